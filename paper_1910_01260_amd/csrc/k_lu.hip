// Batched dense LU with partial pivoting and triangular solves on gfx950.
//
// The reduced space-time system of each query (Sec. 3.2, Eq. (st-galerkin))
// is dense and small (hundreds to a few thousand unknowns); the paper does not
// name its solver, and this is LU with partial pivoting as in LAPACK getrf /
// getrs.  One workgroup factors one query at a time, in place, pulling queries
// from a device work queue ordered largest first (a persistent kernel, so a
// ragged batch runs in one launch).  Matrices are row-major.  Each panel of NB
// columns is factored in registers (the panel's rows are spread over the
// workgroup's threads), its row interchanges are applied to the other columns,
// the NB x (w - p0 - NB) block row is solved against the unit lower panel
// block, and the trailing matrix is updated on the matrix cores with
// v_mfma_{f64,f32}_16x16x4 tiles.
#include "internal.h"

namespace strom {
namespace {

template <typename T>
struct Mfma;

// Lane layouts (checked on gfx950): operand A lane l holds A[l%16][l/16], operand B
// lane l holds B[l/16][l%16]; accumulator register r of lane l holds D[row][l%16] with
// row = l/16 + 4r for the FP64 instruction and row = 4(l/16) + r for the FP32 one.
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ inline v4 op(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

template <typename T>
__device__ inline T wave_shfl_xor(T v, int m) {
  return __shfl_xor(v, m);
}

template <typename T, int NB, int BLOCK, int R>
__global__ __launch_bounds__(BLOCK) void lu_kernel(int32_t n_q, Plan plan, T* __restrict__ mats,
                                                   int32_t* __restrict__ piv) {
  constexpr int NW = BLOCK / 64;
  typedef typename Mfma<T>::v4 v4;
  __shared__ T s_urow[2][NB];
  __shared__ T s_xrow[2][NB];
  __shared__ T s_redv[2][NW];
  __shared__ int32_t s_redr[2][NW];
  __shared__ T s_L11[NB * NB];
  __shared__ int32_t s_piv[NB];
  __shared__ int32_t s_perm[R * BLOCK];  // composed row permutation of the current query
  __shared__ int32_t s_q;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  for (;;) {
    if (tid == 0) s_q = atomicAdd(&plan.counter[0], 1);
    __syncthreads();
    const int32_t idx = s_q;
    __syncthreads();
    if (idx >= n_q) break;
    const int32_t q = plan.order[idx];
    if (plan.info[q] != 0) continue;
    const int32_t w = plan.width[q];
    if (w == 0) continue;
    T* A = mats + plan.mat_off[q];
    int32_t* P = piv + plan.coeff_off[q];
    int32_t zero_piv = 0;
    for (int i = tid; i < w; i += BLOCK) s_perm[i] = i;

    for (int p0 = 0; p0 < w; p0 += NB) {
      const int nb = min(NB, w - p0);
      // ---------------- panel: rows p0.., columns p0..p0+nb, in registers
      T v[R][NB];
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int r = p0 + tid + s * BLOCK;
#pragma unroll
        for (int c = 0; c < NB; ++c) v[s][c] = (r < w && c < nb) ? A[(int64_t)r * w + p0 + c] : T(0);
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < nb) {
          const int buf = c & 1;
          const int diag = p0 + c;
          // pivot search: largest |v| in column c among rows >= diag, lowest row on ties
          T best = T(-1);
          int32_t brow = 0x7fffffff;
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const int r = p0 + tid + s * BLOCK;
            if (r >= diag && r < w) {
              const T a = v[s][c] < T(0) ? -v[s][c] : v[s][c];
              if (a > best) { best = a; brow = r; }
            }
          }
#pragma unroll
          for (int m = 32; m > 0; m >>= 1) {
            const T ob = wave_shfl_xor(best, m);
            const int32_t orow = __shfl_xor(brow, m);
            if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
          }
          if (lane == 0) { s_redv[buf][wave] = best; s_redr[buf][wave] = brow; }
          __syncthreads();
          best = s_redv[buf][0];
          brow = s_redr[buf][0];
#pragma unroll
          for (int k = 1; k < NW; ++k) {
            const T ob = s_redv[buf][k];
            const int32_t orow = s_redr[buf][k];
            if (ob > best || (ob == best && orow < brow)) { best = ob; brow = orow; }
          }
          int32_t prow = brow;
          if (!(best > T(0))) {  // exactly zero (or no finite) pivot: keep the row, record the step
            prow = diag;
            if (zero_piv == 0) zero_piv = diag + 1;
          }
          // exchange rows diag and prow inside the panel; every thread gets the pivot row
          const int tp = (prow - p0) % BLOCK, sp = (prow - p0) / BLOCK;
          if (tid == tp) {
#pragma unroll
            for (int s = 0; s < R; ++s)
              if (s == sp) {
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) s_urow[buf][cc] = v[s][cc];
              }
          }
          if (tid == c) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) s_xrow[buf][cc] = v[0][cc];
          }
          __syncthreads();
          if (tid == c) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) v[0][cc] = s_urow[buf][cc];
          }
          if (tid == tp && prow != diag) {
#pragma unroll
            for (int s = 0; s < R; ++s)
              if (s == sp) {
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) v[s][cc] = s_xrow[buf][cc];
              }
          }
          if (tid == 0) {
            s_piv[c] = prow;
            const int32_t t = s_perm[diag];
            s_perm[diag] = s_perm[prow];
            s_perm[prow] = t;
          }
          const T d = s_urow[buf][c];
          const T inv = (d != T(0)) ? T(1) / d : T(0);
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const int r = p0 + tid + s * BLOCK;
            if (r > diag && r < w) {
              const T l = v[s][c] * inv;
              v[s][c] = l;
#pragma unroll
              for (int cc = c + 1; cc < NB; ++cc) v[s][cc] -= l * s_urow[buf][cc];
            }
          }
        }
      }
      // write the factored panel back
#pragma unroll
      for (int s = 0; s < R; ++s) {
        const int r = p0 + tid + s * BLOCK;
        if (r < w) {
#pragma unroll
          for (int c = 0; c < NB; ++c)
            if (c < nb) A[(int64_t)r * w + p0 + c] = v[s][c];
        }
      }
      __syncthreads();
      // ---------------- row interchanges on the columns outside the panel (in pivot order)
      for (int col = tid; col < w; col += BLOCK) {
        if (col >= p0 && col < p0 + nb) continue;
        for (int c = 0; c < nb; ++c) {
          const int pr = s_piv[c];
          if (pr != p0 + c) {
            T* a = A + (int64_t)(p0 + c) * w + col;
            T* b = A + (int64_t)pr * w + col;
            const T t = *a;
            *a = *b;
            *b = t;
          }
        }
      }
      const int c0 = p0 + nb;
      if (c0 >= w) {
        __syncthreads();
        break;
      }
      // unit lower panel block into LDS
      for (int e = tid; e < nb * nb; e += BLOCK) {
        const int i = e / nb, k = e % nb;
        s_L11[i * NB + k] = A[(int64_t)(p0 + i) * w + p0 + k];
      }
      __syncthreads();
      // ---------------- block row: U12 = L11^{-1} A12 (one column per thread)
      for (int col = c0 + tid; col < w; col += BLOCK) {
        T x[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) x[i] = (i < nb) ? A[(int64_t)(p0 + i) * w + col] : T(0);
#pragma unroll
        for (int i = 1; i < NB; ++i) {
          T acc = x[i];
#pragma unroll
          for (int k = 0; k < i; ++k) acc -= s_L11[i * NB + k] * x[k];
          x[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i < nb) A[(int64_t)(p0 + i) * w + col] = x[i];
      }
      __syncthreads();
      // ---------------- trailing update A22 -= L21 U12 on the matrix cores
      const int m2 = w - c0;
      const int tiles = (m2 + 15) / 16;
      const int li = lane & 15, lk = lane >> 4;
      for (int st = wave; st < tiles; st += NW) {
        const int rb = c0 + st * 16;
        T a[NB / 4];
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk) {
          const int k = kk * 4 + lk;
          const int r = rb + li;
          a[kk] = (r < w && k < nb) ? -A[(int64_t)r * w + p0 + k] : T(0);
        }
        for (int ct = 0; ct < tiles; ++ct) {
          const int cb = c0 + ct * 16;
          const int col = cb + li;
          v4 acc;
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int r = rb + Mfma<T>::row(lk, rr);
            acc[rr] = (r < w && col < w) ? A[(int64_t)r * w + col] : T(0);
          }
#pragma unroll
          for (int kk = 0; kk < NB / 4; ++kk) {
            const int k = kk * 4 + lk;
            const T b = (k < nb && col < w) ? A[(int64_t)(p0 + k) * w + col] : T(0);
            acc = Mfma<T>::op(a[kk], b, acc);
          }
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int r = rb + Mfma<T>::row(lk, rr);
            if (r < w && col < w) A[(int64_t)r * w + col] = acc[rr];
          }
        }
      }
      __syncthreads();
    }
    // row i of P A is row P[i] of A
    for (int i = tid; i < w; i += BLOCK) P[i] = s_perm[i];
    if (tid == 0 && zero_piv) plan.info[q] = zero_piv;
  }
}

// Solve (P^T L U) x = b for each active query: permute b, forward
// substitution with the unit lower factor, back substitution with the upper
// factor, in 64-row blocks (diagonal block by one wave, the rest as wave-wide
// coalesced row dot products).  Accumulation in FP64 whatever T is.
constexpr int kSolveBS = 64;
constexpr int kSolveThreads = 256;

template <typename T>
__global__ __launch_bounds__(kSolveThreads) void lu_solve_kernel(int32_t n_q, Plan plan, const T* __restrict__ mats,
                                                                 const int32_t* __restrict__ piv,
                                                                 const double* __restrict__ b, double* __restrict__ x,
                                                                 int accumulate, const int32_t* __restrict__ active) {
  extern __shared__ __align__(16) double y[];
  __shared__ double dblk[kSolveBS][kSolveBS + 1];
  constexpr int NW = kSolveThreads / 64;
  const int32_t q = blockIdx.x;
  if (plan.info[q] != 0) return;
  if (active && !active[q]) return;
  const int32_t w = plan.width[q];
  if (w == 0) return;
  const int64_t off = plan.coeff_off[q];
  const T* A = mats + plan.mat_off[q];
  const int32_t* P = piv + off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int c = tid; c < w; c += kSolveThreads) y[c] = b[off + P[c]];
  __syncthreads();
  // forward substitution, unit lower triangular
  for (int b0 = 0; b0 < w; b0 += kSolveBS) {
    const int nbk = min(kSolveBS, w - b0);
    for (int e = tid; e < nbk * kSolveBS; e += kSolveThreads) {
      const int i = e / kSolveBS, k = e % kSolveBS;
      dblk[i][k] = (k < nbk) ? (double)A[(int64_t)(b0 + i) * w + b0 + k] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double yi = lane < nbk ? y[b0 + lane] : 0.0;
      for (int k = 0; k < nbk; ++k) {
        const double yk = __shfl(yi, k);
        if (lane > k && lane < nbk) yi -= dblk[lane][k] * yk;
      }
      if (lane < nbk) y[b0 + lane] = yi;
    }
    __syncthreads();
    const double yl = lane < nbk ? y[b0 + lane] : 0.0;
    for (int r = b0 + nbk + wave; r < w; r += NW) {
      double s = lane < nbk ? (double)A[(int64_t)r * w + b0 + lane] * yl : 0.0;
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) y[r] -= s;
    }
    __syncthreads();
  }
  // back substitution, upper triangular
  const int last0 = ((w - 1) / kSolveBS) * kSolveBS;
  for (int b0 = last0; b0 >= 0; b0 -= kSolveBS) {
    const int nbk = min(kSolveBS, w - b0);
    for (int e = tid; e < nbk * kSolveBS; e += kSolveThreads) {
      const int i = e / kSolveBS, k = e % kSolveBS;
      dblk[i][k] = (k < nbk) ? (double)A[(int64_t)(b0 + i) * w + b0 + k] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      double yi = lane < nbk ? y[b0 + lane] : 0.0;
      for (int k = nbk - 1; k >= 0; --k) {
        if (lane == k) yi /= dblk[k][k];
        const double yk = __shfl(yi, k);
        if (lane < k) yi -= dblk[lane][k] * yk;
      }
      if (lane < nbk) y[b0 + lane] = yi;
    }
    __syncthreads();
    const double yl = lane < nbk ? y[b0 + lane] : 0.0;
    for (int r = wave; r < b0; r += NW) {
      double s = lane < nbk ? (double)A[(int64_t)r * w + b0 + lane] * yl : 0.0;
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      if (lane == 0) y[r] -= s;
    }
    __syncthreads();
  }
  for (int c = tid; c < w; c += kSolveThreads) {
    if (accumulate) x[off + c] += y[c];
    else x[off + c] = y[c];
  }
}

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

template <typename T, int NB, int BLOCK, int R>
hipError_t lu_go(int32_t n_q, Plan plan, void* mats, int32_t* piv, int per_cu, hipStream_t s) {
  const int grid = max(1, min(n_q, device_cus() * per_cu));
  hipLaunchKernelGGL((lu_kernel<T, NB, BLOCK, R>), dim3(grid), dim3(BLOCK), 0, s, n_q, plan, (T*)mats, piv);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lu(int32_t n_q, Plan plan, int32_t prec, void* mats, int32_t* piv, int32_t n_max, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  if (n_max <= 1280) {
    if (prec == ST_F64) return lu_go<double, 16, 256, 5>(n_q, plan, mats, piv, 2, s);
    return lu_go<float, 32, 256, 5>(n_q, plan, mats, piv, 2, s);
  }
  if (n_max <= 4096) {
    if (prec == ST_F64) return lu_go<double, 16, 1024, 4>(n_q, plan, mats, piv, 1, s);
    return lu_go<float, 16, 1024, 4>(n_q, plan, mats, piv, 1, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lu_solve(int32_t n_q, Plan plan, int32_t prec, const void* mats, const int32_t* piv, const double* b,
                           double* x, int accumulate, const int32_t* active, int32_t n_max, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  const size_t lds = sizeof(double) * (size_t)n_max;
  hipError_t e = hipFuncSetAttribute(prec == ST_F64 ? (const void*)lu_solve_kernel<double>
                                                    : (const void*)lu_solve_kernel<float>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (prec == ST_F64) {
    hipLaunchKernelGGL(lu_solve_kernel<double>, dim3(n_q), dim3(kSolveThreads), lds, s, n_q, plan,
                       (const double*)mats, piv, b, x, accumulate, active);
  } else {
    hipLaunchKernelGGL(lu_solve_kernel<float>, dim3(n_q), dim3(kSolveThreads), lds, s, n_q, plan, (const float*)mats,
                       piv, b, x, accumulate, active);
  }
  return hipGetLastError();
}

}  // namespace strom
