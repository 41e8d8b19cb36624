// POD on gfx950 (Sec. 4.1, Eq. (snapshotmat), (POD), (SVD), (temporalSVD)),
// computed by the method of snapshots:
//   a1  Gram of the snapshot matrix on the matrix cores (FP64 MFMA, or FP32 /
//       split-BF16 MFMA with FP32 accumulation), lower tiles, split-K;
//   a2  leading eigenpairs in FP64 by subspace iteration: products on the
//       GPU, a one-workgroup classical Gram-Schmidt (twice) orthonormalisation,
//       and a Rayleigh-Ritz step solved by a one-workgroup cyclic Jacobi
//       eigensolver in parallel (round-robin) order;
//   a3  spatial basis: the eigenvectors themselves when the Gram is U U^T,
//       otherwise U V diag(1/sigma) re-orthonormalised by two Cholesky-QR passes;
//   a4  temporal bases: per mode, a one-sided Jacobi SVD of the temporal
//       snapshot matrix, a numerical-rank cut and a DCT-II completion.
#include <math.h>

#include "internal.h"

namespace strom {
namespace {

constexpr int kOneWG = 1024;
constexpr int kTsvdThreads = 1024;  // one workgroup per mode: one wave per column pair of a round
constexpr size_t kOrthMaxLds = 144 * 1024;  // single-workgroup kernels stage their matrices in LDS up to this size
constexpr int kMaxSubspaceDev = 256;        // column limit of the subspace kernels (k <= 256)
constexpr int kOrthBlock = 16;             // column block of the blocked Gram-Schmidt (long columns)

// wavefront reductions of the device library (DPP based, all lanes active)
extern "C" __device__ double __ockl_wfred_add_f64(double);
extern "C" __device__ double __ockl_wfred_max_f64(double);
extern "C" __device__ int __ockl_wfred_min_i32(int);

__device__ inline uint64_t mix64(uint64_t z) {
  // splitmix64 finaliser (Steele, Lea, Flood)
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ inline double rand_pm(uint64_t seed, int64_t i, int64_t j) {
  const uint64_t h = mix64(seed ^ mix64((uint64_t)i * 0x100000001B3ULL + (uint64_t)j));
  return (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

template <typename T>
__device__ inline T block_sum(T v, T* red) {
  // red: LDS of blockDim.x/64 entries; returns the sum to every thread
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = __ockl_wfred_add_f64(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  T s = 0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

__device__ inline double block_max(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = __ockl_wfred_max_f64(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < nw; ++w) s = fmax(s, red[w]);
  return s;
}

__device__ inline int block_min_i(int v, int* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = __ockl_wfred_min_i32(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  int s = red[0];
  for (int w = 1; w < nw; ++w) s = min(s, red[w]);
  return s;
}

// ---------------------------------------------------------------------------
// a1: Gram C = X^T X (p x p) with X of K rows; X element (k, a) at X[k*ks + a*ms].
// 64 x 64 lower output tiles, 4 waves each owning 32 x 32 (2 x 2 MFMA tiles).
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;   // output tile
constexpr int kGK = 32;   // K chunk of the FP32 / split-BF16 Gram
constexpr int kGK64 = 16; // K chunk of the FP64 Gram (smaller LDS and staging: more workgroups per CU;
                          // measured on 2.1M x 8000: 2.52 s against 2.74 s with 32 and 2.65 s with 64)
constexpr int kFlushChunks = 32;  // FP32 Gram accumulators move to FP64 every 32 chunks (1024 terms)

__device__ inline void tile_of(int t, int& ti, int& tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  ti = i;
  tj = t - i * (i + 1) / 2;
}

// A K-chunk of KC rows of one 64-column panel: each of the 256 threads holds
// stage_per<KC>() entries in registers (fetched for the next chunk while the
// matrix cores work on the current one), then writes them to LDS as [k][column].
template <int KC>
constexpr int stage_per() { return KC * kGT / 256; }

template <int KC, typename InT>
__device__ inline void gram_fetch(const InT* __restrict__ X, int p, int64_t ks, int64_t ms, int64_t k0, int64_t kend,
                                  int a0, InT (&v)[stage_per<KC>()]) {
#pragma unroll
  for (int i = 0; i < stage_per<KC>(); ++i) {
    const int e = threadIdx.x + i * 256;
    int kk, a;
    if (ks == 1) { kk = e % KC; a = e / KC; } else { a = e % kGT; kk = e / kGT; }
    const int64_t k = k0 + kk;
    v[i] = (k < kend && a0 + a < p) ? X[k * ks + (int64_t)(a0 + a) * ms] : InT(0);
  }
}

template <int KC, typename InT, typename DstT, int LD>
__device__ inline void gram_put(const InT (&v)[stage_per<KC>()], int64_t ks, DstT (*dst)[LD]) {
#pragma unroll
  for (int i = 0; i < stage_per<KC>(); ++i) {
    const int e = threadIdx.x + i * 256;
    int kk, a;
    if (ks == 1) { kk = e % KC; a = e / KC; } else { a = e % kGT; kk = e / kGT; }
    dst[kk][a] = (DstT)v[i];
  }
}

template <typename InT>
__global__ __launch_bounds__(256) void gram_f64_kernel(int64_t K, int p, const InT* __restrict__ X, int64_t ks,
                                                       int64_t ms, int64_t k_per_split, double* __restrict__ partial) {
  __shared__ double Xa[kGK64][kGT + 1];
  __shared__ double Xb[kGK64][kGT + 1];
  int ti, tj;
  tile_of(blockIdx.x, ti, tj);
  const int a0 = ti * kGT, b0 = tj * kGT;
  const int64_t kbeg = (int64_t)blockIdx.y * k_per_split;
  const int64_t kend = min(K, kbeg + k_per_split);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc[x][y] = d4{0.0, 0.0, 0.0, 0.0};
  const bool two = ti != tj;
  InT va[stage_per<kGK64>()], vb[stage_per<kGK64>()];
  gram_fetch<kGK64, InT>(X, p, ks, ms, kbeg, kend, a0, va);
  if (two) gram_fetch<kGK64, InT>(X, p, ks, ms, kbeg, kend, b0, vb);
  for (int64_t k0 = kbeg; k0 < kend; k0 += kGK64) {
    gram_put<kGK64, InT, double, kGT + 1>(va, ks, Xa);
    if (two) gram_put<kGK64, InT, double, kGT + 1>(vb, ks, Xb);
    __syncthreads();
    if (k0 + kGK64 < kend) {  // the next chunk is in flight while this one is multiplied
      gram_fetch<kGK64, InT>(X, p, ks, ms, k0 + kGK64, kend, a0, va);
      if (two) gram_fetch<kGK64, InT>(X, p, ks, ms, k0 + kGK64, kend, b0, vb);
    }
    double(*B)[kGT + 1] = two ? Xb : Xa;
#pragma unroll
    for (int kk = 0; kk < kGK64; kk += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = Xa[kk + lk][wi * 32 + x * 16 + li];
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = B[kk + lk][wj * 32 + y * 16 + li];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.y * p * p;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + wi * 32 + x * 16 + lk + 4 * r;  // FP64 accumulator row = lane/16 + 4r
        const int b = b0 + wj * 32 + y * 16 + li;
        if (a < p && b < p) out[a + (int64_t)b * p] = acc[x][y][r];
      }
}

// FP32 MFMA (ST_F32) or split-BF16 (ST_BF16X3): inputs rounded to FP32, products accumulated in FP32 over
// 1024-term stretches of K, which are summed in FP64.
__device__ inline short bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ inline float bf16_to_f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

template <typename InT, bool SPLIT>
__global__ __launch_bounds__(256) void gram_f32_kernel(int64_t K, int p, const InT* __restrict__ X, int64_t ks,
                                                       int64_t ms, int64_t k_per_split, double* __restrict__ partial) {
  __shared__ float Xa[kGK][kGT + 4];
  __shared__ float Xb[kGK][kGT + 4];
  int ti, tj;
  tile_of(blockIdx.x, ti, tj);
  const int a0 = ti * kGT, b0 = tj * kGT;
  const int64_t kbeg = (int64_t)blockIdx.y * k_per_split;
  const int64_t kend = min(K, kbeg + k_per_split);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave >> 1, wj = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  f4 acc[2][2];
  double acc64[2][2][4];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) {
      acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};
      for (int r = 0; r < 4; ++r) acc64[x][y][r] = 0.0;
    }
  int chunk = 0;
  const bool two = ti != tj;
  InT va[stage_per<kGK>()], vb[stage_per<kGK>()];
  gram_fetch<kGK, InT>(X, p, ks, ms, kbeg, kend, a0, va);
  if (two) gram_fetch<kGK, InT>(X, p, ks, ms, kbeg, kend, b0, vb);
  for (int64_t k0 = kbeg; k0 < kend; k0 += kGK) {
    if (++chunk == kFlushChunks) {
      // FP32 accumulation only within kFlushChunks * kGK terms; the chunks add up in FP64
      chunk = 0;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc64[x][y][r] += (double)acc[x][y][r];
            acc[x][y][r] = 0.f;
          }
    }
    gram_put<kGK, InT, float, kGT + 4>(va, ks, Xa);
    if (two) gram_put<kGK, InT, float, kGT + 4>(vb, ks, Xb);
    __syncthreads();
    if (k0 + kGK < kend) {  // the next chunk is in flight while this one is multiplied
      gram_fetch<kGK, InT>(X, p, ks, ms, k0 + kGK, kend, a0, va);
      if (two) gram_fetch<kGK, InT>(X, p, ks, ms, k0 + kGK, kend, b0, vb);
    }
    float(*B)[kGT + 4] = two ? Xb : Xa;
    if (!SPLIT) {
#pragma unroll
      for (int kk = 0; kk < kGK; kk += 4) {
        float av[2], bv[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) av[x] = Xa[kk + lk][wi * 32 + x * 16 + li];
#pragma unroll
        for (int y = 0; y < 2; ++y) bv[y] = B[kk + lk][wj * 32 + y * 16 + li];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[x], bv[y], acc[x][y], 0, 0, 0);
      }
    } else {
      // bf16 16x16x16: operand A lane l holds A[l%16][4(l/16) .. 4(l/16)+3], B likewise B[4(l/16)..][l%16]
#pragma unroll
      for (int kk = 0; kk < kGK; kk += 16) {
        s4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float v = Xa[kk + 4 * lk + e][wi * 32 + x * 16 + li];
            const short h = bf16_rne(v);
            ah[x][e] = h;
            al[x][e] = bf16_rne(v - bf16_to_f(h));
          }
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float v = B[kk + 4 * lk + e][wj * 32 + y * 16 + li];
            const short h = bf16_rne(v);
            bh[y][e] = h;
            bl[y][e] = bf16_rne(v - bf16_to_f(h));
          }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[x], bh[y], acc[x][y], 0, 0, 0);
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[x], bl[y], acc[x][y], 0, 0, 0);
            acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[x], bh[y], acc[x][y], 0, 0, 0);
          }
      }
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.y * p * p;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = a0 + wi * 32 + x * 16 + 4 * lk + r;  // FP32 accumulator row = 4(lane/16) + r
        const int b = b0 + wj * 32 + y * 16 + li;
        if (a < p && b < p) out[a + (int64_t)b * p] = acc64[x][y][r] + (double)acc[x][y][r];
      }
}

// G[a,b] = G[b,a] = sum_z partial[z][max + min*p]
__global__ void gram_finish_kernel(int p, int splits, const double* __restrict__ partial, double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pp = (int64_t)p * p;
  if (e >= pp) return;
  const int a = (int)(e % p), b = (int)(e / p);
  const int hi = max(a, b), lo = min(a, b);
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += partial[z * pp + hi + (int64_t)lo * p];
  G[e] = s;
}

// ---------------------------------------------------------------------------
// a2: one-workgroup kernels
// ---------------------------------------------------------------------------

// X (p x k, column-major) <- pseudo-random entries
__global__ void rand_fill_kernel(double* X, int64_t p, int k, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * k) return;
  X[e] = rand_pm(seed, e % p, e / p);
}

// Orthonormalise the k columns of X (p x k, column-major) in place by
// classical Gram-Schmidt applied twice per column; a column that loses all
// but 1e-10 of its norm (dependent on the previous ones) is replaced by a
// pseudo-random vector and orthogonalised again.  With IN_LDS the columns are
// staged in LDS for the whole sweep (every column step touches all previous
// columns, so a global round trip per step would dominate).  As the last step of
// a blocked sweep (X a block of columns col0 .. col0 + k - 1 already projected
// against the columns before it): n0sq holds each column's squared norm before
// that projection (the reference of the dependence test), the pseudo-random
// refills are numbered by col0 + j, and *refilled is set when one was needed
// (the caller then projects the block against the earlier columns again).
template <bool IN_LDS>
__global__ __launch_bounds__(kOneWG) void orth_cgs2_kernel(double* Xg, int64_t p, int k, uint64_t seed,
                                                           const double* __restrict__ n0sq, int col0,
                                                           int* __restrict__ refilled) {
  extern __shared__ __align__(16) double xs_lds[];
  __shared__ double coef[256];
  __shared__ double red[kOneWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kOneWG / 64;
  double* X = IN_LDS ? xs_lds : Xg;
  if (IN_LDS) {
    for (int64_t e = tid; e < p * k; e += kOneWG) X[e] = Xg[e];
    __syncthreads();
  }
  // coef[l] = x_l . x_j for l < lim (one wave per dot, lanes over the rows)
  auto dots = [&](const double* xj, int lim) {
    for (int l = wave; l < lim; l += nw) {
      const double* xl = X + (int64_t)l * p;
      double s = 0.0;
      for (int64_t r = lane; r < p; r += 64) s = fma(xl[r], xj[r], s);
      s = __ockl_wfred_add_f64(s);
      if (lane == 0) coef[l] = s;
    }
  };
  // x_j -= sum_{l < j} coef[l] x_l; returns this thread's share of the new squared norm
  auto project = [&](double* xj, int j) {
    double nn = 0.0;
    for (int64_t r = tid; r < p; r += kOneWG) {
      double v = xj[r];
#pragma unroll 8
      for (int l = 0; l < j; ++l) v = fma(-coef[l], X[(int64_t)l * p + r], v);
      xj[r] = v;
      nn = fma(v, v, nn);
    }
    return nn;
  };
  for (int j = 0; j < k; ++j) {
    double* xj = X + (int64_t)j * p;
    for (int attempt = 0; attempt < 4; ++attempt) {
      // first pass: the projections and the column's own squared norm (slot j) together
      dots(xj, j + 1);
      __syncthreads();
      const double n0 = (n0sq && attempt == 0) ? sqrt(n0sq[j]) : sqrt(coef[j]);
      double nn;
      if (j > 0) {
        project(xj, j);
        __syncthreads();
        dots(xj, j);
        __syncthreads();
        nn = project(xj, j);
      } else {
        nn = 0.0;
        for (int64_t r = tid; r < p; r += kOneWG) nn = fma(xj[r], xj[r], nn);
      }
      const double n1 = sqrt(block_sum(nn, red));
      if (n1 > 1e-10 * n0 && n1 > 0.0) {
        const double inv = 1.0 / n1;
        for (int64_t r = tid; r < p; r += kOneWG) xj[r] *= inv;
        __syncthreads();
        break;
      }
      // dependent column: refill and retry
      for (int64_t r = tid; r < p; r += kOneWG) xj[r] = rand_pm(seed + 7919ULL * (attempt + 1), r, col0 + j);
      if (tid == 0 && refilled) *refilled = 1;
      __syncthreads();
    }
  }
  if (IN_LDS) {
    __syncthreads();
    for (int64_t e = tid; e < p * k; e += kOneWG) Xg[e] = X[e];
  }
}

// Symmetric eigen-decomposition of A (k x k, column-major, overwritten) by
// cyclic Jacobi in round-robin parallel order; eigenvalues descending in
// evals, eigenvectors in the matching columns of Zout.  Work arrays A, Z
// (k*k each) may be global memory; k <= 256.
template <bool IN_LDS>
__global__ __launch_bounds__(kOneWG) void jacobi_eig_kernel(int k, double* Ag, double* Zg, double* evals, double* Zout,
                                                            int max_sweeps) {
  extern __shared__ __align__(16) double az_lds[];
  __shared__ int sp[128], sq[128];
  __shared__ double sc[128], ss[128];
  __shared__ double red[kOneWG / 64];
  __shared__ int s_rot;
  __shared__ int s_rank[256];
  const int tid = threadIdx.x;
  // with IN_LDS the matrix and the rotations are kept in LDS for all sweeps (every round
  // touches two rows and two columns of each and ends in a barrier)
  double* A = IN_LDS ? az_lds : Ag;
  double* Z = IN_LDS ? az_lds + (size_t)k * k : Zg;
  if (IN_LDS)
    for (int e = tid; e < k * k; e += kOneWG) A[e] = Ag[e];
  for (int e = tid; e < k * k; e += kOneWG) Z[e] = (e % k == e / k) ? 1.0 : 0.0;
  const int kk = k + (k & 1);
  const int m = kk - 1;
  double fro = 0.0;
  for (int e = tid; e < k * k; e += kOneWG) fro = fma(A[e], A[e], fro);
  __syncthreads();
  fro = sqrt(block_sum(fro, red));
  const double thr = 1e-22 * fro;
  for (int sweep = 0; sweep < max_sweeps && k > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < m; ++rnd) {
      if (tid < kk / 2) {
        int a, b;
        if (tid == 0) { a = m; b = rnd; }
        else { a = (rnd + tid) % m; b = (rnd - tid + m) % m; }
        if (a > b) { const int t = a; a = b; b = t; }
        double c = 1.0, s = 0.0;
        if (b < k) {
          const double apq = A[a + (int64_t)b * k];
          const double app = A[a + (int64_t)a * k], aqq = A[b + (int64_t)b * k];
          if (fabs(apq) > thr && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            s_rot = 1;
          }
        }
        sp[tid] = a; sq[tid] = b; sc[tid] = c; ss[tid] = s;
      }
      __syncthreads();
      const int np = kk / 2;
      // rows p, q of A
      for (int e = tid; e < np * k; e += kOneWG) {
        const int t = e / k, j = e % k;
        const int a = sp[t], b = sq[t];
        if (b >= k || ss[t] == 0.0) continue;
        const double c = sc[t], s = ss[t];
        const double x = A[a + (int64_t)j * k], y = A[b + (int64_t)j * k];
        A[a + (int64_t)j * k] = c * x - s * y;
        A[b + (int64_t)j * k] = s * x + c * y;
      }
      __syncthreads();
      // columns p, q of A and of Z
      for (int e = tid; e < np * k; e += kOneWG) {
        const int t = e / k, i = e % k;
        const int a = sp[t], b = sq[t];
        if (b >= k || ss[t] == 0.0) continue;
        const double c = sc[t], s = ss[t];
        double x = A[i + (int64_t)a * k], y = A[i + (int64_t)b * k];
        // the rotation annihilates (a, b) and (b, a) exactly in exact arithmetic: store zeros
        A[i + (int64_t)a * k] = (i == b) ? 0.0 : c * x - s * y;
        A[i + (int64_t)b * k] = (i == a) ? 0.0 : s * x + c * y;
        x = Z[i + (int64_t)a * k];
        y = Z[i + (int64_t)b * k];
        Z[i + (int64_t)a * k] = c * x - s * y;
        Z[i + (int64_t)b * k] = s * x + c * y;
      }
      __syncthreads();
    }
    if (!s_rot) break;
    __syncthreads();
  }
  // sort descending (rank by value, ties by index)
  for (int i = tid; i < k; i += kOneWG) {
    const double di = A[i + (int64_t)i * k];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double dj = A[j + (int64_t)j * k];
      if (dj > di || (dj == di && j < i)) ++rank;
    }
    s_rank[i] = rank;
  }
  __syncthreads();
  for (int i = tid; i < k; i += kOneWG) evals[s_rank[i]] = A[i + (int64_t)i * k];
  for (int e = tid; e < k * k; e += kOneWG) {
    const int i = e % k, j = e / k;
    Zout[i + (int64_t)s_rank[j] * k] = Z[e];
  }
  if (IN_LDS)
    for (int e = tid; e < k * k; e += kOneWG) {
      Ag[e] = A[e];
      Zg[e] = Z[e];
    }
}

// Upper Cholesky factor of S (n x n, column-major) and its inverse:
// S = R^T R, Rinv = R^{-1}.  Pivots are floored at 1e-30 of the largest
// diagonal so the second pass of Cholesky-QR can repair a near-singular first.
__global__ __launch_bounds__(kOneWG) void chol_inv_kernel(int n, double* S, double* Rinv) {
  __shared__ double red[kOneWG / 64];
  __shared__ double s_d;
  const int tid = threadIdx.x;
  double dmax = 0.0;
  for (int i = tid; i < n; i += kOneWG) dmax = fmax(dmax, S[i + (int64_t)i * n]);
  dmax = block_max(dmax, red);
  // right-looking: after step j, row j of S holds row j of R
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      double d = S[j + (int64_t)j * n];
      d = sqrt(fmax(d, 1e-30 * dmax));
      s_d = d;
      S[j + (int64_t)j * n] = d;
    }
    __syncthreads();
    const double d = s_d;
    for (int c = j + 1 + tid; c < n; c += kOneWG) S[j + (int64_t)c * n] /= d;
    __syncthreads();
    for (int e = tid; e < (n - j - 1) * (n - j - 1); e += kOneWG) {
      const int r = j + 1 + e % (n - j - 1), c = j + 1 + e / (n - j - 1);
      if (r <= c) S[r + (int64_t)c * n] -= S[j + (int64_t)r * n] * S[j + (int64_t)c * n];
    }
    __syncthreads();
  }
  // Rinv column c: solve R x = e_c (upper), one thread per column
  for (int c = tid; c < n; c += kOneWG) {
    for (int i = n - 1; i >= 0; --i) {
      double v = (i == c) ? 1.0 : 0.0;
      if (i > c) v = 0.0;
      for (int l = i + 1; l <= c; ++l) v -= S[i + (int64_t)l * n] * Rinv[l + (int64_t)c * n];
      Rinv[i + (int64_t)c * n] = (i <= c) ? v / S[i + (int64_t)i * n] : 0.0;
    }
  }
}

// Column j of X (p rows, column-major, ld p) scaled by 1/sigma_j when
// sigma_j > cut * sigma_0, else replaced with a pseudo-random column.
__global__ void scale_or_refill_kernel(double* X, int64_t p, int k, const double* sigma, double cut, uint64_t seed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * k) return;
  const int j = (int)(e / p);
  const double s0 = sigma[0], sj = sigma[j];
  if (sj > cut * s0 && sj > 0.0) X[e] /= sj;
  else X[e] = rand_pm(seed, e % p, j);
}

// sigma_i = sqrt(max(lambda_i, 0))
__global__ void sqrt_clamp_kernel(const double* lam, double* sigma, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) sigma[i] = sqrt(fmax(lam[i], 0.0));
}

// Sign convention: column j of X (ld p) becomes positive at its first entry whose
// magnitude is >= 1/4 of its largest; the same flip is applied to column j of Y.
__global__ __launch_bounds__(256) void sign_fix_kernel(double* X, int64_t p, double* Y, int64_t py) {
  __shared__ double red[4];
  __shared__ int redi[4];
  __shared__ double s_flip;
  const int j = blockIdx.x;
  double* x = X + (int64_t)j * p;
  double m = 0.0;
  for (int64_t r = threadIdx.x; r < p; r += 256) m = fmax(m, fabs(x[r]));
  m = block_max(m, red);
  int first = 0x7fffffff;
  for (int64_t r = threadIdx.x; r < p; r += 256)
    if (m > 0.0 && fabs(x[r]) >= 0.25 * m) { first = (int)r; break; }
  first = block_min_i(first, redi);
  if (threadIdx.x == 0) s_flip = (m > 0.0 && x[first] < 0.0) ? -1.0 : 1.0;
  __syncthreads();
  const double f = s_flip;
  if (f < 0.0) {
    for (int64_t r = threadIdx.x; r < p; r += 256) x[r] = -x[r];
    if (Y)
      for (int64_t r = threadIdx.x; r < py; r += 256) Y[(int64_t)j * py + r] = -Y[(int64_t)j * py + r];
  }
}

// Copy the first n columns of src (ld_src) into dst (ld_dst), p rows each.
__global__ void copy_cols_kernel(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int64_t p, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * n) return;
  const int64_t r = e % p, c = e / p;
  dst[r + c * ld_dst] = src[r + c * ld_src];
}

// ---------------------------------------------------------------------------
// a3 refinement: one-sided (Hestenes) Jacobi SVD of the tall matrix B^T = U^T Q
// (m x k, column-major in global memory), with Q an orthonormal basis of the
// leading left singular subspace.  Because Q comes from the Gram eigenvectors,
// the columns of B^T are already nearly orthogonal (preconditioned Jacobi): the
// resolved modes converge in one or two sweeps, and the Gram's squaring of the
// condition number is undone - the singular vectors are those of U itself, not
// of U^T U.  The rotations are accumulated in J (k x k), so that the refined
// left singular vectors are Q J and the right ones the normalised columns.
// One launch per round of the round-robin (tournament) ordering, one workgroup
// per column pair; rounds of a sweep touch disjoint pairs.
// ---------------------------------------------------------------------------
constexpr int kTallThreads = 256;
// inner two-sided Jacobi of a blocked pass: relative skip threshold and sweep limit
constexpr double kGramInnerEps = 1e-16;
constexpr int kGramInnerSweeps = 10;

// Pair `pr` of round `round` over kk (even) players: player 0 stays, the others rotate.
__device__ inline void tournament_pair(int round, int pr, int kk, int& a, int& b) {
  const int L = kk - 1;
  if (pr == 0) {
    a = 0;
    b = 1 + round % L;
  } else {
    a = 1 + (round + pr) % L;
    b = 1 + (round - pr + L) % L;
  }
}

// atomic max of a non-negative double through its bit pattern (monotone for x >= 0)
__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

__global__ __launch_bounds__(kTallThreads) void tall_jacobi_round_kernel(double* __restrict__ A, int64_t m, int k,
                                                                          int kk, double* __restrict__ J, int round,
                                                                          int sweep, int* __restrict__ rot,
                                                                          double* __restrict__ offmax, double tol) {
  __shared__ double red[3][kTallThreads / 64];
  if (sweep > 0 && rot[sweep - 1] == 0) return;  // the previous sweep rotated nothing: converged
  int a, b;
  tournament_pair(round, blockIdx.x, kk, a, b);
  if (a >= k || b >= k) return;  // padding player of an odd k
  double* x = A + (int64_t)a * m;
  double* y = A + (int64_t)b * m;
  double saa = 0.0, sbb = 0.0, sab = 0.0;
  for (int64_t r = threadIdx.x; r < m; r += kTallThreads) {
    const double u = x[r], v = y[r];
    saa = fma(u, u, saa);
    sbb = fma(v, v, sbb);
    sab = fma(u, v, sab);
  }
  saa = __ockl_wfred_add_f64(saa);
  sbb = __ockl_wfred_add_f64(sbb);
  sab = __ockl_wfred_add_f64(sab);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = saa;
    red[1][wave] = sbb;
    red[2][wave] = sab;
  }
  __syncthreads();
  saa = sbb = sab = 0.0;
  for (int w = 0; w < kTallThreads / 64; ++w) {
    saa += red[0][w];
    sbb += red[1][w];
    sab += red[2][w];
  }
  const double scale = sqrt(saa) * sqrt(sbb);
  const double off = scale > 0.0 ? fabs(sab) / scale : 0.0;
  if (threadIdx.x == 0) atomic_max_nonneg(&offmax[sweep], off);
  if (!(off > tol)) return;  // already orthogonal to the tolerance (uniform decision)
  // rotation that zeroes the inner product of the pair
  const double zeta = (sbb - saa) / (2.0 * sab);
  const double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
  const double c = 1.0 / sqrt(fma(t, t, 1.0));
  const double s = c * t;
  for (int64_t r = threadIdx.x; r < m; r += kTallThreads) {
    const double u = x[r], v = y[r];
    x[r] = c * u - s * v;
    y[r] = s * u + c * v;
  }
  if (J)
    for (int r = threadIdx.x; r < k; r += kTallThreads) {
      const double u = J[r + (int64_t)a * k], v = J[r + (int64_t)b * k];
      J[r + (int64_t)a * k] = c * u - s * v;
      J[r + (int64_t)b * k] = s * u + c * v;
    }
  if (threadIdx.x == 0) atomicAdd(&rot[sweep], 1);
}

// The same one-sided Jacobi in one workgroup with the whole m x k matrix in LDS
// (all sweeps in one launch): one wave per column pair of a round, a barrier per
// round, the sweep loop ends once a sweep rotated nothing.  Records rot[] and
// offmax[] as the per-round kernel does.
__global__ __launch_bounds__(kOneWG) void tall_jacobi_lds_kernel(double* __restrict__ Ag, int64_t m, int k,
                                                                  double* __restrict__ J, int max_sweeps,
                                                                  int* __restrict__ rot,
                                                                  double* __restrict__ offmax, double tol) {
  extern __shared__ __align__(16) double As[];
  __shared__ int s_rot;
  __shared__ double s_off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NWV = kOneWG / 64;
  for (int64_t e = tid; e < m * k; e += kOneWG) As[e] = Ag[e];
  const int kk = (k + 1) / 2 * 2;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (tid == 0) {
      s_rot = 0;
      s_off = 0.0;
    }
    __syncthreads();
    for (int r = 0; r < kk - 1; ++r) {
      for (int pr = wave; pr < kk / 2; pr += NWV) {
        int a, b;
        tournament_pair(r, pr, kk, a, b);
        if (a >= k || b >= k) continue;
        double* x = As + (int64_t)a * m;
        double* y = As + (int64_t)b * m;
        double saa = 0.0, sbb = 0.0, sab = 0.0;
        for (int64_t i = lane; i < m; i += 64) {
          const double u = x[i], v = y[i];
          saa = fma(u, u, saa);
          sbb = fma(v, v, sbb);
          sab = fma(u, v, sab);
        }
        saa = __ockl_wfred_add_f64(saa);
        sbb = __ockl_wfred_add_f64(sbb);
        sab = __ockl_wfred_add_f64(sab);
        const double scale = sqrt(saa) * sqrt(sbb);
        const double off = scale > 0.0 ? fabs(sab) / scale : 0.0;
        if (lane == 0) atomic_max_nonneg(&s_off, off);
        if (!(off > tol)) continue;
        const double zeta = (sbb - saa) / (2.0 * sab);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
        const double c = 1.0 / sqrt(fma(t, t, 1.0));
        const double sn = c * t;
        for (int64_t i = lane; i < m; i += 64) {
          const double u = x[i], v = y[i];
          x[i] = c * u - sn * v;
          y[i] = sn * u + c * v;
        }
        if (J)
          for (int i = lane; i < k; i += 64) {
            const double u = J[i + (int64_t)a * k], v = J[i + (int64_t)b * k];
            J[i + (int64_t)a * k] = c * u - sn * v;
            J[i + (int64_t)b * k] = sn * u + c * v;
          }
        if (lane == 0) atomicAdd(&s_rot, 1);
      }
      __syncthreads();
    }
    const int nrot = s_rot;
    if (tid == 0) {
      rot[sw] = nrot;
      offmax[sw] = s_off;
    }
    __syncthreads();
    if (nrot == 0) break;
  }
  for (int64_t e = tid; e < m * k; e += kOneWG) Ag[e] = As[e];
}

// One pass of the blocked form of the same one-sided Jacobi, for columns too long
// to sweep pair by pair: the caller forms G = A^T A of the current columns; this
// measures its largest |cos| between two columns (offmax[sweep]) and, when that
// exceeds tol, diagonalises G by cyclic two-sided Jacobi (the rotation of each
// pair is the one the one-sided method would take from the same three inner
// products; pairs with |g_ab| <= eps_in sqrt(g_aa g_bb) are skipped) with the
// rotations accumulated in V (k x k, column-major), which the caller applies to
// A and J.  rot[sweep] = 0 when converged, else the inner sweeps that ran (>= 1).
// With IN_LDS, G is copied into LDS; otherwise it is worked on in place.
template <bool IN_LDS>
__global__ __launch_bounds__(kOneWG) void gram_jacobi_kernel(int k, double* __restrict__ Gg, double* __restrict__ V,
                                                             int sweep, int* __restrict__ rot,
                                                             double* __restrict__ offmax, double tol, double eps_in,
                                                             int max_inner) {
  extern __shared__ __align__(16) double gj_lds[];
  __shared__ int sp[kMaxSubspaceDev / 2], sq[kMaxSubspaceDev / 2];
  __shared__ double sc[kMaxSubspaceDev / 2], ss[kMaxSubspaceDev / 2];
  __shared__ double red[kOneWG / 64];
  __shared__ int s_rot;
  const int tid = threadIdx.x;
  double* G = IN_LDS ? gj_lds : Gg;
  if (IN_LDS)
    for (int e = tid; e < k * k; e += kOneWG) G[e] = Gg[e];
  __syncthreads();
  double off = 0.0;
  for (int e = tid; e < k * k; e += kOneWG) {
    const int a = e % k, b = e / k;
    if (a < b) {
      const double d = sqrt(fabs(G[a + (int64_t)a * k])) * sqrt(fabs(G[b + (int64_t)b * k]));
      if (d > 0.0) off = fmax(off, fabs(G[e]) / d);
    }
  }
  off = block_max(off, red);
  if (tid == 0) offmax[sweep] = off;
  if (!(off > tol)) {  // uniform: every thread holds the same maximum
    if (tid == 0) rot[sweep] = 0;
    return;
  }
  for (int e = tid; e < k * k; e += kOneWG) V[e] = (e % k == e / k) ? 1.0 : 0.0;
  const int kk = (k + 1) / 2 * 2, np = kk / 2;
  int used = 0;
  for (int inner = 0; inner < max_inner; ++inner) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < kk - 1; ++rnd) {
      if (tid < np) {
        int a, b;
        tournament_pair(rnd, tid, kk, a, b);
        if (a > b) {
          const int t = a;
          a = b;
          b = t;
        }
        double c = 1.0, sn = 0.0;
        if (b < k) {
          const double gab = G[a + (int64_t)b * k];
          const double gaa = fabs(G[a + (int64_t)a * k]), gbb = fabs(G[b + (int64_t)b * k]);
          if (fabs(gab) > eps_in * sqrt(gaa) * sqrt(gbb)) {
            const double zeta = (gbb - gaa) / (2.0 * gab);
            const double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
            c = 1.0 / sqrt(fma(t, t, 1.0));
            sn = c * t;
            s_rot = 1;
          }
        }
        sp[tid] = a;
        sq[tid] = b;
        sc[tid] = c;
        ss[tid] = sn;
      }
      __syncthreads();
      // rows a and b: G <- R^T G (R: column a -> c a - s b, column b -> s a + c b)
      for (int e = tid; e < np * k; e += kOneWG) {
        const int t = e / k, j = e % k;
        const int a = sp[t], b = sq[t];
        if (b >= k || ss[t] == 0.0) continue;
        const double c = sc[t], sn = ss[t];
        const double x = G[a + (int64_t)j * k], y = G[b + (int64_t)j * k];
        G[a + (int64_t)j * k] = c * x - sn * y;
        G[b + (int64_t)j * k] = sn * x + c * y;
      }
      __syncthreads();
      // columns a and b of G (the pair's own entries become exact zeros) and of V
      for (int e = tid; e < np * k; e += kOneWG) {
        const int t = e / k, i = e % k;
        const int a = sp[t], b = sq[t];
        if (b >= k || ss[t] == 0.0) continue;
        const double c = sc[t], sn = ss[t];
        const double x = G[i + (int64_t)a * k], y = G[i + (int64_t)b * k];
        G[i + (int64_t)a * k] = (i == b) ? 0.0 : c * x - sn * y;
        G[i + (int64_t)b * k] = (i == a) ? 0.0 : sn * x + c * y;
        const double u = V[i + (int64_t)a * k], v = V[i + (int64_t)b * k];
        V[i + (int64_t)a * k] = c * u - sn * v;
        V[i + (int64_t)b * k] = sn * u + c * v;
      }
      __syncthreads();
    }
    const int nrot = s_rot;
    __syncthreads();  // every thread has read s_rot before it is reset
    if (nrot == 0) break;
    ++used;
  }
  if (tid == 0) rot[sweep] = used > 0 ? used : 1;
}

// After the sweeps: column norms (singular values), descending order (ties by
// index), sigma and the permutation of the leading n_out; diagnostics
// (accumulated over calls by maximum) diag[1] = sweeps that rotated, diag[2] =
// largest |cos| between column pairs seen in the last sweep that ran; diag[3] = k;
// diag[4] = pair-by-pair sweeps that followed a stalled blocked pass.  With G (the
// k x k Gram of the final columns, column-major) the norms are its diagonal.
__global__ __launch_bounds__(kOneWG) void tall_jacobi_finish_kernel(const double* __restrict__ A, int64_t m, int k,
                                                                     int n_out, const int* __restrict__ rot,
                                                                     const double* __restrict__ offmax, int max_sweeps,
                                                                     int fallback_sweeps, const double* __restrict__ G,
                                                                     double* __restrict__ sigma, int* __restrict__ perm,
                                                                     double* __restrict__ diag) {
  __shared__ double nrm[kMaxSubspaceDev];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (G) {  // the Gram of the final columns (a blocked pass that rotated nothing) holds their squared norms
    for (int j = tid; j < k; j += kOneWG) nrm[j] = sqrt(fabs(G[j + (int64_t)j * k]));
  } else {
    for (int j = wave; j < k; j += kOneWG / 64) {
      const double* x = A + (int64_t)j * m;
      double s = 0.0;
      for (int64_t r = lane; r < m; r += 64) s = fma(x[r], x[r], s);
      s = __ockl_wfred_add_f64(s);
      if (lane == 0) nrm[j] = sqrt(s);
    }
  }
  __syncthreads();
  for (int j = tid; j < k; j += kOneWG) {
    int rank = 0;
    for (int l = 0; l < k; ++l) rank += (nrm[l] > nrm[j]) || (nrm[l] == nrm[j] && l < j);
    if (rank < n_out) {
      sigma[rank] = nrm[j];
      perm[rank] = j;
    }
  }
  if (tid == 0 && diag) {
    int used = 0;
    while (used < max_sweeps && rot[used] > 0) ++used;
    const int last = used < max_sweeps ? used : max_sweeps - 1;
    diag[1] = fmax(diag[1], (double)used);
    diag[2] = fmax(diag[2], offmax[last]);
    diag[3] = (double)k;
    diag[4] = fmax(diag[4], (double)fallback_sweeps);
  }
}

// V[:, r] = A[:, perm[r]] / sigma[r] (m rows; zero when sigma[r] = 0) and,
// when J is given, Jp[:, r] = J[:, perm[r]] (k rows), r < n.
__global__ void tall_jacobi_gather_kernel(const double* __restrict__ A, int64_t m, const double* __restrict__ J, int k,
                                          const int* __restrict__ perm, const double* __restrict__ sigma, int n,
                                          double* __restrict__ V, double* __restrict__ Jp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rows = m + k;
  if (e >= rows * n) return;
  const int r = (int)(e / rows);
  const int64_t i = e % rows;
  const int src = perm[r];
  if (i < m) {
    const double sg = sigma[r];
    V[i + (int64_t)r * m] = sg > 0.0 ? A[i + (int64_t)src * m] / sg : 0.0;
  } else if (J) {
    const int64_t ii = i - m;
    Jp[ii + (int64_t)r * k] = J[ii + (int64_t)src * k];
  }
}

// J (k x k, if given) <- identity; rot[0..ns) <- 0, offmax[0..ns) <- 0
__global__ void tall_jacobi_init_kernel(double* J, int k, int* rot, double* offmax, int ns) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J && e < (int64_t)k * k) J[e] = (e % k == e / k) ? 1.0 : 0.0;
  if (e < ns) {
    rot[e] = 0;
    offmax[e] = 0.0;
  }
}

// diag[0] = max_{i < n} ||GY_i - lambda_i Y_i|| / lambda_0: the eigen-residual of
// the Ritz pairs (Y p x n column-major, unit columns; GY = G Y).
__global__ __launch_bounds__(kOneWG) void ritz_residual_kernel(const double* __restrict__ GY,
                                                                const double* __restrict__ Y, int64_t p, int n,
                                                                const double* __restrict__ evals,
                                                                double* __restrict__ diag) {
  __shared__ double red[kOneWG / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double worst = 0.0;
  for (int j = wave; j < n; j += kOneWG / 64) {
    const double lam = evals[j];
    double s = 0.0;
    for (int64_t r = lane; r < p; r += 64) {
      const double d = GY[r + (int64_t)j * p] - lam * Y[r + (int64_t)j * p];
      s = fma(d, d, s);
    }
    s = __ockl_wfred_add_f64(s);
    worst = fmax(worst, sqrt(s));
  }
  worst = block_max(worst, red);
  if (tid == 0) {
    diag[0] = evals[0] > 0.0 ? worst / evals[0] : worst;
    diag[1] = 0.0;
    diag[2] = 0.0;
    diag[4] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// a4: temporal bases.  One workgroup per spatial mode i: Y_i[k, q] = V[q*N_t + k, i]
// (N_t x n_mu) in LDS, one-sided Jacobi SVD, rank cut, DCT-II completion.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTsvdThreads) void temporal_svd_kernel(const double* __restrict__ V, int64_t ldV, int N_t, int n_mu,
                                                           const int32_t* __restrict__ moff, double tau_t,
                                                           double* __restrict__ Phi_t, int32_t* __restrict__ rank_out) {
  extern __shared__ __align__(16) double Ys[];  // N_t * n_mu, then n_mu norms
  constexpr int NWV = kTsvdThreads / 64;
  __shared__ double red[NWV];
  __shared__ int redi[NWV];
  __shared__ int s_rot;
  __shared__ int s_order[64];
  __shared__ double s_coef[512];
  const int i = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c0 = moff[i], nt = moff[i + 1] - c0;
  double* out = Phi_t + (int64_t)c0 * N_t;
  double* nrm = Ys + (int64_t)N_t * n_mu;
  for (int e = tid; e < N_t * n_mu; e += kTsvdThreads) {
    const int k = e % N_t, q = e / N_t;
    Ys[e] = V[(int64_t)q * N_t + k + (int64_t)i * ldV];
  }
  __syncthreads();
  // one-sided Jacobi: orthogonalise the columns pairwise (round-robin order, one pair per wave)
  const int nn = n_mu + (n_mu & 1), m = nn - 1;
  for (int sweep = 0; sweep < 40 && n_mu > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < m; ++rnd) {
      for (int t = wave; t < nn / 2; t += NWV) {
        int a, b;
        if (t == 0) { a = m; b = rnd; } else { a = (rnd + t) % m; b = (rnd - t + m) % m; }
        if (a > b) { const int x = a; a = b; b = x; }
        if (b >= n_mu) continue;
        double* ya = Ys + (int64_t)a * N_t;
        double* yb = Ys + (int64_t)b * N_t;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int k = lane; k < N_t; k += 64) {
          al = fma(ya[k], ya[k], al);
          be = fma(yb[k], yb[k], be);
          ga = fma(ya[k], yb[k], ga);
        }
        al = __ockl_wfred_add_f64(al);
        be = __ockl_wfred_add_f64(be);
        ga = __ockl_wfred_add_f64(ga);
        if (fabs(ga) > 1e-15 * sqrt(al * be) && fabs(ga) > 0.0) {
          const double ze = (be - al) / (2.0 * ga);
          const double tt = (ze >= 0.0 ? 1.0 : -1.0) / (fabs(ze) + sqrt(1.0 + ze * ze));
          const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
          for (int k = lane; k < N_t; k += 64) {
            const double x = ya[k], y = yb[k];
            ya[k] = c * x - s * y;
            yb[k] = s * x + c * y;
          }
          if (lane == 0) s_rot = 1;
        }
      }
      __syncthreads();
    }
    if (!s_rot) break;
    __syncthreads();
  }
  // column norms = singular values; order descending
  for (int q = wave; q < n_mu; q += NWV) {
    double s = 0.0;
    for (int k = lane; k < N_t; k += 64) s = fma(Ys[(int64_t)q * N_t + k], Ys[(int64_t)q * N_t + k], s);
    s = __ockl_wfred_add_f64(s);
    if (lane == 0) nrm[q] = sqrt(s);
  }
  __syncthreads();
  if (tid < n_mu) {
    int rank = 0;
    for (int q = 0; q < n_mu; ++q)
      if (nrm[q] > nrm[tid] || (nrm[q] == nrm[tid] && q < tid)) ++rank;
    s_order[rank] = tid;
  }
  __syncthreads();
  const double s1 = n_mu > 0 ? nrm[s_order[0]] : 0.0;
  int r = 0;
  for (int q = 0; q < n_mu; ++q)
    if (s1 > 0.0 && nrm[q] > tau_t * s1) ++r;
  if (tid == 0 && rank_out) rank_out[i] = r;
  const int keep = min(r, nt);
  int have = 0;
  // data vectors: normalised columns in singular-value order
  for (int j = 0; j < keep; ++j) {
    const int q = s_order[j];
    const double inv = 1.0 / nrm[q];
    for (int k = tid; k < N_t; k += kTsvdThreads) out[(int64_t)j * N_t + k] = Ys[(int64_t)q * N_t + k] * inv;
    have = j + 1;
  }
  __syncthreads();
  // DCT-II completion, classical Gram-Schmidt twice against the kept vectors
  double* cand = Ys;  // reuse LDS: N_t doubles
  for (int mfreq = 0; have < nt && mfreq < N_t; ++mfreq) {
    double c2 = 0.0;
    for (int k = tid; k < N_t; k += kTsvdThreads) {
      const double v = cos(M_PI * (double)mfreq * ((double)k + 0.5) / (double)N_t);
      cand[k] = v;
      c2 = fma(v, v, c2);
    }
    c2 = sqrt(block_sum(c2, red));
    for (int pass = 0; pass < 2 && have > 0; ++pass) {
      for (int l = wave; l < have; l += NWV) {
        double s = 0.0;
        for (int k = lane; k < N_t; k += 64) s = fma(out[(int64_t)l * N_t + k], cand[k], s);
        s = __ockl_wfred_add_f64(s);
        if (lane == 0) s_coef[l] = s;
      }
      __syncthreads();
      for (int k = tid; k < N_t; k += kTsvdThreads) {
        double v = cand[k];
        for (int l = 0; l < have; ++l) v = fma(-s_coef[l], out[(int64_t)l * N_t + k], v);
        cand[k] = v;
      }
      __syncthreads();
    }
    double n2 = 0.0;
    for (int k = tid; k < N_t; k += kTsvdThreads) n2 = fma(cand[k], cand[k], n2);
    n2 = sqrt(block_sum(n2, red));
    if (n2 >= 1e-2 * c2) {
      const double inv = 1.0 / n2;
      for (int k = tid; k < N_t; k += kTsvdThreads) out[(int64_t)have * N_t + k] = cand[k] * inv;
      ++have;
    }
    __syncthreads();
  }
  __syncthreads();
  // sign convention on every column of this mode
  for (int j = 0; j < nt; ++j) {
    double* x = out + (int64_t)j * N_t;
    double mx = 0.0;
    for (int k = tid; k < N_t; k += kTsvdThreads) mx = fmax(mx, fabs(x[k]));
    mx = block_max(mx, red);
    int first = 0x7fffffff;
    for (int k = tid; k < N_t; k += kTsvdThreads)
      if (mx > 0.0 && fabs(x[k]) >= 0.25 * mx) { first = k; break; }
    first = block_min_i(first, redi);
    const bool flip = mx > 0.0 && x[first] < 0.0;
    __syncthreads();
    if (flip)
      for (int k = tid; k < N_t; k += kTsvdThreads) x[k] = -x[k];
    __syncthreads();
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t gram_partial_elems(int64_t K, int p) {
  const int64_t nt = (p + kGT - 1) / kGT;
  const int64_t tiles = nt * (nt + 1) / 2;
  int64_t splits = (1024 + tiles - 1) / tiles;
  const int64_t maxs = (K + 1023) / 1024;
  if (splits > maxs) splits = maxs;
  if (splits < 1) splits = 1;
  return (size_t)splits * p * p;
}

hipError_t launch_gram(int64_t K, int p, const void* X, int in_prec, int64_t ks, int64_t ms, int gram_prec, double* G,
                       double* partial, size_t partial_elems, hipStream_t s) {
  const int64_t nt = (p + kGT - 1) / kGT;
  const int64_t tiles = nt * (nt + 1) / 2;
  const int splits = (int)(gram_partial_elems(K, p) / ((size_t)p * p));
  if ((size_t)splits * p * p > partial_elems) return hipErrorInvalidValue;
  int64_t kps = (K + splits - 1) / splits;
  kps = (kps + kGK - 1) / kGK * kGK;
  dim3 grid((unsigned)tiles, splits);
  if (gram_prec == ST_F64) {
    if (in_prec == ST_F64)
      hipLaunchKernelGGL(gram_f64_kernel<double>, grid, dim3(256), 0, s, K, p, (const double*)X, ks, ms, kps, partial);
    else
      hipLaunchKernelGGL(gram_f64_kernel<float>, grid, dim3(256), 0, s, K, p, (const float*)X, ks, ms, kps, partial);
  } else if (gram_prec == ST_F32) {
    if (in_prec == ST_F64)
      hipLaunchKernelGGL((gram_f32_kernel<double, false>), grid, dim3(256), 0, s, K, p, (const double*)X, ks, ms, kps,
                         partial);
    else
      hipLaunchKernelGGL((gram_f32_kernel<float, false>), grid, dim3(256), 0, s, K, p, (const float*)X, ks, ms, kps,
                         partial);
  } else {
    if (in_prec == ST_F64)
      hipLaunchKernelGGL((gram_f32_kernel<double, true>), grid, dim3(256), 0, s, K, p, (const double*)X, ks, ms, kps,
                         partial);
    else
      hipLaunchKernelGGL((gram_f32_kernel<float, true>), grid, dim3(256), 0, s, K, p, (const float*)X, ks, ms, kps,
                         partial);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t pp = (int64_t)p * p;
  hipLaunchKernelGGL(gram_finish_kernel, dim3((unsigned)((pp + 255) / 256)), dim3(256), 0, s, p, splits, partial, G);
  return hipGetLastError();
}

hipError_t launch_rand_fill(double* X, int64_t p, int k, uint64_t seed, hipStream_t s) {
  const int64_t n = p * k;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(rand_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, p, k, seed);
  return hipGetLastError();
}

// n0sq[c] = ||X[:, c]||^2 (one workgroup per column, fixed summation order); the
// first workgroup also clears *flag.
__global__ __launch_bounds__(256) void col_sumsq_kernel(const double* __restrict__ X, int64_t p,
                                                        double* __restrict__ n0sq, int* __restrict__ flag) {
  __shared__ double red[256 / 64];
  const double* x = X + (int64_t)blockIdx.x * p;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < p; r += 256) acc = fma(x[r], x[r], acc);
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    n0sq[blockIdx.x] = acc;
    if (blockIdx.x == 0) *flag = 0;
  }
}

// Xb[:, c] -= Xp C[:, c] for c < nb (Xb p x nb, Xp p x j0, C j0 x nb, all
// column-major, ld p resp. j0; nb <= kOrthBlock): one thread per row, C in LDS.
__global__ __launch_bounds__(256) void sub_mul_kernel(double* __restrict__ Xb, const double* __restrict__ Xp,
                                                      int64_t p, int j0, int nb, const double* __restrict__ C) {
  extern __shared__ __align__(16) double cs[];
  for (int e = threadIdx.x; e < j0 * nb; e += 256) cs[e] = C[e];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= p) return;
  double acc[kOrthBlock];
#pragma unroll
  for (int c = 0; c < kOrthBlock; ++c) acc[c] = c < nb ? Xb[r + (int64_t)c * p] : 0.0;
  for (int l = 0; l < j0; ++l) {
    const double a = Xp[r + (int64_t)l * p];
#pragma unroll
    for (int c = 0; c < kOrthBlock; ++c) acc[c] = fma(-a, cs[l + c * j0], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < kOrthBlock; ++c)
    if (c < nb) Xb[r + (int64_t)c * p] = acc[c];
}

hipError_t launch_orth(double* X, int64_t p, int k, uint64_t seed, const OrthWork& wk, hipStream_t s) {
  const size_t lds = sizeof(double) * (size_t)p * (size_t)k;
  if (lds <= kOrthMaxLds) {
    if (!g_capturing) {
      const hipError_t e = hipFuncSetAttribute((const void*)orth_cgs2_kernel<true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(orth_cgs2_kernel<true>, dim3(1), dim3(kOneWG), lds, s, X, p, k, seed, nullptr, 0, nullptr);
    return hipGetLastError();
  }
  if (!wk.C || !wk.n0sq || !wk.flag || !wk.part) {
    hipLaunchKernelGGL(orth_cgs2_kernel<false>, dim3(1), dim3(kOneWG), 0, s, X, p, k, seed, nullptr, 0, nullptr);
    return hipGetLastError();
  }
  // Block classical Gram-Schmidt with reorthogonalisation (BCGS2) for columns too
  // long for LDS: per block of kOrthBlock columns, two passes of C = X_prev^T X_blk
  // and X_blk -= X_prev C on the whole device, then the one-workgroup CGS2 inside the
  // block (which tests dependence against the norms before the projections).  A block
  // that needed a pseudo-random refill is projected and orthogonalised again.
  hipError_t e = hipSuccess;
  for (int j0 = 0; j0 < k; j0 += kOrthBlock) {
    const int nb = k - j0 < kOrthBlock ? k - j0 : kOrthBlock;
    double* Xb = X + (int64_t)j0 * p;
    for (int attempt = 0; attempt < 3; ++attempt) {
      hipLaunchKernelGGL(col_sumsq_kernel, dim3(nb), dim3(256), 0, s, Xb, p, wk.n0sq, wk.flag);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      for (int pass = 0; pass < 2 && j0 > 0; ++pass) {
        if ((e = launch_tsgemm(p, j0, nb, X, 1, p, Xb, 1, p, wk.C, j0, wk.part, wk.part_elems, s)) != hipSuccess)
          return e;
        hipLaunchKernelGGL(sub_mul_kernel, dim3((unsigned)((p + 255) / 256)), dim3(256),
                           sizeof(double) * (size_t)j0 * nb, s, Xb, X, p, j0, nb, wk.C);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      hipLaunchKernelGGL(orth_cgs2_kernel<false>, dim3(1), dim3(kOneWG), 0, s, Xb, p, nb, seed, wk.n0sq, j0,
                         wk.flag);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (j0 == 0) break;  // nothing earlier to project against
      int refilled = 0;
      if ((e = hipMemcpyAsync(&refilled, wk.flag, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (!refilled) break;
    }
  }
  return hipSuccess;
}

hipError_t launch_jacobi(int k, double* A, double* Z, double* evals, double* Zout, hipStream_t s) {
  const size_t lds = sizeof(double) * 2 * (size_t)k * (size_t)k;
  if (lds <= kOrthMaxLds) {
    if (!g_capturing) {
      const hipError_t e = hipFuncSetAttribute((const void*)jacobi_eig_kernel<true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(jacobi_eig_kernel<true>, dim3(1), dim3(kOneWG), lds, s, k, A, Z, evals, Zout, 60);
  } else {
    hipLaunchKernelGGL(jacobi_eig_kernel<false>, dim3(1), dim3(kOneWG), 0, s, k, A, Z, evals, Zout, 60);
  }
  return hipGetLastError();
}

hipError_t launch_chol_inv(int n, double* S, double* Rinv, hipStream_t s) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(1), dim3(kOneWG), 0, s, n, S, Rinv);
  return hipGetLastError();
}

hipError_t launch_scale_or_refill(double* X, int64_t p, int k, const double* sigma, double cut, uint64_t seed,
                                  hipStream_t s) {
  const int64_t n = p * k;
  hipLaunchKernelGGL(scale_or_refill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, p, k, sigma, cut,
                     seed);
  return hipGetLastError();
}

hipError_t launch_sqrt_clamp(const double* lam, double* sigma, int n, hipStream_t s) {
  hipLaunchKernelGGL(sqrt_clamp_kernel, dim3((n + 255) / 256), dim3(256), 0, s, lam, sigma, n);
  return hipGetLastError();
}

hipError_t launch_sign_fix(double* X, int64_t p, int k, double* Y, int64_t py, hipStream_t s) {
  hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(256), 0, s, X, p, Y, py);
  return hipGetLastError();
}

hipError_t launch_copy_cols(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int64_t p, int n,
                            hipStream_t s) {
  const int64_t e = p * n;
  if (e == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_cols_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, src, ld_src, dst, ld_dst, p,
                     n);
  return hipGetLastError();
}

hipError_t launch_tall_jacobi(double* A, int64_t m, int k, double* J, int* rot, double* offmax, int max_sweeps,
                              double tol, const TallJacobiWork& wk, int* fallback_sweeps, const double** final_gram,
                              hipStream_t s) {
  if (fallback_sweeps) *fallback_sweeps = 0;
  if (final_gram) *final_gram = nullptr;
  if (k < 1 || k > kMaxSubspaceDev || m < 1) return hipErrorInvalidValue;
  const int64_t init = (int64_t)k * k > max_sweeps ? (int64_t)k * k : max_sweeps;
  hipLaunchKernelGGL(tall_jacobi_init_kernel, dim3((unsigned)((init + 255) / 256)), dim3(256), 0, s, J, k, rot, offmax,
                     max_sweeps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || k < 2) return e;
  const size_t abytes = sizeof(double) * (size_t)m * k;
  if (abytes <= kOrthMaxLds) {
    // the whole matrix in LDS: every sweep in one launch
    if ((e = hipFuncSetAttribute((const void*)tall_jacobi_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)abytes)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(tall_jacobi_lds_kernel, dim3(1), dim3(kOneWG), abytes, s, A, m, k, J, max_sweeps, rot, offmax,
                       tol);
    return hipGetLastError();
  }
  // Longer columns: blocked passes while they converge fast -- G = A^T A (one read of
  // A), its two-sided Jacobi in one workgroup, then A <- A V and J <- J V (one read and
  // one write) -- instead of a sweep's k - 1 rounds that each read and write every
  // column.  A pass that does not cut the largest |cos| at least in half (columns
  // so nearly dependent that the rounding of G limits its rotations) hands over to
  // the pair-by-pair sweeps, which take every inner product from the columns
  // themselves.  After each sweep or pass the host reads its rotation count (a stream
  // synchronisation) and stops once one rotated nothing.
  const int kk = (k + 1) / 2 * 2;
  bool blocked = wk.A2 && wk.G && wk.V && (!J || wk.J2) && m <= 0x7fffffff;
  const bool started_blocked = blocked;
  const size_t glds = sizeof(double) * (size_t)k * k;
  const bool g_in_lds = glds <= kOrthMaxLds;
  if (blocked && g_in_lds &&
      (e = hipFuncSetAttribute((const void*)gram_jacobi_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)glds)) != hipSuccess)
    return e;
  double prev = HUGE_VAL;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int nrot = 0;
    if (blocked) {
      if ((e = launch_tsgemm(m, k, k, A, 1, m, A, 1, m, wk.G, k, wk.part, wk.part_elems, s)) != hipSuccess) return e;
      if (g_in_lds)
        hipLaunchKernelGGL(gram_jacobi_kernel<true>, dim3(1), dim3(kOneWG), glds, s, k, wk.G, wk.V, sw, rot, offmax,
                           tol, kGramInnerEps, kGramInnerSweeps);
      else
        hipLaunchKernelGGL(gram_jacobi_kernel<false>, dim3(1), dim3(kOneWG), 0, s, k, wk.G, wk.V, sw, rot, offmax,
                           tol, kGramInnerEps, kGramInnerSweeps);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      double off = 0.0;
      if ((e = hipMemcpyAsync(&nrot, rot + sw, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(&off, offmax + sw, sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
      if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
      if (nrot == 0) {
        if (final_gram) *final_gram = wk.G;  // G holds the Gram of the final columns (the kernel reads it only)
        break;
      }
      if ((e = launch_mul_small(A, m, k, wk.V, wk.A2, s)) != hipSuccess) return e;
      if ((e = hipMemcpyAsync(A, wk.A2, abytes, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
      if (J) {
        if ((e = launch_mul_small(J, k, k, wk.V, wk.J2, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(J, wk.J2, glds, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
      }
      if (off > 0.5 * prev) blocked = false;
      prev = off;
      continue;
    }
    if (started_blocked && fallback_sweeps) ++*fallback_sweeps;
    for (int r = 0; r < kk - 1; ++r) {
      hipLaunchKernelGGL(tall_jacobi_round_kernel, dim3(kk / 2), dim3(kTallThreads), 0, s, A, m, k, kk, J, r, sw, rot,
                         offmax, tol);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = hipMemcpyAsync(&nrot, rot + sw, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (nrot == 0) break;
  }
  return hipSuccess;
}

hipError_t launch_tall_jacobi_finish(const double* A, int64_t m, int k, const double* J, int n_out, const int* rot,
                                     const double* offmax, int max_sweeps, int fallback_sweeps, const double* G,
                                     double* sigma, int* perm, double* V, double* Jp, double* diag, hipStream_t s) {
  if (k < 1 || k > kMaxSubspaceDev || n_out > k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tall_jacobi_finish_kernel, dim3(1), dim3(kOneWG), 0, s, A, m, k, n_out, rot, offmax, max_sweeps,
                     fallback_sweeps, G, sigma, perm, diag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (m + k) * n_out;
  hipLaunchKernelGGL(tall_jacobi_gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, m, J, k, perm,
                     sigma, n_out, V, Jp);
  return hipGetLastError();
}

hipError_t launch_ritz_residual(const double* GY, const double* Y, int64_t p, int n, const double* evals, double* diag,
                                hipStream_t s) {
  hipLaunchKernelGGL(ritz_residual_kernel, dim3(1), dim3(kOneWG), 0, s, GY, Y, p, n, evals, diag);
  return hipGetLastError();
}

hipError_t launch_temporal_svd(const double* V, int64_t ldV, int N_t, int n_mu, int n_s, const int32_t* moff,
                               double tau_t, double* Phi_t, int32_t* rank_out, hipStream_t s) {
  const size_t lds = sizeof(double) * ((size_t)N_t * n_mu + n_mu);
  hipError_t e = hipFuncSetAttribute((const void*)temporal_svd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(temporal_svd_kernel, dim3(n_s), dim3(kTsvdThreads), lds, s, V, ldV, N_t, n_mu, moff, tau_t, Phi_t,
                     rank_out);
  return hipGetLastError();
}

}  // namespace strom
