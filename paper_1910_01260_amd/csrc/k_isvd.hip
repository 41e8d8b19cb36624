// Incremental SVD of a snapshot stream (Sec. 4.2, Alg. 1 and 2).
//
// The factors W (N_s x r), s (r) and V (k x r) live in device memory and are
// updated in place for each snapshot u by five launches, none of which waits
// on the host:
//   dots   l1 = W^T u                                   (row blocks)
//   sub1   res = u - W l1,  l2 = W^T res                (row blocks)
//   sub2   res -= W l2,  p = ||res||; the last workgroup solves the bordered
//          middle matrix [[diag(s), l1 + l2], [0, p]] (bsvd.h) and writes
//          Uq^T, Vq^T, the new s and the step's decisions (Alg. 1 when the
//          basis is empty; dependence, truncation, rank cap)
//   applyW W <- [W, res/p] Uq  in place by rows; the last workgroup applies
//          the orthogonality test of Alg. 2 to the new first and last columns
//   applyV V <- [[V, 0], [0, 1]] Vq  in place by rows; the last workgroup
//          commits the step and, when the test failed, re-orthonormalises W
//          by classical Gram-Schmidt with re-orthogonalisation (the Q factor
//          with a positive diagonal of R, which is dropped).
// Each reduction across workgroups ends in the last workgroup to arrive (an
// atomic ticket), so no workgroup ever waits for another.
#include "bsvd.h"
#include "internal.h"

extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace strom {
namespace {

constexpr int kIT = 256;           // threads of every kernel here
constexpr int kNW = kIT / 64;      // waves per workgroup
constexpr int kApplyRows = 64;     // rows per workgroup of the factor updates
constexpr int kColPass = 8;        // output columns per lane and pass
constexpr int kMaxN = kIsvdMaxRank + 1;

// state slots (the first seven are documented in the public header)
enum : int {
  S_R = 0, S_K = 1, S_QR = 2, S_DEP = 3, S_TRUNC = 4, S_SKIP = 5, S_REFUSED = 6,
  S_RNEW = 8, S_MODE = 9, S_CTR_A = 10, S_CTR_B = 11, S_CTR_C = 12, S_CTR_E = 13, S_CTR_F = 14, S_ORTH = 15
};
enum : int { M_UPDATE = 0, M_NOOP = 1 };
// scalar slots of the workspace
enum : int { C_P2 = 0, C_INVP = 1, C_PART0 = 2 };

__device__ inline double wave_sum(double v) { return __ockl_wfred_add_f64(v); }

__device__ double block_sum(double v) {
  __shared__ double red[kNW];
  __shared__ double tot;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kNW; ++w) t += red[w];
    tot = t;
  }
  __syncthreads();
  const double r = tot;
  __syncthreads();
  return r;
}

// True (in every thread) in the last workgroup to arrive at `ctr`; that
// workgroup then sees the writes of all the others.  The counter is reset for
// the next launch.
__device__ bool last_to_arrive(int32_t* ctr, int nblocks) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int t = atomicAdd(ctr, 1);
    s_last = (t == nblocks - 1);
    if (s_last) atomicExch(ctr, 0);
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// out[c] = sum over rows [row0, row1) of W[row, c] x[row], c < r (one wave per column)
__device__ void block_dots(const double* __restrict__ W, int64_t ldw, int r, const double* x, int64_t row0,
                           int64_t row1, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < r; c += kNW) {
    const double* wc = W + (int64_t)c * ldw;
    double acc = 0.0;
    for (int64_t i = row0 + lane; i < row1; i += 64) acc = fma(wc[i], x[i], acc);
    acc = wave_sum(acc);
    if (lane == 0) out[c] = acc;
  }
}

// out[c] = sum_b part[b * width + c], c < cols
__device__ void reduce_parts(const double* part, int nb, int width, int cols, double* out) {
  for (int c = threadIdx.x; c < cols; c += kIT) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[(int64_t)b * width + c];
    out[c] = s;
  }
}

// x[row] -= sum_c W[row, c] l[c] over rows [row0, row1) (one thread per row);
// returns this thread's share of the new squared norm
__device__ double subtract_block(const double* __restrict__ W, int64_t ldw, int r, const double* l_lds,
                                 const double* x_in, double* x_out, int64_t row0, int64_t row1) {
  double nn = 0.0;
  for (int64_t i = row0 + threadIdx.x; i < row1; i += kIT) {
    double v = x_in[i];
    for (int c = 0; c < r; ++c) v = fma(-W[i + (int64_t)c * ldw], l_lds[c], v);
    x_out[i] = v;
    nn = fma(v, v, nn);
  }
  return nn;
}

__global__ __launch_bounds__(kIT) void isvd_dots_kernel(const double* __restrict__ W, int64_t N_s, int64_t rows_pb,
                                                        const double* __restrict__ u, int32_t* state, double* part,
                                                        int width, double* l1) {
  const int r = state[S_R];
  const int64_t row0 = (int64_t)blockIdx.x * rows_pb, row1 = min(row0 + rows_pb, N_s);
  block_dots(W, N_s, r, u, row0, row1, part + (int64_t)blockIdx.x * width);
  if (last_to_arrive(state + S_CTR_A, gridDim.x)) reduce_parts(part, gridDim.x, width, r, l1);
}

__global__ __launch_bounds__(kIT) void isvd_sub1_kernel(const double* __restrict__ W, int64_t N_s, int64_t rows_pb,
                                                        const double* __restrict__ u, int32_t* state,
                                                        const double* l1, double* res, double* part, int width,
                                                        double* l2) {
  __shared__ double sl[kIsvdMaxRank];
  const int r = state[S_R];
  for (int c = threadIdx.x; c < r; c += kIT) sl[c] = l1[c];
  __syncthreads();
  const int64_t row0 = (int64_t)blockIdx.x * rows_pb, row1 = min(row0 + rows_pb, N_s);
  subtract_block(W, N_s, r, sl, u, res, row0, row1);
  __syncthreads();
  block_dots(W, N_s, r, res, row0, row1, part + (int64_t)blockIdx.x * width);
  if (last_to_arrive(state + S_CTR_B, gridDim.x)) reduce_parts(part, gridDim.x, width, r, l2);
}

// The step's decisions and the SVD of the middle matrix, in one workgroup.
__device__ void bordered_step(int r, int r_max, int64_t m_max, double eps_svd, double eps_sv, double p2,
                              const double* l1, const double* l2, double* s, double* UqT, double* VqT, int ldq,
                              double* scal, int32_t* state) {
  __shared__ double d[kMaxN], z[kMaxN], zh[kMaxN], tau[kMaxN], sg[kMaxN];
  __shared__ double rc[kIsvdMaxRank], rs[kIsvdMaxRank];
  __shared__ int act[kMaxN], org[kMaxN], pos[kMaxN], ri[kIsvdMaxRank], rj[kIsvdMaxRank];
  __shared__ int s_na, s_nrot, s_pact, s_go, s_keep;
  const int tid = threadIdx.x;
  const double p = sqrt(p2);
  const int64_t k = state[S_K];
  for (int t = tid; t < r; t += kIT) {
    d[t] = s[t];
    z[t] = l1[t] + l2[t];
  }
  for (int t = tid; t <= r; t += kIT) pos[t] = -1;
  __syncthreads();
  bsvd::Problem P{r, d, z, act, 0, ri, rj, rc, rs, 0, false};
  if (tid == 0) {
    s_go = 0;
    if (k >= m_max) {
      state[S_MODE] = M_NOOP;
      state[S_RNEW] = r;
    } else if (r == 0) {
      // Alg. 1: the first snapshot whose norm exceeds eps_svd starts the basis
      state[S_MODE] = M_UPDATE;
      if (p > eps_svd) {
        UqT[0] = 1.0;
        VqT[0] = 1.0;
        s[0] = p;
        scal[C_INVP] = 1.0 / p;
        state[S_RNEW] = 1;
      } else {
        scal[C_INVP] = 0.0;
        state[S_RNEW] = 0;
        state[S_SKIP] += 1;
      }
    } else {
      state[S_MODE] = M_UPDATE;
      d[r] = 0.0;
      z[r] = p;
      bsvd::deflate(P, !(p >= eps_svd));
      s_na = P.na;
      s_nrot = P.nrot;
      s_pact = P.p_active ? 1 : 0;
      s_go = 1;
    }
  }
  __syncthreads();
  if (!s_go) return;
  P.na = s_na;
  P.nrot = s_nrot;
  P.p_active = s_pact != 0;
  for (int q = tid; q < P.na; q += kIT) {
    bsvd::root(P, q, org[q], tau[q]);
    pos[act[q]] = q;
  }
  for (int t = tid; t <= r; t += kIT) zh[t] = 0.0;
  __syncthreads();
  for (int q = tid; q < P.na; q += kIT) zh[act[q]] = bsvd::zhat(P, q, org, tau);
  const int ncand = P.p_active ? r + 1 : r;
  for (int t = tid; t < ncand; t += kIT) sg[t] = bsvd::cand_sigma(P, pos, org, tau, t);
  __syncthreads();
  if (tid == 0) {
    double mn = sg[0];
    for (int t = 1; t < ncand; ++t) mn = fmin(mn, sg[t]);
    int keep = ncand;
    if (keep > 0 && mn < eps_sv) --keep;
    if (keep > r_max) keep = r_max;
    if (keep < ncand) state[S_TRUNC] += 1;
    if (!P.p_active) state[S_DEP] += 1;
    s_keep = keep;
    state[S_RNEW] = keep;
    scal[C_INVP] = P.p_active ? 1.0 / p : 0.0;
  }
  __syncthreads();
  const int keep = s_keep;
  for (int t = tid; t < ncand; t += kIT) {
    const int c = bsvd::cand_rank(sg, ncand, t);
    if (c >= keep) continue;
    bsvd::fill_column(P, zh, pos, org, tau, t, UqT + c, VqT + c, ldq);
    s[c] = sg[t];
  }
}

__global__ __launch_bounds__(kIT) void isvd_sub2_kernel(const double* __restrict__ W, int64_t N_s, int64_t rows_pb,
                                                        int32_t* state, const double* l1, const double* l2,
                                                        double* res, double* part, int width, double* scal,
                                                        double* s, double* UqT, double* VqT, int r_max,
                                                        int64_t m_max, double eps_svd, double eps_sv) {
  __shared__ double sl[kIsvdMaxRank];
  const int r = state[S_R];
  for (int c = threadIdx.x; c < r; c += kIT) sl[c] = l2[c];
  __syncthreads();
  const int64_t row0 = (int64_t)blockIdx.x * rows_pb, row1 = min(row0 + rows_pb, N_s);
  const double nn = block_sum(subtract_block(W, N_s, r, sl, res, res, row0, row1));
  if (threadIdx.x == 0) part[(int64_t)blockIdx.x * width] = nn;
  if (!last_to_arrive(state + S_CTR_C, gridDim.x)) return;
  double p2 = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kIT) p2 += part[(int64_t)b * width];
  p2 = block_sum(p2);
  if (threadIdx.x == 0) scal[C_P2] = p2;
  bordered_step(r, r_max, m_max, eps_svd, eps_sv, p2, l1, l2, s, UqT, VqT, r_max + 1, scal, state);
}

// X[row, 0:rnew] <- [X[row, 0:r], extra(row)] M over rows [row0, row1), in
// place (every row is read into LDS before any is written).  MT holds M^T
// row by row: MT[j * ldq + c] = M[j, c].
template <typename Extra>
__device__ void apply_rows(double* __restrict__ X, int64_t ldx, int64_t row0, int64_t row1, int r, int rnew,
                           const double* __restrict__ MT, int ldq, Extra extra, double* tile) {
  const int tid = threadIdx.x;
  const int n_in = r + 1;
  for (int e = tid; e < n_in * kApplyRows; e += kIT) {
    const int j = e / kApplyRows, i = e % kApplyRows;
    const int64_t row = row0 + i;
    double v = 0.0;
    if (row < row1) v = j < r ? X[row + (int64_t)j * ldx] : extra(row);
    tile[e] = v;
  }
  __syncthreads();
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t row = row0 + lane;
  for (int cb = wave * kColPass; cb < rnew; cb += kNW * kColPass) {
    const int cbu = __builtin_amdgcn_readfirstlane(cb);
    double acc[kColPass];
#pragma unroll
    for (int q = 0; q < kColPass; ++q) acc[q] = 0.0;
    for (int j = 0; j < n_in; ++j) {
      const double t = tile[j * kApplyRows + lane];
      const double* m = MT + (int64_t)j * ldq + cbu;
#pragma unroll
      for (int q = 0; q < kColPass; ++q) acc[q] = fma(t, m[q], acc[q]);
    }
    if (row < row1) {
#pragma unroll
      for (int q = 0; q < kColPass; ++q)
        if (cbu + q < rnew) X[row + (int64_t)(cbu + q) * ldx] = acc[q];
    }
  }
}

__global__ __launch_bounds__(kIT) void isvd_apply_w_kernel(double* __restrict__ W, int64_t N_s, int32_t* state,
                                                           const double* __restrict__ res,
                                                           const double* __restrict__ scal,
                                                           const double* __restrict__ UqT, int ldq, double* part,
                                                           double orth_tol) {
  extern __shared__ __align__(16) double tile[];
  const int r = state[S_R], rnew = state[S_RNEW];
  const bool noop = state[S_MODE] == M_NOOP;
  const int64_t row0 = (int64_t)blockIdx.x * kApplyRows, row1 = min(row0 + kApplyRows, N_s);
  if (!noop && rnew > 0) {
    const double invp = scal[C_INVP];
    apply_rows(W, N_s, row0, row1, r, rnew, UqT, ldq, [&](int64_t row) { return res[row] * invp; }, tile);
  }
  __syncthreads();
  // partial of the orthogonality test of Alg. 2: W(:,1)^T W(:,end)
  double v = 0.0;
  if (!noop && rnew > 1 && threadIdx.x < kApplyRows) {
    const int64_t row = row0 + threadIdx.x;
    if (row < row1) v = W[row] * W[row + (int64_t)(rnew - 1) * N_s];
  }
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
  if (!last_to_arrive(state + S_CTR_E, gridDim.x)) return;
  double t = 0.0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += kIT) t += part[b];
  t = block_sum(t);
  if (threadIdx.x == 0) state[S_ORTH] = (!noop && rnew > 1 && fabs(t) > orth_tol) ? 1 : 0;
}

// Q factor of W (N_s x n) with a positive diagonal of R, in place: classical
// Gram-Schmidt, each column projected twice against the finished ones.
__device__ void orthonormalise(double* __restrict__ W, int64_t N_s, int n) {
  __shared__ double coef[kIsvdMaxRank];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = 0; j < n; ++j) {
    double* wj = W + (int64_t)j * N_s;
    for (int pass = 0; pass < 2; ++pass) {
      for (int i = wave; i < j; i += kNW) {
        const double* wi = W + (int64_t)i * N_s;
        double a = 0.0;
        for (int64_t q = lane; q < N_s; q += 64) a = fma(wi[q], wj[q], a);
        a = wave_sum(a);
        if (lane == 0) coef[i] = a;
      }
      __threadfence_block();
      __syncthreads();
      for (int64_t q = threadIdx.x; q < N_s; q += kIT) {
        double v = wj[q];
        for (int i = 0; i < j; ++i) v = fma(-coef[i], W[q + (int64_t)i * N_s], v);
        wj[q] = v;
      }
      __threadfence_block();
      __syncthreads();
    }
    double nn = 0.0;
    for (int64_t q = threadIdx.x; q < N_s; q += kIT) nn = fma(wj[q], wj[q], nn);
    nn = block_sum(nn);
    const double inv = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for (int64_t q = threadIdx.x; q < N_s; q += kIT) wj[q] *= inv;
    __threadfence_block();
    __syncthreads();
  }
}

__global__ __launch_bounds__(kIT) void isvd_apply_v_kernel(double* __restrict__ V, int64_t m_max, int32_t* state,
                                                           const double* __restrict__ VqT, int ldq,
                                                           double* __restrict__ W, int64_t N_s) {
  extern __shared__ __align__(16) double tile[];
  const int r = state[S_R], rnew = state[S_RNEW];
  const bool noop = state[S_MODE] == M_NOOP;
  const int64_t k = state[S_K];
  const int64_t row0 = (int64_t)blockIdx.x * kApplyRows, row1 = min(row0 + kApplyRows, k + 1);
  if (!noop && rnew > 0 && row0 < row1)
    apply_rows(V, m_max, row0, row1, r, rnew, VqT, ldq, [&](int64_t row) { return row == k ? 1.0 : 0.0; }, tile);
  if (!last_to_arrive(state + S_CTR_F, gridDim.x)) return;
  if (noop) {
    if (threadIdx.x == 0) state[S_REFUSED] += 1;
    return;
  }
  if (state[S_ORTH]) orthonormalise(W, N_s, rnew);
  if (threadIdx.x == 0) {
    if (state[S_ORTH]) state[S_QR] += 1;
    state[S_ORTH] = 0;
    state[S_R] = rnew;
    state[S_K] = (int32_t)(k + 1);
  }
}

__global__ void isvd_reset_kernel(int32_t* state) {
  if (threadIdx.x < kIsvdStateInts) state[threadIdx.x] = 0;
}

}  // namespace

int64_t isvd_rows_per_block(int64_t N_s) {
  // row blocks of 512 rows, fewer and longer past 1024 blocks so the final
  // reductions stay short
  int64_t rpb = 512;
  const int64_t nb = (N_s + rpb - 1) / rpb;
  if (nb > 1024) rpb = ((N_s + 1023) / 1024 + 63) / 64 * 64;
  return rpb;
}

int isvd_row_blocks(int64_t N_s) {
  const int64_t rpb = isvd_rows_per_block(N_s);
  return (int)((N_s + rpb - 1) / rpb);
}

size_t isvd_apply_lds_bytes(int r_max) { return sizeof(double) * (size_t)(r_max + 1) * kApplyRows; }

hipError_t launch_isvd_reset(int32_t* state, hipStream_t s) {
  hipLaunchKernelGGL(isvd_reset_kernel, dim3(1), dim3(64), 0, s, state);
  return hipGetLastError();
}

hipError_t launch_isvd_step(const IsvdArgs& a, const double* u, hipStream_t s) {
  const int64_t rpb = isvd_rows_per_block(a.N_s);
  const int G = isvd_row_blocks(a.N_s);
  const int width = a.r_max + 1, ldq = a.r_max + 1;
  const size_t lds = isvd_apply_lds_bytes(a.r_max);
  if (lds > 64 * 1024 && !g_capturing) {
    hipError_t e = hipFuncSetAttribute((const void*)isvd_apply_w_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)isvd_apply_v_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(isvd_dots_kernel, dim3(G), dim3(kIT), 0, s, a.W, a.N_s, rpb, u, a.state, a.part, width, a.l1);
  hipLaunchKernelGGL(isvd_sub1_kernel, dim3(G), dim3(kIT), 0, s, a.W, a.N_s, rpb, u, a.state, a.l1, a.res, a.part,
                     width, a.l2);
  hipLaunchKernelGGL(isvd_sub2_kernel, dim3(G), dim3(kIT), 0, s, a.W, a.N_s, rpb, a.state, a.l1, a.l2, a.res,
                     a.part, width, a.scal, a.s, a.UqT, a.VqT, a.r_max, a.m_max, a.eps_svd, a.eps_sv);
  const int GW = (int)((a.N_s + kApplyRows - 1) / kApplyRows);
  const double orth_tol = fmin(a.eps_svd, bsvd::kEps * (double)a.N_s);
  hipLaunchKernelGGL(isvd_apply_w_kernel, dim3(GW), dim3(kIT), lds, s, a.W, a.N_s, a.state, a.res, a.scal, a.UqT,
                     ldq, a.part, orth_tol);
  const int GV = (int)((a.m_max + kApplyRows - 1) / kApplyRows);
  hipLaunchKernelGGL(isvd_apply_v_kernel, dim3(GV), dim3(kIT), lds, s, a.V, a.m_max, a.state, a.VqT, ldq, a.W,
                     a.N_s);
  return hipGetLastError();
}

}  // namespace strom
