// Incremental SVD of a snapshot stream (Sec. 4.2, Alg. 1 and 2).
//
// The factors W (N_s x r), s (r) and V (k x r) live in device memory and are
// updated in place for each snapshot u, with no host synchronisation:
//   front   l1 = W^T u, res = u - W l1, l2 = W^T res, res -= W l2 (two
//           Gram-Schmidt passes), p = ||res||; then, in one workgroup, the
//           step's decisions (Alg. 1 when the basis is empty; dependence,
//           truncation, rank cap) and the SVD of the bordered middle matrix
//           [[diag(s), l1 + l2], [0, p]] (bsvd.h), which writes Uq^T, Vq^T
//           and the new s.  Snapshots up to kFrontRows long take one
//           workgroup for all of it; longer ones take row-block launches
//           whose partials are summed by launches of their own.
//   applyW  W <- [W, res/p] Uq in place by rows, with the partials of the
//           orthogonality test of Alg. 2 (new first column against new last)
//   applyV  V <- [[V, 0], [0, 1]] Vq in place by rows
//   commit  the test; when it fails W is re-orthonormalised by classical
//           Gram-Schmidt with re-orthogonalisation (the Q factor with a
//           positive diagonal of R, which is dropped); the new rank and count.
// Workgroups never wait for one another: every cross-workgroup sum ends a
// launch and is read by the next.
#include "bsvd.h"
#include "internal.h"

extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace strom {
namespace {

constexpr int kIT = 256;           // threads of every kernel here
constexpr int kNW = kIT / 64;      // waves per workgroup
constexpr int kApplyRows = 64;     // rows per workgroup of the factor updates
constexpr int kColPass = 8;        // output columns per lane and pass
constexpr int kStageElems = 8192;  // rows of M^T staged in LDS by the factor updates (doubles)
constexpr int kStageMaxGrid = 256; // ... when their grid has at most this many workgroups (one per CU)
constexpr size_t kApplyLdsMax = 156 * 1024;  // dynamic LDS of the apply kernels (their static LDS comes on top)
constexpr int kMaxN = kIsvdMaxRank + 1;
constexpr int kGrp = 8;  // lanes per column in the norms of the bordered SVD's vectors
constexpr int64_t kFrontRows = 4096;  // snapshots up to this length take the one-workgroup front

// state slots (the first seven are documented in the public header)
enum : int {
  S_R = 0, S_K = 1, S_QR = 2, S_DEP = 3, S_TRUNC = 4, S_SKIP = 5, S_REFUSED = 6,
  S_RNEW = 8, S_MODE = 9
};
enum : int { M_UPDATE = 0, M_NOOP = 1 };
// scalar slots of the workspace
enum : int { C_P2 = 0, C_INVP = 1, C_PART0 = 2 };

__device__ inline double wave_sum(double v) { return __ockl_wfred_add_f64(v); }

// Sums three values over a group of L lanes; every lane of the group gets
// lane 0's result, so the group takes identical decisions.
template <int L>
struct GroupSum {
  __device__ void operator()(double& a, double& b, double& c) const {
    if constexpr (L > 1) {
#pragma unroll
      for (int m = L / 2; m >= 1; m >>= 1) {
        a += __shfl_xor(a, m, L);
        b += __shfl_xor(b, m, L);
        c += __shfl_xor(c, m, L);
      }
      a = __shfl(a, 0, L);
      b = __shfl(b, 0, L);
      c = __shfl(c, 0, L);
    }
  }
};

template <int NT = kIT>
__device__ double block_sum(double v) {
  constexpr int NW = NT / 64;
  __shared__ double red[NW];
  __shared__ double tot;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += red[w];
    tot = t;
  }
  __syncthreads();
  const double r = tot;
  __syncthreads();
  return r;
}

// out[c * ostride] = sum over rows [row0, row1) of W[row, c] x[row], c < r
// (one wave per column)
__device__ void block_dots(const double* __restrict__ W, int64_t ldw, int r, const double* x, int64_t row0,
                           int64_t row1, double* out, int64_t ostride) {
  constexpr int CB = 4;  // columns per wave and pass: their loads are in flight together
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c0 = wave * CB; c0 < r; c0 += kNW * CB) {
    double acc[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[q] = 0.0;
    for (int64_t i = row0 + lane; i < row1; i += 64) {
      const double xi = x[i];
#pragma unroll
      for (int q = 0; q < CB; ++q)
        if (c0 + q < r) acc[q] = fma(W[i + (int64_t)(c0 + q) * ldw], xi, acc[q]);
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      const double v = wave_sum(acc[q]);
      if (lane == 0 && c0 + q < r) out[(c0 + q) * ostride] = v;
    }
  }
}

// out[c] = sum_b part[c * nb + b], c < cols (one wave per column, lanes over
// the workgroups' partials, always summed in the same order; several loads
// in flight per lane)
template <int NT>
__device__ void reduce_parts(const double* part, int nb, int cols, double* out) {
  constexpr int U = 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < cols; c += NT / 64) {
    const double* pc = part + (int64_t)c * nb;
    double s[U];
#pragma unroll
    for (int q = 0; q < U; ++q) s[q] = 0.0;
    for (int b0 = 0; b0 < nb; b0 += 64 * U) {
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int b = b0 + q * 64 + lane;
        if (b < nb) s[q] += pc[b];
      }
    }
    const double v = wave_sum((s[0] + s[1]) + (s[2] + s[3]));
    if (lane == 0) out[c] = v;
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

// Partials of l1 = W^T u over the workgroup's rows: part[c * G + b].
__global__ __launch_bounds__(kIT) void isvd_dots_kernel(const double* __restrict__ W, int64_t N_s, int64_t rows_pb,
                                                        const double* __restrict__ u, const int32_t* state,
                                                        double* part) {
  const int r = state[S_R];
  const int64_t row0 = (int64_t)blockIdx.x * rows_pb, row1 = min(row0 + rows_pb, N_s);
  block_dots(W, N_s, r, u, row0, row1, part + blockIdx.x, gridDim.x);
}

// out[c] = sum of the G partials of column c, c < r (one workgroup)
constexpr int kRT = 1024;
__global__ __launch_bounds__(kRT) void isvd_reduce_kernel(const double* part, int G, const int32_t* state,
                                                          double* out) {
  reduce_parts<kRT>(part, G, state[S_R], out);
}

// res = u - W l1 over the workgroup's rows, and the partials of l2 = W^T res.
__global__ __launch_bounds__(kIT) void isvd_sub1_kernel(const double* __restrict__ W, int64_t N_s, int64_t rows_pb,
                                                        const double* __restrict__ u, const int32_t* state,
                                                        const double* l1, double* res, double* part) {
  __shared__ double sl[kIsvdMaxRank];
  const int r = state[S_R];
  for (int c = threadIdx.x; c < r; c += kIT) sl[c] = l1[c];
  __syncthreads();
  const int64_t row0 = (int64_t)blockIdx.x * rows_pb, row1 = min(row0 + rows_pb, N_s);
  subtract_block(W, N_s, r, sl, u, res, row0, row1);
  __syncthreads();
  block_dots(W, N_s, r, res, row0, row1, part + blockIdx.x, gridDim.x);
}

// bsvd::deflate spread over the workgroup (same result): the small-z test is
// independent per coordinate, the serial rotation loop runs only when two
// consecutive active coordinates are within tol, and wave 0 compacts the
// active set with ballots.
template <int NT>
__device__ void deflate_block(bsvd::Problem& P, bool dependent, int* s_na, int* s_nrot, int* s_pact) {
  __shared__ int s_close;
  __shared__ double s_tol;
  const int tid = threadIdx.x, r = P.r;
  double zz = 0.0;
  for (int t = tid; t <= r; t += NT) zz += P.z[t] * P.z[t];
  zz = block_sum<NT>(zz);
  if (tid == 0) {
    const double dmax = r > 0 ? P.d[0] : 0.0;
    s_tol = 8.0 * bsvd::kEps * fmax(dmax, sqrt(zz));
    s_close = 0;
  }
  __syncthreads();
  const double tol = s_tol;
  for (int t = tid; t <= r; t += NT)
    if ((t == r && dependent) || fabs(P.z[t]) <= tol) P.z[t] = 0.0;
  __syncthreads();
  for (int t = tid; t < r; t += NT) {
    if (P.z[t] == 0.0) continue;
    int u = t - 1;
    while (u >= 0 && P.z[u] == 0.0) --u;
    if (u >= 0 && P.d[u] - P.d[t] <= tol) s_close = 1;
  }
  __syncthreads();
  if (tid == 0) {
    P.nrot = 0;
    if (s_close) {
      int k0 = -1;
      for (int t = 0; t < r; ++t) {
        if (P.z[t] == 0.0) continue;
        if (k0 >= 0 && P.d[k0] - P.d[t] <= tol) {
          const double rho = hypot(P.z[k0], P.z[t]);
          P.rot_i[P.nrot] = k0;
          P.rot_j[P.nrot] = t;
          P.rot_c[P.nrot] = P.z[k0] / rho;
          P.rot_s[P.nrot] = P.z[t] / rho;
          ++P.nrot;
          P.z[k0] = rho;
          P.z[t] = 0.0;
          P.d[t] = P.d[k0];
        } else {
          k0 = t;
        }
      }
    }
    *s_nrot = P.nrot;
    *s_pact = P.z[r] != 0.0 ? 1 : 0;
  }
  __syncthreads();
  if (tid < 64) {
    int base = 0;
    for (int c0 = 0; c0 <= r; c0 += 64) {
      const int t = c0 + tid;
      const bool on = t <= r && P.z[t] != 0.0;
      const uint64_t m = __ballot(on);
      if (on) {
        const int k = base + __popcll(m & ((1ull << tid) - 1ull));
        P.act[k] = t;
        P.da[k] = P.d[t];
        P.za[k] = P.z[t];
      }
      base += __popcll(m);
    }
    if (tid == 0) *s_na = base;
  }
  __syncthreads();
}

// Every root of the active problem, a group of L lanes per root.
template <int L, int NT>
__device__ void roots_phase(const bsvd::Problem& P, double* org, double* tau, int* pos) {
  const int grp = threadIdx.x / L, gl = threadIdx.x % L;
  for (int q = grp; q < P.na; q += NT / L) {
    double o, tv;
    bsvd::root_group(P, q, gl, L, GroupSum<L>{}, o, tv);
    if (gl == 0) {
      org[q] = o;
      tau[q] = tv;
      pos[P.act[q]] = q;
    }
  }
}

// The step's decisions and the SVD of the middle matrix, in one workgroup of NT threads.
template <int NT>
__device__ void bordered_step(int r, int r_max, int64_t m_max, double eps_svd, double eps_sv, double p2,
                              const double* l1, const double* l2, double* s, double* UqT, double* VqT, int ldq,
                              double* scal, int32_t* state) {
  __shared__ double d[kMaxN], z[kMaxN], zh[kMaxN], tau[kMaxN], org[kMaxN], sg[kMaxN], da[kMaxN], za[kMaxN];
  __shared__ double rc[kIsvdMaxRank], rs[kIsvdMaxRank], inu[kMaxN], inv[kMaxN];
  __shared__ int act[kMaxN], pos[kMaxN], ri[kIsvdMaxRank], rj[kIsvdMaxRank], colsrc[kMaxN];
  __shared__ int s_na, s_nrot, s_pact, s_go, s_keep;
  const int tid = threadIdx.x;
  const double p = sqrt(p2);
  const int64_t k = state[S_K];
  for (int t = tid; t < r; t += NT) {
    d[t] = s[t];
    z[t] = l1[t] + l2[t];
  }
  for (int t = tid; t <= r; t += NT) pos[t] = -1;
  __syncthreads();
  bsvd::Problem P{r, d, z, act, 0, da, za, ri, rj, rc, rs, 0, false};
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
      s_go = 1;
    }
  }
  __syncthreads();
  if (!s_go) return;
  deflate_block<NT>(P, !(p >= eps_svd), &s_na, &s_nrot, &s_pact);
  P.na = s_na;
  P.nrot = s_nrot;
  P.p_active = s_pact != 0;
  const int n = r + 1;
  // roots: a group of lanes per root splits the secular sums; the group is
  // as wide as the workgroup allows with every root in one pass
  if (P.na * 32 <= NT)
    roots_phase<32, NT>(P, org, tau, pos);
  else if (P.na * 16 <= NT)
    roots_phase<16, NT>(P, org, tau, pos);
  else if (P.na * 8 <= NT)
    roots_phase<8, NT>(P, org, tau, pos);
  else if (P.na * 4 <= NT)
    roots_phase<4, NT>(P, org, tau, pos);
  else if (P.na * 2 <= NT)
    roots_phase<2, NT>(P, org, tau, pos);
  else
    roots_phase<1, NT>(P, org, tau, pos);
  for (int t = tid; t <= r; t += NT) zh[t] = 0.0;
  __syncthreads();
  for (int q = tid; q < P.na; q += NT) zh[act[q]] = bsvd::zhat(P, q, org, tau);
  const int ncand = P.p_active ? r + 1 : r;
  for (int t = tid; t < ncand; t += NT) sg[t] = bsvd::cand_sigma(P, pos, org, tau, t);
  __syncthreads();
  // output column c (descending singular values) comes from candidate colsrc[c]
  for (int t = tid; t < ncand; t += NT) colsrc[bsvd::cand_rank(sg, ncand, t)] = t;
  __syncthreads();
  if (tid == 0) {
    const double mn = ncand > 0 ? sg[colsrc[ncand - 1]] : 0.0;
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
  for (int c = tid; c < keep; c += NT) s[c] = sg[colsrc[c]];
  // norms of the unnormalised vectors, a group of kGrp lanes per column
  const int grp = tid / kGrp, gl = tid % kGrp;
  for (int c = grp; c < keep; c += NT / kGrp) {
    const int t = colsrc[c];
    double nu = 1.0, nv = 1.0, w = 0.0;
    if (pos[t] >= 0) {
      const int k = pos[t];
      nu = 0.0;
      nv = 0.0;
      for (int q = gl; q < n; q += kGrp) {
        double a, b;
        bsvd::vec_entry(P, zh, org[k], tau[k], q, a, b);
        nu += a * a;
        nv += b * b;
      }
      GroupSum<kGrp>{}(nu, nv, w);
    }
    if (gl == 0) {
      inu[c] = 1.0 / sqrt(nu);
      inv[c] = 1.0 / sqrt(nv);
    }
  }
  __syncthreads();
  // the entries, consecutive threads on consecutive columns of a row of U_q^T / V_q^T
  for (int e = tid; e < keep * n; e += NT) {
    const int q = e / keep, c = e - q * keep;
    const int t = colsrc[c];
    double a, b;
    if (pos[t] < 0) {
      a = b = (q == t) ? 1.0 : 0.0;
    } else {
      const int k = pos[t];
      bsvd::vec_entry(P, zh, org[k], tau[k], q, a, b);
      a *= inu[c];
      b *= inv[c];
    }
    UqT[(int64_t)q * ldq + c] = a;
    VqT[(int64_t)q * ldq + c] = b;
  }
  if (P.nrot > 0) {
    // undo the deflation rotations, one thread per column
    __threadfence_block();
    __syncthreads();
    for (int c = tid; c < keep; c += NT) {
      bsvd::unrotate(P, UqT + c, ldq);
      bsvd::unrotate(P, VqT + c, ldq);
    }
  }
}

// res -= W l2 over the workgroup's rows; partial of ||res||^2 in part[b].
__global__ __launch_bounds__(kIT) void isvd_sub2_kernel(const double* __restrict__ W, int64_t N_s, int64_t rows_pb,
                                                        const int32_t* state, const double* l2, double* res,
                                                        double* part) {
  __shared__ double sl[kIsvdMaxRank];
  const int r = state[S_R];
  for (int c = threadIdx.x; c < r; c += kIT) sl[c] = l2[c];
  __syncthreads();
  const int64_t row0 = (int64_t)blockIdx.x * rows_pb, row1 = min(row0 + rows_pb, N_s);
  const double nn = block_sum(subtract_block(W, N_s, r, sl, res, res, row0, row1));
  if (threadIdx.x == 0) part[blockIdx.x] = nn;
}

// p = ||res|| from the partials, then the step's decisions and the bordered SVD (one workgroup).
constexpr int kSvdThreads = 1024;  // the bordered SVD alone: more lanes per root and per vector
__global__ __launch_bounds__(kSvdThreads) void isvd_svd_kernel(const double* part, int G, int32_t* state, const double* l1,
                                                       const double* l2, double* scal, double* s, double* UqT,
                                                       double* VqT, int r_max, int64_t m_max, double eps_svd,
                                                       double eps_sv) {
  double p2 = 0.0;
  for (int b = threadIdx.x; b < G; b += kSvdThreads) p2 += part[b];
  p2 = block_sum<kSvdThreads>(p2);
  if (threadIdx.x == 0) scal[C_P2] = p2;
  bordered_step<kSvdThreads>(state[S_R], r_max, m_max, eps_svd, eps_sv, p2, l1, l2, s, UqT, VqT, r_max + 1, scal,
                             state);
}

// The whole front of a step for a short snapshot (N_s up to kFrontRows), in
// one workgroup: l1 = W^T u, res = u - W l1, l2 = W^T res, res -= W l2,
// p = ||res||, then the bordered SVD.
__global__ __launch_bounds__(kIT) void isvd_front_kernel(const double* __restrict__ W, int64_t N_s,
                                                         const double* __restrict__ u, int32_t* state, double* res,
                                                         double* scal, double* s, double* UqT, double* VqT, int r_max,
                                                         int64_t m_max, double eps_svd, double eps_sv) {
  __shared__ double l1[kIsvdMaxRank], l2[kIsvdMaxRank];
  const int r = state[S_R];
  block_dots(W, N_s, r, u, 0, N_s, l1, 1);
  __syncthreads();
  subtract_block(W, N_s, r, l1, u, res, 0, N_s);
  __syncthreads();
  block_dots(W, N_s, r, res, 0, N_s, l2, 1);
  __syncthreads();
  const double p2 = block_sum(subtract_block(W, N_s, r, l2, res, res, 0, N_s));
  if (threadIdx.x == 0) scal[C_P2] = p2;
  bordered_step<kIT>(r, r_max, m_max, eps_svd, eps_sv, p2, l1, l2, s, UqT, VqT, r_max + 1, scal, state);
}

// X[row, 0:rnew] <- [X[row, 0:r], extra(row)] M over rows [row0, row1), in
// place (every row is read into LDS before any is written).  MT holds M^T
// row by row: MT[j * ldq + c] = M[j, c].  With STAGED the rows of MT are first
// copied into LDS (mts, row stride ldm = rnew rounded up to kColPass, zero
// padded) and read from there as broadcasts; otherwise every lane reads them
// through the scalar cache, whose misses then stall each step of the product.
template <bool STAGED, typename Extra>
__device__ void apply_rows(double* __restrict__ X, int64_t ldx, int64_t row0, int64_t row1, int r, int rnew,
                           const double* __restrict__ MT, int ldq, Extra extra, double* tile, double* mts, int ldm) {
  const int tid = threadIdx.x;
  const int n_in = r + 1;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t row = row0 + lane;
  // one row per lane, the waves over the columns (independent loads in flight)
  if (row < row1) {
#pragma unroll 4
    for (int j = wave; j < r; j += kNW) tile[j * kApplyRows + lane] = X[row + (int64_t)j * ldx];
    if (wave == 0) tile[r * kApplyRows + lane] = extra(row);
  } else {
    for (int j = wave; j < n_in; j += kNW) tile[j * kApplyRows + lane] = 0.0;
  }
  if (STAGED)
    for (int e = tid; e < n_in * ldm; e += kIT) {
      const int j = e / ldm, c = e - j * ldm;
      mts[e] = c < rnew ? MT[(int64_t)j * ldq + c] : 0.0;
    }
  __syncthreads();
  for (int cb = wave * kColPass; cb < rnew; cb += kNW * kColPass) {
    const int cbu = __builtin_amdgcn_readfirstlane(cb);
    double acc[kColPass];
#pragma unroll
    for (int q = 0; q < kColPass; ++q) acc[q] = 0.0;
    for (int j = 0; j < n_in; ++j) {
      const double t = tile[j * kApplyRows + lane];
      const double* m = STAGED ? mts + j * ldm + cbu : MT + (int64_t)j * ldq + cbu;
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

// The MT staging area of the apply kernels follows the row tile ((r_max + 1)
// kApplyRows doubles); stage_cap doubles of it (0: none), used when the step's
// (r + 1) x ldm block fits.
__device__ inline bool stage_fits(int r, int rnew, int stage_cap, int& ldm) {
  ldm = (rnew + kColPass - 1) / kColPass * kColPass;
  return (int64_t)(r + 1) * ldm <= stage_cap;
}

__global__ __launch_bounds__(kIT) void isvd_apply_w_kernel(double* __restrict__ W, int64_t N_s,
                                                           const int32_t* state, const double* __restrict__ res,
                                                           const double* __restrict__ scal,
                                                           const double* __restrict__ UqT, int ldq, double* part,
                                                           int stage_cap) {
  extern __shared__ __align__(16) double tile[];
  const int r = state[S_R], rnew = state[S_RNEW];
  const bool noop = state[S_MODE] == M_NOOP;
  const int64_t row0 = (int64_t)blockIdx.x * kApplyRows, row1 = min(row0 + kApplyRows, N_s);
  if (!noop && rnew > 0) {
    const double invp = scal[C_INVP];
    auto extra = [&](int64_t row) { return res[row] * invp; };
    int ldm;
    if (stage_fits(r, rnew, stage_cap, ldm))
      apply_rows<true>(W, N_s, row0, row1, r, rnew, UqT, ldq, extra, tile, tile + ldq * kApplyRows, ldm);
    else
      apply_rows<false>(W, N_s, row0, row1, r, rnew, UqT, ldq, extra, tile, nullptr, 0);
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

__global__ __launch_bounds__(kIT) void isvd_apply_v_kernel(double* __restrict__ V, int64_t m_max,
                                                           const int32_t* state, const double* __restrict__ VqT,
                                                           int ldq, int stage_cap) {
  extern __shared__ __align__(16) double tile[];
  const int r = state[S_R], rnew = state[S_RNEW];
  const bool noop = state[S_MODE] == M_NOOP;
  const int64_t k = state[S_K];
  const int64_t row0 = (int64_t)blockIdx.x * kApplyRows, row1 = min(row0 + kApplyRows, k + 1);
  if (!noop && rnew > 0 && row0 < row1) {
    auto extra = [&](int64_t row) { return row == k ? 1.0 : 0.0; };
    int ldm;
    if (stage_fits(r, rnew, stage_cap, ldm))
      apply_rows<true>(V, m_max, row0, row1, r, rnew, VqT, ldq, extra, tile, tile + ldq * kApplyRows, ldm);
    else
      apply_rows<false>(V, m_max, row0, row1, r, rnew, VqT, ldq, extra, tile, nullptr, 0);
  }
}

// End of a step (one workgroup): the orthogonality test from the W update's
// partials, the re-orthonormalisation when it fails, and the new state.
__global__ __launch_bounds__(kIT) void isvd_commit_kernel(double* __restrict__ W, int64_t N_s, int32_t* state,
                                                          const double* part, int GW, double orth_tol) {
  __shared__ int s_orth;
  const int rnew = state[S_RNEW];
  const bool noop = state[S_MODE] == M_NOOP;
  double t = 0.0;
  for (int b = threadIdx.x; b < GW; b += kIT) t += part[b];
  t = block_sum(t);
  if (threadIdx.x == 0) s_orth = (!noop && rnew > 1 && fabs(t) > orth_tol) ? 1 : 0;
  __syncthreads();
  if (s_orth) orthonormalise(W, N_s, rnew);
  if (threadIdx.x == 0) {
    if (noop) {
      state[S_REFUSED] += 1;
    } else {
      if (s_orth) state[S_QR] += 1;
      state[S_R] = rnew;
      state[S_K] += 1;
    }
  }
}

__global__ void isvd_reset_kernel(int32_t* state) {
  if (threadIdx.x < kIsvdStateInts) state[threadIdx.x] = 0;
}

}  // namespace

int64_t isvd_rows_per_block(int64_t N_s) {
  // row blocks of 128 rows (two per lane and column), longer past 1024 blocks
  // so the final reductions stay short
  int64_t rpb = 128;
  const int64_t nb = (N_s + rpb - 1) / rpb;
  if (nb > 1024) rpb = ((N_s + 1023) / 1024 + 63) / 64 * 64;
  return rpb;
}

int isvd_row_blocks(int64_t N_s) {
  const int64_t rpb = isvd_rows_per_block(N_s);
  return (int)((N_s + rpb - 1) / rpb);
}

// LDS of the apply kernels: the row tile, then up to kStageElems doubles for the
// rows of M^T, as many as fit beside the tile in kApplyLdsMax bytes.
int isvd_stage_cap(int r_max) {
  const int64_t tile = (int64_t)(r_max + 1) * kApplyRows;
  const int64_t want = (int64_t)(r_max + 1) * ((r_max + kColPass - 1) / kColPass * kColPass);
  int64_t cap = want < kStageElems ? want : kStageElems;
  const int64_t room = (int64_t)(kApplyLdsMax / sizeof(double)) - tile;
  if (cap > room) cap = room;
  return cap > 0 ? (int)cap : 0;
}

size_t isvd_apply_lds_bytes(int r_max) {
  return sizeof(double) * ((size_t)(r_max + 1) * kApplyRows + (size_t)isvd_stage_cap(r_max));
}

hipError_t launch_isvd_reset(int32_t* state, hipStream_t s) {
  hipLaunchKernelGGL(isvd_reset_kernel, dim3(1), dim3(64), 0, s, state);
  return hipGetLastError();
}

hipError_t launch_isvd_step(const IsvdArgs& a, const double* u, hipStream_t s) {
  const int ldq = a.r_max + 1;
  const size_t lds = isvd_apply_lds_bytes(a.r_max);
  if (lds > 64 * 1024 && !g_capturing) {
    hipError_t e = hipFuncSetAttribute((const void*)isvd_apply_w_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)isvd_apply_v_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    if (e != hipSuccess) return e;
  }
  if (a.N_s <= kFrontRows) {
    hipLaunchKernelGGL(isvd_front_kernel, dim3(1), dim3(kIT), 0, s, a.W, a.N_s, u, a.state, a.res, a.scal, a.s,
                       a.UqT, a.VqT, a.r_max, a.m_max, a.eps_svd, a.eps_sv);
  } else {
    // row blocks with their partials, each reduction a launch of its own (a
    // kernel boundary orders the workgroups' writes without device-wide fences)
    const int64_t rpb = isvd_rows_per_block(a.N_s);
    const int G = isvd_row_blocks(a.N_s);
    hipLaunchKernelGGL(isvd_dots_kernel, dim3(G), dim3(kIT), 0, s, a.W, a.N_s, rpb, u, a.state, a.part);
    hipLaunchKernelGGL(isvd_reduce_kernel, dim3(1), dim3(kRT), 0, s, a.part, G, a.state, a.l1);
    hipLaunchKernelGGL(isvd_sub1_kernel, dim3(G), dim3(kIT), 0, s, a.W, a.N_s, rpb, u, a.state, a.l1, a.res, a.part);
    hipLaunchKernelGGL(isvd_reduce_kernel, dim3(1), dim3(kRT), 0, s, a.part, G, a.state, a.l2);
    hipLaunchKernelGGL(isvd_sub2_kernel, dim3(G), dim3(kIT), 0, s, a.W, a.N_s, rpb, a.state, a.l2, a.res, a.part);
    hipLaunchKernelGGL(isvd_svd_kernel, dim3(1), dim3(kSvdThreads), 0, s, a.part, G, a.state, a.l1, a.l2, a.scal, a.s,
                       a.UqT, a.VqT, a.r_max, a.m_max, a.eps_svd, a.eps_sv);
  }
  const int GW = (int)((a.N_s + kApplyRows - 1) / kApplyRows);
  const int GV = (int)((a.m_max + kApplyRows - 1) / kApplyRows);
  const double orth_tol = fmin(a.eps_svd, bsvd::kEps * (double)a.N_s);
  // Staging M^T in LDS takes the room of a second workgroup per CU: it pays while
  // the grid leaves CUs idle anyway (measured: the 4-block W and 64-block V updates
  // of 256-row snapshots gain, a 768-block W update of 49152-row ones loses).
  const int cap = isvd_stage_cap(a.r_max);
  const int cap_w = GW <= kStageMaxGrid ? cap : 0, cap_v = GV <= kStageMaxGrid ? cap : 0;
  const size_t tile = sizeof(double) * (size_t)ldq * kApplyRows;
  hipLaunchKernelGGL(isvd_apply_w_kernel, dim3(GW), dim3(kIT), tile + sizeof(double) * (size_t)cap_w, s, a.W, a.N_s,
                     a.state, a.res, a.scal, a.UqT, ldq, a.part, cap_w);
  hipLaunchKernelGGL(isvd_apply_v_kernel, dim3(GV), dim3(kIT), tile + sizeof(double) * (size_t)cap_v, s, a.V,
                     a.m_max, a.state, a.VqT, ldq, cap_v);
  hipLaunchKernelGGL(isvd_commit_kernel, dim3(1), dim3(kIT), 0, s, a.W, a.N_s, a.state, a.part, GW, orth_tol);
  return hipGetLastError();
}

}  // namespace strom
