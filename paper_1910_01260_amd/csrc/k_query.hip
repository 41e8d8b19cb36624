// Per-query kernels of the online phase on gfx950:
//   * plan: widths, packed offsets, validation and a largest-first order;
//   * form: the reduced space-time system of every query (Sec. 4.3,
//     Eq. (ij-block-matrix), (j-block-vector), projection of u0_st),
//     streamed row-major to HBM with coalesced stores;
//   * residual: r = b - Ahat_st(mu) x in FP64 evaluated from the ROM pieces
//     (T, K, Ahat_q), never from a stored matrix;
//   * small bookkeeping kernels for iterative refinement.
#include <type_traits>

#include "internal.h"
#include "wave_ops.h"

namespace strom {
namespace {

constexpr int kPlanThreads = 1024;
constexpr int kFormThreads = 256;
constexpr int kColChunk = 4;      // columns per thread in flight in the form kernel

__device__ inline bool finite_d(double v) { return v == v && v - v == 0.0; }

// Coefficient of P1[a] in the right-hand side for spatial mode i of query q: the
// reduced initial state (Phi_s^T u0)_i, and under Crank-Nicolson the first step's
// explicit half, (Phi_s^T (I + dt_1/2 A(mu)) u0)_i.
__device__ inline double initial_coef(const RomView& rom, const double* __restrict__ thA,
                                      const double* __restrict__ th0, int32_t q, int i) {
  double u0 = 0.0;
  for (int k = 0; k < rom.Q0; ++k) u0 = fma(th0[(int64_t)q * rom.Q0 + k], rom.u0hat[(int64_t)k * rom.n_s + i], u0);
  if (rom.integ == ST_CRANK_NICOLSON && rom.Q0 > 0) {
    double au = 0.0;
    for (int t = 0; t < rom.Q; ++t)
      for (int k = 0; k < rom.Q0; ++k)
        au = fma(thA[(int64_t)q * rom.Q + t] * th0[(int64_t)q * rom.Q0 + k],
                 rom.Au0[((int64_t)t * rom.Q0 + k) * rom.n_s + i], au);
    u0 = fma(0.5 * rom.dt[0], au, u0);
  }
  return u0;
}

// wavefront sum of the device library (DPP based, all lanes active)
extern "C" __device__ double __ockl_wfred_add_f64(double);

// One workgroup.  Writes width, info, coeff_off, mat_off, order, and zeroes the counters.
__global__ __launch_bounds__(kPlanThreads) void plan_kernel(int32_t n_q, int32_t n_s, const int32_t* __restrict__ moff,
                                                            const int32_t* __restrict__ nt_q,
                                                            const int32_t* __restrict__ skip,
                                                            const double* __restrict__ thA,
                                                            const double* __restrict__ thf,
                                                            const double* __restrict__ th0, int32_t Q, int32_t Qf,
                                                            int32_t Q0, int64_t coeff_cap, int64_t mat_cap, Plan plan) {
  __shared__ int64_t s_w[kPlanThreads];
  __shared__ int64_t s_w2[kPlanThreads];
  __shared__ int32_t s_cnt[kMaxWidth + 1];
  const int tid = threadIdx.x;
  // 1. widths and validation
  for (int q = tid; q < n_q; q += kPlanThreads) {
    int32_t code = 0;
    int64_t w = 0;
    for (int i = 0; i < n_s; ++i) {
      const int32_t full = moff[i + 1] - moff[i];
      const int32_t v = nt_q ? nt_q[(int64_t)q * n_s + i] : full;
      if (v < 0 || v > full) code = -4;
      w += v;
    }
    for (int k = 0; k < Q; ++k) if (!finite_d(thA[(int64_t)q * Q + k])) code = code ? code : -5;
    for (int k = 0; k < Qf; ++k) if (!finite_d(thf[(int64_t)q * Qf + k])) code = code ? code : -5;
    for (int k = 0; k < Q0; ++k) if (!finite_d(th0[(int64_t)q * Q0 + k])) code = code ? code : -5;
    if (w > kMaxWidth) code = code ? code : -3;
    if (code == 0 && skip && skip[q]) code = -2;  // keeps its coefficient slot, takes no matrix space
    plan.info[q] = code;
    plan.width[q] = (code == 0 || code == -2) ? (int32_t)w : 0;
  }
  __syncthreads();
  // 2. exclusive prefix sums of w and w^2 over contiguous chunks
  const int per = (n_q + kPlanThreads - 1) / kPlanThreads;
  const int qb = min(n_q, tid * per), qe = min(n_q, qb + per);
  int64_t sw = 0, sw2 = 0;
  for (int q = qb; q < qe; ++q) {
    const int64_t w = plan.width[q];
    sw += w;
    if (plan.info[q] == 0) sw2 += w * w;
  }
  s_w[tid] = sw;
  s_w2[tid] = sw2;
  __syncthreads();
  for (int off = 1; off < kPlanThreads; off <<= 1) {
    int64_t a = 0, b = 0;
    if (tid >= off) { a = s_w[tid - off]; b = s_w2[tid - off]; }
    __syncthreads();
    s_w[tid] += a;
    s_w2[tid] += b;
    __syncthreads();
  }
  int64_t cw = s_w[tid] - sw, cw2 = s_w2[tid] - sw2;
  for (int q = qb; q < qe; ++q) {
    const int64_t w = plan.width[q];
    plan.coeff_off[q] = cw;
    plan.mat_off[q] = cw2;
    cw += w;
    if (plan.info[q] == 0) cw2 += w * w;
    if ((plan.info[q] == 0 || plan.info[q] == -2) && cw > coeff_cap) plan.info[q] = -3;
    if (plan.info[q] == 0 && cw2 > mat_cap) plan.info[q] = -3;
  }
  if (tid == kPlanThreads - 1) {
    plan.coeff_off[n_q] = s_w[tid];
    plan.mat_off[n_q] = s_w2[tid];
  }
  // 3. order by width, largest first (counting sort; order within a width is irrelevant)
  for (int i = tid; i <= kMaxWidth; i += kPlanThreads) s_cnt[i] = 0;
  __syncthreads();
  for (int q = tid; q < n_q; q += kPlanThreads) atomicAdd(&s_cnt[plan.width[q]], 1);
  __syncthreads();
  if (tid == 0) {
    int32_t pos = 0;
    for (int w = kMaxWidth; w >= 0; --w) {
      const int32_t c = s_cnt[w];
      s_cnt[w] = pos;
      pos += c;
    }
  }
  __syncthreads();
  for (int q = tid; q < n_q; q += kPlanThreads) {
    const int32_t p = atomicAdd(&s_cnt[plan.width[q]], 1);
    plan.order[p] = q;
  }
  if (tid < 4) plan.counter[tid] = 0;
}

// Mode-row work items.  The assembly and residual kernels give one workgroup
// the rows of one spatial mode i of one query (its n_t,i(q) temporal rows).  The
// 1-D grid has 8 * per * n_q workgroups (per = ceil(n_s / 8)); workgroups are
// dispatched round-robin over the 8 XCDs, so XCD x receives the linear ids x,
// x + 8, ... and is given the modes x, x + 8, x + 16, ... of every query in turn.
// The rows of the shared contraction T that an XCD reads (those of its modes)
// are then the same for every query and stay in that XCD's L2.
struct ModeItem {
  int32_t q, i;
};

__device__ inline ModeItem mode_item(int32_t n_s) {
  const int32_t L = blockIdx.x;
  const int32_t per = (n_s + 7) >> 3;
  const int32_t k = L >> 3;
  ModeItem it;
  it.q = k / per;
  it.i = (L & 7) + 8 * (k % per);
  return it;
}

inline int32_t mode_grid(int32_t n_q, int32_t n_s) { return 8 * ((n_s + 7) / 8) * n_q; }

// Per-workgroup view of one query: local -> global reduced index and mode of
// every column, local mode offsets, and row i of Ahat(mu) = sum_q theta_q Ahat_q.
struct QueryLds {
  int32_t* gmap;   // w_max
  int16_t* mmap;   // w_max
  int32_t* loff;   // n_s + 1
  double* Ah;      // n_s
};

__device__ inline QueryLds carve_lds(char* base, int n_s, int w_max) {
  QueryLds L;
  L.Ah = reinterpret_cast<double*>(base);
  L.gmap = reinterpret_cast<int32_t*>(base + sizeof(double) * n_s);
  L.loff = L.gmap + w_max;
  L.mmap = reinterpret_cast<int16_t*>(L.loff + n_s + 1);
  return L;
}

__host__ __device__ inline size_t query_lds_bytes(int n_s, int w_max) {
  const size_t b = sizeof(double) * n_s + sizeof(int32_t) * (w_max + n_s + 1) + sizeof(int16_t) * w_max;
  return (b + 15) / 16 * 16;
}

// Local mode offsets by a scan in wave 0 (two modes per lane, n_s <= 128), the
// column maps, and row i of Ahat(mu).
__device__ inline void query_setup(const RomView& rom, int32_t q, int32_t i, const double* __restrict__ thA,
                                   const int32_t* __restrict__ nt_q, QueryLds L) {
  const int n_s = rom.n_s;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int32_t c0 = 0, c1 = 0;
    const int i0 = 2 * lane, i1 = 2 * lane + 1;
    if (i0 < n_s) c0 = nt_q ? nt_q[(int64_t)q * n_s + i0] : rom.moff[i0 + 1] - rom.moff[i0];
    if (i1 < n_s) c1 = nt_q ? nt_q[(int64_t)q * n_s + i1] : rom.moff[i1 + 1] - rom.moff[i1];
    int32_t incl = c0 + c1;
    for (int d = 1; d < 64; d <<= 1) {
      const int32_t v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    const int32_t excl = incl - c0 - c1;
    if (i0 < n_s) L.loff[i0] = excl;
    if (i1 < n_s) L.loff[i1] = excl + c0;
    if (lane == 63) L.loff[n_s] = incl;
  }
  const int ns2 = n_s * n_s;
  for (int ic = threadIdx.x; ic < n_s; ic += blockDim.x) {
    double v = 0.0;
    for (int k = 0; k < rom.Q; ++k)
      v = fma(thA[(int64_t)q * rom.Q + k], rom.Ahat[(int64_t)k * ns2 + (int64_t)ic * n_s + i], v);
    L.Ah[ic] = v;
  }
  __syncthreads();
  // column maps: local column c -> mode (binary search of the offsets) and global index
  const int32_t wq = L.loff[n_s];
  for (int c = threadIdx.x; c < wq; c += blockDim.x) {
    int lo = 0, hi = n_s - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (L.loff[mid] <= c) lo = mid; else hi = mid - 1;
    }
    L.mmap[c] = (int16_t)lo;
    L.gmap[c] = rom.moff[lo] + (c - L.loff[lo]);
  }
  __syncthreads();
}

// Rows handled per pass of the row loops (two rows' loads in flight together).
constexpr int kRowUnroll = 4;
// Rows of one residual pass (their partial sums live in registers).
constexpr int kResRows = 8;

// The rows of one mode i for the columns c = cb + 256 k (k < KC) of one query's
// system outside the mode's own block: -Ahat(mu)[i, mode(c)] T[g0 + j, gmap(c)].
// T symmetric: column g0 + j holds row g0 + j.
template <typename OutT, typename TT, int KC>
__device__ inline void form_columns(const QueryLds& L, int w, int cb, int nti, int g0, int r0, int64_t n,
                                    const TT* __restrict__ tsrc, OutT* __restrict__ M) {
  int gc[KC];
  double ah[KC];
  bool ok[KC];
#pragma unroll
  for (int k = 0; k < KC; ++k) {
    const int c = cb + k * kFormThreads;
    ok[k] = c < w && (c < r0 || c >= r0 + nti);
    gc[k] = c < w ? L.gmap[c] : 0;
    ah[k] = c < w ? -L.Ah[L.mmap[c]] : 0.0;
  }
  constexpr int RU = 8;  // rows whose T loads are in flight together
  if constexpr (std::is_same<OutT, float>::value) {
    // Two batches of RU rows alternate: the next batch's T loads are issued before the
    // current batch's stores.  Loads and stores share one counter of outstanding memory
    // operations, so this order lets a wave wait for its loads without also waiting for
    // the stores issued before them (measured: 2.72 against 2.97 ms on the 4096-query
    // batch; the FP64 systems, with twice the registers per value, are faster as below).
    TT ta[RU][KC], tb[RU][KC];
    auto load = [&](TT (&t)[RU][KC], int j0) {
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int j = min(j0 + u, nti - 1);
        const TT* Trow = tsrc + (int64_t)(g0 + j) * n;
#pragma unroll
        for (int k = 0; k < KC; ++k) t[u][k] = Trow[gc[k]];
      }
    };
    auto store = [&](const TT (&t)[RU][KC], int j0) {
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (j0 + u >= nti) break;
        OutT* Mr = M + (int64_t)(r0 + j0 + u) * w;
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (ok[k]) Mr[cb + k * kFormThreads] = (OutT)(ah[k] * (double)t[u][k]);
      }
    };
    load(ta, 0);
    for (int j0 = 0; j0 < nti; j0 += 2 * RU) {
      if (j0 + RU < nti) load(tb, j0 + RU);
      store(ta, j0);
      if (j0 + RU >= nti) break;
      if (j0 + 2 * RU < nti) load(ta, j0 + 2 * RU);
      store(tb, j0 + RU);
    }
  } else {
    for (int j0 = 0; j0 < nti; j0 += RU) {
      OutT v[RU][KC];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int j = min(j0 + u, nti - 1);
        const TT* Trow = tsrc + (int64_t)(g0 + j) * n;
#pragma unroll
        for (int k = 0; k < KC; ++k) v[u][k] = (OutT)(ah[k] * (double)Trow[gc[k]]);
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (j0 + u >= nti) break;
        OutT* Mr = M + (int64_t)(r0 + j0 + u) * w;
#pragma unroll
        for (int k = 0; k < KC; ++k)
          if (ok[k]) Mr[cb + k * kFormThreads] = v[u][k];
      }
    }
  }
}

template <typename OutT>
__global__ __launch_bounds__(kFormThreads) void form_kernel(RomView rom, int32_t n_q, const double* __restrict__ thA,
                                                            const double* __restrict__ thf,
                                                            const double* __restrict__ th0,
                                                            const int32_t* __restrict__ nt_q, Plan plan,
                                                            OutT* __restrict__ mats, double* __restrict__ rhs,
                                                            int32_t w_max) {
  extern __shared__ __align__(16) char lds[];
  const ModeItem it = mode_item(rom.n_s);
  const int32_t q = it.q, i = it.i;
  if (q >= n_q || i >= rom.n_s || plan.info[q] != 0) return;
  const int32_t nti = nt_q ? nt_q[(int64_t)q * rom.n_s + i] : rom.moff[i + 1] - rom.moff[i];
  if (nti == 0) return;
  const int32_t w = plan.width[q];
  QueryLds L = carve_lds(lds, rom.n_s, w_max);
  query_setup(rom, q, i, thA, nt_q, L);
  const int64_t n = rom.n;
  const int r0 = L.loff[i];
  const int g0 = rom.moff[i];                         // global index of the mode's first temporal vector
  const int ntf = rom.moff[i + 1] - g0;               // full n_t,i (leading dimension of K_i)
  const double* Ki = rom.K + rom.koff[i];            // K_i[j', j] at Ki[j * ntf + j']
  OutT* M = mats + plan.mat_off[q];
  // The FP32 assembly reads the FP32 copy of T: its entries are rounded to FP32
  // anyway, and the FP64 copy's L2 traffic (twice the bytes written) would bound it.
  typedef typename std::conditional<std::is_same<OutT, float>::value, float, double>::type TT;
  const TT* tsrc;
  if constexpr (std::is_same<OutT, float>::value) tsrc = rom.T32;
  else tsrc = rom.Teff;
  // Columns outside the mode's own block: each thread owns the columns c = tid + 256 k,
  // k < KC; their global index and -Ahat(mu) factor stay in registers while the rows
  // of the mode stream past.  KC follows the query's width so that few column slots
  // are empty; the loop is branch-free per element (empty slots and the mode's own
  // columns read T[., 0] or their T entry and are not stored).
  const int kc = (w + kFormThreads - 1) / kFormThreads;
  switch (kc) {
    case 1: form_columns<OutT, TT, 1>(L, w, threadIdx.x, nti, g0, r0, n, tsrc, M); break;
    case 2: form_columns<OutT, TT, 2>(L, w, threadIdx.x, nti, g0, r0, n, tsrc, M); break;
    case 3: form_columns<OutT, TT, 3>(L, w, threadIdx.x, nti, g0, r0, n, tsrc, M); break;
    case 4: form_columns<OutT, TT, 4>(L, w, threadIdx.x, nti, g0, r0, n, tsrc, M); break;
    case 5: form_columns<OutT, TT, 5>(L, w, threadIdx.x, nti, g0, r0, n, tsrc, M); break;
    default:
      for (int cb = threadIdx.x; cb < w; cb += 4 * kFormThreads)
        form_columns<OutT, TT, 4>(L, w, cb, nti, g0, r0, n, tsrc, M);
  }
  // The mode's own block (rows and columns r0 .. r0 + nti - 1): K_i plus the T term,
  // one element per thread.
  {
    const double ahi = -L.Ah[i];
    for (int e = threadIdx.x; e < nti * nti; e += kFormThreads) {
      const int j = e / nti, jj = e % nti;
      M[(int64_t)(r0 + j) * w + r0 + jj] =
          (OutT)fma(ahi, (double)tsrc[(int64_t)(g0 + j) * n + g0 + jj], Ki[(int64_t)jj * ntf + j]);
    }
  }
  // right-hand side of these rows
  for (int j = threadIdx.x; j < nti; j += kFormThreads) {
    const int g = g0 + j;
    double b = 0.0;
    for (int k = 0; k < rom.Qf; ++k)
      b = fma(thf[(int64_t)q * rom.Qf + k] * rom.Wf[(int64_t)k * n + g], rom.bhat[(int64_t)k * rom.n_s + i], b);
    const double u0 = initial_coef(rom, thA, th0, q, i);
    rhs[plan.coeff_off[q] + r0 + j] = fma(rom.P1[g], u0, b);
  }
}

// r = b - Ahat_st(mu) x for the rows of one mode of each active query, in groups
// of kFormRows rows: per-thread partial sums over the thread's columns, then a
// workgroup reduction per row in a fixed order.
__global__ __launch_bounds__(kFormThreads) void residual_kernel(RomView rom, int32_t n_q,
                                                                const double* __restrict__ thA,
                                                                const int32_t* __restrict__ nt_q, Plan plan,
                                                                const double* __restrict__ rhs,
                                                                const double* __restrict__ x, double* __restrict__ r,
                                                                const int32_t* __restrict__ active, int32_t w_max) {
  extern __shared__ __align__(16) char lds[];
  const ModeItem it = mode_item(rom.n_s);
  const int32_t q = it.q, i = it.i;
  if (q >= n_q || i >= rom.n_s || plan.info[q] != 0) return;
  if (active && !active[q]) return;
  const int32_t nti = nt_q ? nt_q[(int64_t)q * rom.n_s + i] : rom.moff[i + 1] - rom.moff[i];
  if (nti == 0) return;
  const int32_t w = plan.width[q];
  QueryLds L = carve_lds(lds, rom.n_s, w_max);
  double* xs = reinterpret_cast<double*>(lds + query_lds_bytes(rom.n_s, w_max));
  const int64_t off = plan.coeff_off[q];
  for (int c = threadIdx.x; c < w; c += kFormThreads) xs[c] = x[off + c];
  query_setup(rom, q, i, thA, nt_q, L);
  const int64_t n = rom.n;
  const int r0 = L.loff[i];
  const int g0 = rom.moff[i];
  const int ntf = rom.moff[i + 1] - g0;
  const double* Ki = rom.K + rom.koff[i];
  __shared__ double s_red[kFormThreads / 64][kResRows];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int jb = 0; jb < nti; jb += kResRows) {
    const int nrow = min(kResRows, nti - jb);
    double acc[kResRows];
#pragma unroll
    for (int rr = 0; rr < kResRows; ++rr) acc[rr] = 0.0;
    for (int cb = threadIdx.x; cb < w; cb += kColChunk * kFormThreads) {
      int ic[kColChunk], gc[kColChunk];
      double xa[kColChunk], ah[kColChunk];
#pragma unroll
      for (int k = 0; k < kColChunk; ++k) {
        const int c = cb + k * kFormThreads;
        ic[k] = c < w ? L.mmap[c] : -1;
        gc[k] = c < w ? L.gmap[c] : 0;
        xa[k] = c < w ? xs[c] : 0.0;
        ah[k] = c < w ? -L.Ah[ic[k]] : 0.0;
      }
#pragma unroll
      for (int rr = 0; rr < kResRows; ++rr) {
        const int j = jb + min(rr, nrow - 1);
        const double* Trow = rom.Teff + (int64_t)(g0 + j) * n;  // row g0 + j of T (or T_cn)
        double sum = 0.0;
#pragma unroll
        for (int k = 0; k < kColChunk; ++k) {
          const double t = ic[k] >= 0 ? Trow[gc[k]] : 0.0;
          const double kv = ic[k] == i ? Ki[(int64_t)(gc[k] - g0) * ntf + j] : 0.0;
          sum = fma(fma(ah[k], t, kv), xa[k], sum);
        }
        acc[rr] += rr < nrow ? sum : 0.0;
      }
    }
#pragma unroll
    for (int rr = 0; rr < kResRows; ++rr) {
      const double t = __ockl_wfred_add_f64(acc[rr]);
      if (lane == 0) s_red[wave][rr] = t;
    }
    __syncthreads();
    if (threadIdx.x < nrow) {
      const int rr = threadIdx.x;
      double t = 0.0;
      for (int wv = 0; wv < kFormThreads / 64; ++wv) t += s_red[wv][rr];
      const int64_t o = off + r0 + jb + rr;
      r[o] = rhs[o] - t;
    }
    __syncthreads();
  }
}

// norms[q] = ||v_q||_2 over the query's segment; one workgroup per query, fixed reduction order.
__global__ __launch_bounds__(256) void vec_norms_kernel(int32_t n_q, Plan plan, const double* __restrict__ v,
                                                        double* __restrict__ norms) {
  __shared__ double red[256];
  const int32_t q = blockIdx.x;
  const int32_t w = plan.width[q];
  const int64_t off = plan.coeff_off[q];
  double s = 0.0;
  if (plan.info[q] == 0)
    for (int c = threadIdx.x; c < w; c += 256) s = fma(v[off + c], v[off + c], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) norms[q] = sqrt(red[0]);
}

// Refinement bookkeeping for step `step` (last != 0: final check).
__global__ void ir_check_kernel(int32_t n_q, Plan plan, const double* __restrict__ rnorm,
                                const double* __restrict__ bnorm, double tol, int32_t step, int32_t last,
                                int32_t* __restrict__ active, double* __restrict__ relres, int32_t* __restrict__ iters) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_q) return;
  if (plan.info[q] != 0) {
    if (last && plan.info[q] != -2) relres[q] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  // queries that converged during refinement keep the residual recorded then
  if (!active[q]) return;
  const double bn = bnorm[q];
  const double rel = bn > 0.0 ? rnorm[q] / bn : rnorm[q];
  if (last) {
    relres[q] = rel;
    if (iters) iters[q] = step;
    if (tol > 0.0 && last > 1 && !(rel <= tol)) plan.info[q] = -1;
    return;
  }
  if (rel <= tol) {
    active[q] = 0;
    relres[q] = rel;
    if (iters) iters[q] = step;
  }
}

// FP64 re-solve plan of the queries whose FP32-LU refinement did not converge
// (plan.info == -1).  One workgroup.  fb shares width, order and coeff_off with
// plan; fb.info is 0 for a query to re-solve and -2 (skip) otherwise, also when
// its FP64 system does not fit in mat_cap elements after the earlier ones;
// fb.mat_off packs the FP64 systems in query order; active marks the queries
// re-solved.
__global__ __launch_bounds__(kPlanThreads) void fallback_plan_kernel(int32_t n_q, Plan plan, Plan fb,
                                                                     int32_t* __restrict__ active, int64_t mat_cap) {
  __shared__ int64_t s_w2[kPlanThreads];
  const int tid = threadIdx.x;
  const int per = (n_q + kPlanThreads - 1) / kPlanThreads;
  const int qb = min(n_q, tid * per), qe = min(n_q, qb + per);
  int64_t sw2 = 0;
  for (int q = qb; q < qe; ++q)
    if (plan.info[q] == -1) sw2 += (int64_t)plan.width[q] * plan.width[q];
  s_w2[tid] = sw2;
  __syncthreads();
  for (int off = 1; off < kPlanThreads; off <<= 1) {
    const int64_t a = tid >= off ? s_w2[tid - off] : 0;
    __syncthreads();
    s_w2[tid] += a;
    __syncthreads();
  }
  int64_t cw2 = s_w2[tid] - sw2;
  for (int q = qb; q < qe; ++q) {
    int32_t code = -2;
    fb.mat_off[q] = cw2;
    if (plan.info[q] == -1) {
      cw2 += (int64_t)plan.width[q] * plan.width[q];
      code = cw2 <= mat_cap ? 0 : -2;
    }
    fb.info[q] = code;
    active[q] = code == 0;
  }
  if (tid == kPlanThreads - 1) fb.mat_off[n_q] = s_w2[tid];
  if (tid < 4) fb.counter[tid] = 0;
}

// After the FP64 re-solve: queries re-solved get info -6 (or the FP64 LU's zero
// pivot); those that did not fit keep -1 and their FP32 iterate and residual.
__global__ void fallback_finish_kernel(int32_t n_q, Plan plan, Plan fb, const int32_t* __restrict__ active) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_q || plan.info[q] != -1 || !active[q]) return;
  const int32_t c = fb.info[q];
  if (c == 0) plan.info[q] = -6;
  else if (c > 0) plan.info[q] = c;
}

__global__ void finalize_kernel(int32_t n_q, Plan plan, double* __restrict__ coeff) {
  const int32_t q = blockIdx.y;
  if (plan.info[q] <= 0) return;
  const int32_t w = plan.width[q];
  const int64_t off = plan.coeff_off[q];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < w; c += gridDim.x * blockDim.x)
    coeff[off + c] = __longlong_as_double(0x7ff8000000000000LL);
}

// right-hand side only (see form_kernel), one thread per reduced index of a query
__global__ __launch_bounds__(256) void rhs_kernel(RomView rom, int32_t n_q, const double* __restrict__ thA,
                                                  const double* __restrict__ thf, const double* __restrict__ th0,
                                                  Plan plan, double* __restrict__ rhs) {
  const int32_t q = blockIdx.y;
  if (plan.info[q] != 0) return;
  const int32_t w = plan.width[q];
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= w) return;  // full-width queries: local index = global index
  const int i = rom.mode[a];
  double b = 0.0;
  for (int k = 0; k < rom.Qf; ++k)
    b = fma(thf[(int64_t)q * rom.Qf + k] * rom.Wf[(int64_t)k * rom.n + a], rom.bhat[(int64_t)k * rom.n_s + i], b);
  const double u0 = initial_coef(rom, thA, th0, q, i);
  rhs[plan.coeff_off[q] + a] = fma(rom.P1[a], u0, b);
}

// right-hand side of queries with per-mode prefixes: one workgroup per (mode,
// query); mode i's local block starts at the sum of the query's earlier prefixes
__global__ __launch_bounds__(256) void rhs_prefix_kernel(RomView rom, int32_t n_q, const double* __restrict__ thA,
                                                         const double* __restrict__ thf,
                                                         const double* __restrict__ th0,
                                                         const int32_t* __restrict__ nt_q, Plan plan,
                                                         double* __restrict__ rhs) {
  const int32_t i = blockIdx.x, q = blockIdx.y;
  if (plan.info[q] != 0) return;
  const int32_t* ntq = nt_q + (int64_t)q * rom.n_s;
  int64_t loff = 0;
  for (int l = 0; l < i; ++l) loff += ntq[l];
  const double u0 = initial_coef(rom, thA, th0, q, i);
  const int32_t a0 = rom.moff[i];
  for (int j = threadIdx.x; j < ntq[i]; j += 256) {
    const int a = a0 + j;
    double b = 0.0;
    for (int k = 0; k < rom.Qf; ++k)
      b = fma(thf[(int64_t)q * rom.Qf + k] * rom.Wf[(int64_t)k * rom.n + a], rom.bhat[(int64_t)k * rom.n_s + i], b);
    rhs[plan.coeff_off[q] + loff + j] = fma(rom.P1[a], u0, b);
  }
}

// coeff[coeff_off[q] + a] = mean[a] + scale[a] * Y[q * n + a] for valid queries
__global__ void destandardize_kernel(int64_t total, int32_t n, const float* __restrict__ Y,
                                     const double* __restrict__ mean, const double* __restrict__ scale, Plan plan,
                                     double* __restrict__ coeff) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int32_t q = (int32_t)(e / n);
  const int a = (int)(e % n);
  if (plan.info[q] != 0 || a >= plan.width[q]) return;
  coeff[plan.coeff_off[q] + a] = fma(scale[a], (double)Y[e], mean[a]);
}

__global__ void certificate_kernel(int32_t n_q, Plan plan, const double* __restrict__ rnorm,
                                   const double* __restrict__ cnorm, double gamma, double tol, double* __restrict__ cert,
                                   int32_t* __restrict__ accept, const double* __restrict__ bnorm,
                                   double* __restrict__ relres) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_q) return;
  double c = __longlong_as_double(0x7ff0000000000000LL);  // +inf
  if (plan.info[q] == 0 && cnorm[q] > 0.0) {
    const double e = rnorm[q] / (gamma * cnorm[q]);
    if (e < 1.0) c = e / (1.0 - e);
  }
  cert[q] = c;
  if (accept) accept[q] = (c <= tol) ? 1 : 0;
  if (relres)
    relres[q] = plan.info[q] != 0 ? __longlong_as_double(0x7ff8000000000000LL)
                                   : (bnorm[q] > 0.0 ? rnorm[q] / bnorm[q] : rnorm[q]);
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Residual r = b - Ahat_st(mu) x of each active query without the reduced matrix.  With
// z_i = Phi_i x_i (the query's prefix of mode i's temporal basis, evaluated on the time
// grid), the blocks of Eq. (ij-block-matrix) give
//   (Ahat_st x)_i = Phi_i^T [ z_i - S z_i - dt .* sum_i' Ahat(mu)[i, i'] z_i' ],
// S the one-step delay ((S z)(k) = z(k - 1), (S z)(0) = 0): the K_i blocks are the
// first two terms, the dt-weighted Gram T the third.  One workgroup per query: z and the
// bracket live in LDS (n_s x N_t each), the temporal bases are read twice per query and
// are shared by all queries (L2 resident), instead of n^2 gathers of T per query.
constexpr int kResMfThreads = 512;
constexpr size_t kResMfMaxLds = 150 * 1024;  // dynamic LDS the matrix-free residual may take

size_t residual_mf_lds_bytes(int n_s, int N_t, int w_max) {
  return sizeof(double) * ((size_t)2 * n_s * N_t + (size_t)n_s * n_s + (size_t)w_max) +
         sizeof(int32_t) * (2 * (size_t)n_s + 1) + sizeof(int16_t) * (size_t)w_max;
}

__global__ __launch_bounds__(kResMfThreads) void residual_mf_kernel(RomView rom, int32_t n_q,
                                                                    const double* __restrict__ thA,
                                                                    const int32_t* __restrict__ nt_q, Plan plan,
                                                                    const double* __restrict__ rhs,
                                                                    const double* __restrict__ x,
                                                                    double* __restrict__ r,
                                                                    const int32_t* __restrict__ active, int32_t w_max) {
  extern __shared__ __align__(16) double sm[];
  const int32_t q = blockIdx.x;
  if (q >= n_q || plan.info[q] != 0) return;
  if (active && !active[q]) return;
  const int32_t w = plan.width[q];
  if (w == 0) return;
  const int n_s = rom.n_s, N_t = rom.N_t;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Z = sm;                          // n_s x N_t, Z[i * N_t + k] = z_i(k)
  double* V = Z + (size_t)n_s * N_t;       // n_s x N_t, the bracket
  double* Ah = V + (size_t)n_s * N_t;      // n_s x n_s, Ah[i * n_s + i'] = Ahat(mu)[i, i']
  double* xs = Ah + (size_t)n_s * n_s;     // w
  int32_t* nt = reinterpret_cast<int32_t*>(xs + w_max);  // n_s
  int32_t* loff = nt + n_s;                                // n_s + 1
  int16_t* cmode = reinterpret_cast<int16_t*>(loff + n_s + 1);  // w: mode of each local column
  const int64_t off = plan.coeff_off[q];
  if (tid == 0) {
    int32_t acc = 0;
    for (int i = 0; i < n_s; ++i) {
      const int32_t c = nt_q ? nt_q[(int64_t)q * n_s + i] : rom.moff[i + 1] - rom.moff[i];
      nt[i] = c;
      loff[i] = acc;
      acc += c;
    }
    loff[n_s] = acc;
  }
  const int ns2 = n_s * n_s;
  for (int e = tid; e < ns2; e += kResMfThreads) {
    const int i = e / n_s, ip = e % n_s;
    double v = 0.0;
    for (int k = 0; k < rom.Q; ++k)
      v = fma(thA[(int64_t)q * rom.Q + k], rom.Ahat[(int64_t)k * ns2 + (int64_t)ip * n_s + i], v);
    Ah[e] = v;
  }
  for (int c = tid; c < w; c += kResMfThreads) xs[c] = x[off + c];
  __syncthreads();
  for (int m = tid; m < n_s; m += kResMfThreads)
    for (int32_t c = loff[m]; c < loff[m + 1]; ++c) cmode[c] = (int16_t)m;
  // z_i(k) = sum_j phi_(i,j)(k) x_(i,j): consecutive threads take consecutive k (coalesced)
  for (int e = tid; e < n_s * N_t; e += kResMfThreads) {
    const int i = e / N_t, k = e % N_t;
    const double* ph = rom.Phit + (int64_t)rom.moff[i] * N_t + k;
    const double* xv = xs + loff[i];
    const int ni = nt[i];
    double z = 0.0;
    // unrolled so that several of the strided Phi_t loads are in flight at once (the FMA
    // order, and so the result, is that of the plain loop)
#pragma unroll 8
    for (int j = 0; j < ni; ++j) z = fma(ph[(int64_t)j * N_t], xv[j], z);
    Z[e] = z;
  }
  __syncthreads();
  // bracket: z_i(k) - z_i(k - 1) - dt_k sum_i' Ahat(mu)[i, i'] z_i'(k)  (backward Euler), or
  // z_i(k) - z_i(k - 1) - dt_k/2 sum_i' Ahat(mu)[i, i'] (z_i'(k) + z_i'(k - 1))  (Crank-Nicolson)
  const bool cn = rom.integ == ST_CRANK_NICOLSON;
  for (int e = tid; e < n_s * N_t; e += kResMfThreads) {
    const int i = e / N_t, k = e % N_t;
    const double* ar = Ah + i * n_s;
    double u = 0.0;
    for (int ip = 0; ip < n_s; ++ip) u = fma(ar[ip], Z[ip * N_t + k], u);
    V[e] = cn ? u : Z[e] - (k > 0 ? Z[e - 1] : 0.0) - rom.dt[k] * u;
  }
  __syncthreads();
  if (cn) {
    // V holds Ahat(mu) z(k); one thread per mode walks its steps backwards (V(k - 1) is
    // still the product when step k is finished)
    for (int i = tid; i < n_s; i += kResMfThreads)
      for (int k = N_t - 1; k >= 0; --k) {
        const int e = i * N_t + k;
        const double az = V[e] + (k > 0 ? V[e - 1] : 0.0);
        V[e] = Z[e] - (k > 0 ? Z[e - 1] : 0.0) - 0.5 * rom.dt[k] * az;
      }
    __syncthreads();
  }
  // (Ahat_st x)_(i,j) = sum_k phi_(i,j)(k) V_i(k): 16 lanes per output (one DPP row), 4
  // outputs per wave per pass; the pass count is uniform per wave
  const int sub = lane >> 4, c16 = lane & 15;
  constexpr int NW = kResMfThreads / 64;
  for (int cb = wave * 4; cb < w; cb += NW * 4) {
    const int c = cb + sub;
    const bool ok = c < w;
    const int m = ok ? cmode[c] : 0;
    const double* ph = rom.Phit + (int64_t)(rom.moff[m] + (ok ? c - loff[m] : 0)) * N_t;
    const double* vm = V + (size_t)m * N_t;
    double acc = 0.0;
    if (ok)
#pragma unroll 8
      for (int k = c16; k < N_t; k += 16) acc = fma(ph[k], vm[k], acc);
    acc = row16_sum(acc);
    if (ok && c16 == 0) r[off + c] = rhs[off + c] - acc;
  }
}

}  // namespace

hipError_t launch_plan(int32_t n_q, int32_t n_s, const int32_t* moff, const int32_t* nt_q, const int32_t* skip,
                       const double* thA, const double* thf, const double* th0, int32_t Q, int32_t Qf, int32_t Q0,
                       int64_t coeff_cap, int64_t mat_cap, Plan plan, hipStream_t s) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, n_q, n_s, moff, nt_q, skip, thA, thf, th0, Q, Qf,
                     Q0, coeff_cap, mat_cap, plan);
  return hipGetLastError();
}

hipError_t launch_rhs(const RomView& rom, int32_t n_q, const double* thA, const double* thf, const double* th0,
                      const int32_t* nt_q, Plan plan, double* rhs, int32_t n_max, hipStream_t s) {
  if (n_q == 0 || n_max == 0) return hipSuccess;
  if (nt_q)
    hipLaunchKernelGGL(rhs_prefix_kernel, dim3(rom.n_s, n_q), dim3(256), 0, s, rom, n_q, thA, thf, th0, nt_q, plan,
                       rhs);
  else
    hipLaunchKernelGGL(rhs_kernel, dim3((n_max + 255) / 256, n_q), dim3(256), 0, s, rom, n_q, thA, thf, th0, plan,
                       rhs);
  return hipGetLastError();
}

hipError_t launch_destandardize(int32_t n_q, int32_t n, const float* Y, const double* mean, const double* scale,
                                Plan plan, double* coeff, hipStream_t s) {
  const int64_t total = (int64_t)n_q * n;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(destandardize_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, n, Y, mean,
                     scale, plan, coeff);
  return hipGetLastError();
}

hipError_t launch_certificate(int32_t n_q, Plan plan, const double* rnorm, const double* cnorm, double gamma, double tol,
                              double* cert, int32_t* accept, const double* bnorm, double* relres, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(certificate_kernel, dim3((n_q + 255) / 256), dim3(256), 0, s, n_q, plan, rnorm, cnorm, gamma, tol,
                     cert, accept, bnorm, relres);
  return hipGetLastError();
}

hipError_t launch_form(const RomView& rom, int32_t n_q, const double* thA, const double* thf, const double* th0,
                       const int32_t* nt_q, Plan plan, int32_t out_prec, void* mats, double* rhs, int32_t n_max,
                       hipStream_t s) {
  if (n_q == 0 || n_max == 0) return hipSuccess;
  const size_t lds = query_lds_bytes(rom.n_s, n_max);
  dim3 grid(mode_grid(n_q, rom.n_s));
  if (out_prec == ST_F64) {
    if (!g_capturing) {
      const hipError_t e = hipFuncSetAttribute((const void*)form_kernel<double>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(form_kernel<double>, grid, dim3(kFormThreads), lds, s, rom, n_q, thA, thf, th0, nt_q, plan,
                       (double*)mats, rhs, n_max);
  } else {
    if (!g_capturing) {
      const hipError_t e = hipFuncSetAttribute((const void*)form_kernel<float>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(form_kernel<float>, grid, dim3(kFormThreads), lds, s, rom, n_q, thA, thf, th0, nt_q, plan,
                       (float*)mats, rhs, n_max);
  }
  return hipGetLastError();
}

hipError_t launch_residual(const RomView& rom, int32_t n_q, const double* thA, const int32_t* nt_q, Plan plan,
                           const double* rhs, const double* x, double* r, double* rnorm, const int32_t* active,
                           int32_t n_max, hipStream_t s) {
  if (n_q == 0 || n_max == 0) return hipSuccess;
  hipError_t e = hipSuccess;
  const size_t lds_mf = residual_mf_lds_bytes(rom.n_s, rom.N_t, n_max);
  if (lds_mf <= kResMfMaxLds) {
    if (!g_capturing) {
      e = hipFuncSetAttribute((const void*)residual_mf_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_mf);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(residual_mf_kernel, dim3(n_q), dim3(kResMfThreads), lds_mf, s, rom, n_q, thA, nt_q, plan, rhs, x,
                       r, active, n_max);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_vec_norms(n_q, plan, r, rnorm, s);
  }
  // n_s x N_t too large for LDS: gather the reduced operator from T and K instead
  const size_t lds = query_lds_bytes(rom.n_s, n_max) + sizeof(double) * n_max;
  if (!g_capturing) {
    e = hipFuncSetAttribute((const void*)residual_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  dim3 grid(mode_grid(n_q, rom.n_s));
  hipLaunchKernelGGL(residual_kernel, grid, dim3(kFormThreads), lds, s, rom, n_q, thA, nt_q, plan, rhs, x, r, active,
                     n_max);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_vec_norms(n_q, plan, r, rnorm, s);
}

hipError_t launch_vec_norms(int32_t n_q, Plan plan, const double* v, double* norms, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(vec_norms_kernel, dim3(n_q), dim3(256), 0, s, n_q, plan, v, norms);
  return hipGetLastError();
}

hipError_t launch_ir_check(int32_t n_q, Plan plan, const double* rnorm, const double* bnorm, double tol, int32_t step,
                           int32_t last, int32_t* active, double* relres, int32_t* iters, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(ir_check_kernel, dim3((n_q + 255) / 256), dim3(256), 0, s, n_q, plan, rnorm, bnorm, tol, step,
                     last, active, relres, iters);
  return hipGetLastError();
}

hipError_t launch_finalize(int32_t n_q, Plan plan, double* coeff, int32_t* info_out, hipStream_t s) {
  (void)info_out;
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(4, n_q), dim3(256), 0, s, n_q, plan, coeff);
  return hipGetLastError();
}

hipError_t launch_fallback_plan(int32_t n_q, Plan plan, Plan fb, int32_t* active, int64_t mat_cap, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(fallback_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, n_q, plan, fb, active, mat_cap);
  return hipGetLastError();
}

hipError_t launch_fallback_finish(int32_t n_q, Plan plan, Plan fb, const int32_t* active, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(fallback_finish_kernel, dim3((n_q + 255) / 256), dim3(256), 0, s, n_q, plan, fb, active);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace strom

// ---------------------------------------------------------------------------
// Reconstruction of the space-time state (Sec. 3.2, the space-time state
// approximation): u(x, t_k) = sum_i Phi_s[x, i] sum_j Phi_t[k, (i, j)] c_(i,j),
// over the query's per-mode prefixes.
// ---------------------------------------------------------------------------
namespace strom {
namespace {

constexpr int kRecThreads = 256;
constexpr int kRecSteps = 16;  // time steps per workgroup

// Y[k, i] = sum_{j < nt_q[q, i]} Phi_t[k, moff[i] + j] c[off + loff[i] + j] for the
// workgroup's time steps (in LDS), then out_q[x, k] = sum_i Phi_s[x, i] Y[k, i] with
// one spatial row per thread: Phi_s rows read once per workgroup, coalesced writes.
__global__ __launch_bounds__(kRecThreads) void reconstruct_kernel(int64_t N_s, int32_t N_t, int32_t n_s,
                                                                  const double* __restrict__ Phi_s, int64_t ldp,
                                                                  const double* __restrict__ Phi_t, int64_t ldt,
                                                                  const int32_t* __restrict__ moff,
                                                                  const int32_t* __restrict__ nt_q,
                                                                  const double* __restrict__ coeff,
                                                                  const int64_t* __restrict__ coeff_off,
                                                                  double* __restrict__ out, int64_t ldo) {
  extern __shared__ __align__(16) double rec_lds[];
  double* Y = rec_lds;                                    // kRecSteps x n_s
  int32_t* loff = reinterpret_cast<int32_t*>(Y + kRecSteps * n_s);  // n_s + 1
  const int32_t q = blockIdx.z;
  const int32_t k0 = blockIdx.y * kRecSteps;
  const int nk = min(kRecSteps, N_t - k0);
  if (threadIdx.x == 0) {
    int32_t o = 0;
    for (int i = 0; i < n_s; ++i) {
      loff[i] = o;
      o += nt_q ? nt_q[(int64_t)q * n_s + i] : moff[i + 1] - moff[i];
    }
    loff[n_s] = o;
  }
  __syncthreads();
  const double* c = coeff + coeff_off[q];
  for (int e = threadIdx.x; e < nk * n_s; e += kRecThreads) {
    const int kk = e / n_s, i = e % n_s;
    const int nti = loff[i + 1] - loff[i];
    double y = 0.0;
#pragma unroll 8  // several strided loads in flight; same FMA order
    for (int j = 0; j < nti; ++j) y = fma(Phi_t[(int64_t)(moff[i] + j) * ldt + k0 + kk], c[loff[i] + j], y);
    Y[kk * n_s + i] = y;
  }
  __syncthreads();
  const int64_t x = (int64_t)blockIdx.x * kRecThreads + threadIdx.x;
  if (x >= N_s) return;
  double acc[kRecSteps];
#pragma unroll
  for (int kk = 0; kk < kRecSteps; ++kk) acc[kk] = 0.0;
  for (int i = 0; i < n_s; ++i) {
    const double p = Phi_s[x + (int64_t)i * ldp];
#pragma unroll
    for (int kk = 0; kk < kRecSteps; ++kk) acc[kk] = fma(p, Y[kk * n_s + i], acc[kk]);
  }
  double* o = out + (int64_t)q * ldo * N_t;
#pragma unroll
  for (int kk = 0; kk < kRecSteps; ++kk)
    if (kk < nk) o[x + (int64_t)(k0 + kk) * ldo] = acc[kk];
}

}  // namespace

hipError_t launch_reconstruct(int64_t N_s, int32_t N_t, int32_t n_s, const double* Phi_s, int64_t ldp,
                              const double* Phi_t, int64_t ldt, const int32_t* moff, const int32_t* nt_q, int32_t n_q,
                              const double* coeff, const int64_t* coeff_off, double* out, int64_t ldo,
                              hipStream_t s) {
  if (n_q == 0 || N_s == 0 || N_t == 0) return hipSuccess;
  const size_t lds = sizeof(double) * kRecSteps * n_s + sizeof(int32_t) * (n_s + 1);
  dim3 grid((unsigned)((N_s + kRecThreads - 1) / kRecThreads), (unsigned)((N_t + kRecSteps - 1) / kRecSteps),
            (unsigned)n_q);
  hipLaunchKernelGGL(reconstruct_kernel, grid, dim3(kRecThreads), lds, s, N_s, N_t, n_s, Phi_s, ldp, Phi_t, ldt, moff,
                     nt_q, coeff, coeff_off, out, ldo);
  return hipGetLastError();
}

}  // namespace strom
