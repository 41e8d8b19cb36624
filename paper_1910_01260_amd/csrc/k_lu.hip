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
#include <type_traits>

#include "internal.h"
#include "wave_ops.h"

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

// Wavefront reductions of the device library (DPP based, all lanes active).
extern "C" __device__ float __ockl_wfred_max_f32(float);
extern "C" __device__ double __ockl_wfred_max_f64(double);
extern "C" __device__ double __ockl_wfred_add_f64(double);

__device__ inline float wave_max(float v) { return __ockl_wfred_max_f32(v); }
__device__ inline double wave_max(double v) { return __ockl_wfred_max_f64(v); }

// Block sizes per element type and workgroup size NT: NBO-wide outer blocks are
// factored as NBI-wide sub-panels held in registers; updates run on the matrix
// cores from LDS tiles of RB rows x K and K x CB columns (K <= NBO), the NW waves
// of the workgroup arranged as WR x 2 over the output tile.  NT = 512 runs one
// workgroup per CU; NT = 256 halves the LDS so that two workgroups (two queries)
// share a CU and overlap their latency-bound phases.
template <typename T, int NT>
struct LuCfg;
template <>
struct LuCfg<float, 512> {
  static constexpr int NBO = 128, RB = 128, CB = 64, CHW = 64;
};
template <>
struct LuCfg<double, 512> {
  static constexpr int NBO = 64, RB = 64, CB = 64, CHW = 64;
};
template <>
struct LuCfg<float, 256> {
  static constexpr int NBO = 64, RB = 64, CB = 64, CHW = 64;
};
template <>
struct LuCfg<double, 256> {
  static constexpr int NBO = 64, RB = 64, CB = 32, CHW = 32;
};

constexpr int kLuThreads = 512;  // the default workgroup size

template <typename T, int NT>
constexpr size_t lu_pool_elems() {
  using C = LuCfg<T, NT>;
  constexpr int NW = NT / 64;
  // max of: update tiles ((RB + 2 CB) x (NBO + 4)), the row-permutation staging
  // (2 NBO x CHW, then a position map of up to kMaxWidth ints) and the unit lower
  // block with its inverse (2 NBO x (NBO + 1)) plus the per-wave strips of the
  // triangular product when they do not fit in the first
  constexpr size_t a = (size_t)(C::RB + 2 * C::CB) * (C::NBO + 4);
  constexpr size_t b = (size_t)2 * C::NBO * C::CHW + (kMaxWidth * sizeof(int32_t) + sizeof(T) - 1) / sizeof(T);
  constexpr size_t strips = (size_t)NW * C::NBO * 16;
  constexpr size_t c = (size_t)2 * C::NBO * (C::NBO + 1) + (strips <= (size_t)C::NBO * (C::NBO + 1) ? 0 : strips);
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

// A[r, c] -= sum_{k < K} A[r, k0 + k] A[k0 + k, c] for r in [r_lo, r_hi), c in
// [c_lo, c_hi), on the matrix cores.  A is row-major with leading dimension w.
// The left factor (RB rows x K) and the right factor (K x CB, stored
// transposed) are staged in LDS with the K index permuted so that the four
// K values a lane feeds to four consecutive MFMA steps are contiguous: one
// 128-bit LDS read per operand per four steps.  Each wave owns an
// (RB/4) x (CB/2) block of the output tile in 16 x 16 MFMA tiles, loaded from
// global memory before the staging barrier so their latency overlaps it.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef float4 type;
  static constexpr int per = 4;
};
template <>
struct Vec4<double> {
  typedef double2 type;
  static constexpr int per = 2;
};

template <typename T, int NT>
__device__ __forceinline__ int kperm(int k) {
  constexpr int Q = LuCfg<T, NT>::NBO / 4;
  return (k & 3) * Q + (k >> 2);
}

template <typename T, int NT>
__device__ __forceinline__ void tile_update(T* __restrict__ A, int w, int r_lo, int r_hi, int c_lo, int c_hi, int k0,
                                            int K, T* __restrict__ pool) {
  using C = LuCfg<T, NT>;
  constexpr int NBO = C::NBO, RB = C::RB, CB = C::CB;
  constexpr int WR = NT / 128;  // wave rows over the output tile (two wave columns)
  constexpr int LDK = NBO + 4;  // row stride of the staged operands (16-byte aligned rows)
  constexpr int Q = NBO / 4;
  constexpr int MR = RB / WR / 16, MC = CB / 2 / 16;
  constexpr int PER = Vec4<T>::per;  // K steps per 128-bit read
  constexpr int UPT = NBO * CB / NT;  // right-factor elements staged per thread
  static_assert(NBO * CB % NT == 0 && RB % (16 * WR) == 0, "update tile shape");
  typedef typename Vec4<T>::type VT;
  typedef typename Mfma<T>::v4 v4;
  if (r_lo >= r_hi || c_lo >= c_hi || K <= 0) return;
  T* Ls = pool;                   // RB x LDK
  T* Us0 = pool + RB * LDK;       // CB x LDK, two buffers (transposed right factor)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * (RB / WR);
  const int wc = (wave & 1) * (CB / 2);
  const int ksteps = (K + 3) / 4;
  const int kchunks = (ksteps + PER - 1) / PER;
  for (int rb = r_lo; rb < r_hi; rb += RB) {
    const int nr = min(RB, r_hi - rb);
    // register tiles for the current column tile and its successor
    v4 acc[MR][MC];
    T ur[UPT];
    auto load_acc = [&](int cb, v4 (&dst)[MR][MC]) {
      const int nc = min(CB, c_hi - cb);
#pragma unroll
      for (int x = 0; x < MR; ++x)
#pragma unroll
        for (int y = 0; y < MC; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = wr + 16 * x + Mfma<T>::row(lk, r);
            const int col = wc + 16 * y + li;
            dst[x][y][r] = (row < nr && col < nc) ? A[(int64_t)(rb + row) * w + cb + col] : T(0);
          }
    };
    auto load_u = [&](int cb) {
      const int nc = min(CB, c_hi - cb);
#pragma unroll
      for (int t = 0; t < UPT; ++t) {
        const int e = tid + t * NT;
        const int k = e / CB, j = e % CB;
        ur[t] = (k < K && j < nc) ? A[(int64_t)(k0 + k) * w + cb + j] : T(0);
      }
    };
    auto store_u = [&](T* Us) {
#pragma unroll
      for (int t = 0; t < UPT; ++t) {
        const int e = tid + t * NT;
        const int k = e / CB, j = e % CB;
        Us[j * LDK + kperm<T, NT>(k)] = ur[t];
      }
    };
    __syncthreads();
    load_u(c_lo);
    load_acc(c_lo, acc);
#pragma unroll 8
    for (int e = tid; e < RB * NBO; e += NT) {
      const int i = e / NBO, k = e % NBO;
      Ls[i * LDK + kperm<T, NT>(k)] = (i < nr && k < K) ? A[(int64_t)(rb + i) * w + k0 + k] : T(0);
    }
    store_u(Us0);
    __syncthreads();
    int buf = 0;
    for (int cb = c_lo; cb < c_hi; cb += CB) {
      const int nc = min(CB, c_hi - cb);
      const bool more = cb + CB < c_hi;
      v4 nxt[MR][MC];
      if (more) {  // successor tile in flight while this one runs on the matrix cores
        load_u(cb + CB);
        load_acc(cb + CB, nxt);
      }
      const T* Us = Us0 + buf * CB * LDK;
      for (int kc = 0; kc < kchunks; ++kc) {
        VT av[MR], bv[MC];
#pragma unroll
        for (int x = 0; x < MR; ++x)
          av[x] = *reinterpret_cast<const VT*>(Ls + (wr + 16 * x + li) * LDK + lk * Q + kc * PER);
#pragma unroll
        for (int y = 0; y < MC; ++y)
          bv[y] = *reinterpret_cast<const VT*>(Us + (wc + 16 * y + li) * LDK + lk * Q + kc * PER);
#pragma unroll
        for (int p = 0; p < PER; ++p)
#pragma unroll
          for (int x = 0; x < MR; ++x)
#pragma unroll
            for (int y = 0; y < MC; ++y) {
              const T a = -reinterpret_cast<const T*>(&av[x])[p];
              const T b = reinterpret_cast<const T*>(&bv[y])[p];
              acc[x][y] = Mfma<T>::op(a, b, acc[x][y]);
            }
      }
#pragma unroll
      for (int x = 0; x < MR; ++x)
#pragma unroll
        for (int y = 0; y < MC; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = wr + 16 * x + Mfma<T>::row(lk, r);
            const int col = wc + 16 * y + li;
            if (row < nr && col < nc) A[(int64_t)(rb + row) * w + cb + col] = acc[x][y][r];
          }
      if (more) {
        store_u(Us0 + (buf ^ 1) * CB * LDK);
#pragma unroll
        for (int x = 0; x < MR; ++x)
#pragma unroll
          for (int y = 0; y < MC; ++y) acc[x][y] = nxt[x][y];
      }
      buf ^= 1;
      __syncthreads();
    }
  }
}

// C[r, c] -= sum_{k < K} A[r, k0 + k] A[k0 + k, c] for r in [r_lo, r_hi), c in [c_lo, c_hi),
// for the narrow updates inside a 64-column outer block (K <= 16, at most 16 NCT columns):
// straight from global memory into MFMA registers, without LDS or barriers.  Every wave holds
// the K x (c_hi - c_lo) right factor in the B-operand layout and walks its own 16-row tiles,
// the next tile's loads in flight while the current one is multiplied.  Ends with a barrier.
template <typename T, int NT, int NCT>
__device__ __forceinline__ void narrow_update(T* __restrict__ A, int w, int r_lo, int r_hi, int c_lo, int c_hi, int k0,
                                              int K) {
  typedef typename Mfma<T>::v4 v4;
  constexpr int NW = NT / 64, KS = 4;  // four MFMA k-steps of 4
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  T b[NCT][KS];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int k = 4 * kk + lk, c = c_lo + 16 * ct + li;
      b[ct][kk] = (k < K && c < c_hi) ? A[(int64_t)(k0 + k) * w + c] : T(0);
    }
  auto load_a = [&](int r0, T (&a)[KS]) {
    const int r = r0 + li;
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int k = 4 * kk + lk;
      a[kk] = (r < r_hi && k < K) ? A[(int64_t)r * w + k0 + k] : T(0);
    }
  };
  auto load_c = [&](int r0, v4 (&cc)[NCT]) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = r0 + Mfma<T>::row(lk, rr), col = c_lo + 16 * ct + li;
        cc[ct][rr] = (row < r_hi && col < c_hi) ? A[(int64_t)row * w + col] : T(0);
      }
  };
  const int ntile = (r_hi - r_lo + 15) / 16;
  T a[KS];
  v4 cc[NCT];
  if (wave < ntile) {
    load_a(r_lo + 16 * wave, a);
    load_c(r_lo + 16 * wave, cc);
  }
  for (int t = wave; t < ntile; t += NW) {
    const int r0 = r_lo + 16 * t;
    const bool more = t + NW < ntile;
    T an[KS];
    v4 cn[NCT];
    if (more) {
      load_a(r0 + 16 * NW, an);
      load_c(r0 + 16 * NW, cn);
    }
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) cc[ct] = Mfma<T>::op(-a[kk], b[ct][kk], cc[ct]);
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = r0 + Mfma<T>::row(lk, rr), col = c_lo + 16 * ct + li;
        if (row < r_hi && col < c_hi) A[(int64_t)row * w + col] = cc[ct][rr];
      }
    if (more) {
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) a[kk] = an[kk];
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) cc[ct] = cn[ct];
    }
  }
  __syncthreads();
}

// The same update as one flat sequence of RB x CB tiles, row-block major: the next tile's
// operands are in flight while the current one runs on the matrix cores also across
// row-block boundaries, where the next left-factor block comes from registers instead of a
// fresh global round trip (one extra barrier).  Used by the 64-column FP32 trailing update.
template <typename T, int NT>
__device__ __forceinline__ void tile_update_flat(T* __restrict__ A, int w, int r_lo, int r_hi, int c_lo, int c_hi,
                                                 int k0, int K, T* __restrict__ pool) {
  using C = LuCfg<T, NT>;
  constexpr int NBO = C::NBO, RB = C::RB, CB = C::CB;
  constexpr int WR = NT / 128, LDK = NBO + 4, Q = NBO / 4;
  constexpr int MR = RB / WR / 16, MC = CB / 2 / 16;
  constexpr int PER = Vec4<T>::per, UPT = NBO * CB / NT, LPT = RB * NBO / NT;
  static_assert(NBO * CB % NT == 0 && RB * NBO % NT == 0 && RB % (16 * WR) == 0, "update tile shape");
  typedef typename Vec4<T>::type VT;
  typedef typename Mfma<T>::v4 v4;
  if (r_lo >= r_hi || c_lo >= c_hi || K <= 0) return;
  T* Ls = pool;
  T* Us0 = pool + RB * LDK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave >> 1) * (RB / WR);
  const int wc = (wave & 1) * (CB / 2);
  const int ksteps = (K + 3) / 4;
  const int kchunks = (ksteps + PER - 1) / PER;
  const int ncb = (c_hi - c_lo + CB - 1) / CB;
  const int ntiles = ncb * ((r_hi - r_lo + RB - 1) / RB);
  auto load_acc = [&](int rb, int cb, v4 (&dst)[MR][MC]) {
    const int nr = min(RB, r_hi - rb), nc = min(CB, c_hi - cb);
#pragma unroll
    for (int x = 0; x < MR; ++x)
#pragma unroll
      for (int y = 0; y < MC; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr + 16 * x + Mfma<T>::row(lk, r);
          const int col = wc + 16 * y + li;
          dst[x][y][r] = (row < nr && col < nc) ? A[(int64_t)(rb + row) * w + cb + col] : T(0);
        }
  };
  T ur[UPT], lr[LPT];
  auto load_u = [&](int cb) {
    const int nc = min(CB, c_hi - cb);
#pragma unroll
    for (int t = 0; t < UPT; ++t) {
      const int e = tid + t * NT;
      const int k = e / CB, j = e % CB;
      ur[t] = (k < K && j < nc) ? A[(int64_t)(k0 + k) * w + cb + j] : T(0);
    }
  };
  auto store_u = [&](T* Us) {
#pragma unroll
    for (int t = 0; t < UPT; ++t) {
      const int e = tid + t * NT;
      const int k = e / CB, j = e % CB;
      Us[j * LDK + kperm<T, NT>(k)] = ur[t];
    }
  };
  auto load_l = [&](int rb) {
    const int nr = min(RB, r_hi - rb);
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
      const int e = tid + t * NT;
      const int i = e / NBO, k = e % NBO;
      lr[t] = (i < nr && k < K) ? A[(int64_t)(rb + i) * w + k0 + k] : T(0);
    }
  };
  auto store_l = [&]() {
#pragma unroll
    for (int t = 0; t < LPT; ++t) {
      const int e = tid + t * NT;
      const int i = e / NBO, k = e % NBO;
      Ls[i * LDK + kperm<T, NT>(k)] = lr[t];
    }
  };
  v4 acc[MR][MC];
  __syncthreads();
  load_u(c_lo);
  load_acc(r_lo, c_lo, acc);
  load_l(r_lo);
  store_l();
  store_u(Us0);
  __syncthreads();
  int buf = 0;
  for (int t = 0; t < ntiles; ++t) {
    const int rb = r_lo + (t / ncb) * RB, cb = c_lo + (t % ncb) * CB;
    const int nr = min(RB, r_hi - rb), nc = min(CB, c_hi - cb);
    const bool more = t + 1 < ntiles;
    const int rbn = r_lo + ((t + 1) / ncb) * RB, cbn = c_lo + ((t + 1) % ncb) * CB;
    const bool newrow = more && rbn != rb;
    v4 nxt[MR][MC];
    if (more) {  // successor tile in flight while this one runs on the matrix cores
      load_u(cbn);
      load_acc(rbn, cbn, nxt);
      if (newrow) load_l(rbn);
    }
    const T* Us = Us0 + buf * CB * LDK;
    for (int kc = 0; kc < kchunks; ++kc) {
      VT av[MR], bv[MC];
#pragma unroll
      for (int x = 0; x < MR; ++x)
        av[x] = *reinterpret_cast<const VT*>(Ls + (wr + 16 * x + li) * LDK + lk * Q + kc * PER);
#pragma unroll
      for (int y = 0; y < MC; ++y)
        bv[y] = *reinterpret_cast<const VT*>(Us + (wc + 16 * y + li) * LDK + lk * Q + kc * PER);
#pragma unroll
      for (int p = 0; p < PER; ++p)
#pragma unroll
        for (int x = 0; x < MR; ++x)
#pragma unroll
          for (int y = 0; y < MC; ++y) {
            const T a = -reinterpret_cast<const T*>(&av[x])[p];
            const T b = reinterpret_cast<const T*>(&bv[y])[p];
            acc[x][y] = Mfma<T>::op(a, b, acc[x][y]);
          }
    }
#pragma unroll
    for (int x = 0; x < MR; ++x)
#pragma unroll
      for (int y = 0; y < MC; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = wr + 16 * x + Mfma<T>::row(lk, r);
          const int col = wc + 16 * y + li;
          if (row < nr && col < nc) A[(int64_t)(rb + row) * w + cb + col] = acc[x][y][r];
        }
    if (more) {
      store_u(Us0 + (buf ^ 1) * CB * LDK);
#pragma unroll
      for (int x = 0; x < MR; ++x)
#pragma unroll
        for (int y = 0; y < MC; ++y) acc[x][y] = nxt[x][y];
    }
    buf ^= 1;
    __syncthreads();
    if (newrow) {  // every wave is done with the current left-factor block
      store_l();
      __syncthreads();
    }
  }
}

// Row interchanges piv[0..n) (step i swaps rows base+i and piv[i] >= base+i),
// composed into a list of moves "row dst receives the old content of row src"
// (a position map in LDS: thread 0 applies the swaps, all threads list the changed
// positions), then applied to the columns [c_lo, c_hi) outside
// [skip_lo, skip_hi) by staging the source row segments through LDS with
// coalesced loads and stores.  Uses s_mv (>= 4 n ints).
template <typename T, int NT>
__device__ __forceinline__ void permute_rows(T* __restrict__ A, int w, int base, int n, const int32_t* __restrict__ piv, int c_lo,
                             int c_hi, int skip_lo, int skip_hi, T* __restrict__ pool, int32_t* __restrict__ s_mv,
                             int32_t* s_nmoves) {
  constexpr int CHW = LuCfg<T, NT>::CHW;
  constexpr int NBO = LuCfg<T, NT>::NBO;
  const int tid = threadIdx.x;
  // content of every position base + p of the range the interchanges can touch, after applying
  // them in order (a dense map in the pool, past the row-staging area)
  int32_t* cmap = reinterpret_cast<int32_t*>(pool + 2 * NBO * CHW);
  int32_t* msrc = s_mv;  // moves: (source row, destination row) pairs
  const int span = w - base;
  for (int p = tid; p < span; p += NT) cmap[p] = base + p;
  if (tid == 0) *s_nmoves = 0;
  __syncthreads();
  if (tid == 0) {
    for (int i = 0; i < n; ++i) {
      const int p = piv[i] - base;
      if (p == i) continue;
      const int t = cmap[i];
      cmap[i] = cmap[p];
      cmap[p] = t;
    }
  }
  __syncthreads();
  for (int p = tid; p < span; p += NT) {
    const int c = cmap[p];
    if (c != base + p) {
      const int t = atomicAdd(s_nmoves, 1);
      msrc[2 * t] = c;
      msrc[2 * t + 1] = base + p;
    }
  }
  __syncthreads();
  const int nm = *s_nmoves;
  if (nm == 0) return;
  if constexpr (NBO <= 64) {
    // 64-column blocks: the moved row segments go through registers, whole columns per
    // round (every move of a column is read before any is written, as the moves may form
    // cycles); a round holds up to KR values per thread, so a few moves cover all columns in
    // one or two rounds.  Rounds touch disjoint columns, so only the reads and writes of one
    // round are separated by a barrier.
    constexpr int KR = 16;
    const int cpr = max(1, (KR * NT) / nm);
    for (int cb = c_lo; cb < c_hi; cb += cpr) {
      const int nc = min(cpr, c_hi - cb);
      const int tot = nm * nc;
      T v[KR];
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int e = tid + k * NT;
        const int t = e / nc, col = cb + e % nc;
        v[k] = (e < tot && (col < skip_lo || col >= skip_hi)) ? A[(int64_t)msrc[2 * t] * w + col] : T(0);
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KR; ++k) {
        const int e = tid + k * NT;
        const int t = e / nc, col = cb + e % nc;
        if (e < tot && (col < skip_lo || col >= skip_hi)) A[(int64_t)msrc[2 * t + 1] * w + col] = v[k];
      }
    }
    __syncthreads();
    return;
  }
  for (int cb = c_lo; cb < c_hi; cb += CHW) {
    if (cb + CHW > skip_lo && cb < skip_hi && cb >= skip_lo && cb + CHW <= skip_hi) continue;
    for (int e = tid; e < nm * CHW; e += NT) {
      const int t = e / CHW, j = e % CHW;
      const int col = cb + j;
      if (col < c_hi && (col < skip_lo || col >= skip_hi)) pool[t * CHW + j] = A[(int64_t)msrc[2 * t] * w + col];
    }
    __syncthreads();
    for (int e = tid; e < nm * CHW; e += NT) {
      const int t = e / CHW, j = e % CHW;
      const int col = cb + j;
      if (col < c_hi && (col < skip_lo || col >= skip_hi)) A[(int64_t)msrc[2 * t + 1] * w + col] = pool[t * CHW + j];
    }
    __syncthreads();
  }
}

// The same for at most 64 NT / 64 columns (the block rows inside a 64-column outer block):
// lane c of the waves holds column c_lo + c of the n rows in registers (row loads are
// coalesced across the lanes) and substitutes down it with the unit lower block broadcast
// from LDS; two barriers in all.
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void block_row_solve_narrow(T* __restrict__ A, int w, int r0, int n, int c_lo, int c_hi,
                                                       T* __restrict__ Ls) {
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, k = e % n;
    Ls[i * NMAX + k] = A[(int64_t)(r0 + i) * w + r0 + k];
  }
  __syncthreads();
  const int c = c_lo + tid;
  if (c < c_hi) {
    T x[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) x[i] = i < n ? A[(int64_t)(r0 + i) * w + c] : T(0);
#pragma unroll
    for (int i = 1; i < NMAX; ++i) {
      T acc = x[i];
#pragma unroll
      for (int k = 0; k < i; ++k) acc -= Ls[i * NMAX + k] * x[k];
      x[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < NMAX; ++i)
      if (i < n) A[(int64_t)(r0 + i) * w + c] = x[i];
  }
  __syncthreads();
}

// Rows [r0, r0 + n) <- L^{-1} rows for the columns [c_lo, c_hi), L the unit
// lower n x n block at A[r0.., r0..] (n <= NMAX <= 32).  Column chunks are
// staged through LDS with coalesced row-segment loads; each thread then
// substitutes down one column in LDS; the chunk is stored back coalesced.
template <typename T, int NMAX, int NT>
__device__ __forceinline__ void block_row_solve(T* __restrict__ A, int w, int r0, int n, int c_lo, int c_hi,
                                                T* __restrict__ Ls, T* __restrict__ pool) {
  constexpr int CW = (64 * 1024) / (sizeof(T) * NMAX) < NT ? (64 * 1024) / (sizeof(T) * NMAX) : NT;
  static_assert((size_t)NMAX * CW <= lu_pool_elems<T, NT>(), "block-row staging exceeds the pool");
  const int tid = threadIdx.x;
  for (int e = tid; e < n * n; e += NT) {
    const int i = e / n, k = e % n;
    Ls[i * NMAX + k] = A[(int64_t)(r0 + i) * w + r0 + k];
  }
  for (int cb = c_lo; cb < c_hi; cb += CW) {
    const int nc = min(CW, c_hi - cb);
    __syncthreads();
#pragma unroll 4
    for (int e = tid; e < n * CW; e += NT) {
      const int i = e / CW, j = e % CW;
      if (j < nc) pool[i * CW + j] = A[(int64_t)(r0 + i) * w + cb + j];
    }
    __syncthreads();
    if (tid < nc) {
      // one column per thread (column-major in LDS, conflict free); the inner products are
      // unrolled so that their LDS reads are issued together
      for (int c = 1; c < n; ++c) {
        T acc = pool[c * CW + tid];
#pragma unroll 8
        for (int k = 0; k < c; ++k) acc -= Ls[c * NMAX + k] * pool[k * CW + tid];
        pool[c * CW + tid] = acc;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int e = tid; e < n * CW; e += NT) {
      const int i = e / CW, j = e % CW;
      if (j < nc) A[(int64_t)(r0 + i) * w + cb + j] = pool[i * CW + j];
    }
  }
  __syncthreads();
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = B .. E-1.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Inverse of the unit lower triangular n x n block L (n <= NB, rows and columns
// from n to NB treated as the identity) into X, both in LDS with leading
// dimension ld; X is written in full (zeros above the diagonal).  Blocked in
// 32 x 32 blocks: the diagonal blocks are inverted one per wave (lane j solves
// for column j), then block row bi of the inverse follows from
// X[bi][bj] = -X[bi][bi] * sum_{bj <= k < bi} L[bi][k] X[k][bj] for all bj < bi
// at once, with the whole workgroup on the products.
template <typename T, int NB, int NT>
__device__ __noinline__ void unit_lower_inverse(const T* __restrict__ L, T* __restrict__ X, int ld, int n) {
  constexpr int SB = 32, NSB = NB / SB;
  constexpr int PER = (NSB > 1 ? (NSB - 1) * SB * SB : 1) / NT + 1;  // outputs per thread per block row
  static_assert(NB % SB == 0 && NSB <= NT / 64, "inverse blocking");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto Lv = [&](int i, int k) -> T { return (i < n && k < n) ? L[i * ld + k] : T(0); };
  // 1. diagonal blocks
  if (wave < NSB && lane < SB) {
    // lane j solves L x = e_j into column j of the block (x_k = 0 for k < j follows from
    // the recurrence); the inner products are unrolled so that their LDS reads issue together
    const int b0 = wave * SB, j = lane;
    for (int i = 0; i < SB; ++i) {
      T acc = i == j ? T(1) : T(0);
#pragma unroll 8
      for (int k = 0; k < i; ++k) acc -= Lv(b0 + i, b0 + k) * X[(b0 + k) * ld + b0 + j];
      X[(b0 + i) * ld + b0 + j] = acc;
    }
  }
  __syncthreads();
  // 2. block rows below the diagonal
  for (int bi = 1; bi < NSB; ++bi) {
    const int cnt = bi * SB * SB;
    // S[bi][bj] = sum_{bj <= k < bi} L[bi][k] X[k][bj], staged in the X[bi][bj] slots
    for (int e = tid; e < cnt; e += NT) {
      const int bj = e / (SB * SB), i = (e / SB) % SB, j = e % SB;
      const int r = bi * SB + i, c = bj * SB + j;
      T acc = T(0);
#pragma unroll 8
      for (int k = bj * SB; k < bi * SB; ++k) acc += Lv(r, k) * X[k * ld + c];  // X[k][c] = 0 for k < c
      X[r * ld + c] = acc;
    }
    __syncthreads();
    T out[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      out[t] = T(0);
      if (e < cnt) {
        const int bj = e / (SB * SB), i = (e / SB) % SB, j = e % SB;
        const T* Dinv = X + (bi * SB + i) * ld + bi * SB;   // row i of X[bi][bi]
        const T* Sc = X + (bi * SB) * ld + bj * SB + j;      // column j of S[bi][bj]
        T acc = T(0);
        for (int k = 0; k <= i; ++k) acc += Dinv[k] * Sc[k * ld];  // X[bi][bi] is lower triangular
        out[t] = -acc;
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * NT;
      if (e < cnt) {
        const int bj = e / (SB * SB), i = (e / SB) % SB, j = e % SB;
        X[(bi * SB + i) * ld + bj * SB + j] = out[t];
      }
    }
    __syncthreads();
  }
  // zeros above the diagonal blocks
  for (int e = tid; e < NB * NB; e += NT) {
    const int i = e / NB, j = e % NB;
    if (j / SB > i / SB) X[i * ld + j] = T(0);
  }
  __syncthreads();
}

// One workgroup factors one query at a time (persistent, work queue).  Row r of
// the query is owned by thread r % NT in register slot r / NT (R slots) while
// its sub-panel is factored.  Pivoting is LAPACK-style partial pivoting; P[i]
// receives the row swapped with row i at step i.  Interchanges are applied
// inside the current outer block and to the columns right of it; columns left
// of the block are never swapped, so the solve interleaves each block's
// interchanges with its forward-substitution step.
template <typename T, int R, int NBI, int NT>
__global__ __launch_bounds__(NT, 2) void lu_kernel(int32_t n_q, Plan plan, T* __restrict__ mats,
                                                        int32_t* __restrict__ piv) {
  using C = LuCfg<T, NT>;
  constexpr int NBO = C::NBO;
  constexpr int BLOCK = NT, NW = NT / 64;
  static_assert(NBO % NBI == 0 && NBI <= 32, "block shape");
  // Carve-up of the dynamic LDS pool (lu_pool_elems<T, NT>() elements of T), phase by phase;
  // phases that reuse it are separated by barriers (each helper ends with one).
  constexpr size_t kPoolBytes = sizeof(T) * lu_pool_elems<T, NT>();
  // sub-panel pivot bookkeeping: pos_of and row_at, 2 (w - i0) ints with w <= R NT
  static_assert(2 * (size_t)R * NT * sizeof(int32_t) <= kPoolBytes, "pos_of / row_at exceed the pool");
  // permute_rows: up to 2 NBO staged row segments of CHW elements, then a position map of w ints
  static_assert(sizeof(T) * 2 * NBO * C::CHW + sizeof(int32_t) * (size_t)R * NT <= kPoolBytes,
                "row staging / position map exceed the pool");
  // tile_update(_flat): the left factor (RB x (NBO + 4)) and two right-factor buffers (CB x (NBO + 4))
  static_assert(sizeof(T) * (size_t)(C::RB + 2 * C::CB) * (NBO + 4) <= kPoolBytes, "update tiles exceed the pool");
  // U12: the unit lower block and its inverse (2 NBO x (NBO + 1)), and the per-wave B strips
  static_assert(sizeof(T) * 2 * (size_t)NBO * (NBO + 1) <= kPoolBytes, "L11 / Linv exceed the pool");
  static_assert(NBO <= 64 || (size_t)NW * NBO * 16 <= (size_t)NBO * (NBO + 1) ||
                    sizeof(T) * ((size_t)2 * NBO * (NBO + 1) + (size_t)NW * NBO * 16) <= kPoolBytes,
                "U12 strips exceed the pool");
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* pool = reinterpret_cast<T*>(lds_raw);
  __shared__ T s_cand[2][NW][NBI];
  __shared__ T s_redv[2][NW];
  __shared__ int32_t s_redr[2][NW];
  __shared__ int32_t s_piv[NBO];
  __shared__ int32_t s_mv[4 * NBO + 8];  // permute_rows: up to 2 n moves (src, dst)
  __shared__ int32_t s_nm;
  __shared__ T s_L[32 * 32];
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

    for (int p0 = 0; p0 < w; p0 += NBO) {
      const int nbo = min(NBO, w - p0);
      // ===================== factor the outer block, one sub-panel at a time
      for (int i0 = p0; i0 < p0 + nbo; i0 += NBI) {
        const int nbi = min(NBI, p0 + nbo - i0);
        T v[R][NBI];
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int r = tid + s * BLOCK;
          const bool live = r >= i0 && r < w;
#pragma unroll
          for (int c = 0; c < NBI; ++c) v[s][c] = (live && c < nbi) ? A[(int64_t)r * w + i0 + c] : T(0);
        }
        // Column steps, unrolled at compile time so that every register index is a
        // constant.  Pivoting is by index: a pivot row stays in its thread's registers
        // and is only marked done; thread 0 tracks the LAPACK interchange sequence
        // (position of every row of the panel, in LDS) and the rows are written to
        // their final positions afterwards.
        int32_t* pos_of = reinterpret_cast<int32_t*>(pool);   // row -> current position (offset i0)
        int32_t* row_at = pos_of + (w - i0);                  // position -> row (offset i0)
        for (int t = tid; t < w - i0; t += BLOCK) {
          pos_of[t] = i0 + t;
          row_at[t] = i0 + t;
        }
        bool done[R];
#pragma unroll
        for (int s = 0; s < R; ++s) done[s] = false;
        static_for<0, NBI>([&](auto CC) {
          constexpr int c = decltype(CC)::value;
          if (c >= nbi) return;
          constexpr int buf = c & 1;
          const int diag = i0 + c;
          T best = T(-1);
          int32_t brow = 0x7fffffff;
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const int r = tid + s * BLOCK;
            if (r >= i0 && r < w && !done[s]) {
              T a = v[s][c] < T(0) ? -v[s][c] : v[s][c];
              a = a == a ? a : T(0);  // a NaN entry never wins over a number
              if (a > best) { best = a; brow = r; }
            }
          }
          const T wbest = wave_max(best);
          const int32_t wrow = __ockl_wfred_min_i32(best == wbest ? brow : 0x7fffffff);
          // One barrier per column: every wave publishes its best value, row index and the
          // whole candidate row.
          if (lane == 0) { s_redv[buf][wave] = wbest; s_redr[buf][wave] = wrow; }
#pragma unroll
          for (int s = 0; s < R; ++s) {
            const int r = tid + s * BLOCK;
            if (r == wrow) {
#pragma unroll
              for (int k = 0; k < NBI; ++k) s_cand[buf][wave][k] = v[s][k];
            }
          }
          __syncthreads();
          // all candidates are read first, then reduced branch-free
          T cv[NW];
          int32_t cr[NW];
#pragma unroll
          for (int k = 0; k < NW; ++k) {
            cv[k] = s_redv[buf][k];
            cr[k] = s_redr[buf][k];
          }
          best = cv[0];
          brow = cr[0];
#pragma unroll
          for (int k = 1; k < NW; ++k) {
            const bool bt = cv[k] > best || (cv[k] == best && cr[k] < brow);
            best = bt ? cv[k] : best;
            brow = bt ? cr[k] : brow;
          }
          const int32_t prow = brow;  // a live row: every live entry compares >= 0 > -1
          // the winning row belongs to thread prow % BLOCK, i.e. to wave (prow % BLOCK) / 64
          const T* urow = s_cand[buf][(prow & (BLOCK - 1)) >> 6];
          if (!(best > T(0)) && zero_piv == 0) zero_piv = diag + 1;  // exactly zero pivot
#pragma unroll
          for (int s = 0; s < R; ++s)
            if (tid + s * BLOCK == prow) done[s] = true;
          if (tid == 0) {
            // LAPACK pivot index: the current position of the pivot row; then exchange
            // the contents of that position and of position diag
            const int pp = pos_of[prow - i0];
            const int other = row_at[c];
            s_piv[diag - p0] = pp;
            P[diag] = pp;
            row_at[pp - i0] = other;
            pos_of[other - i0] = pp;
            row_at[c] = prow;
            pos_of[prow - i0] = diag;
          }
          const T d = urow[c];
          const T inv = (d != T(0)) ? T(1) / d : T(0);
          T um[NBI];
#pragma unroll
          for (int k = c + 1; k < NBI; ++k) um[k] = urow[k];
#pragma unroll
          for (int s = 0; s < R; ++s) {
            if (s * BLOCK >= w) continue;  // slot empty for every thread (uniform)
            const int r = tid + s * BLOCK;
            if (r >= i0 && r < w && !done[s]) {
              const T l = v[s][c] * inv;
              v[s][c] = l;
#pragma unroll
              for (int k = c + 1; k < NBI; ++k) v[s][k] -= l * um[k];
            }
          }
        });
        __syncthreads();
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const int r = tid + s * BLOCK;
          if (r >= i0 && r < w) {
            const int64_t dst = pos_of[r - i0];
#pragma unroll
            for (int c = 0; c < NBI; ++c)
              if (c < nbi) A[dst * w + i0 + c] = v[s][c];
          }
        }
        __syncthreads();
        // this sub-panel's interchanges on the other columns of the outer block
        permute_rows<T, NT>(A, w, i0, nbi, s_piv + (i0 - p0), p0, p0 + nbo, i0, i0 + nbi, pool, s_mv, &s_nm);
        const int cr = i0 + nbi;
        if (cr < p0 + nbo) {
          // pivot rows: solve against the sub-panel's unit lower block; rows below: rank-nbi update
          // (64-column blocks: register forms while the column's rows fit in 64 bytes)
          if constexpr (NBO <= 64 && NBI * sizeof(T) <= 64)
            block_row_solve_narrow<T, NBI, NT>(A, w, i0, nbi, cr, p0 + nbo, s_L);
          else
            block_row_solve<T, NBI, NT>(A, w, i0, nbi, cr, p0 + nbo, s_L, pool);
          if constexpr (NBO <= 64 && NBI <= 16)
            narrow_update<T, NT, (NBO - NBI + 15) / 16>(A, w, cr, w, cr, p0 + nbo, i0, nbi);
          else
            tile_update<T, NT>(A, w, cr, w, cr, p0 + nbo, i0, nbi, pool);
        }
      }
      const int c0 = p0 + nbo;
      if (c0 >= w) {
        __syncthreads();
        break;
      }
      // ===================== the block's interchanges on the columns right of it
      permute_rows<T, NT>(A, w, p0, nbo, s_piv, c0, w, 0, 0, pool, s_mv, &s_nm);
      // ===================== U12 = L11^{-1} A12: explicit inverse of the unit lower
      // block (one column per thread, in LDS), then a triangular product on the
      // matrix cores in 16-column strips per wave (zero blocks of the inverse skipped)
      {
        constexpr int LDL = NBO + 1;
        T* L11 = pool;
        T* Linv = pool + NBO * LDL;
        for (int e = tid; e < nbo * nbo; e += BLOCK) {
          const int i = e / nbo, k = e % nbo;
          L11[i * LDL + k] = A[(int64_t)(p0 + i) * w + p0 + k];
        }
        __syncthreads();
        unit_lower_inverse<T, NBO, NT>(L11, Linv, LDL, nbo);
        typedef typename Mfma<T>::v4 v4;
        const int li = lane & 15, lk = lane >> 4;
        const int n2 = w - c0;
        if constexpr (NBO <= 64) {
          // NBO = 64: this wave's 16-column strips of A12, read straight into the B-operand
          // layout of the MFMA (lane (li, lk) holds rows 4 kk + lk of column li); the next
          // strip's loads are in flight while the current one is multiplied
          constexpr int KB = NBO / 4;
          T bcur[KB], bnxt[KB];
          auto load_b = [&](int st, T (&b)[KB]) {
            const int col = c0 + st * 16 + li;
            const bool ok = st * 16 < n2 && col < w;
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
              const int k = 4 * kk + lk;
              b[kk] = (ok && k < nbo) ? A[(int64_t)(p0 + k) * w + col] : T(0);
            }
          };
          load_b(wave, bcur);
          for (int st = wave; st * 16 < n2; st += NW) {
            load_b(st + NW, bnxt);
            const int col = c0 + st * 16 + li;
#pragma unroll 1
            for (int it = 0; it * 16 < nbo; ++it) {
              v4 acc = {T(0), T(0), T(0), T(0)};
              const T* Lrow = Linv + (16 * it + li) * LDL + lk;
              const int kend = 4 * it + 4;  // the inverse is lower triangular
#pragma unroll
              for (int kk = 0; kk < KB; ++kk)
                if (kk < kend) acc = Mfma<T>::op(Lrow[4 * kk], bcur[kk], acc);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = 16 * it + Mfma<T>::row(lk, r);
                if (row < nbo && col < w) A[(int64_t)(p0 + row) * w + col] = acc[r];
              }
            }
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) bcur[kk] = bnxt[kk];
          }
        } else {
          // NBO = 128: this wave's NBO x 16 strip staged in LDS (in the now free L11 area when
          // all strips fit there, otherwise after the inverse; the pool is sized for either case)
          constexpr bool kStripsInL11 = NW * NBO * 16 <= NBO * LDL;
          T* Sb = (kStripsInL11 ? L11 : Linv + NBO * LDL) + wave * NBO * 16;
          for (int st = wave; st * 16 < n2; st += NW) {
            const int cs = c0 + st * 16;
            for (int e = lane; e < NBO * 16; e += 64) {
              const int k = e >> 4, j = e & 15;
              Sb[e] = (k < nbo && cs + j < w) ? A[(int64_t)(p0 + k) * w + cs + j] : T(0);
            }
            __builtin_amdgcn_wave_barrier();
            const int col = cs + li;
#pragma unroll 1
            for (int it = 0; it * 16 < nbo; ++it) {
              v4 acc = {T(0), T(0), T(0), T(0)};
              const T* Lrow = Linv + (16 * it + li) * LDL + lk;
              const T* Bcol = Sb + lk * 16 + li;
              const int kend = 4 * it + 4;  // the inverse is lower triangular
              for (int kk = 0; kk < kend; ++kk) acc = Mfma<T>::op(Lrow[4 * kk], Bcol[kk * 64], acc);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = 16 * it + Mfma<T>::row(lk, r);
                if (row < nbo && col < w) A[(int64_t)(p0 + row) * w + col] = acc[r];
              }
            }
            __builtin_amdgcn_wave_barrier();
          }
        }
        __syncthreads();
      }
      // ===================== trailing update A22 -= L21 U12 with K = nbo
      if constexpr (NBO <= 64 && sizeof(T) == 4)
        tile_update_flat<T, NT>(A, w, c0, w, c0, w, p0, nbo, pool);
      else
        tile_update<T, NT>(A, w, c0, w, c0, w, p0, nbo, pool);
    }
    if (tid == 0 && zero_piv) plan.info[q] = zero_piv;
  }
}

// Solve (P^T L U) x = b for each active query: permute b, forward
// substitution with the unit lower factor, back substitution with the upper
// factor, in 64-row blocks (diagonal block by one wave, the rows below or above
// it updated with 16 lanes per row).  Accumulation in FP64 whatever T is.
constexpr int kSolveBS = 64;
constexpr int kSolveThreads = 512;
constexpr int kMaxSolveNbo = 128;

// Groups of 4 rows whose loads a wave issues together; with the next groups in flight while
// the current ones are reduced this keeps the solve within 128 VGPRs (two workgroups per CU).
template <typename T>
constexpr int solve_row_groups() {
  return sizeof(T) == 4 ? 4 : 3;
}

// Rows [r, r + 4 solve_row_groups<T>()) of this wave's share of an update against the block
// columns [b0, b0 + nbk): a row is spread over the 16 lanes of a DPP row (lane c holds
// columns c, c + 16, c + 32, c + 48), so one load instruction covers 4 rows.
template <typename T>
struct SolveRows {
  T a[solve_row_groups<T>()][4];
  __device__ __forceinline__ void fetch(const T* __restrict__ A, int w, int b0, int nbk, int r, int r_end) {
    const int lane = threadIdx.x & 63, sub = lane >> 4, c = lane & 15;
#pragma unroll
    for (int u = 0; u < solve_row_groups<T>(); ++u) {
      const int rr = r + 4 * u + sub;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = c + 16 * j;
        a[u][j] = (rr < r_end && col < nbk) ? A[(int64_t)rr * w + b0 + col] : T(0);
      }
    }
  }
  // y[rr] -= row . y_block with one 16-lane reduction per 4 rows; the whole wave must be active
  __device__ __forceinline__ void reduce(const double (&yc)[4], int r, int r_end, double* y) const {
    const int lane = threadIdx.x & 63, sub = lane >> 4, c = lane & 15;
#pragma unroll
    for (int u = 0; u < solve_row_groups<T>(); ++u) {
      double p = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) p += (double)a[u][j] * yc[j];
      p = row16_sum(p);
      const int rr = r + 4 * u + sub;
      if (c == 0 && rr < r_end) y[rr] -= p;
    }
  }
};

// The factor data never depends on the right-hand side, so its loads run ahead of the
// serial chain: the next diagonal block is fetched into registers during the current
// block's update, and each wave's first row group of an update is fetched before the
// diagonal solve that produces the y values it multiplies.
template <typename T>
__global__ __launch_bounds__(kSolveThreads) void lu_solve_kernel(int32_t n_q, Plan plan, const T* __restrict__ mats,
                                                                 const int32_t* __restrict__ piv,
                                                                 const double* __restrict__ b, double* __restrict__ x,
                                                                 int accumulate, const int32_t* __restrict__ active,
                                                                 int NBO) {
  // NBO: the factorisation's outer block (a multiple of kSolveBS, at most kMaxSolveNbo)
  constexpr int NW = kSolveThreads / 64, ROWS = 4 * solve_row_groups<T>(), STRIDE = NW * ROWS;
  constexpr int DPT = kSolveBS * kSolveBS / kSolveThreads;  // diagonal-block entries per thread
  extern __shared__ __align__(16) double y[];
  __shared__ T dblk[kSolveBS][kSolveBS + 1];
  const int32_t q = blockIdx.x;
  if (plan.info[q] != 0) return;
  if (active && !active[q]) return;
  const int32_t w = plan.width[q];
  if (w == 0) return;
  const int64_t off = plan.coeff_off[q];
  const T* A = mats + plan.mat_off[q];
  const int32_t* P = piv + off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  T dreg[DPT];
  auto fetch_dblk = [&](int b0) {
    const int nbk = min(kSolveBS, w - b0);
#pragma unroll
    for (int t = 0; t < DPT; ++t) {
      const int e = tid + t * kSolveThreads, i = e / kSolveBS, k = e % kSolveBS;
      dreg[t] = (i < nbk && k < nbk) ? A[(int64_t)(b0 + i) * w + b0 + k] : T(0);
    }
  };
  auto store_dblk = [&]() {
#pragma unroll
    for (int t = 0; t < DPT; ++t) {
      const int e = tid + t * kSolveThreads;
      dblk[e / kSolveBS][e % kSolveBS] = dreg[t];
    }
  };
  // y values of the columns b0 + c + 16 j held by this lane for the row updates
  auto y_cols = [&](int b0, int nbk, double (&yc)[4]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = (lane & 15) + 16 * j;
      yc[j] = col < nbk ? y[b0 + col] : 0.0;
    }
  };
  SolveRows<T> rows;
  for (int c = tid; c < w; c += kSolveThreads) y[c] = b[off + c];
  fetch_dblk(0);
  __syncthreads();
  // forward substitution, unit lower triangular, each outer block's interchanges first
  for (int b0 = 0; b0 < w; b0 += kSolveBS) {
    const int nbk = min(kSolveBS, w - b0);
    if (b0 % NBO == 0 && wave == 0) {
      // the block's interchanges, in order, by lane 0; a 64-pivot chunk without any
      // interchange (the common case) costs one ballot
      const int nblk = min(NBO, w - b0);
      for (int i0 = 0; i0 < nblk; i0 += 64) {
        const int i = i0 + lane;
        const int p = i < nblk ? P[b0 + i] : b0 + i;
        uint64_t m = __ballot(p != b0 + i);
        while (m) {
          const int l = __builtin_ctzll(m);
          m &= m - 1;
          const int pl = __builtin_amdgcn_readlane(p, l);
          if (lane == 0) {
            const double t = y[b0 + i0 + l];
            y[b0 + i0 + l] = y[pl];
            y[pl] = t;
          }
        }
      }
    }
    store_dblk();
    const int r0 = b0 + nbk + wave * ROWS;
    rows.fetch(A, w, b0, nbk, r0, w);
    __syncthreads();
    if (wave == 0) {
      // lane i holds y[b0 + i]; step k broadcasts y[b0 + k] and updates the lanes below it.
      // The block's entries are read from LDS eight steps ahead of their use.
      double yi = lane < nbk ? y[b0 + lane] : 0.0;
      for (int k0 = 0; k0 < nbk; k0 += 8) {
        double lk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) lk[u] = (double)dblk[lane][k0 + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int k = k0 + u;
          const double yk = readlane_d(yi, k);
          if (lane > k && lane < nbk) yi -= lk[u] * yk;
        }
      }
      if (lane < nbk) y[b0 + lane] = yi;
    }
    if (b0 + kSolveBS < w) fetch_dblk(b0 + kSolveBS);
    __syncthreads();
    double yc[4];
    y_cols(b0, nbk, yc);
    for (int r = r0; r < w; r += STRIDE) {
      SolveRows<T> nxt;  // the wave's next row group is in flight while this one is reduced
      if (r + STRIDE < w) nxt.fetch(A, w, b0, nbk, r + STRIDE, w);
      rows.reduce(yc, r, w, y);
      rows = nxt;
    }
    __syncthreads();
  }
  // back substitution, upper triangular (reciprocals of the diagonal taken off the serial chain)
  const int last0 = ((w - 1) / kSolveBS) * kSolveBS;
  fetch_dblk(last0);
  for (int b0 = last0; b0 >= 0; b0 -= kSolveBS) {
    const int nbk = min(kSolveBS, w - b0);
    store_dblk();
    const int r0 = wave * ROWS;
    rows.fetch(A, w, b0, nbk, r0, b0);
    __syncthreads();
    if (wave == 0) {
      double yi = lane < nbk ? y[b0 + lane] : 0.0;
      const double dinv = lane < nbk ? 1.0 / (double)dblk[lane][lane] : 0.0;
      for (int k0 = ((nbk - 1) / 8) * 8; k0 >= 0; k0 -= 8) {
        double uk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) uk[u] = (double)dblk[lane][k0 + u];
#pragma unroll
        for (int u = 7; u >= 0; --u) {
          const int k = k0 + u;
          if (k >= nbk) continue;
          const double yk = readlane_d(yi, k) * readlane_d(dinv, k);
          if (lane == k) yi = yk;
          if (lane < k) yi -= uk[u] * yk;
        }
      }
      if (lane < nbk) y[b0 + lane] = yi;
    }
    if (b0 > 0) fetch_dblk(b0 - kSolveBS);
    __syncthreads();
    double yc[4];
    y_cols(b0, nbk, yc);
    for (int r = r0; r < b0; r += STRIDE) {
      SolveRows<T> nxt;
      if (r + STRIDE < b0) nxt.fetch(A, w, b0, nbk, r + STRIDE, b0);
      rows.reduce(yc, r, b0, y);
      rows = nxt;
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

template <typename T, int R, int NBI, int NT>
hipError_t lu_go(int32_t n_q, Plan plan, void* mats, int32_t* piv, int32_t n_max, hipStream_t s) {
  // the R register slots of the NT threads must cover every row of the widest query
  if (n_max > R * NT) return hipErrorInvalidValue;
  const size_t lds = sizeof(T) * lu_pool_elems<T, NT>();
  if (!g_capturing) {
    const hipError_t e = hipFuncSetAttribute((const void*)lu_kernel<T, R, NBI, NT>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  // NT = 512: one workgroup per CU; NT = 256: two (their LDS fits together)
  const int grid = max(1, min(n_q, (512 / NT) * device_cus()));
  hipLaunchKernelGGL((lu_kernel<T, R, NBI, NT>), dim3(grid), dim3(NT), lds, s, n_q, plan, (T*)mats, piv);
  return hipGetLastError();
}

}  // namespace

// Batched-LU configurations.  Widths up to 1536: variant 0 = 512 threads, 3 row
// slots, the widest register sub-panel (32 FP32 / 16 FP64 columns); variant 1 = the
// same with half-width sub-panels; variant 2 = 256 threads, 6 row slots, 64-column
// outer blocks, two workgroups per CU.  Widths up to 4096: variants 0 and 1 with 8 row
// slots.  Which is fastest depends on the batch; the autotuner times them.
int lu_variant_count(int32_t prec, int32_t n_max) {
  (void)prec;
  if (n_max <= 3 * kLuThreads) return 3;
  return n_max <= 8 * kLuThreads ? 2 : 0;
}

// Outer block width of a configuration (the triangular solves apply the row
// interchanges block by block, so they need it).
int lu_outer_block(int32_t prec, int32_t n_max, int variant) {
  if (n_max <= 3 * kLuThreads && variant == 2)
    return prec == ST_F64 ? LuCfg<double, 256>::NBO : LuCfg<float, 256>::NBO;
  return prec == ST_F64 ? LuCfg<double, 512>::NBO : LuCfg<float, 512>::NBO;
}

hipError_t launch_lu(int32_t n_q, Plan plan, int32_t prec, void* mats, int32_t* piv, int32_t n_max, int variant,
                     hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  const bool f64 = prec == ST_F64;
  if (n_max <= 3 * kLuThreads) {
    if (variant == 2)
      return f64 ? lu_go<double, 6, 8, 256>(n_q, plan, mats, piv, n_max, s) : lu_go<float, 6, 16, 256>(n_q, plan, mats, piv, n_max, s);
    if (variant == 1)
      return f64 ? lu_go<double, 3, 8, 512>(n_q, plan, mats, piv, n_max, s) : lu_go<float, 3, 16, 512>(n_q, plan, mats, piv, n_max, s);
    return f64 ? lu_go<double, 3, 16, 512>(n_q, plan, mats, piv, n_max, s) : lu_go<float, 3, 32, 512>(n_q, plan, mats, piv, n_max, s);
  }
  if (n_max <= 8 * kLuThreads) {
    if (variant == 1)
      return f64 ? lu_go<double, 8, 4, 512>(n_q, plan, mats, piv, n_max, s) : lu_go<float, 8, 8, 512>(n_q, plan, mats, piv, n_max, s);
    return f64 ? lu_go<double, 8, 8, 512>(n_q, plan, mats, piv, n_max, s) : lu_go<float, 8, 16, 512>(n_q, plan, mats, piv, n_max, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lu_solve(int32_t n_q, Plan plan, int32_t prec, const void* mats, const int32_t* piv, const double* b,
                           double* x, int accumulate, const int32_t* active, int32_t n_max, int nbo, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  if (nbo <= 0 || nbo % kSolveBS != 0 || nbo > kMaxSolveNbo) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (size_t)n_max;
  if (!g_capturing) {
    const hipError_t e = hipFuncSetAttribute(prec == ST_F64 ? (const void*)lu_solve_kernel<double>
                                                            : (const void*)lu_solve_kernel<float>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (prec == ST_F64) {
    hipLaunchKernelGGL(lu_solve_kernel<double>, dim3(n_q), dim3(kSolveThreads), lds, s, n_q, plan,
                       (const double*)mats, piv, b, x, accumulate, active, nbo);
  } else {
    hipLaunchKernelGGL(lu_solve_kernel<float>, dim3(n_q), dim3(kSolveThreads), lds, s, n_q, plan, (const float*)mats,
                       piv, b, x, accumulate, active, nbo);
  }
  return hipGetLastError();
}

}  // namespace strom
