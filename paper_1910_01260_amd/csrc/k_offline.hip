// Offline reduced operators on gfx950:
//   * projection of the affine operator terms onto the spatial basis,
//     Ahat_q = Phi_s^T (A_q Phi_s) (Sec. 3.1, Eq. (galerkin)), as a CSR SpMM
//     against the row-major tall-skinny basis followed by a split-K
//     tall-skinny product;
//   * the mu-independent temporal contractions of the block formulas
//     (Sec. 4.3, Eq. (ij-block-matrix), (j-block-vector)): the dt-weighted
//     temporal Gram T, the per-mode blocks K_i, the input weights Wf and
//     the first-step values P1.
#include "internal.h"

// wavefront sum of the device library (DPP based, all lanes active)
extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace strom {
namespace {

constexpr int kTile = 32;
constexpr int kTile64 = 64;  // output tile of the register-blocked tall-skinny product

__global__ void index_tables_kernel(ModeTable mt, MutRomView rom) {
  // one workgroup; n_s <= kMaxModes
  __shared__ int32_t s_off[kMaxModes + 1];
  const int n_s = mt.n_s;
  if (threadIdx.x == 0) {
    int32_t o = 0;
    int64_t ko = 0;
    for (int i = 0; i < n_s; ++i) {
      s_off[i] = o;
      rom.moff[i] = o;
      rom.koff[i] = ko;
      o += mt.nt[i];
      ko += (int64_t)mt.nt[i] * mt.nt[i];
    }
    s_off[n_s] = o;
    rom.moff[n_s] = o;
    rom.koff[n_s] = ko;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_s; i += blockDim.x)
    for (int j = s_off[i]; j < s_off[i + 1]; ++j) rom.mode[j] = i;
}

// dst (rows x cols, row-major) = src (rows x cols, column-major, leading dimension ld)
__global__ void transpose_kernel(const double* __restrict__ src, int64_t rows, int32_t cols, int64_t ld,
                                 double* __restrict__ dst) {
  __shared__ double tile[kTile][kTile + 1];
  const int64_t r0 = (int64_t)blockIdx.x * kTile;
  const int c0 = blockIdx.y * kTile;
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 32 x 8
  for (int cc = ty; cc < kTile; cc += 8) {
    int64_t r = r0 + tx;
    int c = c0 + cc;
    tile[cc][tx] = (r < rows && c < cols) ? src[r + (int64_t)c * ld] : 0.0;
  }
  __syncthreads();
  for (int rr = ty; rr < kTile; rr += 8) {
    int64_t r = r0 + rr;
    int c = c0 + tx;
    if (r < rows && c < cols) dst[r * cols + c] = tile[tx][rr];
  }
}

// Yr (N x p, row-major) = A (CSR, N x N) * Xr (N x p, row-major); one wave per row,
// lanes across the p columns so every gathered basis row is read contiguously.
__global__ __launch_bounds__(256) void spmm_rowmajor_kernel(int32_t n_rows, const int32_t* __restrict__ row_ptr,
                                                           const int32_t* __restrict__ col_idx,
                                                           const double* __restrict__ val,
                                                           const double* __restrict__ Xr, int32_t p,
                                                           double* __restrict__ Yr) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= n_rows) return;
  const int32_t b = row_ptr[row], e = row_ptr[row + 1];
  for (int m0 = 0; m0 < p; m0 += 64) {
    const int m = m0 + lane;
    double acc = 0.0;
    if (m < p) {
      for (int32_t z = b; z < e; ++z) acc = fma(val[z], Xr[(int64_t)col_idx[z] * p + m], acc);
      Yr[row * p + m] = acc;
    }
  }
}

// Reduced-precision projection.  Z (N x 2p, row-major FP32) holds [Phi_s, A Phi_s]:
// Z[x, m] = Phi_s[x, m] (from the column-major FP64 basis, ld N) ...
__global__ void pack_basis_f32_kernel(const double* __restrict__ Phi, int64_t N, int32_t p, float* __restrict__ Z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * p) return;
  const int64_t x = e / p;
  const int32_t m = (int32_t)(e % p);
  Z[x * 2 * p + m] = (float)Phi[x + (int64_t)m * N];
}

// ... and Z[x, p + m] = (A Phi_s)[x, m] with FP32 products and FP32 accumulation (the
// CSR values rounded to FP32), one wave per row, lanes over m.
__global__ __launch_bounds__(256) void spmm_f32_kernel(int32_t n_rows, const int32_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col_idx,
                                                       const double* __restrict__ val, int32_t p,
                                                       float* __restrict__ Z) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= n_rows) return;
  const int32_t b = row_ptr[row], e = row_ptr[row + 1];
  for (int m0 = 0; m0 < p; m0 += 64) {
    const int m = m0 + lane;
    if (m >= p) continue;
    float acc = 0.f;
    for (int32_t z = b; z < e; ++z) acc = fmaf((float)val[z], Z[(int64_t)col_idx[z] * 2 * p + m], acc);
    Z[row * 2 * p + p + m] = acc;
  }
}

// Ahat[a + b p] = G[a + (p + b) 2p]: the Phi_s^T (A Phi_s) block of the Gram of Z
__global__ void extract_block_kernel(const double* __restrict__ G, int32_t p, double* __restrict__ Ahat) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= p * p) return;
  const int a = e % p, b = e / p;
  Ahat[e] = G[a + (int64_t)(p + b) * 2 * p];
}

// Split-K tall-skinny product: partial[z] (p x q, column-major) = sum over the
// z-th row range of w[r] X[r,:]^T Y[r,:].  32 x 32 output tile per workgroup.
template <typename TX>
__global__ __launch_bounds__(256) void tsgemm_partial_kernel(int64_t N, int32_t p, int32_t q,
                                                            const TX* __restrict__ X, int64_t xrs, int64_t xcs,
                                                            const double* __restrict__ Y, int64_t yrs, int64_t ycs,
                                                            const double* __restrict__ wrow, int64_t rows_per_split,
                                                            double* __restrict__ partial) {
  __shared__ double Xs[kTile][kTile + 1];
  __shared__ double Ys[kTile][kTile + 1];
  const int a0 = blockIdx.x * kTile, b0 = blockIdx.y * kTile;
  const int64_t rbeg = (int64_t)blockIdx.z * rows_per_split;
  const int64_t rend = min(N, rbeg + rows_per_split);
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;  // 32 x 8
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool x_rows_contig = (xrs == 1);
  const bool y_rows_contig = (yrs == 1);
  for (int64_t r0 = rbeg; r0 < rend; r0 += kTile) {
    for (int i = threadIdx.x; i < kTile * kTile; i += blockDim.x) {
      int kk, a;
      if (x_rows_contig) { kk = i % kTile; a = i / kTile; } else { a = i % kTile; kk = i / kTile; }
      const int64_t r = r0 + kk;
      double v = 0.0;
      if (r < rend && a0 + a < p) {
        v = (double)X[r * xrs + (int64_t)(a0 + a) * xcs];
        if (wrow) v *= wrow[r];
      }
      Xs[kk][a] = v;
      int bb;
      if (y_rows_contig) { kk = i % kTile; bb = i / kTile; } else { bb = i % kTile; kk = i / kTile; }
      const int64_t r2 = r0 + kk;
      Ys[kk][bb] = (r2 < rend && b0 + bb < q) ? Y[r2 * yrs + (int64_t)(b0 + bb) * ycs] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kTile; ++kk) {
      const double yv = Ys[kk][tx];
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s] = fma(Xs[kk][ty + 8 * s], yv, acc[s]);
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.z * p * q;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int a = a0 + ty + 8 * s, b = b0 + tx;
    if (a < p && b < q) out[a + (int64_t)b * p] = acc[s];
  }
}

// The same product with a 64 x 64 output tile per workgroup and a 4 x 4 register
// block per thread: eight LDS reads per sixteen FMAs instead of five per four (the
// 32 x 32 form is bound by its LDS reads).  Used when both output sides are >= 64.
template <typename TX>
__global__ __launch_bounds__(256) void tsgemm_partial64_kernel(int64_t N, int32_t p, int32_t q,
                                                              const TX* __restrict__ X, int64_t xrs, int64_t xcs,
                                                              const double* __restrict__ Y, int64_t yrs, int64_t ycs,
                                                              const double* __restrict__ wrow, int64_t rows_per_split,
                                                              double* __restrict__ partial) {
  constexpr int T = kTile64, KC = kTile;  // output tile side, rows per staged chunk
  __shared__ double Xs[KC][T + 1];
  __shared__ double Ys[KC][T + 1];
  const int a0 = blockIdx.x * T, b0 = blockIdx.y * T;
  const int64_t rbeg = (int64_t)blockIdx.z * rows_per_split;
  const int64_t rend = min(N, rbeg + rows_per_split);
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;  // 16 x 16 threads, outputs ty + 16 i, tx + 16 j
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  const bool x_rows_contig = (xrs == 1);
  const bool y_rows_contig = (yrs == 1);
  for (int64_t r0 = rbeg; r0 < rend; r0 += KC) {
    for (int e = threadIdx.x; e < KC * T; e += 256) {
      int kk, a;
      if (x_rows_contig) { kk = e % KC; a = e / KC; } else { a = e % T; kk = e / T; }
      const int64_t r = r0 + kk;
      double v = 0.0;
      if (r < rend && a0 + a < p) {
        v = (double)X[r * xrs + (int64_t)(a0 + a) * xcs];
        if (wrow) v *= wrow[r];
      }
      Xs[kk][a] = v;
      int bb;
      if (y_rows_contig) { kk = e % KC; bb = e / KC; } else { bb = e % T; kk = e / T; }
      const int64_t r2 = r0 + kk;
      Ys[kk][bb] = (r2 < rend && b0 + bb < q) ? Y[r2 * yrs + (int64_t)(b0 + bb) * ycs] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      double xv[4], yv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) xv[i] = Xs[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) yv[j] = Ys[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(xv[i], yv[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.z * p * q;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int a = a0 + ty + 16 * i, b = b0 + tx + 16 * j;
      if (a < p && b < q) out[a + (int64_t)b * p] = acc[i][j];
    }
}

// C[a + b*ldc] = sum_z partial[z][a + b*p], summed in split order (deterministic).
__global__ void tsgemm_reduce_kernel(int32_t p, int32_t q, int32_t splits, const double* __restrict__ partial,
                                     double* __restrict__ C, int32_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t pq = (int64_t)p * q;
  if (e >= pq) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += partial[z * pq + e];
  const int a = (int)(e % p), b = (int)(e / p);
  C[a + (int64_t)b * ldc] = s;
}

// output tile side of a p x q tall-skinny product
inline int tsgemm_tile(int32_t p, int32_t q) { return (p >= kTile64 && q >= kTile64) ? kTile64 : kTile; }

int tsgemm_splits(int64_t N, int32_t p, int32_t q) {
  const int t = tsgemm_tile(p, q);
  const int64_t tiles = (int64_t)((p + t - 1) / t) * ((q + t - 1) / t);
  if (tiles <= 0 || N <= 0) return 1;
  int64_t splits = (512 + tiles - 1) / tiles;
  const int64_t max_splits = (N + 255) / 256;
  if (splits > max_splits) splits = max_splits;
  if (splits < 1) splits = 1;
  return (int)splits;
}

// K_i[j',j] = sum_k phi_ij'(k) phi_ij(k) - sum_{k < N_t - 1} phi_ij'(k+1) phi_ij(k), one mode per workgroup.
__global__ __launch_bounds__(256) void temporal_K_kernel(const double* __restrict__ Phi, int32_t N_t,
                                                        const int32_t* __restrict__ moff,
                                                        const int64_t* __restrict__ koff, double* __restrict__ K) {
  const int i = blockIdx.x;
  const int c0 = moff[i];
  const int nt = moff[i + 1] - c0;
  const double* P = Phi + (int64_t)c0 * N_t;
  for (int e = threadIdx.x; e < nt * nt; e += blockDim.x) {
    const int jp = e % nt, j = e / nt;
    const double* a = P + (int64_t)jp * N_t;
    const double* b = P + (int64_t)j * N_t;
    double g = 0.0, sh = 0.0;
    for (int k = 0; k < N_t; ++k) g = fma(a[k], b[k], g);
    for (int k = 0; k + 1 < N_t; ++k) sh = fma(a[k + 1], b[k], sh);
    K[koff[i] + jp + (int64_t)j * nt] = g - sh;
  }
}

// Wf[q*n + a] = sum_k dt_k g[k,q] phi_a(k) and P1[a] = phi_a(0): one wave per column a.
__global__ __launch_bounds__(256) void temporal_vec_kernel(const double* __restrict__ Phi, int32_t N_t, int32_t n,
                                                          const double* __restrict__ dt,
                                                          const double* __restrict__ g, int32_t Qf,
                                                          double* __restrict__ Wf, double* __restrict__ P1) {
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (a >= n) return;
  const double* col = Phi + (int64_t)a * N_t;
  if (lane == 0) P1[a] = col[0];
  for (int qf = 0; qf < Qf; ++qf) {
    double s = 0.0;
    for (int k = lane; k < N_t; k += 64) s = fma(dt[k] * (g ? g[k + (int64_t)qf * N_t] : 1.0), col[k], s);
    s = __ockl_wfred_add_f64(s);
    if (lane == 0) Wf[(int64_t)qf * n + a] = s;
  }
}

}  // namespace

hipError_t launch_index_tables(const ModeTable& mt, int32_t N_t, MutRomView rom, hipStream_t s) {
  (void)N_t;
  hipLaunchKernelGGL(index_tables_kernel, dim3(1), dim3(256), 0, s, mt, rom);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* src, int64_t rows, int32_t cols, int64_t ld, double* dst, hipStream_t s) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((unsigned)((rows + kTile - 1) / kTile), (unsigned)((cols + kTile - 1) / kTile));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, src, rows, cols, ld, dst);
  return hipGetLastError();
}

hipError_t launch_spmm_rowmajor(const st_csr& A, const double* Xr, int32_t p, double* Yr, hipStream_t s) {
  if (A.n_rows == 0) return hipSuccess;
  const int rows_per_block = 4;
  dim3 grid((unsigned)((A.n_rows + rows_per_block - 1) / rows_per_block));
  hipLaunchKernelGGL(spmm_rowmajor_kernel, grid, dim3(256), 0, s, A.n_rows, A.row_ptr, A.col_idx, A.val, Xr, p, Yr);
  return hipGetLastError();
}

hipError_t launch_pack_basis_f32(const double* Phi, int64_t N, int32_t p, float* Z, hipStream_t s) {
  const int64_t e = N * p;
  hipLaunchKernelGGL(pack_basis_f32_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, Phi, N, p, Z);
  return hipGetLastError();
}

hipError_t launch_spmm_f32(const st_csr& A, int32_t p, float* Z, hipStream_t s) {
  hipLaunchKernelGGL(spmm_f32_kernel, dim3((unsigned)((A.n_rows + 3) / 4)), dim3(256), 0, s, A.n_rows, A.row_ptr,
                     A.col_idx, A.val, p, Z);
  return hipGetLastError();
}

hipError_t launch_extract_block(const double* G, int32_t p, double* Ahat, hipStream_t s) {
  hipLaunchKernelGGL(extract_block_kernel, dim3((p * p + 255) / 256), dim3(256), 0, s, G, p, Ahat);
  return hipGetLastError();
}

__global__ void round_f32_kernel(const double* __restrict__ src, int64_t n, float* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) dst[e] = (float)src[e];
}

__global__ void combine_cn_kernel(const double* __restrict__ T, const double* __restrict__ S, int32_t n,
                                  double* __restrict__ Tcn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int64_t a = e / n, b = e % n;  // row-major destination, column-major sources
  Tcn[e] = 0.5 * (T[a + b * n] + S[a + b * n]);
}

hipError_t launch_combine_cn(const double* T, const double* S, int32_t n, double* Tcn, hipStream_t s) {
  const int64_t e = (int64_t)n * n;
  if (e == 0) return hipSuccess;
  hipLaunchKernelGGL(combine_cn_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, T, S, n, Tcn);
  return hipGetLastError();
}

hipError_t launch_round_f32(const double* src, int64_t n, float* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(round_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, n, dst);
  return hipGetLastError();
}

size_t tsgemm_partial_elems(int64_t N, int32_t p, int32_t q) {
  if (p <= 0 || q <= 0) return 0;
  return (size_t)tsgemm_splits(N, p, q) * (size_t)p * (size_t)q;
}

template <typename TX>
hipError_t tsgemm_go(int64_t N, int32_t p, int32_t q, const TX* X, int64_t xrs, int64_t xcs, const double* Y,
                     int64_t yrs, int64_t ycs, const double* wrow, double* C, int32_t ldc, double* partial,
                     size_t partial_elems, hipStream_t s) {
  if (p == 0 || q == 0) return hipSuccess;
  const int splits = tsgemm_splits(N, p, q);
  if ((size_t)splits * p * q > partial_elems) return hipErrorInvalidValue;
  int64_t rps = (N + splits - 1) / splits;
  rps = (rps + kTile - 1) / kTile * kTile;
  const int t = tsgemm_tile(p, q);
  dim3 grid((p + t - 1) / t, (q + t - 1) / t, splits);
  if (t == kTile64)
    hipLaunchKernelGGL(tsgemm_partial64_kernel<TX>, grid, dim3(256), 0, s, N, p, q, X, xrs, xcs, Y, yrs, ycs, wrow,
                       rps, partial);
  else
    hipLaunchKernelGGL(tsgemm_partial_kernel<TX>, grid, dim3(256), 0, s, N, p, q, X, xrs, xcs, Y, yrs, ycs, wrow, rps,
                       partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t pq = (int64_t)p * q;
  hipLaunchKernelGGL(tsgemm_reduce_kernel, dim3((unsigned)((pq + 255) / 256)), dim3(256), 0, s, p, q, splits,
                     partial, C, ldc);
  return hipGetLastError();
}

hipError_t launch_tsgemm_w(int64_t N, int32_t p, int32_t q, const double* X, int64_t xrs, int64_t xcs, const double* Y,
                           int64_t yrs, int64_t ycs, const double* wrow, double* C, int32_t ldc, double* partial,
                           size_t partial_elems, hipStream_t s) {
  return tsgemm_go<double>(N, p, q, X, xrs, xcs, Y, yrs, ycs, wrow, C, ldc, partial, partial_elems, s);
}

hipError_t launch_tsgemm(int64_t N, int32_t p, int32_t q, const double* X, int64_t xrs, int64_t xcs, const double* Y,
                         int64_t yrs, int64_t ycs, double* C, int32_t ldc, double* partial, size_t partial_elems,
                         hipStream_t s) {
  return tsgemm_go<double>(N, p, q, X, xrs, xcs, Y, yrs, ycs, nullptr, C, ldc, partial, partial_elems, s);
}

// out = A V with A m x k and out m x k column-major (leading dimension m), V k x k
// column-major, k <= 256: the reduction runs over k only, so one split, and the
// tiles write out directly (out must not overlap A or V).
hipError_t launch_mul_small(const double* A, int64_t m, int32_t k, const double* V, double* out, hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  if (k > 256 || m > 0x7fffffff) return hipErrorInvalidValue;
  const int64_t rps = (int64_t)(k + kTile - 1) / kTile * kTile;
  dim3 grid((unsigned)((m + kTile - 1) / kTile), (k + kTile - 1) / kTile, 1);
  hipLaunchKernelGGL(tsgemm_partial_kernel<double>, grid, dim3(256), 0, s, (int64_t)k, (int32_t)m, k, A, m, 1, V,
                     1, k, nullptr, rps, out);
  return hipGetLastError();
}

hipError_t launch_tsgemm_xf(int64_t N, int32_t p, int32_t q, const float* X, int64_t xrs, int64_t xcs, const double* Y,
                            int64_t yrs, int64_t ycs, double* C, int32_t ldc, double* partial, size_t partial_elems,
                            hipStream_t s) {
  return tsgemm_go<float>(N, p, q, X, xrs, xcs, Y, yrs, ycs, nullptr, C, ldc, partial, partial_elems, s);
}

__global__ void mode_offsets_kernel(ModeTable mt, int32_t* moff) {
  if (threadIdx.x == 0) {
    int32_t o = 0;
    for (int i = 0; i < mt.n_s; ++i) {
      moff[i] = o;
      o += mt.nt[i];
    }
    moff[mt.n_s] = o;
  }
}

hipError_t launch_mode_offsets(const ModeTable& mt, int32_t* moff, hipStream_t s) {
  hipLaunchKernelGGL(mode_offsets_kernel, dim3(1), dim3(64), 0, s, mt, moff);
  return hipGetLastError();
}

hipError_t launch_temporal(const double* Phi_t, int32_t N_t, int32_t n, const double* dt, const double* g, int32_t Qf,
                           const ModeTable& mt, MutRomView rom, hipStream_t s) {
  // T is formed by the caller with launch_tsgemm_w (weights dt); this launches K, Wf and P1.
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(temporal_K_kernel, dim3(mt.n_s), dim3(256), 0, s, Phi_t, N_t, (const int32_t*)rom.moff,
                     (const int64_t*)rom.koff, rom.K);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(temporal_vec_kernel, dim3((n + 3) / 4), dim3(256), 0, s, Phi_t, N_t, n, dt, g, Qf, rom.Wf,
                     rom.P1);
  return hipGetLastError();
}

}  // namespace strom
