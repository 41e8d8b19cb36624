// Full-order a-posteriori error bound of space-time ROM solutions (Sec. 5.2,
// Theorem (res-basedErrorBoundforSpaceTime)):
//   ||u_st - u~_st||_inf <= sqrt(N_t) ||A_st^{-1}||_2 ||r_st(u~_st)||_inf,
// with r_st = A_st u~_st - f_st - u0_st (Eq. (stresidual)) and the space-time
// infinity norm max_k ||.||_2 over time steps (Eq. (spacetimeinfnorm)).
//
// The full-order residual of step k is a linear combination of a few fixed
// N_s-vectors.  With u~^(k) = Phi_s y_k, y_k[i] = sum_j Phi_t[k, (i, j)] c_(i,j):
//   r^(k) = Phi_s (y_k - y_{k-1}) - dt_k sum_q theta_q (A_q Phi_s) y_k
//           - dt_k sum_q theta^f_q g[k, q] Bf_q   [- u0(mu) at k = 1, y_0 = 0]
// so every residual vector is D c_k with the dictionary
//   D = [Phi_s, A_1 Phi_s, ..., A_Q Phi_s, Bf_1..Bf_Qf, u0_1..u0_Q0]  (N_s x m_D)
// built once (row-major: one spatial point's m_D entries contiguous), and a
// per-(query, step) coefficient column c_k.  One workgroup per (query, block of
// time steps) forms its coefficient columns in LDS and streams D once,
// reducing ||r^(k)||_2 and ||u~^(k)||_2 = ||Phi_s y_k||_2 without writing the
// N_s x N_t residual.
#include "internal.h"

namespace strom {
namespace {

constexpr int kBoundThreads = 256;
constexpr int kBoundSteps = 32;                       // time steps per workgroup
constexpr int kBoundRowGroups = kBoundThreads / kBoundSteps;

// D[x, 0:n_s] = Phi_s[x, :]; D[x, n_s(Q+1) + q] = Bf[x, q]; D[x, n_s(Q+1) + Qf + q] = u0[x, q]
__global__ void dict_pack_kernel(int64_t N_s, int32_t n_s, int32_t Q, int32_t Qf, int32_t Q0,
                                 const double* __restrict__ Phi_s, const double* __restrict__ Bf,
                                 const double* __restrict__ u0, double* __restrict__ D, int32_t m_D) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t cols = n_s + Qf + Q0;
  if (e >= N_s * cols) return;
  const int64_t x = e / cols;
  const int32_t c = (int32_t)(e % cols);
  double v;
  int32_t dst;
  if (c < n_s) {
    v = Phi_s[x + (int64_t)c * N_s];
    dst = c;
  } else if (c < n_s + Qf) {
    v = Bf[x + (int64_t)(c - n_s) * N_s];
    dst = n_s * (Q + 1) + (c - n_s);
  } else {
    v = u0[x + (int64_t)(c - n_s - Qf) * N_s];
    dst = n_s * (Q + 1) + Qf + (c - n_s - Qf);
  }
  D[x * m_D + dst] = v;
}

// D[x, n_s(1+q) + m] = (A_q Phi_s)[x, m]: one wave per row, lanes over m, reading the
// Phi_s block of D (row-major, so each gathered row is contiguous)
__global__ __launch_bounds__(256) void dict_spmm_kernel(int32_t n_rows, const int32_t* __restrict__ row_ptr,
                                                        const int32_t* __restrict__ col_idx,
                                                        const double* __restrict__ val, int32_t n_s, int32_t col0,
                                                        double* __restrict__ D, int32_t m_D) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (row >= n_rows) return;
  const int32_t b = row_ptr[row], e = row_ptr[row + 1];
  for (int m0 = 0; m0 < n_s; m0 += 64) {
    const int m = m0 + lane;
    if (m >= n_s) continue;
    double acc = 0.0;
    for (int32_t z = b; z < e; ++z) acc = fma(val[z], D[(int64_t)col_idx[z] * m_D + m], acc);
    D[row * m_D + col0 + m] = acc;
  }
}

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax(reinterpret_cast<unsigned long long*>(addr), (unsigned long long)__double_as_longlong(v));
}

// One workgroup per (query q, steps k0 .. k0 + kBoundSteps - 1).  LDS: the
// query's mode offsets, y_k for k0-1 .. k0+KT-1, and the coefficient tile.
__global__ __launch_bounds__(kBoundThreads) void fom_residual_kernel(
    RomView rom, int64_t N_s, const double* __restrict__ D, int32_t m_D, int32_t n_q,
    const double* __restrict__ thA, const double* __restrict__ thf, const double* __restrict__ th0,
    const double* __restrict__ g, const int32_t* __restrict__ nt_q, Plan plan, const double* __restrict__ coeff,
    double* __restrict__ res_inf, double* __restrict__ u_inf) {
  extern __shared__ __align__(16) double lds[];
  __shared__ int32_t s_loff[kMaxFormModes + 1];
  __shared__ double s_r2[kBoundRowGroups][kBoundSteps];
  __shared__ double s_u2[kBoundRowGroups][kBoundSteps];
  const int q = blockIdx.y;
  if (plan.info[q] != 0) return;
  const int n_s = rom.n_s, N_t = rom.N_t;
  const int k0 = blockIdx.x * kBoundSteps;
  const int kt = min(kBoundSteps, N_t - k0);
  const int tid = threadIdx.x;
  double* ys = lds;                                   // (kBoundSteps + 1) x n_s, row s = step k0 - 1 + s
  double* C = lds + (kBoundSteps + 1) * n_s;          // m_D x kBoundSteps
  if (tid == 0) {
    int32_t o = 0;
    for (int i = 0; i < n_s; ++i) {
      s_loff[i] = o;
      o += nt_q ? nt_q[(int64_t)q * n_s + i] : rom.moff[i + 1] - rom.moff[i];
    }
    s_loff[n_s] = o;
  }
  __syncthreads();
  const double* c = coeff + plan.coeff_off[q];
  // y_k[i] = sum_j Phi_t[k, moff_i + j] c[loff_i + j] (y = 0 before the first step)
  for (int e = tid; e < (kBoundSteps + 1) * n_s; e += kBoundThreads) {
    const int srow = e / n_s, i = e % n_s;
    const int k = k0 - 1 + srow;
    double y = 0.0;
    if (k >= 0 && k < N_t) {
      const int nt = s_loff[i + 1] - s_loff[i];
      const double* pt = rom.Phit + (int64_t)rom.moff[i] * N_t + k;
      const double* ci = c + s_loff[i];
#pragma unroll 8  // several strided loads in flight; same FMA order
      for (int j = 0; j < nt; ++j) y = fma(pt[(int64_t)j * N_t], ci[j], y);
    }
    ys[e] = y;
  }
  __syncthreads();
  // coefficient columns
  const int Q = rom.Q, Qf = rom.Qf, Q0 = rom.Q0;
  for (int e = tid; e < m_D * kBoundSteps; e += kBoundThreads) {
    const int m = e / kBoundSteps, kk = e % kBoundSteps;
    const int k = k0 + kk;
    double v = 0.0;
    if (kk < kt) {
      const double dt = rom.dt[k];
      if (m < n_s) {
        v = ys[(kk + 1) * n_s + m] - ys[kk * n_s + m];
      } else if (m < n_s * (Q + 1)) {
        const int t = m / n_s - 1, i = m % n_s;
        v = -dt * thA[(int64_t)q * Q + t] * ys[(kk + 1) * n_s + i];
      } else if (m < n_s * (Q + 1) + Qf) {
        const int t = m - n_s * (Q + 1);
        v = -dt * thf[(int64_t)q * Qf + t] * (g ? g[k + (int64_t)t * N_t] : 1.0);
      } else {
        const int t = m - n_s * (Q + 1) - Qf;
        v = (k == 0) ? -th0[(int64_t)q * Q0 + t] : 0.0;
      }
    }
    C[m * kBoundSteps + kk] = v;
  }
  __syncthreads();
  // r^(k)(x) = D[x, :] c_k and u~^(k)(x) = Phi_s[x, :] y_k, one column per lane group
  const int kk = tid % kBoundSteps, rg = tid / kBoundSteps;
  double r2 = 0.0, u2 = 0.0;
  const double* yk = ys + (kk + 1) * n_s;
  for (int64_t x = rg; x < N_s; x += kBoundRowGroups) {
    const double* dx = D + x * m_D;
    double r = 0.0, u = 0.0;
    for (int m = 0; m < n_s; ++m) {
      const double dv = dx[m];
      r = fma(dv, C[m * kBoundSteps + kk], r);
      u = fma(dv, yk[m], u);
    }
    for (int m = n_s; m < m_D; ++m) r = fma(dx[m], C[m * kBoundSteps + kk], r);
    r2 = fma(r, r, r2);
    u2 = fma(u, u, u2);
  }
  s_r2[rg][kk] = r2;
  s_u2[rg][kk] = u2;
  __syncthreads();
  if (tid < kBoundSteps) {
    double a = 0.0, b = 0.0;
    for (int g2 = 0; g2 < kBoundRowGroups; ++g2) {
      a += s_r2[g2][tid];
      b += s_u2[g2][tid];
    }
    if (tid < kt) {
      atomic_max_nonneg(&res_inf[q], sqrt(a));
      atomic_max_nonneg(&u_inf[q], sqrt(b));
    }
  }
}

__global__ void bound_init_kernel(int32_t n_q, double* res_inf, double* u_inf) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n_q) {
    res_inf[q] = 0.0;
    u_inf[q] = 0.0;
  }
}

__global__ void bound_finish_kernel(int32_t n_q, Plan plan, double scale, double* res_inf, double* u_inf,
                                    double* bound) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n_q) return;
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  if (plan.info[q] != 0) {
    res_inf[q] = nan;
    u_inf[q] = nan;
    bound[q] = nan;
  } else {
    bound[q] = scale * res_inf[q];
  }
}

}  // namespace

size_t fom_bound_lds_bytes(int n_s, int m_D) {
  return sizeof(double) * ((size_t)(kBoundSteps + 1) * n_s + (size_t)m_D * kBoundSteps);
}

hipError_t launch_fom_dict(int64_t N_s, int32_t n_s, int32_t Q, const st_csr* A, int32_t Qf, int32_t Q0,
                           const double* Phi_s, const double* Bf, const double* u0, double* D, int32_t m_D,
                           hipStream_t s) {
  const int64_t e = N_s * (n_s + Qf + Q0);
  hipLaunchKernelGGL(dict_pack_kernel, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, N_s, n_s, Q, Qf, Q0, Phi_s,
                     Bf, u0, D, m_D);
  hipError_t err = hipGetLastError();
  for (int q = 0; q < Q && err == hipSuccess; ++q) {
    hipLaunchKernelGGL(dict_spmm_kernel, dim3((unsigned)((N_s + 3) / 4)), dim3(256), 0, s, (int32_t)N_s,
                       A[q].row_ptr, A[q].col_idx, A[q].val, n_s, n_s * (1 + q), D, m_D);
    err = hipGetLastError();
  }
  return err;
}

hipError_t launch_fom_residual(const RomView& rom, int64_t N_s, const double* D, int32_t m_D, int32_t n_q,
                               const double* thA, const double* thf, const double* th0, const double* g,
                               const int32_t* nt_q, Plan plan, const double* coeff, double inv_norm, double* res_inf,
                               double* u_inf, double* bound, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  hipLaunchKernelGGL(bound_init_kernel, dim3((n_q + 255) / 256), dim3(256), 0, s, n_q, res_inf, u_inf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = fom_bound_lds_bytes(rom.n_s, m_D);
  e = hipFuncSetAttribute((const void*)fom_residual_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  dim3 grid((rom.N_t + kBoundSteps - 1) / kBoundSteps, n_q);
  hipLaunchKernelGGL(fom_residual_kernel, grid, dim3(kBoundThreads), lds, s, rom, N_s, D, m_D, n_q, thA, thf, th0, g,
                     nt_q, plan, coeff, res_inf, u_inf);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(bound_finish_kernel, dim3((n_q + 255) / 256), dim3(256), 0, s, n_q, plan,
                     sqrt((double)rom.N_t) * inv_norm, res_inf, u_inf, bound);
  return hipGetLastError();
}

}  // namespace strom
