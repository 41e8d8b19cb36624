// Spatial Galerkin ROM (Sec. 3.1): the time march of Eq.
// (space_reduced_discretized_ODE) with u_ref = 0,
//   (I - dt_k Ahat(mu)) uhat^(k) = uhat^(k-1) + dt_k Bhat f^(k)(mu),
//   uhat^(0) = Phi_s^T u0(mu),
// and the reduced outputs of Eq. (outputFromReducedsol), y^(k) = Chat^T uhat^(k),
// for a batch of parameter queries.  It is the paper's point of comparison for
// the space-time ROM.  One workgroup per query: (I - dt Ahat(mu))^{-1} is formed
// in LDS by in-place Gauss-Jordan elimination with partial pivoting (again only
// when the step size changes), so each time step is one matrix-vector product
// (one thread per row) instead of a serial triangular solve.
#include "internal.h"

namespace strom {
namespace {

constexpr int kSpThreads = 256;

__device__ inline bool finite_v(double v) { return v == v && v - v == 0.0; }

// Minv (row-major n x n, LDS) <- (I - dt Ahat(mu))^{-1}; returns false if singular
__device__ bool form_inverse(const RomView& rom, const double* __restrict__ thA, int q, double dt, double* Minv,
                             double* f, int* s_piv, int* s_sing) {
  const int n = rom.n_s, tid = threadIdx.x;
  for (int e = tid; e < n * n; e += kSpThreads) {
    const int i = e / n, j = e % n;
    double a = 0.0;
    for (int t = 0; t < rom.Q; ++t)
      a = fma(thA[(int64_t)q * rom.Q + t], rom.Ahat[(int64_t)t * n * n + i + (int64_t)j * n], a);
    Minv[e] = (i == j ? 1.0 : 0.0) - dt * a;
  }
  if (tid == 0) *s_sing = 0;
  __syncthreads();
  for (int p = 0; p < n; ++p) {
    if (tid == 0) {
      int r = p;
      double best = fabs(Minv[p * n + p]);
      for (int i = p + 1; i < n; ++i) {
        const double v = fabs(Minv[i * n + p]);
        if (v > best) { best = v; r = i; }
      }
      s_piv[p] = r;
      if (!(best > 0.0)) *s_sing = 1;
    }
    __syncthreads();
    if (*s_sing) return false;
    const int r = s_piv[p];
    if (r != p)
      for (int j = tid; j < n; j += kSpThreads) {
        const double t = Minv[p * n + j];
        Minv[p * n + j] = Minv[r * n + j];
        Minv[r * n + j] = t;
      }
    __syncthreads();
    const double pinv = 1.0 / Minv[p * n + p];
    for (int i = tid; i < n; i += kSpThreads) f[i] = (i == p) ? 0.0 : Minv[i * n + p];
    __syncthreads();
    for (int j = tid; j < n; j += kSpThreads) Minv[p * n + j] = (j == p ? 1.0 : Minv[p * n + j]) * pinv;
    __syncthreads();
    for (int e = tid; e < n * n; e += kSpThreads) {
      const int i = e / n, j = e % n;
      if (i == p) continue;
      Minv[e] = (j == p ? 0.0 : Minv[e]) - f[i] * Minv[p * n + j];
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int p = n - 1; p >= 0; --p) {
    const int r = s_piv[p];
    if (r != p)
      for (int i = tid; i < n; i += kSpThreads) {
        const double t = Minv[i * n + p];
        Minv[i * n + p] = Minv[i * n + r];
        Minv[i * n + r] = t;
      }
    __syncthreads();
  }
  return true;
}

__global__ __launch_bounds__(kSpThreads) void spatial_march_kernel(RomView rom, int32_t n_q,
                                                                   const double* __restrict__ thA,
                                                                   const double* __restrict__ thf,
                                                                   const double* __restrict__ th0,
                                                                   const double* __restrict__ g, int32_t n_out,
                                                                   const double* __restrict__ Chat,
                                                                   double* __restrict__ traj,
                                                                   double* __restrict__ outs,
                                                                   int32_t* __restrict__ info) {
  extern __shared__ __align__(16) double lds[];
  __shared__ int s_piv[kMaxFormModes];
  __shared__ int s_sing, s_bad;
  const int q = blockIdx.x, tid = threadIdx.x;
  const int n = rom.n_s, N_t = rom.N_t, Qf = rom.Qf;
  double* Minv = lds;                   // n x n
  double* u = Minv + n * n;             // n
  double* rhs = u + n;                  // n
  double* f = rhs + n;                  // n
  double* bq = f + n;                   // Qf x n: theta_f[q, t] bhat_t
  if (tid == 0) {
    int bad = 0;
    for (int t = 0; t < rom.Q; ++t) bad |= !finite_v(thA[(int64_t)q * rom.Q + t]);
    for (int t = 0; t < Qf; ++t) bad |= !finite_v(thf[(int64_t)q * Qf + t]);
    for (int t = 0; t < rom.Q0; ++t) bad |= !finite_v(th0[(int64_t)q * rom.Q0 + t]);
    s_bad = bad;
  }
  __syncthreads();
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  int code = s_bad ? -5 : 0;
  for (int i = tid; i < n; i += kSpThreads) {
    double v = 0.0;
    for (int t = 0; t < rom.Q0; ++t) v = fma(th0[(int64_t)q * rom.Q0 + t], rom.u0hat[(int64_t)t * n + i], v);
    u[i] = v;
    for (int t = 0; t < Qf; ++t) bq[t * n + i] = thf[(int64_t)q * Qf + t] * rom.bhat[(int64_t)t * n + i];
  }
  double dt_prev = nan;
  for (int k = 0; k < N_t; ++k) {
    const double dt = rom.dt[k];
    if (code == 0 && !(dt == dt_prev)) {
      __syncthreads();
      if (!form_inverse(rom, thA, q, dt, Minv, f, s_piv, &s_sing)) code = k + 1;
      dt_prev = dt;
    }
    __syncthreads();
    if (code == 0) {
      for (int i = tid; i < n; i += kSpThreads) {
        double v = u[i];
        for (int t = 0; t < Qf; ++t) v = fma(dt * (g ? g[k + (int64_t)t * N_t] : 1.0), bq[t * n + i], v);
        rhs[i] = v;
      }
      __syncthreads();
      for (int i = tid; i < n; i += kSpThreads) {
        double v = 0.0;
        const double* row = Minv + i * n;
        for (int j = 0; j < n; ++j) v = fma(row[j], rhs[j], v);
        u[i] = v;
      }
      __syncthreads();
    }
    const int64_t base = (int64_t)q * N_t + k;
    if (traj)
      for (int i = tid; i < n; i += kSpThreads) traj[base * n + i] = code == 0 ? u[i] : nan;
    if (outs)
      for (int o = tid; o < n_out; o += kSpThreads) {
        double y = 0.0;
        for (int i = 0; i < n; ++i) y = fma(Chat[i + (int64_t)o * n], u[i], y);
        outs[base * n_out + o] = code == 0 ? y : nan;
      }
  }
  if (tid == 0) info[q] = code;
}

}  // namespace

size_t spatial_march_lds_bytes(int n_s, int Qf) { return sizeof(double) * ((size_t)n_s * n_s + (size_t)(3 + Qf) * n_s); }

hipError_t launch_spatial_march(const RomView& rom, int32_t n_q, const double* thA, const double* thf,
                                const double* th0, const double* g, int32_t n_out, const double* Chat, double* traj,
                                double* outs, int32_t* info, hipStream_t s) {
  if (n_q == 0) return hipSuccess;
  const size_t lds = spatial_march_lds_bytes(rom.n_s, rom.Qf);
  hipError_t e =
      hipFuncSetAttribute((const void*)spatial_march_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(spatial_march_kernel, dim3(n_q), dim3(kSpThreads), lds, s, rom, n_q, thA, thf, th0, g, n_out,
                     Chat, traj, outs, info);
  return hipGetLastError();
}

}  // namespace strom
