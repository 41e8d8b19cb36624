// Surrogate network kernels on gfx950 (not part of the paper's method): a
// multilayer perceptron mu -> reduced space-time coefficients, trained and run
// with BF16 matrix-core products accumulated in FP32, FP32 master weights, and
// Adam.  Its predictions are certified by the FP64 space-time residual.
//
// Layout: samples are rows.  Layer l maps h_{l-1} (batch x in_l) to
// z_l = h_{l-1} W_l^T + b_l with W_l stored out_l x in_l row-major; hidden
// layers apply GELU(z) = z/2 (1 + erf(z / sqrt 2)); the last layer is linear.
// Parameters are one flat FP32 array: W_1, b_1, W_2, b_2, ... in order.
#include <math.h>

#include "internal.h"

namespace strom {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMT = 64;  // output tile
constexpr int kKC = 32;  // K chunk staged per step

__device__ inline short to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));  // inf / nan
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

enum Epi { kStore = 0, kBiasGelu = 1, kBias = 2, kGeluGrad = 3 };

// C (M x N, row-major, ldc) = A (M x K) B (K x N) with general element strides,
// operands rounded to BF16, FP32 accumulation on v_mfma_f32_16x16x16_bf16.
// Epilogues: kStore C = acc; kBias C = acc + bias[n]; kBiasGelu Z = acc + bias[n],
// C = gelu(Z) (Z stored to aux); kGeluGrad C = acc * gelu'(aux[m, n]).
template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const float* __restrict__ A, int64_t sam,
                                                        int64_t sak, const float* __restrict__ B, int64_t sbk,
                                                        int64_t sbn, float* __restrict__ C, int64_t ldc,
                                                        const float* __restrict__ bias, float* __restrict__ aux,
                                                        int64_t ldaux) {
  __shared__ short As[kMT][kKC + 4];  // [m][k]
  __shared__ short Bs[kMT][kKC + 4];  // [n][k] (transposed)
  const int m0 = blockIdx.y * kMT, n0 = blockIdx.x * kMT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  f4 acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc[x][y] = f4{0.f, 0.f, 0.f, 0.f};
  const bool a_k_contig = (sak == 1);
  const bool b_k_contig = (sbk == 1);
  for (int k0 = 0; k0 < K; k0 += kKC) {
    for (int e = tid; e < kMT * kKC; e += 256) {
      int m, k;
      if (a_k_contig) { k = e % kKC; m = e / kKC; } else { m = e % kMT; k = e / kMT; }
      const float v = (m0 + m < M && k0 + k < K) ? A[(int64_t)(m0 + m) * sam + (int64_t)(k0 + k) * sak] : 0.f;
      As[m][k] = to_bf16(v);
      int n, kb;
      if (b_k_contig) { kb = e % kKC; n = e / kKC; } else { n = e % kMT; kb = e / kMT; }
      const float u = (n0 + n < N && k0 + kb < K) ? B[(int64_t)(k0 + kb) * sbk + (int64_t)(n0 + n) * sbn] : 0.f;
      Bs[n][kb] = to_bf16(u);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKC; kk += 16) {
      s4 av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) av[x] = *reinterpret_cast<const s4*>(&As[wm + 16 * x + li][kk + 4 * lk]);
#pragma unroll
      for (int y = 0; y < 2; ++y) bv[y] = *reinterpret_cast<const s4*>(&Bs[wn + 16 * y + li][kk + 4 * lk]);
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * x + 4 * lk + r;  // accumulator row = 4(lane/16) + r
        const int n = n0 + wn + 16 * y + li;
        if (m >= M || n >= N) continue;
        float v = acc[x][y][r];
        if (EPI == kBias || EPI == kBiasGelu) v += bias[n];
        if (EPI == kBiasGelu) {
          aux[(int64_t)m * ldaux + n] = v;
          v = gelu(v);
        }
        if (EPI == kGeluGrad) v *= gelu_grad(aux[(int64_t)m * ldaux + n]);
        C[(int64_t)m * ldc + n] = v;
      }
}

// db[n] = sum_m dZ[m, n]  (one thread per column, fixed order)
__global__ void colsum_kernel(int M, int N, const float* __restrict__ dZ, float* __restrict__ db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += dZ[(int64_t)m * N + n];
  db[n] = s;
}

// dY = 2 (Y - T) / (M N); loss partial sums per block
__global__ void mse_grad_kernel(int64_t n, const float* __restrict__ Y, const float* __restrict__ T, float scale,
                                float* __restrict__ dY, float* __restrict__ partial) {
  __shared__ float red[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float d = 0.f;
  if (i < n) {
    d = Y[i] - T[i];
    dY[i] = 2.f * d * scale;
  }
  red[threadIdx.x] = d * d;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void sum_scale_kernel(int n, const float* __restrict__ partial, float scale, float* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    float s = 0.f;
    for (int i = 0; i < n; ++i) s += partial[i];
    *out = s * scale;
  }
}

// Adam (Kingma and Ba) with bias correction, elementwise.
__global__ void adam_kernel(int64_t n, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-column mean and population standard deviation of an n x d row-major FP64
// matrix, two passes per column (one thread per column: consecutive threads
// read consecutive entries of a row); a zero deviation becomes 1.
__global__ void colstats_kernel(int n, int d, const double* __restrict__ C, double* __restrict__ mean,
                                double* __restrict__ scale) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += C[(int64_t)i * d + j];
  const double mu = s / (double)n;
  double v = 0.0;
  for (int i = 0; i < n; ++i) {
    const double e = C[(int64_t)i * d + j] - mu;
    v = fma(e, e, v);
  }
  const double sd = sqrt(v / (double)n);
  mean[j] = mu;
  scale[j] = sd > 0.0 ? sd : 1.0;
}

// T = FP32((C - mean) / scale), elementwise over n x d row-major
__global__ void standardize_kernel(int64_t nd, int d, const double* __restrict__ C, const double* __restrict__ mean,
                                   const double* __restrict__ scale, float* __restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nd) return;
  const int j = (int)(e % d);
  T[e] = (float)((C[e] - mean[j]) / scale[j]);
}

template <int EPI>
hipError_t gemm(int M, int N, int K, const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbk,
                int64_t sbn, float* C, int64_t ldc, const float* bias, float* aux, int64_t ldaux, hipStream_t s) {
  if (M == 0 || N == 0) return hipSuccess;
  dim3 grid((N + kMT - 1) / kMT, (M + kMT - 1) / kMT);
  hipLaunchKernelGGL(gemm_bf16_kernel<EPI>, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc, bias,
                     aux, ldaux);
  return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------
// network bookkeeping shared with the host API
// ---------------------------------------------------------------------------
int mlp_layers(const st_mlp_shape& s) { return s.n_hidden + 1; }
int mlp_in(const st_mlp_shape& s, int l) { return l == 0 ? s.d_in : s.width; }
int mlp_out(const st_mlp_shape& s, int l) { return l == s.n_hidden ? s.d_out : s.width; }

size_t mlp_param_offset(const st_mlp_shape& s, int l) {  // offset of W_l; b_l follows W_l
  size_t o = 0;
  for (int i = 0; i < l; ++i) o += (size_t)mlp_out(s, i) * mlp_in(s, i) + mlp_out(s, i);
  return o;
}

// activations per layer: Z_l and H_l (batch x out_l) for hidden layers, Y for the last
size_t mlp_act_elems(const st_mlp_shape& s, int32_t batch) {
  size_t e = 0;
  for (int l = 0; l < mlp_layers(s); ++l) e += 2 * (size_t)batch * mlp_out(s, l);
  return e;
}

hipError_t mlp_forward(const st_mlp_shape& s, const float* params, int32_t batch, const float* X, float* acts,
                       float* Y, hipStream_t st) {
  const float* h = X;
  float* z = acts;
  for (int l = 0; l < mlp_layers(s); ++l) {
    const int in = mlp_in(s, l), out = mlp_out(s, l);
    const float* W = params + mlp_param_offset(s, l);
    const float* b = W + (size_t)out * in;
    float* hz = z + (size_t)batch * out;
    hipError_t e;
    if (l < s.n_hidden) {
      // H = gelu(h W^T + b), Z kept in aux
      e = gemm<kBiasGelu>(batch, out, in, h, in, 1, W, 1, in, hz, out, b, z, out, st);
    } else {
      e = gemm<kBias>(batch, out, in, h, in, 1, W, 1, in, Y, out, b, nullptr, 0, st);
    }
    if (e != hipSuccess) return e;
    h = hz;
    z = hz + (size_t)batch * out;
  }
  return hipSuccess;
}

hipError_t mlp_backward(const st_mlp_shape& s, const float* params, int32_t batch, const float* X, const float* acts,
                        float* dY, float* grads, float* tmp0, float* tmp1, hipStream_t st) {
  // dY holds dLoss/dY on entry; walk the layers backwards
  const int L = mlp_layers(s);
  // activation pointers
  const float* Zp[64];
  const float* Hp[64];
  const float* z = acts;
  for (int l = 0; l < L; ++l) {
    const int out = mlp_out(s, l);
    Zp[l] = z;
    Hp[l] = z + (size_t)batch * out;
    z = Hp[l] + (size_t)batch * out;
  }
  const float* dZ = dY;
  float* bufs[2] = {tmp0, tmp1};
  for (int l = L - 1; l >= 0; --l) {
    const int in = mlp_in(s, l), out = mlp_out(s, l);
    const float* W = params + mlp_param_offset(s, l);
    float* dW = grads + mlp_param_offset(s, l);
    float* db = dW + (size_t)out * in;
    const float* hin = l == 0 ? X : Hp[l - 1];
    // dW = dZ^T h_in (out x in), K = batch
    hipError_t e = gemm<kStore>(out, in, batch, dZ, 1, out, hin, in, 1, dW, in, nullptr, nullptr, 0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_kernel, dim3((out + 255) / 256), dim3(256), 0, st, batch, out, dZ, db);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (l > 0) {
      // dZ_{l-1} = (dZ W) * gelu'(Z_{l-1})
      float* nd = bufs[l & 1];
      e = gemm<kGeluGrad>(batch, in, out, dZ, out, 1, W, in, 1, nd, in, nullptr, const_cast<float*>(Zp[l - 1]), in,
                          st);
      if (e != hipSuccess) return e;
      dZ = nd;
    }
  }
  return hipSuccess;
}

hipError_t mlp_mse(int64_t n, const float* Y, const float* T, float* dY, float* partial, float* loss, hipStream_t st) {
  const int blocks = (int)((n + 255) / 256);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(blocks), dim3(256), 0, st, n, Y, T, 1.0f / (float)n, dY, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sum_scale_kernel, dim3(1), dim3(64), 0, st, blocks, partial, 1.0f / (float)n, loss);
  return hipGetLastError();
}

size_t mlp_mse_partials(int64_t n) { return (size_t)((n + 255) / 256); }

hipError_t mlp_colstats(int n, int d, const double* C, double* mean, double* scale, hipStream_t st) {
  hipLaunchKernelGGL(colstats_kernel, dim3((d + 255) / 256), dim3(256), 0, st, n, d, C, mean, scale);
  return hipGetLastError();
}

hipError_t mlp_standardize(int n, int d, const double* C, const double* mean, const double* scale, float* T,
                           hipStream_t st) {
  const int64_t nd = (int64_t)n * d;
  if (nd == 0) return hipSuccess;
  hipLaunchKernelGGL(standardize_kernel, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, st, nd, d, C, mean, scale,
                     T);
  return hipGetLastError();
}

hipError_t adam(int64_t n, float* p, const float* g, float* m, float* v, int32_t t, float lr, float b1, float b2,
                float eps, hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

}  // namespace strom
