// st_solve_noalloc: the batched reduced solve of st_solve for callers that
// cannot allocate device memory.  Its workspace is a fixed static device array
// instead of a caller buffer; everything else (kernels, launch sequence,
// outputs, info codes) is st_solve's.
#include <mutex>

#include "internal.h"

// The workspace of st_solve_noalloc.  Each GPU the library runs on holds its
// own copy for the life of the process.  Host code must not pass this name to
// a kernel or copy: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress below.
static __device__ __align__(256) unsigned char scratch[ST_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Device address of this device's scratch array, looked up once per device
// (with that device current).
st_status scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return ST_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return ST_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ST_EDEVICE;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ST_OK;
}
}  // namespace

extern "C" st_status st_solve_noalloc(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                                      const double* theta_f, const double* theta_0, const int32_t* nt_q,
                                      const int32_t* skip, int32_t lu_prec, double ir_tol, int32_t ir_max,
                                      double* coeff, int64_t coeff_cap, int64_t* coeff_off, double* relres,
                                      int32_t* info, int32_t* iters, void* stream) {
  if (!d || !d->n_t || d->n_s < 1 || n_q < 0 || coeff_cap < 0) return ST_EINVAL;
  if (lu_prec != ST_F64 && lu_prec != ST_F32) return ST_EINVAL;
  if (n_q == 0) return ST_OK;
  int64_t n = 0;
  for (int i = 0; i < d->n_s; ++i) {
    if (d->n_t[i] < 1) return ST_EINVAL;
    n += d->n_t[i];
  }
  // every query at full width must fit: the per-query widths live on the device
  const size_t need = st_solve_workspace(d, n_q, coeff_cap, (int64_t)n_q * n * n, lu_prec);
  if (need == 0) return ST_EINVAL;
  if (need > (size_t)ST_NOALLOC_SCRATCH_BYTES) return ST_EWORKSPACE;
  void* ws = nullptr;
  const st_status st = scratch_of_current_device(&ws);
  if (st != ST_OK) return st;
  return st_solve(d, rom, n_q, theta_A, theta_f, theta_0, nt_q, skip, lu_prec, ir_tol, ir_max, coeff, coeff_cap,
                  coeff_off, relres, info, iters, ws, ST_NOALLOC_SCRATCH_BYTES, stream);
}
