// Host side of the ST-ROM C ABI: argument validation, buffer layouts and the
// launch sequences of st_assemble, st_form and st_solve.  All launches go to
// the caller's stream; nothing here allocates device memory or synchronises.
#include <math.h>
#include <string.h>

#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

using namespace strom;

namespace {

int64_t total_nt(const st_rom_desc* d) {
  int64_t n = 0;
  for (int i = 0; i < d->n_s; ++i) n += d->n_t[i];
  return n;
}

bool desc_ok(const st_rom_desc* d) {
  if (!d || !d->n_t) return false;
  if (d->n_s < 1 || d->n_s > kMaxModes || d->N_t < 1) return false;
  if (d->Q < 1 || d->Q > kMaxTerms || d->Qf < 0 || d->Qf > kMaxTerms || d->Q0 < 0 || d->Q0 > kMaxTerms) return false;
  if (d->integrator != ST_BACKWARD_EULER && d->integrator != ST_CRANK_NICOLSON) return false;
  for (int i = 0; i < d->n_s; ++i)
    if (d->n_t[i] < 1 || d->n_t[i] > d->N_t) return false;
  return true;
}

void layout_of(const st_rom_desc* d, st_rom_layout_t* L) {
  const size_t n_s = (size_t)d->n_s, n = (size_t)total_nt(d);
  size_t k2 = 0;
  for (int i = 0; i < d->n_s; ++i) k2 += (size_t)d->n_t[i] * d->n_t[i];
  size_t o = 0;
  L->Ahat = o;  o = align_up(o + sizeof(double) * d->Q * n_s * n_s);
  L->bhat = o;  o = align_up(o + sizeof(double) * d->Qf * n_s);
  L->u0hat = o; o = align_up(o + sizeof(double) * d->Q0 * n_s);
  L->T = o;     o = align_up(o + sizeof(double) * n * n);
  L->K = o;     o = align_up(o + sizeof(double) * k2);
  L->Wf = o;    o = align_up(o + sizeof(double) * d->Qf * n);
  L->P1 = o;    o = align_up(o + sizeof(double) * n);
  L->mode = o;  o = align_up(o + sizeof(int32_t) * n);
  L->moff = o;  o = align_up(o + sizeof(int32_t) * (n_s + 1));
  L->koff = o;  o = align_up(o + sizeof(int64_t) * (n_s + 1));
  L->Phit = o;  o = align_up(o + sizeof(double) * d->N_t * n);
  L->dt = o;    o = align_up(o + sizeof(double) * d->N_t);
  L->T32 = o;   o = align_up(o + sizeof(float) * n * n);
  const bool cn = d->integrator == ST_CRANK_NICOLSON;
  L->Tcn = o;   o = align_up(o + (cn ? sizeof(double) * n * n : 0));
  L->Au0 = o;   o = align_up(o + (cn ? sizeof(double) * d->Q * d->Q0 * n_s : 0));
  L->total = o;
}

RomView view_of(const st_rom_desc* d, const void* rom) {
  st_rom_layout_t L;
  layout_of(d, &L);
  const char* b = static_cast<const char*>(rom);
  RomView v;
  v.Ahat = reinterpret_cast<const double*>(b + L.Ahat);
  v.bhat = reinterpret_cast<const double*>(b + L.bhat);
  v.u0hat = reinterpret_cast<const double*>(b + L.u0hat);
  v.T = reinterpret_cast<const double*>(b + L.T);
  v.K = reinterpret_cast<const double*>(b + L.K);
  v.Wf = reinterpret_cast<const double*>(b + L.Wf);
  v.P1 = reinterpret_cast<const double*>(b + L.P1);
  v.mode = reinterpret_cast<const int32_t*>(b + L.mode);
  v.moff = reinterpret_cast<const int32_t*>(b + L.moff);
  v.koff = reinterpret_cast<const int64_t*>(b + L.koff);
  v.Phit = reinterpret_cast<const double*>(b + L.Phit);
  v.dt = reinterpret_cast<const double*>(b + L.dt);
  v.T32 = reinterpret_cast<const float*>(b + L.T32);
  v.integ = d->integrator;
  v.Teff = d->integrator == ST_CRANK_NICOLSON ? reinterpret_cast<const double*>(b + L.Tcn) : v.T;
  v.Au0 = reinterpret_cast<const double*>(b + L.Au0);
  v.n_s = d->n_s;
  v.N_t = d->N_t;
  v.n = (int32_t)total_nt(d);
  v.Q = d->Q;
  v.Qf = d->Qf;
  v.Q0 = d->Q0;
  return v;
}

#define ST_TRY(expr)                              \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return ST_EDEVICE;      \
  } while (0)

struct Carver {
  char* base;
  size_t used = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used = align_up(used + sizeof(T) * count);
    return p;
  }
};

size_t plan_bytes(int32_t n_q) {
  size_t o = 0;
  o = align_up(o + sizeof(int32_t) * n_q);        // width
  o = align_up(o + sizeof(int32_t) * n_q);        // order
  o = align_up(o + sizeof(int32_t) * 4);          // counter
  return o;
}

bool query_args_ok(const st_rom_desc* d, const void* rom, int32_t n_q, const double* thA, const double* thf,
                   const double* th0) {
  if (!desc_ok(d) || !rom || n_q < 0) return false;
  if (n_q > 0 && !thA) return false;
  if (n_q > 0 && d->Qf > 0 && !thf) return false;
  if (n_q > 0 && d->Q0 > 0 && !th0) return false;
  return true;
}

}  // namespace

extern "C" {

const char* st_strerror(st_status s) {
  switch (s) {
    case ST_OK: return "success";
    case ST_EINVAL: return "invalid argument";
    case ST_EDEVICE: return "HIP runtime error";
    case ST_EWORKSPACE: return "workspace or output buffer too small";
    case ST_ERANK: return "requested basis exceeds the rank of the data";
    case ST_EUNSUPPORTED: return "size or precision not supported by the kernels";
    default: return "unknown status";
  }
}

int32_t st_version(void) { return 2; }

st_status st_rom_layout(const st_rom_desc* d, st_rom_layout_t* out) {
  if (!desc_ok(d) || !out) return ST_EINVAL;
  layout_of(d, out);
  return ST_OK;
}

size_t st_assemble_workspace(const st_rom_desc* d, int64_t N_s) {
  if (!desc_ok(d) || N_s < 1) return 0;
  const int64_t n = total_nt(d);
  size_t part = tsgemm_partial_elems(N_s, d->n_s, d->n_s);
  part = part > tsgemm_partial_elems(N_s, d->n_s, d->Qf) ? part : tsgemm_partial_elems(N_s, d->n_s, d->Qf);
  part = part > tsgemm_partial_elems(N_s, d->n_s, d->Q0) ? part : tsgemm_partial_elems(N_s, d->n_s, d->Q0);
  part = part > tsgemm_partial_elems(d->N_t, (int32_t)n, (int32_t)n) ? part
                                                                      : tsgemm_partial_elems(d->N_t, (int32_t)n, (int32_t)n);
  if (d->integrator == ST_CRANK_NICOLSON) {
    // the shifted contraction S (n x n) and its partials share the partial area
    const size_t cn = (size_t)n * n + tsgemm_partial_elems(d->N_t > 1 ? d->N_t - 1 : 1, (int32_t)n, (int32_t)n);
    part = part > cn ? part : cn;
  }
  const size_t fp64 = align_up(sizeof(double) * (size_t)N_s * d->n_s) * 2 +
                      align_up(sizeof(double) * (size_t)N_s * d->Q0) * 2 + align_up(sizeof(double) * part);
  // reduced-precision projection: Z (N_s x 2 n_s FP32), its Gram and the Gram's partials
  const int32_t p2 = 2 * d->n_s;
  const size_t red = align_up(sizeof(float) * (size_t)N_s * p2) + align_up(sizeof(double) * (size_t)p2 * p2) +
                     align_up(sizeof(double) * gram_partial_elems(N_s, p2));
  return fp64 > red ? fp64 : red;
}

st_status st_assemble(const st_rom_desc* d, int64_t N_s, const double* Phi_s, const double* Phi_t, const double* dt,
                      const st_csr* A, const double* Bf, const double* g, const double* u0, int32_t proj_prec,
                      void* rom, size_t rom_bytes, void* ws, size_t ws_bytes, void* stream) {
  if (!desc_ok(d) || N_s < 1 || N_s > 0x7fffffff || !Phi_s || !Phi_t || !dt || !A || !rom || !ws) return ST_EINVAL;
  if (proj_prec != ST_F64 && proj_prec != ST_F32 && proj_prec != ST_BF16X3) return ST_EINVAL;
  if (d->n_s > N_s) return ST_ERANK;
  if (d->Qf > 0 && !Bf) return ST_EINVAL;
  if (d->Q0 > 0 && !u0) return ST_EINVAL;
  for (int q = 0; q < d->Q; ++q) {
    if (A[q].n_rows != N_s || A[q].nnz < 0 || !A[q].row_ptr) return ST_EINVAL;
    if (A[q].nnz > 0 && (!A[q].col_idx || !A[q].val)) return ST_EINVAL;
  }
  const int64_t n = total_nt(d);
  if (n > kMaxWidth * 4) return ST_EUNSUPPORTED;
  st_rom_layout_t L;
  layout_of(d, &L);
  if (rom_bytes < L.total) return ST_EWORKSPACE;
  if (ws_bytes < st_assemble_workspace(d, N_s)) return ST_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);

  char* rb = static_cast<char*>(rom);
  MutRomView mv;
  mv.Ahat = reinterpret_cast<double*>(rb + L.Ahat);
  mv.bhat = reinterpret_cast<double*>(rb + L.bhat);
  mv.u0hat = reinterpret_cast<double*>(rb + L.u0hat);
  mv.T = reinterpret_cast<double*>(rb + L.T);
  mv.K = reinterpret_cast<double*>(rb + L.K);
  mv.Wf = reinterpret_cast<double*>(rb + L.Wf);
  mv.P1 = reinterpret_cast<double*>(rb + L.P1);
  mv.mode = reinterpret_cast<int32_t*>(rb + L.mode);
  mv.moff = reinterpret_cast<int32_t*>(rb + L.moff);
  mv.koff = reinterpret_cast<int64_t*>(rb + L.koff);
  mv.Phit = reinterpret_cast<double*>(rb + L.Phit);
  mv.dt = reinterpret_cast<double*>(rb + L.dt);
  mv.T32 = reinterpret_cast<float*>(rb + L.T32);
  mv.Tcn = reinterpret_cast<double*>(rb + L.Tcn);
  mv.Au0 = reinterpret_cast<double*>(rb + L.Au0);

  Carver c(ws);
  double* Phir = c.take<double>((size_t)N_s * d->n_s);
  double* Y = c.take<double>((size_t)N_s * d->n_s);
  double* u0r = c.take<double>((size_t)N_s * d->Q0);  // Crank-Nicolson: u0 terms, row-major
  double* Yu = c.take<double>((size_t)N_s * d->Q0);   //                 A_q u0 terms
  double* part = reinterpret_cast<double*>(c.base + c.used);
  const size_t part_elems = (ws_bytes - c.used) / sizeof(double);

  ModeTable mt;
  memset(&mt, 0, sizeof(mt));
  mt.n_s = d->n_s;
  for (int i = 0; i < d->n_s; ++i) mt.nt[i] = d->n_t[i];
  ST_TRY(launch_index_tables(mt, d->N_t, mv, s));
  const int32_t ns = d->n_s;
  // projection: Ahat_q = Phi_s^T (A_q Phi_s)
  if (proj_prec == ST_F64) {
    ST_TRY(launch_transpose(Phi_s, N_s, ns, N_s, Phir, s));
    for (int q = 0; q < d->Q; ++q) {
      ST_TRY(launch_spmm_rowmajor(A[q], Phir, ns, Y, s));
      ST_TRY(launch_tsgemm(N_s, ns, ns, Phir, ns, 1, Y, ns, 1, mv.Ahat + (size_t)q * ns * ns, ns, part, part_elems,
                           s));
    }
  } else {
    // FP32 SpMM into Z = [Phi_s, A_q Phi_s] (FP32, row-major), then Phi_s^T (A_q Phi_s) as the
    // off-diagonal block of the Gram of Z on the matrix cores (FP32 or split-BF16 MFMA, FP32
    // accumulation); the rest of the ROM stays FP64
    Carver r(ws);
    const int32_t p2 = 2 * ns;
    float* Z = r.take<float>((size_t)N_s * p2);
    double* G = r.take<double>((size_t)p2 * p2);
    double* gpart = r.take<double>(gram_partial_elems(N_s, p2));
    ST_TRY(launch_pack_basis_f32(Phi_s, N_s, ns, Z, s));
    for (int q = 0; q < d->Q; ++q) {
      ST_TRY(launch_spmm_f32(A[q], ns, Z, s));
      ST_TRY(launch_gram(N_s, p2, Z, ST_F32, p2, 1, proj_prec, G, gpart, gram_partial_elems(N_s, p2), s));
      ST_TRY(launch_extract_block(G, ns, mv.Ahat + (size_t)q * ns * ns, s));
    }
    // the row-major FP64 basis for bhat and u0hat below (it reuses Z's memory)
    ST_TRY(launch_transpose(Phi_s, N_s, ns, N_s, Phir, s));
  }
  if (d->Qf > 0) ST_TRY(launch_tsgemm(N_s, ns, d->Qf, Phir, ns, 1, Bf, 1, N_s, mv.bhat, ns, part, part_elems, s));
  if (d->Q0 > 0) ST_TRY(launch_tsgemm(N_s, ns, d->Q0, Phir, ns, 1, u0, 1, N_s, mv.u0hat, ns, part, part_elems, s));
  // temporal contractions
  ST_TRY(launch_tsgemm_w(d->N_t, (int32_t)n, (int32_t)n, Phi_t, 1, d->N_t, Phi_t, 1, d->N_t, dt, mv.T, (int32_t)n, part,
                         part_elems, s));
  ST_TRY(launch_temporal(Phi_t, d->N_t, (int32_t)n, dt, g, d->Qf, mt, mv, s));
  if (d->integrator == ST_CRANK_NICOLSON) {
    // S[a,b] = sum_{k>1} dt_k phi_a(k) phi_b(k-1) (column-major, in the workspace),
    // then T_cn = (T + S)/2, row-major, and its FP32 copy
    const size_t nn = (size_t)n * n;
    double* Sc = part;
    double* part2 = part + nn;
    const size_t part2_elems = part_elems - nn;
    if (d->N_t > 1)
      ST_TRY(launch_tsgemm_w(d->N_t - 1, (int32_t)n, (int32_t)n, Phi_t + 1, 1, d->N_t, Phi_t, 1, d->N_t, dt + 1, Sc,
                             (int32_t)n, part2, part2_elems, s));
    else
      ST_TRY(launch_fill_f64(Sc, (int64_t)nn, 0.0, s));
    ST_TRY(launch_combine_cn(mv.T, Sc, (int32_t)n, mv.Tcn, s));
    ST_TRY(launch_round_f32(mv.Tcn, (int64_t)nn, mv.T32, s));
    // Phi_s^T A_q u0_q0: the initial terms through each operator term
    if (d->Q0 > 0) {
      ST_TRY(launch_transpose(u0, N_s, d->Q0, N_s, u0r, s));
      for (int q = 0; q < d->Q; ++q) {
        ST_TRY(launch_spmm_rowmajor(A[q], u0r, d->Q0, Yu, s));
        ST_TRY(launch_tsgemm(N_s, ns, d->Q0, Phir, ns, 1, Yu, d->Q0, 1, mv.Au0 + (size_t)q * d->Q0 * ns, ns, part,
                             part_elems, s));
      }
    }
  } else {
    ST_TRY(launch_round_f32(mv.T, (int64_t)n * n, mv.T32, s));
  }
  // the bases and steps themselves, for the residual evaluated on the time grid
  ST_TRY(launch_copy_cols(Phi_t, d->N_t, mv.Phit, d->N_t, d->N_t, (int)n, s));
  ST_TRY(launch_copy_cols(dt, d->N_t, mv.dt, d->N_t, d->N_t, 1, s));
  return ST_OK;
}

size_t st_form_workspace(const st_rom_desc* d, int32_t n_q) {
  if (!desc_ok(d) || n_q < 0) return 0;
  return plan_bytes(n_q);
}

st_status st_form(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A, const double* theta_f,
                  const double* theta_0, const int32_t* nt_q, int32_t out_prec, void* mats, int64_t mats_cap,
                  double* rhs, int64_t coeff_cap, int64_t* coeff_off, int64_t* mat_off, int32_t* info, void* ws,
                  size_t ws_bytes, void* stream) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0)) return ST_EINVAL;
  if (out_prec != ST_F64 && out_prec != ST_F32) return ST_EINVAL;
  if (d->n_s > kMaxFormModes) return ST_EUNSUPPORTED;
  if (mats_cap < 0 || coeff_cap < 0) return ST_EINVAL;
  if (n_q == 0) return ST_OK;
  if (!mats || !rhs || !coeff_off || !mat_off || !info || !ws) return ST_EINVAL;
  if (ws_bytes < st_form_workspace(d, n_q)) return ST_EWORKSPACE;
  const int64_t n = total_nt(d);
  if (n > kMaxWidth) return ST_EUNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RomView rv = view_of(d, rom);
  Carver c(ws);
  Plan plan;
  plan.width = c.take<int32_t>(n_q);
  plan.order = c.take<int32_t>(n_q);
  plan.counter = c.take<int32_t>(4);
  plan.mat_off = mat_off;
  plan.coeff_off = coeff_off;
  plan.info = info;
  ST_TRY(launch_plan(n_q, d->n_s, rv.moff, nt_q, nullptr, theta_A, theta_f, theta_0, d->Q, d->Qf, d->Q0, coeff_cap,
                     mats_cap, plan, s));
  ST_TRY(launch_form(rv, n_q, theta_A, theta_f, theta_0, nt_q, plan, out_prec, mats, rhs, (int32_t)n, s));
  return ST_OK;
}

}  // extern "C"

namespace {
bool g_timing = false;
bool g_timing_recorded = false;
hipEvent_t g_events[ST_TIMING_PHASES + 1];
bool g_events_made = false;

hipError_t mark(int i, hipStream_t s) {
  if (!g_timing) return hipSuccess;
  return hipEventRecord(g_events[i], s);
}
}  // namespace

extern "C" {

st_status st_timing_enable(int32_t on) {
  if (on && !g_events_made) {
    for (int i = 0; i <= ST_TIMING_PHASES; ++i)
      if (hipEventCreate(&g_events[i]) != hipSuccess) return ST_EDEVICE;
    g_events_made = true;
  }
  g_timing = on != 0;
  g_timing_recorded = false;
  return ST_OK;
}

int32_t st_timing_read(double* ms, int32_t cap) {
  if (!ms || cap < 0) return ST_EINVAL;
  if (!g_events_made || !g_timing_recorded) return ST_EINVAL;
  const int n = cap < ST_TIMING_PHASES ? cap : ST_TIMING_PHASES;
  for (int i = 0; i < n; ++i) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, g_events[i], g_events[i + 1]) != hipSuccess) return ST_EDEVICE;
    ms[i] = (double)t;
  }
  return ST_TIMING_PHASES;
}

size_t st_solve_workspace(const st_rom_desc* d, int32_t n_q, int64_t sum_w, int64_t sum_w2, int32_t lu_prec) {
  if (!desc_ok(d) || n_q < 0 || sum_w < 0 || sum_w2 < 0) return 0;
  const size_t el = lu_prec == ST_F32 ? sizeof(float) : sizeof(double);
  size_t o = plan_bytes(n_q);
  o = align_up(o + sizeof(int32_t) * n_q);           // active
  o = align_up(o + sizeof(int64_t) * (n_q + 1));     // mat_off
  o = align_up(o + sizeof(double) * n_q) * 1;        // bnorm
  o = align_up(o + sizeof(double) * n_q);            // rnorm
  o = align_up(o + sizeof(double) * sum_w);          // b
  o = align_up(o + sizeof(double) * sum_w);          // r
  o = align_up(o + sizeof(int32_t) * sum_w);         // permutations
  o = align_up(o + sizeof(int64_t) * (n_q + 1));     // FP64 re-solve: matrix offsets
  o = align_up(o + sizeof(int32_t) * n_q);           //                info
  o = align_up(o + sizeof(int32_t) * 4);             //                counters
  o = align_up(o + el * (size_t)sum_w2);             // matrices
  return o;
}

}  // extern "C"

namespace {

// Arguments of one st_solve call (validated), in the form the launch sequence needs.
struct SolveArgs {
  const st_rom_desc* d;
  const void* rom;
  int32_t n_q;
  const double *thA, *thf, *th0;
  const int32_t *nt_q, *skip;
  int32_t lu_prec;
  double ir_tol;
  int32_t ir_max;
  double* coeff;
  int64_t coeff_cap;
  int64_t* coeff_off;
  double* relres;
  int32_t* info;
  int32_t* iters;
  void* ws;
  size_t ws_bytes;
};

// Workspace sections of st_solve.
struct SolveWs {
  Plan plan;
  Plan fb;  // FP64 re-solve of unconverged queries (shares width, order, coeff_off)
  int32_t* active;
  double *bnorm, *rnorm, *b, *r;
  int32_t* perm;
  void* mats;
};

SolveWs solve_ws(const SolveArgs& a) {
  const size_t el = a.lu_prec == ST_F32 ? sizeof(float) : sizeof(double);
  Carver c(a.ws);
  SolveWs w;
  w.plan.width = c.take<int32_t>(a.n_q);
  w.plan.order = c.take<int32_t>(a.n_q);
  w.plan.counter = c.take<int32_t>(4);
  w.active = c.take<int32_t>(a.n_q);
  w.plan.mat_off = c.take<int64_t>(a.n_q + 1);
  w.bnorm = c.take<double>(a.n_q);
  w.rnorm = c.take<double>(a.n_q);
  w.b = c.take<double>(a.coeff_cap);
  w.r = c.take<double>(a.coeff_cap);
  w.perm = c.take<int32_t>(a.coeff_cap);
  w.fb = w.plan;
  w.fb.mat_off = c.take<int64_t>(a.n_q + 1);
  w.fb.info = c.take<int32_t>(a.n_q);
  w.fb.counter = c.take<int32_t>(4);
  w.mats = c.base + c.used;
  w.plan.coeff_off = a.coeff_off;
  w.plan.info = a.info;
  w.fb.width = w.plan.width;
  w.fb.order = w.plan.order;
  w.fb.coeff_off = a.coeff_off;
  (void)el;
  return w;
}

int64_t solve_mats_cap(const SolveArgs& a) {
  const size_t el = a.lu_prec == ST_F32 ? sizeof(float) : sizeof(double);
  const size_t fixed = st_solve_workspace(a.d, a.n_q, a.coeff_cap, 0, a.lu_prec);
  return (int64_t)((a.ws_bytes - fixed) / el);
}

// Autotuned LU variant per (precision, width class); -1 = not tuned (variant 0).
std::mutex g_tune_mu;
int g_lu_choice[2][2] = {{-1, -1}, {-1, -1}};

int width_class(int32_t n_max) { return n_max <= 3 * 512 ? 0 : 1; }

int lu_choice(int32_t prec, int32_t n_max) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int c = g_lu_choice[prec == ST_F32 ? 1 : 0][width_class(n_max)];
  return c < 0 ? 0 : c;
}

// The whole launch sequence of st_solve on stream s.
hipError_t solve_launches(const SolveArgs& a, hipStream_t s) {
  const RomView rv = view_of(a.d, a.rom);
  SolveWs w = solve_ws(a);
  Plan plan = w.plan;
  const int32_t n_max = (int32_t)total_nt(a.d);
  const int32_t n_q = a.n_q;
  const int variant = lu_choice(a.lu_prec, n_max);
  const int nbo = lu_outer_block(a.lu_prec, n_max, variant);
  hipError_t e;
#define SL_TRY(expr)                 \
  do {                               \
    if ((e = (expr)) != hipSuccess) return e; \
  } while (0)
  SL_TRY(mark(0, s));
  SL_TRY(launch_plan(n_q, a.d->n_s, rv.moff, a.nt_q, a.skip, a.thA, a.thf, a.th0, a.d->Q, a.d->Qf, a.d->Q0,
                     a.coeff_cap, solve_mats_cap(a), plan, s));
  SL_TRY(mark(1, s));
  SL_TRY(launch_form(rv, n_q, a.thA, a.thf, a.th0, a.nt_q, plan, a.lu_prec, w.mats, w.b, n_max, s));
  SL_TRY(mark(2, s));
  SL_TRY(launch_vec_norms(n_q, plan, w.b, w.bnorm, s));
  SL_TRY(mark(3, s));
  SL_TRY(launch_lu(n_q, plan, a.lu_prec, w.mats, w.perm, n_max, variant, s));
  SL_TRY(mark(4, s));
  SL_TRY(launch_fill_i32(w.active, n_q, 1, s));
  SL_TRY(launch_lu_solve(n_q, plan, a.lu_prec, w.mats, w.perm, w.b, a.coeff, 0, w.active, n_max, nbo, s));
  SL_TRY(mark(5, s));
  for (int it = 0; it < a.ir_max; ++it) {
    SL_TRY(launch_residual(rv, n_q, a.thA, a.nt_q, plan, w.b, a.coeff, w.r, w.rnorm, w.active, n_max, s));
    SL_TRY(launch_ir_check(n_q, plan, w.rnorm, w.bnorm, a.ir_tol, it, 0, w.active, a.relres, a.iters, s));
    SL_TRY(launch_lu_solve(n_q, plan, a.lu_prec, w.mats, w.perm, w.r, a.coeff, 1, w.active, n_max, nbo, s));
  }
  SL_TRY(mark(6, s));
  // final residual of the queries still active (all of them without refinement)
  SL_TRY(launch_residual(rv, n_q, a.thA, a.nt_q, plan, w.b, a.coeff, w.r, w.rnorm, w.active, n_max, s));
  const int flag = (a.lu_prec == ST_F32 || a.ir_max > 0) ? 2 : 1;
  SL_TRY(launch_ir_check(n_q, plan, w.rnorm, w.bnorm, a.ir_tol, a.ir_max, flag, w.active, a.relres, a.iters, s));
  if (a.lu_prec == ST_F32 && a.ir_tol > 0.0) {
    // queries whose refinement did not converge (info -1): re-form their systems in
    // FP64 in the matrix space (the FP32 factors are no longer needed), factor, solve,
    // and record the FP64 residual (info -6)
    const Plan fb = w.fb;
    const int v64 = lu_choice(ST_F64, n_max);
    const int nbo64 = lu_outer_block(ST_F64, n_max, v64);
    const int64_t cap64 = solve_mats_cap(a) * (int64_t)sizeof(float) / (int64_t)sizeof(double);
    SL_TRY(launch_fallback_plan(n_q, plan, fb, w.active, cap64, s));
    SL_TRY(launch_form(rv, n_q, a.thA, a.thf, a.th0, a.nt_q, fb, ST_F64, w.mats, w.b, n_max, s));
    SL_TRY(launch_lu(n_q, fb, ST_F64, w.mats, w.perm, n_max, v64, s));
    SL_TRY(launch_lu_solve(n_q, fb, ST_F64, w.mats, w.perm, w.b, a.coeff, 0, w.active, n_max, nbo64, s));
    SL_TRY(launch_residual(rv, n_q, a.thA, a.nt_q, fb, w.b, a.coeff, w.r, w.rnorm, w.active, n_max, s));
    SL_TRY(launch_ir_check(n_q, fb, w.rnorm, w.bnorm, a.ir_tol, a.ir_max, 1, w.active, a.relres, a.iters, s));
    SL_TRY(launch_fallback_finish(n_q, plan, fb, w.active, s));
  }
  SL_TRY(launch_finalize(n_q, plan, a.coeff, a.info, s));
  SL_TRY(mark(7, s));
#undef SL_TRY
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// HIP graph cache of st_solve launch sequences, keyed by every argument (the
// description by value, buffers by address) and the LU variant in use.
// ---------------------------------------------------------------------------
bool g_graph = false;
std::mutex g_graph_mu;
std::map<std::vector<uint64_t>, hipGraphExec_t> g_graphs;
hipStream_t g_capture_stream = nullptr;

std::vector<uint64_t> graph_key(const SolveArgs& a, int device) {
  std::vector<uint64_t> k;
  auto put = [&](uint64_t v) { k.push_back(v); };
  auto ptr = [&](const void* p) { put((uint64_t)(uintptr_t)p); };
  put((uint64_t)device);
  put((uint64_t)a.d->n_s); put((uint64_t)a.d->N_t); put((uint64_t)a.d->Q); put((uint64_t)a.d->Qf);
  put((uint64_t)a.d->Q0);
  put((uint64_t)a.d->integrator);
  for (int i = 0; i < a.d->n_s; ++i) put((uint64_t)a.d->n_t[i]);
  ptr(a.rom); put((uint64_t)a.n_q); ptr(a.thA); ptr(a.thf); ptr(a.th0); ptr(a.nt_q); ptr(a.skip);
  put((uint64_t)a.lu_prec);
  uint64_t tb;
  memcpy(&tb, &a.ir_tol, sizeof(tb));
  put(tb); put((uint64_t)a.ir_max);
  ptr(a.coeff); put((uint64_t)a.coeff_cap); ptr(a.coeff_off); ptr(a.relres); ptr(a.info); ptr(a.iters); ptr(a.ws);
  put((uint64_t)a.ws_bytes);
  put((uint64_t)lu_choice(a.lu_prec, (int32_t)total_nt(a.d)));
  put((uint64_t)lu_choice(ST_F64, (int32_t)total_nt(a.d)));
  return k;
}

// Record the launch sequence as a graph (on the library's capture stream; the
// kernels are not run) and instantiate it.
hipError_t capture_solve(const SolveArgs& a, hipGraphExec_t* exec) {
  hipError_t e;
  if (!g_capture_stream && (e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking)) != hipSuccess)
    return e;
  if ((e = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeRelaxed)) != hipSuccess) return e;
  g_capturing = true;
  const hipError_t le = solve_launches(a, g_capture_stream);
  g_capturing = false;
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(g_capture_stream, &graph);
  if (le != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le != hipSuccess ? le : e;
  }
  e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  return e;
}

}  // namespace

namespace strom {
bool g_capturing = false;
}  // namespace strom

extern "C" {

st_status st_solve(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A, const double* theta_f,
                   const double* theta_0, const int32_t* nt_q, const int32_t* skip, int32_t lu_prec, double ir_tol,
                   int32_t ir_max,
                   double* coeff, int64_t coeff_cap, int64_t* coeff_off, double* relres, int32_t* info,
                   int32_t* iters, void* ws, size_t ws_bytes, void* stream) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0)) return ST_EINVAL;
  if (lu_prec != ST_F64 && lu_prec != ST_F32) return ST_EINVAL;
  if (!(ir_tol >= 0.0) || ir_max < 0 || ir_max > 1000 || coeff_cap < 0) return ST_EINVAL;
  if (d->n_s > kMaxFormModes) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!coeff || !coeff_off || !relres || !info || !ws) return ST_EINVAL;
  const int64_t n = total_nt(d);
  if (n > kMaxWidth) return ST_EUNSUPPORTED;
  const size_t fixed = st_solve_workspace(d, n_q, coeff_cap, 0, lu_prec);
  if (ws_bytes < fixed) return ST_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SolveArgs a{d, rom, n_q, theta_A, theta_f, theta_0, nt_q, skip, lu_prec, ir_tol, ir_max,
                    coeff, coeff_cap, coeff_off, relres, info, iters, ws, ws_bytes};
  if (!g_graph || g_timing) {
    ST_TRY(solve_launches(a, s));
    if (g_timing) g_timing_recorded = true;
    return ST_OK;
  }
  int device = 0;
  ST_TRY(hipGetDevice(&device));
  const std::vector<uint64_t> key = graph_key(a, device);
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it != g_graphs.end()) {
    ST_TRY(hipGraphLaunch(it->second, s));
    return ST_OK;
  }
  // first call with these arguments: run eagerly, then record the graph for the next ones
  ST_TRY(solve_launches(a, s));
  hipGraphExec_t exec = nullptr;
  ST_TRY(capture_solve(a, &exec));
  g_graphs.emplace(key, exec);
  return ST_OK;
}

st_status st_reconstruct(const st_rom_desc* d, const void* rom, int64_t N_s, const double* Phi_s, int64_t ldp,
                         const double* Phi_t, int64_t ldt, int32_t n_q, const int32_t* nt_q, const double* coeff,
                         const int64_t* coeff_off, double* out, int64_t ldo, void* stream) {
  if (!desc_ok(d) || !rom || N_s < 1 || n_q < 0) return ST_EINVAL;
  if (ldp < N_s || ldt < d->N_t || ldo < N_s) return ST_EINVAL;
  if (d->n_s > kMaxFormModes) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!Phi_s || !Phi_t || !coeff || !coeff_off || !out) return ST_EINVAL;
  const RomView rv = view_of(d, rom);
  ST_TRY(launch_reconstruct(N_s, d->N_t, d->n_s, Phi_s, ldp, Phi_t, ldt, rv.moff, nt_q, n_q, coeff, coeff_off, out,
                            ldo, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

st_status st_graph_enable(int32_t on) {
  g_graph = on != 0;
  return ST_OK;
}

st_status st_graph_reset(void) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
  g_graphs.clear();
  return ST_OK;
}

int32_t st_graph_count(void) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  return (int32_t)g_graphs.size();
}

st_status st_autotune(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                      const double* theta_f, const double* theta_0, const int32_t* nt_q, int32_t lu_prec,
                      double* coeff, int64_t coeff_cap, int64_t* coeff_off, double* relres, int32_t* info, void* ws,
                      size_t ws_bytes, void* stream, int32_t* choice, double* ms) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0)) return ST_EINVAL;
  if (lu_prec != ST_F64 && lu_prec != ST_F32) return ST_EINVAL;
  if (d->n_s > kMaxFormModes) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!coeff || !coeff_off || !relres || !info || !ws || coeff_cap < 0) return ST_EINVAL;
  const int64_t n = total_nt(d);
  if (n > kMaxWidth) return ST_EUNSUPPORTED;
  if (ws_bytes < st_solve_workspace(d, n_q, coeff_cap, 0, lu_prec)) return ST_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const SolveArgs a{d, rom, n_q, theta_A, theta_f, theta_0, nt_q, nullptr, lu_prec, 0.0, 0,
                    coeff, coeff_cap, coeff_off, relres, info, nullptr, ws, ws_bytes};
  const RomView rv = view_of(d, rom);
  SolveWs w = solve_ws(a);
  const int32_t n_max = (int32_t)n;
  const int nv = lu_variant_count(lu_prec, n_max);
  if (nv <= 0) return ST_EUNSUPPORTED;
  hipEvent_t e0, e1;
  ST_TRY(hipEventCreate(&e0));
  ST_TRY(hipEventCreate(&e1));
  int best = 0;
  float best_ms = 0.f;
  st_status st = ST_OK;
  for (int v = 0; v < nv && st == ST_OK; ++v) {
    // each candidate factors freshly formed systems (the LU works in place); the
    // plan's work-queue counter is reset by re-running the plan
    if (launch_plan(n_q, d->n_s, rv.moff, nt_q, nullptr, theta_A, theta_f, theta_0, d->Q, d->Qf, d->Q0, coeff_cap,
                    solve_mats_cap(a), w.plan, s) != hipSuccess ||
        launch_form(rv, n_q, theta_A, theta_f, theta_0, nt_q, w.plan, lu_prec, w.mats, w.b, n_max, s) != hipSuccess ||
        hipEventRecord(e0, s) != hipSuccess ||
        launch_lu(n_q, w.plan, lu_prec, w.mats, w.perm, n_max, v, s) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
      st = ST_EDEVICE;
      break;
    }
    float t = 0.f;
    if (hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
      st = ST_EDEVICE;
      break;
    }
    if (ms) ms[v] = (double)t;
    if (v == 0 || t < best_ms) {
      best = v;
      best_ms = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != ST_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_lu_choice[lu_prec == ST_F32 ? 1 : 0][width_class(n_max)] = best;
  }
  if (choice) *choice = best;
  return ST_OK;
}

int32_t st_autotune_choice(int32_t lu_prec, int32_t n) {
  if ((lu_prec != ST_F64 && lu_prec != ST_F32) || n < 0 || n > kMaxWidth) return ST_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return g_lu_choice[lu_prec == ST_F32 ? 1 : 0][width_class(n)];
}

st_status st_autotune_set(int32_t lu_prec, int32_t n, int32_t variant) {
  if ((lu_prec != ST_F64 && lu_prec != ST_F32) || n < 0 || n > kMaxWidth) return ST_EINVAL;
  if (variant < -1 || variant >= ST_LU_VARIANTS || variant >= lu_variant_count(lu_prec, n)) return ST_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_lu_choice[lu_prec == ST_F32 ? 1 : 0][width_class(n)] = variant;
  return ST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// st_build_bases (POD)
// ---------------------------------------------------------------------------
namespace {

constexpr int kSubspaceIters = 10;
constexpr int kMaxSubspace = 256;

constexpr int kRefineExtra = 16;    // columns beyond n_s carried into the SVD refinement
constexpr int kRefineSweeps = 30;   // sweep limit of the refinement's one-sided Jacobi

struct PodDims {
  int64_t N_s, m, p;
  int n_s, k, kr, n;
  bool transposed;  // Gram is U U^T (N_s < m)
};

bool pod_dims(int64_t N_s, int32_t N_t, int32_t n_mu, int32_t n_s, const int32_t* n_t, PodDims* d) {
  if (N_s < 1 || N_t < 1 || n_mu < 1 || n_s < 1 || !n_t) return false;
  d->N_s = N_s;
  d->m = (int64_t)n_mu * N_t;
  d->transposed = N_s < d->m;
  d->p = d->transposed ? N_s : d->m;
  d->n_s = n_s;
  int64_t extra = d->p - n_s;
  if (extra > 32) extra = 32;
  d->k = (int)(n_s + (extra > 0 ? extra : 0));
  d->kr = d->k < n_s + kRefineExtra ? d->k : n_s + kRefineExtra;
  int64_t n = 0;
  for (int i = 0; i < n_s; ++i) n += n_t[i];
  d->n = (int)n;
  return true;
}

struct PodWs {
  double *G, *X, *Y, *H, *Z, *Zs, *evals, *sig, *V, *part;
  double *C1, *C2, *Y1, *Y2, *J, *Jp, *sigk, *offmax, *diag, *oC, *on0;
  int32_t *moff, *perm, *rot, *oflag;
  size_t part_elems, total;
};

PodWs pod_ws(const PodDims& d, void* base) {
  Carver c(base);
  PodWs w;
  w.G = c.take<double>((size_t)d.p * d.p);
  w.X = c.take<double>((size_t)d.p * d.k);
  w.Y = c.take<double>((size_t)d.p * d.k);
  w.H = c.take<double>((size_t)d.k * d.k);
  w.Z = c.take<double>((size_t)d.k * d.k);
  w.Zs = c.take<double>((size_t)d.k * d.k);
  w.evals = c.take<double>(d.k);
  w.sig = c.take<double>(d.n_s);
  w.V = c.take<double>((size_t)d.m * d.n_s);
  w.C1 = c.take<double>((size_t)d.N_s * d.kr);
  w.Y1 = c.take<double>((size_t)d.N_s * d.kr);
  w.C2 = c.take<double>((size_t)d.m * d.kr);
  w.Y2 = c.take<double>((size_t)d.m * d.kr);
  w.J = c.take<double>((size_t)d.kr * d.kr);
  w.Jp = c.take<double>((size_t)d.kr * d.n_s);
  w.sigk = c.take<double>(d.k);
  w.offmax = c.take<double>(kRefineSweeps);
  w.diag = c.take<double>(ST_POD_DIAG);
  w.moff = c.take<int32_t>(d.n_s + 1);
  w.perm = c.take<int32_t>(d.kr);
  w.rot = c.take<int32_t>(kRefineSweeps);
  w.oC = c.take<double>((size_t)d.k * 16);  // blocked Gram-Schmidt of the subspace iteration
  w.on0 = c.take<double>(16);
  w.oflag = c.take<int32_t>(1);
  size_t pe = gram_partial_elems(d.transposed ? d.m : d.N_s, (int)d.p);
  const size_t cands[] = {tsgemm_partial_elems(d.p, (int)d.p, d.k), tsgemm_partial_elems(d.p, d.k, d.k),
                          tsgemm_partial_elems(d.k, (int)d.p, d.k), tsgemm_partial_elems(d.N_s, (int)d.m, d.kr),
                          tsgemm_partial_elems(d.m, (int)d.N_s, d.kr), tsgemm_partial_elems(d.kr, (int)d.N_s, d.n_s),
                          tsgemm_partial_elems(d.kr, (int)d.m, d.n_s), tsgemm_partial_elems(d.N_s, d.kr, d.kr),
                          tsgemm_partial_elems(d.m, d.kr, d.kr), tsgemm_partial_elems(d.p, (int)d.p, d.n_s),
                          tsgemm_partial_elems(d.p, 1, 1) * d.k * 16};
  for (size_t v : cands) pe = v > pe ? v : pe;
  w.part = c.take<double>(pe);
  w.part_elems = pe;
  w.total = c.used;
  return w;
}

}  // namespace

extern "C" {

size_t st_build_bases_workspace(int64_t N_s, int32_t N_t, int32_t n_mu, int32_t n_s, const int32_t* n_t,
                                int32_t gram_prec) {
  (void)gram_prec;
  PodDims d;
  if (!pod_dims(N_s, N_t, n_mu, n_s, n_t, &d)) return 0;
  return pod_ws(d, nullptr).total;
}

st_status st_build_bases(const void* U, int32_t U_prec, int64_t ldU, int64_t N_s, int32_t N_t, int32_t n_mu,
                         int32_t n_s, const int32_t* n_t, int32_t gram_prec, double tau_t, double* Phi_s,
                         double* Phi_t, double* sigma, int32_t* rank_t, double* diag, void* ws, size_t ws_bytes,
                         void* stream) {
  PodDims d;
  if (!U || !Phi_s || !Phi_t || !sigma || !ws || !pod_dims(N_s, N_t, n_mu, n_s, n_t, &d)) return ST_EINVAL;
  if (U_prec != ST_F64 && U_prec != ST_F32) return ST_EINVAL;
  if (gram_prec != ST_F64 && gram_prec != ST_F32 && gram_prec != ST_BF16X3) return ST_EINVAL;
  if (ldU < N_s || !(tau_t >= 0.0)) return ST_EINVAL;
  for (int i = 0; i < n_s; ++i)
    if (n_t[i] < 1 || n_t[i] > N_t) return ST_EINVAL;
  if ((int64_t)n_s > d.p) return ST_ERANK;
  if (n_s > kMaxModes || d.k > kMaxSubspace || n_mu > 64 || d.p > 0x7fffffff) return ST_EUNSUPPORTED;
  for (int i = 0; i < n_s; ++i)
    if (n_t[i] > 512) return ST_EUNSUPPORTED;
  if ((size_t)N_t * n_mu * sizeof(double) > 120 * 1024) return ST_EUNSUPPORTED;
  if (ws_bytes < st_build_bases_workspace(N_s, N_t, n_mu, n_s, n_t, gram_prec)) return ST_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PodWs w = pod_ws(d, ws);
  const int p = (int)d.p, k = d.k, ns = d.n_s, kr = d.kr;
  const bool f32in = U_prec == ST_F32;

  // a1: Gram of the snapshots (small side)
  if (!d.transposed)
    ST_TRY(launch_gram(N_s, p, U, U_prec, 1, ldU, gram_prec, w.G, w.part, w.part_elems, s));
  else
    ST_TRY(launch_gram(d.m, p, U, U_prec, ldU, 1, gram_prec, w.G, w.part, w.part_elems, s));

  // a2: subspace iteration on G, then Rayleigh-Ritz
  const uint64_t seed = 0x5EED1910ULL;
  ST_TRY(launch_rand_fill(w.X, p, k, seed, s));
  const OrthWork owk{w.oC, w.on0, w.oflag, w.part, w.part_elems};
  ST_TRY(launch_orth(w.X, p, k, seed + 1, owk, s));
  for (int it = 0; it < kSubspaceIters; ++it) {
    ST_TRY(launch_tsgemm(p, p, k, w.G, 1, p, w.X, 1, p, w.Y, p, w.part, w.part_elems, s));  // Y = G X
    ST_TRY(launch_copy_cols(w.Y, p, w.X, p, p, k, s));
    ST_TRY(launch_orth(w.X, p, k, seed + 2 + it, owk, s));
  }
  ST_TRY(launch_tsgemm(p, p, k, w.G, 1, p, w.X, 1, p, w.Y, p, w.part, w.part_elems, s));    // Y = G X
  ST_TRY(launch_tsgemm(p, k, k, w.X, 1, p, w.Y, 1, p, w.H, k, w.part, w.part_elems, s));    // H = X^T G X
  ST_TRY(launch_jacobi(k, w.H, w.Z, w.evals, w.Zs, s));
  ST_TRY(launch_tsgemm(k, p, k, w.X, p, 1, w.Zs, 1, k, w.Y, p, w.part, w.part_elems, s));   // Ritz vectors Y = X Zs
  // eigen-residual of the leading Ritz pairs (reported; the refinement below
  // makes the result independent of how far the iteration converged)
  ST_TRY(launch_tsgemm(p, p, ns, w.G, 1, p, w.Y, 1, p, w.X, p, w.part, w.part_elems, s));   // X = G Y (n_s cols)
  ST_TRY(launch_ritz_residual(w.X, w.Y, p, ns, w.evals, w.diag, s));

  // a3: SVD refinement in FP64.  The Gram squares the condition number of U
  // (its eigenvectors carry errors ~ eps sigma_1^2 / sigma_i^2, and modes below
  // ~sqrt(eps) sigma_1 are noise), so two half-steps of a subspace iteration in
  // factored form follow, each through U itself and each orthonormalised by a
  // one-sided Jacobi SVD (robust to the graded and nearly dependent columns
  // that plain Cholesky-QR would break down on):
  //   X0 = leading kr eigenvectors of the Gram (orthonormal, on its side)
  //   C1 = op(U) X0      -> Jacobi -> Y1 = normalised columns (other side)
  //   C2 = op(U)^T Y1    -> Jacobi with rotations J -> Z = normalised columns,
  //                         sigma = column norms, and Y1 J on the first side.
  // With a Gram U^T U (m <= N_s) the first side is R^m, so Phi_s = Z and V = Y1 J;
  // with U U^T the first side is R^N_s, so Phi_s = Y1 J and V = Z.
  // Jacobi stops when every pair has |cos| <= tol: 1e-14, widened for very long
  // columns where the rounding of the inner products themselves approaches it
  const double tol_s = 1e-14 * fmax(1.0, sqrt((double)N_s / 65536.0));
  const double tol_m = 1e-14 * fmax(1.0, sqrt((double)d.m / 65536.0));
  // scratch of the blocked Jacobi passes: the buffer that receives the run's normalised
  // columns afterwards (Y1 for C1, Y2 for C2) and the k x k areas of the eigen-step
  const TallJacobiWork wk1{w.Y1, w.H, w.Z, w.Zs, w.part, w.part_elems};
  const TallJacobiWork wk2{w.Y2, w.H, w.Z, w.Zs, w.part, w.part_elems};
  int fb = 0;  // pair-by-pair sweeps after a stalled blocked pass (diagnostic)
  const double* gfin = nullptr;  // Gram of a run's final columns, when its last step was a blocked pass
  if (!d.transposed) {
    // C1 = U X0 (N_s x kr), X0 = Y[:, :kr] in R^m
    if (f32in)
      ST_TRY(launch_tsgemm_xf(d.m, (int)N_s, kr, (const float*)U, ldU, 1, w.Y, 1, p, w.C1, (int)N_s, w.part,
                              w.part_elems, s));
    else
      ST_TRY(launch_tsgemm(d.m, (int)N_s, kr, (const double*)U, ldU, 1, w.Y, 1, p, w.C1, (int)N_s, w.part,
                           w.part_elems, s));
    ST_TRY(launch_tall_jacobi(w.C1, N_s, kr, nullptr, w.rot, w.offmax, kRefineSweeps, tol_s, wk1, &fb, &gfin, s));
    ST_TRY(launch_tall_jacobi_finish(w.C1, N_s, kr, nullptr, kr, w.rot, w.offmax, kRefineSweeps, fb, gfin, w.sigk,
                                     w.perm, w.Y1, nullptr, w.diag, s));
    // C2 = U^T Y1 (m x kr)
    if (f32in)
      ST_TRY(launch_tsgemm_xf(N_s, (int)d.m, kr, (const float*)U, 1, ldU, w.Y1, 1, N_s, w.C2, (int)d.m, w.part,
                              w.part_elems, s));
    else
      ST_TRY(launch_tsgemm(N_s, (int)d.m, kr, (const double*)U, 1, ldU, w.Y1, 1, N_s, w.C2, (int)d.m, w.part,
                           w.part_elems, s));
    ST_TRY(launch_tall_jacobi(w.C2, d.m, kr, w.J, w.rot, w.offmax, kRefineSweeps, tol_m, wk2, &fb, &gfin, s));
    ST_TRY(launch_tall_jacobi_finish(w.C2, d.m, kr, w.J, ns, w.rot, w.offmax, kRefineSweeps, fb, gfin, w.sig, w.perm,
                                     w.V, w.Jp, w.diag, s));
    // Phi_s = Y1 Jp (N_s x n_s)
    ST_TRY(launch_tsgemm(kr, (int)N_s, ns, w.Y1, N_s, 1, w.Jp, 1, kr, Phi_s, (int)N_s, w.part, w.part_elems, s));
  } else {
    // C1 = U^T X0 (m x kr), X0 = Y[:, :kr] in R^N_s
    if (f32in)
      ST_TRY(launch_tsgemm_xf(N_s, (int)d.m, kr, (const float*)U, 1, ldU, w.Y, 1, p, w.C2, (int)d.m, w.part,
                              w.part_elems, s));
    else
      ST_TRY(launch_tsgemm(N_s, (int)d.m, kr, (const double*)U, 1, ldU, w.Y, 1, p, w.C2, (int)d.m, w.part,
                           w.part_elems, s));
    ST_TRY(launch_tall_jacobi(w.C2, d.m, kr, nullptr, w.rot, w.offmax, kRefineSweeps, tol_m, wk2, &fb, &gfin, s));
    ST_TRY(launch_tall_jacobi_finish(w.C2, d.m, kr, nullptr, kr, w.rot, w.offmax, kRefineSweeps, fb, gfin, w.sigk,
                                     w.perm, w.Y2, nullptr, w.diag, s));
    // C2 = U Y1 (N_s x kr), Y1 in R^m
    if (f32in)
      ST_TRY(launch_tsgemm_xf(d.m, (int)N_s, kr, (const float*)U, ldU, 1, w.Y2, 1, d.m, w.C1, (int)N_s, w.part,
                              w.part_elems, s));
    else
      ST_TRY(launch_tsgemm(d.m, (int)N_s, kr, (const double*)U, ldU, 1, w.Y2, 1, d.m, w.C1, (int)N_s, w.part,
                           w.part_elems, s));
    ST_TRY(launch_tall_jacobi(w.C1, N_s, kr, w.J, w.rot, w.offmax, kRefineSweeps, tol_s, wk1, &fb, &gfin, s));
    ST_TRY(launch_tall_jacobi_finish(w.C1, N_s, kr, w.J, ns, w.rot, w.offmax, kRefineSweeps, fb, gfin, w.sig, w.perm,
                                     Phi_s, w.Jp, w.diag, s));
    // V = Y1 Jp (m x n_s)
    ST_TRY(launch_tsgemm(kr, (int)d.m, ns, w.Y2, d.m, 1, w.Jp, 1, kr, w.V, (int)d.m, w.part, w.part_elems, s));
  }
  ST_TRY(launch_sign_fix(Phi_s, N_s, ns, w.V, d.m, s));
  ST_TRY(launch_copy_cols(w.sig, ns, sigma, ns, ns, 1, s));
  if (diag) ST_TRY(launch_copy_cols(w.diag, ST_POD_DIAG, diag, ST_POD_DIAG, ST_POD_DIAG, 1, s));

  // a4: temporal bases
  ModeTable mt;
  memset(&mt, 0, sizeof(mt));
  mt.n_s = ns;
  for (int i = 0; i < ns; ++i) mt.nt[i] = n_t[i];
  ST_TRY(launch_mode_offsets(mt, w.moff, s));
  ST_TRY(launch_temporal_svd(w.V, d.m, N_t, n_mu, ns, w.moff, tau_t, Phi_t, rank_t, s));
  return ST_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// surrogate network and residual certificate
// ---------------------------------------------------------------------------
namespace {
bool mlp_ok(const st_mlp_shape* s) {
  return s && s->d_in >= 1 && s->width >= 1 && s->n_hidden >= 1 && s->n_hidden <= 62 && s->d_out >= 1 &&
         s->d_in <= 65536 && s->width <= 65536 && s->d_out <= 65536;
}

struct MlpWs {
  float *acts, *dY, *tmp0, *tmp1, *partial;
  size_t total;
};

MlpWs mlp_ws(const st_mlp_shape& s, int32_t batch, void* base) {
  Carver c(base);
  MlpWs w;
  w.acts = c.take<float>(mlp_act_elems(s, batch));
  w.dY = c.take<float>((size_t)batch * s.d_out);
  w.tmp0 = c.take<float>((size_t)batch * s.width);
  w.tmp1 = c.take<float>((size_t)batch * s.width);
  w.partial = c.take<float>(mlp_mse_partials((int64_t)batch * s.d_out) + 1);
  w.total = c.used;
  return w;
}
}  // namespace

extern "C" {

int64_t st_mlp_param_count(const st_mlp_shape* s) {
  if (!mlp_ok(s)) return -1;
  return (int64_t)mlp_param_offset(*s, mlp_layers(*s));
}

size_t st_mlp_workspace(const st_mlp_shape* s, int32_t batch) {
  if (!mlp_ok(s) || batch < 0) return 0;
  return mlp_ws(*s, batch, nullptr).total;
}

st_status st_mlp_forward(const st_mlp_shape* s, const float* params, int32_t batch, const float* X, float* Y,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!mlp_ok(s) || batch < 0) return ST_EINVAL;
  if (batch == 0) return ST_OK;
  if (!params || !X || !Y || !ws) return ST_EINVAL;
  if (ws_bytes < st_mlp_workspace(s, batch)) return ST_EWORKSPACE;
  MlpWs w = mlp_ws(*s, batch, ws);
  ST_TRY(mlp_forward(*s, params, batch, X, w.acts, Y, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

st_status st_mlp_grad(const st_mlp_shape* s, const float* params, int32_t batch, const float* X, const float* T,
                      float* grads, float* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!mlp_ok(s) || batch < 1 || !params || !X || !T || !grads || !loss || !ws) return ST_EINVAL;
  if (ws_bytes < st_mlp_workspace(s, batch)) return ST_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  MlpWs w = mlp_ws(*s, batch, ws);
  // forward into a scratch output (the last layer's Z slot of the activations)
  float* Y = w.acts + mlp_act_elems(*s, batch) - 2 * (size_t)batch * s->d_out;
  ST_TRY(mlp_forward(*s, params, batch, X, w.acts, Y, st));
  ST_TRY(mlp_mse((int64_t)batch * s->d_out, Y, T, w.dY, w.partial, loss, st));
  ST_TRY(mlp_backward(*s, params, batch, X, w.acts, w.dY, grads, w.tmp0, w.tmp1, st));
  return ST_OK;
}

st_status st_mlp_adam(int64_t n, float* params, const float* grads, float* m, float* v, int32_t step, float lr,
                      float beta1, float beta2, float eps, void* stream) {
  if (n < 0 || step < 1 || !(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return ST_EINVAL;
  if (n == 0) return ST_OK;
  if (!params || !grads || !m || !v) return ST_EINVAL;
  ST_TRY(adam(n, params, grads, m, v, step, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

st_status st_mlp_colstats(int32_t n, int32_t d, const double* C, double* mean, double* scale, void* stream) {
  if (n < 1 || d < 1 || !C || !mean || !scale) return ST_EINVAL;
  ST_TRY(mlp_colstats(n, d, C, mean, scale, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

st_status st_mlp_standardize(int32_t n, int32_t d, const double* C, const double* mean, const double* scale, float* T,
                             void* stream) {
  if (n < 0 || d < 1 || (n > 0 && (!C || !mean || !scale || !T))) return ST_EINVAL;
  ST_TRY(mlp_standardize(n, d, C, mean, scale, T, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

size_t st_surrogate_check_workspace(const st_rom_desc* d, int32_t n_q) {
  if (!desc_ok(d) || n_q < 0) return 0;
  const size_t n = (size_t)total_nt(d);
  size_t o = plan_bytes(n_q);
  o = align_up(o + sizeof(int64_t) * (n_q + 1));  // coeff offsets
  o = align_up(o + sizeof(int64_t) * (n_q + 1));  // matrix offsets (unused)
  o = align_up(o + sizeof(int32_t) * n_q);        // info
  o = align_up(o + sizeof(double) * n_q);         // ||r||
  o = align_up(o + sizeof(double) * n_q);         // ||c||
  o = align_up(o + sizeof(double) * n_q * n);     // b
  o = align_up(o + sizeof(double) * n_q * n);     // r
  return o;
}

st_status st_surrogate_check(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                             const double* theta_f, const double* theta_0, const float* Y, const double* mean,
                             const double* scale, double gamma, double tol, double* coeff, double* cert,
                             int32_t* accept, void* ws, size_t ws_bytes, void* stream) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0)) return ST_EINVAL;
  if (!(gamma > 0.0) || !(tol >= 0.0)) return ST_EINVAL;
  if (d->n_s > kMaxFormModes) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!Y || !mean || !scale || !coeff || !cert || !accept || !ws) return ST_EINVAL;
  const int64_t n = total_nt(d);
  if (n > kMaxWidth) return ST_EUNSUPPORTED;
  if (ws_bytes < st_surrogate_check_workspace(d, n_q)) return ST_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  RomView rv = view_of(d, rom);
  Carver c(ws);
  Plan plan;
  plan.width = c.take<int32_t>(n_q);
  plan.order = c.take<int32_t>(n_q);
  plan.counter = c.take<int32_t>(4);
  plan.coeff_off = c.take<int64_t>(n_q + 1);
  plan.mat_off = c.take<int64_t>(n_q + 1);
  plan.info = c.take<int32_t>(n_q);
  double* rnorm = c.take<double>(n_q);
  double* cnorm = c.take<double>(n_q);
  double* b = c.take<double>((size_t)n_q * n);
  double* r = c.take<double>((size_t)n_q * n);
  ST_TRY(launch_plan(n_q, d->n_s, rv.moff, nullptr, nullptr, theta_A, theta_f, theta_0, d->Q, d->Qf, d->Q0,
                     (int64_t)n_q * n, (int64_t)1 << 62, plan, s));
  ST_TRY(launch_destandardize(n_q, (int32_t)n, Y, mean, scale, plan, coeff, s));
  ST_TRY(launch_rhs(rv, n_q, theta_A, theta_f, theta_0, nullptr, plan, b, (int32_t)n, s));
  ST_TRY(launch_residual(rv, n_q, theta_A, nullptr, plan, b, coeff, r, rnorm, nullptr, (int32_t)n, s));
  ST_TRY(launch_vec_norms(n_q, plan, coeff, cnorm, s));
  ST_TRY(launch_certificate(n_q, plan, rnorm, cnorm, gamma, tol, cert, accept, nullptr, nullptr, s));
  return ST_OK;
}

double st_coercivity_floor(int32_t N_t) {
  if (N_t < 1) return 0.0;
  return 1.0 - cos(M_PI / (N_t + 1.0));
}

size_t st_certify_workspace(const st_rom_desc* d, int32_t n_q, int64_t coeff_cap) {
  if (!desc_ok(d) || n_q < 0 || coeff_cap < 0) return 0;
  size_t o = plan_bytes(n_q);
  o = align_up(o + sizeof(int64_t) * (n_q + 1));  // coeff offsets
  o = align_up(o + sizeof(int64_t) * (n_q + 1));  // matrix offsets (unused)
  o = align_up(o + sizeof(int32_t) * n_q);        // info
  o = align_up(o + sizeof(double) * n_q);         // ||r||
  o = align_up(o + sizeof(double) * n_q);         // ||c||
  o = align_up(o + sizeof(double) * n_q);         // ||b||
  o = align_up(o + sizeof(double) * coeff_cap);   // b
  o = align_up(o + sizeof(double) * coeff_cap);   // r
  return o;
}

namespace {
int32_t dict_cols(const st_rom_desc* d) { return d->n_s * (d->Q + 1) + d->Qf + d->Q0; }
}  // namespace

size_t st_fom_bound_workspace(const st_rom_desc* d, int64_t N_s, int32_t n_q) {
  if (!desc_ok(d) || N_s < 1 || n_q < 0) return 0;
  size_t o = plan_bytes(n_q);
  o = align_up(o + sizeof(int64_t) * (n_q + 1));                 // coeff offsets
  o = align_up(o + sizeof(int64_t) * (n_q + 1));                 // matrix offsets (unused)
  o = align_up(o + sizeof(int32_t) * n_q);                       // info
  o = align_up(o + sizeof(double) * (size_t)N_s * dict_cols(d));  // dictionary D
  return o;
}

st_status st_fom_bound(const st_rom_desc* d, const void* rom, int64_t N_s, const double* Phi_s, const st_csr* A,
                       const double* Bf, const double* g, const double* u0, int32_t n_q, const double* theta_A,
                       const double* theta_f, const double* theta_0, const int32_t* nt_q, const double* coeff,
                       int64_t coeff_cap, double inv_norm, double* res_inf, double* u_inf, double* bound, void* ws,
                       size_t ws_bytes, void* stream) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0)) return ST_EINVAL;
  if (N_s < 1 || N_s > 0x7fffffff || !Phi_s || !A || coeff_cap < 0 || !(inv_norm >= 0.0)) return ST_EINVAL;
  if (d->n_s > N_s) return ST_ERANK;
  if (d->Qf > 0 && !Bf) return ST_EINVAL;
  if (d->Q0 > 0 && !u0) return ST_EINVAL;
  for (int q = 0; q < d->Q; ++q) {
    if (A[q].n_rows != N_s || A[q].nnz < 0 || !A[q].row_ptr) return ST_EINVAL;
    if (A[q].nnz > 0 && (!A[q].col_idx || !A[q].val)) return ST_EINVAL;
  }
  if (d->n_s > kMaxFormModes || d->integrator != ST_BACKWARD_EULER) return ST_EUNSUPPORTED;
  if (fom_bound_lds_bytes(d->n_s, dict_cols(d)) > 160 * 1024) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!coeff || !res_inf || !u_inf || !bound || !ws) return ST_EINVAL;
  const int64_t n = total_nt(d);
  if (n > kMaxWidth) return ST_EUNSUPPORTED;
  if (ws_bytes < st_fom_bound_workspace(d, N_s, n_q)) return ST_EWORKSPACE;
  if (inv_norm == 0.0) inv_norm = 1.0 / st_coercivity_floor(d->N_t);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RomView rv = view_of(d, rom);
  Carver c(ws);
  Plan plan;
  plan.width = c.take<int32_t>(n_q);
  plan.order = c.take<int32_t>(n_q);
  plan.counter = c.take<int32_t>(4);
  plan.coeff_off = c.take<int64_t>(n_q + 1);
  plan.mat_off = c.take<int64_t>(n_q + 1);
  plan.info = c.take<int32_t>(n_q);
  const int32_t m_D = dict_cols(d);
  double* D = c.take<double>((size_t)N_s * m_D);
  ST_TRY(launch_plan(n_q, d->n_s, rv.moff, nt_q, nullptr, theta_A, theta_f, theta_0, d->Q, d->Qf, d->Q0, coeff_cap,
                     (int64_t)1 << 62, plan, s));
  ST_TRY(launch_fom_dict(N_s, d->n_s, d->Q, A, d->Qf, d->Q0, Phi_s, Bf, u0, D, m_D, s));
  ST_TRY(launch_fom_residual(rv, N_s, D, m_D, n_q, theta_A, theta_f, theta_0, g, nt_q, plan, coeff, inv_norm, res_inf,
                             u_inf, bound, s));
  return ST_OK;
}

st_status st_spatial_march(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                           const double* theta_f, const double* theta_0, const double* g, int32_t n_out,
                           const double* Chat, double* traj, double* outputs, int32_t* info, void* stream) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0) || n_out < 0) return ST_EINVAL;
  if (d->n_s > kMaxFormModes || spatial_march_lds_bytes(d->n_s, d->Qf) > 160 * 1024) return ST_EUNSUPPORTED;
  if (d->integrator != ST_BACKWARD_EULER) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!info || (outputs && (n_out < 1 || !Chat))) return ST_EINVAL;
  ST_TRY(launch_spatial_march(view_of(d, rom), n_q, theta_A, theta_f, theta_0, g, outputs ? n_out : 0, Chat, traj,
                              outputs, info, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

size_t st_project_workspace(int64_t N_s, int32_t n_s, int32_t k) {
  if (N_s < 1 || n_s < 1 || k < 0) return 0;
  return align_up(sizeof(double) * tsgemm_partial_elems(N_s, n_s, k)) + 256;
}

st_status st_project(int64_t N_s, int32_t n_s, const double* Phi_s, int32_t k, const double* X, double* out, void* ws,
                     size_t ws_bytes, void* stream) {
  if (N_s < 1 || n_s < 1 || k < 0 || n_s > N_s) return ST_EINVAL;
  if (k == 0) return ST_OK;
  if (!Phi_s || !X || !out || !ws) return ST_EINVAL;
  if (ws_bytes < st_project_workspace(N_s, n_s, k)) return ST_EWORKSPACE;
  ST_TRY(launch_tsgemm(N_s, n_s, k, Phi_s, 1, N_s, X, 1, N_s, out, n_s, static_cast<double*>(ws),
                       (ws_bytes - 256) / sizeof(double), static_cast<hipStream_t>(stream)));
  return ST_OK;
}

// ---------------------------------------------------------------------------
// incremental SVD
// ---------------------------------------------------------------------------
static_assert(ST_ISVD_STATE == kIsvdStateInts, "state size");
static_assert(ST_ISVD_MAX_RANK == kIsvdMaxRank, "rank limit");

static size_t isvd_part_elems(int64_t N_s, int32_t r_max) {
  const int64_t a = (int64_t)isvd_row_blocks(N_s) * (r_max + 1);
  const int64_t b = (N_s + 63) / 64;  // one partial per 64-row block of the W update
  return (size_t)(a > b ? a : b);
}

static IsvdArgs isvd_carve(int64_t N_s, int32_t r_max, void* ws, size_t* total) {
  Carver c(ws);
  IsvdArgs a;
  memset(&a, 0, sizeof(a));
  const size_t q = (size_t)(r_max + 1) * (r_max + 1) + 16;  // + the tail read by the 8-column passes
  a.l1 = c.take<double>(r_max + 1);
  a.l2 = c.take<double>(r_max + 1);
  a.scal = c.take<double>(8);
  a.part = c.take<double>(isvd_part_elems(N_s, r_max));
  a.res = c.take<double>((size_t)N_s);
  a.UqT = c.take<double>(q);
  a.VqT = c.take<double>(q);
  if (total) *total = c.used;
  return a;
}

size_t st_gram_workspace(int64_t K, int32_t p) {
  if (K < 1 || p < 1 || p > 65535) return 0;
  return align_up(sizeof(double) * gram_partial_elems(K, p));
}

st_status st_gram(const void* X, int32_t X_prec, int64_t ld, int64_t K, int32_t p, int32_t gram_prec, double* G,
                  void* ws, size_t ws_bytes, void* stream) {
  if (!X || !G || !ws || K < 1 || p < 1 || ld < K) return ST_EINVAL;
  if (X_prec != ST_F64 && X_prec != ST_F32) return ST_EINVAL;
  if (gram_prec != ST_F64 && gram_prec != ST_F32 && gram_prec != ST_BF16X3) return ST_EINVAL;
  if (p > 65535) return ST_EUNSUPPORTED;
  if (ws_bytes < st_gram_workspace(K, p)) return ST_EWORKSPACE;
  ST_TRY(launch_gram(K, p, X, X_prec, 1, ld, gram_prec, G, static_cast<double*>(ws), ws_bytes / sizeof(double),
                     static_cast<hipStream_t>(stream)));
  return ST_OK;
}

size_t st_isvd_workspace(int64_t N_s, int32_t r_max) {
  if (N_s < 1 || r_max < 1 || r_max > kIsvdMaxRank) return 0;
  size_t total = 0;
  isvd_carve(N_s, r_max, nullptr, &total);
  return total;
}

st_status st_isvd_reset(int32_t* state, void* stream) {
  if (!state) return ST_EINVAL;
  ST_TRY(launch_isvd_reset(state, static_cast<hipStream_t>(stream)));
  return ST_OK;
}

st_status st_isvd_update(const double* U, int64_t ldU, int64_t N_s, int32_t b, int32_t r_max, int64_t m_max,
                         double eps_svd, double eps_sv, double* W, double* s, double* V, int32_t* state, void* ws,
                         size_t ws_bytes, void* stream) {
  if (N_s < 1 || b < 0 || m_max < 1 || ldU < N_s) return ST_EINVAL;
  if (r_max < 1) return ST_EINVAL;
  if (r_max > kIsvdMaxRank) return ST_EUNSUPPORTED;
  if (!(eps_svd >= 0.0) || !(eps_sv >= 0.0) || !std::isfinite(eps_svd) || !std::isfinite(eps_sv)) return ST_EINVAL;
  if (!W || !s || !V || !state || !ws || (b > 0 && !U)) return ST_EINVAL;
  if (ws_bytes < st_isvd_workspace(N_s, r_max)) return ST_EWORKSPACE;
  IsvdArgs a = isvd_carve(N_s, r_max, ws, nullptr);
  a.N_s = N_s;
  a.r_max = r_max;
  a.m_max = m_max;
  a.eps_svd = eps_svd;
  a.eps_sv = eps_sv;
  a.W = W;
  a.s = s;
  a.V = V;
  a.state = state;
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int32_t c = 0; c < b; ++c) ST_TRY(launch_isvd_step(a, U + (int64_t)c * ldU, st));
  return ST_OK;
}

size_t st_isvd_bases_workspace(int32_t N_t, int32_t n_mu, int32_t n_s) {
  if (N_t < 1 || n_mu < 1 || n_s < 1) return 0;
  Carver c(nullptr);
  c.take<double>((size_t)N_t * n_mu * n_s);
  c.take<int32_t>(n_s + 1);
  return c.used;
}

st_status st_isvd_bases(const double* W, const double* s, const double* V, const int32_t* state, int64_t N_s,
                        int64_t m_max, int32_t N_t, int32_t n_mu, int32_t n_s, const int32_t* n_t, double tau_t,
                        double* Phi_s, double* Phi_t, double* sigma, int32_t* rank_t, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!W || !s || !V || !state || !n_t || !Phi_s || !Phi_t || !sigma || !ws) return ST_EINVAL;
  if (N_s < 1 || N_t < 1 || n_mu < 1 || n_s < 1 || !(tau_t >= 0.0)) return ST_EINVAL;
  const int64_t m = (int64_t)N_t * n_mu;
  if (m > m_max || n_s > N_s) return ST_EINVAL;
  for (int i = 0; i < n_s; ++i)
    if (n_t[i] < 1 || n_t[i] > N_t) return ST_EINVAL;
  if (n_s > kMaxModes || n_mu > 64 || (size_t)m * sizeof(double) > 120 * 1024) return ST_EUNSUPPORTED;
  for (int i = 0; i < n_s; ++i)
    if (n_t[i] > 512) return ST_EUNSUPPORTED;
  if (ws_bytes < st_isvd_bases_workspace(N_t, n_mu, n_s)) return ST_EWORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  int32_t hs[2];
  if (hipMemcpyAsync(hs, state, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return ST_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return ST_EDEVICE;
  if (hs[1] != m || hs[0] < 0) return ST_EINVAL;
  const int rc = hs[0] < n_s ? hs[0] : n_s;
  Carver c(ws);
  double* Vs = c.take<double>((size_t)m * n_s);
  int32_t* moff = c.take<int32_t>(n_s + 1);
  if (rc > 0) {
    ST_TRY(launch_copy_cols(W, N_s, Phi_s, N_s, N_s, rc, st));
    ST_TRY(launch_copy_cols(V, m_max, Vs, m, m, rc, st));
    ST_TRY(launch_copy_cols(s, rc, sigma, rc, rc, 1, st));
  }
  if (rc < n_s) {
    ST_TRY(launch_fill_f64(Phi_s + (int64_t)rc * N_s, (int64_t)(n_s - rc) * N_s, 0.0, st));
    ST_TRY(launch_fill_f64(Vs + (int64_t)rc * m, (int64_t)(n_s - rc) * m, 0.0, st));
    ST_TRY(launch_fill_f64(sigma + rc, n_s - rc, 0.0, st));
  }
  ST_TRY(launch_sign_fix(Phi_s, N_s, n_s, Vs, m, st));
  ModeTable mt;
  memset(&mt, 0, sizeof(mt));
  mt.n_s = n_s;
  for (int i = 0; i < n_s; ++i) mt.nt[i] = n_t[i];
  ST_TRY(launch_mode_offsets(mt, moff, st));
  ST_TRY(launch_temporal_svd(Vs, m, N_t, n_mu, n_s, moff, tau_t, Phi_t, rank_t, st));
  return ST_OK;
}

st_status st_certify(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A, const double* theta_f,
                     const double* theta_0, const int32_t* nt_q, const double* coeff, int64_t coeff_cap, double gamma,
                     double* relres, double* cert, void* ws, size_t ws_bytes, void* stream) {
  if (!query_args_ok(d, rom, n_q, theta_A, theta_f, theta_0)) return ST_EINVAL;
  if (!(gamma >= 0.0) || coeff_cap < 0) return ST_EINVAL;
  if (d->n_s > kMaxFormModes) return ST_EUNSUPPORTED;
  if (n_q == 0) return ST_OK;
  if (!coeff || !relres || !cert || !ws) return ST_EINVAL;
  const int64_t n = total_nt(d);
  if (n > kMaxWidth) return ST_EUNSUPPORTED;
  if (ws_bytes < st_certify_workspace(d, n_q, coeff_cap)) return ST_EWORKSPACE;
  if (gamma == 0.0) gamma = st_coercivity_floor(d->N_t);
  hipStream_t s = static_cast<hipStream_t>(stream);
  RomView rv = view_of(d, rom);
  Carver c(ws);
  Plan plan;
  plan.width = c.take<int32_t>(n_q);
  plan.order = c.take<int32_t>(n_q);
  plan.counter = c.take<int32_t>(4);
  plan.coeff_off = c.take<int64_t>(n_q + 1);
  plan.mat_off = c.take<int64_t>(n_q + 1);
  plan.info = c.take<int32_t>(n_q);
  double* rnorm = c.take<double>(n_q);
  double* cnorm = c.take<double>(n_q);
  double* bnorm = c.take<double>(n_q);
  double* b = c.take<double>(coeff_cap);
  double* r = c.take<double>(coeff_cap);
  ST_TRY(launch_plan(n_q, d->n_s, rv.moff, nt_q, nullptr, theta_A, theta_f, theta_0, d->Q, d->Qf, d->Q0, coeff_cap,
                     (int64_t)1 << 62, plan, s));
  ST_TRY(launch_rhs(rv, n_q, theta_A, theta_f, theta_0, nt_q, plan, b, (int32_t)n, s));
  ST_TRY(launch_residual(rv, n_q, theta_A, nt_q, plan, b, coeff, r, rnorm, nullptr, (int32_t)n, s));
  ST_TRY(launch_vec_norms(n_q, plan, coeff, cnorm, s));
  ST_TRY(launch_vec_norms(n_q, plan, b, bnorm, s));
  ST_TRY(launch_certificate(n_q, plan, rnorm, cnorm, gamma, 0.0, cert, nullptr, bnorm, relres, s));
  return ST_OK;
}

}  // extern "C"
