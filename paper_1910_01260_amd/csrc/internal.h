// Internal declarations shared by the host API and the HIP kernel files of
// the ST-ROM library (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/strom.h"

namespace strom {

constexpr int kMaxModes = 512;     // n_s limit of the index-table kernels (by-value arguments)
constexpr int kMaxFormModes = 128; // n_s limit of the query kernels (Ahat(mu) staged in LDS)
constexpr int kMaxTerms = 16;      // Q, Qf, Q0 limit of the query kernels
constexpr int kMaxWidth = 4096;    // reduced width limit of the query kernels

struct ModeTable {
  int32_t n_s;
  int32_t nt[kMaxModes];
};

// Device view of a ROM buffer.
struct RomView {
  const double* Ahat;   // Q x n_s x n_s
  const double* bhat;   // Qf x n_s
  const double* u0hat;  // Q0 x n_s
  const double* T;      // n x n
  const double* K;      // sum n_t^2
  const double* Wf;     // Qf x n
  const double* P1;     // n
  const int32_t* mode;  // n
  const int32_t* moff;  // n_s + 1
  const int64_t* koff;  // n_s + 1
  const double* Phit;   // N_t x n, column-major (the concatenated temporal bases)
  const double* dt;     // N_t
  const float* T32;     // n x n, the assembly's T rounded to FP32, row-major
  const double* Teff;   // n x n read as row-major: T (symmetric) or, Crank-Nicolson, T_cn
  const double* Au0;    // Q x Q0 x n_s (Crank-Nicolson): Phi_s^T A_q u0_q0
  int32_t n_s, N_t, n, Q, Qf, Q0;
  int32_t integ;        // ST_BACKWARD_EULER or ST_CRANK_NICOLSON
};

struct MutRomView {
  double *Ahat, *bhat, *u0hat, *T, *K, *Wf, *P1;
  int32_t *mode, *moff;
  int64_t* koff;
  double *Phit, *dt;
  float* T32;
  double *Tcn, *Au0;
};

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Query-batch plan written by the plan kernel (device memory in the workspace).
struct Plan {
  int32_t* width;      // n_q
  int32_t* order;      // n_q, queries sorted by width, largest first
  int64_t* mat_off;    // n_q + 1, element offsets of the query matrices
  int64_t* coeff_off;  // n_q + 1, offsets of the query vectors
  int32_t* info;       // n_q
  int32_t* counter;    // 4 work-queue counters
};

// ----------------------------------------------------------------------------
// kernel launchers (each defined in the .hip file that holds the kernel)
// ----------------------------------------------------------------------------

// k_offline.hip: projection (a5) and temporal contractions (a6)
hipError_t launch_index_tables(const ModeTable& mt, int32_t N_t, MutRomView rom, hipStream_t s);
hipError_t launch_transpose(const double* src, int64_t rows, int32_t cols, int64_t ld, double* dst, hipStream_t s);
hipError_t launch_spmm_rowmajor(const st_csr& A, const double* Xr, int32_t p, double* Yr, hipStream_t s);
// C (p x q, column-major, ldc) = X^T Y over N rows; X element (r,a) at X[r*xrs + a*xcs]
hipError_t launch_tsgemm(int64_t N, int32_t p, int32_t q, const double* X, int64_t xrs, int64_t xcs,
                         const double* Y, int64_t yrs, int64_t ycs, double* C, int32_t ldc, double* partial,
                         size_t partial_elems, hipStream_t s);
hipError_t launch_tsgemm_w(int64_t N, int32_t p, int32_t q, const double* X, int64_t xrs, int64_t xcs,
                           const double* Y, int64_t yrs, int64_t ycs, const double* wrow, double* C, int32_t ldc,
                           double* partial, size_t partial_elems, hipStream_t s);
hipError_t launch_tsgemm_xf(int64_t N, int32_t p, int32_t q, const float* X, int64_t xrs, int64_t xcs,
                            const double* Y, int64_t yrs, int64_t ycs, double* C, int32_t ldc, double* partial,
                            size_t partial_elems, hipStream_t s);
size_t tsgemm_partial_elems(int64_t N, int32_t p, int32_t q);
// out = A V (A, out m x k and V k x k, column-major; k <= 256; no overlap)
hipError_t launch_mul_small(const double* A, int64_t m, int32_t k, const double* V, double* out, hipStream_t s);
// reduced-precision projection: Z = [Phi_s, A Phi_s] in FP32 (row-major N x 2p), then the
// Phi_s^T (A Phi_s) block of its Gram
hipError_t launch_pack_basis_f32(const double* Phi, int64_t N, int32_t p, float* Z, hipStream_t s);
hipError_t launch_spmm_f32(const st_csr& A, int32_t p, float* Z, hipStream_t s);
hipError_t launch_extract_block(const double* G, int32_t p, double* Ahat, hipStream_t s);
hipError_t launch_mode_offsets(const ModeTable& mt, int32_t* moff, hipStream_t s);
hipError_t launch_round_f32(const double* src, int64_t n, float* dst, hipStream_t s);
// T_cn (row-major) = (T + S)/2 from column-major T and S (n x n)
hipError_t launch_combine_cn(const double* T, const double* S, int32_t n, double* Tcn, hipStream_t s);
hipError_t launch_temporal(const double* Phi_t, int32_t N_t, int32_t n, const double* dt, const double* g, int32_t Qf,
                           const ModeTable& mt, MutRomView rom, hipStream_t s);

// k_pod.hip: POD (a1-a4)
size_t gram_partial_elems(int64_t K, int p);
hipError_t launch_gram(int64_t K, int p, const void* X, int in_prec, int64_t ks, int64_t ms, int gram_prec, double* G,
                       double* partial, size_t partial_elems, hipStream_t s);
hipError_t launch_rand_fill(double* X, int64_t p, int k, uint64_t seed, hipStream_t s);
// Work areas of launch_orth's blocked sweep for columns too long for LDS: C (k x 16), n0sq
// (16), flag (1 int), part (split partials of the block products, part_elems doubles).
// All null: one workgroup sweeps the columns in global memory.
struct OrthWork {
  double *C, *n0sq;
  int* flag;
  double* part;
  size_t part_elems;
};
hipError_t launch_orth(double* X, int64_t p, int k, uint64_t seed, const OrthWork& wk, hipStream_t s);
hipError_t launch_jacobi(int k, double* A, double* Z, double* evals, double* Zout, hipStream_t s);
hipError_t launch_chol_inv(int n, double* S, double* Rinv, hipStream_t s);
hipError_t launch_scale_or_refill(double* X, int64_t p, int k, const double* sigma, double cut, uint64_t seed,
                                  hipStream_t s);
hipError_t launch_sqrt_clamp(const double* lam, double* sigma, int n, hipStream_t s);
hipError_t launch_sign_fix(double* X, int64_t p, int k, double* Y, int64_t py, hipStream_t s);
hipError_t launch_copy_cols(const double* src, int64_t ld_src, double* dst, int64_t ld_dst, int64_t p, int n,
                            hipStream_t s);
// Work areas of the blocked passes of launch_tall_jacobi: A2 (m x k), G, V and J2
// (k x k each; J2 only with J), part (the split partials of A^T A, part_elems
// doubles).  A2 == nullptr keeps the pair-by-pair sweeps throughout.
struct TallJacobiWork {
  double *A2, *G, *V, *J2, *part;
  size_t part_elems;
};
// one-sided Jacobi SVD of the tall m x k matrix A (in place), rotations accumulated in J
hipError_t launch_tall_jacobi(double* A, int64_t m, int k, double* J, int* rot, double* offmax, int max_sweeps,
                              double tol, const TallJacobiWork& wk, int* fallback_sweeps, const double** final_gram,
                              hipStream_t s);
// fallback_sweeps: the pair-by-pair sweeps that followed a stalled blocked pass (into diag[4]);
// G (may be null): the k x k Gram of the final columns, whose diagonal then gives the norms
// (launch_tall_jacobi's final_gram: set when its last step was a blocked pass that rotated nothing)
hipError_t launch_tall_jacobi_finish(const double* A, int64_t m, int k, const double* J, int n_out, const int* rot,
                                     const double* offmax, int max_sweeps, int fallback_sweeps, const double* G,
                                     double* sigma, int* perm, double* V, double* Jp, double* diag, hipStream_t s);
hipError_t launch_ritz_residual(const double* GY, const double* Y, int64_t p, int n, const double* evals, double* diag,
                                hipStream_t s);
hipError_t launch_temporal_svd(const double* V, int64_t ldV, int N_t, int n_mu, int n_s, const int32_t* moff,
                               double tau_t, double* Phi_t, int32_t* rank_out, hipStream_t s);

// k_query.hip: plan (per-query offsets), assembly (a7), residual
hipError_t launch_plan(int32_t n_q, int32_t n_s, const int32_t* full_nt_dev, const int32_t* nt_q, const int32_t* skip,
                       const double* thA, const double* thf, const double* th0, int32_t Q, int32_t Qf, int32_t Q0,
                       int64_t coeff_cap, int64_t mat_cap, Plan plan, hipStream_t s);
hipError_t launch_rhs(const RomView& rom, int32_t n_q, const double* thA, const double* thf, const double* th0,
                      const int32_t* nt_q,
                      Plan plan, double* rhs, int32_t n_max, hipStream_t s);
hipError_t launch_destandardize(int32_t n_q, int32_t n, const float* Y, const double* mean, const double* scale,
                                Plan plan, double* coeff, hipStream_t s);
hipError_t launch_certificate(int32_t n_q, Plan plan, const double* rnorm, const double* cnorm, double gamma, double tol,
                              double* cert, int32_t* accept, const double* bnorm, double* relres, hipStream_t s);
hipError_t launch_form(const RomView& rom, int32_t n_q, const double* thA, const double* thf, const double* th0,
                       const int32_t* nt_q, Plan plan, int32_t out_prec, void* mats, double* rhs, int32_t n_max,
                       hipStream_t s);
hipError_t launch_residual(const RomView& rom, int32_t n_q, const double* thA, const int32_t* nt_q, Plan plan,
                           const double* rhs, const double* x, double* r, double* rnorm, const int32_t* active,
                           int32_t n_max, hipStream_t s);

// k_lu.hip: batched LU (a8) and triangular solves
int lu_variant_count(int32_t prec, int32_t n_max);
int lu_outer_block(int32_t prec, int32_t n_max, int variant);
hipError_t launch_lu(int32_t n_q, Plan plan, int32_t prec, void* mats, int32_t* piv, int32_t n_max, int variant,
                     hipStream_t s);

// k_bound.hip: full-order space-time residual and Theorem-3 bound per query
size_t fom_bound_lds_bytes(int n_s, int m_D);
hipError_t launch_fom_dict(int64_t N_s, int32_t n_s, int32_t Q, const st_csr* A, int32_t Qf, int32_t Q0,
                           const double* Phi_s, const double* Bf, const double* u0, double* D, int32_t m_D,
                           hipStream_t s);
hipError_t launch_fom_residual(const RomView& rom, int64_t N_s, const double* D, int32_t m_D, int32_t n_q,
                               const double* thA, const double* thf, const double* th0, const double* g,
                               const int32_t* nt_q, Plan plan, const double* coeff, double inv_norm, double* res_inf,
                               double* u_inf, double* bound, hipStream_t s);

// k_spatial.hip: spatial-ROM time march and outputs
size_t spatial_march_lds_bytes(int n_s, int Qf);
hipError_t launch_spatial_march(const RomView& rom, int32_t n_q, const double* thA, const double* thf,
                                const double* th0, const double* g, int32_t n_out, const double* Chat, double* traj,
                                double* outs, int32_t* info, hipStream_t s);

hipError_t launch_reconstruct(int64_t N_s, int32_t N_t, int32_t n_s, const double* Phi_s, int64_t ldp,
                              const double* Phi_t, int64_t ldt, const int32_t* moff, const int32_t* nt_q, int32_t n_q,
                              const double* coeff, const int64_t* coeff_off, double* out, int64_t ldo,
                              hipStream_t s);

// True while st_solve records its launches into a HIP graph: launchers then skip
// hipFuncSetAttribute (set on the eager run that precedes every capture).
// incremental SVD of a snapshot stream (k_isvd.hip)
constexpr int kIsvdMaxRank = 256;   // r_max limit (the bordered SVD keeps r_max + 1 coordinates in LDS)
constexpr int kIsvdStateInts = 16;  // device state words
struct IsvdArgs {
  int64_t N_s;
  int32_t r_max;
  int64_t m_max;
  double eps_svd, eps_sv;
  double *W, *s, *V;
  int32_t* state;
  double *l1, *l2, *scal, *part, *res, *UqT, *VqT;
};
int64_t isvd_rows_per_block(int64_t N_s);
int isvd_row_blocks(int64_t N_s);
size_t isvd_apply_lds_bytes(int r_max);
hipError_t launch_isvd_reset(int32_t* state, hipStream_t s);
// one snapshot u (N_s) through the five launches of the update
hipError_t launch_isvd_step(const IsvdArgs& a, const double* u, hipStream_t s);
extern bool g_capturing;
// x (or x += solution when accumulate) for every active query: solve LU x = b
hipError_t launch_lu_solve(int32_t n_q, Plan plan, int32_t prec, const void* mats, const int32_t* piv, const double* b,
                           double* x, int accumulate, const int32_t* active, int32_t n_max, int nbo, hipStream_t s);
// refinement bookkeeping: relres, convergence flags, NaN for failed queries
hipError_t launch_ir_check(int32_t n_q, Plan plan, const double* rnorm, const double* bnorm, double tol, int32_t step,
                           int32_t last, int32_t* active, double* relres, int32_t* iters, hipStream_t s);
hipError_t launch_vec_norms(int32_t n_q, Plan plan, const double* v, double* norms, hipStream_t s);
hipError_t launch_finalize(int32_t n_q, Plan plan, double* coeff, int32_t* info_out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t s);
// FP64 re-solve of queries whose FP32 refinement did not converge (info -1 -> -6)
hipError_t launch_fallback_plan(int32_t n_q, Plan plan, Plan fb, int32_t* active, int64_t mat_cap, hipStream_t s);
hipError_t launch_fallback_finish(int32_t n_q, Plan plan, Plan fb, const int32_t* active, hipStream_t s);

// k_mlp.hip: surrogate network
int mlp_layers(const st_mlp_shape& s);
int mlp_in(const st_mlp_shape& s, int l);
int mlp_out(const st_mlp_shape& s, int l);
size_t mlp_param_offset(const st_mlp_shape& s, int l);
size_t mlp_act_elems(const st_mlp_shape& s, int32_t batch);
size_t mlp_mse_partials(int64_t n);
hipError_t mlp_forward(const st_mlp_shape& s, const float* params, int32_t batch, const float* X, float* acts,
                       float* Y, hipStream_t st);
hipError_t mlp_backward(const st_mlp_shape& s, const float* params, int32_t batch, const float* X, const float* acts,
                        float* dY, float* grads, float* tmp0, float* tmp1, hipStream_t st);
hipError_t mlp_mse(int64_t n, const float* Y, const float* T, float* dY, float* partial, float* loss, hipStream_t st);
hipError_t mlp_colstats(int n, int d, const double* C, double* mean, double* scale, hipStream_t st);
hipError_t mlp_standardize(int n, int d, const double* C, const double* mean, const double* scale, float* T,
                           hipStream_t st);
hipError_t adam(int64_t n, float* p, const float* g, float* m, float* v, int32_t t, float lr, float b1, float b2,
                float eps, hipStream_t st);

}  // namespace strom
