/*
 * strom.h - C ABI of the space-time reduced-order model (ST-ROM) hot path on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Choi, Brown, Arrighi, Anderson, "Space-time reduced order model for
 * large-scale linear dynamical systems with application to Boltzmann
 * transport problems".  The system is du/dt = A(mu) u + B f(t; mu),
 * u(0) = u0(mu) (Sec. 2, Eq. (Dynamicalstate)), discretised by backward Euler
 * with steps dt_k (Sec. 2, Eq. (fom)).  The library provides:
 *
 *   st_build_bases  POD of the snapshot matrix: spatial basis Phi_s and one
 *                   temporal basis per spatial mode (Sec. 4.1).
 *   st_assemble     projection of the affine operator terms onto Phi_s
 *                   (Sec. 3.1, Eq. (galerkin)) and the mu-independent
 *                   temporal contractions of the block formulas (Sec. 4.3).
 *   st_form         per-query reduced space-time system Ahat_st(mu) and
 *                   right-hand side (Sec. 4.3, Eq. (ij-block-matrix),
 *                   (j-block-vector), and the projection of u0_st).
 *   st_solve        per-query reduced solve Ahat_st c = fhat_st + u0hat_st
 *                   (Sec. 3.2, Eq. (st-galerkin)) for a ragged batch.
 *   st_isvd_*       incremental SVD of a snapshot stream and the bases taken
 *                   from it (Sec. 4.2, Alg. 1-2).
 *   st_mlp_*        a surrogate network mu -> c with a residual check
 *                   (not part of the paper; see the st_mlp section).
 *
 * Conventions (all entry points):
 *   - Every pointer marked [dev] is device memory owned by the caller; the
 *     library never frees it and never keeps it after the call returns.
 *     Pointers marked [host] are read during the call only.
 *   - Dense matrices are column-major FP64 unless stated otherwise.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and is asynchronous: outputs are valid once the caller has
 *     synchronised that stream.  The library allocates no device memory in
 *     st_solve/st_form/st_mlp_*: the caller passes a workspace whose size is
 *     given by the matching *_workspace function.  st_build_bases and
 *     st_assemble likewise take a caller workspace.
 *   - Argument errors are detected on the host before any launch and
 *     reported through the return value; nothing is written then.
 *   - Per-query numerical outcomes are written to a device `info` array:
 *        0  success
 *       k>0 the LU met an exactly zero pivot at step k (1-based); the
 *           query's coefficients are set to NaN
 *       -1  iterative refinement did not reach ir_tol in ir_max steps (the
 *           last iterate is returned); with an FP32 LU only when the FP64
 *           re-solve below did not fit in the workspace
 *       -6  the FP32-LU refinement did not reach ir_tol; the query was
 *           re-formed and re-solved with an FP64 LU (a valid result: relres
 *           is the FP64 solution's residual)
 *       -2  not solved: skipped on request (st_solve's skip mask)
 *       -3  the query did not fit in the coefficient or workspace capacity
 *       -4  invalid per-query temporal profile (nt_q out of range)
 *       -5  non-finite parameter coefficient
 *   - Reduced coordinates are ordered mode-major: spatial mode i's temporal
 *     coefficients j = 0..n_t,i-1 are contiguous.  This is the paper's
 *     ordering i + n_s (j-1) of Eq. (spacetimebasis) up to a symmetric
 *     permutation, and it allows a different temporal basis size per mode.
 */
#ifndef STROM_H
#define STROM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t st_status;

#define ST_OK 0
#define ST_EINVAL (-1)        /* invalid argument (shape, null pointer, range) */
#define ST_EDEVICE (-2)       /* a HIP call failed */
#define ST_EWORKSPACE (-3)    /* workspace or output buffer too small */
#define ST_ERANK (-4)         /* requested basis exceeds the data (n_s > min(N_s, n_mu N_t)) */
#define ST_EUNSUPPORTED (-5)  /* size or precision outside what the kernels handle */

/* arithmetic precisions */
#define ST_F64 0
#define ST_F32 1
#define ST_BF16X3 2           /* split-BF16: x = hi + lo, hi*hi + hi*lo + lo*hi, FP32 accumulate */

/* Static, NUL-terminated description of a status code. */
const char* st_strerror(st_status s);

/* ABI version (incremented on incompatible change). */
int32_t st_version(void);

/* ------------------------------------------------------------------------
 * Square sparse matrix in CSR form; all arrays [dev].  Column indices within
 * a row need not be sorted.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n_rows;          /* N_s */
  int64_t nnz;
  const int32_t* row_ptr;  /* [dev] n_rows + 1 */
  const int32_t* col_idx;  /* [dev] nnz */
  const double* val;       /* [dev] nnz */
} st_csr;

/* ------------------------------------------------------------------------
 * Shape of a reduced model.
 *   n_s    number of spatial modes
 *   N_t    number of time steps
 *   Q      number of affine terms of A(mu) = sum_q theta_A[q] A_q      (>= 1)
 *   Qf     number of input terms  B f^(k) = sum_q theta_f[q] g[k,q] Bf_q (>= 0)
 *   Q0     number of initial-state terms u0 = sum_q theta_0[q] u0_q    (>= 0)
 *   n_t    [host] n_s entries: temporal basis size of each mode (1..N_t);
 *          queries may use any prefix of each mode's basis.
 *   integrator  ST_BACKWARD_EULER (the paper's, Sec. 2 Eq. (fom)) or
 *          ST_CRANK_NICOLSON: (I - dt_k/2 A) u^(k) = (I + dt_k/2 A) u^(k-1)
 *          + dt_k B f^(k), the other block structure Sec. 2 mentions.  The
 *          reduced operator then uses T_cn = (T + S)/2 with
 *          S[a,b] = sum_{k>1} dt_k phi_a(k) phi_b(k-1) in place of T, and the
 *          initial vector phi_a(1) (Phi_s^T (I + dt_1/2 A(mu)) u0)_i.  The input
 *          g[k] is the input of step k (for a time-varying input under
 *          Crank-Nicolson, the average of its values at the step's two ends).
 * n = sum_i n_t[i] is the full reduced dimension.
 * ---------------------------------------------------------------------- */
#define ST_BACKWARD_EULER 0
#define ST_CRANK_NICOLSON 1
typedef struct {
  int32_t n_s;
  int32_t N_t;
  int32_t Q;
  int32_t Qf;
  int32_t Q0;
  const int32_t* n_t;
  int32_t integrator;
} st_rom_desc;

/* Byte offsets of the sections of a ROM buffer (filled by st_rom_layout).
 * All sections are FP64 except the index tables (int32, int64) and T32.
 *   Ahat   Q  x (n_s x n_s)  Ahat_q = Phi_s^T A_q Phi_s           (Eq. (galerkin))
 *   bhat   Qf x n_s          Phi_s^T Bf_q
 *   u0hat  Q0 x n_s          Phi_s^T u0_q
 *   T      n x n             T[a,b] = sum_k dt_k phi_a(k) phi_b(k)  (weighted temporal Gram)
 *   K      sum_i n_t,i^2     per mode, column-major n_t,i x n_t,i:
 *                            K_i[j',j] = sum_k phi_ij'(k) phi_ij(k) - sum_{k<N_t} phi_ij'(k+1) phi_ij(k)
 *   Wf     Qf x n            Wf[q,a] = sum_k dt_k g[k,q] phi_a(k)
 *   P1     n                 P1[a] = phi_a(first step)
 *   mode   n (int32)         spatial mode of reduced index a
 *   moff   n_s + 1 (int32)   mode offsets into the reduced index
 *   koff   n_s + 1 (int64)   element offsets of each K_i inside K
 *   Phit   N_t x n           the concatenated temporal bases, column-major (Phit[k + N_t a] = phi_a(k))
 *   dt     N_t               the time steps
 *   T32    n x n (FP32)      the assembly's T (T, or T_cn) rounded to FP32, row-major
 *   Tcn    n x n             Crank-Nicolson only: T_cn = (T + S)/2, row-major
 *   Au0    Q x Q0 x n_s      Crank-Nicolson only: Phi_s^T A_q u0_q0
 * where phi_a is column a of the concatenated temporal bases (mode-major).
 */
typedef struct {
  size_t Ahat, bhat, u0hat, T, K, Wf, P1, mode, moff, koff, Phit, dt, T32, Tcn, Au0, total;
} st_rom_layout_t;

st_status st_rom_layout(const st_rom_desc* d, st_rom_layout_t* out);

/* ========================================================================
 * st_build_bases - POD (Sec. 4.1, Eq. (snapshotmat), (POD), (SVD),
 * (temporalSVD)).
 *
 * U        [dev] snapshot matrix N_s x (n_mu N_t), column-major with leading
 *          dimension ldU >= N_s, columns parameter-major then time
 *          (U = [U_1 ... U_nmu], U_p = [u^(1) ... u^(N_t)] at mu_p).
 *          U_prec = ST_F64 (double) or ST_F32 (float storage).
 * gram_prec  arithmetic of the snapshot Gram: ST_F64 (FP64 MFMA), ST_F32
 *          (FP32 MFMA) or ST_BF16X3 (split-BF16 MFMA), as st_gram.
 *          The eigen-decomposition and re-orthonormalisation are FP64.
 * n_s      spatial modes, 1 <= n_s <= min(N_s, n_mu N_t).
 * n_t      [host] n_s temporal basis sizes, 1 <= n_t[i] <= N_t.
 * tau_t    relative threshold of the numerical rank of each temporal
 *          snapshot matrix (singular values <= tau_t * largest are dropped).
 *
 * The POD is computed by the method of snapshots, then refined to the SVD
 * of U itself: the smaller of U^T U and U U^T is formed, its leading
 * eigenpairs are found in FP64 by subspace iteration (n_s + min(32, extra)
 * vectors, 10 iterations, Rayleigh-Ritz), and - because the Gram squares
 * the condition number of U - two FP64 passes through U refine them: with
 * X0 the leading k = n_s + (up to 16) eigenvectors, C1 = op(U) X0 and
 * C2 = op(U)^T Y1 are each orthonormalised by a one-sided Jacobi SVD (Y1 the
 * normalised columns of the first), which yields Phi_s, sigma and the right
 * singular vectors.  The singular vectors then carry the accuracy of an SVD
 * of U (error ~ eps sigma_1 / gap) rather than of its Gram (~ eps sigma_1^2
 * / gap^2), down to modes at round-off.  Each temporal snapshot matrix Y_i
 * (N_t x n_mu, Y_i[k,p] = v_i(p N_t + k)) is decomposed by one-sided Jacobi.
 * If U has exact rank r < n_s the trailing columns are zero (sigma = 0).
 * The Jacobi runs in one launch when its matrix fits in LDS (rows x k x 8
 * bytes <= 144 KB); otherwise it takes one launch per round and the host reads
 * each sweep's rotation count, so st_build_bases then synchronises the stream
 * once per sweep (it is an offline call and is not graph-captured).  Temporal bases keep the left singular
 * vectors above tau_t and are completed, when n_t[i] exceeds that rank,
 * with DCT-II vectors cos(pi m (k+1/2)/N_t), m = 0,1,..., each orthogonalised
 * twice against the kept vectors and accepted if >= 1e-2 of its norm
 * survives.  Signs: each vector is made positive at its first entry whose
 * magnitude is >= 1/4 of its largest magnitude.
 *
 * Outputs [dev]: Phi_s N_s x n_s (ld N_s); Phi_t N_t x n (ld N_t),
 * mode-major columns; sigma n_s singular values; rank_t n_s numerical ranks
 * of the temporal snapshot matrices (may be NULL); diag ST_POD_DIAG doubles
 * (may be NULL):
 *   diag[0]  max_{i<n_s} ||G y_i - lambda_i y_i|| / lambda_1 of the Ritz pairs
 *            of the subspace iteration (its convergence; the refinement
 *            does not depend on it being small)
 *   diag[1]  sweeps of the refinement's one-sided Jacobi that rotated (the
 *            larger of its two runs; 30 means the sweep limit was reached);
 *            a run over columns longer than 144 KB counts its blocked passes
 *            (Gram of the columns, its two-sided Jacobi, one product) as sweeps
 *   diag[2]  largest |cos| between two columns seen in the last sweep of
 *            either run (<= 1e-14 max(1, sqrt(rows / 65536)) once converged)
 *   diag[3]  number of columns k of the refinement
 *   diag[4]  pair-by-pair sweeps that followed a blocked pass which did not
 *            halve the largest |cos| (nearly dependent columns; the larger
 *            of the two runs, 0 when the blocked passes converged alone)
 *
 * Limits (ST_EUNSUPPORTED beyond them): n_mu <= 64; N_t n_mu <= 15360
 * (a temporal snapshot matrix is staged in 120 KB of LDS); n_t[i] <= 512;
 * n_s <= 224 (n_s plus the 32 guard vectors of the subspace iteration
 * <= 256); min(N_s, n_mu N_t) < 2^31.
 * ====================================================================== */
#define ST_POD_DIAG 5
size_t st_build_bases_workspace(int64_t N_s, int32_t N_t, int32_t n_mu, int32_t n_s, const int32_t* n_t,
                                int32_t gram_prec);

st_status st_build_bases(const void* U, int32_t U_prec, int64_t ldU, int64_t N_s, int32_t N_t, int32_t n_mu,
                         int32_t n_s, const int32_t* n_t, int32_t gram_prec, double tau_t,
                         double* Phi_s, double* Phi_t, double* sigma, int32_t* rank_t, double* diag,
                         void* ws, size_t ws_bytes, void* stream);

/* ========================================================================
 * st_gram - the snapshot Gram of the method of snapshots (Sec. 4.1, the SVD
 * of Eq. (SVD) through the eigenpairs of U^T U), the first step of
 * st_build_bases, on its own so that its precision can be examined.
 *
 * X        [dev] K x p, column-major with leading dimension ld >= K;
 *          X_prec ST_F64 (double) or ST_F32 (float storage).
 * gram_prec ST_F64 (FP64 MFMA), ST_F32 (FP32 MFMA) or ST_BF16X3 (x = hi + lo
 *          in BF16, hi*hi + hi*lo + lo*hi on BF16 MFMA); both reduced
 *          precisions accumulate in FP32 over 1024-term stretches of K and
 *          sum the stretches in FP64.
 * G        [dev] p x p output, column-major (ld p), full symmetric matrix.
 * Workspace st_gram_workspace(K, p) bytes (split-K partial sums).
 * Limits: 1 <= p <= 65535, K >= 1.
 * ====================================================================== */
size_t st_gram_workspace(int64_t K, int32_t p);
st_status st_gram(const void* X, int32_t X_prec, int64_t ld, int64_t K, int32_t p, int32_t gram_prec, double* G,
                  void* ws, size_t ws_bytes, void* stream);

/* ========================================================================
 * st_assemble - offline reduced operators.
 *
 * Projection (Sec. 3.1, Eq. (galerkin); Sec. 4.3 notes that Ahat is the
 * spatial-ROM operator and can be precomputed): for each affine term,
 * Ahat_q = Phi_s^T (A_q Phi_s) by CSR SpMM against the tall-skinny basis;
 * bhat_q = Phi_s^T Bf_q; u0hat_q = Phi_s^T u0_q (reference state zero).
 * Phi_s^T (I - dt A) Phi_s = I - dt Ahat follows from Phi_s^T Phi_s = I.
 *
 * Temporal contractions (Sec. 4.3, Eq. (ij-block-matrix), (j-block-vector)):
 * T, K, Wf and P1 of the layout above, from the temporal bases and steps
 * (which are also copied into the buffer: Phit and dt).
 *
 * d        [host] model shape; d->n_t must match the bases.
 * Phi_s    [dev] N_s x n_s (ld N_s); Phi_t [dev] N_t x n (ld N_t).
 * dt       [dev] N_t step sizes.
 * A        [host] array of d->Q CSR descriptors (device arrays), N_s rows.
 * Bf       [dev] N_s x Qf (ld N_s) input vectors, or NULL when Qf = 0.
 * g        [dev] N_t x Qf (ld N_t) input time profiles, or NULL (all ones).
 * u0       [dev] N_s x Q0 (ld N_s) initial-state terms, or NULL when Q0 = 0.
 * proj_prec  arithmetic of the projection Ahat_q = Phi_s^T (A_q Phi_s):
 *          ST_F64: FP64 CSR SpMM and FP64 tall-skinny product;
 *          ST_F32: FP32 SpMM (values and basis rounded to FP32, FP32
 *          accumulation), then Phi_s^T (A_q Phi_s) on the matrix cores in FP32
 *          (as a block of the Gram of [Phi_s, A_q Phi_s]), FP32 accumulation;
 *          ST_BF16X3: the same with split-BF16 products (hi*hi + hi*lo + lo*hi).
 *          bhat, u0hat and every temporal contraction are FP64 in all cases.
 * rom      [dev] output buffer of st_rom_layout(d).total bytes.
 * ====================================================================== */
size_t st_assemble_workspace(const st_rom_desc* d, int64_t N_s);

st_status st_assemble(const st_rom_desc* d, int64_t N_s, const double* Phi_s, const double* Phi_t,
                      const double* dt, const st_csr* A, const double* Bf, const double* g, const double* u0,
                      int32_t proj_prec, void* rom, size_t rom_bytes, void* ws, size_t ws_bytes, void* stream);

/* ========================================================================
 * Per-query inputs shared by st_form and st_solve.
 *
 * n_q      number of queries (>= 0; 0 is a no-op).
 * theta_A  [dev] n_q x Q, query-major (row q holds theta_A(mu_q)).
 * theta_f  [dev] n_q x Qf, or NULL when Qf = 0.
 * theta_0  [dev] n_q x Q0, or NULL when Q0 = 0.
 * nt_q     [dev] n_q x n_s, query-major: query q uses the first nt_q[q,i]
 *          temporal vectors of mode i (0 <= nt_q[q,i] <= n_t[i]); NULL means
 *          every query uses the full bases.  A query's reduced system is the
 *          principal submatrix of the full one on its index set.
 * Query q's width is w_q = sum_i nt_q[q,i]; coeff_off[q] = sum_{p<q} w_p.
 * ====================================================================== */

/* ========================================================================
 * st_form - reduced space-time systems for a batch of queries
 * (Sec. 4.3, Eq. (block-reduced-state-mat), (ij-block-matrix),
 * (j-block-vector), and the projection of u0_st).
 *
 * Entry (a, b) of query q's matrix, a = (i', j'), b = (i, j):
 *   delta_{i'i} K_i[j', j] - Ahat(mu_q)[i', i] T[a, b],
 *   Ahat(mu_q) = sum_q theta_A[q] Ahat_q.
 * Right-hand side entry a = (i, j):
 *   sum_q theta_f[q] Wf[q,a] bhat_q[i] + P1[a] (sum_q theta_0[q] u0hat_q[i]).
 * (The printed Eq. (first-block-initial-vector) keeps only the first temporal
 * block; the projection of u0_st gives P1[a] u0hat_i for every a.)
 *
 * out_prec ST_F64 or ST_F32 element type of `mats`.
 * mats     [dev] capacity mats_cap elements; query q's w_q x w_q matrix is
 *          stored ROW-major at element offset mat_off[q] = sum_{p<q} w_p^2.
 * rhs      [dev] coeff_cap doubles, query q at coeff_off[q].
 * coeff_off, mat_off  [dev] n_q + 1 int64 outputs.
 * info     [dev] n_q int32 outputs (codes above).
 * ====================================================================== */
size_t st_form_workspace(const st_rom_desc* d, int32_t n_q);

st_status st_form(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                  const double* theta_f, const double* theta_0, const int32_t* nt_q, int32_t out_prec,
                  void* mats, int64_t mats_cap, double* rhs, int64_t coeff_cap, int64_t* coeff_off,
                  int64_t* mat_off, int32_t* info, void* ws, size_t ws_bytes, void* stream);

/* ========================================================================
 * st_solve - reduced space-time solve for a ragged batch (Sec. 3.2,
 * Eq. (st-galerkin); the paper does not name the dense solver: LU with
 * partial pivoting, as LAPACK gesv).
 *
 * Forms each query's system (as st_form), factors it by a blocked
 * right-looking LU with partial pivoting in lu_prec (ST_F64 or ST_F32), and
 * solves.  With lu_prec = ST_F32 the FP32 factors drive iterative
 * refinement: r = b - Ahat_st x is evaluated in FP64 from the ROM pieces
 * (never from the FP32 matrix), d = LU^{-1} r, x += d, until
 * ||r||_2 <= ir_tol ||b||_2 or ir_max refinement steps were taken.  With
 * ST_F64, ir_max extra refinement steps (usually 0) are taken the same way.
 * The final relative residual ||b - Ahat_st x|| / ||b|| (FP64) is written
 * to relres in both cases.  With ST_F32 and ir_tol > 0, every query still
 * above ir_tol after ir_max steps is re-formed in FP64 inside the matrix
 * workspace (its FP32 factors are no longer needed), factored by the FP64 LU
 * and solved (info = -6); queries whose FP64 system does not fit after the
 * earlier ones (in query order) keep info = -1.
 *
 * skip     [dev] n_q int32 or NULL: a query with skip[q] != 0 is not solved
 *          (info = -2); it keeps its place in coeff (whatever the caller put
 *          there, e.g. certified surrogate coefficients) and its relres entry,
 *          and takes no matrix workspace.
 * coeff    [dev] coeff_cap doubles: query q's solution at coeff_off[q].
 * coeff_off [dev] n_q + 1 int64 outputs.
 * relres   [dev] n_q doubles; info [dev] n_q int32; iters [dev] n_q int32
 *          refinement steps taken (may be NULL).
 * ws       [dev] st_solve_workspace(d, n_q, sum_w, sum_w2, lu_prec) bytes,
 *          where sum_w = sum_q w_q and sum_w2 = sum_q w_q^2 (upper bounds
 *          are fine: n_q * n and n_q * n^2).  A query that does not fit gets
 *          info = -3.
 * ====================================================================== */
size_t st_solve_workspace(const st_rom_desc* d, int32_t n_q, int64_t sum_w, int64_t sum_w2, int32_t lu_prec);

st_status st_solve(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                   const double* theta_f, const double* theta_0, const int32_t* nt_q, const int32_t* skip,
                   int32_t lu_prec, double ir_tol, int32_t ir_max, double* coeff, int64_t coeff_cap,
                   int64_t* coeff_off, double* relres, int32_t* info, int32_t* iters, void* ws, size_t ws_bytes,
                   void* stream);

/* ========================================================================
 * st_solve_noalloc - st_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels, outputs and info codes as st_solve,
 * without ws/ws_bytes: the workspace is a static device array of
 * ST_NOALLOC_SCRATCH_BYTES inside the library (one per GPU, held until the
 * process ends).  The caller still passes inputs and outputs.  The batch must
 * fit with every query at full width n: st_solve_workspace(d, n_q, coeff_cap,
 * n_q * n * n, lu_prec) <= ST_NOALLOC_SCRATCH_BYTES, else ST_EWORKSPACE is
 * returned before any launch.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine).  All calls on one GPU share that
 * GPU's array: calls that overlap in time on one GPU (different streams or
 * threads) race on it and must be serialised by the caller.
 * ====================================================================== */
#define ST_NOALLOC_SCRATCH_BYTES (64u << 20)
st_status st_solve_noalloc(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                           const double* theta_f, const double* theta_0, const int32_t* nt_q, const int32_t* skip,
                           int32_t lu_prec, double ir_tol, int32_t ir_max, double* coeff, int64_t coeff_cap,
                           int64_t* coeff_off, double* relres, int32_t* info, int32_t* iters, void* stream);

/* ========================================================================
 * Surrogate network (not part of the paper).  A multilayer perceptron maps a
 * (scaled) parameter vector to standardized reduced space-time coefficients:
 * x (d_in) -> [Linear + GELU] x n_hidden -> Linear -> y (d_out), GELU in its
 * erf form.  Products run on the matrix cores in BF16 with FP32 accumulation;
 * parameters, gradients and Adam moments are FP32.  Samples are rows of
 * row-major [dev] arrays.  Parameters are one flat array: for each layer l,
 * W_l (out_l x in_l, row-major) then b_l (out_l).
 * ====================================================================== */
typedef struct {
  int32_t d_in, width, n_hidden, d_out;
} st_mlp_shape;

int64_t st_mlp_param_count(const st_mlp_shape* s);
size_t st_mlp_workspace(const st_mlp_shape* s, int32_t batch);

/* Y (batch x d_out) = network(X (batch x d_in)). */
st_status st_mlp_forward(const st_mlp_shape* s, const float* params, int32_t batch, const float* X, float* Y,
                         void* ws, size_t ws_bytes, void* stream);

/* Mean squared error of network(X) against T (batch x d_out), averaged over all
 * outputs, written to *loss [dev]; its gradient with respect to every
 * parameter written to grads [dev] (same layout as params). */
st_status st_mlp_grad(const st_mlp_shape* s, const float* params, int32_t batch, const float* X, const float* T,
                      float* grads, float* loss, void* ws, size_t ws_bytes, void* stream);

/* One Adam step (bias-corrected, step number `step` >= 1) on n parameters. */
st_status st_mlp_adam(int64_t n, float* params, const float* grads, float* m, float* v, int32_t step, float lr,
                      float beta1, float beta2, float eps, void* stream);

/* Output standardisation of the training targets: C [dev] n x d row-major
 * FP64 coefficients (one training solve per row).  st_mlp_colstats writes
 * mean [dev, d] and scale [dev, d], the per-column mean and population
 * standard deviation (1 where it is zero); st_mlp_standardize writes
 * T [dev] n x d FP32 = (C - mean) / scale, the network's training targets
 * (the certificate maps outputs y back to c = mean + scale * y). */
st_status st_mlp_colstats(int32_t n, int32_t d, const double* C, double* mean, double* scale, void* stream);
st_status st_mlp_standardize(int32_t n, int32_t d, const double* C, const double* mean, const double* scale, float* T,
                             void* stream);

/* Residual certificate of surrogate coefficients for full-width queries:
 * c = mean + scale * y (FP64; y = row q of Y, n outputs), r = b(mu) -
 * Ahat_st(mu) c in FP64 from the ROM pieces (Sec. 5.2, Eq. (stresidual) in
 * reduced form), cert = e / (1 - e) with e = ||r||_2 / (gamma ||c||_2) (inf if
 * e >= 1).  When gamma lower-bounds lambda_min(sym Ahat_st(mu)) - e.g.
 * 1 - cos(pi / (N_t + 1)) whenever sym(A(mu)) <= 0 - cert bounds the relative
 * error of c against the exact reduced solution.  accept[q] = cert <= tol.
 * coeff [dev] n_q * n doubles, packed as st_solve packs the same full-width
 * queries (query q at q * n when every query is valid; a query with a
 * non-finite parameter coefficient takes no space and is never accepted),
 * cert [dev] n_q, accept [dev] n_q. */
size_t st_surrogate_check_workspace(const st_rom_desc* d, int32_t n_q);
st_status st_surrogate_check(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                             const double* theta_f, const double* theta_0, const float* Y, const double* mean,
                             const double* scale, double gamma, double tol, double* coeff, double* cert,
                             int32_t* accept, void* ws, size_t ws_bytes, void* stream);

/* ========================================================================
 * Residual certificate of reduced coefficients (any source: st_solve, the
 * surrogate, a caller's iterate), for ragged batches.
 *
 * st_coercivity_floor(N_t) = 1 - cos(pi / (N_t + 1)): a lower bound of
 * lambda_min(sym Ahat_st(mu)) whenever sym(A(mu)) <= 0.  The backward-Euler
 * space-time matrix (Sec. 2, Eq. (stsystemmat)) then has a symmetric part that
 * dominates the tridiagonal Toeplitz matrix (1 on the diagonal, -1/2 beside
 * it) Kronecker I, whose smallest eigenvalue this is, and the Galerkin
 * projection with orthonormal Phi_st (Sec. 3.2) keeps the bound.
 *
 * st_certify: for each query, r = b(mu) - Ahat_st(mu) c in FP64 from the ROM
 * pieces (the reduced form of the space-time residual, Sec. 5.2, Eq.
 * (stresidual)); relres[q] = ||r|| / ||b||; cert[q] = e / (1 - e) with
 * e = ||r|| / (gamma ||c||) (+inf if e >= 1 or c = 0), which bounds
 * ||c - c*|| / ||c*|| against the exact reduced solution c* when gamma <=
 * lambda_min(sym Ahat_st(mu)).  gamma = 0 selects st_coercivity_floor(N_t).
 * coeff [dev] packed as st_solve packs the same queries (nt_q as there).
 * relres, cert [dev] n_q doubles (NaN / +inf for invalid queries).
 * ====================================================================== */
double st_coercivity_floor(int32_t N_t);
size_t st_certify_workspace(const st_rom_desc* d, int32_t n_q, int64_t coeff_cap);
st_status st_certify(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                     const double* theta_f, const double* theta_0, const int32_t* nt_q, const double* coeff,
                     int64_t coeff_cap, double gamma, double* relres, double* cert, void* ws, size_t ws_bytes,
                     void* stream);

/* ========================================================================
 * st_fom_bound - certified full-order error bound of space-time ROM solutions
 * (Sec. 5.2, Theorem (res-basedErrorBoundforSpaceTime)):
 *   ||u_st - u~_st||_inf <= sqrt(N_t) ||A_st^{-1}||_2 ||r_st(u~_st)||_inf,
 * u~_st = Phi_st c the reconstructed space-time state of each query,
 * r_st = A_st u~_st - f_st - u0_st its full-order space-time residual
 * (Eq. (stresidual)), ||.||_inf = max over time steps of the 2-norm
 * (Eq. (spacetimeinfnorm)).  The residual is evaluated exactly in FP64 on
 * the full N_s x N_t grid (never stored): r^(k) = Phi_s (y_k - y_{k-1})
 * - dt_k A(mu) Phi_s y_k - dt_k B f^(k)(mu) (- u0(mu) at the first step),
 * y_k = the query's temporal coefficients at step k.
 *
 * Inputs as st_assemble (N_s, Phi_s, the CSR terms A, Bf, g, u0) plus the
 * ROM buffer (temporal bases, steps) and the packed coefficients of n_q
 * queries (nt_q, coeff, coeff_cap as st_solve).
 * inv_norm  an upper bound of ||A_st(mu)^{-1}||_2 for every query, or 0 for
 *           1 / st_coercivity_floor(N_t), valid whenever sym(A(mu)) <= 0.
 * Outputs [dev] n_q doubles each: res_inf = ||r_st||_inf, u_inf =
 * ||u~_st||_inf, bound = sqrt(N_t) inv_norm res_inf (NaN for invalid queries).
 * Limits: n_s <= 128 and (33 n_s + 32 (n_s (Q+1) + Qf + Q0)) 8 bytes <= 160 KB;
 * backward Euler only (ST_EUNSUPPORTED for a Crank-Nicolson model).
 * ====================================================================== */
size_t st_fom_bound_workspace(const st_rom_desc* d, int64_t N_s, int32_t n_q);
st_status st_fom_bound(const st_rom_desc* d, const void* rom, int64_t N_s, const double* Phi_s, const st_csr* A,
                       const double* Bf, const double* g, const double* u0, int32_t n_q, const double* theta_A,
                       const double* theta_f, const double* theta_0, const int32_t* nt_q, const double* coeff,
                       int64_t coeff_cap, double inv_norm, double* res_inf, double* u_inf, double* bound, void* ws,
                       size_t ws_bytes, void* stream);

/* ========================================================================
 * Spatial Galerkin ROM (Sec. 3.1): the paper's point of comparison for the
 * space-time ROM.
 *
 * st_spatial_march: for each query, the backward-Euler march of Eq.
 * (space_reduced_discretized_ODE) with u_ref = 0,
 *   (I - dt_k Ahat(mu)) uhat^(k) = uhat^(k-1) + dt_k sum_q theta_f[q] g[k,q] bhat_q,
 *   uhat^(0) = sum_q theta_0[q] u0hat_q,
 * from the ROM buffer's Ahat_q, bhat_q, u0hat_q and steps, and the reduced
 * outputs of Eq. (outputFromReducedsol), y^(k) = Chat^T uhat^(k).
 * g        [dev] N_t x Qf input time profiles (ld N_t) or NULL (all ones).
 * Chat     [dev] n_s x n_out (ld n_s) reduced output matrix Phi_s^T C (see
 *          st_project), or NULL when outputs is NULL.
 * traj     [dev] n_q x N_t x n_s (query, step, mode; uhat^(1..N_t)) or NULL.
 * outputs  [dev] n_q x N_t x n_out or NULL.
 * info     [dev] n_q: 0, -5 (non-finite parameter coefficient), or k > 0 when
 *          I - dt_k Ahat(mu) is singular (its entries are then NaN).
 * Each query factors I - dt Ahat(mu) once per distinct step size (an explicit
 * inverse by Gauss-Jordan elimination with partial pivoting, FP64), then
 * marches.  n_s <= 128 and (n_s^2 + (3 + Qf) n_s) 8 bytes <= 160 KB; backward
 * Euler only (ST_EUNSUPPORTED for a Crank-Nicolson model).
 *
 * st_project: out (n_s x k, ld n_s) = Phi_s^T X, X N_s x k (ld N_s), FP64,
 * e.g. Chat = Phi_s^T C (Eq. (galerkin)).
 * ====================================================================== */
st_status st_spatial_march(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                           const double* theta_f, const double* theta_0, const double* g, int32_t n_out,
                           const double* Chat, double* traj, double* outputs, int32_t* info, void* stream);
size_t st_project_workspace(int64_t N_s, int32_t n_s, int32_t k);
st_status st_project(int64_t N_s, int32_t n_s, const double* Phi_s, int32_t k, const double* X, double* out, void* ws,
                     size_t ws_bytes, void* stream);

/* ========================================================================
 * st_isvd_* - incremental SVD of a snapshot stream (Sec. 4.2, Alg. 1 and 2,
 * Eq. (factorization2), (middleMat), (svdMiddleMat), (rankOneUpdateSVD2)).
 *
 * Snapshots are taken one at a time, as a full-order solver produces them,
 * and U_k = W diag(s) V^T is updated without keeping U.  For a snapshot u:
 * l = W^T u and p = ||u - W l|| (two Gram-Schmidt passes); the middle matrix
 * [[diag(s), l], [0, p]] is decomposed (secular equation with deflation and
 * Loewner-recomputed vectors) and W <- [W, (u - W l)/p] Uq,
 * V <- [[V, 0], [0, 1]] Vq, s <- the new singular values.  Decisions, in the
 * paper's order:
 *   - empty basis (Alg. 1): u starts it if ||u|| > eps_svd, else u is
 *     skipped (V still gains a zero row, so row c of V belongs to snapshot c);
 *   - p < eps_svd (or p at the rounding level of the middle matrix, 8 eps
 *     times its norm): u is dependent, the rank stays, only the leading r
 *     triplets are kept;
 *   - the smallest new singular value < eps_sv: its triplet is dropped;
 *   - the rank never exceeds r_max: the trailing triplet is dropped (the
 *     basis is kept, not restarted);
 *   - |W(:,1)^T W(:,end)| > min(eps_svd, eps N_s) (eps the machine epsilon):
 *     W is replaced by the Q factor of its QR factorisation with a positive
 *     diagonal of R (classical Gram-Schmidt with re-orthogonalisation in one
 *     workgroup), R is dropped.
 *
 * Buffers [dev], owned by the caller and passed unchanged to every call of
 * one stream: W N_s x r_max (ld N_s), s r_max, V m_max x r_max (ld m_max),
 * state ST_ISVD_STATE int32 words (clear it with st_isvd_reset before the
 * first snapshot), workspace of st_isvd_workspace(N_s, r_max) bytes.
 * Columns 0..r-1 of W and V and s[0..r-1] hold the factors, r = state[0];
 * the rest is stale.  Public state words:
 *   state[0] r, the current rank         state[1] k, snapshots taken
 *   state[2] re-orthonormalisations      state[3] dependent snapshots
 *   state[4] truncated triplets          state[5] snapshots skipped by Alg. 1
 *   state[6] snapshots refused because k had reached m_max (no update made)
 * Words 7..15 are internal.
 *
 * st_isvd_update streams the b columns of U (N_s x b, ld ldU >= N_s) in
 * order: four kernel launches each for N_s <= 4096, nine beyond, with no host
 * synchronisation and no allocation.
 * Limits: 1 <= r_max <= ST_ISVD_MAX_RANK, N_s >= 1, m_max >= 1.  Calls on one
 * state must not overlap (use one stream).
 *
 * st_isvd_bases: Eq. (spatialincrementalbasis), (incrementaltemporalsnapshotmat),
 * (temporalincrementalbasis): once the stream holds all n_mu N_t snapshots
 * (parameter-major, then time, as st_build_bases's U), Phi_s = W(:, 1:n_s),
 * sigma = s(1:n_s), and the temporal bases of the columns of V with the
 * same completion, threshold and sign rules as st_build_bases (columns
 * beyond the rank are zero).  Synchronises the stream to read the state;
 * ST_EINVAL when state[1] != n_mu N_t.  Same limits as st_build_bases's
 * temporal part (n_mu <= 64, N_t n_mu 8 bytes <= 120 KB, n_t[i] <= 512).
 * ====================================================================== */
#define ST_ISVD_STATE 16
#define ST_ISVD_MAX_RANK 256
size_t st_isvd_workspace(int64_t N_s, int32_t r_max);
st_status st_isvd_reset(int32_t* state, void* stream);
st_status st_isvd_update(const double* U, int64_t ldU, int64_t N_s, int32_t b, int32_t r_max, int64_t m_max,
                         double eps_svd, double eps_sv, double* W, double* s, double* V, int32_t* state, void* ws,
                         size_t ws_bytes, void* stream);
size_t st_isvd_bases_workspace(int32_t N_t, int32_t n_mu, int32_t n_s);
st_status st_isvd_bases(const double* W, const double* s, const double* V, const int32_t* state, int64_t N_s,
                        int64_t m_max, int32_t N_t, int32_t n_mu, int32_t n_s, const int32_t* n_t, double tau_t,
                        double* Phi_s, double* Phi_t, double* sigma, int32_t* rank_t, void* ws, size_t ws_bytes,
                        void* stream);

/* ========================================================================
 * Phase timing (measurement tools).  After st_timing_enable(1), every st_solve
 * records HIP events on its stream at its phase boundaries; after the caller
 * has synchronised that stream, st_timing_read fills ms[p] with the elapsed
 * milliseconds of phase p of the most recent st_solve and returns the number
 * of phases (or a negative status).  Phases: 0 plan, 1 form (assembly of
 * every query's system), 2 right-hand-side norms, 3 batched LU, 4 first
 * triangular solves, 5 all refinement steps, 6 final residual and checks.
 * Not thread-safe; timing one solve at a time is the intended use.
 * ====================================================================== */
#define ST_TIMING_PHASES 7
st_status st_timing_enable(int32_t on);
int32_t st_timing_read(double* ms, int32_t cap);

/* ========================================================================
 * st_reconstruct - space-time state of each query (Sec. 3.2, the space-time
 * state approximation): out_q[x, k] = sum_i Phi_s[x, i] sum_j Phi_t[k, (i, j)] c_q[(i, j)]
 * over query q's per-mode prefixes (nt_q as in st_solve; NULL = full bases).
 *
 * rom       [dev] ROM buffer of d (its mode offsets are used).
 * Phi_s     [dev] N_s x n_s column-major, leading dimension ldp >= N_s.
 * Phi_t     [dev] N_t x n column-major, leading dimension ldt >= N_t.
 * coeff, coeff_off [dev] packed coefficients as written by st_solve.
 * out       [dev] n_q blocks of ldo x N_t (column-major, ldo >= N_s); block q
 *           starts at out + q * ldo * N_t.  Validation only (the full-order
 *           state is large): not part of the online solve.
 * ====================================================================== */
st_status st_reconstruct(const st_rom_desc* d, const void* rom, int64_t N_s, const double* Phi_s, int64_t ldp,
                         const double* Phi_t, int64_t ldt, int32_t n_q, const int32_t* nt_q, const double* coeff,
                         const int64_t* coeff_off, double* out, int64_t ldo, void* stream);

/* ========================================================================
 * HIP graph replay of st_solve.  After st_graph_enable(1), the first st_solve
 * call with a given set of arguments runs eagerly and records its whole launch
 * sequence as a HIP graph; later calls with the same arguments (the
 * description by value; every pointer, size, precision and tolerance; and the
 * LU variant in use) replay it with one hipGraphLaunch on the caller's stream.
 * The data behind the pointers may change between calls; the buffers must stay
 * allocated while a graph using them is cached (st_graph_reset destroys every
 * cached graph).  Graphs are bypassed while phase timing is on.  The cache is
 * guarded by a mutex; st_graph_count returns its size.
 * ====================================================================== */
st_status st_graph_enable(int32_t on);
st_status st_graph_reset(void);
int32_t st_graph_count(void);

/* ========================================================================
 * LU autotuner.  st_autotune times every batched-LU configuration (register
 * sub-panel widths; for n <= 1536 also a 256-thread configuration that runs two
 * queries per compute unit) on the given batch, forming the systems afresh before each,
 * records the fastest for the batch's LU precision and width class (total
 * reduced width n <= 1536, or n <= 4096) and st_solve uses it from then on.
 * Arguments as st_solve, with the same workspace size; coeff_off and info
 * receive the plan, while coeff and the workspace are used as scratch (no
 * solution is produced).  choice [host, may be NULL] receives the chosen
 * variant, ms [host, may be NULL, >= ST_LU_VARIANTS entries] each candidate's
 * time.  Synchronises the stream.
 * st_autotune_choice returns the recorded variant for (lu_prec, n), -1 if
 * none (variant 0 is then used); st_autotune_set records one directly.
 * ====================================================================== */
#define ST_LU_VARIANTS 3
st_status st_autotune(const st_rom_desc* d, const void* rom, int32_t n_q, const double* theta_A,
                      const double* theta_f, const double* theta_0, const int32_t* nt_q, int32_t lu_prec,
                      double* coeff, int64_t coeff_cap, int64_t* coeff_off, double* relres, int32_t* info, void* ws,
                      size_t ws_bytes, void* stream, int32_t* choice, double* ms);
int32_t st_autotune_choice(int32_t lu_prec, int32_t n);
st_status st_autotune_set(int32_t lu_prec, int32_t n, int32_t variant);

#ifdef __cplusplus
}
#endif

#endif /* STROM_H */
