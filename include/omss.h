/*
 * omss.h -- C ABI of the optomechanical steady-state solver library
 * (libomss.so): the Lindblad Liouvillian of a driven optomechanical system,
 * its trace-constrained steady-state system, reverse Cuthill-McKee
 * reordering, a dual-threshold incomplete-LU preconditioner and restarted
 * GMRES, after Nation, Johansson, Blencowe and Rimberg, "Iterative solutions
 * to the steady state density matrix for optomechanical systems".
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Every call returns om_status; none throws or aborts across the ABI.  On a
 *    status other than OM_OK, om_last_error() (thread-local) holds a message.
 *  - Complex vectors are interleaved (re, im): complex128 = two doubles,
 *    complex64 = two floats.  Batched vectors are stored batch-major: item b
 *    of a batch occupies elements [b*n, (b+1)*n).
 *  - "device" pointers are HIP device memory owned by the caller (e.g. a
 *    contiguous torch tensor); the library never frees or reallocates them.
 *    "host" pointers are ordinary host memory owned by the caller.
 *  - Handles (om_csr, om_ilu) are created by the library and released with
 *    om_csr_free / om_ilu_free.
 *  - `stream` is a hipStream_t passed as void* (0 = the null stream).  Device
 *    work is ordered on it.  Calls that take convergence decisions
 *    (gmres_solve, steady_state) or move data to the host (rcm_permute,
 *    ilu_factor) synchronise the stream before returning.
 *  - Sizes: n = (nc*nm)^2 rows; row pointers of the system matrix are 32-bit
 *    (nnz < 2^31), factor storage is 64-bit indexed.
 */
#ifndef OMSS_H
#define OMSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OM_OK = 0,
    OM_EINVAL = 1,      /* invalid argument (NaN, negative rate, bad size, ...) */
    OM_ENOMEM = 2,      /* device or host allocation failed / would not fit */
    OM_EHIP = 3,        /* a HIP runtime call failed */
    OM_ENOTCONV = 4,    /* iteration limit reached; x holds the last iterate */
    OM_EBREAKDOWN = 5,  /* NaN/Inf produced, or an unrecoverable pivot */
    OM_ETIMEOUT = 6     /* a bounded device-side wait expired (no hang) */
} om_status;

typedef enum { OM_C128 = 0, OM_C64 = 1 } om_dtype;

/* How the trace condition Tr rho = 1 enters the system (Eq. (5)). */
typedef enum {
    OM_TRACE_NONE = 0,          /* plain L (singular); rhs = 0 */
    OM_TRACE_REPLACE_ROW0 = 1,  /* row 0 := w t^T, rhs = w e_0 (default) */
    OM_TRACE_ADD_ROW0 = 2       /* row 0 := L_0 + w t^T, rhs = w e_0 (Eq. (5)) */
} om_trace;

/* Model parameters of Eq. (1) and Eq. (3), in units of omega_m, with the
 * Fock truncation: Hilbert index k = i*nm + j (Sec. III ordering). */
typedef struct {
    int32_t nc, nm;     /* cavity / mechanical Fock cutoffs, each >= 2 */
    double delta;       /* detuning Delta = omega_p - omega_c */
    double omega_m;     /* mechanical frequency */
    double g0;          /* radiation-pressure coupling */
    double E;           /* pump amplitude */
    double kappa;       /* cavity damping rate, >= 0 */
    double gamma_m;     /* mechanical damping rate Gamma_m, >= 0 */
    double n_th;        /* thermal occupation of the mechanical bath, >= 0 */
    double g2;          /* quadratic coupling g2 (b + b^dag)^2 a^dag a added to the
                           Hamiltonian of Eq. (1) (the "membrane in the middle"
                           variant of Sec. V); 0 for Eq. (1) itself */
} om_params;

typedef struct om_csr om_csr;   /* device CSR: one pattern, `batch` value sets */
typedef struct om_ilu om_ilu;   /* device ILU factors (+ solve schedules) per batch item */

/* Bandwidth/profile statistics (Sec. II definitions) before (0) and after (1)
 * reordering. */
typedef struct {
    int64_t ub0, lb0, B0, P0;
    int64_t ub1, lb1, B1, P1;
} om_order_stats;

typedef struct {
    double fill;             /* (nnz(L strict) + nnz(U incl. diag)) / nnz(A), max over batch */
    double condest;          /* ||(L U)^{-1} e||_inf (Sec. IV), max over batch; 0 if not requested */
    int64_t nnz_L, nnz_U;    /* summed over the batch */
    int64_t depth_L, depth_U;/* level-schedule depth (max over the batch) */
    int64_t repaired_pivots; /* summed over the batch */
    double t_factor_s;       /* wall time of the host factorisation */
} om_ilu_stats;

typedef enum { OM_PREC_FP64 = 0, OM_PREC_IR_C64 = 1 } om_precision;

typedef struct {
    int32_t m;          /* restart length (Arnoldi steps per cycle) */
    int32_t maxiter;    /* limit on total Arnoldi steps (per batch item) */
    int32_t precision;  /* om_precision */
    int32_t max_outer;  /* GMRES-IR: limit on refinement steps */
    double tol;         /* stop when ||b - A x||_2 / ||b||_2 <= tol (FP64, true residual) */
    double inner_tol;   /* GMRES-IR: relative tolerance of each inner c64 solve */
} om_gmres_opts;

typedef struct {
    int32_t iters;          /* Arnoldi steps (max over batch) */
    int32_t restarts;       /* completed cycles (max over batch) */
    int32_t outer_iters;    /* GMRES-IR refinement steps */
    int32_t converged;      /* number of batch items that met tol */
    double relres_true;     /* max over batch of the final FP64 true relative residual */
    double relres_est;      /* max over batch of the last Arnoldi residual estimate */
    double t_spmv_s, t_ilu_s, t_orth_s, t_total_s;
} om_gmres_info;

typedef struct {
    double drop_tol;        /* ILUT drop tolerance d */
    double fill_factor;     /* ILUT fill limit p (per-row cap); INFINITY = none */
    om_gmres_opts gmres;
    int32_t trace_mode;     /* om_trace */
    int32_t nth0_fix;       /* n_th == 0 is built as n_th = 1e-15 (Sec. IV) */
    int32_t reorder;        /* 1 = RCM (default), 0 = natural order */
    int32_t want_adjoint;   /* keep conjugate-transposed factors for adjoint solves */
    int32_t share_factor;   /* one ILU factor (of item 0) preconditions the whole batch */
} om_ss_opts;

typedef struct {
    om_order_stats order;
    om_ilu_stats ilu;
    om_gmres_info gmres;
    double t_build_s, t_rcm_s, t_factor_s, t_solve_s, t_post_s;
} om_ss_info;

/* Per-item results of steady_state, host arrays of length `batch` (nullable). */
typedef struct {
    double* trace_err;      /* |Tr rho - 1| before normalisation */
    double* herm_err;       /* ||rho - rho^H||_F / ||rho||_F */
    double* n_a;            /* <a^dag a> */
    double* n_b;            /* <b^dag b> */
    double* fano;           /* <(Delta N_b)^2> / <N_b> */
    double* relres;         /* final true relative residual */
} om_ss_results;

/* ---- library ------------------------------------------------------------ */

const char* om_last_error(void);
const char* om_version(void);

/* ---- liouvillian_build ---------------------------------------------------
 * Assemble on the device the sparse matrix of the Liouvillian of Eq. (3) in
 * the Fock basis with column-stacked vec(rho) (Eq. (4)), and impose the trace
 * condition of Eq. (5) with the weight w = mean of diag(L) (Sec. IV).
 * params: host array of `batch` >= 1 parameter sets with the same (nc, nm) and
 *   the same zero pattern (a parameter zero in one item is zero in all); the
 *   items share one sparsity pattern.  Entries that evaluate to exactly zero
 *   are not stored.
 * flags: OM_BUILD_C64 also keeps a complex64 copy of the values.
 * w_out: host array of `batch` doubles (nullable) receiving w.
 * Errors: OM_EINVAL for nc or nm < 2, non-finite values, negative rates, or a
 *   mismatched batch; OM_ENOMEM if the matrix would exceed 2^31 nonzeros or
 *   does not fit. */
#define OM_BUILD_C64 1u
om_status liouvillian_build(const om_params* params, int32_t batch, int32_t trace_mode,
                            uint32_t flags, om_csr** A_out, double* w_out, void* stream);

/* Query sizes of a CSR handle (any pointer may be null). */
om_status om_csr_info(const om_csr* A, int64_t* n, int64_t* nnz, int32_t* batch, int32_t* N);

/* Copy a CSR handle to host arrays: row_ptr[n+1], col[nnz], val[batch*nnz]
 * complex128 interleaved (any may be null). */
om_status om_csr_export(const om_csr* A, int64_t* row_ptr, int32_t* col, double* val, void* stream);

/* ---- rcm_permute ---------------------------------------------------------
 * Reverse Cuthill-McKee ordering of the structure of A + A^T (Sec. III):
 * breadth-first search from an unvisited node of lowest degree (degree = row
 * count of A + A^T including the diagonal; ties to the lower index), each
 * node's unvisited neighbours enqueued by ascending (degree, index), repeated
 * per connected component, order reversed.  Produces A_perm = P A P^T with
 * A_perm[i, j] = A[perm[i], perm[j]] on the device (same batch).
 * perm_host: host int32[n] (nullable) receiving perm[new] = old.
 * st: bandwidth/profile before and after (nullable). */
om_status rcm_permute(const om_csr* A, int32_t* perm_host, om_csr** A_perm_out,
                      om_order_stats* st, void* stream);

/* Apply a caller-given symmetric permutation perm[new] = old (host int32[n]). */
om_status csr_permute(const om_csr* A, const int32_t* perm_host, om_csr** A_perm_out, void* stream);

/* ---- ilu_factor ----------------------------------------------------------
 * Dual-threshold incomplete LU of every batch item of A (Sec. II): row-wise
 * elimination in increasing column order; a multiplier with
 * |l_ik| < drop_tol * ||a_i||_inf is dropped before use; after the row is
 * eliminated every off-diagonal entry below that threshold is dropped and at
 * most floor((fill_factor * nnz(a_i) - 1) / 2) entries (largest modulus, ties
 * to the lower column) are kept in each triangle; no pivoting; a pivot below
 * 1e-14 ||a_i||_inf is raised to that floor and counted.  drop_tol = 0 with
 * fill_factor = INFINITY gives the complete LU.  Runs on host threads (one
 * per batch item), then uploads the factors with their solve schedules.
 * flags: OM_ILU_C64 keeps complex64 copies for ilu_apply(OM_C64);
 *        OM_ILU_ADJOINT keeps the conjugate-transposed factors;
 *        OM_ILU_CONDEST fills st->condest;
 *        OM_ILU_KEEP_HOST keeps a host copy of the CSR factors for
 *        om_ilu_export (costs host memory of the size of the factors);
 *        OM_ILU_SHARED factors batch item 0 only (with all host threads) and
 *        uses that factor as the preconditioner of every batch item (items
 *        that differ only in parameter values share one structure).
 * Errors: OM_EINVAL (drop_tol < 0, fill_factor <= 0), OM_ENOMEM. */
#define OM_ILU_C64 1u
#define OM_ILU_ADJOINT 2u
#define OM_ILU_CONDEST 4u
#define OM_ILU_KEEP_HOST 8u
#define OM_ILU_SHARED 16u
om_status ilu_factor(const om_csr* A, double drop_tol, double fill_factor, uint32_t flags,
                     om_ilu** M_out, om_ilu_stats* st, void* stream);

/* Copy the factors of batch item b to host CSR arrays (any may be null):
 * L strictly lower (unit diagonal implied), U upper with the diagonal first in
 * each row; values complex128 interleaved.  Sizes from om_ilu_info.  Needs a
 * handle from om_host_ilut or from ilu_factor with OM_ILU_KEEP_HOST. */
om_status om_ilu_info(const om_ilu* M, int32_t b, int64_t* n, int64_t* nnz_L, int64_t* nnz_U);
om_status om_ilu_export(const om_ilu* M, int32_t b, int64_t* l_ptr, int32_t* l_col, double* l_val,
                        int64_t* u_ptr, int32_t* u_col, double* u_val);

/* ---- ilu_apply -----------------------------------------------------------
 * Preconditioner solve on the device for every batch item:
 *   adjoint = 0: y = (L U)^{-1} x   (forward then backward substitution)
 *   adjoint = 1: y = (L U)^{-H} x   (needs OM_ILU_ADJOINT)
 * x, y: device arrays of batch*n complex values of `dtype` (OM_C64 needs
 * OM_ILU_C64); x and y may alias. */
om_status ilu_apply(const om_ilu* M, int32_t adjoint, int32_t dtype, const void* x, void* y,
                    void* stream);

/* ---- csr_spmv -------------------------------------------------------------
 * y = A x (adjoint = 0) or y = A^H x (adjoint = 1) for every batch item, in
 * complex128 (OM_C128) or complex64 (OM_C64, needs OM_BUILD_C64).  x and y
 * are device arrays of batch*n complex values and must not alias. */
om_status csr_spmv(const om_csr* A, int32_t adjoint, int32_t dtype, const void* x, void* y,
                   void* stream);

/* ---- liouvillian_apply ----------------------------------------------------
 * y = A x for every batch item without reading A's stored entries: A must be
 * a matrix built by liouvillian_build (possibly permuted by rcm_permute), and
 * each row's entries are re-evaluated from its model parameters (Eq. (3) in
 * the Fock basis with column-stacked rho, Eq. (4), and the trace row of
 * Eq. (5) as A was built with).  The values are those liouvillian_build
 * stores, so y equals csr_spmv(A, 0, ...) up to the order of the additions;
 * only x, y and the permutation cross memory.  dtype OM_C128 or OM_C64
 * (values rounded to complex64 as OM_BUILD_C64 stores them; no complex64 copy
 * of A is needed).  x and y: device arrays of batch*n complex values, not
 * aliased.  Errors: OM_EINVAL if A carries no model description or for a bad
 * dtype or aliasing.  With OMSS_SPMV=stencil in the environment the solver's
 * own products with A (not A^H) use this path too. */
om_status liouvillian_apply(const om_csr* A, int32_t dtype, const void* x, void* y, void* stream);

/* ---- gmres_solve ----------------------------------------------------------
 * Restarted GMRES(m) with right preconditioning M (nullable = none) on every
 * batch item: solves A x = b (adjoint = 0) or A^H x = b (adjoint = 1) to the
 * FP64 true relative residual opts->tol.  Arnoldi uses classical Gram-Schmidt
 * with reorthogonalisation; the Hessenberg matrix, Givens rotations and
 * least-squares solve are FP64 on the device.  With precision OM_PREC_IR_C64
 * the residual and update stay FP64 while each correction is solved by a
 * complex64 GMRES (c64 SpMV, c64 factors, c64 basis, FP64 dot products).
 * b: device complex128[batch*n]; x: device complex128[batch*n], in: initial
 * guess, out: solution (on OM_ENOTCONV the last iterate).
 * info: host (nullable). */
om_status gmres_solve(const om_csr* A, const om_ilu* M, int32_t adjoint, const void* b, void* x,
                      const om_gmres_opts* opts, om_gmres_info* info, void* stream);

/* ---- steady_state --------------------------------------------------------
 * The whole method for `batch` parameter sets sharing one structure:
 * liouvillian_build -> rcm_permute -> ilu_factor -> gmres_solve -> un-permute,
 * rho = unvec(x), rho /= Tr rho, observables.
 * rho: device complex128[batch * N * N], column-major N x N per item,
 * N = nc*nm.  info, res: host (nullable). */
om_status steady_state(const om_params* params, int32_t batch, const om_ss_opts* opts, void* rho,
                       om_ss_info* info, om_ss_results* res, void* stream);

/* Default options for a given problem (gmres m = 50, tol = 1e-10, ...). */
void om_ss_opts_default(om_ss_opts* opts);

/* ---- observables and parameter derivatives (adjoint gradients) ------------
 * For a solution x of the constrained system (device complex128[batch*n], in
 * the ordering of A, Tr rho = 1):
 * om_observables: host double[batch*3] receives <a^dag a>, <b^dag b>, Fano F.
 * om_objective_vectors: device complex128[3*batch*n] receives conj(o_f) for
 *   f = (n_a, n_b, F) -- vector f of item b at (f*batch + b)*n -- the
 *   right-hand sides of the adjoint system A^H lambda = conj(o_f) (for F:
 *   o_2/m_1 - (2 + F/m_1) o_1, with m_1 = <b^dag b>).
 * om_param_gradient: grad[(b*nrhs + f)*5 + t] = -Re lambda_f^H P0 (dL/dtheta_t) x
 *   for theta = (Delta, g0, E, kappa, Gamma_m); lambda: device
 *   complex128[nrhs*batch*n] laid out like the objective vectors (1 <= nrhs
 *   <= 3); P0 zeroes row 0 (the trace row).  A must carry model parameters
 *   (built by liouvillian_build, possibly permuted). */
om_status om_observables(const om_csr* A, const void* x, double* obs_host, void* stream);
om_status om_objective_vectors(const om_csr* A, const void* x, void* g, void* stream);
om_status om_param_gradient(const om_csr* A, const void* x, const void* lambda, int32_t nrhs,
                            double* grad_host, void* stream);

void om_csr_free(om_csr* A);
void om_ilu_free(om_ilu* M);

/* ---- kernel timing (diagnostics) -----------------------------------------
 * When enabled, every launch of an instrumented kernel class records a pair of
 * HIP events on the stream it is launched on, together with the algorithmic
 * bytes that launch moves.  Classes:
 *   "trsv"  one triangular solve over all batch items (two per ilu_apply);
 *           bytes = sum over items of nnz_T * (s + 4) + 2 n s (+ n s for the
 *           pivot scaling of U-type solves), s = 16 (complex128) or 8;
 *   "spmv"  one SpMV or FP64 residual over all batch items;
 *           bytes = sum over items of nnz (s + 4) + 4 (n + 1) + 2 n s;
 *   "orth"  one Gram-Schmidt pass (dots or update) of an Arnoldi step.
 * om_profile_query waits for the recorded events of the class and returns the
 * number of launches, their summed duration (ms) and summed bytes.  The
 * counters are process-wide; om_profile_reset clears them. */
void om_profile_enable(int32_t on);
void om_profile_reset(void);
om_status om_profile_query(const char* kernel_class, int64_t* launches, double* total_ms, double* bytes);

/* ---- host-only entry points (no device; used for CPU checks of the host
 * algorithms) ------------------------------------------------------------- */

/* RCM of the n x n pattern (row_ptr int64[n+1], col int32[nnz], sorted per
 * row), as rcm_permute.  perm: int32[n] receives perm[new] = old. */
om_status om_host_rcm(int64_t n, const int64_t* row_ptr, const int32_t* col, int32_t* perm);

/* ILUT of a host CSR (values complex128 interleaved), as ilu_factor.  The
 * factors stay inside an om_ilu with no device part; read them with
 * om_ilu_info / om_ilu_export. */
om_status om_host_ilut(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* val,
                       double drop_tol, double fill_factor, om_ilu** M_out, om_ilu_stats* st);

#ifdef __cplusplus
}
#endif

#endif /* OMSS_H */
