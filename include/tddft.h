/*
 * libtddft — full (non-Tamm-Dancoff) linear-response TDDFT in two localised function
 * sets, on one MI355X (gfx950).
 *
 * Method: T. J. Zuehlsdorff, N. D. M. Hine, M. C. Payne, P. D. Haynes,
 * "Linear-scaling time-dependent density-functional theory beyond the Tamm-Dancoff
 * approximation ..." (arXiv:1507.08157).
 *
 * Notation.  The o-set {o_b} spans the occupied space (the paper's phi_beta), the
 * u-set {u_a} the low unoccupied space (the paper's chi_alpha).  Response kernels P^p,
 * P^q have u-set rows and o-set columns (Sec. III.A).  K^v, K^c are the valence and
 * conduction density kernels (Sec. II.C), S and H the overlap and Hamiltonian matrices
 * of each set.  All matrices are contravariant; the metric is Tr[X^T S^u Y S^o].
 *
 * Patterns.  M is the cutoff pattern of the auxiliary matrices L (Sec. III.A, Eq.
 * auxiliary); the response kernels are P = K^c S^u L S^o K^v and live on the response
 * pattern R: the blocks that product reaches from M, or M itself in the linear-scaling
 * mode (tddft_options.truncate_p, Sec. IV.C) (computed by tddft_create, exported by
 * tddft_response_pattern).  Response-kernel arrays at this interface hold the values of R's
 * blocks in (block row, block column) order, each block dense row-major.
 *
 * Conventions of this interface
 *   - Every call returns an int status (TDDFT_OK = 0, negative = error, positive =
 *     informational warning).  No call aborts or exits the process.
 *   - Host arrays passed to tddft_create are read during the call only; the caller keeps
 *     ownership and may free them on return.
 *   - Device arrays passed to tddft_apply / tddft_pcg_solve are caller-owned device
 *     memory of the GPU that was current at tddft_create; they must not alias each
 *     other.  Work is issued on the stream given at tddft_create (NULL = the default
 *     stream) and the calls return after it completes; a solve whose options name another
 *     stream is ordered after the work already queued there.
 *   - A handle is not thread-safe: use one handle per host thread.
 *   - Grid arrays index points as x + nx * (y + ny * z).
 */
#ifndef TDDFT_H
#define TDDFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDDFT_ABI_VERSION 1

/* ---- status codes ------------------------------------------------------------------ */
#define TDDFT_OK                 0
#define TDDFT_E_INVALID         -1  /* bad shapes, patterns, NaN/Inf, asymmetric S or H  */
#define TDDFT_E_NOMEM           -2  /* device or host allocation failed                  */
#define TDDFT_E_DEVICE          -3  /* HIP runtime error; text in tddft_last_error       */
#define TDDFT_E_NOT_PD          -4  /* Tsiper numerator/denominator not positive, or a
                                       non-positive Kohn-Sham gap detected              */
#define TDDFT_E_NO_CONVERGENCE  -5  /* outputs hold the last (best) iterate              */
#define TDDFT_W_FALLBACK         1  /* learned preconditioner rejected at least once     */

/* ---- precision modes --------------------------------------------------------------- */
#define TDDFT_FP64       0  /* everything FP64                                            */
#define TDDFT_FP32       1  /* grid samples, fields, sparse products FP32; traces FP64    */
#define TDDFT_BF16_GRID  2  /* grid samples BF16 (FP32 accumulation), rest as TDDFT_FP32  */

/* ---- coupling kernel ------------------------------------------------------------------ */
#define TDDFT_XC_ALDA_X  0  /* Hartree + adiabatic LDA exchange kernel (Sec. II.A)        */
#define TDDFT_XC_NONE    1  /* Hartree only                                                */
#define TDDFT_HXC_NONE   2  /* no coupling (A = B + D, B = 0): test closed form            */

/* ---- preconditioners (Sec. III.B) ------------------------------------------------------ */
#define TDDFT_PC_NONE       0
#define TDDFT_PC_KSDIFF_CG  1  /* solve Eq. precond by CG to relative tolerance eps_tol    */
#define TDDFT_PC_LEARNED    2  /* learned block correction, KSDIFF_CG as fallback          */

/* Block-sparse matrix in BSR form with variable block sizes (1 to 5 functions per atom).
 * Blocks are dense and row-major; their values are concatenated in (block row, colind)
 * order.  rowptr and colind describe the block pattern; colind is sorted within each block
 * row.  For a pattern-only matrix (M) val is NULL.  The largest u-set and o-set blocks set
 * the padded shape BU x BO of the kernels, which must be one of 3 x 2, 1 x 1, 2 x 2,
 * 3 x 3, 4 x 4 or 5 x 2 (the joint unoccupied representation of Eq. proj: o- and
 * u-functions of an atom in one u-set block); other shapes fail with TDDFT_E_INVALID. */
typedef struct {
  int32_t nbr, nbc;          /* number of block rows / block columns (atoms)            */
  const int32_t *row_off;    /* [nbr+1] first function of each block row               */
  const int32_t *col_off;    /* [nbc+1] first function of each block column            */
  const int64_t *rowptr;     /* [nbr+1] offsets into colind                            */
  const int32_t *colind;     /* [nnzb]                                                 */
  const double  *val;        /* [sum of block sizes] or NULL                           */
} tddft_bsr;

/* Grid-sampled localised functions.  Function f is given on a box of grid points with
 * corner origin[3f..3f+2] = (x, y, z) and dimensions extent[3f..3f+2]; the box wraps
 * periodically and must not exceed the cell.  val[off[f] .. off[f+1]) holds its values,
 * x fastest; values outside the function's support are zero.  Function f belongs to the
 * block (atom) whose row_off range contains f in the matrices of its set. */
typedef struct {
  int32_t n_fn;
  const int32_t *origin;     /* [3 * n_fn]                                             */
  const int32_t *extent;     /* [3 * n_fn]                                             */
  const int64_t *off;        /* [n_fn + 1]                                             */
  const double  *val;
} tddft_functions;

/* One system: a periodic orthorhombic cell with n[d] points along side L[d] (bohr). */
typedef struct {
  int32_t n[3];
  double  L[3];
  tddft_functions occ;       /* o-set                                                  */
  tddft_functions vir;       /* u-set                                                  */
  tddft_bsr S_o, H_o, K_v;   /* n_o x n_o, symmetric; same block structure             */
  tddft_bsr S_u, H_u, K_c;   /* n_u x n_u, symmetric; same block structure             */
  tddft_bsr M;               /* cutoff pattern of the auxiliary matrices L (u x o blocks) */
} tddft_system;

typedef struct {
  int32_t  precision;        /* TDDFT_FP64 | TDDFT_FP32 | TDDFT_BF16_GRID               */
  int32_t  xc;               /* TDDFT_XC_ALDA_X | TDDFT_XC_NONE | TDDFT_HXC_NONE        */
  double   rho_floor;        /* f_xc = 0 where rho0 < rho_floor (bohr^-3)               */
  double   coupling_scale;   /* K -> s K (test knob; 1 = the method)                    */
  int32_t  precond;          /* TDDFT_PC_*                                              */
  double   eps_tol;          /* inner CG relative tolerance (Sec. III.B)                */
  double   tol_omega;        /* Ha: stop when max |d omega| < tol and max |g| < sqrt(tol) */
  int32_t  max_iter;         /* outer iterations                                        */
  int32_t  max_inner;        /* inner CG iterations                                     */
  int32_t  refresh;          /* recompute F = apply(P) every `refresh` iterations       */
  int32_t  restart;          /* steepest-descent restart period                         */
  uint64_t seed;             /* initial guess when none is given                        */
  const void *model;         /* learned-preconditioner weights blob, or NULL           */
  int64_t  model_bytes;
  void    *stream;           /* hipStream_t, or NULL for the default stream             */
  double   eps_loose;        /* > eps_tol: adaptive inner tolerance eps_loose |g| / |g_0|
                                (max_i ||g_i||_S now and at the first iteration) clamped
                                to [eps_tol, eps_loose] (Sec. IV.A); 0 = constant eps_tol */
  int32_t  tda;              /* 1: Tamm-Dancoff mode (B = 0, Sec. II.B): both halves see
                                A = D + K, f_p = A P^p and f_q = A P^q; the solver keeps
                                p = q (started from Pq) and returns eig(A).  Fixed at
                                tddft_create like xc */
  int32_t  truncate_p;       /* 1: linear-scaling mode of Sec. IV.C: the response kernels
                                are truncated to M as well, so R = M and the trial vectors
                                are P = mask_M(K^c S^u L S^o K^v) (the invariance
                                constraint then holds only approximately, Sec. III.A after
                                Eq. auxiliary); 0: R is the pattern the exact product
                                reaches from M.  Fixed at tddft_create */
  int32_t  graphs;           /* 1 (default): a solve captures each distinct operator
                                application (its kernels on the handle's two streams) in a
                                HIP graph once and replays it; 0: direct launches.  Results
                                are identical either way */
  int32_t  autotune;         /* 1 (default): tddft_create times the candidate launch shapes
                                of the FFT passes (threads per workgroup), the response
                                density (tiles per workgroup), the sparse products
                                (columns per thread, pairs per round trip) and the dense
                                products (output tile) on the system's own data and keeps
                                the fastest; choices are remembered per process for
                                systems of the same shapes.  No choice changes a result.
                                0: fixed defaults */
  int32_t  density_pbcast;   /* -1 (default): the tuner's choice (scalar P when autotune
                                is 0); 0: the response density keeps P blocks in scalar
                                registers; 1: in vector registers shared by DPP row
                                broadcasts.  Results are identical either way */
  int32_t  gemm_tile;        /* -1 (default): the tuner's choice (0 when autotune is 0);
                                0, 1, 2: the output tile shape of every dense
                                (complete-pattern) MFMA product (left: 128x64, 64x64,
                                64x128; right: 64x64, 128x64, 64x128 rows x columns).  All
                                shapes share the k-slab depth: results are identical */
  int32_t  sparse_cw;        /* -1 (default, with sparse_pairs -1): the tuner's choice
                                (1 column, 4 pairs when autotune is 0).  Otherwise every
                                sparse-pattern product takes sparse_cw columns per thread
                                and sparse_pairs operand block pairs per memory round
                                trip, one of (1, 1), (1, 2), (1, 4), (1, 8), (2, 1),
                                (2, 2), (2, 4), (4, 1), (4, 2); both -1 or neither.  The
                                pairs are summed in the same order: results are identical */
  int32_t  sparse_pairs;
} tddft_options;

/* Per-solve statistics (host memory, caller-owned).  The log arrays are optional. */
typedef struct {
  int32_t iterations;        /* outer iterations done                                   */
  int32_t converged;
  int32_t inner_total;       /* inner CG iterations summed over all columns' maxima     */
  int32_t applies;           /* operator applications (each one for all states)         */
  int32_t fallbacks;         /* learned-preconditioner rejections                       */
  double  setup_ms;          /* tddft_create wall time                                  */
  double  solve_ms;          /* tddft_pcg_solve wall time                               */
  double  apply_ms;          /* summed device time of operator applications             */
  int32_t log_capacity;      /* entries the caller provided (0 = no log)                */
  int32_t log_len;           /* entries written                                         */
  double *log_omega;         /* [log_capacity * n_states] ascending omega per iteration */
  double *log_time_ms;       /* [log_capacity] wall time since solve entry              */
  double *log_gnorm;         /* [log_capacity] max_i ||g_i||_S                          */
  int32_t graph_replays;     /* operator applications replayed from captured HIP graphs */
} tddft_stats;

/* Sizes of the structures a handle built (for work and traffic accounting). */
typedef struct {
  int32_t n[3];              /* grid                                                    */
  int32_t tiles;             /* 4x4x4 grid tiles                                        */
  int32_t block_rows, block_cols;   /* padded block shape of response kernels (BU x BO)  */
  int32_t max_rows_o;        /* most o-set sample rows touching one tile                 */
  int32_t precision;
  int64_t sample_rows_u;     /* tile sample rows (64 points each) of the u-set          */
  int64_t sample_rows_o;     /* ... of the o-set                                        */
  int64_t pair_points;       /* sum over tiles of (u rows x o rows x 64)                */
  int64_t blocks_m;          /* blocks of M                                              */
  int64_t blocks_r;          /* blocks of the response pattern R                         */
  int64_t blocks_o;          /* blocks of the overlap pattern of the potential integrals */
  int64_t blocks_m2, blocks_m3, blocks_m4;  /* intermediate patterns of the sandwiches  */
  int64_t pairs_kshift;      /* block products of one K^c H^u X plus X H^o K^v (per column) */
  int64_t pairs_project;     /* ... of the projection                                   */
  int64_t pairs_project_t;   /* ... of its adjoint                                       */
  int64_t pairs_covariant;   /* ... of S^u X S^o                                        */
  int64_t pairs_sandwich;    /* ... of K^c V K^v                                        */
  int64_t partial_pairs;     /* function pairs with per-tile partial integral sums       */
  double  setup_ms;
  int64_t samples_u_nz;      /* nonzero grid samples of the u-set (points inside spheres) */
  int64_t samples_o_nz;      /* ... of the o-set                                         */
  int64_t pair_points_nz;    /* sum over grid points of (u-functions nonzero there) x
                                (o-functions nonzero there): the method's own work unit of
                                the response density and the potential integrals          */
  /* launch shapes in use (see tddft_options.autotune) */
  int32_t fft_threads[3];    /* FFT threads per workgroup per axis (0 = two-buffer form)  */
  int32_t density_waves;     /* response density: tiles per workgroup                    */
  int32_t kshift_cw[2];      /* K-shift products: columns per thread (left, right)       */
  int32_t density_pbcast;    /* response density: 1 = P blocks in vector registers
                                shared by DPP row broadcasts, 0 = P in scalar registers   */
  int32_t kshift_tile[2];    /* K-shift products in the dense form: output tile shape
                                (tddft_options.gemm_tile numbering; 0 for sparse forms)   */
  int32_t kshift_pairs[2];   /* K-shift products in the sparse form: operand block pairs
                                loaded per memory round trip (1, 2, 4 or 8; the dense
                                form does not use it, like kshift_cw)                    */
} tddft_info;

typedef struct tddft_handle tddft_handle;

/* Defaults: FP64, ALDA exchange, rho_floor 1e-10, coupling 1, KSDIFF_CG, eps_tol 1e-4,
 * tol_omega 1e-7, max_iter 300, max_inner 50, refresh 10, restart 20, seed 0, eps_loose 0,
 * tda 0, truncate_p 0, graphs 1, autotune 1, density_pbcast -1, gemm_tile -1,
 * sparse_cw -1, sparse_pairs -1. */
void tddft_default_options(tddft_options *opts);

/* Build a handle for one system (Sec. III.A: sparse K^v, K^c, S and H, the cutoff
 * pattern M and grid-sampled functions).  Validates the input (TDDFT_E_INVALID on bad
 * shapes, unsorted or out-of-range patterns, NaN/Inf, asymmetric S/H, functions whose
 * boxes exceed the cell, grid edges outside [2, 4096] or with a prime factor above 7, grid
 * edges whose FFT line buffers exceed a workgroup's LDS: with 160 KiB, FP64 edges of 640
 * points or more, or of more than 316 points with a factor 7, FP32 twice these), uploads
 * it to the current GPU, builds the
 * grid tiles and the sparse-product plans, and computes rho0 = 2 sum o_b K^v_bb' o_b' and
 * the ALDA kernel f_xc(r) (Sec. II.A) once.  opts->precision fixes the storage precision
 * of the grid samples for the handle's lifetime.  On success *out owns all device state. */
int tddft_create(const tddft_system *sys, const tddft_options *opts, tddft_handle **out);

int tddft_get_info(const tddft_handle *h, tddft_info *out);

/* Number of values of one response kernel (sum of the block sizes of R). */
int64_t tddft_nnz_p(const tddft_handle *h);

/* The response pattern R: rowptr [n_u blocks + 1] and colind [nnzb] (host arrays, either
 * may be NULL to query only).  Returns the number of blocks of R. */
int64_t tddft_response_pattern(const tddft_handle *h, int64_t *rowptr, int32_t *colind);

/* The operator of Eq. operator_RPA for n_states states at once:
 *   f_p = mask_R(K^c H^u P^p - P^p H^o K^v)
 *   f_q = mask_R(K^c H^u P^q - P^q H^o K^v + 2 s K^c V_SCF[P^q] K^v)
 * with V_SCF[P]_ab = h^3 sum_r u_a (V_H[rho] + f_xc rho) o_b, rho = sum u_a P_ab o_b,
 * V_H the periodic Hartree potential (G = 0 dropped) and s the coupling scale.
 * Pp, Pq, fp, fq: DEVICE arrays [n_states][tddft_nnz_p] FP64 in R's value order
 * (contravariant).  Every product is exact; only results are restricted to R.
 * n_states in [1, 32].  Internal arithmetic follows the handle's precision. */
int tddft_apply(tddft_handle *h, int32_t n_states, const double *Pp, const double *Pq,
                double *fp, double *fq);

/* tddft_apply without any device allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, arithmetic and results as tddft_apply; the column sets, grid fields, FFT
 * buffer and per-tile partial sums live in one device array that the library holds per GPU
 * for the life of the process, of tddft_apply_noalloc_limit() bytes (256 MiB).  An
 * application whose workspace exceeds that (large grids or many states; e.g. a 320^3 grid
 * at 32 FP32 states) fails with TDDFT_E_INVALID and a message naming the bytes needed.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * threads, other handles, other streams) race.  Nothing in it needs to start at zero.
 * The handle's GPU must be current.  While the handle's stream (a non-default stream
 * given at tddft_create) is being captured into a HIP graph, the call records its kernels
 * (on that stream and the handle's second stream, joined back) and returns without
 * waiting; every replay then applies the operator to what Pp and Pq hold at that time.
 * Otherwise it returns after the work completes. */
int tddft_apply_noalloc(tddft_handle *h, int32_t n_states, const double *Pp, const double *Pq,
                        double *fp, double *fq);
int64_t tddft_apply_noalloc_limit(void);

/* Lowest n_states positive excitation energies by preconditioned CG on the Tsiper sum
 * functional (Secs. III.A-III.C).  omega: HOST [n_states], ascending (Ha).
 * Pp, Pq: DEVICE [n_states][tddft_nnz_p] FP64 (R's layout) or NULL.  On input, if
 * non-NULL, their blocks on M are the initial auxiliary matrices L (Eq. auxiliary; other
 * blocks are ignored) and the trial vectors start at P = K^c S^u L S^o K^v; if NULL a seeded
 * N(0,1) guess on M is used.  On output (if non-NULL) they hold the converged
 * Tsiper-orthonormal vectors, rotated to the eigenvectors of the subspace matrix.
 * The optimisation variable is L on M.  Preconditioner (opts->precond): KSDIFF_CG solves
 * the Kohn-Sham-difference equation of Eq. precond by inner CG (on the trial-vector space
 * when M is complete, expressed on L otherwise); LEARNED scales each gradient block
 * elementwise by the output of the model blob opts->model (see tddft_mlp_export) evaluated
 * once per solve on tddft_block_features, falls back to KSDIFF_CG in any iteration where
 * that is not a descent direction for every state, and, when Pp/Pq are NULL, scales the
 * random initial L block by block by the model's guess head.  opts may be NULL (handle's
 * create options).  stats may be NULL.  precision, xc, rho_floor, coupling_scale, tda and
 * truncate_p belong to the handle: solve options that differ in them are rejected with
 * TDDFT_E_INVALID.
 * Returns TDDFT_E_NO_CONVERGENCE with the last iterate when max_iter is reached, and
 * TDDFT_W_FALLBACK (converged) when the learned scaling was rejected at least once. */
int tddft_pcg_solve(tddft_handle *h, int32_t n_states, const tddft_options *opts,
                    double *omega, double *Pp, double *Pq, tddft_stats *stats);

/* Oscillator strengths of converged excitations in the velocity form (the line strengths
 * listed with the excitation energies in Sec. IV.A, Table tab:azo, and broadened into the
 * spectra of Sec. IV.B; the paper prints no formula, and in a periodic cell the position
 * operator has no matrix elements between the functions):
 *   f_n = 2 / (3 omega_n) sum_alpha D_n,alpha^2,   D_n,alpha = sum_ab P^p_n,ab G^alpha_ab,
 *   G^alpha_ab = h^3 sum_r u_a(r) (d_alpha o_b)(r)
 * with d_alpha the second-order central difference on the periodic grid (G is built once
 * by tddft_create, FP64) and P^p_n = X_n - Y_n Tsiper-normalised, <p_n, q_n> = 1, as
 * tddft_pcg_solve returns them.  omega: HOST [n_states]; Pp: DEVICE [n_states][tddft_nnz_p]
 * FP64; f: HOST [n_states] out; moments: HOST [n_states][3] out (D_n, x y z) or NULL. */
int tddft_oscillator_strengths(tddft_handle *h, int32_t n_states, const double *omega,
                               const double *Pp, double *f, double *moments);

/* Solves of several systems at once (a work queue over systems): up to max_workers host
 * threads (0 = one per system, at most 16) each take the next unsolved system and run
 * tddft_pcg_solve on it on a private non-blocking stream of the handle's GPU, so the
 * kernels and host round trips of different systems overlap.  hs[k], n_states[k],
 * omega[k] (HOST [n_states[k]]), Pp[k] / Pq[k] (DEVICE or NULL; Pp and Pq may themselves
 * be NULL) and stats[k] (or stats NULL) are the per-system arguments of tddft_pcg_solve;
 * opts (or NULL for each handle's create options) is shared.  status[k] (HOST) receives
 * each system's return code; the call returns TDDFT_OK when every system was attempted
 * (check status), TDDFT_E_INVALID on bad arguments.  Results are identical to solving
 * the systems one after another.  Distinct handles only; no handle may be used by
 * another thread during the call.  The private streams are not ordered after other work:
 * device inputs must be complete (e.g. the device synchronised) before the call. */
int tddft_pcg_solve_batched(tddft_handle *const *hs, int32_t n_sys, const int32_t *n_states,
                            const tddft_options *opts, double *const *omega, double *const *Pp,
                            double *const *Pq, tddft_stats *stats, int32_t *status,
                            int32_t max_workers);

void tddft_destroy(tddft_handle *h);

/* ---- building blocks of the solver, exposed for training and testing -------------------- */

/* Pi(L) = mask_R(K^c S^u L S^o K^v) (Sec. III.A, Eq. auxiliary) for n_states auxiliary
 * matrices.  L, P: DEVICE [n_states][tddft_nnz_p] FP64 in R's layout; only L's blocks on M
 * are read.  n_states in [1, 32]. */
int tddft_project(tddft_handle *h, int32_t n_states, const double *L, double *P);

/* Eq. precond (Sec. III.B): K^c H^u G - G H^o K^v = g solved by CG in the metric
 * Tr[X^T S^u Y S^o] from G = 0, per state, to relative residual eps_tol or max_inner steps
 * (or non-positive curvature).  g, G: DEVICE [n_states][tddft_nnz_p] FP64.  Requires a
 * complete M (the trial vectors' own space); TDDFT_E_INVALID otherwise. */
int tddft_precondition(tddft_handle *h, int32_t n_states, const double *g, double *G,
                       double eps_tol, int32_t max_inner);

/* Two-atom features of every block (I, J) of R, in R's block order, for the learned
 * preconditioner: the upper triangles (row-major) of S^u_II, H^u_II, S^o_JJ, H^o_JJ; the
 * generalised eigenvalues of (H^u_II, S^u_II) and (H^o_JJ, S^o_JJ), ascending; their
 * differences (u index outer); the minimum-image distance (bohr) between the centres of
 * the two atoms' function boxes.  out: DEVICE [blocks of R][tddft_n_features] FP32. */
int32_t tddft_n_features(const tddft_handle *h);
int tddft_block_features(tddft_handle *h, float *out);

/* Guess targets from converged vectors: t_IJ = log10(sum_i ||P^q_i,IJ||^2 /
 * sum_i ||P^q_i||^2 + 1e-8) per block of R.  Pq: DEVICE [n_states][tddft_nnz_p] FP64;
 * t: DEVICE [blocks of R] FP32. */
int tddft_guess_targets(tddft_handle *h, int32_t n_states, const double *Pq, float *t);

/* ---- the learned preconditioner's network ----------------------------------------------
 * y = W3 a(W2 a(W1 x^ + b1) + b2) + b3 with a(z) = z / (1 + e^-z), x^ = (x - mean) / std,
 * hidden width `width`; outputs: y[0..E-1] elementwise scaling of a gradient block,
 * y[E] the guess head.  Master parameters and Adam moments are FP32; the forward and
 * backward passes use BF16 copies of the weight matrices (round to nearest even) with
 * FP32 accumulation.  Parameters are packed as W1 [n_in][width], b1, W2 [width][width],
 * b2, W3 [width][n_out], b3.  All row arrays are DEVICE FP32, row-major.  Work runs on the
 * stream given at creation.  Not thread-safe. */
typedef struct tddft_mlp tddft_mlp;

/* Weights ~ N(0, 2 / fan_in) from a seeded generator, zero biases, mean 0, std 1. */
int tddft_mlp_create(int32_t n_in, int32_t width, int32_t n_out, uint64_t seed, void *stream,
                     tddft_mlp **out);
void tddft_mlp_destroy(tddft_mlp *m);
int64_t tddft_mlp_n_params(const tddft_mlp *m);
/* host arrays: params [n_params] (packed order above), mean and std [n_in] (either pair
 * may be NULL to leave it unchanged / not read back) */
int tddft_mlp_set_params(tddft_mlp *m, const float *params, const float *mean, const float *std);
int tddft_mlp_get_params(const tddft_mlp *m, float *params, float *mean, float *std);
/* mean and std of each input column over rows X [rows][n_in] (FP64 sums; std floored at
 * 1e-6), stored as the network's input normalisation */
int tddft_mlp_fit_normalisation(tddft_mlp *m, int64_t rows, const float *X);
int tddft_mlp_forward(tddft_mlp *m, int64_t rows, const float *X, float *Y);
/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the loss
 *   sum_rows [ 1/2 ||y[0..E-1] * g - gstar||^2 / loss_scale + 1/2 (y[E] - t)^2 ]
 * with g, gstar [rows][E] and t [rows] (E = n_out - 1).  loss: HOST, the loss before the
 * step; grad: DEVICE [n_params] or NULL, the gradient used. */
int tddft_mlp_train_step(tddft_mlp *m, int64_t rows, const float *X, const float *g,
                         const float *gstar, const float *t, double loss_scale, double lr,
                         double *loss, float *grad);
/* Model blob for tddft_options.model: *size bytes (query with blob NULL). */
int tddft_mlp_export(const tddft_mlp *m, void *blob, int64_t cap, int64_t *size);
int tddft_mlp_import(const void *blob, int64_t size, void *stream, tddft_mlp **out);
const char *tddft_mlp_last_error(const tddft_mlp *m);

/* Device-time profiling of the kernel stages (HIP events recorded on the handle's stream
 * around each stage; enabling it adds event records and host waits, not extra kernels).
 * Outside profiling an application runs its K-shift products on a second stream of the
 * handle, beside the coupling term; while profiling is on, every stage runs on the
 * handle's stream one after another, so that each stage's time is its own.
 * tddft_profile(h, 1) enables and zeroes the counters, tddft_profile(h, 0) disables.
 * tddft_profile_read copies up to cap entries of accumulated milliseconds and execution
 * counts per stage (caller-owned host arrays) and returns the number of stages;
 * tddft_profile_stage_name names stage k (NULL when out of range). */
int tddft_profile(tddft_handle *h, int enable);
int tddft_profile_read(tddft_handle *h, int cap, double *ms, int64_t *count);
const char *tddft_profile_stage_name(int k);

const char *tddft_strerror(int code);
/* Detail of the last failing call on this handle (or of the last failing tddft_create
 * on this thread when h is NULL). */
const char *tddft_last_error(const tddft_handle *h);
int tddft_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TDDFT_H */
