/*
 * dgdft_alb.h -- C ABI of the MI355X library for DGDFT's adaptive-local-basis
 * (ALB) generation step.
 *
 * What the library computes (Hu, Lin, Yang, "DGDFT: a massively parallel
 * method for large scale density functional theory calculations"):
 *
 *   For every extended element Q_K of a batch, the lowest J_K eigenpairs of
 *   the local Kohn-Sham operator  -1/2 Laplacian + V_eff^Q + V_nl^Q  with the
 *   normalisation  integral over Q_K of psi_j psi_j' = delta  (Sec. II.A,
 *   Eq. localproblem), discretised by planewaves on the periodic box of Q_K
 *   (Sec. II.B, grid rule Eq. Ngecut) and solved by Teter-preconditioned
 *   LOBPCG (Sec. II.B, "Generation of the ALB functions"); the nonlocal part
 *   is of Kleinman-Bylander form  sum_p gamma_p |b_p><b_p|  (Eq. DGvar).
 *   The eigenvectors are then restricted to the element E_K and
 *   orthonormalised (Sec. II.A after Eq. localproblem; Eq. orthonormal), here
 *   as an SVD truncation to n_alb functions.
 *
 * Conventions shared by every entry point
 *   - Grids are flattened x fastest: flat = i + n1*(j + n2*k).
 *   - Block matrices are column-major, one orbital per column, leading
 *     dimension = rows (no padding at the ABI).
 *   - Batched arrays are the per-element arrays concatenated in element order.
 *   - Units: Hartree atomic units (bohr, Ha).  All floating point is FP64 at
 *     the ABI.
 *   - "device" pointers are HIP device memory of the device current at
 *     dgdft_alb_create; "host" pointers are ordinary host memory.
 *   - Work is enqueued on the caller's hipStream_t (passed as void*; NULL =
 *     the null stream).  Entry points that return results to the host
 *     (status, stats) synchronise that stream before returning.
 *   - No entry point aborts or throws; failures return a negative status and
 *     leave a message for dgdft_alb_last_error.
 *   - One handle must not be used from two threads at once; distinct handles
 *     are independent.
 */
#ifndef DGDFT_ALB_H
#define DGDFT_ALB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define DGDFT_OK               0   /* success                                     */
#define DGDFT_NOT_CONVERGED    1   /* warning: outputs written, some element did  *
                                    * not reach tol within max_iter (see stats)   */
#define DGDFT_EINVAL          -1   /* bad argument: null pointer, bad shape,      *
                                    * non-finite input, box outside the grid ...  */
#define DGDFT_EUNSUPPORTED    -2   /* grid edge with a prime factor > 5, plane or *
                                    * pencil tile above the LDS limit, J > 1024   */
#define DGDFT_ENOMEM          -3   /* device allocation failed                    */
#define DGDFT_EHIP            -4   /* HIP runtime error (message in last_error)   */
#define DGDFT_EBREAKDOWN      -5   /* initial block rank deficient (CholQR)       */

#define DGDFT_PREC_FP64        0
#define DGDFT_PREC_MIXED       1   /* FP32 transforms of the preconditioner; with *
                                    * the orthonormalised direction (no guard      *
                                    * columns, or tol < 1e-7) also FP32 transforms *
                                    * for H W and FP32 MFMA products for the       *
                                    * projection and normalisation of W; Grams of  *
                                    * S, Rayleigh-Ritz, X/HX/P/HP updates, final   *
                                    * check and ALBs stay FP64                     */

#define DGDFT_PRECOND_TETER    0
#define DGDFT_PRECOND_LEARNED  1   /* Teter factor times a learned per-shell gain *
                                    * (network below), Teter fallback per band    */
#define DGDFT_PRECOND_NONE     2   /* identity (for tests)                        */

typedef struct dgdft_alb dgdft_alb;   /* opaque handle */

/* Options for dgdft_alb_create.  Zero-initialise, then set fields; a NULL
 * options pointer means all defaults.  Array fields are host pointers with
 * one entry (or three, for boxes) per element, copied at create. */
typedef struct dgdft_alb_opts {
    int32_t precision;        /* DGDFT_PREC_*, default FP64                        */
    int32_t precond;          /* DGDFT_PRECOND_*, default TETER                    */
    double  tol;              /* residual tolerance, default 1e-8 (0 = default)   *
                               * converged iff max_i ||H x_i - theta_i x_i||_2     *
                               * <= tol for unit x_i, in FP64                      */
    int32_t max_iter;         /* LOBPCG iteration cap, default 500 (0 = default)  */
    int32_t poll_every;       /* host convergence poll period in iterations,      *
                               * default 1                                         */
    const int32_t* elem_lo;   /* [n_elem][3] restriction box, half-open; NULL =   */
    const int32_t* elem_hi;   /*   central floor(n/3) points per axis             */
    const int32_t* n_alb;     /* [n_elem] ALBs per element; NULL = (J-n_guard)/2  */
    const float* mlp_weights; /* device [DGDFT_MLP_NTOT]: network of the learned  *
                               * preconditioner (read at every solve; may also be  *
                               * set later with dgdft_alb_set_mlp)                 */
    int32_t graph_iters;      /* K > 0: each element group runs K LOBPCG          *
                               * iterations per launch of a HIP graph captured     *
                               * for its active set (re-captured when the set      *
                               * changes); elements are checked between launches, *
                               * so one that converges inside a launch runs the    *
                               * rest of its K iterations.  0 = one launch per     *
                               * kernel, checks every iteration (default)          */
    int32_t tune;             /* 1: at create, time the split-K chunk count of    *
                               * the N_g-long Gram products per element shape and  *
                               * keep the fastest (see dgdft_alb_get_tuning)       */
    int32_t n_guard;          /* guard columns (default 0): the last n_guard of    *
                               * each element's n_states columns iterate with the  *
                               * block but are not held to tol, and the ALBs (and  *
                               * the volume terms) use only the first              *
                               * n_states - n_guard states.  The block then        *
                               * converges at the rate set by the gap to state     *
                               * n_states + 1 instead of n_states - n_guard + 1    *
                               * (LOBPCG, Sec. II.B, computes the lowest J_K       *
                               * states; guards are an addition of this library).  *
                               * Must be < every n_states.  Outputs keep all       *
                               * n_states columns; the guard ones are returned as  *
                               * they stand                                        */
    int32_t n_streams;        /* element groups iterating on their own HIP         *
                               * streams, 1 or 2 (0 = 2): with two, one group's    *
                               * small dense steps overlap the other's block       *
                               * products                                          */
    uint64_t seed;            /* seed of the start block drawn when               *
                               * dgdft_alb_solve gets X0 == NULL (see             *
                               * dgdft_alb_initial_guess)                          */
} dgdft_alb_opts;

/* Kleinman-Bylander projectors of the whole batch, CSR by projector
 * (the b_{I,l}, gamma_{I,l} of Eq. DGvar).  Projector p of element e covers
 * idx/val[ptr[p] .. ptr[p+1]); projectors are numbered element after element.
 *   n_proj  host   [n_elem]          projectors per element (may be 0)
 *   gamma   device [sum n_proj]      coupling constants (Ha)
 *   ptr     device [sum n_proj + 1]  offsets into idx/val (ptr[0] = 0)
 *   idx     device [nnz]             flat grid index within the element's grid
 *   val     device [nnz]             b_p sampled on the grid, normalised so that
 *                                    dV * sum val^2 = 1 (bohr^-3/2)
 * The library copies these arrays to the host once per dgdft_alb_solve /
 * dgdft_alb_set_potential and re-lays them out for its kernels. */
typedef struct dgdft_kb {
    const int32_t* n_proj;
    const double*  gamma;
    const int64_t* ptr;
    const int32_t* idx;
    const double*  val;
} dgdft_kb;

#define DGDFT_PHASES 5

/* Per-element results of dgdft_alb_solve (host array, one per element). */
typedef struct dgdft_alb_stats {
    int32_t iters;            /* LOBPCG iterations performed                       */
    int32_t converged;        /* 1 iff the final FP64 residual max <= tol          */
    double  max_res;          /* final max_i residual (FP64); with guard columns   *
                               * both fields cover only the wanted states          *
                               * (the first n_states - n_guard columns)            */
    int32_t n_chol_fallback;  /* W orthonormalisations that fell back to SVQB      */
    int32_t n_rr_fallback;    /* Rayleigh-Ritz steps with a rank-deficient basis   */
    int32_t n_p_drop;         /* Rayleigh-Ritz steps without P (its block was      *
                               * numerically dependent on [X W])                   */
    int32_t n_ql_fail;        /* small eigensolves whose QL iteration hit its cap  *
                               * (SVQB and the reduction of a rank-deficient     *
                               * basis)                                           */
    int32_t n_teter_fallback; /* bands switched to the Teter factor (learned mode)  */
    int32_t graph_launches;   /* graph launches that advanced this element          */
    int32_t n_rr_cholesky;    /* Rayleigh-Ritz steps reduced by a Cholesky of S^T S */
    int32_t n_rr_series;      /* ... by the series for (S^T S)^-1/2 (basis nearly   *
                               * orthonormal, ||S^T S - I||_F <= 1e-4)              */
    double  ms_by_phase[DGDFT_PHASES];  /* wall time of the solve's phases for    *
                               * the whole batch (the same in every element's      *
                               * record; the stream is synchronised at each phase  *
                               * boundary): potential load, start (X0, CholQR,      *
                               * H X, Rayleigh-Ritz on X), LOBPCG iterations, final *
                               * FP64 checks, restriction + SVD truncation         */
} dgdft_alb_stats;

/* Create a handle for a batch of n_elem extended elements.
 *   grid     host [n_elem][3]  grid points per axis; each edge >= 2 with prime
 *                              factors in {2,3,5}
 *   box      host [n_elem][3]  box lengths L_d (bohr), > 0
 *   n_states host [n_elem]     J_K, 1 <= J_K <= min(N_g, 1024)
 *   opts     host or NULL
 * Allocates the device workspace for the whole batch on the current device.
 * On failure *out is NULL and dgdft_alb_last_error(NULL) explains. */
int32_t dgdft_alb_create(dgdft_alb** out, const int32_t* grid, const double* box,
                         int32_t n_elem, const int32_t* n_states,
                         const dgdft_alb_opts* opts);

/* Release everything the handle owns.  NULL is a no-op. */
void dgdft_alb_destroy(dgdft_alb* h);

/* Sizes and offsets of element `elem` in the concatenated arrays.
 * Any output pointer may be NULL.  offsets (if non-NULL) receives 4 values:
 * offset of the element in V/eigvecs rows-space (sum of N_g of earlier
 * elements), in eigvecs (sum N_g*J), in eigvals (sum J), in albs (sum N_E*n_alb).
 */
int32_t dgdft_alb_sizes(const dgdft_alb* h, int32_t elem, int64_t* ng, int64_t* ne,
                        int32_t* n_states, int32_t* n_alb, int64_t* offsets);

/* Tuned parameters of element `elem` (host outputs, nullable): the split-K
 * chunk count of its N_g-long Gram products (0 = the default rule). */
int32_t dgdft_alb_get_tuning(const dgdft_alb* h, int32_t elem, int32_t* gram_split);

/* Cached tuning: set element `elem`'s split-K chunk count (0 = the default
 * rule, else 1..8), e.g. a value dgdft_alb_get_tuning returned for a
 * handle of the same element shapes created with opts.tune = 1, so that a
 * new handle skips the timing runs.  The three tuning modes are thus: off
 * (opts.tune = 0), full (opts.tune = 1), cached (opts.tune = 0, then this
 * call per element).  Synchronous; EINVAL for an index or count out of
 * range.  Not concurrent with a solve on h. */
int32_t dgdft_alb_set_tuning(dgdft_alb* h, int32_t elem, int32_t gram_split);

/* Load the restricted potentials of all elements (V_eff^Q and V_nl^Q of
 * Sec. II.A).  V: device [sum N_g] (Ha); kb as above (n_proj may be NULL for
 * no projectors).  Validates finiteness; the data are copied, so the caller
 * may free them afterwards. */
int32_t dgdft_alb_set_potential(dgdft_alb* h, const double* V, const dgdft_kb* kb,
                                void* stream);

/* Solve every element: LOBPCG from X0 to the tolerance, final FP64 check,
 * then restriction + SVD truncation (Sec. II.A-B).
 *   V, kb    as in dgdft_alb_set_potential; V == NULL keeps the loaded ones
 *   X0       device [sum N_g*J] initial guesses (full column rank), read only;
 *            NULL: the seeded N(0,1) block of dgdft_alb_initial_guess with
 *            opts.seed
 *   eigvals  device [sum J]        ascending per element (Ha)
 *   eigvecs  device [sum N_g*J] or NULL; dV * sum psi^2 = 1 (Eq. localproblem)
 *   albs     device [sum N_E*n_alb] or NULL; dV * sum_E phi^2 = 1, descending
 *            singular value, largest-|entry| positive (Eq. orthonormal)
 *   sigma    device [sum n_alb] or NULL; singular values of the restricted
 *            unit eigenvectors
 *   stats    host [n_elem] or NULL
 * Returns DGDFT_OK, DGDFT_NOT_CONVERGED (outputs still written) or an error.
 * Synchronises `stream` before returning. */
int32_t dgdft_alb_solve(dgdft_alb* h, const double* V, const dgdft_kb* kb,
                        const double* X0, double* eigvals, double* eigvecs,
                        double* albs, double* sigma, dgdft_alb_stats* stats,
                        void* stream);

/* The start block the solver draws when it is given no initial guess (the
 * seeded random start of Sec. II.B's LOBPCG): X0 (device [sum N_g*J], the
 * layout of dgdft_alb_solve's X0) with entries of standard normal law.  Rows
 * 2q, 2q+1 of column j of batch element e come from the counter-based
 * generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) at counter
 * (q, j, e, 0) and key (seed mod 2^32, seed div 2^32): its outputs w0..w3
 * give u1 = (w0 2^21 + w1 div 2^11) 2^-53 and u2 from (w2, w3), and the
 * Box-Muller transform x_2q = r cos(2 pi u2), x_2q+1 = r sin(2 pi u2),
 * r = sqrt(-2 ln(1 - u1)) (an odd N_g drops the last sine). */
int32_t dgdft_alb_initial_guess(dgdft_alb* h, uint64_t seed, double* X0, void* stream);

/* Apply the discrete operator of element `elem` (loaded potential) to ncols
 * unit-basis columns: HX = (F^-1 diag(|G|^2/2) F + diag(V) +
 * sum_p gamma_p beta_p beta_p^T) X with beta_p = sqrt(dV) b_p
 * (Eq. localproblem with the KB term of Eq. DGvar; the operation-1 of the
 * LOBPCG list in Sec. II.B).  X, HX: device [N_g*ncols]; 1 <= ncols <= J.
 * A handle created with DGDFT_PREC_MIXED applies the kinetic term with FP32
 * transforms, as inside its iteration (V and KB terms in FP64). */
int32_t dgdft_alb_apply_h(dgdft_alb* h, int32_t elem, const double* X, double* HX,
                          int32_t ncols, void* stream);

/* Teter preconditioner of element `elem` (Sec. II.B; Payne, Teter, Allan et
 * al.): W_i = F^-1 K(|G|^2/2 / T_i) F R_i with T_i = the kinetic energy of the
 * unit vector X_i, floored at (2 pi / L_max)^2 / 2, and
 * K(x) = (27+18x+12x^2+8x^3)/(27+18x+12x^2+8x^3+16x^4).
 * R, X, W: device [N_g*ncols]; W may equal R.  FP32 transforms for a
 * DGDFT_PREC_MIXED handle (T_i in FP64). */
int32_t dgdft_alb_precondition(dgdft_alb* h, int32_t elem, const double* R,
                               const double* X, double* W, int32_t ncols, void* stream);

/* Block orthonormalisation step of the LOBPCG iteration (Sec. II.B: the
 * correction block W is made orthonormal before H is applied to it), on the
 * solver's own kernel, exported so its branches can be tested: for the
 * J x J Gram G = Y^T Y of a block Y (J = n_states of element `elem`;
 * device, column-major, upper triangle read) returns T (device [J*J],
 * column-major) with Y T orthonormal:
 *   CholQR: T = D^-1 L^-T with D^-1 G D^-1 = L L^T, D = diag(G)^1/2, when
 *           every pivot^2 of L exceeds 1e-10;
 *   SVQB:   otherwise T = D^-1 U Lambda^-1/2, D^-1 G D^-1 = U Lambda U^T
 *           with Lambda clamped below at 1e-10 max(Lambda).
 * init = 1 treats the block as the initial guess: a failed pivot test then
 * marks breakdown (flags[3]) instead of taking SVQB (T is still written).
 * flags: host [6] = SVQB fallbacks, Rayleigh-Ritz fallbacks, P drops,
 * breakdown, Rayleigh-Ritz reduction path, eigensolver iteration-cap hits.
 * Uses the element's workspace; not concurrent with a solve on h. */
int32_t dgdft_alb_orthonormalise(dgdft_alb* h, int32_t elem, const double* G, double* T,
                                 int32_t init, int32_t* flags, void* stream);

/* Rayleigh-Ritz step of the LOBPCG iteration (operation 4 of the list in
 * Sec. II.B) on the solver's own kernels, exported so its branches can be
 * tested.  With J = n_states of element `elem` and n = kb J (kb = 1: the
 * basis X alone; 2: [X W]; 3: [X P W]), Hh and M (device, n x n column-major,
 * upper triangles read) are S^T H S and S^T S.  Outputs (device): theta [J]
 * the lowest generalised eigenvalues of (Hh, M) ascending; C [n*J] the
 * coefficients with C^T M C = I; for kb > 1, D [n*J] the coefficients of
 * the next search direction P' = S D, in the form the solver uses for the
 * handle:
 *   - handles without guard columns and handles with a tolerance below
 *     1e-7: the part of [0; C_P; C_W] (C with its
 *     first J rows zeroed) M-orthogonal to C, normalised so that
 *     D^T M D = I, or all zero when that normalisation breaks down (P is
 *     then dropped, flags[2]);
 *   - handles with guard columns (opts.n_guard > 0) and opts.tol >= 1e-7:
 *     Knyazev's form,
 *     D = C with its first J rows zeroed (P' = [P W] [C_P; C_W], neither
 *     normalised nor orthogonal to X' = S C).  For kb = 3, where the
 *     solver's X and W blocks are orthonormal and mutually orthogonal, the
 *     P block is first orthonormalised against [X W] through a scaled
 *     Cholesky of its Schur complement M_PP - M_XP^T M_XP - M_WP^T M_WP;
 *     if that breaks, P is dropped for the step (flags[2]; C_P = 0, the step
 *     runs on [X W]: the P block of the reduced problem is decoupled with
 *     M_PP = I and a diagonal above every kept Ritz value).
 * Reductions: the binomial series for M^-1/2 when ||M - I||_F <= 1e-4
 * (kb > 1), a scaled Cholesky of M, or, when M is not numerically positive
 * definite, its eigenvectors above 1e-10 of the largest eigenvalue
 * (flags[1]; fewer than J of them sets flags[3]).  flags: host [6] as for
 * dgdft_alb_orthonormalise.  Uses the element's
 * workspace; not concurrent with a solve on h. */
int32_t dgdft_alb_rayleigh_ritz(dgdft_alb* h, int32_t elem, int32_t kb, const double* Hh,
                                const double* M, double* theta, double* C, double* D,
                                int32_t* flags, void* stream);

/* Batched FP64 symmetric eigensolver used for the Rayleigh-Ritz step
 * (operation 4 of the LOBPCG list in Sec. II.B): for each of `count` n x n
 * matrices A (device, column-major, lda = n, only the upper triangle read),
 * w = eigenvalues ascending (device [count*n]) and Z = the first k unit
 * eigenvectors (device [count*n*k]).  n <= 3072.
 * method 0: Householder tridiagonalisation, bisection and inverse iteration
 *           for the k lowest only (w[0..k) written per matrix) -- the path of
 *           the solver; for 513 <= n <= 832 the tridiagonalisation runs over
 *           eight workgroups per matrix, one kernel launch per Householder
 *           step (n + 1 launches in all, e.g. in a captured graph);
 *           method 1: implicit QL on the whole spectrum. */
int32_t dgdft_small_syev(int32_t count, int32_t n, int32_t k, const double* A,
                         double* w, double* Z, int32_t method, void* stream);

/* dgdft_small_syev without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and kernels; the eigensolver's
 * workspace is a static device array of 4 Mi doubles (32 MiB) that every GPU
 * the library runs on holds until the process ends, so
 *   count * (2 n^2 + 8 n + 6 n k) <= 4194304
 * or DGDFT_EINVAL (message in dgdft_alb_last_error(NULL)).  A, w, Z stay the
 * caller's.  All calls on one GPU share that GPU's workspace: calls that
 * overlap in time on one GPU (two streams, two threads) race and must be
 * serialised by the caller.  The workspace keeps the last call's contents;
 * the kernels write every part of it they read.  Synchronises `stream`. */
int32_t dgdft_small_syev_noalloc(int32_t count, int32_t n, int32_t k, const double* A,
                                 double* w, double* Z, int32_t method, void* stream);

/* Batched tall-skinny product on matrix cores (operations 2 and 3 of the
 * LOBPCG list in Sec. II.B), exported for tests:
 *   trans & 1 == 1: C (m x n) = A^T B with A (K x m), B (K x n)
 *   trans & 1 == 0: C (K x n) = alpha A B + beta C with A (K x m), B (m x n)
 * all column-major with leading dimension = rows, `count` independent
 * problems laid out back to back.  Device pointers, FP64 storage.  trans & 2
 * selects the kernels of the mixed form: operands rounded to FP32 as they
 * are staged, FP32 products and accumulation within a split-K chunk (Gram)
 * or the whole inner dimension (update), FP64 chunk sums and output. */
int32_t dgdft_gemm_batched(int32_t trans, int32_t count, int64_t K, int32_t m,
                           int32_t n, double alpha, const double* A, const double* B,
                           double beta, double* C, void* stream);

/* ---- per-kernel timing (diagnostics) ---------------------------------
 * When enabled, every launch of the listed kernel classes is bracketed by
 * HIP events on the launch stream; durations are accumulated at the host
 * polls.  Algorithmic work per launch: Gram products count 2 K m n flops
 * (K m (m+1) for the symmetric, upper-triangle products) and 8 K (m + n)
 * bytes; update products 2 K kA n flops and 8 K (kA + n) bytes (+8 K n when
 * accumulating); FFT passes count the HBM bytes of their input and output;
 * the strided-batched products of dgdft_alb_dg_volume count 2 M N K per
 * problem and the bytes of their operands (a shared operand once) and result. */
#define DGDFT_K_GRAM         0
#define DGDFT_K_GRAM_REDUCE  1
#define DGDFT_K_UPDATE       2
#define DGDFT_K_FFT_XY_FWD   3
#define DGDFT_K_FFT_Z        4
#define DGDFT_K_FFT_XY_INV   5
#define DGDFT_K_KB_PROJECT   6
#define DGDFT_K_RESID        7
#define DGDFT_K_RR           8
#define DGDFT_K_CHOLQR       9
#define DGDFT_K_OTHER       10
#define DGDFT_K_SGEMM       11
#define DGDFT_K_BGEMM       12
#define DGDFT_KCLASS_COUNT  13

/* Enable (1) or disable (0) timing and reset the counters. */
int32_t dgdft_alb_profile(dgdft_alb* h, int32_t enable);

/* Accumulated launches, milliseconds, algorithmic flops and bytes of one
 * kernel class since the last dgdft_alb_profile call.  Outputs nullable. */
int32_t dgdft_alb_kernel_stats(const dgdft_alb* h, int32_t kclass, int64_t* launches,
                               double* ms, double* flops, double* bytes);

/* Kernel symbol name of a class ("dg_gram", ...). */
const char* dgdft_kernel_class_name(int32_t kclass);

/* Batched products of the small Rayleigh-Ritz matrices (operation 4 of the
 * LOBPCG list in Sec. II.B works on matrices of size n = kb*J), exported for
 * tests: C = alpha op(A) op(B) + beta C with each dimension d* = 0 -> n,
 * 1 -> J (dm rows of C, dn columns of C, dk inner), op = transpose when
 * ta/tb = 1.  `count` problems back to back, each column-major with leading
 * dimension = rows as stored.  J <= 1024, kb in 1..3.  Device pointers. */
int32_t dgdft_small_gemm_batched(int32_t ta, int32_t tb, int32_t count, int32_t J,
                                 int32_t kb, int32_t dm, int32_t dn, int32_t dk,
                                 double alpha, const double* A, const double* B,
                                 double beta, double* C, void* stream);

/* ---- learned preconditioner --------------------------------------------
 * Not in the paper: a refinement of its Teter preconditioner (Sec. II.B).
 * Band i of an element gets the factor
 *   K_i(G) = K_Teter(t / T_i) * exp(f(u)),  f = 2 tanh(z(u) / 2),  t = |G|^2/2,
 *   u = ((log max(t / T_i, 1e-3), theta_i, Vbar) - mu) / sd,
 * with T_i as for Teter, theta_i = x_i^T H x_i and Vbar the mean of V.  z is a
 * perceptron 3 -> 64 -> 64 -> 1 with SiLU activations, evaluated in FP32 with
 * its trained weights rounded to bfloat16; the bound keeps K_i within a factor
 * e^2 of Teter's.  K_i depends on G through |G|^2
 * only, so it is tabulated per shell (distinct value of |G|^2 on the grid).
 * A band whose residual has not fallen below 0.9 times its value three
 * iterations earlier uses the Teter factor for the rest of the solve.
 *
 * Parameter vector, FP32, DGDFT_MLP_NTOT values: W1 [64][3] (row = hidden
 * unit), b1 [64], W2 [64][64] (row = output unit), b2 [64], w3 [64], b3,
 * mu [3], sd [3] (the last six are not trained). */
#define DGDFT_MLP_HIDDEN  64
#define DGDFT_MLP_NW      4481
#define DGDFT_MLP_NTOT    4487

/* Replace the network used by DGDFT_PRECOND_LEARNED (device pointer, read at
 * every solve; the caller keeps it alive). */
int32_t dgdft_alb_set_mlp(dgdft_alb* h, const float* weights);

/* Shells of element `elem`: n_shell (host) and, if t_shell is non-NULL, the
 * ascending values of |G|^2/2 (host [n_shell]).  Equal values up to 1e-12
 * relative form one shell. */
int32_t dgdft_alb_shells(const dgdft_alb* h, int32_t elem, int32_t* n_shell, double* t_shell);

/* Training pairs.  A sample is one band of one element at one LOBPCG
 * iteration; its rows are the element's shells.  With r the residual of the
 * band and e = (I - X X^T) x~ its ideal correction (x~: the band's Ritz
 * vector projected on the converged eigenvectors of its cluster, i.e. of
 * eigenvalues within 1e-6 Ha), under the unnormalised DFT:
 *   a[row] = sum_{G in shell} Re(conj(r^(G)) e^(G)),  b[row] = sum |r^(G)|^2,
 *   s_feat[4 s + 3] = e2 = sum_G |e^(G)|^2.
 * The training loss of a sample is 1 - (sum K a)^2 / ((sum K^2 b) e2) with K
 * the factor above on each shell.  All arrays are device memory. */
typedef struct dgdft_pairs {
    int64_t n_samples;
    int32_t n_elem;
    const int64_t* shell_off;  /* [n_elem + 1] offsets into t_shell               */
    const double*  t_shell;    /* |G|^2/2 per shell, per element                  */
    const int32_t* s_elem;     /* [n_samples] element of the sample               */
    const int64_t* s_row;      /* [n_samples] first row of the sample in a, b     */
    const double*  s_feat;     /* [n_samples][4] theta, T, Vbar, e2               */
    const double*  a;
    const double*  b;
} dgdft_pairs;

/* Number of samples and rows dgdft_alb_log_pairs writes for max_log
 * iterations: samples sum_e max_log J_e, rows sum_e max_log J_e n_shell_e. */
int32_t dgdft_alb_log_capacity(const dgdft_alb* h, int32_t max_log, int64_t* n_samples,
                               int64_t* n_rows);

/* Generate training pairs with the solver itself: a first solve from X0
 * gives the converged eigenvectors; a second solve from X0 records, at each
 * of its first max_log iterations, every band's shell sums (before the
 * preconditioner is applied).  Sample of element e, iteration k, band i:
 * index sum_{e' < e} max_log J_e' + k J_e + i; its rows follow the same
 * order (n_shell_e each).  Outputs (device, sized by
 * dgdft_alb_log_capacity): s_elem, s_row, s_feat, a, b; n_logged (host
 * [n_elem]) = iterations recorded per element (samples of later iterations
 * are left with e2 = 0).  V, kb as in dgdft_alb_solve.  Requires J >= 2 and
 * at most 4096 shells per element. */
int32_t dgdft_alb_log_pairs(dgdft_alb* h, const double* V, const dgdft_kb* kb, const double* X0,
                            int32_t max_log, int32_t* s_elem, int64_t* s_row, double* s_feat,
                            double* a, double* b, int32_t* n_logged, void* stream);

/* Training options (zero-initialise; 0 = default). */
typedef struct dgdft_train_opts {
    int32_t epochs;           /* default 10                                     */
    int32_t batch;            /* samples per Adam step, default 256             */
    double  lr;               /* default 1e-3                                   */
    double  beta1, beta2, eps;/* defaults 0.9, 0.999, 1e-8                       */
    uint64_t seed;            /* minibatch order                                */
    int32_t set_norm;         /* 1: set mu, sd from the selected samples first  */
} dgdft_train_opts;

/* Train the network on the GPU (hand-written forward, backward and Adam
 * kernels; FP32 master weights, bfloat16 evaluation, FP32 accumulation).
 * index: host [n_index] samples to use (NULL = all); samples with e2 <= 0
 * are skipped.  weights: device [DGDFT_MLP_NTOT], updated in place.
 * loss_hist: host [epochs] mean sample loss of each epoch, or NULL. */
int32_t dgdft_mlp_train(const dgdft_pairs* data, const int64_t* index, int64_t n_index,
                        const dgdft_train_opts* opts, float* weights, double* loss_hist,
                        void* stream);

/* Mean loss (host) and its gradient with respect to the DGDFT_MLP_NW trained
 * parameters (device [DGDFT_MLP_NW], FP64) over the selected samples, at the
 * bfloat16-rounded weights (one forward + backward pass; exported for the
 * gradient check). */
int32_t dgdft_mlp_grad(const dgdft_pairs* data, const int64_t* index, int64_t n_index,
                       const float* weights, double* loss, double* grad, void* stream);

/* f (after the bound) for n raw input rows feat (device [n][3] = x, theta, Vbar with x = t/T;
 * the logarithm and standardisation are applied inside) into f (device [n]).
 * Exported for tests. */
int32_t dgdft_mlp_eval(const double* feat, int64_t n, const float* weights, double* f,
                       void* stream);

/* ---- element-local DG quantities from the ALBs -------------------------
 * albs: device [sum N_E n_alb], the layout dgdft_alb_solve writes (per
 * element N_E x n_alb column-major, rows in element-box order x fastest,
 * dV sum phi^2 = 1). */

/* Electron density on every element box from the diagonal blocks of the
 * density matrix (Sec. II.A, Eq. newdensity: the ALBs of different elements
 * do not overlap, so only P_{K;K} enters):
 *   rho_K(x) = sum_{j,j'} phi_{K,j}(x) P_{K,j;K,j'} phi_{K,j'}(x).
 * P: device [sum n_alb^2], per element n_alb x n_alb column-major.
 * rho: device [sum N_E]. */
int32_t dgdft_alb_density(dgdft_alb* h, const double* albs, const double* P, double* rho,
                          void* stream);

/* Kleinman-Bylander term of the DG Hamiltonian for one element and itself
 * (Sec. II.A, Eq. DGHamiltonian, second bracket with K = K'):
 *   H_K[j][j'] = sum_p gamma_p <phi_{K,j}, b_p> <b_p, phi_{K,j'}>,
 * inner products = dV sums over the element box on the element's uniform
 * grid, projectors of the loaded potential.  Coupling to neighbouring
 * elements is not formed.  out: device [sum n_alb^2], column-major. */
int32_t dgdft_alb_nonlocal_block(dgdft_alb* h, const double* albs, double* out, void* stream);

/* Volume terms of the diagonal DG block of every element (Sec. II.A,
 * Eq. DGHamiltonian, first bracket; Sec. III, construction of the DG
 * Hamiltonian):
 *   A_K[j][j'] = 1/2 <grad phi_{K,j}, grad phi_{K,j'}>_E + <phi_{K,j}, V phi_{K,j'}>_E
 * as Gauss quadratures on the element's Legendre-Gauss-Lobatto grid with
 * lgl_ratio * (hi_d - lo_d) points along axis d (the paper uses twice the
 * uniform grid, lgl_ratio = 2) and gradients by LGL differentiation matrices.
 * E_K along axis d is [lo_d h_d, hi_d h_d], grid point i at i h_d.  The ALBs
 * are sampled on the LGL grid as phi = psi T: psi, the eigenvectors of the
 * extended element, evaluated by trigonometric interpolation on its periodic
 * box (an even-n Nyquist mode as a cosine), and T = dV psi_E^T phi sigma^-2
 * the map from the restricted eigenvectors to the ALBs (zero column where
 * sigma = 0).  V: the potential loaded last, interpolated likewise.
 * eigvecs, albs, sigma: device, as dgdft_alb_solve writes them (eigvecs per
 * element N_g x J column-major with dV sum psi^2 = 1; with guard columns
 * only the first J - n_guard enter, as for the ALBs).  out: device
 * [sum n_alb^2], per element n_alb x n_alb column-major.  lgl_ratio in 1..8
 * with at most 1024 points per axis, else DGDFT_EINVAL.  The library holds a
 * workspace for the largest element between calls (released by destroy). */
int32_t dgdft_alb_dg_volume(dgdft_alb* h, const double* eigvecs, const double* albs,
                            const double* sigma, int32_t lgl_ratio, double* out, void* stream);

/* Message of the last failure on h (NULL: of the last failed create). */
const char* dgdft_alb_last_error(const dgdft_alb* h);

/* Static description of a status code. */
const char* dgdft_strerror(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* DGDFT_ALB_H */
