/*
 * feasthip -- non-Hermitian FEAST (Kestyn, Polizzi, Tang, "FEAST eigensolver
 * for non-Hermitian problems") on AMD MI355X (gfx950).
 *
 * C ABI.  No torch or HIP types appear in the signatures: device buffers are
 * plain pointers, the stream is an opaque pointer (a hipStream_t).
 *
 * Conventions shared by every call
 * --------------------------------
 * complex numbers  interleaved (re, im) pairs of double (complex128) unless a
 *                  call says otherwise; a "complex array of length k" is 2k
 *                  doubles.
 * block vectors    Y, Yh, Q, Qh, X ...: n x m0 complex, ROW-major: entry
 *                  (i, k) at offset i*ld + k, ld >= m0 (ld = m0 when not given).
 * dense matrices   n x n complex, ROW-major with leading dimension ld.
 * CSR matrices     0-based int32 row pointers (n+1) and column indices (nnz),
 *                  column indices sorted within each row; values real (FH_R64)
 *                  or complex (FH_C128).
 * ownership        every buffer passed in belongs to the caller and is never
 *                  freed by the library; input matrices are never modified.
 *                  Workspace (device memory) lives in the handle and in
 *                  prepared problems and is freed in fh_destroy /
 *                  fh_problem_destroy; it comes from the allocator given to
 *                  fh_create (see fh_allocator), else from hipMalloc.
 * streams          all GPU work of a handle runs on the handle's stream; calls
 *                  return after that work has completed.  A handle is not
 *                  thread-safe.
 * return codes     0 success; -k argument k invalid (1-based, LAPACK style);
 *                  positive codes below; fh_last_error() gives a message.
 */
#ifndef FEASTHIP_H
#define FEASTHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define FH_OK                0
#define FH_NO_EIG_INSIDE     1   /* no Ritz value inside the contour after max_iter  */
#define FH_NOT_CONVERGED     2   /* max_iter reached; best pairs and res are filled   */
#define FH_M0_TOO_SMALL      3   /* max_iter reached with all m0 Ritz values inside
                                    the contour: m0 is probably not above m        */
#define FH_SINGULAR_SHIFT    4   /* zero pivot / breakdown at a node (bad_node = j)   */
#define FH_INNER_FAILED      5   /* an iterative inner solve missed its tolerance     */
#define FH_NONFINITE         6   /* non-finite input or state                          */
#define FH_EIG_FAILED        7   /* reduced eigenproblem (QR iteration) did not converge */
#define FH_HIP_ERROR       100   /* HIP runtime error or out of memory                 */

enum { FH_DENSE = 0, FH_CSR = 1 };
enum { FH_R64 = 0, FH_C128 = 1 };
enum { FH_PREC_FP64 = 0, FH_PREC_MIXED = 1 };        /* solve precision            */
enum { FH_SOLVER_LU = 0, FH_SOLVER_BGMRES = 1 };      /* shifted-system solver      */
enum { FH_PC_NONE = 0, FH_PC_JACOBI = 1, FH_PC_ILU0 = 2, FH_PC_LEARNED = 3 };

/* most constant input fields a learned preconditioner takes */
enum { FH_NET_MAX_FIELDS = 11 };

typedef struct fh_ctx*  fh_handle;
typedef struct fh_prob* fh_problem;
typedef struct fh_net_s* fh_net;

/* A matrix operand; all pointers are DEVICE pointers owned by the caller. */
typedef struct {
    int kind;             /* FH_DENSE or FH_CSR                               */
    int dtype;            /* FH_R64 (CSR only) or FH_C128                     */
    int n;                /* order                                            */
    int ld;               /* dense: leading dimension (>= n)                  */
    long long nnz;        /* CSR: number of stored entries                    */
    const void* val;      /* dense: n*ld values; CSR: nnz values              */
    const int* rowptr;    /* CSR: n+1                                         */
    const int* colind;    /* CSR: nnz                                         */
} fh_mat;

/* Search contour: ellipse z(t) = c + e^{i angle} (a cos t + i ratio*a sin t).
 * Paper Section 2.1 (complex midpoint, radius, axis ratio, rotation angle).
 * Or, with nv >= 3, a polygon (the paper's custom contours, e.g. the squares
 * of its multi-contour experiment): vertices verts (host, nv complex values,
 * either orientation, not self-intersecting), ne / nv trapezoid intervals on
 * each side (ne a multiple of nv; 16 nodes = 4 per side of a square), the
 * inside test (step 5.a) point-in-polygon, alpha of eq:res |g| + max_k
 * |v_k - g| with g the mean of the vertices; c_re .. angle are then unused. */
typedef struct {
    double c_re, c_im;    /* centre lambda_mid                                */
    double a;             /* horizontal semi-axis (radius for a circle)       */
    double ratio;         /* vertical / horizontal semi-axis (1 = circle)     */
    double angle;         /* rotation in radians                              */
    int ne;               /* number of quadrature nodes                       */
    int nv;               /* polygon: number of vertices (0 = the ellipse)    */
    const double* verts;  /* polygon: nv complex vertices (re, im pairs)      */
} fh_contour;

typedef struct {
    int m0;               /* search subspace size (columns of Y)              */
    int max_iter;         /* FEAST iterations                                 */
    double eps;           /* threshold of eq:res                              */
    int precision;        /* FH_PREC_FP64 or FH_PREC_MIXED                    */
    int solver;           /* FH_SOLVER_LU (dense) or FH_SOLVER_BGMRES (CSR)   */
    int restart;          /* GMRES restart length (Krylov steps per cycle)    */
    int block;            /* reserved (0): every right-hand side carries its own
                             Krylov space, all columns advance in lockstep    */
    int precond;          /* FH_PC_*                                          */
    double inner_tol;     /* relative residual target of each inner solve     */
    int max_restarts;     /* GMRES cycles per solve (FP64) / per refinement step */
    double mixed_inner_tol; /* mixed: FP32 inner-solve target per refinement step */
    int max_refine;       /* mixed: FP64 refinement steps                     */
    int save_factors;     /* keep per-node factorizations across calls         */
    int resume;           /* fh_feast: 1 = the start columns of Y / Yh are Ritz
                             vectors whose Ritz values are passed in lambda
                             (resume from a previous call's subspace)         */
    int fallback;         /* FH_PC_LEARNED only: preconditioner that takes over
                             for the rest of a solve when a restart cycle with
                             the network cuts the worst relative residual by
                             less than half (FH_PC_NONE, _JACOBI or _ILU0)    */
    int graph;            /* dense grouped solves (fh_feast_batched, mixed dense
                             filter): 1 = capture each solve / refinement step
                             into a HIP graph once per layout and replay it   */
    int orth;             /* GMRES orthogonalization: 0 = classical Gram-Schmidt
                             with reorthogonalization (two projections),
                             1 = one projection (one pass over the basis less),
                             2 = delayed reorthogonalization (the second
                             projection of each vector shares the next step's
                             pass: two passes over the basis per step instead
                             of three); 2 applies when restart <= 31 (FP64
                             and complex-FP32 solves alike), longer cycles
                             use 0 */
    int batch_nodes;      /* sparse filter: quadrature nodes whose right and
                             left systems are solved together (their Krylov
                             bases live in device memory at once); 0 = as many
                             as fit in half of the device memory.  The filter
                             sums the chunks' contributions, so the result
                             does not depend on it beyond rounding and the
                             inner tolerances */
    int sym;              /* sparse problems: 1 = complex symmetric (A = A^T).
                             The left eigenvectors are then the conjugates of
                             the right ones, so the filter solves only the
                             n_e right systems instead of 2 n_e (paper,
                             reduced-workload cases, complex symmetric; Table
                             tab:solve) and takes for the left block
                             Qh = conj(Q) D, D = diag(conj(1 / (y_i^T y_i))):
                             the left filter of conj(Y) D, the left block
                             with yh_i^H y_i = 1 that FEAST's left Ritz
                             vectors have; Yh is not read by the filter.  The
                             call returns -2 if A is not symmetric.
                             0 = general.  Dense problems ignore it */
    int confirm;          /* exit rule.  0 (default) = the paper's steps 5.c /
                             5.d: with m_r Ritz values inside and m_s flagged
                             spurious, converged when the m = m_r - m_s
                             smallest inside residuals are below eps, and
                             exactly those m pairs are returned.  1 = a
                             stricter exit that is not in the paper: when the
                             test passes only because flagged pairs were
                             passed over, the next iteration must pass with
                             the same number of converged inside pairs, and
                             every inside pair below eps is returned.  2 =
                             the paper's exit iteration, and every inside pair
                             below eps is returned (not only the m of step
                             5.d): for runs where the number of flagged pairs
                             changes from one iteration to the next, so that
                             1 finds no confirming iteration, while the paper's
                             m = m_r - m_s leaves converged pairs out */
    int conj_pairs;       /* sparse problems with real A (FH_R64): 1 (default)
                             = when the nodes are symmetric about the real
                             axis (each lower node the conjugate of an upper
                             one, with the conjugate weight), factorize only
                             the upper and real-axis nodes and solve a lower
                             node's systems as its partner's with conjugated
                             right-hand sides (paper, reduced-workload cases,
                             real non-symmetric with a contour symmetric about
                             the real axis: n_e/2 factorizations; Table
                             tab:solve).  The solves stay 2 n_e: the start
                             block is complex.
                             2 = the same factorizations, and n_e solves
                             instead of 2 n_e (n_e/2 with sym = 1; the
                             table's n_e total solves): fh_feast drops the
                             imaginary part of the start blocks (not with
                             resume), so that in exact arithmetic every
                             search subspace is closed under conjugation; before
                             each filter it pairs the Ritz values as
                             conjugates, makes the pairs exact (x_k =
                             conj(x_i), lambda_k = conj(lambda_i), the vectors
                             of real Ritz values real: a change at rounding
                             level), and solves only the upper nodes' systems,
                             a lower node's solution being the conjugate of
                             its partner's for the partner column.  fh_filter
                             does the same when Y and Yh are real (zero
                             imaginary parts), else it behaves as with 1.
                             0 = factorize every node */
} fh_opts;

typedef struct {
    int info;             /* status code of the call                          */
    int m;                /* converged eigenpairs returned                    */
    int iters;            /* FEAST iterations performed                       */
    int m0_final;         /* subspace size after resizing                     */
    int bad_node;         /* node index for FH_SINGULAR_SHIFT / inner failure  */
    int m_s;              /* spurious Ritz values flagged in the last iteration */
    long long n_factor;   /* factorizations performed (Table tab:solve)       */
    long long n_solve;    /* m0-column shifted solves performed                */
    long long inner_steps;/* block Krylov steps (all systems) in the last filter */
    double inner_relres;  /* worst final relative residual of the last filter  */
    double t_filter_ms;   /* time of the last contour integration             */
    double t_iter_ms;     /* time of the last full FEAST iteration            */
    long long n_fallback; /* solves a fallback took over (cumulative): sparse,
                             the learned preconditioner replaced by
                             opts.fallback; dense complex FP32, systems whose
                             refinement stalled above inner_tol, solved again
                             with FP64 factors                                */
    int n_bq_retry;       /* B_Q eigendecompositions that exhausted the shifted
                             QR budget and were run again on the reversed
                             basis order (cumulative)                         */
} fh_report;

/* ---- handle -----------------------------------------------------------
 * Device-memory provider.  alloc(bytes, stream, user) returns device memory
 * of at least `bytes` bytes on the handle's device, usable in stream order on
 * `stream` (the handle's stream at the time of the request), or NULL when it
 * cannot (the call then fails with FH_HIP_ERROR).  free(ptr, bytes, stream,
 * user) gives back a block with the size and stream of its alloc; the
 * library waits for the device before it frees a block.  Blocks are requested
 * inside the library's calls (workspace grows to the largest problem seen and
 * is kept) and freed when a workspace grows, in fh_problem_destroy,
 * fh_net_destroy and fh_destroy, which may run after fh_destroy of the
 * handle that made the request: the callbacks must stay valid until the
 * last of them.  A binding can route both to its framework's caching
 * allocator (the Python binding uses torch's). */
typedef struct {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* ptr, size_t bytes, void* stream, void* user);
    void* user;
} fh_allocator;

/* h: out; device: HIP device index (-2 if out of range); hip_stream: the
 * stream every call of the handle runs on (a hipStream_t, NULL = the null
 * stream); alloc: NULL = hipMalloc / hipFree, else both callbacks must be set
 * (-4 otherwise); the struct is copied. */
int         fh_create(fh_handle* h, int device, void* hip_stream, const fh_allocator* alloc);
int         fh_destroy(fh_handle h);
int         fh_set_stream(fh_handle h, void* hip_stream);
const char* fh_last_error(fh_handle h);
void        fh_default_opts(fh_opts* o);

/* ---- contour (host, FP64) ---------------------------------------------
 * Trapezoidal nodes t_j = 2 pi (j - 1/2)/ne and weights w_j = z'(t_j)/(i ne):
 * the rational filter rho_a(z) = sum_j w_j/(z_j - z) of eq:rational
 * approximating the Cauchy integral eq:cauchy (Sections 1, 2.1, 2.3).
 * z, w: host complex arrays of length ne. */
int fh_contour_nodes(const fh_contour* c, double* z, double* w);
/* rho_a at nlam host points (eq:rational).  lam, rho: host complex arrays. */
int fh_rational(int ne, const double* z, const double* w, int nlam, const double* lam, double* rho);

/* ---- prepared problem ---------------------------------------------------
 * Holds A, B (B == NULL means B = I) and, once computed, the per-node
 * factorizations that the paper keeps across FEAST iterations (Section 4.1:
 * saving the factorizations).  Dense problems use complex LU with partial
 * pivoting; CSR problems use ILU(0) of (z_j B - A), natural ordering, as the
 * preconditioner of block GMRES.  CSR B must be NULL (identity). */
int fh_problem_create(fh_handle h, const fh_mat* A, const fh_mat* B, fh_problem* p);
int fh_problem_destroy(fh_problem p);

/* ---- contour filter (the hot path alone), eq:qr and eq:ql ---------------
 *   Q  = sum_j w_j       (z_j B - A)^{-1}  B   Y
 *   Qh = sum_j conj(w_j) (z_j B - A)^{-H}  B^H Yh
 * z, w: host complex arrays of length ne.  Y, Yh, Q, Qh: device n x m0 row-
 * major blocks (ld = m0).  One factorization per node serves both sides
 * (Section 2.4).  rep may be NULL. */
int fh_filter(fh_handle h, fh_problem p, int ne, const double* z, const double* w, int m0,
              const void* Y, const void* Yh, void* Q, void* Qh, const fh_opts* o, fh_report* rep);

/* ---- non-Hermitian FEAST (complete algorithm figure, steps 0-5) ----------
 * Y, Yh   in: start subspaces (n x m0, device, step 0); out: the m converged
 *         right / left eigenvectors in columns 0..m-1 (ld = m0), normalised
 *         so that Xh^H B X = I (step 5.d), followed by the other Ritz vectors
 *         of the final search subspace in columns m..m0_final-1 (so that the
 *         subspace can be reused as a start, see opts->resume).  When not
 *         converged (FH_NOT_CONVERGED), m = 0 and all m0_final columns hold the
 *         current Ritz vectors.
 * lambda  device complex array, length m0: Ritz values of the returned
 *         columns; the m eigenvalues first, sorted by (Re, Im).  Input when
 *         opts->resume = 1.
 * res     host array, length m0: eq:res of the returned columns (may be NULL).
 * z, w    host nodes/weights (length c->ne) or NULL to generate them from c.
 * The contour c also defines the inside test (step 5.a) and alpha of eq:res. */
int fh_feast(fh_handle h, fh_problem p, const fh_contour* c, const double* z, const double* w,
             const fh_opts* o, void* Y, void* Yh, void* lambda, double* res, fh_report* rep);

/* ---- many dense problems at once (sizes may differ) ---------------------
 * FEAST on each problem i with its own contour contours[i] and start
 * subspaces Y[i], Yh[i] (device n_i x m0, in/out exactly as in fh_feast;
 * lambda[i]: device m0; res[i]: host m0 or NULL; reports[i] optional).  The
 * contour filters of all problems run together every iteration: one
 * factorization of (z_j B_i - A_i) per (problem, node), made once for all
 * problems by grouped launches in which every launch advances every matrix
 * by one panel, then grouped 'N' and 'C' solves.  With o->precision ==
 * FH_PREC_MIXED the factors and solves are complex FP32 (GEMM updates on
 * MFMA, tile autotuned per shape class) inside FP64 iterative refinement of
 * every right-hand side (o->inner_tol, o->max_refine); otherwise FP64.
 * Steps 2-5 run per problem.  All problems must be dense; o->m0 <= every n_i;
 * nodes are generated from the contours (Section 2.4 trapezoidal rule).
 * Returns FH_OK when every problem converged, else the first other status
 * (each report holds its own). */
int fh_feast_batched(fh_handle h, int count, const fh_problem* problems, const fh_contour* contours,
                     const fh_opts* o, void* const* Y, void* const* Yh, void* const* lambda, double* const* res,
                     fh_report* reports);

/* ---- kernel timing ---------------------------------------------------------
 * fh_profile(h, 1) resets and enables per-kernel timing with HIP events on
 * the handle's stream (a small overhead per launch); fh_profile_read returns
 * entry idx (0-based; 1 when idx is past the end): kernel name, launches,
 * total milliseconds, algorithmic bytes and flops summed over launches. */
int fh_profile(fh_handle h, int enable);
int fh_profile_read(fh_handle h, int idx, char* name, int namelen, long long* count, double* ms, double* bytes,
                    double* flops);

/* ---- components (exposed for parity tests of single steps) -------------- */

/* Stochastic estimate of the number of eigenvalues inside the contour (the
 * eigenvalue-count estimator the paper's section on the FEAST v3.0 software
 * cites): the filter applied to p probe vectors, Q = sum_j w_j (z_j B - A)^{-1} B V
 * (right solves only), and est = (1/p) trace(V^H Q) = (1/p) sum_k v_k^H Q e_k,
 * which estimates trace(rho_a) = sum_i rho_a(lambda_i).  V: device n x p
 * row-major complex (the probes: the caller draws them, e.g. Rademacher or
 * Gaussian entries; V = I with p = n gives the exact trace).  1 <= p <= 256.
 * est: host double[2] (real, imaginary part).  Returns FH_OK or -k. */
int fh_count_estimate(fh_handle h, fh_problem p, int ne, const double* z, const double* w, int nprobe,
                      const void* V, const fh_opts* o, double* est, fh_report* rep);

/* Step 2.a: BQ (m x m, device, row-major) = Qh^H B Q. */
int fh_reduced_matrix(fh_handle h, fh_problem p, int m, const void* Qh, const void* Q, void* BQ);

/* Allocation-free variant of fh_reduced_matrix, for callers that cannot
 * allocate device memory during the call: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same operands and
 * result (BQ = Qh^H B Q, m x m, device, row-major); it calls no hipMalloc,
 * hipFree or allocator callback.  Its workspace (the split-K partial sums,
 * and B Q when the problem has a B matrix) is a static device array of
 * FH_NOALLOC_SCRATCH_BYTES per device, held from library load until the
 * process ends, whose device address fh_create resolves once per device.
 * Limits: m*m*16 bytes (plus n*m*16 with a B matrix) must fit in it,
 * else -3 and fh_last_error says why.  Every call on one device shares that
 * array and overwrites it (nothing in it has to start at zero); calls that
 * overlap on one device, e.g. from two streams or threads, race.  When the
 * partial sums of fh_reduced_matrix's split fit, the split and so the result
 * are the same; otherwise a coarser split changes only the summation order. */
#define FH_NOALLOC_SCRATCH_BYTES (32u << 20)
int fh_reduced_matrix_noalloc(fh_handle h, fh_problem p, int m, const void* Qh, const void* Q, void* BQ);

/* Steps 3.a-3.c on the GPU: B_Q = V Gamma Vh^H, sort by decreasing |gamma|
 * (stable), count m0t = #{|gamma_i| >= eta max|gamma|}, and return the
 * bi-orthonormalizing factors S = V[:, :m0t] Gamma^{-1/2} and
 * Sh = Vh[:, :m0t] conj(Gamma^{-1/2}) (so that U = Q S, Uh = Qh Sh; eq:uu).
 * BQ, S, Sh: device m x m row-major; gamma: device complex length m (sorted);
 * m0t: host int. */
int fh_biortho_factors(fh_handle h, int m, const void* BQ, double eta, void* gamma, void* S, void* Sh,
                       int* m0t);

/* Step 4.b on the GPU: A_U W = B_U W Lambda, A_U^H Wh = B_U^H Wh Lambda^*,
 * Wh^H B_U W = I; W has unit 2-norm columns.  All device, m x m row-major. */
int fh_reduced_eig(fh_handle h, int m, const void* AU, const void* BU, void* lambda, void* W, void* Wh);

/* Shifted operator on a batch of blocks (sparse or dense A):
 *   Out_s = shift_s X_s - A X_s       (side 0)
 *   Out_s = shift_s X_s - A^H X_s     (side 1)
 * for s = 0..nsys-1, each X_s / Out_s an n x m block (device, contiguous,
 * system-major).  shifts: host complex array of length nsys. */
int fh_shifted_apply(fh_handle h, fh_problem p, int side, int nsys, const double* shifts, int m,
                     const void* X, void* Out);

/* Training pairs of the learned preconditioner (not part of the paper's
 * method; the pairs of the residual-norm loss): for s = 0..nsys-1, with
 * M_s = shift_s I - op(A) (op = A for side 0, A^H for side 1),
 *   R_s = B_s - M_s X_s    (residual of the iterate X_s)
 *   E_s = Xt_s - X_s       (its error against the exact solution Xt_s)
 * so that M_s E_s = R_s up to rounding when B_s = M_s Xt_s.  CSR problems
 * only.  Every block is n x m (device, contiguous, system-major, complex
 * double); shifts: host complex array of length nsys.  R and E must not
 * overlap the inputs.  Returns FH_OK, or -k for an invalid argument k (-2
 * for a dense problem). */
int fh_residual_pair(fh_handle h, fh_problem p, int side, int nsys, const double* shifts, int m, const void* B,
                     const void* X, const void* Xt, void* R, void* E);

/* ILU(0) of (z B - A) for a CSR problem (natural ordering): factor values
 * aligned with A's CSR pattern (L strictly left of the diagonal, unit
 * diagonal implied; U on and right of it).  lu: device complex, nnz. */
int fh_ilu0(fh_handle h, fh_problem p, double z_re, double z_im, void* lu);

/* Preconditioner apply: Out = (LU)^{-1} X (side 0) or (LU)^{-H} X (side 1)
 * with the ILU(0) of (z B - A); X, Out: device n x m blocks. */
int fh_ilu0_apply(fh_handle h, fh_problem p, double z_re, double z_im, int side, int m,
                  const void* X, void* Out);

/* The same apply in complex FP32, as the mixed-precision Krylov solves use
 * it: the ILU(0) is computed in FP64 and its factors are rounded to FP32;
 * X, Out: device complex-FP32 (interleaved float pairs) n x m blocks.
 * Returns FH_OK, -k for an invalid argument k, FH_SINGULAR_SHIFT on a zero
 * pivot. */
int fh_ilu0_apply_c64(fh_handle h, fh_problem p, double z_re, double z_im, int side, int m,
                      const void* X, void* Out);

/* Shifted solves, the linear systems of the contour filter (Section 2.4,
 * eq:qr and eq:ql) for arbitrary shifts:
 *   sides[s] == 0:  (z_s B - A) X_s = B_s
 *   sides[s] == 1:  (z_s B - A)^H X_s = B_s
 * s = 0..nsys-1; all right systems (side 0) must come before the left ones.
 * z: host complex array of nsys shifts; B, X: device complex, nsys blocks of
 * n x m (system-major, row-major n x m each).
 * Dense problem: one LU with partial pivoting per system (FP64), direct
 * solves; only o->save_factors is read.
 * CSR problem (B = I): GMRES with m <= 256; restart, max_restarts,
 * inner_tol, precision, mixed_inner_tol, max_refine and precond come from
 * *o.  With precond == FH_PC_LEARNED the network attached by
 * fh_problem_set_net is the (nonlinear) preconditioner, the flexible
 * variant of GMRES is used and o->fallback takes over when a restart cycle
 * does not halve the worst relative residual.  rep (optional): n_factor,
 * n_solve, inner_steps (Krylov steps), inner_relres (largest final relative
 * residual), n_fallback.
 * Returns FH_OK, -k for an invalid argument k, FH_SINGULAR_SHIFT on a zero
 * pivot, or an error status with fh_last_error set. */
int fh_shifted_solve(fh_handle h, fh_problem p, int nsys, const double* z, const int* sides, int m,
                     const fh_opts* o, const void* B, void* X, fh_report* rep);

/* Learned preconditioner (not part of the paper's method: a flexible
 * preconditioner for the iterative shifted solves of Section 2.4).
 * A 3-layer convolutional network on an nz x ny x nx grid (vector index
 * i = (z * ny + y) * nx + x, so n = nz * ny * nx): 3x3 convolutions (nz = 1)
 * or 3x3x3 convolutions (nz > 1) with zero padding, cin -> 16 -> 16 -> 2
 * channels, bias, ReLU after the first two layers.
 * Input channels: Re and Im of v / ||v||_2, Re and Im of the operator shift
 * divided by alpha (z for a right system, conj(z) for a left one), the side
 * (0 or 1), then nfields constant fields.  Output:
 * e = ||v||_2 out_scale (o_0 + i o_1), an approximation of (z B - A)^{-1} v
 * (side 0) or (z B - A)^{-H} v (side 1); out_scale sets the magnitude of
 * the operator's inverse (about 1 / max |a_ii| for a stiff operator).
 * Parameters are kept in FP32 (Adam master copy) and used in BF16 by the
 * kernels, which accumulate in FP32.  Parameter vector layout (floats), with
 * T = 9 (nz = 1) or 27 taps:
 *   w1 [16][cin][T], b1 [16], w2 [16][16][T], b2 [16], w3 [2][16][T], b3 [2]
 * with cin = 5 + nfields and tap index (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
 * (dz = 0 when nz = 1), where the tap reads the input at (z+dz, y+dy, x+dx).
 *
 * fh_net_create: fields = host [nfields][n] (may be NULL if nfields is 0);
 * alpha > 0 scales the shift channels, out_scale > 0 the output; He-normal
 * initial weights drawn from seed.  The network belongs to h's device;
 * destroy it with fh_net_destroy after detaching it from every problem. */
int fh_net_create(fh_handle h, int nz, int ny, int nx, int nfields, const double* fields, double alpha,
                  double out_scale, unsigned long long seed, fh_net* net);
int fh_net_destroy(fh_net net);
/* number of floats in the parameter vector (or a negative error) */
int fh_net_param_count(fh_net net);
/* copy the FP32 parameters to / from host memory; set also resets Adam */
int fh_net_get_params(fh_handle h, fh_net net, float* params);
int fh_net_set_params(fh_handle h, fh_net net, const float* params);
/* replace the constant input fields (host [nfields][n], as at creation), e.g.
 * to train one network on the operators of several coefficient fields */
int fh_net_set_fields(fh_handle h, fh_net net, const double* fields);
/* activations of the network's inference passes (fh_net_forward and the
 * preconditioner applications inside the Krylov solves): 0 (default) = FP32,
 * each activation entering the MFMA layers as two BF16 terms (FP32-level
 * accuracy); 1 = BF16, one term (the inputs of the first two layers rounded
 * to BF16: half the operand loads and MFMA work, about 3 significant
 * digits).  Training passes always use FP32 activations.  Returns FH_OK,
 * -1 for a null net, -2 for another mode. */
int fh_net_set_activations(fh_net net, int bf16);
/* Out_s = network(V_s) for nsys blocks (device, [nsys][n][m] complex);
 * z, sides as in fh_shifted_solve. */
int fh_net_forward(fh_handle h, fh_net net, int nsys, int m, const double* z, const int* sides,
                   const void* V, void* Out);
/* One training step on (residual, error) pairs R_s, E_s (device, [nsys][n][m],
 * E_s an exact or accurate solution of M_s E_s = R_s).  With t = e / ||r||
 * and o the network's raw output (both in units of out_scale), the loss is
 * the mean over the nsys*m columns of
 *   p == NULL:   ||o - t||^2 / ||t||^2                      (error norm)
 *   p != NULL:   ||M (o - t)||^2 / ||M t||^2                (residual norm)
 * where M is the column's shifted operator of the CSR problem p (n = ny*nx,
 * m <= 256); the second form measures how close M net(r) is to r and is the
 * one that trains a useful preconditioner for stiff operators.  The gradient
 * with respect to the BF16 parameters goes to grad (host, optional,
 * param_count floats); if update != 0 one Adam step (beta 0.9 / 0.999,
 * eps 1e-8, learning rate lr) is applied to the FP32 parameters.
 * loss: host, optional. */
int fh_net_train_step(fh_handle h, fh_net net, fh_problem p, int nsys, int m, const double* z,
                      const int* sides, const void* R, const void* E, double lr, int update, double* loss,
                      float* grad);
/* attach (net != NULL) or detach (NULL) the learned preconditioner used by
 * fh_filter / fh_feast / fh_shifted_solve on a CSR problem when
 * opts.precond == FH_PC_LEARNED; the grid must have n points.  Not owned. */
int fh_problem_set_net(fh_problem p, fh_net net);

#ifdef __cplusplus
}
#endif
#endif /* FEASTHIP_H */
