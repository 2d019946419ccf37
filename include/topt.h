/*
 * topt.h -- C ABI of the MI355X (gfx950) SIMP minimum-compliance hot path.
 *
 * Method: F. Ferrari and O. Sigmund, "A new generation 99 line Matlab code for
 * compliance Topology Optimization and its extension to 3D" (arXiv:2005.05436).
 * Equations are cited by their number in order of appearance as typeset:
 * (1) projection, (2) filter, (5) state equation, (6) SIMP, (7)-(8)
 * sensitivities, (9) projection derivative, (10)-(11) OC rule, (14) reduced
 * index set, (15) full-matrix recovery, (17) volume-preserving threshold,
 * (19) multiplier estimate.
 *
 * Conventions shared by every entry point
 *  - Pointers named d_* or documented as "device" are device addresses (e.g. a
 *    torch tensor's data_ptr()); pointers named h_* are host addresses.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    call except to_plan_create and to_plan_export only enqueues work on it and
 *    never synchronises the host.
 *  - The library allocates no device memory.  Plan data and every scratch
 *    buffer live in one caller-owned device workspace whose size
 *    to_plan_query reports.  One plan must not be used by two streams at once
 *    (its scratch buffers would race).
 *  - Numbering (0-based, y fastest):  element e = iy + nely*ix (2D),
 *    e = iy + nely*(iz + nelz*ix) (3D); node n = iy + (nely+1)*ix (2D),
 *    n = iy + (nely+1)*(iz + (nelz+1)*ix) (3D); DOF = dim*n + component.
 *    Row iy = 0 is the top edge (physical y points to smaller iy).
 *  - Field dtype: TO_F64 fields are double, TO_F32 fields are float.  The
 *    displacement u and the load f are always double.  Reductions are always
 *    accumulated in double in a fixed order (results are bitwise repeatable).
 *  - Argument errors return TO_EINVAL before anything is enqueued; HIP runtime
 *    failures return TO_EHIP; details in to_last_error() (thread-local).
 *    Data-dependent outcomes (CG not converged, Newton or bisection cap hit,
 *    non-finite values) are never errors: they are flags in the device stats.
 *  - No C++ exception ever crosses this interface.
 */
#ifndef TOPT_H
#define TOPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TO_OK = 0,
    TO_EINVAL = 1,        /* bad argument (null pointer, size, mode) */
    TO_EHIP = 2,          /* HIP runtime error */
    TO_EWORKSPACE = 3,    /* workspace too small or misaligned (256 B) */
    TO_EUNSUPPORTED = 4   /* valid request this build does not implement */
} to_status;

typedef enum { TO_F32 = 0, TO_F64 = 1 } to_dtype;

/* Passive element codes (Sec. 2: active set A, passive solid P1, void P0). */
enum { TO_ACTIVE = 0, TO_SOLID = 1, TO_VOID = 2 };

/* Mesh and material description (Sec. 3, blocks PRE.1-PRE.3 of both codes). */
typedef struct {
    int32_t dim;                 /* 2 (Q4 plane stress) or 3 (Hex8) */
    int32_t nelx, nely, nelz;    /* elements per axis; nelz ignored in 2D */
    double E0, Emin, nu;         /* solid / void Young moduli, Poisson ratio */
    double rmin;                 /* filter radius in element widths, > 0 */
    char bc;                     /* filter boundary rule: 'D' zero padding, 'N' mirror */
    const uint8_t* h_passive;    /* host, m codes TO_ACTIVE/SOLID/VOID, or NULL (all active) */
    const int32_t* h_fixed;      /* host, fixed DOFs (any order, duplicates allowed) */
    int64_t n_fixed;
} to_mesh_desc;

typedef struct to_plan to_plan;   /* opaque: host header + views into the workspace */

/* Sizes of a plan (host copy). */
typedef struct {
    int32_t dim, d, dtilde;      /* element DOFs d = 8 | 24, d~ = d(d+1)/2 */
    int64_t m, nnode, n;         /* elements, nodes, DOFs */
    int64_t n_pairs;             /* |I_r| = m d~  (eq. (14)) */
    int64_t nnz_lower;           /* non-zeros of K^(s) incl. diagonal */
    int64_t n_active, n_solid, n_void, n_free;
    int32_t filter_radius;       /* R = ceil(rmin) - 1 */
    int32_t coop_blocks;         /* blocks of the persistent kernels */
    size_t workspace_bytes;
} to_plan_info;

/* Workspace size for a mesh.  The workspace must be 256-byte aligned.
 * Returns TO_EINVAL for a bad description (dim not 2/3, non-positive sizes,
 * rmin <= 0, bc not 'D'/'N', fixed DOF out of range, more than 2^31-1 index
 * pairs). */
to_status to_plan_query(const to_mesh_desc* desc, size_t* ws_bytes);

/* Builds the plan (Sec. 3, blocks PRE.2 and PRE.5): connectivity, the reduced
 * index set I_r of eq. (14), the lower-triangular CSR pattern of K^(s) with
 * every DOF kept (row_ptr, col_idx ascending within a row), the stable
 * (row, col)-sort permutation of I_r that assembly reduces through (seg_ptr
 * delimits each slot's pairs, in ascending pair order), the element matrix
 * Ke by Gauss quadrature, the cone filter table and its weights Hs.  Uploads
 * them into `ws` on `stream` and synchronises that stream before returning.
 * The plan header is host memory owned by the library until to_plan_destroy;
 * `ws` must outlive the plan. */
to_status to_plan_create(const to_mesh_desc* desc, void* ws, size_t ws_bytes, void* stream,
                         to_plan** out);
void to_plan_destroy(to_plan* plan);
to_status to_plan_get_info(const to_plan* plan, to_plan_info* out);

/* Copies one plan array to host memory `h_dst` (synchronous on `stream`):
 *   TO_X_PAIRS   int32 [n_pairs][2]  I_r as (row, col), row >= col
 *   TO_X_PERM    int32 [n_pairs]     stable sort permutation of I_r
 *   TO_X_SEGPTR  int32 [nnz_lower+1]
 *   TO_X_ROWPTR  int32 [n+1]
 *   TO_X_COLIDX  int32 [nnz_lower]
 *   TO_X_HS      double [m]          filter weights Hs = h * 1 (eq. (2))
 *   TO_X_KE      double [d~]         lower triangle of Ke, column by column
 *   TO_X_FREE    uint8 [n]           1 = free DOF
 *   TO_X_KERNEL  double [(2R+1)^dim] cone weights h, y fastest */
enum { TO_X_PAIRS = 0, TO_X_PERM, TO_X_SEGPTR, TO_X_ROWPTR, TO_X_COLIDX, TO_X_HS, TO_X_KE,
       TO_X_FREE, TO_X_KERNEL };
to_status to_plan_export(const to_plan* plan, int what, void* h_dst, size_t dst_bytes,
                         void* stream);

/* Builds one of the arrays above on the host, without a device, with the same
 * host code to_plan_create runs (for checks on machines without a GPU).
 * TO_X_HS is device-computed: TO_EUNSUPPORTED. */
to_status to_plan_build_host(const to_mesh_desc* desc, int what, void* h_dst, size_t dst_bytes);

const char* to_status_string(to_status s);
const char* to_last_error(void);

/* ---------------------------------------------------------------------------
 * to_init_state -- the initial state of a run (Sec. 3, block PRE.6 of both
 * codes), on the device:
 *   x_e = (volfrac (m - |P0|) - |P1|) / |A| on active elements, 1 on passive
 *         solid, 0 on passive void (the mean of x over all m elements is
 *         volfrac);
 *   xphys = x;  xphys_old = 1 (every element);
 *   dv_e = 1 / (m volfrac) on active elements, 0 on passive ones (the codes'
 *         constant volume derivative, which carries the 1/volfrac scale);
 *   u = 0.
 * x: device, m values of `dtype` (required); xphys, xphys_old, dv: device, m
 * values of `dtype`, each nullable (not written); u: device double n,
 * nullable.  Returns TO_EINVAL when volfrac is outside (0, 1), the plan has no
 * active element, or the active value falls outside [0, 1]. */
to_status to_init_state(const to_plan* plan, to_dtype dtype, double volfrac, void* x, void* xphys,
                        void* xphys_old, void* dv, double* u, void* stream);

/* ---------------------------------------------------------------------------
 * to_filter -- density filter, eq. (2), and its adjoint, eq. (8) read as the
 * chain rule (the 2D code's back-filter).
 *   mode TO_FILTER_FWD:  out = (h * in) / Hs                         (s unused)
 *   mode TO_FILTER_ADJ:  out = h * (in . s / Hs)   = H^T (s . in)   (s NULL -> 1)
 *   mode TO_FILTER_ADJ2: two adjoints sharing one pass: out = h*(in.s/Hs) and
 *                        out2 = h*(in2.s/Hs)
 * in, in2, s, out, out2: device, m values of `dtype`, element order.  `out`
 * may not alias an input. */
enum { TO_FILTER_FWD = 0, TO_FILTER_ADJ = 1, TO_FILTER_ADJ2 = 2 };
to_status to_filter(const to_plan* plan, to_dtype dtype, int mode, const void* in,
                    const void* in2, const void* s, void* out, void* out2, void* stream);

/* ---------------------------------------------------------------------------
 * to_project -- physical density (block RL.1): eq. (1) projection, eq. (9)
 * derivative, eq. (17) volume-preserving threshold by Newton (ft = 3).
 *   xpre  = xtilde on active elements, 1 on passive solid, 0 on passive void;
 *   ft = 1: xphys = xpre, dprj = 1;  ft = 2: projection at the given eta;
 *   ft = 3: Newton on g(eta) = mean(prj(xpre, eta)) - target from *d_eta until
 *           |g| <= 1e-6 (at most 50 steps), target = `target`, or mean(xtilde)
 *           when target is NaN;
 *   xphys = prj(xpre, eta, beta); dprj = d prj/d x at xtilde.
 * d_eta: device double, in/out.  xphys_old: device, nullable; when given,
 * ch = |xphys - xphys_old|_2 / sqrt(m).  d_stats: device to_project_stats. */
typedef struct {
    double eta, g, ch, vol;      /* final eta, residual g, change, mean(xphys) */
    int32_t n_newton, converged; /* Newton steps; 1 if |g| <= 1e-6 */
    int32_t pad[2];
} to_project_stats;
to_status to_project(const to_plan* plan, to_dtype dtype, int ft, const void* xtilde,
                     const void* x, void* xphys, void* dprj, double beta, double* d_eta,
                     double target, const void* xphys_old, to_project_stats* d_stats,
                     void* stream);

/* ---------------------------------------------------------------------------
 * to_assemble -- K^(s) values (block RL.2, eq. (6) and (14)):
 *   E_e = Emin + xphys_e^penal (E0 - Emin);  sK[e d~ + k] = Ke[k] E_e;
 *   kval[s] = sum of sK[perm[t]] for t = seg_ptr[s] .. seg_ptr[s+1]-1, ascending.
 * xphys: device, m; kval: device, nnz_lower (CSR order of the plan). */
to_status to_assemble(const to_plan* plan, to_dtype dtype, const void* xphys, double penal,
                      void* kval, void* stream);

/* ---------------------------------------------------------------------------
 * to_solve -- K(free, free) u = f (eq. (5)) by Jacobi-preconditioned CG
 * (or the multigrid-preconditioned flexible CG, precond TO_PREC_GMG).
 * Fixed DOFs hold u = 0.  The stop test is on the 2-norm over free DOFs:
 * |f - K u| <= rtol |f|, checked on the recursive residual and confirmed on a
 * recomputed one (CG restarts from the recomputed residual otherwise).
 *   dtype TO_F64: plain FP64 PCG with the operator chosen by `op`.
 *   dtype TO_F32, precision AUTO or F64: FP64 PCG on the FP64 matrix-free
 *                 operator (moduli from the FP32 design promoted to FP64);
 *                 with op TO_OP_ASSEMBLED its Jacobi diagonal is read from the
 *                 FP32 assembled kval, with TO_OP_MATFREE it is matrix-free.
 *   dtype TO_F32, precision MIXED: mixed precision -- CG with FP32 directions, FP32 SpMV (the
 *                 FP32 assembled kval, or FP32 moduli with op TO_OP_MATFREE)
 *                 and FP32 Jacobi; the iterate u accumulates in FP64, and
 *                 each time the FP32 residual has dropped by the factor
 *                 inner_rtol since the last replacement, the residual is
 *                 recomputed in FP64 as f - K64 u (matrix-free, FP64 moduli
 *                 from the same xphys) and replaces the FP32 one (the search
 *                 direction is kept).  Convergence is judged on those FP64
 *                 residuals (also recomputed every 64 iterations).  If they
 *                 stop improving (3 replacements without halving the best),
 *                 grow, or half of maxit is spent, the solve restarts from the
 *                 best iterate with FP64 matrix-free PCG (flagged in the stats).
 *   dtype TO_F64, op TO_OP_HYBRID: FP64 PCG on the matrix-free operator with
 *                 the Jacobi diagonal read from the FP64 assembled kval.
 * kval: device, nnz_lower values of dtype (needed unless op is
 * TO_OP_MATFREE); xphys: device m values of dtype (moduli for the matrix-free
 * operator); f, u: device double n; u holds the initial guess on entry. */
enum { TO_OP_ASSEMBLED = 0, TO_OP_MATFREE = 1, TO_OP_HYBRID = 2 };
enum { TO_SOLVE_AUTO = 0, TO_SOLVE_F64 = 1, TO_SOLVE_MIXED = 2 };
typedef struct {
    double rtol;                 /* default 1e-8 */
    double inner_rtol;           /* mixed precision replacement factor, default 0.1 */
    int32_t maxit;               /* total CG iteration cap, default 200000 */
    int32_t op;                  /* TO_OP_ASSEMBLED | TO_OP_MATFREE | TO_OP_HYBRID: the FP64
                                    matrix-free operator with the Jacobi diagonal read from the
                                    assembled kval (either field dtype; the mixed scheme takes it as
                                    TO_OP_ASSEMBLED) */
    int32_t precision;           /* TO_SOLVE_AUTO or TO_SOLVE_F64: FP64 PCG (for TO_F32 fields the
                                    operator is the FP64 matrix-free one built from the FP32
                                    design, and with op TO_OP_ASSEMBLED the Jacobi diagonal is
                                    taken from the FP32 assembled kval);
                                    TO_SOLVE_MIXED: the mixed scheme (TO_F32 fields only) */
    int32_t zero_x0;             /* 1: ignore u on entry, start from 0 */
    int32_t grid_blocks;         /* 0: automatic; else blocks of the persistent solve kernel
                                    (clamped to what can be co-resident) */
    int32_t precond;             /* TO_PREC_JACOBI (default) or TO_PREC_GMG: geometric multigrid
                                    V-cycle (2D and 3D meshes; FP64 vectors and operators for
                                    either field precision; op and precision are then ignored) */
    int32_t budget;              /* TO_PREC_GMG only.  0: the host reads the device stop flag after
                                    every 8 outer iterations and stops once convergence is confirmed
                                    (synchronises the stream; not capturable).  > 0: enqueue-only --
                                    `budget` outer iterations (rounded up to a multiple of 8) are
                                    enqueued, each predicated on the device stop flag (after
                                    convergence they return at once), with no host synchronisation;
                                    capturable into a caller's graph.  If the budget ends before
                                    convergence, the stats say converged = 0 (call again from u to
                                    continue).  Ignored by the Jacobi PCG, which is enqueue-only
                                    always.  0 .. 1,000,000. */
    int32_t pad;
} to_solve_opts;
enum { TO_PREC_JACOBI = 0, TO_PREC_GMG = 1 };
typedef struct {
    double residual;             /* final true relative residual (FP64) */
    double bnorm;                /* |f_free|_2 */
    int32_t iterations;          /* CG iterations (inner + fallback) */
    int32_t outer;               /* FP64 residual replacements (mixed) */
    int32_t converged;           /* 1 if residual <= rtol */
    int32_t fallback;            /* 1 if a fallback ran: the FP64 PCG after a mixed-precision solve
                                    that stalled, or the single-sum PCG after a pipelined one whose
                                    recurrences ran away (it continues from the best iterate) */
    int32_t restarts;            /* residual-replacement restarts */
    int32_t pad;
} to_solve_stats;
to_status to_solve(const to_plan* plan, to_dtype dtype, const void* kval, const void* xphys,
                   double penal, const double* f, double* u, const to_solve_opts* h_opts,
                   to_solve_stats* d_stats, void* stream);

/* ---------------------------------------------------------------------------
 * to_sensitivity -- eq. (7): dc_e = -penal (E0 - Emin) xphys_e^(penal-1)
 * u_e^T Ke u_e on active elements, 0 on passive ones; and the compliance
 * c = f^T u written to d_compliance (device double).  f may be NULL (then c
 * is not written). */
to_status to_sensitivity(const to_plan* plan, to_dtype dtype, const void* xphys,
                         const double* u, const double* f, double penal, void* dc,
                         double* d_compliance, void* stream);

/* to_sensitivity_noalloc -- to_sensitivity for callers that cannot allocate
 * device memory or take part in allocation at all (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, kernels and results (bit-identical) as to_sensitivity; the
 * compliance sum's scratch (at most 1024 FP64 block partials and 832 arrival
 * counters, 11.3 KiB) lives in a file-scope device array of the library, one
 * per device, held until the process ends, instead of the plan workspace.
 * Allocates nothing (no hipMalloc, no library allocation).  The counters are
 * cleared by a small kernel at the start of every call with f and
 * d_compliance given.  Calls on one device share that array: two such calls
 * that overlap in time on one device (different streams, or threads) race and
 * give wrong compliance values; serialise them.  Returns TO_EINVAL for bad
 * arguments, or if a launch would need more block partials than the array
 * holds (no mesh does: the launch clamps its grid); TO_EHIP if the device
 * address of the array cannot be obtained. */
to_status to_sensitivity_noalloc(const to_plan* plan, to_dtype dtype, const void* xphys,
                                 const double* u, const double* f, double penal, void* dc,
                                 double* d_compliance, void* stream);

/* ---------------------------------------------------------------------------
 * to_oc_update -- OC rule eq. (10)-(11) with bisection on sqrt(lambda) over
 * [0, sqrt(lambda#)] of eq. (19) (block RL.4 of the 2D code):
 *   ocP = x sqrt(max(0, -dc/dv)) on active elements;
 *   l1 = 0, l2 = mean_active(ocP)/volfrac;
 *   while (l2-l1)/(l2+l1) > 1e-4 (at most 200 steps):
 *       lmid = (l1+l2)/2; x_act = clamp(ocP/lmid, max(0, x-move), min(1, x+move));
 *       mean_all(x) > volfrac ? l1 = lmid : l2 = lmid.
 * The volume sums are double-double, so the decisions match an exactly
 * rounded sum.  The GPU evaluates 15 bisection candidates per pass (the next
 * four levels of the bisection tree) and follows the same decision path.
 * x: device, m, in/out; dc, dv: device, m (already back-filtered). */
typedef struct {
    double lmid, l1, l2, vol;    /* last midpoint, final bracket, final mean(x) */
    int32_t n_bs, capped;        /* bisection steps, 1 if the 200 cap was hit */
    int32_t passes, pad;         /* device passes over the design */
} to_oc_stats;
to_status to_oc_update(const to_plan* plan, to_dtype dtype, void* x, const void* dc,
                       const void* dv, double volfrac, double move, to_oc_stats* d_stats,
                       void* stream);

/* ---------------------------------------------------------------------------
 * to_oc_update_pd -- the OC update with the explicit primal-dual iteration
 * for lm = sqrt(lambda) (Appendix A, the primal and dual maps and the code
 * given with them) instead of bisection.  On the active set, with
 * xU' = min(x + move, 1), xL' = max(x - move, 0), ocP = x sqrt(max(0, -dc/dv)):
 *   lm = mean(ocP) / volfrac; repeat while |lm - lm_old| > 1e-10 (cap 200):
 *     tmp = ocP / lm; U = {tmp > xU'}, L = {tmp < xL'}, M = {xL' < tmp < xU'}
 *     (tmp exactly on a bound with xL' < xU' is in no set; xL' = xU' = tmp is
 *     in M); lm = sum_M ocP / (volfrac m - sum_passive x - sum_U xU' - sum_L xL');
 *   x = clip(ocP / lm, xL', xU').
 * The constraint is the mean of the design over all m elements (the volume of
 * x: volume-preserving for the density filter alone).  A non-positive
 * denominator stops the iteration, and a multiplier that is not positive and
 * finite leaves x unchanged; both set capped.  Stats: lmid = l2 = lm, l1 = the
 * previous lm, vol = the design volume of the last pass, n_bs = passes =
 * iterations.  Arguments as to_oc_update. */
to_status to_oc_update_pd(const to_plan* plan, to_dtype dtype, void* x, const void* dc,
                          const void* dv, double volfrac, double move, to_oc_stats* d_stats,
                          void* stream);

/* ---------------------------------------------------------------------------
 * to_oc_update_filtered -- the bisection of to_oc_update with the volume test
 * taken on the physical field of each candidate (Sec. 3.2, the code given for
 * a fixed threshold): xf = forward filter of the candidate (eq. (2), the
 * plan's boundary rule); xf = 1 / 0 on passive solid / void elements; for
 * ft > 1, xf = prj(xf, eta, beta) (eq. (1)); l1 = lmid if mean(xf) > volfrac
 * else l2 = lmid.  Same bracket and stop test as to_oc_update; at most 48
 * steps (capped is set when the cap ends the loop).  d_eta: device double
 * (read for ft > 1, may be NULL for ft = 1).  Every step costs one filter
 * application; the steps are enqueued without host synchronisation and the
 * ones after the stop return at once.  Uses the plan's scratch vectors (as
 * to_solve does).  Stats as to_oc_update (passes = n_bs). */
to_status to_oc_update_filtered(const to_plan* plan, to_dtype dtype, int ft, void* x,
                                const void* dc, const void* dv, double volfrac, double move,
                                double beta, const double* d_eta, to_oc_stats* d_stats,
                                void* stream);

/* ---------------------------------------------------------------------------
 * to_step -- one redesign iteration (blocks RL.1-RL.4): filter, projection,
 * change, assembly, solve, sensitivities + compliance, back-filter of dc and
 * dV, OC, then parameter continuation.  All buffers are device memory of
 * `dtype` unless noted; the caller allocates them (m or n entries).  The
 * host-side fields of to_step_state (penal, beta, loop) are updated. */
typedef struct {
    int32_t istart, isteps;      /* continuation starts at loop istart, every isteps */
    double maxpar, delta;        /* up to maxpar, by +delta (mul = 0) or *delta (mul = 1) */
    int32_t mul, enabled;
} to_sched;
enum { TO_OC_BISECT = 0, TO_OC_PD = 1, TO_OC_FILTERED = 2 };
typedef struct {
    double volfrac, move;
    int32_t ft;                  /* 1, 2 or 3 */
    int32_t oc;                  /* TO_OC_BISECT (to_oc_update), TO_OC_PD (to_oc_update_pd) or
                                    TO_OC_FILTERED (to_oc_update_filtered with the state's beta and eta) */
    double target;               /* Newton target; NaN -> volfrac (the codes' choice) */
    to_sched penal_sched, beta_sched;
    to_solve_opts solve;
} to_step_params;
typedef struct {
    void *x, *xtilde, *xphys, *xphys_old, *dprj, *dc, *dcf, *dv, *dv0, *kval;
    double* u;                   /* n, warm start in / solution out */
    const double* f;             /* n */
    double* eta;                 /* device scalar */
    double* compliance;          /* device scalar */
    to_project_stats* pstats;    /* device */
    to_solve_stats* sstats;      /* device */
    to_oc_stats* ostats;         /* device */
    double penal, beta;          /* host: current continuation parameters */
    int32_t loop;                /* host: iterations done */
    int32_t pad;
} to_step_state;
to_status to_step(const to_plan* plan, to_dtype dtype, to_step_state* h_state,
                  const to_step_params* h_params, void* stream);

/* Continuation rule of Sec. 3 (host scalar): par grows by delta (or times
 * delta) after iteration `loop` when loop >= istart, par < maxpar and
 * loop % isteps == 0. */
double to_continuation(double par, const to_sched* sched, int32_t loop);

/* ---------------------------------------------------------------------------
 * Learned warm start of the state solve (2D and 3D meshes).  The paper has no
 * network; the prediction only seeds the PCG of eq. (5), whose own true
 * residual still decides convergence.
 *
 * to_warm_start -- the minimiser of the energy 1/2 u.K u - f.u of eq. (5)
 * over span{uhat, uprev} (K: the free-DOF stiffness built from xphys and
 * penal by eq. (6), applied matrix-free in FP64).  Writes u (n, device FP64;
 * may alias uprev; zero on fixed DOFs) and, if d_coef is not NULL, the device
 * doubles (a, b, energy, case) with u = a uhat + b uprev; case 3 = both
 * vectors, 1 or 2 = the better one-vector fit (singular 2x2 system), 0 = both
 * vectors zero (u = 0).  uhat, uprev: device FP64, n. */
to_status to_warm_start(const to_plan* plan, to_dtype dtype, const void* xphys, double penal,
                        const double* f, const double* uhat, const double* uprev, double* u,
                        double* d_coef, void* stream);

/* The network: a U-Net on the node grid, bfloat16 weights and activations on
 * the matrix cores with FP32 accumulation, 15 layers of 3x3 (3D: 3x3x3)
 * convolutions, leaky ReLU of slope 1/8, 2x2 (2x2x2) average pooling,
 * nearest upsampling, additive skips, 4 levels.  2D: image rows ix, columns
 * iy (padded to multiples of 8), inputs (mean filtered density around the
 * node, f_x, f_y), outputs the two displacement components divided by the
 * RMS of u; channels 16, 32, 64, 128 (293,922 parameters).  3D: image planes
 * ix, rows iz, columns iy, inputs (density, f_x, f_y, f_z), three outputs;
 * channels 8, 16, 32, 64 (221,267 parameters).  Parameters: an FP32 vector
 * of to_nn_query's n_params entries, per layer W[t][co][ci] (2D: t = 3 (dr +
 * 1) + (dc + 1) for the offset (dr, dc) in (row, column); 3D: t = 9 (dp + 1)
 * + 3 (dr + 1) + (dc + 1) for (plane, row, column)) then b[co]; layers in the
 * order e1a e1b e2a e2b e3a e3b ba bb d3a d3b d2a d2b d1a d1b out.
 *
 * to_nn_query: workspace bytes for a mesh (dim 2 or 3; nelz ignored in 2D),
 *   and the parameter count.
 * to_nn_create: binds a plan (mesh size, free mask) and a caller-owned
 *   device workspace (256-byte aligned) of to_nn_query's size.
 * to_nn_set_params: copies device FP32 parameters in, clears the Adam moments.
 * to_nn_forward: xtilde (m, dtype) and f (n, FP64) -> uhat (n, FP64, zero on
 *   fixed DOFs; may be NULL to keep the output image only).
 * to_nn_backward: after to_nn_forward on the same sample, the mean squared
 *   error against u / rms(u) over the real nodes (device double d_loss, may
 *   be NULL) and the gradient of every parameter.
 * to_nn_adam: one Adam step (bias-corrected) with the last gradient.
 * to_nn_train_step: forward, backward and Adam (0.9, 0.999, 1e-8) on one sample.
 * to_nn_get: copies to device memory `out` the parameters or the gradient
 *   (n_params floats), the output image (pixels x 16 floats), the bfloat16
 *   output of layer i < 14 (TO_NN_ACT + i: pixels_l x c_out padded to 16,
 *   raw 16-bit values; level l images are 2^l times smaller along each axis)
 *   or, for the three layers with a skip, the activation before the skip is
 *   added (TO_NN_PRESKIP + i).
 * Every sum of the backward pass (weight and bias gradients, the loss and
 * the target scale) is taken in a fixed order: training is bitwise
 * repeatable. */
typedef struct to_nn to_nn;
enum { TO_NN_PARAMS = 0, TO_NN_GRAD = 1, TO_NN_OUTPUT = 2, TO_NN_ACT = 16, TO_NN_PRESKIP = 32 };
to_status to_nn_query(int32_t dim, int32_t nelx, int32_t nely, int32_t nelz, size_t* ws_bytes,
                      int64_t* n_params);
to_status to_nn_create(const to_plan* plan, void* ws, size_t ws_bytes, to_nn** out);
void to_nn_destroy(to_nn* nn);
to_status to_nn_set_params(to_nn* nn, const float* params, void* stream);
to_status to_nn_get(const to_nn* nn, int what, void* out, void* stream);
to_status to_nn_forward(to_nn* nn, to_dtype dtype, const void* xtilde, const double* f, double* uhat,
                        void* stream);
to_status to_nn_backward(to_nn* nn, const double* u, double* d_loss, void* stream);
to_status to_nn_adam(to_nn* nn, float lr, float beta1, float beta2, float eps, void* stream);
to_status to_nn_train_step(to_nn* nn, to_dtype dtype, const void* xtilde, const double* f,
                           const double* u, float lr, double* d_loss, void* stream);

/* ---------------------------------------------------------------------------
 * Launch-shape autotuning.  to_plan_autotune times, on the plan's own arrays,
 * the candidate shapes of the 2D filter kernel (output columns per tile 4 or
 * 8; waves per block automatic or equal to the columns; for FP32 also the
 * four tiles of the matrix-core variant, which computes the same sums with
 * v_mfma_f32_16x16x4_f32 and falls back to the stencil kernel where its tile
 * does not fit in LDS) and of the assembly
 * kernel (either form, 128, 256 or 512 threads per block; only when kval, a device buffer
 * of nnz_lower entries of `dtype`, is given) and keeps the fastest in the
 * plan (the waves per block separately for the one-field and the fused
 * two-field filter).  It synchronises `stream` and overwrites the plan's scratch arrays
 * (moduli, filter staging) and kval.  Every shape computes the same
 * quantities (the filter sums taps in a shape-dependent order).
 * to_plan_set_tuning / to_plan_get_tuning force or read the shapes. */
typedef struct {
    int32_t filt_v;              /* 4 or 8 */
    int32_t filt_parts;          /* waves per block, one field: 0 (automatic) .. 16 */
    int32_t asm_block;           /* 128, 256 or 512 */
    int32_t tuned;               /* 1 once autotuned */
    int32_t filt_parts2;         /* waves per block, fused double adjoint: 0 .. 16 */
    int32_t filt_mfma;           /* 2D FP32 filter on the matrix cores, one field: 0 off, 1..4 the tile
                                    (1: 32 x 64, 2: 16 x 64, 3: 32 x 32, 4: 16 x 32 outputs) */
    int32_t filt_mfma2;          /* the same for the fused double adjoint */
    int32_t coop_launch;         /* projection and OC kernels (their blocks meet at grid barriers):
                                    0 = plain launch with a grid that fits the device at once (default;
                                    the waits are bounded, a block that never arrives turns into a
                                    barrier-timeout error), 1 = the runtime's cooperative launch (about
                                    17 us more per launch; residency guaranteed also when other
                                    streams run kernels on the device at the same time) */
    int32_t asm_rows;            /* assembly kernel: 0 = segmented sum over the permutation of I_r,
                                    1 = one thread per slot, the row from row_ptr and the contributing
                                    elements from the grid, 2 = (2D) one thread per node, its two rows
                                    from the moduli of the elements around it (3D meshes take 0); the
                                    same terms in the same order: identical values */
} to_tuning;
to_status to_plan_autotune(to_plan* plan, to_dtype dtype, void* kval, to_tuning* h_out, void* stream);
to_status to_plan_set_tuning(to_plan* plan, const to_tuning* h_tuning);
to_status to_plan_get_tuning(const to_plan* plan, to_tuning* h_out);

/* ---------------------------------------------------------------------------
 * Batches: many independent designs of different sizes advanced together
 * by one redesign iteration each (the iteration of to_step for every design).
 * The projection (with its threshold Newton), the PCG state solve and the OC
 * bisection each run as ONE cooperative launch for the whole batch, its
 * blocks split into per-design groups in proportion to the design sizes; the
 * moduli, the 2D assembly and the sensitivities are one ordinary launch each
 * with per-design block groups, and each 2D filter pass is one launch over
 * the tiles of every design (3D designs filter and assemble per design; a
 * multigrid solve runs per design on side streams).  With
 * use_graph the iteration is captured into a HIP graph on first use and
 * replayed while every design's (penal, beta, volfrac, move, target, ft)
 * stay the same; any change recaptures it.
 *
 * to_batch_query: device workspace bytes for `count` designs.
 * to_batch_create: plans[count], one to_step_state and one to_step_params per
 *   design (the state buffers are bound to the batch: to_step_batched must get
 *   the same device pointers; ft and the solve options are fixed and must be
 *   equal for all designs, and all designs 2D or all 3D).  autotune != 0 runs
 *   to_plan_autotune on every plan not yet tuned (synchronising).  The
 *   workspace is caller-owned device memory (256-byte aligned).  Returns
 *   TO_EUNSUPPORTED when there are more designs than blocks that can be
 *   co-resident for a stage.
 * to_step_batched: one iteration of every design on `stream`; updates each
 *   state's host fields (loop, penal, beta) as to_step does.
 * to_batch_get_info: int32[8] = designs, blocks of the projection, solve and
 *   OC launches, graph captures, graph launches, blocks of the moduli /
 *   assembly / sensitivity launches, and 1 if each 2D stencil pass is one
 *   launch for the whole batch (0: one launch per design, as for 3D designs
 *   or when the largest radius's tile does not fit the LDS). */
typedef struct to_batch to_batch;
to_status to_batch_query(int32_t count, size_t* ws_bytes);
to_status to_batch_create(to_plan* const* plans, int32_t count, to_dtype dtype, const to_step_state* states,
                          const to_step_params* params, int32_t autotune, void* ws, size_t ws_bytes,
                          void* stream, to_batch** out);
to_status to_step_batched(to_batch* batch, to_step_state* states, const to_step_params* params,
                          int32_t use_graph, void* stream);
to_status to_batch_get_info(const to_batch* batch, int32_t* h_out);
void to_batch_destroy(to_batch* batch);

/* ---------------------------------------------------------------------------
 * to_pae_step -- periodic Anderson extrapolation of the OC iteration (Section
 * 3.3, eq. (20)-(23), following the code given there).  Call after the OC
 * update of iteration `loop` with x = the design after it (device, m, in/out)
 * and x_pre = the design before it (device, m).  For it = loop - q0 >= 0:
 * r = x - x_pre on active elements; mix = xi if it % q == 0 else alpha; from
 * it = 2 on the history column (it - 1) % mr receives x_pre - x_pre_old and
 * r - r_old; when it > 1 and (it - 1) % q == 0, gamma solves
 * R^T R gamma = R^T r (Gaussian elimination with partial pivoting; a zero
 * pivot sets that coefficient to 0) over the min(it, mr) columns and
 * dp = (X + mix R) gamma, else dp = 0; x = clip(x_pre + mix r - dp, 0, 1) on
 * active elements.  Before q0 nothing is done.  ws: caller-owned device
 * memory of to_pae_query bytes holding the FP64 history; it must be zeroed
 * before the first call of a run and kept between calls.  d_gamma (nullable):
 * device doubles receiving the coefficients.  mr <= 8, q >= 1. */
typedef struct {
    int32_t mr, q, q0, pad;
    double alpha, xi;
} to_pae_params;
to_status to_pae_query(const to_plan* plan, const to_pae_params* h_params, size_t* ws_bytes);
to_status to_pae_step(const to_plan* plan, to_dtype dtype, void* x, const void* x_pre, int32_t loop,
                      const to_pae_params* h_params, void* ws, double* d_gamma, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TOPT_H */
