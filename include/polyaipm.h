/*
 * polyaipm.h -- C ABI of libpolyaipm.so: Polya set-up and primal-dual
 * interior-point solver for robust stability of dx/dt = A(alpha) x on the
 * unit simplex (Kamyar, Peet & Peet, IEEE TAC 2013), on one AMD MI355X.
 *
 * Problem (Section II, Theorem 1): find a homogeneous matrix polynomial
 * P(alpha) = sum_{h in W_dp} P_h alpha^h with P(alpha) > 0 and
 * A(alpha)^T P(alpha) + P(alpha) A(alpha) < 0 on the simplex.  Polya's theorem
 * (Section II, Theorem 2) turns both into LMIs on the coefficients of
 * (sum alpha)^d1 P and (sum alpha)^d2 (A^T P + P A) (Section III-A,
 * eq. LMI_3/LMI_4), which form the block-diagonal SDP of Section III-B
 * (eq. primal/dual, C, Ai, Aij, a).  The SDP is solved by the predictor-
 * corrector primal-dual method of Section IV (Alg. 2).
 *
 * Conventions
 *  - All functions return 0 on success or a negative PSDP_E* status; no C++
 *    exception crosses this boundary.  A thread-local message describing the
 *    last error is returned by psdp_last_error().
 *  - A FEASIBLE / INFEASIBLE / UNKNOWN verdict is a result, not an error.
 *  - Host pointers are read or written only during the call; inputs are
 *    copied.  Handles are owned by the library and released by psdp_free().
 *  - Matrices are row-major FP64.  Exponent sets W_d are in the paper's
 *    descending lexicographic order (Notation section).
 *  - Device work runs on the stream given in the options (NULL = the null
 *    stream) and every call synchronises that stream before returning.
 *  - Argument validation happens before any device call, so invalid input
 *    is rejected without touching the GPU.
 */
#ifndef POLYAIPM_H
#define POLYAIPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define PSDP_OK         0
#define PSDP_EINVAL    -1   /* NULL pointer, bad dimension, non-finite input   */
#define PSDP_EOVERFLOW -2   /* a multinomial exceeds int64, or sizes overflow  */
#define PSDP_ENOMEM    -3   /* host or device allocation failed                */
#define PSDP_EDEVICE   -4   /* a HIP runtime call failed                       */
#define PSDP_ENUMERIC  -5   /* unrecoverable numerical failure                 */

/* verdicts */
#define PSDP_FEASIBLE   0   /* certificate found and checked by FP64 block Cholesky */
#define PSDP_INFEASIBLE 1   /* no certificate exists at this (dp, d1, d2)           */
#define PSDP_UNKNOWN    2

/* exit reasons of the paper's SDP run (psdp_result.reason) */
#define PSDP_R_CONVERGED 0
#define PSDP_R_FARKAS    1
#define PSDP_R_STALL     2
#define PSDP_R_MAXITER   3
#define PSDP_R_LADDER    4
#define PSDP_R_CHOL      5
#define PSDP_R_NONFINITE 6

/* verdict pipelines */
#define PSDP_VERDICT_PAPER_THEN_PHASE1 0
#define PSDP_VERDICT_PAPER_ONLY        1
#define PSDP_VERDICT_PHASE1_ONLY       2

/* arithmetic of the Schur complement assembly (the Cholesky is FP64 always).
 * FP32 / BF16: the block products are rounded to FP32 / BF16 (BF16 through
 * FP32, nearest-even) and multiplied on MFMA with FP32 accumulation; every
 * Newton solve is refined against the FP64 matrix-free Schur product, and a
 * system falls back to FP64 assembly when the refinement stops converging
 * (see ir_eta_max). */
#define PSDP_PREC_FP64 0
#define PSDP_PREC_FP32 1
#define PSDP_PREC_BF16 2

/* stopping tests of the paper's SDP run (psdp_opts.stop_rule).
 * RELATIVE: |psi - phi| / max(|psi|, |phi|) <= gap_tol and relative primal and
 * dual residuals <= feas_tol.  ABSOLUTE: the printed test of Section IV-A,
 * |a^T y - tr(C X)| <= gap_tol alone, with no feasibility test. */
#define PSDP_STOP_RELATIVE 0
#define PSDP_STOP_ABSOLUTE 1

/* centring parameter of the corrector (psdp_opts.sigma_rule).
 * FIXED: mu = sigma tr(ZX) / m.  MEHROTRA: sigma = (mu_aff / mu)^3 clipped to
 * [0, 1], where mu_aff = tr((Z + t_d dZ^)(X + t_p dX^)) / m uses the step
 * lengths the ladder gives the predictor directions (the fixed sigma stays
 * when either ladder finds no step). */
#define PSDP_SIGMA_FIXED    0
#define PSDP_SIGMA_MEHROTRA 1

typedef struct psdp_sdp psdp_sdp;  /* opaque handle: one structured SDP */

/* stability notion (psdp_setup_opts.form).
 * CONTINUOUS: x' = A(alpha) x, the Lyapunov LMIs of Theorem 1 (Section III).
 * DISCRETE:   x+ = A(alpha) x, as an instance of the generalized LMI of
 *   Section III-C: P(alpha) > 0 and [[P, P A], [A^T P, P]] > 0 (equivalent
 *   to A^T P A - P < 0).  Every block of the SDP has order 2n: the Polya
 *   coefficient for gamma in W_{dp+da+d2} is
 *   [[b P_h, P_h H], [H^T P_h, b P_h]] summed over h, with
 *   b_{h,gamma} = (da+d2)!/(gamma-h)! and H_{h,gamma} as in the continuous
 *   set-up; the P-blocks hold blockdiag(beta P, beta P).  y, K and the
 *   objective are unchanged (P_h stays n x n). */
#define PSDP_FORM_CONTINUOUS 0
#define PSDP_FORM_DISCRETE   1

typedef struct {
    int    da;            /* degree of A(alpha); 1 = affine, A holds the l vertices  */
    int    d1, d2;        /* Polya exponents; -1 = take d from psdp_polya_setup      */
    double delta;         /* P-block margin: C_j = delta * s_j * I   (eq. Cj; 1e-3)   */
    double eps;           /* derivative-block margin eps * s_j * I (1e-3)            */
    int    paper_literal; /* 1: derivative blocks of C are 0 as printed (eq. Cj)     */
    int    a_on_device;   /* 1: the A pointer is a device address                    */
    int    form;          /* PSDP_FORM_* (CONTINUOUS)                                 */
} psdp_setup_opts;

typedef struct {
    int n, l, da, dp, d1, d2;
    int L0;               /* card W_dp            (eq. L0) */
    int L;                /* card W_{dp+d1}       (eq. L)  */
    int M;                /* card W_{dp+da+d2}    (eq. M)  */
    int Na;               /* card W_da                      */
    int Nt;               /* n (n+1) / 2                    */
    int64_t K;            /* L0 * Nt              (eq. K)  */
    int64_t Kpad;         /* K rounded up to the Schur tile */
    int64_t device_bytes; /* device memory one solve of this SDP needs */
    int form;             /* PSDP_FORM_*                    */
    int bo;               /* order of every block: n, or 2n (discrete form) */
} psdp_dims;

/* launch classes timed with HIP events when psdp_opts.prof is set */
#define PSDP_PROF_CHOLINV      0   /* block Cholesky + inverse of Z              */
#define PSDP_PROF_BT           1   /* B^T(y) (eq. AT)                            */
#define PSDP_PROF_B            2   /* B(W)                                       */
#define PSDP_PROF_PRE          3   /* Schur pre-products Z^-1 H^T, X H^T, ...    */
#define PSDP_PROF_ASSEMBLE     4   /* Schur complement assembly (eq. T2)         */
#define PSDP_PROF_CHOL_PANEL   5   /* Schur Cholesky: diagonal + panel solve     */
#define PSDP_PROF_CHOL_UPDATE  6   /* Schur Cholesky: trailing update            */
#define PSDP_PROF_TRSV         7   /* the two triangular solves                  */
#define PSDP_PROF_GEMM         8   /* block products of the directions           */
#define PSDP_PROF_LADDER       9   /* step-length ladder                         */
#define PSDP_PROF_MISC        10   /* residuals, reductions, updates             */
#define PSDP_PROF_CERT        11   /* certificate check                          */
#define PSDP_PROF_PHASE1      12   /* phase-I transforms                         */
#define PSDP_NPROF            16

typedef struct {
    double gap_tol;       /* relative duality gap tolerance (1e-8)                   */
    double feas_tol;      /* relative primal / dual residual tolerance (1e-8)        */
    int    max_iter;      /* per IPM run (100)                                       */
    double sigma;         /* centring: mu = sigma tr(ZX) / m (1/3)                   */
    double step_frac;     /* fraction of the largest PD step (0.95)                  */
    double ladder_rho;    /* ratio of the step ladder (0.9)                          */
    int    ladder_len;    /* rungs of the ladder (300)                               */
    int    verdict_mode;  /* PSDP_VERDICT_*                                          */
    int    precision;     /* PSDP_PREC_*: arithmetic of the Schur assembly           */
    int    ir_max;        /* most refinement corrections per Newton solve against   */
                          /* the matrix-free FP64 product B(Z^-1 B^T(v) X); a solve */
                          /* stops early once its residual ratio reaches 1e-14 or    */
                          /* stops falling below 1e-10. -1 = 0 for FP64, 6 for FP32 */
    void*  stream;        /* hipStream_t, NULL = null stream: the solve runs on a    */
                          /* private stream ordered after it and returns when done  */
    int    record_history;/* 1: fill psdp_result.history (host memory, caller owns)  */
    double* prof;         /* NULL, or a caller array [PSDP_NPROF][2] that receives,  */
                          /* per launch class, the summed device time (ms) and the   */
                          /* number of launches, measured with HIP events on the     */
                          /* solver stream (accumulated, not cleared)                */
    /* Warm start (NULL = cold start X = Z = I, y = 0).  Per system (array of
     * count host pointers, entries may be NULL): warm_y[s] holds K dual values
     * in the library's dual order (psdp_basis), warm_logx[s] holds L+M values
     * s_j.  The start is projected into the interior: y = warm_y,
     * Z_j = B^T(y)_j - C_j + tau_j I with tau_j = max(0, theta s_j' - lambda_min)
     * (s_j' the block scale, lambda_min by bisection on FP64 Cholesky), and
     * X_j from exp(s_j) (see warm_center; s_j = 0 without warm_logx).  The
     * warm run is the paper's SDP run only, capped at warm_iter_cap
     * iterations (0: max_iter); a warm-started system that ends without a
     * certified FEASIBLE verdict or a Farkas ray is solved again from the cold
     * start (with phase-I as usual); the result says which run it reports. */
    const double* const* warm_y;
    const double* const* warm_logx;
    int    warm_iter_cap;
    double warm_margin;   /* theta in tau_j = max(0, theta s_j' - lambda_min) (1e-6)  */
    int    warm_center;   /* 0: X_j = exp(s_j) I; 1 (default): X_j = exp(s_j) n       */
                          /* Z_j^-1 / tr(Z_j^-1), the projected Z's centred partner   */
                          /* with block trace exp(s_j) n                              */
    int    asm_path;      /* Schur assembly kernels: 1 whole (h, h') pairs per        */
                          /* workgroup (n^2 <= 128), 0 grouped 64 x 64 tiles, -1     */
                          /* (default) chosen per block order by the autotuner       */
    int    solve_path;    /* triangular solves: 1 one workgroup per system (at most  */
                          /* 32 tiles of 64), 0 by groups of 8 tiles (two launches   */
                          /* per group and sweep), -1 (default) chosen per tile      */
                          /* count by the autotuner                                  */
    int    use_graph;     /* 1 (default): each iteration's launches are captured once */
                          /* into two hipGraphs and replayed; 0: launched one by one */
    double label_gap;     /* > 0: record in psdp_result.label_y / label_logx the     */
                          /* iterate of the paper's SDP run at the first iteration    */
                          /* whose relative gap is <= label_gap (training labels of   */
                          /* the learned warm start)                                  */
    /* Failure of the FP64 Schur factorisation (Alg. 2, root step 1, assumes
     * it succeeds; near the optimum a pivot can turn non-positive by
     * rounding).  The step is then retried on Lambda + tau I with
     * tau = f max_i Lambda_ii, f = 1e-14 first and x100 per further failure
     * while f <= chol_shift_max, and both Newton solves of that step are
     * refined against the unshifted FP64 product B(Z^-1 B^T(v) X) (up to six
     * corrections; ir_max when larger).  A retried step is not counted as an
     * iteration.  Past chol_shift_max the run ends with PSDP_R_CHOL. */
    double chol_shift_max;   /* largest f (1e-6); 0 = no shift, a failure ends the run */
    double chol_shift_force; /* > 0: every factorisation starts at f = this value      */
                             /* (then x100 on failure), 0 (default) = unshifted first  */
    int    stop_rule;        /* PSDP_STOP_* (RELATIVE)                                  */
    int    sigma_rule;       /* PSDP_SIGMA_* (FIXED)                                    */
    int    chol_panels;      /* Schur Cholesky: 64-wide panels per super-panel, whose   */
                             /* trailing update is one pass of depth 64 chol_panels     */
                             /* (1..32); -1 = left-looking (one launch per tile column, */
                             /* each tile updated once); -2 = right-looking with each   */
                             /* step's panel solve folded into its update (one launch   */
                             /* per step); -3 = look-ahead right-looking (one launch    */
                             /* per step: the next column's diagonal factorisation and  */
                             /* panel solve beside the update); 0 (default) = chosen    */
                             /* per tile-count bucket by the autotuner among -1, -2,    */
                             /* -3 (below 64 tiles) and widths 4, 8 and 16              */
    int    chol_subpanels;   /* with chol_panels = w > 0: split each super-panel in     */
                             /* sub-panels of this many panels (a divisor of w); the    */
                             /* narrow updates stay inside a sub-panel and each         */
                             /* sub-panel's end brings one update of depth 64 of these  */
                             /* panels to the rest of its super-panel. 0 = none         */
} psdp_opts;

typedef struct {
    int    iter;
    double phi, psi, gap_rel, pinf, dinf, mu, tp, td;
} psdp_iter_rec;

typedef struct {
    int     verdict;        /* PSDP_FEASIBLE / INFEASIBLE / UNKNOWN                  */
    int     reason;         /* exit reason of the paper's SDP run (PSDP_R_*)         */
    double* P;              /* caller buffer [L0][n][n] or NULL: the coefficients P_h */
    double* y;              /* caller buffer [K] or NULL: the dual variable          */
    double  phi, psi;       /* primal tr(CX) and dual a^T y objectives               */
    double  gap_abs, gap_rel, pinf, dinf;
    double  margin;         /* min_j lambda_min(B^T(y)_j) / s_j (certificate check)  */
    double  margin_P, margin_D;
    int     iterations;     /* iterations of the paper's SDP run                     */
    int     phase1_used;
    int     phase1_iterations;
    double  t_star;         /* phase-I optimum (normalised margin), NaN if unused    */
    double  time_solve_s;   /* wall time of the solve call                           */
    int     iters_lowprec;  /* iterations whose Schur matrix was assembled in FP32   */
    int     ir_steps;       /* refinement steps applied to this system's solves      */
    double  ir_eta_max;     /* largest ||Omega - Lambda v0|| / ||Omega|| (inf norms) */
                            /* after the unrefined solve, over those iterations;     */
                            /* NaN if none. A ratio above 0.1, a solve that the      */
                            /* refinement cannot bring below 1e-10, or a failed      */
                            /* Cholesky of the reduced-precision matrix switches the */
                            /* system to FP64 assembly for the rest of the run       */
    int     warm_used;      /* 1: the reported run started from the warm start       */
    int     warm_fallback;  /* 1: the warm run was rejected and a cold run followed  */
    int     warm_iterations;/* iterations of the warm-started run (0 if none)        */
    double* logx;           /* caller buffer [L+M] or NULL: log(tr(X_j) / n) of the  */
                            /* final primal iterate of the paper's SDP run           */
    double* label_y;        /* caller buffers [K] and [L+M] or NULL: y and           */
    double* label_logx;     /* log(tr(X_j) / n) at the label_gap iterate             */
    int     label_iter;     /* that iteration (-1: not reached)                      */
    int     asm_path;       /* paths this system took (see psdp_opts)                */
    int     solve_path;
    psdp_iter_rec* history; /* caller buffer of history_cap records, or NULL         */
    int     history_cap;
    int     history_len;
    int     chol_shifts;    /* Newton steps (both runs) whose Schur factorisation    */
                            /* needed a diagonal shift                               */
    int     graph_replays;  /* hipGraph launches of the call: each iteration replays  */
                            /* two or three captured graphs (0: every kernel launched */
                            /* eagerly; the same count in every result of a batch)    */
    int     phase1_reason;  /* exit reason (PSDP_R_*) of the phase-I run, -1 if none  */
    int     chol_panels;    /* super-panel width the Schur Cholesky used (0: left-   */
                            /* looking, -2: panel solves folded into the updates,     */
                            /* -3: look-ahead steps)                                  */
    int     chol_subpanels; /* its sub-panel width (= chol_panels: no sub-panels)    */
    /* wall time of the solve call's phases (seconds; one batch shares them):   */
    double  time_prepare_s; /* kernel-path tuning, tables, first iterate           */
    double  time_warm_s;    /* warm-start projection (0 without a warm start)     */
    double  time_paper_s;   /* the paper's SDP run (Alg. 2)                       */
    double  time_phase1_s;  /* the phase-I margin SDP run (0 if no system used it)*/
    double  time_cert_s;    /* certificate checks and the extraction of P and y   */
} psdp_result;

/* Defaults for the option structs. */
void psdp_setup_opts_default(psdp_setup_opts* o);
void psdp_opts_default(psdp_opts* o);

/*
 * psdp_polya_setup -- Section III, Alg. 1 (set-up): from the coefficients of
 * A(alpha) build the structured SDP.  Computes on the device, exactly:
 *   beta_{h,g} = d1! / (g-h)!            (closed form of eq. beta_init/beta)
 *   c[h][g][lam] = d2! / (g-h-lam)!      (closed form of eq. H_init/H)
 *   H_{h,g} = sum_lam c[h][g][lam] A_lam (FP64, ascending lam, no contraction)
 *   s_j, the multinomial block scales, and C_j (eq. C, Cj).
 * A: [Na][n][n] row-major FP64, Na = card W_da (da = 1: the l vertices).
 * n in [1, 128], l >= 1, dp >= 0, d >= 0.  Multinomials of degree > 20 are
 * rejected with PSDP_EOVERFLOW.  *out receives a new handle.
 */
int psdp_polya_setup(const double* A, int n, int l, int dp, int d,
                     const psdp_setup_opts* o, psdp_sdp** out);

/*
 * psdp_polya_setup_batched -- the set-up of psdp_polya_setup (Section III,
 * Alg. 1) for count systems in one call: A[i] (host or device per o, as for
 * psdp_polya_setup), n[i], l[i], dp[i], d[i] describe system i; o (or NULL)
 * applies to all.  One device allocation holds every system's set-up, each
 * set-up kernel is one launch over all systems and one read-back serves
 * them all, so the call costs about one set-up, not count of them.  out
 * (count handles, owned by the caller as from psdp_polya_setup) is all set
 * on success; the shared device allocation is returned when the last of the
 * count handles is freed.  On any error no handle is returned (out[i] =
 * NULL), nothing stays allocated, and the message names the failing system.
 */
int psdp_polya_setup_batched(int count, const double* const* A, const int* n, const int* l,
                             const int* dp, const int* d, const psdp_setup_opts* o,
                             psdp_sdp** out);

/* Sizes of an SDP handle (eq. L0, L, M, K). */
int psdp_query(const psdp_sdp* sdp, psdp_dims* out);

/*
 * Copies the exact set-up back to host buffers (any may be NULL):
 * beta [L0][L] int64, coef [L0][M][Na] int64, H [M][L0][n][n] FP64,
 * scale [L+M] FP64 (s_j), cdiag [L+M] FP64 (C_j = cdiag_j I).
 */
int psdp_get_polya(const psdp_sdp* sdp, int64_t* beta, int64_t* coef, double* H,
                   double* scale, double* cdiag);

/*
 * psdp_ipm_solve -- Section IV, Alg. 2: solve the SDP to the requested gap
 * and return the verdict, P coefficients and duality gap.  The solver is the
 * predictor-corrector primal-dual method started at X = Z = I, y = 0; the
 * certificate is accepted only if every block of B^T(y) passes an FP64
 * Cholesky.  On a stall the phase-I margin SDP decides the verdict.
 */
int psdp_ipm_solve(psdp_sdp* sdp, const psdp_opts* opts, psdp_result* res);

/*
 * Solves count independent SDPs together: every kernel of an iteration
 * covers all systems still running (systems may differ in n, l, dp, d).
 * res is an array of count results.  Equivalent, system by system, to
 * psdp_ipm_solve.
 */
int psdp_ipm_solve_batched(psdp_sdp* const* sdps, int count, const psdp_opts* opts,
                           psdp_result* res);

/*
 * psdp_ipm_solve_noalloc -- psdp_ipm_solve for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, same results as psdp_ipm_solve run
 * with the same kernel paths; it calls no hipMalloc, hipFree, hipHostMalloc
 * or other allocating routine.  Every table and array of the solve lives in
 * one static device array of PSDP_NOALLOC_SCRATCH_BYTES that the library
 * holds on each device it runs on until the process ends; a system whose
 * solve needs more (the Schur matrix alone is 8 Kpad^2 bytes: about K <= 3800
 * fits) is rejected with PSDP_EINVAL before any device work.  The solve runs
 * eagerly on opts->stream (no private stream, no graphs, no autotuner: the
 * kernel paths are opts->asm_path / solve_path, -1 = the defaults; the class
 * profiler is off) and synchronises it before returning.  The array keeps
 * the last call's contents; each call initialises everything it reads.
 * Calls that overlap on one device race for the array and must not be made.
 */
#define PSDP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int psdp_ipm_solve_noalloc(psdp_sdp* sdp, const psdp_opts* opts, psdp_result* res);

/*
 * Hot-path evaluation at a fixed iterate, for parity checks of single steps
 * (Alg. 2, processors step 1 and root step 1).  Host buffers:
 *   X, Z: [L+M][n][n] symmetric positive definite blocks; y: [K].
 * Outputs (any may be NULL):
 *   Zi    [L+M][n][n]  block inverses Z_j^{-1}
 *   BTy   [L+M][n][n]  B^T(y)                         (eq. AT)
 *   BX    [K]          B(X)
 *   Lam   [K][K]       Schur complement Omega (eq. T2), full symmetric (built on
 *                      the device as its lower triangle and mirrored here)
 *   LamL  [K][K]       its lower Cholesky factor (upper part zero)
 *   sol   [K]          Omega^{-1} y
 * chol_panels / chol_subpanels pick the factorisation as the psdp_opts
 * fields of those names do (-1: left-looking, -2: panel solves folded into
 * the updates, -3: look-ahead steps, 1..32: super-panel width; a divisor of
 * it: sub-panel width),
 * 0 = the default width 8 without sub-panels.
 * The basis order of the dual variable is the library's (see psdp_basis).
 */
int psdp_eval_newton(psdp_sdp* sdp, const double* X, const double* Z, const double* y,
                     double* Zi, double* BTy, double* BX, double* Lam, double* LamL,
                     double* sol, int chol_panels, int chol_subpanels, void* stream);

/*
 * The Schur complement Omega (Alg. 2 eq. T2) assembled at a fixed iterate in
 * the arithmetic of a precision form (PSDP_PREC_*: FP64, or block products
 * rounded to FP32 / BF16 with FP32 accumulation), for measuring the reduced
 * forms' error.  X, Z: host [L+M][n][n] symmetric positive definite; Lam:
 * host [K][K] (full symmetric; the library's dual order, see psdp_basis).
 */
int psdp_eval_schur(psdp_sdp* sdp, const double* X, const double* Z, int precision, double* Lam,
                    void* stream);

/*
 * Step-length ladder of the line search on fixed blocks (host buffers
 * [L+M][n][n]): largest r_k = rho^k (k <= ladder_len) such that
 * V_j + (r_k / step_frac) dV_j passes Cholesky for every block j.
 * *step = 0 and *kstar = -1 when some block never passes.
 */
int psdp_eval_ladder(psdp_sdp* sdp, const double* V, const double* dV, const psdp_opts* opts,
                     double* step, int* kstar);

/*
 * Basis order of the dual variable: pairs[2*b], pairs[2*b+1] = (p, q), p <= q,
 * for b < Nt; y index k = b + Nt * h.  The order groups indices in tiles of 8
 * so that Schur tiles are contiguous.
 */
int psdp_basis(const psdp_sdp* sdp, int* pairs);

/*
 * psdp_poly_on_simplex -- the homogeneous representation of Section II and
 * the translated simplices of Section V (Examples 1 and 2).  A is given as
 * count terms A(x) = sum_t mats[t] x^exps[t] in lx variables x (any degrees
 * <= da, a constant term allowed): exps [count][lx] int, mats [count][n][n]
 * FP64 row-major.  G [lx][l] row-major maps the unit simplex onto the region
 * of interest, x = G alpha (NULL: the identity, lx = l).  out [f(l,da)][n][n]
 * receives the coefficients, on W_da in descending lexicographic order, of
 *   B(alpha) = sum_t (sum_j alpha_j)^(da - |exps[t]|) mats[t] (G alpha)^exps[t],
 * a homogeneous polynomial equal to A(G alpha) on Delta_l: the A argument
 * psdp_polya_setup takes with psdp_setup_opts.da = da.  Host memory only;
 * no device work.  EINVAL: NULL or non-positive sizes, a negative exponent,
 * a term of degree above da, non-finite input; EOVERFLOW: da > 20.
 */
int psdp_poly_on_simplex(int n, int lx, int count, const int* exps, const double* mats, int l,
                         const double* G, int da, double* out);

typedef struct {
    double t;           /* parameter value tried                                  */
    int    verdict;     /* PSDP_FEASIBLE / INFEASIBLE / UNKNOWN                   */
    int    iterations;  /* IPM iterations of that trial (paper run + phase-I)     */
    double margin;      /* certificate margin (NaN without a certificate)         */
} psdp_bisect_rec;

/*
 * psdp_bisect_simplex -- the bisection of Section V (Example 1: the largest
 * rho; Example 2: the smallest L) over regions x = G(t) alpha, alpha in the
 * unit simplex, G(t) = G0 + t G1 (both [lx][l] row-major).  For every trial t
 * the system A on the region becomes B = psdp_poly_on_simplex(A, G(t)), whose
 * Polya SDP at (dp, d) is set up and solved on the device (setup options so
 * or NULL, its da replaced by A's degree; solver options opts or NULL).  t_feas
 * is tried first; if it has no certificate, *t_cert = NaN.  Otherwise each
 * round solves `width` trial values splitting the bracket [t_cert, t_other]
 * evenly as one batch, moves t_cert to the last certified value before the
 * first trial without a certificate (FEASIBLE only: UNKNOWN counts as none)
 * and t_other to that trial, until |t_cert - t_other| <= tol.  On return
 * *t_cert is the certified end (stability is proved on its region) and
 * *t_other the other end of the final bracket.  recs (caller buffer of
 * rec_cap records, or NULL with rec_cap = 0) receives the trials in order,
 * *nrec their number.  width in [1, 64] (1: plain bisection).
 */
int psdp_bisect_simplex(int n, int lx, int count, const int* exps, const double* mats, int l,
                        const double* G0, const double* G1, int dp, int d, double t_feas,
                        double t_infeas, double tol, int width, const psdp_setup_opts* so,
                        const psdp_opts* opts, double* t_cert, double* t_other, psdp_bisect_rec* recs,
                        int rec_cap, int* nrec);

/* Release a handle (NULL is ignored).  Device memory of a batched set-up
 * is returned with the last handle of that call. */
void psdp_free(psdp_sdp* sdp);

/* Thread-local description of the last error of this thread. */
const char* psdp_last_error(void);

/* Library version string. */
const char* psdp_version(void);

/* Measurement support for callers that report a roofline (not a step of the
 * method): the attainable FP64 matrix-core rate of the current device in
 * TFLOP/s, from independent chains of v_mfma_f64_16x16x4 on register
 * operands at four waves per SIMD, the best of three timed launches on
 * `stream` (synchronised before returning).  Allocates and frees a small
 * device buffer.  EINVAL for a NULL tflops, EDEVICE on a HIP error. */
int psdp_fp64_mfma_rate(double* tflops, void* stream);

/* ---------------------------------------------------------------------------
 * Learned warm start: the network that proposes a starting point (not part of
 * the paper).  A three-layer perceptron d0 -> d1 -> d2 -> d3 with GELU
 * (x Phi(x)) on the two hidden layers, trained on the mean squared error
 * sum_b ||out_b - t_b||^2 / (2 batch) with Adam.  Products run on MFMA with
 * FP32 accumulation, their operands in FP32 or rounded to BF16
 * (precision = PSDP_PREC_FP32 / PSDP_PREC_BF16).  Parameters are one FP32
 * array [W1, b1, W2, b2, W3, b3], W_i row-major [d_i x d_{i-1}].
 * x, t and out are DEVICE pointers to row-major FP32 [batch x width];
 * every call synchronizes its stream.
 * ------------------------------------------------------------------------- */
typedef struct psdp_mlp psdp_mlp;

int psdp_mlp_create(const int* dims /*[4]*/, int precision, int max_batch, psdp_mlp** out);
int64_t psdp_mlp_param_count(const psdp_mlp* m);
/* host FP32 arrays of psdp_mlp_param_count entries; set resets Adam */
int psdp_mlp_set_params(psdp_mlp* m, const float* host);
int psdp_mlp_get_params(const psdp_mlp* m, float* host /*or NULL*/, float* grad_host /*or NULL*/);
/* out [batch x d3] */
int psdp_mlp_forward(psdp_mlp* m, const float* x, int batch, float* out, void* stream);
/* forward + backward: the gradient stays on the device (psdp_mlp_get_params
 * reads it); *loss (host, may be NULL) receives the loss */
int psdp_mlp_loss_grad(psdp_mlp* m, const float* x, const float* t, int batch, double* loss,
                       void* stream);
/* one Adam step with the last gradient (bias-corrected moments) */
int psdp_mlp_adam(psdp_mlp* m, float lr, float b1, float b2, float eps, void* stream);
void psdp_mlp_free(psdp_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* POLYAIPM_H */
