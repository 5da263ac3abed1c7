/*
 * frkc2.h -- C ABI of libfrkc2, the FRKC2 superstep on AMD MI355X (gfx950).
 *
 * Method: S. O'Sullivan, "Factorized Runge-Kutta-Chebyshev Methods",
 * arXiv:1702.03818. A superstep of length T advances w' = f(w) (Sec. 1, the
 * semi-discrete system with a Jacobian whose eigenvalues lie near the
 * negative real axis) by L = s ordered forward Euler steps with complex
 * stepsizes (Sec. 3, the Euler-step equation of the FRKC2 scheme):
 *     W^0 = w^n,  W^{l+1} = W^l + T a_l f(W^l),  w^{n+1} = Re W^L.
 * The a_l come from the roots of the damped second-order FRKC stability
 * polynomial (Sec. 2 and Sec. 2.1) in the internal-stability order of
 * Sec. 2.2. f is a diffusion operator on a uniform grid, fused into the
 * GPU kernels (ops below). Everything is FP64.
 *
 * Conventions for every entry point:
 *  - Arrays are flat, x fastest: index = x + n[0]*(y + n[1]*z).
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller. The library
 *    never frees caller memory and allocates no device memory in any call
 *    except the batched graph (see frkc2_step_batched) and its own small
 *    host-side caches.
 *  - Work is enqueued on the caller's stream `st` (0 = null stream). Calls
 *    that return a host value synchronise that stream; others are
 *    asynchronous unless stated.
 *  - Arguments are validated before any HIP call. A negative return value is
 *    an error (frkc2_status); frkc2_last_error() then describes it. A GPU
 *    fault of an earlier asynchronous call surfaces as FRKC2_EHIP at the next
 *    call that synchronises.
 *  - Floating point: the kernels evaluate each grid point's arithmetic in one
 *    fixed order (faces x-, x+, y-, y+, z-, z+, each accumulated with one
 *    correctly rounded fused multiply-add; the Euler update as two nested
 *    fused multiply-adds per component), so results do not depend on tiling,
 *    temporal blocking or launch shape.
 */
#ifndef FRKC2_H
#define FRKC2_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FRKC2_OK = 0,
    FRKC2_WQBOUND = 1,      /* coefficients: no n <= 64 met Q <= 10 L^2; lowest-Q order kept */
    FRKC2_EINVAL = -1,      /* invalid argument */
    FRKC2_ENOMEM = -2,      /* workspace too small, or a host allocation failed */
    FRKC2_EHIP = -3,        /* HIP runtime error (including earlier asynchronous faults) */
    FRKC2_EUNSTABLE = -4,   /* T * rho > betabar: the superstep would leave the stability interval */
    FRKC2_ENONFINITE = -5,  /* a norm or bound came out NaN or infinite */
    FRKC2_ETIMEOUT = -6,    /* frkc2_integrate: attempt limit reached before the end time */
    FRKC2_EDISABLED = -7    /* the call is switched off in this version (its block says why) */
} frkc2_status;

typedef enum { FRKC2_BC_PERIODIC = 0, FRKC2_BC_DIRICHLET0 = 1 } frkc2_bc;

/*
 * Diffusion operators f (cell-centred, faces in the order x-, x+, y-, y+, z-, z+):
 *  LAPLACE  f = d_const * sum_f (W_nb - W_c) / h^2
 *  VARCOEF  f = sum_f D_f (W_nb - W_c) / h^2,  D_f = D_c/2 + D_nb/2 (the mean; each
 *           half is exact, so this equals (D_c + D_nb)/2 bit for bit for
 *           normal diffusivities)
 *  POROUS2  f = div(u^2 grad u): sum_f Q_f (W_nb - W_c) / h^2 with
 *           Q_f = (W_c^2 + W_nb^2)/2, evaluated on the complex stage values
 *           (the continuation of u^2 is holomorphic, as the complex Euler
 *           steps of Sec. 3 require).
 *  BRUSS2   the two-species Brusselator of Sec. 3.1 (the default problem of
 *           the paper's public code), periodic 2D grids only:
 *           v_t = d lap v + 1 - 4v + w v^2, w_t = d lap w + 3v - v^2 w,
 *           d = d_const. The state holds 2N values, v then w (each x fastest);
 *           D is not used. Faces as LAPLACE per species; then
 *           p = v^2 = (fma(vr, vr, -(vi*vi)), 2*(vr*vi)), q = w p =
 *           (fma(wr, pr, -(wi*pi)), fma(wr, pi, wi*pr)), R_v = (fma(-4, vr, 1) + qr,
 *           fma(-4, vi, qi)), R_w = (fma(3, vr, -qr), fma(3, vi, -qi)) and
 *           f = fma(acc, 1/h^2, R) per component. Gershgorin bound:
 *           (2/h^2)(4d) + max_c max(|2vw - 4| + v^2, v^2 + |3 - 2vw|).
 *           frkc2_step and frkc2_integrate fuse 2 to 6 stages per pass
 *           (default 4); not available to the batched and adjoint calls.
 *  ADVDIFF  f = d lap u - v . grad u with central differences (Sec. 2.1:
 *           damping makes the schemes usable for problems with a small
 *           hyperbolic part): a LAPLACE stencil whose face coefficients are
 *           d + (0.5 h) v_k on the minus face and d - (0.5 h) v_k on the plus
 *           face of dimension k (d = d_const, v = vel). Gershgorin bound:
 *           (|sum_f c_f| + sum_f |c_f|) / h^2. The spectrum leaves the real
 *           axis; a damping nu that keeps it inside the stability domain is
 *           the caller's choice (the real extent shrinks by about nu).
 *           Not available to the batched and adjoint calls.
 * Dirichlet-zero boundaries use a ghost value W = 0 and, for VARCOEF, a ghost
 * diffusivity equal to the boundary cell's own D.
 */
typedef enum {
    FRKC2_OP_LAPLACE = 0,
    FRKC2_OP_VARCOEF = 1,
    FRKC2_OP_POROUS2 = 2,
    FRKC2_OP_BRUSS2 = 3,
    FRKC2_OP_ADVDIFF = 4
} frkc2_op;

typedef struct {
    int ndim;          /* 1, 2 or 3 */
    int n[3];          /* points per dimension, x first; unused dimensions = 1 */
    double h;          /* grid spacing (all dimensions); the stencil uses 1/(h*h) */
    int bc;            /* frkc2_bc */
    int op;            /* frkc2_op */
    double d_const;    /* diffusivity of FRKC2_OP_LAPLACE, BRUSS2 and ADVDIFF */
    double vel[3];     /* advection velocity per dimension (FRKC2_OP_ADVDIFF only) */
} frkc2_grid;

typedef struct {
    double beta;         /* real extent of the damped polynomial: |R(x)| <= 1 on [-beta, 0] */
    double beta_bar;     /* (1 - n C) beta, C = 1e-4: the usable extent, T rho <= beta_bar */
    double q_realised;   /* max over x in [-beta, 0] and stage runs j..k of prod |1 + a_l x| */
    double mu_re, mu_im; /* damping parameter of the first root group */
    int n_shrink;        /* n of Sec. 2.2 */
    int q_bound_met;     /* q_realised <= 10 L^2 */
} frkc2_coeff_info;

typedef struct {
    double T_last;       /* superstep length of the last superstep */
    double rho_last;     /* Gershgorin bound used for it (0 when not computed) */
    double im_ratio;     /* ||Im W^L||_2 / ||W^L||_2 of the last superstep */
    int supersteps;      /* supersteps completed */
} frkc2_step_stats;

/* Workspace flags for frkc2_workspace_bytes. */
#define FRKC2_WS_STEP    0
#define FRKC2_WS_ADJOINT 1
#define FRKC2_WS_ADAPT   2
#define FRKC2_WS_STAGES  3
#define FRKC2_WS_ADJOINT_STORED 4

/*
 * frkc2_coeffs -- the s ordered stepsizes a_l (Sec. 2, 2.1, 2.2).
 *   s       even, 2 <= s <= 514 (the range of the paper's table, M <= 257, Sec. 3.1)
 *   nu      damping, 0 <= nu < 1 (Sec. 2.1: nu = nu0/N)
 *   a_re, a_im  host arrays of length s, caller-owned; receive a_l in execution order
 *               (may be NULL to query info only)
 *   info    host, may be NULL
 * Host only, no GPU use; results are cached per (s, nu). Returns FRKC2_OK,
 * FRKC2_WQBOUND (usable, flagged) or FRKC2_EINVAL.
 */
int frkc2_coeffs(int s, double nu, double *a_re, double *a_im, frkc2_coeff_info *info);

/*
 * frkc4_coeffs -- the s ordered stepsizes of the fourth-order (N = 4) FRKC
 * polynomial (Sec. 2: B = d0 + 2 sum_{k=1..4} d_k C_{kM}, L = 4M, the d_k from
 * the linear order conditions R^(n)(0) = 1, n = 1..4), in the internal-stability
 * order of Sec. 2.2; the linear flows of the split scheme FRKC4s (Sec. 4.1).
 * Readings: R(x) = P(C_M(z))/P(1), z = 1 + x/(M^2 alpha_M), P of degree 4 fixed
 * by the order conditions for a given alpha_M; damping nu (Sec. 2.1) sets
 * alpha_M so that P(-1) = 1 - 4 nu (the marginal real-axis points get
 * |R| = 1 - 4 nu; nu = 0 gives the largest extent, |P| <= 1 on [-1, 1]); the
 * 2M stepsizes from the roots of P with positive imaginary part are ordered
 * greedily and followed by their conjugates. M = 1 is classical RK4.
 *   s       multiple of 4, 4 <= s <= 512
 *   nu      0 <= nu < 0.25
 *   a_re, a_im, info  as for frkc2_coeffs (info->mu_re holds alpha_M, mu_im 0)
 * Host only; cached per (s, nu). Returns FRKC2_OK, FRKC2_WQBOUND or FRKC2_EINVAL.
 */
int frkc4_coeffs(int s, double nu, double *a_re, double *a_im, frkc2_coeff_info *info);

/*
 * frkc2_write_table -- the stepsize table in the layout of the paper's public
 * code (Sec. 3.1, "FRKC2 public code"): for M = 1 .. m_max (s = 2M stages),
 * line 3M-2 holds betabar and the realised Q, line 3M-1 the real parts and
 * line 3M the imaginary parts of a_1 .. a_s in execution order (%.17g,
 * space separated). The section prints "lines 3M-2 and 3M" for the real and
 * imaginary parts; with betabar and Q already on line 3M-2 the real parts are
 * taken to be on line 3M-1.
 *   path   file to write (created or truncated), host string
 *   nu     damping, 0 <= nu < 1
 *   m_max  1 .. 257
 * Host only, no GPU use. Errors: FRKC2_EINVAL (arguments, file).
 */
int frkc2_write_table(const char *path, double nu, int m_max);

/*
 * frkc2_workspace_bytes -- device workspace needed by the calls below for grid g.
 * A systems pattern of this library (the caller owns all device memory); no
 * passage of the paper defines it.
 *   FRKC2_WS_STEP: frkc2_step and frkc2_rho_bound (two complex state buffers
 *   plus reduction scratch); FRKC2_WS_ADJOINT: frkc2_step_adjoint (s stored
 *   complex stages, two complex adjoint buffers, one real gradient buffer);
 *   FRKC2_WS_ADAPT: frkc2_integrate (two complex and two real state buffers
 *   plus scratch; s is ignored); FRKC2_WS_STAGES: the stage store of
 *   frkc2_step_store and frkc2_step_adjoint_stored (s complex states, each
 *   slot rounded up to 256 bytes); FRKC2_WS_ADJOINT_STORED:
 *   frkc2_step_adjoint_stored (two complex adjoint buffers, one real gradient
 *   buffer, scratch; s is ignored).
 * Returns 0 for an invalid grid (or an invalid s where s sets the size).
 */
size_t frkc2_workspace_bytes(const frkc2_grid *g, int s, int flags);

/*
 * frkc2_rho_bound -- Gershgorin bound on the spectral radius of the Jacobian
 * of f at the real state w, the largest row sum |a_cc| + sum_nb |a_cn|. This
 * is the rho of the stability requirement T rho <= beta_bar (Sec. 2:
 * |R(T lambda)| <= 1 on the spectrum).
 *   LAPLACE, VARCOEF: rho = (2/h^2) * max_c sum_f D_f.
 *   POROUS2: the face value Q_f = (w_c^2 + w_nb^2)/2 depends on the state, so
 *     with dw = w_nb - w_c the row is a_cc = sum_f (w_c dw - Q_f) / h^2 and
 *     a_cn = (w_nb dw + Q_f) / h^2 (a Dirichlet ghost, fixed at 0, adds to
 *     a_cc only): rho = (1/h^2) * max_c (|sum_f (w_c dw - Q_f)| +
 *     sum_f |w_nb dw + Q_f|), per face in the order x-, x+, y-, y+, z-, z+.
 *   BRUSS2: the diffusion rows plus the reaction rows (see the operator list).
 *   ADVDIFF: (|sum_f c_f| + sum_f |c_f|) / h^2, computed on the host.
 *   w   device, N doubles (read for POROUS2 only; may be NULL otherwise)
 *   D   device, N doubles (VARCOEF only; NULL otherwise)
 *   rho host, receives the bound. Synchronises st.
 */
int frkc2_rho_bound(const frkc2_grid *g, const double *w, const double *D, double *rho,
                    void *ws, size_t ws_bytes, hipStream_t st);

/*
 * frkc2_step -- nsteps FRKC2 supersteps of s stages (Sec. 3, Euler-step equation).
 *   w       device, N doubles, in/out: w^n on entry, w^{n+nsteps} on return
 *   D       device, N doubles (VARCOEF only; NULL otherwise)
 *   T, cfl  exactly one is positive. T > 0: fixed superstep length.
 *           cfl > 0: before each superstep T = (cfl * beta_bar) / rho(w^n).
 *   s, nu   as for frkc2_coeffs
 *   ws      device workspace of at least frkc2_workspace_bytes(g, s, FRKC2_WS_STEP)
 *   stats   host, may be NULL; when given, the call synchronises st and fills it
 * Before the first superstep (and before every superstep for the
 * state-dependent operators POROUS2 and BRUSS2) rho is computed and the call
 * fails with FRKC2_EUNSTABLE if T * rho > beta_bar; those checks synchronise
 * st. Otherwise asynchronous. A 1D grid of up to 4096 points runs each
 * superstep in one LDS-resident launch, and for a linear operator (one T) all
 * supersteps of the call but a last one that fills stats in one launch.
 */
int frkc2_step(const frkc2_grid *g, double *w, const double *D, double T, double cfl, int s,
               double nu, int nsteps, void *ws, size_t ws_bytes, hipStream_t st,
               frkc2_step_stats *stats);

/*
 * frkc2_step_noalloc -- frkc2_step for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Same arguments and results as frkc2_step (bit for bit),
 * without ws: the two complex state buffers, reduction partials and stepsize
 * table come from a static device array of the library, one per GPU, of
 * FRKC2_NOALLOC_MAX_VALUES * 32 bytes + 64 KiB (64 MiB + 64 KiB), held from
 * the first call on that GPU until the process ends. The call itself performs
 * no hipMalloc, hipFree or other device allocation.
 *   States of more than FRKC2_NOALLOC_MAX_VALUES values (2^21, e.g. 128^3)
 *   are refused with FRKC2_ENOMEM before any HIP call.
 *   Every call on one GPU shares that GPU's array, which keeps the last
 *   call's contents (nothing in it has to start at zero: every buffer is
 *   written before it is read). Calls that overlap on one GPU (other streams,
 *   other threads) race on it; the caller serialises them.
 * Errors: those of frkc2_step (FRKC2_ENOMEM means the size limit above).
 */
#define FRKC2_NOALLOC_MAX_VALUES 2097152
int frkc2_step_noalloc(const frkc2_grid *g, double *w, const double *D, double T, double cfl,
                       int s, double nu, int nsteps, hipStream_t st, frkc2_step_stats *stats);

/*
 * frkc2_step_adjoint -- reverse-mode derivative of one superstep (VARCOEF or LAPLACE):
 * the transpose of the Sec. 3 Euler-step recursion W^{l+1} = W^l + T a_l f(W^l),
 * applied stage by stage in reverse order.
 * With w^{n+1} = S(w^n; D) the superstep from w_n with fixed T:
 *   lam_next  device, N doubles: dJ/dw^{n+1}
 *   lam_n     device, N doubles, out: dJ/dw^n = S^T lam_next
 *   grad_logD device, N doubles, accumulated (+=): D * dJ/dD for this superstep
 *             (VARCOEF; may be NULL for LAPLACE)
 * The forward stages are recomputed from w_n and stored in ws (s complex
 * stages), then the transposed stages run in reverse order:
 * lam <- lam + conj(tau_l) A lam (A is symmetric), with the face-diffusivity
 * derivative -Re(tau_l conj(lam_nb - lam_c)(W_nb - W_c))/h^2 of each stage
 * accumulated per cell. On request two reverse stages share an HBM pass on
 * 3D grids (FRKC2_OPT_ADJ_STAGES), with the same bits. lam_n may alias
 * lam_next.
 * Asynchronous.
 */
int frkc2_step_adjoint(const frkc2_grid *g, const double *w_n, const double *D, double T, int s,
                       double nu, const double *lam_next, double *lam_n, double *grad_logD,
                       void *ws, size_t ws_bytes, hipStream_t st);

/*
 * frkc2_step_store -- one superstep (Sec. 3, Euler-step equation; VARCOEF or
 * LAPLACE) that keeps its stage states for frkc2_step_adjoint_stored, so that
 * the backward pass need not recompute them: memory (s complex states per
 * superstep) for the recomputation's time.
 *   w       device, N doubles, in/out: w^n on entry, w^{n+1} on return, with the
 *           bits frkc2_step gives for the same T, s and nu
 *   D       device, N doubles (VARCOEF only; NULL otherwise)
 *   T       fixed superstep length, positive and finite
 *   stages  device, caller-owned, at least frkc2_workspace_bytes(g, s,
 *           FRKC2_WS_STAGES) bytes, 16-byte aligned; out: W^0 .. W^{s-1}, the
 *           complex state before stage l at byte offset l * slot, slot =
 *           16 N rounded up to 256, interleaved (re, im) per point in the
 *           grid's x-fastest order
 *   ws      device, reduction scratch of at least 65536 bytes (any
 *           FRKC2_WS_STEP workspace serves); may be NULL for LAPLACE
 * The stability requirement is checked as frkc2_step checks it (FRKC2_EUNSTABLE
 * if T * rho > beta_bar; the check synchronises st for VARCOEF). Otherwise
 * asynchronous.
 */
int frkc2_step_store(const frkc2_grid *g, double *w, const double *D, double T, int s, double nu,
                     double *stages, size_t stages_bytes, void *ws, size_t ws_bytes,
                     hipStream_t st);

/*
 * frkc2_step_adjoint_stored -- frkc2_step_adjoint with the forward stages taken
 * from a store that frkc2_step_store filled for the same g, D, T, s and nu
 * (the same bits as frkc2_step_adjoint from that superstep's w_n).
 *   stages    device, the store as frkc2_step_store left it (read only)
 *   lam_next, lam_n, grad_logD  as for frkc2_step_adjoint (lam_n may alias
 *             lam_next)
 *   ws        device, at least frkc2_workspace_bytes(g, s,
 *             FRKC2_WS_ADJOINT_STORED) bytes, 16-byte aligned
 * Asynchronous.
 */
int frkc2_step_adjoint_stored(const frkc2_grid *g, const double *stages, size_t stages_bytes,
                              const double *D, double T, int s, double nu,
                              const double *lam_next, double *lam_n, double *grad_logD, void *ws,
                              size_t ws_bytes, hipStream_t st);

/*
 * frkc2_step_batched -- one superstep (Sec. 3, Euler-step equation) for each of
 * nprob independent problems (VARCOEF or LAPLACE, 2D or 3D, each with its own
 * grid, T and s) in a single HIP graph launch. Batching is a systems pattern
 * of this library; no passage of the paper defines it. The graph has
 * concurrent branches: 3D problems (two interleaved groups, one branch each)
 * advance in pass levels (level L: stages k3 L .. k3 L + k3 - 1 of every
 * problem that has them, fused in one HBM pass, then the remaining single
 * stages), 2D problems likewise with passes of k2 stages (s = k: k single
 * stages); k3 = 3, k2 = 4 and the fused 3D tiles' width come from
 * frkc2_batched_autotune or the FRKC2_OPT_BATCH_* options (built-in: 3, the
 * width with less modelled work, 4).
 *   grids  host array of nprob grids
 *   w      host array of nprob device pointers (in/out states, real)
 *   D      host array of nprob device pointers (NULL entries for LAPLACE)
 *   T      host array of nprob superstep lengths
 *   s      host array of nprob even stage counts (2..514)
 *   ws     device workspace of at least frkc2_batched_workspace_bytes(...),
 *          256-byte aligned; it holds the work tables and two complex
 *          buffers per problem and must not be shared by concurrent calls
 * The first call for a given set of arguments checks every problem's
 * stability (T rho <= betabar(s), rho the Gershgorin bound of frkc2_rho_bound;
 * FRKC2_EUNSTABLE names the first problem that fails, before any state is
 * touched), builds the work tables and captures the graph (synchronising st);
 * later calls with identical arguments upload the tables again (about 1 MB
 * for 512 problems, asynchronous, so ws need not keep its contents between
 * calls) and replay the graph. The check is not repeated on replays: D must
 * not change while the graph is cached. The graph stays cached for ws until
 * frkc2_batched_release(ws). Each problem's result is bit-identical to
 * frkc2_step on it. frkc2_batched_status synchronises st and reports any
 * HIP error of the replays.
 */
size_t frkc2_batched_workspace_bytes(int nprob, const frkc2_grid *grids, const int *s);
int frkc2_step_batched(int nprob, const frkc2_grid *grids, double *const *w,
                       const double *const *D, const double *T, const int *s, double nu,
                       void *ws, size_t ws_bytes, hipStream_t st);
int frkc2_batched_status(void *ws, hipStream_t st);   /* synchronises st */
int frkc2_batched_release(void *ws);                  /* frees the graph cached for ws */

/*
 * frkc2_batched_autotune -- pick the launch configuration of
 * frkc2_step_batched for a problem set by timing. A batch runs its 3D problems
 * in fused passes of k3 stages (2 or 3) over tiles of 32 or 64 output columns
 * and its 2D problems in fused passes of k2 stages (2, 3, 4 or 6); which is
 * fastest depends on the mix of sizes and stage counts. Candidates: the
 * built-in configuration, every (k3, width) with its k2 (widths 32, 64 and
 * 1, one per problem, as FRKC2_OPT_BATCH_COLS numbers them), then every k2
 * with the best (k3, width); each
 * runs one warm-up and `reps` timed supersteps of the whole batch (graph
 * replays, HIP events on st). The fastest (the built-in one unless a
 * candidate beats it by more than 2 %) is stored for problem sets of the same
 * dimensions, extents, boundaries, operators and s, in the same order, and
 * used by the graphs frkc2_step_batched builds for them while the
 * FRKC2_OPT_BATCH_* options are 0.
 *   nprob .. ws_bytes  as for frkc2_step_batched (the same stability check)
 *   reps               timed supersteps per candidate, 1..100
 *   res                host; receives the choice, the number of
 *                      configurations timed and the average superstep time
 *                      of the choice and of the built-in configuration
 * Every timed superstep advances the states w in place, (reps + 1) per
 * candidate: pass copies of the states to keep them. Every configuration
 * gives the same bits. Synchronises st; drops the graph cached for ws.
 * Errors: FRKC2_EINVAL (arguments), FRKC2_EUNSTABLE, FRKC2_ENONFINITE,
 * FRKC2_ENOMEM (workspace), FRKC2_EHIP.
 * SWITCHED OFF in this version: after validating its arguments the call returns
 * FRKC2_EDISABLED without touching the GPU. Two test runs that rebuilt the
 * batch graph for every candidate ended in a host heap corruption detected
 * inside this call (glibc "free(): invalid pointer"), and its cause was not
 * found; frkc2_step_batched uses the FRKC2_OPT_BATCH_* options or the built-in
 * configuration meanwhile.
 */
/*
 * frkc2_batched_config -- the launch configuration frkc2_step_batched would
 * build a graph with for this problem set now: the FRKC2_OPT_BATCH_* options
 * where set, else what frkc2_batched_autotune stored for the set, else the
 * built-in one. Host only, no GPU use.
 *   nprob, grids, s  as for frkc2_step_batched
 *   k3, cols3, k2    host, out: stages per fused 3D pass, output columns of
 *                    its tiles (1: per problem), stages per fused 2D pass
 * Errors: FRKC2_EINVAL.
 */
int frkc2_batched_config(int nprob, const frkc2_grid *grids, const int *s, int *k3, int *cols3,
                         int *k2);

typedef struct {
    int k3;             /* stages per fused 3D pass */
    int cols3;          /* output columns of the fused 3D tiles (1: per problem) */
    int k2;             /* stages per fused 2D pass */
    int candidates;     /* configurations timed */
    double ms_best;     /* average superstep time of the choice */
    double ms_default;  /* ... and of the built-in configuration */
} frkc2_batch_tune_result;
int frkc2_batched_autotune(int nprob, const frkc2_grid *grids, double *const *w,
                           const double *const *D, const double *T, const int *s, double nu,
                           int reps, void *ws, size_t ws_bytes, hipStream_t st,
                           frkc2_batch_tune_result *res);

/*
 * frkc2_reduce -- deterministic FP64 reductions over n elements (device x, y).
 *   op 0: sum x_i^2    1: sum x_i    2: max x_i^2    3: sum (x_i - y_i)^2
 *      4: sum x_i y_i
 *   result host, synchronises st. ws needs 8 KiB.
 */
#define FRKC2_RED_SUMSQ 0
#define FRKC2_RED_SUM 1
#define FRKC2_RED_MAXSQ 2
#define FRKC2_RED_SUMSQDIFF 3
#define FRKC2_RED_DOT 4
int frkc2_reduce(int op, const double *x, const double *y, size_t n, double *result,
                 void *ws, size_t ws_bytes, hipStream_t st);

/*
 * frkc2_integrate -- error-controlled FRKC2 integration over a time span
 * (Sec. 3, error control). Each attempt runs one superstep that also carries
 * the embedded first-order solution What (real parts of the stepsizes and of
 * f(W^l) only: What^{l+1} = What^l + T Re(a_l) Re f(W^l)), estimates
 *   err = max_points |W^L - What^L| / (tol (1 + max(|W^L|, |What^L|)))
 * (complex modulus), rejects the step if err > 1 and retries with T scaled by
 * SAFE / sqrt(err), and otherwise keeps Re W^L and sets the next length with
 * the predictive controller T (SAFE / sqrt(err_n)) (T_n / T_{n-1})
 * sqrt(err_{n-1} / err_n), SAFE = 0.8 (after two consecutive accepted steps;
 * T SAFE / sqrt(err) otherwise; err floored at 1e-12, growth capped at 5).
 * The stage count of each attempt is the smallest even s with
 * betabar(s) >= T rho (rho the Gershgorin bound, recomputed per step for
 * POROUS2); beyond s = 514, T is cut to 0.99 betabar(514) / rho. The last step
 * ends exactly at t_span.
 *   g, w, D, nu  as for frkc2_step; w (device) is advanced in place by t_span
 *   t_span       time to advance, > 0
 *   T0           first superstep length to try, > 0
 *   tol          error tolerance of the estimate, > 0
 *   max_attempts bound on supersteps tried (accepted + rejected); exceeding
 *                it returns FRKC2_ETIMEOUT with w at the last accepted step
 *   ws, ws_bytes frkc2_workspace_bytes(g, 0, FRKC2_WS_ADAPT) bytes, 16-byte aligned
 *   trace        host array of 5 * trace_cap doubles or NULL: per attempt
 *                (t, T, s, err, accepted 1/0), the first trace_cap attempts
 *   stats        host or NULL
 * Synchronises st once per attempt (the accept decision is taken on the
 * host). 3D grids (full-width tiles), 2D grids (rows of 256, depth 2..4) and
 * the Brusselator fuse stages per HBM pass as frkc2_step does (the embedded
 * solution adds 16 B per point and species and pass); 1D grids of up to 4096
 * points run each attempt's superstep in one LDS-resident launch; other
 * depths, tile shapes and longer 1D grids run one stage per pass. Results are
 * identical, bit for bit, to the same procedure evaluated on the CPU in the
 * library's arithmetic order. Errors:
 * FRKC2_EINVAL (arguments, checked before any HIP call), FRKC2_ENOMEM
 * (workspace), FRKC2_ENONFINITE (non-finite error estimate), FRKC2_ETIMEOUT,
 * FRKC2_EHIP.
 */
typedef struct {
    double t;           /* time reached (t_span on success) */
    double T_next;      /* length the controller proposes for the next superstep */
    double err_last;    /* error estimate of the last accepted superstep */
    long long stages;   /* stages (f evaluations) over all attempts */
    int attempts, accepted, rejected;
    int s_last;         /* stage count of the last attempt */
} frkc2_adapt_stats;
int frkc2_integrate(const frkc2_grid *g, double *w, const double *D, double t_span, double T0,
                    double tol, double nu, int max_attempts, void *ws, size_t ws_bytes,
                    hipStream_t st, double *trace, int trace_cap, frkc2_adapt_stats *stats);

/*
 * frkc2_step_user -- supersteps with a caller-supplied operator, the split of
 * the paper's public code into the scheme's core and the problem's f
 * (Sec. 3.1). The library keeps the complex stage W (interleaved re, im, n
 * values) and the stepsizes; per stage it calls f(W, F, n, user, st), which
 * must write F = f(W) (complex, the holomorphic continuation of the caller's
 * real operator) on stream st and return 0, and then applies
 * W <- W + T a_l F on the GPU (fma order of frkc2_step). The first stage
 * starts from (w, 0); the superstep keeps Re W^L in w.
 *   n, w     values per state, device state (in/out)
 *   f, user  callback and its context; W and F are device pointers into ws
 *   T, rho   superstep length and a bound on the spectral radius of f's
 *            Jacobian (T rho <= betabar(s) is required; rho = 0 skips it)
 *   s, nu, nsteps  as for frkc2_step
 *   ws       frkc2_user_workspace_bytes(n, FRKC2_WS_STEP) bytes, 16-byte
 *            aligned
 * Errors: FRKC2_EINVAL (arguments, checked before any HIP call; a non-zero
 * return of f), FRKC2_EUNSTABLE, FRKC2_ENOMEM, FRKC2_EHIP.
 */
typedef int (*frkc2_user_f)(const double *W, double *F, long long n, void *user, hipStream_t st);
int frkc2_step_user(long long n, double *w, frkc2_user_f f, void *user, double T, double rho,
                    int s, double nu, int nsteps, void *ws, size_t ws_bytes, hipStream_t st);

/*
 * frkc2_user_workspace_bytes -- device workspace of frkc2_step_user
 * (flags FRKC2_WS_STEP) or frkc2_integrate_user (FRKC2_WS_ADAPT) for states of
 * n values; 0 for n < 1 or other flags.
 */
size_t frkc2_user_workspace_bytes(long long n, int flags);

/*
 * frkc2_integrate_user -- the error control of frkc2_integrate (Sec. 3, the
 * same readings and controller) around a caller-supplied operator as in
 * frkc2_step_user: the paper's public code runs its error-controlled core
 * around the user's f in the same way (Sec. 3.1). Per attempt the library
 * starts W from (w, 0) and the embedded solution from w, calls f before each
 * stage and applies W <- W + tau_l F and What <- What + Re tau_l Re F (fma
 * order of frkc2_step), then takes the error estimate and the accept decision.
 *   n, w, f, user      as for frkc2_step_user
 *   rho_f, rho_const   spectral-radius bound of f's Jacobian: rho_f(w, n, user,
 *                      st, &rho) is called on the host with the current real
 *                      state before the first attempt and after every accepted
 *                      step and must return 0 and a positive finite rho; with
 *                      rho_f NULL the constant rho_const (> 0) is used
 *   t_span, T0, tol, nu, max_attempts, trace, trace_cap, stats
 *                      as for frkc2_integrate
 *   ws                 frkc2_user_workspace_bytes(n, FRKC2_WS_ADAPT) bytes,
 *                      16-byte aligned
 * Errors: FRKC2_EINVAL (arguments, checked before any HIP call; a non-zero
 * return of f or rho_f), FRKC2_ENOMEM, FRKC2_ENONFINITE, FRKC2_ETIMEOUT,
 * FRKC2_EHIP.
 */
typedef int (*frkc2_user_rho)(const double *w, long long n, void *user, hipStream_t st,
                              double *rho);
int frkc2_integrate_user(long long n, double *w, frkc2_user_f f, frkc2_user_rho rho_f,
                         double rho_const, void *user, double t_span, double T0, double tol,
                         double nu, int max_attempts, void *ws, size_t ws_bytes, hipStream_t st,
                         double *trace, int trace_cap, frkc2_adapt_stats *stats);

/*
 * frkc4s_step -- nsteps steps of the fourth-order split scheme FRKC4s (Sec. 4.1,
 * "Complex splitting") on the two-species Brusselator (g->op = FRKC2_OP_BRUSS2,
 * periodic 2D, d = g->d_const): w' = A w + f_B(w) with A = d lap per species and
 * f_B the reaction of Sec. 3.1. One step of length T is
 *   w <- Re[ e^{b1 T B} e^{T/4 A} e^{b2 T B} e^{T/4 A} e^{b3 T B} e^{T/4 A}
 *            e^{b2 T B} e^{T/4 A} e^{b1 T B} w ],
 * b1 = (3 + i)/30, b2 = (4 - 2i)/15, b3 = (4 + 3i)/15 (the symmetric
 * composition with four equal real A steps; consistency and the third-order
 * conditions leave this conjugate pair, the paper prints no coefficients).
 * Each A flow is one superstep of s stages of the fourth-order polynomial
 * (frkc4_coeffs) on the complex state, per species, fused as frkc2_step
 * fuses stages; each B flow integrates dY/dsig = (b T) f_B(Y), sig in [0, 1], by
 * nsub classical Runge-Kutta steps per grid point (arithmetic order in
 * frkc4.hip). The first B flow starts from (w, 0); the step keeps Re.
 *   w      device, 2N doubles (v then w), in/out
 *   T      step length, > 0; (T/4) rho <= betabar_4(s) is required,
 *          rho = 8 d / h^2 (FRKC2_EUNSTABLE otherwise)
 *   s      multiple of 4, 4..512; nu as for frkc4_coeffs
 *   nsub   1..64
 *   ws     frkc4s_workspace_bytes(g) bytes, 16-byte aligned
 * Asynchronous. Errors: FRKC2_EINVAL (arguments, checked before any HIP call),
 * FRKC2_EUNSTABLE, FRKC2_ENOMEM, FRKC2_EHIP.
 */
size_t frkc4s_workspace_bytes(const frkc2_grid *g);
int frkc4s_step(const frkc2_grid *g, double *w, double T, int s, int nsub, double nu, int nsteps,
                void *ws, size_t ws_bytes, hipStream_t st);

/*
 * frkc2_autotune -- pick the launch configuration of frkc2_step's passes for
 * one grid by timing. The stages of a superstep are applied one after the
 * other (Sec. 3, the Euler-step recursion), so any number k of consecutive
 * stages can share one HBM pass; the best k, tile shape and z chunk length
 * depend on the grid and the operator. Every candidate (k = 1 and each
 * supported fused depth, tile shape, chunk length) runs `reps` whole
 * supersteps of s stages at T = betabar / (2 rho) on the caller's data, timed
 * with HIP events on st; the fastest (the built-in default unless a candidate
 * beats it by more than 3 %) is stored for grids of the same shape,
 * operator and boundary and used by later frkc2_step calls while
 * FRKC2_OPT_TBLOCK is 0 (automatic).
 *   g, w, D, s, nu  as for frkc2_step; w and D are only read.
 *   reps            timed supersteps per candidate, 1..100 (one more warms up)
 *   ws, ws_bytes    frkc2_workspace_bytes(g, s, 0) bytes, 16-byte aligned
 *   res             host; receives the chosen configuration and the average
 *                   superstep time of it and of the built-in default
 * Synchronises st. Results of frkc2_step are identical, bit for bit, for
 * every configuration, so tuning changes only the time. Errors: FRKC2_EINVAL
 * (arguments, checked before any HIP call), FRKC2_ENOMEM (workspace),
 * FRKC2_EHIP.
 */
typedef struct {
    int tblock;         /* stages per fused pass (1 = one stage per pass) */
    int tile;           /* tile shape, as FRKC2_OPT_TILE numbers it (>= 1) */
    int zchunk;         /* z planes (2D: rows) per workgroup, 0 = automatic */
    int candidates;     /* configurations timed */
    double ms_best;     /* average superstep time of the chosen configuration */
    double ms_default;  /* ... and of the built-in default */
} frkc2_tune_result;
int frkc2_autotune(const frkc2_grid *g, const double *w, const double *D, int s, double nu,
                   int reps, void *ws, size_t ws_bytes, hipStream_t st, frkc2_tune_result *res);

/*
 * frkc2_set_option -- tuning knobs (process-wide, not thread-safe to change
 * while other threads call the library):
 *   FRKC2_OPT_TBLOCK  stages fused per HBM pass of frkc2_step: 1, or 2 and 3
 *                     (3D), 2, 3, 4, 6 and 8 (2D), 2 to 6 (BRUSS2: 64x40
 *                     tiles of both species, its own shape, TILE and ZCHUNK
 *                     do not apply); an unsupported depth runs one stage per
 *                     pass; 0 = automatic (the entry frkc2_autotune stored for
 *                     the grid, else 3 in 3D, 4 in 2D, 1 in 1D)
 *   FRKC2_OPT_TILE    tile shape of the fused passes: 0 = automatic (3D 4 or
 *                     5, whichever a pass-time model prefers for the grid;
 *                     2D 1); 3D 1 = 64x16 extended columns, 2 = 64x32 (k = 2),
 *                     3 = 64x32 (k = 2) or 64x24 (k = 3) with 512 threads,
 *                     4 = 64-column output rows with halo wavefronts (64x11
 *                     outputs for k = 2, 64x8 for k = 3), 5 = 32-column output
 *                     rows, two per wavefront (32x24 for k = 2, 32x20 for
 *                     k = 3); 2D 1 = rows of 256, 2 = rows of 512
 *   FRKC2_OPT_ZCHUNK  z planes (2D: rows) per workgroup of every pass of
 *                     frkc2_step, 0 = automatic (3D shapes 4 and 5: the length
 *                     with the most useful planes per CU-step over whole
 *                     rounds of one workgroup per CU; otherwise halve from the
 *                     whole depth until >= 512 workgroups for 3D fused passes,
 *                     >= 2048 otherwise)
 *   FRKC2_OPT_CLEAR_TUNED  forget every configuration frkc2_autotune and
 *                     frkc2_batched_autotune stored (value ignored)
 *   FRKC2_OPT_ADJ_STAGES  reverse stages per pass of frkc2_step_adjoint: 0 =
 *                     automatic (one), 1, or 2 (3D grids; others run one;
 *                     two move 44 instead of 72 bytes per cell and stage but
 *                     take longer at 128^3, their extra arithmetic and
 *                     barriers being the limit)
 *   FRKC2_OPT_BATCH_K3, FRKC2_OPT_BATCH_COLS, FRKC2_OPT_BATCH_K2  the launch
 *                     configuration of every frkc2_step_batched graph built
 *                     afterwards: stages per fused 3D pass (2 or 3), output
 *                     columns of its tiles (32 or 64 for all 3D problems, or
 *                     1: each problem the width with less modelled work for
 *                     it, the two widths on separate graph branches), stages
 *                     per fused 2D pass (2, 3, 4 or 6); 0 = automatic (what
 *                     frkc2_batched_autotune stored for the problem set, else
 *                     the built-in configuration of frkc2_step_batched)
 * Results are identical, bit for bit, for every setting.
 */
#define FRKC2_OPT_TBLOCK 1
#define FRKC2_OPT_TILE 3
#define FRKC2_OPT_CLEAR_TUNED 4
#define FRKC2_OPT_ZCHUNK 5
#define FRKC2_OPT_ADJ_STAGES 9
#define FRKC2_OPT_BATCH_K3 6
#define FRKC2_OPT_BATCH_COLS 7
#define FRKC2_OPT_BATCH_K2 8
int frkc2_set_option(int key, int value);

/*
 * frkc2_stream_copy -- a measurement helper, not part of the method: copies
 * `bytes` (a multiple of 16) from src to dst (device, 16-byte aligned, not
 * overlapping) with 128-bit accesses per lane, blocks_per_cu workgroups of
 * 256 threads per CU (1..64), plain (nontemporal = 0) or nontemporal accesses.
 * Timed by the caller, it gives the HBM streaming ceiling the stage kernels'
 * bandwidth is compared with. Asynchronous.
 */
int frkc2_stream_copy(const void *src, void *dst, size_t bytes, int blocks_per_cu, int nontemporal,
                      hipStream_t st);

/* Thread-local description of the last error. */
const char *frkc2_last_error(void);

/* Library version string. */
const char *frkc2_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FRKC2_H */
