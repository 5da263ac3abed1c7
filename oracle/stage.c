/*
 * Oracle for the FRKC2 superstep: plain CPU FP64 stage loops.
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library. It shares no code with the GPU
 * library; the two meet only in the seeded inputs and in the stepsizes each
 * computes on its own.
 *
 * Method: O'Sullivan, "Factorized Runge-Kutta-Chebyshev Methods",
 * arXiv:1702.03818, Sec. 3 ("FRKC2 schemes"): a superstep of length T is the
 * ordered sequence of L = s forward Euler steps W^{l+1} = W^l + T a_l f(W^l),
 * W^0 = w^n, w^{n+1} = W^L, with complex a_l, so the stages are complex.
 * The caller passes tau_l = T a_l. The result kept is Re W^L.
 *
 * f is the semi-discrete diffusion operator of Sec. 1 (w' = f(t, w) with a
 * Jacobian whose eigenvalues lie near the negative real axis), here on a
 * uniform grid of spacing h, cell-centred, x fastest:
 *   op 0 (Laplace):    f = d sum_faces (W_nb - W_c) / h^2
 *   op 1 (var. coef.): f = sum_faces D_f (W_nb - W_c) / h^2, D_f = (D_c + D_nb)/2
 *   op 2 (porous):     f = sum_faces Q_f (W_nb - W_c) / h^2, Q_f = (W_c^2 + W_nb^2)/2
 *                      (div(u^2 grad u); u^2 is holomorphic, so it is applied
 *                      to the complex stage values unchanged)
 * Boundaries: periodic (wrap), or Dirichlet zero (ghost W = 0 and, for op 1,
 * ghost D equal to the cell's own D, so the boundary face carries D_c).
 *
 * Evaluation order (fixed; the paper fixes none, and the GPU library
 * evaluates the same expressions in the same order, so results agree to the
 * last bit). fma(a, b, c) is the correctly rounded a*b + c (C99):
 *   faces in the order x-, x+, y-, y+, z-, z+; dr = Wr_nb - Wr_c, di likewise;
 *   op 1:   Df = 0.5*D_c + 0.5*D_nb (each half exact; equal to (D_c + D_nb)/2
 *           to the last bit whenever the halves are normal and the sum finite);
 *   op 0/1: acc_r = fma(Df, dr, acc_r), acc_i = fma(Df, di, acc_i);
 *   op 2:   q = W^2 as (fma(Wr, Wr, -(Wi*Wi)), 2*(Wr*Wi)) for cell and
 *           neighbour, Qr = qr_c/2 + qr_nb/2, Qi likewise (halves exact: the
 *           same bits as (qr_c + qr_nb)/2 whenever they are normal),
 *           acc_r = fma(Qr, dr, fma(-Qi, di, acc_r)),
 *           acc_i = fma(Qr, di, fma(Qi, dr, acc_i));
 *   f = acc*inv_h2 with inv_h2 = 1/(h*h);
 *   Wr = fma(tr, fr, fma(-ti, fi, Wr)), Wi = fma(tr, fi, fma(ti, fr, Wi)).
 * Built with -ffp-contract=off, so no other multiply-add is fused.
 *
 * The adjoint runs the transposed stages in reverse order. Because A is
 * symmetric, the adjoint of W <- W + tau A W is lam <- lam + conj(tau) A lam
 * for lam = dJ/dWr + i dJ/dWi; the derivative with respect to a face
 * diffusivity is -Re(tau conj(lam_nb - lam_c) (W_nb - W_c))/h^2, with
 * lam = lam^{l+1} and W = W^l, split half to each cell of an interior face
 * and fully to the cell of a Dirichlet boundary face.
 */
#include <math.h>

/* FMA is the correctly rounded fused multiply-add of C99 (the arithmetic order
 * above). Built with -DORACLE_UNFUSED it is the plain a*b + c (two roundings):
 * that variant only measures how far the fused order moves results from the
 * unfused one; it is not the reference the tests compare against. */
#ifdef ORACLE_UNFUSED
#define FMA(a, b, c) ((a) * (b) + (c))
#else
#define FMA(a, b, c) fma((a), (b), (c))
#endif
#include <stdlib.h>
#include <string.h>

enum { BC_PERIODIC = 0, BC_DIRICHLET0 = 1 };
enum { OP_LAPLACE = 0, OP_VARCOEF = 1, OP_POROUS2 = 2, OP_BRUSS2 = 3, OP_ADVDIFF = 4 };

typedef struct {
    int ndim;
    long n[3];
    int bc, op;
    double inv_h2, d_const;
    double fc[6];   /* op 4: coefficient of face f = 2*dim + side */
} grid_t;

/* Op 4, advection-diffusion f = d lap u - v . grad u with central differences
 * (Sec. 2.1: the damped schemes for problems with a small hyperbolic part):
 * the flux form d (u_nb - u_c)/h^2 per face plus -v_k (u_{+} - u_{-})/(2h)
 * per dimension gives face coefficients d + v_k h/2 (minus side) and
 * d - v_k h/2 (plus side); the caller passes them in fc, computed as
 * d + (0.5*h)*v_k and d - (0.5*h)*v_k. */

static long npts(const grid_t *g) { return g->n[0] * g->n[1] * g->n[2]; }

/* Face coefficients of op 4 for the calls that follow (set from Python before
 * each call; the oracle is not called from several threads at once). */
static double g_fc[6];
static int g_fc_set = 0;

void oracle_set_faces(const double *fc)
{
    g_fc_set = fc != NULL;
    for (int f = 0; f < 6; ++f) g_fc[f] = fc ? fc[f] : 0.0;
}

/* Values per grid point: the Brusselator carries two species (v then w). */
static int nfield(const grid_t *g) { return g->op == OP_BRUSS2 ? 2 : 1; }
static long nstate(const grid_t *g) { return nfield(g) * npts(g); }

/* Index of the neighbour of point (i[0], i[1], i[2]) across face f
 * (f = 2*dim + side, side 0 = minus, 1 = plus), or -1 for a Dirichlet ghost. */
static long neighbour(const grid_t *g, const long i[3], int f)
{
    long j[3] = {i[0], i[1], i[2]};
    int d = f / 2;
    j[d] += (f % 2) ? 1 : -1;
    if (j[d] < 0 || j[d] >= g->n[d]) {
        if (g->bc == BC_DIRICHLET0) return -1;
        j[d] = (j[d] + g->n[d]) % g->n[d];
    }
    return j[0] + g->n[0] * (j[1] + g->n[1] * j[2]);
}

static void coords(const grid_t *g, long p, long i[3])
{
    i[0] = p % g->n[0];
    i[1] = (p / g->n[0]) % g->n[1];
    i[2] = p / (g->n[0] * g->n[1]);
}

/*
 * Two-species Brusselator of Sec. 3.1 (the default problem of the paper's
 * public code): v_t = d lap v + 1 - 4v + w v^2, w_t = d lap w + 3v - v^2 w,
 * with d = d_const, applied to complex stage values (a polynomial, so the
 * complex stages need no continuation). State layout: v at [0, N), w at
 * [N, 2N). Per point: each species' faces as for op 0 (acc = fma(d, nb - c,
 * acc)); p = v^2 = (fma(vr, vr, -(vi*vi)), 2*(vr*vi)); q = w p =
 * (fma(wr, pr, -(wi*pi)), fma(wr, pi, wi*pr)); R_v = (fma(-4, vr, 1) + qr,
 * fma(-4, vi, qi)); R_w = (fma(3, vr, -qr), fma(3, vi, -qi));
 * f = fma(acc, inv_h2, R) per component.
 */
static void apply_bruss(const grid_t *g, const double *wr, const double *wi, double *fr,
                        double *fi)
{
    long N = npts(g);
    double d = g->d_const;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        long i[3];
        coords(g, p, i);
        double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        for (int s = 0; s < 2; ++s) {
            const double *ur = wr + s * N, *ui = wi + s * N;
            for (int f = 0; f < 2 * g->ndim; ++f) {
                long q = neighbour(g, i, f);
                double nr = (q < 0) ? 0.0 : ur[q];
                double ni = (q < 0) ? 0.0 : ui[q];
                acc[s][0] = FMA(d, nr - ur[p], acc[s][0]);
                acc[s][1] = FMA(d, ni - ui[p], acc[s][1]);
            }
        }
        double vr = wr[p], vi = wi[p], xr = wr[N + p], xi = wi[N + p];
        double pr = FMA(vr, vr, -(vi * vi)), pi = 2.0 * (vr * vi);
        double qr = FMA(xr, pr, -(xi * pi)), qi = FMA(xr, pi, xi * pr);
        double rvr = FMA(-4.0, vr, 1.0) + qr, rvi = FMA(-4.0, vi, qi);
        double rwr = FMA(3.0, vr, -qr), rwi = FMA(3.0, vi, -qi);
        fr[p] = FMA(acc[0][0], g->inv_h2, rvr);
        fi[p] = FMA(acc[0][1], g->inv_h2, rvi);
        fr[N + p] = FMA(acc[1][0], g->inv_h2, rwr);
        fi[N + p] = FMA(acc[1][1], g->inv_h2, rwi);
    }
}

/* F = f(W) for complex W = (wr, wi), all points. */
static void apply_op(const grid_t *g, const double *D, const double *wr, const double *wi,
                     double *fr, double *fi)
{
    if (g->op == OP_BRUSS2) {
        apply_bruss(g, wr, wi, fr, fi);
        return;
    }
    long N = npts(g);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        long i[3];
        coords(g, p, i);
        double acc_r = 0.0, acc_i = 0.0;
        for (int f = 0; f < 2 * g->ndim; ++f) {
            long q = neighbour(g, i, f);
            double nr = (q < 0) ? 0.0 : wr[q];
            double ni = (q < 0) ? 0.0 : wi[q];
            double dr = nr - wr[p];
            double di = ni - wi[p];
            if (g->op == OP_POROUS2) {
                double qr_c = FMA(wr[p], wr[p], -(wi[p] * wi[p]));
                double qi_c = 2.0 * (wr[p] * wi[p]);
                double qr_n = FMA(nr, nr, -(ni * ni));
                double qi_n = 2.0 * (nr * ni);
                double Dr = 0.5 * qr_c + 0.5 * qr_n;
                double Di = 0.5 * qi_c + 0.5 * qi_n;
                acc_r = FMA(Dr, dr, FMA(-Di, di, acc_r));
                acc_i = FMA(Dr, di, FMA(Di, dr, acc_i));
            } else {
                double Df;
                if (g->op == OP_LAPLACE) {
                    Df = g->d_const;
                } else if (g->op == OP_ADVDIFF) {
                    Df = g->fc[f];
                } else {
                    double Dn = (q < 0) ? D[p] : D[q];
                    Df = 0.5 * D[p] + 0.5 * Dn;
                }
                acc_r = FMA(Df, dr, acc_r);
                acc_i = FMA(Df, di, acc_i);
            }
        }
        fr[p] = acc_r * g->inv_h2;
        fi[p] = acc_i * g->inv_h2;
    }
}

static int make_grid(grid_t *g, int ndim, const long *n, int bc, int op, double inv_h2,
                     double d_const)
{
    for (int f = 0; f < 6; ++f) g->fc[f] = (op == OP_ADVDIFF && g_fc_set) ? g_fc[f] : d_const;
    if (ndim < 1 || ndim > 3) return -1;
    g->ndim = ndim;
    for (int d = 0; d < 3; ++d) g->n[d] = (d < ndim) ? n[d] : 1;
    for (int d = 0; d < 3; ++d) if (g->n[d] < 1) return -1;
    g->bc = bc;
    g->op = op;
    g->inv_h2 = inv_h2;
    g->d_const = d_const;
    return 0;
}

/*
 * One superstep. w: real W^0 on entry, Re W^L on exit; wi_out (may be NULL):
 * Im W^L; store (may be NULL): every stage W^0 .. W^{s-1} (re then im);
 * emb_out (may be NULL): the embedded first-order solution of Sec. 3, which
 * uses only the real parts of the stepsizes and of f(W^l):
 *   What^0 = W^0, What^{l+1} = What^l + T Re(a_l) Re f(W^l),
 * evaluated as What = fma(tr, Re f, What) with tr = Re(tau_l).
 */
int oracle_superstep(int ndim, const long *n, int bc, int op, double inv_h2, double d_const,
                     const double *D, int s, const double *tau_re, const double *tau_im,
                     double *w, double *wi_out, double *store, double *emb_out)
{
    grid_t g;
    if (make_grid(&g, ndim, n, bc, op, inv_h2, d_const)) return -1;
    long N = nstate(&g);   /* values per state (both species for op 3) */
    double *wr = malloc(sizeof(double) * N), *wi = malloc(sizeof(double) * N);
    double *fr = malloc(sizeof(double) * N), *fi = malloc(sizeof(double) * N);
    if (!wr || !wi || !fr || !fi) { free(wr); free(wi); free(fr); free(fi); return -2; }
    memcpy(wr, w, sizeof(double) * N);
    memset(wi, 0, sizeof(double) * N);
    if (emb_out) memcpy(emb_out, w, sizeof(double) * N);
    for (int l = 0; l < s; ++l) {
        if (store) {
            memcpy(store + (size_t)2 * N * l, wr, sizeof(double) * N);
            memcpy(store + (size_t)2 * N * l + N, wi, sizeof(double) * N);
        }
        apply_op(&g, D, wr, wi, fr, fi);
        double tr = tau_re[l], ti = tau_im[l];
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) {
            double nr = FMA(tr, fr[p], FMA(-ti, fi[p], wr[p]));
            double ni = FMA(tr, fi[p], FMA(ti, fr[p], wi[p]));
            wr[p] = nr;
            wi[p] = ni;
            if (emb_out) emb_out[p] = FMA(tr, fr[p], emb_out[p]);
        }
    }
    memcpy(w, wr, sizeof(double) * N);
    if (wi_out) memcpy(wi_out, wi, sizeof(double) * N);
    free(wr); free(wi); free(fr); free(fi);
    return 0;
}

/*
 * One forward Euler stage W <- W + tau f (Sec. 3, the Euler-step equation)
 * for a caller-supplied f, in the same expressions as the stage loop above;
 * emb (may be NULL) is the embedded first-order solution of Sec. 3's error
 * estimate, advanced by Re tau Re f.
 */
void oracle_euler_update(long N, double *wr, double *wi, const double *fr, const double *fi,
                         double tr, double ti, double *emb)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        double nr = FMA(tr, fr[p], FMA(-ti, fi[p], wr[p]));
        double ni = FMA(tr, fi[p], FMA(ti, fr[p], wi[p]));
        wr[p] = nr;
        wi[p] = ni;
        if (emb) emb[p] = FMA(tr, fr[p], emb[p]);
    }
}

/*
 * Adjoint of one superstep (ops 0 and 1). Given w_n, the stepsizes and
 * lam_next = dJ/dw^{n+1}, writes lam_n = dJ/dw^n and adds D * dJ/dD to
 * grad_logD (op 1 only; grad_logD may be NULL for op 0).
 */
int oracle_adjoint(int ndim, const long *n, int bc, int op, double inv_h2, double d_const,
                   const double *D, int s, const double *tau_re, const double *tau_im,
                   const double *w_n, const double *lam_next, double *lam_n, double *grad_logD)
{
    grid_t g;
    if (op == OP_POROUS2 || op == OP_BRUSS2 || op == OP_ADVDIFF) return -1;
    if (make_grid(&g, ndim, n, bc, op, inv_h2, d_const)) return -1;
    long N = npts(&g);
    double *store = malloc(sizeof(double) * 2 * N * (size_t)s);
    double *w = malloc(sizeof(double) * N);
    double *lr = malloc(sizeof(double) * N), *li = malloc(sizeof(double) * N);
    double *gr = malloc(sizeof(double) * N), *gi = malloc(sizeof(double) * N);
    double *gD = calloc(N, sizeof(double));
    if (!store || !w || !lr || !li || !gr || !gi || !gD) {
        free(store); free(w); free(lr); free(li); free(gr); free(gi); free(gD);
        return -2;
    }
    memcpy(w, w_n, sizeof(double) * N);
    oracle_superstep(ndim, n, bc, op, inv_h2, d_const, D, s, tau_re, tau_im, w, NULL, store, NULL);
    memcpy(lr, lam_next, sizeof(double) * N);
    memset(li, 0, sizeof(double) * N);
    for (int l = s - 1; l >= 0; --l) {
        const double *Wr = store + (size_t)2 * N * l, *Wi = Wr + N;
        double tr = tau_re[l], ti = tau_im[l];
        if (op == OP_VARCOEF) {
#pragma omp parallel for schedule(static)
            for (long p = 0; p < N; ++p) {
                long i[3];
                coords(&g, p, i);
                double gsum = 0.0;
                for (int f = 0; f < 2 * ndim; ++f) {
                    long q = neighbour(&g, i, f);
                    double dWr = ((q < 0) ? 0.0 : Wr[q]) - Wr[p];
                    double dWi = ((q < 0) ? 0.0 : Wi[q]) - Wi[p];
                    double dLr = ((q < 0) ? 0.0 : lr[q]) - lr[p];
                    double dLi = ((q < 0) ? 0.0 : li[q]) - li[p];
                    double pr = dLr * dWr + dLi * dWi;
                    double pi = dLr * dWi - dLi * dWr;
                    double e = tr * pr - ti * pi;
                    double wgt = (q < 0) ? 1.0 : 0.5;
                    gsum = gsum + wgt * e;
                }
                gD[p] = gD[p] - gsum * inv_h2;
            }
        }
        apply_op(&g, D, lr, li, gr, gi);
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) {
            double nr = lr[p] + (tr * gr[p] + ti * gi[p]);
            double ni = li[p] + (tr * gi[p] - ti * gr[p]);
            lr[p] = nr;
            li[p] = ni;
        }
    }
    memcpy(lam_n, lr, sizeof(double) * N);
    if (op == OP_VARCOEF && grad_logD) {
        for (long p = 0; p < N; ++p) grad_logD[p] = grad_logD[p] + D[p] * gD[p];
    }
    free(store); free(w); free(lr); free(li); free(gr); free(gi); free(gD);
    return 0;
}

/*
 * Gershgorin bound on the spectral radius of the Jacobian of f at real w
 * (the rho of the stability requirement T rho <= betabar, Sec. 2):
 *  ops 0, 1: the operator is linear, the row of cell c has diagonal
 *            -sum_f D_f / h^2 and off-diagonal entries D_f / h^2, so
 *            rho = (2*inv_h2) * max_c sum_faces D_f.
 *  op 2:     f_c = sum_f Q_f (w_nb - w_c) / h^2 with Q_f = (w_c^2 + w_nb^2)/2
 *            depends on w through Q_f as well, so the Jacobian row is
 *            d f_c / d w_c  = sum_f (w_c (w_nb - w_c) - Q_f) / h^2,
 *            d f_c / d w_nb = (w_nb (w_nb - w_c) + Q_f) / h^2
 *            (a Dirichlet ghost, w_nb = 0, is no unknown: it adds to the
 *            diagonal only), and rho = inv_h2 * max_c (|diag| + sum |off|),
 *            evaluated per face as dw = w_nb - w_c, Q = 0.5*(w_c*w_c + w_nb*w_nb),
 *            diag = diag + (w_c*dw - Q), off = off + fabs(w_nb*dw + Q).
 *  op 3:     adds the reaction rows: rho = (2*inv_h2) * (4d) + max_c
 *            max(|2vw - 4| + v^2, v^2 + |3 - 2vw|) (diagonal and coupling
 *            entries of each row).
 */
double oracle_rho_bound(int ndim, const long *n, int bc, int op, double inv_h2, double d_const,
                        const double *D, const double *w)
{
    grid_t g;
    if (make_grid(&g, ndim, n, bc, op, inv_h2, d_const)) return -1.0;
    /* the state-dependent bounds need the state, the variable one its D */
    if (((op == OP_POROUS2 || op == OP_BRUSS2) && !w) || (op == OP_VARCOEF && !D)) return -1.0;
    if (op == OP_ADVDIFF) {
        /* |a_ii| + sum_j |a_ij| with a_ii = -sum_f fc_f / h^2, a_ij = fc_f / h^2 */
        double sum = 0.0, asum = 0.0;
        for (int f = 0; f < 2 * ndim; ++f) {
            sum = sum + g.fc[f];
            asum = asum + fabs(g.fc[f]);
        }
        return (fabs(sum) + asum) * inv_h2;
    }
    long N = npts(&g);
    double m = 0.0;
    for (long p = 0; p < N; ++p) {
        long i[3];
        coords(&g, p, i);
        double sum = 0.0, diag = 0.0;
        for (int f = 0; f < 2 * ndim; ++f) {
            long q = neighbour(&g, i, f);
            double Df;
            if (op == OP_LAPLACE || op == OP_BRUSS2) {
                Df = d_const;
            } else if (op == OP_VARCOEF) {
                Df = 0.5 * D[p] + 0.5 * ((q < 0) ? D[p] : D[q]);
            } else {
                double un = (q < 0) ? 0.0 : w[q];
                double dw = un - w[p];
                double Q = 0.5 * (w[p] * w[p] + un * un);
                diag = diag + (w[p] * dw - Q);
                if (q >= 0) sum = sum + fabs(un * dw + Q);
                continue;
            }
            sum = sum + Df;
        }
        if (op == OP_POROUS2) sum = fabs(diag) + sum;
        if (sum > m) m = sum;
    }
    if (op == OP_BRUSS2) {
        double r = 0.0;
        for (long p = 0; p < N; ++p) {
            double v = w[p], x = w[N + p];
            double vx = v * x, v2 = v * v;
            double a = fabs(2.0 * vx - 4.0) + v2;
            double b = v2 + fabs(3.0 - 2.0 * vx);
            double c = a > b ? a : b;
            if (c > r) r = c;
        }
        return (2.0 * inv_h2) * m + r;
    }
    if (op == OP_POROUS2) return inv_h2 * m;
    return (2.0 * inv_h2) * m;
}

/*
 * One superstep of s stages on a complex state (Sec. 3, Euler-step equation with
 * complex W^0): (wr, wi) in, W^s out, every stage as in oracle_superstep. The A flows
 * of the split scheme of Sec. 4.1 start from complex states.
 */
int oracle_superstep_c(int ndim, const long *n, int bc, int op, double inv_h2, double d_const,
                       const double *D, int s, const double *tau_re, const double *tau_im,
                       double *wr, double *wi)
{
    grid_t g;
    if (make_grid(&g, ndim, n, bc, op, inv_h2, d_const)) return -1;
    long N = nstate(&g);
    double *fr = malloc(sizeof(double) * N), *fi = malloc(sizeof(double) * N);
    if (!fr || !fi) { free(fr); free(fi); return -2; }
    for (int l = 0; l < s; ++l) {
        apply_op(&g, D, wr, wi, fr, fi);
        double tr = tau_re[l], ti = tau_im[l];
#pragma omp parallel for schedule(static)
        for (long p = 0; p < N; ++p) {
            double nr = FMA(tr, fr[p], FMA(-ti, fi[p], wr[p]));
            double ni = FMA(tr, fi[p], FMA(ti, fr[p], wi[p]));
            wr[p] = nr;
            wi[p] = ni;
        }
    }
    free(fr); free(fi);
    return 0;
}

/*
 * Reaction flow of the two-species Brusselator (Sec. 3.1) over a complex time tau, the
 * B flow of the split scheme of Sec. 4.1: dY/ds = tau f_B(Y), s in [0, 1], with
 * f_B(v, w) = (1 - 4v + v^2 w, 3v - v^2 w) continued to complex v, w, by nsub classical
 * Runge-Kutta steps of length 1/nsub in s. The caller passes c = tau/nsub, c/2 and c/6
 * (re, im). Arithmetic in this order, no multiply-add fused:
 *   f:  v2 = (vr*vr - vi*vi, 2*(vr*vi)), q = v2 w = (v2r*wr - v2i*wi, v2r*wi + v2i*wr),
 *       fv = ((1 - 4*vr) + qr, qi - 4*vi), fw = (3*vr - qr, 3*vi - qi);
 *   y + c k = (yr + (cr*kr - ci*ki), yi + (cr*ki + ci*kr)) per species;
 *   k1 = f(y), k2 = f(y + (c/2) k1), k3 = f(y + (c/2) k2), k4 = f(y + c k3),
 *   y <- y + (c/6) (((k1 + 2 k2) + 2 k3) + k4).
 * State: v at [0, N), w at [N, 2N), real parts in zr, imaginary parts in zi.
 */
typedef struct { double vr, vi, wr, wi; } bz_t;

static bz_t bz_f(bz_t y)
{
    double v2r = y.vr * y.vr - y.vi * y.vi;
    double v2i = 2.0 * (y.vr * y.vi);
    double qr = v2r * y.wr - v2i * y.wi;
    double qi = v2r * y.wi + v2i * y.wr;
    bz_t f;
    f.vr = (1.0 - 4.0 * y.vr) + qr;
    f.vi = qi - 4.0 * y.vi;
    f.wr = 3.0 * y.vr - qr;
    f.wi = 3.0 * y.vi - qi;
    return f;
}

static bz_t bz_axpy(bz_t y, double cr, double ci, bz_t k)
{
    bz_t o;
    o.vr = y.vr + (cr * k.vr - ci * k.vi);
    o.vi = y.vi + (cr * k.vi + ci * k.vr);
    o.wr = y.wr + (cr * k.wr - ci * k.wi);
    o.wi = y.wi + (cr * k.wi + ci * k.wr);
    return o;
}

void oracle_react_flow(long N, double *zr, double *zi, double cr, double ci, double c2r,
                       double c2i, double c6r, double c6i, int nsub)
{
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; ++p) {
        bz_t y = {zr[p], zi[p], zr[N + p], zi[N + p]};
        for (int j = 0; j < nsub; ++j) {
            bz_t k1 = bz_f(y);
            bz_t k2 = bz_f(bz_axpy(y, c2r, c2i, k1));
            bz_t k3 = bz_f(bz_axpy(y, c2r, c2i, k2));
            bz_t k4 = bz_f(bz_axpy(y, cr, ci, k3));
            bz_t S;
            S.vr = ((k1.vr + 2.0 * k2.vr) + 2.0 * k3.vr) + k4.vr;
            S.vi = ((k1.vi + 2.0 * k2.vi) + 2.0 * k3.vi) + k4.vi;
            S.wr = ((k1.wr + 2.0 * k2.wr) + 2.0 * k3.wr) + k4.wr;
            S.wi = ((k1.wi + 2.0 * k2.wi) + 2.0 * k3.wi) + k4.wi;
            y = bz_axpy(y, c6r, c6i, S);
        }
        zr[p] = y.vr;
        zi[p] = y.vi;
        zr[N + p] = y.wr;
        zi[N + p] = y.wi;
    }
}

/* Threads the OpenMP loops above use (1 when built without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
#endif
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the OpenMP loops that follow (the CPU baseline times 1 and all). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
