// FRKC2 stepsizes on the host: roots of the damped second-order FRKC
// polynomial in the internal-stability order.
//
// O'Sullivan, arXiv:1702.03818:
//  * Sec. 2: the N = 2 FRKC polynomial is d0 + 2 d1 C_M(z) + 2 d2 C_2M(z)
//    (L = 2M) and a_l = 1 / (M^2 alpha_M (1 - zeta_l)) from its roots.
//    Maximising the real extent under the order conditions R'(0) = R''(0) = 1
//    gives d1 = 0 and alpha_M = (4 - 1/M^2)/3, so the roots solve
//    C_L(zeta) = -(2L^2 + 1)/(L^2 - 1):
//        zeta_j = cos(theta_j), theta_j = (pi (2j+1) + i eta)/L,
//        eta = arccosh((2L^2 + 1)/(L^2 - 1)),  M^2 alpha_M = (L^2 - 1)/3.
//  * Sec. 2.1: damping nu replaces a_l by
//        (1 - mu) / ((1 - nu) M^2 alpha_M ((1 - zeta_l) + 2 mu zeta_l)),
//    one mu for the M roots with C_M(zeta) = +i sinh(eta/2) (odd j) and its
//    conjugate for the others, fixed by Newton-Raphson on R'(0) = R''(0) = 1.
//  * Sec. 2.2: greedy ordering that keeps the estimate Qbar small on L
//    samples of [-betabar, 0], betabar = (1 - nC) beta, C = 1e-4, with n
//    increased until the realised Q is at most 10 L^2.
//
// Precision: roots and damping in IEEE binary128 (libquadmath), rounded once
// to FP64; the real extent is located by bisection on doubles with a
// binary128 test |R| <= 1; the ordering runs in FP64 log-magnitudes.
#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"

namespace frkc2 {
namespace {

typedef __float128 q_t;

struct qc {   // binary128 complex with the few operations the construction needs
    q_t re, im;
};
inline qc operator+(qc a, qc b) { return {a.re + b.re, a.im + b.im}; }
inline qc operator-(qc a, qc b) { return {a.re - b.re, a.im - b.im}; }
inline qc operator*(qc a, qc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline qc operator*(q_t a, qc b) { return {a * b.re, a * b.im}; }
inline qc operator/(qc a, qc b)
{
    q_t d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

const double kShrinkC = 1e-4;
const int kShrinkMax = 64;
const double kTieRel = 1e-12;

// Odd-j roots zeta_j and 1 - zeta_j = 2 sin^2(theta_j/2) (no cancellation).
void first_group_roots(int L, std::vector<qc> &zeta, std::vector<qc> &one_minus)
{
    q_t L2 = (q_t)L * (q_t)L;
    q_t eta = acoshq((2 * L2 + 1) / (L2 - 1));
    q_t v = eta / L;
    zeta.clear();
    one_minus.clear();
    for (int j = 1; j < L; j += 2) {
        q_t u = M_PIq * (2 * j + 1) / L;
        qc z = {cosq(u) * coshq(v), -sinq(u) * sinhq(v)};
        qc sh = {sinq(u / 2) * coshq(v / 2), cosq(u / 2) * sinhq(v / 2)};
        qc om = (q_t)2 * (sh * sh);
        zeta.push_back(z);
        one_minus.push_back(om);
    }
}

// Newton-Raphson for mu (Sec. 2.1); returns the first-group stepsizes.
std::vector<qc> damp(int L, double nu, qc &mu_out)
{
    std::vector<qc> z, om;
    first_group_roots(L, z, om);
    const size_t M = z.size();
    q_t K = (q_t)3 / (((q_t)1 - (q_t)nu) * ((q_t)L * (q_t)L - 1));
    qc mu = {0, 0};
    std::vector<qc> a(M), da(M);
    for (int it = 0; it < 100; ++it) {
        qc F = {0, 0}, G = {0, 0}, Fp = {0, 0}, Gp = {0, 0};
        for (size_t i = 0; i < M; ++i) {
            qc den = om[i] + (q_t)2 * (mu * z[i]);
            qc one = {1, 0};
            a[i] = K * ((one - mu) / den);
            da[i] = ((q_t)-1 * K) * ((one + z[i]) / (den * den));
            F = F + a[i];
            G = G + a[i] * a[i];
            Fp = Fp + da[i];
            Gp = Gp + (q_t)2 * (a[i] * da[i]);
        }
        // equations 2 Re F = 1, 2 Re G = 0; d Re H/d Re mu = Re H', d Re H/d Im mu = -Im H'
        q_t e1 = 2 * F.re - 1, e2 = 2 * G.re;
        q_t j11 = 2 * Fp.re, j12 = -2 * Fp.im, j21 = 2 * Gp.re, j22 = -2 * Gp.im;
        q_t det = j11 * j22 - j12 * j21;
        q_t dp = (e1 * j22 - j12 * e2) / det;
        q_t dq = (j11 * e2 - j21 * e1) / det;
        mu.re -= dp;
        mu.im -= dq;
        if (fabsq(dp) + fabsq(dq) <= 1e-30Q) break;
    }
    for (size_t i = 0; i < M; ++i) {
        qc one = {1, 0};
        a[i] = K * ((one - mu) / (om[i] + (q_t)2 * (mu * z[i])));
    }
    mu_out = mu;
    return a;
}

// sum over the first group of log|1 + a x| (|R(x)| = exp(2 * this) for real x)
double log_abs_half(const std::vector<double> &ar, const std::vector<double> &ai, double x)
{
    double s = 0.0;
    for (size_t i = 0; i < ar.size(); ++i) s += std::log(std::hypot(1.0 + ar[i] * x, ai[i] * x));
    return s;
}

bool stable_q(const std::vector<double> &ar, const std::vector<double> &ai, double b)
{
    q_t x = -(q_t)b, p = 1;
    for (size_t i = 0; i < ar.size(); ++i) {
        q_t re = 1 + (q_t)ar[i] * x, im = (q_t)ai[i] * x;
        p *= re * re + im * im;
    }
    return p <= 1 + 1e-20Q;
}

// Largest double b with |R(-x)| <= 1 on [0, b]: scan dense where C_L
// oscillates fastest (8 samples per half period in z, then past z = -1), then
// bisect on doubles with the binary128 test.
double real_extent(const std::vector<double> &ar, const std::vector<double> &ai, int L,
                   double beta0)
{
    std::vector<double> xs;
    for (int k = 1; k <= 8 * L; ++k) {
        double zk = std::cos((double)k * M_PI / (double)(8 * L));
        xs.push_back((zk - 1.0) * (beta0 / 2.0));
    }
    for (int j = 1; j <= 40; ++j) xs.push_back(-beta0 * (1.0 + 1e-3 * j));
    for (int j = 1; j <= 20; ++j) xs.push_back(-beta0 * (1.04 + 0.05 * j));   // past 1.04 beta0
    size_t i = 0;
    for (; i < xs.size(); ++i)
        if (2.0 * log_abs_half(ar, ai, xs[i]) > 1e-12) break;
    if (i == xs.size()) return -1.0;
    double lo = (i == 0) ? 0.0 : -xs[i - 1];
    double hi = -xs[i];
    for (;;) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (stable_q(ar, ai, mid)) lo = mid; else hi = mid;
    }
    return lo;
}

// Greedy order of the first group on Qbar (Sec. 2.2). Returns indices.
std::vector<int> greedy(const std::vector<double> &ar, const std::vector<double> &ai,
                        double beta_bar, int L)
{
    const int M = (int)ar.size();
    std::vector<double> lv((size_t)M * L);
    for (int k = 1; k <= L; ++k) {
        double x = -(beta_bar * (double)k) / (double)L;
        for (int j = 0; j < M; ++j)
            lv[(size_t)j * L + (k - 1)] = std::log(std::hypot(1.0 + ar[j] * x, ai[j] * x));
    }
    std::vector<double> placed(L, 0.0), rest(L);
    std::vector<int> S(M), order;
    for (int j = 0; j < M; ++j) S[j] = j;
    std::vector<double> score;
    for (int step = 0; step < M; ++step) {
        std::fill(rest.begin(), rest.end(), 0.0);
        for (int c : S)
            for (int k = 0; k < L; ++k) rest[k] += lv[(size_t)c * L + k];
        score.assign(S.size(), 0.0);
        double m = INFINITY;
        for (size_t ci = 0; ci < S.size(); ++ci) {
            const double *v = &lv[(size_t)S[ci] * L];
            double sc = 0.0;
            for (int k = 0; k < L; ++k) {
                double pre = placed[k] + v[k], suf = rest[k] - v[k];
                sc += std::exp(pre > suf ? pre : suf);
            }
            score[ci] = sc;
            if (sc < m) m = sc;
        }
        size_t pick = 0;
        while (!(score[pick] <= m * (1.0 + kTieRel))) ++pick;
        int c = S[pick];
        S.erase(S.begin() + pick);
        order.push_back(c);
        for (int k = 0; k < L; ++k) placed[k] += lv[(size_t)c * L + k];
    }
    return order;
}

// Realised Q: max over x on max(4000, 10 L) points of [-beta, 0] of the best
// contiguous run of log|1 + a_l x| (Kadane).
double realised_q(const std::vector<std::complex<double>> &seq, double beta, int L)
{
    int G = std::max(4000, 10 * L);
    double step = (0.0 - (-beta)) / (double)(G - 1);
    double best = -INFINITY;
    for (int g = 0; g < G; ++g) {
        double x = (g == G - 1) ? 0.0 : -beta + (double)g * step;
        double cur = 0.0, bx = -INFINITY;
        for (size_t l = 0; l < seq.size(); ++l) {
            double t = std::log(std::abs(1.0 + seq[l] * x));
            cur = std::max(t, cur + t);
            bx = std::max(bx, cur);
        }
        best = std::max(best, bx);
    }
    return std::exp(best);
}

struct Entry {
    std::vector<double> re, im;
    frkc2_coeff_info info;
    int status;
};

std::mutex g_mu;
std::map<std::pair<int, double>, Entry> g_cache;

Entry compute(int s, double nu)
{
    const int L = s;
    Entry e;
    qc mu;
    std::vector<qc> aq = damp(L, nu, mu);
    std::vector<double> ar(aq.size()), ai(aq.size());
    for (size_t i = 0; i < aq.size(); ++i) {
        ar[i] = (double)aq[i].re;
        ai[i] = (double)aq[i].im;
    }
    double beta = real_extent(ar, ai, L, 2.0 * (double)(L * L - 1) / 3.0);
    double bound = 10.0 * (double)L * (double)L;
    double best_q = INFINITY, best_bb = 0.0;
    int best_n = 0;
    std::vector<std::complex<double>> best_seq;
    for (int n = 1; n <= kShrinkMax; ++n) {
        double beta_bar = (1.0 - n * kShrinkC) * beta;
        std::vector<int> ord = greedy(ar, ai, beta_bar, L);
        std::vector<std::complex<double>> seq;
        for (int j : ord) seq.emplace_back(ar[j], ai[j]);
        for (int j : ord) seq.emplace_back(ar[j], -ai[j]);
        double q = realised_q(seq, beta, L);
        if (q < best_q) {
            best_q = q;
            best_n = n;
            best_bb = beta_bar;
            best_seq = seq;
        }
        if (q <= bound) break;
    }
    for (auto &c : best_seq) {
        e.re.push_back(c.real());
        e.im.push_back(c.imag());
    }
    e.info.beta = beta;
    e.info.beta_bar = best_bb;
    e.info.q_realised = best_q;
    e.info.mu_re = (double)mu.re;
    e.info.mu_im = (double)mu.im;
    e.info.n_shrink = best_n;
    e.info.q_bound_met = best_q <= bound;
    e.status = e.info.q_bound_met ? FRKC2_OK : FRKC2_WQBOUND;
    return e;
}

// ---- Fourth order (N = 4), the A flows of the split scheme (Sec. 4.1) ----
//
// R(x) = P(C_M(z)) / P(1), z = 1 + x / (M^2 alpha_M), P of degree 4 in y = C_M(z).
// For a given alpha_M the four order conditions R^(n)(0) = 1 fix the
// derivatives p_k = P^(k)(1) / P(1) (chain rule for P(g(x)) with
// g^(n)(0) = C_M^(n)(1) / (M^2 alpha_M)^n, C_M^(n)(1) = prod_{j<n} (M^2 - j^2)/(2j+1)).
// |R| <= 1 on [-2 M^2 alpha_M, 0] iff |P| <= 1 on [-1, 1]; alpha_M is taken
// with P(-1) = 1 - 4 nu (damping: the marginal real-axis points keep
// |R| = 1 - 4 nu). Stepsizes from the roots: C_M(zeta) = y for each root y
// of P, zeta = cos((acos(y) + 2 pi j)/M), a = 1/(M^2 alpha_M (1 - zeta)).

void taylor_p4(int M, q_t alpha, q_t p[4])
{
    q_t c[4], v = 1;
    for (int j = 0; j < 4; ++j) {
        v = v * ((q_t)M * (q_t)M - (q_t)(j * j)) / (q_t)(2 * j + 1);
        c[j] = v;
    }
    const q_t sc = (q_t)M * (q_t)M * alpha;
    q_t g[4];
    q_t pw = sc;
    for (int k = 0; k < 4; ++k) {
        g[k] = c[k] / pw;
        pw = pw * sc;
    }
    const q_t g1 = g[0];
    p[0] = 1 / g1;
    p[1] = (1 - p[0] * g[1]) / (g1 * g1);
    p[2] = (1 - 3 * p[1] * g1 * g[1] - p[0] * g[2]) / (g1 * g1 * g1);
    p[3] = (1 - 6 * p[2] * g1 * g1 * g[1] - p[1] * (3 * g[1] * g[1] + 4 * g1 * g[2]) - p[0] * g[3]) /
           (g1 * g1 * g1 * g1);
}

// coefficients of y^0 .. y^4 of P(y) = 1 + sum_k p_k (y - 1)^k / k!
void poly4(int M, q_t alpha, q_t coef[5])
{
    q_t p[4];
    taylor_p4(M, alpha, p);
    for (int j = 0; j < 5; ++j) coef[j] = 0;
    coef[0] = 1;
    q_t fact = 1;
    for (int k = 1; k <= 4; ++k) {
        fact *= k;
        q_t binom = 1;   // C(k, j)
        for (int j = 0; j <= k; ++j) {
            const q_t sign = ((k - j) % 2) ? -1 : 1;
            coef[j] += p[k - 1] / fact * binom * sign;
            binom = binom * (q_t)(k - j) / (q_t)(j + 1);
        }
    }
}

q_t p_minus1(int M, q_t alpha)
{
    q_t p[4];
    taylor_p4(M, alpha, p);
    q_t v = 1, fact = 1, pw = 1;
    for (int k = 1; k <= 4; ++k) {
        fact *= k;
        pw *= -2;
        v += p[k - 1] * pw / fact;
    }
    return v;
}

// alpha_M with P(-1) = 1 - 4 nu by bisection on [0.5, 3]; < 0 if not bracketed
q_t alpha4(int M, double nu)
{
    const q_t target = 1 - 4 * (q_t)nu;
    q_t lo = 0.5Q, hi = 3;
    if (!(p_minus1(M, lo) - target < 0 && p_minus1(M, hi) - target > 0)) return -1;
    for (int it = 0; it < 200; ++it) {
        q_t mid = (lo + hi) / 2;
        if (p_minus1(M, mid) - target < 0) lo = mid; else hi = mid;
    }
    return (lo + hi) / 2;
}

qc poly_eval(const q_t c[5], qc z)
{
    qc v = {c[4], 0};
    for (int j = 3; j >= 0; --j) v = v * z + qc{c[j], 0};
    return v;
}

qc poly_deriv(const q_t c[5], qc z)
{
    qc v = {4 * c[4], 0};
    for (int j = 3; j >= 1; --j) v = v * z + qc{(q_t)j * c[j], 0};
    return v;
}

// the four roots of c4 y^4 + ... + c0: Weierstrass (Durand-Kerner) iteration,
// then Newton steps on each root
void quartic_roots(const q_t c[5], qc r[4])
{
    const qc seed = {0.4Q, 0.9Q};
    qc z = {1, 0};
    for (int i = 0; i < 4; ++i) {
        r[i] = z;
        z = z * seed;
    }
    for (int it = 0; it < 500; ++it) {
        q_t change = 0;
        for (int i = 0; i < 4; ++i) {
            qc den = {c[4], 0};
            for (int j = 0; j < 4; ++j)
                if (j != i) den = den * (r[i] - r[j]);
            qc d = poly_eval(c, r[i]) / den;
            r[i] = r[i] - d;
            change += fabsq(d.re) + fabsq(d.im);
        }
        if (change < 1e-33Q) break;
    }
    for (int i = 0; i < 4; ++i)
        for (int it = 0; it < 4; ++it) r[i] = r[i] - poly_eval(c, r[i]) / poly_deriv(c, r[i]);
}

qc q_cos(qc t) { return {cosq(t.re) * coshq(t.im), -sinq(t.re) * sinhq(t.im)}; }
qc q_sin(qc t) { return {sinq(t.re) * coshq(t.im), cosq(t.re) * sinhq(t.im)}; }

// principal acos(y): the double-precision value refined by Newton on cos(t) = y
qc q_acos(qc y)
{
    std::complex<double> t0 = std::acos(std::complex<double>((double)y.re, (double)y.im));
    qc t = {(q_t)t0.real(), (q_t)t0.imag()};
    for (int it = 0; it < 8; ++it) {
        qc s = q_sin(t);
        t = t + (q_cos(t) - y) / s;   // t - (cos t - y) / (-sin t)
    }
    return t;
}

// stepsizes from the two roots of P with Im y > 0 (sorted by real, then imaginary part)
std::vector<qc> half_group4(int M, double nu, q_t &alpha)
{
    std::vector<qc> a;
    alpha = alpha4(M, nu);
    if (!(alpha > 0)) return a;
    q_t c[5];
    poly4(M, alpha, c);
    qc r[4];
    quartic_roots(c, r);
    std::vector<qc> up;
    for (int i = 0; i < 4; ++i)
        if (r[i].im > 0) up.push_back(r[i]);
    if (up.size() != 2) return a;
    if (up[1].re < up[0].re || (up[1].re == up[0].re && up[1].im < up[0].im)) std::swap(up[0], up[1]);
    const q_t sc = (q_t)M * (q_t)M * alpha;
    for (const qc &y : up) {
        const qc th0 = q_acos(y);
        for (int j = 0; j < M; ++j) {
            const qc th = {(th0.re + 2 * M_PIq * (q_t)j) / (q_t)M, th0.im / (q_t)M};
            const qc sh = q_sin(qc{th.re / 2, th.im / 2});
            const qc om = (q_t)2 * (sh * sh);
            a.push_back(qc{1, 0} / (sc * om));
        }
    }
    return a;
}

Entry compute4(int s, double nu)
{
    const int L = s, M = s / 4;
    Entry e;
    q_t alpha;
    std::vector<qc> aq = half_group4(M, nu, alpha);
    if (aq.empty()) {
        e.info.beta = -1.0;
        e.status = FRKC2_EINVAL;
        return e;
    }
    std::vector<double> ar(aq.size()), ai(aq.size());
    for (size_t i = 0; i < aq.size(); ++i) {
        ar[i] = (double)aq[i].re;
        ai[i] = (double)aq[i].im;
    }
    const double alpha_d = (double)alpha;
    double beta = real_extent(ar, ai, L, 2.0 * (double)M * (double)M * alpha_d);
    double bound = 10.0 * (double)L * (double)L;
    double best_q = INFINITY, best_bb = 0.0;
    int best_n = 0;
    std::vector<std::complex<double>> best_seq;
    for (int n = 1; n <= kShrinkMax; ++n) {
        double beta_bar = (1.0 - n * kShrinkC) * beta;
        std::vector<int> ord = greedy(ar, ai, beta_bar, L);
        std::vector<std::complex<double>> seq;
        for (int j : ord) seq.emplace_back(ar[j], ai[j]);
        for (int j : ord) seq.emplace_back(ar[j], -ai[j]);
        double q = realised_q(seq, beta, L);
        if (q < best_q) {
            best_q = q;
            best_n = n;
            best_bb = beta_bar;
            best_seq = seq;
        }
        if (q <= bound) break;
    }
    for (auto &c : best_seq) {
        e.re.push_back(c.real());
        e.im.push_back(c.imag());
    }
    e.info.beta = beta;
    e.info.beta_bar = best_bb;
    e.info.q_realised = best_q;
    e.info.mu_re = alpha_d;
    e.info.mu_im = 0.0;
    e.info.n_shrink = best_n;
    e.info.q_bound_met = best_q <= bound;
    e.status = e.info.q_bound_met ? FRKC2_OK : FRKC2_WQBOUND;
    return e;
}

std::map<std::pair<int, double>, Entry> g_cache4;

}  // namespace

int coeffs4_cached(int s, double nu, const double **re, const double **im, frkc2_coeff_info *info)
{
    if (s < 4 || s > kMaxStages4 || (s % 4) != 0) {
        set_error("frkc4_coeffs: s must be a multiple of 4 with 4 <= s <= %d (got %d)",
                  kMaxStages4, s);
        return FRKC2_EINVAL;
    }
    if (!(nu >= 0.0 && nu < 0.25)) {
        set_error("frkc4_coeffs: nu must lie in [0, 0.25) (got %g)", nu);
        return FRKC2_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(s, nu);
    auto it = g_cache4.find(key);
    if (it == g_cache4.end()) it = g_cache4.emplace(key, compute4(s, nu)).first;
    if (it->second.info.beta <= 0.0) {
        set_error("frkc4_coeffs: construction failed for s=%d", s);
        return FRKC2_EINVAL;
    }
    if (re) *re = it->second.re.data();
    if (im) *im = it->second.im.data();
    if (info) *info = it->second.info;
    return it->second.status;
}

int coeffs_cached(int s, double nu, const double **re, const double **im, frkc2_coeff_info *info)
{
    if (s < 2 || s > kMaxStages || (s % 2) != 0) {
        set_error("frkc2_coeffs: s must be even with 2 <= s <= 514 (got %d)", s);
        return FRKC2_EINVAL;
    }
    if (!(nu >= 0.0 && nu < 1.0)) {
        set_error("frkc2_coeffs: nu must lie in [0, 1) (got %g)", nu);
        return FRKC2_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(s, nu);
    auto it = g_cache.find(key);
    if (it == g_cache.end()) it = g_cache.emplace(key, compute(s, nu)).first;
    if (it->second.info.beta <= 0.0) {
        set_error("frkc2_coeffs: no end of the stability interval found for s=%d", s);
        return FRKC2_EINVAL;
    }
    if (re) *re = it->second.re.data();
    if (im) *im = it->second.im.data();
    if (info) *info = it->second.info;
    return it->second.status;
}

}  // namespace frkc2

extern "C" int frkc2_coeffs(int s, double nu, double *a_re, double *a_im, frkc2_coeff_info *info)
{
    const double *re = nullptr, *im = nullptr;
    int rc = frkc2::coeffs_cached(s, nu, &re, &im, info);
    if (rc < 0) return rc;
    if (a_re) std::memcpy(a_re, re, sizeof(double) * (size_t)s);
    if (a_im) std::memcpy(a_im, im, sizeof(double) * (size_t)s);
    return rc;
}

extern "C" int frkc4_coeffs(int s, double nu, double *a_re, double *a_im, frkc2_coeff_info *info)
{
    const double *re = nullptr, *im = nullptr;
    int rc = frkc2::coeffs4_cached(s, nu, &re, &im, info);
    if (rc < 0) return rc;
    if (a_re) std::memcpy(a_re, re, sizeof(double) * (size_t)s);
    if (a_im) std::memcpy(a_im, im, sizeof(double) * (size_t)s);
    return rc;
}

extern "C" int frkc2_write_table(const char *path, double nu, int m_max)
{
    if (!path || m_max < 1 || m_max > frkc2::kMaxStages / 2) {
        frkc2::set_error("write_table: need a path and 1 <= m_max <= %d", frkc2::kMaxStages / 2);
        return FRKC2_EINVAL;
    }
    if (!(nu >= 0.0 && nu < 1.0)) {
        frkc2::set_error("write_table: nu must lie in [0, 1) (got %g)", nu);
        return FRKC2_EINVAL;
    }
    // generate everything first, so a bad entry leaves no partial file
    std::vector<const double *> re(m_max + 1), im(m_max + 1);
    std::vector<frkc2_coeff_info> info(m_max + 1);
    for (int M = 1; M <= m_max; ++M) {
        const int rc = frkc2::coeffs_cached(2 * M, nu, &re[M], &im[M], &info[M]);
        if (rc < 0) return rc;
    }
    FILE *f = std::fopen(path, "w");
    if (!f) {
        frkc2::set_error("write_table: cannot open %s for writing", path);
        return FRKC2_EINVAL;
    }
    for (int M = 1; M <= m_max; ++M) {
        std::fprintf(f, "%.17g %.17g\n", info[M].beta_bar, info[M].q_realised);
        for (int part = 0; part < 2; ++part) {
            const double *a = part ? im[M] : re[M];
            for (int l = 0; l < 2 * M; ++l) std::fprintf(f, l ? " %.17g" : "%.17g", a[l]);
            std::fputc('\n', f);
        }
    }
    const bool bad = std::ferror(f) != 0;
    if (std::fclose(f) != 0 || bad) {
        frkc2::set_error("write_table: write to %s failed", path);
        return FRKC2_EINVAL;
    }
    return FRKC2_OK;
}
