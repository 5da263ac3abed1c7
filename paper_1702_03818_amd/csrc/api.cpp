// Host orchestration and C ABI of libfrkc2 (declarations and contracts in
// include/frkc2.h).
//
// A superstep (O'Sullivan, arXiv:1702.03818, Sec. 3) is s stage launches on
// the caller's stream: the first reads the real state w, the last writes Re W^L
// back into w, the ones between ping-pong two complex workspace buffers. The
// stepsizes tau_l = T a_l are formed here in FP64 and passed by value. The
// stability requirement T rho <= betabar (Sec. 2, |R| <= 1 on the spectrum)
// is checked against a Gershgorin bound computed on the GPU.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace frkc2 {

namespace {
thread_local char g_err[512] = "";
int g_tblock = 0;
int g_tile = 0;
int g_zchunk = 0;
int g_adj_stages = 0;   // reverse stages per pass of the adjoint: 0 automatic, 1, 2

constexpr size_t kAlign = 256;
constexpr size_t kScratch = 64 * 1024;   // reduction partials + stepsize table

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int hip_fail(hipError_t e, const char *what)
{
    set_error("%s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
    return FRKC2_EHIP;
}

#define HIP_TRY(expr, what)                                   \
    do {                                                      \
        hipError_t e_ = (hipError_t)(expr);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what);      \
    } while (0)

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Operators whose Jacobian (and so the Gershgorin bound) depends on the state.
bool nonlinear(const KGrid &kg)
{
    return kg.op == FRKC2_OP_POROUS2 || kg.op == FRKC2_OP_BRUSS2;
}

}  // namespace

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

bool make_kgrid(const frkc2_grid *g, KGrid &k)
{
    if (!g) {
        set_error("grid is NULL");
        return false;
    }
    if (g->ndim < 1 || g->ndim > 3) {
        set_error("ndim must be 1, 2 or 3 (got %d)", g->ndim);
        return false;
    }
    for (int d = 0; d < 3; ++d) {
        const int n = g->n[d];
        if (d < g->ndim ? n < 1 : n != 1) {
            set_error("n[%d] = %d invalid (used dimensions >= 1, unused = 1)", d, n);
            return false;
        }
    }
    if (!(g->h > 0.0) || !std::isfinite(g->h)) {
        set_error("h must be positive and finite");
        return false;
    }
    if (g->bc != FRKC2_BC_PERIODIC && g->bc != FRKC2_BC_DIRICHLET0) {
        set_error("unknown boundary condition %d", g->bc);
        return false;
    }
    if (g->op != FRKC2_OP_LAPLACE && g->op != FRKC2_OP_VARCOEF && g->op != FRKC2_OP_POROUS2 &&
        g->op != FRKC2_OP_BRUSS2 && g->op != FRKC2_OP_ADVDIFF) {
        set_error("unknown operator %d", g->op);
        return false;
    }
    if ((g->op == FRKC2_OP_LAPLACE || g->op == FRKC2_OP_BRUSS2 || g->op == FRKC2_OP_ADVDIFF) &&
        !(g->d_const >= 0.0 && std::isfinite(g->d_const))) {
        set_error("d_const must be finite and non-negative");
        return false;
    }
    if (g->op == FRKC2_OP_BRUSS2 && (g->ndim != 2 || g->bc != FRKC2_BC_PERIODIC)) {
        set_error("the Brusselator runs on periodic 2D grids");
        return false;
    }
    const long long N = (long long)g->n[0] * g->n[1] * g->n[2];
    if (N > (1LL << 34)) {
        set_error("grid too large");
        return false;
    }
    k.ndim = g->ndim;
    k.bc = g->bc;
    k.op = g->op;
    k.nfield = (g->op == FRKC2_OP_BRUSS2) ? 2 : 1;
    k.inv_h2 = 1.0 / (g->h * g->h);
    k.d_const = g->d_const;
    // face coefficients: d, or d + (0.5 h) v_k / d - (0.5 h) v_k for ADVDIFF,
    // in the caller's dimension order and in the kernels' (2D grids march in z)
    for (int f = 0; f < 6; ++f) k.fcg[f] = g->d_const;
    if (g->op == FRKC2_OP_ADVDIFF) {
        for (int d = 0; d < g->ndim; ++d) {
            if (!std::isfinite(g->vel[d])) {
                set_error("vel must be finite");
                return false;
            }
            k.fcg[2 * d] = g->d_const + (0.5 * g->h) * g->vel[d];
            k.fcg[2 * d + 1] = g->d_const - (0.5 * g->h) * g->vel[d];
        }
    }
    for (int f = 0; f < 6; ++f) k.fc[f] = g->d_const;
    const int kd[3] = {0, g->ndim == 2 ? 2 : 1, 2};   // kernel dimension of caller dimension d
    for (int d = 0; d < g->ndim; ++d) {
        k.fc[2 * kd[d]] = k.fcg[2 * d];
        k.fc[2 * kd[d] + 1] = k.fcg[2 * d + 1];
    }
    if (g->ndim == 1) { k.nx = g->n[0]; k.ny = 1; k.nz = 1; }
    else if (g->ndim == 2) { k.nx = g->n[0]; k.ny = 1; k.nz = g->n[1]; }
    else { k.nx = g->n[0]; k.ny = g->n[1]; k.nz = g->n[2]; }
    return true;
}

namespace {

struct StepLayout {
    size_t bufA, bufB, scratch, total;
};

StepLayout step_layout(long long N)
{
    StepLayout L;
    const size_t cbytes = align_up((size_t)N * 16);
    L.bufA = 0;
    L.bufB = cbytes;
    L.scratch = 2 * cbytes;
    L.total = L.scratch + kScratch;
    return L;
}

struct AdaptLayout {
    size_t bufA, bufB, embA, embB, scratch, total;
};

AdaptLayout adapt_layout(long long N)
{
    AdaptLayout L;
    const size_t cbytes = align_up((size_t)N * 16), rbytes = align_up((size_t)N * 8);
    L.bufA = 0;
    L.bufB = cbytes;
    L.embA = 2 * cbytes;
    L.embB = L.embA + rbytes;
    L.scratch = L.embB + rbytes;
    L.total = L.scratch + kScratch;
    return L;
}

struct AdjLayout {
    size_t store, lamA, lamB, gD, scratch, total;
};

// s == 0: no stage store (frkc2_step_adjoint_stored, whose caller holds the
// stages)
AdjLayout adj_layout(long long N, int s)
{
    AdjLayout L;
    const size_t cbytes = align_up((size_t)N * 16);
    L.store = 0;
    L.lamA = (size_t)s * cbytes;
    L.lamB = L.lamA + cbytes;
    L.gD = L.lamB + cbytes;
    L.scratch = L.gD + align_up((size_t)N * 8);
    L.total = L.scratch + kScratch;
    return L;
}

// Gershgorin bound on the Jacobian of f: (2/h^2) max_c sum_f D_f for the linear
// operators, (1/h^2) max_c (|diag| + sum |off|) of the state-dependent rows for
// POROUS2, plus the reaction rows for BRUSS2; synchronises st.
int rho_bound_impl(const KGrid &kg, const double *w, const double *D, double *partials,
                   double *rho, hipStream_t st)
{
    if (kg.op == FRKC2_OP_ADVDIFF) {
        // |a_ii| + sum_j |a_ij|, a_ii = -sum_f c_f / h^2, a_ij = c_f / h^2
        double sum = 0.0, asum = 0.0;
        for (int f = 0; f < 2 * kg.ndim; ++f) {
            sum = sum + kg.fcg[f];
            asum = asum + std::fabs(kg.fcg[f]);
        }
        *rho = (std::fabs(sum) + asum) * kg.inv_h2;
        return FRKC2_OK;
    }
    double m;
    if (kg.op == FRKC2_OP_LAPLACE || kg.op == FRKC2_OP_BRUSS2) {
        double sum = 0.0;
        for (int f = 0; f < 2 * kg.ndim; ++f) sum = sum + kg.d_const;
        m = sum;
    } else {
        HIP_TRY(launch_rho(kg, w, D, partials, st), "rho bound launch");
        HIP_TRY(hipMemcpyAsync(&m, partials + kReduceBlocks, sizeof(double), hipMemcpyDeviceToHost,
                               st),
                "rho bound copy");
        HIP_TRY(hipStreamSynchronize(st), "rho bound");
    }
    *rho = (kg.op == FRKC2_OP_POROUS2) ? kg.inv_h2 * m : (2.0 * kg.inv_h2) * m;
    if (kg.op == FRKC2_OP_BRUSS2) {
        // reaction rows of the Jacobian (diagonal and species coupling)
        double r = 0.0;
        HIP_TRY(launch_bruss_react_max(kg, w, partials, st), "rho bound launch");
        HIP_TRY(launch_max_partials(partials, st), "rho bound launch");
        HIP_TRY(hipMemcpyAsync(&r, partials + kReduceBlocks, sizeof(double), hipMemcpyDeviceToHost,
                               st),
                "rho bound copy");
        HIP_TRY(hipStreamSynchronize(st), "rho bound");
        *rho = *rho + r;
    }
    if (!std::isfinite(*rho)) {
        set_error("Gershgorin bound is not finite");
        return FRKC2_ENONFINITE;
    }
    return FRKC2_OK;
}

// Launch configuration of a superstep's passes: stages fused per pass, tile
// shape and z planes per workgroup (0 = automatic).
struct PassCfg {
    int k, tile, zchunk;
};

// Configurations measured by frkc2_autotune, per grid shape and operator.
struct TuneEntry {
    int ndim, op, bc, nx, ny, nz;
    PassCfg cfg;
};
std::vector<TuneEntry> g_tuned;
std::mutex g_tune_mu;

bool same_shape(const TuneEntry &e, const KGrid &kg)
{
    return e.ndim == kg.ndim && e.op == kg.op && e.bc == kg.bc && e.nx == kg.nx &&
           e.ny == kg.ny && e.nz == kg.nz;
}

bool lookup_tuned(const KGrid &kg, PassCfg &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry &e : g_tuned)
        if (same_shape(e, kg)) {
            c = e.cfg;
            return true;
        }
    return false;
}

void store_tuned(const KGrid &kg, const PassCfg &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (TuneEntry &e : g_tuned)
        if (same_shape(e, kg)) {
            e.cfg = c;
            return;
        }
    g_tuned.push_back(TuneEntry{kg.ndim, kg.op, kg.bc, kg.nx, kg.ny, kg.nz, c});
}

// Measured best depth per dimension when nothing else is known (3D: K = 3
// with full-width tiles beat K = 2 by 2-3 % at 128^3 and 256^3; 2D rows have
// little halo overhead and take K = 4).
int default_depth(const KGrid &kg) { return (kg.ndim == 3) ? 3 : (kg.ndim == 2 ? 4 : 1); }

// Tile shapes as the launchers number them (the option's value minus one):
// 3D 0 = 64x16 extended columns, 1 = 64x32, 2 = 64x32 / 64x24 with 512
// threads, 3 = 64-column output rows with halo wavefronts, 4 = the same with
// 32-column rows, two per wavefront; 2D 0 = rows of 256, 1 = rows of 512.
// The 3D default is the full-width tile whose width the pass-time model
// prefers for this grid.
int default_tile(const KGrid &kg)
{
    if (kg.ndim != 3 || !tb3d_plane_ok(kg)) return 0;
    return tb3d_pick_cols(kg, default_depth(kg)) == 32 ? 4 : 3;
}

// The options if the depth is set, else the tuned entry for this grid, else
// the default depth with the tile and chunk options.
PassCfg pass_cfg(const KGrid &kg)
{
    PassCfg c{g_tblock, g_tile > 0 ? g_tile - 1 : default_tile(kg), g_zchunk};
    if (c.k == 0) {
        if (lookup_tuned(kg, c)) return c;
        c.k = default_depth(kg);
    }
    if (c.k >= 2 && !tblock_supported(kg, c.k)) c.k = 1;
    return c;
}

// One superstep of s stages from the real state w: passes of k fused stages,
// the remainder as single stages. The first pass reads w, the last writes
// Re W^L to w (or, with last_complex, the complex W^L to a buffer, returned).
int run_superstep(const KGrid &kg, const PassCfg &cfg, double *w, const double *D, double Tn,
                  const double *are, const double *aim, int s, bool last_complex,
                  double *const buf[2], const double **last_out, hipStream_t st)
{
    const int k = cfg.k;
    int l = 0, pass = 0;
    const double *in = nullptr;
    while (l < s) {
        // passes of k stages; a remainder of r >= 2 stages as one pass of
        // depth r where the tile supports it
        int kk = (k >= 2 && s - l >= k) ? k : 1;
        // a pass that would leave one stage leaves two: a lone stage is a
        // whole-grid pass of its own, about twice the time of a fused stage
        if (kk >= 3 && s - l - kk == 1 && tblock_supported(kg, kk - 1)) kk -= 1;
        if (kk == 1 && k > 2 && s - l >= 2 && tblock_supported(kg, s - l)) kk = s - l;
        // A fused pass reads its input around each tile and chunk (halo), so it
        // must not write into the array it reads: the pass that starts from w
        // may not also be the one that writes w back.
        if (l == 0 && kk == s) {
            kk = s - 1;
            while (kk >= 2 && !tblock_supported(kg, kk)) --kk;
        }
        PassArgs pa{};
        pa.k = kk;
        pa.zchunk = cfg.zchunk;
        pa.D = D;
        if (l == 0) pa.in_re = w;
        else pa.in_c = in;
        const bool last = (l + kk == s);
        double *out = buf[pass & 1];
        if (last && !last_complex) pa.out_re = w;
        else pa.out_c = out;
        for (int i = 0; i < kk; ++i) {
            pa.tr[i] = Tn * are[l + i];
            pa.ti[i] = Tn * aim[l + i];
        }
        // consecutive fused passes march in opposite directions, so that each
        // starts on the planes the one before touched last (still cached)
        pa.rev = pass & 1;
        const int rc = (kk == 1) ? launch_pass(kg, pa, 1, st) : launch_tblock(kg, pa, cfg.tile, st);
        if (rc != 0) return rc;
        in = out;
        l += kk;
        ++pass;
    }
    if (last_out) *last_out = in;
    return 0;
}

bool check_s_nu(int s, double nu)
{
    if (s < 2 || s > kMaxStages || (s % 2) != 0) {
        set_error("s must be even with 2 <= s <= 514 (got %d)", s);
        return false;
    }
    if (!(nu >= 0.0 && nu < 1.0)) {
        set_error("nu must lie in [0, 1) (got %g)", nu);
        return false;
    }
    return true;
}

}  // namespace


}  // namespace frkc2

using namespace frkc2;

extern "C" const char *frkc2_last_error(void) { return g_err; }

extern "C" const char *frkc2_version(void) { return "frkc2-mi355x 0.1 (gfx950, fp64)"; }

extern "C" int frkc2_set_option(int key, int value)
{
    if (key == FRKC2_OPT_TBLOCK) {
        if (value < 0 || value > kMaxTBlock) {
            set_error("temporal block depth must lie in [0, %d]", kMaxTBlock);
            return FRKC2_EINVAL;
        }
        g_tblock = value;
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_TILE) {
        if (value < 0 || value > 5) {
            set_error("tile shape must lie in [0, 5]");
            return FRKC2_EINVAL;
        }
        g_tile = value;
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_ZCHUNK) {
        if (value < 0 || value > (1 << 20)) {
            set_error("z chunk length must lie in [0, 2^20]");
            return FRKC2_EINVAL;
        }
        g_zchunk = value;
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_CLEAR_TUNED) {
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned.clear();
        }
        batched_clear_tuned();
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_ADJ_STAGES) {
        if (value < 0 || value > 2) {
            set_error("adjoint stages per pass must be 0 (automatic), 1 or 2");
            return FRKC2_EINVAL;
        }
        g_adj_stages = value;
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_BATCH_K3 || key == FRKC2_OPT_BATCH_COLS || key == FRKC2_OPT_BATCH_K2)
        return batched_set_option(key, value);
    set_error("unknown option %d", key);
    return FRKC2_EINVAL;
}

extern "C" size_t frkc2_workspace_bytes(const frkc2_grid *g, int s, int flags)
{
    KGrid kg;
    if (!make_kgrid(g, kg)) return 0;
    if (flags == FRKC2_WS_ADJOINT) {
        if (s < 2 || s > kMaxStages || (s % 2)) return 0;
        return adj_layout(kg.npts(), s).total;
    }
    if (flags == FRKC2_WS_ADJOINT_STORED) return adj_layout(kg.npts(), 0).total;
    if (flags == FRKC2_WS_STAGES) {
        if (s < 2 || s > kMaxStages || (s % 2)) return 0;
        return (size_t)s * align_up((size_t)kg.npts() * 16);
    }
    if (flags == FRKC2_WS_ADAPT) return adapt_layout(kg.nstate()).total;
    return step_layout(kg.nstate()).total;
}

extern "C" int frkc2_rho_bound(const frkc2_grid *g, const double *w, const double *D, double *rho,
                               void *ws, size_t ws_bytes, hipStream_t st)
{
    KGrid kg;
    if (!make_kgrid(g, kg)) return FRKC2_EINVAL;
    if (!rho) {
        set_error("rho is NULL");
        return FRKC2_EINVAL;
    }
    if (kg.op == FRKC2_OP_VARCOEF && !D) {
        set_error("VARCOEF needs D");
        return FRKC2_EINVAL;
    }
    if ((kg.op == FRKC2_OP_POROUS2 || kg.op == FRKC2_OP_BRUSS2) && !w) {
        set_error("the POROUS2 and BRUSS2 bounds need the state w");
        return FRKC2_EINVAL;
    }
    const bool host_only = kg.op == FRKC2_OP_LAPLACE || kg.op == FRKC2_OP_ADVDIFF;
    if (!host_only && (!ws || ws_bytes < kScratch || !aligned16(ws))) {
        set_error("workspace needs at least %zu bytes, 16-byte aligned", kScratch);
        return FRKC2_ENOMEM;
    }
    return rho_bound_impl(kg, w, D, static_cast<double *>(ws), rho, st);
}

namespace frkc2 {

size_t step_workspace_bytes(long long nstate) { return step_layout(nstate).total; }

// Argument checks of frkc2_step (no HIP call).
int step_validate(const frkc2_grid *g, const double *w, const double *D, double T, double cfl,
                  int s, double nu, int nsteps, KGrid &kg)
{
    if (!make_kgrid(g, kg)) return FRKC2_EINVAL;
    if (!w) {
        set_error("w is NULL");
        return FRKC2_EINVAL;
    }
    if (kg.op == FRKC2_OP_VARCOEF && !D) {
        set_error("VARCOEF needs D");
        return FRKC2_EINVAL;
    }
    if (!check_s_nu(s, nu)) return FRKC2_EINVAL;
    if (nsteps < 0) {
        set_error("nsteps must be >= 0");
        return FRKC2_EINVAL;
    }
    const bool fixedT = T > 0.0 && std::isfinite(T);
    const bool adaptive = cfl > 0.0 && std::isfinite(cfl);
    if (fixedT == adaptive || (!(T >= 0.0) || !(cfl >= 0.0))) {
        set_error("exactly one of T and cfl must be positive and finite (T=%g, cfl=%g)", T, cfl);
        return FRKC2_EINVAL;
    }
    return FRKC2_OK;
}

// frkc2_step's body; ws is the caller's workspace or the library's static
// scratch (frkc2_step_noalloc).
int step_core(const frkc2_grid *g, double *w, const double *D, double T, double cfl, int s,
              double nu, int nsteps, void *ws, size_t ws_bytes, hipStream_t st,
              frkc2_step_stats *stats)
{
    KGrid kg;
    const int vrc = step_validate(g, w, D, T, cfl, s, nu, nsteps, kg);
    if (vrc < 0) return vrc;
    const bool adaptive = cfl > 0.0 && std::isfinite(cfl);
    const long long N = kg.nstate();
    const StepLayout L = step_layout(N);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("workspace needs %zu bytes (got %zu), 16-byte aligned", L.total, ws_bytes);
        return FRKC2_ENOMEM;
    }
    const double *are, *aim;
    frkc2_coeff_info info;
    int crc = coeffs_cached(s, nu, &are, &aim, &info);
    if (crc < 0) return crc;
    char *base = static_cast<char *>(ws);
    double *buf[2] = {reinterpret_cast<double *>(base + L.bufA),
                      reinterpret_cast<double *>(base + L.bufB)};
    double *partials = reinterpret_cast<double *>(base + L.scratch);
    double *tau_dev = partials + 2 * (kReduceBlocks + 8);

    double rho = 0.0, Tn = T;
    const PassCfg cfg = pass_cfg(kg);
    static thread_local std::vector<double> tau_host;
    for (int step = 0; step < nsteps; ++step) {
        if (step == 0 || nonlinear(kg)) {
            int rc = rho_bound_impl(kg, w, D, partials, &rho, st);
            if (rc < 0) return rc;
            if (adaptive) {
                if (!(rho > 0.0)) {
                    set_error("adaptive T needs a positive Gershgorin bound (got %g)", rho);
                    return FRKC2_ENONFINITE;
                }
                Tn = (cfl * info.beta_bar) / rho;
            }
            if (Tn * rho > info.beta_bar) {
                set_error("T*rho = %g exceeds beta_bar = %g", Tn * rho, info.beta_bar);
                return FRKC2_EUNSTABLE;
            }
        }
        const bool last_step = (step == nsteps - 1);
        const bool want_stats = stats && last_step;
        if (stage1d_lds_fits(kg) && !want_stats) {
            // A linear operator keeps T, and so every stepsize, for the rest of
            // the call: its remaining supersteps (all but a last one that
            // reports statistics) run in one launch, the state staying in LDS.
            const int run = nonlinear(kg) ? 1 : (stats ? nsteps - 1 : nsteps) - step;
            tau_host.resize(2 * (size_t)s);
            for (int l = 0; l < s; ++l) {
                tau_host[2 * l] = Tn * are[l];
                tau_host[2 * l + 1] = Tn * aim[l];
            }
            HIP_TRY(hipMemcpyAsync(tau_dev, tau_host.data(), sizeof(double) * 2 * s,
                                   hipMemcpyHostToDevice, st),
                    "stepsize upload");
            HIP_TRY(launch_stage1d_lds(kg, w, w, D, tau_dev, s, run, st), "1D stage launch");
            step += run - 1;
            continue;
        }
        const double *last_out = nullptr;
        HIP_TRY(run_superstep(kg, cfg, w, D, Tn, are, aim, s, want_stats, buf, &last_out, st),
                "stage launch");
        if (want_stats) {
            HIP_TRY(launch_finalize(kg, last_out, w, partials, st), "finalize launch");
            double sums[2];
            HIP_TRY(hipMemcpyAsync(sums, partials + 2 * kReduceBlocks, sizeof(sums),
                                   hipMemcpyDeviceToHost, st),
                    "stats copy");
            HIP_TRY(hipStreamSynchronize(st), "stats");
            stats->im_ratio = sums[1] > 0.0 ? std::sqrt(sums[0] / sums[1]) : 0.0;
        }
    }
    if (stats) {
        stats->T_last = Tn;
        stats->rho_last = rho;
        stats->supersteps = nsteps;
        if (nsteps == 0) stats->im_ratio = 0.0;
        HIP_TRY(hipStreamSynchronize(st), "step");
    }
    return crc;
}

}  // namespace frkc2

extern "C" int frkc2_step(const frkc2_grid *g, double *w, const double *D, double T, double cfl,
                          int s, double nu, int nsteps, void *ws, size_t ws_bytes, hipStream_t st,
                          frkc2_step_stats *stats)
{
    return step_core(g, w, D, T, cfl, s, nu, nsteps, ws, ws_bytes, st, stats);
}

namespace {

// Distinct launch configurations worth timing for a grid: every supported
// depth, the tile shapes that differ for it, and a few chunk lengths.
std::vector<PassCfg> tune_candidates(const KGrid &kg)
{
    std::vector<PassCfg> out;
    std::vector<int> zcs{0};
    for (int zc : {8, 16, 32, 64, 128})   // the Brusselator's tiles have no chunk length
        if (zc < kg.nz && kg.op != FRKC2_OP_BRUSS2) zcs.push_back(zc);
    auto add = [&](int k, int tile) {
        if (k >= 2 && !tblock_supported(kg, k)) return;
        for (int zc : zcs) {
            if (k >= 2 && zc != 0 && zc < 2 * k) continue;   // halo planes would dominate
            out.push_back(PassCfg{k, tile, zc});
        }
    };
    add(1, 0);
    if (kg.ndim == 3) {
        add(2, 0);
        add(2, 1);
        add(2, 2);
        add(2, 3);
        add(2, 4);
        add(3, 0);
        add(3, 2);
        add(3, 3);
        add(3, 4);
    } else if (kg.ndim == 2) {
        for (int k : {2, 3, 4, 6, 8}) {
            add(k, 0);
            if (kg.op != FRKC2_OP_BRUSS2) add(k, 1);   // the Brusselator has one tile
        }
    }
    return out;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

}  // namespace

extern "C" int frkc2_autotune(const frkc2_grid *g, const double *w, const double *D, int s,
                              double nu, int reps, void *ws, size_t ws_bytes, hipStream_t st,
                              frkc2_tune_result *res)
{
    KGrid kg;
    if (!make_kgrid(g, kg)) return FRKC2_EINVAL;
    if (!w || !res || (kg.op == FRKC2_OP_VARCOEF && !D)) {
        set_error("w and result (and D for VARCOEF) must be non-NULL");
        return FRKC2_EINVAL;
    }
    if (!check_s_nu(s, nu)) return FRKC2_EINVAL;
    if (reps < 1 || reps > 100) {
        set_error("reps must lie in [1, 100] (got %d)", reps);
        return FRKC2_EINVAL;
    }
    const StepLayout L = step_layout(kg.nstate());
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("workspace needs %zu bytes (got %zu), 16-byte aligned", L.total, ws_bytes);
        return FRKC2_ENOMEM;
    }
    const double *are, *aim;
    frkc2_coeff_info info;
    const int crc = coeffs_cached(s, nu, &are, &aim, &info);
    if (crc < 0) return crc;
    char *base = static_cast<char *>(ws);
    double *buf[2] = {reinterpret_cast<double *>(base + L.bufA),
                      reinterpret_cast<double *>(base + L.bufB)};
    double *partials = reinterpret_cast<double *>(base + L.scratch);
    double rho = 0.0;
    int rc = rho_bound_impl(kg, w, D, partials, &rho, st);
    if (rc < 0) return rc;
    // a stable step, so that the timed values stay bounded
    const double Tn = (rho > 0.0 && std::isfinite(rho)) ? 0.5 * info.beta_bar / rho : 0.0;

    EventPair ev;
    HIP_TRY(hipEventCreate(&ev.a), "autotune: event");
    HIP_TRY(hipEventCreate(&ev.b), "autotune: event");
    // Each candidate runs whole supersteps that end in the complex buffers,
    // so the caller's w is only read.
    auto time_cfg = [&](const PassCfg &c, double *ms) -> int {
        HIP_TRY(run_superstep(kg, c, const_cast<double *>(w), D, Tn, are, aim, s, true, buf,
                              nullptr, st),
                "autotune: warm-up");
        HIP_TRY(hipEventRecord(ev.a, st), "autotune: event");
        for (int r = 0; r < reps; ++r)
            HIP_TRY(run_superstep(kg, c, const_cast<double *>(w), D, Tn, are, aim, s, true, buf,
                                  nullptr, st),
                    "autotune: superstep");
        HIP_TRY(hipEventRecord(ev.b, st), "autotune: event");
        HIP_TRY(hipEventSynchronize(ev.b), "autotune: sync");
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, ev.a, ev.b), "autotune: elapsed");
        *ms = (double)t / reps;
        return FRKC2_OK;
    };

    PassCfg dflt{default_depth(kg), default_tile(kg), 0};
    if (dflt.k >= 2 && !tblock_supported(kg, dflt.k)) dflt.k = 1;
    double ms_default = 0.0;
    rc = time_cfg(dflt, &ms_default);
    if (rc < 0) return rc;
    PassCfg best = dflt;
    double ms_best = ms_default;
    int n = 1;
    for (const PassCfg &c : tune_candidates(kg)) {
        double ms = 0.0;
        rc = time_cfg(c, &ms);
        if (rc < 0) return rc;
        ++n;
        if (ms < ms_best) {
            ms_best = ms;
            best = c;
        }
    }
    // The default ran first, while clocks and caches settle: time it again and
    // keep it unless a candidate is clearly faster, so that timing noise does
    // not flip the configuration from run to run.
    double ms_again = 0.0;
    rc = time_cfg(dflt, &ms_again);
    if (rc < 0) return rc;
    ms_default = std::min(ms_default, ms_again);
    if (ms_default <= 1.03 * ms_best) {
        best = dflt;
        ms_best = ms_default;
    }
    store_tuned(kg, best);
    res->tblock = best.k;
    res->tile = best.tile + 1;
    res->zchunk = best.zchunk;
    res->candidates = n;
    res->ms_best = ms_best;
    res->ms_default = ms_default;
    return crc;
}

namespace {

// One linear flow of s stages on the complex state Z (Sec. 3 Euler steps with
// complex W^0): passes as run_superstep schedules them, the first reading Z,
// the last writing Z, the ones between ping-ponging buf. A fused pass reads a
// halo around its tiles, so a single pass may not read and write Z: the
// first pass then takes one stage less.
int run_flow_c(const KGrid &kg, const PassCfg &cfg, double *Z, double Tn, const double *are,
               const double *aim, int s, double *const buf[2], hipStream_t st)
{
    const int k = cfg.k;
    int l = 0, pass = 0;
    const double *in = Z;
    while (l < s) {
        int kk = (k >= 2 && s - l >= k) ? k : 1;
        // a pass that would leave one stage leaves two: a lone stage is a
        // whole-grid pass of its own, about twice the time of a fused stage
        if (kk >= 3 && s - l - kk == 1 && tblock_supported(kg, kk - 1)) kk -= 1;
        if (kk == 1 && k > 2 && s - l >= 2 && tblock_supported(kg, s - l)) kk = s - l;
        if (l == 0 && kk == s && s > 1) {
            kk = s - 1;
            while (kk >= 2 && !tblock_supported(kg, kk)) --kk;
        }
        PassArgs pa{};
        pa.k = kk;
        pa.zchunk = cfg.zchunk;
        pa.in_c = in;
        const bool last = (l + kk == s);
        double *out = last ? Z : buf[pass & 1];
        pa.out_c = out;
        for (int i = 0; i < kk; ++i) {
            pa.tr[i] = Tn * are[l + i];
            pa.ti[i] = Tn * aim[l + i];
        }
        const int rc = (kk == 1) ? launch_pass(kg, pa, 1, st) : launch_tblock(kg, pa, cfg.tile, st);
        if (rc != 0) return rc;
        in = out;
        l += kk;
        ++pass;
    }
    return 0;
}

// The B steps of the split scheme: b1 = (3 + i)/30, b2 = (4 - 2i)/15,
// b3 = (4 + 3i)/15, in the order b1 b2 b3 b2 b1.
const double kSplitB[5][2] = {{3.0 / 30.0, 1.0 / 30.0}, {4.0 / 15.0, -2.0 / 15.0},
                              {4.0 / 15.0, 3.0 / 15.0}, {4.0 / 15.0, -2.0 / 15.0},
                              {3.0 / 30.0, 1.0 / 30.0}};

struct SplitLayout {
    size_t Z, bufA, bufB, total;
};

SplitLayout split_layout(long long N)
{
    SplitLayout L;
    L.Z = 0;
    L.bufA = align_up((size_t)N * 32);
    L.bufB = L.bufA + align_up((size_t)N * 16);
    L.total = L.bufB + align_up((size_t)N * 16) + kScratch;
    return L;
}

bool split_grid(const frkc2_grid *g, KGrid &kb, KGrid &ka)
{
    if (!make_kgrid(g, kb)) return false;
    if (kb.op != FRKC2_OP_BRUSS2) {
        set_error("frkc4s_step: the split scheme runs the Brusselator (op BRUSS2)");
        return false;
    }
    frkc2_grid gl = *g;
    gl.op = FRKC2_OP_LAPLACE;
    return make_kgrid(&gl, ka);
}

}  // namespace

extern "C" size_t frkc4s_workspace_bytes(const frkc2_grid *g)
{
    KGrid kb, ka;
    if (!split_grid(g, kb, ka)) return 0;
    return split_layout(ka.npts()).total;
}

extern "C" int frkc4s_step(const frkc2_grid *g, double *w, double T, int s, int nsub, double nu,
                           int nsteps, void *ws, size_t ws_bytes, hipStream_t st)
{
    KGrid kb, ka;
    if (!split_grid(g, kb, ka)) return FRKC2_EINVAL;
    if (!w) {
        set_error("frkc4s_step: w is NULL");
        return FRKC2_EINVAL;
    }
    if (!(T > 0.0) || !std::isfinite(T) || nsub < 1 || nsub > 64 || nsteps < 0) {
        set_error("frkc4s_step: need T > 0 finite, 1 <= nsub <= 64, nsteps >= 0");
        return FRKC2_EINVAL;
    }
    const double *are, *aim;
    frkc2_coeff_info info;
    const int crc = coeffs4_cached(s, nu, &are, &aim, &info);
    if (crc < 0) return crc;
    // stability of the linear flows of length T/4 (Sec. 2): Gershgorin bound of
    // the periodic Laplacian, 2 (4 d) / h^2, exact
    double dsum = 0.0;
    for (int f = 0; f < 2 * ka.ndim; ++f) dsum = dsum + ka.d_const;
    const double rho = (2.0 * ka.inv_h2) * dsum;
    const double TA = T * 0.25;
    if (TA * rho > info.beta_bar) {
        set_error("frkc4s_step: (T/4)*rho = %g exceeds beta_bar(%d) = %g", TA * rho, s,
                  info.beta_bar);
        return FRKC2_EUNSTABLE;
    }
    const long long N = ka.npts();
    const SplitLayout L = split_layout(N);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("frkc4s_step: workspace needs %zu bytes (got %zu), 16-byte aligned", L.total,
                  ws_bytes);
        return FRKC2_ENOMEM;
    }
    char *base = static_cast<char *>(ws);
    double *Z = reinterpret_cast<double *>(base + L.Z);
    double *buf[2] = {reinterpret_cast<double *>(base + L.bufA),
                      reinterpret_cast<double *>(base + L.bufB)};
    const PassCfg cfg = pass_cfg(ka);
    for (int step = 0; step < nsteps; ++step) {
        HIP_TRY(launch_real_to_complex(2 * N, w, Z, st), "split: state upload");
        for (int j = 0; j < 5; ++j) {
            const double tr = kSplitB[j][0] * T, ti = kSplitB[j][1] * T;
            const double cr = tr / (double)nsub, ci = ti / (double)nsub;
            const double c[6] = {cr, ci, cr / 2.0, ci / 2.0, cr / 6.0, ci / 6.0};
            HIP_TRY(launch_react_flow(Z, N, c, nsub, st), "split: reaction flow");
            if (j == 4) break;
            for (int sp = 0; sp < 2; ++sp)
                HIP_TRY(run_flow_c(ka, cfg, Z + 2 * N * sp, TA, are, aim, s, buf, st),
                        "split: diffusion flow");
        }
        HIP_TRY(launch_take_real(Z, w, 2 * N, st), "split: real part");
    }
    return crc;
}

namespace {

// Argument checks shared by the adjoint entry points (no HIP call).
int adjoint_validate(const frkc2_grid *g, const double *D, double T, int s, double nu, KGrid &kg)
{
    if (!make_kgrid(g, kg)) return FRKC2_EINVAL;
    if (nonlinear(kg) || kg.op == FRKC2_OP_ADVDIFF) {
        set_error("the adjoint supports the symmetric operators (LAPLACE, VARCOEF)");
        return FRKC2_EINVAL;
    }
    if (kg.op == FRKC2_OP_VARCOEF && !D) {
        set_error("VARCOEF needs D");
        return FRKC2_EINVAL;
    }
    if (!check_s_nu(s, nu)) return FRKC2_EINVAL;
    if (!(T > 0.0) || !std::isfinite(T)) {
        set_error("T must be positive and finite");
        return FRKC2_EINVAL;
    }
    return FRKC2_OK;
}

// The forward stages W^0 .. W^{s-1} of the superstep from the real state w_n
// (Sec. 3, Euler-step equation) into the slots S(0) .. S(s-1) of store (slot
// stride cbytes): 3D grids fuse three stages per pass (two for a remainder of
// two) and write the intermediate states as well.
int store_stages(const KGrid &kg, const double *w_n, const double *D, double T,
                 const double *are, const double *aim, int s, char *store, size_t cbytes,
                 hipStream_t st)
{
    auto S = [&](int l) { return reinterpret_cast<double *>(store + (size_t)l * cbytes); };
    int rc = launch_real_to_complex(kg.npts(), w_n, S(0), st);
    for (int l = 0; rc == 0 && l + 1 < s;) {
        const int left = s - 1 - l;
        const int k = (kg.ndim == 3 && tb3d_plane_ok(kg) && left >= 2) ? (left >= 3 ? 3 : 2) : 1;
        PassArgs pa{};
        pa.k = k;
        pa.D = D;
        pa.in_c = S(l);
        pa.out_c = S(l + k);
        for (int i = 0; i < k; ++i) {
            pa.tr[i] = T * are[l + i];
            pa.ti[i] = T * aim[l + i];
        }
        if (k > 1) {
            pa.cols = tb3d_pick_cols(kg, 3);
            pa.lvl_out = S(l + 1);
            pa.lvl_stride = (long long)(cbytes / 16);
            rc = launch_tb3d(kg, pa, st);
        } else {
            rc = launch_pass(kg, pa, 0, st);
        }
        l += k;
    }
    return rc;
}

// The transposed stages in reverse order (stage l = s-1 .. 0) from lam_next to
// lam_n, with W^l in the slots of store; lam[2] are complex scratch states,
// gD the real per-cell accumulator (VARCOEF). Pass q writes lam[q & 1].
int reverse_stages(const KGrid &kg, const char *store, size_t cbytes, const double *D, double T,
                   const double *are, const double *aim, int s, const double *lam_next,
                   double *lam_n, double *grad_logD, double *const lam[2], double *gD,
                   hipStream_t st)
{
    const bool vc = kg.op == FRKC2_OP_VARCOEF;
    int rc = vc ? launch_zero(kg.npts(), gD, st) : 0;
    if (rc) return rc;
    // On request, 3D grids run two stages per pass (s is even) in the same
    // per-cell arithmetic; measured slower than one per pass, so not the
    // default. One pass of two would read lam_next and write lam_n, so it needs
    // the two to be distinct.
    const bool pairs = kg.ndim == 3 && g_adj_stages == 2 && !(s == 2 && lam_n == lam_next);
    auto rev = [&](int r, int q_in, int q_out) {
        const int l = s - 1 - r;
        AdjArgs a{};
        if (r == 0) a.lam_in_re = lam_next;
        else a.lam_in_c = lam[q_in & 1];
        if (r == s - 1) a.lam_out_re = lam_n;
        else a.lam_out_c = lam[q_out & 1];
        a.W = reinterpret_cast<const double *>(store + (size_t)l * cbytes);
        a.D = D;
        a.gD = vc ? gD : nullptr;
        a.tr = T * are[l];
        a.ti = T * aim[l];
        return a;
    };
    if (pairs) {
        for (int r = 0, q = 0; r < s && rc == 0; r += 2, ++q)
            rc = launch_adjoint_pair(kg, rev(r, q - 1, q), rev(r + 1, q - 1, q), st);
    } else {
        for (int r = 0; r < s && rc == 0; ++r) rc = launch_adjoint_stage(kg, rev(r, r - 1, r), st);
    }
    if (rc == 0 && vc && grad_logD) rc = launch_grad_finish(kg.npts(), D, gD, grad_logD, st);
    return rc;
}

}  // namespace

extern "C" int frkc2_step_adjoint(const frkc2_grid *g, const double *w_n, const double *D,
                                  double T, int s, double nu, const double *lam_next,
                                  double *lam_n, double *grad_logD, void *ws, size_t ws_bytes,
                                  hipStream_t st)
{
    KGrid kg;
    const int vrc = adjoint_validate(g, D, T, s, nu, kg);
    if (vrc < 0) return vrc;
    if (!w_n || !lam_next || !lam_n) {
        set_error("w_n, lam_next and lam_n must be non-NULL");
        return FRKC2_EINVAL;
    }
    const long long N = kg.npts();
    const AdjLayout L = adj_layout(N, s);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("adjoint workspace needs %zu bytes (got %zu), 16-byte aligned", L.total,
                  ws_bytes);
        return FRKC2_ENOMEM;
    }
    const double *are, *aim;
    int crc = coeffs_cached(s, nu, &are, &aim, nullptr);
    if (crc < 0) return crc;
    char *base = static_cast<char *>(ws);
    const size_t cbytes = align_up((size_t)N * 16);
    double *lam[2] = {reinterpret_cast<double *>(base + L.lamA),
                      reinterpret_cast<double *>(base + L.lamB)};
    double *gD = reinterpret_cast<double *>(base + L.gD);
    HIP_TRY(store_stages(kg, w_n, D, T, are, aim, s, base + L.store, cbytes, st),
            "adjoint: forward recompute");
    HIP_TRY(reverse_stages(kg, base + L.store, cbytes, D, T, are, aim, s, lam_next, lam_n,
                           grad_logD, lam, gD, st),
            "adjoint: reverse stages");
    return crc;
}

extern "C" int frkc2_step_store(const frkc2_grid *g, double *w, const double *D, double T, int s,
                                double nu, double *stages, size_t stages_bytes, void *ws,
                                size_t ws_bytes, hipStream_t st)
{
    KGrid kg;
    const int vrc = adjoint_validate(g, D, T, s, nu, kg);
    if (vrc < 0) return vrc;
    if (!w || !stages) {
        set_error("w and stages must be non-NULL");
        return FRKC2_EINVAL;
    }
    const long long N = kg.npts();
    const size_t cbytes = align_up((size_t)N * 16);
    if (stages_bytes < (size_t)s * cbytes || !aligned16(stages)) {
        set_error("the stage store needs %zu bytes (got %zu), 16-byte aligned",
                  (size_t)s * cbytes, stages_bytes);
        return FRKC2_ENOMEM;
    }
    const bool host_only = kg.op == FRKC2_OP_LAPLACE;
    if (!host_only && (!ws || ws_bytes < kScratch || !aligned16(ws))) {
        set_error("workspace needs at least %zu bytes, 16-byte aligned", kScratch);
        return FRKC2_ENOMEM;
    }
    const double *are, *aim;
    frkc2_coeff_info info;
    int crc = coeffs_cached(s, nu, &are, &aim, &info);
    if (crc < 0) return crc;
    // stability as frkc2_step checks it (Sec. 2: T rho <= beta_bar)
    double rho = 0.0;
    const int rc = rho_bound_impl(kg, w, D, static_cast<double *>(ws), &rho, st);
    if (rc < 0) return rc;
    if (T * rho > info.beta_bar) {
        set_error("T*rho = %g exceeds beta_bar = %g", T * rho, info.beta_bar);
        return FRKC2_EUNSTABLE;
    }
    char *store = reinterpret_cast<char *>(stages);
    HIP_TRY(store_stages(kg, w, D, T, are, aim, s, store, cbytes, st), "store: stages");
    // the last stage from W^{s-1}, its real part into w
    PassArgs pa{};
    pa.k = 1;
    pa.D = D;
    pa.in_c = reinterpret_cast<const double *>(store + (size_t)(s - 1) * cbytes);
    pa.out_re = w;
    pa.tr[0] = T * are[s - 1];
    pa.ti[0] = T * aim[s - 1];
    HIP_TRY(launch_pass(kg, pa, 0, st), "store: last stage");
    return crc;
}

extern "C" int frkc2_step_adjoint_stored(const frkc2_grid *g, const double *stages,
                                         size_t stages_bytes, const double *D, double T, int s,
                                         double nu, const double *lam_next, double *lam_n,
                                         double *grad_logD, void *ws, size_t ws_bytes,
                                         hipStream_t st)
{
    KGrid kg;
    const int vrc = adjoint_validate(g, D, T, s, nu, kg);
    if (vrc < 0) return vrc;
    if (!stages || !lam_next || !lam_n) {
        set_error("stages, lam_next and lam_n must be non-NULL");
        return FRKC2_EINVAL;
    }
    const long long N = kg.npts();
    const size_t cbytes = align_up((size_t)N * 16);
    if (stages_bytes < (size_t)s * cbytes || !aligned16(stages)) {
        set_error("the stage store needs %zu bytes (got %zu), 16-byte aligned",
                  (size_t)s * cbytes, stages_bytes);
        return FRKC2_ENOMEM;
    }
    const AdjLayout L = adj_layout(N, 0);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("adjoint workspace needs %zu bytes (got %zu), 16-byte aligned", L.total,
                  ws_bytes);
        return FRKC2_ENOMEM;
    }
    const double *are, *aim;
    int crc = coeffs_cached(s, nu, &are, &aim, nullptr);
    if (crc < 0) return crc;
    char *base = static_cast<char *>(ws);
    double *lam[2] = {reinterpret_cast<double *>(base + L.lamA),
                      reinterpret_cast<double *>(base + L.lamB)};
    double *gD = reinterpret_cast<double *>(base + L.gD);
    HIP_TRY(reverse_stages(kg, reinterpret_cast<const char *>(stages), cbytes, D, T, are, aim, s,
                           lam_next, lam_n, grad_logD, lam, gD, st),
            "adjoint: reverse stages");
    return crc;
}


// ---- error-controlled integration (Sec. 3) ----

namespace {

constexpr double kSafe = 0.8;        // safety factor of the paper's controller
constexpr double kFacMax = 5.0;      // growth cap (the paper gives none)
constexpr double kErrFloor = 1e-12;  // error estimates below this count as this

// One superstep from the real state w that also carries the embedded
// first-order solution; W^L (complex) and What^L are left in the workspace.
// Fused passes of cfg.k stages where the tile has an embedded variant (3D
// full-width tiles, the Brusselator, 2D rows of 256 with k <= 4); other grids
// and tile shapes run one stage per pass.
int run_superstep_emb(const KGrid &kg, const PassCfg &cfg, const double *w, const double *D,
                      double Tn, const double *are, const double *aim, int s,
                      double *const buf[2], double *const emb[2], const double **WL,
                      const double **EL, double *tau_dev, hipStream_t st)
{
    if (stage1d_lds_fits(kg)) {
        // a 1D grid that fits in LDS: the whole superstep in one launch, the
        // stepsizes from a device table (tau_dev, 2 s doubles)
        static thread_local std::vector<double> tau_host;
        tau_host.resize(2 * (size_t)s);
        for (int l = 0; l < s; ++l) {
            tau_host[2 * l] = Tn * are[l];
            tau_host[2 * l + 1] = Tn * aim[l];
        }
        int rc = (int)hipMemcpyAsync(tau_dev, tau_host.data(), sizeof(double) * 2 * s,
                                     hipMemcpyHostToDevice, st);
        if (rc != 0) return rc;
        rc = launch_stage1d_lds_emb(kg, w, buf[0], emb[0], D, tau_dev, s, st);
        if (rc != 0) return rc;
        *WL = buf[0];
        *EL = emb[0];
        return 0;
    }
    const bool fused = cfg.k >= 2 && tblock_emb_supported(kg, cfg.k, cfg.tile);
    const int k = fused ? cfg.k : 1;
    int l = 0, pass = 0;
    const double *in = nullptr, *ein = nullptr;
    while (l < s) {
        int kk = (k >= 2 && s - l >= k) ? k : 1;
        if (kk == 1 && k > 2 && s - l >= 2 && tblock_emb_supported(kg, s - l, cfg.tile))
            kk = s - l;
        PassArgs pa{};
        pa.k = kk;
        pa.zchunk = cfg.zchunk;
        pa.D = D;
        if (l == 0) pa.in_re = w;
        else {
            pa.in_c = in;
            pa.emb_in = ein;
        }
        pa.out_c = buf[pass & 1];
        pa.emb_out = emb[pass & 1];
        pa.cols = (cfg.tile == 4) ? 32 : 64;
        for (int i = 0; i < kk; ++i) {
            pa.tr[i] = Tn * are[l + i];
            pa.ti[i] = Tn * aim[l + i];
        }
        const int rc = (kk == 1) ? launch_pass(kg, pa, 1, st)
                                 : launch_tblock(kg, pa, cfg.tile, st);
        if (rc != 0) return rc;
        in = buf[pass & 1];
        ein = emb[pass & 1];
        l += kk;
        ++pass;
    }
    *WL = in;
    *EL = ein;
    return 0;
}

// Smallest even s with betabar(s) >= x, searched from the estimate
// betabar ~ 0.33 s^2 (s = 2 ceil(sqrt(x / 1.32))) down and up in steps of 2.
int choose_s(double x, double nu, double *bbar)
{
    auto bb = [&](int s, double *v) -> int {
        const double *re, *im;
        frkc2_coeff_info info;
        const int rc = coeffs_cached(s, nu, &re, &im, &info);
        if (rc < 0) return rc;
        *v = info.beta_bar;
        return 0;
    };
    const double r = std::sqrt(x / 1.32);
    int m = (r < kMaxStages / 2) ? (int)std::ceil(r) : kMaxStages / 2;
    if (m < 1) m = 1;
    int s = 2 * m;
    double v = 0.0;
    while (s > 2) {
        const int rc = bb(s - 2, &v);
        if (rc < 0) return rc;
        if (!(v >= x)) break;
        s -= 2;
    }
    while (true) {
        const int rc = bb(s, &v);
        if (rc < 0) return rc;
        if (v >= x || s >= kMaxStages) break;
        s += 2;
    }
    *bbar = v;
    return s;
}

}  // namespace

namespace {

// The controller of Sec. 3 with the readings stated in frkc2.h: attempts until t reaches
// t_span. rho_fn(&rho) bounds the spectral radius of the current state (before the first
// attempt and, with rho_every, after every accepted step); step_fn(Tn, s, a_re, a_im, &WL,
// &EL) runs one superstep from w that carries the embedded solution and leaves W^L
// (complex) and What^L in the workspace. Both return a frkc2_status.
template <class RhoFn, class StepFn>
int adapt_loop(long long N, double *w, double t_span, double T0, double tol, double nu,
               int max_attempts, bool rho_every, double *partials, hipStream_t st,
               double *trace, int trace_cap, frkc2_adapt_stats *stats, RhoFn rho_fn,
               StepFn step_fn)
{
    double t = 0.0, T = T0, T_prev = 0.0, err_prev = 0.0, err_last = 0.0, rho = 0.0;
    bool have_prev = false, need_rho = true;
    int attempts = 0, accepted = 0, rejected = 0, s_last = 0;
    long long stages = 0;
    while (t < t_span) {
        if (attempts >= max_attempts) {
            set_error("no end after %d attempts (t = %g of %g)", attempts, t, t_span);
            return FRKC2_ETIMEOUT;
        }
        if (need_rho) {
            const int rc = rho_fn(&rho);
            if (rc < 0) return rc;
            need_rho = false;
        }
        double Tn = std::min(T, t_span - t);
        const double x = Tn * rho;
        double bbar = 0.0;
        const int s = choose_s(x, nu, &bbar);
        if (s < 0) return s;
        if (bbar < x) Tn = 0.99 * bbar / rho;
        const double *are, *aim;
        frkc2_coeff_info info;
        int crc = coeffs_cached(s, nu, &are, &aim, &info);
        if (crc < 0) return crc;
        const double *WL = nullptr, *EL = nullptr;
        const int src = step_fn(Tn, s, are, aim, &WL, &EL);
        if (src < 0) return src;
        HIP_TRY(launch_err_max(WL, EL, N, tol, partials, st), "error estimate launch");
        double err = 0.0;
        HIP_TRY(hipMemcpyAsync(&err, partials + kReduceBlocks, sizeof(double),
                               hipMemcpyDeviceToHost, st),
                "error estimate copy");
        HIP_TRY(hipStreamSynchronize(st), "error estimate");
        stages += s;
        s_last = s;
        if (trace && attempts < trace_cap) {
            double *r = trace + 5 * (size_t)attempts;
            r[0] = t;
            r[1] = Tn;
            r[2] = s;
            r[3] = err;
            r[4] = (err > 1.0) ? 0.0 : 1.0;
        }
        ++attempts;
        if (!std::isfinite(err)) {
            set_error("non-finite error estimate at t = %g (T = %g, s = %d)", t, Tn, s);
            return FRKC2_ENONFINITE;
        }
        if (err > 1.0) {
            ++rejected;
            T = Tn * (kSafe / std::sqrt(err));
            have_prev = false;
            continue;
        }
        HIP_TRY(launch_take_real(WL, w, N, st), "accept launch");
        ++accepted;
        t = t + Tn;
        err_last = err;
        const double e = std::max(err, kErrFloor);
        double fac = kSafe / std::sqrt(e);
        if (have_prev) fac = fac * (Tn / T_prev) * std::sqrt(err_prev / e);
        fac = std::min(fac, kFacMax);
        T_prev = Tn;
        err_prev = e;
        have_prev = true;
        T = Tn * fac;
        if (rho_every) need_rho = true;
    }
    HIP_TRY(hipStreamSynchronize(st), "integrate");
    if (stats) {
        stats->t = t;
        stats->T_next = T;
        stats->err_last = err_last;
        stats->stages = stages;
        stats->attempts = attempts;
        stats->accepted = accepted;
        stats->rejected = rejected;
        stats->s_last = s_last;
    }
    return FRKC2_OK;
}

bool check_adapt_args(double t_span, double T0, double tol, double nu, int max_attempts,
                      double *trace, int trace_cap)
{
    if (!(t_span > 0.0) || !std::isfinite(t_span) || !(T0 > 0.0) || !std::isfinite(T0) ||
        !(tol > 0.0) || !std::isfinite(tol)) {
        set_error("t_span, T0 and tol must be positive and finite");
        return false;
    }
    if (!(nu >= 0.0 && nu < 1.0)) {
        set_error("nu must lie in [0, 1) (got %g)", nu);
        return false;
    }
    if (max_attempts < 1 || trace_cap < 0 || (trace_cap > 0 && !trace)) {
        set_error("max_attempts must be >= 1 and trace non-NULL when trace_cap > 0");
        return false;
    }
    return true;
}

}  // namespace

extern "C" int frkc2_integrate(const frkc2_grid *g, double *w, const double *D, double t_span,
                               double T0, double tol, double nu, int max_attempts, void *ws,
                               size_t ws_bytes, hipStream_t st, double *trace, int trace_cap,
                               frkc2_adapt_stats *stats)
{
    KGrid kg;
    if (!make_kgrid(g, kg)) return FRKC2_EINVAL;
    if (!w || (kg.op == FRKC2_OP_VARCOEF && !D)) {
        set_error("w (and D for VARCOEF) must be non-NULL");
        return FRKC2_EINVAL;
    }
    if (!check_adapt_args(t_span, T0, tol, nu, max_attempts, trace, trace_cap)) return FRKC2_EINVAL;
    const long long N = kg.nstate();
    const AdaptLayout L = adapt_layout(N);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("workspace needs %zu bytes (got %zu), 16-byte aligned", L.total, ws_bytes);
        return FRKC2_ENOMEM;
    }
    char *base = static_cast<char *>(ws);
    double *buf[2] = {reinterpret_cast<double *>(base + L.bufA),
                      reinterpret_cast<double *>(base + L.bufB)};
    double *emb[2] = {reinterpret_cast<double *>(base + L.embA),
                      reinterpret_cast<double *>(base + L.embB)};
    double *partials = reinterpret_cast<double *>(base + L.scratch);
    const PassCfg cfg = pass_cfg(kg);
    return adapt_loop(
        N, w, t_span, T0, tol, nu, max_attempts, nonlinear(kg), partials, st, trace, trace_cap,
        stats, [&](double *rho) { return rho_bound_impl(kg, w, D, partials, rho, st); },
        [&](double Tn, int s, const double *are, const double *aim, const double **WL,
            const double **EL) -> int {
            HIP_TRY(run_superstep_emb(kg, cfg, w, D, Tn, are, aim, s, buf, emb, WL, EL,
                                      partials + 2 * (kReduceBlocks + 8), st),
                    "embedded superstep launch");
            return FRKC2_OK;
        });
}

extern "C" size_t frkc2_user_workspace_bytes(long long n, int flags)
{
    if (n < 1) return 0;
    if (flags == FRKC2_WS_STEP) return step_layout(n).total;
    if (flags == FRKC2_WS_ADAPT) return adapt_layout(n).total;
    return 0;
}

extern "C" int frkc2_integrate_user(long long n, double *w, frkc2_user_f f,
                                    frkc2_user_rho rho_f, double rho_const, void *user,
                                    double t_span, double T0, double tol, double nu,
                                    int max_attempts, void *ws, size_t ws_bytes, hipStream_t st,
                                    double *trace, int trace_cap, frkc2_adapt_stats *stats)
{
    if (n < 1 || !w || !f) {
        set_error("user integrate: need n >= 1, w and f");
        return FRKC2_EINVAL;
    }
    if (!rho_f && (!(rho_const > 0.0) || !std::isfinite(rho_const))) {
        set_error("user integrate: need rho_f or a positive finite rho_const");
        return FRKC2_EINVAL;
    }
    if (!check_adapt_args(t_span, T0, tol, nu, max_attempts, trace, trace_cap)) return FRKC2_EINVAL;
    const AdaptLayout L = adapt_layout(n);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("workspace needs %zu bytes (got %zu), 16-byte aligned", L.total, ws_bytes);
        return FRKC2_ENOMEM;
    }
    char *base = static_cast<char *>(ws);
    double *W = reinterpret_cast<double *>(base + L.bufA);
    double *F = reinterpret_cast<double *>(base + L.bufB);
    double *E = reinterpret_cast<double *>(base + L.embA);
    double *partials = reinterpret_cast<double *>(base + L.scratch);
    return adapt_loop(
        n, w, t_span, T0, tol, nu, max_attempts, rho_f != nullptr, partials, st, trace,
        trace_cap, stats,
        [&](double *rho) -> int {
            if (!rho_f) {
                *rho = rho_const;
                return FRKC2_OK;
            }
            double r = -1.0;
            const int urc = rho_f(w, n, user, st, &r);
            if (urc != 0 || !(r > 0.0) || !std::isfinite(r)) {
                set_error("user integrate: rho_f returned %d with rho = %g", urc, r);
                return FRKC2_EINVAL;
            }
            *rho = r;
            return FRKC2_OK;
        },
        [&](double Tn, int s, const double *are, const double *aim, const double **WL,
            const double **EL) -> int {
            HIP_TRY(launch_real_to_complex(n, w, W, st), "user integrate: W^0");
            HIP_TRY(hipMemcpyAsync(E, w, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st),
                    "user integrate: What^0");
            for (int l = 0; l < s; ++l) {
                const int urc = f(W, F, n, user, st);
                if (urc != 0) {
                    set_error("user integrate: f returned %d at stage %d", urc, l);
                    return FRKC2_EINVAL;
                }
                HIP_TRY(launch_euler_axpy(n, W, F, Tn * are[l], Tn * aim[l], st, E),
                        "user integrate: update");
            }
            *WL = W;
            *EL = E;
            return FRKC2_OK;
        });
}

extern "C" int frkc2_step_user(long long n, double *w, frkc2_user_f f, void *user, double T,
                               double rho, int s, double nu, int nsteps, void *ws,
                               size_t ws_bytes, hipStream_t st)
{
    if (n < 1 || !w || !f) {
        set_error("user step: need n >= 1, w and f");
        return FRKC2_EINVAL;
    }
    if (!check_s_nu(s, nu)) return FRKC2_EINVAL;
    if (nsteps < 0 || !(T > 0.0) || !std::isfinite(T) || !(rho >= 0.0) || !std::isfinite(rho)) {
        set_error("user step: need nsteps >= 0, T > 0 and rho >= 0, finite");
        return FRKC2_EINVAL;
    }
    const StepLayout L = step_layout(n);
    if (!ws || ws_bytes < L.total || !aligned16(ws)) {
        set_error("workspace needs %zu bytes (got %zu), 16-byte aligned", L.total, ws_bytes);
        return FRKC2_ENOMEM;
    }
    const double *are, *aim;
    frkc2_coeff_info info;
    const int crc = coeffs_cached(s, nu, &are, &aim, &info);
    if (crc < 0) return crc;
    if (T * rho > info.beta_bar) {
        set_error("T*rho = %g exceeds beta_bar = %g", T * rho, info.beta_bar);
        return FRKC2_EUNSTABLE;
    }
    char *base = static_cast<char *>(ws);
    double *W = reinterpret_cast<double *>(base + L.bufA);
    double *F = reinterpret_cast<double *>(base + L.bufB);
    for (int step = 0; step < nsteps; ++step) {
        HIP_TRY(launch_real_to_complex(n, w, W, st), "user step: W^0");
        for (int l = 0; l < s; ++l) {
            const int urc = f(W, F, n, user, st);
            if (urc != 0) {
                set_error("user step: f returned %d at stage %d", urc, l);
                return FRKC2_EINVAL;
            }
            HIP_TRY(launch_euler_axpy(n, W, F, T * are[l], T * aim[l], st), "user step: update");
        }
        HIP_TRY(launch_take_real(W, w, n, st), "user step: Re W^L");
    }
    return crc;
}

extern "C" int frkc2_reduce(int op, const double *x, const double *y, size_t n, double *result,
                            void *ws, size_t ws_bytes, hipStream_t st)
{
    if (op < FRKC2_RED_SUMSQ || op > FRKC2_RED_DOT) {
        set_error("unknown reduction %d", op);
        return FRKC2_EINVAL;
    }
    if (!x || !result || ((op == FRKC2_RED_SUMSQDIFF || op == FRKC2_RED_DOT) && !y)) {
        set_error("reduction operands must be non-NULL");
        return FRKC2_EINVAL;
    }
    const size_t need = sizeof(double) * (kReduceBlocks + 8);
    if (!ws || ws_bytes < need || !aligned16(ws)) {
        set_error("reduction workspace needs %zu bytes", need);
        return FRKC2_ENOMEM;
    }
    double *partials = static_cast<double *>(ws);
    HIP_TRY(launch_reduce(op, x, y, (long long)n, partials, st), "reduce launch");
    HIP_TRY(hipMemcpyAsync(result, partials + kReduceBlocks, sizeof(double), hipMemcpyDeviceToHost,
                           st),
            "reduce copy");
    HIP_TRY(hipStreamSynchronize(st), "reduce");
    return FRKC2_OK;
}
