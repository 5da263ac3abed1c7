// Host side of frkc2_step_batched: validation, work tables, workspace layout
// and the cached HIP graph (per stage level one kernel over the 3D problems
// and one over the 2D problems).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <vector>

#include "internal.h"

namespace frkc2 {
namespace {

constexpr size_t kAlign = 256;
constexpr int kChunkPlanes = 32;   // z planes (3D) or rows (2D) per one-stage tile
// The 3D problems run as kGroups3 interleaved groups (alternate problems in
// order of decreasing s), each a chain of pass levels on its own graph
// branch, so that the tail of one group's level, when few tiles are left,
// shares the GPU with the other group's work.
constexpr int kGroups3 = 2;
constexpr int kChunkPlanes3 = 128;  // z planes per fused 3D tile (nz <= 128: one chunk)
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    size_t probs[2], tau, bufs, total;             // index 0: 3D list, 1: 2D list
    size_t partials;                               // reduction scratch of the rho check
    size_t pass3;                                  // 3D pass tables: kGroups3 * 2 * levels3 rows of n3 + 1
    int levels3;                                   // most pass levels of the 3D list (any depth)
    size_t pass2;                                  // 2D pass tables: 2 * levels2 rows of n2 + 1
    int levels2;
    std::vector<size_t> buf_off;                   // per problem (caller's order)
};

// Passes of a problem: fused passes of k stages, then single stages. A lone
// fused pass would read and write w (its tiles read a halo around them), so
// s = k runs as single stages.
int nfull(int s, int k) { return (s == k) ? 0 : s / k; }
int npass(int s, int k) { return nfull(s, k) + (s - k * nfull(s, k)); }
constexpr int kK3[] = {2, 3};
constexpr int kK2[] = {2, 3, 4, 6};
// Most pass levels any supported depth gives s stages (the tables' capacity).
int max_levels(int s, bool three)
{
    int m = 0;
    if (three)
        for (int k : kK3) m = std::max(m, npass(s, k));
    else
        for (int k : kK2) m = std::max(m, npass(s, k));
    return m;
}

bool validate(int nprob, const frkc2_grid *grids, const int *s, std::vector<KGrid> &kg)
{
    if (nprob < 1 || !grids || !s) {
        set_error("batched: need nprob >= 1 and non-NULL grids and s");
        return false;
    }
    kg.resize(nprob);
    for (int i = 0; i < nprob; ++i) {
        if (!make_kgrid(&grids[i], kg[i])) return false;
        if (kg[i].ndim < 2 ||
            (kg[i].op != FRKC2_OP_LAPLACE && kg[i].op != FRKC2_OP_VARCOEF)) {
            set_error("batched: problem %d must be 2D or 3D with a linear operator", i);
            return false;
        }
        if (s[i] < 2 || s[i] > kMaxStages || (s[i] % 2)) {
            set_error("batched: problem %d has invalid s = %d", i, s[i]);
            return false;
        }
        if (kg[i].ndim == 3 && !tb3d_plane_ok(kg[i])) {
            set_error("batched: problem %d has planes of 2^27 points or more", i);
            return false;
        }
    }
    return true;
}

Layout layout(int nprob, const std::vector<KGrid> &kg, const int *s)
{
    Layout L;
    int n3 = 0;
    L.levels3 = 0;
    L.levels2 = 0;
    for (int i = 0; i < nprob; ++i)
        if (kg[i].ndim == 3) {
            ++n3;
            L.levels3 = std::max(L.levels3, max_levels(s[i], true));
        } else {
            L.levels2 = std::max(L.levels2, max_levels(s[i], false));
        }
    const int cnt[2] = {n3, nprob - n3};
    const size_t sum_s = std::accumulate(s, s + nprob, (size_t)0);
    size_t o = 0;
    for (int d = 0; d < 2; ++d) {
        L.probs[d] = o;
        o = align_up(o + sizeof(BatchProblem) * (cnt[d] + 1));
    }
    L.pass3 = o;
    o = align_up(o + sizeof(long long) * kGroups3 * 2 * (size_t)L.levels3 * (n3 + 1));
    L.pass2 = o;
    o = align_up(o + sizeof(long long) * 2 * (size_t)L.levels2 * (cnt[1] + 1));
    L.tau = o;
    o = align_up(o + sizeof(double) * 2 * sum_s);
    L.partials = o;
    o = align_up(o + sizeof(double) * (kReduceBlocks + 2));
    L.bufs = o;
    L.buf_off.resize(nprob);
    for (int i = 0; i < nprob; ++i) {
        L.buf_off[i] = o;
        o = align_up(o + 2 * align_up((size_t)kg[i].npts() * 16));
    }
    L.total = o;
    return L;
}

struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<BatchProblem> probs[2];   // host copies of the uploaded tables
    std::vector<long long> pass3;         // 3D: per level, fused then single-stage prefixes
    std::vector<long long> pass2;         // 2D: the same
    int levels3 = 0, levels2 = 0;         // pass levels under cfg
    BatchCfg cfg;                         // resolved (cols3 set)
    int gcols[kGroups3] = {};             // output columns of each 3D group's fused tiles
    std::vector<double> tau;
};

std::mutex g_mu;
std::map<void *, GraphEntry> g_graphs;
// The timing autotuner is switched off (frkc2_batched_autotune's header block).
constexpr bool g_autotune_enabled = false;
BatchCfg g_forced{0, 0, 0};                                  // FRKC2_OPT_BATCH_*
std::map<std::vector<unsigned char>, BatchCfg> g_tuned;      // by problem-set shape
hipStream_t g_capture = nullptr, g_capture2 = nullptr;   // 3D group 0 and 2D branches
hipStream_t g_group[kGroups3] = {};                       // 3D groups 1.. (0 = g_capture)
hipEvent_t g_fork = nullptr, g_join = nullptr, g_gjoin[kGroups3] = {};

void append(std::vector<unsigned char> &k, const void *p, size_t n)
{
    const unsigned char *c = static_cast<const unsigned char *>(p);
    k.insert(k.end(), c, c + n);
}

int hip_err(hipError_t e, const char *what)
{
    set_error("batched: %s: HIP error %d (%s)", what, (int)e, hipGetErrorString(e));
    return FRKC2_EHIP;
}

// Upload the work tables (host copies kept in E) into ws on st, asynchronously.
// Every call uploads them, replays included, so that ws need not keep its
// contents between calls (a caller's allocator may hand the memory to other
// tensors in between).
hipError_t upload_tables(const GraphEntry &E, const Layout &L, char *base, hipStream_t st)
{
    hipError_t e = hipSuccess;
    if (!E.pass3.empty())
        e = hipMemcpyAsync(base + L.pass3, E.pass3.data(), sizeof(long long) * E.pass3.size(),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !E.pass2.empty())
        e = hipMemcpyAsync(base + L.pass2, E.pass2.data(), sizeof(long long) * E.pass2.size(),
                           hipMemcpyHostToDevice, st);
    for (int d = 0; d < 2 && e == hipSuccess; ++d) {
        if (E.probs[d].empty()) continue;
        e = hipMemcpyAsync(base + L.probs[d], E.probs[d].data(),
                           sizeof(BatchProblem) * E.probs[d].size(), hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(base + L.tau, E.tau.data(), sizeof(double) * E.tau.size(),
                           hipMemcpyHostToDevice, st);
    return e;
}

// The problem set as far as the launch configuration depends on it:
// dimension, extents, boundary, operator and s of every problem, in order.
std::vector<unsigned char> shape_key(int nprob, const std::vector<KGrid> &kg, const int *s)
{
    std::vector<unsigned char> k;
    append(k, &nprob, sizeof(nprob));
    for (int i = 0; i < nprob; ++i) {
        const int v[7] = {kg[i].ndim, kg[i].nx, kg[i].ny, kg[i].nz, kg[i].bc, kg[i].op, s[i]};
        append(k, v, sizeof(v));
    }
    return k;
}

// Output columns of the fused 3D tiles with less modelled work over every 3D
// problem's fused passes (one width per batch: a pass kernel that carries both
// widths needs more registers than it has). The items always fill the GPU, so
// work decides.
int model_cols(int nprob, const std::vector<KGrid> &kg, const int *s, int k3)
{
    long long w32 = 0, w64 = 0;
    for (int i = 0; i < nprob; ++i) {
        if (kg[i].ndim != 3) continue;
        const int zc = std::min(kg[i].nz, kChunkPlanes3);
        const long long f = nfull(s[i], k3);
        w32 += f * tb3d_work(k3, 32, kg[i].nx, kg[i].ny, kg[i].nz, zc);
        w64 += f * tb3d_work(k3, 64, kg[i].nx, kg[i].ny, kg[i].nz, zc);
    }
    return (w32 < w64) ? 32 : 64;
}

// The width with less modelled work for one problem.
int problem_cols(const KGrid &g, int k3)
{
    const int zc = std::min(g.nz, kChunkPlanes3);
    return tb3d_work(k3, 32, g.nx, g.ny, g.nz, zc) < tb3d_work(k3, 64, g.nx, g.ny, g.nz, zc) ? 32
                                                                                           : 64;
}

// Built-in configuration: depths 3 and 4, the modelled width.
BatchCfg default_cfg(int nprob, const std::vector<KGrid> &kg, const int *s)
{
    BatchCfg c;
    c.cols3 = model_cols(nprob, kg, s, c.k3);
    return c;
}

// Forced options where set, else the tuned entry, else the built-in one.
// Caller holds g_mu.
BatchCfg resolve_cfg(int nprob, const std::vector<KGrid> &kg, const int *s)
{
    BatchCfg c = default_cfg(nprob, kg, s);
    auto it = g_tuned.find(shape_key(nprob, kg, s));
    if (it != g_tuned.end()) c = it->second;
    if (g_forced.k3) c.k3 = g_forced.k3;
    if (g_forced.k2) c.k2 = g_forced.k2;
    if (g_forced.cols3) c.cols3 = g_forced.cols3;
    else if (g_forced.k3 && it == g_tuned.end()) c.cols3 = model_cols(nprob, kg, s, c.k3);
    return c;
}

void drop(GraphEntry &E)
{
    if (E.exec) hipGraphExecDestroy(E.exec);
    if (E.graph) hipGraphDestroy(E.graph);
    E.exec = nullptr;
    E.graph = nullptr;
    E.key.clear();
}

// Arguments shared by every batched call after validation.
struct Batch {
    int nprob;
    const frkc2_grid *grids;
    double *const *w;
    const double *const *D;
    const double *T;
    const int *s;
    double nu;
    std::vector<KGrid> kg;
};

int check_args(const Batch &B)
{
    if (!B.w || !B.D || !B.T) {
        set_error("batched: w, D and T arrays must be non-NULL");
        return FRKC2_EINVAL;
    }
    if (!(B.nu >= 0.0 && B.nu < 1.0)) {
        set_error("batched: nu must lie in [0, 1)");
        return FRKC2_EINVAL;
    }
    for (int i = 0; i < B.nprob; ++i) {
        if (!B.w[i] || (B.kg[i].op == FRKC2_OP_VARCOEF && !B.D[i])) {
            set_error("batched: problem %d lacks w or D", i);
            return FRKC2_EINVAL;
        }
        if (!(B.T[i] > 0.0) || !std::isfinite(B.T[i])) {
            set_error("batched: problem %d has invalid T", i);
            return FRKC2_EINVAL;
        }
    }
    return FRKC2_OK;
}

// Graph key: every argument the graph and its tables depend on, and the
// configuration.
std::vector<unsigned char> graph_key(const Batch &B, size_t ws_bytes, const BatchCfg &c)
{
    std::vector<unsigned char> key;
    append(key, &B.nprob, sizeof(B.nprob));
    append(key, B.grids, sizeof(frkc2_grid) * B.nprob);
    append(key, B.w, sizeof(double *) * B.nprob);
    append(key, B.D, sizeof(double *) * B.nprob);
    append(key, B.T, sizeof(double) * B.nprob);
    append(key, B.s, sizeof(int) * B.nprob);
    append(key, &B.nu, sizeof(B.nu));
    append(key, &ws_bytes, sizeof(ws_bytes));
    const int cv[3] = {c.k3, c.cols3, c.k2};
    append(key, cv, sizeof(cv));
    return key;
}

// Stability of every problem (Sec. 2: T rho <= betabar(s)). Synchronises st.
int check_stability(const Batch &B, const Layout &L, char *base, hipStream_t st)
{
    double *partials = reinterpret_cast<double *>(base + L.partials);
    std::vector<double> rmax(B.nprob, 0.0);
    for (int i = 0; i < B.nprob; ++i) {
        const KGrid &g = B.kg[i];
        if (g.op == FRKC2_OP_LAPLACE) {
            double sum = 0.0;
            for (int f = 0; f < 2 * g.ndim; ++f) sum = sum + g.d_const;
            rmax[i] = sum;
            continue;
        }
        hipError_t e = (hipError_t)launch_rho(g, B.w[i], B.D[i], partials, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&rmax[i], partials + kReduceBlocks, sizeof(double),
                               hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return hip_err(e, "rho check");
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e, "rho check");
    for (int i = 0; i < B.nprob; ++i) {
        frkc2_coeff_info info;
        int crc = coeffs_cached(B.s[i], B.nu, nullptr, nullptr, &info);
        if (crc < 0) return crc;
        const double rho = (2.0 * B.kg[i].inv_h2) * rmax[i];
        if (!std::isfinite(rho)) {
            set_error("batched: problem %d has a non-finite Gershgorin bound", i);
            return FRKC2_ENONFINITE;
        }
        if (B.T[i] * rho > info.beta_bar) {
            set_error("batched: problem %d: T*rho = %g exceeds beta_bar = %g", i, B.T[i] * rho,
                      info.beta_bar);
            return FRKC2_EUNSTABLE;
        }
    }
    return FRKC2_OK;
}

// Work tables of configuration c into E (host copies).
int build_tables(GraphEntry &E, const Batch &B, const Layout &L, const BatchCfg &c, char *base)
{
    const int *s = B.s;
    // 3D and 2D lists, each sorted by decreasing s (stable)
    std::vector<int> order(B.nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return s[a] > s[b]; });
    E.cfg = c;
    E.tau.clear();
    E.levels3 = E.levels2 = 0;
    for (int d = 0; d < 2; ++d) E.probs[d].clear();
    for (int i : order) {
        const KGrid &g = B.kg[i];
        const int d = (g.ndim == 3) ? 0 : 1;
        const double *are, *aim;
        int crc = coeffs_cached(s[i], B.nu, &are, &aim, nullptr);
        if (crc < 0) return crc;
        const size_t toff = E.tau.size();
        for (int l = 0; l < s[i]; ++l) {
            E.tau.push_back(B.T[i] * are[l]);
            E.tau.push_back(B.T[i] * aim[l]);
        }
        BatchProblem P{};
        P.w = B.w[i];
        P.D = B.D[i];
        P.bufA = reinterpret_cast<double *>(base + L.buf_off[i]);
        P.bufB = reinterpret_cast<double *>(base + L.buf_off[i] + align_up((size_t)g.npts() * 16));
        P.tau = reinterpret_cast<const double *>(base + L.tau) + toff;
        P.nx = g.nx;
        P.ny = g.ny;
        P.nz = g.nz;
        P.ndim = g.ndim;
        P.bc = g.bc;
        P.op = g.op;
        P.s = s[i];
        int bx, by;
        batched_tile(P.ndim, &bx, &by);
        P.zchunk = std::min(P.nz, kChunkPlanes);
        P.ntx = (P.nx + bx - 1) / bx;
        P.nty = (P.ndim == 3) ? (P.ny + by - 1) / by : 1;
        P.ntiles = P.ntx * P.nty * ((P.nz + P.zchunk - 1) / P.zchunk);
        P.zc3 = std::min(P.nz, kChunkPlanes3);
        if (P.ndim == 3) {
            int bx3, by3;
            P.nfull = nfull(P.s, c.k3);
            P.npass = npass(P.s, c.k3);
            P.cols3 = (c.cols3 == kColsPerProblem) ? problem_cols(g, c.k3) : c.cols3;
            batched_tile3(P.cols3, c.k3, &bx3, &by3);
            P.ntx3 = (P.nx + bx3 - 1) / bx3;
            P.nty3 = (P.ny + by3 - 1) / by3;
            P.ntiles3 = P.ntx3 * P.nty3 * ((P.nz + P.zc3 - 1) / P.zc3);
            E.levels3 = std::max(E.levels3, P.npass);
        } else {
            // fused rows: batched_row2(k2) output columns, up to kChunkPlanes3 rows
            const int row = batched_row2(c.k2);
            P.nfull = nfull(P.s, c.k2);
            P.npass = npass(P.s, c.k2);
            P.ntx3 = (P.nx + row - 1) / row;
            P.nty3 = 1;
            P.ntiles3 = P.ntx3 * ((P.nz + P.zc3 - 1) / P.zc3);
            E.levels2 = std::max(E.levels2, P.npass);
        }
        P.inv_h2 = g.inv_h2;
        P.d_const = g.d_const;
        E.probs[d].push_back(P);
    }
    if (E.levels3 > L.levels3 || E.levels2 > L.levels2) {
        set_error("batched: internal error: pass levels exceed the workspace tables");
        return FRKC2_EINVAL;
    }
    // 3D groups: alternate problems of the list (decreasing s); with a width
    // per problem, the 32-column problems and the 64-column ones (each group
    // runs one kernel, so one width), alternating if all have one width.
    const int n3 = (int)E.probs[0].size();
    std::vector<int> grp(n3);
    bool mixed = false;
    for (int j = 1; j < n3; ++j) mixed = mixed || E.probs[0][j].cols3 != E.probs[0][0].cols3;
    for (int j = 0; j < n3; ++j) grp[j] = mixed ? (E.probs[0][j].cols3 == 64) : (j % kGroups3);
    for (int g = 0; g < kGroups3; ++g)
        E.gcols[g] = mixed ? (g == 1 ? 64 : 32) : (n3 ? E.probs[0][0].cols3 : 64);
    // 3D pass tables: row (g, L, kind) = group g's items of pass level L
    // (kind 0 fused, 1 single stage), prefix sums over the 3D list
    E.pass3.assign(kGroups3 * 2 * (size_t)E.levels3 * (n3 + 1), 0);
    for (int g = 0; g < kGroups3; ++g)
        for (int lv = 0; lv < E.levels3; ++lv) {
            const size_t r0 = (size_t)(g * 2 * E.levels3 + 2 * lv);
            long long *fa = &E.pass3[r0 * (n3 + 1)];
            long long *sg = &E.pass3[(r0 + 1) * (n3 + 1)];
            for (int j = 0; j < n3; ++j) {
                const BatchProblem &P = E.probs[0][j];
                const bool mine = grp[j] == g;
                fa[j + 1] = fa[j] + (mine && lv < P.nfull ? P.ntiles3 : 0);
                sg[j + 1] = sg[j] + (mine && lv >= P.nfull && lv < P.npass ? P.ntiles : 0);
            }
        }
    // 2D pass tables, the same layout over the 2D list
    const int n2 = (int)E.probs[1].size();
    E.pass2.assign(2 * (size_t)E.levels2 * (n2 + 1), 0);
    for (int lv = 0; lv < E.levels2; ++lv) {
        long long *fa = &E.pass2[(size_t)(2 * lv) * (n2 + 1)];
        long long *sg = &E.pass2[(size_t)(2 * lv + 1) * (n2 + 1)];
        for (int j = 0; j < n2; ++j) {
            const BatchProblem &P = E.probs[1][j];
            fa[j + 1] = fa[j] + (lv < P.nfull ? P.ntiles3 : 0);
            sg[j + 1] = sg[j] + (lv >= P.nfull && lv < P.npass ? P.ntiles : 0);
        }
    }
    return FRKC2_OK;
}

// Tables of configuration c, uploaded, and the graph captured and
// instantiated into E (not launched). Synchronises st. Caller holds g_mu.
int build_graph(GraphEntry &E, const Batch &B, const Layout &L, const BatchCfg &c, char *base,
                hipStream_t st)
{
    drop(E);
    int rc = build_tables(E, B, L, c, base);
    if (rc < 0) return rc;
    hipError_t e = upload_tables(E, L, base, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e, "table upload");

    // ---- capture: the 3D groups' pass levels on one branch each, the 2D
    // levels on another, forked from and joined into the capture stream ----
    if (!g_capture) {
        e = hipStreamCreate(&g_capture);
        if (e == hipSuccess) e = hipStreamCreate(&g_capture2);
        for (int g = 1; g < kGroups3 && e == hipSuccess; ++g) {
            e = hipStreamCreate(&g_group[g]);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&g_gjoin[g], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g_join, hipEventDisableTiming);
        if (e != hipSuccess) return hip_err(e, "capture streams");
    }
    int grid_max[2] = {batched_grid_size(3), batched_grid_size(2)};
    if (grid_max[0] <= 0 || grid_max[1] <= 0) return hip_err(hipErrorInvalidValue, "occupancy query");
    e = hipStreamBeginCapture(g_capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_err(e, "begin capture");
    const int n3 = (int)E.probs[0].size(), n2 = (int)E.probs[1].size();
    const bool has2 = n2 > 0;
    int lrc = (int)hipEventRecord(g_fork, g_capture);
    for (int g = 1; g < kGroups3 && lrc == 0; ++g) lrc = (int)hipStreamWaitEvent(g_group[g], g_fork, 0);
    if (has2 && lrc == 0) lrc = (int)hipStreamWaitEvent(g_capture2, g_fork, 0);
    auto grid_for = [&](int d, long long items) {
        long long grid = std::min<long long>(grid_max[d], (items + 7) / 8 * 8);
        return (int)std::max<long long>(grid, 1);
    };
    const long long *pass3_dev = reinterpret_cast<const long long *>(base + L.pass3);
    for (int g = 0; g < kGroups3 && lrc == 0; ++g)
        for (int lv = 0; lv < E.levels3 && lrc == 0; ++lv) {
            for (int kind = 0; kind < 2 && lrc == 0; ++kind) {
                const size_t row = (size_t)(g * 2 * E.levels3 + 2 * lv + kind) * (n3 + 1);
                const long long items = E.pass3[row + n3];
                if (items == 0) continue;
                // fused items: one workgroup each; single-stage items: a
                // grid that fills the GPU, each workgroup a range of items
                if (kind == 0 && items > 0x7fffffffLL) {
                    lrc = (int)hipErrorInvalidValue;
                    break;
                }
                lrc = launch_batched_pass3(
                    kind == 0, E.gcols[g], c.k3,
                    reinterpret_cast<const BatchProblem *>(base + L.probs[0]), pass3_dev + row,
                    items, n3, lv, kind == 0 ? (int)items : grid_for(0, items),
                    g == 0 ? g_capture : g_group[g]);
            }
        }
    const long long *pass2_dev = reinterpret_cast<const long long *>(base + L.pass2);
    for (int lv = 0; lv < E.levels2 && lrc == 0 && has2; ++lv) {
        for (int kind = 0; kind < 2 && lrc == 0; ++kind) {
            const size_t row = (size_t)(2 * lv + kind) * (n2 + 1);
            const long long items = E.pass2[row + n2];
            if (items == 0) continue;
            lrc = launch_batched_pass2(kind == 0, c.k2,
                                       reinterpret_cast<const BatchProblem *>(base + L.probs[1]),
                                       pass2_dev + row, items, n2, lv, grid_for(1, items),
                                       g_capture2);
        }
    }
    for (int g = 1; g < kGroups3; ++g) {
        const int r1 = (int)hipEventRecord(g_gjoin[g], g_group[g]);
        const int r2 = (int)hipStreamWaitEvent(g_capture, g_gjoin[g], 0);
        if (lrc == 0) lrc = r1 ? r1 : r2;
    }
    if (has2) {
        const int r1 = (int)hipEventRecord(g_join, g_capture2);
        const int r2 = (int)hipStreamWaitEvent(g_capture, g_join, 0);
        if (lrc == 0) lrc = r1 ? r1 : r2;
    }
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(g_capture, &graph);
    if (lrc != 0) {
        if (graph) hipGraphDestroy(graph);
        return hip_err((hipError_t)lrc, "capture launch");
    }
    if (e2 != hipSuccess) return hip_err(e2, "end capture");
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return hip_err(e, "instantiate");
    }
    E.graph = graph;
    E.exec = exec;
    return FRKC2_OK;
}

int launch_graph(const GraphEntry &E, const Layout &L, char *base, hipStream_t st)
{
    hipError_t e = upload_tables(E, L, base, st);
    if (e == hipSuccess) e = hipGraphLaunch(E.exec, st);
    return e == hipSuccess ? FRKC2_OK : hip_err(e, "graph launch");
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

int batched_set_option(int key, int value)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (key == FRKC2_OPT_BATCH_K3 && (value == 0 || value == 2 || value == 3)) {
        g_forced.k3 = value;
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_BATCH_COLS &&
        (value == 0 || value == kColsPerProblem || value == 32 || value == 64)) {
        g_forced.cols3 = value;
        return FRKC2_OK;
    }
    if (key == FRKC2_OPT_BATCH_K2 && (value == 0 || value == 2 || value == 3 || value == 4 ||
                                       value == 6)) {
        g_forced.k2 = value;
        return FRKC2_OK;
    }
    set_error("batched option %d: unsupported value %d (3D depth 2 or 3, width 32, 64 or 1 "
              "(per problem), 2D depth 2, 3, 4 or 6; 0 = automatic)", key, value);
    return FRKC2_EINVAL;
}

void batched_clear_tuned()
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_tuned.clear();
}

}  // namespace frkc2

using namespace frkc2;

extern "C" size_t frkc2_batched_workspace_bytes(int nprob, const frkc2_grid *grids, const int *s)
{
    std::vector<KGrid> kg;
    if (!validate(nprob, grids, s, kg)) return 0;
    return layout(nprob, kg, s).total;
}

extern "C" int frkc2_step_batched(int nprob, const frkc2_grid *grids, double *const *w,
                                  const double *const *D, const double *T, const int *s,
                                  double nu, void *ws, size_t ws_bytes, hipStream_t st)
{
    Batch B{nprob, grids, w, D, T, s, nu, {}};
    if (!validate(nprob, grids, s, B.kg)) return FRKC2_EINVAL;
    int rc = check_args(B);
    if (rc < 0) return rc;
    const Layout L = layout(nprob, B.kg, s);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) {
        set_error("batched: workspace needs %zu bytes (got %zu), 256-byte aligned", L.total,
                  ws_bytes);
        return FRKC2_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const BatchCfg cfg = resolve_cfg(nprob, B.kg, s);
    std::vector<unsigned char> key = graph_key(B, ws_bytes, cfg);
    GraphEntry &E = g_graphs[ws];
    char *base = static_cast<char *>(ws);
    if (E.exec && E.key == key) return launch_graph(E, L, base, st);
    drop(E);
    // stability, checked when the graph is built; replays assume the same D,
    // as the graph does
    rc = check_stability(B, L, base, st);
    if (rc < 0) return rc;
    rc = build_graph(E, B, L, cfg, base, st);
    if (rc < 0) return rc;
    E.key = key;
    return launch_graph(E, L, base, st);
}

extern "C" int frkc2_batched_autotune(int nprob, const frkc2_grid *grids, double *const *w,
                                      const double *const *D, const double *T, const int *s,
                                      double nu, int reps, void *ws, size_t ws_bytes,
                                      hipStream_t st, frkc2_batch_tune_result *res)
{
    Batch B{nprob, grids, w, D, T, s, nu, {}};
    if (!validate(nprob, grids, s, B.kg)) return FRKC2_EINVAL;
    int rc = check_args(B);
    if (rc < 0) return rc;
    if (!res || reps < 1 || reps > 100) {
        set_error("batched autotune: need a result pointer and 1 <= reps <= 100 (got %d)", reps);
        return FRKC2_EINVAL;
    }
    const Layout L = layout(nprob, B.kg, s);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) {
        set_error("batched: workspace needs %zu bytes (got %zu), 256-byte aligned", L.total,
                  ws_bytes);
        return FRKC2_ENOMEM;
    }
    if (!g_autotune_enabled) {
        set_error("batched autotune: switched off in this version (runs that rebuilt the batch "
                  "graph per candidate ended in a host heap corruption inside this call, cause "
                  "not found); frkc2_step_batched uses the options or the built-in "
                  "configuration");
        return FRKC2_EDISABLED;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    GraphEntry &E = g_graphs[ws];
    char *base = static_cast<char *>(ws);
    drop(E);
    rc = check_stability(B, L, base, st);
    if (rc < 0) return rc;
    EventPair ev;
    hipError_t e = hipEventCreate(&ev.a);
    if (e == hipSuccess) e = hipEventCreate(&ev.b);
    if (e != hipSuccess) return hip_err(e, "autotune: event");
    // One warm-up superstep, then reps timed ones; each advances w.
    auto time_cfg = [&](const BatchCfg &c, double *ms) -> int {
        int r = build_graph(E, B, L, c, base, st);
        if (r < 0) return r;
        if ((r = launch_graph(E, L, base, st)) < 0) return r;
        hipError_t he = hipEventRecord(ev.a, st);
        if (he != hipSuccess) return hip_err(he, "autotune: event");
        for (int i = 0; i < reps; ++i)
            if ((r = launch_graph(E, L, base, st)) < 0) return r;
        he = hipEventRecord(ev.b, st);
        if (he == hipSuccess) he = hipEventSynchronize(ev.b);
        float t = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&t, ev.a, ev.b);
        if (he != hipSuccess) return hip_err(he, "autotune: timing");
        *ms = (double)t / reps;
        return FRKC2_OK;
    };
    bool has3 = false, has2 = false;
    for (const KGrid &g : B.kg) (g.ndim == 3 ? has3 : has2) = true;
    const BatchCfg dflt = default_cfg(nprob, B.kg, s);
    double ms_default = 0.0;
    rc = time_cfg(dflt, &ms_default);
    if (rc < 0) return rc;
    BatchCfg best = dflt;
    double ms_best = ms_default;
    int n = 1;
    std::vector<BatchCfg> tried{dflt};
    auto consider = [&](const BatchCfg &c) -> int {
        for (const BatchCfg &t : tried)
            if (c.k3 == t.k3 && c.cols3 == t.cols3 && c.k2 == t.k2) return FRKC2_OK;
        tried.push_back(c);
        double ms = 0.0;
        int r = time_cfg(c, &ms);
        if (r < 0) return r;
        ++n;
        if (ms < ms_best) {
            ms_best = ms;
            best = c;
        }
        return FRKC2_OK;
    };
    // the 3D depth and width with the default 2D depth, then the 2D depth
    // with the best of those (the 2D passes run beside the 3D ones)
    if (has3)
        for (int k3 : kK3)
            for (int cols : {32, 64, kColsPerProblem}) {
                BatchCfg c = best;
                c.k3 = k3;
                c.cols3 = cols;
                if ((rc = consider(c)) < 0) return rc;
            }
    if (has2)
        for (int k2 : kK2) {
            BatchCfg c = best;
            c.k2 = k2;
            if ((rc = consider(c)) < 0) return rc;
        }
    // The default ran first, while clocks and caches settle: time it again
    // and keep it unless a candidate is clearly faster, so that timing noise
    // does not flip the configuration from run to run.
    double ms_again = 0.0;
    rc = time_cfg(dflt, &ms_again);
    if (rc < 0) return rc;
    ms_default = std::min(ms_default, ms_again);
    if (ms_default <= 1.02 * ms_best) {
        best = dflt;
        ms_best = ms_default;
    }
    drop(E);   // the next frkc2_step_batched builds the chosen configuration
    g_tuned[shape_key(nprob, B.kg, s)] = best;
    res->k3 = best.k3;
    res->cols3 = best.cols3;
    res->k2 = best.k2;
    res->candidates = n;
    res->ms_best = ms_best;
    res->ms_default = ms_default;
    return FRKC2_OK;
}

extern "C" int frkc2_batched_config(int nprob, const frkc2_grid *grids, const int *s, int *k3,
                                    int *cols3, int *k2)
{
    std::vector<KGrid> kg;
    if (!validate(nprob, grids, s, kg)) return FRKC2_EINVAL;
    if (!k3 || !cols3 || !k2) {
        set_error("batched config: output pointers must be non-NULL");
        return FRKC2_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const BatchCfg c = resolve_cfg(nprob, kg, s);
    *k3 = c.k3;
    *cols3 = c.cols3;
    *k2 = c.k2;
    return FRKC2_OK;
}

extern "C" int frkc2_batched_status(void *ws, hipStream_t st)
{
    if (!ws) {
        set_error("batched: workspace is NULL");
        return FRKC2_EINVAL;
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_graphs.find(ws);
        if (it == g_graphs.end() || !it->second.exec) {
            set_error("batched: no batched launch recorded for this workspace");
            return FRKC2_EINVAL;
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e, "status");
    return FRKC2_OK;
}

extern "C" int frkc2_batched_release(void *ws)
{
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_graphs.find(ws);
    if (it == g_graphs.end()) return FRKC2_OK;
    drop(it->second);
    g_graphs.erase(it);
    return FRKC2_OK;
}
