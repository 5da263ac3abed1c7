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
    int levels3;                                   // pass levels of the 3D list
    size_t pass2;                                  // 2D pass tables: 2 * levels2 rows of n2 + 1
    int levels2;
    std::vector<size_t> buf_off;                   // per problem (caller's order)
};

// Passes of a 3D problem: fused passes of kBatchK stages, then single stages.
int nfull3(int s) { return s / kBatchK; }
int npass3(int s) { return nfull3(s) + (s - kBatchK * nfull3(s)); }
// 2D: fused passes of kBatchK2 stages, then single stages. A lone fused pass
// would read and write w (its tiles read a halo around them), so s = kBatchK2
// runs as single stages.
int nfull2(int s) { return (s == kBatchK2) ? 0 : s / kBatchK2; }
int npass2(int s) { return nfull2(s) + (s - kBatchK2 * nfull2(s)); }

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
            L.levels3 = std::max(L.levels3, npass3(s[i]));
        } else {
            L.levels2 = std::max(L.levels2, npass2(s[i]));
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
    int cols3 = 64;                       // 3D fused tiles: output columns (one width per batch)
    std::vector<double> tau;
};

std::mutex g_mu;
std::map<void *, GraphEntry> g_graphs;
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

void drop(GraphEntry &E)
{
    if (E.exec) hipGraphExecDestroy(E.exec);
    if (E.graph) hipGraphDestroy(E.graph);
    E.exec = nullptr;
    E.graph = nullptr;
    E.key.clear();
}

}  // namespace
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
    std::vector<KGrid> kg;
    if (!validate(nprob, grids, s, kg)) return FRKC2_EINVAL;
    if (!w || !D || !T) {
        set_error("batched: w, D and T arrays must be non-NULL");
        return FRKC2_EINVAL;
    }
    if (!(nu >= 0.0 && nu < 1.0)) {
        set_error("batched: nu must lie in [0, 1)");
        return FRKC2_EINVAL;
    }
    for (int i = 0; i < nprob; ++i) {
        if (!w[i] || (kg[i].op == FRKC2_OP_VARCOEF && !D[i])) {
            set_error("batched: problem %d lacks w or D", i);
            return FRKC2_EINVAL;
        }
        if (!(T[i] > 0.0) || !std::isfinite(T[i])) {
            set_error("batched: problem %d has invalid T", i);
            return FRKC2_EINVAL;
        }
    }
    const Layout L = layout(nprob, kg, s);
    if (!ws || ws_bytes < L.total || ((uintptr_t)ws & 255u)) {
        set_error("batched: workspace needs %zu bytes (got %zu), 256-byte aligned", L.total,
                  ws_bytes);
        return FRKC2_ENOMEM;
    }
    std::vector<unsigned char> key;
    append(key, &nprob, sizeof(nprob));
    append(key, grids, sizeof(frkc2_grid) * nprob);
    append(key, w, sizeof(double *) * nprob);
    append(key, D, sizeof(double *) * nprob);
    append(key, T, sizeof(double) * nprob);
    append(key, s, sizeof(int) * nprob);
    append(key, &nu, sizeof(nu));
    append(key, &ws_bytes, sizeof(ws_bytes));

    std::lock_guard<std::mutex> lk(g_mu);
    GraphEntry &E = g_graphs[ws];
    char *base = static_cast<char *>(ws);
    if (E.exec && E.key == key) {
        hipError_t e = upload_tables(E, L, base, st);
        if (e == hipSuccess) e = hipGraphLaunch(E.exec, st);
        return e == hipSuccess ? FRKC2_OK : hip_err(e, "graph launch");
    }
    drop(E);
    // ---- stability of every problem (Sec. 2: T rho <= betabar(s)), checked
    // when the graph is built; replays assume the same D, as the graph does ----
    {
        double *partials = reinterpret_cast<double *>(base + L.partials);
        std::vector<double> rmax(nprob, 0.0);
        for (int i = 0; i < nprob; ++i) {
            if (kg[i].op == FRKC2_OP_LAPLACE) {
                double sum = 0.0;
                for (int f = 0; f < 2 * kg[i].ndim; ++f) sum = sum + kg[i].d_const;
                rmax[i] = sum;
                continue;
            }
            int rc = launch_rho(kg[i], w[i], D[i], partials, st);
            hipError_t e = (hipError_t)rc;
            if (e == hipSuccess)
                e = hipMemcpyAsync(&rmax[i], partials + kReduceBlocks, sizeof(double),
                                   hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) return hip_err(e, "rho check");
        }
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_err(e, "rho check");
        for (int i = 0; i < nprob; ++i) {
            frkc2_coeff_info info;
            int crc = coeffs_cached(s[i], nu, nullptr, nullptr, &info);
            if (crc < 0) return crc;
            const double rho = (2.0 * kg[i].inv_h2) * rmax[i];
            if (!std::isfinite(rho)) {
                set_error("batched: problem %d has a non-finite Gershgorin bound", i);
                return FRKC2_ENONFINITE;
            }
            if (T[i] * rho > info.beta_bar) {
                set_error("batched: problem %d: T*rho = %g exceeds beta_bar = %g", i, T[i] * rho,
                          info.beta_bar);
                return FRKC2_EUNSTABLE;
            }
        }
    }
    // ---- work tables: 3D and 2D lists, each sorted by decreasing s (stable) ----
    std::vector<int> order(nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return s[a] > s[b]; });
    // One tile width for all 3D problems (a pass kernel that carries both
    // widths needs more registers than it has): the one with less total work
    // over the fused passes. The items always fill the GPU, so work decides.
    {
        long long w32 = 0, w64 = 0;
        for (int i = 0; i < nprob; ++i) {
            if (kg[i].ndim != 3) continue;
            const int zc = std::min(kg[i].nz, kChunkPlanes3);
            w32 += (long long)nfull3(s[i]) * tb3d_work(32, kg[i].nx, kg[i].ny, kg[i].nz, zc);
            w64 += (long long)nfull3(s[i]) * tb3d_work(64, kg[i].nx, kg[i].ny, kg[i].nz, zc);
        }
        E.cols3 = (w32 < w64) ? 32 : 64;
    }
    E.tau.clear();
    for (int d = 0; d < 2; ++d) E.probs[d].clear();
    for (int i : order) {
        const int d = (kg[i].ndim == 3) ? 0 : 1;
        const double *are, *aim;
        int crc = coeffs_cached(s[i], nu, &are, &aim, nullptr);
        if (crc < 0) return crc;
        const size_t toff = E.tau.size();
        for (int l = 0; l < s[i]; ++l) {
            E.tau.push_back(T[i] * are[l]);
            E.tau.push_back(T[i] * aim[l]);
        }
        BatchProblem P{};
        P.w = w[i];
        P.D = D[i];
        P.bufA = reinterpret_cast<double *>(base + L.buf_off[i]);
        P.bufB = reinterpret_cast<double *>(base + L.buf_off[i] + align_up((size_t)kg[i].npts() * 16));
        P.tau = reinterpret_cast<const double *>(base + L.tau) + toff;
        P.nx = kg[i].nx;
        P.ny = kg[i].ny;
        P.nz = kg[i].nz;
        P.ndim = kg[i].ndim;
        P.bc = kg[i].bc;
        P.op = kg[i].op;
        P.s = s[i];
        int bx, by;
        batched_tile(P.ndim, &bx, &by);
        P.zchunk = std::min(P.nz, kChunkPlanes);
        P.ntx = (P.nx + bx - 1) / bx;
        P.nty = (P.ndim == 3) ? (P.ny + by - 1) / by : 1;
        P.ntiles = P.ntx * P.nty * ((P.nz + P.zchunk - 1) / P.zchunk);
        if (P.ndim == 3) {
            int bx3, by3;
            P.nfull = nfull3(P.s);
            P.npass = npass3(P.s);
            P.zc3 = std::min(P.nz, kChunkPlanes3);
            P.cols3 = E.cols3;
            batched_tile3(P.cols3, &bx3, &by3);
            P.ntx3 = (P.nx + bx3 - 1) / bx3;
            P.nty3 = (P.ny + by3 - 1) / by3;
            P.ntiles3 = P.ntx3 * P.nty3 * ((P.nz + P.zc3 - 1) / P.zc3);
        } else {
            // fused rows: batched_row2() output columns, up to kChunkPlanes3 rows
            P.nfull = nfull2(P.s);
            P.npass = npass2(P.s);
            P.zc3 = std::min(P.nz, kChunkPlanes3);
            P.ntx3 = (P.nx + batched_row2() - 1) / batched_row2();
            P.nty3 = 1;
            P.ntiles3 = P.ntx3 * ((P.nz + P.zc3 - 1) / P.zc3);
        }
        P.inv_h2 = kg[i].inv_h2;
        P.d_const = kg[i].d_const;
        E.probs[d].push_back(P);
    }
    // 3D pass tables: row 2L = fused items of level L, row 2L+1 = single-stage items
    const int n3 = (int)E.probs[0].size();
    // row (g, L, kind): group g's items of pass level L (kind 0 fused, 1 single)
    E.pass3.assign(kGroups3 * 2 * (size_t)L.levels3 * (n3 + 1), 0);
    for (int g = 0; g < kGroups3; ++g)
        for (int lv = 0; lv < L.levels3; ++lv) {
            const size_t r0 = (size_t)(g * 2 * L.levels3 + 2 * lv);
            long long *fa = &E.pass3[r0 * (n3 + 1)];
            long long *sg = &E.pass3[(r0 + 1) * (n3 + 1)];
            for (int j = 0; j < n3; ++j) {
                const BatchProblem &P = E.probs[0][j];
                const bool mine = (j % kGroups3) == g;
                fa[j + 1] = fa[j] + (mine && lv < P.nfull ? P.ntiles3 : 0);
                sg[j + 1] = sg[j] + (mine && lv >= P.nfull && lv < P.npass ? P.ntiles : 0);
            }
        }
    // 2D pass tables, the same layout over the 2D list
    const int n2 = (int)E.probs[1].size();
    E.pass2.assign(2 * (size_t)L.levels2 * (n2 + 1), 0);
    for (int lv = 0; lv < L.levels2; ++lv) {
        long long *fa = &E.pass2[(size_t)(2 * lv) * (n2 + 1)];
        long long *sg = &E.pass2[(size_t)(2 * lv + 1) * (n2 + 1)];
        for (int j = 0; j < n2; ++j) {
            const BatchProblem &P = E.probs[1][j];
            fa[j + 1] = fa[j] + (lv < P.nfull ? P.ntiles3 : 0);
            sg[j + 1] = sg[j] + (lv >= P.nfull && lv < P.npass ? P.ntiles : 0);
        }
    }
    hipError_t e = upload_tables(E, L, base, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_err(e, "table upload");

    // ---- capture: the 3D pass levels on one stream, the 2D stage levels on a
    // second one forked from it, joined before the end ----
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
    int lrc = 0;
    const bool has2 = !E.probs[1].empty();
    lrc = (int)hipEventRecord(g_fork, g_capture);
    for (int g = 1; g < kGroups3 && lrc == 0; ++g) lrc = (int)hipStreamWaitEvent(g_group[g], g_fork, 0);
    if (has2 && lrc == 0) lrc = (int)hipStreamWaitEvent(g_capture2, g_fork, 0);
    auto grid_for = [&](int d, long long items) {
        long long grid = std::min<long long>(grid_max[d], (items + 7) / 8 * 8);
        return (int)std::max<long long>(grid, 1);
    };
    const long long *pass3_dev = reinterpret_cast<const long long *>(base + L.pass3);
    for (int g = 0; g < kGroups3 && lrc == 0; ++g)
        for (int lv = 0; lv < L.levels3 && lrc == 0; ++lv) {
            for (int kind = 0; kind < 2 && lrc == 0; ++kind) {
                const size_t row = (size_t)(g * 2 * L.levels3 + 2 * lv + kind) * (n3 + 1);
                const long long items = E.pass3[row + n3];
                if (items == 0) continue;
                lrc = launch_batched_pass3(
                    kind == 0, E.cols3, reinterpret_cast<const BatchProblem *>(base + L.probs[0]),
                    pass3_dev + row, items, n3, lv, grid_for(0, items),
                    g == 0 ? g_capture : g_group[g]);
            }
        }
    const long long *pass2_dev = reinterpret_cast<const long long *>(base + L.pass2);
    for (int lv = 0; lv < L.levels2 && lrc == 0 && has2; ++lv) {
        for (int kind = 0; kind < 2 && lrc == 0; ++kind) {
            const size_t row = (size_t)(2 * lv + kind) * (n2 + 1);
            const long long items = E.pass2[row + n2];
            if (items == 0) continue;
            lrc = launch_batched_pass2(kind == 0,
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
    E.key = key;
    e = hipGraphLaunch(E.exec, st);
    return e == hipSuccess ? FRKC2_OK : hip_err(e, "graph launch");
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
