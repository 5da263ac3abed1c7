// Temporally blocked 3D stages with full-width output tiles: K consecutive
// Euler stages W <- W + tau_l f(W) (O'Sullivan, arXiv:1702.03818, Sec. 3,
// Euler-step equation) in one HBM pass.
//
// Same pipeline as tb_stage (tblock.hip): a workgroup marches through a chunk
// of z planes and at time step t computes level m (the state after m stages
// of the pass) at plane t - m from level m-1, whose x/y neighbours sit in LDS
// and whose z neighbours the thread keeps in registers. What differs is the
// tile geometry and the synchronisation:
//
//  * The output tile is 64 columns wide, one wavefront per row, so it lines
//    up with 512-byte segments of the grid and a 256-wide grid needs exactly
//    4 tiles across. The K halo columns on each side of every row are
//    computed by one or two extra "halo" wavefronts whose lanes each own one
//    (row, halo column) pair. A wavefront computes the levels one of its
//    lanes needs (level m is used within K - m cells of the output), so rows
//    near the tile edge skip whole levels.
//  * The LDS planes are double-buffered by time-step parity, so one barrier
//    per time step separates the writes of step t from the reads of step
//    t + 1. The diffusivity ring holds K + 2 planes for the same reason. The
//    plane row stride is odd, which keeps the column-wise halo wavefronts
//    free of bank conflicts.
//  * The thread's own diffusivity of planes t-2 .. t comes from its register
//    ring; only x/y neighbours (and older planes) are read from LDS. The
//    level windows live in a register ring indexed by the unrolled step.
//
// Every value is computed with the same per-point arithmetic, in the same
// order, as the one-stage kernel (faces x-, x+, y-, y+, z-, z+; face() and
// euler() of device_common.h), so the results are identical to the last bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tb3d_tile.h"

namespace frkc2 {
namespace {

using namespace dev;

// tb3d_stage: one workgroup per tile, the block index remapped so that each
// XCD receives a contiguous range of tiles.
template <int OP, int BC, int K, bool IN_REAL, bool OUT_REAL, bool EMB = false, bool ST = false,
          int W = 64, bool REV = false>
__global__ __launch_bounds__(1024) void tb3d_stage(Tb3Args a)
{
    __shared__ double2 sL[Tb3Lds<OP, K, W, EMB>::L];
    __shared__ double sD[Tb3Lds<OP, K, W, EMB>::D];   // the D ring where EMB turns the faces off
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % a.ntx;
    lb /= a.ntx;
    const int by = lb % a.nty;
    const int bz = lb / a.nty;
    tb3d_tile<OP, BC, K, IN_REAL, OUT_REAL, EMB, ST, W, !EMB, true, REV>(a, bx, by, bz, sL, sD);
}

// Chunk length: one workgroup fills a CU (its LDS), so the launch runs in
// rounds of n_cu workgroups, each as long as a full chunk of zc + 2K steps.
// Pick the chunk length (every one down to 8 planes) that maximises the
// useful planes per CU-step, tiles * nz / (rounds * n_cu * (zc + 2K)); on a
// tie the longest.
int cu_count()
{
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            v > 0)
            n_cu = v;
        else
            n_cu = 256;
    }
    return n_cu;
}

int choose_zchunk3(long long tiles, int nz, int K)
{
    const int n_cu = cu_count();
    // every chunk length down to 8 planes (a host loop of at most nz steps);
    // the longest of equally good ones
    int best = nz;
    double best_eff = -1.0;
    for (int zc = nz; zc >= 1; --zc) {
        if (zc < 8 && zc < nz) break;
        const long long nblk = tiles * ((nz + zc - 1) / zc);
        const long long rounds = (nblk + n_cu - 1) / n_cu;
        const double eff =
            (double)tiles * nz / ((double)rounds * n_cu * (zc + 2.0 * K));
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = zc;
        }
    }
    return best;
}

template <int OP, int BC, int K, int W>
int launch3_k(const Tb3Args &a0, bool ir, bool orl, bool rev, hipStream_t st)
{
    Tb3Args a = a0;
    a.ntx = (a.nx + W - 1) / W;
    a.nty = (a.ny + Tb3Shape<K, W>::BYO - 1) / Tb3Shape<K, W>::BYO;
    const long long tiles = (long long)a.ntx * a.nty;
    a.zchunk = (a0.zchunk > 0) ? min(a0.zchunk, a.nz) : choose_zchunk3(tiles, a.nz, K);
    const long long nblk = tiles * ((a.nz + a.zchunk - 1) / a.zchunk);
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(1024);
    if (a.lvl_out) {
        // stage states of the adjoint's forward recompute: complex in and out
        if (ir || orl || a.emb_out || !(OP == LAP || OP == VAR)) return (int)hipErrorInvalidValue;
        if constexpr (OP == LAP || OP == VAR)
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, false, false, false, true, W>), grid, block, 0,
                               st, a);
        return (int)hipGetLastError();
    }
    if (a.emb_out) {
        if (orl) return (int)hipErrorInvalidValue;
        if (ir)
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, true, false, true, false, W>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, false, false, true, false, W>), grid, block, 0, st, a);
        return (int)hipGetLastError();
    }
    if (rev) {
        if (ir && orl)
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, true, true, false, false, W, true>), grid, block, 0, st, a);
        else if (ir)
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, true, false, false, false, W, true>), grid, block, 0, st, a);
        else if (orl)
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, false, true, false, false, W, true>), grid, block, 0, st, a);
        else
            hipLaunchKernelGGL((tb3d_stage<OP, BC, K, false, false, false, false, W, true>), grid, block, 0, st, a);
        return (int)hipGetLastError();
    }
    if (ir && orl)
        hipLaunchKernelGGL((tb3d_stage<OP, BC, K, true, true, false, false, W>), grid, block, 0, st, a);
    else if (ir)
        hipLaunchKernelGGL((tb3d_stage<OP, BC, K, true, false, false, false, W>), grid, block, 0, st, a);
    else if (orl)
        hipLaunchKernelGGL((tb3d_stage<OP, BC, K, false, true, false, false, W>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((tb3d_stage<OP, BC, K, false, false, false, false, W>), grid, block, 0, st, a);
    return (int)hipGetLastError();
}

template <int OP, int BC>
int launch3_kk(int k, int cols, const Tb3Args &a, bool ir, bool orl, bool rev, hipStream_t st)
{
    if (cols == 32) {
        if (k == 2) return launch3_k<OP, BC, 2, 32>(a, ir, orl, rev, st);
        if (k == 3) return launch3_k<OP, BC, 3, 32>(a, ir, orl, rev, st);
        return (int)hipErrorInvalidValue;
    }
    if (k == 2) return launch3_k<OP, BC, 2, 64>(a, ir, orl, rev, st);
    if (k == 3) return launch3_k<OP, BC, 3, 64>(a, ir, orl, rev, st);
    return (int)hipErrorInvalidValue;
}

template <int OP>
int launch3_bc(const KGrid &g, int k, int cols, const Tb3Args &a, bool ir, bool orl, bool rev,
               hipStream_t st)
{
    if (g.bc == PER) return launch3_kk<OP, PER>(k, cols, a, ir, orl, rev, st);
    return launch3_kk<OP, DIR>(k, cols, a, ir, orl, rev, st);
}

// Predicted time of a pass in units of one time step of the 64-column tile:
// rounds of n_cu workgroups, each zc + 2K steps of the tile's step cost.
template <int K, int W>
double tb3d_cost(const KGrid &g)
{
    const long long tiles = (long long)((g.nx + W - 1) / W) *
                            ((g.ny + Tb3Shape<K, W>::BYO - 1) / Tb3Shape<K, W>::BYO);
    const int zc = choose_zchunk3(tiles, g.nz, K);
    const long long nblk = tiles * ((g.nz + zc - 1) / zc);
    const long long rounds = (nblk + cu_count() - 1) / cu_count();
    return (double)rounds * (zc + 2.0 * K) * Tb3Shape<K, W>::STEP_COST;
}

}  // namespace

bool tb3d_plane_ok(const KGrid &g) { return (long long)g.nx * g.ny < (1LL << 27); }

int launch_tb3d(const KGrid &g, const PassArgs &p, hipStream_t st)
{
    if (g.ndim != 3 || (p.k != 2 && p.k != 3) || !tb3d_plane_ok(g)) return (int)hipErrorInvalidValue;
    Tb3Args a{};
    a.in_re = p.in_re;
    a.in_c = reinterpret_cast<const double2 *>(p.in_c);
    a.out_re = p.out_re;
    a.out_c = reinterpret_cast<double2 *>(p.out_c);
    a.D = p.D;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.inv_h2 = g.inv_h2;
    a.d_const = g.d_const;
    a.zchunk = p.zchunk;
    a.emb_in = p.emb_in;
    a.emb_out = p.emb_out;
    a.lvl_out = reinterpret_cast<double2 *>(p.lvl_out);
    a.lvl_stride = p.lvl_stride;
    for (int i = 0; i < kMaxTBlock; ++i) {
        a.tr[i] = p.tr[i];
        a.ti[i] = p.ti[i];
    }
    for (int k = 0; k < 6; ++k) a.fc[k] = g.fc[k];
    const bool ir = p.in_re != nullptr, orl = p.out_re != nullptr;
    const bool rev = p.rev != 0;
    const int cols = (p.cols == 32) ? 32 : 64;
    if (g.op == LAP) return launch3_bc<LAP>(g, p.k, cols, a, ir, orl, rev, st);
    if (g.op == ADV) return launch3_bc<ADV>(g, p.k, cols, a, ir, orl, rev, st);
    if (g.op == VAR) return launch3_bc<VAR>(g, p.k, cols, a, ir, orl, rev, st);
    return launch3_bc<POR>(g, p.k, cols, a, ir, orl, rev, st);
}

int tb3d_pick_cols(const KGrid &g, int k)
{
    if (k == 2) return tb3d_cost<2, 32>(g) < tb3d_cost<2, 64>(g) ? 32 : 64;
    return tb3d_cost<3, 32>(g) < tb3d_cost<3, 64>(g) ? 32 : 64;
}

namespace {
template <int K, int W>
long long tb3d_work_kw(int nx, int ny, int nz, int zc)
{
    using S = Tb3Shape<K, W>;
    const long long tiles = (long long)((nx + W - 1) / W) * ((ny + S::BYO - 1) / S::BYO);
    const int chunks = (nz + zc - 1) / zc;
    return tiles * ((long long)nz + 2LL * K * chunks) * S::STEP_COST;
}
}  // namespace

long long tb3d_work(int k, int cols, int nx, int ny, int nz, int zc)
{
    // steps x step cost of all tiles of a grid with chunk zc (batched items)
    if (k == 2) return cols == 32 ? tb3d_work_kw<2, 32>(nx, ny, nz, zc) : tb3d_work_kw<2, 64>(nx, ny, nz, zc);
    return cols == 32 ? tb3d_work_kw<3, 32>(nx, ny, nz, zc) : tb3d_work_kw<3, 64>(nx, ny, nz, zc);
}

}  // namespace frkc2
