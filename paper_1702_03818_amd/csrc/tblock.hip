// Temporally blocked FRKC2 stages: K consecutive Euler stages
// W <- W + tau_l f(W) (O'Sullivan, arXiv:1702.03818, Sec. 3, Euler-step
// equation) in one HBM pass.
//
// The stages of a superstep are strictly sequential, but stage l+1 at a
// point only needs stage l within one cell of it, so K stages of a tile can
// be computed from the tile's input extended by a K-cell halo. Each
// workgroup owns an extended tile of BXE x BYE columns (3D; 2D tiles are one
// row of BXE) and marches through a chunk of z planes with a software
// pipeline: at time step t it has level 0 (the pass input) of plane t and
// computes level m (the state after m stages of the pass) at plane t - m for
// m = 1..K. Level m at plane p needs level m-1 at planes p-1, p, p+1 of the
// same column, which the thread keeps in registers, and level m-1 at the x/y
// neighbours of plane p, which sit in LDS (one plane per level, written in
// the previous time step). The diffusivity planes t-K-1 .. t-1 live in an LDS
// ring. Two barriers per time step separate the LDS reads from the writes
// (one for 2D rows, whose planes are double-buffered where LDS allows).
//
// Level 0 is prefetched two time steps ahead into a five-slot register ring;
// the time loop is unrolled by five so the slot indices are compile-time
// constants and a load in flight is never copied (a copy would have to wait
// for it). Dirichlet ghosts are zeroed when a plane is first used, not where
// it is loaded, for the same reason.
//
// Only level K inside the inner (BXE-2K) x (BYE-2K) region is written back;
// the ring of halo columns is recomputed by the neighbouring tile (their
// input is read twice, mostly through L2). HBM traffic per pass is the input
// (16 B complex or 8 B real, plus 8 B of D) and the output (16 B or 8 B), so
// per stage it drops roughly by K.
//
// Every value is computed with the same per-point arithmetic, in the same
// order, as the one-stage kernel (faces x-, x+, y-, y+, z-, z+; face() and
// euler() of device_common.h), so the results are identical to the last bit.
#include <hip/hip_runtime.h>

#include "tb_tile.h"

namespace frkc2 {
namespace {

using namespace dev;

template <int OP, int BC, int NDIM, int BXE, int TY, int R, int K, bool IN_REAL, bool OUT_REAL,
          bool EMB = false>
__global__ __launch_bounds__(BXE *TY) void tb_stage(TbArgs a)
{
    using S = TbLds<OP, NDIM, BXE, TY, R, K>;
    __shared__ double2 sL[S::L];
    __shared__ double sD[S::D];
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % a.ntx;
    lb /= a.ntx;
    const int by = lb % a.nty;
    const int bz = lb / a.nty;
    tb_tile<OP, BC, NDIM, BXE, TY, R, K, IN_REAL, OUT_REAL, EMB>(a, bx, by, bz, sL, sD);
}

int choose_zchunk(long long tiles, int nz, int target_blocks)
{
    int zc = nz;
    while (zc > 16 && tiles * ((nz + zc - 1) / zc) < target_blocks) zc = (zc + 1) / 2;
    return zc;
}

template <int OP, int BC, int NDIM, int BXE, int TY, int R, int K>
int launch_k(const TbArgs &a0, bool ir, bool orl, bool emb, hipStream_t st)
{
    TbArgs a = a0;
    constexpr int BXO = BXE - 2 * K;
    constexpr int BYO = (NDIM == 3) ? TY * R - 2 * K : 1;
    a.ntx = (a.nx + BXO - 1) / BXO;
    a.nty = (NDIM == 3) ? (a.ny + BYO - 1) / BYO : 1;
    const long long tiles = (long long)a.ntx * a.nty;
    a.zchunk = (a0.zchunk > 0) ? min(a0.zchunk, a.nz)
                               : choose_zchunk(tiles, a.nz, NDIM == 3 ? 512 : 2048);
    const long long nblk = tiles * ((a.nz + a.zchunk - 1) / a.zchunk);
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(BXE * TY);
    if (emb) {   // 2D rows of 256, K <= 4 only (tblock_emb_supported)
        if constexpr (NDIM == 2 && BXE == 256 && K <= 4) {
            if (ir)
                hipLaunchKernelGGL((tb_stage<OP, BC, NDIM, BXE, TY, R, K, true, false, true>), grid,
                                   block, 0, st, a);
            else
                hipLaunchKernelGGL((tb_stage<OP, BC, NDIM, BXE, TY, R, K, false, false, true>), grid,
                                   block, 0, st, a);
            return (int)hipGetLastError();
        }
        return (int)hipErrorInvalidValue;
    }
    if (ir && orl)
        hipLaunchKernelGGL((tb_stage<OP, BC, NDIM, BXE, TY, R, K, true, true>), grid, block, 0, st, a);
    else if (ir)
        hipLaunchKernelGGL((tb_stage<OP, BC, NDIM, BXE, TY, R, K, true, false>), grid, block, 0, st, a);
    else if (orl)
        hipLaunchKernelGGL((tb_stage<OP, BC, NDIM, BXE, TY, R, K, false, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((tb_stage<OP, BC, NDIM, BXE, TY, R, K, false, false>), grid, block, 0, st, a);
    return (int)hipGetLastError();
}

// Tile shapes, chosen to fit LDS (160 KiB per workgroup) and registers:
//  3D shape 0: 64 x 16 extended columns, 1024 threads, one row each
//  3D shape 1: 64 x 32 extended columns, 1024 threads, two rows each (K = 2)
//  3D shape 2: 64 x 32 (K = 2) or 64 x 24 (K = 3) with 512 threads
//  2D shape 0: rows of 256 extended columns; shape 1: rows of 512.
template <int OP, int BC, int K>
int launch_shape(int ndim, int shape, const TbArgs &a, bool ir, bool orl, bool emb, hipStream_t st)
{
    if (ndim == 3) {
        if (emb) return (int)hipErrorInvalidValue;
        if constexpr (K == 2) {
            if (shape == 1) return launch_k<OP, BC, 3, 64, 16, 2, K>(a, ir, orl, false, st);
            if (shape == 2) return launch_k<OP, BC, 3, 64, 8, 4, K>(a, ir, orl, false, st);
        }
        if constexpr (K == 3) {
            if (shape == 2) return launch_k<OP, BC, 3, 64, 8, 3, K>(a, ir, orl, false, st);
        }
        if constexpr (K <= 3) return launch_k<OP, BC, 3, 64, 16, 1, K>(a, ir, orl, false, st);
        else return (int)hipErrorInvalidValue;
    }
    if (shape == 1) return launch_k<OP, BC, 2, 512, 1, 1, K>(a, ir, orl, emb, st);
    return launch_k<OP, BC, 2, 256, 1, 1, K>(a, ir, orl, emb, st);
}

template <int OP, int BC>
int launch_kk(int ndim, int k, int shape, const TbArgs &a, bool ir, bool orl, bool emb,
              hipStream_t st)
{
    switch (k) {
    case 2: return launch_shape<OP, BC, 2>(ndim, shape, a, ir, orl, emb, st);
    case 3: return launch_shape<OP, BC, 3>(ndim, shape, a, ir, orl, emb, st);
    case 4: return launch_shape<OP, BC, 4>(ndim, shape, a, ir, orl, emb, st);
    case 6: return launch_shape<OP, BC, 6>(ndim, shape, a, ir, orl, emb, st);
    case 8: return launch_shape<OP, BC, 8>(ndim, shape, a, ir, orl, emb, st);
    default: return (int)hipErrorInvalidValue;
    }
}

template <int OP>
int launch_bc(const KGrid &g, int k, int shape, const TbArgs &a, bool ir, bool orl, bool emb,
              hipStream_t st)
{
    if (g.bc == PER) return launch_kk<OP, PER>(g.ndim, k, shape, a, ir, orl, emb, st);
    return launch_kk<OP, DIR>(g.ndim, k, shape, a, ir, orl, emb, st);
}

}  // namespace

bool tblock_supported(const KGrid &g, int k)
{
    if (g.op == FRKC2_OP_BRUSS2) return k >= 2 && k <= 6;
    if (g.ndim == 3) return k == 2 || k == 3;
    if (g.ndim == 2) return k == 2 || k == 3 || k == 4 || k == 6 || k == 8;
    return false;
}

bool tblock_emb_supported(const KGrid &g, int k, int shape)
{
    if (g.op == FRKC2_OP_BRUSS2) return tblock_supported(g, k);
    if (g.ndim == 3) return (shape == 3 || shape == 4) && tblock_supported(g, k);
    return g.ndim == 2 && shape == 0 && k >= 2 && k <= 4;
}

int launch_tblock(const KGrid &g, const PassArgs &p, int shape, hipStream_t st)
{
    if (!tblock_supported(g, p.k)) return (int)hipErrorInvalidValue;
    if (g.op == FRKC2_OP_BRUSS2) return launch_bruss_tb(g, p, st);
    if (g.ndim == 3 && (shape == 3 || shape == 4) && !tb3d_plane_ok(g)) shape = 0;
    if (g.ndim == 3 && (shape == 3 || shape == 4)) {
        PassArgs q = p;
        q.cols = (shape == 4) ? 32 : 64;
        return launch_tb3d(g, q, st);
    }
    TbArgs a{};
    a.in_re = p.in_re;
    a.in_c = reinterpret_cast<const double2 *>(p.in_c);
    a.out_re = p.out_re;
    a.out_c = reinterpret_cast<double2 *>(p.out_c);
    a.emb_in = p.emb_in;
    a.emb_out = p.emb_out;
    a.D = p.D;
    a.nx = g.nx;
    a.ny = g.ny;
    a.nz = g.nz;
    a.inv_h2 = g.inv_h2;
    a.d_const = g.d_const;
    a.zchunk = p.zchunk;
    for (int i = 0; i < kMaxTBlock; ++i) {
        a.tr[i] = p.tr[i];
        a.ti[i] = p.ti[i];
    }
    for (int k = 0; k < 6; ++k) a.fc[k] = g.fc[k];
    const bool ir = p.in_re != nullptr, orl = p.out_re != nullptr, emb = p.emb_out != nullptr;
    if (emb && (orl || !tblock_emb_supported(g, p.k, shape) || (!ir && !p.emb_in)))
        return (int)hipErrorInvalidValue;
    if (g.op == LAP) return launch_bc<LAP>(g, p.k, shape, a, ir, orl, emb, st);
    if (g.op == ADV) return launch_bc<ADV>(g, p.k, shape, a, ir, orl, emb, st);
    if (g.op == VAR) return launch_bc<VAR>(g, p.k, shape, a, ir, orl, emb, st);
    return launch_bc<POR>(g, p.k, shape, a, ir, orl, emb, st);
}

}  // namespace frkc2
