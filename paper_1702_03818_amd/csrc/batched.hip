// Batched FRKC2 supersteps: many independent problems of uneven size and
// stage count advanced by one HIP graph launch.
//
// Stage l of problem i is the Euler step W <- W + tau_l f(W) of its own
// superstep (O'Sullivan, arXiv:1702.03818, Sec. 3). Stages of one problem are
// sequential; different problems are independent. The graph holds, for each
// stage level l = 0 .. max(s)-1, one kernel over the 3D problems and one over
// the 2D problems with s > l (each list sorted by decreasing s, so the active
// problems are a prefix). Consecutive kernels in the graph are ordered, and
// that ordering is the only synchronisation: a kernel boundary makes every
// XCD's writes visible to every other XCD, which an in-kernel wait between
// workgroups could only get by writing back and invalidating the L2 caches
// around every dependency.
//
// A work item is one tile of the one-stage plane-march kernel (plane_tile.h):
// 64 x 4 columns over a chunk of z planes for 3D problems (256 threads), a
// row of 64 columns over a chunk of rows for 2D problems (64 threads, so the
// many narrow 2D problems do not idle three quarters of a 256-wide row). The
// items of a level are split into eight contiguous ranges, one per XCD
// (workgroup b runs on XCD b % 8), so neighbouring tiles share an L2.
//
// The per-point arithmetic is the one of the plain stage kernels (faces
// x-, x+, y-, y+, z-, z+, face() and euler()), so each problem's result
// equals, bit for bit, the result of frkc2_step on it.
#include <hip/hip_runtime.h>

#include "plane_tile.h"

namespace frkc2 {
namespace {

using namespace dev;

struct LevelArgs {
    const BatchProblem *probs;         // one dimension's list, sorted by decreasing s
    const long long *item_prefix;      // prefix sums of tiles per stage over that list
    long long items;                   // tiles of the active problems at this level
    int active;                        // problems with s > level
    int level;
};

template <int NDIM, int BX, int BY, int OP, int BC, bool IR, bool OR>
__device__ void run_tile(const BatchProblem &P, const PlaneArgs &a, long long c, double2 *sW,
                         double *sD)
{
    const int bx = (int)(c % P.ntx);
    const long long r = c / P.ntx;
    const int by = (int)(r % P.nty);
    const int bz = (int)(r / P.nty);
    plane_tile<OP, BC, NDIM, BX, BY, IR, OR>(a, bx, by, bz, sW, sD);
}

template <int NDIM, int BX, int BY, int OP, int BC>
__device__ void run_io(const BatchProblem &P, const PlaneArgs &a, long long c, bool ir, bool orl,
                       double2 *sW, double *sD)
{
    if (ir) run_tile<NDIM, BX, BY, OP, BC, true, false>(P, a, c, sW, sD);
    else if (orl) run_tile<NDIM, BX, BY, OP, BC, false, true>(P, a, c, sW, sD);
    else run_tile<NDIM, BX, BY, OP, BC, false, false>(P, a, c, sW, sD);
}

template <int NDIM, int BX, int BY>
__global__ __launch_bounds__(BX *BY) void batched_level(LevelArgs t)
{
    using S = TileShape<VAR, DIR, NDIM, BX, BY>;   // the largest LDS footprint
    __shared__ double2 sW[S::LDS_W];
    __shared__ double sD[S::LDS_D];
    const int xcd = blockIdx.x & 7;
    const int per_xcd = (int)(gridDim.x >> 3);
    long long hi, step, first;
    if (per_xcd > 0 && (int)blockIdx.x < per_xcd * 8) {
        const long long span = (t.items + 7) / 8;
        const long long lo = xcd * span;
        hi = lo + span < t.items ? lo + span : t.items;
        first = lo + (blockIdx.x >> 3);
        step = per_xcd;
    } else {
        hi = (per_xcd > 0) ? 0 : t.items;
        first = blockIdx.x;
        step = gridDim.x;
    }
    const int l = t.level;
    for (long long g = first; g < hi; g += step) {
        int a = 0, b = t.active - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (t.item_prefix[mid] <= g) a = mid;
            else b = mid - 1;
        }
        const BatchProblem &P = t.probs[a];
        const long long c = g - t.item_prefix[a];
        PlaneArgs pa{};
        const bool ir = (l == 0), orl = (l == P.s - 1);
        pa.in_re = P.w;
        pa.in_c = reinterpret_cast<const double2 *>((l & 1) ? P.bufA : P.bufB);
        pa.out_re = P.w;
        pa.out_c = reinterpret_cast<double2 *>((l & 1) ? P.bufB : P.bufA);
        pa.D = P.D;
        pa.nx = P.nx;
        pa.ny = P.ny;
        pa.nz = P.nz;
        pa.zchunk = P.zchunk;
        pa.ntx = P.ntx;
        pa.nty = P.nty;
        pa.inv_h2 = P.inv_h2;
        pa.d_const = P.d_const;
        pa.tr = P.tau[2 * l];
        pa.ti = P.tau[2 * l + 1];
        const bool per = (P.bc == PER), var = (P.op == VAR);
        if (var) {
            if (per) run_io<NDIM, BX, BY, VAR, PER>(P, pa, c, ir, orl, sW, sD);
            else run_io<NDIM, BX, BY, VAR, DIR>(P, pa, c, ir, orl, sW, sD);
        } else {
            if (per) run_io<NDIM, BX, BY, LAP, PER>(P, pa, c, ir, orl, sW, sD);
            else run_io<NDIM, BX, BY, LAP, DIR>(P, pa, c, ir, orl, sW, sD);
        }
        __syncthreads();   // the next item reuses the LDS tile
    }
}

constexpr int kBX3 = 64, kBY3 = 4, kBX2 = 64;

}  // namespace

void batched_tile(int ndim, int *bx, int *by) { *bx = ndim == 3 ? kBX3 : kBX2; *by = ndim == 3 ? kBY3 : 1; }

int launch_batched_level(int ndim, const BatchProblem *probs, const long long *item_prefix,
                         long long items, int active, int level, int grid, hipStream_t st)
{
    LevelArgs t{probs, item_prefix, items, active, level};
    if (ndim == 3)
        hipLaunchKernelGGL((batched_level<3, kBX3, kBY3>), dim3(grid), dim3(kBX3 * kBY3), 0, st, t);
    else
        hipLaunchKernelGGL((batched_level<2, kBX2, 1>), dim3(grid), dim3(kBX2), 0, st, t);
    return (int)hipGetLastError();
}

int batched_grid_size(int ndim)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e = (ndim == 3)
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_level<3, kBX3, kBY3>, kBX3 * kBY3, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_level<2, kBX2, 1>, kBX2, 0);
    if (e != hipSuccess) return 0;
    return cus * (per > 0 ? per : 1);
}

}  // namespace frkc2
