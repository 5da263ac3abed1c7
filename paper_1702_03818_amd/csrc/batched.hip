// Batched FRKC2 supersteps: many independent problems of uneven size and
// stage count advanced by one HIP graph launch.
//
// Stage l of problem i is the Euler step W <- W + tau_l f(W) of its own
// superstep (O'Sullivan, arXiv:1702.03818, Sec. 3). Stages of one problem are
// sequential; different problems are independent. The graph holds one kernel
// per stage level l = 0 .. max(s)-1; the kernel of level l covers stage l of
// every problem with s > l (problems are sorted by decreasing s, so these are
// a prefix of the problem list), split into work items of up to kChunk
// consecutive grid points. Consecutive kernels in the graph are ordered, and
// that ordering is the only synchronisation: a kernel boundary makes every
// XCD's writes visible to every other XCD, which an in-kernel wait between
// workgroups could only get by writing back and invalidating the L2 caches
// around every dependency.
//
// Within a level kernel each workgroup takes items in a grid-stride loop; the
// items are split into eight contiguous ranges, one per XCD (workgroup b runs
// on XCD b % 8), so the halos of neighbouring chunks are shared through one
// L2.
//
// The per-point arithmetic is the one of the plain stage kernels (faces
// x-, x+, y-, y+, z-, z+, no fused multiply-adds), so each problem's result
// equals, bit for bit, the result of frkc2_step on it.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace {

using namespace dev;

constexpr int kThreads = 256;
constexpr int kChunk = 16384;          // points per work item

struct LevelArgs {
    const BatchProblem *probs;         // sorted by decreasing s
    const long long *chunk_prefix;     // prefix sums of chunks over the sorted problems
    long long items;                   // chunks of the active problems at this level
    int active;                        // problems with s > level
    int level;
};

template <int NDIM, int OP, int BC>
__device__ void chunk_body(const BatchProblem &P, int l, long long p0, long long p1)
{
    const Dims dm{P.nx, P.ny, P.nz};
    const bool first = (l == 0), last = (l == P.s - 1);
    const double *in_re = P.w;
    const double2 *in_c = reinterpret_cast<const double2 *>((l & 1) ? P.bufA : P.bufB);
    double2 *out_c = reinterpret_cast<double2 *>((l & 1) ? P.bufB : P.bufA);
    const double tr = P.tau[2 * l], ti = P.tau[2 * l + 1];
    const bool dir = (BC == DIR);
    for (long long p = p0 + threadIdx.x; p < p1; p += kThreads) {
        const int x = (int)(p % P.nx);
        const long long rest = p / P.nx;
        const int y = (int)(rest % P.ny);
        const int z = (int)(rest / P.ny);
        auto ld = [&](int gx, int gy, int gz) {
            return first ? load_c<BC, true>(dm, in_re, nullptr, gx, gy, gz)
                         : load_c<BC, false>(dm, nullptr, in_c, gx, gy, gz);
        };
        auto ldd = [&](int gx, int gy, int gz) {
            return (OP == VAR) ? load_r<BC>(dm, P.D, gx, gy, gz) : 0.0;
        };
        const double2 c = ld(x, y, z);
        const double dc = ldd(x, y, z);
        double acc_r = 0.0, acc_i = 0.0;
        face<OP>(acc_r, acc_i, c, ld(x - 1, y, z), dc, ldd(x - 1, y, z), dir && x == 0, 0.0, 0.0,
                 P.d_const);
        face<OP>(acc_r, acc_i, c, ld(x + 1, y, z), dc, ldd(x + 1, y, z), dir && x == P.nx - 1,
                 0.0, 0.0, P.d_const);
        if (NDIM == 3) {
            face<OP>(acc_r, acc_i, c, ld(x, y - 1, z), dc, ldd(x, y - 1, z), dir && y == 0, 0.0,
                     0.0, P.d_const);
            face<OP>(acc_r, acc_i, c, ld(x, y + 1, z), dc, ldd(x, y + 1, z),
                     dir && y == P.ny - 1, 0.0, 0.0, P.d_const);
        }
        face<OP>(acc_r, acc_i, c, ld(x, y, z - 1), dc, ldd(x, y, z - 1), dir && z == 0, 0.0, 0.0,
                 P.d_const);
        face<OP>(acc_r, acc_i, c, ld(x, y, z + 1), dc, ldd(x, y, z + 1), dir && z == P.nz - 1,
                 0.0, 0.0, P.d_const);
        const double2 v = euler(c, acc_r, acc_i, P.inv_h2, tr, ti);
        if (last) P.w[p] = v.x;
        else out_c[p] = v;
    }
}

__device__ void dispatch_chunk(const BatchProblem &P, int l, long long p0, long long p1)
{
    const bool three = (P.ndim == 3), per = (P.bc == PER), var = (P.op == VAR);
    if (three) {
        if (var) {
            if (per) chunk_body<3, VAR, PER>(P, l, p0, p1);
            else chunk_body<3, VAR, DIR>(P, l, p0, p1);
        } else {
            if (per) chunk_body<3, LAP, PER>(P, l, p0, p1);
            else chunk_body<3, LAP, DIR>(P, l, p0, p1);
        }
    } else {
        if (var) {
            if (per) chunk_body<2, VAR, PER>(P, l, p0, p1);
            else chunk_body<2, VAR, DIR>(P, l, p0, p1);
        } else {
            if (per) chunk_body<2, LAP, PER>(P, l, p0, p1);
            else chunk_body<2, LAP, DIR>(P, l, p0, p1);
        }
    }
}

__global__ __launch_bounds__(kThreads) void batched_level(LevelArgs t)
{
    // items are split into 8 contiguous ranges; workgroup b serves range b % 8
    const int xcd = blockIdx.x & 7;
    const int per_xcd = (int)(gridDim.x >> 3);
    const int lane_b = (int)(blockIdx.x >> 3);
    long long lo, hi, step, first;
    if (per_xcd > 0 && (int)blockIdx.x < per_xcd * 8) {
        const long long span = (t.items + 7) / 8;
        lo = xcd * span;
        hi = lo + span < t.items ? lo + span : t.items;
        first = lo + lane_b;
        step = per_xcd;
    } else {   // blocks beyond a multiple of 8 (small grids): plain grid stride
        lo = 0;
        hi = (per_xcd > 0) ? 0 : t.items;
        first = blockIdx.x;
        step = gridDim.x;
    }
    for (long long g = first; g < hi; g += step) {
        int a = 0, b = t.active - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (t.chunk_prefix[mid] <= g) a = mid;
            else b = mid - 1;
        }
        const BatchProblem &P = t.probs[a];
        const long long c = g - t.chunk_prefix[a];
        const long long n = (long long)P.nx * P.ny * P.nz;
        const long long p0 = c * kChunk;
        const long long p1 = (p0 + kChunk < n) ? p0 + kChunk : n;
        dispatch_chunk(P, t.level, p0, p1);
    }
}

}  // namespace

int batched_chunk_points() { return kChunk; }

int launch_batched_level(const BatchProblem *probs, const long long *chunk_prefix, long long items,
                         int active, int level, int grid, hipStream_t st)
{
    LevelArgs t{probs, chunk_prefix, items, active, level};
    hipLaunchKernelGGL(batched_level, dim3(grid), dim3(kThreads), 0, st, t);
    return (int)hipGetLastError();
}

int batched_grid_size()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_level, kThreads, 0) !=
        hipSuccess)
        return 0;
    return cus * (per > 0 ? per : 1);
}

}  // namespace frkc2
