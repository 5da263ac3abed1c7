// Batched FRKC2 supersteps: many independent problems of uneven size and
// stage count advanced by one HIP graph launch.
//
// Stage l of problem i is the Euler step W <- W + tau_l f(W) of its own
// superstep (O'Sullivan, arXiv:1702.03818, Sec. 3). Stages of one problem are
// sequential; different problems are independent. The graph has independent
// branches: the 3D problems in two interleaved groups (so that one group's
// level tail shares the GPU with the other's work) and the 2D problems. A 3D
// branch holds, per pass level L, one kernel
// for the fused passes (stages 3L .. 3L+2 of every problem that has them, as
// full-width temporally blocked tiles of tb3d_tile.h, 64 or 32 output columns
// wide, one width for the whole batch) and one for the
// single-stage passes that finish each superstep (s mod 3 stages, 64 x 16
// plane-march tiles). The 2D branch is built the same way with passes of 4
// stages, as rows of 64 extended columns (tb_tile.h, one wavefront each, so
// the many narrow 2D problems do not idle most of a wide row) marching up to
// 128 rows, and 64-column plane-march tiles for the single stages (s mod 4;
// a problem with s = 4 runs single stages, since one fused pass would read
// and write its state in place). Kernels of one
// branch are ordered, and that ordering is the only synchronisation: a kernel
// boundary makes every XCD's writes visible to every other XCD, which an
// in-kernel wait between workgroups could only get by writing back and
// invalidating the L2 caches around every dependency.
//
// A work item is one tile of a problem. A fused item is one workgroup, the
// block index remapped so that each XCD (workgroup b runs on XCD b % 8) takes
// a contiguous range of items; the single-stage items of a level are split
// into eight contiguous ranges, one per XCD, that the workgroups walk. Either
// way neighbouring tiles share an L2. An item's problem descriptor is moved to
// scalar registers, since the whole workgroup works on one problem.
//
// The per-point arithmetic is the one of the plain stage kernels (faces
// x-, x+, y-, y+, z-, z+, face() and euler()), so each problem's result
// equals, bit for bit, the result of frkc2_step on it.
#include <hip/hip_runtime.h>

#include "plane_tile.h"
#include "tb3d_tile.h"
#include "tb_tile.h"

namespace frkc2 {
namespace {

using namespace dev;


// A value the whole workgroup shares, moved to scalar registers (the compiler
// cannot prove that loads of the problem table are uniform).
template <typename T>
__device__ __forceinline__ T uni(T v)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    union {
        T v;
        int w[sizeof(T) / 4];
    } u;
    u.v = v;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) u.w[i] = __builtin_amdgcn_readfirstlane(u.w[i]);
    return u.v;
}

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

constexpr int kBX2 = 64;             // single-stage 2D items: 64-column plane-march tiles
constexpr int kPBX = 64, kPBY = 16;   // single-stage items of the 3D pass kernel (1024 threads)
constexpr int kBXE2 = 64;             // fused 2D items: rows of 64 extended columns (one wavefront)

// Range of items of this workgroup: eight contiguous ranges, one per XCD.
__device__ __forceinline__ void xcd_range(long long items, long long &first, long long &hi,
                                          long long &step)
{
    const int xcd = blockIdx.x & 7;
    const int per_xcd = (int)(gridDim.x >> 3);
    if (per_xcd > 0 && (int)blockIdx.x < per_xcd * 8) {
        const long long span = (items + 7) / 8;
        const long long lo = xcd * span;
        hi = lo + span < items ? lo + span : items;
        first = lo + (blockIdx.x >> 3);
        step = per_xcd;
    } else {
        hi = (per_xcd > 0) ? 0 : items;
        first = blockIdx.x;
        step = gridDim.x;
    }
}

struct Pass3Args {
    const BatchProblem *probs;         // all 3D problems
    const long long *item_prefix;      // items of this pass level per problem (0: not active)
    long long items;
    int nprob, level;
};

template <int OP, int BC, bool IR, bool OR, int W, int KB>
__device__ void run_fused(const BatchProblem &P, Tb3Args &a, long long c, double2 *sL, double *sD)
{
    const int bx = (int)(c % P.ntx3);
    const long long r = c / P.ntx3;
    tb3d_tile<OP, BC, KB, IR, OR, false, false, W, true, true>(a, bx, (int)(r % P.nty3),
                                                                 (int)(r / P.nty3), sL, sD);
}

template <int OP, int BC, int W, int KB>
__device__ void fused_io_w(const BatchProblem &P, Tb3Args &a, long long c, bool ir, bool orl,
                           double2 *sL, double *sD)
{
    if (ir) run_fused<OP, BC, true, false, W, KB>(P, a, c, sL, sD);
    else if (orl) run_fused<OP, BC, false, true, W, KB>(P, a, c, sL, sD);
    else run_fused<OP, BC, false, false, W, KB>(P, a, c, sL, sD);
}


template <int OP, int BC, int KB>
__device__ void row_io(const TbArgs &a, int bx, int bz, bool ir, bool orl, double2 *sL, double *sD)
{
    if (ir) tb_tile<OP, BC, 2, kBXE2, 1, 1, KB, true, false>(a, bx, 0, bz, sL, sD);
    else if (orl) tb_tile<OP, BC, 2, kBXE2, 1, 1, KB, false, true>(a, bx, 0, bz, sL, sD);
    else tb_tile<OP, BC, 2, kBXE2, 1, 1, KB, false, false>(a, bx, 0, bz, sL, sD);
}

// One pass level of the 3D problems. FUSED: each active problem's pass of
// KB stages (stages KB*level ..), as tb3d_tile items with the diffusivity
// faces in registers, one item per workgroup (a loop over items around the
// tile keeps more registers live than the face ring leaves, and spills);
// otherwise its single-stage pass (the stages left after the fused ones), as
// 64 x 16 plane-march items, each workgroup a range of items. A problem's
// first pass reads w, its last writes w, the passes between ping-pong the
// workspace buffers.
template <bool FUSED, int W, int KB>
__device__ __forceinline__ void pass3_item(const Pass3Args &t, long long g, double2 *sL, double *sD)
{
    const int L = t.level;
    int a = 0, b = t.nprob - 1;
    while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (t.item_prefix[mid] <= g) a = mid;
        else b = mid - 1;
    }
    a = uni(a);
    BatchProblem P = t.probs[a];
    P.w = uni(P.w);
    P.D = uni(P.D);
    P.bufA = uni(P.bufA);
    P.bufB = uni(P.bufB);
    P.tau = uni(P.tau);
    P.nx = uni(P.nx);
    P.ny = uni(P.ny);
    P.nz = uni(P.nz);
    P.bc = uni(P.bc);
    P.op = uni(P.op);
    P.zchunk = uni(P.zchunk);
    P.ntx = uni(P.ntx);
    P.nty = uni(P.nty);
    P.nfull = uni(P.nfull);
    P.npass = uni(P.npass);
    P.zc3 = uni(P.zc3);
    P.ntx3 = uni(P.ntx3);
    P.nty3 = uni(P.nty3);
    P.inv_h2 = uni(P.inv_h2);
    P.d_const = uni(P.d_const);
    const long long c = uni(g - t.item_prefix[a]);
    const bool ir = (L == 0), orl = (L == P.npass - 1);
    const double *in_c = (L & 1) ? P.bufA : P.bufB;   // pass L-1 wrote buffer (L-1) & 1
    double *out_c = (L & 1) ? P.bufB : P.bufA;
    const bool per = (P.bc == PER), var = (P.op == VAR);
    if (FUSED) {
        Tb3Args ta{};
        ta.in_re = P.w;
        ta.in_c = reinterpret_cast<const double2 *>(in_c);
        ta.out_re = P.w;
        ta.out_c = reinterpret_cast<double2 *>(out_c);
        ta.D = P.D;
        ta.nx = P.nx;
        ta.ny = P.ny;
        ta.nz = P.nz;
        ta.zchunk = P.zc3;
        ta.ntx = P.ntx3;
        ta.nty = P.nty3;
        ta.inv_h2 = P.inv_h2;
        ta.d_const = P.d_const;
        for (int k = 0; k < 6; ++k) ta.fc[k] = P.d_const;
        const int l0 = KB * L;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            ta.tr[i] = uni(P.tau[2 * (l0 + i)]);
            ta.ti[i] = uni(P.tau[2 * (l0 + i) + 1]);
        }
        if (var) {
            if (per) fused_io_w<VAR, PER, W, KB>(P, ta, c, ir, orl, sL, sD);
            else fused_io_w<VAR, DIR, W, KB>(P, ta, c, ir, orl, sL, sD);
        } else {
            if (per) fused_io_w<LAP, PER, W, KB>(P, ta, c, ir, orl, sL, sD);
            else fused_io_w<LAP, DIR, W, KB>(P, ta, c, ir, orl, sL, sD);
        }
    } else {
        const int l = KB * P.nfull + (L - P.nfull);
        PlaneArgs pa{};
        pa.in_re = P.w;
        pa.in_c = reinterpret_cast<const double2 *>(in_c);
        pa.out_re = P.w;
        pa.out_c = reinterpret_cast<double2 *>(out_c);
        pa.D = P.D;
        pa.nx = P.nx;
        pa.ny = P.ny;
        pa.nz = P.nz;
        pa.zchunk = P.zchunk;
        pa.ntx = P.ntx;
        pa.nty = P.nty;
        pa.inv_h2 = P.inv_h2;
        pa.d_const = P.d_const;
        for (int k = 0; k < 6; ++k) pa.fc[k] = P.d_const;
        pa.tr = uni(P.tau[2 * l]);
        pa.ti = uni(P.tau[2 * l + 1]);
        if (var) {
            if (per) run_io<3, kPBX, kPBY, VAR, PER>(P, pa, c, ir, orl, sL, sD);
            else run_io<3, kPBX, kPBY, VAR, DIR>(P, pa, c, ir, orl, sL, sD);
        } else {
            if (per) run_io<3, kPBX, kPBY, LAP, PER>(P, pa, c, ir, orl, sL, sD);
            else run_io<3, kPBX, kPBY, LAP, DIR>(P, pa, c, ir, orl, sL, sD);
        }
    }
}

template <bool FUSED, int W, int KB>
__global__ __launch_bounds__(1024) void batched_pass3(Pass3Args t)
{
    using S1 = TileShape<VAR, DIR, 3, kPBX, kPBY>;
    constexpr int NL = FUSED ? Tb3Lds<VAR, KB, W>::L : S1::LDS_W;
    constexpr int ND = FUSED ? Tb3Lds<VAR, KB, W>::D : S1::LDS_D;
    __shared__ double2 sL[NL];
    __shared__ double sD[ND];
    if constexpr (FUSED) {
        // consecutive items (neighbouring tiles of a problem) on one XCD
        const int g = xcd_remap(blockIdx.x, gridDim.x);
        if (g < t.items) pass3_item<FUSED, W, KB>(t, g, sL, sD);
    } else {
        long long first, hi, step;
        xcd_range(t.items, first, hi, step);
        for (long long g = first; g < hi; g += step) {
            pass3_item<FUSED, W, KB>(t, g, sL, sD);
            __syncthreads();   // the next item reuses the LDS
        }
    }
}

// One pass level of the 2D problems. FUSED: each active problem's pass of
// KB stages (stages KB*level ..), as row items of tb_tile.h (64
// extended columns marching up to 128 rows); otherwise its single-stage pass,
// as 64-column plane-march items. Buffers as in the 3D pass kernel.
template <bool FUSED, int KB>
__global__ __launch_bounds__(64) void batched_pass2(Pass3Args t)
{
    using S1 = TileShape<VAR, DIR, 2, kBX2, 1>;
    using S2 = TbLds<VAR, 2, kBXE2, 1, 1, KB>;
    __shared__ double2 sL[FUSED ? S2::L : S1::LDS_W];
    __shared__ double sD[FUSED ? S2::D : S1::LDS_D];
    long long first, hi, step;
    xcd_range(t.items, first, hi, step);
    const int L = t.level;
    for (long long g = first; g < hi; g += step) {
        int a = 0, b = t.nprob - 1;
        while (a < b) {
            const int mid = (a + b + 1) >> 1;
            if (t.item_prefix[mid] <= g) a = mid;
            else b = mid - 1;
        }
        a = uni(a);
        BatchProblem P = t.probs[a];
        P.w = uni(P.w);
        P.D = uni(P.D);
        P.bufA = uni(P.bufA);
        P.bufB = uni(P.bufB);
        P.tau = uni(P.tau);
        P.nx = uni(P.nx);
        P.ny = uni(P.ny);
        P.nz = uni(P.nz);
        P.bc = uni(P.bc);
        P.op = uni(P.op);
        P.zchunk = uni(P.zchunk);
        P.ntx = uni(P.ntx);
        P.nty = uni(P.nty);
        P.nfull = uni(P.nfull);
        P.npass = uni(P.npass);
        P.zc3 = uni(P.zc3);
        P.ntx3 = uni(P.ntx3);
        P.inv_h2 = uni(P.inv_h2);
        P.d_const = uni(P.d_const);
        const long long c = uni(g - t.item_prefix[a]);
        const bool ir = (L == 0), orl = (L == P.npass - 1);
        const double *in_c = (L & 1) ? P.bufA : P.bufB;   // pass L-1 wrote buffer (L-1) & 1
        double *out_c = (L & 1) ? P.bufB : P.bufA;
        const bool per = (P.bc == PER), var = (P.op == VAR);
        if (FUSED) {
            TbArgs ta{};
            ta.in_re = P.w;
            ta.in_c = reinterpret_cast<const double2 *>(in_c);
            ta.out_re = P.w;
            ta.out_c = reinterpret_cast<double2 *>(out_c);
            ta.D = P.D;
            ta.nx = P.nx;
            ta.ny = P.ny;
            ta.nz = P.nz;
            ta.zchunk = P.zc3;
            ta.ntx = P.ntx3;
            ta.nty = 1;
            ta.inv_h2 = P.inv_h2;
            ta.d_const = P.d_const;
            for (int k = 0; k < 6; ++k) ta.fc[k] = P.d_const;
            const int l0 = KB * L;
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                ta.tr[i] = uni(P.tau[2 * (l0 + i)]);
                ta.ti[i] = uni(P.tau[2 * (l0 + i) + 1]);
            }
            const int bx = (int)(c % P.ntx3), bz = (int)(c / P.ntx3);
            if (var) {
                if (per) row_io<VAR, PER, KB>(ta, bx, bz, ir, orl, sL, sD);
                else row_io<VAR, DIR, KB>(ta, bx, bz, ir, orl, sL, sD);
            } else {
                if (per) row_io<LAP, PER, KB>(ta, bx, bz, ir, orl, sL, sD);
                else row_io<LAP, DIR, KB>(ta, bx, bz, ir, orl, sL, sD);
            }
        } else {
            const int l = KB * P.nfull + (L - P.nfull);
            PlaneArgs pa{};
            pa.in_re = P.w;
            pa.in_c = reinterpret_cast<const double2 *>(in_c);
            pa.out_re = P.w;
            pa.out_c = reinterpret_cast<double2 *>(out_c);
            pa.D = P.D;
            pa.nx = P.nx;
            pa.ny = P.ny;
            pa.nz = P.nz;
            pa.zchunk = P.zchunk;
            pa.ntx = P.ntx;
            pa.nty = P.nty;
            pa.inv_h2 = P.inv_h2;
            pa.d_const = P.d_const;
            for (int k = 0; k < 6; ++k) pa.fc[k] = P.d_const;
            pa.tr = uni(P.tau[2 * l]);
            pa.ti = uni(P.tau[2 * l + 1]);
            if (var) {
                if (per) run_io<2, kBX2, 1, VAR, PER>(P, pa, c, ir, orl, sL, sD);
                else run_io<2, kBX2, 1, VAR, DIR>(P, pa, c, ir, orl, sL, sD);
            } else {
                if (per) run_io<2, kBX2, 1, LAP, PER>(P, pa, c, ir, orl, sL, sD);
                else run_io<2, kBX2, 1, LAP, DIR>(P, pa, c, ir, orl, sL, sD);
            }
        }
        __syncthreads();   // the next item reuses the LDS
    }
}

}  // namespace

void batched_tile(int ndim, int *bx, int *by) { *bx = ndim == 3 ? kPBX : kBX2; *by = ndim == 3 ? kPBY : 1; }

void batched_tile3(int cols, int k, int *bx, int *by)
{
    *bx = cols;
    if (k == 2) *by = (cols == 32) ? Tb3Shape<2, 32>::BYO : Tb3Shape<2, 64>::BYO;
    else *by = (cols == 32) ? Tb3Shape<3, 32>::BYO : Tb3Shape<3, 64>::BYO;
}

bool batched_cfg_supported(int k3, int cols3, int k2)
{
    return (k3 == 2 || k3 == 3) && (cols3 == 32 || cols3 == 64) &&
           (k2 == 2 || k2 == 3 || k2 == 4 || k2 == 6);
}

namespace {

template <bool FUSED, int W, int KB>
void launch3(const Pass3Args &t, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((batched_pass3<FUSED, W, KB>), dim3(grid), dim3(1024), 0, st, t);
}

template <bool FUSED, int KB>
void launch2(const Pass3Args &t, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((batched_pass2<FUSED, KB>), dim3(grid), dim3(64), 0, st, t);
}

}  // namespace

int launch_batched_pass3(bool fused, int cols, int k, const BatchProblem *probs,
                         const long long *item_prefix, long long items, int nprob, int level,
                         int grid, hipStream_t st)
{
    Pass3Args t{probs, item_prefix, items, nprob, level};
    // the single-stage items do not depend on the width
    if (k == 2) {
        if (!fused) launch3<false, 64, 2>(t, grid, st);
        else if (cols == 32) launch3<true, 32, 2>(t, grid, st);
        else launch3<true, 64, 2>(t, grid, st);
    } else if (k == 3) {
        if (!fused) launch3<false, 64, 3>(t, grid, st);
        else if (cols == 32) launch3<true, 32, 3>(t, grid, st);
        else launch3<true, 64, 3>(t, grid, st);
    } else {
        return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int batched_row2(int k) { return kBXE2 - 2 * k; }

int launch_batched_pass2(bool fused, int k, const BatchProblem *probs,
                         const long long *item_prefix, long long items, int nprob, int level,
                         int grid, hipStream_t st)
{
    Pass3Args t{probs, item_prefix, items, nprob, level};
    switch (k) {
    case 2: fused ? launch2<true, 2>(t, grid, st) : launch2<false, 2>(t, grid, st); break;
    case 3: fused ? launch2<true, 3>(t, grid, st) : launch2<false, 3>(t, grid, st); break;
    case 4: fused ? launch2<true, 4>(t, grid, st) : launch2<false, 4>(t, grid, st); break;
    case 6: fused ? launch2<true, 6>(t, grid, st) : launch2<false, 6>(t, grid, st); break;
    default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

int batched_grid_size(int ndim)
{
    // every pass kernel of a dimension has the same workgroup size and fits the
    // same number of workgroups per CU (one for 3D: its LDS; the 2D rows are
    // bound by waves per CU), so one query per dimension serves all
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    hipError_t e = (ndim == 3)
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_pass3<true, 64, 3>, 1024, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batched_pass2<true, 4>, 64, 0);
    if (e != hipSuccess) return 0;
    return cus * (per > 0 ? per : 1);
}

}  // namespace frkc2
