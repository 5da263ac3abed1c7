// Stage kernel of the two-species Brusselator (O'Sullivan, arXiv:1702.03818,
// Sec. 3.1, the default problem of the paper's public code):
//   v_t = d lap v + 1 - 4v + w v^2,   w_t = d lap w + 3v - v^2 w,
// advanced by one FRKC2 Euler stage W <- W + tau f(W) (Sec. 3) on complex
// stage values; periodic 2D grid, state v then w (N values each).
//
// A workgroup of 64 x 8 threads loads its tile of both species with a
// one-cell periodic halo into LDS (complex, 16 B each), then every thread
// updates one point: faces x-, x+, y-, y+ of each species (fma(d, nb - c,
// acc), as face<LAPLACE>), then p = v^2, q = w p, R_v = (fma(-4, vr, 1) + qr,
// fma(-4, vi, qi)), R_w = (fma(3, vr, -qr), fma(3, vi, -qi)),
// f = fma(acc, inv_h2, R), and the Euler update of euler(). The CPU check
// evaluates the same expressions in the same order. With EMB the embedded
// first-order solution of the error estimate is advanced as well.
//
// HBM traffic per point and stage: 32 B in (two complex values; 16 B real on
// a first stage), 32 B out, plus the tile halos (1.16 x the reads); with EMB
// 16 B more each way.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace {

using namespace dev;

constexpr int kBBX = 64, kBBY = 8;

struct BrussArgs {
    const double *in_re;        // first stage: real state (v then w)
    const double2 *in_c;        // complex stage (v then w)
    double *out_re;
    double2 *out_c;
    const double *emb_in;
    double *emb_out;
    int nx, ny, ntx;
    long long n;                // points per species
    double inv_h2, d, tr, ti;
};

template <bool IN_REAL, bool OUT_REAL, bool EMB>
__global__ __launch_bounds__(kBBX *kBBY) void bruss_stage(BrussArgs a)
{
    constexpr int SX = kBBX + 2, SY = kBBY + 2, PL = SX * SY;
    __shared__ double2 sV[PL], sW[PL];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int x0 = (lb % a.ntx) * kBBX, y0 = (lb / a.ntx) * kBBY;
    const int tid = threadIdx.x;
    for (int k = tid; k < PL; k += kBBX * kBBY) {
        const int gx = wrap(x0 - 1 + k % SX, a.nx), gy = wrap(y0 - 1 + k / SX, a.ny);
        const long long i = gx + (long long)a.nx * gy;
        if (IN_REAL) {
            sV[k] = make_double2(a.in_re[i], 0.0);
            sW[k] = make_double2(a.in_re[a.n + i], 0.0);
        } else {
            sV[k] = a.in_c[i];
            sW[k] = a.in_c[a.n + i];
        }
    }
    __syncthreads();
    const int tx = tid % kBBX, ty = tid / kBBX;
    const int x = x0 + tx, y = y0 + ty;
    if (x >= a.nx || y >= a.ny) return;
    const int sl = (ty + 1) * SX + tx + 1;
    const double2 v = sV[sl], w = sW[sl];
    double avr = 0.0, avi = 0.0, awr = 0.0, awi = 0.0;
    const int nb[4] = {sl - 1, sl + 1, sl - SX, sl + SX};
#pragma unroll
    for (int f = 0; f < 4; ++f)
        face<LAP>(avr, avi, v, sV[nb[f]], 0.0, 0.0, false, 0.0, 0.0, a.d);
#pragma unroll
    for (int f = 0; f < 4; ++f)
        face<LAP>(awr, awi, w, sW[nb[f]], 0.0, 0.0, false, 0.0, 0.0, a.d);
    double pr, pi;
    csq(v, pr, pi);
    const double qr = fma(w.x, pr, -(w.y * pi)), qi = fma(w.x, pi, w.y * pr);
    const double rvr = fma(-4.0, v.x, 1.0) + qr, rvi = fma(-4.0, v.y, qi);
    const double rwr = fma(3.0, v.x, -qr), rwi = fma(3.0, v.y, -qi);
    const double fvr = fma(avr, a.inv_h2, rvr), fvi = fma(avi, a.inv_h2, rvi);
    const double fwr = fma(awr, a.inv_h2, rwr), fwi = fma(awi, a.inv_h2, rwi);
    const double2 nv = make_double2(fma(a.tr, fvr, fma(-a.ti, fvi, v.x)),
                                    fma(a.tr, fvi, fma(a.ti, fvr, v.y)));
    const double2 nw = make_double2(fma(a.tr, fwr, fma(-a.ti, fwi, w.x)),
                                    fma(a.tr, fwi, fma(a.ti, fwr, w.y)));
    const long long i = x + (long long)a.nx * y;
    if (OUT_REAL) {
        a.out_re[i] = nv.x;
        a.out_re[a.n + i] = nw.x;
    } else {
        a.out_c[i] = nv;
        a.out_c[a.n + i] = nw;
    }
    if (EMB) {
        a.emb_out[i] = fma(a.tr, fvr, IN_REAL ? v.x : a.emb_in[i]);
        a.emb_out[a.n + i] = fma(a.tr, fwr, IN_REAL ? w.x : a.emb_in[a.n + i]);
    }
}

// Reaction part of the Gershgorin bound, per cell
// max(|2vw - 4| + v^2, v^2 + |3 - 2vw|), maximised over the grid in
// partials[kReduceBlocks] (first pass here, second pass in reduce.hip's
// order: a maximum is exact in any order).
__global__ __launch_bounds__(256) void bruss_react_max(const double *s, long long n,
                                                       double *partials)
{
    double m = 0.0;
    for (long long p = blockIdx.x * 256LL + threadIdx.x; p < n; p += (long long)gridDim.x * 256) {
        const double v = s[p], x = s[n + p];
        const double vx = v * x, v2 = v * v;
        const double aa = fabs(2.0 * vx - 4.0) + v2;
        const double bb = v2 + fabs(3.0 - 2.0 * vx);
        const double c = aa > bb ? aa : bb;
        m = c > m ? c : m;
    }
    __shared__ double sm[4];
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sm[0];
        for (int k = 1; k < 4; ++k) r = sm[k] > r ? sm[k] : r;
        partials[blockIdx.x] = r;
    }
}

}  // namespace

int launch_bruss(const KGrid &g, const PassArgs &p, hipStream_t st)
{
    if (g.op != FRKC2_OP_BRUSS2 || g.ndim != 2 || p.k != 1) return (int)hipErrorInvalidValue;
    BrussArgs a{};
    a.in_re = p.in_re;
    a.in_c = reinterpret_cast<const double2 *>(p.in_c);
    a.out_re = p.out_re;
    a.out_c = reinterpret_cast<double2 *>(p.out_c);
    a.emb_in = p.emb_in;
    a.emb_out = p.emb_out;
    a.nx = g.nx;
    a.ny = g.nz;   // 2D grids keep their second dimension in nz
    a.ntx = (g.nx + kBBX - 1) / kBBX;
    a.n = g.npts();
    a.inv_h2 = g.inv_h2;
    a.d = g.d_const;
    a.tr = p.tr[0];
    a.ti = p.ti[0];
    const long long nblk = (long long)a.ntx * ((a.ny + kBBY - 1) / kBBY);
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    const dim3 grid((unsigned)nblk), block(kBBX * kBBY);
    const bool ir = p.in_re != nullptr, orl = p.out_re != nullptr;
    if (p.emb_out) {
        if (orl) return (int)hipErrorInvalidValue;
        if (ir) hipLaunchKernelGGL((bruss_stage<true, false, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((bruss_stage<false, false, true>), grid, block, 0, st, a);
    } else if (ir && orl) {
        hipLaunchKernelGGL((bruss_stage<true, true, false>), grid, block, 0, st, a);
    } else if (ir) {
        hipLaunchKernelGGL((bruss_stage<true, false, false>), grid, block, 0, st, a);
    } else if (orl) {
        hipLaunchKernelGGL((bruss_stage<false, true, false>), grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL((bruss_stage<false, false, false>), grid, block, 0, st, a);
    }
    return (int)hipGetLastError();
}

int launch_bruss_react_max(const KGrid &g, const double *w, double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(bruss_react_max, dim3(kReduceBlocks), dim3(256), 0, st, w, g.npts(),
                       partials);
    return (int)hipGetLastError();
}

}  // namespace frkc2
