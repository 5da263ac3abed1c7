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
// 16 B more each way. bruss_tb (below) fuses 2..4 stages per pass: 64 B per
// point and pass plus its halo reads, spread over the pass's stages.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace {

using namespace dev;

constexpr int kBBX = 64, kBBY = 8;

// One Euler stage at one point from the point's and its four neighbours'
// values of both species (x-, x+, y-, y+): the fixed arithmetic of the header
// comment. fvr, fwr: Re f of each species (for the embedded solution).
__device__ __forceinline__ void bruss_point(double2 v, double2 w, double2 vxm, double2 vxp,
                                            double2 vym, double2 vyp, double2 wxm, double2 wxp,
                                            double2 wym, double2 wyp, double d, double inv_h2,
                                            double tr, double ti, double2 &nv, double2 &nw,
                                            double &fvr, double &fwr)
{
    double avr = 0.0, avi = 0.0, awr = 0.0, awi = 0.0;
    face<LAP>(avr, avi, v, vxm, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(avr, avi, v, vxp, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(avr, avi, v, vym, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(avr, avi, v, vyp, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(awr, awi, w, wxm, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(awr, awi, w, wxp, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(awr, awi, w, wym, 0.0, 0.0, false, 0.0, 0.0, d);
    face<LAP>(awr, awi, w, wyp, 0.0, 0.0, false, 0.0, 0.0, d);
    double pr, pi;
    csq(v, pr, pi);
    const double qr = fma(w.x, pr, -(w.y * pi)), qi = fma(w.x, pi, w.y * pr);
    const double rvr = fma(-4.0, v.x, 1.0) + qr, rvi = fma(-4.0, v.y, qi);
    const double rwr = fma(3.0, v.x, -qr), rwi = fma(3.0, v.y, -qi);
    fvr = fma(avr, inv_h2, rvr);
    fwr = fma(awr, inv_h2, rwr);
    const double fvi = fma(avi, inv_h2, rvi), fwi = fma(awi, inv_h2, rwi);
    nv = make_double2(fma(tr, fvr, fma(-ti, fvi, v.x)), fma(tr, fvi, fma(ti, fvr, v.y)));
    nw = make_double2(fma(tr, fwr, fma(-ti, fwi, w.x)), fma(tr, fwi, fma(ti, fwr, w.y)));
}

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
    double2 nv, nw;
    double fvr, fwr;
    bruss_point(v, w, sV[sl - 1], sV[sl + 1], sV[sl - SX], sV[sl + SX], sW[sl - 1], sW[sl + 1],
                sW[sl - SX], sW[sl + SX], a.d, a.inv_h2, a.tr, a.ti, nv, nw, fvr, fwr);
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

// K stages (2..6) in one HBM pass. A workgroup of NW wavefronts works on a
// 64 x (NW R) extended tile of both species (periodic wrap) and writes its
// (64 - 2K) x (NW R - 2K) centre. Lane x of wavefront r owns column x, rows
// rR .. rR+R-1, and keeps their complex values of both species in registers
// through all K stages: x neighbours come from the adjacent lanes (DPP
// wavefront shifts), y neighbours from the thread's own rows, except the two
// rows beyond its strip, which the wavefronts above and below publish in LDS
// once per stage (two slots by stage parity, one barrier per stage). Stage m
// updates every column of the rows m .. NW R - 1 - m (rows outside are left as
// they are; the test is uniform over a wavefront); only the points at least m
// cells inside the tile then hold stage m values (lanes 0 and 63 take
// shifted-in values), so the centre is exact after K stages. bruss_point() does the arithmetic, so the result
// equals K single-stage passes bit for bit. With EMB each thread also carries
// the embedded first-order solution of its points (real, advanced by Re tau
// Re f per stage as in bruss_stage; it needs no neighbours).
constexpr int kTBX = 64;

struct BrussTbArgs {
    const double *in_re;
    const double2 *in_c;
    double *out_re;
    double2 *out_c;
    const double *emb_in;       // embedded solution in (complex input) and out
    double *emb_out;
    int nx, ny, ntx;
    long long n;
    double inv_h2, d;
    double tr[kMaxTBlock], ti[kMaxTBlock];
};

// The value of lane i - 1 (SHR) or i + 1 (SHL) of the wavefront; 0 at the end
// lane (the DPP move's bound control writes 0 where the source lane is out of
// the wavefront, so no destination has to be cleared first).
template <bool SHR>
__device__ __forceinline__ double lane_shift(double v)
{
    constexpr int ctrl = SHR ? 0x138 : 0x130;   // DPP wave_shr:1 / wave_shl:1
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <bool SHR>
__device__ __forceinline__ double2 lane_shift2(double2 v)
{
    return make_double2(lane_shift<SHR>(v.x), lane_shift<SHR>(v.y));
}

template <int K, bool IN_REAL, bool OUT_REAL, bool EMB, int NW, int R>
__global__ __launch_bounds__(kTBX *NW) void bruss_tb(BrussTbArgs a)
{
    constexpr int TY = NW * R, OX = kTBX - 2 * K, OY = TY - 2 * K;
    // [parity][wavefront][top, bottom row][lane]: v, w
    __shared__ double2 sEdge[2][NW][2][kTBX][2];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % a.ntx, by = lb / a.ntx;
    const int tx = threadIdx.x & (kTBX - 1), wv = threadIdx.x >> 6, r0 = wv * R;
    const int xs = bx * OX - K + tx, ys = by * OY - K + r0;
    double2 v[R], w[R];
    double ev[EMB ? R : 1], ew[EMB ? R : 1];   // embedded solution (real), EMB only
    {
        const long long gx = wrap(xs, a.nx);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const long long i = gx + (long long)a.nx * wrap(ys + j, a.ny);
            if (IN_REAL) {
                v[j] = make_double2(a.in_re[i], 0.0);
                w[j] = make_double2(a.in_re[a.n + i], 0.0);
            } else {
                v[j] = a.in_c[i];
                w[j] = a.in_c[a.n + i];
            }
            if (EMB) {
                ev[j] = IN_REAL ? v[j].x : a.emb_in[i];
                ew[j] = IN_REAL ? w[j].x : a.emb_in[a.n + i];
            }
        }
    }
    const int wu = wv > 0 ? wv - 1 : wv, wd = wv < NW - 1 ? wv + 1 : wv;
#pragma unroll
    for (int m = 0; m < K; ++m) {
        const int par = m & 1;
        sEdge[par][wv][0][tx][0] = v[0];
        sEdge[par][wv][0][tx][1] = w[0];
        sEdge[par][wv][1][tx][0] = v[R - 1];
        sEdge[par][wv][1][tx][1] = w[R - 1];
        __syncthreads();
        // the row above the strip (the wavefront above's bottom row; the tile's
        // top wavefront repeats its own top row) and the row below it
        double2 vu = sEdge[par][wu][wv > 0 ? 1 : 0][tx][0];
        double2 wu2 = sEdge[par][wu][wv > 0 ? 1 : 0][tx][1];
        const double2 vdn = sEdge[par][wd][wv < NW - 1 ? 0 : 1][tx][0];
        const double2 wdn = sEdge[par][wd][wv < NW - 1 ? 0 : 1][tx][1];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const double2 vd = (j + 1 < R) ? v[j + 1] : vdn, wd2 = (j + 1 < R) ? w[j + 1] : wdn;
            const double2 vo = v[j], wo = w[j];
            // rows outside the stage's range are left as they are (the test is
            // uniform over the wavefront)
            if (r0 + j > m && r0 + j < TY - 1 - m) {
                double fvr, fwr;
                bruss_point(vo, wo, lane_shift2<true>(vo), lane_shift2<false>(vo), vu, vd,
                            lane_shift2<true>(wo), lane_shift2<false>(wo), wu2, wd2, a.d,
                            a.inv_h2, a.tr[m], a.ti[m], v[j], w[j], fvr, fwr);
                if (EMB) {
                    ev[j] = fma(a.tr[m], fvr, ev[j]);
                    ew[j] = fma(a.tr[m], fwr, ew[j]);
                }
            }
            vu = vo;
            wu2 = wo;
        }
    }
    if (tx < K || tx >= kTBX - K || xs >= a.nx) return;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int e = r0 + j;
        if (e >= K && e < TY - K && ys + j < a.ny) {
            const long long i = xs + (long long)a.nx * (ys + j);
            if (OUT_REAL) {
                a.out_re[i] = v[j].x;
                a.out_re[a.n + i] = w[j].x;
            } else {
                a.out_c[i] = v[j];
                a.out_c[a.n + i] = w[j];
            }
            if (EMB) {
                a.emb_out[i] = ev[j];
                a.emb_out[a.n + i] = ew[j];
            }
        }
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

// 4 wavefronts of 10 rows: 64 x 40 tiles, about 150 VGPRs, three workgroups
// per CU (8 and 12 rows, 8 wavefronts x 8 rows, 16 x 4 and a 128-VGPR cap
// measured 2-20 % slower at 2048^2).
constexpr int kTbWaves = 4, kTbRows = 10;

template <int K>
int launch_bruss_tb_k(const BrussTbArgs &a, unsigned nblk, bool ir, bool orl, hipStream_t st)
{
    constexpr int NW = kTbWaves, R = kTbRows;
    const dim3 grid(nblk), block(kTBX * NW);
    if (a.emb_out) {
        if (ir) hipLaunchKernelGGL((bruss_tb<K, true, false, true, NW, R>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((bruss_tb<K, false, false, true, NW, R>), grid, block, 0, st, a);
    } else if (ir && orl) {
        hipLaunchKernelGGL((bruss_tb<K, true, true, false, NW, R>), grid, block, 0, st, a);
    } else if (ir) {
        hipLaunchKernelGGL((bruss_tb<K, true, false, false, NW, R>), grid, block, 0, st, a);
    } else if (orl) {
        hipLaunchKernelGGL((bruss_tb<K, false, true, false, NW, R>), grid, block, 0, st, a);
    } else {
        hipLaunchKernelGGL((bruss_tb<K, false, false, false, NW, R>), grid, block, 0, st, a);
    }
    return (int)hipGetLastError();
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

int launch_bruss_tb(const KGrid &g, const PassArgs &p, hipStream_t st)
{
    if (g.op != FRKC2_OP_BRUSS2 || g.ndim != 2 || p.k < 2 || p.k > 6)
        return (int)hipErrorInvalidValue;
    // the embedded variant writes complex W and reads emb_in after the first stage
    if (p.emb_out && (p.out_re || (!p.in_re && !p.emb_in))) return (int)hipErrorInvalidValue;
    if ((p.in_re != nullptr) == (p.in_c != nullptr) ||
        (p.out_re != nullptr) == (p.out_c != nullptr))
        return (int)hipErrorInvalidValue;
    BrussTbArgs a{};
    a.in_re = p.in_re;
    a.in_c = reinterpret_cast<const double2 *>(p.in_c);
    a.out_re = p.out_re;
    a.out_c = reinterpret_cast<double2 *>(p.out_c);
    a.emb_in = p.emb_in;
    a.emb_out = p.emb_out;
    a.nx = g.nx;
    a.ny = g.nz;   // 2D grids keep their second dimension in nz
    a.n = g.npts();
    a.inv_h2 = g.inv_h2;
    a.d = g.d_const;
    for (int m = 0; m < p.k; ++m) {
        a.tr[m] = p.tr[m];
        a.ti[m] = p.ti[m];
    }
    const int ox = kTBX - 2 * p.k, oy = kTbWaves * kTbRows - 2 * p.k;
    a.ntx = (a.nx + ox - 1) / ox;
    const long long nblk = (long long)a.ntx * ((a.ny + oy - 1) / oy);
    if (nblk <= 0) return 0;
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    const bool ir = p.in_re != nullptr, orl = p.out_re != nullptr;
    if (p.k == 2) return launch_bruss_tb_k<2>(a, (unsigned)nblk, ir, orl, st);
    if (p.k == 3) return launch_bruss_tb_k<3>(a, (unsigned)nblk, ir, orl, st);
    if (p.k == 4) return launch_bruss_tb_k<4>(a, (unsigned)nblk, ir, orl, st);
    if (p.k == 5) return launch_bruss_tb_k<5>(a, (unsigned)nblk, ir, orl, st);
    return launch_bruss_tb_k<6>(a, (unsigned)nblk, ir, orl, st);
}

int launch_bruss_react_max(const KGrid &g, const double *w, double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(bruss_react_max, dim3(kReduceBlocks), dim3(256), 0, st, w, g.npts(),
                       partials);
    return (int)hipGetLastError();
}

}  // namespace frkc2
