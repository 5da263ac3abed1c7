// Reverse-mode stage kernel of the FRKC2 superstep (linear operators).
//
// A stage W^{l+1} = W^l + tau_l A(D) W^l (O'Sullivan, arXiv:1702.03818,
// Sec. 3, Euler-step equation) with A real symmetric has, for the adjoint
// lam = dJ/dRe W + i dJ/dIm W, the transpose lam^l = lam^{l+1} + conj(tau_l) A lam^{l+1}.
// Its dependence on the face diffusivity D_f of the face between cells c and
// nb is dJ/dD_f = -Re(tau_l conj(lam_nb - lam_c) (W_nb - W_c)) / h^2 with
// lam = lam^{l+1} and W = W^l; D_f = D_c/2 + D_nb/2 hands half of it to each
// cell, a Dirichlet boundary face (D_f = D_c, ghost W = lam = 0) all of it.
// The kernel fuses both: for every cell it accumulates its share into gD and
// writes lam^l. The stages run in reverse order; the reversed sequence has
// the same internal amplification Q as the forward one (contiguous runs are
// the same runs), so the adjoint is as stable (Sec. 2.2).
//
// Same plane-march tiling as the forward stage: lam, W and D of plane z with
// a one-cell halo in LDS, z-neighbours in registers.
//
// Per-cell arithmetic order (shared with the CPU check): faces x-, x+, y-,
// y+, z-, z+; pr = dLr*dWr + dLi*dWi, pi = dLr*dWi - dLi*dWr,
// e = tr*pr - ti*pi, gsum = gsum + w_f*e; gD = gD - gsum*inv_h2; the A lam
// sum as in the forward stage; lam_r + (tr*g_r + ti*g_i), lam_i + (tr*g_i - ti*g_r).
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace {

using namespace dev;

struct AdjPlaneArgs {
    const double *lin_re;
    const double2 *lin_c;
    double *lout_re;
    double2 *lout_c;
    const double2 *W;
    const double *D;
    double *gD;
    int nx, ny, nz;
    int zchunk, ntx, nty;
    double inv_h2, d_const, tr, ti;
};

template <int OP>
__device__ __forceinline__ void adj_face(double &gsum, double &acc_r, double &acc_i, double2 lc,
                                         double2 ln, double2 wc, double2 wn, double dc,
                                         double dn, bool ghost, double tr, double ti,
                                         double d_const)
{
    if (OP == VAR) {
        const double dWr = wn.x - wc.x, dWi = wn.y - wc.y;
        const double dLr = ln.x - lc.x, dLi = ln.y - lc.y;
        const double pr = dLr * dWr + dLi * dWi;
        const double pi = dLr * dWi - dLi * dWr;
        const double e = tr * pr - ti * pi;
        const double wgt = ghost ? 1.0 : 0.5;
        gsum = gsum + wgt * e;
    }
    face<OP>(acc_r, acc_i, lc, ln, dc, dn, ghost, 0.0, 0.0, d_const);
}

template <int OP, int BC, int NDIM, int BX, int BY, bool IN_REAL, bool OUT_REAL>
__global__ __launch_bounds__(BX *BY) void adjoint_stage(AdjPlaneArgs a)
{
    constexpr int SX = BX + 2;
    constexpr int SY = (NDIM == 3) ? BY + 2 : 1;
    constexpr int NH = 2 * BY + (NDIM == 3 ? 2 * BX : 0);
    static_assert(NH <= BX * BY, "one halo cell per thread at most");
    constexpr bool VC = (OP == VAR);
    __shared__ double2 sL[2][SY * SX];
    __shared__ double2 sW[2][VC ? SY * SX : 1];
    __shared__ double sD[2][VC ? SY * SX : 1];

    const Dims dm{a.nx, a.ny, a.nz};
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % a.ntx;
    lb /= a.ntx;
    const int by = lb % a.nty;
    const int bz = lb / a.nty;
    const int x0 = bx * BX, y0 = by * BY;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < a.nx && y < a.ny;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);

    int hx = 0, hy = 0;
    const bool has_halo = tid < NH;
    if (has_halo) {
        if (tid < 2 * BY) {
            hy = tid % BY;
            hx = (tid < BY) ? -1 : BX;
        } else {
            const int hh = tid - 2 * BY;
            hx = hh % BX;
            hy = (hh < BX) ? -1 : BY;
        }
    }
    const int hslot = (NDIM == 3 ? (hy + 1) * SX : 0) + (hx + 1);
    const int oslot = (NDIM == 3 ? (ty + 1) * SX : 0) + (tx + 1);

    auto ldL = [&](int gx, int gy, int gz) {
        return load_c<BC, IN_REAL>(dm, a.lin_re, a.lin_c, gx, gy, gz);
    };
    auto ldW = [&](int gx, int gy, int gz) {
        return load_c<BC, false>(dm, nullptr, a.W, gx, gy, gz);
    };

    double2 Lm = ldL(x, y, z0 - 1), Lc = ldL(x, y, z0), Lp = ldL(x, y, z0 + 1);
    double2 Wm = make_double2(0.0, 0.0), Wc = Wm, Wp = Wm;
    double Dm = 0.0, Dc = 0.0, Dp = 0.0;
    if (VC) {
        Wm = ldW(x, y, z0 - 1);
        Wc = ldW(x, y, z0);
        Wp = ldW(x, y, z0 + 1);
        Dm = 0.5 * load_r<BC>(dm, a.D, x, y, z0 - 1);
        Dc = 0.5 * load_r<BC>(dm, a.D, x, y, z0);
        Dp = 0.5 * load_r<BC>(dm, a.D, x, y, z0 + 1);
    }
    double2 hL = make_double2(0.0, 0.0), hW = hL;
    double hD = 0.0;
    if (has_halo) {
        hL = ldL(x0 + hx, y0 + hy, z0);
        if (VC) {
            hW = ldW(x0 + hx, y0 + hy, z0);
            hD = 0.5 * load_r<BC>(dm, a.D, x0 + hx, y0 + hy, z0);
        }
    }

    for (int z = z0; z < z1; ++z) {
        const int b = z & 1;
        sL[b][oslot] = Lc;
        if (VC) {
            sW[b][oslot] = Wc;
            sD[b][oslot] = Dc;
        }
        if (has_halo) {
            sL[b][hslot] = hL;
            if (VC) {
                sW[b][hslot] = hW;
                sD[b][hslot] = hD;
            }
        }
        __syncthreads();
        if (has_halo && z + 1 < z1) {
            hL = ldL(x0 + hx, y0 + hy, z + 1);
            if (VC) {
                hW = ldW(x0 + hx, y0 + hy, z + 1);
                hD = 0.5 * load_r<BC>(dm, a.D, x0 + hx, y0 + hy, z + 1);
            }
        }
        if (active) {
            const bool dir = (BC == DIR);
            double gsum = 0.0, acc_r = 0.0, acc_i = 0.0;
            const double2 zero = make_double2(0.0, 0.0);
            auto S = [&](int off) {
                return VC ? sW[b][oslot + off] : zero;
            };
            auto SD = [&](int off) { return VC ? sD[b][oslot + off] : 0.0; };
            adj_face<OP>(gsum, acc_r, acc_i, Lc, sL[b][oslot - 1], Wc, S(-1), Dc, SD(-1),
                         dir && x == 0, a.tr, a.ti, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, Lc, sL[b][oslot + 1], Wc, S(1), Dc, SD(1),
                         dir && x == a.nx - 1, a.tr, a.ti, a.d_const);
            if (NDIM == 3) {
                adj_face<OP>(gsum, acc_r, acc_i, Lc, sL[b][oslot - SX], Wc, S(-SX), Dc, SD(-SX),
                             dir && y == 0, a.tr, a.ti, a.d_const);
                adj_face<OP>(gsum, acc_r, acc_i, Lc, sL[b][oslot + SX], Wc, S(SX), Dc, SD(SX),
                             dir && y == a.ny - 1, a.tr, a.ti, a.d_const);
            }
            if (NDIM >= 2) {
                adj_face<OP>(gsum, acc_r, acc_i, Lc, Lm, Wc, Wm, Dc, Dm, dir && z == 0, a.tr,
                             a.ti, a.d_const);
                adj_face<OP>(gsum, acc_r, acc_i, Lc, Lp, Wc, Wp, Dc, Dp, dir && z == a.nz - 1,
                             a.tr, a.ti, a.d_const);
            }
            const long long i = x + (long long)a.nx * (y + (long long)a.ny * z);
            if (VC) a.gD[i] = a.gD[i] - gsum * a.inv_h2;
            const double gr = acc_r * a.inv_h2;
            const double gi = acc_i * a.inv_h2;
            const double nr = Lc.x + (a.tr * gr + a.ti * gi);
            const double ni = Lc.y + (a.tr * gi - a.ti * gr);
            if (OUT_REAL) a.lout_re[i] = nr;
            else a.lout_c[i] = make_double2(nr, ni);
        }
        Lm = Lc;
        Lc = Lp;
        if (VC) {
            Wm = Wc;
            Wc = Wp;
            Dm = Dc;
            Dc = Dp;
        }
        if (z + 1 < z1) {
            Lp = ldL(x, y, z + 2);
            if (VC) {
                Wp = ldW(x, y, z + 2);
                Dp = 0.5 * load_r<BC>(dm, a.D, x, y, z + 2);
            }
        }
    }
}

__global__ void grad_finish_kernel(const double *D, const double *gD, double *g, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        g[i] = g[i] + D[i] * gD[i];
}

int choose_zchunk(long long tiles_xy, int nz)
{
    int zc = nz;
    while (zc > 8 && tiles_xy * ((nz + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
    return zc;
}

template <int OP, int BC, int NDIM, int BX, int BY>
int launch_t(const AdjPlaneArgs &a0, bool ir, bool orl, hipStream_t st)
{
    AdjPlaneArgs a = a0;
    a.ntx = (a.nx + BX - 1) / BX;
    a.nty = (a.ny + BY - 1) / BY;
    a.zchunk = choose_zchunk((long long)a.ntx * a.nty, a.nz);
    const long long nblk = (long long)a.ntx * a.nty * ((a.nz + a.zchunk - 1) / a.zchunk);
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(BX * BY);
    if (ir && orl)
        hipLaunchKernelGGL((adjoint_stage<OP, BC, NDIM, BX, BY, true, true>), grid, block, 0, st, a);
    else if (ir)
        hipLaunchKernelGGL((adjoint_stage<OP, BC, NDIM, BX, BY, true, false>), grid, block, 0, st, a);
    else if (orl)
        hipLaunchKernelGGL((adjoint_stage<OP, BC, NDIM, BX, BY, false, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((adjoint_stage<OP, BC, NDIM, BX, BY, false, false>), grid, block, 0, st, a);
    return (int)hipGetLastError();
}

template <int OP, int BC>
int launch_dim(const KGrid &g, const AdjPlaneArgs &a, bool ir, bool orl, hipStream_t st)
{
    if (g.ndim == 3) return launch_t<OP, BC, 3, 64, 4>(a, ir, orl, st);
    if (g.ndim == 2) return launch_t<OP, BC, 2, 256, 1>(a, ir, orl, st);
    return launch_t<OP, BC, 1, 256, 1>(a, ir, orl, st);
}

template <int OP>
int launch_bc(const KGrid &g, const AdjPlaneArgs &a, bool ir, bool orl, hipStream_t st)
{
    if (g.bc == PER) return launch_dim<OP, PER>(g, a, ir, orl, st);
    return launch_dim<OP, DIR>(g, a, ir, orl, st);
}

}  // namespace

int launch_adjoint_stage(const KGrid &g, const AdjArgs &a, hipStream_t st)
{
    AdjPlaneArgs p{};
    p.lin_re = a.lam_in_re;
    p.lin_c = reinterpret_cast<const double2 *>(a.lam_in_c);
    p.lout_re = a.lam_out_re;
    p.lout_c = reinterpret_cast<double2 *>(a.lam_out_c);
    p.W = reinterpret_cast<const double2 *>(a.W);
    p.D = a.D;
    p.gD = a.gD;
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    p.inv_h2 = g.inv_h2;
    p.d_const = g.d_const;
    p.tr = a.tr;
    p.ti = a.ti;
    const bool ir = a.lam_in_re != nullptr, orl = a.lam_out_re != nullptr;
    if (g.op == VAR) return launch_bc<VAR>(g, p, ir, orl, st);
    if (g.op == LAP) return launch_bc<LAP>(g, p, ir, orl, st);
    return (int)hipErrorInvalidValue;
}

int launch_grad_finish(long long n, const double *D, const double *gD, double *grad_logD,
                       hipStream_t st)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(grad_finish_kernel, dim3((unsigned)blocks), dim3(256), 0, st, D, gD,
                       grad_logD, n);
    return (int)hipGetLastError();
}

}  // namespace frkc2
