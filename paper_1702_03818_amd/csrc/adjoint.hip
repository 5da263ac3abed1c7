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

    // Loads without branches (clamped index, a Dirichlet ghost selected to
    // 0 afterwards), so that a plane's loads are all in flight together.
    auto ldL = [&](int gx, int gy, int gz) {
        return load_c_nb<BC, IN_REAL>(dm, a.lin_re, a.lin_c, gx, gy, gz);
    };
    auto ldW = [&](int gx, int gy, int gz) {
        return load_c_nb<BC, false>(dm, nullptr, a.W, gx, gy, gz);
    };
    auto ldD = [&](int gx, int gy, int gz) { return 0.5 * load_r_nb<BC>(dm, a.D, gx, gy, gz); };
    // the dJ/dD accumulator of the lane's cell (any cell for an idle lane:
    // the read is then discarded), read one plane ahead of its update
    const long long pst = (long long)a.nx * a.ny;
    const long long ixy = min(x, a.nx - 1) + (long long)a.nx * min(y, a.ny - 1);

    double2 Lm = ldL(x, y, z0 - 1), Lc = ldL(x, y, z0), Lp = ldL(x, y, z0 + 1);
    double2 Wm = make_double2(0.0, 0.0), Wc = Wm, Wp = Wm;
    double Dm = 0.0, Dc = 0.0, Dp = 0.0, Gc = 0.0;
    if (VC) {
        Wm = ldW(x, y, z0 - 1);
        Wc = ldW(x, y, z0);
        Wp = ldW(x, y, z0 + 1);
        Dm = ldD(x, y, z0 - 1);
        Dc = ldD(x, y, z0);
        Dp = ldD(x, y, z0 + 1);
        Gc = a.gD[ixy + pst * z0];
    }
    double2 hL = make_double2(0.0, 0.0), hW = hL;
    double hD = 0.0;
    if (has_halo) {
        hL = ldL(x0 + hx, y0 + hy, z0);
        if (VC) {
            hW = ldW(x0 + hx, y0 + hy, z0);
            hD = ldD(x0 + hx, y0 + hy, z0);
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
                hD = ldD(x0 + hx, y0 + hy, z + 1);
            }
        }
        // next plane's accumulator, in flight during this plane's work
        const double Gn = (VC && z + 1 < z1) ? a.gD[ixy + pst * (z + 1)] : 0.0;
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
            if (VC) a.gD[i] = Gc - gsum * a.inv_h2;
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
            Gc = Gn;
        }
        if (z + 1 < z1) {
            Lp = ldL(x, y, z + 2);
            if (VC) {
                Wp = ldW(x, y, z + 2);
                Dp = ldD(x, y, z + 2);
            }
        }
    }
}

// Two reverse stages in one pass (3D grids). The pass takes lam^{l+1} to
// lam^{l-1} through stages l and l-1, with the same per-cell arithmetic as
// adjoint_stage at each (so the same bits), and subtracts both stages'
// dJ/dD shares from gD in that order: 88 bytes per cell and pair (lam in and
// out, W^l and W^{l-1}, D, gD read and written) against 144 for two passes.
//
// Tile: kPX x kPY threads, one column each, of an extended tile whose
// kPK-cell rim is halo: 32 x 24 output columns. The tile marches up its z
// chunk; at step t the first stage (level 1) computes plane t-1 from lam^{l+1}
// and W^l, the second (level 2) plane t-2 from level 1 and W^{l-1}, so the
// chunk takes zchunk + 2 steps. z neighbours are in per-thread register
// rings (the t-3 planes level 2 reads in LDS rings); x and y neighbours of the
// planes a step reads are written to LDS first (one buffer per plane, a
// barrier before and after the writes). Level 1 is
// valid one cell in from the tile edge, level 2 two cells in (the outputs).
// A Dirichlet ghost column never writes LDS, which starts at zero (lam = W =
// 0 there); a ghost plane's level-1 value is set to 0.
constexpr int kPX = 36, kPY = 21, kPK = 2;
constexpr int kPairThreads = kPX * kPY;

struct AdjPairArgs {
    const double *lin_re;       // lam^{l+1}: real (first pass) or complex
    const double2 *lin_c;
    double *lout_re;            // lam^{l-1}: real (last pass) or complex
    double2 *lout_c;
    const double2 *W1, *W2;     // stored stages W^l and W^{l-1}
    const double *D;
    double *gD;
    int nx, ny, nz;
    int zchunk, ntx, nty;
    double inv_h2, d_const, tr1, ti1, tr2, ti2;
};

template <int OP, int BC, bool IN_REAL, bool OUT_REAL>
__global__ __launch_bounds__(kPairThreads) void adjoint_pair(AdjPairArgs a)
{
    constexpr int SX = kPX + 2, SY = kPY + 2, PL = SX * SY;
    constexpr bool VC = (OP == VAR);
    constexpr bool dir = (BC == DIR);
    __shared__ double2 sL0[PL], sL1[2][PL];
    __shared__ double2 sW1[VC ? PL : 1], sW2[2][VC ? PL : 1];
    __shared__ double sD[3][VC ? PL : 1];     // D/2 of plane p in slot p mod 3

    const int tid = threadIdx.x;
    const int lx = tid % kPX, ly = tid / kPX;
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % a.ntx;
    lb /= a.ntx;
    const int by = lb % a.nty;
    const int bz = lb / a.nty;
    const int x = bx * (kPX - 2 * kPK) - kPK + lx;
    const int y = by * (kPY - 2 * kPK) - kPK + ly;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const bool ghost_col = dir && !(x >= 0 && x < a.nx && y >= 0 && y < a.ny);
    const int need = min(min(lx, kPX - 1 - lx), min(ly, kPY - 1 - ly));
    const bool out_col = need >= kPK && x < a.nx && y < a.ny;
    const int slot = (ly + 1) * SX + lx + 1;
    const int cx = (BC == PER) ? wrap(x, a.nx) : min(max(x, 0), a.nx - 1);
    const int cy = (BC == PER) ? wrap(y, a.ny) : min(max(y, 0), a.ny - 1);
    const long long ixy = cx + (long long)a.nx * cy;
    const long long pst = (long long)a.nx * a.ny;
    auto zi = [&](int gz) {
        return pst * ((BC == PER) ? wrap(gz, a.nz) : min(max(gz, 0), a.nz - 1));
    };
    auto pout = [&](int p) { return dir && (p < 0 || p >= a.nz); };
    const double2 zero = make_double2(0.0, 0.0);
    // loads at plane p: lam and W are 0 at a Dirichlet ghost; D is halved
    // once (its ghost value is never used: ghost faces take D_c)
    auto LL = [&](int p) {
        const long long i = ixy + zi(p);
        double2 v = IN_REAL ? make_double2(a.lin_re[i], 0.0) : a.lin_c[i];
        return (ghost_col || pout(p)) ? zero : v;
    };
    auto LW = [&](const double2 *W, int p) {
        if (!VC) return zero;
        const double2 v = W[ixy + zi(p)];
        return (ghost_col || pout(p)) ? zero : v;
    };
    auto LD = [&](int p) { return VC ? 0.5 * a.D[ixy + zi(p)] : 0.0; };

    auto m3 = [](int p) { return ((p % 3) + 3) % 3; };
    for (int i = tid; i < PL; i += kPairThreads) {
        sL0[i] = zero;
        sL1[0][i] = zero;
        sL1[1][i] = zero;
        if (VC) {
            sW1[i] = zero;
            sW2[0][i] = zero;
            sW2[1][i] = zero;
            sD[0][i] = 0.0;
            sD[1][i] = 0.0;
            sD[2][i] = 0.0;
        }
    }
    // rings at the first step t = z0
    double2 l0m = LL(z0 - 2), l0c = LL(z0 - 1), l0p = LL(z0);          // lam^{l+1}: t-2 .. t
    double2 w1m = LW(a.W1, z0 - 2), w1c = LW(a.W1, z0 - 1), w1p = LW(a.W1, z0);   // t-2 .. t
    double2 w2c = LW(a.W2, z0 - 2), w2p = LW(a.W2, z0 - 1);            // W^{l-1}: t-2, t-1
    double d2 = LD(z0 - 2), d1 = LD(z0 - 1), d0 = LD(z0);               // D/2: t-2 .. t
    double2 l1c = zero;                                                 // level 1: t-2
    double gs1 = 0.0;                 // level 1's face sum at t-2
    double gin = 0.0;                 // gD at t-2 as read
    __syncthreads();

    for (int t = z0; t <= z1 + 1; ++t) {
        // planes for the next step
        const double2 l0n = LL(t + 1);
        const double2 w1n = LW(a.W1, t + 1);
        const double dnn = LD(t + 1);
        const double2 w2n = LW(a.W2, t);
        const int p2 = t - 2;
        const double gn = (VC && out_col && p2 + 1 >= z0 && p2 + 1 < z1)
                              ? a.gD[ixy + pst * (p2 + 1)] : 0.0;

        // lam^{l+1} and W^l at t-1, level 1 and W^{l-1} at t-2 (t-3 in the
        // other slot, written a step before), D at t-1 (t-2, t-3 in the others)
        if (!ghost_col) {
            sL0[slot] = l0c;
            sL1[t & 1][slot] = l1c;
            if (VC) {
                sW1[slot] = w1c;
                sW2[t & 1][slot] = w2c;
                sD[m3(t - 1)][slot] = d1;
            }
        }
        __syncthreads();

        // level 1 (stage l) at plane p1 = t-1
        const int p1 = t - 1;
        double2 l1n;
        double gs1n;
        {
            const double *Dp = VC ? sD[m3(p1)] : nullptr;
            auto S = [&](int off) { return VC ? sW1[slot + off] : zero; };
            auto SD = [&](int off) { return VC ? Dp[slot + off] : 0.0; };
            double gsum = 0.0, acc_r = 0.0, acc_i = 0.0;
            adj_face<OP>(gsum, acc_r, acc_i, l0c, sL0[slot - 1], w1c, S(-1), d1, SD(-1),
                         dir && x == 0, a.tr1, a.ti1, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l0c, sL0[slot + 1], w1c, S(1), d1, SD(1),
                         dir && x == a.nx - 1, a.tr1, a.ti1, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l0c, sL0[slot - SX], w1c, S(-SX), d1, SD(-SX),
                         dir && y == 0, a.tr1, a.ti1, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l0c, sL0[slot + SX], w1c, S(SX), d1, SD(SX),
                         dir && y == a.ny - 1, a.tr1, a.ti1, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l0c, l0m, w1c, w1m, d1, d2, dir && p1 == 0,
                         a.tr1, a.ti1, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l0c, l0p, w1c, w1p, d1, d0, dir && p1 == a.nz - 1,
                         a.tr1, a.ti1, a.d_const);
            const double gr = acc_r * a.inv_h2;
            const double gi = acc_i * a.inv_h2;
            l1n = make_double2(l0c.x + (a.tr1 * gr + a.ti1 * gi),
                               l0c.y + (a.tr1 * gi - a.ti1 * gr));
            if (pout(p1)) l1n = zero;
            gs1n = gsum;
        }
        // keep level 2's LDS reads after level 1 (their registers would not fit beside it)
        __builtin_amdgcn_sched_barrier(0);
        // level 2 (stage l-1) at plane p2, an output plane from t = z0 + 2 on;
        // gD takes stage l's share, then stage l-1's
        if (p2 >= z0) {
            const double *Dp = VC ? sD[m3(p2)] : nullptr;
            const double2 *L1 = sL1[t & 1], *W2 = VC ? sW2[t & 1] : nullptr;
            auto S = [&](int off) { return VC ? W2[slot + off] : zero; };
            auto SD = [&](int off) { return VC ? Dp[slot + off] : 0.0; };
            // plane t-3 from the other slots
            const double2 l1m = sL1[(t + 1) & 1][slot];
            const double2 w2m = VC ? sW2[(t + 1) & 1][slot] : zero;
            const double d3 = VC ? sD[m3(t - 3)][slot] : 0.0;
            double gsum = 0.0, acc_r = 0.0, acc_i = 0.0;
            adj_face<OP>(gsum, acc_r, acc_i, l1c, L1[slot - 1], w2c, S(-1), d2, SD(-1),
                         dir && x == 0, a.tr2, a.ti2, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l1c, L1[slot + 1], w2c, S(1), d2, SD(1),
                         dir && x == a.nx - 1, a.tr2, a.ti2, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l1c, L1[slot - SX], w2c, S(-SX), d2, SD(-SX),
                         dir && y == 0, a.tr2, a.ti2, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l1c, L1[slot + SX], w2c, S(SX), d2, SD(SX),
                         dir && y == a.ny - 1, a.tr2, a.ti2, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l1c, l1m, w2c, w2m, d2, d3, dir && p2 == 0,
                         a.tr2, a.ti2, a.d_const);
            adj_face<OP>(gsum, acc_r, acc_i, l1c, l1n, w2c, w2p, d2, d1, dir && p2 == a.nz - 1,
                         a.tr2, a.ti2, a.d_const);
            if (out_col) {
                const long long i = ixy + pst * p2;
                if (VC) a.gD[i] = (gin - gs1 * a.inv_h2) - gsum * a.inv_h2;
                const double gr = acc_r * a.inv_h2;
                const double gi = acc_i * a.inv_h2;
                const double nr = l1c.x + (a.tr2 * gr + a.ti2 * gi);
                const double ni = l1c.y + (a.tr2 * gi - a.ti2 * gr);
                if (OUT_REAL) a.lout_re[i] = nr;
                else a.lout_c[i] = make_double2(nr, ni);
            }
        }
        __syncthreads();   // this step's LDS reads end before the next step's writes
        l0m = l0c;
        l0c = l0p;
        l0p = l0n;
        w1m = w1c;
        w1c = w1p;
        w1p = w1n;
        w2c = w2p;
        w2p = w2n;
        d2 = d1;
        d1 = d0;
        d0 = dnn;
        l1c = l1n;
        gs1 = gs1n;
        gin = gn;
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

template <int OP, int BC>
int launch_pair_bc(const AdjPairArgs &a, bool ir, bool orl, int nblk, hipStream_t st)
{
    dim3 grid((unsigned)nblk), block(kPairThreads);
    if (ir && orl)
        hipLaunchKernelGGL((adjoint_pair<OP, BC, true, true>), grid, block, 0, st, a);
    else if (ir)
        hipLaunchKernelGGL((adjoint_pair<OP, BC, true, false>), grid, block, 0, st, a);
    else if (orl)
        hipLaunchKernelGGL((adjoint_pair<OP, BC, false, true>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((adjoint_pair<OP, BC, false, false>), grid, block, 0, st, a);
    return (int)hipGetLastError();
}

}  // namespace

int launch_adjoint_pair(const KGrid &g, const AdjArgs &a1, const AdjArgs &a2, hipStream_t st)
{
    if (g.ndim != 3 || (g.op != VAR && g.op != LAP)) return (int)hipErrorInvalidValue;
    AdjPairArgs p{};
    p.lin_re = a1.lam_in_re;
    p.lin_c = reinterpret_cast<const double2 *>(a1.lam_in_c);
    p.lout_re = a2.lam_out_re;
    p.lout_c = reinterpret_cast<double2 *>(a2.lam_out_c);
    p.W1 = reinterpret_cast<const double2 *>(a1.W);
    p.W2 = reinterpret_cast<const double2 *>(a2.W);
    p.D = a1.D;
    p.gD = a1.gD;
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    p.inv_h2 = g.inv_h2;
    p.d_const = g.d_const;
    p.tr1 = a1.tr;
    p.ti1 = a1.ti;
    p.tr2 = a2.tr;
    p.ti2 = a2.ti;
    p.ntx = (g.nx + kPX - 2 * kPK - 1) / (kPX - 2 * kPK);
    p.nty = (g.ny + kPY - 2 * kPK - 1) / (kPY - 2 * kPK);
    // chunk length: fewest rounds of one workgroup per CU (the LDS allows
    // one) times the zchunk + 2 steps of a tile, the longer chunk on a tie
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        return (int)hipErrorInvalidValue;
    const long long txy = (long long)p.ntx * p.nty;
    long long best = -1;
    for (int zc = g.nz; zc >= 1; --zc) {
        const long long chunks = (g.nz + zc - 1) / zc;
        const long long rounds = (txy * chunks + cus - 1) / cus;
        const long long cost = rounds * (zc + 2);
        if (best < 0 || cost < best) {
            best = cost;
            p.zchunk = zc;
        }
    }
    const long long nblk = txy * ((g.nz + p.zchunk - 1) / p.zchunk);
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    const bool ir = a1.lam_in_re != nullptr, orl = a2.lam_out_re != nullptr;
    if (g.op == VAR) {
        if (g.bc == PER) return launch_pair_bc<VAR, PER>(p, ir, orl, (int)nblk, st);
        return launch_pair_bc<VAR, DIR>(p, ir, orl, (int)nblk, st);
    }
    if (g.bc == PER) return launch_pair_bc<LAP, PER>(p, ir, orl, (int)nblk, st);
    return launch_pair_bc<LAP, DIR>(p, ir, orl, (int)nblk, st);
}

namespace {
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
