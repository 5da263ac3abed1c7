// One tile of the temporally blocked stage kernel tb_stage (tblock.hip),
// shared with the batched pass kernels: K consecutive Euler stages
// W <- W + tau_l f(W) (O'Sullivan, arXiv:1702.03818, Sec. 3, Euler-step
// equation) of one extended tile in one HBM pass. The design is described in
// tblock.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace dev {

struct TbArgs {
    const double *in_re;
    const double2 *in_c;
    double *out_re;
    double2 *out_c;
    const double *emb_in;       // EMB: embedded first-order solution in (complex input) and out
    double *emb_out;
    const double *D;
    int nx, ny, nz;
    int zchunk, ntx, nty;
    double inv_h2, d_const;
    double tr[kMaxTBlock], ti[kMaxTBlock];
    double fc[6];
};

__device__ __forceinline__ double2 keep(double2 v, bool ghost)
{
    v.x = ghost ? 0.0 : v.x;
    v.y = ghost ? 0.0 : v.y;
    return v;
}

// LDS of one tile (level planes and diffusivity ring), for the caller to
// declare: the same shape computations as the tile itself.
template <int OP, int NDIM, int BXE, int TY, int R, int K>
struct TbLds {
    static constexpr int BYE = TY * R;
    static constexpr int SX = BXE + 2;
    static constexpr int SY = (NDIM == 3) ? BYE + 2 : 1;
    static constexpr int PL = SX * SY;
    static constexpr bool VC = (OP == FRKC2_OP_VARCOEF);
    static constexpr bool DB = (NDIM == 2) &&
                               (2 * K * PL * 16 + (VC ? (K + 2) * PL * 8 : 0) <= 160 * 1024);
    static constexpr int NB = DB ? 2 : 1;
    static constexpr int ND = DB ? K + 2 : K + 1;
    static constexpr int L = NB * K * PL;
    static constexpr int D = VC ? ND * PL : 1;
};

// NDIM 3: threads BXE x TY, each owning R rows (ty + r*TY) of an extended
// tile BXE x (TY*R). NDIM 2: one row, TY = R = 1, "z" is the second grid
// dimension. EMB (2D only): each level also advances the embedded first-order
// solution of the error estimate, What <- What + Re tau Re f(W) at the same
// point (no neighbours), carried in a register ring beside the level windows
// and written with the last level.
template <int OP, int BC, int NDIM, int BXE, int TY, int R, int K, bool IN_REAL, bool OUT_REAL,
          bool EMB = false>
__device__ __forceinline__ void tb_tile(const TbArgs &a, int bx, int by, int bz, double2 *sLp,
                                        double *sDp)
{
    static_assert(!EMB || (NDIM == 2 && K > 1 && !OUT_REAL), "embedded variant: 2D rows, complex out");
    constexpr int BYE = TY * R;
    constexpr bool SKIP_ROWS = (BXE == 64);         // one extended row per wavefront
    constexpr int SX = BXE + 2;
    constexpr int SY = (NDIM == 3) ? BYE + 2 : 1;
    constexpr int PL = SX * SY;                     // padded plane
    constexpr bool VC = (OP == VAR);
    // 2D rows are small: where LDS allows, their level planes are
    // double-buffered by step parity, so one barrier per step suffices; 3D
    // tiles keep one buffer and separate reads from writes with a second
    // barrier.
    constexpr bool DB = (NDIM == 2) &&
                        (2 * K * PL * 16 + (VC ? (K + 2) * PL * 8 : 0) <= 160 * 1024);
    constexpr int NB = DB ? 2 : 1;
    constexpr int ND = DB ? K + 2 : K + 1;          // D ring: planes t-K-1 .. t-1 (and t)
    constexpr int BXO = BXE - 2 * K;                // output tile
    constexpr int BYO = (NDIM == 3) ? BYE - 2 * K : 1;
    static_assert(BXO > 0 && BYO > 0, "tile too small for K");
    // level m plane (m = 0..K-1) by buffer; D ring
    double2 (*sL)[K][PL] = reinterpret_cast<double2 (*)[K][PL]>(sLp);
    double (*sD)[VC ? PL : 1] = reinterpret_cast<double (*)[VC ? PL : 1]>(sDp);

    const Dims dm{a.nx, a.ny, a.nz};
    const int tid = threadIdx.x;
    const int tx = tid % BXE, ty = tid / BXE;
    const int xe0 = bx * BXO - K;
    const int ye0 = (NDIM == 3) ? by * BYO - K : 0;
    const int x = xe0 + tx;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const bool dir = (BC == DIR);
    const bool x_in = x >= 0 && x < a.nx;
    const bool x_out = tx >= K && tx < BXE - K && x < a.nx;

    int yr[R], slot[R];
    bool col_ghost[R], out_col[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int ly = ty + r * TY;                 // row inside the extended tile
        yr[r] = ye0 + ly;
        slot[r] = (NDIM == 3 ? (ly + 1) * SX : 0) + tx + 1;
        const bool y_in = (NDIM == 3) ? (yr[r] >= 0 && yr[r] < a.ny) : true;
        col_ghost[r] = dir && !(x_in && y_in);      // Dirichlet ghost column: all levels 0
        const bool y_out = (NDIM == 3) ? (ly >= K && ly < BYE - K && yr[r] < a.ny) : true;
        out_col[r] = x_out && y_out;
    }
    auto LW = [&](int gy, int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, x, gy, gz, g);
        return IN_REAL ? make_double2(a.in_re[i], 0.0) : a.in_c[i];
    };
    auto LE = [&](int gy, int gz) {   // embedded solution in (EMB with complex input)
        bool g;
        const long long i = bc_index_nb<BC>(dm, x, gy, gz, g);
        return (EMB && !IN_REAL) ? a.emb_in[i] : 0.0;
    };
    auto LD = [&](int gy, int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, x, gy, gz, g);
        return VC ? 0.5 * a.D[i] : 0.0;   // D/2, as the face rule takes it
    };
    auto pout = [&](int p) { return dir && (p < 0 || p >= a.nz); };
    auto dslot = [](int p) { return ((p % ND) + ND) % ND; };

    // Level 0 ring: plane p in slot (p - t_begin) % NR, its D alongside. At
    // time step t planes t-2, t-1, t are in use and t+1 .. t+PF in flight.
    // Register windows of levels 1..K-1: planes (q-1, q, q+1) around the
    // plane that the next level computes.
    constexpr int PF = 2;
    constexpr int NR = PF + 3;
    const int t_begin = z0 - K, t_end = z1 + K;     // level 0 planes z0-K .. z1+K-1
    double2 L0[NR][R];
    double D0[NR][R];
    double2 wm[K > 1 ? K - 1 : 1][R], wc[K > 1 ? K - 1 : 1][R], wp[K > 1 ? K - 1 : 1][R];
    // 2D rows compute every level on every lane, so their level windows can
    // live in a ring indexed by the unrolled step (slot of step t = plane t-m
    // of level m) instead of being shifted through registers every step; 3D
    // tiles skip levels per row and keep the shifting windows.
    constexpr bool RING = (NDIM == 2) && (K > 1);
    double2 WR[RING ? K - 1 : 1][RING ? NR : 1][R];
    // EMB: embedded solution of level 0 (read beside W; the real input itself
    // on a first pass) and of levels 1..K-1, in the same ring slots
    constexpr bool ER0 = EMB && !IN_REAL;
    double E0[ER0 ? NR : 1][R];
    double ER[EMB ? K - 1 : 1][EMB ? NR : 1][R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gy = (NDIM == 3) ? yr[r] : 0;
#pragma unroll
        for (int q = 0; q < NR; ++q) {
            L0[q][r] = make_double2(0.0, 0.0);
            D0[q][r] = 0.0;
            if (ER0) E0[q][r] = 0.0;
            if (EMB) {
#pragma unroll
                for (int m = 0; m + 1 < K; ++m) ER[m][q][r] = 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int tq = min(t_begin + q, t_end - 1);
            L0[q][r] = LW(gy, tq);
            D0[q][r] = LD(gy, tq);
            if (ER0) E0[q][r] = LE(gy, tq);
        }
#pragma unroll
        for (int m = 0; m + 1 < K; ++m) wm[m][r] = wc[m][r] = wp[m][r] = make_double2(0.0, 0.0);
        if (RING) {
#pragma unroll
            for (int m = 0; m + 1 < K; ++m)
#pragma unroll
                for (int q = 0; q < NR; ++q) WR[m][q][r] = make_double2(0.0, 0.0);
        }
    }

    for (int tb = t_begin; tb < t_end; tb += NR) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int t = tb + u;
        if (t >= t_end) break;
        // slot of plane t + d
        auto rs = [u](int d) { return (u + d + 2 * NR) % NR; };
        // prefetch plane t+PF into the slot of plane t-3
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int gy = (NDIM == 3) ? yr[r] : 0;
            const int tn = min(t + PF, t_end - 1);  // nothing past the last plane is used
            L0[rs(PF)][r] = LW(gy, tn);
            D0[rs(PF)][r] = LD(gy, tn);
            if (ER0) E0[rs(PF)][r] = LE(gy, tn);
        }
        // plane t of level 0 is consumed from here on: zero its Dirichlet
        // ghosts once, in its ring slot
#pragma unroll
        for (int r = 0; r < R; ++r) L0[rs(0)][r] = keep(L0[rs(0)][r], col_ghost[r] || pout(t));
        const int rb = DB ? ((t - 1) & 1) : 0, wb = DB ? (t & 1) : 0;
        // levels 1..K at planes t-1 .. t-K
#pragma unroll
        for (int m = 1; m <= K; ++m) {
            const int p = t - m;
            const double2 *L = sL[rb][m - 1];
            const double *Dc_ = VC ? sD[dslot(p)] : nullptr;
            const double *Dm_ = VC ? sD[dslot(p - 1)] : nullptr;
            const double *Dp_ = VC ? sD[dslot(p + 1)] : nullptr;
            const bool pghost = pout(p);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                // Level m is only used within m cells of the output rows; in
                // 3D a row of 64 columns is one wavefront, so rows outside
                // that band skip the level as a whole.
                if (NDIM == 3 && SKIP_ROWS) {
                    const int ly = ty + r * TY;
                    if (ly < m || ly >= BYE - m) continue;
                }
                const int sl = slot[r];
                double2 c, zm, zp;
                if (m == 1) {
                    // level 0 from the ring: planes t-2, t-1, t
                    zm = L0[rs(-2)][r];
                    c = L0[rs(-1)][r];
                    zp = L0[rs(0)][r];
                } else {
                    if (RING) {
                        zm = WR[(m - 2) % (K - 1)][rs(-2)][r];
                        c = WR[(m - 2) % (K - 1)][rs(-1)][r];
                        zp = WR[(m - 2) % (K - 1)][rs(0)][r];
                    } else {
                        zm = wm[m - 2][r];
                        c = wc[m - 2][r];
                        zp = wp[m - 2][r];
                    }
                }
                double dc = 0.0, dzm = 0.0, dzp = 0.0;
                if (VC) {
                    dc = Dc_[sl];
                    dzm = Dm_[sl];
                    dzp = (m == 1) ? D0[rs(0)][r] : Dp_[sl];   // plane t is not in LDS yet
                }
                double qr_c = 0.0, qi_c = 0.0;
                if (OP == POR) {
                    csqh(c, qr_c, qi_c);
                }
                double acc_r = 0.0, acc_i = 0.0;
                // A Dirichlet ghost holds W = 0 and the D of the boundary cell
                // it faces (loads are clamped), so every face takes the plain
                // mean, which there equals D_c bit for bit.
                face<OP>(acc_r, acc_i, c, L[sl - 1], dc, VC ? Dc_[sl - 1] : 0.0, false, qr_c,
                         qi_c, a.fc[0]);
                face<OP>(acc_r, acc_i, c, L[sl + 1], dc, VC ? Dc_[sl + 1] : 0.0, false, qr_c,
                         qi_c, a.fc[1]);
                if (NDIM == 3) {
                    face<OP>(acc_r, acc_i, c, L[sl - SX], dc, VC ? Dc_[sl - SX] : 0.0, false,
                             qr_c, qi_c, a.fc[2]);
                    face<OP>(acc_r, acc_i, c, L[sl + SX], dc, VC ? Dc_[sl + SX] : 0.0, false,
                             qr_c, qi_c, a.fc[3]);
                }
                face<OP>(acc_r, acc_i, c, zm, dc, dzm, false, qr_c, qi_c, a.fc[4]);
                face<OP>(acc_r, acc_i, c, zp, dc, dzp, false, qr_c, qi_c, a.fc[5]);
                double2 v = euler(c, acc_r, acc_i, a.inv_h2, a.tr[m - 1], a.ti[m - 1]);
                v = keep(v, col_ghost[r] || pghost);
                double eh = 0.0;
                if (EMB) {
                    // level m-1's embedded value at this point: plane t-m
                    const double base = (m == 1) ? (IN_REAL ? c.x : E0[ER0 ? rs(-1) : 0][r])
                                                 : ER[(m - 2) % (K - 1)][rs(-1)][r];
                    eh = fma(a.tr[m - 1], acc_r * a.inv_h2, base);
                }
                if (m < K) {
                    if (EMB) ER[(m - 1) % (K - 1)][rs(0)][r] = eh;
                    if (RING) {
                        WR[(m - 1) % (K - 1)][rs(0)][r] = v;
                    } else {
                        wm[m - 1][r] = wc[m - 1][r];
                        wc[m - 1][r] = wp[m - 1][r];
                        wp[m - 1][r] = v;
                    }
                } else if (out_col[r] && p >= z0 && p < z1) {
                    const int gy = (NDIM == 3) ? yr[r] : 0;
                    const long long i = x + (long long)a.nx * (gy + (long long)a.ny * p);
                    if (OUT_REAL) a.out_re[i] = v.x;
                    else a.out_c[i] = v;
                    if (EMB) a.emb_out[i] = eh;
                }
            }
        }
        if (!DB) __syncthreads();   // every read of the LDS planes of this step is done
#pragma unroll
        for (int r = 0; r < R; ++r) {
            sL[wb][0][slot[r]] = L0[rs(0)][r];
#pragma unroll
            for (int m = 1; m < K; ++m)
                sL[wb][m][slot[r]] = RING ? WR[(m - 1) % (K - 1)][rs(0)][r] : wp[m - 1][r];
            if (VC) sD[dslot(t)][slot[r]] = D0[rs(0)][r];
        }
        __syncthreads();   // the planes of step t are visible to step t+1
    }
    }
}

}  // namespace dev
}  // namespace frkc2
