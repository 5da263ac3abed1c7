// One tile of the full-width temporally blocked 3D stage kernel, shared by
// tb3d_stage and the batched pass kernels. See tb3d.hip for the design.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace dev {

struct Tb3Args {
    const double *in_re;
    const double2 *in_c;
    double *out_re;
    double2 *out_c;
    const double *D;
    const double *emb_in;       // embedded first-order solution (EMB; first pass: real input)
    double *emb_out;
    int nx, ny, nz;
    int zchunk, ntx, nty;
    double inv_h2, d_const;
    double tr[kMaxTBlock], ti[kMaxTBlock];
    double fc[6];               // face coefficients x-, x+, y-, y+, z-, z+ (LAPLACE, ADVDIFF)
};

// Rows of the extended tile (one wavefront each) and halo wavefronts for
// 1024 threads: 2K halo columns per row must fit in the halo wavefronts.
template <int K>
struct Tb3Shape {
    static constexpr int NHW = (K == 2) ? 1 : 2;
    static constexpr int BYE = 16 - NHW;
    static constexpr int BXE = 64 + 2 * K;
    static constexpr int BYO = BYE - 2 * K;
    static_assert(2 * K * BYE <= 64 * NHW, "halo columns must fit the halo wavefronts");
    // Role of wavefront w (rows 0..BYE-1, then the halo wavefronts). The
    // wavefronts of a workgroup are dealt to the CU's four SIMDs in turn
    // (w % 4), and a row computes min(row, BYE-1-row, K) levels, so the roles
    // are permuted to give every SIMD the same work before the barrier: for
    // K = 3 each SIMD gets 8 row-levels (rows 3 4 2 0 | 5 6 11 13 | 7 8 A B |
    // 9 10 1 12) instead of 7 to 10 in natural order; for K = 2 the natural
    // order is already balanced (6 6 6 7).
    static __device__ __forceinline__ int role(int w)
    {
        if (K != 3) return w;
        constexpr int perm[16] = {3, 5, 7, 9, 4, 6, 8, 10, 2, 11, 14, 1, 0, 13, 15, 12};
        return perm[w];
    }
};

__device__ __forceinline__ double2 keep3(double2 v, bool ghost)
{
    v.x = ghost ? 0.0 : v.x;
    v.y = ghost ? 0.0 : v.y;
    return v;
}

// LDS of one tile: level planes (double2) and the diffusivity ring (double).
template <int OP, int K>
struct Tb3Lds {
    static constexpr int PL = (Tb3Shape<K>::BXE + 2) * (Tb3Shape<K>::BYE + 2);
    static constexpr int L = 2 * K * PL;
    static constexpr int D = (OP == FRKC2_OP_VARCOEF) ? (K + 2) * PL : 1;
};

// EMB: also advance the embedded first-order solution of the error estimate
// (Sec. 3): What^m = fma(tr_m, Re f(W^{m-1}), What^{m-1}) at every level, a
// pointwise recursion carried in registers next to the level windows.
template <int OP, int BC, int K, bool IN_REAL, bool OUT_REAL, bool EMB = false>
__device__ __forceinline__ void tb3d_tile(const Tb3Args &a, int bx, int by, int bz, double2 *sLp,
                                          double *sDp)
{
    using S = Tb3Shape<K>;
    constexpr int BXE = S::BXE, BYE = S::BYE, BYO = S::BYO;
    constexpr int SX = BXE + 2, SY = BYE + 2;      // one padding cell around each plane
    constexpr int PL = SX * SY;
    constexpr bool VC = (OP == VAR);
    constexpr int ND = K + 2;                       // D ring: planes t-K-1 .. t
    // level m plane, by step parity; D ring
    double2 (*sL)[K][PL] = reinterpret_cast<double2 (*)[K][PL]>(sLp);
    double (*sD)[VC ? PL : 1] = reinterpret_cast<double (*)[VC ? PL : 1]>(sDp);

    const Dims dm{a.nx, a.ny, a.nz};
    const int tid = threadIdx.x;
    const int wv = S::role(tid >> 6), lane = tid & 63;
    int lx, ly;                                     // position in the extended tile
    if (wv < BYE) {
        lx = K + lane;
        ly = wv;
    } else {
        // halo lane: depth d = 1..K from the output columns, side, row;
        // spare lanes repeat depth-K lanes (same values, never used)
        int j = (wv - BYE) * 64 + lane;
        if (j >= 2 * K * BYE) j = 2 * (K - 1) * BYE + (j % (2 * BYE));
        const int d = 1 + j / (2 * BYE);
        const int rem = j % (2 * BYE);
        ly = rem % BYE;
        lx = (rem < BYE) ? K - d : K + 63 + d;
    }
    // level m is needed where the tile edge is at least m cells away
    const int need = min(min(lx, BXE - 1 - lx), min(ly, BYE - 1 - ly));

    const int x = bx * 64 - K + lx;
    const int y = by * BYO - K + ly;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const bool dir = (BC == DIR);
    const bool col_ghost = dir && !(x >= 0 && x < a.nx && y >= 0 && y < a.ny);
    const bool out_col = lx >= K && lx < K + 64 && ly >= K && ly < BYE - K && x < a.nx &&
                         y < a.ny;
    const int slot = (ly + 1) * SX + lx + 1;

    auto LW = [&](int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, x, y, gz, g);
        return IN_REAL ? make_double2(a.in_re[i], 0.0) : a.in_c[i];
    };
    auto LD = [&](int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, x, y, gz, g);
        return VC ? a.D[i] : 0.0;
    };
    auto LE = [&](int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, x, y, gz, g);
        return (EMB && !IN_REAL) ? a.emb_in[i] : 0.0;
    };
    auto pout = [&](int p) { return dir && (p < 0 || p >= a.nz); };
    auto dslot = [](int p) { return ((p % ND) + ND) % ND; };

    // Level 0 ring: plane p in slot (p - t_begin) % NR with its D; at step t
    // planes t-2 .. t are in use and t+1, t+2 in flight. Windows of levels
    // 1..K-1: planes (q-1, q, q+1) around the plane the next level computes.
    constexpr int PF = 2;
    constexpr int NR = PF + 3;
    const int t_begin = z0 - K, t_end = z1 + K;     // level 0 planes z0-K .. z1+K-1
    double2 L0[NR];
    double D0[NR];
    constexpr bool ER = EMB && !IN_REAL;            // embedded input read from memory
    double E0[ER ? NR : 1];
    double ehc[K - 1], ehn[K - 1];                  // What of levels 1..K-1: last step, this step
    double2 wm[K - 1], wc[K - 1], wp[K - 1];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        L0[q] = make_double2(0.0, 0.0);
        D0[q] = 0.0;
        if (ER) E0[q] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int tq = min(t_begin + q, t_end - 1);
        L0[q] = LW(tq);
        D0[q] = LD(tq);
        if (ER) E0[q] = LE(tq);
    }
#pragma unroll
    for (int m = 0; m + 1 < K; ++m) ehc[m] = ehn[m] = 0.0;
#pragma unroll
    for (int m = 0; m + 1 < K; ++m) wm[m] = wc[m] = wp[m] = make_double2(0.0, 0.0);

    for (int tb = t_begin; tb < t_end; tb += NR) {
#pragma unroll
    for (int u = 0; u < NR; ++u) {
        const int t = tb + u;
        if (t >= t_end) break;
        auto rs = [u](int d) { return (u + d + 2 * NR) % NR; };   // slot of plane t + d
        {
            const int tn = min(t + PF, t_end - 1);  // nothing past the last plane is used
            L0[rs(PF)] = LW(tn);
            D0[rs(PF)] = LD(tn);
            if (ER) E0[rs(PF)] = LE(tn);
        }
        L0[rs(0)] = keep3(L0[rs(0)], col_ghost || pout(t));
        const int rb = (t - 1) & 1, wb = t & 1;     // LDS buffers read / written at step t
        // LDS operands of level m: x/y neighbours of level m-1 and their D,
        // and the cell's own D where the register ring no longer holds it.
        // Level m+1's operands are read before level m is computed, by every
        // lane (all slots are in range), so their latency overlaps the work.
        struct Nb {
            double2 w[4];
            double d[4], dc, dzm, dzp;
        };
        auto read = [&](int m) {
            Nb n;
            const int p = t - m;
            const double2 *L = sL[rb][m - 1];
            n.w[0] = L[slot - 1];
            n.w[1] = L[slot + 1];
            n.w[2] = L[slot - SX];
            n.w[3] = L[slot + SX];
            n.dc = n.dzm = n.dzp = 0.0;
            n.d[0] = n.d[1] = n.d[2] = n.d[3] = 0.0;
            if (VC) {
                const double *Dp = sD[dslot(p)];
                n.d[0] = Dp[slot - 1];
                n.d[1] = Dp[slot + 1];
                n.d[2] = Dp[slot - SX];
                n.d[3] = Dp[slot + SX];
                if (m == 1) {
                    n.dzm = D0[rs(-2)];
                    n.dc = D0[rs(-1)];
                    n.dzp = D0[rs(0)];
                } else {
                    n.dc = (m == 2) ? D0[rs(-2)] : Dp[slot];
                    n.dzm = sD[dslot(p - 1)][slot];
                    n.dzp = (m == 2) ? D0[rs(-1)] : (m == 3 ? D0[rs(-2)] : sD[dslot(p + 1)][slot]);
                }
            }
            return n;
        };
        // (For K = 3, or with the embedded solution, the operands of two levels
        // do not fit the registers of four wavefronts per SIMD: there each
        // level reads its own.)
        constexpr bool RA = (K <= 2) && !EMB;
        Nb cur = read(1);
#pragma unroll
        for (int m = 1; m <= K; ++m) {
            Nb nxt = cur;
            if (RA && m < K) nxt = read(m + 1);
            if (need >= m) {
                const int p = t - m;
                double2 c, zm, zp;
                if (m == 1) {
                    zm = L0[rs(-2)];
                    c = L0[rs(-1)];
                    zp = L0[rs(0)];
                } else {
                    zm = wm[m - 2];
                    c = wc[m - 2];
                    zp = wp[m - 2];
                }
                double qr_c = 0.0, qi_c = 0.0;
                if (OP == POR) {
                    csq(c, qr_c, qi_c);
                }
                // A Dirichlet ghost holds W = 0 and the D of the boundary cell
                // it faces (loads are clamped), so every face takes the plain
                // mean, which there equals D_c bit for bit.
                const double dc = cur.dc;
                double acc_r = 0.0, acc_i = 0.0;
                face<OP>(acc_r, acc_i, c, cur.w[0], dc, cur.d[0], false, qr_c, qi_c, a.fc[0]);
                face<OP>(acc_r, acc_i, c, cur.w[1], dc, cur.d[1], false, qr_c, qi_c, a.fc[1]);
                face<OP>(acc_r, acc_i, c, cur.w[2], dc, cur.d[2], false, qr_c, qi_c, a.fc[2]);
                face<OP>(acc_r, acc_i, c, cur.w[3], dc, cur.d[3], false, qr_c, qi_c, a.fc[3]);
                face<OP>(acc_r, acc_i, c, zm, dc, cur.dzm, false, qr_c, qi_c, a.fc[4]);
                face<OP>(acc_r, acc_i, c, zp, dc, cur.dzp, false, qr_c, qi_c, a.fc[5]);
                double2 v = euler(c, acc_r, acc_i, a.inv_h2, a.tr[m - 1], a.ti[m - 1]);
                v = keep3(v, col_ghost || pout(p));
                double eh = 0.0;
                if (EMB) {
                    // What^{m-1} at plane p: the input (level 1) or last step's level m-1
                    const double base =
                        (m == 1) ? (IN_REAL ? c.x : E0[ER ? rs(-1) : 0]) : ehc[m - 2];
                    eh = fma(a.tr[m - 1], acc_r * a.inv_h2, base);
                }
                if (m < K) {
                    wm[m - 1] = wc[m - 1];
                    wc[m - 1] = wp[m - 1];
                    wp[m - 1] = v;
                    if (EMB) ehn[m - 1] = eh;
                } else if (out_col && p >= z0 && p < z1) {
                    const long long i = x + (long long)a.nx * (y + (long long)a.ny * p);
                    if (OUT_REAL) a.out_re[i] = v.x;
                    else a.out_c[i] = v;
                    if (EMB) a.emb_out[i] = eh;
                }
            }
            if (!RA && m < K) nxt = read(m + 1);
            cur = nxt;
        }
        // All LDS writes of the step come after all its reads, so the reads
        // of every level can be issued early. A lane that skipped level m
        // stores a stale value that no needed cell reads.
        sL[wb][0][slot] = L0[rs(0)];
#pragma unroll
        for (int m = 1; m < K; ++m) sL[wb][m][slot] = wp[m - 1];
        if (EMB) {
#pragma unroll
            for (int m = 0; m + 1 < K; ++m) ehc[m] = ehn[m];
        }
        if (VC) sD[dslot(t)][slot] = D0[rs(0)];
        __syncthreads();   // step t's planes are visible to step t+1, whose
                           // writes go to the other buffer
    }
    }
}

}  // namespace dev
}  // namespace frkc2
