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
    double2 *lvl_out;           // ST: level m (1..K-1) written to lvl_out + (m-1)*lvl_stride
    long long lvl_stride;
};

// Extended tile of W output columns (64: one row per wavefront; 32: two
// rows per wavefront, lanes 0-31 and 32-63) plus K halo columns on each side,
// which the halo wavefronts compute: 2K halo columns per row must fit in them.
// 1024 threads either way.
template <int K, int W = 64>
struct Tb3Shape {
    static_assert(W == 64 || W == 32, "64 or 32 output columns");
    static constexpr int RPW = 64 / W;                           // rows per row wavefront
    static constexpr int NHW = (W == 64) ? (K == 2 ? 1 : 2) : (K == 2 ? 2 : 3);
    static constexpr int NRW = 16 - NHW;                         // row wavefronts
    static constexpr int BYE = NRW * RPW;
    static constexpr int BXE = W + 2 * K;
    static constexpr int BYO = BYE - 2 * K;
    static_assert(2 * K * BYE <= 64 * NHW, "halo columns must fit the halo wavefronts");
    // LDS row stride in cells: at least one padding cell on each side, made
    // odd so that the halo wavefronts, whose consecutive lanes walk down a
    // column, hit distinct banks (an even stride of 72 cells put 16-byte
    // accesses of a 16-lane group on two bank groups only).
    static constexpr int SX = (BXE + 2) | 1;
    static constexpr int SY = BYE + 2;
    // Role of wavefront w (row wavefronts first, then the halo wavefronts).
    // The wavefronts of a workgroup are dealt to the CU's four SIMDs in turn
    // (w % 4), and a wavefront computes as many levels as its most central
    // cell needs, so the roles are permuted to even out the levels per SIMD
    // before each barrier: 8 8 8 8 (W = 64, K = 3; 7 to 10 in natural order)
    // and 10 10 9 9 (W = 32, K = 3; 8 to 11); the other shapes are balanced
    // in natural order.
    static __device__ __forceinline__ int role(int w)
    {
        if (K == 3 && W == 64) {
            constexpr int perm[16] = {3, 5, 7, 9, 4, 6, 8, 10, 2, 11, 14, 1, 0, 13, 15, 12};
            return perm[w];
        }
        if (K == 3 && W == 32) {
            constexpr int perm[16] = {1, 2, 3, 0, 5, 6, 7, 4, 9, 10, 11, 8, 12, 14, 15, 13};
            return perm[w];
        }
        return w;
    }
    // The largest per-SIMD level count above: the work of one time step
    static constexpr int STEP_COST = (K == 3) ? (W == 64 ? 8 : 10) : 7;
};

// LDS of one tile: level planes (double2), double-buffered by step parity,
// and for the diffusion operator D/2 (double): one plane double-buffered
// where the faces live in registers, a ring of K + 2 planes where the
// levels read their D neighbours themselves (DRING).
template <int OP, int K, int W = 64, bool DRING = false>
struct Tb3Lds {
    static constexpr int PL = Tb3Shape<K, W>::SX * Tb3Shape<K, W>::SY;
    static constexpr int L = 2 * K * PL;
    static constexpr int D = (OP == FRKC2_OP_VARCOEF) ? (DRING ? K + 2 : 2) * PL : 1;
};

// EMB: also advance the embedded first-order solution of the error estimate
// (Sec. 3): What^m = fma(tr_m, Re f(W^{m-1}), What^{m-1}) at every level, a
// pointwise recursion carried in registers next to the level windows.
// ST: also write the intermediate levels 1..K-1 of the output columns (the
// stage states the adjoint's reverse sweep reads).
// FACES: the diffusion operator's faces from a register ring (below); off
// where the registers are taken (the embedded solution; the batch's kernels,
// which hold the code of two operators), with the D ring of Tb3Lds<..., true>.
// BUF: global accesses through buffer resources (below); off in the batch's
// kernels, which address through 64-bit lane pointers.
// REV: march the chunk from its top plane down (with the face ring only).
// Every point takes the same operands in the same order, so the results are
// the same bits; consecutive passes that alternate the direction start on
// the planes the previous pass touched last, which the last-level cache
// (256 MB) still holds.
template <int OP, int BC, int K, bool IN_REAL, bool OUT_REAL, bool EMB = false, bool ST = false,
          int W = 64, bool FACES = !EMB, bool BUF = true, bool REV = false>
__device__ __forceinline__ void tb3d_tile(const Tb3Args &a, int bx, int by, int bz, double2 *sLp,
                                          double *sDp)
{
    using S = Tb3Shape<K, W>;
    constexpr int BXE = S::BXE, BYE = S::BYE, BYO = S::BYO;
    constexpr int SX = S::SX;                       // padding cells around each plane
    constexpr int PL = Tb3Lds<OP, K, W>::PL;
    constexpr bool VC = (OP == VAR);
    // Diffusivity faces D_f = D_c/2 + D_nb/2: from a register ring (FR), or
    // per level from D/2 planes in LDS (DR)
    constexpr bool FR = VC && FACES, DR = VC && !FACES;
    static_assert(!REV || (FACES && !EMB && !ST), "the reversed march: face ring, plain passes");
    constexpr int ND = DR ? K + 2 : 2;              // D/2 planes in LDS
    // level m plane by step parity; D/2 planes
    double2 (*sL)[K][PL] = reinterpret_cast<double2 (*)[K][PL]>(sLp);
    double (*sD)[VC ? PL : 1] = reinterpret_cast<double (*)[VC ? PL : 1]>(sDp);

    const int tid = threadIdx.x;
    const int wv = S::role(tid >> 6), lane = tid & 63;
    int lx, ly;                                     // position in the extended tile
    if (wv < S::NRW) {
        lx = K + lane % W;
        ly = wv * S::RPW + lane / W;
    } else {
        // halo lane: depth d = 1..K from the output columns, side, row;
        // spare lanes repeat depth-K lanes (same values, never used)
        int j = (wv - S::NRW) * 64 + lane;
        if (j >= 2 * K * BYE) j = 2 * (K - 1) * BYE + (j % (2 * BYE));
        const int d = 1 + j / (2 * BYE);
        const int rem = j % (2 * BYE);
        ly = rem % BYE;
        lx = (rem < BYE) ? K - d : K + W - 1 + d;
    }
    const int x = bx * W - K + lx;
    const int y = by * BYO - K + ly;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const bool dir = (BC == DIR);
    const bool col_ghost = dir && !(x >= 0 && x < a.nx && y >= 0 && y < a.ny);
    // Level m is needed where the tile edge is at least m cells away. A
    // wavefront computes every level one of its lanes needs, on all lanes, so
    // each level's registers are rewritten every step; a lane that does not
    // need the level computes a value nobody reads. A Dirichlet ghost column
    // never writes LDS, whose planes start at 0, the ghost value its
    // neighbours read.
    const int need = min(min(lx, BXE - 1 - lx), min(ly, BYE - 1 - ly));
    int wneed = 0;
#pragma unroll
    for (int m = 1; m <= K; ++m)
        if (__any(need >= m)) wneed = m;
    wneed = __builtin_amdgcn_readfirstlane(wneed);
    const bool out_col = lx >= K && lx < K + W && ly >= K && ly < BYE - K && x < a.nx &&
                         y < a.ny;
    const int slot = (ly + 1) * SX + lx + 1;

    // Global accesses: buffer loads and stores whose resource (scalar
    // registers) starts at the plane and spans its bytes, plus the lane's
    // column offset in bytes (clamped into the grid for Dirichlet, wrapped for
    // periodic) in one 32-bit vector register, so no lane holds a 64-bit
    // pointer. The host sends planes of 2^27 points or more elsewhere, so
    // every offset and extent fits 31 bits.
    // (Without BUF: a 64-bit pointer per lane to its column plus a uniform
    // plane offset.)
    const int cx = (BC == PER) ? wrap(x, a.nx) : min(max(x, 0), a.nx - 1);
    const int cy = (BC == PER) ? wrap(y, a.ny) : min(max(y, 0), a.ny - 1);
    const unsigned oxy = (unsigned)cx + (unsigned)a.nx * (unsigned)cy;
    const unsigned o8 = 8u * oxy, o16 = 16u * oxy;
    const long long pst = (long long)a.nx * a.ny;
    const int pb8 = (int)(8 * pst), pb16 = (int)(16 * pst);   // plane extents in bytes
    // The march runs over q = z0-K .. z1+K-1 (planes below, in and above the
    // chunk); plane(q) is the plane it stands for: q itself, or its mirror in
    // the chunk with REV.
    auto plane = [&](int q) { return REV ? z0 + z1 - 1 - q : q; };
    auto zoff = [&](int q) {
        const int gz = plane(q);
        return pst * ((BC == PER) ? wrap(gz, a.nz) : min(max(gz, 0), a.nz - 1));
    };
    const double2 *pWc = (BUF || IN_REAL) ? nullptr : a.in_c + oxy;
    const double *pWr = (BUF || !IN_REAL) ? nullptr : a.in_re + oxy;
    const double *pD = (BUF || !VC) ? nullptr : a.D + oxy;
    const double *pE = (BUF || !(EMB && !IN_REAL)) ? nullptr : a.emb_in + oxy;
    auto LW = [&](int gz) {
        if constexpr (!BUF) return IN_REAL ? make_double2(pWr[zoff(gz)], 0.0) : pWc[zoff(gz)];
        if (IN_REAL) {
            const double v = buf_load_f64(a.in_re + zoff(gz), pb8, o8);
            return make_double2(v, 0.0);
        }
        return buf_load_c(a.in_c + zoff(gz), pb16, o16);
    };
    // D as loaded: with the face ring it is halved (the face rule takes D/2)
    // when its plane enters use, so the multiply never waits on a load still
    // in flight; with the per-level reads (HL) as it is loaded
    constexpr bool HL = !FACES;
    auto LD = [&](int gz) {
        if constexpr (!VC) return 0.0;
        const double d = BUF ? buf_load_f64(a.D + zoff(gz), pb8, o8) : pD[zoff(gz)];
        return HL ? 0.5 * d : d;
    };
    auto LE = [&](int gz) {
        if constexpr (!(EMB && !IN_REAL)) return 0.0;
        return BUF ? buf_load_f64(a.emb_in + zoff(gz), pb8, o8) : pE[zoff(gz)];
    };
    auto pout = [&](int q) {
        const int p = plane(q);
        return dir && (p < 0 || p >= a.nz);
    };

    // Level 0 ring: plane p in slot (p - t_begin) % NR with its D; at step t
    // planes t-2 .. t are in use and the next PF planes in flight. Windows of levels
    // 1..K-1: planes (q-1, q, q+1) around the plane the next level computes.
    // Planes loaded ahead: one for the diffusion operator, whose face ring
    // takes the registers (two measured no faster where they fit), and with
    // the embedded solution (its rings)
    constexpr int PF = (EMB || (VC && FACES)) ? 1 : 2;
    constexpr int NR = PF + 3;
    static_assert(K < NR, "the face rings hold K + 1 planes");
    // Steps z0-K .. z0-1 only fill the levels below the chunk. At a Dirichlet
    // lower end those planes are ghosts, 0 at every level, which the rings
    // and LDS hold from the start: the march begins at plane 0, with the
    // ghost plane's D in place (below).
    const bool lead_ghost = dir && (REV ? z1 == a.nz : z0 == 0);
    const int t_begin = lead_ghost ? z0 : z0 - K, t_end = z1 + K;   // level 0 planes
    double2 L0[NR];
    double D0[NR];
    constexpr bool ER = EMB && !IN_REAL;            // embedded input read from memory
    double E0[ER ? NR : 1];
    double ehc[K - 1], ehn[K - 1];                  // What of levels 1..K-1: last step, this step
    // Levels 1..K-1 by step: WR[m-1][slot of step t] holds level m at plane
    // t-m; the window of level m+1 at step t is the slots of steps t-2..t.
    // The step loop is unrolled by NR, so every index is static.
    double2 WR[K - 1][NR];
    // FR: the faces, the operand of every face term, formed once per plane
    // instead of once per level. At step t the lane forms the four x/y faces
    // of plane t-1 from the neighbours' D/2 in LDS, and the z face between
    // planes t-1 and t, into the slot of step t; level m (plane t-m) then
    // finds its x/y faces in the slot of step t-m+1, its z- face in the slot
    // of step t-m and its z+ face in the slot of step t-m+1. The sums are the
    // ones the per-level form computes, so every result keeps its bits.
    double FX[FR ? NR : 1][4];
    double FZ[FR ? NR : 1];
    double dhp = 0.0;                               // D/2 of plane t-1
    // DR: D/2 of planes t-2 .. t in registers (the D ring, halved as loaded),
    // older planes in the LDS ring
    static_assert(!DR || HL, "the per-level reads take D/2 from the load ring");
    double (&DH)[NR] = D0;
    auto dslot = [](int p) { return ((p % ND) + ND) % ND; };
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        L0[q] = make_double2(0.0, 0.0);
        D0[q] = 0.0;
        if (ER) E0[q] = 0.0;
        if constexpr (FR) {
            FX[q][0] = FX[q][1] = FX[q][2] = FX[q][3] = 0.0;
            FZ[q] = 0.0;
        }
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
    for (int m = 0; m + 1 < K; ++m) {
#pragma unroll
        for (int q = 0; q < NR; ++q) WR[m][q] = make_double2(0.0, 0.0);
    }

    if (dir) {
        for (int i = tid; i < 2 * K * PL; i += 1024) sLp[i] = make_double2(0.0, 0.0);
        if (VC && lead_ghost) {
            // the ghost planes (clamped loads: plane 0's D) as the steps
            // before plane 0 leave them, in registers and in LDS
            if constexpr (FR) {
                dhp = 0.5 * LD(t_begin - 1);
                sD[(t_begin - 1) & 1][slot] = dhp;
            } else {
                DH[NR - 1] = LD(-1);
                DH[NR - 2] = LD(-2);
                sD[dslot(-1)][slot] = DH[NR - 1];
            }
        }
        __syncthreads();
    }

    // A plane outside the grid (Dirichlet) holds the ghost value 0 at every
    // level. The test is uniform and true only near the ends of the grid;
    // the empty asm keeps it a branch rather than selects on every step.
    auto zero_if = [](bool c, double2 &v) {
        if (c) {
            asm volatile("" ::: "memory");
            v = make_double2(0.0, 0.0);
        }
    };
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
        // D/2 of plane t, loaded PF steps ago
        const double dht = VC ? (HL ? D0[rs(0)] : 0.5 * D0[rs(0)]) : 0.0;
        zero_if(pout(t), L0[rs(0)]);
        const int rb = (t - 1) & 1, wb = t & 1;     // LDS buffers read / written at step t
        if constexpr (FR) {
            const double *Dp = sD[rb];              // D/2 of plane t-1
            FX[rs(0)][0] = dhp + Dp[slot - 1];
            FX[rs(0)][1] = dhp + Dp[slot + 1];
            FX[rs(0)][2] = dhp + Dp[slot - SX];
            FX[rs(0)][3] = dhp + Dp[slot + SX];
            FZ[rs(0)] = dhp + dht;
        }
        // x/y neighbours of level m-1 at plane t-m, written at step t-1.
        // With RA, level m+1's are read before level m is computed, so their
        // latency overlaps the work.
        struct Nb {
            double2 w[4];
            double d[4], dc, dzm, dzp;              // DR: D/2 of neighbours and cell
        };
        auto readw = [&](int m, Nb &n) {
            const double2 *L = sL[rb][m - 1];
            n.w[0] = L[slot - 1];
            n.w[1] = L[slot + 1];
            n.w[2] = L[slot - SX];
            n.w[3] = L[slot + SX];
            if constexpr (DR) {
                // plane p = t-m: the x/y neighbours from its LDS plane; the
                // cell and its z neighbours from the registers while they hold
                // them (planes t-2 .. t), else from LDS
                const int p = t - m;
                const double *Dp = sD[dslot(p)];
                n.d[0] = Dp[slot - 1];
                n.d[1] = Dp[slot + 1];
                n.d[2] = Dp[slot - SX];
                n.d[3] = Dp[slot + SX];
                if (m == 1) {
                    n.dzm = DH[rs(-2)];
                    n.dc = DH[rs(-1)];
                    n.dzp = DH[rs(0)];
                } else {
                    n.dc = (m == 2) ? DH[rs(-2)] : Dp[slot];
                    n.dzm = sD[dslot(p - 1)][slot];
                    n.dzp = (m == 2) ? DH[rs(-1)] : DH[rs(-2)];
                }
            }
        };
        // (With the embedded solution the operands of two levels do not fit
        // the registers of four wavefronts per SIMD: there each level reads
        // its own.)
        constexpr bool RA = (K <= 2) && !EMB;
        static_assert(K <= 3, "the register D/2 ring covers three levels");
        Nb cur;
        readw(1, cur);
#pragma unroll
        for (int m = 1; m <= K; ++m) {
            Nb nxt = cur;
            if (RA && m < K) readw(m + 1, nxt);
            const int p = t - m;
            if (m > wneed) {
                // keep the slot written every step (the value is never read)
                if (m < K) WR[m - 1][rs(0)] = make_double2(0.0, 0.0);
                if (EMB && m < K) ehn[m - 1] = 0.0;
            } else {
                double2 c, zm, zp;
                if (m == 1) {
                    zm = L0[rs(-2)];
                    c = L0[rs(-1)];
                    zp = L0[rs(0)];
                } else {
                    zm = WR[m - 2][rs(-2)];
                    c = WR[m - 2][rs(-1)];
                    zp = WR[m - 2][rs(0)];
                }
                double qr_c = 0.0, qi_c = 0.0;
                if (OP == POR) {
                    csqh(c, qr_c, qi_c);
                }
                double acc_r = 0.0, acc_i = 0.0;
                // A Dirichlet ghost holds W = 0 and the D of the boundary cell
                // it faces (loads are clamped), so every face takes the plain
                // mean, which there equals D_c bit for bit.
                if constexpr (FR) {
                    const double *fx = FX[rs(1 - m)];
                    face<LAP>(acc_r, acc_i, c, cur.w[0], 0.0, 0.0, false, 0.0, 0.0, fx[0]);
                    face<LAP>(acc_r, acc_i, c, cur.w[1], 0.0, 0.0, false, 0.0, 0.0, fx[1]);
                    face<LAP>(acc_r, acc_i, c, cur.w[2], 0.0, 0.0, false, 0.0, 0.0, fx[2]);
                    face<LAP>(acc_r, acc_i, c, cur.w[3], 0.0, 0.0, false, 0.0, 0.0, fx[3]);
                    // the face toward the lower plane first
                    if (REV) {
                        face<LAP>(acc_r, acc_i, c, zp, 0.0, 0.0, false, 0.0, 0.0, FZ[rs(1 - m)]);
                        face<LAP>(acc_r, acc_i, c, zm, 0.0, 0.0, false, 0.0, 0.0, FZ[rs(-m)]);
                    } else {
                        face<LAP>(acc_r, acc_i, c, zm, 0.0, 0.0, false, 0.0, 0.0, FZ[rs(-m)]);
                        face<LAP>(acc_r, acc_i, c, zp, 0.0, 0.0, false, 0.0, 0.0, FZ[rs(1 - m)]);
                    }
                } else {
                    const double dc = cur.dc;
                    face<OP>(acc_r, acc_i, c, cur.w[0], dc, cur.d[0], false, qr_c, qi_c, a.fc[0]);
                    face<OP>(acc_r, acc_i, c, cur.w[1], dc, cur.d[1], false, qr_c, qi_c, a.fc[1]);
                    face<OP>(acc_r, acc_i, c, cur.w[2], dc, cur.d[2], false, qr_c, qi_c, a.fc[2]);
                    face<OP>(acc_r, acc_i, c, cur.w[3], dc, cur.d[3], false, qr_c, qi_c, a.fc[3]);
                    // the face toward the lower plane first, with its coefficient
                    if (REV) {
                        face<OP>(acc_r, acc_i, c, zp, dc, cur.dzp, false, qr_c, qi_c, a.fc[4]);
                        face<OP>(acc_r, acc_i, c, zm, dc, cur.dzm, false, qr_c, qi_c, a.fc[5]);
                    } else {
                        face<OP>(acc_r, acc_i, c, zm, dc, cur.dzm, false, qr_c, qi_c, a.fc[4]);
                        face<OP>(acc_r, acc_i, c, zp, dc, cur.dzp, false, qr_c, qi_c, a.fc[5]);
                    }
                }
                double2 v = euler(c, acc_r, acc_i, a.inv_h2, a.tr[m - 1], a.ti[m - 1]);
                zero_if(pout(p), v);
                double eh = 0.0;
                if (EMB) {
                    // What^{m-1} at plane p: the input (level 1) or last step's level m-1
                    const double base =
                        (m == 1) ? (IN_REAL ? c.x : E0[ER ? rs(-1) : 0]) : ehc[m - 2];
                    eh = fma(a.tr[m - 1], acc_r * a.inv_h2, base);
                }
                if (m < K) {
                    WR[m - 1][rs(0)] = v;
                    if (EMB) ehn[m - 1] = eh;
                    if (ST && out_col && p >= z0 && p < z1) {
                        double2 *lv = a.lvl_out + (m - 1) * a.lvl_stride + pst * plane(p);
                        if constexpr (BUF) buf_store_c(lv, pb16, o16, v);
                        else lv[oxy] = v;
                    }
                } else if (out_col && p >= z0 && p < z1) {
                    // an output column is inside the grid: oxy is its own offset
                    const long long po = pst * plane(p);
                    if constexpr (BUF) {
                        if (OUT_REAL) buf_store_f64(a.out_re + po, pb8, o8, v.x);
                        else buf_store_c(a.out_c + po, pb16, o16, v);
                        if (EMB) buf_store_f64(a.emb_out + po, pb8, o8, eh);
                    } else {
                        const long long i = oxy + po;
                        if (OUT_REAL) a.out_re[i] = v.x;
                        else a.out_c[i] = v;
                        if (EMB) a.emb_out[i] = eh;
                    }
                }
            }
            if (!RA && m < K) readw(m + 1, nxt);
            cur = nxt;
        }
        // All LDS writes of the step come after all its reads, so the reads
        // of every level can be issued early. A wavefront stores the levels
        // it computed (a lane of it that does not need level m stores a value
        // no needed cell reads; the levels it skips no needed cell reads
        // either); a ghost column stores nothing, so its cells keep the ghost
        // value 0.
        if (!col_ghost) {
            sL[wb][0][slot] = L0[rs(0)];
#pragma unroll
            for (int m = 1; m < K; ++m)
                if (m <= wneed) sL[wb][m][slot] = WR[m - 1][rs(0)];
        }
        if (EMB) {
#pragma unroll
            for (int m = 0; m + 1 < K; ++m) ehc[m] = ehn[m];
        }
        if constexpr (FR) {
            sD[wb][slot] = dht;
            dhp = dht;
        }
        if constexpr (DR) sD[dslot(t)][slot] = dht;
        __syncthreads();   // step t's planes are visible to step t+1, whose
                           // writes go to the other buffer
    }
    }
}

}  // namespace dev
}  // namespace frkc2
