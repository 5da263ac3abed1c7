// One tile of the one-stage plane-march kernel, shared by the plain stage
// kernel and the batched level kernels. See stage.hip for the design.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace dev {

struct PlaneArgs {
    const double *in_re;
    const double2 *in_c;
    double *out_re;
    double2 *out_c;
    const double *D;
    const double *emb_in;       // embedded first-order solution in (EMB, not first stage)
    double *emb_out;            // ... and out (EMB)
    int nx, ny, nz;
    int zchunk, ntx, nty;
    double inv_h2, d_const, tr, ti;
    double fc[6];               // face coefficient per face x-, x+, y-, y+, z-, z+ (LAPLACE,
                                // ADVDIFF; d_const for LAPLACE)
};

template <int BC, bool IN_REAL>
__device__ __forceinline__ double2 load_w(const PlaneArgs &a, int gx, int gy, int gz)
{
    return load_c<BC, IN_REAL>(Dims{a.nx, a.ny, a.nz}, a.in_re, a.in_c, gx, gy, gz);
}

template <int OP, int BC, int NDIM, int BX, int BY>
struct TileShape {
    static constexpr int SX = BX + 2;
    static constexpr int SY = (NDIM == 3) ? BY + 2 : 1;   // 1D/2D tiles need only the x halo
    static constexpr int PL = SX * SY;
    static constexpr int LDS_W = 2 * PL;                   // double2 entries
    static constexpr int LDS_D = (OP == FRKC2_OP_VARCOEF) ? 2 * PL : 1;
};

// One tile (bx, by) of BX x BY columns over the z planes of chunk bz; sWp and
// sDp are the tile's LDS (TileShape::LDS_W double2, ::LDS_D doubles). With
// EMB the tile also advances the embedded first-order solution of the error
// estimate (O'Sullivan, arXiv:1702.03818, Sec. 3): What + Re(tau) Re f(W),
// evaluated as fma(tr, f_r, What); a first stage (IN_REAL) starts it from the
// real input.
template <int OP, int BC, int NDIM, int BX, int BY, bool IN_REAL, bool OUT_REAL, bool EMB = false>
__device__ __forceinline__ void plane_tile(const PlaneArgs &a, int bx, int by, int bz,
                                           double2 *sWp, double *sDp)
{
    constexpr int SX = BX + 2;
    constexpr int SY = (NDIM == 3) ? BY + 2 : 1;   // 1D/2D tiles need only the x halo
    constexpr int NT = BX * BY;
    constexpr int NH = 2 * BY + (NDIM == 3 ? 2 * BX : 0);   // halo cells per plane
    static_assert(NH <= NT, "one halo cell per thread at most");
    double2 (*sW)[SY * SX] = reinterpret_cast<double2 (*)[SY * SX]>(sWp);
    double (*sD)[SY * SX] = reinterpret_cast<double (*)[SY * SX]>(sDp);

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int x0 = bx * BX, y0 = by * BY;
    const int x = x0 + tx, y = y0 + ty;
    const bool active = x < a.nx && y < a.ny;
    const int z0 = bz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);

    // this thread's halo cell (if any), as plane-local (hx, hy)
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

    // Own column: planes z-1, z, z+1 in use and z+2 in flight; halo cell of
    // plane z in use and of z+1 in flight. All loads are branch-free (a
    // thread without a halo cell re-reads its own point), so the prefetches
    // stay outstanding across the barrier.
    const Dims dm{a.nx, a.ny, a.nz};
    const int hgx = has_halo ? x0 + hx : x, hgy = has_halo ? y0 + hy : y;
    // Raw loads at clamped (or wrapped) addresses; a Dirichlet ghost is zeroed
    // only where the value is consumed, so nothing waits for a prefetch early.
    auto LW = [&](int gx, int gy, int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, gx, gy, gz, g);
        return IN_REAL ? make_double2(a.in_re[i], 0.0) : a.in_c[i];
    };
    auto LD = [&](int gx, int gy, int gz) {
        bool g;
        const long long i = bc_index_nb<BC>(dm, gx, gy, gz, g);
        return (OP == VAR) ? 0.5 * a.D[i] : 0.0;   // D/2 (face rule); ghost D is never used
    };
    const bool dirichlet = (BC == DIR);
    const bool own_out = dirichlet && !(x < a.nx && y < a.ny);
    const bool halo_out = dirichlet && !(hgx >= 0 && hgx < a.nx && hgy >= 0 && hgy < a.ny);
    auto keep = [&](double2 v, bool ghost) {
        v.x = ghost ? 0.0 : v.x;
        v.y = ghost ? 0.0 : v.y;
        return v;
    };
    auto zout = [&](int p) { return dirichlet && (p < 0 || p >= a.nz); };
    // Plane p of the own column sits in ring slot (p - z0 + 1) & 3 and the
    // halo cell of plane p in slot (p - z0) & 1. The z loop is unrolled by
    // four, so every slot index is a compile-time constant: a new plane is
    // loaded straight into the slot it will be used from, and no register
    // copy has to wait for a load in flight.
    double2 Wr[4] = {LW(x, y, z0 - 1), LW(x, y, z0), LW(x, y, z0 + 1), LW(x, y, z0 + 2)};
    double Dr[4] = {LD(x, y, z0 - 1), LD(x, y, z0), LD(x, y, z0 + 1), LD(x, y, z0 + 2)};
    double2 hWr[2] = {LW(hgx, hgy, z0), LW(hgx, hgy, z0 + 1)};
    double hDr[2] = {LD(hgx, hgy, z0), LD(hgx, hgy, z0 + 1)};

    // Planes z0-1 and z0 are consumed first; every later plane gets its
    // Dirichlet ghosts zeroed in its ring slot when it is first used (as the
    // z+ neighbour).
    Wr[0] = keep(Wr[0], own_out || zout(z0 - 1));
    Wr[1] = keep(Wr[1], own_out || zout(z0));
    for (int zb = z0; zb < z1; zb += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int z = zb + u;
        if (z >= z1) break;
        Wr[(u + 2) & 3] = keep(Wr[(u + 2) & 3], own_out || zout(z + 1));
        const long long iz = x + (long long)a.nx * (y + (long long)a.ny * z);
        double eh = 0.0;
        if (EMB && !IN_REAL && active) eh = a.emb_in[iz];   // issued before the barrier
        const double2 Wm = Wr[u & 3];
        const double2 Wc = Wr[(u + 1) & 3];
        const double2 Wp = Wr[(u + 2) & 3];
        const double Dm = Dr[u & 3], Dc = Dr[(u + 1) & 3], Dp = Dr[(u + 2) & 3];
        const int b = z & 1;
        sW[b][oslot] = Wc;
        if (OP == VAR) sD[b][oslot] = Dc;
        if (has_halo) {
            sW[b][hslot] = keep(hWr[u & 1], halo_out || zout(z));
            if (OP == VAR) sD[b][hslot] = hDr[u & 1];
        }
        __syncthreads();
        // planes past the chunk are never used: clamp so the tail re-reads a
        // cached line instead of fetching new data
        const int zh = min(z + 2, z1 - 1);
        hWr[u & 1] = LW(hgx, hgy, zh);
        hDr[u & 1] = LD(hgx, hgy, zh);
        if (active) {
            const double2 c = Wc;
            double qr_c = 0.0, qi_c = 0.0;
            if (OP == POR) {
                csqh(c, qr_c, qi_c);
            }
            double acc_r = 0.0, acc_i = 0.0;
            // A Dirichlet ghost holds W = 0 and the D of the boundary cell it
            // faces (loads are clamped), so every face takes the plain mean,
            // which there equals D_c bit for bit.
            face<OP>(acc_r, acc_i, c, sW[b][oslot - 1], Dc, (OP == VAR) ? sD[b][oslot - 1] : 0.0,
                     false, qr_c, qi_c, a.fc[0]);
            face<OP>(acc_r, acc_i, c, sW[b][oslot + 1], Dc, (OP == VAR) ? sD[b][oslot + 1] : 0.0,
                     false, qr_c, qi_c, a.fc[1]);
            if (NDIM == 3) {
                face<OP>(acc_r, acc_i, c, sW[b][oslot - SX], Dc,
                         (OP == VAR) ? sD[b][oslot - SX] : 0.0, false, qr_c, qi_c, a.fc[2]);
                face<OP>(acc_r, acc_i, c, sW[b][oslot + SX], Dc,
                         (OP == VAR) ? sD[b][oslot + SX] : 0.0, false, qr_c, qi_c, a.fc[3]);
            }
            if (NDIM >= 2) {
                face<OP>(acc_r, acc_i, c, Wm, Dc, Dm, false, qr_c, qi_c, a.fc[4]);
                face<OP>(acc_r, acc_i, c, Wp, Dc, Dp, false, qr_c, qi_c, a.fc[5]);
            }
            const double2 nv = euler(c, acc_r, acc_i, a.inv_h2, a.tr, a.ti);
            const long long i = iz;
            if (OUT_REAL) a.out_re[i] = nv.x;
            else a.out_c[i] = nv;
            if (EMB) {
                const double fr = acc_r * a.inv_h2;
                a.emb_out[i] = fma(a.tr, fr, IN_REAL ? c.x : eh);
            }
        }
        const int zq = min(z + 3, z1);   // plane z1 is the last one used (z+ of z1-1)
        Wr[u & 3] = LW(x, y, zq);        // into the slot of plane z-1
        Dr[u & 3] = LD(x, y, zq);
    }
    }
}


}  // namespace dev
}  // namespace frkc2
