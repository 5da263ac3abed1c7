// Device helpers shared by the stage, adjoint and batched kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace frkc2 {
namespace dev {

enum { LAP = FRKC2_OP_LAPLACE, VAR = FRKC2_OP_VARCOEF, POR = FRKC2_OP_POROUS2,
       ADV = FRKC2_OP_ADVDIFF };
enum { PER = FRKC2_BC_PERIODIC, DIR = FRKC2_BC_DIRICHLET0 };

struct Dims {
    int nx, ny, nz;
};

__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
    // Dispatch places block b on XCD b % 8. Give XCD i the logical blocks
    // [i*per, (i+1)*per) so that tiles sharing halos share an L2.
    const int per = nb >> 3;
    if (bid >= (per << 3)) return bid;
    return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ int wrap(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

// Flat index of (gx, gy, gz) after applying the boundary condition; -1 for a
// Dirichlet ghost outside the grid.
template <int BC>
__device__ __forceinline__ long long bc_index(const Dims &d, int gx, int gy, int gz)
{
    if (BC == PER) {
        gx = wrap(gx, d.nx);
        gy = wrap(gy, d.ny);
        gz = wrap(gz, d.nz);
    } else if (gx < 0 || gx >= d.nx || gy < 0 || gy >= d.ny || gz < 0 || gz >= d.nz) {
        return -1;
    }
    return gx + (long long)d.nx * (gy + (long long)d.ny * gz);
}

// Complex value at (gx, gy, gz); a real input is read as (w, 0); a Dirichlet
// ghost is 0.
template <int BC, bool IN_REAL>
__device__ __forceinline__ double2 load_c(const Dims &d, const double *re, const double2 *c,
                                          int gx, int gy, int gz)
{
    const long long i = bc_index<BC>(d, gx, gy, gz);
    if (i < 0) return make_double2(0.0, 0.0);
    if (IN_REAL) return make_double2(re[i], 0.0);
    return c[i];
}

// Real value at (gx, gy, gz); 0 for a Dirichlet ghost (a ghost face takes the
// boundary cell's own diffusivity, so this value is never used).
template <int BC>
__device__ __forceinline__ double load_r(const Dims &d, const double *v, int gx, int gy, int gz)
{
    const long long i = bc_index<BC>(d, gx, gy, gz);
    return i < 0 ? 0.0 : v[i];
}

// Branch-free versions for software pipelining: the load is always issued
// (at a clamped in-range address) and a Dirichlet ghost is selected to 0
// afterwards, so no control flow separates a prefetch from its use and the
// compiler can keep several loads in flight across barriers.
template <int BC>
__device__ __forceinline__ long long bc_index_nb(const Dims &d, int gx, int gy, int gz, bool &ghost)
{
    if (BC == PER) {
        ghost = false;
        gx = wrap(gx, d.nx);
        gy = wrap(gy, d.ny);
        gz = wrap(gz, d.nz);
    } else {
        ghost = (gx < 0) | (gx >= d.nx) | (gy < 0) | (gy >= d.ny) | (gz < 0) | (gz >= d.nz);
        gx = min(max(gx, 0), d.nx - 1);
        gy = min(max(gy, 0), d.ny - 1);
        gz = min(max(gz, 0), d.nz - 1);
    }
    return gx + (long long)d.nx * (gy + (long long)d.ny * gz);
}

template <int BC, bool IN_REAL>
__device__ __forceinline__ double2 load_c_nb(const Dims &d, const double *re, const double2 *c,
                                             int gx, int gy, int gz)
{
    bool ghost;
    const long long i = bc_index_nb<BC>(d, gx, gy, gz, ghost);
    double2 v;
    if (IN_REAL) v = make_double2(re[i], 0.0);
    else v = c[i];
    v.x = ghost ? 0.0 : v.x;
    v.y = ghost ? 0.0 : v.y;
    return v;
}

template <int BC>
__device__ __forceinline__ double load_r_nb(const Dims &d, const double *v, int gx, int gy, int gz)
{
    bool ghost;
    const long long i = bc_index_nb<BC>(d, gx, gy, gz, ghost);
    const double r = v[i];
    return ghost ? 0.0 : r;
}

// Buffer accesses: a resource (scalar registers) whose base is the given
// pointer and whose extent is `bytes`, addressed by a 32-bit byte offset per
// lane. An offset at or past the extent reads 0 and drops a store. The third
// word is the CDNA raw-buffer format (no swizzle, no stride).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, 0x00020000);
}

__device__ __forceinline__ double buf_load_f64(const double *base, int bytes, unsigned off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(buf_rsrc(base, bytes), off, 0, 0);
    return __builtin_bit_cast(double, v);
}

__device__ __forceinline__ double2 buf_load_c(const double2 *base, int bytes, unsigned off)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(buf_rsrc(base, bytes), off, 0, 0);
    return __builtin_bit_cast(double2, v);
}

__device__ __forceinline__ void buf_store_f64(double *base, int bytes, unsigned off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(HIP_vector_base<unsigned, 2>::Native_vec_, v),
                                          buf_rsrc(base, bytes), off, 0, 0);
}

__device__ __forceinline__ void buf_store_c(double2 *base, int bytes, unsigned off, double2 v)
{
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(HIP_vector_base<unsigned, 4>::Native_vec_, v),
                                           buf_rsrc(base, bytes), off, 0, 0);
}

// W^2 of a complex value in the fixed order the library and its CPU check
// share: (fma(re, re, -(im*im)), 2*(re*im)).
__device__ __forceinline__ void csq(double2 c, double &qr, double &qi)
{
    qr = fma(c.x, c.x, -(c.y * c.y));
    qi = 2.0 * (c.x * c.y);
}

// W^2 / 2 of a complex value: (0.5 * fma(re, re, -(im*im)), re*im), the exact
// halves of csq(); a porous face value is the sum of the two cells' halves.
__device__ __forceinline__ void csqh(double2 c, double &qr, double &qi)
{
    qr = 0.5 * fma(c.x, c.x, -(c.y * c.y));
    qi = c.x * c.y;
}

// Porous face with both cells' W^2/2 given: Q = qh_c + qh_n,
// acc_r = fma(Qr, dr, fma(-Qi, di, acc_r)), acc_i = fma(Qr, di, fma(Qi, dr, acc_i)).
__device__ __forceinline__ void face_por(double &acc_r, double &acc_i, double2 c, double2 nb,
                                         double qr_c, double qi_c, double qr_n, double qi_n)
{
    const double dr = nb.x - c.x;
    const double di = nb.y - c.y;
    const double Dr = qr_c + qr_n;
    const double Di = qi_c + qi_n;
    acc_r = fma(Dr, dr, fma(-Di, di, acc_r));
    acc_i = fma(Dr, di, fma(Di, dr, acc_i));
}

// One face of the flux sum of the diffusion operator, in the fixed order the
// library and its CPU check share (fused multiply-adds, correctly rounded).
// nb: neighbour value (0 for a Dirichlet ghost); dc, dn: halves of the cell
// and neighbour diffusivity (0.5 * D, exact; the kernels halve D once when
// they load it), D_f = dc + dn, the mean of the two; ghost takes dn = dc, so
// the face carries D_c; qr_c, qi_c: W_c^2/2 (csqh) for the porous operator; d_const:
// the face's coefficient for LAPLACE (d) and ADVDIFF (d -+ v h/2).
template <int OP>
__device__ __forceinline__ void face(double &acc_r, double &acc_i, double2 c, double2 nb,
                                     double dc, double dn, bool ghost, double qr_c, double qi_c,
                                     double d_const)
{
    if (OP == POR) {
        double qr_n, qi_n;
        csqh(nb, qr_n, qi_n);
        face_por(acc_r, acc_i, c, nb, qr_c, qi_c, qr_n, qi_n);
    } else {
        const double dr = nb.x - c.x;
        const double di = nb.y - c.y;
        double Df;
        if (OP == LAP || OP == ADV) Df = d_const;   // the face's own coefficient
        else Df = dc + (ghost ? dc : dn);
        acc_r = fma(Df, dr, acc_r);
        acc_i = fma(Df, di, acc_i);
    }
}

// Forward Euler update W + tau f with f = acc * inv_h2:
// (fma(tr, fr, fma(-ti, fi, Wr)), fma(tr, fi, fma(ti, fr, Wi))).
__device__ __forceinline__ double2 euler(double2 c, double acc_r, double acc_i, double inv_h2,
                                         double tr, double ti)
{
    const double fr = acc_r * inv_h2;
    const double fi = acc_i * inv_h2;
    return make_double2(fma(tr, fr, fma(-ti, fi, c.x)), fma(tr, fi, fma(ti, fr, c.y)));
}

}  // namespace dev
}  // namespace frkc2
