// Reaction flow of the two-species Brusselator over a complex time: the B flow of
// the split fourth-order scheme FRKC4s (O'Sullivan, arXiv:1702.03818, Sec. 4.1,
// "Complex splitting"; the Brusselator is the problem of Sec. 3.1).
//
// The splitting alternates flows of the linear diffusion A (FRKC4 supersteps,
// run by the stage kernels on complex states) with flows of the reaction
// f_B(v, w) = (1 - 4v + v^2 w, 3v - v^2 w), whose steps tau = b T are complex.
// The reaction is pointwise, so its flow is integrated on each grid point by
// itself: dY/ds = tau f_B(Y) for s in [0, 1], f_B continued to complex v, w
// (a polynomial), by nsub classical Runge-Kutta steps of length 1/nsub in s.
//
// The arithmetic order is fixed (no multiply-add fused; the file is compiled
// with contraction off) and shared with the CPU check:
//   f:  v2 = (vr*vr - vi*vi, 2*(vr*vi)), q = v2 w = (v2r*wr - v2i*wi,
//       v2r*wi + v2i*wr), fv = ((1 - 4*vr) + qr, qi - 4*vi),
//       fw = (3*vr - qr, 3*vi - qi);
//   y + c k = (yr + (cr*kr - ci*ki), yi + (cr*ki + ci*kr)) per species;
//   k1 = f(y), k2 = f(y + (c/2) k1), k3 = f(y + (c/2) k2), k4 = f(y + c k3),
//   y <- y + (c/6) (((k1 + 2 k2) + 2 k3) + k4),
// with c = tau / nsub, c/2 and c/6 formed on the host.
//
// Memory: one pass reads and writes both species' complex values of a point,
// 64 B per point and flow; XCD-contiguous grid-stride blocks.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace frkc2 {
namespace {

using namespace dev;

struct Bz {
    double vr, vi, wr, wi;
};

__device__ __forceinline__ Bz bz_f(const Bz &y)
{
    const double v2r = y.vr * y.vr - y.vi * y.vi;
    const double v2i = 2.0 * (y.vr * y.vi);
    const double qr = v2r * y.wr - v2i * y.wi;
    const double qi = v2r * y.wi + v2i * y.wr;
    return Bz{(1.0 - 4.0 * y.vr) + qr, qi - 4.0 * y.vi, 3.0 * y.vr - qr, 3.0 * y.vi - qi};
}

__device__ __forceinline__ Bz bz_axpy(const Bz &y, double cr, double ci, const Bz &k)
{
    return Bz{y.vr + (cr * k.vr - ci * k.vi), y.vi + (cr * k.vi + ci * k.vr),
              y.wr + (cr * k.wr - ci * k.wi), y.wi + (cr * k.wi + ci * k.wr)};
}

constexpr int kReactThreads = 256;

__global__ __launch_bounds__(kReactThreads) void bruss_react_flow(double2 *Z, long long n,
                                                                  double cr, double ci,
                                                                  double c2r, double c2i,
                                                                  double c6r, double c6i, int nsub)
{
    const long long stride = (long long)gridDim.x * kReactThreads;
    const long long b = xcd_remap(blockIdx.x, gridDim.x);
    for (long long p = b * kReactThreads + threadIdx.x; p < n; p += stride) {
        const double2 v = Z[p], w = Z[n + p];
        Bz y{v.x, v.y, w.x, w.y};
        for (int j = 0; j < nsub; ++j) {
            const Bz k1 = bz_f(y);
            const Bz k2 = bz_f(bz_axpy(y, c2r, c2i, k1));
            const Bz k3 = bz_f(bz_axpy(y, c2r, c2i, k2));
            const Bz k4 = bz_f(bz_axpy(y, cr, ci, k3));
            const Bz S{((k1.vr + 2.0 * k2.vr) + 2.0 * k3.vr) + k4.vr,
                       ((k1.vi + 2.0 * k2.vi) + 2.0 * k3.vi) + k4.vi,
                       ((k1.wr + 2.0 * k2.wr) + 2.0 * k3.wr) + k4.wr,
                       ((k1.wi + 2.0 * k2.wi) + 2.0 * k3.wi) + k4.wi};
            y = bz_axpy(y, c6r, c6i, S);
        }
        Z[p] = make_double2(y.vr, y.vi);
        Z[n + p] = make_double2(y.wr, y.wi);
    }
}

}  // namespace

int launch_react_flow(double *Zc, long long n, const double c[6], int nsub, hipStream_t st)
{
    long long blocks = (n + kReactThreads - 1) / kReactThreads;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(bruss_react_flow, dim3((unsigned)blocks), dim3(kReactThreads), 0, st,
                       reinterpret_cast<double2 *>(Zc), n, c[0], c[1], c[2], c[3], c[4], c[5],
                       nsub);
    return (int)hipGetLastError();
}

}  // namespace frkc2
