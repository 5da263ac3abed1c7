// Deterministic FP64 reductions for norms, the loss and the Gershgorin bound.
//
// First pass: a fixed grid of kReduceBlocks workgroups strides over the
// input; each thread accumulates in a fixed order, the wavefront folds its 64
// lanes with cross-lane shuffles, the waves of a workgroup combine through
// LDS, and each workgroup writes one partial. Second pass: one workgroup folds
// the partials in index order. The grid is fixed, so the summation order (and
// the result) does not depend on the device or the run.
//
// The Gershgorin bound (stability requirement T rho <= betabar of Sec. 2,
// |R(T lambda)| <= 1 on the spectrum) is the largest row sum |a_cc| + sum |a_cn|
// of the Jacobian of f, faces in the order x-, x+, y-, y+, z-, z+. For the
// linear operators the row sum is 2 sum_f D_f / h^2 with the operator's face
// diffusivity. For div(u^2 grad u) the face value Q_f = (w_c^2 + w_nb^2)/2
// depends on the state, so the row is diag = sum_f (w_c dw - Q_f),
// off_nb = w_nb dw + Q_f with dw = w_nb - w_c (over h^2; a Dirichlet ghost adds
// to the diagonal only); rho_pass1 yields max_c (|diag| + sum |off|) and the
// host multiplies by 1/h^2. A maximum is exact in any order.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace frkc2 {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

enum { R_SUMSQ = FRKC2_RED_SUMSQ, R_SUM = FRKC2_RED_SUM, R_MAXSQ = FRKC2_RED_MAXSQ,
       R_SQDIFF = FRKC2_RED_SUMSQDIFF, R_DOT = FRKC2_RED_DOT, R_MAX = 100 };

template <int OP>
__device__ __forceinline__ double combine(double a, double b)
{
    if (OP == R_MAXSQ || OP == R_MAX) return a > b ? a : b;
    return a + b;
}

template <int OP>
__device__ __forceinline__ double block_reduce(double v)
{
    __shared__ double s[kWaves];
    for (int off = 32; off > 0; off >>= 1) v = combine<OP>(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s[wave] = v;
    __syncthreads();
    double r = s[0];
    for (int i = 1; i < kWaves; ++i) r = combine<OP>(r, s[i]);
    return r;
}

template <int OP>
__global__ __launch_bounds__(kThreads) void reduce_pass1(const double *x, const double *y,
                                                         long long n, double *partials)
{
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kThreads) {
        const double v = x[i];
        double t;
        if (OP == R_SUMSQ || OP == R_MAXSQ) t = v * v;
        else if (OP == R_SUM) t = v;
        else if (OP == R_SQDIFF) {
            const double d = v - y[i];
            t = d * d;
        } else if (OP == R_DOT) t = v * y[i];
        else t = v;
        acc = combine<OP>(acc, t);
    }
    const double r = block_reduce<OP>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <int OP>
__global__ __launch_bounds__(kThreads) void reduce_pass2(double *partials, int nb)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += kThreads) acc = combine<OP>(acc, partials[i]);
    const double r = block_reduce<OP>(acc);
    if (threadIdx.x == 0) partials[nb] = r;
}

// per-cell Jacobian row sum (without the 1/h^2 factor; linear operators also
// without their factor 2), then max
constexpr int kRhoThreads = 1024;   // a full CU of wavefronts over the grid's loads

template <int OP, int BC, int NDIM>
__global__ __launch_bounds__(kRhoThreads) void rho_pass1(const double *w, const double *D, int nx,
                                                      int ny, int nz, double d_const,
                                                      double *partials)
{
    // Work items of up to kRhoThreads points: a segment of one x row, or
    // several whole rows when they are shorter, so that the row and its y, z
    // follow from one (uniform) division per item
    const int tpr = nx < kRhoThreads ? nx : kRhoThreads;     // threads per row segment
    const int rpi = kRhoThreads / tpr;                        // rows per item
    const int cpr = (nx + tpr - 1) / tpr;                     // segments per row
    const long long rows = (long long)ny * nz;
    const long long items = (long long)cpr * ((rows + rpi - 1) / rpi);
    const int trow = (int)threadIdx.x / tpr, tx = (int)threadIdx.x % tpr;
    double m = 0.0;
    for (long long it = blockIdx.x; it < items; it += gridDim.x) {
        const long long rg = it / cpr;
        const long long r = rg * rpi + trow;
        const int x = (int)(it - rg * cpr) * tpr + tx;
        if (trow >= rpi || r >= rows || x >= nx) continue;
        int y, z;
        if (rows <= 0xffffffffLL) {   // 32-bit division where the rows allow (uniform)
            y = (int)((unsigned)r % (unsigned)ny);
            z = (int)((unsigned)r / (unsigned)ny);
        } else {
            y = (int)(r % ny);
            z = (int)(r / ny);
        }
        const long long p = x + (long long)nx * r;
        double sum = 0.0, diag = 0.0;
        // Every neighbour is loaded, with no branch around the loads (so they
        // are all in flight together): a Dirichlet ghost at the clamped index,
        // which is the cell itself, then set aside by a select.
        const double Dc = (OP == FRKC2_OP_VARCOEF) ? D[p] : 0.0;
        const double wc = (OP == FRKC2_OP_POROUS2) ? w[p] : 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const int d = f >> 1;
            if (NDIM == 1 && d > 0) continue;
            if (NDIM == 2 && d == 1) continue;   // 2D grids march in z
            int j[3] = {x, y, z};
            const int nd[3] = {nx, ny, nz};
            const int jd = j[d] + ((f & 1) ? 1 : -1);
            const bool out = jd < 0 || jd >= nd[d];
            const bool ghost = (BC == FRKC2_BC_DIRICHLET0) && out;
            j[d] = (BC == FRKC2_BC_DIRICHLET0) ? min(max(jd, 0), nd[d] - 1)
                                               : (out ? (jd < 0 ? jd + nd[d] : jd - nd[d]) : jd);
            const long long q = j[0] + (long long)nx * (j[1] + (long long)ny * j[2]);
            double Df;
            if (OP == FRKC2_OP_LAPLACE) {
                Df = d_const;
            } else if (OP == FRKC2_OP_VARCOEF) {
                Df = 0.5 * Dc + 0.5 * D[q];   // a ghost's clamped D is D_c
            } else {
                const double wq = w[q];
                const double un = ghost ? 0.0 : wq;
                const double dw = un - wc;
                const double Q = 0.5 * (wc * wc + un * un);
                diag = diag + (wc * dw - Q);
                if (!ghost) sum = sum + fabs(un * dw + Q);
                continue;
            }
            sum = sum + Df;
        }
        if (OP == FRKC2_OP_POROUS2) sum = fabs(diag) + sum;
        m = m > sum ? m : sum;
    }
    // block maximum (exact in any order): wavefronts, then their maxima
    __shared__ double sm[kRhoThreads / 64];
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(m, off, 64);
        m = m > o ? m : o;
    }
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sm[0];
        for (int i = 1; i < kRhoThreads / 64; ++i) r = r > sm[i] ? r : sm[i];
        partials[blockIdx.x] = r;
    }
}

template <int OP>
int launch_red(const double *x, const double *y, long long n, double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_pass1<OP>, dim3(kReduceBlocks), dim3(kThreads), 0, st, x, y, n,
                       partials);
    hipLaunchKernelGGL(reduce_pass2<OP>, dim3(1), dim3(kThreads), 0, st, partials,
                       kReduceBlocks);
    return (int)hipGetLastError();
}

template <int OP, int BC>
int launch_rho_t(const KGrid &g, const double *w, const double *D, double *partials,
                 hipStream_t st)
{
    dim3 grid(kReduceBlocks), block(kRhoThreads);
    if (g.ndim == 3)
        hipLaunchKernelGGL((rho_pass1<OP, BC, 3>), grid, block, 0, st, w, D, g.nx, g.ny, g.nz,
                           g.d_const, partials);
    else if (g.ndim == 2)
        hipLaunchKernelGGL((rho_pass1<OP, BC, 2>), grid, block, 0, st, w, D, g.nx, g.ny, g.nz,
                           g.d_const, partials);
    else
        hipLaunchKernelGGL((rho_pass1<OP, BC, 1>), grid, block, 0, st, w, D, g.nx, g.ny, g.nz,
                           g.d_const, partials);
    hipLaunchKernelGGL(reduce_pass2<R_MAX>, dim3(1), dim3(kThreads), 0, st, partials,
                       kReduceBlocks);
    return (int)hipGetLastError();
}

template <int OP>
int launch_rho_bc(const KGrid &g, const double *w, const double *D, double *partials,
                  hipStream_t st)
{
    if (g.bc == FRKC2_BC_PERIODIC) return launch_rho_t<OP, FRKC2_BC_PERIODIC>(g, w, D, partials, st);
    return launch_rho_t<OP, FRKC2_BC_DIRICHLET0>(g, w, D, partials, st);
}

// Scaled error of the embedded pair (O'Sullivan, arXiv:1702.03818, Sec. 3):
// per point |W - What| / (tol (1 + max(|W|, |What|))) with the complex
// modulus sqrt(re*re + im*im), then the maximum over points (exact in any
// order). A NaN counts as infinity so that it cannot be lost in the maximum.
__global__ __launch_bounds__(kThreads) void err_pass1(const double2 *W, const double *E,
                                                      long long n, double tol, double *partials)
{
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kThreads) {
        const double2 w = W[i];
        const double e = E[i];
        const double dr = w.x - e;
        const double num = sqrt(dr * dr + w.y * w.y);
        const double mw = sqrt(w.x * w.x + w.y * w.y);
        const double ae = fabs(e);
        const double den = tol * (1.0 + (mw > ae ? mw : ae));
        double q = num / den;
        q = (q == q) ? q : __builtin_inf();
        acc = combine<R_MAX>(acc, q);
    }
    const double r = block_reduce<R_MAX>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ __launch_bounds__(kThreads) void take_real(const double2 *W, double *w, long long n)
{
    for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kThreads)
        w[i] = W[i].x;
}

}  // namespace

int launch_reduce(int op, const double *x, const double *y, long long n, double *partials,
                  hipStream_t st)
{
    switch (op) {
    case R_SUMSQ: return launch_red<R_SUMSQ>(x, y, n, partials, st);
    case R_SUM: return launch_red<R_SUM>(x, y, n, partials, st);
    case R_MAXSQ: return launch_red<R_MAXSQ>(x, y, n, partials, st);
    case R_SQDIFF: return launch_red<R_SQDIFF>(x, y, n, partials, st);
    case R_DOT: return launch_red<R_DOT>(x, y, n, partials, st);
    default: return (int)hipErrorInvalidValue;
    }
}

int launch_rho(const KGrid &g, const double *w, const double *D, double *partials, hipStream_t st)
{
    if (g.op == FRKC2_OP_LAPLACE) return launch_rho_bc<FRKC2_OP_LAPLACE>(g, w, D, partials, st);
    if (g.op == FRKC2_OP_VARCOEF) return launch_rho_bc<FRKC2_OP_VARCOEF>(g, w, D, partials, st);
    return launch_rho_bc<FRKC2_OP_POROUS2>(g, w, D, partials, st);
}

}  // namespace frkc2

namespace frkc2 {

int launch_err_max(const double *Wc, const double *E, long long n, double tol, double *partials,
                   hipStream_t st)
{
    hipLaunchKernelGGL(err_pass1, dim3(kReduceBlocks), dim3(kThreads), 0, st,
                       reinterpret_cast<const double2 *>(Wc), E, n, tol, partials);
    hipLaunchKernelGGL(reduce_pass2<R_MAX>, dim3(1), dim3(kThreads), 0, st, partials,
                       kReduceBlocks);
    return (int)hipGetLastError();
}

int launch_max_partials(double *partials, hipStream_t st)
{
    hipLaunchKernelGGL(reduce_pass2<R_MAX>, dim3(1), dim3(kThreads), 0, st, partials,
                       kReduceBlocks);
    return (int)hipGetLastError();
}

int launch_take_real(const double *Wc, double *w, long long n, hipStream_t st)
{
    long long nb = (n + kThreads - 1) / kThreads;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(take_real, dim3((unsigned)nb), dim3(kThreads), 0, st,
                       reinterpret_cast<const double2 *>(Wc), w, n);
    return (int)hipGetLastError();
}

}  // namespace frkc2
