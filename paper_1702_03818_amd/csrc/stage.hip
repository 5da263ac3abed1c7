// FRKC2 stage kernels for gfx950: one forward Euler step with a complex
// stepsize, W <- W + tau f(W) (O'Sullivan, arXiv:1702.03818, Sec. 3, the
// Euler-step equation of the FRKC2 scheme), with the diffusion operator f
// fused into the update.
//
// Data layout in HBM: the real state w and the diffusivity D are the
// caller's flat FP64 arrays (x fastest); complex stage values live in
// workspace buffers as interleaved (re, im) pairs, 16 B per point, so one
// 128-bit load or store moves a whole complex value.
//
// plane_stage: a workgroup owns a BX x BY tile of the (x, y) plane and marches
// through a chunk of z planes. The z-neighbours of a point stay in registers
// (planes z-1, z, z+1 of the thread's own column); the x/y neighbours come
// from an LDS copy of plane z with a one-cell halo, double-buffered so one
// barrier per plane suffices; the halo of the next plane is prefetched into
// registers while the current plane is computed. Every input value is read
// from HBM once per pass except the tile halos, which are shared through L2:
// the block index is remapped so that each XCD receives a contiguous range of
// tiles (round-robin dispatch would scatter neighbouring tiles over all eight
// L2 caches). 2D grids march along their second dimension with BY = 1; 1D
// grids use a single plane.
//
// Arithmetic order (identical in every kernel and in the CPU check, see
// face() and euler() in device_common.h): faces x-, x+, y-, y+, z-, z+;
// acc = fma(Df, W_nb - W_c, acc) per face; f = acc*inv_h2;
// W_r = fma(tr, f_r, fma(-ti, f_i, W_r)), W_i = fma(tr, f_i, fma(ti, f_r, W_i)).
// The library is compiled with -ffp-contract=off, so no other operation is
// fused and the result is independent of the tile shape.
#include <hip/hip_runtime.h>

#include "plane_tile.h"

namespace frkc2 {
namespace {

using namespace dev;

template <int OP, int BC, int NDIM, int BX, int BY, bool IN_REAL, bool OUT_REAL, bool EMB = false>
__global__ __launch_bounds__(BX *BY) void plane_stage(PlaneArgs a)
{
    using S = TileShape<OP, BC, NDIM, BX, BY>;
    __shared__ double2 sW[S::LDS_W];
    __shared__ double sD[S::LDS_D];
    int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = lb % a.ntx;
    lb /= a.ntx;
    const int by = lb % a.nty;
    const int bz = lb / a.nty;
    plane_tile<OP, BC, NDIM, BX, BY, IN_REAL, OUT_REAL, EMB>(a, bx, by, bz, sW, sD);
}

// Whole 1D grid resident in LDS: every stage of every superstep in one
// launch, two barriers per stage. Used when the grid fits (small 1D cases).
constexpr int k1dThreads = 1024;
constexpr int k1dMaxPts = 4096;
constexpr int k1dPerThread = k1dMaxPts / k1dThreads;

template <int OP, int BC, bool EMB>
__global__ __launch_bounds__(k1dThreads) void stage1d_lds(const double *w_in, double *w_out,
                                                          const double *D, const double2 *tau,
                                                          int n, int s, int nsteps,
                                                          double inv_h2, double fcl, double fcr,
                                                          double2 *out_c, double *emb_out)
{
    extern __shared__ double2 s1[];
    double2 *sW = s1;
    double *sD = reinterpret_cast<double *>(s1 + n);
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += k1dThreads) {
        sW[i] = make_double2(w_in[i], 0.0);
        if (OP == VAR) sD[i] = 0.5 * D[i];   // D/2, as the face rule takes it
    }
    // EMB (one superstep): the embedded first-order solution of each thread's
    // points, What <- What + Re tau Re f(W) per stage, in registers; W^L is
    // then written complex to out_c and What^L to emb_out.
    double ev[EMB ? k1dPerThread : 1];
    if (EMB) {
#pragma unroll
        for (int p = 0; p < k1dPerThread; ++p) {
            const int i = tid + p * k1dThreads;
            ev[p] = (i < n) ? w_in[i] : 0.0;
        }
    }
    __syncthreads();
    for (int step = 0; step < nsteps; ++step) {
        for (int l = 0; l < s; ++l) {
            const double tr = tau[l].x, ti = tau[l].y;
            const bool last = (l == s - 1) && !EMB;
            double2 nv[k1dPerThread];
#pragma unroll
            for (int p = 0; p < k1dPerThread; ++p) {
                const int i = tid + p * k1dThreads;
                if (i >= n) break;
                const double2 c = sW[i];
                double qr_c = 0.0, qi_c = 0.0;
                if (OP == POR) {
                    csqh(c, qr_c, qi_c);
                }
                const bool gl = (BC == DIR) && i == 0;
                const bool gr = (BC == DIR) && i == n - 1;
                const int il = (i == 0) ? n - 1 : i - 1;
                const int ir = (i == n - 1) ? 0 : i + 1;
                const double2 wl = gl ? make_double2(0.0, 0.0) : sW[il];
                const double2 wr = gr ? make_double2(0.0, 0.0) : sW[ir];
                const double dc = (OP == VAR) ? sD[i] : 0.0;
                double acc_r = 0.0, acc_i = 0.0;
                face<OP>(acc_r, acc_i, c, wl, dc, (OP == VAR) ? sD[il] : 0.0, gl, qr_c, qi_c,
                         fcl);
                face<OP>(acc_r, acc_i, c, wr, dc, (OP == VAR) ? sD[ir] : 0.0, gr, qr_c, qi_c,
                         fcr);
                const double2 u = euler(c, acc_r, acc_i, inv_h2, tr, ti);
                if (EMB) ev[p] = fma(tr, acc_r * inv_h2, ev[p]);
                // a superstep keeps Re W^L; the next one starts from a real state
                nv[p] = make_double2(u.x, last ? 0.0 : u.y);
            }
            __syncthreads();
#pragma unroll
            for (int p = 0; p < k1dPerThread; ++p) {
                const int i = tid + p * k1dThreads;
                if (i >= n) break;
                sW[i] = nv[p];
            }
            __syncthreads();
        }
    }
    if (EMB) {
#pragma unroll
        for (int p = 0; p < k1dPerThread; ++p) {
            const int i = tid + p * k1dThreads;
            if (i < n) {
                out_c[i] = sW[i];
                emb_out[i] = ev[p];
            }
        }
    } else {
        for (int i = tid; i < n; i += k1dThreads) w_out[i] = sW[i].x;
    }
}

// w = Re W and per-block partial sums of (Im W)^2 and |W|^2.
constexpr int kFinThreads = 256;
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(const double2 *in, double *out,
                                                               long long n, double *partials)
{
    __shared__ double s_im[kFinThreads], s_all[kFinThreads];
    double im2 = 0.0, all2 = 0.0;
    for (long long i = blockIdx.x * (long long)kFinThreads + threadIdx.x; i < n;
         i += (long long)gridDim.x * kFinThreads) {
        const double2 v = in[i];
        out[i] = v.x;
        im2 = im2 + v.y * v.y;
        all2 = all2 + (v.x * v.x + v.y * v.y);
    }
    s_im[threadIdx.x] = im2;
    s_all[threadIdx.x] = all2;
    __syncthreads();
    for (int w = kFinThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_im[threadIdx.x] = s_im[threadIdx.x] + s_im[threadIdx.x + w];
            s_all[threadIdx.x] = s_all[threadIdx.x] + s_all[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s_im[0];
        partials[2 * blockIdx.x + 1] = s_all[0];
    }
}

__global__ __launch_bounds__(256) void finalize_sum(double *partials, int nb)
{
    // the partials staged in LDS by all threads, then summed in index order
    __shared__ double s[2 * kReduceBlocks];
    for (int i = threadIdx.x; i < 2 * nb; i += blockDim.x) s[i] = partials[i];
    __syncthreads();
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < nb; ++i) {
            a = a + s[2 * i];
            b = b + s[2 * i + 1];
        }
        partials[2 * nb] = a;
        partials[2 * nb + 1] = b;
    }
}

__global__ void real_to_complex(const double *in, double2 *out, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = make_double2(in[i], 0.0);
}

// W <- W + tau F for a user-supplied F = f(W) (Sec. 3, Euler step), in the
// library's order: (fma(tr, Fr, fma(-ti, Fi, Wr)), fma(tr, Fi, fma(ti, Fr, Wi))).
// emb (may be null): the embedded first-order solution of the error estimate
// (Sec. 3), advanced by Re tau Re f.
__global__ void euler_axpy(double2 *W, const double2 *F, double *emb, long long n, double tr,
                           double ti)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double2 w = W[i], f = F[i];
        W[i] = make_double2(fma(tr, f.x, fma(-ti, f.y, w.x)), fma(tr, f.y, fma(ti, f.x, w.y)));
        if (emb) emb[i] = fma(tr, f.x, emb[i]);
    }
}

// ---- launch ----

template <int BX, int BY>
struct TileCfg {
    static constexpr int bx = BX, by = BY;
};

int choose_zchunk(long long tiles_xy, int nz)
{
    // aim for >= 2048 workgroups (8 per CU on 256 CUs) with chunks of >= 8 planes
    int zc = nz;
    while (zc > 8 && tiles_xy * ((nz + zc - 1) / zc) < 2048) zc = (zc + 1) / 2;
    return zc;
}

template <int OP, int BC, int NDIM, int BX, int BY>
int launch_plane_t(const PlaneArgs &pa0, bool in_real, bool out_real, hipStream_t st)
{
    PlaneArgs pa = pa0;
    pa.ntx = (pa.nx + BX - 1) / BX;
    pa.nty = (pa.ny + BY - 1) / BY;
    pa.zchunk = (pa0.zchunk > 0) ? min(pa0.zchunk, pa.nz)
                                 : choose_zchunk((long long)pa.ntx * pa.nty, pa.nz);
    const long long nzc = (pa.nz + pa.zchunk - 1) / pa.zchunk;
    const long long nblk = (long long)pa.ntx * pa.nty * nzc;
    if (nblk > 0x7fffffffLL) return (int)hipErrorInvalidValue;
    dim3 grid((unsigned)nblk), block(BX * BY);
    if (pa.emb_out) {
        // embedded solution: the stage output stays complex
        if (out_real) return (int)hipErrorInvalidValue;
        if (in_real)
            hipLaunchKernelGGL((plane_stage<OP, BC, NDIM, BX, BY, true, false, true>), grid, block, 0,
                               st, pa);
        else
            hipLaunchKernelGGL((plane_stage<OP, BC, NDIM, BX, BY, false, false, true>), grid, block,
                               0, st, pa);
        return (int)hipGetLastError();
    }
    if (in_real && out_real)
        hipLaunchKernelGGL((plane_stage<OP, BC, NDIM, BX, BY, true, true>), grid, block, 0, st, pa);
    else if (in_real)
        hipLaunchKernelGGL((plane_stage<OP, BC, NDIM, BX, BY, true, false>), grid, block, 0, st, pa);
    else if (out_real)
        hipLaunchKernelGGL((plane_stage<OP, BC, NDIM, BX, BY, false, true>), grid, block, 0, st, pa);
    else
        hipLaunchKernelGGL((plane_stage<OP, BC, NDIM, BX, BY, false, false>), grid, block, 0, st, pa);
    return (int)hipGetLastError();
}

template <int OP, int BC>
int launch_plane_dim(const KGrid &g, const PlaneArgs &pa, bool ir, bool orl, hipStream_t st)
{
    if (g.ndim == 3) return launch_plane_t<OP, BC, 3, 64, 4>(pa, ir, orl, st);
    if (g.ndim == 2) return launch_plane_t<OP, BC, 2, 256, 1>(pa, ir, orl, st);
    return launch_plane_t<OP, BC, 1, 256, 1>(pa, ir, orl, st);
}

template <int OP>
int launch_plane_bc(const KGrid &g, const PlaneArgs &pa, bool ir, bool orl, hipStream_t st)
{
    if (g.bc == PER) return launch_plane_dim<OP, PER>(g, pa, ir, orl, st);
    return launch_plane_dim<OP, DIR>(g, pa, ir, orl, st);
}

}  // namespace

int launch_pass(const KGrid &g, const PassArgs &a, int /*tblock_hint*/, hipStream_t st)
{
    // one stage per pass (k = 1)
    if (a.k != 1) return (int)hipErrorInvalidValue;
    if (g.op == FRKC2_OP_BRUSS2) return launch_bruss(g, a, st);
    PlaneArgs pa{};
    pa.in_re = a.in_re;
    pa.in_c = reinterpret_cast<const double2 *>(a.in_c);
    pa.out_re = a.out_re;
    pa.out_c = reinterpret_cast<double2 *>(a.out_c);
    pa.D = a.D;
    pa.nx = g.nx;
    pa.ny = g.ny;
    pa.nz = g.nz;
    pa.inv_h2 = g.inv_h2;
    pa.d_const = g.d_const;
    pa.zchunk = a.zchunk;
    pa.emb_in = a.emb_in;
    pa.emb_out = a.emb_out;
    pa.tr = a.tr[0];
    pa.ti = a.ti[0];
    for (int k = 0; k < 6; ++k) pa.fc[k] = g.fc[k];
    const bool ir = a.in_re != nullptr, orl = a.out_re != nullptr;
    if (g.op == LAP) return launch_plane_bc<LAP>(g, pa, ir, orl, st);
    if (g.op == ADV) return launch_plane_bc<ADV>(g, pa, ir, orl, st);
    if (g.op == VAR) return launch_plane_bc<VAR>(g, pa, ir, orl, st);
    return launch_plane_bc<POR>(g, pa, ir, orl, st);
}

bool stage1d_lds_fits(const KGrid &g) { return g.ndim == 1 && g.nx <= k1dMaxPts; }

namespace {
struct Launch1d {
    const double *w_in;
    double *w_out;              // Re W^L (nsteps supersteps), or
    double2 *out_c;             // ... with emb_out: W^L complex and What^L (one superstep)
    double *emb_out;
    const double *D;
    const double *tau;
    int s, nsteps;
};

template <int OP, int BC, bool EMB>
int launch_1d_t(const KGrid &g, const Launch1d &q, hipStream_t st)
{
    const size_t shm = (size_t)g.nx * (sizeof(double2) + sizeof(double));
    auto kern = stage1d_lds<OP, BC, EMB>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(k1dThreads), shm, st, q.w_in, q.w_out, q.D,
                       reinterpret_cast<const double2 *>(q.tau), g.nx, q.s, q.nsteps, g.inv_h2,
                       g.fc[0], g.fc[1], q.out_c, q.emb_out);
    return (int)hipGetLastError();
}
template <int OP>
int launch_1d_bc(const KGrid &g, const Launch1d &q, hipStream_t st)
{
    if (q.emb_out) {
        if (g.bc == PER) return launch_1d_t<OP, PER, true>(g, q, st);
        return launch_1d_t<OP, DIR, true>(g, q, st);
    }
    if (g.bc == PER) return launch_1d_t<OP, PER, false>(g, q, st);
    return launch_1d_t<OP, DIR, false>(g, q, st);
}
int launch_1d(const KGrid &g, const Launch1d &q, hipStream_t st)
{
    if (!stage1d_lds_fits(g)) return (int)hipErrorInvalidValue;
    if (g.op == LAP) return launch_1d_bc<LAP>(g, q, st);
    if (g.op == ADV) return launch_1d_bc<ADV>(g, q, st);
    if (g.op == VAR) return launch_1d_bc<VAR>(g, q, st);
    return launch_1d_bc<POR>(g, q, st);
}
}  // namespace

int launch_stage1d_lds(const KGrid &g, const double *w_in, double *w_out, const double *D,
                       const double *tau, int s, int nsteps, hipStream_t st)
{
    return launch_1d(g, Launch1d{w_in, w_out, nullptr, nullptr, D, tau, s, nsteps}, st);
}

int launch_stage1d_lds_emb(const KGrid &g, const double *w_in, double *out_c, double *emb_out,
                           const double *D, const double *tau, int s, hipStream_t st)
{
    if (!out_c || !emb_out) return (int)hipErrorInvalidValue;
    return launch_1d(g, Launch1d{w_in, nullptr, reinterpret_cast<double2 *>(out_c), emb_out, D,
                                 tau, s, 1},
                     st);
}

int launch_finalize(const KGrid &g, const double *in_c, double *out_re, double *partials,
                    hipStream_t st)
{
    const long long n = g.nstate();
    hipLaunchKernelGGL(finalize_kernel, dim3(kReduceBlocks), dim3(kFinThreads), 0, st,
                       reinterpret_cast<const double2 *>(in_c), out_re, n, partials);
    hipLaunchKernelGGL(finalize_sum, dim3(1), dim3(256), 0, st, partials, kReduceBlocks);
    return (int)hipGetLastError();
}

int launch_euler_axpy(long long n, double *W, const double *F, double tr, double ti,
                      hipStream_t st, double *emb)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(euler_axpy, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<double2 *>(W), reinterpret_cast<const double2 *>(F), emb,
                       n, tr, ti);
    return (int)hipGetLastError();
}

int launch_real_to_complex(long long n, const double *in, double *out_c, hipStream_t st)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(real_to_complex, dim3((unsigned)blocks), dim3(256), 0, st, in,
                       reinterpret_cast<double2 *>(out_c), n);
    return (int)hipGetLastError();
}

}  // namespace frkc2

namespace frkc2 {
namespace {
__global__ void zero_kernel(double *p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.0;
}
}  // namespace

int launch_zero(long long n, double *p, hipStream_t st)
{
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, st, p, n);
    return (int)hipGetLastError();
}
}  // namespace frkc2
