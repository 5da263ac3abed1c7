// Internal declarations shared by the host and kernel translation units of
// libfrkc2. Not part of the public ABI.
#pragma once

#include <cstddef>
#include <cstdint>

#include "../../include/frkc2.h"

namespace frkc2 {

constexpr int kMaxStages = 514;     // M <= 257 (the paper's table range)
constexpr int kMaxTBlock = 8;       // stages fused into one HBM pass

void set_error(const char *fmt, ...);

// Cached ordered stepsizes (host pointers valid for the process lifetime).
int coeffs_cached(int s, double nu, const double **re, const double **im, frkc2_coeff_info *info);
// ... of the fourth-order polynomial (s = 4M stages; info.mu_re holds alpha_M).
constexpr int kMaxStages4 = 512;
int coeffs4_cached(int s, double nu, const double **re, const double **im, frkc2_coeff_info *info);

// Grid description as the kernels see it. For ndim = 1 and 2 the last used
// dimension is the "march" dimension: (nx, ny, nz) = (n0, 1, 1) in 1D,
// (n0, 1, n1) in 2D and (n0, n1, n2) in 3D, so that index = x + nx*(y + ny*z)
// equals the public flat index in every case.
struct KGrid {
    int ndim, nx, ny, nz;
    int bc, op;
    int nfield;                 // values per point: 2 for the Brusselator (v, then w)
    double inv_h2, d_const;
    double fc[6];               // face coefficients in kernel order x-, x+, y-, y+, z-, z+
                                // (d_const, or d -+ v h/2 for ADVDIFF)
    double fcg[6];              // the same in grid order (dimension 0, 1, 2 of the caller)
    long long npts() const { return (long long)nx * ny * nz; }
    long long nstate() const { return nfield * npts(); }
};

bool make_kgrid(const frkc2_grid *g, KGrid &k);

// frkc2_step's argument checks (no HIP call), frkc2_step on a given workspace
// (api.cpp), and the workspace it needs for a state of nstate values.
int step_validate(const frkc2_grid *g, const double *w, const double *D, double T, double cfl,
                  int s, double nu, int nsteps, KGrid &kg);
int step_core(const frkc2_grid *g, double *w, const double *D, double T, double cfl, int s,
              double nu, int nsteps, void *ws, size_t ws_bytes, hipStream_t st,
              frkc2_step_stats *stats);
size_t step_workspace_bytes(long long nstate);

// One pass of k consecutive stages over the whole grid.
struct PassArgs {
    const double *in_re;        // real input (first pass) or nullptr
    const double *in_c;         // complex input, interleaved (re, im), or nullptr
    double *out_re;             // real output (last pass) or nullptr
    double *out_c;              // complex output, interleaved, or nullptr
    const double *D;            // diffusivity (VARCOEF) or nullptr
    double tr[kMaxTBlock];      // tau_l = T a_l of the pass's stages
    double ti[kMaxTBlock];
    int k;                      // stages in this pass
    int zchunk;                 // z planes per workgroup (0: automatic)
    const double *emb_in;       // embedded first-order solution in (not the first stage)
    double *emb_out;            // ... and out; non-null selects the embedded variant (k = 1)
    double *lvl_out;            // 3D fused passes: levels 1..k-1 also written to
    long long lvl_stride;       // lvl_out + (m-1)*lvl_stride complex values (non-null selects it)
    int cols;                   // 3D fused passes: output columns per tile, 64 (0) or 32
    int rev;                    // 3D full-width fused passes: march each chunk downwards
                                // (same bits; alternate passes reuse the cached planes)
};

// Launchers (stage.hip). Return hipError_t as int.
int launch_pass(const KGrid &g, const PassArgs &a, int tblock_hint, hipStream_t st);
int launch_stage1d_lds(const KGrid &g, const double *w_in, double *w_out, const double *D,
                       const double *tau, int s, int nsteps, hipStream_t st);
bool stage1d_lds_fits(const KGrid &g);
// One superstep with the embedded solution: W^L (complex) to out_c, What^L to emb_out.
int launch_stage1d_lds_emb(const KGrid &g, const double *w_in, double *out_c, double *emb_out,
                           const double *D, const double *tau, int s, hipStream_t st);
int launch_finalize(const KGrid &g, const double *in_c, double *out_re, double *partials,
                    hipStream_t st);
int launch_real_to_complex(long long n, const double *in, double *out_c, hipStream_t st);
// W <- W + tau F (complex, interleaved); emb, if given, <- emb + Re tau Re F
int launch_euler_axpy(long long n, double *W, const double *F, double tr, double ti,
                      hipStream_t st, double *emb = nullptr);
int launch_zero(long long n, double *p, hipStream_t st);   // fill kernel (graph-safe)

// Two-species Brusselator (bruss.hip): one stage per pass, or p.k = 2..4
// stages per pass (no embedded variant); reaction part of the Gershgorin
// bound into partials[kReduceBlocks].
int launch_bruss(const KGrid &g, const PassArgs &p, hipStream_t st);
int launch_bruss_tb(const KGrid &g, const PassArgs &p, hipStream_t st);
int launch_bruss_react_max(const KGrid &g, const double *w, double *partials, hipStream_t st);
int launch_max_partials(double *partials, hipStream_t st);   // max of kReduceBlocks partials

// Temporally blocked passes (tblock.hip): p.k stages in one HBM pass.
bool tblock_supported(const KGrid &g, int k);
// ... and with the embedded solution (p.emb_out): 3D full-width tiles
// (launch_tb3d), the Brusselator, 2D rows of 256 with k = 2..4.
bool tblock_emb_supported(const KGrid &g, int k, int shape);
int launch_tblock(const KGrid &g, const PassArgs &p, int shape, hipStream_t st);
// 3D passes with 64-column output tiles and halo wavefronts (tb3d.hip), k = 2, 3.
int launch_tb3d(const KGrid &g, const PassArgs &p, hipStream_t st);
// The full-width 3D tile addresses a plane with 32-bit byte offsets: planes
// of fewer than 2^27 points (other grids take the other 3D tiles).
bool tb3d_plane_ok(const KGrid &g);
// Output columns (64 or 32) of the fused 3D tile with the lower predicted
// pass time on this grid (rounds of workgroups x steps x step cost).
int tb3d_pick_cols(const KGrid &g, int k);
// Steps x step cost of all fused-tile items of one batched 3D problem.
long long tb3d_work(int k, int cols, int nx, int ny, int nz, int zc);

// Reductions (reduce.hip). partials must hold kReduceBlocks doubles + 2.
constexpr int kReduceBlocks = 512;
int launch_reduce(int op, const double *x, const double *y, long long n, double *partials,
                  hipStream_t st);
int launch_rho(const KGrid &g, const double *w, const double *D, double *partials, hipStream_t st);
// Embedded-pair error estimate: max over points into partials[kReduceBlocks].
int launch_err_max(const double *Wc, const double *E, long long n, double tol, double *partials,
                   hipStream_t st);
int launch_take_real(const double *Wc, double *w, long long n, hipStream_t st);

// Brusselator reaction flow over a complex time (frkc4.hip), in place on the
// complex state (v then w, n points each); c = {c, c/2, c/6} as (re, im) pairs,
// c = tau / nsub.
int launch_react_flow(double *Zc, long long n, const double c[6], int nsub, hipStream_t st);

// Adjoint (adjoint.hip).
struct AdjArgs {
    const double *lam_in_re;    // real lambda (first reverse stage) or nullptr
    const double *lam_in_c;     // complex lambda^{l+1}
    double *lam_out_re;         // real lambda^0 (last reverse stage) or nullptr
    double *lam_out_c;          // complex lambda^l
    const double *W;            // stored complex stage W^l
    const double *D;
    double *gD;                 // per-cell dJ/dD accumulator (VARCOEF) or nullptr
    double tr, ti;
};
int launch_adjoint_stage(const KGrid &g, const AdjArgs &a, hipStream_t st);
// Reverse stages a1 (stage l) then a2 (stage l-1) in one pass, 3D LAPLACE or
// VARCOEF: lam in from a1, lam out to a2 (they must not alias), W^l = a1.W,
// W^{l-1} = a2.W, D and gD from a1.
int launch_adjoint_pair(const KGrid &g, const AdjArgs &a1, const AdjArgs &a2, hipStream_t st);
int launch_grad_finish(long long n, const double *D, const double *gD, double *grad_logD,
                       hipStream_t st);

// Batched engine (batched.hip, batched_host.cpp).
struct BatchProblem {           // one problem's descriptor in device memory
    double *w;                  // caller state (real)
    const double *D;
    double *bufA, *bufB;        // complex ping-pong buffers in the workspace
    const double *tau;          // 2*s doubles (re, im interleaved)
    int nx, ny, nz, ndim, bc, op;   // kernel layout: 3D (n0, n1, n2), 2D (n0, 1, n1)
    int s, ntiles;                  // stages, tiles per one-stage pass
    int zchunk, ntx, nty;           // one-stage tile grid: ntx * nty * ceil(nz / zchunk)
    int nfull, npass;               // fused passes of k3 (3D) / k2 (2D) stages, then single stages
    int zc3, ntx3, nty3, ntiles3;   // fused-pass tile grid (3D: full-width tiles; 2D: rows)
    int cols3;                      // 3D: its output columns per tile (64 or 32)
    double inv_h2, d_const;
};
// Launch configuration of a batch: stages per fused 3D pass (2, 3), output
// columns of the fused 3D tiles (32, 64, or kColsPerProblem), stages per fused
// 2D pass (2, 3, 4, 6). Every configuration gives the same bits.
constexpr int kColsPerProblem = 1;  // BatchCfg::cols3: each 3D problem its modelled width
struct BatchCfg {
    int k3 = 3, cols3 = 64, k2 = 4;
};
bool batched_cfg_supported(int k3, int cols3, int k2);
void batched_tile(int ndim, int *bx, int *by);
void batched_tile3(int cols, int k, int *bx, int *by);
int batched_row2(int k);            // output columns of a fused 2D row item of k stages
int batched_grid_size(int ndim);
// 2D pass level: fused == true runs the k-stage passes of level `level`,
// otherwise the single-stage passes; item_prefix spans all nprob 2D problems.
int launch_batched_pass2(bool fused, int k, const BatchProblem *probs,
                         const long long *item_prefix, long long items, int nprob, int level,
                         int grid, hipStream_t st);
// 3D pass level: fused == true runs the k-stage passes (cols output columns)
// of level `level`, otherwise the single-stage passes; item_prefix spans all
// nprob 3D problems.
int launch_batched_pass3(bool fused, int cols, int k, const BatchProblem *probs,
                         const long long *item_prefix, long long items, int nprob, int level,
                         int grid, hipStream_t st);
// frkc2_set_option's batch keys (FRKC2_OPT_BATCH_*: a configuration forced
// for every batch, 0 = automatic), and forgetting what frkc2_batched_autotune
// stored.
int batched_set_option(int key, int value);
void batched_clear_tuned();

}  // namespace frkc2
