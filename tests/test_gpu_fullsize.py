"""Full-size parity: the configurations the benchmark and the paper-scale workloads use,
compared with the CPU oracle on one superstep (or on sampled problems of the batch), in
the launch configuration bench.py times (default block depth and tiles)."""
import numpy as np
import pytest

from oracle import frkc2_coeffs, stage
from paper_1702_03818_amd import frkc2 as F
from paper_1702_03818_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()
    F.frkc2_set_option(F.OPT_TBLOCK, 0)
    yield
    F.release_workspaces()


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")


def check(got, ref, what):
    r = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert np.isfinite(got).all(), what
    assert r <= 1e-12, "%s: rel L2 %.3e" % (what, r)
    assert np.array_equal(got, ref), "%s: %d values differ (rel %.2e)" % (
        what, int(np.sum(got != ref)), r)


@pytest.fixture(scope="module")
def c2_reference():
    p = wl.diffusion3d()
    c = frkc2_coeffs(100, 0.01)
    rho = stage.rho_bound(p)
    T = 0.9 * c.beta_bar / rho
    return p, c, rho, T, stage.superstep(p, p.w0, T * c.a_re, T * c.a_im)


@pytest.mark.parametrize("k,tile,zchunk", [(0, 0, 0), (2, 4, 32), (3, 4, 128), (2, 1, 0),
                                          (3, 5, 0)])
def test_diffusion3d_256_superstep(c2_reference, k, tile, zchunk):
    """256^3 variable D, Dirichlet, s = 100 (the benchmark workload) in the launch
    configurations the benchmark's autotuner chooses between."""
    p, c, rho, T, ref = c2_reference
    w = dev(p.w0)
    D = dev(p.D)
    assert F.frkc2_rho_bound(p, None, D) == rho
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    F.frkc2_set_option(F.OPT_TILE, tile)
    F.frkc2_set_option(F.OPT_ZCHUNK, zchunk)
    try:
        F.frkc2_step(p, w, D, T=T, s=100, nsteps=1)
    finally:
        F.frkc2_set_option(F.OPT_TBLOCK, 0)
        F.frkc2_set_option(F.OPT_TILE, 0)
        F.frkc2_set_option(F.OPT_ZCHUNK, 0)
    check(w.cpu().numpy(), ref, "3D 256^3 s=100 k=%d tile=%d zchunk=%d" % (k, tile, zchunk))


def test_diffusion3d_256_ten_supersteps_contract():
    """The timed 10 supersteps: every superstep contracts the L2 norm (|R| <= 1 on the
    spectrum of the symmetric operator) and the imaginary part of W^L stays at roundoff."""
    p = wl.diffusion3d()
    c = frkc2_coeffs(100, 0.01)
    D = dev(p.D)
    T = 0.9 * c.beta_bar / F.frkc2_rho_bound(p, None, D)
    w = dev(p.w0)
    prev = float(torch.linalg.vector_norm(w))
    for _ in range(10):
        st = F.frkc2_step(p, w, D, T=T, s=100, nsteps=1, stats=True)
        now = float(torch.linalg.vector_norm(w))
        assert now <= prev * (1 + 1e-14)
        assert st["im_ratio"] < 1e-12
        prev = now


def test_porous2d_4096_superstep():
    """4096^2 div(u^2 grad u), periodic, s = 400, adaptive T at the stable cfl."""
    p = wl.porous2d()
    c = frkc2_coeffs(400, 0.01)
    cfl = 0.002
    ref, Ts = stage.run(p, 400, 1, cfl=cfl, coeffs=c)
    w = dev(p.w0)
    st = F.frkc2_step(p, w, None, cfl=cfl, s=400, nsteps=1, stats=True)
    assert st["T_last"] == Ts[0]
    check(w.cpu().numpy(), ref, "2D porous 4096^2 s=400")


def test_heat1d_20_supersteps():
    p = wl.heat1d()
    c = frkc2_coeffs(16, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    ref, _ = stage.run(p, 16, 20, T=T, coeffs=c)
    w = dev(p.w0)
    F.frkc2_step(p, w, None, T=T, s=16, nsteps=20)
    check(w.cpu().numpy(), ref, "1D heat")


def test_batched_512_sampled():
    """The 512-problem batch: every problem equals the plain path bit for bit, and a seeded
    sample of six problems (the largest 3D one among them) equals the oracle."""
    probs = wl.batched()
    ws_list, D_list, T_list, s_list = [], [], [], []
    for p, s in probs:
        D = dev(p.D)
        c = F.frkc2_coeffs(s, 0.01)[2]
        T_list.append(0.9 * c["beta_bar"] / F.frkc2_rho_bound(p, None, D))
        ws_list.append(dev(p.w0))
        D_list.append(D)
        s_list.append(s)
    args = F.BatchedArgs([p for p, _ in probs], ws_list, D_list, T_list, s_list)
    F.frkc2_step_batched(args)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2024)
    big = max(range(len(probs)), key=lambda i: probs[i][0].npoints * (probs[i][0].ndim == 3))
    sample = set(rng.choice(len(probs), 5, replace=False).tolist()) | {big}
    for i, ((p, s), wb, D, T) in enumerate(zip(probs, ws_list, D_list, T_list)):
        w = dev(p.w0)
        F.frkc2_step(p, w, D, T=T, s=s, nsteps=1)
        assert torch.equal(w, wb), "problem %d (%s, s=%d)" % (i, p.n, s)
        if i in sample:
            c = frkc2_coeffs(s, 0.01)
            ref = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im)
            check(wb.cpu().numpy(), ref, "batched problem %d %s s=%d" % (i, p.n, s))
    F.frkc2_batched_release()


def test_adjoint_128_superstep():
    """128^3 adjoint configuration (s = 64): one superstep's adjoint equals the oracle's."""
    p, target = wl.adjoint3d()
    s = 64
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    lam_next = 2.0 * (p.w0.reshape(-1) - target.reshape(-1))
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, T * c.a_re, T * c.a_im)
    lam_n = torch.empty(p.npoints, dtype=torch.float64, device="cuda")
    g = torch.zeros(p.npoints, dtype=torch.float64, device="cuda")
    F.frkc2_step_adjoint(p, dev(p.w0), dev(p.D), T, s, dev(lam_next), lam_n, g)
    torch.cuda.synchronize()
    check(lam_n.cpu().numpy(), ref_lam, "adjoint lambda 128^3")
    gg = g.cpu().numpy()
    assert np.linalg.norm(gg - ref_g) <= 1e-12 * np.linalg.norm(ref_g)


def test_adjoint_128_stage_store():
    """128^3 adjoint configuration (s = 64) through the stage store, as the autograd function
    runs it there: the forward superstep equals the oracle's, and the reverse stages on the
    store equal the oracle's adjoint."""
    p, target = wl.adjoint3d()
    s = 64
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    w = dev(p.w0)
    D = dev(p.D)
    st = F.stage_store(p, s)
    F.frkc2_step_store(p, w, D, T, s, st)
    torch.cuda.synchronize()
    ref_w = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im).reshape(-1)
    check(w.cpu().numpy(), ref_w, "stage-store forward 128^3")
    lam_next = 2.0 * (ref_w - target.reshape(-1))
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, T * c.a_re, T * c.a_im)
    lam_n = torch.empty(p.npoints, dtype=torch.float64, device="cuda")
    g = torch.zeros(p.npoints, dtype=torch.float64, device="cuda")
    F.frkc2_step_adjoint_stored(p, st, D, T, s, dev(lam_next), lam_n, g)
    torch.cuda.synchronize()
    check(lam_n.cpu().numpy(), ref_lam, "stored adjoint lambda 128^3")
    gg = g.cpu().numpy()
    assert np.linalg.norm(gg - ref_g) <= 1e-12 * np.linalg.norm(ref_g)
    del st


def test_integrate_256(c2_reference):
    """Error-controlled integration on the benchmark grid (fused embedded passes, default
    configuration) over three superstep lengths: every attempt and the state equal the
    oracle's."""
    from oracle import adaptive
    p, c, rho, T, _ = c2_reference
    span = 3 * T
    w_ref, trace_ref, T_ref = adaptive.integrate(p, span, T, 1e-3)
    w = dev(p.w0)
    st, trace = F.frkc2_integrate(p, w, dev(p.D), t_span=span, T0=T, tol=1e-3,
                                  trace_cap=len(trace_ref) + 4)
    torch.cuda.synchronize()
    assert np.array_equal(trace, np.array(trace_ref))
    assert st["T_next"] == T_ref
    check(w.cpu().numpy(), w_ref, "integrate 256^3")
