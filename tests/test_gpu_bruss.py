"""GPU parity of the two-species Brusselator (Sec. 3.1): Gershgorin bound, supersteps with the
bound recomputed per superstep (one stage per pass and 2..4 fused stages per pass, on square,
non-square and tiny periodic grids that the 64 x 32 tiles wrap around several times), the
imaginary-part diagnostic and error-controlled integration (the embedded solution through the
same fused passes), bit for bit against the oracle."""
import numpy as np
import pytest

from oracle import adaptive, frkc2_coeffs, stage
from paper_1702_03818_amd import frkc2 as F
from paper_1702_03818_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()
    yield
    torch.cuda.synchronize()


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")


def perturbed(n, seed=3):
    p = wl.brusselator(n)
    rng = np.random.default_rng(seed)
    p.w0 = p.w0 + 0.05 * rng.standard_normal(p.w0.shape)
    return p


def rect(nx, ny, seed=7):
    """A non-square periodic Brusselator grid near the steady state (v, w) = (1, 3)."""
    p = wl.Problem(2, (nx, ny, 1), 1.0 / max(nx, ny), wl.BC_PERIODIC, wl.OP_BRUSS2, 0.02)
    p.w0 = np.stack([1.0 + 0.1 * wl.random_state((ny, nx), seed, smooth=1.0),
                     3.0 + 0.1 * wl.random_state((ny, nx), seed + 1, smooth=1.0)])
    return p


@pytest.mark.parametrize("n", [200, 70, 9])
def test_rho_bound(n):
    p = perturbed(n)
    assert F.frkc2_rho_bound(p, dev(p.w0)) == stage.rho_bound(p, p.w0)


@pytest.mark.parametrize("n,s,nsteps", [(200, 16, 3), (200, 100, 2), (70, 16, 3), (9, 8, 4)])
def test_supersteps_match_oracle(n, s, nsteps):
    p = perturbed(n)
    c = frkc2_coeffs(s, 0.01)
    ref, Ts = stage.run(p, s, nsteps, cfl=0.9, coeffs=c)
    w = dev(p.w0)
    st = F.frkc2_step(p, w, None, cfl=0.9, s=s, nsteps=nsteps, stats=True)
    assert st["T_last"] == Ts[-1]
    got = w.cpu().numpy()
    assert np.array_equal(got, ref), "%d values differ" % int(np.sum(got != ref))


def test_imaginary_part_diagnostic():
    p = wl.brusselator(64)
    c = frkc2_coeffs(16, 0.01)
    rho = stage.rho_bound(p, p.w0)
    T = 0.5 * c.beta_bar / rho
    wr, wi = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im, want_imag=True)
    w = dev(p.w0)
    st = F.frkc2_step(p, w, None, T=T, s=16, nsteps=1, stats=True)
    ref = float(np.sqrt(np.sum(wi * wi) / np.sum(wr * wr + wi * wi)))
    assert abs(st["im_ratio"] - ref) <= 1e-10 * ref + 1e-300


def test_integrate_matches_oracle():
    """Error control on the paper's 200 x 200 problem from its initial data."""
    p = wl.brusselator(200)
    t_span, T0, tol = 0.5, 0.05, 1e-4
    w_ref, trace_ref, T_ref = adaptive.integrate(p, t_span, T0, tol)
    w = dev(p.w0)
    st, trace = F.frkc2_integrate(p, w, None, t_span=t_span, T0=T0, tol=tol,
                                  trace_cap=len(trace_ref) + 4)
    torch.cuda.synchronize()
    assert np.array_equal(trace, np.array(trace_ref))
    assert st["T_next"] == T_ref
    assert np.array_equal(w.cpu().numpy(), w_ref)


@pytest.mark.parametrize("grid,k", [((57, 131), 2), ((131, 57), 3), ((64, 40), 4), ((5, 3), 4),
                                    ((200, 200), 1), ((57, 131), 6), ((90, 33), 5)])
def test_integrate_fused_depths_match_oracle(grid, k):
    """Error control with the embedded solution carried through fused passes of k stages
    (k = 1: one stage per pass), on non-square and tiny periodic grids."""
    p = rect(*grid)
    t_span, T0, tol = 1.0, 0.05, 1e-2      # steps of s = 4 .. 70 stages
    w_ref, trace_ref, T_ref = adaptive.integrate(p, t_span, T0, tol)
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    try:
        w = dev(p.w0)
        st, trace = F.frkc2_integrate(p, w, None, t_span=t_span, T0=T0, tol=tol,
                                      trace_cap=len(trace_ref) + 4)
        torch.cuda.synchronize()
    finally:
        F.frkc2_set_option(F.OPT_TBLOCK, 0)
    assert np.array_equal(trace, np.array(trace_ref))
    assert st["T_next"] == T_ref
    assert np.array_equal(w.cpu().numpy(), w_ref)


def test_rho_bound_non_square():
    p = rect(57, 131)
    assert F.frkc2_rho_bound(p, dev(p.w0)) == stage.rho_bound(p, p.w0)


# (grid, s, fused depth, cfl or None for a fixed T = 0.05)
FUSED = [((200, 200), 16, 2, 0.9), ((200, 200), 16, 3, 0.9), ((200, 200), 16, 4, 0.9),
         ((200, 200), 18, 4, 0.9), ((200, 200), 34, 3, 0.9), ((70, 70), 50, 4, 0.5),
         ((57, 131), 18, 3, 0.9), ((131, 57), 22, 4, 0.9), ((512, 512), 16, 4, 0.9),
         ((512, 512), 14, 2, 0.9), ((5, 3), 8, 4, None), ((1, 1), 6, 3, None),
         ((64, 1), 8, 4, None), ((1, 40), 10, 2, None), ((200, 200), 18, 5, 0.9),
         ((131, 57), 22, 6, 0.9), ((5, 3), 12, 6, None), ((300, 77), 16, 5, 0.9)]


@pytest.mark.parametrize("grid,s,k,cfl", FUSED)
def test_fused_passes_match_oracle(grid, s, k, cfl):
    """Fused passes of k stages, the remainder of s as the library schedules it (one fused pass
    of the remaining depth, else single stages), three supersteps."""
    p = perturbed(grid[0]) if grid[0] == grid[1] and grid[0] >= 64 else rect(*grid)
    c = frkc2_coeffs(s, 0.01)
    if cfl is None:
        ref, _ = stage.run(p, s, 3, T=0.05, coeffs=c)
    else:
        ref, Ts = stage.run(p, s, 3, cfl=cfl, coeffs=c)
    assert np.isfinite(ref).all()
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    try:
        w = dev(p.w0)
        if cfl is None:
            F.frkc2_step(p, w, None, T=0.05, s=s, nsteps=3)
        else:
            st = F.frkc2_step(p, w, None, cfl=cfl, s=s, nsteps=3, stats=True)
            assert st["T_last"] == Ts[-1]
        torch.cuda.synchronize()
    finally:
        F.frkc2_set_option(F.OPT_TBLOCK, 0)
    got = w.cpu().numpy()
    assert np.array_equal(got, ref), "%d of %d values differ" % (int(np.sum(got != ref)), got.size)


def test_default_depth_matches_oracle():
    """No option set: the automatic depth (four stages per pass) on a ragged grid."""
    p = rect(300, 77)
    c = frkc2_coeffs(40, 0.01)
    ref, _ = stage.run(p, 40, 2, cfl=0.9, coeffs=c)
    w = dev(p.w0)
    F.frkc2_step(p, w, None, cfl=0.9, s=40, nsteps=2)
    torch.cuda.synchronize()
    assert np.array_equal(w.cpu().numpy(), ref)


def test_autotune_picks_a_supported_depth():
    p = perturbed(128)
    r = F.frkc2_autotune(p, dev(p.w0), None, s=16, reps=1)
    try:
        assert r["tblock"] in (1, 2, 3, 4, 5, 6)
        c = frkc2_coeffs(16, 0.01)
        ref, _ = stage.run(p, 16, 2, cfl=0.9, coeffs=c)
        w = dev(p.w0)
        F.frkc2_step(p, w, None, cfl=0.9, s=16, nsteps=2)   # runs the tuned configuration
        torch.cuda.synchronize()
        assert np.array_equal(w.cpu().numpy(), ref)
    finally:
        F.frkc2_set_option(F.OPT_CLEAR_TUNED, 0)
