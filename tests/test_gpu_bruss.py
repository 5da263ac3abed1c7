"""GPU parity of the two-species Brusselator (Sec. 3.1): Gershgorin bound, supersteps with the
bound recomputed per superstep, the imaginary-part diagnostic and error-controlled integration,
bit for bit against the oracle."""
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


def test_autotune_keeps_one_stage_passes():
    p = wl.brusselator(64)
    r = F.frkc2_autotune(p, dev(p.w0), None, s=16, reps=1)
    F.frkc2_set_option(F.OPT_CLEAR_TUNED, 0)
    assert r["tblock"] == 1
