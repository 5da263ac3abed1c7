"""GPU parity of the error-controlled integration (Sec. 3): every attempt (start time, T, s,
error estimate, accept flag), the proposed next T and the final state equal the oracle's
bit for bit, with the embedded solution in one-stage passes and in fused 3D and 2D passes."""
import numpy as np
import pytest

from oracle import adaptive, stage
from paper_1702_03818_amd import frkc2 as F
from paper_1702_03818_amd import workloads as wl

from test_gpu_parity import dev, host, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()
    yield
    torch.cuda.synchronize()


def run_both(p, t_span, T0, tol):
    w_ref, trace_ref, T_ref = adaptive.integrate(p, t_span, T0, tol)
    w = dev(p.w0)
    D = dev(p.D) if p.D is not None else None
    st, trace = F.frkc2_integrate(p, w, D, t_span=t_span, T0=T0, tol=tol,
                                  trace_cap=len(trace_ref) + 8)
    torch.cuda.synchronize()
    ref = np.array(trace_ref, dtype=np.float64)
    assert st["attempts"] == len(trace_ref)
    assert st["accepted"] == int(ref[:, 4].sum())
    assert np.array_equal(trace, ref), "first difference at attempt %d" % int(
        np.argmax(np.any(trace != ref, axis=1)))
    assert st["T_next"] == T_ref
    assert st["t"] == t_span
    got = host(w)
    assert np.array_equal(got, w_ref), "%d values differ" % int(np.sum(got != w_ref))
    return st, ref


@pytest.mark.parametrize("kind,n", [("3d-var-dir", (70, 37, 21)), ("2d-por-per", (64, 64, 1)),
                                    ("2d-var-dir", (300, 37, 1)), ("1d-lap-per", (1024, 1, 1)),
                                    ("3d-lap-per", (65, 5, 12)), ("3d-var-per", (67, 6, 10)),
                                    ("3d-por-dir", (70, 37, 21)), ("3d-por-per", (67, 30, 18))])
def test_integrate_matches_oracle(kind, n):
    p = problem(kind, n)
    span, T0 = 1500.0, 800.0
    if p.ndim == 3 and p.op == wl.OP_POROUS2:
        # the complex stages of the 3D porous medium diverge from T rho of about 800
        p.w0 = 1.0 + 0.4 * p.w0 / np.max(np.abs(p.w0))
        span, T0 = 600.0, 200.0
    rho = stage.rho_bound(p, p.w0)
    st, ref = run_both(p, span / rho, T0 / rho, 1e-3)
    assert (ref[:, 4] == 0).any(), "the first, long attempt should be rejected"


def test_integrate_heat1d_many_steps():
    p = wl.heat1d()
    st, ref = run_both(p, 2e-3, 1e-5, 1e-5)
    assert st["accepted"] > 200


def test_integrate_zero_state():
    """All-zero state: the error estimate is 0 and the controller grows T by its cap."""
    p = problem("2d-var-dir", (64, 9, 1))
    p.w0 = np.zeros_like(p.w0)
    rho = stage.rho_bound(p, p.w0)
    st, ref = run_both(p, 100.0 / rho, 1.0 / rho, 1e-3)
    assert (ref[:, 3] == 0).all()


@pytest.mark.parametrize("k,tile,zchunk", [(1, 0, 0), (2, 4, 0), (3, 4, 0), (2, 4, 5), (3, 4, 7),
                                          (2, 1, 0), (3, 5, 0), (2, 5, 6)])
def test_integrate_launch_configurations(k, tile, zchunk):
    """The embedded solution in fused 3D passes (K = 2, 3, chunk lengths) and one stage per
    pass gives the same attempts and state."""
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    F.frkc2_set_option(F.OPT_TILE, tile)
    F.frkc2_set_option(F.OPT_ZCHUNK, zchunk)
    try:
        p = problem("3d-var-dir", (70, 37, 21))
        rho = stage.rho_bound(p, p.w0)
        run_both(p, 1500.0 / rho, 800.0 / rho, 1e-3)
        p = problem("3d-lap-per", (65, 5, 12))
        rho = stage.rho_bound(p, p.w0)
        run_both(p, 1500.0 / rho, 800.0 / rho, 1e-3)
        p = problem("3d-por-dir", (70, 37, 21))
        p.w0 = 1.0 + 0.4 * p.w0 / np.max(np.abs(p.w0))
        rho = stage.rho_bound(p, p.w0)
        run_both(p, 600.0 / rho, 200.0 / rho, 1e-3)
    finally:
        F.frkc2_set_option(F.OPT_TBLOCK, 0)
        F.frkc2_set_option(F.OPT_TILE, 0)
        F.frkc2_set_option(F.OPT_ZCHUNK, 0)


@pytest.mark.parametrize("k,tile,zchunk", [(2, 1, 0), (3, 1, 0), (4, 1, 0), (4, 1, 9), (4, 2, 0),
                                          (6, 1, 0), (1, 0, 0)])
def test_integrate_2d_launch_configurations(k, tile, zchunk):
    """The embedded solution in fused 2D rows of 256 (K = 2..4, a forced chunk length); rows
    of 512 and K = 6 fall back to one-stage embedded passes. Every 2D operator, both
    boundaries, ragged sizes."""
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    F.frkc2_set_option(F.OPT_TILE, tile)
    F.frkc2_set_option(F.OPT_ZCHUNK, zchunk)
    try:
        # (kind, grid, t_span and first T in units of 1/rho)
        for kind, n, span, T0 in (("2d-por-per", (64, 64, 1), 1500.0, 800.0),
                                  ("2d-var-dir", (300, 37, 1), 1500.0, 800.0),
                                  ("2d-lap-per", (517, 23, 1), 1500.0, 800.0),
                                  ("2d-por-dir", (41, 90, 1), 300.0, 50.0),
                                  ("2d-var-per", (3, 250, 1), 1500.0, 800.0)):
            p = problem(kind, n)
            if p.op == wl.OP_POROUS2:
                p.w0 = 1.0 + 0.4 * p.w0 / np.max(np.abs(p.w0))
            rho = stage.rho_bound(p, p.w0)
            run_both(p, span / rho, T0 / rho, 1e-3)
    finally:
        F.frkc2_set_option(F.OPT_TBLOCK, 0)
        F.frkc2_set_option(F.OPT_TILE, 0)
        F.frkc2_set_option(F.OPT_ZCHUNK, 0)


@pytest.mark.parametrize("kind,n", [("1d-lap-per", (4096, 1, 1)), ("1d-var-dir", (777, 1, 1)),
                                    ("1d-por-per", (300, 1, 1)), ("1d-lap-per", (1, 1, 1)),
                                    ("1d-var-dir", (5000, 1, 1))])
def test_integrate_1d(kind, n):
    """1D grids that fit in LDS run each attempt's superstep, embedded solution included, in
    one launch; a grid of 5000 points runs one pass per stage. Same attempts and state."""
    p = problem(kind, n)
    if p.op == wl.OP_POROUS2:
        p.w0 = 1.0 + 0.4 * p.w0 / np.max(np.abs(p.w0))
    rho = stage.rho_bound(p, p.w0)
    run_both(p, 1500.0 / rho, 800.0 / rho, 1e-3)
