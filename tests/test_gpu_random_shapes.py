"""Seeded sweep of the fused 3D passes over random grid shapes: both tile widths (64 and 32
output columns), both depths, both boundary conditions, constant and variable coefficients,
automatic and forced chunk lengths, against the oracle bit for bit."""
import numpy as np
import pytest

from oracle import frkc2_coeffs, stage
from paper_1702_03818_amd import frkc2 as F
from paper_1702_03818_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _cases(count=36, seed=2026):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = (int(rng.integers(1, 141)), int(rng.integers(1, 61)), int(rng.integers(1, 31)))
        bc = int(rng.integers(0, 2))
        op = int(rng.integers(0, 2))
        k = int(rng.integers(2, 4))
        tile = int(rng.integers(4, 6))
        zchunk = 0 if rng.random() < 0.5 else int(rng.integers(1, n[2] + 1))
        s = int(rng.choice([4, 8, 16, 34]))
        out.append((i, n, bc, op, k, tile, zchunk, s))
    return out


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()
    yield
    for key in (F.OPT_TBLOCK, F.OPT_TILE, F.OPT_ZCHUNK):
        F.frkc2_set_option(key, 0)
    torch.cuda.synchronize()


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")


@pytest.mark.parametrize("i,n,bc,op,k,tile,zchunk,s", _cases())
def test_random_shape_matches_oracle(i, n, bc, op, k, tile, zchunk, s):
    rng = np.random.default_rng(1000 + i)
    h = 1.0 / (max(n) + (1 if bc == wl.BC_DIRICHLET0 else 0))
    D = wl.lognormal_D(n[::-1], 2.0, rng) if op == wl.OP_VARCOEF else None
    p = wl.Problem(3, n, h, bc, op, 0.7 if op == wl.OP_LAPLACE else 1.0, D)
    p.w0 = wl.random_state(p.shape, 10 + i, smooth=1.0)
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    ref, _ = stage.run(p, s, 2, T=T, coeffs=c)
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    F.frkc2_set_option(F.OPT_TILE, tile)
    F.frkc2_set_option(F.OPT_ZCHUNK, zchunk)
    try:
        w = dev(p.w0)
        F.frkc2_step(p, w, dev(D) if D is not None else None, T=T, s=s, nsteps=2)
        torch.cuda.synchronize()
    finally:
        for key in (F.OPT_TBLOCK, F.OPT_TILE, F.OPT_ZCHUNK):
            F.frkc2_set_option(key, 0)
    got = w.cpu().numpy()
    assert np.isfinite(got).all()
    assert np.array_equal(got, ref), "%d of %d values differ" % (int(np.sum(got != ref)), got.size)


def _store_cases(count=12, seed=2027):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = (int(rng.integers(1, 100)), int(rng.integers(1, 45)), int(rng.integers(1, 25)))
        out.append((i, n, int(rng.integers(0, 2)), int(rng.integers(0, 2)),
                    int(rng.choice([2, 4, 6, 8, 10, 20, 34]))))
    return out


@pytest.mark.parametrize("i,n,bc,op,s", _store_cases())
def test_random_shape_stage_store_and_adjoint(i, n, bc, op, s):
    """Random 3D shapes through the stage store (fused storing passes on ragged tiles) and
    the reverse stages on it: w, lambda and the accumulated D dJ/dD against the oracle."""
    rng = np.random.default_rng(2000 + i)
    h = 1.0 / (max(n) + (1 if bc == wl.BC_DIRICHLET0 else 0))
    D = wl.lognormal_D(n[::-1], 2.0, rng) if op == wl.OP_VARCOEF else None
    p = wl.Problem(3, n, h, bc, op, 0.7 if op == wl.OP_LAPLACE else 1.0, D)
    p.w0 = wl.random_state(p.shape, 30 + i, smooth=1.0)
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tr, ti = T * c.a_re, T * c.a_im
    lam_next = wl.random_state(p.shape, 60 + i).reshape(-1)
    ref_w = stage.superstep(p, p.w0, tr, ti).reshape(-1)
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, tr, ti,
                                   grad_logD=np.zeros(p.npoints) if D is not None else None)
    Dd = dev(D) if D is not None else None
    w = dev(p.w0)
    st = F.stage_store(p, s)
    F.frkc2_step_store(p, w, Dd, T, s, st)
    lam = dev(lam_next)
    g = torch.zeros(p.npoints, dtype=torch.float64, device="cuda") if D is not None else None
    F.frkc2_step_adjoint_stored(p, st, Dd, T, s, lam, lam, g)
    torch.cuda.synchronize()
    what = "case %d n=%s bc=%d op=%d s=%d" % (i, n, bc, op, s)
    assert np.array_equal(w.cpu().numpy(), ref_w), what
    assert np.array_equal(lam.cpu().numpy(), ref_lam), what
    if D is not None:
        assert np.array_equal(g.cpu().numpy(), ref_g), what
