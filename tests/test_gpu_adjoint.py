"""GPU adjoint: frkc2_step_adjoint against the oracle adjoint, and the autograd
wrapper against central finite differences of the GPU forward."""
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
    yield


def dev(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _prob(kind):
    rng = np.random.default_rng(3)
    if kind == "3d-var-dir":
        p = wl.diffusion3d(n_xyz=(70, 13, 11), nblobs=2)
    elif kind == "3d-var-per":
        p = wl.Problem(3, (20, 9, 6), 1.0 / 20, wl.BC_PERIODIC, wl.OP_VARCOEF, 1.0,
                       wl.lognormal_D((6, 9, 20), 2.0, rng))
    elif kind == "2d-var-dir":
        p = wl.Problem(2, (260, 17, 1), 1.0 / 261, wl.BC_DIRICHLET0, wl.OP_VARCOEF, 1.0,
                       wl.lognormal_D((17, 260), 3.0, rng))
    elif kind == "3d-lap-dir":
        p = wl.Problem(3, (30, 10, 7), 1.0 / 31, wl.BC_DIRICHLET0, wl.OP_LAPLACE, 0.7)
    p.w0 = wl.random_state(p.shape, 5, smooth=1.5)
    return p


@pytest.mark.parametrize("kind", ["3d-var-dir", "3d-var-per", "2d-var-dir", "3d-lap-dir"])
@pytest.mark.parametrize("s", [2, 6, 8, 16, 64, 512, 514])   # 3D: 3-stage forward passes + 0..2 single
def test_adjoint_matches_oracle(kind, s):
    p = _prob(kind)
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    lam_next = wl.random_state(p.shape, 9).reshape(-1)
    g0 = wl.random_state(p.shape, 10).reshape(-1)
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, T * c.a_re, T * c.a_im,
                                   grad_logD=g0.copy() if p.D is not None else None)
    lam_n = torch.empty(p.npoints, dtype=torch.float64, device="cuda")
    g = dev(g0) if p.D is not None else None
    D = dev(p.D) if p.D is not None else None
    F.frkc2_step_adjoint(p, dev(p.w0), D, T, s, dev(lam_next), lam_n, g)
    torch.cuda.synchronize()
    got = host(lam_n)
    assert np.array_equal(got, ref_lam), "lambda differs: rel %.3e" % (
        np.linalg.norm(got - ref_lam) / np.linalg.norm(ref_lam))
    if p.D is not None:
        gg = host(g)
        r = np.linalg.norm(gg - ref_g) / np.linalg.norm(ref_g)
        assert r <= 1e-12, r
        assert np.array_equal(gg, ref_g)


def _pair_prob(n, bc, op, seed):
    rng = np.random.default_rng(seed)
    h = 1.0 / (n[0] + (1 if bc == wl.BC_DIRICHLET0 else 0))
    D = wl.lognormal_D(n[::-1], 2.0, rng) if op == wl.OP_VARCOEF else None
    p = wl.Problem(3, n, h, bc, op, 1.0 if op == wl.OP_VARCOEF else 0.6, D)
    p.w0 = wl.random_state(p.shape, seed + 1, smooth=1.0)
    return p


@pytest.mark.parametrize("n", [(70, 50, 37), (33, 25, 3), (5, 3, 2), (1, 1, 9), (64, 17, 130)])
@pytest.mark.parametrize("bc", [wl.BC_DIRICHLET0, wl.BC_PERIODIC])
@pytest.mark.parametrize("op", [wl.OP_VARCOEF, wl.OP_LAPLACE])
@pytest.mark.parametrize("s", [2, 4, 16])
def test_reverse_pairs_match_oracle(n, bc, op, s):
    """Two reverse stages per pass (an option on 3D grids) and one per pass: both give the
    oracle's lambda and dJ/dD bit for bit, on ragged shapes over several tiles and z chunks."""
    p = _pair_prob(n, bc, op, 11)
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    lam_next = wl.random_state(p.shape, 12).reshape(-1)
    g0 = wl.random_state(p.shape, 13).reshape(-1)
    vc = p.D is not None
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, T * c.a_re, T * c.a_im,
                                   grad_logD=g0.copy() if vc else None)
    D = dev(p.D) if vc else None
    try:
        for k in (2, 1):
            F.frkc2_set_option(F.OPT_ADJ_STAGES, k)
            lam_n = torch.empty(p.npoints, dtype=torch.float64, device="cuda")
            g = dev(g0) if vc else None
            F.frkc2_step_adjoint(p, dev(p.w0), D, T, s, dev(lam_next), lam_n, g)
            torch.cuda.synchronize()
            got = host(lam_n)
            assert np.array_equal(got, ref_lam), "k=%d: %d lambda values differ" % (
                k, int(np.sum(got != ref_lam)))
            if vc:
                assert np.array_equal(host(g), ref_g), "k=%d: dJ/dD differs" % k
    finally:
        F.frkc2_set_option(F.OPT_ADJ_STAGES, 0)


def test_reverse_pair_with_aliased_lambda():
    """s = 2 with lam_n the same buffer as lam_next (allowed), two reverse stages per pass
    requested: that pass would read and write one buffer, so the library runs the two stages
    apart; the result is the oracle's."""
    p = _pair_prob((40, 30, 20), wl.BC_DIRICHLET0, wl.OP_VARCOEF, 21)
    c = frkc2_coeffs(2, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    lam_next = wl.random_state(p.shape, 22).reshape(-1)
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, T * c.a_re, T * c.a_im,
                                   grad_logD=np.zeros(p.npoints))
    lam = dev(lam_next)
    g = torch.zeros(p.npoints, dtype=torch.float64, device="cuda")
    try:
        F.frkc2_set_option(F.OPT_ADJ_STAGES, 2)
        F.frkc2_step_adjoint(p, dev(p.w0), dev(p.D), T, 2, lam, lam, g)
        torch.cuda.synchronize()
    finally:
        F.frkc2_set_option(F.OPT_ADJ_STAGES, 0)
    assert np.array_equal(host(lam), ref_lam)
    assert np.array_equal(host(g), ref_g)


def test_autograd_against_finite_differences():
    """J = sum (w(3T) - target)^2 over 3 supersteps, 3D variable D: dJ/du0 (central differences
    are exact for a quadratic) and dJ/dlogD (step 1e-4) in seeded directions."""
    from paper_1702_03818_amd.autograd import superstep_fn
    p = wl.diffusion3d(n_xyz=(24, 20, 16), nblobs=3)
    p.w0 = wl.random_state(p.shape, 1, smooth=1.5)
    s, nsteps = 16, 3
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    target = dev(wl.random_state(p.shape, 2, smooth=2.0))
    u0 = dev(p.w0).requires_grad_(True)
    logD = dev(np.log(p.D)).requires_grad_(True)

    def J(u, ld):
        w = superstep_fn(u, ld, p, T, s, nsteps)
        return ((w - target) ** 2).sum()

    loss = J(u0, logD)
    loss.backward()
    gu, gl = u0.grad.detach().clone(), logD.grad.detach().clone()
    rng = np.random.default_rng(7)
    with torch.no_grad():
        for _ in range(4):
            d = dev(rng.standard_normal(p.npoints))
            h = 1e-3
            fd = (J(u0 + h * d, logD) - J(u0 - h * d, logD)) / (2 * h)
            an = (gu * d).sum()
            assert abs(float(fd - an)) <= 1e-8 * max(1.0, abs(float(fd)))
            h = 1e-4
            fd = (J(u0, logD + h * d) - J(u0, logD - h * d)) / (2 * h)
            an = (gl * d).sum()
            assert abs(float(fd - an)) <= 1e-6 * max(1.0, abs(float(fd)))


def test_autograd_matches_oracle_chain():
    """The autograd gradients equal the oracle's adjoint chained over the supersteps."""
    from paper_1702_03818_amd.autograd import superstep_fn
    p = _prob("3d-var-dir")
    s, nsteps = 8, 2
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    target = wl.random_state(p.shape, 4).reshape(-1)
    u0 = dev(p.w0).requires_grad_(True)
    logD = dev(np.log(p.D)).requires_grad_(True)
    w = superstep_fn(u0, logD, p, T, s, nsteps)
    ((w - dev(target)) ** 2).sum().backward()
    # oracle chain
    tr, ti = T * c.a_re, T * c.a_im
    w1 = stage.superstep(p, p.w0, tr, ti)
    w2 = stage.superstep(p, w1, tr, ti)
    lam = 2 * (w2 - target)
    g = np.zeros(p.npoints)
    lam, g = stage.adjoint(p, w1, lam, tr, ti, grad_logD=g)
    lam, g = stage.adjoint(p, p.w0.reshape(-1), lam, tr, ti, grad_logD=g)
    # D = exp(logD) is formed by torch on the GPU and by the test's oracle
    # input (p.D) on the host, which may differ in the last bit: compare at the
    # 1e-12 gate instead of bit for bit (bitwise parity with the same D is
    # covered by test_adjoint_matches_oracle).
    def rel(a, b):
        return np.linalg.norm(a - b) / np.linalg.norm(b)
    assert rel(host(w), w2) <= 1e-12
    assert rel(host(u0.grad), lam) <= 1e-12
    assert rel(host(logD.grad), g) <= 1e-10


def _stored_stage(st, l, slot, n):
    """W^l of a stage store as (re, im) host arrays."""
    v = host(st[l * slot:l * slot + 16 * n].view(torch.float64)).reshape(n, 2)
    return v[:, 0], v[:, 1]


@pytest.mark.parametrize("kind", ["3d-var-dir", "3d-var-per", "2d-var-dir", "3d-lap-dir"])
@pytest.mark.parametrize("s", [2, 6, 8, 16, 64, 514])   # 3D: forward passes of three, two and one
def test_stage_store_and_stored_adjoint(kind, s):
    """frkc2_step_store gives the oracle's w^{n+1} bit for bit and leaves the oracle's stage
    states W^l in the store; frkc2_step_adjoint_stored on that store gives the oracle's adjoint
    bit for bit (lam_n and the accumulated D dJ/dD)."""
    p = _prob(kind)
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tr, ti = T * c.a_re, T * c.a_im
    D = dev(p.D) if p.D is not None else None
    w = dev(p.w0)
    st = F.stage_store(p, s)
    F.frkc2_step_store(p, w, D, T, s, st)
    torch.cuda.synchronize()
    assert np.array_equal(host(w), stage.superstep(p, p.w0, tr, ti).reshape(-1))
    n = p.npoints
    slot = F.frkc2_workspace_bytes(p, s, F.WS_STAGES) // s
    for l in sorted({0, 1, 2, 3, 4, s // 2, s - 2, s - 1}):
        if l >= s:
            continue
        wr = p.w0.reshape(-1).astype(np.float64).copy()
        wi = np.zeros_like(wr)
        if l > 0:
            stage.superstep_complex(p, wr, wi, tr[:l].copy(), ti[:l].copy())
        gr, gi = _stored_stage(st, l, slot, n)
        assert np.array_equal(gr, wr), "stage %d (real part)" % l
        assert np.array_equal(gi, wi), "stage %d (imaginary part)" % l
    lam_next = wl.random_state(p.shape, 9).reshape(-1)
    g0 = wl.random_state(p.shape, 10).reshape(-1)
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, tr, ti,
                                   grad_logD=g0.copy() if p.D is not None else None)
    lam_n = torch.empty(n, dtype=torch.float64, device="cuda")
    g = dev(g0) if p.D is not None else None
    F.frkc2_step_adjoint_stored(p, st, D, T, s, dev(lam_next), lam_n, g)
    torch.cuda.synchronize()
    assert np.array_equal(host(lam_n), ref_lam)
    if p.D is not None:
        assert np.array_equal(host(g), ref_g)


def test_stored_adjoint_aliased_lambda_and_pairs():
    """lam_n may alias lam_next, and two reverse stages per pass (on request) read the store
    as the one-stage passes do: both give the oracle's bits."""
    p = _prob("3d-var-dir")
    s = 16
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tr, ti = T * c.a_re, T * c.a_im
    D = dev(p.D)
    st = F.stage_store(p, s)
    F.frkc2_step_store(p, dev(p.w0), D, T, s, st)
    lam_next = wl.random_state(p.shape, 11).reshape(-1)
    ref_lam, ref_g = stage.adjoint(p, p.w0, lam_next, tr, ti, grad_logD=np.zeros(p.npoints))
    try:
        for stages in (1, 2):
            assert F.frkc2_set_option(F.OPT_ADJ_STAGES, stages) == 0
            lam = dev(lam_next)
            g = torch.zeros(p.npoints, dtype=torch.float64, device="cuda")
            F.frkc2_step_adjoint_stored(p, st, D, T, s, lam, lam, g)
            torch.cuda.synchronize()
            assert np.array_equal(host(lam), ref_lam), "stages per pass %d" % stages
            assert np.array_equal(host(g), ref_g), "stages per pass %d" % stages
    finally:
        F.frkc2_set_option(F.OPT_ADJ_STAGES, 0)


def test_autograd_stage_store_matches_checkpoints():
    """The autograd function with the stage store and with per-superstep checkpoints gives the
    same w and the same gradients, bit for bit."""
    from paper_1702_03818_amd.autograd import superstep_fn
    p = _prob("3d-var-per")
    s, nsteps = 16, 3
    c = frkc2_coeffs(s, 0.01)
    T = 0.9 * c.beta_bar / stage.rho_bound(p)
    tgt = dev(wl.random_state(p.shape, 4))
    res = []
    for store in (False, True, None):
        u = dev(p.w0).requires_grad_(True)
        ld = dev(np.log(p.D)).requires_grad_(True)
        w = superstep_fn(u, ld, p, T, s, nsteps, store_stages=store)
        ((w - tgt) ** 2).sum().backward()
        res.append((host(w), host(u.grad), host(ld.grad)))
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a, b)
