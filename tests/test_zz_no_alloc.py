"""frkc2_step_noalloc (the entry point for callers that cannot allocate device memory) against
frkc2_step on the same inputs, through the C ABI: bit for bit, on two calls in a row, the
second on a smaller grid (the static scratch keeps the first call's contents), and on the
largest state it accepts; a larger one is refused before any HIP call."""
import numpy as np
import pytest

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


def both(p, s, nsteps, **kw):
    D = dev(p.D) if p.D is not None else None
    a = dev(p.w0)
    b = dev(p.w0)
    sa = F.frkc2_step(p, a, D, s=s, nsteps=nsteps, stats=True, **kw)
    sb = F.frkc2_step_noalloc(p, b, D, s=s, nsteps=nsteps, stats=True, **kw)
    torch.cuda.synchronize()
    return a, b, sa, sb


def test_two_calls_second_smaller():
    big = wl.diffusion3d(n_xyz=(70, 37, 21), nblobs=3)
    big.w0 = wl.random_state(big.shape, 3, smooth=1.5)
    rho = F.frkc2_rho_bound(big, None, dev(big.D))
    _, _, info, _ = F.frkc2_coeffs(100, 0.01)
    a, b, sa, sb = both(big, 100, 2, T=0.9 * info["beta_bar"] / rho)
    assert torch.equal(a, b)
    assert sa == sb
    small = wl.Problem(2, (67, 19, 1), 1.0 / 67, wl.BC_PERIODIC, wl.OP_POROUS2, 1.0)
    small.w0 = 1.0 + 0.3 * wl.random_state(small.shape, 4, smooth=2.0)
    a, b, sa, sb = both(small, 16, 3, cfl=0.5)
    assert torch.equal(a, b)
    assert sa == sb


def test_largest_accepted_state():
    p = wl.diffusion3d(n_xyz=(128, 128, 128), nblobs=4)
    assert p.npoints == F.NOALLOC_MAX_VALUES
    rho = F.frkc2_rho_bound(p, None, dev(p.D))
    _, _, info, _ = F.frkc2_coeffs(16, 0.01)
    a, b, sa, sb = both(p, 16, 1, T=0.9 * info["beta_bar"] / rho)
    assert torch.equal(a, b)
    assert sa == sb


def test_larger_state_is_refused():
    p = wl.Problem(3, (129, 128, 128), 1.0 / 130, wl.BC_DIRICHLET0, wl.OP_LAPLACE, 1.0)
    w = torch.zeros(p.npoints, dtype=torch.float64, device="cuda")
    with pytest.raises(F.Frkc2Error) as e:
        F.frkc2_step_noalloc(p, w, None, T=1e-9, s=4)
    assert e.value.status == -2
    assert "static scratch" in str(e.value)
