"""Launch configurations: every z chunk length and the configuration the autotuner picks
give the oracle's superstep bit for bit; the autotuner only reads the caller's state."""
import numpy as np
import pytest

from oracle import frkc2_coeffs, stage
from paper_1702_03818_amd import frkc2 as F

import test_gpu_parity as P
from test_gpu_parity import check, dev, host, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    F.load()
    yield
    for key in (F.OPT_TBLOCK, F.OPT_TILE, F.OPT_ZCHUNK, F.OPT_CLEAR_TUNED):
        F.frkc2_set_option(key, 0)
    torch.cuda.synchronize()


ZC_CASES = [
    ("3d-var-dir", (70, 37, 21), 1), ("3d-var-dir", (70, 37, 21), 2), ("3d-var-dir", (70, 37, 21), 3),
    ("3d-var-per", (67, 30, 18), 2), ("3d-lap-per", (9, 5, 4), 3),
    ("2d-var-dir", (300, 37, 1), 4), ("2d-por-per", (260, 33, 1), 8), ("2d-var-per", (257, 19, 1), 1),
]


@pytest.mark.parametrize("kind,n,k", ZC_CASES)
@pytest.mark.parametrize("zchunk", [1, 3, 8, 17])
def test_zchunk_matches_oracle(kind, n, k, zchunk, tile=1):
    """Chunks shorter than the fused depth, ragged last chunks and one-plane chunks."""
    F.frkc2_set_option(F.OPT_TBLOCK, k)
    F.frkc2_set_option(F.OPT_TILE, tile)
    F.frkc2_set_option(F.OPT_ZCHUNK, zchunk)
    try:
        P.test_superstep_matches_oracle(kind, n, 16)
    finally:
        F.frkc2_set_option(F.OPT_TBLOCK, 0)
        F.frkc2_set_option(F.OPT_TILE, 0)
        F.frkc2_set_option(F.OPT_ZCHUNK, 0)


@pytest.mark.parametrize("kind,n,k", [("3d-var-dir", (70, 37, 21), 2), ("3d-var-dir", (70, 37, 21), 3),
                                      ("3d-var-per", (67, 30, 18), 3), ("3d-lap-per", (9, 5, 4), 2)])
@pytest.mark.parametrize("zchunk", [1, 2, 5, 16])
@pytest.mark.parametrize("tile", [4, 5])
def test_zchunk_full_width_tiles(kind, n, k, zchunk, tile):
    test_zchunk_matches_oracle(kind, n, k, zchunk, tile=tile)


@pytest.mark.parametrize("kind,n", [("3d-var-dir", (72, 40, 36)), ("2d-por-per", (260, 33, 1)),
                                    ("2d-var-dir", (300, 37, 1))])
def test_autotune_then_step(kind, n):
    p = problem(kind, n)
    s = 16
    w = dev(p.w0)
    D = dev(p.D) if p.D is not None else None
    before = host(w).copy()
    r = F.frkc2_autotune(p, w, D, s=s, reps=1)
    torch.cuda.synchronize()
    assert np.array_equal(host(w), before), "autotune wrote the state"
    assert r["candidates"] > 10
    assert r["ms_best"] > 0 and r["ms_best"] <= r["ms_default"]
    assert r["tblock"] in ((1, 2, 3) if p.ndim == 3 else (1, 2, 3, 4, 6, 8))
    assert r["tile"] in ((1, 2, 3, 4) if p.ndim == 3 else (1, 2)) and r["zchunk"] >= 0
    try:
        c = frkc2_coeffs(s, 0.01)
        if p.op == 2:
            cfl = 0.9
            ref, _ = stage.run(p, s, 1, cfl=cfl, coeffs=c)
            F.frkc2_step(p, w, None, cfl=cfl, s=s, nsteps=1)
        else:
            T = 0.9 * c.beta_bar / stage.rho_bound(p)
            ref = stage.superstep(p, p.w0, T * c.a_re, T * c.a_im)
            F.frkc2_step(p, w, D, T=T, s=s, nsteps=1)
        torch.cuda.synchronize()
        check(host(w), ref, "%s %s after autotune %s" % (kind, n, r))
    finally:
        F.frkc2_set_option(F.OPT_CLEAR_TUNED, 0)
