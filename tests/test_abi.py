"""CPU tests of the C-ABI library: loading, exported symbols, host-side
stepsizes against the oracle, and argument validation (which runs before any
HIP call, so no GPU is needed)."""
import ctypes
import re

import numpy as np
import pytest

from oracle.coeffs import frkc2_coeffs as oracle_coeffs
from paper_1702_03818_amd import frkc2 as F
from paper_1702_03818_amd import workloads as wl

HEADER = "include/frkc2.h"


def header_functions():
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, HEADER)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(frkc(?:2|4s?)_\w+)\s*\(", src)))


def test_library_exports_every_declared_function():
    lib = F.load()
    names = header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(F.exported_symbols())


def test_version():
    assert "gfx950" in F.frkc2_version()


@pytest.mark.parametrize("s", [2, 4, 6, 8, 10, 16, 20, 32, 50, 64, 100, 128, 200, 256, 400, 514])
def test_coeffs_bitwise_equal_to_oracle(s):
    """Library (binary128 host code) and oracle (50-digit mpmath) round to the same doubles and
    pick the same stage order; beta, betabar and n agree exactly, Q to rounding."""
    re_, im_, info, rc = F.frkc2_coeffs(s, 0.01)
    o = oracle_coeffs(s, 0.01)
    assert np.array_equal(re_, o.a_re)
    assert np.array_equal(im_, o.a_im)
    assert info["beta"] == o.beta
    assert info["beta_bar"] == o.beta_bar
    assert info["n_shrink"] == o.n_shrink
    assert abs(info["q_realised"] / o.q_realised - 1) < 1e-12
    assert bool(info["q_bound_met"]) == o.q_bound_met
    assert rc == (F.FRKC2_OK if o.q_bound_met else F.FRKC2_WQBOUND)
    assert complex(info["mu_re"], info["mu_im"]) == o.mu


@pytest.mark.parametrize("nu", [0.0, 0.05, 0.3])
def test_coeffs_other_damping(nu):
    for s in (8, 64):
        re_, im_, info, _ = F.frkc2_coeffs(s, nu)
        o = oracle_coeffs(s, nu)
        assert np.array_equal(re_, o.a_re) and np.array_equal(im_, o.a_im)
        assert info["beta"] == o.beta


@pytest.mark.parametrize("s,nu", [(0, 0.01), (3, 0.01), (516, 0.01), (8, -0.1), (8, 1.0),
                                  (8, float("nan"))])
def test_coeffs_rejects(s, nu):
    with pytest.raises(F.Frkc2Error) as e:
        F.frkc2_coeffs(s, nu)
    assert e.value.status == -1


def grid(**kw):
    d = dict(ndim=3, n=(8, 8, 8), h=0.1, bc=1, op=1, d_const=1.0)
    d.update(kw)
    return F.make_grid(d)


@pytest.mark.parametrize("kw", [dict(ndim=0), dict(ndim=4), dict(n=(0, 8, 8)), dict(ndim=2, n=(8, 8, 8)),
                                dict(h=0.0), dict(h=float("inf")), dict(bc=7), dict(op=9),
                                dict(op=0, d_const=-1.0)])
def test_workspace_bytes_invalid_grid(kw):
    g = grid(**kw)
    assert F.load().frkc2_workspace_bytes(ctypes.byref(g), 16, F.WS_STEP) == 0


def test_workspace_bytes_sizes():
    lib = F.load()
    g = grid(n=(256, 256, 256))
    N = 256 ** 3
    step = lib.frkc2_workspace_bytes(ctypes.byref(g), 100, F.WS_STEP)
    adj = lib.frkc2_workspace_bytes(ctypes.byref(g), 64, F.WS_ADJOINT)
    assert 32 * N <= step < 32 * N + (1 << 20)
    assert (64 + 2) * 16 * N + 8 * N <= adj < (64 + 2) * 16 * N + 8 * N + (1 << 20)


def _step(g, w=1, D=1, T=1e-3, cfl=0.0, s=16, nu=0.01, nsteps=1, ws=1, ws_bytes=1 << 40):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    return lib.frkc2_step(ctypes.byref(g), p(w), p(D), T, cfl, s, nu, nsteps, p(ws), ws_bytes, None,
                          None)


@pytest.mark.parametrize("kw,expect", [
    (dict(w=0), -1), (dict(D=0), -1), (dict(s=7), -1), (dict(s=600), -1), (dict(nu=1.5), -1),
    (dict(nsteps=-1), -1), (dict(T=0.0), -1), (dict(T=1e-3, cfl=0.5), -1),
    (dict(T=float("nan")), -1), (dict(T=-1.0), -1), (dict(ws=0), -2), (dict(ws_bytes=100), -2),
])
def test_step_validation(kw, expect):
    g = grid()
    assert _step(g, **kw) == expect
    assert F.frkc2_last_error()


def test_stage_store_workspace_sizes():
    """The stage store holds s complex states in 256-byte-rounded slots; the stored adjoint's
    workspace two complex adjoint buffers, one real gradient buffer and scratch."""
    lib = F.load()
    g = grid(n=(70, 13, 11))
    N = 70 * 13 * 11
    slot = (16 * N + 255) // 256 * 256
    for s in (2, 64, 514):
        assert lib.frkc2_workspace_bytes(ctypes.byref(g), s, F.WS_STAGES) == s * slot
    for s in (0, 7, 516):
        assert lib.frkc2_workspace_bytes(ctypes.byref(g), s, F.WS_STAGES) == 0
    adj = lib.frkc2_workspace_bytes(ctypes.byref(g), 64, F.WS_ADJOINT_STORED)
    assert 2 * 16 * N + 8 * N <= adj < 2 * 16 * N + 8 * N + (1 << 20)
    assert lib.frkc2_workspace_bytes(ctypes.byref(g), 64, F.WS_ADJOINT) == 64 * slot + adj


def _store(g, w=1, D=1, T=1e-3, s=16, nu=0.01, st=1, st_bytes=1 << 40, ws=1, ws_bytes=1 << 40):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    return lib.frkc2_step_store(ctypes.byref(g), p(w), p(D), T, s, nu, p(st), st_bytes, p(ws),
                                ws_bytes, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(w=0), -1), (dict(D=0), -1), (dict(st=0), -1), (dict(s=7), -1), (dict(nu=1.5), -1),
    (dict(T=0.0), -1), (dict(T=float("inf")), -1), (dict(st_bytes=1000), -2),
    (dict(ws=0), -2), (dict(ws_bytes=1000), -2),
])
def test_step_store_validation(kw, expect):
    assert _store(grid(), **kw) == expect
    assert F.frkc2_last_error()


def _stored_adj(g, st=1, st_bytes=1 << 40, D=1, T=1e-3, s=16, nu=0.01, ln=1, l0=1, ws=1,
                ws_bytes=1 << 40):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    return lib.frkc2_step_adjoint_stored(ctypes.byref(g), p(st), st_bytes, p(D), T, s, nu, p(ln),
                                         p(l0), None, p(ws), ws_bytes, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(st=0), -1), (dict(D=0), -1), (dict(ln=0), -1), (dict(l0=0), -1), (dict(s=3), -1),
    (dict(T=-1.0), -1), (dict(st_bytes=1000), -2), (dict(ws=0), -2), (dict(ws_bytes=1000), -2),
])
def test_step_adjoint_stored_validation(kw, expect):
    assert _stored_adj(grid(), **kw) == expect
    assert F.frkc2_last_error()


def test_stage_store_rejects_nonlinear_operator():
    for op in (2, 3, 4):
        assert _store(grid(op=op)) == -1
        assert _stored_adj(grid(op=op)) == -1


def test_adjoint_rejects_nonlinear_operator():
    lib = F.load()
    g = grid(op=2)
    p = ctypes.c_void_p(4096)
    rc = lib.frkc2_step_adjoint(ctypes.byref(g), p, None, 1e-3, 16, 0.01, p, p, None, p, 1 << 40,
                                None)
    assert rc == -1


def test_reduce_validation():
    lib = F.load()
    out = ctypes.c_double()
    assert lib.frkc2_reduce(9, ctypes.c_void_p(4096), None, 10, ctypes.byref(out),
                            ctypes.c_void_p(4096), 1 << 20, None) == -1
    assert lib.frkc2_reduce(3, ctypes.c_void_p(4096), None, 10, ctypes.byref(out),
                            ctypes.c_void_p(4096), 1 << 20, None) == -1
    assert lib.frkc2_reduce(0, ctypes.c_void_p(4096), None, 10, ctypes.byref(out),
                            ctypes.c_void_p(4096), 8, None) == -2


def test_set_option_validation():
    assert F.load().frkc2_set_option(F.OPT_TBLOCK, 99) == -1
    assert F.load().frkc2_set_option(12345, 1) == -1
    assert F.frkc2_set_option(F.OPT_TBLOCK, 0) == 0
    assert F.load().frkc2_set_option(F.OPT_TILE, 6) == -1
    assert F.frkc2_set_option(F.OPT_TILE, 5) == 0
    assert F.frkc2_set_option(F.OPT_TILE, 0) == 0


@pytest.mark.parametrize("key,good,bad", [("OPT_ADJ_STAGES", (0, 1, 2), (3, -1)),
                                          ("OPT_BATCH_K3", (0, 2, 3), (1, 4, -1)),
                                          ("OPT_BATCH_COLS", (0, 1, 32, 64), (2, 16, 48, 128)),
                                          ("OPT_BATCH_K2", (0, 2, 3, 4, 6), (1, 5, 8))])
def test_batch_option_validation(key, good, bad):
    lib = F.load()
    for v in bad:
        assert lib.frkc2_set_option(getattr(F, key), v) == -1
    for v in good:
        assert lib.frkc2_set_option(getattr(F, key), v) == 0
    assert lib.frkc2_set_option(getattr(F, key), 0) == 0


def test_batched_autotune_validation():
    """Argument errors come back before any HIP call."""
    lib = F.load()
    g = (F.Grid * 1)(grid(n=(8, 8, 8), op=0))
    s = (ctypes.c_int * 1)(8)
    w = (ctypes.c_void_p * 1)(None)
    D = (ctypes.c_void_p * 1)(None)
    T = (ctypes.c_double * 1)(0.001)
    r = F.BatchTuneResult()
    assert lib.frkc2_batched_autotune(1, g, w, D, T, s, 0.01, 2, None, 0, None,
                                      ctypes.byref(r)) == -1          # w[0] NULL
    w2 = (ctypes.c_void_p * 1)(16)
    for reps in (0, 101):
        assert lib.frkc2_batched_autotune(1, g, w2, D, T, s, 0.01, reps, None, 0, None,
                                          ctypes.byref(r)) == -1
    assert lib.frkc2_batched_autotune(1, g, w2, D, T, s, 0.01, 2, None, 0, None, None) == -1
    s_bad = (ctypes.c_int * 1)(7)
    assert lib.frkc2_batched_autotune(1, g, w2, D, T, s_bad, 0.01, 2, None, 0, None,
                                      ctypes.byref(r)) == -1
    assert lib.frkc2_batched_autotune(1, g, w2, D, T, s, 0.01, 2, None, 0, None,
                                      ctypes.byref(r)) == -2          # no workspace


def test_batched_autotune_is_switched_off():
    """With valid arguments the switched-off autotuner refuses before any HIP call and says
    why."""
    lib = F.load()
    g = (F.Grid * 1)(grid(n=(8, 8, 8), op=0))
    s = (ctypes.c_int * 1)(8)
    w = (ctypes.c_void_p * 1)(16)
    D = (ctypes.c_void_p * 1)(None)
    T = (ctypes.c_double * 1)(0.001)
    r = F.BatchTuneResult()
    need = lib.frkc2_batched_workspace_bytes(1, g, s)
    assert need > 0
    ws = ctypes.c_void_p(1 << 20)   # never dereferenced: the call returns before using it
    assert lib.frkc2_batched_autotune(1, g, w, D, T, s, 0.01, 2, ws, need, None,
                                      ctypes.byref(r)) == -7
    assert b"switched off" in lib.frkc2_last_error()


def test_batched_workspace_covers_every_depth():
    """The work tables are sized for the most pass levels any supported depth gives."""
    lib = F.load()
    g3 = (F.Grid * 1)(grid(n=(8, 8, 8), op=0))
    small = lib.frkc2_batched_workspace_bytes(1, g3, (ctypes.c_int * 1)(2))
    big = lib.frkc2_batched_workspace_bytes(1, g3, (ctypes.c_int * 1)(514))
    assert 0 < small < big


def test_grid_from_problem():
    p = wl.heat1d()
    g = F.make_grid(p)
    assert g.ndim == 1 and list(g.n) == [1024, 1, 1] and g.h == p.h


def _tune(g, w=1, D=1, s=16, nu=0.01, reps=2, ws=1, ws_bytes=1 << 40, res=True):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    r = F.TuneResult()
    return lib.frkc2_autotune(ctypes.byref(g), p(w), p(D), s, nu, reps, p(ws), ws_bytes, None,
                              ctypes.byref(r) if res else None)


@pytest.mark.parametrize("kw,expect", [
    (dict(w=0), -1), (dict(D=0), -1), (dict(res=False), -1), (dict(s=5), -1), (dict(nu=-1.0), -1),
    (dict(reps=0), -1), (dict(reps=101), -1), (dict(ws=0), -2), (dict(ws_bytes=64), -2),
])
def test_autotune_validation(kw, expect):
    assert _tune(grid(), **kw) == expect
    assert F.frkc2_last_error()


def test_autotune_invalid_grid():
    assert _tune(grid(ndim=5)) == -1


def test_clear_tuned_option():
    assert F.frkc2_set_option(F.OPT_CLEAR_TUNED, 0) == 0


def _integrate(g, w=1, D=1, t_span=1e-3, T0=1e-5, tol=1e-4, nu=0.01, max_attempts=10, ws=1,
               ws_bytes=1 << 40, trace_cap=0):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    st = F.AdaptStats()
    return lib.frkc2_integrate(ctypes.byref(g), p(w), p(D), t_span, T0, tol, nu, max_attempts, p(ws),
                               ws_bytes, None, None, trace_cap, ctypes.byref(st))


@pytest.mark.parametrize("kw,expect", [
    (dict(w=0), -1), (dict(D=0), -1), (dict(t_span=0.0), -1), (dict(t_span=float("inf")), -1),
    (dict(T0=-1.0), -1), (dict(tol=0.0), -1), (dict(nu=1.0), -1), (dict(max_attempts=0), -1),
    (dict(trace_cap=3), -1), (dict(ws=0), -2), (dict(ws_bytes=1024), -2),
])
def test_integrate_validation(kw, expect):
    assert _integrate(grid(), **kw) == expect
    assert F.frkc2_last_error()


def test_adapt_workspace_bytes():
    lib = F.load()
    g = grid(n=(64, 32, 16))
    N = 64 * 32 * 16
    b = lib.frkc2_workspace_bytes(ctypes.byref(g), 0, F.WS_ADAPT)
    assert 48 * N <= b < 48 * N + (1 << 20)


@pytest.mark.parametrize("nu", [0.01, 0.25])
def test_write_table_layout_and_values(tmp_path, nu):
    """Three lines per M: betabar and Q, then Re a and Im a of the s = 2M stages, equal to the
    oracle's stepsizes (betabar and a exactly, Q to rounding)."""
    path = tmp_path / "frkc2arks.dat"
    m_max = 12
    F.frkc2_write_table(str(path), nu, m_max)
    lines = path.read_text().splitlines()
    assert len(lines) == 3 * m_max
    for M in range(1, m_max + 1):
        bb, q = (float(v) for v in lines[3 * M - 3].split())
        re_ = np.array([float(v) for v in lines[3 * M - 2].split()])
        im_ = np.array([float(v) for v in lines[3 * M - 1].split()])
        o = oracle_coeffs(2 * M, nu)
        assert bb == o.beta_bar
        assert abs(q / o.q_realised - 1) < 1e-12
        assert np.array_equal(re_, o.a_re) and np.array_equal(im_, o.a_im)


def test_write_table_rejects():
    assert F.load().frkc2_write_table(b"/tmp/x", 0.01, 0) == -1
    assert F.load().frkc2_write_table(b"/tmp/x", 0.01, 258) == -1
    assert F.load().frkc2_write_table(b"/nonexistent-dir/x", 0.01, 2) == -1
    assert F.load().frkc2_write_table(None, 0.01, 2) == -1


def test_step_user_validation():
    lib = F.load()
    cb = F.USER_F(lambda W, Fp, n, user, st: 0)   # never called: validation fails first
    p = ctypes.c_void_p(4096 * 16)
    ok = dict(n=1000, w=p, f=cb, T=1e-3, rho=10.0, s=16, nu=0.01, nsteps=1, ws=p, wsb=1 << 40)

    def call(**kw):
        a = dict(ok)
        a.update(kw)
        return lib.frkc2_step_user(a["n"], a["w"], a["f"], None, a["T"], a["rho"], a["s"], a["nu"],
                                   a["nsteps"], a["ws"], a["wsb"], None)
    assert call(n=0) == -1
    assert call(w=None) == -1
    assert call(f=F.USER_F()) == -1
    assert call(s=7) == -1
    assert call(T=0.0) == -1
    assert call(rho=-1.0) == -1
    assert call(nsteps=-1) == -1
    assert call(ws=None) == -2
    assert call(wsb=100) == -2
    assert call(T=1.0, rho=1e6) == -4          # T rho beyond betabar(16)


@pytest.mark.parametrize("ndim,vel,bc", [(1, (12.0,), 0), (2, (3.0, -40.0), 1), (3, (1.0, 2.0, 500.0), 0)])
def test_advdiff_rho_bound_on_host(ndim, vel, bc):
    """The advection-diffusion bound is computed on the host: equal to the oracle's."""
    from oracle import stage as ostage
    n = (16, 12, 10)[:ndim]
    p = wl.Problem(ndim, tuple(n) + (1,) * (3 - ndim), 0.05, bc, wl.OP_ADVDIFF, 0.7)
    p.vel = tuple(vel) + (0.0,) * (3 - ndim)
    g = F.make_grid(p)
    rho = ctypes.c_double()
    assert F.load().frkc2_rho_bound(ctypes.byref(g), None, None, ctypes.byref(rho), None, 0,
                                    None) == 0
    assert rho.value == ostage.rho_bound(p)


def test_advdiff_rejects_nonfinite_velocity():
    g = grid(op=4, vel=(1.0, float("nan"), 0.0))
    assert F.load().frkc2_workspace_bytes(ctypes.byref(g), 16, F.WS_STEP) == 0


def test_user_workspace_and_integrate_validation():
    lib = F.load()
    assert lib.frkc2_user_workspace_bytes(0, F.WS_STEP) == 0
    assert lib.frkc2_user_workspace_bytes(1000, 7) == 0
    step = lib.frkc2_user_workspace_bytes(1000, F.WS_STEP)
    adapt = lib.frkc2_user_workspace_bytes(1000, F.WS_ADAPT)
    assert step >= 32 * 1000 and adapt >= step + 16 * 1000
    f = F.USER_F(lambda *a: 0)
    nul = ctypes.cast(None, F.USER_RHO)
    args = dict(t_span=1.0, T0=0.1, tol=1e-3, nu=0.01, max_attempts=10)

    def call(n=8, w=1, fn=f, rho_f=nul, rho_const=1.0, **kw):
        a = dict(args, **kw)
        return lib.frkc2_integrate_user(n, ctypes.c_void_p(w), fn, rho_f, rho_const, None,
                                        a["t_span"], a["T0"], a["tol"], a["nu"],
                                        a["max_attempts"], None, 0, None, None, 0, None)

    assert call(n=0) == -1
    assert call(fn=ctypes.cast(None, F.USER_F)) == -1
    assert call(rho_const=0.0) == -1
    assert call(rho_const=float("inf")) == -1
    assert call(tol=0.0) == -1
    assert call(nu=1.0) == -1
    assert call(max_attempts=0) == -1
    assert call() == -2            # arguments fine, no workspace


def _noalloc(g, w=1, D=1, T=1e-3, cfl=0.0, s=16, nu=0.01, nsteps=1):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    return lib.frkc2_step_noalloc(ctypes.byref(g), p(w), p(D), T, cfl, s, nu, nsteps, None, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(w=0), -1), (dict(D=0), -1), (dict(s=7), -1), (dict(nsteps=-1), -1), (dict(T=0.0), -1),
])
def test_step_noalloc_validation(kw, expect):
    assert _noalloc(grid(), **kw) == expect
    assert F.frkc2_last_error()


def test_step_noalloc_size_limit():
    """States beyond the static scratch (2^21 values) are refused before any HIP call."""
    assert F.NOALLOC_MAX_VALUES == 2 ** 21
    assert _noalloc(grid(n=(129, 128, 128))) == -2
    assert "static scratch" in F.frkc2_last_error()
    assert _noalloc(grid(ndim=2, n=(1449, 1449, 1), op=0)) == -2


@pytest.mark.parametrize("nu", [0.0, 0.01, 0.05])
def test_frkc4_coeffs_bitwise_equal_to_oracle(nu):
    """Fourth-order stepsizes: library (binary128 bisection, Weierstrass roots, Newton acos)
    and oracle (50-digit mpmath) round to the same doubles, the same order and extent."""
    from oracle import frkc4
    for s in list(range(4, 68, 4)) + [100, 128, 200, 256, 512]:
        re_, im_, info, rc = F.frkc4_coeffs(s, nu)
        o = frkc4.frkc4_coeffs(s, nu)
        assert np.array_equal(re_, o.a_re) and np.array_equal(im_, o.a_im), s
        assert info["beta"] == o.beta and info["beta_bar"] == o.beta_bar, s
        assert info["n_shrink"] == o.n_shrink and bool(info["q_bound_met"]) == o.q_bound_met
        assert info["mu_re"] == o.alpha


@pytest.mark.parametrize("s,nu", [(0, 0.01), (6, 0.01), (516, 0.01), (8, -0.1), (8, 0.25)])
def test_frkc4_coeffs_rejects(s, nu):
    with pytest.raises(F.Frkc2Error) as e:
        F.frkc4_coeffs(s, nu)
    assert e.value.status == -1


def _split(g, w=1, T=1e-3, s=8, nsub=4, nu=0.01, nsteps=1, ws=1, ws_bytes=1 << 40):
    lib = F.load()
    p = lambda v: ctypes.c_void_p(4096 * 16) if v else None  # never dereferenced: validation fails first
    return lib.frkc4s_step(ctypes.byref(g), p(w), T, s, nsub, nu, nsteps, p(ws), ws_bytes, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(w=0), -1), (dict(T=0.0), -1), (dict(s=6), -1), (dict(s=516), -1), (dict(nsub=0), -1),
    (dict(nsub=65), -1), (dict(nsteps=-1), -1), (dict(nu=0.3), -1), (dict(ws=0), -2),
    (dict(ws_bytes=1024), -2), (dict(T=1.0, s=4), -4),
])
def test_frkc4s_validation(kw, expect):
    g = F.make_grid(dict(ndim=2, n=(64, 64, 1), h=1 / 64, bc=0, op=3, d_const=0.02))
    assert _split(g, **kw) == expect
    assert F.frkc2_last_error()


def test_frkc4s_needs_brusselator():
    g = grid(op=1)
    assert _split(g) == -1
    assert F.load().frkc4s_workspace_bytes(ctypes.byref(g)) == 0


def test_batched_refuses_oversized_planes():
    """A 3D batch problem whose planes reach 2^27 points is refused before any HIP call (the
    fused tiles address a plane with 32-bit byte offsets); one point fewer is accepted."""
    lib = F.load()
    s = (ctypes.c_int * 1)(16)
    big = grid(n=(1 << 14, 1 << 13, 2))
    assert lib.frkc2_batched_workspace_bytes(1, ctypes.byref(big), s) == 0
    assert b"2^27" in lib.frkc2_last_error()
    ok = grid(n=(1 << 14, (1 << 13) - 1, 2))
    assert lib.frkc2_batched_workspace_bytes(1, ctypes.byref(ok), s) > 0


def test_batched_shapes_match_the_batch():
    """batched_shapes draws the same grids and stage counts as batched (first 6 problems)."""
    full = wl.batched(count=6)
    shapes = wl.batched_shapes(count=6)
    for (p, s), (q, t) in zip(full, shapes):
        assert (p.ndim, p.n, p.h, s) == (q.ndim, q.n, q.h, t)


def test_batched_config_query():
    """The configuration a graph would be built with: built-in (depths 3 and 4, the width
    with less modelled work: 32 columns for the 512-problem batch, 64 for one 256^3 grid),
    then the options, which override it per key; host only."""
    batch = wl.batched_shapes()
    grids = [p for p, _ in batch]
    ss = [s for _, s in batch]
    assert F.frkc2_batched_config(grids, ss) == (3, 32, 4)
    big = wl.Problem(3, (256, 256, 256), 1.0 / 257, wl.BC_DIRICHLET0, wl.OP_VARCOEF)
    assert F.frkc2_batched_config([big], [100]) == (3, 64, 4)
    try:
        assert F.frkc2_set_option(F.OPT_BATCH_K2, 6) == 0
        assert F.frkc2_batched_config(grids, ss) == (3, 32, 6)
        assert F.frkc2_set_option(F.OPT_BATCH_COLS, 1) == 0
        assert F.frkc2_batched_config(grids, ss) == (3, 1, 6)
        assert F.frkc2_set_option(F.OPT_BATCH_K3, 2) == 0
        assert F.frkc2_batched_config(grids, ss) == (2, 1, 6)
        assert F.frkc2_set_option(F.OPT_BATCH_COLS, 0) == 0
        k3, cols, k2 = F.frkc2_batched_config(grids, ss)
        assert (k3, k2) == (2, 6) and cols in (32, 64)
    finally:
        for key in (F.OPT_BATCH_K3, F.OPT_BATCH_COLS, F.OPT_BATCH_K2):
            F.frkc2_set_option(key, 0)
    assert F.frkc2_batched_config(grids, ss) == (3, 32, 4)
    lib = F.load()
    one = (F.Grid * 1)(F.make_grid(big))
    sarr = (ctypes.c_int * 1)(100)
    v = ctypes.c_int()
    assert lib.frkc2_batched_config(0, one, sarr, ctypes.byref(v), ctypes.byref(v),
                                    ctypes.byref(v)) == -1
    assert lib.frkc2_batched_config(1, one, sarr, None, ctypes.byref(v), ctypes.byref(v)) == -1
