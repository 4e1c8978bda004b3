"""The D2Q9 per-cell arithmetic of the GPU kernels (``csrc/cm_math2d.hpp``),
built for the host, against the oracle (CPU only).

The kernel works in the factorised central-moment form; the oracle's generic
collision on the D2Q9 lattice is itself pinned to the paper's printed D2Q9
formulas (Secs. 8-11), so agreement here ties the kernel arithmetic to the
paper's own lattice.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import collide as C
from oracle import d2q9_paper as PP
from oracle.lattice import Relax, d2q9

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOSTLIB = os.path.join(ROOT, "paper_1202_6074_amd", "libcmlbm_hostmath.so")
LAT = d2q9()
W = dict(w3=1.21, ws=1.37, w6=0.93, w7=1.41, w8=1.12)


@pytest.fixture(scope="module")
def hm():
    if not os.path.exists(HOSTLIB):
        from paper_1202_6074_amd.build import build_hostmath
        build_hostmath()
    lib = ctypes.CDLL(HOSTLIB)
    P = ctypes.c_void_p
    for name in ("cmhost_collide9_f64", "cmhost_collide9_f32"):
        getattr(lib, name).argtypes = [P, P, P, ctypes.c_int, ctypes.c_long, P]
    lib.cmhost_equilibrium9_f64.argtypes = [P, P, P, ctypes.c_double, ctypes.c_long, P, ctypes.c_int]
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _relax(cs=0.0, rc=False, fact=False):
    return Relax(omega_shear=W["ws"], omega_bulk=W["w3"], d2q9_omega678=(W["w6"], W["w7"], W["w8"]), cs_smag=cs,
                 reduced_compressibility=rc, factorized=fact)


def host_collide(hm, f, F, cs=0.0, rc=False, fact=False, dtype=np.float64, rho0=1.0):
    f = np.ascontiguousarray(f, dtype=dtype)
    F = np.ascontiguousarray(F, dtype=dtype)
    out = np.empty_like(f)
    flags = (1 if fact else 0) | (2 if rc else 0)
    rates = np.array([rho0, W["w3"], W["ws"], W["w6"], W["w7"], W["w8"], cs, float(flags)])
    fn = hm.cmhost_collide9_f64 if dtype == np.float64 else hm.cmhost_collide9_f32
    fn(_ptr(f), _ptr(F), _ptr(rates), int(cs > 0), f.shape[1], _ptr(out))
    return out


def _state(n=300, seed=31, famp=0.01, uamp=0.1):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = uamp * rng.standard_normal((2, n))
    F = famp * rng.standard_normal((2, n))
    feq = C.product_equilibrium(rho, u, LAT)
    f = feq * (1 + 0.05 * rng.standard_normal(feq.shape))
    return f, F


def test_paper_order_and_weights():
    # the host entries take the paper's velocity order (Sec. 2), as the oracle lattice
    assert LAT.e.tolist() == [[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]]


@pytest.mark.parametrize("cs", [0.0, 0.15])
def test_collision_f64_matches_oracle(hm, cs):
    f, F = _state()
    got = host_collide(hm, f, F, cs)
    want = C.collide(f, F, LAT, _relax(cs))
    assert np.abs(got - want).max() < 2e-15


@pytest.mark.parametrize("rc,fact", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("cs", [0.0, 0.15])
def test_collision_variants_f64_match_oracle(hm, cs, rc, fact):
    f, F = _state(seed=32)
    got = host_collide(hm, f, F, cs, rc, fact)
    want = C.collide(f, F, LAT, _relax(cs, rc, fact), rho0=1.0)
    assert np.abs(got - want).max() < 3e-15


def test_force_free_collision_equals_paper_literal(hm):
    # Secs. 9-11 as printed (no force): the kernel equals the literal formulas
    f, F = _state(seed=33)
    F[:] = 0.0
    got = host_collide(hm, f, F)
    want = PP.collide(f, F, (W["w3"], W["ws"], W["ws"], W["w6"], W["w7"], W["w8"]))
    assert np.abs(got - want).max() < 2e-15


def test_collision_f32_matches_oracle(hm):
    f, F = _state(seed=34)
    f32, F32 = f.astype(np.float32), F.astype(np.float32)
    got = host_collide(hm, f32, F32, dtype=np.float32).astype(np.float64)
    want = C.collide(f32.astype(np.float64), F32.astype(np.float64), LAT, _relax())
    assert np.abs(got - want).max() < 1e-7


def test_equilibrium_matches_oracle(hm):
    rng = np.random.default_rng(35)
    n = 60
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = np.ascontiguousarray(0.1 * rng.standard_normal((2, n)))
    F = np.ascontiguousarray(0.01 * rng.standard_normal((2, n)))
    out = np.empty((9, n))
    for rc in (0, 1):
        hm.cmhost_equilibrium9_f64(_ptr(rho), _ptr(u), _ptr(F), 1.0, n, _ptr(out), rc)
        want = C.equilibrium_state(rho, u, F, LAT, 1.0 if rc else None)
        assert np.abs(out - want).max() < 2e-16 * 8


@pytest.mark.parametrize("rc,fact", [(False, False), (True, True)])
def test_collision_with_sgs_force_matches_oracle(hm, rc, fact):
    """Sec. 14 on the paper's lattice: force F + rho a', and the sub-grid stress
    (xx, yy, xy) of the step from the pre-collision moments (oracle.sgs)."""
    from oracle import sgs as SG
    hm.cmhost_collide9_sgs_f64.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_long] + [ctypes.c_void_p] * 2
    f, F = _state(seed=36)
    rng = np.random.default_rng(37)
    acc = np.ascontiguousarray(1e-3 * rng.standard_normal(F.shape))
    flags = (1 if fact else 0) | (2 if rc else 0) | 4
    cs = 0.3
    rates = np.array([1.0, W["w3"], W["ws"], W["w6"], W["w7"], W["w8"], cs, float(flags)])
    out = np.empty_like(f)
    st = np.empty((3, f.shape[1]))
    hm.cmhost_collide9_sgs_f64(_ptr(f), _ptr(F), _ptr(acc), _ptr(rates), f.shape[1], _ptr(out), _ptr(st))
    r = Relax(omega_shear=W["ws"], omega_bulk=W["w3"], d2q9_omega678=(W["w6"], W["w7"], W["w8"]), cs_smag=cs,
              sgs_force=True, reduced_compressibility=rc, factorized=fact)
    rho = f.sum(axis=0)
    want, parts = C.collide(f, F + rho * acc, LAT, r, return_parts=True, rho0=1.0)
    assert np.abs(out - want).max() < 3e-15
    rho_s = np.ones_like(rho) if rc else parts["rho"]
    Rw = SG.sgs_stress(parts["kbar"], rho_s, LAT, W["ws"], cs)
    want_st = np.array([Rw[0, 0], Rw[1, 1], Rw[0, 1]])
    assert np.abs(st - want_st).max() < 1e-12 * np.abs(want_st).max()
    assert np.abs(want_st).max() > 1e-6
