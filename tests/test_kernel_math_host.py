"""The GPU kernels' per-cell arithmetic, built for the host, against the oracle (CPU only).

``libcmlbm_hostmath.so`` compiles the same header the HIP kernels use
(``csrc/cm_math.hpp``) with g++. These tests check, without a GPU, that the
factorised transforms, source recursion, relaxation and eddy viscosity agree
with the oracle's matrix route, and that the hand-written adjoint is the exact
transpose of the collision's Jacobian.
"""
import ctypes
import os

import numpy as np
import pytest

from oracle import collide as C
from oracle.lattice import Relax, d3q27

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOSTLIB = os.path.join(ROOT, "paper_1202_6074_amd", "libcmlbm_hostmath.so")
LAT = d3q27()
RATES = dict(omega_shear=1.37, omega_bulk=1.21, omega3=(0.93, 1.41, 1.12), omega4=(1.31, 0.87), omega5=1.19,
             omega6=1.63)


@pytest.fixture(scope="module")
def hm():
    if not os.path.exists(HOSTLIB):
        from paper_1202_6074_amd.build import build_hostmath
        build_hostmath()
    lib = ctypes.CDLL(HOSTLIB)
    P = ctypes.c_void_p
    for name in ("cmhost_collide_f64", "cmhost_collide_f32"):
        getattr(lib, name).argtypes = [P, P, P, ctypes.c_int, ctypes.c_long, P]
    lib.cmhost_adjoint_f64.argtypes = [P, P, P, ctypes.c_int, P, ctypes.c_long, P, P]
    lib.cmhost_equilibrium_f64.argtypes = [P, P, P, ctypes.c_double, ctypes.c_long, P, ctypes.c_int]
    return lib


def _rates(r: Relax, rho0=1.0):
    flags = (1 if r.factorized else 0) | (2 if r.reduced_compressibility else 0)
    return np.array([rho0, r.omega_shear, r.omega_bulk, *r.omega3, *r.omega4, r.omega5, r.omega6, r.cs_smag,
                     float(flags)])


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def host_collide(hm, f, F, relax, dtype=np.float64):
    f = np.ascontiguousarray(f, dtype=dtype)
    F = np.ascontiguousarray(F, dtype=dtype)
    out = np.empty_like(f)
    rates = _rates(relax)
    fn = hm.cmhost_collide_f64 if dtype == np.float64 else hm.cmhost_collide_f32
    fn(_ptr(f), _ptr(F), _ptr(rates), int(relax.cs_smag > 0), f.shape[1], _ptr(out))
    return out


def host_adjoint(hm, f, F, relax, lam_post):
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    lam_post = np.ascontiguousarray(lam_post, dtype=np.float64)
    lam_pre = np.empty_like(f)
    gF = np.empty_like(F)
    rates = _rates(relax)
    hm.cmhost_adjoint_f64(_ptr(f), _ptr(F), _ptr(rates), int(relax.cs_smag > 0), _ptr(lam_post), f.shape[1],
                          _ptr(lam_pre), _ptr(gF))
    return lam_pre, gF


def _state(n=200, seed=21, famp=0.01, uamp=0.1):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = uamp * rng.standard_normal((3, n))
    F = famp * rng.standard_normal((3, n))
    feq = C.product_equilibrium(rho, u, LAT)
    f = feq * (1 + 0.05 * rng.standard_normal(feq.shape))
    return f, F


@pytest.mark.parametrize("cs", [0.0, 0.12])
def test_collision_f64_matches_oracle(hm, cs):
    f, F = _state()
    r = Relax(cs_smag=cs, **RATES)
    got = host_collide(hm, f, F, r)
    want = C.collide(f, F, LAT, r)
    assert np.abs(got - want).max() < 2e-15


@pytest.mark.parametrize("rc,fact", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("cs", [0.0, 0.12])
def test_collision_variants_f64_match_oracle(hm, cs, rc, fact):
    f, F = _state()
    r = Relax(cs_smag=cs, reduced_compressibility=rc, factorized=fact, **RATES)
    got = host_collide(hm, f, F, r)
    want = C.collide(f, F, LAT, r, rho0=1.0)
    assert np.abs(got - want).max() < 3e-15


@pytest.mark.parametrize("cs", [0.0, 0.12])
def test_collision_f32_matches_oracle(hm, cs):
    f, F = _state()
    r = Relax(cs_smag=cs, **RATES)
    got = host_collide(hm, f, F, r, np.float32).astype(np.float64)
    want = C.collide(f.astype(np.float32).astype(np.float64), F.astype(np.float32).astype(np.float64), LAT, r)
    # FP32 arithmetic on deviations from the rest state: errors ~ eps * |f - w|
    assert np.abs(got - want).max() < 2e-7


def test_equilibrium_matches_oracle(hm):
    rng = np.random.default_rng(5)
    n = 50
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((3, n))
    F = 0.01 * rng.standard_normal((3, n))
    out = np.empty((27, n))
    for rc in (0, 1):
        hm.cmhost_equilibrium_f64(_ptr(rho), _ptr(np.ascontiguousarray(u)), _ptr(np.ascontiguousarray(F)), 1.0, n,
                                  _ptr(out), rc)
        want = C.equilibrium_state(rho, u, F, LAT, 1.0 if rc else None)
        assert np.abs(out - want).max() < 2e-16 * 8


ADJ_CASES = [(0.0, False, False), (0.3, False, False), (0.0, True, False), (0.0, False, True), (0.3, True, True)]


@pytest.mark.parametrize("cs,fact,rc", ADJ_CASES)
def test_adjoint_dot_product_and_finite_differences(hm, cs, fact, rc):
    """<J v, w> = <v, J^T w> with J from central differences of the host
    collision (exact to FD error), and the same for dC/dF; with the eddy rate
    (cs > 0) the Jacobian includes the rate's dependence on the moments, with
    the Sec. 12-13 flags that of the velocity and the attractors."""
    f, F = _state(n=40, seed=3)
    r = Relax(cs_smag=cs, factorized=fact, reduced_compressibility=rc, **RATES)
    rng = np.random.default_rng(4)
    w = rng.standard_normal(f.shape)
    lam_pre, gF = host_adjoint(hm, f, F, r, w)
    # the central differences' error is eps^2 times the third derivatives,
    # which the eddy rate's square roots make larger (1e-8 at eps = 1e-6)
    eps = 1e-6 if cs == 0 else 1e-7
    for trial in range(3):
        v = rng.standard_normal(f.shape)
        Jv = (host_collide(hm, f + eps * v, F, r) - host_collide(hm, f - eps * v, F, r)) / (2 * eps)
        lhs = (Jv * w).sum(axis=0)
        rhs = (v * lam_pre).sum(axis=0)
        assert np.abs(lhs - rhs).max() < 1e-8 * np.abs(rhs).max()
        vF = rng.standard_normal(F.shape)
        JF = (host_collide(hm, f, F + eps * vF, r) - host_collide(hm, f, F - eps * vF, r)) / (2 * eps)
        lhsF = (JF * w).sum(axis=0)
        rhsF = (vF * gF).sum(axis=0)
        assert np.abs(lhsF - rhsF).max() < 1e-8 * np.abs(rhsF).max()


@pytest.mark.parametrize("cs,fact,rc", ADJ_CASES)
def test_adjoint_matches_oracle_jacobian(hm, cs, fact, rc):
    """The adjoint against the oracle's collision differentiated by central
    differences (with cs > 0, through the oracle's Smagorinsky rate; with the
    flags, through the oracle's Sec. 12-13 operators)."""
    f, F = _state(n=6, seed=9)
    r = Relax(cs_smag=cs, factorized=fact, reduced_compressibility=rc, **RATES)
    rng = np.random.default_rng(10)
    w = rng.standard_normal(f.shape)
    lam_pre, gF = host_adjoint(hm, f, F, r, w)
    eps = 1e-6
    J = np.zeros((27, 27, f.shape[1]))
    for i in range(27):
        d = np.zeros_like(f)
        d[i] = eps
        J[:, i] = (C.collide(f + d, F, LAT, r) - C.collide(f - d, F, LAT, r)) / (2 * eps)
    want = np.einsum("ijc,ic->jc", J, w)
    assert np.abs(lam_pre - want).max() < 1e-7 * np.abs(want).max()
    JF = np.zeros((27, 3, f.shape[1]))
    for dd in range(3):
        d = np.zeros_like(F)
        d[dd] = eps
        JF[:, dd] = (C.collide(f, F + d, LAT, r) - C.collide(f, F - d, LAT, r)) / (2 * eps)
    wantF = np.einsum("ijc,ic->jc", JF, w)
    assert np.abs(gF - wantF).max() < 1e-7 * np.abs(wantF).max()


def test_adjoint_with_eddy_rate_at_isotropic_state_is_the_plain_adjoint(hm):
    """Where the traceless second moments vanish (Q = 0: the rest state, F = 0)
    the eddy rate is omega_shear and its derivative is taken as 0, so the
    adjoint with eddy viscosity equals the plain one bit for bit; at a generic
    state the two differ."""
    n = 8
    f = np.repeat(LAT.w[:, None], n, axis=1).astype(np.float64)
    F = np.zeros((3, n))
    rng = np.random.default_rng(12)
    w = rng.standard_normal(f.shape)
    les = host_adjoint(hm, f, F, Relax(cs_smag=0.3, **RATES), w)
    plain = host_adjoint(hm, f, F, Relax(**RATES), w)
    assert np.array_equal(les[0], plain[0]) and np.array_equal(les[1], plain[1])
    f2, F2 = _state(n=n, seed=13)
    les2 = host_adjoint(hm, f2, F2, Relax(cs_smag=0.3, **RATES), w)
    plain2 = host_adjoint(hm, f2, F2, Relax(**RATES), w)
    assert np.abs(les2[0] - plain2[0]).max() > 1e-6


@pytest.mark.parametrize("rc,fact", [(False, False), (True, True)])
def test_collision_with_sgs_force_matches_oracle(hm, rc, fact):
    """Sec. 14 coupling: force F + rho a', and the sub-grid stress of the step
    from the pre-collision moments (oracle.sgs)."""
    from oracle import sgs as SG
    hm.cmhost_collide_sgs_f64.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_long] + [ctypes.c_void_p] * 2
    f, F = _state(seed=41)
    rng = np.random.default_rng(42)
    acc = np.ascontiguousarray(1e-3 * rng.standard_normal(F.shape))
    r = Relax(cs_smag=0.3, sgs_force=True, reduced_compressibility=rc, factorized=fact, **RATES)
    rates = _rates(r)
    rates[-1] += 4.0
    out = np.empty_like(f)
    st = np.empty((6, f.shape[1]))
    hm.cmhost_collide_sgs_f64(_ptr(f), _ptr(F), _ptr(acc), _ptr(rates), f.shape[1], _ptr(out), _ptr(st))
    rho = f.sum(axis=0)
    Ft = F + rho * acc
    want, parts = C.collide(f, Ft, LAT, r, return_parts=True, rho0=1.0)
    assert np.abs(out - want).max() < 3e-15
    rho_s = np.ones_like(rho) if rc else parts["rho"]
    Rw = SG.sgs_stress(parts["kbar"], rho_s, LAT, r.omega_shear, r.cs_smag)
    want_st = np.array([Rw[0, 0], Rw[1, 1], Rw[2, 2], Rw[0, 1], Rw[0, 2], Rw[1, 2]])
    assert np.abs(st - want_st).max() < 1e-12 * np.abs(want_st).max()
    assert np.abs(want_st).max() > 1e-6
