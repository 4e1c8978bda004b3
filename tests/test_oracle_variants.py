"""Pins of the reduced-compressibility (Sec. 12) and factorized-attractor
(Sec. 13) variants of the collision (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import collide as C
from oracle import d2q9_paper as P
from oracle.lattice import Relax, d2q9, d3q27
from oracle.sim import OracleSim

L2 = d2q9()
L3 = d3q27()
W = (1.1, 1.3, 1.4, 0.9, 1.7, 1.2)
COMBOS = [(False, True), (True, False), (True, True)]


def relax2(rc, fact):
    return Relax(omega_shear=1.3, omega_bulk=W[0], d2q9_omega45=(W[1], W[2]), d2q9_omega678=W[3:],
                 reduced_compressibility=rc, factorized=fact)


def _inputs(n=40, seed=21, famp=0.01):
    rng = np.random.default_rng(seed)
    f = L2.w[:, None] * (1 + 0.2 * rng.standard_normal((9, n)))
    return f, famp * rng.standard_normal((2, n))


@pytest.mark.parametrize("rc,fact", COMBOS)
def test_force_free_variants_equal_paper(rc, fact):
    f, F = _inputs()
    F[:] = 0
    got = C.collide(f, F, L2, relax2(rc, fact), rho0=1.0)
    want = P.collide(f, F, W, rho0=1.0 if rc else None, factorized=fact)
    assert np.abs(got - want).max() < 1e-14


@pytest.mark.parametrize("rc,fact", COMBOS)
def test_forced_variants_second_order_and_sigma_structure(rc, fact):
    f, F = _inputs(famp=0.02)
    got, parts = C.collide(f, F, L2, relax2(rc, fact), return_parts=True, rho0=1.0)
    want = P.collide(f, F, W, rho0=1.0 if rc else None, factorized=fact)
    u, sig = parts["u"], parts["sigma"]
    d = C.central_moments(want, u, L2) - C.central_moments(got, u, L2)
    for e in ((0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1)):
        assert np.abs(d[L2.moment_index(e)]).max() < 1e-15, e
    ixxy, ixyy, i4 = L2.moment_index((2, 1)), L2.moment_index((1, 2)), L2.moment_index((2, 2))
    assert np.abs(d[ixxy] - W[3] * sig[ixxy]).max() < 1e-16
    assert np.abs(d[ixyy] - W[4] * sig[ixyy]).max() < 1e-16
    extra = 0.0
    if fact:
        # Sec. 13 replaces rho/9 in g_8, which it calls kappabar^M_xxyy, by the
        # transformed factorized attractor (Eq. factorxxyyfinal, which already
        # carries -sigma_xxyy/2). But rho/9 is the untransformed kappa^M_xxyy:
        # g_8 takes -sigma/2 through sigma'_xxyy as well, so the printed
        # replacement subtracts sigma_xxyy/2 twice. The oracle relaxes towards
        # kappa^at - sigma/2 once.
        extra = -W[5] * 0.5 * sig[i4]
    assert np.abs(d[i4] + W[5] * (u[1] * sig[ixxy] + u[0] * sig[ixyy]) - extra).max() < 4e-16


def test_factorized_attractor_is_maxwellian_at_equilibrium():
    # with the post-collision second moments at rho cs^2 the product / rho is rho cs^4 (Sec. 13)
    rng = np.random.default_rng(3)
    n = 10
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((3, n))
    feq = C.product_equilibrium(rho, u, L3)
    r = Relax(omega_shear=1.4, omega4=(0.8, 1.2), omega6=0.7, factorized=True)
    assert np.abs(C.collide(feq, np.zeros((3, n)), L3, r) - feq).max() < 1e-15


@pytest.mark.parametrize("rc,fact", COMBOS)
def test_variants_conserve_mass_and_add_force(rc, fact):
    rng = np.random.default_rng(4)
    n = 30
    feq = C.product_equilibrium(1 + 0.05 * rng.standard_normal(n), 0.08 * rng.standard_normal((3, n)), L3)
    f = feq * (1 + 0.05 * rng.standard_normal(feq.shape))
    F = 0.01 * rng.standard_normal((3, n))
    r = Relax(omega_shear=1.5, omega_bulk=1.2, omega3=(1.1, 0.9, 1.3), cs_smag=0.1, reduced_compressibility=rc,
              factorized=fact)
    post = C.collide(f, F, L3, r, rho0=1.0)
    assert np.abs((post - f).sum(axis=0)).max() < 1e-15
    assert np.abs(L3.e.T @ (post - f) - F).max() < 1e-15


def test_factorized_is_galilean_invariant():
    rng = np.random.default_rng(6)
    n = 20
    F = 0.01 * rng.standard_normal((3, n))
    feq = C.product_equilibrium(1 + 0.05 * rng.standard_normal(n), 0.05 * rng.standard_normal((3, n)), L3)
    f_ref = feq * (1 + 0.05 * rng.standard_normal(feq.shape))
    _, u_r = C.macroscopic(f_ref, F, L3)
    kbar = C.central_moments(f_ref, u_r, L3)
    r = Relax(omega_shear=1.5, omega4=(0.8, 1.1), factorized=True, cs_smag=0.1)
    outs = []
    for shift in (np.zeros(3), np.array([0.07, -0.04, 0.03])):
        u = u_r + shift[:, None]
        f = L3.Minv @ C.frame_shift(kbar, u, L3)
        outs.append(C.central_moments(C.collide(f, F, L3, r), u, L3))
    assert np.abs(outs[1] - outs[0]).max() < 1e-14


def test_reduced_compressibility_equilibrium_reads_back():
    rng = np.random.default_rng(7)
    n = 12
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((3, n))
    F = 0.01 * rng.standard_normal((3, n))
    f0 = C.equilibrium_state(rho, u, F, L3, rho0=1.0)
    r2, u2 = C.macroscopic(f0, F, L3, rho0=1.0)
    assert np.abs(r2 - rho).max() < 1e-14 and np.abs(u2 - u).max() < 1e-15
    # force-free: a fixed point of the reduced-compressibility collision
    f1 = C.equilibrium_state(rho, u, 0 * F, L3, rho0=1.0)
    r = Relax(omega_shear=1.3, reduced_compressibility=True, factorized=True)
    assert np.abs(C.collide(f1, 0 * F, L3, r, rho0=1.0) - f1).max() < 1e-15


@pytest.mark.parametrize("rc,fact", COMBOS)
def test_variants_keep_chapman_enskog_viscosity(rc, fact):
    omega = 1.8
    L = 32
    shape = (1, L, 1)
    sim = OracleSim(shape, Relax(omega_shear=omega, reduced_compressibility=rc, factorized=fact))
    rho, u = synth.shear_wave(shape, amp=1e-4)
    sim.init_equilibrium(rho, u)
    k = 2 * np.pi / L
    nu = (1 / omega - 0.5) / 3
    y = np.arange(L)
    amp = lambda: 2 * np.mean(sim.moments()[1][0, 0, :, 0] * np.sin(k * y))
    t1, t2 = int(0.1 / (nu * k * k)), int(0.6 / (nu * k * k))
    sim.step(t1)
    a1 = amp()
    sim.step(t2 - t1)
    a2 = amp()
    assert abs(np.log(a1 / a2) / (k * k * (t2 - t1)) / nu - 1) < 5e-3
