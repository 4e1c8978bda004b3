"""Pins for the torch/autograd reference gradient (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import collide as C
from oracle.grad import TorchStep, energy_gradient
from oracle.lattice import Relax, d3q27
from oracle.sim import OracleSim

LAT = d3q27()
RELAX = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3))


def test_torch_collision_equals_oracle():
    import torch
    rng = np.random.default_rng(1)
    n = 30
    f = C.product_equilibrium(1 + 0.05 * rng.standard_normal(n), 0.1 * rng.standard_normal((3, n)), LAT)
    f *= 1 + 0.05 * rng.standard_normal(f.shape)
    F = 0.01 * rng.standard_normal((3, n))
    got = TorchStep(LAT, RELAX).collide(torch.tensor(f), torch.tensor(F)).numpy()
    assert np.abs(got - C.collide(f, F, LAT, RELAX)).max() < 1e-15


def test_energy_and_gradient_against_oracle_and_finite_differences():
    shape = (4, 4, 4)
    n = 64
    rho, u = synth.taylor_green_3d(shape, u0=0.02)
    F = synth.smooth_random_force(shape, sigma=1.0, frms=1e-4).reshape(3, n)
    f0 = C.equilibrium_state(rho.reshape(-1), u.reshape(3, -1), np.zeros((3, n)), LAT)
    E, g = energy_gradient(LAT, RELAX, f0, F, 6, shape)
    sim = OracleSim(shape, RELAX, force=F)
    sim.set_populations(f0)
    sim.step(6)
    assert abs(sim.reduce()["ke"] - E) < 1e-15
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.standard_normal(F.shape)
        eps = 1e-6
        ep = energy_gradient(LAT, RELAX, f0, F + eps * v, 6, shape)[0]
        em = energy_gradient(LAT, RELAX, f0, F - eps * v, 6, shape)[0]
        fd = (ep - em) / (2 * eps)
        assert abs(fd - (g * v).sum()) < 1e-6 * abs(fd)


def test_torch_stream_with_walls_equals_oracle_stream():
    import torch
    from oracle.stream import stream
    rng = np.random.default_rng(3)
    shape = (3, 5, 4)
    fpost = rng.standard_normal((27,) + shape)
    u_lo, u_hi = (0.01, -0.02, 0.005), (0.03, 0.0, -0.01)
    st = TorchStep(LAT, RELAX, walls=True, u_lo=u_lo, u_hi=u_hi)
    got = st.stream(torch.tensor(fpost.reshape(27, -1)), shape).numpy().reshape(fpost.shape)
    ref = stream(fpost, LAT, True, u_lo, u_hi)
    assert np.abs(got - ref).max() == 0.0


def test_energy_gradient_with_moving_walls_against_oracle_and_finite_differences():
    shape = (3, 5, 4)   # (nz, ny, nx)
    n = 60
    walls = dict(walls=True, u_lo=(0.0, 0.0, 0.0), u_hi=(0.02, 0.0, 0.0))
    rho, u = synth.taylor_green_3d(shape, u0=0.02)
    F = synth.smooth_random_force(shape, sigma=1.0, frms=1e-4).reshape(3, n)
    f0 = C.equilibrium_state(rho.reshape(-1), u.reshape(3, -1), np.zeros((3, n)), LAT)
    E, g = energy_gradient(LAT, RELAX, f0, F, 5, shape, **walls)
    sim = OracleSim(shape, RELAX, force=F, walls=True, u_lo=walls["u_lo"], u_hi=walls["u_hi"])
    sim.set_populations(f0)
    sim.step(5)
    assert abs(sim.reduce()["ke"] - E) < 1e-14 * abs(E)
    rng = np.random.default_rng(5)
    for _ in range(3):
        v = rng.standard_normal(F.shape)
        eps = 1e-6
        ep = energy_gradient(LAT, RELAX, f0, F + eps * v, 5, shape, **walls)[0]
        em = energy_gradient(LAT, RELAX, f0, F - eps * v, 5, shape, **walls)[0]
        fd = (ep - em) / (2 * eps)
        assert abs(fd - (g * v).sum()) < 1e-6 * abs(fd)


RELAX_LES = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), cs_smag=0.3)


def test_torch_collision_with_eddy_rate_equals_oracle():
    import torch
    rng = np.random.default_rng(11)
    n = 30
    f = C.product_equilibrium(1 + 0.05 * rng.standard_normal(n), 0.1 * rng.standard_normal((3, n)), LAT)
    f *= 1 + 0.05 * rng.standard_normal(f.shape)
    F = 0.01 * rng.standard_normal((3, n))
    got = TorchStep(LAT, RELAX_LES).collide(torch.tensor(f), torch.tensor(F)).numpy()
    want = C.collide(f, F, LAT, RELAX_LES)
    assert np.abs(got - want).max() < 1e-15
    assert np.abs(want - C.collide(f, F, LAT, RELAX)).max() > 1e-5   # the eddy rate acts


def test_eddy_rate_derivative_is_zero_where_the_traceless_moments_vanish():
    """Q = sqrt(2 Pi^d : Pi^d) has no derivative at Pi^d = 0; the reference takes
    it as 0 there, so the rate is omega_shear with a zero gradient."""
    import torch
    st = TorchStep(LAT, RELAX_LES)
    kbar = torch.zeros((27, 4), dtype=torch.float64)
    for a in range(3):
        ex = [0, 0, 0]
        ex[a] = 2
        kbar[LAT.moment_index(ex)] = 1.0 / 3.0   # isotropic: Pi^d = 0
    kbar.requires_grad_(True)
    rho = torch.ones(4, dtype=torch.float64, requires_grad=True)
    om = st.eddy_rate(kbar, rho)
    om.sum().backward()
    assert torch.equal(om.detach(), torch.full((4,), 1.6, dtype=torch.float64))
    assert not kbar.grad.any() and not rho.grad.any()


def test_energy_gradient_with_eddy_viscosity_against_oracle_and_finite_differences():
    shape = (4, 4, 4)
    n = 64
    rho, u = synth.taylor_green_3d(shape, u0=0.05)
    F = synth.smooth_random_force(shape, sigma=1.0, frms=1e-4).reshape(3, n)
    f0 = C.equilibrium_state(rho.reshape(-1), u.reshape(3, -1), np.zeros((3, n)), LAT)
    E, g = energy_gradient(LAT, RELAX_LES, f0, F, 6, shape)
    sim = OracleSim(shape, RELAX_LES, force=F)
    sim.set_populations(f0)
    sim.step(6)
    assert abs(sim.reduce()["ke"] - E) < 1e-14 * abs(E)
    assert abs(E - energy_gradient(LAT, RELAX, f0, F, 6, shape)[0]) > 1e-6 * abs(E)   # the eddy rate acts
    rng = np.random.default_rng(6)
    for _ in range(3):
        v = rng.standard_normal(F.shape)
        eps = 1e-6
        ep = energy_gradient(LAT, RELAX_LES, f0, F + eps * v, 6, shape)[0]
        em = energy_gradient(LAT, RELAX_LES, f0, F - eps * v, 6, shape)[0]
        fd = (ep - em) / (2 * eps)
        assert abs(fd - (g * v).sum()) < 1e-6 * abs(fd)


@pytest.mark.parametrize("fact,rc,cs", [(True, False, 0.0), (False, True, 0.0), (True, True, 0.0), (True, True, 0.3)])
def test_torch_collision_with_variants_equals_oracle(fact, rc, cs):
    """Secs. 12-13: reduced compressibility (rho0 u = sum fbar e + F/2) and the
    factorized attractors, with and without the eddy rate, against
    oracle.collide."""
    import torch
    rng = np.random.default_rng(21)
    n = 30
    f = C.product_equilibrium(1 + 0.05 * rng.standard_normal(n), 0.1 * rng.standard_normal((3, n)), LAT)
    f *= 1 + 0.05 * rng.standard_normal(f.shape)
    F = 0.01 * rng.standard_normal((3, n))
    r = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), omega4=(1.3, 0.8), cs_smag=cs,
              factorized=fact, reduced_compressibility=rc)
    got = TorchStep(LAT, r).collide(torch.tensor(f), torch.tensor(F)).numpy()
    want = C.collide(f, F, LAT, r)
    assert np.abs(got - want).max() < 1e-15
    plain = C.collide(f, F, LAT, Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), omega4=(1.3, 0.8),
                                       cs_smag=cs))
    assert np.abs(want - plain).max() > 1e-6   # the variant acts


@pytest.mark.parametrize("fact,rc", [(True, True), (True, False), (False, True)])
def test_energy_gradient_with_variants_against_oracle_and_finite_differences(fact, rc):
    shape = (4, 4, 4)
    n = 64
    r = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), omega4=(1.3, 0.8), cs_smag=0.2,
              factorized=fact, reduced_compressibility=rc)
    rho, u = synth.taylor_green_3d(shape, u0=0.05)
    F = synth.smooth_random_force(shape, sigma=1.0, frms=1e-4).reshape(3, n)
    f0 = C.equilibrium_state(rho.reshape(-1), u.reshape(3, -1), np.zeros((3, n)), LAT, 1.0 if rc else None)
    E, g = energy_gradient(LAT, r, f0, F, 6, shape)
    sim = OracleSim(shape, r, force=F)
    sim.set_populations(f0)
    sim.step(6)
    assert abs(sim.reduce()["ke"] - E) < 1e-12 * abs(E)   # the same E, summed in another order
    rng = np.random.default_rng(8)
    for _ in range(3):
        v = rng.standard_normal(F.shape)
        eps = 1e-6
        ep = energy_gradient(LAT, r, f0, F + eps * v, 6, shape)[0]
        em = energy_gradient(LAT, r, f0, F - eps * v, 6, shape)[0]
        fd = (ep - em) / (2 * eps)
        assert abs(fd - (g * v).sum()) < 1e-6 * abs(fd)
