"""GPU adjoint: the hand-written adjoint step and the checkpointed backward
pass against the FP64 autograd reference and finite differences."""
import numpy as np
import pytest

import synth
from oracle import collide as C
from oracle.grad import energy_gradient
from oracle.lattice import Relax, d3q27

pytestmark = pytest.mark.gpu
LAT = d3q27()
RELAX = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3))
RELAX_LES = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), cs_smag=0.3)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(shape_xyz, storage, F, u0=0.03, walls=False, relax=RELAX):
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    nx, ny, nz = shape_xyz
    lat = Lattice(shape_xyz, storage=storage, walls=walls, wall_u_hi=(0.02, 0.0, 0.0) if walls else (0.0, 0.0, 0.0))
    lat.set_relaxation(relax.omega_shear, relax.omega_bulk, relax.omega3, relax.omega4, cs_smag=relax.cs_smag,
                       factorized=relax.factorized, reduced_compressibility=relax.reduced_compressibility)
    dt = lat.dtype
    lat.set_force((0, 0, 0), torch.tensor(F, device="cuda", dtype=dt))
    rho, u = synth.taylor_green_3d((nz, ny, nx), u0=u0)
    # initial populations independent of F: force-free equilibrium
    lat.set_force((0, 0, 0), torch.zeros_like(torch.tensor(F, device="cuda", dtype=dt)))
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    f0_state = lat.state_buffer().clone()
    f0 = lat.populations().cpu().numpy().reshape(27, -1)
    return lat, f0_state, f0


@pytest.mark.parametrize("K", [5, 4, 13, 100])   # 13, 100 >= nsteps: every state kept
def test_checkpointed_gradient_fp64_matches_autograd(K):
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (6, 5, 4)
    nx, ny, nz = shape
    F = synth.smooth_random_force((nz, ny, nx), sigma=1.0, frms=1e-3)
    lat, f0_state, f0 = _setup(shape, "f64", F)
    nsteps = 13
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, nsteps, K)
    E_ref, g_ref = energy_gradient(LAT, RELAX, f0, F.reshape(3, -1), nsteps, (nz, ny, nx))
    assert abs(E - E_ref) < 1e-13 * abs(E_ref)
    g = g.cpu().numpy().reshape(3, -1)
    assert np.abs(g - g_ref).max() < 1e-10 * np.abs(g_ref).max()


@pytest.mark.parametrize("walls", [False, True])
def test_adjoint_fp32_matches_fp64_reference(walls):
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (8, 8, 8)
    F = synth.smooth_random_force((8, 8, 8), sigma=2.0, frms=1e-4)
    lat, f0_state, f0 = _setup(shape, "f32", F, walls=walls)
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda", dtype=torch.float32), f0_state, 20, 6)
    wk = dict(walls=True, u_hi=(0.02, 0.0, 0.0)) if walls else {}
    E_ref, g_ref = energy_gradient(LAT, RELAX, f0, F.reshape(3, -1), 20, (8, 8, 8), **wk)
    g = g.cpu().numpy().reshape(3, -1).astype(np.float64)
    assert abs(E - E_ref) < 1e-5 * abs(E_ref)
    assert np.abs(g - g_ref).max() < 1e-3 * np.abs(g_ref).max()


@pytest.mark.parametrize("les", [False, True])
@pytest.mark.parametrize("walls", [False, True])
def test_adjoint_step_dot_product_fp64(walls, les):
    """<P C(f + eps v) - P C(f - eps v), w> / 2 eps = <v, adjoint(w)> for one step
    (with walls, the upper one moving: the wall term is a constant and cancels;
    with eddy viscosity, the rate's dependence on the moments included)."""
    torch = _torch()
    shape = (9, 7, 5)
    rng = np.random.default_rng(7)
    F = 1e-3 * rng.standard_normal((3, 5, 7, 9))
    lat, _, _ = _setup(shape, "f64", F, u0=0.05, walls=walls, relax=RELAX_LES if les else RELAX)
    lat.set_force((0, 0, 0), torch.tensor(F, device="cuda"))
    f = lat.populations()
    if les:
        # away from the Taylor-Green nodes where u = 0: there Q is of the
        # order of |F|^2, and a perturbation of 1e-6 would cross the cone
        # Q = |Pi^d| that has no derivative at its tip
        f = f * (1 + 0.05 * torch.tensor(rng.standard_normal(f.shape), device="cuda"))
    v = torch.tensor(rng.standard_normal(f.shape), device="cuda")
    w = torch.tensor(rng.standard_normal(f.shape), device="cuda")
    eps = 1e-6 if not les else 1e-7   # central differences: error ~ eps^2 x third derivatives
    outs = []
    for sgn in (1, -1):
        lat.set_populations(f + sgn * eps * v)
        lat.step(1)
        outs.append(lat.populations())
    lhs = float(((outs[0] - outs[1]) / (2 * eps) * w).sum())
    lat.set_populations(f)
    lam = lat.lam_buffer()
    gF = torch.zeros((3, 5, 7, 9), dtype=torch.float64, device="cuda")
    lat.adjoint_step(lat.state_buffer(), lat.lam_from_planes(w), lam, gF)
    rhs = float((v * lat.lam_to_planes(lam)).sum())
    assert abs(lhs - rhs) < 1e-7 * abs(rhs)


def test_zero_steps_and_invalid_arguments():
    """nsteps = 0: E is the energy of the initial state, which depends on F
    only through the F/2 term of u (the energy seed's gradient); K < 1 and
    nsteps < 0 are refused before any work."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (6, 5, 4)
    nx, ny, nz = shape
    F = synth.smooth_random_force((nz, ny, nx), sigma=1.0, frms=1e-3)
    lat, f0_state, f0 = _setup(shape, "f64", F)
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, 0, 5)
    E_ref, g_ref = energy_gradient(LAT, RELAX, f0, F.reshape(3, -1), 0, (nz, ny, nx))
    assert abs(E - E_ref) < 1e-13 * abs(E_ref)
    assert np.abs(g.cpu().numpy().reshape(3, -1) - g_ref).max() < 1e-12 * np.abs(g_ref).max()
    for nsteps, K in ((5, 0), (-1, 5)):
        with pytest.raises(ValueError):
            energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, nsteps, K)


def test_keep_every_state_gives_the_checkpointed_gradient_bitwise():
    """K >= nsteps keeps every forward state instead of recomputing segments:
    the same kernels run on the same states, so E and dE/dF are bitwise those
    of the checkpointed pass."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (16, 12, 10)
    nx, ny, nz = shape
    F = synth.smooth_random_force((nz, ny, nx), sigma=2.0, frms=1e-4)
    out = []
    for K in (4, 40):
        lat, f0_state, _ = _setup(shape, "f32", F)
        E, g = energy_and_grad(lat, torch.tensor(F, device="cuda", dtype=torch.float32), f0_state, 17, K)
        out.append((E, g.cpu().numpy()))
        lat.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("K", [4, 13])   # checkpointed, and every state kept
def test_gradient_with_moving_walls_fp64_matches_autograd(K):
    """Halfway bounce-back walls at y = -1/2 and ny - 1/2, the upper one moving:
    the adjoint transposes the bounce-back (reference: autograd through the
    oracle's wall streaming)."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    from paper_1202_6074_amd.lattice import Lattice
    nx, ny, nz = 6, 5, 4
    u_hi = (0.02, 0.0, 0.0)
    lat = Lattice((nx, ny, nz), storage="f64", walls=True, wall_u_hi=u_hi)
    lat.set_relaxation(RELAX.omega_shear, RELAX.omega_bulk, RELAX.omega3)
    F = synth.smooth_random_force((nz, ny, nx), sigma=1.0, frms=1e-3)
    rho, u = synth.taylor_green_3d((nz, ny, nx), u0=0.03)
    lat.set_force((0, 0, 0), torch.zeros((3, nz, ny, nx), dtype=torch.float64, device="cuda"))
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    f0_state = lat.state_buffer().clone()
    f0 = lat.populations().cpu().numpy().reshape(27, -1)
    nsteps = 13
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, nsteps, K)
    E_ref, g_ref = energy_gradient(LAT, RELAX, f0, F.reshape(3, -1), nsteps, (nz, ny, nx),
                                   walls=True, u_hi=u_hi)
    assert abs(E - E_ref) < 1e-13 * abs(E_ref)
    g = g.cpu().numpy().reshape(3, -1)
    assert np.abs(g - g_ref).max() < 1e-10 * np.abs(g_ref).max()


@pytest.mark.parametrize("K", [5, 100])   # checkpointed, and every state kept
@pytest.mark.parametrize("walls", [False, True])
def test_gradient_with_eddy_viscosity_fp64_matches_autograd(K, walls):
    """Smagorinsky eddy viscosity (C_s = 0.3, strong enough to matter): the GPU
    FP64 checkpointed adjoint against autograd through the reference step with
    the eddy rate, over 13 steps of a Taylor-Green start."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (6, 5, 4)
    nx, ny, nz = shape
    F = synth.smooth_random_force((nz, ny, nx), sigma=1.0, frms=1e-3)
    lat, f0_state, f0 = _setup(shape, "f64", F, u0=0.05, walls=walls, relax=RELAX_LES)
    nsteps = 13
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, nsteps, K)
    wk = dict(walls=True, u_hi=(0.02, 0.0, 0.0)) if walls else {}
    E_ref, g_ref = energy_gradient(LAT, RELAX_LES, f0, F.reshape(3, -1), nsteps, (nz, ny, nx), **wk)
    E_plain, g_plain = energy_gradient(LAT, RELAX, f0, F.reshape(3, -1), nsteps, (nz, ny, nx), **wk)
    assert np.abs(g_ref - g_plain).max() > 1e-3 * np.abs(g_ref).max()   # the eddy rate matters here
    assert abs(E - E_ref) < 1e-13 * abs(E_ref)
    g = g.cpu().numpy().reshape(3, -1)
    assert np.abs(g - g_ref).max() < 1e-10 * np.abs(g_ref).max()


def test_adjoint_fp32_with_eddy_viscosity_matches_fp64_reference():
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (8, 8, 8)
    F = synth.smooth_random_force((8, 8, 8), sigma=2.0, frms=1e-4)
    relax = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), cs_smag=0.12)
    lat, f0_state, f0 = _setup(shape, "f32", F, u0=0.05, relax=relax)
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda", dtype=torch.float32), f0_state, 20, 6)
    E_ref, g_ref = energy_gradient(LAT, relax, f0, F.reshape(3, -1), 20, (8, 8, 8))
    g = g.cpu().numpy().reshape(3, -1).astype(np.float64)
    assert abs(E - E_ref) < 1e-5 * abs(E_ref)
    assert np.abs(g - g_ref).max() < 1e-3 * np.abs(g_ref).max()


def test_energy_seed_in_the_row_layout_of_lambda():
    """lambda uses the populations' row layout ((z ny + y) 27 + i) nx + x: the
    seed read back through lam_to_planes is u.e_i - |u|^2/2 at every cell, with
    u of Eq. velocitycalculation, and the plane conversions invert each other."""
    torch = _torch()
    shape = (9, 7, 5)
    rng = np.random.default_rng(17)
    F = 1e-3 * rng.standard_normal((3, 5, 7, 9))
    lat, _, _ = _setup(shape, "f64", F, u0=0.05)
    lat.set_force((0, 0, 0), torch.tensor(F, device="cuda"))
    lam = lat.lam_buffer()
    g = torch.empty((3, 5, 7, 9), dtype=torch.float64, device="cuda")
    lat.energy_seed(lat.state_buffer(), lam, g)
    _, u = lat.moments()
    planes = lat.lam_to_planes(lam)
    hu2 = 0.5 * (u * u).sum(0)
    for i in range(27):
        e = LAT.e[i]
        want = e[0] * u[0] + e[1] * u[1] + e[2] * u[2] - hu2
        assert torch.abs(planes[i] - want).max() < 1e-15
    assert torch.abs(g - 0.5 * u).max() < 1e-16
    assert torch.equal(lat.lam_from_planes(planes), lam)
    assert lam.shape == (5, 7, 27, 9)


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("les,walls", [(False, False), (True, True)])
def test_adjoint_over_many_planes_in_chunks_and_one_launch(storage, les, walls):
    """Lattices of more than 128 z-planes run the adjoint as launches over
    chunks of planes: bitwise the same lambda and gradient as one launch
    (tuning bit 7), and the chunked step passes the dot-product test against
    central differences of the forward step (FP64)."""
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    nx, ny, nz = 8, 4, 300   # chunks of 128, 128 and 44 planes
    rng = np.random.default_rng(23)
    F = 1e-3 * rng.standard_normal((3, nz, ny, nx))
    rho, u = synth.taylor_green_3d((nz, ny, nx), u0=0.05)
    relax = RELAX_LES if les else RELAX
    res = []
    for tuning in (0, 128):
        lat = Lattice((nx, ny, nz), storage=storage, walls=walls, tuning=tuning,
                      wall_u_hi=(0.02, 0.0, 0.0) if walls else (0.0, 0.0, 0.0))
        lat.set_relaxation(relax.omega_shear, relax.omega_bulk, relax.omega3, cs_smag=relax.cs_smag)
        dt = lat.dtype
        lat.set_force((0, 0, 0), torch.tensor(F, device="cuda", dtype=dt))
        lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
        f = lat.populations()
        f = f * (1 + 0.05 * torch.tensor(rng.standard_normal(f.shape), device="cuda", dtype=dt)) if not res else f_pert
        f_pert = f
        lat.set_populations(f)
        w = torch.tensor(np.random.default_rng(29).standard_normal(f.shape), device="cuda", dtype=dt)
        lam = lat.lam_buffer()
        gF = torch.zeros((3, nz, ny, nx), dtype=dt, device="cuda")
        lat.adjoint_step(lat.state_buffer(), lat.lam_from_planes(w), lam, gF)
        torch.cuda.synchronize()
        res.append((lat.lam_to_planes(lam).cpu(), gF.cpu()))
        if storage == "f64" and tuning == 0:
            v = torch.tensor(np.random.default_rng(31).standard_normal(f.shape), device="cuda")
            eps = 1e-7
            outs = []
            for sgn in (1, -1):
                lat.set_populations(f + sgn * eps * v)
                lat.step(1)
                outs.append(lat.populations())
            lhs = float(((outs[0] - outs[1]) / (2 * eps) * w).sum())
            rhs = float((v * res[-1][0].to("cuda")).sum())
            assert abs(lhs - rhs) < 1e-7 * abs(rhs)
        lat.close()
    assert torch.equal(res[0][0], res[1][0])
    assert torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("storage,tol", [("f32s", 1e-5), ("f16s", 2e-3)])   # measured 4e-7, 2e-4
def test_adjoint_with_shifted_storage_matches_fp64_reference(storage, tol):
    """Shifted FP32 and FP16 storage: the forward steps store rounded
    populations and the adjoint linearises the collision at the stored values
    (the rounding itself is not differentiated); the gradient against the
    FP64 autograd reference, to the storage's accuracy (8^3, 20 steps, K = 6)."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (8, 8, 8)
    F = synth.smooth_random_force((8, 8, 8), sigma=2.0, frms=1e-4)
    lat, f0_state, f0 = _setup(shape, storage, F)
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda", dtype=torch.float32), f0_state, 20, 6)
    E_ref, g_ref = energy_gradient(LAT, RELAX, f0, F.reshape(3, -1), 20, (8, 8, 8))
    g = g.cpu().numpy().reshape(3, -1).astype(np.float64)
    gerr = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"\n{storage}: E rel err {abs(E - E_ref) / abs(E_ref):.2e}, gradient max rel err {gerr:.2e}")
    assert abs(E - E_ref) < tol * abs(E_ref)
    assert gerr < tol


@pytest.mark.parametrize("fact,rc,cs,walls", [(True, False, 0.0, False), (False, True, 0.0, False),
                                              (True, True, 0.3, False), (True, True, 0.3, True)])
def test_gradient_with_sec12_13_operators_fp64_matches_autograd(fact, rc, cs, walls):
    """Factorized attractors (Sec. 13) and reduced compressibility (Sec. 12),
    with and without the eddy rate and walls: the GPU FP64 checkpointed adjoint
    against autograd through the reference step with the same operators (E with
    the velocity of the operator, rho0 u = sum fbar e + F/2 under Sec. 12)."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    shape = (6, 5, 4)
    nx, ny, nz = shape
    relax = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), omega4=(1.3, 0.8), cs_smag=cs,
                  factorized=fact, reduced_compressibility=rc)
    F = synth.smooth_random_force((nz, ny, nx), sigma=1.0, frms=1e-3)
    lat, f0_state, f0 = _setup(shape, "f64", F, u0=0.05, walls=walls, relax=relax)
    nsteps = 13
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, nsteps, 5)
    wk = dict(walls=True, u_hi=(0.02, 0.0, 0.0)) if walls else {}
    E_ref, g_ref = energy_gradient(LAT, relax, f0, F.reshape(3, -1), nsteps, (nz, ny, nx), **wk)
    plain = Relax(omega_shear=1.6, omega_bulk=1.1, omega3=(1.2, 0.9, 1.3), omega4=(1.3, 0.8), cs_smag=cs)
    g_plain = energy_gradient(LAT, plain, f0, F.reshape(3, -1), nsteps, (nz, ny, nx), **wk)[1]
    assert np.abs(g_ref - g_plain).max() > 1e-4 * np.abs(g_ref).max()   # the operators change the gradient
    assert abs(E - E_ref) < 1e-13 * abs(E_ref)
    g = g.cpu().numpy().reshape(3, -1)
    assert np.abs(g - g_ref).max() < 1e-10 * np.abs(g_ref).max()
