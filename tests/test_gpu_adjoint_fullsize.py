"""The checkpointed gradient at the adjoint workload's full size, and its
independence from what happens to the lattice between the two passes.

Workload: 128^3 periodic, rest initial state, omega = 1.6, force parameter =
white noise filtered by a Gaussian of 4 cells, per-component rms 1e-5 (seed
42); E = sum rho |u|^2 / 2 after 500 steps (Eq. velocitycalculation for u),
checkpoints every 50 steps. The discrete adjoint is the transpose of the
linearised step of Sec. 6 (Eqs. cascadedcollision1, cascadedstreaming1).
"""
import numpy as np
import pytest

import synth
from oracle.grad import energy_gradient
from oracle.lattice import Relax, d3q27

pytestmark = pytest.mark.gpu
LAT = d3q27()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rest_lattice(shape_xyz, storage, omega=1.6):
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    nx, ny, nz = shape_xyz
    lat = Lattice(shape_xyz, storage=storage)
    lat.set_relaxation(omega)
    lat.set_force((0, 0, 0), torch.zeros((3, nz, ny, nx), device="cuda", dtype=lat.dtype))
    lat.init_equilibrium(torch.zeros((3, nz, ny, nx), device="cuda", dtype=torch.float32))
    return lat, lat.state_buffer().clone()


def _energy(lat, f0_state, F, nsteps):
    """E after nsteps from f0_state with force field F (forward only)."""
    lat.set_force((0, 0, 0), F)
    lat.state_buffer().copy_(f0_state)
    lat.step(nsteps)
    return lat.reduce()["ke"]


def test_adjoint_workload_gradient_against_central_differences_and_fp64():
    """128^3, 500 steps, K = 50: <dE/dF, v> of the FP32 checkpointed adjoint and of
    the FP64 one against central differences of E in FP64 storage along four
    seeded smooth random directions v. The differences are Richardson-extrapolated
    from steps h and 2h (E is nearly quadratic in F: starting at rest, u grows
    linearly with F up to the weak advection), which removes their h^2 error."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    n, nsteps, K = 128, 500, 50
    shape = (n, n, n)
    Fnp = synth.smooth_random_force(shape, sigma=4.0, frms=1e-5)
    dirs = [synth.smooth_random_force(shape, sigma=4.0, frms=1e-5, seed=1000 + k) for k in range(4)]
    lat32, f0_32 = _rest_lattice(shape, "f32")
    E32, g32 = energy_and_grad(lat32, torch.tensor(Fnp, device="cuda", dtype=torch.float32), f0_32, nsteps, K)
    g32 = g32.double()
    lat32.close()
    del lat32, f0_32
    torch.cuda.empty_cache()
    lat64, f0_64 = _rest_lattice(shape, "f64")
    F64 = torch.tensor(Fnp, device="cuda", dtype=torch.float64)
    E64, g64 = energy_and_grad(lat64, F64, f0_64, nsteps, K)
    print(f"\nE: FP32 {E32:.10e}, FP64 {E64:.10e} (rel {abs(E32 - E64) / E64:.2e})")
    gerr = float((g32 - g64).norm() / g64.norm())
    print(f"|g32 - g64| / |g64| = {gerr:.3e}")
    h = 1e-2
    for k, vnp in enumerate(dirs):
        v = torch.tensor(vnp, device="cuda", dtype=torch.float64)
        e = {s: _energy(lat64, f0_64, F64 + s * h * v, nsteps) for s in (-2, -1, 1, 2)}
        d1 = (e[1] - e[-1]) / (2 * h)
        d2 = (e[2] - e[-2]) / (4 * h)
        fd = (4 * d1 - d2) / 3
        a64 = float((g64 * v).sum())
        a32 = float((g32 * v).sum())
        r64, r32 = abs(a64 - fd) / abs(fd), abs(a32 - fd) / abs(fd)
        print(f"direction {k}: FD {fd:.10e} (h: {d1:.10e}, 2h: {d2:.10e}); "
              f"FP64 adjoint rel {r64:.2e}; FP32 adjoint rel {r32:.2e}")
        assert r64 < 1e-6
        assert r32 < 1e-3
    assert abs(E32 - E64) < 1e-3 * E64
    assert gerr < 1e-3
    lat64.close()


def test_fp64_gradient_16_cubed_100_steps_matches_autograd():
    """FP64 checkpointed adjoint (K = 10) against the FP64 CPU autograd reference
    over 100 steps on a 16^3 box (Taylor-Green start, smooth random force):
    the largest case the reference runs in seconds."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import energy_and_grad
    from paper_1202_6074_amd.lattice import Lattice
    n, nsteps, K = 16, 100, 10
    shape = (n, n, n)
    relax = Relax(omega_shear=1.6)
    F = synth.smooth_random_force(shape, sigma=2.0, frms=1e-4)
    rho, u = synth.taylor_green_3d(shape, u0=0.03)
    lat = Lattice(shape, storage="f64")
    lat.set_relaxation(1.6)
    lat.set_force((0, 0, 0), torch.zeros((3, n, n, n), dtype=torch.float64, device="cuda"))
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    f0_state = lat.state_buffer().clone()
    f0 = lat.populations().cpu().numpy().reshape(27, -1)
    E, g = energy_and_grad(lat, torch.tensor(F, device="cuda"), f0_state, nsteps, K)
    E_ref, g_ref = energy_gradient(LAT, relax, f0, F.reshape(3, -1), nsteps, shape)
    g = g.cpu().numpy().reshape(3, -1)
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"\n16^3 x 100 steps: dE {abs(E - E_ref) / abs(E_ref):.2e}, gradient rel err {err:.2e}")
    assert abs(E - E_ref) < 1e-12 * abs(E_ref)
    assert err < 1e-10


@pytest.mark.parametrize("K", [5, 100])   # checkpointed, and every state kept
def test_interleaved_passes_give_each_forward_its_own_gradient(K):
    """Two forward passes with different force fields on one lattice, a step and
    another force bound in between, then the two backward passes in reverse
    order: each gradient is bitwise the one of a clean run with its own F."""
    torch = _torch()
    from paper_1202_6074_amd.adjoint import EnergyAdjoint, energy_and_grad
    shape = (10, 8, 6)
    nx, ny, nz = shape
    nsteps = 12
    Fa = torch.tensor(synth.smooth_random_force((nz, ny, nx), sigma=1.5, frms=1e-3, seed=5), device="cuda",
                      dtype=torch.float32)
    Fb = torch.tensor(synth.smooth_random_force((nz, ny, nx), sigma=1.5, frms=1e-3, seed=6), device="cuda",
                      dtype=torch.float32)
    lat, f0 = _rest_lattice(shape, "f32")
    ref = {}
    for name, F in (("a", Fa), ("b", Fb)):
        ref[name] = energy_and_grad(lat, F, f0, nsteps, K)
    pa = Fa.clone().requires_grad_(True)
    pb = Fb.clone().requires_grad_(True)
    Ea = EnergyAdjoint.apply(pa, lat, f0, nsteps, K)
    Eb = EnergyAdjoint.apply(pb, lat, f0, nsteps, K)
    with torch.no_grad():
        pa.mul_(3.0)   # the caller changes its tensor; the forward pass kept a copy
    lat.set_force((0, 0, 0), torch.zeros_like(Fa))
    lat.step(3)
    Eb.backward()
    lat.step(2)
    Ea.backward()
    assert float(Ea.detach()) == ref["a"][0] and float(Eb.detach()) == ref["b"][0]
    assert torch.equal(pa.grad, ref["a"][1])
    assert torch.equal(pb.grad, ref["b"][1])
    assert not torch.equal(ref["a"][1], ref["b"][1])
