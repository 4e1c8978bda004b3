"""Time steps recorded in a HIP graph (Lattice.capture_steps) and replayed.

A replay launches the same kernels on the same buffers as the eager steps, so
after every replay the state is bitwise that of a lattice stepped eagerly the
same number of times; between replays the program does eager work of its own
(read-outs and synchronisation), and eager steps may follow the replays. One
case is also checked against the oracle. Cases: FP64 with the eddy viscosity,
FP32 over 300 planes (launches over chunks of planes), walls (interior and
wall-row launches), in-place streaming (even and odd kernels), the sub-grid
stress as a force (alternating stress buffers) and D2Q9.
"""
import numpy as np
import pytest

import synth
from oracle.lattice import Relax
from oracle.sim import OracleSim

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


CASES = {
    "f64_les": dict(shape=(20, 12, 10), storage="f64", relax=dict(omega_shear=1.7, cs_smag=0.2)),
    "f32_300_planes": dict(shape=(16, 6, 300), storage="f32", relax=dict(omega_shear=1.8, cs_smag=0.12)),
    "f32s_walls": dict(shape=(24, 10, 8), storage="f32s", walls=True, relax=dict(omega_shear=1.6)),
    "f32_in_place": dict(shape=(16, 12, 10), storage="f32", in_place=True, relax=dict(omega_shear=1.9, cs_smag=0.1)),
    "f32_sgs_force": dict(shape=(20, 12, 8), storage="f32",
                          relax=dict(omega_shear=1.7, cs_smag=0.3, factorized=True, sgs_force=True)),
    "f16s_d2q9": dict(shape=(64, 48), storage="f16s", lattice="d2q9", relax=dict(omega_shear=1.8, cs_smag=0.1)),
}


def _make(case):
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    c = CASES[case]
    lat = Lattice(c["shape"], storage=c["storage"], walls=c.get("walls", False), wall_u_hi=(0.02, 0.0, 0.0),
                  in_place=c.get("in_place", False), lattice=c.get("lattice", "d3q27"))
    lat.set_relaxation(**c["relax"])
    rng = np.random.default_rng(5)
    shp = (lat.D, lat.nz, lat.ny, lat.nx)
    lat.set_force((0, 0, 0), torch.tensor(1e-4 * rng.standard_normal(shp), device="cuda", dtype=lat.dtype))
    lat.init_equilibrium(torch.tensor(0.04 * rng.standard_normal(shp), device="cuda"))
    return lat


@pytest.mark.parametrize("case", list(CASES))
def test_replays_match_eager_steps_bitwise(case):
    torch = _torch()
    eager, graphed = _make(case), _make(case)
    g = graphed.capture_steps(4)
    for rep in range(3):
        eager.step(4)
        g.replay()
        graphed.moments()   # eager work of the program between replays
        torch.cuda.synchronize()
        assert torch.equal(eager.populations(), graphed.populations()), (case, rep)
        if CASES[case]["relax"].get("sgs_force"):
            assert torch.equal(eager.sgs_stress(), graphed.sgs_stress()), (case, rep)
    g.replay(2)
    eager.step(8)
    eager.step(3)    # eager steps after replays continue from the replayed state
    graphed.step(3)
    assert torch.equal(eager.populations(), graphed.populations()), case
    eager.close()
    graphed.close()


def test_replayed_steps_match_the_oracle():
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    shape = (12, 10, 8)
    nx, ny, nz = shape
    relax = Relax(omega_shear=1.7, cs_smag=0.2)
    rho, u = synth.taylor_green_3d((nz, ny, nx), u0=0.04)
    F = synth.smooth_random_force((nz, ny, nx), sigma=2.0, frms=1e-4)
    lat = Lattice(shape, storage="f64")
    lat.set_relaxation(relax.omega_shear, cs_smag=relax.cs_smag)
    lat.set_force((0, 0, 0), torch.tensor(F, device="cuda"))
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    f0 = lat.populations().cpu().numpy().reshape(27, -1)
    g = lat.capture_steps(6)
    g.replay()
    torch.cuda.synchronize()
    sim = OracleSim((nz, ny, nx), relax, force=F.reshape(3, -1))
    sim.set_populations(f0)
    sim.step(6)
    got = lat.populations().cpu().numpy().reshape(27, -1)
    assert np.abs(got - sim.f).max() < 1e-13


def test_odd_step_counts_are_refused():
    lat = _make("f64_les")
    for n in (0, 3, -2):
        with pytest.raises(ValueError):
            lat.capture_steps(n)
    lat.close()
