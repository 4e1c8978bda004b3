"""GPU parity of the Sec. 14 coupling: sub-grid stresses as a force.

The kernel reads the stress of the previous step, forms a' = -div R by
central differences, collides with F + rho a' and writes this step's stress;
the oracle (``oracle.sgs`` inside ``OracleSim``) does the same on whole
fields with np.roll. Populations, the stress field and the moments are
compared after several steps, per storage mode, with the same tolerances as
the plain step (the stress itself is compared relative to its size).
"""
import numpy as np
import pytest

import synth
from oracle import collide as C
from oracle import sgs as SG
from oracle.lattice import Relax, d3q27
from oracle.sim import OracleSim

pytestmark = pytest.mark.gpu
LAT = d3q27()
TOL = {"f64": 1e-14, "f32": 1.5e-7, "f32s": 5e-8, "f16s": 1e-4}
STRESS_TOL = {"f64": 1e-11, "f32": 2e-4, "f32s": 5e-5, "f16s": 3e-2}   # relative to max |R|
RATES = dict(omega_shear=1.55, omega_bulk=1.2, omega3=(1.1, 0.95, 1.3), omega4=(1.05, 0.9), omega5=1.2,
             omega6=1.4)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_np(t):
    return t.detach().to("cpu").numpy()


def stress_planes(R):
    """(3, 3, ...) oracle stress -> the library's plane order xx, yy, zz, xy, xz, yz."""
    return np.stack([R[0, 0], R[1, 1], R[2, 2], R[0, 1], R[0, 2], R[1, 2]])


def make(shape, storage, relax: Relax, force):
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice(shape, storage=storage)
    lat.set_relaxation(relax.omega_shear, relax.omega_bulk, relax.omega3, relax.omega4, relax.omega5, relax.omega6,
                       relax.cs_smag, relax.factorized, relax.reduced_compressibility, sgs_force=relax.sgs_force)
    if np.ndim(force) > 1:
        lat.set_force((0, 0, 0), torch.tensor(np.asarray(force), device="cuda"))
    else:
        lat.set_force(tuple(force))
    return lat


CASES = [
    # shape (nx, ny, nz), storage, force field, factorized, reduced compressibility
    ((37, 11, 5), "f64", True, False, False),
    ((37, 11, 5), "f64", False, True, True),
    ((37, 11, 5), "f32", True, False, False),
    ((37, 11, 5), "f32s", True, True, True),
    ((64, 4, 4), "f16s", True, True, True),
    ((300, 3, 2), "f32", True, True, False),
    ((1, 1, 1), "f64", False, False, False),
    ((2, 3, 1), "f64", True, False, True),
]


@pytest.mark.parametrize("shape,storage,ffield,fact,rc", CASES)
def test_sgs_step_matches_oracle(shape, storage, ffield, fact, rc):
    torch = _torch()
    nx, ny, nz = shape
    rng = np.random.default_rng(sum(shape) + 5)
    s = (nz, ny, nx)
    rho = 1 + 0.02 * rng.standard_normal(s)
    u = 0.05 * rng.standard_normal((3,) + s)
    F = 1e-3 * rng.standard_normal((3,) + s)
    relax = Relax(cs_smag=0.4, sgs_force=True, factorized=fact, reduced_compressibility=rc, **RATES)
    force = F if ffield else (2e-4, -1e-4, 5e-5)
    lat = make(shape, storage, relax, force)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    sim = OracleSim(s, relax, force=np.asarray(force).reshape(3, -1) if ffield else force)
    sim.set_populations(to_np(lat.populations()).reshape(27, -1))
    assert np.abs(to_np(lat.sgs_stress())).max() == 0.0
    for k in range(8):
        lat.step(1)
        sim.step(1)
    err = np.abs(to_np(lat.populations()).reshape(27, -1) - sim.f).max()
    Rg = to_np(lat.sgs_stress()).reshape(6, -1)
    Ro = stress_planes(sim.R_prev)
    scale = np.abs(Ro).max()
    errR = np.abs(Rg - Ro).max() / scale
    print(f"sgs {shape} {storage} ffield={ffield} fact={fact} rc={rc}: max |df| = {err:.3e}, "
          f"stress rel err {errR:.3e} (|R| max {scale:.2e})")
    assert err < TOL[storage]
    if shape != (1, 1, 1):   # one cell has no gradient: zero stress
        assert scale > 1e-7
        assert errR < STRESS_TOL[storage]
    rg, ug = lat.moments()
    ro, uo = sim.moments()
    assert np.abs(to_np(ug).reshape(3, -1) - uo.reshape(3, -1)).max() < 40 * TOL[storage]
    red, ref = lat.reduce(), sim.reduce()
    assert abs(red["ke"] - ref["ke"]) < 1e-6 * ref["ke"] + 40 * TOL[storage]
    assert np.abs(np.array(red["momentum"]) - ref["momentum"]).max() < 1e-6 * ref["mass"] * 1e-3 + 40 * TOL[storage]


def test_sgs_state_reset_and_errors():
    torch = _torch()
    from paper_1202_6074_amd import _lib
    shape = (16, 8, 4)
    rng = np.random.default_rng(2)
    u = 0.05 * rng.standard_normal((3, 4, 8, 16))
    relax = Relax(omega_shear=1.6, cs_smag=0.4, sgs_force=True)
    lat = make(shape, "f64", relax, (0.0, 0.0, 0.0))
    lat.init_equilibrium(torch.tensor(u, device="cuda"))
    lat.step(4)
    assert np.abs(to_np(lat.sgs_stress())).max() > 0
    f = lat.populations()
    lat.set_populations(f)   # a new state starts without sub-grid force
    assert np.abs(to_np(lat.stress[0])).max() == 0.0 and np.abs(to_np(lat.stress[1])).max() == 0.0
    sim = OracleSim((4, 8, 16), relax)
    sim.set_populations(to_np(f).reshape(27, -1))
    lat.step(3)
    sim.step(3)
    assert np.abs(to_np(lat.populations()).reshape(27, -1) - sim.f).max() < 1e-14
    # step_from cannot carry the stress
    with pytest.raises(_lib.CmlbmError) as e:
        lat.step_from(lat.buf[0], lat.buf[1])
    assert e.value.status == _lib.EINVAL
    # walls are rejected, and the flag without buffers leaves the handle unusable for steps
    from paper_1202_6074_amd.lattice import Lattice
    lw = Lattice(shape, storage="f32", walls=True)
    with pytest.raises(_lib.CmlbmError) as e:
        lw.set_relaxation(1.6, cs_smag=0.2, sgs_force=True)
    assert e.value.status == _lib.EINVAL
    lb = Lattice(shape, storage="f32")
    r = _lib.Relax()
    r.omega_shear = r.omega_bulk = r.omega5 = r.omega6 = 1.0
    r.omega3[:] = [1.0, 1.0, 1.0]
    r.omega4[:] = [1.0, 1.0]
    r.cs_smag = 0.2
    r.flags = _lib.SGS_FORCE
    _lib.cmlbm_set_relaxation(lb.h, r)
    lb.init_equilibrium(torch.zeros((3, 4, 8, 16), device="cuda"))
    with pytest.raises(_lib.CmlbmError) as e:
        lb.step(1)
    assert e.value.status == _lib.ESTATE
    with pytest.raises(_lib.CmlbmError) as e:
        lb.reduce()
    assert e.value.status == _lib.ESTATE


def test_sgs_full_size_sampled_step():
    """The benchmarked Sec. 14 configuration (256^3 FP32, factorized attractors,
    reduced compressibility, stress as a force with C_s = 0.12, band forcing,
    turbulence initial field): one step after 3 warm-up steps, 1500 sampled
    cells recomputed by the oracle from the GPU state fbar(n) and stress R(n-1)
    (collide the upstream cells with F + rho a', stream), and the stress R(n)
    at the sampled cells."""
    torch = _torch()
    n = 256
    shape = (n, n, n)
    u = synth.turbulence_velocity(shape, k0=4.0, urms=0.03)
    F = synth.band_forcing(shape, frms=1e-4)
    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice(shape, storage="f32")
    lat.set_relaxation(1.95, cs_smag=0.12, factorized=True, reduced_compressibility=True, sgs_force=True)
    Fd = torch.tensor(F, device="cuda", dtype=torch.float32)
    lat.set_force((0, 0, 0), Fd)
    lat.init_equilibrium(torch.tensor(u, device="cuda", dtype=torch.float32))
    del u
    relax = Relax(omega_shear=1.95, cs_smag=0.12, factorized=True, reduced_compressibility=True, sgs_force=True)
    lat.step(3)
    f_n = lat.populations(torch.float64).reshape(27, -1)
    R_prev = lat.sgs_stress().double().reshape(6, -1)
    rng = np.random.default_rng(256)
    pts = np.concatenate([np.stack([rng.integers(0, n, 1500) for _ in range(3)], 1),
                          np.array([[0, 0, 0], [n - 1, n - 1, n - 1], [0, n - 1, 0],
                                    [5, 7, n // 2 - 1], [9, 200, n // 2]])])   # the planes where the launches meet
    src = np.array([[(x - LAT.e[i, 0]) % n, (y - LAT.e[i, 1]) % n, (z - LAT.e[i, 2]) % n]
                    for (x, y, z) in pts for i in range(27)])
    uniq, inv = np.unique(src, axis=0, return_inverse=True)
    # a' at the upstream cells from the stress at their six neighbours
    acc = np.zeros((3, len(uniq)))
    plane = {(0, 0): 0, (1, 1): 1, (2, 2): 2, (0, 1): 3, (1, 0): 3, (0, 2): 4, (2, 0): 4, (1, 2): 5, (2, 1): 5}
    for a in range(3):
        for b in range(3):
            off = np.zeros(3, int)
            off[b] = 1
            cp = (uniq + off) % n
            cm = (uniq - off) % n
            ip = torch.tensor(cp[:, 0] + n * (cp[:, 1] + n * cp[:, 2]), device="cuda")
            im = torch.tensor(cm[:, 0] + n * (cm[:, 1] + n * cm[:, 2]), device="cuda")
            k = plane[(a, b)]
            acc[a] -= 0.5 * (R_prev[k, ip] - R_prev[k, im]).cpu().numpy()
    it = torch.tensor(uniq[:, 0] + n * (uniq[:, 1] + n * uniq[:, 2]), device="cuda")
    fu = f_n[:, it].cpu().numpy()
    Fu = Fd.reshape(3, -1)[:, it].double().cpu().numpy() + fu.sum(axis=0) * acc
    post, parts = C.collide(fu, Fu, LAT, relax, return_parts=True, rho0=1.0)
    inv = inv.reshape(len(pts), 27)
    want = np.array([[post[i, inv[k, i]] for i in range(27)] for k in range(len(pts))])
    # stress of this step at the sampled cells themselves (upstream index of the rest population)
    Rs = SG.sgs_stress(parts["kbar"], np.ones(len(uniq)), LAT, 1.95, 0.12)
    want_R = stress_planes(Rs)[:, inv[:, 13]]
    del f_n, R_prev
    lat.step(1)
    idx = torch.tensor(pts[:, 0] + n * (pts[:, 1] + n * pts[:, 2]), device="cuda")
    got = lat.populations(torch.float64).reshape(27, -1)[:, idx].T.cpu().numpy()
    got_R = lat.sgs_stress().double().reshape(6, -1)[:, idx].cpu().numpy()
    err = np.abs(got - want).max()
    errR = np.abs(got_R - want_R).max() / np.abs(want_R).max()
    print(f"sgs 256^3 sampled: max |df| = {err:.3e}, stress rel err {errR:.3e}, |R| max {np.abs(want_R).max():.2e}")
    assert err < 2e-7
    assert errR < 1e-3


def test_sgs_results_identical_across_tuning_hints():
    """Row-loop, workgroup-order, per-lane-gather and one-launch hints change
    which lane loads a value, which workgroup computes a row and how the planes
    are split between launches, never the arithmetic (also with the stress
    stencil): bitwise identical populations and stress."""
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    # per-lane gather; LDS exchange unless bit 5; 300 planes: launches over
    # chunks of 128, 128 and 44 planes unless bit 7
    for shape in ((300, 6, 5), (37, 11, 5), (16, 4, 300)):
        nx, ny, nz = shape
        rng = np.random.default_rng(9)
        u = 0.05 * rng.standard_normal((3, nz, ny, nx))
        F = 1e-3 * rng.standard_normal((3, nz, ny, nx))
        outs = []
        for tuning in (0, 4, 8, 16, 32, 4 | 8, 4 | 16, 32 | 16, 128, 128 | 24):
            lat = Lattice(shape, storage="f32", tuning=tuning)
            lat.set_relaxation(1.7, cs_smag=0.3, factorized=True, sgs_force=True)
            lat.set_force((0, 0, 0), torch.tensor(F, device="cuda"))
            lat.init_equilibrium(torch.tensor(u, device="cuda"))
            lat.step(5)
            outs.append((to_np(lat.populations()), to_np(lat.sgs_stress())))
        for f, R in outs[1:]:
            assert np.array_equal(f, outs[0][0]) and np.array_equal(R, outs[0][1]), shape
