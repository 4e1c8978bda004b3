"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Every test runs the library's kernels on cuda:0 and compares element by
element with the oracle on the same seeded inputs. Tolerances per storage
mode (absolute, on populations of order w_i ~ 0.3):
  f64: 1e-14 after a few steps (rounding order only; no FMA in the oracle)
  f32: 1.5e-7; f32 shifted: 5e-8; f16 shifted: 1e-4 (8 steps)
derived from half a unit in the last place of what is stored per step
(f ~ 0.3 for plain storage: 1.5e-8 in FP32; f - w ~ 0.05 for shifted
storage: 1.9e-9 in FP32, 1.5e-5 in FP16), plus FP32 arithmetic on O(1)
intermediates (the rest mass of a line, rho) of a few 1e-9 per step,
accumulated linearly over the 8 steps. Measured on MI355X: 4e-16, 2.4e-8,
6e-9 and 5.5e-6 respectively.
"""
import os

import numpy as np
import pytest

import synth
from oracle import collide as C
from oracle.lattice import Relax, d3q27
from oracle.sim import OracleSim

pytestmark = pytest.mark.gpu
LAT = d3q27()
TOL = {"f64": 1e-14, "f32": 1.5e-7, "f32s": 5e-8, "f16s": 1e-4}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make(shape, storage, relax: Relax, walls=False, u_lo=(0, 0, 0), u_hi=(0, 0, 0), force=None):
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice(shape, storage=storage, walls=walls, wall_u_lo=u_lo, wall_u_hi=u_hi)
    lat.set_relaxation(relax.omega_shear, relax.omega_bulk, relax.omega3, relax.omega4, relax.omega5,
                       relax.omega6, relax.cs_smag, relax.factorized, relax.reduced_compressibility)
    if force is not None and np.ndim(force) > 1:
        lat.set_force((0, 0, 0), torch.tensor(np.asarray(force), device="cuda"))
    elif force is not None:
        lat.set_force(tuple(force))
    return lat


def to_np(t):
    return t.detach().to("cpu").numpy()


def grid_fields(shape_xyz, seed=3, uamp=0.05, famp=1e-3):
    nx, ny, nz = shape_xyz
    rng = np.random.default_rng(seed)
    s = (nz, ny, nx)
    rho = 1 + 0.02 * rng.standard_normal(s)
    u = uamp * rng.standard_normal((3,) + s)
    F = famp * rng.standard_normal((3,) + s)
    return rho, u, F


RATES = Relax(omega_shear=1.55, omega_bulk=1.2, omega3=(1.1, 0.95, 1.3), omega4=(1.05, 0.9), omega5=1.2,
              omega6=1.4)


def test_library_is_the_in_tree_native_build():
    _torch()
    from paper_1202_6074_amd import _lib
    lib = _lib.load()
    assert os.path.abspath(lib._name) == os.path.abspath(_lib.LIB_PATH)
    with open("/proc/self/maps") as fh:
        maps = fh.read()
    assert "libcmlbm.so" in maps


@pytest.mark.parametrize("storage", ["f64", "f32", "f32s", "f16s"])
def test_init_equilibrium_matches_oracle(storage):
    torch = _torch()
    shape = (37, 11, 5)
    rho, u, F = grid_fields(shape)
    lat = make(shape, storage, RATES, force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    got = to_np(lat.populations()).reshape(27, -1)
    want = C.equilibrium_state(rho.reshape(-1), u.reshape(3, -1), F.reshape(3, -1), LAT)
    # FP32 modes receive rho and u rounded to FP32: error ~ 6e-8 * rho * w_i
    tol = {"f64": 1e-15, "f32": 6e-8, "f32s": 6e-8, "f16s": 3e-5}[storage]
    err = np.abs(got - want).max()
    print(f"init {storage}: max |df| = {err:.3e}")
    assert err < tol
    r2, u2 = lat.moments()
    assert np.abs(to_np(r2) - rho).max() < max(tol * 27, 1e-14)
    assert np.abs(to_np(u2) - u).max() < max(tol * 60, 1e-14)


CASES = [
    # shape (nx, ny, nz), storage, walls, les, force field
    ((37, 11, 5), "f64", False, False, True),
    ((37, 11, 5), "f64", True, True, True),
    ((37, 11, 5), "f32", False, True, True),
    ((37, 11, 5), "f32s", True, False, False),
    ((37, 11, 5), "f32s", False, True, True),
    ((37, 11, 5), "f16s", False, True, True),
    ((130, 3, 2), "f32", True, True, True),
    ((1, 1, 1), "f64", False, False, False),
    ((1, 5, 1), "f64", True, True, False),
    ((3, 2, 1), "f32s", False, True, True),
    ((64, 4, 4), "f16s", True, True, False),
    ((256, 3, 2), "f32", False, True, True),     # one full workgroup per row
    ((255, 4, 3), "f16s", True, True, True),     # one idle lane, walls
    ((300, 4, 3), "f16s", False, True, True),    # FP16 rows of 258-512 cells: two cells per lane
    ((512, 2, 2), "f16s", False, False, False),  # two cells per lane, every lane busy, uniform force
    ((258, 3, 2), "f16s", False, True, True),    # two cells per lane, 127 idle lanes
    ((300, 5, 3), "f16s", True, True, True),     # walls: interior rows two cells per lane
]


@pytest.mark.parametrize("shape,storage,walls,les,ffield", CASES)
def test_step_matches_oracle(shape, storage, walls, les, ffield):
    torch = _torch()
    nsteps = 8
    rho, u, F = grid_fields(shape, seed=sum(shape))
    relax = Relax(**{**RATES.__dict__, "cs_smag": 0.15 if les else 0.0})
    force = F if ffield else (2e-4, -1e-4, 5e-5)
    u_lo, u_hi = (0.01, 0.0, -0.02), (0.03, 0.0, 0.01)
    lat = make(shape, storage, relax, walls=walls, u_lo=u_lo, u_hi=u_hi, force=force)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    f0 = to_np(lat.populations())
    nx, ny, nz = shape
    sim = OracleSim((nz, ny, nx), relax, force=np.asarray(force).reshape(3, -1) if ffield else force,
                    walls=walls, u_lo=u_lo, u_hi=u_hi)
    sim.set_populations(f0.reshape(27, -1))
    lat.step(nsteps)
    sim.step(nsteps)
    got = to_np(lat.populations()).reshape(27, -1)
    err = np.abs(got - sim.f).max()
    print(f"step {shape} {storage} walls={walls} les={les} ffield={ffield}: max |df| = {err:.3e}")
    assert err < TOL[storage], f"max |df| = {err:.3e}"
    rg, ug = lat.moments()
    ro, uo = sim.moments()
    assert np.abs(to_np(ug) - uo).max() < 40 * TOL[storage]


VARIANT_CASES = [
    ((37, 11, 5), "f64", False, True, True, True, False),
    ((37, 11, 5), "f64", True, True, True, False, True),
    ((37, 11, 5), "f64", False, False, True, True, True),
    ((37, 11, 5), "f32s", False, True, True, True, True),
    ((64, 4, 4), "f16s", True, True, False, True, True),
    ((300, 4, 3), "f16s", False, True, True, True, True),   # two cells per lane
]


@pytest.mark.parametrize("shape,storage,walls,les,ffield,fact,rc", VARIANT_CASES)
def test_variant_step_matches_oracle(shape, storage, walls, les, ffield, fact, rc):
    """Factorized attractors (Sec. 13) and reduced compressibility (Sec. 12):
    init, 8 steps and moments against the oracle."""
    torch = _torch()
    nsteps = 8
    rho, u, F = grid_fields(shape, seed=7 + sum(shape))
    relax = Relax(**{**RATES.__dict__, "cs_smag": 0.15 if les else 0.0, "factorized": fact,
                     "reduced_compressibility": rc})
    force = F if ffield else (2e-4, -1e-4, 5e-5)
    lat = make(shape, storage, relax, walls=walls, u_lo=(0.01, 0, 0), u_hi=(0, 0, 0.02), force=force)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    nx, ny, nz = shape
    sim = OracleSim((nz, ny, nx), relax, force=np.asarray(force).reshape(3, -1) if ffield else force,
                    walls=walls, u_lo=(0.01, 0, 0), u_hi=(0, 0, 0.02))
    if storage == "f64":
        sim.init_equilibrium(rho, u)
        assert np.abs(to_np(lat.populations()).reshape(27, -1) - sim.f).max() < 1e-15
        r0, u0 = lat.moments()
        assert np.abs(to_np(u0) - u).max() < 1e-15
    else:
        sim.set_populations(to_np(lat.populations()).reshape(27, -1))
    lat.step(nsteps)
    sim.step(nsteps)
    err = np.abs(to_np(lat.populations()).reshape(27, -1) - sim.f).max()
    print(f"variant {shape} {storage} fact={fact} rc={rc} les={les}: max |df| = {err:.3e}")
    assert err < TOL[storage]
    rg, ug = lat.moments()
    ro, uo = sim.moments()
    assert np.abs(to_np(ug) - uo).max() < 40 * TOL[storage]
    red, ref = lat.reduce(), sim.reduce()
    assert abs(red["ke"] - ref["ke"]) < 1e-6 * ref["ke"] + 40 * TOL[storage]


@pytest.mark.parametrize("storage,walls", [("f64", False), ("f32", True), ("f16s", False)])
def test_row_mapping_hints_give_identical_results(storage, walls):
    """The tuning hints (row loop, workgroup order, per-lane gather instead of
    the LDS exchange) change only which lane loads a value and which block
    computes a cell, never the arithmetic: results are bitwise identical.
    (300, 6, 5): two blocks of 256 per row, ragged tail (per-lane gather);
    (37, 11, 5), (200, 5, 4): one block per row (LDS exchange unless bit 5
    is set), with idle lanes. For FP16 storage the row loop (bit 2) also
    switches the step kernel from scalar-base to vector addressing, and on
    (300, 6, 5) the default is the two-cells-per-lane kernel, which bits 2, 5
    and 6 turn off. The workgroup orders need block counts divisible by 8
    (XCD-aware) or by 256 (runs of 32 rows), else they fall back to the plain
    order: (40, 16, 16), (40, 18, 16) (256 interior rows between walls),
    (300, 8, 32) (256 pair rows, 512 per-lane blocks), (130, 16, 16)
    (runs of 32 by default for FP32) and (300, 64, 32) (runs of 256 pair rows
    by default for FP16) take them; (40, 4, 260) runs its FP32 steps as
    launches over chunks of 128 z-planes, which bit 7 turns off."""
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    for shape in ((300, 6, 5), (37, 11, 5), (200, 5, 4), (40, 16, 16), (40, 18, 16), (300, 8, 32), (130, 16, 16),
                  (300, 64, 32), (40, 4, 260)):
        rho, u, F = grid_fields(shape, seed=4)
        outs = []
        for tuning in (0, 4, 8, 16, 24, 32, 4 | 8, 4 | 16, 32 | 16, 32 | 4, 64, 64 | 16, 64 | 24, 128):
            lat = Lattice(shape, storage=storage, walls=walls, wall_u_lo=(0.01, 0, 0), tuning=tuning)
            lat.set_relaxation(1.7, cs_smag=0.12)
            lat.set_force((0, 0, 0), torch.tensor(F, device="cuda"))
            lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
            lat.step(5)
            outs.append(to_np(lat.populations()))
            r_, u_ = lat.moments()
            outs.append(to_np(u_))
        for k in range(2, len(outs), 2):
            assert np.array_equal(outs[k], outs[0]) and np.array_equal(outs[k + 1], outs[1]), (shape, k)


def test_cfg1_taylor_green_fp64_200_steps():
    """32^3 periodic FP64 Taylor-Green vortex, u0 = 0.02, omega = 1.6, F = (1e-5, 0, 0), 200 steps."""
    torch = _torch()
    shape = (32, 32, 32)
    relax = Relax(omega_shear=1.6)
    F = (1e-5, 0.0, 0.0)
    rho, u = synth.taylor_green_3d((32, 32, 32), u0=0.02)
    lat = make(shape, "f64", relax, force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    sim = OracleSim((32, 32, 32), relax, force=F)
    sim.init_equilibrium(rho, u)
    assert np.abs(to_np(lat.populations()).reshape(27, -1) - sim.f).max() < 1e-15
    lat.step(200)
    sim.step(200)
    got = to_np(lat.populations()).reshape(27, -1)
    assert np.abs(got - sim.f).max() / np.abs(sim.f).max() < 1e-11
    rg, ug = lat.moments()
    ro, uo = sim.moments()
    assert np.abs(to_np(rg) - ro).max() < 1e-12
    assert np.abs(to_np(ug) - uo).max() < 1e-12
    red = lat.reduce()
    ref = sim.reduce()
    assert abs(red["mass"] - ref["mass"]) < 1e-12 * ref["mass"]
    assert np.abs(np.array(red["momentum"]) - ref["momentum"]).max() < 1e-12 * 32 ** 3
    assert abs(red["ke"] - ref["ke"]) < 1e-11 * ref["ke"]
    # exact global invariants of the step (Sec. 9): mass constant, momentum + N F per step
    assert abs(red["mass"] - 32 ** 3 * float(rho.mean())) < 1e-9
    assert abs(red["momentum"][0] - (32 ** 3 * (rho * u[0]).mean() + 200 * 32 ** 3 * F[0])) < 1e-9


@pytest.mark.parametrize("storage", ["f64", "f32", "f32s", "f16s"])
def test_populations_roundtrip(storage):
    torch = _torch()
    for walls in (False, True):
        shape = (19, 6, 3)
        lat = make(shape, storage, RATES, walls=walls, u_lo=(0.02, 0, 0), u_hi=(0, 0, 0.01))
        rng = np.random.default_rng(4)
        f = LAT.w[:, None, None, None] * (1 + 0.1 * rng.standard_normal((27, 3, 6, 19)))
        lat.set_populations(torch.tensor(f, device="cuda"))
        back = to_np(lat.populations())
        # set converts f to the stored form (f - w rho0 for the compute, rounded to
        # the storage type), get converts back: half an ulp of the stored magnitude
        # plus one FP64 rounding of f ~ 0.3. For FP16 |f - w| <= 0.095 here, below
        # 0.125, where the binary16 ulp is 2^-14: half an ulp is 3.05e-5 (the FP32
        # rounding before it adds at most 4e-9)
        tol = {"f64": 1e-16, "f32": 6e-8, "f32s": 4e-9, "f16s": 3.06e-5}[storage]
        assert np.abs(back - f).max() <= tol


def test_reduce_matches_oracle_and_flags_nonfinite():
    torch = _torch()
    from paper_1202_6074_amd import _lib
    shape = (24, 10, 6)
    rho, u, F = grid_fields(shape)
    lat = make(shape, "f64", RATES, force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    lat.step(3)
    sim = OracleSim((6, 10, 24), RATES, force=F.reshape(3, -1))
    sim.set_populations(to_np(lat.populations()).reshape(27, -1))
    red, ref = lat.reduce(), sim.reduce()
    assert abs(red["mass"] - ref["mass"]) < 1e-12 * ref["mass"]
    assert np.abs(np.array(red["momentum"]) - ref["momentum"]).max() < 1e-13 * ref["mass"]
    assert abs(red["ke"] - ref["ke"]) < 1e-12 * ref["ke"]
    assert abs(red["rho_min"] - ref["rho_min"]) < 1e-14 and abs(red["umax"] - ref["umax"]) < 1e-14
    assert red["nonfinite"] == 0
    f = lat.populations()
    f[5, 2, 3, 4] = float("nan")
    f[0, 1, 1, 1] = float("inf")
    lat.set_populations(f)
    with pytest.raises(_lib.CmlbmError) as e:
        lat.reduce()
    assert e.value.status == _lib.ENONFINITE
    red = lat.reduce(raise_nonfinite=False)
    assert red["nonfinite"] == 2 and red["status"] == _lib.ENONFINITE


def test_deterministic_replay_and_resume():
    torch = _torch()
    shape = (48, 12, 8)
    rho, u, F = grid_fields(shape, uamp=0.05)
    relax = Relax(omega_shear=1.9, cs_smag=0.12)
    outs = []
    for _ in range(2):
        lat = make(shape, "f32", relax, force=F)
        lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
        lat.step(20)
        outs.append(to_np(lat.state_buffer()).copy())
        lat.close()
    assert np.array_equal(outs[0], outs[1])
    # resume from a device copy of the internal state after 10 steps
    lat = make(shape, "f32", relax, force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    lat.step(10)
    ck = lat.state_buffer().clone()
    lat2 = make(shape, "f32", relax, force=F)
    lat2.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    lat2.state_buffer().copy_(ck)
    lat2.step(10)
    assert np.array_equal(to_np(lat2.state_buffer()), outs[0])


def test_invalid_relaxation_on_device_handle():
    _torch()
    from paper_1202_6074_amd import _lib
    lat = make((8, 8, 8), "f32", RATES)
    with pytest.raises(_lib.CmlbmError) as e:
        lat.set_relaxation(2.5)
    assert e.value.status == _lib.EINVAL
    lat_w = make((8, 8, 8), "f32s", RATES, walls=True)
    import torch
    z = torch.zeros((27, 8, 8, 8), device="cuda")
    with pytest.raises(ValueError, match="lam_in"):   # lambda in the compute type (float32), not float64
        lat_w.adjoint_step(lat_w.state_buffer(), z.double(), z.clone(), torch.zeros((3, 8, 8, 8), device="cuda"))


@pytest.mark.parametrize("case,msg", [
    ("in_place", "two-buffer"), ("sgs_force", "sub-grid stress"), ("d2q9", "D3Q27")])
def test_adjoint_rejects_unsupported_configurations(case, msg):
    """The adjoint covers the D3Q27 collision (two buffers, every storage mode,
    with or without eddy viscosity and the Sec. 12-13 flags, not the sub-grid
    stress as a force); every other configuration is refused on the host before
    any launch."""
    torch = _torch()
    from paper_1202_6074_amd import _lib
    from paper_1202_6074_amd.lattice import Lattice
    shape = (8, 6, 4)
    lat = Lattice(shape if case != "d2q9" else (8, 6), storage="f32",
                  in_place=case == "in_place", lattice="d2q9" if case == "d2q9" else "d3q27")
    lat.set_relaxation(1.5, cs_smag=0.1 if case == "sgs_force" else 0.0, factorized=case == "factorized",
                       reduced_compressibility=case == "reduced_compressibility", sgs_force=case == "sgs_force")
    Q = lat.Q
    z = torch.zeros((Q,) + tuple(lat.buf[0].shape[1:]), device="cuda")
    g = torch.zeros((lat.D,) + tuple(lat.buf[0].shape[1:]), device="cuda")
    with pytest.raises(_lib.CmlbmError, match=msg):
        _lib.cmlbm_adjoint_step(lat.h, lat.buf[0].data_ptr(), z.data_ptr(), z.clone().data_ptr(), g.data_ptr())
    with pytest.raises(_lib.CmlbmError, match=msg):
        _lib.cmlbm_energy_seed(lat.h, lat.buf[0].data_ptr(), z.data_ptr(), g.data_ptr())
    lat.close()
