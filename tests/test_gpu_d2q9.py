"""GPU parity of the D2Q9 path (the paper's own lattice) against the FP64 oracle.

The kernels run on cuda:0 through the C ABI (desc.lattice = D2Q9); the oracle
is the generic central-moment collision on the D2Q9 lattice in the paper's
velocity order, which the CPU tests pin to the paper's printed D2Q9 formulas.
Tolerances per storage mode follow the same derivation as for D3Q27 (half an
ulp of what is stored per step plus FP32 arithmetic on O(1) intermediates,
accumulated over the steps); the largest population is w_0 = 4/9 here.
"""
import numpy as np
import pytest

from oracle import collide as C
from oracle import d2q9_paper as PP
from oracle.lattice import Relax, d2q9
from oracle.sim import OracleSim
from oracle.stream import stream

pytestmark = pytest.mark.gpu
LAT = d2q9()
TOL = {"f64": 1e-14, "f32": 2e-7, "f32s": 5e-8, "f16s": 1e-4}
W = dict(w3=1.2, ws=1.55, w6=1.1, w7=0.95, w8=1.3)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def relax(cs=0.0, fact=False, rc=False, ws=None):
    return Relax(omega_shear=ws or W["ws"], omega_bulk=W["w3"], d2q9_omega678=(W["w6"], W["w7"], W["w8"]),
                 cs_smag=cs, factorized=fact, reduced_compressibility=rc)


def make(shape, storage, r: Relax, walls=False, u_lo=(0, 0, 0), u_hi=(0, 0, 0), force=None, tuning=0):
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice(shape, storage=storage, walls=walls, wall_u_lo=u_lo, wall_u_hi=u_hi, lattice="d2q9",
                  tuning=tuning)
    o6, o7, o8 = r.d2q9_omega678
    lat.set_relaxation(r.omega_shear, r.omega_bulk, omega3=(o6, o7, 1.0), omega4=(o8, 1.0), cs_smag=r.cs_smag,
                       factorized=r.factorized, reduced_compressibility=r.reduced_compressibility)
    if force is not None and np.ndim(force) > 1:
        lat.set_force((0, 0, 0), torch.tensor(np.asarray(force), device="cuda"))
    elif force is not None:
        lat.set_force(tuple(force) + (0.0,))
    return lat


def to_np(t):
    return t.detach().to("cpu").numpy()


def fields(shape_xy, seed=3, uamp=0.05, famp=1e-3):
    nx, ny = shape_xy
    rng = np.random.default_rng(seed)
    rho = 1 + 0.02 * rng.standard_normal((ny, nx))
    u = uamp * rng.standard_normal((2, ny, nx))
    F = famp * rng.standard_normal((2, ny, nx))
    return rho, u, F


@pytest.mark.parametrize("storage", ["f64", "f32", "f32s", "f16s"])
def test_init_equilibrium_matches_oracle(storage):
    torch = _torch()
    shape = (37, 11)
    rho, u, F = fields(shape)
    lat = make(shape, storage, relax(), force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    got = to_np(lat.populations()).reshape(9, -1)
    want = C.equilibrium_state(rho.reshape(-1), u.reshape(2, -1), F.reshape(2, -1), LAT)
    tol = {"f64": 1e-15, "f32": 6e-8, "f32s": 6e-8, "f16s": 3e-5}[storage]
    err = np.abs(got - want).max()
    print(f"d2q9 init {storage}: max |df| = {err:.3e}")
    assert err < tol
    r2, u2 = lat.moments()
    assert np.abs(to_np(r2)[0] - rho).max() < max(tol * 9, 1e-14)
    assert np.abs(to_np(u2)[:, 0] - u).max() < max(tol * 60, 1e-14)


CASES = [
    # shape (nx, ny), storage, walls, les, force field
    ((67, 13), "f64", False, False, False),
    ((67, 13), "f64", True, True, True),
    ((67, 13), "f32", False, True, True),
    ((67, 13), "f32s", True, False, False),
    ((67, 13), "f32s", False, True, True),
    ((67, 13), "f16s", False, True, True),
    ((300, 3), "f32", True, True, True),
    ((1, 1), "f64", False, False, False),
    ((1, 5), "f64", True, True, False),
    ((2, 2), "f32s", False, True, True),
]


@pytest.mark.parametrize("shape,storage,walls,les,ffield", CASES)
def test_step_matches_oracle(shape, storage, walls, les, ffield):
    torch = _torch()
    nsteps = 8
    rho, u, F = fields(shape, seed=sum(shape))
    r = relax(0.15 if les else 0.0)
    force = F if ffield else (2e-4, -1e-4)
    u_lo, u_hi = (0.01, 0.0, 0.0), (0.03, 0.0, 0.0)
    lat = make(shape, storage, r, walls=walls, u_lo=u_lo, u_hi=u_hi, force=force)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    nx, ny = shape
    sim = OracleSim((ny, nx), r, lat=LAT, force=np.asarray(force).reshape(2, -1) if ffield else force,
                    walls=walls, u_lo=u_lo, u_hi=u_hi)
    sim.set_populations(to_np(lat.populations()).reshape(9, -1))
    lat.step(nsteps)
    sim.step(nsteps)
    err = np.abs(to_np(lat.populations()).reshape(9, -1) - sim.f).max()
    print(f"d2q9 step {shape} {storage} walls={walls} les={les} ffield={ffield}: max |df| = {err:.3e}")
    assert err < TOL[storage], f"max |df| = {err:.3e}"
    rg, ug = lat.moments()
    ro, uo = sim.moments()
    assert np.abs(to_np(ug)[:, 0] - uo).max() < 40 * TOL[storage]


@pytest.mark.parametrize("storage,fact,rc,les", [("f64", True, False, True), ("f64", False, True, True),
                                                 ("f64", True, True, False), ("f32s", True, True, True)])
def test_variant_step_matches_oracle(storage, fact, rc, les):
    """Factorized attractor (Sec. 13) and reduced compressibility (Sec. 12) on D2Q9."""
    torch = _torch()
    shape = (45, 17)
    rho, u, F = fields(shape, seed=19)
    r = relax(0.15 if les else 0.0, fact, rc)
    lat = make(shape, storage, r, force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    sim = OracleSim((17, 45), r, lat=LAT, force=F.reshape(2, -1))
    if storage == "f64":
        sim.init_equilibrium(rho, u)
        assert np.abs(to_np(lat.populations()).reshape(9, -1) - sim.f).max() < 1e-15
    else:
        sim.set_populations(to_np(lat.populations()).reshape(9, -1))
    lat.step(8)
    sim.step(8)
    err = np.abs(to_np(lat.populations()).reshape(9, -1) - sim.f).max()
    print(f"d2q9 variant {storage} fact={fact} rc={rc} les={les}: max |df| = {err:.3e}")
    assert err < TOL[storage]
    red, ref = lat.reduce(), sim.reduce()
    assert abs(red["ke"] - ref["ke"]) < 1e-6 * ref["ke"] + 40 * TOL[storage]


def test_force_free_step_equals_paper_literal_formulas():
    """One FP64 step against the paper's printed D2Q9 collision (Secs. 9-11,
    force-free, where the printed brackets and the stated relaxation agree)
    followed by standard streaming (Eq. cascadedstreaming1)."""
    torch = _torch()
    shape = (29, 23)
    rng = np.random.default_rng(12)
    f0 = LAT.w[:, None, None] * (1 + 0.2 * rng.standard_normal((9, 23, 29)))
    lat = make(shape, "f64", relax(), force=(0.0, 0.0))
    lat.set_populations(torch.tensor(f0[:, None], device="cuda"))
    lat.step(1)
    post = PP.collide(f0.reshape(9, -1), np.zeros((2, f0[0].size)), (W["w3"], W["ws"], W["ws"], W["w6"], W["w7"],
                                                                       W["w8"]))
    want = stream(post.reshape(9, 23, 29), LAT)
    err = np.abs(to_np(lat.populations())[:, 0] - want).max()
    print(f"d2q9 literal paper step: max |df| = {err:.3e}")
    assert err < 1e-15


@pytest.mark.parametrize("storage", ["f64", "f32", "f32s", "f16s"])
def test_populations_roundtrip_paper_order(storage):
    torch = _torch()
    for walls in (False, True):
        lat = make((19, 6), storage, relax(), walls=walls, u_lo=(0.02, 0, 0), u_hi=(-0.01, 0, 0))
        rng = np.random.default_rng(4)
        f = LAT.w[:, None, None, None] * (1 + 0.1 * rng.standard_normal((9, 1, 6, 19)))
        lat.set_populations(torch.tensor(f, device="cuda"))
        back = to_np(lat.populations())
        tol = {"f64": 1e-16, "f32": 6e-8, "f32s": 4e-9, "f16s": 6.2e-5}[storage]
        assert np.abs(back - f).max() <= tol
    # the plane order is the paper's: a state with mass only in alpha = 1 (e = (1, 0))
    # streams one cell in +x
    f = np.zeros((9, 1, 6, 19))
    f[1, 0, 2, 5] = 1.0
    lat = make((19, 6), "f64", Relax(omega_shear=1.0, omega_bulk=1.0, d2q9_omega678=(1.0, 1.0, 1.0)))
    lat.set_populations(torch.tensor(f, device="cuda"))
    rho, u = lat.moments()
    assert abs(to_np(rho)[0, 2, 5] - 1.0) < 1e-15 and abs(to_np(u)[0, 0, 2, 5] - 1.0) < 1e-15
    assert abs(to_np(u)[1, 0, 2, 5]) < 1e-15


def test_reduce_matches_oracle_and_flags_nonfinite():
    torch = _torch()
    from paper_1202_6074_amd import _lib
    shape = (40, 14)
    rho, u, F = fields(shape)
    lat = make(shape, "f64", relax(), force=F)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    lat.step(3)
    sim = OracleSim((14, 40), relax(), lat=LAT, force=F.reshape(2, -1))
    sim.set_populations(to_np(lat.populations()).reshape(9, -1))
    red, ref = lat.reduce(), sim.reduce()
    assert abs(red["mass"] - ref["mass"]) < 1e-12 * ref["mass"]
    assert np.abs(np.array(red["momentum"][:2]) - ref["momentum"]).max() < 1e-13 * ref["mass"]
    assert red["momentum"][2] == 0.0
    assert abs(red["ke"] - ref["ke"]) < 1e-12 * ref["ke"]
    assert abs(red["rho_min"] - ref["rho_min"]) < 1e-14 and abs(red["umax"] - ref["umax"]) < 1e-14
    f = lat.populations()
    f[5, 0, 3, 4] = float("nan")
    lat.set_populations(f)
    red = lat.reduce(raise_nonfinite=False)
    assert red["nonfinite"] == 1 and red["status"] == _lib.ENONFINITE


@pytest.mark.parametrize("storage,walls", [("f64", True), ("f32", False), ("f16s", True)])
def test_layout_and_row_mapping_hints_give_identical_results(storage, walls):
    torch = _torch()
    shape = (300, 7)
    rho, u, F = fields(shape, seed=6)
    outs = []
    for tuning in (0, 4, 8, 16, 32, 4 | 8, 4 | 16):
        lat = make(shape, storage, relax(0.12), walls=walls, u_lo=(0.01, 0, 0), force=F, tuning=tuning)
        lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
        lat.step(5)
        outs.append(to_np(lat.populations()))
    for k in range(1, len(outs)):
        assert np.array_equal(outs[k], outs[0])


def test_poiseuille_20000_steps_f32s_against_oracle_and_closed_form():
    """Force-driven channel between resting walls (halfway bounce-back),
    H = 32, omega = 1.2, F = 1e-6, 20000 steps from rest (steady: the first
    start-up mode has decayed to 5e-10). The GPU profile agrees with the
    oracle's run to FP32 rounding, and both with the parabola
    u(y) = F (y + 1/2)(H - 1/2 - y) / (2 nu), nu = (1/omega - 1/2)/3, to the
    scheme's discretisation error (1.09e-4 of u_max in the oracle)."""
    torch = _torch()
    H, Fx, omega = 32, 1e-6, 1.2
    r = Relax(omega_shear=omega, omega_bulk=1.0, d2q9_omega678=(1.0, 1.0, 1.0))
    lat = make((1, H), "f32s", r, walls=True, force=(Fx, 0.0))
    lat.init_equilibrium(torch.zeros((2, 1, H, 1), device="cuda"))
    lat.step(20000)
    _, u = lat.moments()
    ux = to_np(u)[0, 0, :, 0]
    sim = OracleSim((H, 1), r, lat=LAT, force=(Fx, 0.0), walls=True)
    sim.init_equilibrium(1.0, np.zeros((2, H, 1)))
    sim.step(20000)
    uo = sim.moments()[1][0, :, 0]
    nu = (1.0 / omega - 0.5) / 3.0
    y = np.arange(H) + 0.5
    exact = Fx * y * (H - y) / (2 * nu)
    d_oracle = np.abs(ux - uo).max() / exact.max()
    d_exact = np.abs(ux - exact).max() / exact.max()
    print(f"d2q9 Poiseuille H={H}: |gpu - oracle| = {d_oracle:.3e}, |gpu - parabola| = {d_exact:.3e} (of u_max)")
    assert d_oracle < 3e-5
    assert d_exact < 1.5e-4
    assert float(u[1].abs().max()) < 1e-8


def test_adjoint_is_rejected_on_d2q9():
    torch = _torch()
    from paper_1202_6074_amd import _lib
    lat = make((8, 8), "f64", relax())
    z = torch.zeros((9, 1, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.CmlbmError) as e:
        _lib.cmlbm_adjoint_step(lat.h, lat.state_buffer().data_ptr(), z.data_ptr(), z.clone().data_ptr(),
                                torch.zeros((2, 1, 8, 8), dtype=torch.float64, device="cuda").data_ptr())
    assert e.value.status == _lib.EINVAL and "D3Q27" in str(e.value)


def test_full_size_8192_sampled_step_and_invariants():
    """The benchmarked D2Q9 configuration (8192^2 FP32 LES, Kolmogorov force
    field, 2D turbulence): one step after 3 warm-up steps, 2000 sampled cells
    recomputed one by one by the oracle (collide the upstream cells, stream),
    plus mass conservation and the momentum gain sum(F) per step on the whole
    field (FP64 reductions)."""
    torch = _torch()
    import synth
    n = 8192
    u = synth.turbulence_velocity_2d((n, n), k0=8.0, urms=0.03)
    F = synth.kolmogorov_force_2d((n, n), kf=4, amp=1e-5)
    r = Relax(omega_shear=1.95, omega_bulk=1.0, d2q9_omega678=(1.0, 1.0, 1.0), cs_smag=0.12)
    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice((n, n), storage="f32", lattice="d2q9")
    lat.set_relaxation(1.95, cs_smag=0.12)
    Fd = torch.tensor(F, device="cuda", dtype=torch.float32)
    lat.set_force((0, 0, 0), Fd)
    lat.init_equilibrium(torch.tensor(u, device="cuda", dtype=torch.float32))
    del u
    lat.step(3)
    r0 = lat.reduce()
    f_n = lat.populations(torch.float64).reshape(9, -1)
    rng = np.random.default_rng(8192)
    pts = np.concatenate([np.stack([rng.integers(0, n, 2000), rng.integers(0, n, 2000)], 1),
                          np.array([[0, 0], [n - 1, n - 1], [0, n - 1], [n - 1, 0]])])
    src = np.array([[(x - LAT.e[a, 0]) % n, (y - LAT.e[a, 1]) % n] for (x, y) in pts for a in range(9)])
    uniq, inv = np.unique(src, axis=0, return_inverse=True)
    it = torch.tensor(uniq[:, 0] + n * uniq[:, 1], device="cuda")
    fu = f_n[:, it].cpu().numpy()
    Fu = Fd.reshape(2, -1)[:, it].double().cpu().numpy()
    post = C.collide(fu, Fu, LAT, r)
    inv = inv.reshape(len(pts), 9)
    want = np.array([[post[a, inv[k, a]] for a in range(9)] for k in range(len(pts))])
    del f_n
    lat.step(1)
    idx = torch.tensor(pts[:, 0] + n * pts[:, 1], device="cuda")
    got = lat.populations(torch.float64).reshape(9, -1)[:, idx].T.cpu().numpy()
    err = np.abs(got - want).max()
    print(f"d2q9 8192^2 sampled max |df| = {err:.3e}")
    assert err < 2e-7
    r1 = lat.reduce()
    assert abs(r1["mass"] - r0["mass"]) < 1e-6 * n * n * 1e-3
    dp = r1["momentum"][0] - r0["momentum"][0]
    assert abs(dp - float(F[0].sum())) < 1e-3 * abs(float(np.abs(F[0]).sum())) + 1e-4


@pytest.mark.parametrize("storage,fact,rc", [("f64", False, False), ("f64", True, True), ("f32", True, False),
                                             ("f32s", True, True), ("f16s", False, True)])
def test_sgs_force_step_matches_oracle(storage, fact, rc):
    """Sec. 14 on the paper's own lattice: sub-grid stress as a force (a' = -div R
    of the previous step), 8 steps, populations, stress (xx, yy, xy) and moments."""
    torch = _torch()
    shape = (45, 17)
    rho, u, F = fields(shape, seed=23)
    r = Relax(omega_shear=W["ws"], omega_bulk=W["w3"], d2q9_omega678=(W["w6"], W["w7"], W["w8"]), cs_smag=0.4,
              sgs_force=True, factorized=fact, reduced_compressibility=rc)
    from paper_1202_6074_amd.lattice import Lattice
    lat = Lattice(shape, storage=storage, lattice="d2q9")
    lat.set_relaxation(r.omega_shear, r.omega_bulk, omega3=(W["w6"], W["w7"], 1.0), omega4=(W["w8"], 1.0),
                       cs_smag=0.4, factorized=fact, reduced_compressibility=rc, sgs_force=True)
    lat.set_force((0, 0, 0), torch.tensor(F, device="cuda"))
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    sim = OracleSim((17, 45), r, lat=LAT, force=F.reshape(2, -1))
    sim.set_populations(to_np(lat.populations()).reshape(9, -1))
    lat.step(8)
    sim.step(8)
    err = np.abs(to_np(lat.populations()).reshape(9, -1) - sim.f).max()
    Rg = to_np(lat.sgs_stress()).reshape(3, -1)
    Ro = np.stack([sim.R_prev[0, 0], sim.R_prev[1, 1], sim.R_prev[0, 1]])
    errR = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    print(f"d2q9 sgs {storage} fact={fact} rc={rc}: max |df| = {err:.3e}, stress rel err {errR:.3e}, "
          f"|R| max {np.abs(Ro).max():.2e}")
    assert err < TOL[storage]
    assert np.abs(Ro).max() > 1e-7
    assert errR < {"f64": 1e-11, "f32": 2e-4, "f32s": 5e-5, "f16s": 3e-2}[storage]
    rg, ug = lat.moments()
    ro, uo = sim.moments()
    assert np.abs(to_np(ug)[:, 0] - uo).max() < 40 * TOL[storage]
    red, ref = lat.reduce(), sim.reduce()
    assert abs(red["ke"] - ref["ke"]) < 1e-6 * ref["ke"] + 40 * TOL[storage]
