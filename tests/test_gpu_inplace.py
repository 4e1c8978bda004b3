"""In-place streaming (one buffer, alternating even and odd steps) on the GPU.

The in-place kernels run the same collision on the same values as the
two-buffer pull scheme and only address memory differently, so after any
number of steps the populations, moments and reductions are bitwise equal to
the two-buffer run's; one case is also checked against the oracle. Odd step
counts leave the buffer in the swapped arrangement, which every read-out must
undo.
"""
import numpy as np
import pytest

from oracle.lattice import Relax
from oracle.sim import OracleSim

pytestmark = pytest.mark.gpu
RATES = dict(omega_shear=1.55, omega_bulk=1.2, omega3=(1.1, 0.95, 1.3), omega4=(1.05, 0.9), omega5=1.2,
             omega6=1.4)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_np(t):
    return t.detach().to("cpu").numpy()


def pair(shape, storage, walls, les, ffield, fact=False, rc=False, seed=0):
    """The same initial state on a two-buffer and an in-place lattice."""
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    nx, ny, nz = shape
    rng = np.random.default_rng(seed + sum(shape))
    s = (nz, ny, nx)
    rho = torch.tensor(1 + 0.02 * rng.standard_normal(s), device="cuda")
    u = torch.tensor(0.05 * rng.standard_normal((3,) + s), device="cuda")
    F = torch.tensor(1e-3 * rng.standard_normal((3,) + s), device="cuda")
    out = []
    for in_place in (False, True):
        lat = Lattice(shape, storage=storage, walls=walls, wall_u_lo=(0.01, 0, -0.02), wall_u_hi=(0.03, 0, 0.01),
                      in_place=in_place)
        lat.set_relaxation(cs_smag=0.15 if les else 0.0, factorized=fact, reduced_compressibility=rc, **RATES)
        if ffield:
            lat.set_force((0, 0, 0), F)
        else:
            lat.set_force((2e-4, -1e-4, 5e-5))
        lat.init_equilibrium(u, rho)
        out.append(lat)
    return out


CASES = [
    # shape, storage, walls, les, force field
    ((37, 11, 5), "f64", True, True, True),
    ((37, 11, 5), "f32", False, True, True),
    ((37, 11, 5), "f32s", True, False, False),
    ((64, 4, 4), "f16s", True, True, True),
    ((300, 4, 3), "f16s", False, True, True),   # two-buffer step: two cells per lane
    ((300, 3, 2), "f32", True, True, True),
    ((256, 4, 3), "f32s", False, True, True),
    ((1, 1, 1), "f64", False, False, False),
    ((1, 5, 1), "f64", True, True, False),
    ((3, 2, 1), "f32", False, True, True),
    # 256 rows of 129-256 cells: the default order of periodic 4-byte storage
    # there (runs of 32 rows per XCD) applies
    ((130, 16, 16), "f32", False, True, True),
    ((136, 16, 16), "f32s", False, True, True),
]


@pytest.mark.parametrize("shape,storage,walls,les,ffield", CASES)
def test_in_place_bitwise_equal_to_two_buffers(shape, storage, walls, les, ffield):
    torch = _torch()
    a, b = pair(shape, storage, walls, les, ffield)
    assert np.array_equal(to_np(a.populations()), to_np(b.populations()))
    done = 0
    for n in (1, 1, 2, 3):   # parities odd, even, even, odd
        a.step(n)
        b.step(n)
        done += n
        fa, fb = to_np(a.populations()), to_np(b.populations())
        assert np.array_equal(fa, fb), f"after {done} steps"
        (ra, ua), (rb, ub) = a.moments(), b.moments()
        assert np.array_equal(to_np(ra), to_np(rb)) and np.array_equal(to_np(ua), to_np(ub))
        xa, xb = a.reduce(), b.reduce()
        assert xa["mass"] == xb["mass"] and xa["ke"] == xb["ke"] and xa["momentum"] == xb["momentum"]
    assert len(a.buf) == 2 and len(b.buf) == 1


@pytest.mark.parametrize("fact,rc", [(True, False), (False, True), (True, True)])
def test_in_place_variants_bitwise(fact, rc):
    a, b = pair((37, 11, 5), "f64", True, True, True, fact=fact, rc=rc, seed=3)
    a.step(5)
    b.step(5)
    assert np.array_equal(to_np(a.populations()), to_np(b.populations()))


def test_in_place_against_oracle_odd_parity():
    torch = _torch()
    shape = (23, 9, 6)
    relax = Relax(cs_smag=0.15, **RATES)
    _, b = pair(shape, "f64", True, True, False)
    sim = OracleSim((6, 9, 23), relax, force=(2e-4, -1e-4, 5e-5), walls=True, u_lo=(0.01, 0, -0.02),
                    u_hi=(0.03, 0, 0.01))
    sim.set_populations(to_np(b.populations()).reshape(27, -1))
    b.step(7)
    sim.step(7)
    assert np.abs(to_np(b.populations()).reshape(27, -1) - sim.f).max() < 1e-14


def test_set_populations_resets_parity_and_errors():
    torch = _torch()
    from paper_1202_6074_amd import _lib
    a, b = pair((16, 6, 4), "f32", True, False, True)
    a.step(3)
    b.step(3)
    f = b.populations(torch.float32)
    a.set_populations(f)
    b.set_populations(f)                 # odd parity -> natural arrangement again
    # the storage round trip rounds (see the populations round-trip tests); both
    # schemes round alike
    assert np.array_equal(to_np(a.populations(torch.float32)), to_np(b.populations(torch.float32)))
    assert np.abs(to_np(b.populations(torch.float32)) - to_np(f)).max() < 6e-8
    a.step(2)
    b.step(2)
    assert np.array_equal(to_np(a.populations()), to_np(b.populations()))
    with pytest.raises(_lib.CmlbmError) as e:
        b.step_from(b.buf[0], a.buf[1])
    assert e.value.status == _lib.EINVAL
    with pytest.raises(_lib.CmlbmError) as e:
        b.set_relaxation(1.5, cs_smag=0.2, sgs_force=True)
    assert e.value.status == _lib.EINVAL
    from paper_1202_6074_amd.lattice import Lattice
    c = Lattice((8, 8, 8), storage="f32", in_place=True)
    z = torch.zeros((27, 8, 8, 8), device="cuda")
    with pytest.raises(_lib.CmlbmError) as e:
        c.adjoint_step(c.state_buffer(), z, z.clone(), torch.zeros((3, 8, 8, 8), device="cuda"))
    assert e.value.status == _lib.EINVAL


def test_in_place_full_size_bitwise():
    """The headline configuration (256^3 FP32, LES, force field): 3 steps (odd
    parity) in place against the two-buffer kernel, bitwise, on the whole field."""
    torch = _torch()
    import synth
    from paper_1202_6074_amd.lattice import Lattice
    n = 256
    u = torch.tensor(synth.turbulence_velocity((n, n, n), k0=4.0, urms=0.03), device="cuda", dtype=torch.float32)
    F = torch.tensor(synth.band_forcing((n, n, n), frms=1e-4), device="cuda", dtype=torch.float32)
    outs = []
    for in_place in (False, True):
        lat = Lattice((n, n, n), storage="f32", in_place=in_place)
        lat.set_relaxation(1.95, cs_smag=0.12)
        lat.set_force((0, 0, 0), F)
        lat.init_equilibrium(u)
        lat.step(3)
        outs.append(lat.populations(torch.float32))
        lat.close()
        del lat
    assert torch.equal(outs[0], outs[1])
