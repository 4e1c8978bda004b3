"""cmlbm_reduce_noalloc (the reductions for callers that cannot allocate device
memory) against cmlbm_reduce, through the C ABI: two calls in a row on one
device, the second on a smaller lattice, then a D2Q9 lattice with a
non-finite cell."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(lat):
    """(cmlbm_reduce's 8 values, cmlbm_reduce_noalloc's 8 values)."""
    torch = _torch()
    from paper_1202_6074_amd import _lib
    ref, _ = _lib.cmlbm_reduce(lat.h, raise_nonfinite=False)
    out = torch.full((8,), float("nan"), dtype=torch.float64, device=lat.device)
    _lib.cmlbm_reduce_noalloc(lat.h, out.data_ptr())
    lat.stream.synchronize()
    return np.array(ref), out.cpu().numpy()


def _check(ref, got):
    # sums (mass, momentum, kinetic energy): FP64 rounding of another summation order
    for k in (0, 1, 2, 3, 4):
        assert abs(got[k] - ref[k]) <= 1e-12 * max(abs(ref[0]), 1.0), (k, ref[k], got[k])
    # count, min and max do not depend on the order
    assert got[5] == ref[5] and got[6] == ref[6] and got[7] == ref[7]


def test_noalloc_reduce_matches_reduce_on_two_calls_the_second_smaller():
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    # 1: 256^3 LES state after a few steps (65,536 row chunks: the static
    #    partials are combined over many chunks per workgroup)
    n = 256
    print(f"\nnoalloc reduce: {n}^3 f32", flush=True)
    lat = Lattice((n, n, n), storage="f32")
    lat.set_relaxation(1.95, cs_smag=0.12)
    lat.set_force((0, 0, 0), torch.tensor(synth.band_forcing((n, n, n), frms=1e-4), device="cuda"))
    lat.init_equilibrium(torch.tensor(synth.turbulence_velocity((n, n, n), k0=4.0, urms=0.03), device="cuda"))
    lat.step(3)
    ref, got = _both(lat)
    _check(ref, got)
    assert got[5] == 0
    lat.close()
    del lat
    # 2: a smaller, ragged walled lattice in FP64 (fewer chunks than workgroups)
    print("noalloc reduce: 37x11x6 f64 walls", flush=True)
    shape = (37, 11, 6)
    lat = Lattice(shape, storage="f64", walls=True, wall_u_hi=(0.02, 0.0, 0.0))
    lat.set_relaxation(1.3)
    lat.set_force((1e-5, 0.0, 0.0))
    rho, u = synth.taylor_green_3d(shape[::-1], u0=0.04)
    lat.init_equilibrium(torch.tensor(u, device="cuda"), torch.tensor(rho, device="cuda"))
    lat.step(2)
    ref, got = _both(lat)
    _check(ref, got)
    # and with one non-finite cell
    f = lat.populations()
    f[:, 3, 5, 7] = float("nan")
    lat.set_populations(f)
    ref, got = _both(lat)
    assert ref[5] == 1
    _check(ref, got)
    lat.close()


def test_noalloc_reduce_d2q9_and_sgs_force():
    torch = _torch()
    from paper_1202_6074_amd.lattice import Lattice
    print("\nnoalloc reduce: D2Q9 300x40 f16s, sub-grid force", flush=True)
    nx, ny = 300, 40
    lat = Lattice((nx, ny), storage="f16s", lattice="d2q9")
    lat.set_relaxation(1.8, cs_smag=0.15, sgs_force=True)
    u = synth.turbulence_velocity_2d((ny, nx), k0=4.0, urms=0.05)
    lat.init_equilibrium(torch.tensor(u, device="cuda"))
    lat.step(4)
    ref, got = _both(lat)
    _check(ref, got)
    lat.close()
