"""The C ABI library loads, exports every declared symbol and validates its
arguments on the host (CPU only: no call here reaches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cmlbm.h")


@pytest.fixture(scope="module")
def L():
    from paper_1202_6074_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcmlbm.so not built (run __graft_entry__.build())")
    _lib.load()
    return _lib


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:cmlbm_status|const char\*|int32_t)\s+(cmlbm_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("cmlbm_create", "cmlbm_destroy", "cmlbm_set_relaxation", "cmlbm_set_force",
                 "cmlbm_init_equilibrium", "cmlbm_step", "cmlbm_read_moments", "cmlbm_get_populations",
                 "cmlbm_set_populations", "cmlbm_reduce", "cmlbm_adjoint_step", "cmlbm_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, name


def test_struct_layouts_match_header(L):
    assert ctypes.sizeof(L.Desc) == 88
    assert L.Desc.lattice.offset == 80 and L.Desc.rho0.offset == 72
    assert ctypes.sizeof(L.Relax) == 88


def _desc(L, **kw):
    d = L.Desc()
    d.nx, d.ny, d.nz = kw.get("shape", (8, 8, 8))
    d.storage = kw.get("storage", L.F32)
    d.walls = kw.get("walls", 0)
    d.tuning = kw.get("tuning", 0)
    d.rho0 = kw.get("rho0", 1.0)
    d.lattice = kw.get("lattice", L.D3Q27)
    d.streaming = kw.get("streaming", 0)
    return d


@pytest.mark.parametrize("kw,msg", [
    (dict(shape=(0, 8, 8)), "must be >= 1"),
    (dict(shape=(2048, 2048, 1024)), "< 2^31"),
    (dict(storage=7), "storage"),
    (dict(walls=2), "walls"),
    (dict(tuning=256), "tuning"),
    (dict(tuning=1), "bits 2-7"),
    (dict(rho0=0.0), "rho0"),
    (dict(rho0=float("nan")), "rho0"),
    (dict(lattice=2), "unknown lattice"),
    (dict(lattice=1, shape=(8, 8, 2)), "nz == 1"),
    (dict(streaming=2), "streaming"),
    (dict(streaming=1, lattice=1, shape=(8, 8, 1)), "in-place"),
])
def test_create_rejects_invalid_descriptions(L, kw, msg):
    with pytest.raises(L.CmlbmError) as e:
        L.cmlbm_create(_desc(L, **kw), 0x1000, 0x2000, 1 << 40, 0)
    assert e.value.status == L.EINVAL and msg in str(e.value)


def test_create_rejects_small_or_aliased_buffers(L):
    with pytest.raises(L.CmlbmError, match="too small"):
        L.cmlbm_create(_desc(L), 0x1000, 0x2000, 27 * 512 * 4 - 1, 0)
    with pytest.raises(L.CmlbmError, match="distinct"):
        L.cmlbm_create(_desc(L), 0x1000, 0x1000, 1 << 30, 0)
    # D2Q9 needs 9 values per cell
    with pytest.raises(L.CmlbmError, match="too small"):
        L.cmlbm_create(_desc(L, lattice=L.D2Q9, shape=(16, 8, 1)), 0x1000, 0x2000, 9 * 128 * 4 - 1, 0)


@pytest.mark.parametrize("field,val", [("omega_shear", 2.0), ("omega_shear", 0.0), ("omega_bulk", -1.0),
                                       ("omega5", float("inf")), ("cs_smag", -0.1)])
def test_relaxation_rates_are_validated(L, field, val):
    r = L.Relax()
    for f in ("omega_shear", "omega_bulk", "omega5", "omega6"):
        setattr(r, f, 1.0)
    r.omega3[:] = [1.0, 1.0, 1.0]
    r.omega4[:] = [1.0, 1.0]
    setattr(r, field, val)
    with pytest.raises(L.CmlbmError) as e:
        L.cmlbm_set_relaxation(None, r)
    assert e.value.status == L.EINVAL and ("(0, 2)" in str(e.value) or "cs_smag" in str(e.value))


def test_null_handle_is_rejected(L):
    r = L.Relax()
    for f in ("omega_shear", "omega_bulk", "omega5", "omega6"):
        setattr(r, f, 1.0)
    r.omega3[:] = [1.0, 1.0, 1.0]
    r.omega4[:] = [1.0, 1.0]
    with pytest.raises(L.CmlbmError, match="null handle"):
        L.cmlbm_set_relaxation(None, r)
    with pytest.raises(L.CmlbmError, match="null handle"):
        L.cmlbm_step(None, 1)
    assert L.cmlbm_version() >= 10000


def test_relaxation_flags_and_sgs_buffers_are_validated(L):
    r = L.Relax()
    for f in ("omega_shear", "omega_bulk", "omega5", "omega6"):
        setattr(r, f, 1.0)
    r.omega3[:] = [1.0, 1.0, 1.0]
    r.omega4[:] = [1.0, 1.0]
    r.flags = 8
    with pytest.raises(L.CmlbmError, match="bits 0-2"):
        L.cmlbm_set_relaxation(None, r)
    r.flags = L.FACTORIZED | L.REDUCED_COMPRESSIBILITY | L.SGS_FORCE
    with pytest.raises(L.CmlbmError, match="null handle"):   # the flags themselves are valid
        L.cmlbm_set_relaxation(None, r)
    with pytest.raises(L.CmlbmError, match="null handle"):
        L.cmlbm_set_sgs_buffers(None, 0x1000, 0x2000, 1 << 20)


def test_in_place_streaming_takes_one_buffer(L):
    with pytest.raises(L.CmlbmError, match="one buffer"):
        L.cmlbm_create(_desc(L, streaming=1), 0x1000, 0x2000, 1 << 30, 0)
    with pytest.raises(L.CmlbmError, match="two distinct"):
        L.cmlbm_create(_desc(L, streaming=0), 0x1000, None, 1 << 30, 0)


# Longest rows the kernels can address with 32-bit per-lane byte offsets:
# 3 nx E and nx C below 2^32 (E storage, C compute element size).
ROW_LIMITS = {0: (2 ** 32 - 1) // 24, 1: (2 ** 32 - 1) // 12, 2: (2 ** 32 - 1) // 12, 3: (2 ** 32 - 1) // 6}


@pytest.mark.parametrize("storage", [0, 1, 2, 3])
def test_create_rejects_rows_beyond_32bit_lane_offsets(L, storage):
    nx = ROW_LIMITS[storage]
    assert nx < 2 ** 31
    with pytest.raises(L.CmlbmError) as e:
        L.cmlbm_create(_desc(L, shape=(nx + 1, 1, 1), storage=storage), 0x1000, 0x2000, 1 << 46, 0)
    assert e.value.status == L.EINVAL and "32-bit byte offsets" in str(e.value)
    # D2Q9 rows obey the same rule
    with pytest.raises(L.CmlbmError, match="32-bit byte offsets"):
        L.cmlbm_create(_desc(L, shape=(nx + 1, 1, 1), storage=storage, lattice=1), 0x1000, 0x2000, 1 << 46, 0)


@pytest.mark.parametrize("storage", [0, 1, 2, 3])
def test_create_accepts_the_longest_addressable_row(L, storage):
    """At the limit the description passes validation: without a device the call
    then fails only at the scratch allocation (CMLBM_EHIP)."""
    nx = ROW_LIMITS[storage]
    try:
        h = L.cmlbm_create(_desc(L, shape=(nx, 1, 1), storage=storage), 0x1000, 0x2000, 1 << 46, 0)
    except L.CmlbmError as e:
        assert e.status == L.EHIP, str(e)
    else:
        L.cmlbm_destroy(h)
