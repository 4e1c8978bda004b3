"""PyTorch-facing wrapper of the cmlbm C ABI.

PyTorch provides device memory and the HIP stream; every operation on the
lattice runs in the HIP kernels of ``libcmlbm.so``. Tensors follow the
library's structure-of-arrays layout: populations (Q, nz, ny, nx), vectors
(D, nz, ny, nx), scalars (nz, ny, nx), x fastest; Q, D = 27, 3 on D3Q27 and
9, 2 on D2Q9 (nz = 1, populations in the paper's velocity order).
"""
from __future__ import annotations

import torch

from . import _lib as L

COMPUTE_DTYPE = {L.F64: torch.float64, L.F32: torch.float32, L.F32_SHIFTED: torch.float32,
                 L.F16_SHIFTED: torch.float32}
STORAGE_DTYPE = {L.F64: torch.float64, L.F32: torch.float32, L.F32_SHIFTED: torch.float32,
                 L.F16_SHIFTED: torch.float16}
_DT = {torch.float64: L.DT_F64, torch.float32: L.DT_F32}


def _check_tensor(t: torch.Tensor, numel: int, dtype, device, name: str):
    """The kernels index these arrays by cell: shape, type and placement must match."""
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor on {device}")
    if t.numel() != numel:
        raise ValueError(f"{name}: expected {numel} elements, got {t.numel()}")


def _storage_id(storage) -> int:
    if isinstance(storage, str):
        return L.STORAGE_NAMES[storage]
    return int(storage)


class Lattice:
    """A cascaded central-moment lattice (D3Q27, or the paper's D2Q9) on one GPU.

    shape = (nx, ny, nz), or (nx, ny) for D2Q9; storage in {'f64', 'f32',
    'f32s', 'f16s'} (the last two store populations shifted by w_i rho0);
    walls=True puts halfway bounce-back planes at y = -1/2 and y = ny - 1/2;
    in_place=True streams in one buffer (AA pattern, D3Q27); tuning: the
    performance hints of cmlbm_desc.tuning (bit 2 row loop, bits 3-4 workgroup
    order, bit 5 per-lane gather, bit 6 no two-cell FP16 kernel, bit 7 one
    launch per step and adjoint step; results are identical). On D2Q9 the rates of
    set_relaxation map to the paper's as omega_bulk =
    omega_3, omega_shear = omega_4 = omega_5, omega3[0] = omega_6,
    omega3[1] = omega_7, omega4[0] = omega_8.
    """

    def __init__(self, shape, storage="f32", walls=False, wall_u_lo=(0.0, 0.0, 0.0), wall_u_hi=(0.0, 0.0, 0.0),
                 rho0=1.0, device="cuda", stream=None, tuning=0, lattice="d3q27", in_place=False):
        L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("cmlbm needs a HIP device (torch.cuda.is_available() is False)")
        self.lattice = L.LATTICE_NAMES[lattice] if isinstance(lattice, str) else int(lattice)
        self.Q, self.D = (9, 2) if self.lattice == L.D2Q9 else (27, 3)
        shape = tuple(int(s) for s in shape)
        if len(shape) == 2:
            shape = shape + (1,)
        self.nx, self.ny, self.nz = shape
        self.N = self.nx * self.ny * self.nz
        self.storage = _storage_id(storage)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dtype = COMPUTE_DTYPE[self.storage]
        self.sdtype = STORAGE_DTYPE[self.storage]
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.in_place = bool(in_place)
        self.buf = [torch.empty((self.Q, self.nz, self.ny, self.nx), dtype=self.sdtype, device=self.device)
                    for _ in range(1 if self.in_place else 2)]
        desc = L.Desc()
        desc.nx, desc.ny, desc.nz = self.nx, self.ny, self.nz
        desc.storage = self.storage
        desc.walls = 1 if walls else 0
        desc.tuning = int(tuning)
        desc.wall_u_lo[:] = [float(v) for v in wall_u_lo]
        desc.wall_u_hi[:] = [float(v) for v in wall_u_hi]
        desc.rho0 = float(rho0)
        desc.lattice = self.lattice
        desc.streaming = L.STREAM_IN_PLACE if self.in_place else L.STREAM_TWO_BUFFERS
        self.rho0 = float(rho0)
        self.walls = bool(walls)
        nbytes = self.buf[0].numel() * self.buf[0].element_size()
        self.h = L.cmlbm_create(desc, self.buf[0].data_ptr(), None if self.in_place else self.buf[1].data_ptr(),
                                nbytes, self.stream.cuda_stream)
        self._force_field = None

    # -- configuration ---------------------------------------------------------
    def set_relaxation(self, omega_shear, omega_bulk=1.0, omega3=(1.0, 1.0, 1.0), omega4=(1.0, 1.0), omega5=1.0,
                       omega6=1.0, cs_smag=0.0, factorized=False, reduced_compressibility=False, sgs_force=False):
        """sgs_force=True: the sub-grid stress (Smagorinsky, C_s = cs_smag) acts
        as a force (Sec. 14) instead of an eddy viscosity in the collision; the
        two stress buffers are allocated here on first use."""
        r = L.Relax()
        r.omega_shear, r.omega_bulk = float(omega_shear), float(omega_bulk)
        r.omega3[:] = [float(v) for v in omega3]
        r.omega4[:] = [float(v) for v in omega4]
        r.omega5, r.omega6, r.cs_smag = float(omega5), float(omega6), float(cs_smag)
        r.flags = ((L.FACTORIZED if factorized else 0) | (L.REDUCED_COMPRESSIBILITY if reduced_compressibility else 0)
                   | (L.SGS_FORCE if sgs_force else 0))
        r.reserved = 0
        L.cmlbm_set_relaxation(self.h, r)
        if sgs_force and getattr(self, "stress", None) is None:
            planes = 3 if self.lattice == L.D2Q9 else 6
            self.stress = [torch.zeros((planes, self.nz, self.ny, self.nx), dtype=self.dtype, device=self.device)
                           for _ in range(2)]
            nbytes = self.stress[0].numel() * self.stress[0].element_size()
            L.cmlbm_set_sgs_buffers(self.h, self.stress[0].data_ptr(), self.stress[1].data_ptr(), nbytes)

    def sgs_stress(self) -> torch.Tensor:
        """The sub-grid stress of the previous step: (6, nz, ny, nx) planes xx, yy, zz,
        xy, xz, yz on D3Q27; (3, 1, ny, nx) planes xx, yy, xy on D2Q9."""
        state = self.state_buffer()
        k = 0 if state.data_ptr() == self.buf[0].data_ptr() else 1
        return self.stress[k]

    def _after_use(self, *tensors):
        """The kernels run asynchronously on self.stream: tell torch's allocator that
        these inputs are in use there, so that their memory is not handed out again
        before the work that reads them has run."""
        for t in tensors:
            if t is not None:
                t.record_stream(self.stream)

    def set_force(self, uniform=(0.0, 0.0, 0.0), field: torch.Tensor | None = None):
        if field is not None:
            field = field.to(device=self.device, dtype=self.dtype).contiguous()
            _check_tensor(field, self.D * self.N, self.dtype, self.device, "force field")
            self._after_use(field)
        self._force_field = field   # borrowed by the library until replaced
        L.cmlbm_set_force(self.h, uniform, field.data_ptr() if field is not None else None)

    # -- state -----------------------------------------------------------------
    def init_equilibrium(self, u: torch.Tensor, rho: torch.Tensor | None = None):
        dt = torch.float64 if self.dtype == torch.float64 else torch.float32
        u = u.to(device=self.device, dtype=dt).contiguous()
        rho = rho.to(device=self.device, dtype=dt).contiguous() if rho is not None else None
        _check_tensor(u, self.D * self.N, dt, self.device, "u")
        if rho is not None:
            _check_tensor(rho, self.N, dt, self.device, "rho")
        L.cmlbm_init_equilibrium(self.h, rho.data_ptr() if rho is not None else None, u.data_ptr(), _DT[dt])
        self._after_use(u, rho)
        return self

    def step(self, nsteps=1):
        L.cmlbm_step(self.h, nsteps)

    def capture_steps(self, nsteps: int) -> "StepGraph":
        """Record nsteps time steps (cmlbm_step) in a HIP graph and return a
        StepGraph whose replay() enqueues them on self.stream again, without
        the host-side cost of each launch (which dominates small lattices).

        nsteps must be even and positive: the buffers then alternate back to
        where they started (the two-buffer state, the in-place parity, the
        sub-grid stress buffers), so the handle's host state is the same after
        every replay and eager calls may follow. The graph keeps the buffers,
        force field, rates and flags of the moment of capture: capture again
        after changing any of them. Call it after the lattice has been set up
        (init_equilibrium or set_populations), so that the library's kernels
        are loaded before the capture starts. If the capture fails, the
        handle's record of which buffer holds the state may have moved: set
        the state again before further steps."""
        nsteps = int(nsteps)
        if nsteps <= 0 or nsteps % 2:
            raise ValueError("capture an even, positive number of steps: a replay must end in the buffer "
                             "it started from")
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream(device=self.device)
        cap.wait_stream(self.stream)
        L.cmlbm_set_stream(self.h, cap.cuda_stream)
        try:
            with torch.cuda.graph(graph, stream=cap):
                L.cmlbm_step(self.h, nsteps)
        finally:
            L.cmlbm_set_stream(self.h, self.stream.cuda_stream)
        self.stream.wait_stream(cap)
        keep = list(self.buf) + list(getattr(self, "stress", None) or [])
        if self._force_field is not None:
            keep.append(self._force_field)
        return StepGraph(graph, self.stream, nsteps, keep)

    def step_from(self, src: torch.Tensor, dst: torch.Tensor):
        for t, nm in ((src, "src"), (dst, "dst")):
            _check_tensor(t, self.Q * self.N, self.sdtype, self.device, nm)
        L.cmlbm_step_from(self.h, src.data_ptr(), dst.data_ptr())
        self._after_use(src, dst)

    def state_buffer(self) -> torch.Tensor:
        ptr, _ = L.cmlbm_state_buffer(self.h)
        for b in self.buf:
            if b.data_ptr() == ptr:
                return b
        raise RuntimeError("state buffer is not one of this lattice's buffers")

    def moments(self, dtype=torch.float64):
        rho = torch.empty((self.nz, self.ny, self.nx), dtype=dtype, device=self.device)
        u = torch.empty((self.D, self.nz, self.ny, self.nx), dtype=dtype, device=self.device)
        L.cmlbm_read_moments(self.h, rho.data_ptr(), u.data_ptr(), _DT[dtype])
        return rho, u

    def populations(self, dtype=torch.float64):
        f = torch.empty((self.Q, self.nz, self.ny, self.nx), dtype=dtype, device=self.device)
        L.cmlbm_get_populations(self.h, f.data_ptr(), _DT[dtype])
        return f

    def set_populations(self, f: torch.Tensor):
        dt = torch.float64 if f.dtype == torch.float64 else torch.float32
        f = f.to(device=self.device, dtype=dt).contiguous()
        _check_tensor(f, self.Q * self.N, dt, self.device, "f")
        L.cmlbm_set_populations(self.h, f.data_ptr(), _DT[dt])
        self._after_use(f)

    def reduce(self, raise_nonfinite=True):
        out, status = L.cmlbm_reduce(self.h, raise_nonfinite)
        return dict(mass=out[0], momentum=tuple(out[1:4]), ke=out[4], nonfinite=int(out[5]), rho_min=out[6],
                    umax=out[7], status=status)

    # -- adjoint ---------------------------------------------------------------
    # The adjoint arrays lambda (27*N) use the row layout of the population
    # buffers: element (i, x, y, z) at ((z*ny + y)*27 + i)*nx + x, i.e. a
    # (nz, ny, 27, nx) array. The two helpers below convert to and from
    # (27, nz, ny, nx) planes (index copies, for callers that inspect lambda).
    def lam_buffer(self) -> torch.Tensor:
        """An uninitialised lambda array, shaped (nz, ny, 27, nx)."""
        return torch.empty((self.nz, self.ny, self.Q, self.nx), dtype=self.dtype, device=self.device)

    def lam_to_planes(self, lam: torch.Tensor) -> torch.Tensor:
        return lam.reshape(self.nz, self.ny, self.Q, self.nx).permute(2, 0, 1, 3).contiguous()

    def lam_from_planes(self, planes: torch.Tensor) -> torch.Tensor:
        return planes.reshape(self.Q, self.nz, self.ny, self.nx).permute(1, 2, 0, 3).contiguous()

    def adjoint_step(self, state: torch.Tensor, lam_in: torch.Tensor, lam_out: torch.Tensor,
                     grad_F: torch.Tensor):
        self._check_adjoint_args(state, lam_in, lam_out, grad_F)
        L.cmlbm_adjoint_step(self.h, state.data_ptr(), lam_in.data_ptr(), lam_out.data_ptr(), grad_F.data_ptr())
        self._after_use(state, lam_in, lam_out, grad_F)

    def _check_adjoint_args(self, state, lam_in, lam_out, grad_F):
        _check_tensor(state, 27 * self.N, self.sdtype, self.device, "state")
        for t, nm in ((lam_in, "lam_in"), (lam_out, "lam_out")):
            if t is not None:
                _check_tensor(t, 27 * self.N, self.dtype, self.device, nm)
        _check_tensor(grad_F, 3 * self.N, self.dtype, self.device, "grad_F")

    def energy_seed(self, state: torch.Tensor, lam_out: torch.Tensor, grad_F: torch.Tensor):
        self._check_adjoint_args(state, None, lam_out, grad_F)
        L.cmlbm_energy_seed(self.h, state.data_ptr(), lam_out.data_ptr(), grad_F.data_ptr())
        self._after_use(state, lam_out, grad_F)

    # -- teardown --------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            L.cmlbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class StepGraph:
    """nsteps captured time steps of one Lattice (Lattice.capture_steps).
    replay() enqueues them on the lattice's stream; the tensors the graph reads
    and writes are held here, so that they stay allocated while it exists.
    Keep it until its replays have run (a synchronisation of the stream)."""

    def __init__(self, graph, stream, nsteps, tensors):
        self.graph, self.stream, self.nsteps = graph, stream, nsteps
        self._keep = tensors

    def replay(self, times: int = 1):
        with torch.cuda.stream(self.stream):
            for _ in range(int(times)):
                self.graph.replay()
