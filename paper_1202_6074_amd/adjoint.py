"""Gradient of the flow's kinetic energy with respect to the body-force field.

Loss: E(F) = sum_x rho |u|^2 / 2 after ``nsteps`` steps from a fixed initial
state (the populations do not depend on F), with u from
Eq. velocitycalculation (so E depends on F also through the F/2 term).

Backward pass (discrete adjoint, project addition): the forward run keeps a
device copy of the state every K steps. For each segment, last to first, the
K-1 steps after its checkpoint are recomputed into a stash of K-1 buffers
(the checkpoint itself is the segment's first state), then K adjoint steps
run in reverse. With K >= nsteps the forward run writes every
state into a buffer of its own (nsteps population buffers, e.g. 113 GB for
500 steps at 128^3 in FP32) and the backward pass runs the adjoint steps only,
without recomputation; the gradient is bitwise the same. Every step's work is done by the library's
HIP kernels (``cmlbm_step_from``, ``cmlbm_adjoint_step``,
``cmlbm_energy_seed``, ``cmlbm_reduce``); torch provides buffers and copies.
"""
from __future__ import annotations

import torch

from .lattice import Lattice


def _keep_all(nsteps: int, K: int) -> bool:
    return nsteps >= 1 and K >= nsteps


def _forward(lat: Lattice, F: torch.Tensor, f0_state: torch.Tensor, nsteps: int, K: int):
    """Run the forward pass from f0_state with force field F. Returns E, the
    checkpoints and a buffer of its own holding the final state fbar(nsteps),
    so that the backward pass does not depend on what the lattice does in
    between."""
    if nsteps < 0 or K < 1:
        raise ValueError(f"nsteps must be >= 0 and K >= 1 (got nsteps={nsteps}, K={K})")
    lat.set_force((0.0, 0.0, 0.0), F)
    cur = lat.state_buffer()
    cur.copy_(f0_state)
    if _keep_all(nsteps, K):
        # every state kept, ckpts[n] = fbar(n) for n < nsteps, in one allocation
        # whose last entry receives the last step and then holds fbar(nsteps)
        states = torch.empty((nsteps + 1,) + tuple(cur.shape), dtype=cur.dtype, device=cur.device)
        ckpts = [states[n] for n in range(nsteps)]
        ckpts[0].copy_(cur)
        for n in range(nsteps - 1):
            lat.step_from(ckpts[n], ckpts[n + 1])
        final = states[nsteps]
        lat.step_from(ckpts[nsteps - 1], final)
        cur.copy_(final)   # the lattice's state is fbar(nsteps) afterwards, as with checkpoints
        E = lat.reduce()["ke"]
        return E, ckpts, final
    # the checkpoints in one allocation (one request to the allocator instead of
    # one per checkpoint)
    states = torch.empty(((nsteps + K - 1) // K,) + tuple(cur.shape), dtype=cur.dtype, device=cur.device)
    ckpts = []
    for n0 in range(0, nsteps, K):
        ckpts.append(states[n0 // K])
        ckpts[-1].copy_(lat.state_buffer())
        lat.step(min(K, nsteps - n0))
    E = lat.reduce()["ke"]
    return E, ckpts, lat.state_buffer().clone()


def _backward(lat: Lattice, F: torch.Tensor, ckpts, final: torch.Tensor, nsteps: int, K: int):
    """dE/dF for the forward pass that used force field F and left `final`.
    Binds F to the lattice again (the adjoint and the recomputed steps read
    it), so that other work on the lattice between the passes does not change
    the result; the lattice's state is not touched."""
    lat.set_force((0.0, 0.0, 0.0), F)
    lam = lat.lam_buffer()
    lam2 = torch.empty_like(lam)
    gF = torch.empty((3, lat.nz, lat.ny, lat.nx), dtype=lat.dtype, device=lat.device)
    lat.energy_seed(final, lam, gF)
    if nsteps == 0:   # E of the initial state: F enters only through u's F/2 term
        return gF
    if _keep_all(nsteps, K):
        for k in range(nsteps - 1, -1, -1):
            lat.adjoint_step(ckpts[k], lam, lam2, gF)
            lam, lam2 = lam2, lam
        return gF
    # stash[k] holds fbar(n0 + k) of the current segment; its first entry is the
    # checkpoint itself (only read), so no copy of it is made; the others share
    # one allocation (the first backward pass measured 1 % faster than with K - 1
    # separate ones at 128^3, K = 50)
    block = torch.empty((max(K - 1, 1),) + tuple(ckpts[0].shape), dtype=ckpts[0].dtype, device=ckpts[0].device)
    stash = [None] + [block[k] for k in range(K - 1)]
    nseg = len(ckpts)
    for s in range(nseg - 1, -1, -1):
        n0 = s * K
        steps = min(K, nsteps - n0)
        stash[0] = ckpts[s]
        for k in range(steps - 1):
            lat.step_from(stash[k], stash[k + 1])
        for k in range(steps - 1, -1, -1):
            lat.adjoint_step(stash[k], lam, lam2, gF)
            lam, lam2 = lam2, lam
    return gF


class EnergyAdjoint(torch.autograd.Function):
    """E = EnergyAdjoint.apply(F, lattice, f0_state, nsteps, K).

    F: (3, nz, ny, nx) force field in the lattice's compute dtype; f0_state: an
    internal-layout population buffer (e.g. a copy of ``lattice.state_buffer()``
    after ``init_equilibrium``). Returns E as a 0-d float64 tensor on the
    lattice's device; ``backward`` returns dE/dF. The forward pass keeps its own
    copies of F, of the checkpoints and of the final state, so several applies
    on one lattice, and steps or force changes between forward and backward,
    leave each gradient that of its own forward pass. After either pass the
    lattice's force field is the F of that pass.
    """

    @staticmethod
    def forward(ctx, F, lat, f0_state, nsteps, K):
        Fs = F.detach().to(device=lat.device, dtype=lat.dtype).clone()
        E, ckpts, final = _forward(lat, Fs, f0_state, int(nsteps), int(K))
        ctx.lat, ctx.F, ctx.ckpts, ctx.final = lat, Fs, ckpts, final
        ctx.nsteps, ctx.K = int(nsteps), int(K)
        return torch.tensor(E, dtype=torch.float64, device=F.device)

    @staticmethod
    def backward(ctx, gE):
        gF = _backward(ctx.lat, ctx.F, ctx.ckpts, ctx.final, ctx.nsteps, ctx.K)
        ctx.ckpts = ctx.final = None
        return (gE.to(gF.dtype) * gF), None, None, None, None


def energy_and_grad(lat: Lattice, F: torch.Tensor, f0_state: torch.Tensor, nsteps: int, K: int = 50):
    """Convenience wrapper: (E, dE/dF)."""
    Fp = F.detach().clone().requires_grad_(True)
    E = EnergyAdjoint.apply(Fp, lat, f0_state, nsteps, K)
    E.backward()
    return float(E.detach()), Fp.grad
