"""Small driver around ``collide`` and ``stream`` (oracle; test infrastructure).

State convention: ``self.f`` holds fbar(n), the transformed populations after
streaming and before collision (Eq. cascadedLBE3); one ``step`` is collision
(Eq. cascadedcollision1) followed by streaming (Eq. cascadedstreaming1).
Moments at step n come from fbar(n) (Eqs. densitycalculation, velocitycalculation).
"""
from __future__ import annotations

import numpy as np

from . import collide as C
from . import sgs as SG
from .lattice import Lattice, Relax, d3q27
from .stream import stream


class OracleSim:
    def __init__(self, shape, relax: Relax, lat: Lattice | None = None, force=None,
                 walls=False, u_lo=(0.0, 0.0, 0.0), u_hi=(0.0, 0.0, 0.0), rho0=1.0, chunk=1 << 16):
        self.lat = lat or d3q27()
        self.shape = tuple(shape)            # (nz, ny, nx) or (ny, nx)
        self.relax = relax
        self.walls = walls
        self.u_lo, self.u_hi, self.rho0 = u_lo, u_hi, rho0
        self.chunk = chunk
        n = int(np.prod(self.shape))
        D = self.lat.D
        if force is None:
            force = np.zeros(D)
        force = np.asarray(force, dtype=np.float64)
        if force.ndim == 1:
            force = np.repeat(force[:, None], n, axis=1)
        self.F = force.reshape(D, n)
        self.f = np.empty((self.lat.Q, n))
        # sub-grid stress of the previous step (Sec. 14 coupling; zero before the first step)
        self.R_prev = np.zeros((D, D, n))

    # -- initial state ---------------------------------------------------
    def init_equilibrium(self, rho, u):
        n = self.f.shape[1]
        rho = np.broadcast_to(np.asarray(rho, dtype=np.float64).reshape(-1), (n,)).copy()
        u = np.asarray(u, dtype=np.float64).reshape(self.lat.D, n)
        rc = self.relax.reduced_compressibility
        self.f = C.equilibrium_state(rho, u, self.F, self.lat, self.rho0 if rc else None)
        self.R_prev[:] = 0.0

    def set_populations(self, f):
        self.f = np.array(f, dtype=np.float64).reshape(self.lat.Q, -1)
        self.R_prev[:] = 0.0

    # -- forcing -------------------------------------------------------------
    def force_total(self):
        """Force of the collision at the current step: F_ext, plus rho a' with
        a' = -div R(n-1) when the sub-grid stress acts as a force (Sec. 14)."""
        if not self.relax.sgs_force:
            return self.F
        D = self.lat.D
        a = SG.stress_divergence(self.R_prev.reshape((D, D) + self.shape), self.shape).reshape(D, -1)
        return self.F + self.f.sum(axis=0) * a

    # -- time stepping -----------------------------------------------------
    def collide_all(self):
        out = np.empty_like(self.f)
        n = self.f.shape[1]
        F = self.force_total()
        sgs = self.relax.sgs_force
        R_next = np.empty_like(self.R_prev) if sgs else None
        rc = self.relax.reduced_compressibility
        for s in range(0, n, self.chunk):
            e = min(n, s + self.chunk)
            res = C.collide(self.f[:, s:e], F[:, s:e], self.lat, self.relax, rho0=self.rho0, return_parts=sgs)
            if sgs:
                out[:, s:e], parts = res
                rho_s = np.full(e - s, self.rho0) if rc else parts["rho"]
                R_next[:, :, s:e] = SG.sgs_stress(parts["kbar"], rho_s, self.lat, self.relax.omega_shear,
                                                  self.relax.cs_smag)
            else:
                out[:, s:e] = res
        if sgs:
            self.R_prev = R_next
        return out

    def step(self, nsteps=1):
        for _ in range(nsteps):
            post = self.collide_all().reshape((self.lat.Q,) + self.shape)
            self.f = stream(post, self.lat, self.walls, self.u_lo, self.u_hi, self.rho0).reshape(self.lat.Q, -1)

    # -- outputs -----------------------------------------------------------
    def _macro(self):
        rc = self.relax.reduced_compressibility
        return C.macroscopic(self.f, self.force_total(), self.lat, self.rho0 if rc else None)

    def moments(self):
        rho, u = self._macro()
        return rho.reshape(self.shape), u.reshape((self.lat.D,) + self.shape)

    def reduce(self):
        """mass, momentum (D), kinetic energy, non-finite count, min rho, max |u|."""
        rho, u = self._macro()
        mom = (rho[None, :] * u).sum(axis=1)
        ke = 0.5 * (rho * (u ** 2).sum(axis=0)).sum()
        bad = int((~np.isfinite(rho) | ~np.isfinite(u).all(axis=0)).sum())
        umax = float(np.sqrt((u ** 2).sum(axis=0)).max())
        return dict(mass=float(rho.sum()), momentum=mom, ke=float(ke), nonfinite=bad,
                    rho_min=float(rho.min()), umax=umax)
