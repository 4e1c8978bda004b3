"""Reference gradients: the LBM step in torch FP64 on the CPU, differentiated
by autograd (oracle; test infrastructure).

The collision is written again in torch, following the same definition as
``oracle.collide`` (raw moments by the monomial matrix, central moments by the
binomial shift of Eq. binomialtheorem, sources from the identity of Sec. 5
taken order by order, relaxation towards kappa^M - sigma/2 by groups, return
by the inverse shift and M^{-1}; with cs_smag > 0 the shear rate of each cell
is the Smagorinsky rate of ``oracle.collide.eddy_omega``, whose norm
Q = sqrt(2 Pi^d : Pi^d) is given the derivative 0 where Q = 0, the one point
where it has none; with the Sec. 12 and 13 flags, the reduced-compressibility
velocity rho0 u = sum fbar e + F/2 (rho0 = 1) and the factorized attractors
of ``oracle.collide.factorized_attractor``); streaming is ``torch.roll``
(periodic), with
optional halfway bounce-back walls at y = -1/2 and y = ny - 1/2 following the
rule of ``oracle.stream`` (a population arriving from a wall is the opposite
population of the same cell plus the moving-wall correction).
The loss is E = sum_x rho |u|^2 / 2 at the final step, with
rho u = sum fbar e + F/2 (Eq. velocitycalculation; rho0 u with reduced
compressibility, Sec. 12).

Parity: pinned in tests against ``oracle.collide`` and ``oracle.stream``
(forward values) and by central finite differences (gradients).
"""
from __future__ import annotations

import numpy as np
import torch

from .lattice import CS2, Lattice, Relax, binomial_pairs, maxwell_unit_moment, relaxation_groups


class TorchStep:
    def __init__(self, lat: Lattice, relax: Relax, walls: bool = False, u_lo=(0.0, 0.0, 0.0),
                 u_hi=(0.0, 0.0, 0.0), rho_w: float = 1.0):
        if relax.sgs_force:
            raise ValueError("reference gradients are for the collision with an eddy rate or none, "
                             "not for the sub-grid stress as a force")
        self.lat = lat
        self.relax = relax
        self.walls = walls
        self.u_lo, self.u_hi, self.rho_w = np.asarray(u_lo, float), np.asarray(u_hi, float), float(rho_w)
        t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))
        self.M = t(lat.M)
        self.Minv = t(lat.Minv)
        self.E = t(lat.e.T.astype(np.float64))
        self.pairs = binomial_pairs(lat)
        self.unit = t([maxwell_unit_moment(p) for p in lat.exps])
        self.order = [int(p) for p in np.argsort(lat.exps.sum(axis=1), kind="stable")]
        self.groups = [(list(idx), t(G), t(np.linalg.inv(G)), names)
                       for idx, G, names in relaxation_groups(lat, relax)]

    def shift(self, m, s):
        out = [torch.zeros_like(m[0]) for _ in range(self.lat.Q)]
        for p, q, c, dexp in self.pairs:
            coef = c
            for d, k in enumerate(dexp):
                if k:
                    coef = coef * s[d] ** k
            out[p] = out[p] + coef * m[q]
        return torch.stack(out)

    def eddy_rate(self, kbar, rho):
        """Per-cell shear rate with the Smagorinsky eddy viscosity: the
        traceless second-order central moments Pi^d of fbar, Q = sqrt(2 Pi^d : Pi^d)
        and tau = (tau_0 + sqrt(tau_0^2 + 2 C_s^2 Q / (rho cs^4))) / 2, omega = 1 / tau."""
        lat, D = self.lat, self.lat.D
        Pi = [[None] * D for _ in range(D)]
        for a in range(D):
            for b in range(D):
                ex = np.zeros(D, dtype=int)
                ex[a] += 1
                ex[b] += 1
                Pi[a][b] = kbar[lat.moment_index(ex)]
        tr = sum(Pi[a][a] for a in range(D)) / D
        for a in range(D):
            Pi[a][a] = Pi[a][a] - tr
        q2 = 2.0 * sum(Pi[a][b] ** 2 for a in range(D) for b in range(D))
        pos = q2 > 0
        Q = torch.where(pos, torch.sqrt(torch.where(pos, q2, torch.ones_like(q2))), torch.zeros_like(q2))
        tau0 = 1.0 / self.relax.omega_shear
        tau = 0.5 * (tau0 + torch.sqrt(tau0 ** 2 + 2.0 * self.relax.cs_smag ** 2 * Q / (rho * CS2 ** 2)))
        return 1.0 / tau

    def factorized_targets(self, post, rho, sigma):
        """Sec. 13 attractors of the even moments of order >= 4 from the
        post-collision second-order moments (oracle.collide.factorized_attractor)."""
        lat, out = self.lat, {}
        for p, ep in enumerate(lat.exps):
            if ep.sum() >= 4 and not (ep % 2).any():
                val, k = torch.ones_like(rho), 0
                for d in range(lat.D):
                    if ep[d] == 2:
                        e2 = np.zeros(lat.D, dtype=int)
                        e2[d] = 2
                        val = val * post[lat.moment_index(e2)]
                        k += 1
                out[p] = val / rho ** (k - 1) - 0.5 * sigma[p]
        return out

    def collide(self, f, F):
        lat = self.lat
        rc = self.relax.reduced_compressibility
        rho = f.sum(0)
        u = (self.E @ f + 0.5 * F) / (1.0 if rc else rho)
        kbar = self.shift(self.M @ f, -u)
        om = self.eddy_rate(kbar, torch.ones_like(rho) if rc else rho) if self.relax.cs_smag else self.relax.omega_shear
        sigma = [torch.zeros_like(rho) for _ in range(lat.Q)]
        kappa = [None] * lat.Q
        for p in self.order:
            ep = lat.exps[p]
            acc = torch.zeros_like(rho)
            for d in range(lat.D):
                if ep[d] > 0:
                    low = ep.copy()
                    low[d] -= 1
                    acc = acc + float(ep[d]) * (F[d] / rho) * kappa[lat.moment_index(low)]
            sigma[p] = acc
            # the first-order central moments of f vanish by the definition of u;
            # with reduced compressibility kbar_1 no longer equals -sigma_1/2, and
            # the sources keep kappa_1 = 0 (as oracle.collide does)
            kappa[p] = torch.zeros_like(rho) if ep.sum() == 1 else kbar[p] + 0.5 * acc
        sigma = torch.stack(sigma)
        target = self.unit[:, None] * rho[None, :] - 0.5 * sigma
        post = [kbar[p] for p in range(lat.Q)]
        for idx, G, Ginv, names in self.groups:
            if self.relax.factorized and lat.exps[idx[0]].sum() >= 4:
                target = target.clone()
                for p, v in self.factorized_targets(post, rho, sigma).items():
                    target[p] = v
            D = target[idx] - kbar[idx]
            y = G @ D
            y = torch.stack([(om if nm == "shear" else float(nm)) * y[r] for r, nm in enumerate(names)])
            upd = Ginv @ y
            for r, p in enumerate(idx):
                post[p] = kbar[p] + upd[r]
        kpost = torch.stack(post) + sigma
        return self.Minv @ self.shift(kpost, u)

    def stream(self, fpost, shape):
        nz, ny, nx = shape
        g = fpost.reshape(self.lat.Q, nz, ny, nx)
        out = []
        for i in range(self.lat.Q):
            ex, ey, ez = (int(v) for v in self.lat.e[i])
            out.append(torch.roll(g[i], shifts=(ez, ey, ex), dims=(0, 1, 2)))
        if self.walls:
            D = self.lat.D
            for i in range(self.lat.Q):
                ey = int(self.lat.e[i, 1])
                if ey == 0:
                    continue
                ib = int(self.lat.opp[i])   # the direction that left towards the wall
                U, yrow = (self.u_lo, 0) if ey == 1 else (self.u_hi, ny - 1)
                corr = -2.0 * self.lat.w[ib] * self.rho_w * float(np.dot(self.lat.e[ib], U[:D])) / CS2
                o = out[i].clone()
                o[:, yrow, :] = g[ib][:, yrow, :] + corr
                out[i] = o
        return torch.stack(out).reshape(self.lat.Q, -1)

    def energy(self, f0, F, nsteps, shape):
        """E = sum rho |u|^2 / 2 after nsteps, u as read by oracle.sim (Eq.
        velocitycalculation; rho0 u = sum fbar e + F/2 with reduced
        compressibility, Sec. 12)."""
        f = f0
        for _ in range(nsteps):
            f = self.stream(self.collide(f, F), shape)
        rho = f.sum(0)
        j = self.E @ f + 0.5 * F
        if self.relax.reduced_compressibility:
            return 0.5 * (rho * (j ** 2).sum(0)).sum()   # rho0 = 1
        return 0.5 * ((j ** 2).sum(0) / rho).sum()


def energy_gradient(lat: Lattice, relax: Relax, f0: np.ndarray, F: np.ndarray, nsteps: int, shape, **walls):
    """E and dE/dF for a periodic box (or with walls: walls=True, u_lo, u_hi);
    f0 (Q, n) canonical, F (3, n)."""
    st = TorchStep(lat, relax, **walls)
    Ft = torch.tensor(np.asarray(F, dtype=np.float64), requires_grad=True)
    E = st.energy(torch.tensor(np.asarray(f0, dtype=np.float64)), Ft, nsteps, shape)
    E.backward()
    return float(E.detach()), Ft.grad.numpy()
