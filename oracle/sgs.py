"""Sub-grid stresses as a force: the filtered kinetic equation of Sec. 14
(oracle; test infrastructure, imported only by tests, smoke() and the CPU
baseline of the benchmark).

Sec. 14 takes the unresolved motion out of the collision: the resolved
populations feel the acceleration a' = -div R, R the filtered product of the
unresolved velocities (the equations for a'_x, a'_y), whose source central
moments obey the same exact identity as a body force with a' in place of
F/rho; the momentum is rho0 u = sum fbar e + rho a'/2
(Eq. resolvedvelocitycalculation) with reduced compressibility, and
rho u = sum fbar e + F/2 with F = rho a' otherwise. The discrete equation is
Eq. resolvedcascadedLBE, i.e. the step of Sec. 11 with this force.

The paper leaves the closure of R open ("any conventional macroscopic
turbulence model"). Readings taken here (each a plain definition):
  * Smagorinsky closure of the deviatoric part, R^d = -2 nu_t S,
    nu_t = (C_s Delta)^2 |S|, Delta = 1 cell, |S| = sqrt(2 S:S); the isotropic
    part of R is absorbed into the pressure;
  * the strain rate from the non-equilibrium second central moments of fbar
    (Chapman-Enskog with the collision's own rate omega0):
    S = -omega0 Pi^d / (2 rho cs^2), Pi^d the traceless part of the second
    central moments (rho0 in place of rho with reduced compressibility, as
    in the eddy-viscosity collision);
  * a'(n) = -div R(n-1) by second-order central differences, R(n-1) taken
    from the pre-collision moments of step n-1 (one step of lag keeps the
    step explicit); R = 0 before the first step; periodic lattices only;
  * the force of the collision at step n is F_ext + rho(n) a'(n).

Parity: the difference operator is pinned to its closed form on Fourier
modes, the stress to a plain shear flow, and the coupled scheme to the steady
Kolmogorov flow of the Smagorinsky closure and to the eddy-viscosity
collision, which it equals at the Chapman-Enskog level.
"""
from __future__ import annotations

import numpy as np

from .lattice import CS2, Lattice


def second_moment_tensor(kbar: np.ndarray, lat: Lattice) -> np.ndarray:
    """(D, D, n) second central moments Pi_ab = kappabar_{e_a + e_b}."""
    D = lat.D
    Pi = np.zeros((D, D) + kbar.shape[1:])
    for a in range(D):
        for b in range(D):
            ex = np.zeros(D, dtype=int)
            ex[a] += 1
            ex[b] += 1
            Pi[a, b] = kbar[lat.moment_index(ex)]
    return Pi


def strain_rate(kbar: np.ndarray, rho: np.ndarray, lat: Lattice, omega0: float) -> np.ndarray:
    """S = -omega0 Pi^d / (2 rho cs^2) from the central moments of fbar."""
    Pi = second_moment_tensor(kbar, lat)
    tr = np.trace(Pi, axis1=0, axis2=1) / lat.D
    for a in range(lat.D):
        Pi[a, a] = Pi[a, a] - tr
    return -omega0 * Pi / (2.0 * rho * CS2)


def sgs_stress(kbar: np.ndarray, rho: np.ndarray, lat: Lattice, omega0: float, cs_smag: float) -> np.ndarray:
    """Deviatoric sub-grid stress R^d = -2 (C_s^2 |S|) S, (D, D, n)."""
    S = strain_rate(kbar, rho, lat, omega0)
    Smag = np.sqrt(2.0 * (S ** 2).sum(axis=(0, 1)))
    return -2.0 * cs_smag ** 2 * Smag * S


def stress_divergence(R: np.ndarray, grid_shape) -> np.ndarray:
    """a'_a = -sum_b (R_ab(x + e_b) - R_ab(x - e_b)) / 2 on a periodic grid.

    R: (D, D) + grid_shape with grid axes ([z,] y, x); returns (D,) + grid_shape.
    """
    D = R.shape[0]
    a = np.zeros((D,) + tuple(grid_shape))
    for i in range(D):
        for b in range(D):
            axis = len(grid_shape) - 1 - b   # x is the last grid axis
            a[i] -= 0.5 * (np.roll(R[i, b], -1, axis=axis) - np.roll(R[i, b], 1, axis=axis))
    return a
