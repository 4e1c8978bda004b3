"""Streaming step (oracle; test infrastructure).

Standard streaming fbar_a(x + e_a, t+1) = fbar~_a(x, t) (Eq. cascadedstreaming1;
the paper keeps the standard discretisation, Sec. 6). Arrays have shape
(Q, nz, ny, nx) for D3Q27 and (Q, ny, nx) for D2Q9, x fastest.

Periodic wrap is ``np.roll``. Walls (project addition, not in the paper) are
halfway bounce-back planes at y = -1/2 and y = ny - 1/2 moving with velocity
U_w: a population leaving a fluid cell towards the wall returns to the same
cell in the opposite direction one step later, with the momentum correction
-2 w_a rho_w (e_a . U_w) / cs^2 of the outgoing direction a (rho_w = rho_0).

Parity: pinned by exact bookkeeping tests (mass conservation, bijection) and by
the Poiseuille and Couette closed forms.
"""
from __future__ import annotations

import numpy as np

from .lattice import CS2, Lattice


def stream(fpost: np.ndarray, lat: Lattice, walls: bool = False,
           u_lo=(0.0, 0.0, 0.0), u_hi=(0.0, 0.0, 0.0), rho_w: float = 1.0) -> np.ndarray:
    D = lat.D
    yaxis = fpost.ndim - 1 - 1  # axes: (Q, [z,] y, x) -> y is second to last
    out = np.empty_like(fpost)
    for a in range(lat.Q):
        shifted = fpost[a]
        for d in range(D):
            k = int(lat.e[a, d])
            if k:
                axis = fpost.ndim - 2 - d  # x -> last axis
                shifted = np.roll(shifted, k, axis=axis)
        out[a] = shifted
    if walls:
        ny = fpost.shape[yaxis]
        for a in range(lat.Q):
            ey = int(lat.e[a, 1])
            if ey == 0:
                continue
            ab = lat.opp[a]  # outgoing direction that bounces back into a
            corr_lo = -2.0 * lat.w[ab] * rho_w * float(np.dot(lat.e[ab], np.asarray(u_lo)[:D])) / CS2
            corr_hi = -2.0 * lat.w[ab] * rho_w * float(np.dot(lat.e[ab], np.asarray(u_hi)[:D])) / CS2
            idx_out = [slice(None)] * (fpost.ndim - 1)
            if ey == 1:      # arrives at row 0 from the lower wall
                idx_out[yaxis - 1] = 0
                out[a][tuple(idx_out)] = fpost[ab][tuple(idx_out)] + corr_lo
            else:            # arrives at row ny-1 from the upper wall
                idx_out[yaxis - 1] = ny - 1
                out[a][tuple(idx_out)] = fpost[ab][tuple(idx_out)] + corr_hi
    return out
