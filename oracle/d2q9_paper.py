"""The paper's own D2Q9 formulas, written out (oracle; test infrastructure only).

This module exists to pin ``oracle.collide`` on the one lattice the paper
derives: it restates, equation by equation, Sec. 9 (raw moments, raw source
moments, central moments from raw ones, projected source moments, source terms
in velocity space), Sec. 10 (cascaded collision kernel g_3 .. g_8) and Sec. 11
(post-collision update). Everything is vectorised over cells; fbar has shape
(9, n) in the paper's velocity order, F has shape (2, n).

Readings of garbled or erroneous passages:

* Eq. rawmomentsourceterm4 prints sigma'_yy = 2 F_x u_y; by symmetry with
  Eq. rawmomentsourceterm3 and consistency with Eqs. sourceterm3/4 it is
  2 F_y u_y (used here).
* The inversion before Eq. vsourceterms0 states K^{-1} = K^T D^{-1}; with K's
  columns K_beta, K^T K = D, so K^{-1} = D^{-1} K^T. The printed S_alpha agree
  with the latter, and are used as printed.
* In the brackets of g_6 and g_7 the source moment is printed without a prime.
  ``g67_sigma`` selects 'raw' (sigma'_xxy, sigma'_xyy of Eqs.
  rawmomentsourceterm6/7) or 'central' (sigma_xxy, sigma_xyy of Eq.
  centralmomentforcingtransformed). Neither makes the third- and fourth-order
  post-collision moments equal to relaxation towards the attractor that
  Sec. 8 states; tests quantify the difference. With F = 0 all readings agree.
"""
from __future__ import annotations

import numpy as np

# Eq. collisionmatrix2 (columns are K_0 .. K_8)
K_MATRIX = np.array([
    [1, 0, 0, -4, 0, 0, 0, 0, 4],
    [1, 1, 0, -1, 1, 0, 0, 2, -2],
    [1, 0, 1, -1, -1, 0, 2, 0, -2],
    [1, -1, 0, -1, 1, 0, 0, -2, -2],
    [1, 0, -1, -1, -1, 0, -2, 0, -2],
    [1, 1, 1, 2, 0, 1, -1, -1, 1],
    [1, -1, 1, 2, 0, -1, -1, 1, 1],
    [1, -1, -1, 2, 0, 1, 1, 1, 1],
    [1, 1, -1, 2, 0, -1, 1, -1, 1],
], dtype=float)
D_DIAG = np.array([9, 6, 6, 36, 4, 4, 12, 12, 36], dtype=float)

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def macroscopic(f, F):
    rho = f.sum(axis=0)
    ux = (EX @ f + 0.5 * F[0]) / rho
    uy = (EY @ f + 0.5 * F[1]) / rho
    return rho, ux, uy


def raw_moments(f):
    """Eqs. rawmomenttransformed3-8 via the subsets A_3 .. B_7."""
    kxx = f[1] + f[3] + f[5] + f[6] + f[7] + f[8]
    kyy = f[2] + f[4] + f[5] + f[6] + f[7] + f[8]
    kxy = (f[5] + f[7]) - (f[6] + f[8])
    kxxy = (f[5] + f[6]) - (f[7] + f[8])
    kxyy = (f[5] + f[8]) - (f[6] + f[7])
    kxxyy = f[5] + f[6] + f[7] + f[8]
    return dict(xx=kxx, yy=kyy, xy=kxy, xxy=kxxy, xyy=kxyy, xxyy=kxxyy)


def central_from_raw(r, rho, ux, uy, Fx, Fy):
    """Eqs. kxxtransform - kxxytransform."""
    c = {}
    c["xx"] = r["xx"] + Fx * ux - rho * ux ** 2
    c["yy"] = r["yy"] + Fy * uy - rho * uy ** 2
    c["xy"] = r["xy"] + 0.5 * (Fx * uy + Fy * ux) - rho * ux * uy
    c["xyy"] = (r["xyy"] - 2 * uy * r["xy"] - ux * r["yy"] - 0.5 * Fx * uy ** 2
                - Fy * ux * uy + 2 * rho * ux * uy ** 2)
    c["xxy"] = (r["xxy"] - 2 * ux * r["xy"] - uy * r["xx"] - 0.5 * Fy * ux ** 2
                - Fx * ux * uy + 2 * rho * ux ** 2 * uy)
    return c


def raw_source_moments(c, rho, ux, uy, Fx, Fy):
    """Eqs. rawmomentsourceterm0-8 (sigma'_yy read as 2 F_y u_y)."""
    s = {}
    s["0"] = np.zeros_like(rho)
    s["x"], s["y"] = Fx, Fy
    s["xx"] = 2 * Fx * ux
    s["yy"] = 2 * Fy * uy
    s["xy"] = Fx * uy + Fy * ux
    s["xxy"] = 2 * Fx * (c["xy"] / rho + ux * uy) + Fy * (c["xx"] / rho + ux ** 2)
    s["xyy"] = Fx * (c["yy"] / rho + uy ** 2) + 2 * Fy * (c["xy"] / rho + ux * uy)
    s["xxyy"] = (2 * Fx * ux * (c["yy"] / rho + uy ** 2) + 2 * Fy * uy * (c["xx"] / rho + ux ** 2)
                 + 2 * Fx / rho * c["xyy"] + 2 * Fy / rho * c["xxy"]
                 + Fx ** 2 / rho ** 2 * c["yy"] + Fy ** 2 / rho ** 2 * c["xx"]
                 + 4 * (Fx * uy / rho + Fy * ux / rho + Fx * Fy / rho ** 2) * c["xy"])
    return s


def central_source_moments(c, rho, Fx, Fy):
    """Eq. centralmomentforcingtransformed."""
    return dict(
        x=Fx, y=Fy,
        xxy=2 * Fx / rho * c["xy"] + Fy / rho * c["xx"],
        xyy=Fx / rho * c["yy"] + 2 * Fy / rho * c["xy"],
        xxyy=(2 * Fx / rho * c["xyy"] + 2 * Fy / rho * c["xxy"] + Fy ** 2 / rho ** 2 * c["xx"]
              + Fx ** 2 / rho ** 2 * c["yy"] + 4 * Fx * Fy / rho ** 2 * c["xy"]),
    )


def projected_source_moments(c, rho, ux, uy, Fx, Fy):
    """Eqs. sourceterm0-8."""
    m = [None] * 9
    m[0] = np.zeros_like(rho)
    m[1], m[2] = Fx, Fy
    m[3] = 6 * (Fx * ux + Fy * uy)
    m[4] = 2 * (Fx * ux - Fy * uy)
    m[5] = Fx * uy + Fy * ux
    m[6] = -6 * Fx * (c["xy"] / rho + ux * uy) - 3 * Fy * (c["xx"] / rho + ux ** 2 - 2.0 / 3.0)
    m[7] = -3 * Fx * (c["yy"] / rho + uy ** 2 - 2.0 / 3.0) - 6 * Fy * (c["xy"] / rho + ux * uy)
    m[8] = (18 * Fx * ux * (c["yy"] / rho + uy ** 2 - 2.0 / 3.0)
            + 18 * Fy * uy * (c["xx"] / rho + ux ** 2 - 2.0 / 3.0)
            + 18 * Fx / rho * c["xyy"] + 18 * Fy / rho * c["xxy"]
            + 9 * Fx ** 2 / rho ** 2 * c["yy"] + 9 * Fy ** 2 / rho ** 2 * c["xx"]
            + 36 * (Fx * uy / rho + Fy * ux / rho + Fx * Fy / rho ** 2) * c["xy"])
    return m


def source_velocity_space(m):
    """Eqs. vsourceterms0-8."""
    S = [None] * 9
    S[0] = (-m[3] + m[8]) / 9
    S[1] = (6 * m[1] - m[3] + 9 * m[4] + 6 * m[7] - 2 * m[8]) / 36
    S[2] = (6 * m[2] - m[3] - 9 * m[4] + 6 * m[6] - 2 * m[8]) / 36
    S[3] = (-6 * m[1] - m[3] + 9 * m[4] - 6 * m[7] - 2 * m[8]) / 36
    S[4] = (-6 * m[2] - m[3] - 9 * m[4] - 6 * m[6] - 2 * m[8]) / 36
    S[5] = (6 * m[1] + 6 * m[2] + 2 * m[3] + 9 * m[5] - 3 * m[6] - 3 * m[7] + m[8]) / 36
    S[6] = (-6 * m[1] + 6 * m[2] + 2 * m[3] - 9 * m[5] - 3 * m[6] + 3 * m[7] + m[8]) / 36
    S[7] = (-6 * m[1] - 6 * m[2] + 2 * m[3] + 9 * m[5] + 3 * m[6] + 3 * m[7] + m[8]) / 36
    S[8] = (6 * m[1] - 6 * m[2] + 2 * m[3] - 9 * m[5] + 3 * m[6] - 3 * m[7] + m[8]) / 36
    return np.array(S)


def collision_kernel(r, s, sig6, sig7, rho, ux, uy, w, rho0=None, att_xxyy=None):
    """Eqs. collisionkernelg3-g8; w = (omega_3, ..., omega_8).

    With ``rho0`` the reduced-compressibility kernel of Sec. 12 (Eqs.
    collisionkernelcompact3-8): rho in the velocity terms becomes
    rho0 - drho, 2 rho0 - drho, 3 rho0 - drho. ``att_xxyy`` (a callable of
    g_3, g_4) replaces the attractor rho/9 of g_8 (factorized model, Sec. 13).
    """
    w3, w4, w5, w6, w7, w8 = w
    if rho0 is None:
        a1, a2, a3 = rho, 2 * rho, 3 * rho
    else:
        drho = rho - rho0
        a1, a2, a3 = rho0 - drho, 2 * rho0 - drho, 3 * rho0 - drho
    g3 = w3 / 12 * (2.0 / 3.0 * rho + a1 * (ux ** 2 + uy ** 2) - (r["xx"] + r["yy"])
                    - 0.5 * (s["xx"] + s["yy"]))
    g4 = w4 / 4 * (a1 * (ux ** 2 - uy ** 2) - (r["xx"] - r["yy"]) - 0.5 * (s["xx"] - s["yy"]))
    g5 = w5 / 4 * (a1 * ux * uy - r["xy"] - 0.5 * s["xy"])
    g6 = (w6 / 4 * (a2 * ux ** 2 * uy + r["xxy"] - 2 * ux * r["xy"] - uy * r["xx"] - 0.5 * sig6)
          - 0.5 * uy * (3 * g3 + g4) - 2 * ux * g5)
    g7 = (w7 / 4 * (a2 * ux * uy ** 2 + r["xyy"] - 2 * uy * r["xy"] - ux * r["yy"] - 0.5 * sig7)
          - 0.5 * ux * (3 * g3 - g4) - 2 * uy * g5)
    bracket = (r["xxyy"] - 2 * ux * r["xyy"] - 2 * uy * r["xxy"] + ux ** 2 * r["yy"]
               + uy ** 2 * r["xx"] + 4 * ux * uy * r["xy"])
    att = rho / 9 if att_xxyy is None else att_xxyy(g3, g4)
    g8 = (w8 / 4 * (att + a3 * ux ** 2 * uy ** 2 - bracket - 0.5 * s["xxyy"])
          - 2 * g3 - 0.5 * uy ** 2 * (3 * g3 + g4) - 0.5 * ux ** 2 * (3 * g3 - g4)
          - 4 * ux * uy * g5 - 2 * uy * g6 - 2 * ux * g7)
    return g3, g4, g5, g6, g7, g8


def central_direct(f, ux, uy):
    """Central moments of fbar about (ux, uy) from their definition (sums over the
    nine directions); used where the raw-to-central formulas of Sec. 9 assume
    rho u = sum fbar e + F/2, i.e. not with reduced compressibility."""
    dx = EX[:, None] - ux[None, :]
    dy = EY[:, None] - uy[None, :]
    m = lambda a, b: (f * dx ** a * dy ** b).sum(axis=0)
    return dict(xx=m(2, 0), yy=m(0, 2), xy=m(1, 1), xxy=m(2, 1), xyy=m(1, 2))


def collide(f, F, w, g67_sigma="raw", return_parts=False, rho0=None, factorized=False):
    """Post-collision fbar~ of Sec. 11 for D2Q9; w = (omega_3, ..., omega_8).

    rho0: reduced compressibility (Sec. 12: rho0 u = sum fbar e + F/2 and the
    kernel of Eqs. collisionkernelcompact3-8). factorized: the fourth-order
    attractor of Eq. factorxxyyfinal (Sec. 13), read with the product divided
    by rho, in the reduced-compressibility form when rho0 is given."""
    f = np.asarray(f, dtype=np.float64)
    Fx, Fy = np.asarray(F[0], dtype=np.float64), np.asarray(F[1], dtype=np.float64)
    rho, ux, uy = macroscopic(f, np.array([Fx, Fy]))
    if rho0 is not None:
        ux = (EX @ f + 0.5 * Fx) / rho0
        uy = (EY @ f + 0.5 * Fy) / rho0
    r = raw_moments(f)
    c = central_from_raw(r, rho, ux, uy, Fx, Fy) if rho0 is None else central_direct(f, ux, uy)
    s = raw_source_moments(c, rho, ux, uy, Fx, Fy)
    if g67_sigma == "raw":
        sig6, sig7 = s["xxy"], s["xyy"]
    elif g67_sigma == "central":
        cs = central_source_moments(c, rho, Fx, Fy)
        sig6, sig7 = cs["xxy"], cs["xyy"]
    else:
        raise ValueError(g67_sigma)
    att = None
    if factorized:
        a1 = rho if rho0 is None else 2 * rho0 - rho
        half_sigma_xxyy = (Fx / rho * c["xyy"] + Fy / rho * c["xxy"] + Fy ** 2 / (2 * rho ** 2) * c["xx"]
                           + Fx ** 2 / (2 * rho ** 2) * c["yy"] + 2 * Fx * Fy / rho ** 2 * c["xy"])

        def att(g3, g4):
            kxx = r["xx"] - a1 * ux ** 2 + Fx * ux + (6 * g3 + 2 * g4)
            kyy = r["yy"] - a1 * uy ** 2 + Fy * uy + (6 * g3 - 2 * g4)
            return kxx * kyy / rho - half_sigma_xxyy
    g3, g4, g5, g6, g7, g8 = collision_kernel(r, s, sig6, sig7, rho, ux, uy, w, rho0=rho0, att_xxyy=att)
    S = source_velocity_space(projected_source_moments(c, rho, ux, uy, Fx, Fy))
    out = np.empty_like(f)
    out[0] = f[0] - 4 * (g3 - g8) + S[0]
    out[1] = f[1] - g3 + g4 + 2 * (g7 - g8) + S[1]
    out[2] = f[2] - g3 - g4 + 2 * (g6 - g8) + S[2]
    out[3] = f[3] - g3 + g4 - 2 * (g7 + g8) + S[3]
    out[4] = f[4] - g3 - g4 - 2 * (g6 + g8) + S[4]
    out[5] = f[5] + 2 * g3 + g5 - g6 - g7 + g8 + S[5]
    out[6] = f[6] + 2 * g3 - g5 - g6 + g7 + g8 + S[6]
    out[7] = f[7] + 2 * g3 + g5 + g6 + g7 + g8 + S[7]
    out[8] = f[8] + 2 * g3 - g5 + g6 - g7 + g8 + S[8]
    if return_parts:
        return out, dict(S=S, g=(g3, g4, g5, g6, g7, g8), central=c, raw_source=s)
    return out
