"""Collision step of the cascaded central-moment LBE, FP64 (oracle; test infrastructure).

Written in central-moment space with dense matrices and explicit binomial
sums, one function per step of the method, vectorised over cells
(arrays have shape (Q, ncells) or (D, ncells)).

Steps and the passages they follow:

1. ``macroscopic``       rho = sum_a fbar_a, rho u = sum_a fbar_a e_a + F/2
                         (Eqs. densitycalculation, velocitycalculation).
2. ``raw_moments``       raw moments of fbar, monomial basis (Eq.
                         rawmomenttransformeddistribution1).
3. ``frame_shift``       raw <-> central moments by the binomial theorem
                         (Eq. binomialtheorem).
4. ``source_moments``    central moments sigma of the source from the exact
                         identity Gamma_{x^m y^n} = m F_x/rho Pi_{x^{m-1}y^n} + ...
                         (Eq. centralmomentforceexactidentity2, matched to the
                         discrete moments by Eq. centralmomentforcing), where the
                         moments of the untransformed f follow from those of fbar
                         by kappa = kappabar + sigma/2 (Eq. transformedcentralmoments),
                         taken order by order (Sec. 8).
5. ``attractor``         transformed Maxwellian attractor
                         kappabar^M = kappa^M - sigma/2 (Eq. centralmomenttransformed).
6. ``eddy_omega``        Smagorinsky eddy-viscosity rate (project addition; the
                         paper only places turbulence closures in the kinetic
                         equation, Sec. 14); uses nu = cs^2 (1/omega - 1/2) of Sec. 10.
7. ``collide``           relax each non-conserved central moment of fbar towards
                         its attractor with its group's rate and add the source's
                         central moments (Eq. cascadedcollision1 with the
                         relaxation principle stated at the end of Sec. 8 and in
                         Sec. 10), then return to velocity space exactly.

Reading of the paper taken here (see the design notes): the cascaded kernel
g_3 .. g_8 of Sec. 10 is read as "relax kappabar to kappabar^M, then add S".
The printed third- and fourth-order brackets differ from this reading by
terms proportional to sigma; tests show what they differ by.

Parity: pinned in tests against the literal D2Q9 formulas of the paper
(force-free collision, source terms S_alpha, second-order moments), exact
conservation, Galilean invariance, the BGK special case, brute-force source
moments, and physical closed forms.
"""
from __future__ import annotations

import numpy as np

from .lattice import CS2, Lattice, Relax, binomial_pairs, maxwell_unit_moment, relaxation_groups

_PAIRS_CACHE: dict = {}


def _pairs(lat: Lattice):
    if lat.name not in _PAIRS_CACHE:
        _PAIRS_CACHE[lat.name] = binomial_pairs(lat)
    return _PAIRS_CACHE[lat.name]


def macroscopic(fbar: np.ndarray, F: np.ndarray, lat: Lattice, rho0: float | None = None):
    """rho and u from the transformed populations (Eqs. densitycalculation, velocitycalculation).

    With ``rho0`` given (reduced compressibility, Sec. 12) the momentum is
    rho0 u = sum fbar e + F/2 instead of rho u."""
    rho = fbar.sum(axis=0)
    j = lat.e.T.astype(float) @ fbar
    u = (j + 0.5 * F) / (rho if rho0 is None else rho0)
    return rho, u


def raw_moments(fbar: np.ndarray, lat: Lattice) -> np.ndarray:
    return lat.M @ fbar


def frame_shift(m: np.ndarray, s: np.ndarray, lat: Lattice) -> np.ndarray:
    """Moments about a frame moving with velocity -s relative to the input's frame.

    out_p = sum_{q <= p} prod_d C(p_d, q_d) s_d^(p_d - q_d) m_q.
    With s = -u this maps raw to central moments (Eq. binomialtheorem);
    with s = +u it maps central back to raw.
    """
    out = np.zeros_like(m)
    for p, q, c, dexp in _pairs(lat):
        coef = c
        for d, k in enumerate(dexp):
            if k:
                coef = coef * s[d] ** k
        out[p] += coef * m[q]
    return out


def central_moments(fbar, u, lat):
    return frame_shift(raw_moments(fbar, lat), -u, lat)


def source_moments(kbar: np.ndarray, F: np.ndarray, rho: np.ndarray, lat: Lattice, first_order_zero: bool = True):
    """Central moments sigma of the source term, and kappa of the untransformed f.

    sigma_0 = 0 and, for every other moment p in order of increasing total order,
    sigma_p = sum_d p_d (F_d / rho) kappa_{p - e_d}          (exact identity, Sec. 5)
    kappa_p = kappabar_p + sigma_p / 2                      (Sec. 7)
    Only lower orders appear on the right, so the sweep is explicit.
    With ``first_order_zero`` the first-order kappa are set to their defining
    value 0 (Sec. 8: u is the velocity of f), which the recursion also gives
    for any fbar read with Eq. velocitycalculation; without it the general
    relations of Sec. 8 (before the conserved-moment simplification) result.
    """
    sigma = np.zeros_like(kbar)
    kappa = np.zeros_like(kbar)
    orders = lat.exps.sum(axis=1)
    order = np.argsort(orders, kind="stable")
    for p in order:
        ep = lat.exps[p]
        acc = np.zeros_like(rho)
        for d in range(lat.D):
            if ep[d] > 0:
                lower = ep.copy()
                lower[d] -= 1
                acc = acc + ep[d] * (F[d] / rho) * kappa[lat.moment_index(lower)]
        sigma[p] = acc
        # first-order central moments of f vanish by the definition of u
        # (Sec. 8); the source expressions keep this also with reduced
        # compressibility (Sec. 12)
        if orders[p] == 1 and first_order_zero:
            kappa[p] = 0.0 * kbar[p]
        else:
            kappa[p] = kbar[p] + 0.5 * sigma[p]
    return sigma, kappa


def maxwell_moments(rho: np.ndarray, lat: Lattice) -> np.ndarray:
    """Discrete central moments of the Maxwellian attractor, kappa^M (Eq. centralmomentMaxwelldistribution)."""
    unit = np.array([maxwell_unit_moment(p) for p in lat.exps])
    return unit[:, None] * rho[None, :]


def attractor(rho, sigma, lat):
    """kappabar^M = kappa^M - sigma / 2 (Eq. centralmomenttransformed)."""
    return maxwell_moments(rho, lat) - 0.5 * sigma


def eddy_omega(kbar: np.ndarray, rho: np.ndarray, lat: Lattice, relax: Relax) -> np.ndarray:
    """Per-cell shear relaxation rate with a Smagorinsky eddy viscosity (project addition).

    Pi^d = traceless part of the second-order central moments of fbar. The
    second-order source moments vanish (Eq. centralmomentforcingtransformed),
    so these equal the moments of f (Sec. 8). Chapman-Enskog gives
    Pi^d = -2 rho cs^2 tau S^d with tau = 1/omega, and nu = cs^2 (tau - 1/2).
    Requiring nu_eff = nu_0 + (C_s Delta)^2 |S|, |S| = sqrt(2 S:S), Delta = 1,
    and Q = sqrt(2 Pi^d:Pi^d) = 2 rho cs^2 tau_eff |S|, gives
    tau_eff = tau_0 + C_s^2 |S| / cs^2, i.e. the quadratic
    tau_eff^2 - tau_0 tau_eff - C_s^2 Q / (2 rho cs^4) = 0, whose positive root is
    tau_eff = (tau_0 + sqrt(tau_0^2 + 2 C_s^2 Q / (rho cs^4))) / 2.
    """
    tau0 = 1.0 / relax.omega_shear
    if relax.cs_smag == 0.0 or relax.sgs_force:
        return np.full_like(rho, relax.omega_shear)
    D = lat.D
    Pi = np.zeros((D, D) + rho.shape)
    for a in range(D):
        for b in range(D):
            ex = np.zeros(D, dtype=int)
            ex[a] += 1
            ex[b] += 1
            Pi[a, b] = kbar[lat.moment_index(ex)]
    tr = sum(Pi[a, a] for a in range(D)) / D
    for a in range(D):
        Pi[a, a] = Pi[a, a] - tr
    Qn = np.sqrt(2.0 * (Pi ** 2).sum(axis=(0, 1)))
    tau = 0.5 * (tau0 + np.sqrt(tau0 ** 2 + 2.0 * relax.cs_smag ** 2 * Qn / (rho * CS2 ** 2)))
    return 1.0 / tau


def factorized_attractor(kpost2, rho, sigma, lat: Lattice):
    """Sec. 13 (with the 1/rho of the design notes): the attractor of a moment whose
    exponents are all even is the product over axes of the post-collision
    second-order central moments kappa~_{x^2}, kappa~_{y^2}, ... divided by rho
    for every factor beyond the first, minus sigma/2. Moments with an odd
    exponent contain a first-order factor and keep the Maxwellian value 0.
    Returns {moment index: attractor} for the even moments of order >= 4."""
    out = {}
    for p, ep in enumerate(lat.exps):
        if ep.sum() >= 4 and not (ep % 2).any():
            val = np.ones_like(rho)
            k = 0
            for d in range(lat.D):
                if ep[d] == 2:
                    e2 = np.zeros(lat.D, dtype=int)
                    e2[d] = 2
                    val = val * kpost2[lat.moment_index(e2)]
                    k += 1
            out[p] = val / rho ** (k - 1) - 0.5 * sigma[p]
    return out


def relax_moments(kbar, target, rates_shear, lat: Lattice, relax: Relax, rho=None, sigma=None):
    """Group-wise relaxation of the non-conserved central moments towards ``target``.

    Returns kbar + G^-1 diag(omega) G (target - kbar) order by order; conserved
    moments (orders 0 and 1) are returned unchanged. With ``relax.factorized``
    the even fourth- and sixth-order targets are replaced, after the
    second-order moments are relaxed, by the factorized attractor (Sec. 13).
    """
    out = kbar.copy()
    for idx, G, names in relaxation_groups(lat, relax):
        if relax.factorized and lat.exps[idx[0]].sum() >= 4:
            fa = factorized_attractor(out, rho, sigma, lat)
            target = target.copy()
            for p, v in fa.items():
                target[p] = v
        Dv = target[idx] - kbar[idx]
        y = G @ Dv
        for r, name in enumerate(names):
            rate = rates_shear if name == "shear" else name
            y[r] = rate * y[r]
        out[idx] = kbar[idx] + np.linalg.solve(G, y)
    return out


def collide(fbar: np.ndarray, F: np.ndarray, lat: Lattice, relax: Relax, return_parts=False, rho0=1.0):
    """Post-collision transformed populations (Eq. cascadedcollision1).

    fbar: (Q, n) pre-collision populations; F: (D, n) force per cell. ``rho0``
    is used only with reduced compressibility (Sec. 12).
    """
    fbar = np.asarray(fbar, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    rc = relax.reduced_compressibility
    rho, u = macroscopic(fbar, F, lat, rho0 if rc else None)
    kbar = central_moments(fbar, u, lat)
    sigma, _ = source_moments(kbar, F, rho, lat)
    target = attractor(rho, sigma, lat)
    om = eddy_omega(kbar, np.full_like(rho, rho0) if rc else rho, lat, relax)
    kpost = relax_moments(kbar, target, om, lat, relax, rho, sigma) + sigma
    mpost = frame_shift(kpost, u, lat)
    fpost = lat.Minv @ mpost
    if return_parts:
        return fpost, dict(rho=rho, u=u, kbar=kbar, sigma=sigma, kpost=kpost, omega=om)
    return fpost


def equilibrium_state(rho: np.ndarray, u: np.ndarray, F: np.ndarray, lat: Lattice,
                      rho0: float | None = None) -> np.ndarray:
    """Populations fbar whose central moments equal the attractor kappabar^M(rho, u, F).

    At this state kappa = kappa^M (the untransformed f is the discrete
    Maxwellian), so sigma is the identity of Sec. 5 evaluated on kappa^M and
    kappabar = kappa^M - sigma/2 (Sec. 7-8). Reading rho and u back with
    Eqs. densitycalculation and velocitycalculation returns the inputs.
    """
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    F = np.asarray(F, dtype=np.float64)
    kM = maxwell_moments(rho, lat)
    sigma = np.zeros_like(kM)
    for p in range(lat.Q):
        ep = lat.exps[p]
        for d in range(lat.D):
            if ep[d] > 0:
                lower = ep.copy()
                lower[d] -= 1
                sigma[p] = sigma[p] + ep[d] * (F[d] / rho) * kM[lat.moment_index(lower)]
    kbar = kM - 0.5 * sigma
    if rho0 is not None:
        # reduced compressibility (Sec. 12): rho0 u = sum fbar e + F/2, so the
        # first central moments of fbar about u are (rho0 - rho) u - F/2
        for d in range(lat.D):
            e1 = np.zeros(lat.D, dtype=int)
            e1[d] = 1
            kbar[lat.moment_index(e1)] = (rho0 - rho) * u[d] - 0.5 * F[d]
    return lat.Minv @ frame_shift(kbar, u, lat)


def product_equilibrium(rho, u, lat):
    """Textbook product-form equilibrium rho prod_d phi(e_d, u_d), with
    phi(0,u) = 2/3 - u^2 and phi(+-1,u) = (1/3 + u^2 +- u)/2. Its central
    moments are the Maxwellian ones of Sec. 4 on the tensor-product lattice."""
    out = np.ones((lat.Q,) + np.shape(rho))
    for i in range(lat.Q):
        for d in range(lat.D):
            ed = lat.e[i, d]
            ud = u[d]
            if ed == 0:
                out[i] = out[i] * (2.0 / 3.0 - ud * ud)
            else:
                out[i] = out[i] * 0.5 * (1.0 / 3.0 + ud * ud + ed * ud)
    return out * rho
