"""Exact invariants of the D3Q27 oracle collision (CPU only).

These pin the three-dimensional generalisation where the paper prints no
values: conservation (Sec. 9, moments of the collision kernel), the
force-free equilibrium as fixed point, the textbook BGK special case,
Galilean invariance of the collision (the paper's central claim, Secs. 1 and
15), a brute-force construction of the source from the exact identity of
Sec. 5, and cubic lattice symmetry.
"""
import itertools

import numpy as np
import pytest

from oracle import collide as C
from oracle.lattice import Relax, d3q27

LAT = d3q27()
RATES = dict(omega_shear=1.37, omega_bulk=1.21, omega3=(0.93, 1.41, 1.12), omega4=(1.31, 0.87),
             omega5=1.19, omega6=1.63)


def _state(n=50, seed=1, famp=0.01, uamp=0.08):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = uamp * rng.standard_normal((3, n))
    F = famp * rng.standard_normal((3, n))
    feq = C.product_equilibrium(rho, u, LAT)
    f = feq * (1 + 0.05 * rng.standard_normal(feq.shape))
    return f, F


@pytest.mark.parametrize("cs", [0.0, 0.17])
def test_mass_and_momentum_exact(cs):
    f, F = _state()
    post = C.collide(f, F, LAT, Relax(cs_smag=cs, **RATES))
    dm = (post - f).sum(axis=0)
    dj = LAT.e.T @ (post - f)
    assert np.abs(dm).max() < 1e-15
    assert np.abs(dj - F).max() < 1e-15


@pytest.mark.parametrize("cs", [0.0, 0.2])
def test_force_free_equilibrium_is_fixed_point(cs):
    rng = np.random.default_rng(2)
    n = 20
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((3, n))
    feq = C.product_equilibrium(rho, u, LAT)
    post = C.collide(feq, np.zeros((3, n)), LAT, Relax(cs_smag=cs, **RATES))
    assert np.abs(post - feq).max() < 1e-15


def test_forced_equilibrium_state_reads_back_and_is_rate_independent():
    rng = np.random.default_rng(3)
    n = 20
    rho = 1 + 0.05 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((3, n))
    F = 0.01 * rng.standard_normal((3, n))
    f0 = C.equilibrium_state(rho, u, F, LAT)
    r2, u2 = C.macroscopic(f0, F, LAT)
    assert np.abs(r2 - rho).max() < 1e-14 and np.abs(u2 - u).max() < 1e-15
    a = C.collide(f0, F, LAT, Relax(**RATES))
    b = C.collide(f0, F, LAT, Relax(omega_shear=0.6, omega_bulk=1.9, omega3=(0.5, 0.6, 0.7)))
    assert np.abs(a - b).max() < 1e-15


@pytest.mark.parametrize("omega", [0.8, 1.0, 1.6, 1.95])
def test_bgk_special_case(omega):
    # All rates equal and F = 0: f~ = f + omega (f^eq - f) with the product equilibrium.
    f, F = _state(seed=4)
    rho, u = C.macroscopic(f, 0 * F, LAT)
    r = Relax(omega_shear=omega, omega_bulk=omega, omega3=(omega,) * 3, omega4=(omega,) * 2,
              omega5=omega, omega6=omega)
    post = C.collide(f, 0 * F, LAT, r)
    feq = C.product_equilibrium(rho, u, LAT)
    assert np.abs(post - (f + omega * (feq - f))).max() < 1e-15


@pytest.mark.parametrize("cs", [0.0, 0.15])
def test_galilean_invariance_of_collision(cs):
    """Two states with identical central moments about different velocities
    (and the same F) have identical post-collision central moments."""
    rng = np.random.default_rng(6)
    n = 30
    rho = 1 + 0.05 * rng.standard_normal(n)
    F = 0.01 * rng.standard_normal((3, n))
    f_ref, _ = _state(n=n, seed=7)
    rho_r, u_r = C.macroscopic(f_ref, F, LAT)
    kbar = C.central_moments(f_ref, u_r, LAT)   # kappabar_100 = -F/2 automatically
    outs = []
    for shift in (np.zeros(3), np.array([0.05, -0.03, 0.02]), np.array([-0.1, 0.07, 0.04])):
        u = u_r + shift[:, None]
        f = LAT.Minv @ C.frame_shift(kbar, u, LAT)
        rr, uu = C.macroscopic(f, F, LAT)
        assert np.abs(uu - u).max() < 1e-14
        post = C.collide(f, F, LAT, Relax(cs_smag=cs, **RATES))
        outs.append(C.central_moments(post, u, LAT))
    assert np.abs(outs[1] - outs[0]).max() < 1e-14
    assert np.abs(outs[2] - outs[0]).max() < 1e-14
    del rho, rho_r


def test_source_recursion_matches_brute_force_identity():
    """Build an untransformed f, evaluate sigma directly from the identity
    Gamma_p = sum_d p_d (F_d/rho) Pi_{p-e_d} on the moments of f, form
    S = M^{-1} shift(sigma) and fbar = f - S/2 (Sec. 6). The collision's
    order-by-order recursion applied to fbar must return the same sigma."""
    rng = np.random.default_rng(9)
    n = 25
    f, _ = _state(n=n, seed=10)
    F = 0.02 * rng.standard_normal((3, n))
    rho = f.sum(axis=0)
    u = (LAT.e.T @ f) / rho                      # velocity of the untransformed f
    kappa = C.central_moments(f, u, LAT)
    sigma = np.zeros_like(kappa)
    for p in range(LAT.Q):
        for d in range(3):
            ep = LAT.exps[p].copy()
            if ep[d]:
                c = ep[d]
                ep[d] -= 1
                sigma[p] += c * (F[d] / rho) * kappa[LAT.moment_index(ep)]
    S = LAT.Minv @ C.frame_shift(sigma, u, LAT)
    fbar = f - 0.5 * S
    rho_b, u_b = C.macroscopic(fbar, F, LAT)
    assert np.abs(rho_b - rho).max() < 1e-15 and np.abs(u_b - u).max() < 1e-15
    kbar = C.central_moments(fbar, u_b, LAT)
    sigma_rec, kappa_rec = C.source_moments(kbar, F, rho_b, LAT)
    assert np.abs(sigma_rec - sigma).max() < 1e-16
    assert np.abs(kappa_rec - kappa).max() < 1e-15


def _axis_perm_tables(perm, flip):
    """Direction and moment permutations for x_new[d] = flip[d] * x_old[perm[d]]."""
    dirs = np.empty(27, dtype=int)
    for i, e in enumerate(LAT.e):
        enew = np.array([flip[d] * e[perm[d]] for d in range(3)])
        dirs[i] = int(np.where((LAT.e == enew).all(axis=1))[0][0])
    return dirs


@pytest.mark.parametrize("perm,flip", [((1, 0, 2), (1, 1, 1)), ((2, 0, 1), (1, -1, 1)),
                                       ((0, 1, 2), (-1, 1, -1))])
def test_cubic_symmetry(perm, flip):
    f, F = _state(seed=12)
    r = Relax(cs_smag=0.1, **RATES)
    post = C.collide(f, F, LAT, r)
    dirs = _axis_perm_tables(perm, flip)
    # rotated input: population i of the new state is population j of the old with e_i = R e_j
    f_rot = np.empty_like(f)
    p_rot = np.empty_like(post)
    f_rot[dirs] = f
    p_rot[dirs] = post
    F_rot = np.array([flip[d] * F[perm[d]] for d in range(3)])
    got = C.collide(f_rot, F_rot, LAT, r)
    assert np.abs(got - p_rot).max() < 1e-15


def test_eddy_rate_reduces_viscosity_rate_and_is_frame_free():
    f, F = _state(seed=13)
    r0 = Relax(**RATES)
    r1 = Relax(cs_smag=0.12, **RATES)
    _, p0 = C.collide(f, F, LAT, r0, return_parts=True)
    _, p1 = C.collide(f, F, LAT, r1, return_parts=True)
    assert np.allclose(p0["omega"], RATES["omega_shear"])
    assert (p1["omega"] < RATES["omega_shear"]).all() and (p1["omega"] > 0).all()
    # the eddy rate uses only central moments: a pure bulk (isotropic) deviation leaves it unchanged
    rho, u = C.macroscopic(f, F, LAT)
    kb = C.central_moments(f, u, LAT)
    for e in ((2, 0, 0), (0, 2, 0), (0, 0, 2)):
        kb[LAT.moment_index(e)] += 0.01
    om_a = C.eddy_omega(C.central_moments(f, u, LAT), rho, LAT, r1)
    om_b = C.eddy_omega(kb, rho, LAT, r1)
    assert np.abs(om_a - om_b).max() < 1e-14


def test_relaxation_groups_are_complete():
    from oracle.lattice import relaxation_groups
    seen = []
    for idx, G, names in relaxation_groups(LAT, Relax(**RATES)):
        assert abs(np.linalg.det(G)) > 0.1
        seen += list(idx)
    orders = LAT.exps.sum(axis=1)
    assert sorted(seen) == sorted(int(i) for i in np.where(orders >= 2)[0])
    assert len(set(itertools.chain(seen))) == 23
