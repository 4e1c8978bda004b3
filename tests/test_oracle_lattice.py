"""Pins for the oracle's lattice tables and frame transforms (CPU only)."""
import itertools

import numpy as np
import pytest

from oracle import collide as C
from oracle.lattice import CS2, d2q9, d3q27, maxwell_unit_moment

LATS = [d2q9(), d3q27()]


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_weights_isotropy(lat):
    # sum w = 1, sum w e = 0, sum w e_a e_b = cs^2 delta_ab (rest state of the Maxwellian, Sec. 4)
    assert abs(lat.w.sum() - 1.0) < 1e-15
    assert np.abs(lat.w @ lat.e).max() < 1e-15
    second = np.einsum("i,ia,ib->ab", lat.w, lat.e, lat.e)
    assert np.allclose(second, CS2 * np.eye(lat.D), atol=1e-15)
    # fourth-order isotropy for the tensor-product weights: sum w ex^2 ey^2 = cs^4
    assert abs(np.sum(lat.w * lat.e[:, 0] ** 2 * lat.e[:, 1] ** 2) - CS2 ** 2) < 1e-15


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_monomial_matrix_invertible_and_opposites(lat):
    assert abs(np.linalg.det(lat.M)) > 1e-6
    assert np.allclose(lat.M @ lat.Minv, np.eye(lat.Q), atol=1e-13)
    assert (lat.e[lat.opp] == -lat.e).all()
    assert (lat.opp[lat.opp] == np.arange(lat.Q)).all()


def test_d3q27_index_convention():
    lat = d3q27()
    for i, (ex, ey, ez) in enumerate(lat.e):
        assert i == (ex + 1) + 3 * (ey + 1) + 9 * (ez + 1)
        assert lat.opp[i] == 26 - i
    for k, (a, b, c) in enumerate(lat.exps):
        assert k == a + 3 * b + 9 * c


def test_maxwell_moments_match_paper_list():
    # Sec. 4: Pi^M_0 = rho, Pi^M_xx = cs^2 rho, Pi^M_xxyy = cs^4 rho, odd ones vanish
    assert maxwell_unit_moment((0, 0)) == 1.0
    assert maxwell_unit_moment((1, 0)) == 0.0
    assert maxwell_unit_moment((2, 0)) == pytest.approx(1 / 3)
    assert maxwell_unit_moment((1, 1)) == 0.0
    assert maxwell_unit_moment((2, 1)) == 0.0
    assert maxwell_unit_moment((2, 2)) == pytest.approx(1 / 9)
    assert maxwell_unit_moment((4,)) == pytest.approx(3 / 9)   # cs^4 (4-1)!!


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_frame_shift_matches_brute_force_central_moments(lat):
    rng = np.random.default_rng(3)
    n = 7
    f = rng.standard_normal((lat.Q, n))
    u = 0.3 * rng.standard_normal((lat.D, n))
    got = C.central_moments(f, u, lat)
    # brute force: sum_i f_i prod_d (e_id - u_d)^p_d
    want = np.zeros_like(got)
    for k, p in enumerate(lat.exps):
        for i in range(lat.Q):
            term = f[i].copy()
            for d in range(lat.D):
                term = term * (lat.e[i, d] - u[d]) ** p[d]
            want[k] += term
    assert np.abs(got - want).max() < 1e-13
    # shifting back by +u restores the raw moments
    back = C.frame_shift(got, u, lat)
    assert np.abs(back - lat.M @ f).max() < 1e-13


def test_product_equilibrium_has_maxwell_central_moments():
    lat = d3q27()
    rng = np.random.default_rng(4)
    n = 5
    rho = 1 + 0.1 * rng.standard_normal(n)
    u = 0.1 * rng.standard_normal((3, n))
    feq = C.product_equilibrium(rho, u, lat)
    k = C.central_moments(feq, u, lat)
    want = C.maxwell_moments(rho, lat)
    assert np.abs(k - want).max() < 1e-14


def test_all_exponents_present():
    lat = d3q27()
    got = {tuple(p) for p in lat.exps}
    assert got == set(itertools.product(range(3), repeat=3))
