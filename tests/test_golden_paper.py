"""Values the paper prints, stored under tests/golden/ with their citations,
against the oracle and against the paper's own formulas (CPU only).

- d2q9_moment_basis_K.txt: the orthogonal D2Q9 basis matrix (Eq.
  collisionmatrix2); its columns must equal the printed basis-vector formulas
  evaluated on the velocities of Eq. velocityd2q9 (so a transcription error in
  the fixture or in the oracle fails here), and the oracle's copy must equal it.
- d2q9_basis_norms_D.txt: D = K^T K (Sec. 8, before Eq. vsourceterms0).
- maxwell_central_moments_d2q9.txt: the Maxwellian central moments of Sec. 5
  (Eq. centralmomentMaxwelldistribution), against the central moments of the
  oracle's equilibrium populations.
"""
import os

import numpy as np

from oracle import d2q9_paper as P
from oracle.lattice import d2q9

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=1)


def test_printed_basis_matrix_equals_printed_basis_formulas():
    K = _load("d2q9_moment_basis_K.txt")
    assert K.shape == (9, 9)
    e = d2q9().e.astype(float)          # paper order alpha = 0..8 (Eq. velocityd2q9)
    ex, ey = e[:, 0], e[:, 1]
    # rest, then (+-1, 0), (0, +-1), then the diagonals, as Eq. velocityd2q9 lists them
    assert np.array_equal(np.abs(e).sum(1), [0, 1, 1, 1, 1, 2, 2, 2, 2])
    one = np.ones(9)
    cols = [one, ex, ey, 3 * (ex ** 2 + ey ** 2) - 4 * one, ex ** 2 - ey ** 2, ex * ey,
            -3 * ex ** 2 * ey + 2 * ey, -3 * ex * ey ** 2 + 2 * ex,
            9 * ex ** 2 * ey ** 2 - 6 * (ex ** 2 + ey ** 2) + 4 * one]
    assert np.array_equal(np.stack(cols, 1), K)


def test_oracle_basis_equals_the_printed_one():
    assert np.array_equal(P.K_MATRIX, _load("d2q9_moment_basis_K.txt"))
    assert np.array_equal(P.D_DIAG, _load("d2q9_basis_norms_D.txt"))


def test_printed_norms_are_the_gram_diagonal():
    K = _load("d2q9_moment_basis_K.txt")
    D = _load("d2q9_basis_norms_D.txt")
    assert np.array_equal(K.T @ K, np.diag(D))
    assert np.allclose(np.linalg.inv(K), np.diag(1 / D) @ K.T)


def test_equilibrium_central_moments_are_the_printed_maxwellian_ones():
    """The oracle's force-free equilibrium populations (D2Q9, paper order) have
    central moments about u equal to rho times the printed values; the D3Q27
    tensor extension (reading R9) gives the same values on its c = 0 moments."""
    from oracle import collide as C
    from oracle.lattice import d3q27
    rows = _load("maxwell_central_moments_d2q9.txt").reshape(-1, 4)
    rng = np.random.default_rng(3)
    n = 7
    rho = 1 + 0.1 * rng.standard_normal(n)
    for lat in (d2q9(), d3q27()):
        u = 0.05 * rng.standard_normal((lat.D, n))
        f = C.equilibrium_state(rho, u, np.zeros((lat.D, n)), lat)
        kappa = C.central_moments(f, u, lat)
        for m, k, num, den in rows:
            e = (int(m), int(k)) + (0,) * (lat.D - 2)
            np.testing.assert_allclose(kappa[lat.moment_index(np.array(e))], rho * num / den, rtol=0, atol=1e-14)
