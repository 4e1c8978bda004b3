"""Velocity sets, moment exponents and relaxation groups (oracle; test infrastructure).

D2Q9 follows the paper's ordering of particle velocities (Sec. 2,
Eq. velocityd2q9) and its non-orthogonal monomial basis e_x^m e_y^n.

D3Q27 is the three-dimensional generalisation the paper says is possible but
does not derive (end of Sec. 2; Sec. 15): the tensor product of the 1D set
{-1, 0, +1}. Direction index i = (ex+1) + 3(ey+1) + 9(ez+1); the moment with
exponents (a, b, c) in {0,1,2}^3 has index a + 3b + 9c. Weights are products
of the 1D weights (1/6, 2/3, 1/6).

Parity: the tables are pinned in tests by exact properties (invertibility of
the monomial matrix, weight sums and isotropy, opposite-direction symmetry).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

CS2 = 1.0 / 3.0  # squared lattice sound speed (Sec. 4, after Eq. Maxwellian)


@dataclass
class Lattice:
    name: str
    D: int
    e: np.ndarray        # (Q, D) integer velocities
    w: np.ndarray        # (Q,) rest-state weights
    exps: np.ndarray     # (Q, D) moment exponents, one row per moment
    M: np.ndarray = field(init=False)      # (Q, Q) raw-moment matrix: M[k, i] = prod_d e_id^exps_kd
    Minv: np.ndarray = field(init=False)
    opp: np.ndarray = field(init=False)    # opposite direction index

    def __post_init__(self):
        Q = self.e.shape[0]
        M = np.ones((Q, Q))
        for k in range(Q):
            for d in range(self.D):
                M[k] *= self.e[:, d].astype(float) ** self.exps[k, d]
        self.M = M
        self.Minv = np.linalg.inv(M)
        opp = np.empty(Q, dtype=int)
        for i in range(Q):
            opp[i] = int(np.where((self.e == -self.e[i]).all(axis=1))[0][0])
        self.opp = opp

    @property
    def Q(self) -> int:
        return self.e.shape[0]

    def moment_index(self, exps) -> int:
        hit = np.where((self.exps == np.asarray(exps)).all(axis=1))[0]
        if len(hit) != 1:
            raise KeyError(exps)
        return int(hit[0])


def d2q9() -> Lattice:
    """D2Q9 in the paper's order: rest, (+-1,0),(0,+-1), diagonals (Eq. velocityd2q9)."""
    e = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
                  [1, 1], [-1, 1], [-1, -1], [1, -1]])
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    # Monomials in the ascending order the paper lists them (Sec. 2):
    # 1, x, y, xx, yy, xy, xxy, xyy, xxyy
    exps = np.array([[0, 0], [1, 0], [0, 1], [2, 0], [0, 2], [1, 1],
                     [2, 1], [1, 2], [2, 2]])
    return Lattice("D2Q9", 2, e, w, exps)


def d3q27() -> Lattice:
    e = np.array([[ex, ey, ez] for ez in (-1, 0, 1) for ey in (-1, 0, 1) for ex in (-1, 0, 1)])
    w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    w = np.array([w1[a] * w1[b] * w1[c] for a, b, c in e])
    exps = np.array([[a, b, c] for c in range(3) for b in range(3) for a in range(3)])
    return Lattice("D3Q27", 3, e, w, exps)


# ---------------------------------------------------------------- relaxation
#
# The paper fixes D2Q9 rates omega_3 .. omega_8 (Sec. 10): omega_3 on the
# trace of the second-order moments (bulk viscosity), omega_4 = omega_5 on the
# deviatoric second-order moments (shear viscosity,
# nu = cs^2 (1/omega - 1/2)), the rest free. For D3Q27 the grouping below is
# a generalisation of that choice: within each order, moments that the cubic
# symmetry maps onto each other share a rate.

@dataclass
class Relax:
    """Relaxation rates. ``omega_shear`` and ``omega_bulk`` follow Sec. 10;
    the higher-order rates are free parameters (default 1)."""
    omega_shear: float
    omega_bulk: float = 1.0
    omega3: tuple = (1.0, 1.0, 1.0)   # D3Q27: (xyy+xzz)-type, (xyy-xzz)-type, xyz
    omega4: tuple = (1.0, 1.0)        # D3Q27: xxyy-type, xxyz-type
    omega5: float = 1.0
    omega6: float = 1.0
    cs_smag: float = 0.0              # Smagorinsky constant; 0 = no eddy viscosity
    # Sec. 12: rho0 u = sum fbar e + F/2 (density fluctuations removed from the momentum)
    reduced_compressibility: bool = False
    # Sec. 13: fourth- and sixth-order attractors as Cartesian products of the
    # post-collision second-order central moments (divided by rho per extra factor)
    factorized: bool = False
    # Sec. 14: the sub-grid stresses act as a force (acceleration a' = -div R)
    # instead of an eddy viscosity in the collision; cs_smag then sets the
    # stress closure (oracle.sgs) and the collision keeps omega_shear
    sgs_force: bool = False
    # D2Q9 only: the paper's omega_6, omega_7, omega_8 (omega_3 = omega_bulk,
    # omega_4 = omega_5 = omega_shear unless d2q9_omega45 is given)
    d2q9_omega678: tuple = (1.0, 1.0, 1.0)
    d2q9_omega45: tuple | None = None


def relaxation_groups(lat: Lattice, relax: Relax):
    """Return a list of (moment indices, G, rate names) for every non-conserved order.

    Within an order the deficit vector D (attractor minus moment) is mapped to
    group coordinates y = G D, each row relaxed with its own rate, and mapped
    back with G^{-1}. Rate names are 'shear' (may be replaced per cell by the
    eddy-viscosity rate) or a float.
    """
    groups = []
    idx = lambda *p: lat.moment_index(p)
    if lat.name == "D2Q9":
        o45 = relax.d2q9_omega45 or ("shear", "shear")
        o6, o7, o8 = relax.d2q9_omega678
        two = [idx(2, 0), idx(0, 2), idx(1, 1)]
        G2 = np.array([[1.0, 1.0, 0.0], [1.0, -1.0, 0.0], [0.0, 0.0, 1.0]])
        groups.append((two, G2, [relax.omega_bulk, o45[0], o45[1]]))
        groups.append(([idx(2, 1)], np.eye(1), [o6]))
        groups.append(([idx(1, 2)], np.eye(1), [o7]))
        groups.append(([idx(2, 2)], np.eye(1), [o8]))
        return groups
    if lat.name != "D3Q27":
        raise ValueError(lat.name)
    # order 2: xx, yy, zz, xy, xz, yz
    two = [idx(2, 0, 0), idx(0, 2, 0), idx(0, 0, 2), idx(1, 1, 0), idx(1, 0, 1), idx(0, 1, 1)]
    G2 = np.zeros((6, 6))
    G2[0, :3] = 1.0                      # trace -> bulk
    G2[1, 0], G2[1, 1] = 1.0, -1.0       # xx - yy -> shear
    G2[2, 0], G2[2, 2] = 1.0, -1.0       # xx - zz -> shear
    G2[3, 3] = G2[4, 4] = G2[5, 5] = 1.0 # off-diagonal -> shear
    groups.append((two, G2, [relax.omega_bulk] + ["shear"] * 5))
    # order 3: xyy, xzz, xxy, yzz, xxz, yyz, xyz
    three = [idx(1, 2, 0), idx(1, 0, 2), idx(2, 1, 0), idx(0, 1, 2), idx(2, 0, 1), idx(0, 2, 1),
             idx(1, 1, 1)]
    G3 = np.zeros((7, 7))
    for k in range(3):
        G3[k, 2 * k], G3[k, 2 * k + 1] = 1.0, 1.0
        G3[3 + k, 2 * k], G3[3 + k, 2 * k + 1] = 1.0, -1.0
    G3[6, 6] = 1.0
    o3a, o3b, o3c = relax.omega3
    groups.append((three, G3, [o3a] * 3 + [o3b] * 3 + [o3c]))
    four = [idx(2, 2, 0), idx(2, 0, 2), idx(0, 2, 2), idx(2, 1, 1), idx(1, 2, 1), idx(1, 1, 2)]
    o4a, o4b = relax.omega4
    groups.append((four, np.eye(6), [o4a] * 3 + [o4b] * 3))
    five = [idx(2, 2, 1), idx(2, 1, 2), idx(1, 2, 2)]
    groups.append((five, np.eye(3), [relax.omega5] * 3))
    groups.append(([idx(2, 2, 2)], np.eye(1), [relax.omega6]))
    return groups


def maxwell_unit_moment(exps) -> float:
    """Central moment of the continuous Maxwellian per unit density (Sec. 4):
    product over axes of cs^n (n-1)!! for even n, zero for odd n."""
    out = 1.0
    for n in exps:
        n = int(n)
        if n % 2:
            return 0.0
        dfact = 1.0
        for k in range(n - 1, 0, -2):
            dfact *= k
        out *= CS2 ** (n // 2) * dfact
    return out


def binomial_pairs(lat: Lattice):
    """All (p, q, coeff_exponents) with q <= p componentwise, for the frame shift
    of Eq. binomialtheorem: sum_q prod_d C(p_d, q_d) s_d^(p_d - q_d) m_q."""
    from math import comb
    pairs = []
    for p in range(lat.Q):
        for q in range(lat.Q):
            ep, eq = lat.exps[p], lat.exps[q]
            if np.all(eq <= ep):
                c = 1.0
                for d in range(lat.D):
                    c *= comb(int(ep[d]), int(eq[d]))
                pairs.append((p, q, c, tuple(int(x) for x in (ep - eq))))
    return pairs


def moment_orders(lat: Lattice):
    return lat.exps.sum(axis=1)


def all_exponent_tuples(D, nmax=2):
    return [t for t in itertools.product(range(nmax + 1), repeat=D)]
