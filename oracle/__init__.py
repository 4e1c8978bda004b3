"""FP64 CPU oracle for the cascaded central-moment lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it. It shares no code with the HIP library.

What it computes (Premnath & Banerjee, "Inertial frame independent forcing
for discrete velocity Boltzmann equation", arXiv:1202.6074):

* ``lattice``   velocity sets (D2Q9 of Sec. 2, and its D3Q27 tensor-product
                generalisation), monomial moment matrices, relaxation groups.
* ``collide``   the collision step written in central-moment space with
                dense matrices and explicit binomial sums (Secs. 7-10:
                Eqs. binomialtheorem, centralmomentforceexactidentity2,
                transformedcentralmoments, centralmomenttransformed,
                densitycalculation, velocitycalculation).
* ``stream``    standard streaming (Eq. cascadedstreaming1) with periodic
                wrap and, as a project addition, halfway bounce-back walls.
* ``sim``       a small driver: initial state, N steps, moments, FP64 sums.
* ``d2q9_paper`` a literal transcription of the paper's D2Q9 formulas
                (Secs. 9-11), used only to pin ``collide`` on D2Q9.
* ``grad``      the same step in torch FP64 on the CPU, differentiated by
                autograd (reference gradients for the adjoint).

Parity status per function is stated in each module header. The only part
with no value fixed by the paper or by an exact identity is the accuracy of
the three-dimensional higher-order source moments (the paper derives D2Q9
only); their structure is pinned by exact invariants (see tests).
"""
