"""Pins of the oracle's variance theory (Section 2).

- Theorem 1, eq. varAr: equals ||offdiag(A_R)||_F^2 computed directly, for a
  random complex matrix and for the inverse of a small Wilson matrix;
- eq. vA-vAR: equals the difference of the two direct norms;
- the 3x3 example of Section 2 reproduces the four regimes the paper states.
"""
import numpy as np
import pytest

from oracle import estimator, lattice, theory
from paper_1603_05988_amd.workloads import gauge_links


def _mats():
    rs = np.random.default_rng(2)
    A = rs.standard_normal((40, 40)) + 1j * rs.standard_normal((40, 40))
    L = (2, 2, 2, 4)
    D = lattice.dense_wilson(gauge_links(L, 0.6, 3), L, -0.1)
    return [A, estimator.exact_inverse(D)]


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("k", [0, 1, 7])
def test_theorem1_variance(which, k):
    A = _mats()[which]
    direct = estimator.offdiag_frobenius2(theory.deflated_remainder(A, k))
    formula = theory.variance_deflated_theorem1(A, k)
    assert abs(direct - formula) <= 1e-10 * estimator.offdiag_frobenius2(A)
    diff = theory.variance_difference_theorem1(A, k)
    ref = estimator.offdiag_frobenius2(A) - direct
    assert abs(diff - ref) <= 1e-10 * estimator.offdiag_frobenius2(A)


def test_3x3_example_regimes():
    ds = np.linspace(0.01, 4.0, 60)
    # s = 0.5: deflation never helps (Var(A_r) >= Var(A) <=> ratio <= 1)
    assert all(theory.example_3x3_ratio(0.5, d) <= 1 + 1e-12 for d in ds)
    # d = 0.001: no (appreciable) reduction regardless of the separation
    for s in (0.5, 1.0, 2.0, 5.0):
        assert abs(theory.example_3x3_ratio(s, 0.001) - 1) <= 1e-4
    # s = 1: no reduction for d <= 1, reduction for d > 1
    assert all(theory.example_3x3_ratio(1.0, d) <= 1 + 1e-9 for d in ds if d <= 1.0)
    assert all(theory.example_3x3_ratio(1.0, d) > 1 for d in ds if d > 1.0 + 1e-9)
    # s = 2: reduction for all d (away from the degenerate d -> 0 limit)
    assert all(theory.example_3x3_ratio(2.0, d) > 1 for d in ds if d >= 0.05)
