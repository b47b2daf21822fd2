"""The library's Theorem 2 predictor (dht_theorem2, host only) against the
oracle (oracle/theory.py, itself pinned by Haar Monte Carlo): expected
deflated and undeflated variances, mu_k and V_k, and the Corollary's verdict,
for non-Hermitian spectra, Hermitian positive definite and indefinite ones,
k = 0..N; the inputs are only what a user knows in practice (the sum and sum
of squares of all values and the k deflated ones).

Report (not asserted: the model assumes random singular vectors, which a
Wilson matrix does not have): on the 4^4 Wilson matrix, Theorem 2's
prediction of the Z4 variance of t(D^-1) and of the deflated remainder next
to the exact ||offdiag(.)||_F^2, for k = 0..16 deflated eigenvectors of Q.
"""
import numpy as np
import pytest

from oracle import estimator, lattice, theory
from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links


def _lib():
    from paper_1603_05988_amd import _lib as L
    L.load()
    return L


@pytest.mark.parametrize("kind", ["nonherm", "hpd", "indefinite"])
def test_predictor_matches_oracle(kind):
    L = _lib()
    rs = np.random.default_rng({"nonherm": 1, "hpd": 2, "indefinite": 3}[kind])
    herm = kind != "nonherm"
    for N in (1, 2, 7, 50, 300):
        v = np.exp(rs.normal(0, 1, N))
        if kind == "indefinite":
            v *= rs.choice([-1.0, 1.0], N)
        srt = v[np.argsort(-np.abs(v), kind="stable")]
        for k in sorted({0, 1, N // 3, N - 1, N}):
            out = L.theorem2(N, k, herm, v.sum(), np.sum(v ** 2), srt[:k])
            ref = theory.theorem2_expected_variance(v, k, herm)
            ref0 = theory.remark4_undeflated(v, herm)
            scale = max(ref0, 1e-300)
            assert abs(out["var_k"] - ref) <= 1e-10 * scale, (N, k, out["var_k"], ref)
            assert abs(out["var_0"] - ref0) <= 1e-10 * scale
            if k < N:
                r = srt[k:]
                assert abs(out["mu_k"] - r.mean()) <= 1e-10 * np.abs(v).max()
                assert abs(out["V_k"] - r.var()) <= 1e-8 * np.sum(v ** 2) / max(1, N - k)
            if herm and 0 < k < N and abs(ref - ref0) > 1e-9 * scale:
                assert out["reduces"] == int(theory.corollary_hermitian_reduces(v, k))
            if not herm and k > 0:
                assert out["reduces"] == 1 or ref == ref0


def test_predictor_errors():
    L = _lib()
    with pytest.raises(RuntimeError):
        L.theorem2(10, 11, False, 1.0, 1.0, np.ones(11))
    with pytest.raises(RuntimeError):
        L.theorem2(10, 2, False, float("nan"), 1.0, np.array([1.0, 1.0]))   # squares exceed the total
    with pytest.raises(RuntimeError):
        L.theorem2(10, 0, True, float("nan"), 1.0, [])                      # Hermitian needs the sum
    assert L.theorem2(10, 0, False, float("nan"), 4.0, [])["var_0"] == pytest.approx(3.6)


def test_report_wilson_4444(capsys):
    L = _lib()
    w = WORKLOADS["c1"]
    D = lattice.dense_wilson(gauge_links(w.L, w.eps, w.seed), w.L, w.mass)
    g5 = lattice.gamma5_full(w.V)
    Dinv = estimator.exact_inverse(D)
    N = D.shape[0]
    lam, W = estimator.q_eigenpairs(D, g5, w.k)
    sigma = 1.0 / np.abs(lam)             # the largest singular values of D^-1
    frob2 = float(np.sum(np.abs(Dinv) ** 2))
    rows = []
    for k in range(0, w.k + 1, 4):
        pred = L.theorem2(N, k, False, float("nan"), frob2, sigma[:k])
        AR = Dinv - estimator.deflation_matrix(W[:, :k], np.diag(1.0 / lam[:k]), g5) if k else Dinv
        rows.append((k, pred["var_k"], estimator.offdiag_frobenius2(AR)))
    with capsys.disabled():
        print("\nTheorem 2 on the 4^4 Wilson matrix: k, predicted E Var, exact Var")
        for k, p, e in rows:
            print(f"  {k:3d} {p:12.4f} {e:12.4f}")
    # deflation lowers both the predicted and the exact variance here
    assert rows[-1][1] < rows[0][1] and rows[-1][2] < rows[0][2]
