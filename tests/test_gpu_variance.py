"""Variance analysis on the 8^3x16 operator over 40 runs of Algorithm 1
(Sections 6.2-6.3): k = 64 eigenvectors of Q from the library's eigensolver
(FP64 storage, Galerkin M), 40 runs (base vectors z0) of 32 hierarchical-
probing probes each, solved in mixed precision to 1e-8, with their projection
coefficients; 256 plain Z4 probes give the Monte Carlo variance V_stoc.
The report (variance_c2.json in the directory DHT_REPORT_DIR names, if set) holds
V_hp(s) with Jackknife errors and R_s at s = 1 .. 32, undeflated and
deflated, and the playback of the deflated estimate with k = 0 .. 64.

Asserted (consistency, not the size of the gains, which the paper's
matrices do not share): playback with all 64 vectors reproduces the records'
deflated quadratures and T_D; with none, the undeflated ones; the deflated
estimate equals the undeflated one within their errors (both are unbiased).
"""
import json

import numpy as np
import pytest

from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links
from reports import write_report

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_variance_report_c2():
    from paper_1603_05988_amd import _lib as L
    w = WORKLOADS["c2"]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    lam, res, st, TD = ctx.eigensolve(w.k, L.FP64, tol=1e-9, max_iter=400, degree=16, seed=11)
    assert st["converged"] == w.k
    H, G5, diag = ctx.deflation_galerkin()
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-8, maxiter=5000)
    R, S = 40, 32
    q = np.zeros((R, S), dtype=np.complex128)
    qd = np.zeros((R, S), dtype=np.complex128)
    coef = np.zeros((R, 2, w.k, S), dtype=np.complex128)
    for r in range(R):
        recs, c1, c2 = ctx.trace_batch(w.seed, 100 + r, True, 0, S, prm, want_coef=True)
        q[r] = [x["q"] for x in recs]
        qd[r] = [x["q_defl"] for x in recs]
        coef[r, 0], coef[r, 1] = c1, c2
    mc = []
    for b in range(0, 256, 64):
        mc += [x["q"] for x in ctx.trace_batch(w.seed, 7, False, b, 64, prm)]
    mc = np.array(mc)
    v_stoc = float(np.sum(np.abs(mc - mc.mean()) ** 2) / (len(mc) - 1))
    s_list = list(range(1, S + 1))
    und = L.hp_variance(q, s_list, v_stoc)
    dfl = L.hp_variance(qd, s_list, v_stoc)
    # playback over k at s = 32, all runs
    k_list = [0, 8, 16, 32, 48, 64]
    play = []
    t_runs = {kk: [] for kk in k_list}
    for r in range(R):
        pq, ptd = L.playback(H, G5, coef[r], q[r], k_list, diagonal=diag)
        if r == 0:
            assert np.abs(pq[-1] - qd[r]).max() <= 1e-10 * np.abs(q[r]).max()
            assert abs(ptd[-1] - TD) <= 1e-12 * abs(TD)
            assert np.array_equal(pq[0], q[r])
        for a, kk in enumerate(k_list):
            t_runs[kk].append(pq[a])
    for kk in k_list:
        o = L.hp_variance(np.array(t_runs[kk]), [S], v_stoc)[0]
        play.append({"k": kk, "var": o["var"], "var_err": o["var_err"], "rs": o["rs"], "rs_err": o["rs_err"]})
    m_u = complex(und[-1]["mean_re"], und[-1]["mean_im"])
    m_d = complex(dfl[-1]["mean_re"], dfl[-1]["mean_im"]) + TD
    assert abs(m_u - m_d) <= 5 * np.hypot(und[-1]["mean_err"], dfl[-1]["mean_err"]), (m_u, m_d)
    out = {"lattice": list(w.L), "runs": R, "probes_per_run": S, "k": w.k, "T_D": [TD.real, TD.imag],
           "sigma_min": float(np.abs(lam).min()), "v_stoc": v_stoc, "mc_probes": len(mc),
           "trace_undeflated": [m_u.real, m_u.imag], "trace_deflated": [m_d.real, m_d.imag],
           "hp": [{"s": a["s"], "var": a["var"], "var_err": a["var_err"], "rs": a["rs"], "rs_err": a["rs_err"],
                   "var_defl": b["var"], "var_defl_err": b["var_err"], "rs_defl": b["rs"], "rs_defl_err": b["rs_err"]}
                  for a, b in zip(und, dfl)],
           "playback_s32": play}
    print(json.dumps(out)[:2000])
    write_report("variance_c2.json", out)
    ctx.close()


def test_variance_report_c3():
    """The same analysis on the 16^3x32 operator (Section 6.2's procedure at the
    third configuration): k = 200 vectors from the preconditioned block
    eigensolver (FP32 storage, Galerkin M), 40 runs of 256 hierarchical-probing
    probes, 256 plain Z4 probes for V_stoc; V_hp(s) and R_s at s = 1 .. 256,
    undeflated and deflated, and playback at s = 256 over k = 0 .. 200.  Written
    to variance_c3.json in the directory DHT_REPORT_DIR names, if set.  Asserted as for
    8^3x16: playback with all vectors reproduces the records, with none the
    undeflated forms, and the two estimates agree within their errors.  Also
    reported: W_d of 10 sampled rows (plain, deflated, masked to 32 HP vectors,
    both; the mask leaves no entry at distance 1) and Theorem 2's predicted
    Monte Carlo variances from ||D^-1||_F^2 (N x the sampled mean squared row
    norm) and the 200 deflated values 1 / sigma, beside the measured ones."""
    from paper_1603_05988_amd import _lib as L
    w = WORKLOADS["c3"]
    U = gauge_links(w.L, w.eps, w.seed)
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    sig, res, st, TD = ctx.lobpcg(w.k, L.FP32, tol=1e-9, max_iter=2000, block=64, precond=True, seed=5)
    assert st["converged"] == w.k
    H, G5, diag = ctx.deflation_galerkin()
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-8, maxiter=5000)
    R, S, B = 40, w.nprobe, w.batch
    q = np.zeros((R, S), dtype=np.complex128)
    qd = np.zeros((R, S), dtype=np.complex128)
    coef = np.zeros((R, 2, w.k, S), dtype=np.complex128)
    for r in range(R):
        for b in range(0, S, B):
            recs, c1, c2 = ctx.trace_batch(w.seed, 100 + r, True, b, B, prm, want_coef=True)
            q[r, b:b + B] = [x["q"] for x in recs]
            qd[r, b:b + B] = [x["q_defl"] for x in recs]
            coef[r, 0, :, b:b + B], coef[r, 1, :, b:b + B] = c1, c2
    mc, mcd = [], []
    for b in range(0, 256, B):
        recs = ctx.trace_batch(w.seed, 7, False, b, B, prm)
        mc += [x["q"] for x in recs]
        mcd += [x["q_defl"] for x in recs]
    mc, mcd = np.array(mc), np.array(mcd)
    v_stoc = float(np.sum(np.abs(mc - mc.mean()) ** 2) / (len(mc) - 1))
    v_stoc_defl = float(np.sum(np.abs(mcd - mcd.mean()) ** 2) / (len(mcd) - 1))
    s_list = [1, 2, 4, 8, 16, 32, 64, 128, 256]
    und = L.hp_variance(q, s_list, v_stoc)
    dfl = L.hp_variance(qd, s_list, v_stoc)
    k_list = [0, 25, 50, 100, 150, 200]
    t_runs = {kk: [] for kk in k_list}
    for r in range(R):
        pq, ptd = L.playback(H, G5, coef[r], q[r], k_list, diagonal=diag)
        if r == 0:
            assert np.abs(pq[-1] - qd[r]).max() <= 1e-10 * np.abs(q[r]).max()
            assert abs(ptd[-1] - TD) <= 1e-12 * abs(TD)
            assert np.array_equal(pq[0], q[r])
        for a, kk in enumerate(k_list):
            t_runs[kk].append(pq[a])
    play = []
    for kk in k_list:
        o = L.hp_variance(np.array(t_runs[kk]), [S], v_stoc)[0]
        play.append({"k": kk, "var": o["var"], "var_err": o["var_err"], "rs": o["rs"], "rs_err": o["rs_err"]})
    m_u = complex(und[-1]["mean_re"], und[-1]["mean_im"])
    m_d = complex(dfl[-1]["mean_re"], dfl[-1]["mean_im"]) + TD
    assert abs(m_u - m_d) <= 5 * np.hypot(und[-1]["mean_err"], dfl[-1]["mean_err"]), (m_u, m_d)
    # W_d profiles of 10 sampled rows (Section 6.2) and Theorem 2's prediction
    # (Section 2.1) from what one knows in practice: ||D^-1||_F^2 estimated as N
    # times the mean squared row norm of the sampled rows, and the k deflated
    # singular values 1 / sigma of D^-1
    rows = np.random.default_rng(12).choice(w.N, 10, replace=False)
    prof = {}
    for name, defl, hp in (("monte_carlo", False, 0), ("deflation", True, 0), ("hp32", False, 32),
                           ("hp32_deflation", True, 32)):
        Wg, m = ctx.distance_profile(rows, prm, deflate=defl, hp_vectors=hp)
        prof[name] = Wg.mean(axis=0).tolist()
    frob2 = float(w.N * np.dot(prof["monte_carlo"], m))   # N x the mean squared row norm
    frob2_defl = float(w.N * np.dot(prof["deflation"], m))
    thm = L.theorem2(w.N, w.k, False, float("nan"), frob2, 1.0 / np.sort(sig))
    assert prof["hp32"][1] == 0.0 and prof["hp32"][0] > 0.0
    out = {"lattice": list(w.L), "runs": R, "probes_per_run": S, "k": w.k, "T_D": [TD.real, TD.imag],
           "sigma_min": float(np.min(sig)), "v_stoc": v_stoc, "v_stoc_deflated": v_stoc_defl, "mc_probes": len(mc),
           "trace_undeflated": [m_u.real, m_u.imag], "trace_deflated": [m_d.real, m_d.imag],
           "hp": [{"s": a["s"], "var": a["var"], "var_err": a["var_err"], "rs": a["rs"], "rs_err": a["rs_err"],
                   "var_defl": b["var"], "var_defl_err": b["var_err"], "rs_defl": b["rs"], "rs_defl_err": b["rs_err"]}
                  for a, b in zip(und, dfl)],
           "playback_s%d" % S: play,
           "wd_rows": rows.tolist(), "wd_m": m.tolist(), "wd": prof,
           "theorem2": {"frob2_sampled": frob2, "frob2_deflated_sampled": frob2_defl,
                        "frob2_minus_deflated_sigma2": frob2 - float(np.sum(1.0 / np.asarray(sig) ** 2)),
                        "predicted_var_0": thm["var_0"], "predicted_var_k": thm["var_k"], "predicted_ratio": thm["ratio"],
                        "measured_var_0": v_stoc, "measured_var_k": v_stoc_defl,
                        "measured_ratio": v_stoc_defl / v_stoc}}
    print(json.dumps(out)[:2000])
    write_report("variance_c3.json", out)
    ctx.close()
