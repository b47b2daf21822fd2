"""Benchmark: RHS solves/s of Algorithm 1 batches on one MI355X.

One step = one pass of the whole hot path over one batch of B = 16
hierarchical-probing probes on the 32^3x64 Wilson lattice (N = 25,165,824):
probe generation, the solve D X = Z to relative true residual 1e-8 (FP64
defect correction around an FP32- or BF16-storage BiCGStab on the even/odd
system), the deflation projection against a k = 1000 BF16 basis (MFMA), the
FP64 quadratic forms and the running estimates.  Inputs (links, basis) are
resident in HBM before the timed region.

The basis here is synthetic (Gaussian columns rounded to BF16 with the
diagonal Galerkin inverse): the projection streams exactly the bytes and
performs exactly the flops of a k = 1000 eigenvector basis, and the estimator
stays unbiased for any basis; computing 1000 eigenvectors at this size is
setup outside the measured path.

Prints one JSON line.  --gpus N with N > 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RHS solves/s (res 1e-8) at 32^3x64, mixed+learned vs FP64; dslash GB/s"
HBM_PEAK_GBPS = 8000.0
BF16_MFMA_PEAK_TFLOPS = 2500.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 PMC summaries, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except ValueError:
        return None
    ent = data.get(kernel + "@" + workload)
    if not ent or ent.get("source_hash") != source_hash(ent.get("sources", [])):
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(U, w, k: int, hp: bool):
    """The oracle (plain-C FP64 stencil BiCGStab, full lattice) on a bounded
    sample: one probe of the same workload solved to the same tolerance, its
    z^H x, and the projection on 8 basis columns scaled to k."""
    import numpy as np
    from oracle import rng, stencil
    z = rng.probe(w.L, w.seed, 0, hp, 0)
    t0 = time.time()
    x, st, it, rr = stencil.solve(U, w.L, w.mass, z, w.tol, 5000)
    t_solve = time.time() - t0
    t0 = time.time()
    q = np.vdot(z, x.ravel())
    t_q = time.time() - t0
    rs = np.random.default_rng(0)
    Wc = (rs.standard_normal((8, z.size)) + 1j * rs.standard_normal((8, z.size)))
    t1 = time.time()
    stencil.project(Wc, z)
    t_proj = (time.time() - t1) * (k / 8.0)
    total = t_solve + t_q + t_proj
    return {
        "value": 1.0 / total,
        "unit": "RHS solves/s",
        "cores": stencil.num_threads(),
        "kind": "oracle",
        "sample": ("1 probe of the 32^3x64 workload: C-oracle FP64 BiCGStab to %.0e (%d iterations, %.1f s, "
                   "true residual %.1e) plus its projection on 8 basis columns scaled to k=%d (%.1f s)"
                   % (w.tol, it, t_solve, rr, k, t_proj)),
        "status": st,
        "q": [q.real, q.imag],
    }


def host_info():
    """Cores, CPU model and memory of the host the CPU baseline runs on."""
    info = {"nproc": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["mem_gb"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def small_config_legs(L, torch, np, run_cpu: bool):
    """The 8^3x16 (64 right-hand sides) and 16^3x32 (16) solves to 1e-8 on the
    GPU (mixed BiCGStab, Z4 probes, no deflation) and, beside them, the oracle's
    C stencil FP64 BiCGStab on the host cores for the same probes."""
    from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links
    out = {}
    for name, nrhs in (("c2", 64), ("c3", 16)):
        w = WORKLOADS[name]
        U = gauge_links(w.L, w.eps, w.seed)
        c = L.Context(w.L, w.mass)
        c.set_gauge(torch.from_numpy(U).cuda())
        prm = c.params(L.SOLVER_DC_BICGSTAB, inner=L.BF16, tol=1e-8, maxiter=5000)
        c.trace_batch(w.seed, 0, False, 0, nrhs, prm)   # warm-up
        torch.cuda.synchronize()
        t0 = time.time()
        reps = 3
        for r in range(reps):
            recs = c.trace_batch(w.seed, 0, False, 0, nrhs, prm)
        torch.cuda.synchronize()
        gpu = reps * nrhs / (time.time() - t0)
        c.close()
        ent = {"lattice": list(w.L), "nrhs": nrhs, "gpu_rhs_per_s": round(gpu, 2),
               "gpu_worst_residual": max(r["true_resid"] for r in recs)}
        if run_cpu:
            from oracle import rng, stencil
            t0 = time.time()
            its = []
            for j in range(nrhs):
                z = rng.probe(w.L, w.seed, 0, False, j)
                x, st, it, rr = stencil.solve(U, w.L, w.mass, z, 1e-8, 5000)
                its.append(it)
            el = time.time() - t0
            ent.update({"cpu_rhs_per_s": round(nrhs / el, 3), "cpu_seconds": round(el, 2),
                        "cpu_mean_iters": float(np.mean(its)), "gpu_over_cpu": round(gpu / (nrhs / el), 1)})
        out[w.name] = ent
    return out


def train_network(L, torch, np, npairs: int, epochs: int):
    """The learned preconditioner of the 8^3x16 recipe: (residual, error) pairs
    from FGMRES(4) restarts of Z4 probes (x* from FP64 BiCGStab to 1e-12),
    Adam on the GPU; returns the weights and a summary (held-out losses of the
    Jacobi term alone and of the trained network)."""
    from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links
    w4 = WORKLOADS["c4"]
    c4 = L.Context(w4.L, w4.mass)
    c4.set_gauge(torch.from_numpy(gauge_links(w4.L, w4.eps, w4.seed)).cuda())
    t0 = time.time()
    Rs, Es, n, run = [], [], 0, 1000
    while n < npairs:
        R, E = c4.nn_make_pairs(w4.seed, run, False, 0, 16, 4, min(512, npairs - n))
        Rs.append(R.clone())
        Es.append(E.clone())
        n += R.shape[0]
        run += 1
        del R, E
    R = torch.cat(Rs)
    E = torch.cat(Es)
    del Rs, Es
    Rh, Eh = c4.nn_make_pairs(w4.seed, 300, False, 0, 16, 4, 32)   # held out
    t_pairs = time.time() - t0
    skip = 1.0 / (4.0 + w4.mass)
    c4.nn_init(0)
    c4.nn_set_skip(skip)
    init = c4.nn_get_weights()
    c4.nn_set_weights([np.zeros_like(x) for x in init])
    l_jac, _ = c4.nn_grad(Rh, Eh)
    c4.nn_set_weights(init)
    t0 = time.time()
    last = c4.nn_train(R, E, epochs=epochs, batch=16, lr=3e-4)
    torch.cuda.synchronize()
    t_train = time.time() - t0
    l_tr, _ = c4.nn_grad(Rh, Eh)
    weights = c4.nn_get_weights()
    c4.close()
    del R, E, Rh, Eh
    torch.cuda.empty_cache()
    return weights, {"trained_on": w4.name, "pairs": n, "epochs": epochs, "pair_seconds": round(t_pairs, 1),
                     "train_seconds": round(t_train, 1), "last_epoch_loss": last,
                     "heldout_loss_jacobi_only": l_jac, "heldout_loss_trained": l_tr}


def dirac_basis(np):
    """The 16 products of the chiral-basis gamma matrices (g5 = diag(1, 1, -1, -1))."""
    sig = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    z, one = np.zeros((2, 2)), np.eye(2)
    g = [np.block([[z, -1j * s_], [1j * s_, z]]) for s_ in sig] + [np.block([[z, one], [one, z]])]
    out = []
    for mask in range(16):
        m = np.eye(4, dtype=np.complex128)
        for mu in range(4):
            if mask >> mu & 1:
                m = m @ g[mu]
        out.append(m)
    return np.array(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--inner", default="bf16", choices=["fp32", "bf16"])
    ap.add_argument("--inner-tol", type=float, default=0.0, help="inner relative residual per outer cycle (0: library default)")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--proj-window", type=int, default=64,
                    help="probes per pass over the deflation basis (0: each batch on its own)")
    ap.add_argument("--fp64-steps", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel HIP-event timing")
    ap.add_argument("--tune", default="auto", choices=["auto", "off"],
                    help="autotune the hopping-kernel shape before timing (off: built-in default)")
    ap.add_argument("--tune-cache", default=None, help="JSON table to load the shapes from / save them to")
    ap.add_argument("--gamma-steps", type=int, default=2,
                    help="timed batches of Tr(Gamma D^-1) for the 16 Dirac matrices at once (0: skip)")
    ap.add_argument("--nn-steps", type=int, default=2, help="timed batches of FGMRES + learned preconditioner (0: skip)")
    ap.add_argument("--nn-pairs", type=int, default=20480, help="training pairs of the network (8^3x16 recipe)")
    ap.add_argument("--nn-epochs", type=int, default=4)
    ap.add_argument("--nn-restart", type=int, default=16,
                    help="FGMRES restart at 32^3x64 (its FP32 bases must fit beside the 100 GB deflation basis)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (--gpus %d requested); probes shard across GPUs "
              "by design, but no multi-GPU path is built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1603_05988_amd import _lib as L
    from paper_1603_05988_amd.workloads import WORKLOADS, gauge_links

    w = WORKLOADS[args.workload]
    k = args.k if args.k is not None else w.k
    B = w.batch
    small = small_config_legs(L, torch, np, not args.no_cpu)
    for nm, ent in small.items():
        log("%s: GPU %.1f RHS/s%s" % (nm, ent["gpu_rhs_per_s"], (", CPU oracle %.2f RHS/s (%.1f s)" % (
            ent["cpu_rhs_per_s"], ent["cpu_seconds"])) if "cpu_rhs_per_s" in ent else ""))
    nn_weights, nn_info = None, None
    if args.nn_steps > 0:   # trained first: its pairs are freed before the large lattice is set up
        nn_weights, nn_info = train_network(L, torch, np, args.nn_pairs, args.nn_epochs)
        log("network trained on %d pairs (%d epochs, %.1f s): held-out loss %.4f (Jacobi term alone %.4f)"
            % (nn_info["pairs"], args.nn_epochs, nn_info["train_seconds"], nn_info["heldout_loss_trained"],
               nn_info["heldout_loss_jacobi_only"]))
    t0 = time.time()
    U = gauge_links(w.L, w.eps, w.seed)
    log("links generated in %.1f s" % (time.time() - t0))
    ctx = L.Context(w.L, w.mass)
    ctx.set_gauge(torch.from_numpy(U).cuda())
    if args.no_cpu:
        del U

    # synthetic BF16 basis, generated on the device in blocks
    t0 = time.time()
    g = torch.Generator(device="cuda")
    g.manual_seed(w.seed)
    ctx.begin_deflation(k, L.BF16)
    blk = 32
    for j in range(0, k, blk):
        n = min(blk, k - j)
        Wb = torch.randn((n, w.N), dtype=torch.complex128, device="cuda", generator=g)
        Wb /= torch.linalg.vector_norm(Wb, dim=1, keepdim=True)
        ctx.set_deflation_columns(j, Wb)
        del Wb
    torch.cuda.empty_cache()
    TD = ctx.finalize_deflation(diagonal=True)
    t_setup = time.time() - t0
    log("deflation basis k=%d set up in %.1f s, T_D = %.6g" % (k, t_setup, TD.real))

    inner = L.FP32 if args.inner == "fp32" else L.BF16
    prm = ctx.params(L.SOLVER_DC_BICGSTAB, inner=inner, tol=w.tol, maxiter=5000, inner_tol=args.inner_tol)
    ctx.set_projection_window(args.proj_window)
    ws_bytes = ctx.workspace_size(B, prm)   # the caller-owned workspace this configuration would need
    log("workspace plan for batches of %d: %.2f GB" % (B, ws_bytes / 1e9))
    proj_tune = None
    if args.tune == "auto":   # split of the basis over the MFMA projection's workgroups, for the window
        proj_tune = ctx.autotune_projection(min(64, args.proj_window or B), reps=3)
        log("projection split: %d workgroups, %.2f ms per pass" % (proj_tune["workgroups"], proj_tune["ms_per_pass"]))

    # launch shapes of the hopping kernel for the inner and the FP64 outer
    # precision (and FP32, which updates the late residuals of BF16 solves)
    # at this batch: from the cache if it was measured on this lattice, else
    # timed now (setup, outside the measured region)
    if args.tune == "auto":
        want = {(inner, B), (L.FP64, B), (L.FP32, B)}
        if args.tune_cache and os.path.exists(args.tune_cache):
            ctx.load_tuning(args.tune_cache)
        have = set(ctx._tuned)
        for prec, nb in sorted(want - have):
            r = ctx.autotune_hop(prec, nb, reps=5)
            log("autotune prec %d B %d: %s %s ms (default %s ms, %d shapes per class, %d rejected)"
                % (prec, nb, r["best"], r["best_ms"], r["default_ms"], r["candidates"], r["rejected"]))
        if args.tune_cache:
            ctx.save_tuning(args.tune_cache)
    shapes = {}
    for prec in sorted({inner, L.FP64, L.FP32}):
        name = "fp64" if prec == L.FP64 else ("fp32" if prec == L.FP32 else "bf16")
        for cls, cname in L.HOP_CLASSES.items():
            v_ = ctx.hop_config(prec, B, cls)
            v_["form"] = L.HOP_FORMS[v_["form"]]
            shapes[name + "_" + cname] = v_

    # a plain 1 GiB device copy (untimed) so that hardware-counter runs of this
    # command carry their own calibration of FETCH_SIZE / WRITE_SIZE
    cal_a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    cal_b = torch.empty_like(cal_a)
    cal_b.copy_(cal_a)
    torch.cuda.synchronize()
    del cal_a, cal_b
    nprobe = w.nprobe

    def run(prm, steps, first0=0, profile=False):
        recs = []
        # a fresh window: every projection the timed batches use is computed
        # inside the timed region (a last window that reaches past it is
        # computed in full, so a step count that is not a multiple of the
        # window counts extra projection work, never less)
        ctx.set_projection_window(args.proj_window)
        if profile:
            ctx.profile(True)
            ctx.profile_reset()
        torch.cuda.synchronize()
        t0 = time.time()
        for s in range(steps):
            first = (first0 + s * B) % nprobe
            recs += ctx.trace_batch(w.seed, 0, w.hp, first, B, prm, allow_not_converged=True)
        torch.cuda.synchronize()
        el = time.time() - t0
        if profile:
            ctx.profile(False)
        return el, recs

    run(prm, args.warmup)
    ctx.reset_estimate()
    el, recs = run(prm, args.steps, profile=not args.no_profile)
    ms_step = 1e3 * el / args.steps
    value = args.steps * B / el
    worst = max(r["true_resid"] for r in recs)
    iters = float(np.mean([r["iters"] for r in recs]))
    outer = float(np.mean([r["outer"] for r in recs]))
    est = ctx.estimate()
    log("running estimate over %d probes: mean z^H D^-1 z = %.6g%+.6gi (synthetic basis: deflated value not physical)"
        % (est["n"], est["mean_re"], est["mean_im"]))
    tm = ctx.timings()
    log("mixed: %.2f ms/step, %.2f RHS/s, worst residual %.2e, mean inner iters %.1f, outer %.1f"
        % (ms_step, value, worst, iters, outer))

    roof = None
    dslash = None
    proj = None
    if not args.no_profile:
        stats = {name: ctx.profile_get(name) for name in ctx.PROF_CLASSES}
        for name, s in stats.items():
            if s["count"]:
                log("  %-12s %6d launches  %9.2f ms  %8.1f GB/s" % (name, s["count"], s["ms"], s["bytes"] / s["ms"] / 1e6))
        dom = max(stats, key=lambda n: stats[n]["ms"])
        s = stats[dom]
        avg_ms = s["ms"] / s["count"]
        bpl = s["bytes"] / s["count"]
        achieved = bpl / avg_ms / 1e6
        traffic = load_traffic(dom, w.name)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": dom, "avg_launch_ms": round(avg_ms, 4), "alg_bytes_per_launch": bpl,
                "launches": s["count"]}
        hop = stats["hop_fp32" if inner == L.FP32 else "hop_bf16"]
        if hop["count"]:
            dslash = round(hop["bytes"] / hop["ms"] / 1e6, 1)
        pm = stats["proj_mfma"]
        if pm["count"]:
            # each pass multiplies every complex entry of W (k x N) with the window's probes:
            # 8 real flops per complex multiply-add
            wprobes = min(64, args.proj_window or B)
            fl = 8.0 * k * w.N * wprobes
            avg = pm["ms"] / pm["count"]
            proj = {"launches": pm["count"], "avg_launch_ms": round(avg, 3), "probes_per_pass": wprobes,
                    "alg_GBps": round(pm["bytes"] / pm["ms"] / 1e6, 1),
                    "hbm_frac": round(pm["bytes"] / pm["ms"] / 1e6 / HBM_PEAK_GBPS, 4),
                    "mfma_tflops": round(fl / avg / 1e9, 1),
                    "mfma_frac": round(fl / avg / 1e9 / BF16_MFMA_PEAK_TFLOPS, 4)}
            log("projection: %.2f ms per %d-probe pass, %.0f GB/s algorithmic (%.3f of HBM), %.0f TFLOP/s "
                "(%.3f of the BF16 MFMA peak)" % (avg, wprobes, proj["alg_GBps"], proj["hbm_frac"],
                                                  proj["mfma_tflops"], proj["mfma_frac"]))

    # the plain FP64 BiCGStab path on the same GPU, same probes
    fp64_value = None
    if args.fp64_steps > 0:
        prm64 = ctx.params(L.SOLVER_BICGSTAB_FP64, tol=w.tol, maxiter=5000)
        run(prm64, 1)
        el64, recs64 = run(prm64, args.fp64_steps)
        fp64_value = args.fp64_steps * B / el64
        log("fp64: %.2f ms/step, %.2f RHS/s" % (1e3 * el64 / args.fp64_steps, fp64_value))

    # the traces Tr(Gamma D^-1) of all 16 Dirac matrices from the same solves
    # and deflation space (spin-pair projections and quadratic forms)
    gam = None
    if args.gamma_steps > 0:
        td_g = ctx.gamma_set(dirac_basis(np))
        ctx.trace_gamma_batch(w.seed, 0, w.hp, 0, B, prm, allow_not_converged=True)   # warm-up
        ctx.profile(True)
        ctx.profile_reset()
        torch.cuda.synchronize()
        t0 = time.time()
        for s_ in range(args.gamma_steps):
            ctx.trace_gamma_batch(w.seed, 0, w.hp, (s_ * B) % nprobe, B, prm, allow_not_converged=True)
        torch.cuda.synchronize()
        elg = time.time() - t0
        ctx.profile(False)
        sp = ctx.profile_get("proj_sp")
        gam = {"value": round(args.gamma_steps * B / elg, 3), "unit": "probes/s (16 traces each)",
               "ms_per_step": round(1e3 * elg / args.gamma_steps, 1), "matrices": 16,
               "time_vs_one_trace": round((elg / args.gamma_steps) / (ms_step / 1e3), 3)}
        if sp["count"]:
            # 16 probes x 4 target spins per entry of W: 8 real flops per complex multiply-add
            spf = 8.0 * k * w.N * 64 / (sp["ms"] / sp["count"]) / 1e9
            gam["proj_sp"] = {"launches": sp["count"], "avg_launch_ms": round(sp["ms"] / sp["count"], 3),
                              "alg_GBps": round(sp["bytes"] / sp["ms"] / 1e6, 1),
                              "mfma_tflops": round(spf, 1), "mfma_frac": round(spf / BF16_MFMA_PEAK_TFLOPS, 4),
                              "share_of_step": round(sp["ms"] / (1e3 * elg), 3)}
        log("gamma traces: %.1f ms/step (%.3f of a plain trace step), %.2f probes/s for 16 matrices%s"
            % (gam["ms_per_step"], gam["time_vs_one_trace"], gam["value"],
               (", spin-pair projection %.2f ms/launch at %.0f GB/s" % (gam["proj_sp"]["avg_launch_ms"],
                                                                        gam["proj_sp"]["alg_GBps"]))
               if "proj_sp" in gam else ""))

    # the learned leg: FGMRES(restart) with the network as right preconditioner
    # inside FP64 defect correction, same probes and projection window
    learned = None
    if args.nn_steps > 0:
        ctx.workspace_trim()   # the BiCGStab legs' fields make room for the FGMRES bases
        ctx.nn_set_weights(nn_weights)
        ctx.nn_set_skip(1.0 / (4.0 + w.mass))
        prm_nn = ctx.params(L.SOLVER_DC_FGMRES_NN, tol=w.tol, restart=args.nn_restart, maxiter=20000)
        elw, _ = run(prm_nn, 1, first0=0)
        log("learned leg: warm-up batch %.1f s" % elw)
        eln, recn = run(prm_nn, args.nn_steps, first0=0, profile=not args.no_profile)
        conv = ctx.profile_get("conv") if not args.no_profile else None
        learned = {
            "value": round(args.nn_steps * B / eln, 4), "unit": "RHS solves/s",
            "ms_per_step": round(1e3 * eln / args.nn_steps, 1),
            "solver": "FGMRES(%d) in FP32, learned preconditioner (BF16 matrix cores), FP64 defect correction"
                      % args.nn_restart,
            "mean_iters": round(float(np.mean([r["iters"] for r in recn])), 2),
            "mean_outer_cycles": round(float(np.mean([r["outer"] for r in recn])), 2),
            "worst_true_residual": max(r["true_resid"] for r in recn),
            "fallbacks_to_bicgstab": int(sum(1 for r in recn if r["status"] == 4)),
            "network": nn_info,
        }
        if conv and conv["count"]:
            tf = conv["bytes"] / conv["ms"] / 1e9
            learned["conv"] = {"launches": conv["count"], "avg_launch_ms": round(conv["ms"] / conv["count"], 3),
                               "achieved_tflops": round(tf, 1), "peak_tflops": BF16_MFMA_PEAK_TFLOPS,
                               "mfma_frac": round(tf / BF16_MFMA_PEAK_TFLOPS, 4),
                               "share_of_step": round(conv["ms"] / (1e3 * eln), 3)}
        log("learned: %.1f ms/step, %.3f RHS/s, mean iters %.1f, worst residual %.2e%s"
            % (learned["ms_per_step"], learned["value"], learned["mean_iters"], learned["worst_true_residual"],
               (", conv %.1f TFLOP/s (%.3f of BF16 MFMA peak)" % (learned["conv"]["achieved_tflops"],
                                                                 learned["conv"]["mfma_frac"]))
               if "conv" in learned else ""))

    cpu = None
    if not args.no_cpu:
        t0 = time.time()
        cpu = cpu_baseline(U, w, k, w.hp)
        log("cpu baseline: %.4f RHS/s (%.1f s)" % (cpu["value"], time.time() - t0))
        cpu.pop("q", None)
        cpu.pop("status", None)
        cpu["host"] = host_info()
        cpu["small_configs"] = {nm: ent for nm, ent in small.items()}

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "RHS solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32" if inner == L.FP32 else "bf16-storage/f32") + "+f64-defect-correction",
        "data": "synthetic",
        "config": {
            "workload": w.name, "lattice": list(w.L), "N": w.N, "mass": w.mass, "link_eps": w.eps,
            "batch": B, "probes": "hierarchical probing (Z4 base x Hadamard)" if w.hp else "Z4",
            "deflation_k": k, "deflation_storage": "bf16 (synthetic basis, diagonal Galerkin inverse)",
            "projection_window": args.proj_window,
            "solver": "even/odd BiCGStab, %s inner, FP64 defect correction" % args.inner,
            "preconditioner": "none (the learned FGMRES leg is reported as mixed_learned)", "tol": w.tol,
            "hop_shapes": shapes,
            "workspace_bytes": ws_bytes, "projection_split": proj_tune,
            "mean_inner_iters": round(iters, 2), "mean_outer_cycles": round(outer, 2),
            "worst_true_residual": worst,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "small_configs": small,
        "gamma_traces": gam,
        "mixed_learned": learned,
        "mixed_learned_value": learned["value"] if learned else None,
        "fp64_bicgstab_value": round(fp64_value, 3) if fp64_value else None,
        "speedup_vs_fp64": round(value / fp64_value, 3) if fp64_value else None,
        "dslash_GBps": dslash,
        "projection": proj,
        "phase_ms_last_step": {kk: round(v, 3) for kk, v in tm.items()},
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
