"""Benchmark: Rademacher probe solves/s at 1e-8 residual on 16^3x32, with dslash HBM GB/s.

One step = one deflated Hutchinson estimate through the C-ABI (lqt_trace): 128 real
Rademacher probes generated on the device, the deflation projections U^+ z and U^+ g5 z
against a k = 64 basis of A g5 eigenvectors (FP64 MFMA), batched restarted s-step GMRES(15)
(basis of hopping-term powers, one Gram pass and an FP64 Cholesky per cycle) with FP16 links
and Krylov vectors, FP32 accumulation, residuals carried between cycles and FP64 defect
correction until the FP64 true residual is <= 1e-8, the probe samples and the estimate.
Gauge field, mass, basis and dslash tiling are set up before the timed region (the
basis build is reported separately).  Inputs are synthetic (seeded random SU(3) links).

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MG_METRIC = "Rademacher probe solves/s at 1e-8 residual (32^3x64, multigrid deflation k=256)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="wilson16x32_mixed")
    ap.add_argument("--nprobes", type=int, default=None, help="override the probe count (profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GMRES comparison")
    ap.add_argument("--dslash-sweep", action="store_true",
                    help="only time the Wilson operator at its tuned tile for every storage precision and "
                         "n in {1, 8, 16, 32, 64} right-hand sides on 16^3x32 and 32^3x64, beside a device copy, "
                         "one JSON line per case, and exit")
    ap.add_argument("--train-pairs", type=int, default=None,
                    help="transport-net workload: training pairs (default: the workload's)")
    ap.add_argument("--train-epochs", type=int, default=None,
                    help="transport-net workload: training epochs (default: the workload's)")
    ap.add_argument("--pair-xi", type=float, default=None,
                    help="transport-net workload: errors of the training pairs from FP32 solves of Gaussian fields "
                         "to this tolerance (0: the Gaussian fields themselves; default: the workload's)")
    ap.add_argument("--dslash-tile", default=None, metavar="R,BLOCK,CHUNK,KIND",
                    help="use this operator tile for the inner storage instead of the autotuner's choice "
                         "(for counter runs of a given tile)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB 5 times (HBM counter calibration) and exit")
    ap.add_argument("--inner-prec", choices=["f32", "f16", "bf16"], default=None,
                    help="override the workload's inner storage precision")
    ap.add_argument("--no-orth-bound", action="store_true",
                    help="multigrid workload: skip the orthogonal-projector variance (the lower bound of Section 2.1)")
    ap.add_argument("--mass", type=float, default=None, help="override the workload's bare mass (conditioning scans)")
    ap.add_argument("--basis-iters", type=int, default=400,
                    help="cap on the filtered iterations of the A g5 eigensolver before the timed region (it stops "
                         "once all k pairs meet the Table 1 test; about 65 at m = -1.90 and 270 at m = -1.95 on 16^3x32)")
    return ap.parse_args()


def cpu_baseline(U, dims, mass, iters_per_probe, budget_s=15.0):
    """Oracle FP64 GMRES(32) timed on the host for a bounded number of iterations of one probe
    solve, scaled to probe solves/s with the iteration count the identical FP64 algorithm
    needs per probe (measured on the device)."""
    import numpy as np

    from oracle import core

    N = 12 * int(np.prod(dims))
    z = core.probes(1001, 1, N)[0].astype(np.complex128)
    core.gmres(U, dims, mass, z, 1e-8, m=32, maxit=2)  # warm the library
    its = 32
    t0 = time.perf_counter()
    core.gmres(U, dims, mass, z, 1e-8, m=32, maxit=its)
    dt = time.perf_counter() - t0
    if dt < budget_s / 3:  # whole restart cycles filling about budget_s
        its = 32 * max(1, int(budget_s / dt))
        t0 = time.perf_counter()
        core.gmres(U, dims, mass, z, 1e-8, m=32, maxit=its)
        dt = time.perf_counter() - t0
    per_iter = dt / its
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    # the oracle's FP64 operator on one right-hand side, by the operator's algorithmic bytes
    V = int(np.prod(dims))
    napp = 10
    t0 = time.perf_counter()
    for _ in range(napp):
        core.apply(U, dims, mass, core.OP_A, z)
    dt_op = (time.perf_counter() - t0) / napp
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": 1.0 / (per_iter * iters_per_probe),
        "unit": "probe solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{its} Arnoldi steps of FP64 GMRES(32) on one probe ({dt:.1f} s, {per_iter*1e3:.1f} ms/step), "
                  f"scaled by the {iters_per_probe:.0f} steps per probe the same algorithm takes on the device",
        "dslash_fp64_ms": round(dt_op * 1e3, 2),
        "dslash_fp64_gbps": round(V * (72 * 8 + 48 * 8) / dt_op / 1e9, 2),
        "cpu_model": model,
    }


VALU_PEAK_TFLOPS = 78.6  # FP32/FP64 FMA on the vector ALUs: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz
MFMA_F32_PEAK_TFLOPS = 157.3  # dense FP32 matrix-core peak of the MI355X
# useful flops of one transport-net application per site and field: channel mixing
# 9 paths x (4*8 + 8*8 + 8*8 + 8*4) complex products x 3 colours, transports 8 paths x
# (4 + 8 + 8 + 8) input features x 9 complex products, 8 flops per complex product
NET_FLOPS_PER_SITE_FIELD = 8 * (9 * (32 + 64 + 64 + 32) * 3 + 8 * 28 * 9)


def dslash_flops(byt, calls, sites, b):
    """Flops of the timed dslash launches from their algorithmic bytes: each launch moves
    sites*(72 b + 48 b n) bytes for n right-hand sides and does 1392 flops per site and
    right-hand side (1320 hopping term, 72 for the mass term and the 1/2)."""
    site_rhs = (byt - 72.0 * b * sites * calls) / (48.0 * b)
    return 1392.0 * site_rhs


def _measured_traffic(family, tile=None, workload=None):
    """HBM bytes per launch of a kernel family from the recorded counter runs (one record per
    measured workload and tile), or None when the kernel's source has changed since they were
    taken (hash mismatch), the workload or the tuned tile is none of those measured, or none
    exist."""
    import hashlib

    try:
        with open(os.path.join(ROOT, "paper_1909_12234_amd", "traffic.json")) as f:
            recs = json.load(f)["kernels"].get(family)
        if recs is None:
            return None
        if isinstance(recs, dict):
            recs = [recs]
        for rec in recs:
            if rec.get("workload") != workload:
                continue
            if tile is not None and "tile" in rec and list(rec["tile"]) != list(tile):
                continue
            with open(os.path.join(ROOT, "paper_1909_12234_amd", rec["source"]), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest()[:16] != rec["sha256_16"]:
                    return None
            return rec["fetch_bytes"] + rec["write_bytes"]
        return None
    except (OSError, KeyError, ValueError):
        return None


def _roofline(kt, sites=None, b=None, tile=None, workload=None):
    """Dominant kernel family by device time among those with algorithmic bytes.  The
    reduced-precision Wilson operator with FP32 arithmetic on the vector ALUs (tile kind 0) is
    reported against their FMA peak; the packed-FP16 and matrix-core operators (kinds 2, 3, 1)
    and the other families against HBM; the transport net against the FP32 matrix peak."""
    kind = tile[3] if tile else 0
    fam = max((f for f in kt if kt[f][2] > 0), key=lambda f: kt[f][0])
    ms, calls, byt = kt[fam]
    base = {"kernel": fam, "traffic": _measured_traffic(fam, tile if fam == "dslash" else None, workload),
            "launches": calls,
            "avg_launch_us": round(ms * 1e3 / max(calls, 1), 2)}
    if fam == "dslash" and sites and b and b < 8 and kind == 0:
        tf = dslash_flops(byt, calls, sites, b) / (ms * 1e-3) / 1e12
        base.update({"bound": "alu", "achieved": round(tf, 2), "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / VALU_PEAK_TFLOPS, 4),
                     "hbm_algorithmic_gbps": round(byt / (ms * 1e-3) / 1e9, 1)})
        return base
    if fam == "net" and sites and b:
        # the timer counts 12 (2b) bytes in and out per site and field, 4 FP32 activation
        # fields of 24 complex numbers and the FP32 links of each of the 4 layers
        site_fields = (byt - 4.0 * 72 * 4 * sites * calls) / (48.0 * b + 768.0)
        tf = NET_FLOPS_PER_SITE_FIELD * site_fields / (ms * 1e-3) / 1e12
        base.update({"bound": "mfma", "achieved": round(tf, 2), "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tf / MFMA_F32_PEAK_TFLOPS, 4),
                     "hbm_algorithmic_gbps": round(byt / (ms * 1e-3) / 1e9, 1)})
        return base
    achieved = byt / (ms * 1e-3) / 1e9
    base.update({"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4)})
    return base


def _line(a, value, elapsed, dtype, config, extra, metric=None):
    out = {"metric": metric or "Rademacher probe solves/s at 1e-8 residual (16^3x32) + dslash HBM GB/s",
           "value": round(value, 3),
           "unit": "probe solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": round(elapsed / a.steps * 1e3, 2), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def run_batched(a, w):
    """Three lattices solved together: every kernel of a cycle is one launch over all of them
    and the cycles are replayed from HIP graphs.  One step = the probes of every lattice."""
    import numpy as np
    import torch

    import paper_1909_12234_amd as lq
    import synth

    torch.cuda.set_device(0)
    lats = [d for d, _ in w["lattices"]]
    links = [synth.su3_links(d, w["eps"], sd) for d, sd in w["lattices"]]
    ctx = lq.Context(lats, [w["mass"]] * len(lats))
    ctx.set_gauge(np.concatenate([u.ravel() for u in links]))
    per = (a.nprobes or w["nprobes"]) // len(lats)
    ctx.tune(lq.F32, per)
    ctx.tune(lq.F64, 1)
    opts = dict(prec=lq.F32, restart=16)

    def step(graph):
        return ctx.trace_lattices(per, w["probe_seed"], w["xi"], graph=graph, **opts)

    for _ in range(a.warmup):
        step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = [step(1) for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ok = sum(r[0]["nsolves"] - r[0]["nfailed"] for r in res) * len(lats)
    # per-kernel timing needs eager launches: one more step with the timers on
    ctx.kernel_times(mode=2)
    t1 = time.perf_counter()
    step(0)
    torch.cuda.synchronize()
    eager = time.perf_counter() - t1
    kt = ctx.kernel_times(mode=3)
    d_ms, _, d_b = kt["dslash"]
    _line(a, ok / elapsed, elapsed, "f32",
          {"workload": f"wilson_batched3: lattices {lats} solved together, eps={w['eps']}, m={w['mass']}, "
                       f"{per} probes per lattice, FP32 inner GMRES(16), xi={w['xi']}, graph-captured cycles",
           "lattices": lats, "probes": per * len(lats), "restart": 16},
          {"roofline": _roofline(kt), "roofline_from": "one eager step with per-kernel HIP events",
           "eager_step_ms": round(eager * 1e3, 2), "graph_speedup": round(eager / (elapsed / a.steps), 3),
           "dslash_hbm_gbps": round(d_b / (d_ms * 1e-3) / 1e9, 1) if d_ms > 0 else None,
           "traces": [r["trace_re"] for r in res[-1]], "jackknife_err": [r["jackknife_err"] for r in res[-1]],
           "iters_per_probe": res[-1][0]["iters_total"] / max(1, res[-1][0]["nsolves"])})


def run_net(a, w):
    """16^3x32 with the transport net as FGMRES right preconditioner (trained before the
    timed region), beside the plain path on the same probes."""
    import torch

    import paper_1909_12234_amd as lq
    import synth

    torch.cuda.set_device(0)
    U = synth.su3_links(w["dims"], w["eps"], w["seed"])
    ctx = lq.Context(w["dims"], w["mass"])
    ctx.set_gauge(U)
    nprobes = a.nprobes or w["nprobes"]
    ctx.tune(lq.BF16, nprobes)
    ctx.tune(lq.F64, 1)
    t_train = time.perf_counter()
    npairs = a.train_pairs or w.get("train_pairs", 256)
    epochs = a.train_epochs or w.get("train_epochs", 4)
    pair_xi = a.pair_xi if a.pair_xi is not None else w.get("pair_xi", 0.0)
    loss = ctx.precond_train(npairs, seed=5, epochs=epochs, lr=3e-3, batch=8, pair_xi=pair_xi, verbose=1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    res = {}
    for net in (1, 0):
        def step():
            return ctx.trace(nprobes, w["probe_seed"], w["xi"], prec=lq.BF16, use_net=net, restart=w.get("restart", 32))
        for _ in range(a.warmup):
            step()
        torch.cuda.synchronize()
        ctx.kernel_times(mode=2)
        t0 = time.perf_counter()
        rr = [step() for _ in range(a.steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[net] = (rr, el, ctx.kernel_times(mode=3))
    rr, el, kt = res[1]
    ok = sum(r["nsolves"] - r["nfailed"] for r in rr)
    rp, elp, _ = res[0]
    okp = sum(r["nsolves"] - r["nfailed"] for r in rp)
    _line(a, ok / el, el, "bf16",
          {"workload": f"wilson16x32_net: 16^3x32, eps={w['eps']}, m={w['mass']}, {nprobes} probes, transport-net "
                       f"FGMRES({w.get('restart', 32)}), BF16 inner, xi={w['xi']}",
           "lattice": list(w["dims"]), "probes": nprobes, "restart": w.get("restart", 32)},
          {"roofline": _roofline(kt, 16 * 16 * 16 * 32, 2), "net_ms": round(kt["net"][0], 2),
           "iters_per_probe_net": rr[-1]["iters_total"] / rr[-1]["nsolves"],
           "iters_per_probe_plain": rp[-1]["iters_total"] / rp[-1]["nsolves"],
           "plain_same_probes_solves_per_s": round(okp / elp, 3), "train_s": round(t_train, 2),
           "train_pairs": npairs, "train_epochs": epochs, "train_pair_xi": pair_xi, "train_loss": loss,
           **({} if a.no_fp64 else fp64_plain(ctx, w, ok / el, w.get("restart", 32)))})


def fp64_plain(ctx, w, value, restart):
    """Plain FP64 GPU GMRES legs: one right-hand side at a time on a sample of 4 of the
    workload's probes, with the timed path's restart length, 8 and 32, and 32 probes batched in
    one lock-step GMRES(8) solve.  `speedup_vs_fp64_plain` divides by the fastest of all of
    them; `speedup_vs_fp64_single_rhs` by the fastest one-at-a-time leg."""
    import numpy as np
    import torch

    import paper_1909_12234_amd as lq

    out = {}
    zs = ctx.probes(w["probe_seed"], 4)
    restarts = sorted({restart, 8, 32})
    for m in restarts:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its = []
        for j in range(zs.shape[0]):
            _, st, _ = ctx.solve(zs[j:j + 1], w["xi"], prec=lq.F64, restart=m)
            its.append(st[0][1])
        torch.cuda.synchronize()
        rate = zs.shape[0] / (time.perf_counter() - t1)
        out[f"fp64_plain_gmres{m}_solves_per_s"] = round(rate, 3)
        out[f"fp64_plain_gmres{m}_iters_per_probe"] = float(np.mean(its))
    single_rate = max(out[f"fp64_plain_gmres{m}_solves_per_s"] for m in restarts)
    out["fp64_plain_iters_per_probe"] = out["fp64_plain_gmres32_iters_per_probe"]
    # FP64 batched: 32 of the workload's probes in one lock-step GMRES(8) solve (FP64 operator
    # and Krylov vectors), which separates the gain of batching from that of reduced storage
    zb = ctx.probes(w["probe_seed"], 32)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st, _ = ctx.solve(zb, w["xi"], prec=lq.F64, restart=8)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    out["fp64_batched32_gmres8_solves_per_s"] = round(sum(1 for s in st if s[0]) / dt, 3)
    out["fp64_batched32_gmres8_iters_per_probe"] = float(np.mean([s[1] for s in st]))
    best = max(single_rate, out["fp64_batched32_gmres8_solves_per_s"])
    out["fp64_plain_best_solves_per_s"] = best
    out["speedup_vs_fp64_plain"] = round(value / best, 2)
    out["speedup_vs_fp64_single_rhs"] = round(value / single_rate, 2)
    return out


def run_mg(a, w):
    """Algorithm 2 at 32^3x64.  Untimed setup: near-null vectors, the prolongator W, the
    explicit coarse operator and the k coarse eigenvectors (their kernel times reported
    apart).  Timed step: the trace over the workload's probes, oblique g5 projector on
    X = W U_c, probes solved in batches of the workload's size."""
    import numpy as np
    import torch

    import paper_1909_12234_amd as lq
    import synth
    from paper_1909_12234_amd.workloads import PREC

    if a.mass is not None:
        w = dict(w, mass=a.mass)
    dims, mass, eps = w["dims"], w["mass"], w["eps"]
    nprobes = a.nprobes or w["nprobes"]
    prec = PREC[a.inner_prec or w["inner_prec"]]
    V = int(np.prod(dims))
    torch.cuda.set_device(0)
    t_setup = time.perf_counter()
    U = synth.su3_links(dims, eps, w["seed"])
    ctx = lq.Context(dims, mass)
    ctx.set_gauge(U)
    del U
    _, tile = ctx.tune(prec, w["batch"], return_tile=True)
    ctx.tune(prec, w["nv"])
    ctx.tune(0, 1)
    solver = dict(prec=prec, restart=w["restart"], sstep=w["sstep"])
    ctx.kernel_times(mode=2)
    t_basis = time.perf_counter()
    if "block2" in w:
        basis = ctx.basis_prolongator2(w["block"], w["nv"], w["block2"], w["nv2"], w["k"], null_xi=1e-2,
                                       null_maxit=200, verbose=1, outer_maxit=a.basis_iters, **solver)
    else:
        basis = ctx.basis_prolongator(w["block"], w["nv"], w["k"], null_xi=1e-2, null_maxit=200, verbose=1,
                                      outer_maxit=a.basis_iters, **solver)
    torch.cuda.synchronize()
    t_basis = time.perf_counter() - t_basis
    kt_setup = ctx.kernel_times(mode=3)
    lam = basis.eigenvalues().numpy().real
    t_setup = time.perf_counter() - t_setup

    def step():
        return ctx.trace(nprobes, w["probe_seed"], w["xi"], basis=basis, rank_curve=True, max_batch=w["batch"],
                         **solver)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times(mode=2)
    t0 = time.perf_counter()
    results = [step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = ctx.kernel_times(mode=3)
    ok = sum(r["nsolves"] - r["nfailed"] for r in results)
    # the orthogonal projector onto the same span W U_c on the same probes: the rough lower
    # bound of Section 2.1 for the variance of any projector of this rank (untimed; its t0
    # takes k more solves)
    r_orth = None
    if not a.no_orth_bound:
        t_orth = time.perf_counter()
        r_orth = ctx.trace(nprobes, w["probe_seed"], w["xi"], basis=basis, projector=lq.ORTH, max_batch=w["batch"],
                           **solver)
        torch.cuda.synchronize()
        t_orth = time.perf_counter() - t_orth
    bpr = {0: 8, 1: 4, 2: 2, 3: 2}[prec]
    pr_ms, pr_calls, pr_b = kt["prolongator"]
    pr_gbs = pr_b / (pr_ms * 1e-3) / 1e9 if pr_ms > 0 else None
    spr_ms, spr_calls, spr_b = kt_setup["prolongator"]
    last = results[-1]
    curve = last["rank_curve"].numpy()
    smax = ctx.sigma_max()
    extra = {
        "dtype_detail": f"{w['inner_prec']} links and Krylov vectors, fp32 accumulate, fp64 defect correction; "
                        "fp64 prolongator, coarse operator and projections",
        "roofline": _roofline(kt, V, bpr, tile=tile, workload=a.workload),
        "kernel_ms": {f: round(kt[f][0], 2) for f in kt},
        "iters_per_probe_mixed": round(sum(r["iters_total"] for r in results) / max(1, sum(r["nsolves"] for r in results)), 1),
        # restriction of the probes (W streamed once per 32 probes), algorithmic bytes / time
        "pr_hbm_gbps": round(pr_gbs, 1) if pr_gbs else None,
        "pr_frac_of_peak": round(pr_gbs / HBM_PEAK_GBS, 4) if pr_gbs else None,
        "pr_launches": pr_calls,
        # setup: restriction / prolongation / explicit coarse operator applications of the coarse eigensolve
        "setup_pr_ms": round(spr_ms, 1),
        "setup_pr_hbm_gbps": round(spr_b / (spr_ms * 1e-3) / 1e9, 1) if spr_ms > 0 else None,
        "setup_kernel_ms": {f: round(kt_setup[f][0], 1) for f in kt_setup},
        "estimate": {"trace": last["trace_re"], "var_sample": last["var_sample"],
                     "jackknife_err": last["jackknife_err"], "nfailed": last["nfailed"]},
        "estimate_undeflated": {"trace": float(curve[0, 0]), "var_sample": float(curve[0, 1]),
                                "jackknife_err": float(curve[0, 2])},
        "variance_ratio_undeflated_over_deflated": round(float(curve[0, 1]) / last["var_sample"], 4),
        "rank_min_var": {"rank": int(np.argmin(curve[:, 1])), "var_sample": float(np.min(curve[:, 1]))},
        "estimate_orthogonal_projector": ({"trace": r_orth["trace_re"], "var_sample": r_orth["var_sample"],
                                           "jackknife_err": r_orth["jackknife_err"], "nfailed": r_orth["nfailed"],
                                           "seconds": round(t_orth, 1)} if r_orth else None),
        "setup_s": round(t_setup, 2),
        "basis_s": round(t_basis, 2),
        "basis_min_abs_lambda": float(np.min(np.abs(lam))),
        "basis_max_abs_lambda": float(np.max(np.abs(lam))),
        "basis_iters": a.basis_iters,
        "basis_all_pairs_converged": bool(basis.converged),
        "sigma_max": round(smax, 4),
        "sigma_min_coarse": float(np.min(np.abs(lam))),
        "cpu_baseline": None,
        "cpu_baseline_note": "the oracle is timed on the 16^3x32 workload's line only",
    }
    lvl2 = (f", second level {w['block2'][0]}^4 blocks of the coarse lattice with nv2={w['nv2']}"
            if "block2" in w else "")
    config = {"workload": f"{a.workload}: Wilson-Dirac {dims[0]}^3x{dims[3]}, eps={eps}, m={mass}, {nprobes} "
                          f"Rademacher probes, xi={w['xi']}, oblique g5 deflation on X = W U_c: {w['block'][0]}^4 "
                          f"aggregates, nv={w['nv']} per chirality{lvl2}, k={w['k']} coarse eigenvectors, s-step "
                          f"GMRES({w['restart']}) in batches of {w['batch']}",
              "lattice": list(dims), "probes": nprobes, "block": list(w["block"]), "nv": w["nv"],
              "deflation_rank": w["k"], "batch": w["batch"], "levels": 2 if "block2" in w else 1}
    _line(a, ok / elapsed, elapsed, w["inner_prec"], config, extra, metric=MG_METRIC)


def run_dslash_sweep(a):
    """The Wilson operator alone: for each lattice, storage precision and number of right-hand
    sides, the autotuner's tile, then 5 launches timed by the library's HIP events; algorithmic
    bytes V (72 b + 48 b n) per launch against 8 TB/s and against a plain device copy (4 GiB
    read + 4 GiB written, timed with events on the current stream)."""
    import torch

    import paper_1909_12234_amd as lq
    import synth

    torch.cuda.set_device(0)
    nb = 1 << 30
    src = torch.ones(nb, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * 4 * nb / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    print(json.dumps({"copy_gbps": round(copy_gbs, 1), "copy_bytes": 8 * nb}), flush=True)
    names = {lq.F64: "f64", lq.F32: "f32", lq.F16: "f16", lq.BF16: "bf16"}
    for dims in [(16, 16, 16, 32), (32, 32, 32, 64)]:
        U = synth.su3_links(dims, 0.5, 1)
        ctx = lq.Context(dims, -1.9)
        ctx.set_gauge(U)
        del U
        N = ctx.N
        for prec in (lq.F64, lq.F32, lq.F16, lq.BF16):
            for n in (1, 8, 16, 32, 64):
                dt = torch.complex128 if prec == lq.F64 else torch.complex64
                x = torch.randn((n, N), dtype=dt, device="cuda")
                ms_tune, tile = ctx.tune(prec, n, return_tile=True)
                ctx.apply(x, prec=prec)
                torch.cuda.synchronize()
                ctx.kernel_times(mode=2)
                for _ in range(5):
                    y = ctx.apply(x, prec=prec)
                torch.cuda.synchronize()
                ms, calls, byt = ctx.kernel_times(mode=3)["dslash"]
                gbs = byt / (ms * 1e-3) / 1e9
                print(json.dumps({"lattice": list(dims), "prec": names[prec], "nrhs": n, "tile": list(tile),
                                  "us_per_launch": round(ms * 1e3 / calls, 2), "alg_bytes": round(byt / calls),
                                  "gbps": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                                  "frac_copy": round(gbs / copy_gbs, 4), "tuner_us": round(ms_tune * 1e3, 2)}),
                      flush=True)
                del x, y
        ctx.close()
        torch.cuda.empty_cache()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the probes are independent "
              "solves, so several GPUs would each take a share of them", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if a.dslash_sweep:
        return run_dslash_sweep(a)
    if a.calibrate_copy:
        n = a.calibrate_copy * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}), flush=True)
        return

    import paper_1909_12234_amd as lq
    import synth
    from paper_1909_12234_amd.workloads import PREC, WORKLOADS

    w = WORKLOADS[a.workload]
    if "block" in w:
        return run_mg(a, w)
    if "lattices" in w:
        return run_batched(a, w)
    if a.workload == "wilson16x32_net":
        return run_net(a, w)
    if a.mass is not None:
        w = dict(w, mass=a.mass)
    dims, mass, eps = w["dims"], w["mass"], w["eps"]
    nprobes = a.nprobes or w["nprobes"]
    if a.inner_prec:
        w = dict(w, inner_prec=a.inner_prec)
    prec = PREC[w["inner_prec"]]
    V = int(np.prod(dims))
    torch.cuda.set_device(0)

    t_setup = time.perf_counter()
    U = synth.su3_links(dims, eps, w["seed"])
    ctx = lq.Context(dims, mass)
    ctx.set_gauge(U)
    _, tile = ctx.tune(prec, nprobes, return_tile=True)
    if a.dslash_tile:
        tile = tuple(int(v) for v in a.dslash_tile.split(","))
        ctx.set_tile(prec, nprobes, tile)
    ctx.tune(0, 1)
    t_basis = time.perf_counter()
    basis = (ctx.basis_eig(w["k"], xi=1e-2, verbose=1, outer_maxit=a.basis_iters) if w.get("k") else None)
    torch.cuda.synchronize()
    t_basis = time.perf_counter() - t_basis
    lam = basis.eigenvalues().numpy().real if basis is not None else np.array([1.0])
    t_setup = time.perf_counter() - t_setup

    def step():
        return ctx.trace(nprobes, w["probe_seed"], w["xi"], basis=basis, prec=prec, restart=w.get("restart", 32),
                         sstep=w.get("sstep", 0), rank_curve=basis is not None)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times(mode=2)  # zero and start the kernel timers
    t0 = time.perf_counter()
    results = []
    for _ in range(a.steps):
        results.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kt = ctx.kernel_times(mode=3)
    ok = sum(r["nsolves"] - r["nfailed"] for r in results)
    value = ok / elapsed
    iters_mixed = sum(r["iters_total"] for r in results) / max(1, sum(r["nsolves"] for r in results))

    # roofline of the dominant kernel family (by device time), from live HIP events
    bpr = {0: 8, 1: 4, 2: 2, 3: 2}[prec]  # bytes per real of the inner storage
    roof = _roofline(kt, V, bpr, tile=tile, workload=a.workload)
    d_ms, d_calls, d_b = kt["dslash"]
    dslash_gbs = d_b / (d_ms * 1e-3) / 1e9 if d_ms > 0 else None

    out = {
        "metric": "Rademacher probe solves/s at 1e-8 residual (16^3x32) + dslash HBM GB/s",
        "value": round(value, 3),
        "unit": "probe solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w["inner_prec"],
        "dtype_detail": f"{w['inner_prec']} links and Krylov vectors, fp32 accumulate, fp64 defect correction"
                        + (" (operator half spinors in packed fp16)" if tile[3] in (2, 3) else ""),
        "data": "synthetic",
        "config": {"workload": f"{a.workload}: Wilson-Dirac {dims[0]}^3x{dims[3]}, eps={eps}, m={mass}, "
                               f"{nprobes} Rademacher probes, xi={w['xi']}, oblique g5 deflation k={w.get('k', 0)}, "
                               f"{'s-step ' if w.get('sstep') else ''}GMRES({w.get('restart', 32)})",
                   "lattice": list(dims), "probes": nprobes, "restart": w.get("restart", 32), "sstep": w.get("sstep", 0),
                   "deflation_rank": w.get("k", 0)},
        "dslash_hbm_gbps": round(dslash_gbs, 1) if dslash_gbs else None,
        "dslash_frac_of_peak": round(dslash_gbs / HBM_PEAK_GBS, 4) if dslash_gbs else None,
        "roofline": roof,
        "dslash_tile": {"per_thread_or_lane": tile[0], "block": tile[1], "chunk": tile[2],
                        "kernel": {0: "vector ALUs, fp32", 1: "matrix cores", 2: "vector ALUs, packed fp16",
                                   3: "vector ALUs, packed fp16, links staged in LDS for 8 groups"}[tile[3]]},
        "kernel_ms": {f: round(kt[f][0], 2) for f in kt},
        "iters_per_probe_mixed": round(iters_mixed, 1),
        "estimate": {"trace": results[-1]["trace_re"], "var_sample": results[-1]["var_sample"],
                     "jackknife_err": results[-1]["jackknife_err"], "nfailed": results[-1]["nfailed"]},
        # the same probes' samples without the deflation correction (rank 0 of the rank curve)
        "estimate_undeflated": ({"trace": float(results[-1]["rank_curve"][0, 0]),
                                 "var_sample": float(results[-1]["rank_curve"][0, 1]),
                                 "jackknife_err": float(results[-1]["rank_curve"][0, 2])}
                                if basis is not None else None),
        # a-posteriori rank (Section 2.2): the prefix of the basis with the smallest sample variance
        "rank_min_var": ({"rank": int(np.argmin(results[-1]["rank_curve"][:, 1].numpy())),
                          "var_sample": float(np.min(results[-1]["rank_curve"][:, 1].numpy()))}
                         if basis is not None else None),
        "setup_s": round(t_setup, 2),
        "basis_s": round(t_basis, 2),
        "basis_min_abs_lambda": float(np.min(np.abs(lam))),
        "basis_iters": a.basis_iters,
        "basis_all_pairs_converged": bool(getattr(basis, "converged", True)) if basis is not None else None,
    }
    # conditioning of the timed operator: sigma_min = min |lambda(A g5)| from the basis (the
    # smallest eigenvalue in modulus when the basis converged), sigma_max by the library's
    # power iteration on A g5
    smax = ctx.sigma_max()
    out["sigma_max"] = round(smax, 4)
    if basis is not None:
        out["sigma_min"] = float(np.min(np.abs(lam)))
        out["kappa"] = round(smax / out["sigma_min"], 1)

    if not a.no_fp64:
        out.update(fp64_plain(ctx, w, value, w.get("restart", 32)))
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(U, dims, mass, out.get("fp64_plain_iters_per_probe", 604.0))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
