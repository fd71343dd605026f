"""Throughput of the CCWSIM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step is one ccwsim_simulate call: every patch of every realization of
the workload goes through data-event extraction, the CCW scan over all
candidates, top-K + draw, inverse DWT, boundary cut and paste.  The default
workload is the largest one-GPU configuration: 16 realizations of a 2000^2
grid from a 1000^2 three-facies TI (T 48, OV 12, J 2, K 10), plain form.
Inputs (TI, hard data) are resident in HBM before the timed region.  Prints
one JSON line.

The roofline object is measured live: after the timed region, the same K
steps run again with the library's event profiler on (the scan and finalize
launches carry start/stop events recorded by their own dispatch); the
dominant kernel's algorithmic work per launch divided by its average launch
time gives `achieved`.  Algorithmic work: the scan's contraction, 2 flops
per (overlap block, candidate, patch); the finalize's bytes, 6 T^d per patch
(the grid and pattern windows read, the coefficients read, the window
written).
The CPU baseline is the oracle, as it stands, on a bounded sample of the same
workload: one realization on one core, and the same realization in one
process per host core at once.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_FP16_TFLOPS = 2500.0      # MI355X dense fp16 MFMA
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E

METRIC = "simulated cells/s + CCF candidates/s (fraction of MFMA/HBM peak), plain vs learned"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5_learned")
    ap.add_argument("--n-real", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched and precision-split side measurements")
    ap.add_argument("--no-next", action="store_true",
                    help="skip dense conditioning, the level x grid-size sweep and the ensemble statistics")
    ap.add_argument("--traffic-json", default=os.path.join(HERE, "profiles", "traffic.json"),
                    help="HBM bytes per launch measured with rocprofv3 counters (optional)")
    ap.add_argument("--cdf97-only", action="store_true",
                    help="print only the CDF 9/7 measurements (transform, exact and split selection)")
    ap.add_argument("--lp-lists", type=int, default=None, help="inverted lists of the learned proposer's index")
    ap.add_argument("--lp-eval-seeds", type=int, default=None, help="evaluation seeds 1..N of the learned sweep")
    ap.add_argument("--lp-kmeans-iters", type=int, default=None, help="k-means rounds of the learned index")
    ap.add_argument("--lp-points", default=None,
                    help="(lists probed[:gate]) points of the learned sweep, comma-separated, e.g. 8,12,8:0.2")
    ap.add_argument("--lp-epochs", type=int, default=None,
                    help="training epochs of the learned proposer (default: the built-in schedule)")
    ap.add_argument("--learned-only", action="store_true",
                    help="only the learned proposer's measurement (training, offline metrics, gate sweep)")
    ap.add_argument("--oracle-worker", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--oracle-procs", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB five times (counter calibration)")
    return ap.parse_args()


def calibrate_copy(mib):
    """A plain copy kernel of known size, for scaling the HBM byte counters."""
    import torch
    n = mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 5}), flush=True)


def kernel_source_hash():
    """Hash of the HIP sources: counter readings taken on other sources are stale."""
    import hashlib
    d = os.path.join(HERE, "paper_2404_00441_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(d, name), "rb").read())
    return h.hexdigest()[:16]


ORACLE_KEYS = ("ti", "grid", "tmpl", "overlap", "level", "top_k", "n_real", "n_facies", "seed", "path_mode",
               "score_mode", "nc_margin", "cut")


def _oracle_sample(workload, scale, n_real):
    """Realization 0 of the workload through the oracle (one thread); returns
    (seconds, cells).  Runs in a process that never touches the GPU."""
    from oracle import oracle as orc
    from paper_2404_00441_amd import workloads as wl
    p, ti, hd = wl.make(workload, scale=scale, n_real=n_real)
    q = dict(p, n_real=1)
    if hd is not None:
        sel = hd[0] == 0
        hd = (hd[0][sel], hd[1][sel], hd[2][sel])
    sp = orc.SimParams(**{k: q[k] for k in ORACLE_KEYS}, wavelet=q.get("wavelet", 0))
    t0 = time.perf_counter()
    orc.simulate(sp, ti, hd)
    cells = 1
    for n in p["grid"]:
        cells *= n
    return time.perf_counter() - t0, cells


def _host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_worker_main(workload, n_proc):
    """Child process of cpu_baseline: the oracle on realization 0, first alone
    (one core), then in n_proc processes at once (one per core)."""
    import multiprocessing as mp
    from oracle import oracle as orc
    orc.build_oracle(force=False)
    t1, cells = _oracle_sample(workload, 1.0, None)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(n_proc) as pool:
        res = pool.starmap(_oracle_sample, [(workload, 1.0, None)] * n_proc)
    tw = time.perf_counter() - t0
    print(json.dumps({"t_single": t1, "cells": cells, "t_all": tw, "n_proc": n_proc,
                      "t_each": [r[0] for r in res]}), flush=True)


def cpu_baseline(workload, n_real):
    """The oracle on realization 0 of the workload: one core, then one process
    per host core (each simulating the same realization), in a child process
    that never initialises the GPU.  cells/s counts the realization's cells
    per process."""
    import subprocess
    n_proc = _host_cores()
    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-worker", workload, "--oracle-procs", str(n_proc)]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=HERE)
    if r.returncode != 0:
        raise RuntimeError(f"oracle worker failed: {r.stderr[-2000:]}")
    d = json.loads(r.stdout.strip().splitlines()[-1])
    cells = d["cells"]
    single = cells / d["t_single"]
    allc = cells * d["n_proc"] / d["t_all"]
    return {"value": allc, "unit": "cells/s", "cores": d["n_proc"], "kind": "oracle",
            "sample": f"realization 0 of the workload ({cells} cells) in {d['n_proc']} processes at once, "
                      f"{d['t_all']:.1f} s wall; the workload has {n_real} realizations, each the same work",
            "single_core": {"value": single, "unit": "cells/s", "cores": 1,
                            "sample": f"realization 0 alone, {d['t_single']:.1f} s"},
            "host": {"cpu_model": _cpu_model(), "nproc": os.cpu_count(), "cores_used": d["n_proc"]}}


def _time_runs(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def measure_scan_kernel(cc, wl, dev, reps=20):
    """The scan kernel alone at the largest filter counts of the batched
    workloads: M = candidates, K = overlap blocks of an L-shaped overlap,
    N = filters in flight (realizations x wavefront concurrency).  Data events
    are synthetic block sums on that overlap.  Two forms: the selection fused
    into the scan (each filter's 10 best keys, no score map; the energy term
    in the contraction), and the whole score map in every layout.  Timing
    comes from events recorded by the scan launch itself."""
    import numpy as np
    import torch
    out = []
    for name, n_filters in (("c4_batched", 384), ("c5_learned", 448)):
        p, ti, _ = wl.make(name, n_real=1)
        level, T, OV = p["level"], p["tmpl"], p["overlap"]
        b = 2 ** level
        tc = [-(-t // b) for t in T]
        ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
        approx, _ = cc.dwt(ti_d, level)
        # block counts of the L-shaped overlap (bands on both axes)
        u = np.zeros((T[1], T[0]), bool)
        u[:OV[1], :] = True
        u[:, :OV[0]] = True
        pad = np.zeros((tc[1] * b, tc[0] * b), int)
        pad[:T[1], :T[0]] = u
        n_beta = pad.reshape(tc[1], b, tc[0], b).sum(axis=(1, 3))
        rng = np.random.default_rng(7)
        or_n = np.broadcast_to(n_beta, (n_filters,) + n_beta.shape).astype(np.int32).copy()
        or_m = (rng.integers(0, p["n_facies"], size=or_n.shape) * or_n).astype(np.int32)
        or_n_d = torch.from_numpy(or_n).to(dev)
        or_m_d = torch.from_numpy(or_m).to(dev)
        real = torch.arange(n_filters, dtype=torch.int32, device=dev) % 16
        step = torch.arange(n_filters, dtype=torch.int64, device=dev)
        cand = [(p["ti"][a] - T[a]) // b + 1 for a in range(2)]
        ncand = cand[0] * cand[1]
        blocks = int((n_beta > 0).sum())
        flops = 2.0 * blocks * ncand * n_filters

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            cc.profile_enable(True)
            cc.profile_read()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            prof = cc.profile_read()
            cc.profile_enable(False)
            return 1e3 * prof["scan"][0] / max(prof["scan"][1], 1)

        us_fused = timed(lambda: cc.ccf_scan(p["ti"], level, p["n_facies"] - 1, approx, T, or_n_d, or_m_d, top_k=10,
                                             seed=1, realization=real, step=step))
        # every layout of the whole score map: candidate-major with 1, 2, 4, 8
        # tiles per workgroup, filter-major (-1); 0 is the library's default
        variants = {}
        for V in (0, 1, 2, 4, 8, -1):
            cc.set_scan_group(V)
            try:
                variants[V] = timed(lambda: cc.ccf_scan(p["ti"], level, p["n_facies"] - 1, approx, T, or_n_d, or_m_d))
            finally:
                cc.set_scan_group(0)
        best_v = min(variants, key=variants.get)
        us_map = variants[best_v]
        map_bytes = 8.0 * ncand * n_filters + 2.0 * approx.numel() + 512.0 * n_filters
        tf = flops / (us_fused * 1e-6) / 1e12
        out.append({"shape": f"{name}: M={ncand} candidates, K={blocks} overlap blocks (padded to "
                             f"{-(-blocks // 16) * 16}), N={n_filters} filters",
                    "flops_per_launch": flops,
                    "fused_top10": {"us_per_launch": us_fused, "tflops_algorithmic": tf,
                                    "frac_mfma_fp16": tf / PEAK_FP16_TFLOPS},
                    "score_map": {"us_per_launch": us_map, "tflops_algorithmic": flops / (us_map * 1e-6) / 1e12,
                                  "frac_mfma_fp16": flops / (us_map * 1e-6) / 1e12 / PEAK_FP16_TFLOPS,
                                  "gbs_algorithmic": map_bytes / (us_map * 1e-6) / 1e9,
                                  "layout": {0: "default", -1: "filter-major"}.get(best_v, f"{best_v} tiles per workgroup"),
                                  "us_per_layout": {str(k): round(v, 2) for k, v in variants.items()}}})
    return out


def measure_certified(cc, wl, dev, dims=(16,)):
    """C5 with the certified principal-component proposer against the plain
    scan: same realizations (checked), cells/s, and how many candidate rows
    were rescored exactly per patch before the K best were certified."""
    import numpy as np
    import torch
    p, ti, _ = wl.make("c5_learned")
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    cells = p["n_real"] * int(np.prod(p["grid"]))
    rows = (p["ti"][1] - p["tmpl"][1]) // 2 ** p["level"] + 1
    sim0 = cc.Simulator(p, device=dev)
    ref = sim0.run(ti_d)
    t_plain = _time_runs(lambda: sim0.run(ti_d), 2)
    res = {"workload": wl.describe(p), "ms_plain": t_plain * 1e3, "cells_per_s_plain": cells / t_plain,
           "candidate_rows": rows, "by_dim": []}
    del sim0
    for D in dims:
        simL = cc.Simulator(dict(p, proposer_dim=D), device=dev)
        got = simL.run(ti_d)
        torch.cuda.synchronize()
        rep = simL.report()
        same = bool(torch.equal(got, ref))
        t = _time_runs(lambda: simL.run(ti_d), 2)
        res["by_dim"].append({"proposer_dim": D, "ms": t * 1e3, "cells_per_s": cells / t, "speedup": t_plain / t,
                              "identical_to_plain": same,
                              "rows_rescored_per_patch": rep["proposer_rows"] / max(rep["proposer_patches"], 1)})
        del simL
    return res


LP_TRAIN_SEEDS = (1001, 1002, 1003, 1004)   # plain simulations whose data events train the proposer
LP_HELDOUT_SEED = 2001
LP_EPOCHS, LP_BATCH, LP_LR = 6, 512, 2e-3
LP_LISTS = 512
LP_KMEANS_ITERS = 10
# (lists probed, gate): None lets every proposal stand
LP_POINTS = ((4, None), (5, None), (6, None), (8, None), (12, None), (16, None), (8, 0.2), (8, 0.15))
LP_EVAL_SEEDS = (1, 2, 3, 4, 5, 6, 7, 8)     # each form simulated with each seed; errors pooled


def measure_learned(cc, wl, dev, reps=3, epochs=None, lists=None, points=None, eval_seeds=None, kmeans_iters=None):
    """C5 with the learned convolutional proposer against the plain form on
    the same GPU.  Training pairs: the data events of plain simulations of
    the C5 workload with other seeds and their exact-best candidates; a
    held-out simulation gives the offline metrics (cross-entropy, recall of
    the exact best among the proxy's top 256, exact-score regret of that
    shortlist's best).  Then the workload is simulated with seeds 1, 2 and
    3 (the bench's own and two more), plain and with the index of the
    trained keys for several (lists probed, gate) points: cells/s, the match error of the drawn
    candidates (mean, p95, pooled over the seeds) against the plain form's,
    and the fraction of patches the gate sent to the full scan.  The equal-error
    point is the fastest point whose mean match error is within 1 % of the
    plain form's."""
    import numpy as np
    import torch
    from paper_2404_00441_amd import learn
    p, ti, _ = wl.make("c5_learned")
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    cells = p["n_real"] * int(np.prod(p["grid"]))
    approx, _ = cc.dwt(ti_d, p["level"])
    t0 = time.perf_counter()
    on, om, lab, best, sb, nk = learn.training_pairs(p, ti_d, LP_TRAIN_SEEDS)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    von, vom, vlab, vbest, vsb, vnk = learn.training_pairs(dict(p, n_real=2), ti_d, [LP_HELDOUT_SEED])
    t0 = time.perf_counter()
    epochs = epochs or LP_EPOCHS
    w, hist = learn.train(p, approx, on, om, lab, epochs=epochs, batch=LP_BATCH, lr=LP_LR, seed=7)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ev = learn.evaluate(p, w, approx, von, vom, vlab, vbest, vsb, vnk)
    t0 = time.perf_counter()
    lists = lists or LP_LISTS
    eval_seeds = eval_seeds or LP_EVAL_SEEDS
    kmeans_iters = kmeans_iters or LP_KMEANS_ITERS
    index = cc.lp_build_index(w, approx, p["ti"], p["level"], p["tmpl"], lists, iters=kmeans_iters)
    torch.cuda.synchronize()
    t_index = time.perf_counter() - t0

    def run(q):
        # every evaluation seed: time per call and the drawn candidates'
        # match errors, pooled over the seeds
        ts, errs, fbs, acc, scored, n = [], [], 0, 0, 0, 0
        for sd in eval_seeds:
            sim = cc.Simulator(dict(q, seed=sd), device=dev)
            ts.append(_time_runs(lambda: sim.run(ti_d), reps))
            e = sim.match_errors()
            errs.append(e[e >= 0].double())
            rep = sim.report()
            fbs += rep["proposer_fallbacks"]
            acc += rep["proposer_patches"]
            scored += rep["proposer_rows"]
            n += sim.n_patches()
            del sim
        e = torch.cat(errs)
        return sum(ts) / len(ts), float(e.mean()), float(torch.quantile(e, 0.95)), fbs / max(n, 1), \
            scored / max(acc, 1)

    t_plain, e_plain, e95_plain, _, _ = run(p)
    res = {"workload": wl.describe(p), "training": {
        "pairs": int(on.shape[0]), "pair_seeds": list(LP_TRAIN_SEEDS), "pairs_s": t_pairs,
        "labels_per_pair": int(lab.shape[1]),
        "epochs": epochs, "batch": LP_BATCH, "lr": LP_LR, "train_s": t_train,
        "loss_per_epoch": hist, "index_lists": lists, "kmeans_iters": kmeans_iters, "index_s": t_index},
        "heldout": dict(ev, seed=LP_HELDOUT_SEED),
        "eval_seeds": list(eval_seeds),
        "plain": {"ms": t_plain * 1e3, "cells_per_s": cells / t_plain, "match_error_mean": e_plain,
                  "match_error_p95": e95_plain},
        "by_gate": []}
    for probe, gate in (points or LP_POINTS):
        q = dict(p, proposer_dim=64, proposer=index, lp_probe=probe, lp_gate=1e30 if gate is None else gate)
        t, em, e95, fbr, spp = run(q)
        res["by_gate"].append({
            "gate": gate, "probe": probe, "ms": t * 1e3, "cells_per_s": cells / t, "speedup": t_plain / t,
            "match_error_mean": em, "match_error_p95": e95, "match_error_vs_plain": em / e_plain,
            "fallback_rate": fbr, "members_scored_per_patch": spp})
    # equal match error: within 1 % of plain's mean, either way
    ok = [r for r in res["by_gate"] if abs(r["match_error_vs_plain"] - 1.0) <= 0.01]
    res["equal_error"] = max(ok, key=lambda r: r["speedup"]) if ok else None
    # realization statistics beside the TI's (the first evaluation seed):
    # the match error depends on the realizations themselves, so the forms'
    # realizations are compared directly
    forms = [("plain", p)] + [(f"probe {r['probe']}" + ("" if r["gate"] is None else f" gate {r['gate']}"),
                               dict(p, proposer_dim=64, proposer=index, lp_probe=r["probe"],
                                    lp_gate=1e30 if r["gate"] is None else r["gate"]))
                              for r in res["by_gate"] if r["gate"] is None]
    res["realization_stats"] = _realization_stats(cc, p, ti_d, forms, eval_seeds[0])
    return res


def _realization_stats(cc, p, ti_d, forms, seed, lags=(1, 5, 10, 20, 50, 100)):
    """Per form: facies proportions, indicator variograms of facies 1 along x
    and y and its probability of connection along x at a few lags, for the
    realizations of one call, with the TI's; and the mean absolute
    difference of the two variograms from the TI's over those lags."""
    import numpy as np
    import torch
    nf, max_lag = p["n_facies"], max(lags)
    g, t_ext = p["grid"], p["ti"]
    lag_i = [h - 1 for h in lags]

    def stats(imgs, ext):
        n = imgs.shape[0]
        cells = n * int(np.prod(ext))
        pi, _ = cc.stats_histogram(imgs, nf, per_cell=False)
        vx, vy = cc.stats_variogram(imgs, nf, 0, max_lag), cc.stats_variogram(imgs, nf, 1, max_lag)
        bx, cx = cc.stats_connectivity(imgs, nf, 0, max_lag)
        gam = {}
        for name, v, a in (("x", vx, 0), ("y", vy, 1)):
            pairs = np.array([cc.pair_count(ext, a, h) for h in lags], dtype=np.float64)
            gam[name] = v.cpu().numpy().sum(axis=0)[1, lag_i] / (2.0 * pairs * n)
        b, c = bx.cpu().numpy().sum(axis=0)[1, lag_i], cx.cpu().numpy().sum(axis=0)[1, lag_i]
        return {"proportions": (pi.cpu().numpy().sum(axis=0) / cells).round(4).tolist(),
                "variogram_x": gam["x"].round(4).tolist(), "variogram_y": gam["y"].round(4).tolist(),
                "connection_x": np.where(b > 0, c / np.maximum(b, 1), np.nan).round(4).tolist()}

    out = {"lags": list(lags), "facies": 1, "seed": seed, "ti": stats(ti_d.view(1, *ti_d.shape), t_ext)}
    tv = np.array(out["ti"]["variogram_x"] + out["ti"]["variogram_y"])
    for name, q in forms:
        sim = cc.Simulator(dict(q, seed=seed), device=ti_d.device)
        real = sim.run(ti_d).view(torch.int8)
        st = stats(real, g)
        st["variogram_mad_vs_ti"] = float(np.abs(np.array(st["variogram_x"] + st["variogram_y"]) - tv).mean())
        out[name] = st
        del sim, real
    return out


def _time_case(cc, p, ti, hd, dev, reps=3):
    import numpy as np
    import torch
    nd = len(p["ti"])
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    hd_d = cc.hd_to_device(hd, nd, device=dev)
    sim = cc.Simulator(p, device=dev)
    sim.run(ti_d, hd_d)                      # first call: tuning runs
    t = _time_runs(lambda: sim.run(ti_d, hd_d), reps)
    cc.profile_enable(True)
    cc.profile_read()
    sim.run(ti_d, hd_d)
    torch.cuda.synchronize()
    prof = cc.profile_read()
    cc.profile_enable(False)
    cells = p["n_real"] * int(np.prod(p["grid"]))
    st = cc.simulate_stats(p)
    return {"ms": t * 1e3, "cells_per_s": cells / t, "wavefront_steps": st["wavefront_steps"],
            "hard_data": 0 if hd is None else int(len(hd[0])),
            "kernel_ms": {k: round(v[0], 4) for k, v in prof.items() if v[1]}}


def measure_next(cc, wl, dev):
    """C2 with the 5/3 wavelet beside Haar, dense conditioning (C2 with 300,
    4000, 8000 hard data) and the level x grid-size sweep (C2 training image,
    T 32, OV 8, 1000 hard data per 512^2; 512^2 also with 2000)."""
    out = {"dense_conditioning": [], "level_grid": [], "wavelet": []}
    # another mother wavelet: C2 with the LeGall 5/3 integer lifting beside Haar
    for wav in (0, 1):
        p, ti, hd = wl.make("c2_scale2d")
        p["wavelet"] = wav
        out["wavelet"].append(dict(_time_case(cc, p, ti, hd, dev), wavelet="haar" if wav == 0 else "legall53"))
    for n_hd in (300, 4000, 8000):
        p, ti, hd = wl.dense_conditioning(n_hd)
        out["dense_conditioning"].append(dict(_time_case(cc, p, ti, hd, dev), workload=wl.describe(p)))
    for level in (1, 2, 3):
        for n in (128, 256, 512, 1024, 2048):
            p, ti, hd = wl.level_grid_case(level, n)
            out["level_grid"].append(dict(_time_case(cc, p, ti, hd, dev), level=level, grid=n))
        p, ti, hd = wl.level_grid_case(level, 512, hd_per_512=2000)
        out["level_grid"].append(dict(_time_case(cc, p, ti, hd, dev), level=level, grid=512))
    out["cdf97"] = measure_cdf97(cc, wl, dev)
    return out


def measure_cdf97(cc, wl, dev, n_events=448, k=10, reps=10):
    """The CDF 9/7 path at the 2000^2 x 16 workload's scan shape (1000^2
    three-facies training image, J = 2, T = 48, 448 data events: 28 patches
    in flight x 16 realizations): the transform, the exact fp32 selection
    (every candidate rescored) and the precision split (fp16 / bf16 MFMA bulk,
    fp32 rescoring of a 64 or 128 shortlist), with the share of the exact
    path's 10 best that each split keeps.  Events are crops of the level-2
    approximation of a second seeded channel image at random block
    positions, known on an L-shaped band of 3 blocks."""
    import numpy as np
    import torch
    from paper_2404_00441_amd import synthetic as syn
    p, ti, _ = wl.make("c5_learned", n_real=1)
    level, T = p["level"], p["tmpl"]
    b = 2 ** level
    tc = [-(-t // b) for t in T]
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    ref = syn.channel_image_2d(p["grid"][0] // 2, p["grid"][1] // 2, 50, p["n_facies"], seed=4242)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_dwt = timed(lambda: cc.dwt97(ti_d, level))
    K, _ = cc.dwt97(ti_d, level)
    Kr, _ = cc.dwt97(torch.from_numpy(np.ascontiguousarray(ref)).to(dev), level)
    Kr = Kr.cpu().numpy()
    rng = np.random.default_rng(17)
    ov = 3
    mask = np.zeros((tc[1], tc[0]), bool)
    mask[:ov, :] = True
    mask[:, :ov] = True
    n = np.broadcast_to(mask, (n_events,) + mask.shape).astype(np.int32).copy()
    A = np.zeros(n.shape, np.float32)
    for e in range(n_events):
        y, x = rng.integers(0, Kr.shape[0] - tc[1] + 1), rng.integers(0, Kr.shape[1] - tc[0] + 1)
        A[e][mask] = Kr[y: y + tc[1], x: x + tc[0]][mask]
    n_d = torch.from_numpy(n.reshape(n_events, -1)).to(dev)
    A_d = torch.from_numpy(A.reshape(n_events, -1)).to(dev)
    real = torch.arange(n_events, dtype=torch.int32, device=dev) % 16
    step = torch.arange(n_events, dtype=torch.int64, device=dev)
    cand = [(p["ti"][a] - T[a]) // b + 1 for a in range(2)]
    ncand = cand[0] * cand[1]
    nk = int(mask.sum())

    def run(shortlist, precision=0):
        return cc.ccf_scan97(p["ti"], level, K, T, n_d, A_d, top_k=k, shortlist=shortlist, precision=precision,
                             seed=1, realization=real, step=step)[1]

    exact = run(0).cpu()
    ex_idx = [set((exact[e] & 0xFFFFF).tolist()) for e in range(n_events)]
    ms_exact = timed(lambda: run(0))
    res = {"workload": f"1000^2 TI, J={level}, T={T[0]}, {n_events} events x {ncand} candidates, "
                       f"{nk} known blocks per event, K={k}",
           "dwt97_ms": ms_dwt,
           "exact_fp32": {"ms_per_call": ms_exact,
                          "gflops_fp32": 3.0 * nk * ncand * n_events / (ms_exact * 1e-3) / 1e9},
           "split": []}
    for prec, name in ((0, "fp16"), (1, "bf16")):
        for R in (64, 128):
            keys = run(R, prec).cpu()
            same = np.mean([len(ex_idx[e] & set((keys[e] & 0xFFFFF).tolist())) / k for e in range(n_events)])
            ms = timed(lambda: run(R, prec))
            res["split"].append({"bulk": name, "shortlist": R, "ms_per_call": ms,
                                 "speedup_vs_exact": ms_exact / ms,
                                 "top10_same_as_exact": float(same),
                                 "bulk_tflops_algorithmic": 2.0 * 2 * nk * ncand * n_events / (ms * 1e-3) / 1e12})
    return res


def measure_stats(cc, wl, dev, n_real=100, max_lag=200):
    """An ensemble of C2 realizations in one call (the same 300 hard data for
    each), then its statistics beside the TI's: facies counts and ensemble
    map, indicator variograms along x and y, probability of connection
    along x (each timed with events on the launch stream)."""
    import numpy as np
    import torch
    p, ti, hd = wl.ensemble(n_real)
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    hd_d = cc.hd_to_device(hd, len(p["ti"]), device=dev)
    sim = cc.Simulator(p, device=dev)
    out = sim.run(ti_d, hd_d)
    t_sim = _time_runs(lambda: sim.run(ti_d, hd_d, out=out), 2)
    del sim
    real = out.view(torch.int8)
    nf = p["n_facies"]
    res = {"workload": wl.describe(p), "simulate_ms": t_sim * 1e3,
           "simulate_cells_per_s": n_real * int(np.prod(p["grid"])) / t_sim, "max_lag": max_lag}

    def timed(fn, reps=3):
        fn()
        st = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        for _ in range(reps):
            r = fn()
        b.record(st)
        b.synchronize()
        return a.elapsed_time(b) / reps, r

    ms = {}
    ms["histogram"], (pi, pc) = timed(lambda: cc.stats_histogram(real, nf))
    ms["variogram_x"], vx = timed(lambda: cc.stats_variogram(real, nf, 0, max_lag))
    ms["variogram_y"], vy = timed(lambda: cc.stats_variogram(real, nf, 1, max_lag))
    ms["connectivity_x"], (bx, cx) = timed(lambda: cc.stats_connectivity(real, nf, 0, max_lag))
    ms["connectivity_y"], _ = timed(lambda: cc.stats_connectivity(real, nf, 1, max_lag))
    res["ms"] = ms
    cells = n_real * int(np.prod(p["grid"]))
    res["cells_per_s"] = {k: cells / (v * 1e-3) for k, v in ms.items()}
    # the TI's statistics and the ensemble's, as ratios
    tid = ti_d.view(1, *ti_d.shape)
    tpi, _ = cc.stats_histogram(tid, nf, per_cell=False)
    tvx, tvy = cc.stats_variogram(tid, nf, 0, max_lag), cc.stats_variogram(tid, nf, 1, max_lag)
    tbx, tcx = cc.stats_connectivity(tid, nf, 0, max_lag)
    g, t_ext = p["grid"], p["ti"]
    lags = np.arange(1, max_lag + 1)
    n_r = {a: np.array([cc.pair_count(g, a, h) for h in lags], dtype=np.float64) for a in (0, 1)}
    n_t = {a: np.array([cc.pair_count(t_ext, a, h) for h in lags], dtype=np.float64) for a in (0, 1)}

    def gam(v, n):
        return v.cpu().numpy().sum(axis=0) / (2.0 * n * v.shape[0])

    def tau(b, c):
        b, c = b.cpu().numpy().sum(axis=0), c.cpu().numpy().sum(axis=0)
        return np.where(b > 0, c / np.maximum(b, 1), np.nan)

    pick = [h for h in (1, 5, 10, 20, 50, 100, 200) if h <= max_lag]
    q = {"proportions_ti": (tpi.cpu().numpy()[0] / np.prod(t_ext)).round(4).tolist(),
         "proportions_realizations": (pi.cpu().numpy().sum(axis=0) / cells).round(4).tolist(),
         "ensemble_map_hard_data_cells": None, "lags": pick}
    for name, v_r, v_t, a in (("variogram_x", vx, tvx, 0), ("variogram_y", vy, tvy, 1)):
        gr, gt = gam(v_r, n_r[a]), gam(v_t, n_t[a])
        q[name] = {"facies": 1, "ti": [round(float(gt[1, h - 1]), 4) for h in pick],
                   "realizations": [round(float(gr[1, h - 1]), 4) for h in pick]}
    tr, tt = tau(bx, cx), tau(tbx, tcx)
    q["connection_x"] = {"facies": 1, "ti": [round(float(tt[1, h - 1]), 4) for h in pick],
                         "realizations": [round(float(tr[1, h - 1]), 4) for h in pick]}
    # the ensemble map at hard-data cells: every realization honours them
    pos = hd[1][: len(hd[1]) // n_real]
    val = hd[2][: len(hd[2]) // n_real]
    pcn = pc.cpu().numpy()
    q["ensemble_map_hard_data_cells"] = float(np.mean([pcn[v, y, x] / n_real for (x, y), v in zip(pos, val)]))
    res["quality"] = q
    return res


def measure_forms(cc, wl, dev):
    """Side measurements of the batched and precision-split forms.

    batched: the 64-realization workload in one call against the same 64
    realizations simulated one call at a time (same kernels, same results).
    precision_split: the 3D workload with an fp16 bulk scan and exact
    rescoring of a 32-shortlist; the report gives the largest bulk-vs-exact
    score difference over every rescored candidate."""
    import numpy as np
    import torch
    out = {}
    p, ti, hd = wl.make("c4_batched")
    nd = len(p["ti"])
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    sim = cc.Simulator(p, device=dev)
    hd_d = cc.hd_to_device(hd, nd, device=dev)
    t_batch = _time_runs(lambda: sim.run(ti_d, hd_d), 3)
    cells = p["n_real"] * int(np.prod(p["grid"]))
    # one realization per call: realization r keeps its own hard data
    p1 = dict(p, n_real=1)
    sims, hds = [], []
    for r in range(p["n_real"]):
        q = dict(p1, seed=p["seed"])
        sel = hd[0] == r
        hr = (np.zeros(int(sel.sum()), np.int32), hd[1][sel], hd[2][sel])
        q["max_hard_data"] = int(sel.sum())
        sims.append(cc.Simulator(q, device=dev))
        hds.append(cc.hd_to_device(hr, nd, device=dev))
    def one_at_a_time():
        for s_, h_ in zip(sims, hds):
            s_.run(ti_d, h_)
    t_single = _time_runs(one_at_a_time, 2)
    out["batched"] = {"workload": wl.describe(p), "ms_batched": t_batch * 1e3,
                      "ms_one_at_a_time": t_single * 1e3, "cells_per_s_batched": cells / t_batch,
                      "cells_per_s_one_at_a_time": cells / t_single, "speedup": t_single / t_batch}
    out["learned"] = measure_learned(cc, wl, dev)
    out["certified_proposer"] = measure_certified(cc, wl, dev)
    p3, ti3, hd3 = wl.make("c3_split3d")
    sim3 = cc.Simulator(p3, device=dev)
    ti3_d = torch.from_numpy(np.ascontiguousarray(ti3)).to(dev)
    t3 = _time_runs(lambda: sim3.run(ti3_d, None), 3)
    rep = sim3.report()
    p3b = dict(p3, shortlist=0)
    sim3b = cc.Simulator(p3b, device=dev)
    t3b = _time_runs(lambda: sim3b.run(ti3_d, None), 3)
    out["precision_split"] = {"workload": wl.describe(p3), "bulk": "fp16 in / fp32 accumulate",
                              "shortlist": p3["shortlist"], "cells_per_s": int(np.prod(p3["grid"])) / t3,
                              "cells_per_s_without_rescoring": int(np.prod(p3["grid"])) / t3b,
                              "max_abs_score_error_vs_exact": rep["max_abs_error"],
                              "candidates_rescored": rep["rescored"], "topk_changed": rep["topk_changed"]}
    return out


def main():
    a = parse()
    if a.oracle_worker:
        oracle_worker_main(a.oracle_worker, a.oracle_procs)
        return
    if a.calibrate_copy:
        calibrate_copy(a.calibrate_copy)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {a.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2404_00441_amd import ccwsim as cc
    from paper_2404_00441_amd import workloads as wl

    if a.learned_only:
        pts = tuple((int(v.split(":")[0]), float(v.split(":")[1]) if ":" in v else None)
                    for v in a.lp_points.split(",")) if a.lp_points else None
        seeds = tuple(range(1, a.lp_eval_seeds + 1)) if a.lp_eval_seeds else None
        print(json.dumps({"learned": measure_learned(cc, wl, torch.device("cuda:0"), epochs=a.lp_epochs,
                                                     lists=a.lp_lists, points=pts, eval_seeds=seeds,
                                                     kmeans_iters=a.lp_kmeans_iters)}), flush=True)
        return
    if a.cdf97_only:
        print(json.dumps({"cdf97": measure_cdf97(cc, wl, torch.device("cuda:0"))}), flush=True)
        return
    p, ti, hd = wl.make(a.workload, n_real=a.n_real)
    nd = len(p["ti"])
    dev = torch.device("cuda:0")
    ti_d = torch.from_numpy(np.ascontiguousarray(ti)).to(dev)
    hd_d = cc.hd_to_device(hd, nd, device=dev)
    sim = cc.Simulator(p, device=dev)
    out = torch.empty((p["n_real"],) + tuple(p["grid"][::-1]), dtype=torch.int8, device=dev)
    stats = cc.simulate_stats(p)

    for _ in range(a.warmup):
        sim.run(ti_d, hd_d, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        sim.run(ti_d, hd_d, out=out)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / a.steps
    print(f"timed {a.steps} steps: {dt * 1e3:.3f} ms/step", file=sys.stderr, flush=True)

    cells = stats["cells"]
    scanned = stats["patches"]          # every patch scans all candidates (the first scores 0)
    res = {
        "metric": METRIC,
        "value": cells / dt,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16",
        "data": "synthetic",
        "config": {"workload": wl.describe(p), "hard_data": 0 if hd is None else int(len(hd[0])),
                   "path": "seeded" if p["path_mode"] else "raster", "form": "plain"},
        "ccf_candidates_per_s": scanned * stats["candidates"] / dt,
        "scan_tflops_algorithmic": stats["scan_flops"] / dt / 1e12,
    }

    if not a.no_roofline:
        cc.profile_enable(True)
        cc.profile_read()
        for _ in range(a.steps):
            sim.run(ti_d, hd_d, out=out)
        torch.cuda.synchronize()
        prof = cc.profile_read()
        cc.profile_enable(False)
        kern = {k: {"ms_per_step": v[0] / a.steps, "launches_per_step": v[1] / a.steps,
                    "us_per_launch": (1e3 * v[0] / v[1]) if v[1] else 0.0} for k, v in prof.items()}
        res["kernels"] = kern
        dom = max(prof, key=lambda k: prof[k][0])
        # algorithmic work of each kind per step
        tcells = 1
        for t in p["tmpl"]:
            tcells *= t
        per_step_work = {
            "scan": ("mfma", stats["scan_flops"], "TFLOP/s", PEAK_FP16_TFLOPS, 1e12),
            # 6 T^d bytes per patch: windows read, coefficients read, window written
            "finalize": ("hbm", 6.0 * tcells * stats["patches"], "GB/s", PEAK_HBM_GBS, 1e9),
        }
        kind = dom if dom in per_step_work else "scan"
        bound, work, unit, peak, scale = per_step_work[kind]
        launches = prof[kind][1] / a.steps
        us = kern[kind]["us_per_launch"]
        achieved = (work / launches) / (us * 1e-6) / scale if us > 0 else 0.0
        traffic = None
        if os.path.exists(a.traffic_json):
            try:
                tj = json.load(open(a.traffic_json))
                if (tj.get("kernel") == kind and tj.get("workload") == a.workload
                        and tj.get("source_hash") == kernel_source_hash()):
                    traffic = tj.get("bytes_per_launch")
            except (OSError, ValueError):
                traffic = None
        res["roofline"] = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                           "frac": achieved / peak, "traffic": traffic, "kernel": kind,
                           "dominant_by_time": dom, "us_per_launch": us,
                           "work_per_launch": work / launches}
        # the other per-step kernel against its own roofline
        other = "finalize" if kind == "scan" else "scan"
        if prof.get(other, (0, 0))[1]:
            b2, w2, u2, pk2, sc2 = per_step_work[other]
            us2 = kern[other]["us_per_launch"]
            a2 = (w2 / (prof[other][1] / a.steps)) / (us2 * 1e-6) / sc2
            res["roofline_other"] = {"kernel": other, "bound": b2, "achieved": a2, "peak": pk2, "unit": u2,
                                     "frac": a2 / pk2, "us_per_launch": us2}

    if a.workload != "c2_scale2d" and not a.no_next:
        # the one-realization workload (1000^2, 300 hard data) beside the headline
        p2, ti2, hd2 = wl.make("c2_scale2d")
        res["c2_scale2d"] = dict(_time_case(cc, p2, ti2, hd2, dev, reps=10), workload=wl.describe(p2))
    if not a.no_forms:
        res["forms"] = measure_forms(cc, wl, dev)
        res["scan_kernel"] = measure_scan_kernel(cc, wl, dev)
    if not a.no_next:
        res["next"] = measure_next(cc, wl, dev)
        res["stats"] = measure_stats(cc, wl, dev)

    if not a.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(a.workload, p["n_real"])
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
