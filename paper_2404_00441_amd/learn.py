"""Training and evaluation of the learned candidate proposer.

The proposer (two convolutional encoders over level-J approximation
coefficients, Sec. 3.1 and 4.3) is trained on pairs (data event, best
candidate): the events are those of plain simulations run through
``ccwsim_simulate`` (every patch's overlap as the scan sees it), and each
label is the candidate with the smallest exact score (``ccwsim_ccf_scan``
score map, then ``ccwsim_lp_labels``: the K candidates with the smallest
exact scores, the set the simulation draws from).  Training steps, the index
build and the proposal all run in the library's kernels; this module only
moves buffers between them and summarises results.
"""
from __future__ import annotations

import time

import torch

from . import ccwsim as cc


def max_code_of(p: dict) -> int:
    return int(p.get("n_facies", 2)) - 1


def training_pairs(p: dict, ti: torch.Tensor, seeds, chunk: int = 1024, n_pos: int | None = None):
    """Data events of plain simulations of ``p`` (one call per seed) with a
    non-empty overlap, and their best candidates.  Returns or_n, or_m
    (int32 [N, T_c cells]), labels (int32 [N, n_pos]: the n_pos candidates
    with the smallest exact scores, K of the workload by default), best
    (int32 [N]: one with the smallest), and, per event, the best exact
    score and the known-cell count (int64 [N] each)."""
    if n_pos is None:
        n_pos = int(p["top_k"])
    dev = ti.device
    ext = tuple(p["ti"])
    approx, _ = cc.dwt(ti, p["level"])
    ons, oms, labs, bests, sbest, nks = [], [], [], [], [], []
    for s in seeds:
        q = dict(p, seed=int(s), proposer_dim=0, proposer=None)
        sim = cc.Simulator(q, device=dev)
        sim.run(ti)
        on, om, rr, ss = sim.events()
        nk = on.sum(dim=1)
        keep = nk > 0
        on, om, rr, ss, nk = on[keep], om[keep], rr[keep], ss[keep], nk[keep]
        for i in range(0, on.shape[0], chunk):
            a, b = on[i: i + chunk].contiguous(), om[i: i + chunk].contiguous()
            S = cc.ccf_scan(ext, p["level"], max_code_of(p), approx, p["tmpl"], a, b)
            lab = cc.lp_labels(S, n_pos)
            sl = S.gather(1, lab.long())
            first = sl.argmin(dim=1, keepdim=True)
            labs.append(lab)
            bests.append(lab.gather(1, first)[:, 0].contiguous())
            sbest.append(sl.gather(1, first)[:, 0].to(torch.int64))
        ons.append(on)
        oms.append(om)
        nks.append(nk.to(torch.int64))
        del sim
    return (torch.cat(ons), torch.cat(oms), torch.cat(labs), torch.cat(bests), torch.cat(sbest), torch.cat(nks))


def train(p: dict, approx: torch.Tensor, on, om, labels, epochs: int = 2, batch: int = 512, lr: float = 2e-3,
          seed: int = 7, log=None):
    """Adam on the softmax cross-entropy over every candidate against each
    event's label set (int32 [N, L]) or best candidate ([N]).  Returns the
    weights and the mean loss of each epoch."""
    dev = approx.device
    ext = tuple(p["ti"])
    w = cc.lp_init(seed, device=dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    ws = cc.LpWorkspace(ext, p["level"], p["tmpl"], batch, device=dev)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    n = on.shape[0]
    steps = n // batch
    t = 0
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, device=dev, generator=g)
        tot = torch.zeros((), dtype=torch.float64, device=dev)
        t0 = time.time()
        for s in range(steps):
            idx = perm[s * batch: (s + 1) * batch]
            t += 1
            loss, _ = cc.lp_train_step(w, m, v, t, lr, approx, ws, on[idx].contiguous(), om[idx].contiguous(),
                                       labels[idx].contiguous())
            tot += loss.double().sum()
        hist.append(float(tot) / max(1, steps * batch))
        if log:
            log(f"epoch {ep}: mean loss {hist[-1]:.4f} ({time.time() - t0:.1f} s, {steps} steps)")
    return w, hist


def evaluate(p: dict, w, approx, on, om, labels, best, sbest, nk, k: int = 256, batch: int = 512):
    """Held-out metrics of the proxy scores: mean cross-entropy against the
    exact best candidate, recall@k of it and the mean share of the label set
    (the K best) in the proxy's top k, and the exact-score regret of the best
    of the top k (in match-error units: the score difference over |beta|^2
    times the known cells).  Returns a dict."""
    dev = approx.device
    ext = tuple(p["ti"])
    beta = (2 ** p["level"]) ** len(ext)
    ws = cc.LpWorkspace(ext, p["level"], p["tmpl"], batch, device=dev)
    zeros_m = torch.zeros_like(w)
    zeros_v = torch.zeros_like(w)
    ce, hit, hitset, reg = [], [], [], []
    for i in range(0, on.shape[0] - batch + 1, batch):
        a, b = on[i: i + batch].contiguous(), om[i: i + batch].contiguous()
        lab = best[i: i + batch].contiguous()
        # the loss at unchanged weights (learning rate 0, scratch moments)
        loss, _ = cc.lp_train_step(w, zeros_m.zero_(), zeros_v.zero_(), 1, 0.0, approx, ws, a, b, lab)
        ce.append(loss)
        _, _, S = cc.lp_encode(w, approx, ws, a, b, want_keys=False, want_scores=True)
        idx = cc.lp_shortlist(S, k)
        hit.append((idx == lab[:, None]).any(dim=1))
        lset = labels[i: i + batch]
        hitset.append((lset[:, :, None] == idx[:, None, :]).any(dim=2).double().mean(dim=1))
        ex = cc.ccf_scan(ext, p["level"], max_code_of(p), approx, p["tmpl"], a, b)
        s_sl = ex.gather(1, idx.long()).min(dim=1).values.to(torch.int64)
        reg.append((s_sl - sbest[i: i + batch]).double() / (beta * beta * nk[i: i + batch].double()))
    ce = torch.cat(ce).double()
    hit = torch.cat(hit).double()
    hitset = torch.cat(hitset)
    reg = torch.cat(reg)
    return {"ce_loss": float(ce.mean()), f"recall_at_{k}": float(hit.mean()),
            f"set_recall_at_{k}": float(hitset.mean()), "label_set": int(labels.shape[1]),
            "regret_mean": float(reg.mean()), "regret_p95": float(torch.quantile(reg, 0.95)),
            "events": int(ce.numel())}
