"""GPU checks of the learned proposer inside the hot path, against the CPU
oracle.

* The standalone proposal: the query equals the float64 reference encoder
  at the window's centre; the probed lists are those whose centroids score
  best; the keys it returns are, bit for bit, the K best of the oracle's
  keys over the scored members (oracle scores, oracle tie-break).
* A simulation whose gate sends every patch to the scan gives the oracle's
  realizations byte for byte.
* A simulation whose gate accepts every proposal draws, at every patch,
  the oracle's choice among the proposal's members, and logs the oracle's
  match error for it.
* The data events a simulation exports are the oracle's.

Weights are the seeded initialisation (the checks do not depend on how
well the proposer ranks)."""
import sys

import numpy as np
import pytest

from paper_2404_00441_amd import workloads as wl
from tests import lp_ref

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_00441_amd import ccwsim
    ccwsim.load()
    return ccwsim


def _t(a, dtype=None):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a if dtype is None else a.astype(dtype))).cuda()


def _sp(p, orc):
    keys = ("ti", "grid", "tmpl", "overlap", "level", "top_k", "n_real", "n_facies", "seed", "path_mode",
            "score_mode", "nc_margin", "cut")
    return orc.SimParams(**{k: p[k] for k in keys})


N_LISTS, PROBE = 16, 4


@pytest.fixture(scope="module")
def setup(cc, orc):
    p, ti, _ = wl.make("c5_learned", scale=0.2, n_real=2)
    _say("learned setup", p["ti"], p["grid"])
    tig = _t(ti)
    approx, _ = cc.dwt(tig, p["level"])
    w = cc.lp_init(5)
    index = cc.lp_build_index(w, approx, p["ti"], p["level"], p["tmpl"], N_LISTS, iters=5)
    K = orc.dwt(ti, p["level"])[0]
    return p, ti, tig, approx, w, index, K


def _events(cc, p, tig, extra=None):
    q = dict(p)
    q.update(extra or {})
    sim = cc.Simulator(q)
    out = sim.run(tig)
    on, om, rr, ss = sim.events()
    return sim, out, on, om, rr, ss


def test_events_are_the_oracles(cc, orc, setup):
    p, ti, tig, approx, w, index, K = setup
    _say("events vs oracle")
    sim, out, on, om, rr, ss = _events(cc, p, tig)
    geo = orc.geometry(_sp(p, orc))
    _, chosen = orc.simulate(_sp(p, orc), ti)
    on, om = on.cpu().numpy(), om.cpu().numpy()
    rr, ss = rr.cpu().numpy(), ss.cpu().numpy()
    tc = geo["tc"][:2][::-1]
    b = geo["beta_cells"]
    # each exported event, scored by the oracle, leads to the oracle's choice
    # at that (realization, step)
    rng = np.random.default_rng(0)
    for i in rng.choice(len(on), size=40, replace=False):
        S = orc.scores(K, geo["cand"][:2], on[i].reshape(tc), om[i].reshape(tc), b)
        c, _ = orc.select(S, None, p["top_k"], p["seed"], int(rr[i]), int(ss[i]))
        assert c == chosen[rr[i], ss[i]], (i, rr[i], ss[i])


def test_proposal_matches_oracle(cc, orc, setup):
    p, ti, tig, approx, w, index, K = setup
    _say("standalone proposal vs oracle")
    sim, out, on, om, rr, ss = _events(cc, p, tig)
    nk = on.sum(dim=1).cpu().numpy()
    sel = np.nonzero(nk > 0)[0][:48]
    import torch
    on, om = on[sel].contiguous(), om[sel].contiguous()
    rr, ss = rr[sel].contiguous(), ss[sel].to(torch.int64).contiguous()
    keys, mem, nmem, q, err = cc.lp_propose(index, approx, p["ti"], p["level"], p["n_facies"] - 1, p["tmpl"], on, om,
                                            PROBE, p["top_k"], seed=p["seed"], realization=rr, step=ss)
    geo = orc.geometry(_sp(p, orc))
    tc = geo["tc"][:2][::-1]
    cand = geo["cand"][:2]
    b = geo["beta_cells"]
    keys = keys.cpu().numpy().view(np.uint64)
    mem, nmem, q, err = mem.cpu().numpy(), nmem.cpu().numpy(), q.cpu().numpy(), err.cpu().numpy()
    onn, omn, rrn, ssn = on.cpu().numpy(), om.cpu().numpy(), rr.cpu().numpy(), ss.cpu().numpy()
    # the index: header, query weights, centroids, lists
    ixb = index.cpu().numpy()
    hdr = ixb[:128].view(np.int64)
    # header: 4 int32, 3 x int32[3] and padding, then ncand and the offsets (int64)
    off_w, off_cent, off_list, off_mem = (int(x) for x in hdr[8:12])
    assert int(hdr[7]) == int(np.prod(cand))
    nq = sum(co * ci * t + co for (co, ci, t) in lp_ref.layer_shapes(2))
    wq = ixb[off_w: off_w + 4 * nq].view(np.float32).astype(np.float64)
    wn = w.cpu().numpy().astype(np.float64)
    assert np.array_equal(wq, wn[wn.size - nq:])
    cent = ixb[off_cent: off_cent + 4 * N_LISTS * 64].view(np.float32).reshape(N_LISTS, 64).astype(np.float64)
    loff = ixb[off_list: off_list + 4 * (N_LISTS + 1)].view(np.int32)
    lmem = ixb[off_mem: off_mem + 4 * int(np.prod(cand))].view(np.int32)
    assert loff[0] == 0 and loff[-1] == np.prod(cand)
    assert np.array_equal(np.sort(lmem), np.arange(np.prod(cand)))
    list_of = np.empty(int(np.prod(cand)), np.int64)
    for j in range(N_LISTS):
        assert np.all(np.diff(lmem[loff[j]: loff[j + 1]]) > 0)
        list_of[lmem[loff[j]: loff[j + 1]]] = j
    # queries: the reference encoder's output at the window's centre
    ev = np.stack([omn, onn], axis=1).reshape(len(sel), 2, tc[0], tc[1]) / float(b)
    _, q_ref, _, _ = lp_ref.forward(wn, K, b, ev, cand, tc[::-1])
    assert np.abs(q - q_ref).max() <= 1e-4 * max(1.0, np.abs(q_ref).max())
    for i in range(len(sel)):
        # probed lists: no unprobed list scores clearly above a probed one
        cs = cent @ q_ref[i]
        n = int(nmem[i])
        members = mem[i, :n]
        probed = sorted({int(list_of[c]) for c in members})
        rest = [j for j in range(N_LISTS) if j not in probed]
        if rest and len(probed) == PROBE:
            assert cs[probed].min() >= cs[rest].max() - 1e-4 * np.abs(cs).max()
        # members are whole lists (the last one may be cut only when alone)
        tot = sum(loff[j + 1] - loff[j] for j in probed)
        assert n == tot or (len(probed) == 1 and n == cc.LP_CAND_MAX)
        # keys: the K best oracle keys over the members
        S = orc.scores(K, cand, onn[i].reshape(tc), omn[i].reshape(tc), b).ravel()
        Sm = np.full_like(S, 2 ** 31 - 1)
        Sm[members] = S[members]
        _, kref = orc.select(Sm, None, p["top_k"], p["seed"], int(rrn[i]), int(ssn[i]))
        assert np.array_equal(keys[i], kref), i
        # best match error of the proposal
        B = b   # |beta|, the cells of a level-J block
        m, nn = omn[i].astype(np.float64), onn[i].astype(np.float64)
        ct = (B * B * m[nn > 0] ** 2 / nn[nn > 0]).sum()
        e_ref = (S[members].min() + ct) / (B * B * nn.sum())
        assert abs(err[i] - e_ref) <= 1e-5 * max(1.0, abs(e_ref))


def test_gate_forced_to_fallback_gives_oracle_realizations(cc, orc, setup):
    p, ti, tig, approx, w, index, K = setup
    _say("learned, gate always falls back")
    q = dict(p, proposer_dim=64, proposer=index, lp_probe=PROBE, lp_gate=-1.0)
    sim = cc.Simulator(q)
    out = sim.run(tig).cpu().numpy()
    ref, _ = orc.simulate(_sp(p, orc), ti)
    assert np.array_equal(out, ref)
    rep = sim.report()
    assert rep["proposer_patches"] == 0 and rep["proposer_fallbacks"] == sim.n_patches()


def test_learned_draws_the_oracles_choice_among_members(cc, orc, setup):
    import torch
    p, ti, tig, approx, w, index, K = setup
    _say("learned, gate accepts every proposal")
    q = dict(p, proposer_dim=64, proposer=index, lp_probe=PROBE, lp_gate=1e30)
    sim = cc.Simulator(q)
    geo = orc.geometry(_sp(p, orc))
    chosen = torch.full((p["n_real"], geo["nsteps"]), -1, dtype=torch.int32, device="cuda")
    sim.run(tig, chosen=chosen)
    rep = sim.report()
    on, om, rr, ss = sim.events()
    err = sim.match_errors().cpu().numpy()
    n = sim.n_patches()
    nk = on.sum(dim=1).cpu().numpy()
    keys, mem, nmem, _, _ = cc.lp_propose(index, approx, p["ti"], p["level"], p["n_facies"] - 1, p["tmpl"], on, om,
                                          PROBE, p["top_k"], seed=p["seed"], realization=rr,
                                          step=ss.to(torch.int64))
    # the scan decides where the overlap is empty or too few members were scored
    fb = (nk == 0) | (nmem.cpu().numpy() < p["top_k"])
    assert rep["proposer_patches"] == int((~fb).sum()) and rep["proposer_fallbacks"] == int(fb.sum())
    ch = chosen.cpu().numpy()
    onn, omn, rrn, ssn = on.cpu().numpy(), om.cpu().numpy(), rr.cpu().numpy(), ss.cpu().numpy()
    mem, nmem = mem.cpu().numpy(), nmem.cpu().numpy()
    tc = geo["tc"][:2][::-1]
    cand = geo["cand"][:2]
    b = geo["beta_cells"]
    B = b   # |beta|, the cells of a level-J block
    rng = np.random.default_rng(1)
    picks = list(np.nonzero(fb)[0][:3]) + list(rng.choice(np.nonzero(~fb)[0], size=60, replace=False))
    for i in picks:
        S = orc.scores(K, cand, onn[i].reshape(tc), omn[i].reshape(tc), b).ravel()
        if not fb[i]:
            Sm = np.full_like(S, 2 ** 31 - 1)
            members = mem[i, : nmem[i]]
            Sm[members] = S[members]
        else:
            Sm = S   # no overlap: the full scan decides
        c, _ = orc.select(Sm, None, p["top_k"], p["seed"], int(rrn[i]), int(ssn[i]))
        assert c == ch[rrn[i], ssn[i]], i
        if nk[i] > 0:
            m, nn = omn[i].astype(np.float64), onn[i].astype(np.float64)
            ct = (B * B * m[nn > 0] ** 2 / nn[nn > 0]).sum()
            e_ref = (S[c] + ct) / (B * B * nn.sum())
            assert abs(err[i] - e_ref) <= 1e-5 * max(1.0, abs(e_ref)), i
        else:
            assert err[i] == -1.0
    assert len(err) == n


def test_plain_match_errors_are_the_oracles(cc, orc, setup):
    p, ti, tig, approx, w, index, K = setup
    _say("plain match errors")
    sim, out, on, om, rr, ss = _events(cc, p, tig)
    err = sim.match_errors().cpu().numpy()
    _, chosen = orc.simulate(_sp(p, orc), ti)
    geo = orc.geometry(_sp(p, orc))
    tc = geo["tc"][:2][::-1]
    b = geo["beta_cells"]
    B = b   # |beta|, the cells of a level-J block
    onn, omn, rrn, ssn = on.cpu().numpy(), om.cpu().numpy(), rr.cpu().numpy(), ss.cpu().numpy()
    rng = np.random.default_rng(2)
    for i in rng.choice(len(onn), size=40, replace=False):
        nn, m = onn[i].astype(np.float64), omn[i].astype(np.float64)
        if nn.sum() == 0:
            assert err[i] == -1.0
            continue
        S = orc.scores(K, geo["cand"][:2], onn[i].reshape(tc), omn[i].reshape(tc), b).ravel()
        c = chosen[rrn[i], ssn[i]]
        e_ref = (S[c] + (B * B * m[nn > 0] ** 2 / nn[nn > 0]).sum()) / (B * B * nn.sum())
        assert abs(err[i] - e_ref) <= 1e-5 * max(1.0, abs(e_ref)), i
        assert e_ref >= -1e-9   # a sum of squares


def test_training_pairs_spot_checked_by_the_oracle(cc, orc, setup):
    # the proposer's training pairs: 1 % (at least 25) of the labels checked
    # against the oracle's scores of the same data event
    from paper_2404_00441_amd import learn
    p, ti, tig, approx, w, index, K = setup
    _say("training pairs vs oracle")
    on, om, lab, best, sbest, nk = learn.training_pairs(p, tig, [11, 12])
    geo = orc.geometry(_sp(p, orc))
    tc = geo["tc"][:2][::-1]
    b = geo["beta_cells"]
    onn, omn, labn, bestn, sbn = (x.cpu().numpy() for x in (on, om, lab, best, sbest))
    assert (nk.cpu().numpy() > 0).all()
    assert labn.shape[1] == p["top_k"]
    rng = np.random.default_rng(3)
    n = max(25, len(onn) // 100)
    for i in rng.choice(len(onn), size=n, replace=False):
        S = orc.scores(K, geo["cand"][:2], onn[i].reshape(tc), omn[i].reshape(tc), b).ravel()
        assert S[bestn[i]] == S.min() == sbn[i], i
        # the label set: the K smallest scores (ties to the smaller index)
        want = np.sort(np.argsort(S, kind="stable")[: p["top_k"]])
        assert np.array_equal(np.sort(labn[i]), want), i


EDGE_CASES = [
    # (lists, probe): one list holding every candidate (cut at the member
    # cap); more lists probed than exist; the most lists (one or two candidates each)
    (1, 4), (3, 16), (1024, 16),
]


@pytest.mark.parametrize("n_lists,probe", EDGE_CASES, ids=[f"L{a}_P{b}" for a, b in EDGE_CASES])
def test_proposal_edge_cases_match_oracle(cc, orc, setup, n_lists, probe):
    import torch
    p, ti, tig, approx, w, index, K = setup
    _say("proposal edge case", n_lists, probe)
    geo = orc.geometry(_sp(p, orc))
    tc = geo["tc"][:2][::-1]
    cand = geo["cand"][:2]
    b = geo["beta_cells"]
    ncand = int(np.prod(cand))
    n_lists = min(n_lists, ncand)
    ix = cc.lp_build_index(w, approx, p["ti"], p["level"], p["tmpl"], n_lists, iters=3)
    sim, out, on, om, rr, ss = _events(cc, p, tig)
    # events with an overlap, one without (every score 0), one with a single
    # known block
    sel = np.nonzero(on.sum(dim=1).cpu().numpy() > 0)[0][:6]
    on_s, om_s = on[sel].clone(), om[sel].clone()
    on_s[0] = 0
    om_s[0] = 0
    on_s[1] = 0
    om_s[1] = 0
    on_s[1, 5] = b
    om_s[1, 5] = b
    rr_s, ss_s = rr[sel].contiguous(), ss[sel].to(torch.int64).contiguous()
    keys, mem, nmem, _, _ = cc.lp_propose(ix, approx, p["ti"], p["level"], p["n_facies"] - 1, p["tmpl"],
                                          on_s.contiguous(), om_s.contiguous(), probe, p["top_k"], seed=p["seed"],
                                          realization=rr_s, step=ss_s)
    keys = keys.cpu().numpy().view(np.uint64)
    mem, nmem = mem.cpu().numpy(), nmem.cpu().numpy()
    onn, omn, rrn, ssn = on_s.cpu().numpy(), om_s.cpu().numpy(), rr_s.cpu().numpy(), ss_s.cpu().numpy()
    for i in range(len(sel)):
        n = int(nmem[i])
        assert 1 <= n <= min(ncand, cc.LP_CAND_MAX)
        members = mem[i, :n]
        assert len(np.unique(members)) == n and members.min() >= 0 and members.max() < ncand
        if n_lists == 1:
            assert n == min(ncand, cc.LP_CAND_MAX) and np.array_equal(members, np.arange(n))
        S = orc.scores(K, cand, onn[i].reshape(tc), omn[i].reshape(tc), b).ravel()
        Sm = np.full_like(S, 2 ** 31 - 1)
        Sm[members] = S[members]
        if n >= p["top_k"]:
            _, kref = orc.select(Sm, None, p["top_k"], p["seed"], int(rrn[i]), int(ssn[i]))
            assert np.array_equal(keys[i], kref), i
        else:
            assert np.all(keys[i] == np.uint64(2 ** 64 - 1))


def test_learned_simulation_with_hard_data_falls_back_there(cc, orc):
    # patches with hard data in their virtual template go to the scan, so a
    # conditional run honours every datum; with the gate closed the
    # realizations are the oracle's
    p, ti, hd = wl.make("c2_scale2d", scale=0.3)
    _say("learned with hard data", p["ti"], p["grid"], len(hd[0]))
    tig = _t(ti)
    approx, _ = cc.dwt(tig, p["level"])
    w = cc.lp_init(9)
    ix = cc.lp_build_index(w, approx, p["ti"], p["level"], p["tmpl"], 16, iters=3)
    nd = len(p["ti"])
    hdd = cc.hd_to_device(hd, nd)
    q = dict(p, proposer_dim=64, proposer=ix, lp_probe=4, lp_gate=1e30)
    sim = cc.Simulator(q)
    out = sim.run(tig, hdd).cpu().numpy()
    for r, pos, v in zip(*hd):
        assert out[(r,) + tuple(pos[::-1])] == v
    rep = sim.report()
    assert rep["proposer_fallbacks"] > 0 and rep["proposer_patches"] > 0
    q = dict(q, lp_gate=-1.0)
    sim2 = cc.Simulator(q)
    out2 = sim2.run(tig, hdd).cpu().numpy()
    ref, _ = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(out2, ref)
