"""GPU parity: every entry point of the C ABI against the CPU oracle.

All comparisons are bit-exact: every quantity of the method is an integer
(integer Haar coefficients, integer scores, indices, codes).  Inputs are
seeded and synthetic (``paper_2404_00441_amd.synthetic``); expected values
come from ``oracle/`` only.
"""
import sys

import numpy as np
import pytest

from paper_2404_00441_amd import synthetic as syn
from paper_2404_00441_amd import workloads as wl

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
    d = {k: p[k] for k in keys}
    d["wavelet"] = p.get("wavelet", 0)
    return orc.SimParams(**d)


# --------------------------------------------------------------------------
# A1 DWT
# --------------------------------------------------------------------------
DWT_CASES = [((13, 17), 1), ((150, 150), 1), ((500, 500), 2), ((61, 47), 3), ((33, 20), 0),
             ((20, 18, 9), 2), ((180, 150, 60), 2), ((7, 9, 5), 1)]


@pytest.mark.parametrize("shape,J", DWT_CASES, ids=[f"{'x'.join(map(str, s))}_J{j}" for s, j in DWT_CASES])
def test_dwt_parity(cc, orc, shape, J):
    _say("dwt", shape, J)
    rng = np.random.default_rng(sum(shape) + J)
    if len(shape) == 2:
        x = syn.channel_image_2d(shape[1], shape[0], 5, 3, seed=7) if min(shape) >= 40 else \
            rng.integers(0, 3, size=shape).astype(np.int8)
    else:
        x = rng.integers(0, 2, size=shape).astype(np.int8)
    a_gpu, d_gpu = cc.dwt(_t(x), J)
    a_orc, d_orc = orc.dwt(x, J)
    assert np.array_equal(a_gpu.cpu().numpy().astype(np.int64), a_orc)
    if J > 0:
        assert np.array_equal(d_gpu.cpu().numpy().astype(np.int64), orc.details_flat(d_orc))


# --------------------------------------------------------------------------
# A7 inverse DWT of patterns
# --------------------------------------------------------------------------
IDWT_CASES = [((150, 150), (24, 24), 1), ((500, 500), (40, 40), 2), ((101, 77), (13, 9), 2),
              ((180, 150, 60), (30, 30, 10), 2), ((40, 30, 20), (7, 5, 6), 1), ((50, 40), (11, 7), 0)]


@pytest.mark.parametrize("ext,patch,J", IDWT_CASES, ids=[f"{'x'.join(map(str, e))}_J{j}" for e, _, j in IDWT_CASES])
def test_idwt_parity(cc, orc, ext, patch, J):
    _say("idwt", ext, patch, J)
    rng = np.random.default_rng(len(ext) * 100 + J)
    shape = ext[::-1]
    x = rng.integers(0, 3, size=shape).astype(np.int8)
    a_gpu, d_gpu = cc.dwt(_t(x), J)
    b = 2 ** J
    nd = len(ext)
    G = [-(-e // b) for e in ext]
    tc = [-(-t // b) for t in patch]
    n = 40
    org = np.zeros((n, 3), dtype=np.int32)
    for a in range(nd):
        org[:, a] = rng.integers(0, G[a] - tc[a] + 1, size=n)
        org[0, a] = 0
        org[1, a] = G[a] - tc[a]
    pats = cc.idwt(a_gpu, d_gpu, ext, J, _t(org), patch).cpu().numpy()
    a_orc, d_orc = orc.dwt(x, J)
    xp = np.pad(x, [(0, (-s) % b) for s in shape], mode="edge")
    for i in range(n):
        sl = tuple(slice(b * org[i, a], b * org[i, a] + patch[a]) for a in range(nd))[::-1]
        reg = orc.idwt_region(a_orc, d_orc, ext, J, list(org[i, :nd]), tc)
        want = reg[tuple(slice(0, patch[a]) for a in range(nd))[::-1]]
        assert np.array_equal(want, xp[sl])
        assert np.array_equal(pats[i].astype(np.int64), want)


DWT53_CASES = [((13, 17), 1), ((150, 150), 1), ((500, 500), 2), ((61, 47), 3), ((33, 20), 0),
               ((20, 18, 9), 2), ((180, 150, 60), 2), ((7, 9, 5), 1)]


@pytest.mark.parametrize("shape,J", DWT53_CASES, ids=[f"{'x'.join(map(str, s))}_J{j}" for s, j in DWT53_CASES])
def test_dwt53_parity(cc, orc, shape, J):
    # the LeGall 5/3 transform with every sub-band, and its inverse: the
    # approximation and details equal the oracle's, and the patterns rebuilt
    # from them equal the edge-replicated image's windows
    _say("dwt53", shape, J)
    rng = np.random.default_rng(sum(shape) + J + 53)
    if len(shape) == 2:
        x = syn.channel_image_2d(shape[1], shape[0], 5, 3, seed=7) if min(shape) >= 40 else \
            rng.integers(0, 3, size=shape).astype(np.int8)
    else:
        x = rng.integers(0, 2, size=shape).astype(np.int8)
    a_gpu, d_gpu = cc.dwt(_t(x), J, wavelet=1)
    a_orc, d_orc = orc.dwt53(x, J)
    assert np.array_equal(a_gpu.cpu().numpy().astype(np.int64), a_orc)
    if J > 0:
        assert np.array_equal(d_gpu.cpu().numpy().astype(np.int64), orc.details_flat(d_orc))
    # patterns from the coefficients
    nd = len(shape)
    ext = shape[::-1]
    b = 2 ** J
    G = [-(-e // b) for e in ext]
    patch = [max(1, min(e, 11)) for e in ext]
    tc = [-(-t // b) for t in patch]
    n = 12
    org = np.zeros((n, 3), dtype=np.int32)
    for a in range(nd):
        org[:, a] = rng.integers(0, G[a] - tc[a] + 1, size=n)
        org[1, a] = G[a] - tc[a]
    org[2, 0] = G[0]   # outside the grid: -1
    pats = cc.idwt(a_gpu, d_gpu, ext, J, _t(org), patch, wavelet=1).cpu().numpy()
    xp = orc.idwt53(a_orc, d_orc)
    for i in range(n):
        if i == 2:
            assert (pats[i] == -1).all()
            continue
        sl = tuple(slice(b * org[i, a], b * org[i, a] + patch[a]) for a in range(nd))[::-1]
        assert np.array_equal(pats[i].astype(np.int64), xp[sl]), i


def test_idwt_rejects_origin_outside_grid(cc):
    x = np.random.default_rng(0).integers(0, 2, size=(40, 40)).astype(np.int8)
    a, d = cc.dwt(_t(x), 1)
    org = np.array([[19, 0, 0], [-1, 0, 0], [0, 15, 0]], dtype=np.int32)  # tc = 6 -> only [0..14] fit
    pats = cc.idwt(a, d, (40, 40), 1, _t(org), (12, 12)).cpu().numpy()
    assert (pats == -1).all()


# --------------------------------------------------------------------------
# A3/A4 scan
# --------------------------------------------------------------------------
def _events(rng, T, J, nf, ncode, kind):
    """nf data events over the T window: random masks, or overlap bands."""
    b = 2 ** J
    tc = [-(-t // b) for t in T]
    nd = len(T)
    nb = np.zeros((nf,) + tuple(tc[::-1]), dtype=np.int64)
    mb = np.zeros_like(nb)
    for f in range(nf):
        vals = rng.integers(0, ncode, size=T[::-1])
        if kind == "random":
            mask = rng.random(T[::-1]) < rng.uniform(0.05, 1.0)
        else:
            mask = np.zeros(T[::-1], dtype=bool)
            ov = [max(1, t // 4) for t in T]
            for a in range(nd):
                if rng.random() < 0.6:
                    sl = [slice(None)] * nd
                    sl[nd - 1 - a] = slice(0, ov[a]) if rng.random() < 0.5 else slice(T[a] - ov[a], T[a])
                    mask[tuple(sl)] = True
        for u in zip(*np.nonzero(mask)):
            bk = tuple(ui // b for ui in u)
            nb[(f,) + bk] += 1
            mb[(f,) + bk] += vals[u]
    return nb, mb


SCAN_CASES = [
    # ext (x,y[,z]), T, J, n_filters, n_facies, kind, mode
    ((150, 150), (24, 24), 1, 3, 2, "bands", 0),
    ((500, 500), (40, 40), 2, 17, 3, "bands", 0),
    ((400, 400), (32, 32), 2, 70, 3, "random", 0),
    ((97, 131), (18, 22), 1, 33, 3, "random", 1),
    ((60, 50), (9, 7), 0, 5, 3, "random", 0),
    ((180, 150, 60), (30, 30, 10), 2, 46, 2, "bands", 0),
    ((45, 40, 21), (9, 11, 6), 1, 9, 3, "random", 1),
]


@pytest.mark.parametrize("case", SCAN_CASES, ids=[f"{'x'.join(map(str, c[0]))}_J{c[2]}_F{c[3]}_m{c[6]}"
                                                  for c in SCAN_CASES])
def test_scan_parity(cc, orc, case):
    ext, T, J, nf, nfac, kind, mode = case
    _say("scan", case)
    rng = np.random.default_rng(nf + J)
    shape = ext[::-1]
    if len(ext) == 2 and min(ext) >= 60:
        x = syn.channel_image_2d(ext[0], ext[1], 8, nfac, seed=nf)
    else:
        x = rng.integers(0, nfac, size=shape).astype(np.int8)
    a_gpu, _ = cc.dwt(_t(x), J)
    nb, mb = _events(rng, T, J, nf, nfac, kind)
    S = cc.ccf_scan(ext, J, nfac - 1, a_gpu, T, _t(nb, np.int32), _t(mb, np.int32), score_mode=mode)
    S = S.cpu().numpy()
    a_orc, _ = orc.dwt(x, J)
    b = 2 ** J
    cand = [(ext[a] - T[a]) // b + 1 for a in range(len(ext))]
    for f in range(nf):
        want = orc.scores(a_orc, cand, nb[f], mb[f], b ** len(ext), mode=mode).ravel()
        assert np.array_equal(S[f].astype(np.int64), want), f"filter {f}"


@pytest.mark.parametrize("G", [1, 2, 4, 8, -1])
def test_scan_tile_groups(cc, orc, G):
    # several 32-filter tiles per workgroup share one A gather; results must
    # not depend on how many (the last group is ragged for G = 2, 4, 8)
    ext, T, J, nf, nfac = (400, 400), (32, 32), 2, 70, 3
    _say("scan groups", G)
    rng = np.random.default_rng(5)
    x = syn.channel_image_2d(ext[0], ext[1], 8, nfac, seed=9)
    a_gpu, _ = cc.dwt(_t(x), J)
    nb, mb = _events(rng, T, J, nf, nfac, "bands")
    cc.set_scan_group(G)
    try:
        S = cc.ccf_scan(ext, J, nfac - 1, a_gpu, T, _t(nb, np.int32), _t(mb, np.int32)).cpu().numpy()
    finally:
        cc.set_scan_group(0)
    a_orc, _ = orc.dwt(x, J)
    cand = [(ext[a] - T[a]) // 4 + 1 for a in range(2)]
    for f in range(nf):
        want = orc.scores(a_orc, cand, nb[f], mb[f], 16).ravel()
        assert np.array_equal(S[f].astype(np.int64), want), f"filter {f}"


FUSED_SCAN_CASES = [
    # SCAN_CASES index, top_k, precision
    (0, 5, 0), (1, 10, 0), (2, 16, 0), (3, 7, 0), (4, 3, 0), (5, 10, 0), (6, 4, 0), (1, 10, 1), (2, 1, 0),
]


@pytest.mark.parametrize("case", FUSED_SCAN_CASES,
                         ids=[f"{'x'.join(map(str, SCAN_CASES[c[0]][0]))}_k{c[1]}_p{c[2]}" for c in FUSED_SCAN_CASES])
def test_scan_fused_topk(cc, orc, case):
    # the selection fused into the scan: each filter's K best keys equal the
    # oracle's selection over its full score map (same tie-break keys)
    import torch
    ci, k, prec = case
    ext, T, J, nf, nfac, kind, mode = SCAN_CASES[ci]
    _say("scan fused", case)
    rng = np.random.default_rng(nf + J + 100)
    shape = ext[::-1]
    if len(ext) == 2 and min(ext) >= 60:
        x = syn.channel_image_2d(ext[0], ext[1], 8, nfac, seed=nf)
    else:
        x = rng.integers(0, nfac, size=shape).astype(np.int8)
    a_gpu, _ = cc.dwt(_t(x), J)
    nb, mb = _events(rng, T, J, nf, nfac, kind)
    real = rng.integers(0, 50, size=nf).astype(np.int32)
    step = rng.integers(0, 5000, size=nf).astype(np.int64)
    seed = 4242
    S, keys = cc.ccf_scan(ext, J, nfac - 1, a_gpu, T, _t(nb, np.int32), _t(mb, np.int32), score_mode=mode,
                          precision=prec, top_k=k, seed=seed, realization=_t(real), step=_t(step),
                          want_scores=(ci % 2 == 0))
    torch.cuda.synchronize()
    keys = keys.cpu().numpy().view(np.uint64)
    a_orc, _ = orc.dwt(x, J)
    b = 2 ** J
    cand = [(ext[a] - T[a]) // b + 1 for a in range(len(ext))]
    for f in range(nf):
        Sf = orc.scores(a_orc, cand, nb[f], mb[f], b ** len(ext), mode=mode)
        _, want = orc.select(Sf, None, k, seed, int(real[f]), int(step[f]))
        assert np.array_equal(keys[f], want), f"filter {f}"
        if S is not None:
            assert np.array_equal(S[f].cpu().numpy().astype(np.int64), Sf.ravel()), f"filter {f}"


@pytest.mark.timeout(600)
def test_scan_fused_c5_shape_full(cc, orc):
    # the fused scan at the largest batched shape (1000^2 TI, T 48, J 2, an
    # L-shaped overlap of 63 level-J blocks, 448 filters), as the benchmark
    # times it: every filter's 10 best keys against the oracle
    import torch
    p, ti, _ = wl.make("c5_learned", n_real=1)
    level, T, OV = p["level"], p["tmpl"], p["overlap"]
    b = 2 ** level
    tc = [-(-t // b) for t in T]
    nf = 448
    _say("scan fused c5 shape", nf)
    u = np.zeros((T[1], T[0]), bool)
    u[:OV[1], :] = True
    u[:, :OV[0]] = True
    pad = np.zeros((tc[1] * b, tc[0] * b), int)
    pad[:T[1], :T[0]] = u
    n_beta = pad.reshape(tc[1], b, tc[0], b).sum(axis=(1, 3))
    rng = np.random.default_rng(7)
    nb = np.broadcast_to(n_beta, (nf,) + n_beta.shape).astype(np.int32).copy()
    mb = (rng.integers(0, p["n_facies"], size=nb.shape) * nb).astype(np.int32)
    real = np.arange(nf, dtype=np.int32) % 16
    step = np.arange(nf, dtype=np.int64) * 7
    a_gpu, _ = cc.dwt(_t(ti), level)
    _, keys = cc.ccf_scan(p["ti"], level, p["n_facies"] - 1, a_gpu, T, _t(nb), _t(mb), top_k=10, seed=9,
                          realization=_t(real), step=_t(step))
    torch.cuda.synchronize()
    keys = keys.cpu().numpy().view(np.uint64)
    a_orc, _ = orc.dwt(ti, level)
    cand = [(p["ti"][a] - T[a]) // b + 1 for a in range(2)]
    for f in range(0, nf, 7):
        Sf = orc.scores(a_orc, cand, nb[f], mb[f], b * b)
        _, want = orc.select(Sf, None, 10, 9, int(real[f]), int(step[f]))
        assert np.array_equal(keys[f], want), f"filter {f}"


def test_scan_rejects_inexact_range(cc):
    x = np.zeros((64, 64), dtype=np.int8)
    a, _ = cc.dwt(_t(x), 3)   # |beta| = 64: block sums up to 64 * 126 > 2048
    nb = np.zeros((1, 2, 2), np.int32)
    with pytest.raises(cc.CcwsimError):
        cc.ccf_scan((64, 64), 3, 126, a, (16, 16), _t(nb), _t(nb))


# --------------------------------------------------------------------------
# A6 select
# --------------------------------------------------------------------------
SELECT_CASES = [(1, 5, False), (7, 10, True), (4096, 5, False), (13456, 10, True), (57121, 16, False),
                (8649, 1, True), (300, 16, True)]


@pytest.mark.parametrize("n,k,with_mis", SELECT_CASES, ids=[f"n{c[0]}_k{c[1]}_{c[2]}" for c in SELECT_CASES])
def test_select_parity(cc, orc, n, k, with_mis):
    import torch
    _say("select", n, k, with_mis)
    rng = np.random.default_rng(n + k)
    nf = 12
    S = (rng.integers(-40, 40, size=(nf, n)) * rng.integers(1, 1000, size=(nf, 1))).astype(np.int32)
    S[0] = 0                                 # one filter of pure ties (first patch)
    mis = rng.integers(0, 4, size=(nf, n)).astype(np.int16) if with_mis else None
    if with_mis:
        mis[1] = 5000                        # saturates at 4095
    real = rng.integers(0, 64, size=nf).astype(np.int32)
    step = rng.integers(0, 4000, size=nf).astype(np.int64)
    seed = 12345
    chosen, keys = cc.select(_t(S), _t(mis) if with_mis else None, k, seed, _t(real), _t(step), want_keys=True)
    chosen = chosen.cpu().numpy()
    keys = keys.cpu().numpy().view(np.uint64)
    for f in range(nf):
        c, kk = orc.select(S[f], None if mis is None else mis[f], k, seed, int(real[f]), int(step[f]))
        assert chosen[f] == c, f"filter {f}"
        assert np.array_equal(keys[f], kk), f"filter {f}"


# --------------------------------------------------------------------------
# whole path
# --------------------------------------------------------------------------
def _run(cc, p, ti, hd):
    import torch
    sim = cc.Simulator(p)
    nd = len(p["ti"])
    geo_steps = 1
    for a in range(nd):
        s = p["tmpl"][a] - p["overlap"][a]
        geo_steps *= max(1, -(-(p["grid"][a] - p["overlap"][a]) // s))
    chosen = torch.full((p["n_real"], geo_steps), -7, dtype=torch.int32, device="cuda")
    out = sim.run(_t(ti), cc.hd_to_device(hd, nd), chosen=chosen)
    torch.cuda.synchronize()
    return out.cpu().numpy(), chosen.cpu().numpy()


def _compare(cc, orc, p, ti, hd):
    out, chosen = _run(cc, p, ti, hd)
    oout, ochosen = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(chosen, ochosen), f"first differing step {np.argwhere(chosen != ochosen)[:3]}"
    assert np.array_equal(out, oout)
    return out


def _tiny(over, nhd, seed=11):
    p = dict(nc_margin=(-1, -1, -1), n_facies=3, seed=seed, score_mode=0, name="tiny")
    p.update(over)
    nd = len(p["ti"])
    if nd == 2:
        ti = syn.channel_image_2d(p["ti"][0], p["ti"][1], 4, 3, seed=21)
        ref = syn.channel_image_2d(p["grid"][0], p["grid"][1], 4, 3, seed=22)
    else:
        ti = syn.tube_image_3d(*p["ti"], 4, seed=21)
        ref = syn.tube_image_3d(*p["grid"], 4, seed=22)
        p["n_facies"] = 2
    hd = syn.sample_hard_data(ref, [nhd] * p["n_real"], seed=23) if nhd else None
    p["max_hard_data"] = 0 if hd is None else int(len(hd[0]))
    return p, ti, hd


SIM_TINY = [
    ("fixed_2d_j1", dict(ti=(40, 36), grid=(50, 47), tmpl=(10, 10), overlap=(3, 3), level=1, top_k=3,
                         path_mode=0, n_real=1, cut=1), 0),
    ("seeded_2d_j1_hd_batch", dict(ti=(48, 40), grid=(45, 52), tmpl=(12, 10), overlap=(3, 2), level=1,
                                   top_k=4, path_mode=1, n_real=6, cut=1), 30),
    ("partial_blocks_j2", dict(ti=(70, 66), grid=(61, 58), tmpl=(14, 11), overlap=(5, 3), level=2, top_k=5,
                               path_mode=1, n_real=3, cut=1), 20),
    ("level0_nocut", dict(ti=(30, 28), grid=(40, 33), tmpl=(7, 6), overlap=(2, 2), level=0, top_k=3,
                          path_mode=1, n_real=2, cut=0), 10),
    ("raw_score", dict(ti=(60, 60), grid=(64, 64), tmpl=(16, 16), overlap=(4, 4), level=1, top_k=6,
                       path_mode=0, n_real=2, cut=1, score_mode=1), 0),
    ("sequential_schedule", dict(ti=(50, 50), grid=(40, 44), tmpl=(10, 10), overlap=(6, 6), level=1,
                                 top_k=3, path_mode=1, n_real=3, cut=1), 8),
    ("one_column_lattice", dict(ti=(60, 60), grid=(20, 90), tmpl=(24, 24), overlap=(6, 6), level=1,
                                top_k=5, path_mode=1, n_real=4, cut=1), 5),
    ("single_patch", dict(ti=(40, 40), grid=(16, 16), tmpl=(16, 16), overlap=(4, 4), level=2, top_k=16,
                          path_mode=0, n_real=2, cut=1), 3),
    ("k_exceeds_candidates", dict(ti=(24, 24), grid=(40, 40), tmpl=(20, 20), overlap=(5, 5), level=1,
                                  top_k=16, path_mode=1, n_real=2, cut=1), 0),
    ("seeded_3d_j1", dict(ti=(24, 22, 16), grid=(30, 26, 18), tmpl=(8, 8, 6), overlap=(2, 2, 2), level=1,
                          top_k=4, path_mode=1, n_real=3, cut=1), 12),
    ("fixed_3d_j2", dict(ti=(40, 36, 20), grid=(44, 40, 22), tmpl=(12, 12, 8), overlap=(3, 3, 2), level=2,
                         top_k=6, path_mode=0, n_real=2, cut=1), 0),
    ("partial_blocks_j3", dict(ti=(90, 84), grid=(75, 70), tmpl=(21, 18), overlap=(6, 5), level=3, top_k=5,
                               path_mode=1, n_real=3, cut=1), 25),
    ("seeded_3d_j3", dict(ti=(40, 36, 34), grid=(36, 34, 30), tmpl=(17, 16, 16), overlap=(4, 4, 4), level=3,
                          top_k=4, path_mode=1, n_real=2, cut=1), 10),
]


@pytest.mark.parametrize("case", SIM_TINY, ids=[c[0] for c in SIM_TINY])
def test_simulate_small_cases(cc, orc, case):
    name, over, nhd = case
    _say("simulate", name)
    p, ti, hd = _tiny(over, nhd)
    out = _compare(cc, orc, p, ti, hd)
    assert out.min() >= 0


WORKLOAD_CASES = [("c1_plain2d", 1.0, None), ("c2_scale2d", 0.3, None), ("c4_batched", 0.5, 8),
                  ("c3_split3d", 0.4, None), ("c5_learned", 0.12, 2)]


@pytest.mark.parametrize("name,scale,nr", WORKLOAD_CASES, ids=[f"{c[0]}_s{c[1]}" for c in WORKLOAD_CASES])
def test_simulate_workloads_scaled(cc, orc, name, scale, nr):
    _say("workload", name, scale, nr)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    out = _compare(cc, orc, p, ti, hd)
    if hd is not None:
        for r, pos, v in zip(*hd):
            assert out[(r,) + tuple(pos[::-1])] == v


@pytest.mark.parametrize("name,nr", [("c2_scale2d", None), ("c1_plain2d", None), ("c4_batched", 16)])
def test_simulate_full_size(cc, orc, name, nr):
    # the full workload sizes, in the launch configuration the benchmark times
    _say("full", name, nr)
    p, ti, hd = wl.make(name, n_real=nr)
    out = _compare(cc, orc, p, ti, hd)
    assert out.min() >= 0
    if hd is not None:
        for r, pos, v in zip(*hd):
            assert out[(r,) + tuple(pos[::-1])] == v


# The configurations the benchmark reports, at their full sizes and in the
# launch configuration it times.  The batched calls run every realization on
# the GPU; realization r depends only on (seed, r), so a shorter oracle run
# gives realizations 0 .. n_cmp - 1 of the same batch.
FULL_BENCH_CASES = [("c5_learned", 16, 2), ("c4_batched", 64, 64), ("c3_split3d", None, None)]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name,nr,n_cmp", FULL_BENCH_CASES, ids=[c[0] for c in FULL_BENCH_CASES])
def test_simulate_full_size_bench_configs(cc, orc, name, nr, n_cmp):
    _say("full bench config", name, nr, n_cmp)
    p, ti, hd = wl.make(name, n_real=nr)
    out, chosen = _run(cc, p, ti, hd)
    q = dict(p)
    if n_cmp is not None:
        q["n_real"] = n_cmp
        if hd is not None:
            sel = hd[0] < n_cmp
            hd = (hd[0][sel], hd[1][sel], hd[2][sel])
    oout, ochosen = orc.simulate(_sp(q, orc), ti, hd)
    m = q["n_real"]
    assert np.array_equal(chosen[:m], ochosen), f"first differing step {np.argwhere(chosen[:m] != ochosen)[:3]}"
    assert np.array_equal(out[:m], oout)
    assert out.min() >= 0


@pytest.mark.timeout(600)
def test_scan_c5_shape_full(cc, orc):
    # the standalone scan at the largest batched shape (1000^2 TI, T 48,
    # J 2, an L-shaped overlap of 63 level-J blocks, 448 filters), the
    # configuration the benchmark times, against the oracle's scores
    import torch
    p, ti, _ = wl.make("c5_learned", n_real=1)
    level, T, OV = p["level"], p["tmpl"], p["overlap"]
    b = 2 ** level
    tc = [-(-t // b) for t in T]
    nf = 448
    _say("scan c5 shape", nf)
    u = np.zeros((T[1], T[0]), bool)
    u[:OV[1], :] = True
    u[:, :OV[0]] = True
    pad = np.zeros((tc[1] * b, tc[0] * b), int)
    pad[:T[1], :T[0]] = u
    n_beta = pad.reshape(tc[1], b, tc[0], b).sum(axis=(1, 3))
    rng = np.random.default_rng(7)
    nb = np.broadcast_to(n_beta, (nf,) + n_beta.shape).astype(np.int32).copy()
    mb = (rng.integers(0, p["n_facies"], size=nb.shape) * nb).astype(np.int32)
    a_gpu, _ = cc.dwt(_t(ti), level)
    S = cc.ccf_scan(p["ti"], level, p["n_facies"] - 1, a_gpu, T, _t(nb), _t(mb)).cpu().numpy()
    torch.cuda.synchronize()
    a_orc, _ = orc.dwt(ti, level)
    cand = [(p["ti"][a] - T[a]) // b + 1 for a in range(2)]
    for f in range(nf):
        want = orc.scores(a_orc, cand, nb[f], mb[f], b * b).ravel()
        assert np.array_equal(S[f].astype(np.int64), want), f"filter {f}"


def test_simulate_tile_groups(cc, orc):
    # steps wider than one tile: the scan's A operand spans the whole
    # template window and a workgroup takes 1, 2, 4 or 8 tiles, or the tuned
    # count; every choice must give the oracle's realizations
    p, ti, hd = wl.make("c4_batched", scale=0.5, n_real=40)
    _say("simulate groups", p["n_real"])
    oout, ochosen = orc.simulate(_sp(p, orc), ti, hd)
    for G in (1, 2, 4, 8, -1, 0):
        cc.set_scan_group(G)
        try:
            out, chosen = _run(cc, p, ti, hd)
        finally:
            cc.set_scan_group(0)
        assert np.array_equal(chosen, ochosen), f"G={G}: first differing step {np.argwhere(chosen != ochosen)[:3]}"
        assert np.array_equal(out, oout), f"G={G}"


def test_simulate_group_table_in_memory(cc):
    # 4,096 realizations of the batched workload put more than 64 groups of
    # two tiles into a step, so the scan reads its group table from memory
    # instead of the launch arguments; the realizations must equal those of
    # the one-tile layout (no group table), which the test above ties to the
    # oracle on the same workload
    p, ti, hd = wl.make("c4_batched", scale=0.5, n_real=4096)
    _say("group table in memory", p["n_real"])
    res = {}
    for G in (1, 2):
        cc.set_scan_group(G)
        try:
            res[G] = _run(cc, p, ti, hd)
        finally:
            cc.set_scan_group(0)
    assert np.array_equal(res[1][1], res[2][1])
    assert np.array_equal(res[1][0], res[2][0])


@pytest.mark.parametrize("name,scale,nr", [("c2_scale2d", 0.3, None), ("c3_split3d", 0.3, None),
                                           ("c1_plain2d", 1.0, None)])
def test_simulate_filter_major_scan(cc, orc, name, scale, nr):
    # the filter-major scan layout on 2D and 3D workloads with hard data
    _say("filter-major", name)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    cc.set_scan_group(-1)
    try:
        _compare(cc, orc, p, ti, hd)
    finally:
        cc.set_scan_group(0)


HD_PATH_CASES = [c for c in SIM_TINY if c[2] > 0] + [
    ("wide_margin_j2", dict(ti=(70, 66), grid=(61, 58), tmpl=(14, 11), overlap=(5, 3), level=2, top_k=5,
                            path_mode=1, n_real=3, cut=1, nc_margin=(9, 7, -1)), 60),
    ("wide_margin_3d", dict(ti=(24, 22, 16), grid=(30, 26, 18), tmpl=(8, 8, 6), overlap=(2, 2, 2), level=1,
                            top_k=4, path_mode=1, n_real=2, cut=1, nc_margin=(5, 3, 4)), 40),
]


@pytest.mark.parametrize("case", HD_PATH_CASES, ids=[c[0] for c in HD_PATH_CASES])
def test_hard_data_paths(cc, orc, case):
    # hard-data mismatches from the bit table and from the TI codes, in the
    # tile-group and filter-major scans
    name, over, nhd = case
    p, ti, hd = _tiny(over, nhd)
    oout, ochosen = orc.simulate(_sp(p, orc), ti, hd)
    for hd_direct in (0, 1):
        for G in (1, 2, -1):
            _say("hard-data paths", name, hd_direct, G)
            cc.set_scan_group(G)
            try:
                out, chosen = _run(cc, dict(p, hd_direct=hd_direct), ti, hd)
            finally:
                cc.set_scan_group(0)
            assert np.array_equal(chosen, ochosen), f"hd_direct={hd_direct} G={G}"
            assert np.array_equal(out, oout), f"hd_direct={hd_direct} G={G}"


SEL_CASES = [c for c in SIM_TINY if c[1].get("score_mode", 0) == 0]


@pytest.mark.parametrize("case", SEL_CASES, ids=[c[0] for c in SEL_CASES])
def test_row_minima_selection_small(cc, orc, case):
    # the scan writes row minima only; the K best come from exact rescoring
    # of rows in order of their minima
    name, over, nhd = case
    p, ti, hd = _tiny(over, nhd)
    oout, ochosen = orc.simulate(_sp(p, orc), ti, hd)
    for G in (1, -1, 2):
        _say("row minima", name, G)
        cc.set_selection(2)
        cc.set_scan_group(G)
        try:
            out, chosen = _run(cc, p, ti, hd)
        finally:
            cc.set_scan_group(0)
            cc.set_selection(0)
        assert np.array_equal(chosen, ochosen), f"G={G}"
        assert np.array_equal(out, oout), f"G={G}"


@pytest.mark.parametrize("name,scale,nr", WORKLOAD_CASES + [("c2_scale2d", 1.0, None)],
                         ids=[f"{c[0]}_s{c[1]}" for c in WORKLOAD_CASES] + ["c2_full"])
def test_row_minima_selection_workloads(cc, orc, name, scale, nr):
    _say("row minima workload", name, scale, nr)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    cc.set_selection(2)
    try:
        _compare(cc, orc, p, ti, hd)
    finally:
        cc.set_selection(0)


@pytest.mark.parametrize("hd_direct", [0, 1])
def test_row_minima_selection_dense(cc, orc, hd_direct):
    p, ti, hd = wl.dense_conditioning(8000, scale=0.3)
    p["hd_direct"] = hd_direct
    _say("row minima dense", hd_direct)
    cc.set_selection(2)
    try:
        _compare(cc, orc, p, ti, hd)
    finally:
        cc.set_selection(0)


def test_selection_validation(cc):
    with pytest.raises(cc.CcwsimError):
        cc.set_selection(4)


# --------------------------------------------------------------------------
# Selection fused into the scan: per candidate row only the candidates that
# can be among the row's K best keys are written
# --------------------------------------------------------------------------
def _compare_fused(cc, orc, p, ti, hd, n_cmp=None):
    cc.set_selection(3)
    try:
        out, chosen = _run(cc, p, ti, hd)
    finally:
        cc.set_selection(0)
    q = dict(p)
    if n_cmp is not None:
        q["n_real"] = n_cmp
        if hd is not None:
            sel = hd[0] < n_cmp
            hd = (hd[0][sel], hd[1][sel], hd[2][sel])
    oout, ochosen = orc.simulate(_sp(q, orc), ti, hd)
    m = q["n_real"]
    assert np.array_equal(chosen[:m], ochosen), f"first differing step {np.argwhere(chosen[:m] != ochosen)[:3]}"
    assert np.array_equal(out[:m], oout)
    return out


@pytest.mark.parametrize("case", SIM_TINY, ids=[c[0] for c in SIM_TINY])
def test_fused_selection_small(cc, orc, case):
    name, over, nhd = case
    _say("fused selection", name)
    p, ti, hd = _tiny(over, nhd)
    _compare_fused(cc, orc, p, ti, hd)


@pytest.mark.parametrize("name,scale,nr", WORKLOAD_CASES + [("c2_scale2d", 1.0, None)],
                         ids=[f"{c[0]}_s{c[1]}" for c in WORKLOAD_CASES] + ["c2_full"])
def test_fused_selection_workloads(cc, orc, name, scale, nr):
    _say("fused selection workload", name, scale, nr)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    _compare_fused(cc, orc, p, ti, hd)


@pytest.mark.timeout(900)
def test_fused_selection_c5_full(cc, orc):
    # the headline configuration: 16 realizations of 2000^2 in one call,
    # realizations 0 and 1 against the oracle
    _say("fused selection c5 full")
    p, ti, hd = wl.make("c5_learned")
    _compare_fused(cc, orc, p, ti, hd, n_cmp=2)


@pytest.mark.parametrize("n_hd", [4000, 8000])
def test_fused_selection_dense(cc, orc, n_hd):
    p, ti, hd = wl.dense_conditioning(n_hd, scale=0.3)
    _say("fused selection dense", n_hd)
    out = _compare_fused(cc, orc, p, ti, hd)
    for r, pos, v in zip(*hd):
        assert out[(r,) + tuple(pos[::-1])] == v


@pytest.mark.parametrize("case", [("c3_split3d", 0.4, None, 32, 0), ("c3_split3d", 0.4, None, 32, 1),
                                  ("c2_scale2d", 0.3, None, 16, 1), ("c4_batched", 0.5, 8, 10, 0)],
                         ids=["c3_S32_fp16", "c3_S32_bf16", "c2_S16_bf16", "c4_S10_fp16"])
def test_fused_selection_precision_split(cc, orc, case):
    import torch
    name, scale, nr, S, prec = case
    _say("fused precision", case)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    p.update(shortlist=S, precision=prec)
    cc.set_selection(3)
    try:
        sim = cc.Simulator(p)
        out = sim.run(_t(ti), cc.hd_to_device(hd, len(p["ti"])))
        torch.cuda.synchronize()
        rep = sim.report()
    finally:
        cc.set_selection(0)
    oout, _ = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(out.cpu().numpy(), oout)
    assert rep["max_abs_error"] == 0 and rep["topk_changed"] == 0


@pytest.mark.parametrize("case", [c for c in SIM_TINY if c[0] in ("partial_blocks_j2", "seeded_3d_j1",
                                                                   "seeded_2d_j1_hd_batch")],
                         ids=lambda c: c[0])
def test_fused_selection_wavelet53(cc, orc, case):
    name, over, nhd = case
    _say("fused selection 5/3", name)
    p, ti, hd = _tiny(over, nhd)
    p["wavelet"] = 1
    _compare_fused(cc, orc, p, ti, hd)


# --------------------------------------------------------------------------
# Another mother wavelet: LeGall 5/3 integer lifting
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", SIM_TINY, ids=[c[0] for c in SIM_TINY])
def test_wavelet53_small_cases(cc, orc, case):
    name, over, nhd = case
    _say("5/3", name)
    p, ti, hd = _tiny(dict(over, wavelet=1), nhd)
    _compare(cc, orc, p, ti, hd)


W53_CASES = [("c1_plain2d", 1.0, None, {}), ("c2_scale2d", 0.3, None, {}), ("c4_batched", 0.5, 8, {}),
             ("c3_split3d", 0.4, None, {"shortlist": 0}), ("c5_learned", 0.12, 2, {}),
             ("c2_scale2d", 0.3, None, {"precision": 1}), ("c2_scale2d", 1.0, None, {})]


@pytest.mark.parametrize("name,scale,nr,over", W53_CASES,
                         ids=[f"{c[0]}_s{c[1]}_{'_'.join(c[3]) or 'plain'}" for c in W53_CASES])
def test_wavelet53_workloads(cc, orc, name, scale, nr, over):
    _say("5/3 workload", name, scale, nr, over)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    p.update(over, wavelet=1)
    out = _compare(cc, orc, p, ti, hd)
    if hd is not None:
        for r, pos, v in zip(*hd):
            assert out[(r,) + tuple(pos[::-1])] == v


def test_wavelet53_scan_layouts(cc, orc):
    p, ti, hd = wl.make("c4_batched", scale=0.5, n_real=12)
    p["wavelet"] = 1
    oout, ochosen = orc.simulate(_sp(p, orc), ti, hd)
    for G in (1, 2, -1):
        cc.set_scan_group(G)
        try:
            out, chosen = _run(cc, p, ti, hd)
        finally:
            cc.set_scan_group(0)
        assert np.array_equal(chosen, ochosen) and np.array_equal(out, oout), G


def test_caches_stay_bounded_over_seeds(cc, orc):
    # one plan and one graph per seed: the caches keep at most 16 plans and
    # the graphs captured on them, and the last call still equals the oracle
    p, ti, hd = wl.make("c1_plain2d", scale=0.3)
    _say("cache bound", 40)
    cc.release_caches()
    import torch
    ti_d = _t(ti)
    for seed in range(40):
        p["seed"] = 1000 + seed
        sim = cc.Simulator(p)
        out = sim.run(ti_d)
        plans, graphs = cc.cache_counts()
        assert plans <= 16 and graphs <= 16, (plans, graphs)
    torch.cuda.synchronize()
    oout, _ = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(out.cpu().numpy(), oout)


def test_simulate_is_deterministic(cc):
    p, ti, hd = wl.make("c2_scale2d", scale=0.3)
    a, ca = _run(cc, p, ti, hd)
    b, cb = _run(cc, p, ti, hd)
    assert np.array_equal(a, b) and np.array_equal(ca, cb)


def test_simulate_rejects_bad_workspace(cc):
    import torch
    p, ti, hd = wl.make("c1_plain2d")
    q = cc.params_of(p)
    import ctypes
    out = torch.empty((1, 100, 100), dtype=torch.int8, device="cuda")
    st = cc.load().ccwsim_simulate(ctypes.byref(q), ctypes.c_void_p(_t(ti).data_ptr()), 0, None, None, None,
                                   ctypes.c_void_p(out.data_ptr()), None, None, 0, None)
    assert st == 3


def test_graph_replays_match_eager(cc, orc):
    # the captured launch sequence, replayed several times with unrelated
    # eager work and synchronisations in between, must give the eager result
    import torch
    p, ti, hd = wl.make("c4_batched", scale=0.4, n_real=4)
    nd = len(p["ti"])
    sim = cc.Simulator(p)
    ti_d = _t(ti)
    hd_d = cc.hd_to_device(hd, nd)
    cc.set_graphs(False)
    eager = sim.run(ti_d, hd_d).cpu().numpy()
    cc.set_graphs(True)
    out = torch.empty((p["n_real"],) + tuple(p["grid"][::-1]), dtype=torch.int8, device="cuda")
    for rep in range(4):
        out.fill_(-5)
        junk = torch.randn(256, 256, device="cuda") @ torch.randn(256, 256, device="cuda")
        torch.cuda.synchronize()
        sim.run(ti_d, hd_d, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {rep}"
        del junk
    oout, _ = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(eager, oout)


PRECISION_CASES = [
    # name, scale, n_real, overrides
    ("c3_split3d", 0.4, None, dict(shortlist=32, precision=0)),
    ("c3_split3d", 0.4, None, dict(shortlist=32, precision=1)),
    ("c2_scale2d", 0.3, None, dict(shortlist=16, precision=1)),
    ("c4_batched", 0.4, 4, dict(shortlist=10, precision=0)),
]


@pytest.mark.parametrize("case", PRECISION_CASES,
                         ids=[f"{c[0]}_S{c[3]['shortlist']}_p{c[3]['precision']}" for c in PRECISION_CASES])
def test_precision_split(cc, orc, case):
    # bulk scan in fp16 or bf16, exact integer rescoring of the shortlist:
    # for Haar on integer codes the bulk is exact, so the rescoring changes
    # nothing and the realization equals the oracle's exact-score one
    import torch
    name, scale, nr, over = case
    _say("precision", case)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    p.update(over)
    sim = cc.Simulator(p)
    out = sim.run(_t(ti), cc.hd_to_device(hd, len(p["ti"])))
    torch.cuda.synchronize()
    rep = sim.report()
    oout, _ = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(out.cpu().numpy(), oout)
    geo = orc.geometry(_sp(p, orc))
    npatch = p["n_real"] * geo["nsteps"]
    assert rep["max_abs_error"] == 0 and rep["topk_changed"] == 0
    assert rep["patches"] == npatch
    assert rep["rescored"] == npatch * min(p["shortlist"], geo["ncand"])


# --------------------------------------------------------------------------
# A9 learned proposer: certified bounds, so the realizations are the oracle's
# --------------------------------------------------------------------------
LEARN_CASES = [
    # workload, scale, n_real, proposer dimension
    ("c1_plain2d", 1.0, None, 8),
    ("c2_scale2d", 0.3, None, 16),
    ("c4_batched", 0.4, 6, 8),
    ("c5_learned", 0.12, 2, 32),
    ("c3_split3d", 0.3, None, 16),
]


@pytest.mark.parametrize("case", LEARN_CASES, ids=[f"{c[0]}_s{c[1]}_D{c[3]}" for c in LEARN_CASES])
def test_learned_proposer_matches_oracle(cc, orc, case):
    import torch
    name, scale, nr, D = case
    _say("learned", case)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    p = dict(p, proposer_dim=D, shortlist=0)
    sim = cc.Simulator(p)
    nd = len(p["ti"])
    steps = 1
    for a in range(nd):
        st_ = p["tmpl"][a] - p["overlap"][a]
        steps *= max(1, -(-(p["grid"][a] - p["overlap"][a]) // st_))
    chosen = torch.full((p["n_real"], steps), -7, dtype=torch.int32, device="cuda")
    out = sim.run(_t(ti), cc.hd_to_device(hd, nd), chosen=chosen)
    torch.cuda.synchronize()
    rep = sim.report()
    oout, ochosen = orc.simulate(_sp(p, orc), ti, hd)
    got_c = chosen.cpu().numpy()
    assert np.array_equal(got_c, ochosen), f"first differing step {np.argwhere(got_c != ochosen)[:3]}"
    assert np.array_equal(out.cpu().numpy(), oout)
    assert rep["proposer_patches"] == p["n_real"] * steps
    rows = (p["ti"][1] - p["tmpl"][1]) // 2 ** p["level"] + 1
    if nd == 3:
        rows *= (p["ti"][2] - p["tmpl"][2]) // 2 ** p["level"] + 1
    # every patch rescored at least one row and never more than all of them
    assert rep["proposer_patches"] <= rep["proposer_rows"] <= rep["proposer_patches"] * rows


SKEW_CASES = [("c2_scale2d", 0.3, None, 16, 1.0), ("c5_learned", 0.12, 2, 32, 2.0), ("c4_batched", 0.4, 6, 8, 0.5)]


@pytest.mark.parametrize("case", SKEW_CASES, ids=[f"{c[0]}_D{c[3]}_skew{c[4]}" for c in SKEW_CASES])
def test_certified_proposer_with_a_skewed_basis(cc, orc, case):
    # the bound is a lower bound for any basis: with rows that are neither
    # orthogonal nor normalised the realizations are still the oracle's
    name, scale, nr, D, skew = case
    _say("certified proposer, skewed basis", case)
    p, ti, hd = wl.make(name, scale=scale, n_real=nr)
    p = dict(p, proposer_dim=D, shortlist=0)
    cc.set_proposer_skew(skew)
    try:
        sim = cc.Simulator(p)
        out = sim.run(_t(ti), cc.hd_to_device(hd, len(p["ti"])))
        out = out.cpu().numpy()
    finally:
        cc.set_proposer_skew(0.0)
    oout, _ = orc.simulate(_sp(p, orc), ti, hd)
    assert np.array_equal(out, oout)


# --------------------------------------------------------------------------
# Dense conditioning and the level x grid-size cases
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n_hd", [4000, 8000])
@pytest.mark.parametrize("hd_direct", [0, 1])
def test_dense_conditioning(cc, orc, n_hd, hd_direct):
    p, ti, hd = wl.dense_conditioning(n_hd, scale=0.3)
    p["hd_direct"] = hd_direct
    _say("dense", n_hd, len(hd[0]), hd_direct)
    out = _compare(cc, orc, p, ti, hd)
    for r, pos, v in zip(*hd):
        assert out[(r,) + tuple(pos[::-1])] == v


@pytest.mark.parametrize("level,grid_n", [(1, 128), (2, 160), (3, 128), (3, 200)])
def test_level_grid_cases(cc, orc, level, grid_n):
    p, ti, hd = wl.level_grid_case(level, grid_n)
    _say("level x grid", level, grid_n)
    out = _compare(cc, orc, p, ti, hd)
    for r, pos, v in zip(*hd):
        assert out[(r,) + tuple(pos[::-1])] == v
