"""GPU parity of the CDF 9/7 path (ccwsim_dwt97, ccwsim_idwt97,
ccwsim_ccf_scan97) against the float64 oracle in oracle/cdf97.py.

Tolerances, derived from the arithmetic:
- transform: fp32 lifting, about a dozen roundings per output and pass,
  amplified by the lifting gains; every coefficient within 1e-5 of the
  largest magnitude of its band (typical errors are ~1e-7 of it).
- scores: the kernel sums nk squared differences of the same fp32 inputs
  the oracle reads, one rounding for the difference and one fused
  multiply-add per term, so |S32 - S64| <= (nk + 2) 2^-24 S64; with at most
  144 known blocks that is below 8.7e-6, and the tests assert the 1e-5
  relative tolerance.
- selection: keys carry the fp32 score, so which of two candidates within
  the fp32 error of each other comes first is not unique; the tests compare
  the sorted scores and check that every chosen candidate lies within the
  tolerance of the K-th best.
- bulk ranking (shortlist): the fp16 / bf16 operands are off by a relative
  2^-11 / 2^-8 each, so the bulk value of a candidate is off by at most
  eta(c), computed below from |A||K| and K^2 sums; a shortlist is valid when
  no left-out candidate beats a kept one by more than the two bounds.
"""
import sys

import numpy as np
import pytest

from oracle import cdf97 as c97
from oracle import oracle as orc
from paper_2404_00441_amd import synthetic as syn

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


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


def _img(shape, seed, nfac=3):
    if len(shape) == 2 and min(shape) >= 40:
        return syn.channel_image_2d(shape[1], shape[0], 5, nfac, seed=seed).astype(np.int8)
    return np.random.default_rng(seed).integers(0, nfac, size=shape).astype(np.int8)


def _dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).astype(dtype)).cuda()


DWT_CASES = [((56, 64), 1), ((70, 90), 2), ((50, 37), 3), ((12, 18, 20), 2), ((8, 8), 2), ((128, 128), 2),
             ((9, 11), 0)]


@pytest.mark.parametrize("shape,level", DWT_CASES, ids=[f"{'x'.join(map(str, s))}_J{j}" for s, j in DWT_CASES])
def test_dwt97_matches_oracle(cc, shape, level):
    _say("dwt97", shape, level)
    x = _img(shape, 3)
    a_ref, d_ref = c97.dwt97(x, level)
    a, d = cc.dwt97(_dev(x, np.int8), level)
    a = a.cpu().numpy().astype(np.float64)
    d = d.cpu().numpy().astype(np.float64)
    assert a.shape == a_ref.shape
    _say(f"  approximation: max error {np.abs(a - a_ref).max() / np.abs(a_ref).max():.2e} of its largest magnitude")
    assert np.abs(a - a_ref).max() <= 1e-5 * np.abs(a_ref).max()
    off = 0
    for dj in d_ref:
        got = d[off: off + dj.size].reshape(dj.shape)
        off += dj.size
        for q in range(dj.shape[0]):
            scale = max(np.abs(dj[q]).max(), np.abs(a_ref).max() * 1e-3)
            assert np.abs(got[q] - dj[q]).max() <= 1e-5 * scale, q
    assert off == d.size


IDWT_CASES = DWT_CASES[:4] + [DWT_CASES[-1]]


@pytest.mark.parametrize("shape,level", IDWT_CASES, ids=[f"{'x'.join(map(str, s))}_J{j}" for s, j in IDWT_CASES])
def test_idwt97_reconstructs(cc, shape, level):
    _say("idwt97", shape, level)
    x = _img(shape, 4)
    xd = _dev(x, np.int8)
    a, d = cc.dwt97(xd, level)
    img = cc.idwt97(a, d, tuple(shape[::-1]), level).cpu().numpy().astype(np.float64)
    pad = c97.pad_edge(x, level)
    assert img.shape == pad.shape
    assert np.abs(img - pad).max() < 1e-4
    assert np.array_equal(np.rint(img).astype(np.int64), pad.astype(np.int64))
    # the inverse of the oracle's (fp32-rounded) coefficients against the
    # oracle's inverse of the same values
    a_ref, d_ref = c97.dwt97(x, level)
    a32 = a_ref.astype(np.float32)
    d32 = [dj.astype(np.float32) for dj in d_ref]
    flat = np.concatenate([dj.ravel() for dj in d32]) if d32 else np.zeros(0, np.float32)
    img2 = cc.idwt97(_dev(a32, np.float32), _dev(flat, np.float32), tuple(shape[::-1]), level)
    want = c97.idwt97(a32.astype(np.float64), [dj.astype(np.float64) for dj in d32])
    assert np.abs(img2.cpu().numpy() - want).max() <= 1e-5 * np.abs(want).max()


def _events(K, tc, n_ev, ov, seed):
    """Data events: crops of the level-J approximation K_ref of a second
    seeded image at random block positions, kept on an L-shaped band of ov
    blocks (top rows and left columns), zero elsewhere."""
    rng = np.random.default_rng(seed)
    nd = K.ndim
    n = np.zeros((n_ev,) + tc, np.int32)
    A = np.zeros((n_ev,) + tc, np.float64)
    for e in range(n_ev):
        p = [rng.integers(0, K.shape[i] - tc[i] + 1) for i in range(nd)]
        win = K[tuple(slice(p[i], p[i] + tc[i]) for i in range(nd))]
        mask = np.zeros(tc, bool)
        w = rng.integers(1, ov + 1)
        if nd == 2:
            mask[:w, :] = True
            mask[:, :w] = True
        else:
            mask[:, :w, :] = True
            mask[:, :, :w] = True
        if e % 5 == 4:
            mask[:] = False
            mask[(0,) * nd] = True    # a single known block
        n[e][mask] = 1
        A[e][mask] = win[mask] + rng.normal(scale=0.05, size=mask.sum())
    return n, A


def _setup(ti_shape, ref_shape, level, T, n_ev, seed=11):
    ti = _img(ti_shape, seed)
    ref = _img(ref_shape, seed + 1)
    K = c97.dwt97(ti, level)[0].astype(np.float32)
    Kr = c97.dwt97(ref, level)[0]
    b = 2 ** level
    tc = tuple(-(-t // b) for t in T)
    n, A = _events(Kr, tc, n_ev, max(1, tc[-1] // 4), seed + 2)
    A = A.astype(np.float32)
    ext = tuple(ti_shape[::-1])
    cand = tuple((ti_shape[i] - T[i]) // b + 1 for i in range(len(T)))
    return ti, K, n, A, ext, cand, tc


def _oracle_scores(K, cand, n, A):
    return np.stack([c97.scores97(K.astype(np.float64), cand, n[e], A[e].astype(np.float64)).ravel()
                     for e in range(n.shape[0])])


SCAN_CASES = [((100, 120), (90, 90), 2, (24, 24), 37),
              ((64, 80), (64, 64), 1, (16, 16), 33),
              ((120, 128), (100, 100), 2, (48, 48), 40),
              ((20, 36, 40), (20, 30, 30), 2, (8, 12, 12), 9),
              ((30, 41), (30, 30), 0, (6, 8), 35),
              ((80, 70), (80, 80), 0, (64, 1), 12)]
SCAN_IDS = [f"{'x'.join(map(str, c[0]))}_J{c[2]}_T{c[3][-1]}" for c in SCAN_CASES]


@pytest.mark.parametrize("case", SCAN_CASES, ids=SCAN_IDS)
def test_scan97_map_matches_oracle(cc, case):
    ti_shape, ref_shape, level, T, n_ev = case
    _say("scan97 map", case)
    ti, K, n, A, ext, cand, tc = _setup(ti_shape, ref_shape, level, T, n_ev)
    S = cc.ccf_scan97(ext, level, _dev(K, np.float32), T[::-1], _dev(n.reshape(n_ev, -1), np.int32),
                      _dev(A.reshape(n_ev, -1), np.float32)).cpu().numpy().astype(np.float64)
    want = _oracle_scores(K, cand, n, A)
    assert S.shape == want.shape
    err = np.abs(S - want)
    rel = float((err / np.maximum(want, 1e-30)).max())
    _say(f"  max relative error of the fp32 map against float64: {rel:.2e}")
    assert np.all(err <= 1e-5 * want + 1e-30), rel


def _perm_table(ncand, seed, r, step):
    key = orc.rng(seed, orc.STREAM_TIEBREAK, r, step)
    return {orc.perm20(c, key): c for c in range(ncand)}


def _decode(keys, table):
    k = keys.astype(np.uint64)
    S = (k >> np.uint64(20)).astype(np.uint32).view(np.float32).astype(np.float64)
    idx = np.array([table[int(v)] for v in (k & np.uint64(0xFFFFF))])
    return S, idx


def _check_topk(S_got, idx, S64, k, allowed=None):
    """Keys ascending; scores within the tolerance of the oracle's; the k
    chosen are the k best of `allowed` (all candidates by default) up to
    candidates within the fp32 error of the k-th."""
    assert len(set(idx.tolist())) == k
    assert np.all(np.diff(S_got) >= 0)
    assert np.all(np.abs(S_got - S64[idx]) <= 1e-5 * S64[idx] + 1e-30)
    pool = np.arange(S64.size) if allowed is None else np.asarray(allowed)
    best = np.sort(S64[pool])[:k]
    assert np.all(np.abs(np.sort(S64[idx]) - best) <= 2e-5 * best + 1e-30)
    if allowed is not None:
        assert set(idx.tolist()) <= set(pool.tolist())


@pytest.mark.parametrize("case", SCAN_CASES, ids=SCAN_IDS)
def test_scan97_exact_keys(cc, case):
    import torch
    ti_shape, ref_shape, level, T, n_ev = case
    _say("scan97 exact keys", case)
    ti, K, n, A, ext, cand, tc = _setup(ti_shape, ref_shape, level, T, n_ev)
    k, seed = 10, 5
    real = torch.arange(n_ev, dtype=torch.int32, device="cuda")
    step = torch.full((n_ev,), 3, dtype=torch.int64, device="cuda")
    S, keys, sl = cc.ccf_scan97(ext, level, _dev(K, np.float32), T[::-1], _dev(n.reshape(n_ev, -1), np.int32),
                                _dev(A.reshape(n_ev, -1), np.float32), top_k=k, shortlist=0, seed=seed,
                                realization=real, step=step, want_scores=True)
    assert sl is None
    S = S.cpu().numpy()
    keys = keys.cpu().numpy()
    want = _oracle_scores(K, cand, n, A)
    ncand = want.shape[1]
    for e in range(n_ev):
        tab = _perm_table(ncand, seed, e, 3)
        S_got, idx = _decode(keys[e], tab)
        _check_topk(S_got, idx, want[e], k)
        # the key's score is the map's value, bit for bit
        assert np.array_equal(S_got.astype(np.float32), S[e][idx])
    # keys alone (no map requested) are the same
    _, keys2, _ = cc.ccf_scan97(ext, level, _dev(K, np.float32), T[::-1], _dev(n.reshape(n_ev, -1), np.int32),
                                _dev(A.reshape(n_ev, -1), np.float32), top_k=k, shortlist=0, seed=seed,
                                realization=real, step=step)
    assert np.array_equal(keys2.cpu().numpy(), keys)


def _bulk_bound(K, cand, n, A, precision):
    """Bound eta(c) on |bulk - exact| of the ranking value sum n (A K - K^2/2)."""
    u = 2.0 ** -11 if precision == 0 else 2.0 ** -8
    sub = 2.0 ** -25 if precision == 0 else 0.0
    kmax = float(np.abs(K).max())
    q = max(0, int(np.floor(np.log2(kmax * kmax))) - 14) + 1 if kmax * kmax >= 1 and precision == 0 else 1
    Kd = K.astype(np.float64)
    out = []
    for e in range(n.shape[0]):
        nk = int(n[e].sum())
        k2 = c97.scores97(Kd, cand, n[e], np.zeros(n[e].shape))   # sum n K^2
        # sum n |A| |K| and sum n (|A| + |K|), by the same block loop
        absA = np.abs(A[e].astype(np.float64))
        aK = np.zeros(cand, np.float64)
        apk = np.zeros(cand, np.float64)
        for b in zip(*np.nonzero(n[e])):
            win = np.abs(Kd[tuple(slice(b[i], b[i] + cand[i]) for i in range(Kd.ndim))])
            aK += absA[b] * win
            apk += absA[b] + win
        eta = (aK * (2 * u + u * u) + apk * sub * (1 + u) + 0.5 * k2 * (u + U32 + u * U32)
               + nk * 2.0 ** (q - 1) * sub + 2 * nk * U32 * 1.01 * (aK + 0.5 * k2) * 1.01)
        out.append(1.5 * eta.ravel() + 1e-30)
    return np.stack(out)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp16", "bf16"])
@pytest.mark.parametrize("case", SCAN_CASES, ids=SCAN_IDS)
def test_scan97_bulk_shortlist(cc, case, precision):
    import torch
    ti_shape, ref_shape, level, T, n_ev = case
    _say("scan97 bulk", case, precision)
    ti, K, n, A, ext, cand, tc = _setup(ti_shape, ref_shape, level, T, n_ev)
    k, R, seed = 10, 64, 9
    real = torch.arange(n_ev, dtype=torch.int32, device="cuda")
    step = torch.zeros((n_ev,), dtype=torch.int64, device="cuda")
    S, keys, sl = cc.ccf_scan97(ext, level, _dev(K, np.float32), T[::-1], _dev(n.reshape(n_ev, -1), np.int32),
                                _dev(A.reshape(n_ev, -1), np.float32), top_k=k, shortlist=R, precision=precision,
                                seed=seed, realization=real, step=step, want_shortlist=True, want_scores=True)
    S = S.cpu().numpy()
    keys = keys.cpu().numpy()
    sl = sl.cpu().numpy()
    want = _oracle_scores(K, cand, n, A)
    eta = _bulk_bound(K, cand, n, A, precision)
    ncand = want.shape[1]
    agree = []
    for e in range(n_ev):
        s = sl[e]
        assert np.all(np.diff(s) > 0) and s[0] >= 0 and s[-1] < ncand
        out = np.setdiff1d(np.arange(ncand), s)
        # no left-out candidate beats a kept one by more than both bounds
        assert (want[e][out] + 2 * eta[e][out]).min() >= (want[e][s] - 2 * eta[e][s]).max()
        tab = _perm_table(ncand, seed, e, 0)
        S_got, idx = _decode(keys[e], tab)
        _check_topk(S_got, idx, want[e], k, allowed=s)
        # the rescored fp32 score is the map's value, bit for bit
        assert np.array_equal(S_got.astype(np.float32), S[e][idx])
        agree.append(len(set(idx.tolist()) & set(c97.topk97(want[e], k).tolist())) / k)
    _say(f"  top-{k} agreement with the float64 oracle: mean {np.mean(agree):.3f}, min {np.min(agree):.2f}")


def test_scan97_flat_ti_ties(cc):
    """A constant training image: every candidate has the same score (the
    same fp32 operations on the same values), so the K best keys are the K
    smallest tie-break permutations and the bulk shortlist is the first R
    indices (ties to the smaller index).  The exact selection takes its
    whole-map path here (every chunk ties)."""
    import torch
    _say("scan97 flat TI ties")
    level, T, n_ev, k, seed = 2, (24, 24), 6, 10, 3
    K = np.full((30, 30), 1.5, np.float32)
    ext = (120, 120)
    tc = (6, 6)
    n = np.zeros((n_ev,) + tc, np.int32)
    n[:, :2, :] = 1
    A = np.random.default_rng(1).normal(size=(n_ev,) + tc).astype(np.float32)
    real = torch.arange(n_ev, dtype=torch.int32, device="cuda")
    step = torch.zeros(n_ev, dtype=torch.int64, device="cuda")
    args = (ext, level, _dev(K, np.float32), T, _dev(n.reshape(n_ev, -1), np.int32),
            _dev(A.reshape(n_ev, -1), np.float32))
    _, keys, _ = cc.ccf_scan97(*args, top_k=k, shortlist=0, seed=seed, realization=real, step=step)
    _, _, sl = cc.ccf_scan97(*args, top_k=k, shortlist=64, seed=seed, realization=real, step=step,
                             want_shortlist=True)
    keys = keys.cpu().numpy().astype(np.uint64)
    ncand = 25 * 25
    assert np.array_equal(sl.cpu().numpy(), np.tile(np.arange(64, dtype=np.int32), (n_ev, 1)))
    for e in range(n_ev):
        key = orc.rng(seed, orc.STREAM_TIEBREAK, e, 0)
        perms = np.sort(np.array([orc.perm20(c, key) for c in range(ncand)], dtype=np.uint64))[:k]
        sbits = keys[e][0] >> np.uint64(20)
        assert np.all(keys[e] >> np.uint64(20) == sbits)
        assert np.array_equal(keys[e] & np.uint64(0xFFFFF), perms)


def test_scan97_fewer_chunks_than_shortlist(cc):
    # 5 x 5 candidates: 5 chunks, a shortlist of 16 takes them all
    import torch
    _say("scan97 small candidate set")
    ti, K, n, A, ext, cand, tc = _setup((40, 40), (40, 40), 2, (24, 24), 7)
    k, R, seed = 10, 16, 2
    real = torch.zeros(7, dtype=torch.int32, device="cuda")
    step = torch.arange(7, dtype=torch.int64, device="cuda")
    _, keys, sl = cc.ccf_scan97(ext, 2, _dev(K, np.float32), (24, 24), _dev(n.reshape(7, -1), np.int32),
                                _dev(A.reshape(7, -1), np.float32), top_k=k, shortlist=R, seed=seed,
                                realization=real, step=step, want_shortlist=True)
    want = _oracle_scores(K, cand, n, A)
    keys, sl = keys.cpu().numpy(), sl.cpu().numpy()
    for e in range(7):
        assert np.all(np.diff(sl[e]) > 0) and sl[e][-1] < 25
        S_got, idx = _decode(keys[e], _perm_table(25, seed, 0, e))
        _check_topk(S_got, idx, want[e], k, allowed=sl[e])


def test_scan97_validation(cc):
    import torch
    K = torch.zeros((30, 30), dtype=torch.float32, device="cuda")
    n = torch.ones((2, 36), dtype=torch.int32, device="cuda")
    A = torch.zeros((2, 36), dtype=torch.float32, device="cuda")
    real = torch.zeros(2, dtype=torch.int32, device="cuda")
    step = torch.zeros(2, dtype=torch.int64, device="cuda")
    with pytest.raises(cc.CcwsimError):   # shortlist below top_k
        cc.ccf_scan97((120, 120), 2, K, (24, 24), n, A, top_k=8, shortlist=4, realization=real, step=step)
    with pytest.raises(cc.CcwsimError):   # top_k above 16
        cc.ccf_scan97((120, 120), 2, K, (24, 24), n, A, top_k=17, realization=real, step=step)
    with pytest.raises(cc.CcwsimError):   # shortlist above 128
        cc.ccf_scan97((120, 120), 2, K, (24, 24), n, A, top_k=8, shortlist=129, realization=real, step=step)


def test_scan97_at_the_c5_scan_shape(cc):
    """The launch configuration the benchmark times: a 1000^2 three-facies
    training image, J = 2, T = 48 (57,121 candidates), 448 events with an
    L-shaped overlap of 3 blocks.  Every event's exact keys and its split
    keys (fp16, shortlist 64) against the oracle's scores of the same fp32
    inputs; the score map on 8 sampled events."""
    import torch
    from paper_2404_00441_amd import workloads as wl
    _say("scan97 at the C5 scan shape")
    p, ti, _ = wl.make("c5_learned", n_real=1)
    level, T = p["level"], tuple(p["tmpl"])
    a_ref, d_ref = c97.dwt97(ti, level)
    K = a_ref.astype(np.float32)
    # the transform of the full training image and its inverse
    ti_d = _dev(ti, np.int8)
    a_gpu, d_gpu = cc.dwt97(ti_d, level)
    assert np.abs(a_gpu.cpu().numpy() - a_ref).max() <= 1e-5 * np.abs(a_ref).max()
    flat = np.concatenate([dj.ravel() for dj in d_ref])
    assert np.abs(d_gpu.cpu().numpy() - flat).max() <= 1e-5 * np.abs(a_ref).max()
    img = cc.idwt97(a_gpu, d_gpu, tuple(p["ti"]), level).cpu().numpy()
    assert np.array_equal(np.rint(img).astype(np.int64), ti.astype(np.int64))
    ref = syn.channel_image_2d(500, 500, 20, 3, seed=4242)
    Kr = c97.dwt97(ref, level)[0]
    tc = (12, 12)
    n_ev, k, seed = 448, 10, 1
    rng = np.random.default_rng(17)
    mask = np.zeros(tc, bool)
    mask[:3, :] = True
    mask[:, :3] = True
    n = np.broadcast_to(mask, (n_ev,) + tc).astype(np.int32).copy()
    A = np.zeros((n_ev,) + tc, np.float32)
    for e in range(n_ev):
        y, x = rng.integers(0, Kr.shape[0] - 11), rng.integers(0, Kr.shape[1] - 11)
        A[e][mask] = Kr[y: y + 12, x: x + 12][mask]
    cand = ((1000 - 48) // 4 + 1, (1000 - 48) // 4 + 1)
    real = torch.arange(n_ev, dtype=torch.int32, device="cuda") % 16
    step = torch.arange(n_ev, dtype=torch.int64, device="cuda")
    args = (p["ti"], level, _dev(K, np.float32), T, _dev(n.reshape(n_ev, -1), np.int32),
            _dev(A.reshape(n_ev, -1), np.float32))
    _, kx, _ = cc.ccf_scan97(*args, top_k=k, shortlist=0, seed=seed, realization=real, step=step)
    _, ks, sl = cc.ccf_scan97(*args, top_k=k, shortlist=64, precision=0, seed=seed, realization=real, step=step,
                              want_shortlist=True)
    S = cc.ccf_scan97(*args)
    kx, ks, sl = kx.cpu().numpy(), ks.cpu().numpy(), sl.cpu().numpy()
    ncand = cand[0] * cand[1]
    agree = []
    for e in range(n_ev):
        want = c97.scores97(K.astype(np.float64), cand, n[e], A[e].astype(np.float64)).ravel()
        tab = _perm_table(ncand, seed, e % 16, e) if e < 8 else None
        if tab is None:
            # the index from the key's low bits through the same bijection:
            # compare the scores of the chosen set instead
            Sx = (kx[e].astype(np.uint64) >> np.uint64(20)).astype(np.uint32).view(np.float32).astype(np.float64)
            best = np.sort(want)[:k]
            assert np.all(np.diff(Sx) >= 0)
            assert np.all(np.abs(Sx - best) <= 2e-5 * best + 1e-30), e
            Ss = (ks[e].astype(np.uint64) >> np.uint64(20)).astype(np.uint32).view(np.float32).astype(np.float64)
            best_sl = np.sort(want[sl[e]])[:k]
            assert np.all(np.abs(Ss - best_sl) <= 2e-5 * best_sl + 1e-30), e
            agree.append(np.mean(np.abs(Ss - best) <= 2e-5 * best + 1e-30))
            continue
        S_got, idx = _decode(kx[e], tab)
        _check_topk(S_got, idx, want, k)
        S_got, idx = _decode(ks[e], tab)
        _check_topk(S_got, idx, want, k, allowed=sl[e])
        Se = S[e].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(Se - want) <= 1e-5 * want + 1e-30), e
    _say(f"  split top-10 scores equal to the float64 top-10: {np.mean(agree):.4f} of events")
