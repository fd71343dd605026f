"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a
published known-answer vector, a closed form, an invariant, a library
routine on a special case, or brute force on tiny inputs (``bruteforce.py``).
"""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import signal

from paper_2404_00441_amd import synthetic as syn
from paper_2404_00441_amd import workloads as wl
from tests import bruteforce as bf

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------
def test_splitmix64_known_answers(orc):
    with open(os.path.join(GOLD, "splitmix64_kat.txt")) as f:
        kat = [int(l, 16) for l in f if l.strip() and not l.startswith("#")]
    golden = 0x9E3779B97F4A7C15
    state = 0
    for want in kat:
        # the oracle exposes "first output from state x"; the published
        # sequence advances the state by the golden increment per output
        assert orc.splitmix_first(state) == want
        state = (state + golden) % 2 ** 64


def test_rng_streams_distinct(orc):
    vals = {orc.rng(1, s, a, b) for s in range(1, 4) for a in range(8) for b in range(8)}
    assert len(vals) == 3 * 64
    # swapping the two counters must change the value
    assert orc.rng(5, 2, 1, 0) != orc.rng(5, 2, 0, 1)


def test_perm20_is_bijection(orc):
    for key in (0, 0x123456789ABCDEF, 2 ** 64 - 1):
        seen = np.zeros(1 << 20, dtype=bool)
        vals = np.fromiter((orc.perm20(x, key) for x in range(1 << 20)), dtype=np.int64,
                           count=1 << 20)
        assert vals.min() >= 0 and vals.max() < (1 << 20)
        seen[vals] = True
        assert seen.all()


def test_draw_is_uniform_over_k(orc):
    # the draw index j = floor(u32 * k / 2^32) must be uniform over 0..k-1
    k, n = 10, 20000
    counts = np.zeros(k, dtype=np.int64)
    for step in range(n):
        u = orc.rng(7, 3, 0, step) >> 32
        counts[(u * k) >> 32] += 1
    expected = n / k
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    assert chi2 < 30.0  # 9 dof, p ~ 4e-4


# --------------------------------------------------------------------------
# Haar DWT
# --------------------------------------------------------------------------
def _edge_pad(x, b):
    pads = [(0, (-s) % b) for s in x.shape]
    return np.pad(x, pads, mode="edge")


def _block_sums(x, b):
    xp = _edge_pad(x, b).astype(np.int64)
    if x.ndim == 2:
        ny, nx = xp.shape
        return xp.reshape(ny // b, b, nx // b, b).sum(axis=(1, 3))
    nz, ny, nx = xp.shape
    return xp.reshape(nz // b, b, ny // b, b, nx // b, b).sum(axis=(1, 3, 5))


@pytest.mark.parametrize("shape,J", [((13, 17), 1), ((20, 24), 2), ((31, 9), 3), ((7, 6, 10), 1),
                                     ((9, 12, 14), 2)])
def test_dwt_approx_is_block_sum(orc, shape, J):
    # Haar scaling function = box (Sec. 4.2): the level-J approximation is the
    # block sum (times 2^(-dJ/2) in orthonormal units)
    rng = np.random.default_rng(1)
    x = rng.integers(0, 3, size=shape).astype(np.int8)
    a, _ = orc.dwt(x, J)
    assert np.array_equal(a, _block_sums(x, 2 ** J))


def test_dwt_worked_size_example(orc):
    # Sec. 4.3: 2000 x 2000 at level 3 -> 250 x 250 = 62,500 coefficients
    with open(os.path.join(GOLD, "paper_facts.json")) as f:
        facts = json.load(f)
    ex = facts["worked_size_example"]
    x = np.zeros(tuple(ex["ti"]), dtype=np.int8)
    a, det = orc.dwt(x, ex["level"])
    assert list(a.shape) == ex["approx"] and a.size == ex["approx_cells"]
    # Sec. 3.1: each sub-band is 1/4^j of the image
    for j, d in enumerate(det, start=1):
        assert d.shape[0] == 3
        assert d[0].size == x.size * facts["subband_fraction"]["per_level_fraction_2d"] ** j


def test_dwt_signs_on_one_block(orc):
    # 2x2 image [[p, q], [r, s]] (rows y): with the Haar wavelet +1 on the first
    # half and -1 on the second (Sec. 4.2), integer form:
    #   x-detail = (p - q) + (r - s); y-detail = (p + q) - (r + s);
    #   diagonal = (p - q) - (r - s); approximation = p + q + r + s
    p, q, r, s = 5, 1, 2, 7
    a, det = orc.dwt(np.array([[p, q], [r, s]], dtype=np.int8), 1)
    assert int(a[0, 0]) == p + q + r + s
    d = det[0][:, 0, 0]
    assert list(d) == [(p - q) + (r - s), (p + q) - (r + s), (p - q) - (r - s)]


@pytest.mark.parametrize("shape,J", [((16, 16), 2), ((12, 20), 1), ((8, 8, 8), 2), ((6, 10, 4), 1)])
def test_dwt_parseval(orc, shape, J):
    # orthonormal basis (Sec. 3.1): energy is preserved.  Integer coefficients
    # after p passes are 2^(p/2) times the orthonormal ones, so
    #   2^(dJ) sum x^2 = sum a^2 + sum_j 2^(d(J-j)) sum d_j^2
    rng = np.random.default_rng(2)
    x = rng.integers(0, 3, size=shape).astype(np.int8)
    d = x.ndim
    a, det = orc.dwt(x, J)
    lhs = (2 ** (d * J)) * int((x.astype(np.int64) ** 2).sum())
    rhs = int((a ** 2).sum()) + sum((2 ** (d * (J - j))) * int((dj ** 2).sum())
                                   for j, dj in enumerate(det, start=1))
    assert lhs == rhs


@pytest.mark.parametrize("shape,J", [((16, 16), 2), ((13, 17), 1), ((21, 11), 3), ((9, 12, 14), 2),
                                     ((5, 7, 6), 1)])
def test_idwt_perfect_reconstruction(orc, shape, J):
    # bijective filters (Sec. 3.1): IDWT(DWT(x)) == x (on the extended image)
    rng = np.random.default_rng(3)
    x = rng.integers(0, 3, size=shape).astype(np.int8)
    a, det = orc.dwt(x, J)
    full = orc.idwt_region(a, det, x.shape[::-1], J, [0] * x.ndim, list(a.shape[::-1]))
    assert np.array_equal(full, _edge_pad(x, 2 ** J))


def test_idwt_region_is_crop(orc):
    # Sec. 3.2 / Algorithm 1 "Inv-DWT": the pattern rebuilt from a block range
    # of coefficients is the TI crop there
    rng = np.random.default_rng(4)
    x = syn.channel_image_2d(64, 48, 4, 3, seed=9)
    for J in (1, 2):
        a, det = orc.dwt(x, J)
        b = 2 ** J
        for _ in range(10):
            nc = [int(rng.integers(1, 5)), int(rng.integers(1, 5))]
            c0 = [int(rng.integers(0, a.shape[1] - nc[0] + 1)), int(rng.integers(0, a.shape[0] - nc[1] + 1))]
            reg = orc.idwt_region(a, det, x.shape[::-1], J, c0, nc)
            want = _edge_pad(x, b)[c0[1] * b:(c0[1] + nc[1]) * b, c0[0] * b:(c0[0] + nc[0]) * b]
            assert np.array_equal(reg, want)


# --------------------------------------------------------------------------
# CCW score
# --------------------------------------------------------------------------
def _random_event(rng, T, J, ndim, ncode):
    """Random overlap mask over a T^d window and its data values."""
    b = 2 ** J
    tc = [(t + b - 1) // b for t in T]
    mask = rng.random(T[::-1]) < rng.uniform(0.2, 0.9)
    vals = rng.integers(0, ncode, size=T[::-1])
    nb = np.zeros(tc[::-1], dtype=np.int64)
    mb = np.zeros(tc[::-1], dtype=np.int64)
    for u in itertools.product(*[range(t) for t in T[::-1]]):
        if mask[u]:
            bk = tuple(ui // b for ui in u)
            nb[bk] += 1
            mb[bk] += vals[u]
    return mask, vals, nb, mb


@pytest.mark.parametrize("J", [0, 1, 2])
@pytest.mark.parametrize("ndim", [2, 3])
def test_score_equals_spatial_ssd_of_block_means(orc, J, ndim):
    # S(c) + |b|^2 sum m^2/n == |b|^2 sum_{u in OR} (mean_TI(u) - mean_OR(u))^2,
    # the wavelet-domain CCF against a brute-force spatial-domain SSD
    rng = np.random.default_rng(10 + J + 10 * ndim)
    b = 2 ** J
    for trial in range(6 if ndim == 2 else 3):
        if ndim == 2:
            Nti = [int(rng.integers(8, 17)), int(rng.integers(8, 17))]
            T = [int(rng.integers(2, 8)), int(rng.integers(2, 8))]
        else:
            Nti = [int(rng.integers(6, 10)) for _ in range(3)]
            T = [int(rng.integers(2, 5)) for _ in range(3)]
        T = [min(t, n) for t, n in zip(T, Nti)]
        ti = rng.integers(0, 3, size=Nti[::-1]).astype(np.int8)
        a, _ = orc.dwt(ti, J)
        mask, vals, nb, mb = _random_event(rng, T, J, ndim, 3)
        cand = [(Nti[k] - T[k]) // b + 1 for k in range(ndim)]
        beta = b ** ndim
        S = orc.scores(a, cand, nb, mb, beta, mode=0)
        tip = _edge_pad(ti, b).astype(np.int64)
        const = sum(Fraction(int(mb[k]) ** 2, int(nb[k])) for k in np.ndindex(nb.shape) if nb[k] > 0)
        for c in itertools.product(*[range(n) for n in cand[::-1]]):      # numpy order
            ssd = Fraction(0)
            for u in zip(*np.nonzero(mask)):
                bk = tuple(ui // b for ui in u)
                lo = [b * c[k] + b * bk[k] for k in range(ndim)]
                blk = tip[tuple(slice(l, l + b) for l in lo)]
                pti = Fraction(int(blk.sum()), beta)
                por = Fraction(int(mb[bk]), int(nb[bk]))
                ssd += (pti - por) ** 2
            assert S[c] + beta * beta * const == beta * beta * ssd


def test_score_level0_is_masked_template_matching(orc):
    # J = 0: S = sum_OR (TI - OR)^2 - sum_OR OR^2 (textbook masked SSD), and the
    # raw CCW is the cross-correlation of the TI with the zero-filled OR
    rng = np.random.default_rng(5)
    ti = rng.integers(0, 3, size=(20, 23)).astype(np.int8)
    T = [7, 5]
    mask, vals, nb, mb = _random_event(rng, T, 0, 2, 3)
    or_img = np.where(mask, vals, 0).astype(np.int64)
    a, _ = orc.dwt(ti, 0)
    cand = [23 - 7 + 1, 20 - 5 + 1]
    S = orc.scores(a, cand, nb, mb, 1, mode=0)
    raw = orc.scores(a, cand, nb, mb, 1, mode=1)
    t64 = ti.astype(np.int64)
    xc = signal.correlate(t64, or_img, mode="valid", method="direct")
    e = signal.correlate(t64 ** 2, mask.astype(np.int64), mode="valid", method="direct")
    assert np.array_equal(raw, -xc)
    assert np.array_equal(S, e - 2 * xc)


def test_raw_ccw_is_coarse_cross_correlation(orc):
    # Sec. 4.3 CCW equation: sum of products of TI and OR approximations over
    # the template footprint, at every coarse candidate
    rng = np.random.default_rng(6)
    ti = syn.channel_image_2d(60, 44, 5, 3, seed=3)
    for J in (1, 2):
        a, _ = orc.dwt(ti, J)
        T = [16, 12]
        mask, vals, nb, mb = _random_event(rng, T, J, 2, 3)
        b = 2 ** J
        cand = [(60 - 16) // b + 1, (44 - 12) // b + 1]
        raw = orc.scores(a, cand, nb, mb, b * b, mode=1)
        xc = signal.correlate(a.astype(np.int64), mb, mode="valid", method="direct")
        assert np.array_equal(raw, -xc[: cand[1], : cand[0]])


# --------------------------------------------------------------------------
# K best and the draw
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n,k,with_mis", [(1, 5, False), (7, 10, True), (500, 10, False), (3000, 16, True)])
def test_select_matches_plain_sort(orc, n, k, with_mis):
    # Sec. 4.4: sort, keep the K best, draw one uniformly; checked against a
    # plain tuple sort of (mismatch, score, tie-break)
    rng = np.random.default_rng(n + k)
    for trial in range(5):
        S = rng.integers(-50, 50, size=n) * (trial + 1)          # many ties
        mis = rng.integers(0, 3, size=n) if with_mis else None
        seed, r, step = 77 + trial, trial, 3 * trial + 1
        chosen, keys = orc.select(S, mis, k, seed, r, step)
        tkey = orc.rng(seed, 2, r, step)
        order = sorted(range(n), key=lambda c: (0 if mis is None else int(mis[c]), int(S[c]),
                                                orc.perm20(c, tkey)))
        kk = min(k, n)
        j = ((orc.rng(seed, 3, r, step) >> 32) * kk) >> 32
        assert chosen == order[j]
        want = [((0 if mis is None else int(mis[c])) << 52) | ((int(S[c]) + 2 ** 31) << 20)
                | orc.perm20(c, tkey) for c in order[:kk]]
        assert [int(x) for x in keys] == want


# --------------------------------------------------------------------------
# minimal-error boundary cut
# --------------------------------------------------------------------------
@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 4), (4, 1), (5, 3), (6, 4), (4, 6)])
def test_mincut_matches_enumeration(orc, rows, cols):
    rng = np.random.default_rng(rows * 10 + cols)
    for _ in range(15):
        e = rng.integers(0, 4, size=(rows, cols)) ** 2
        seam = orc.mincut(e)
        want, cost = bf.best_seam(e)
        assert np.array_equal(seam, want)
        assert sum(int(e[y, seam[y]]) for y in range(rows)) == cost


def test_mincut_ties_follow_the_rule(orc):
    # all-equal errors: the seam stays at the outer edge (column 0)
    assert list(orc.mincut(np.zeros((5, 4), dtype=np.int64))) == [0] * 5
    # a single cheap column drags the seam onto it
    e = np.full((4, 3), 9, dtype=np.int64)
    e[:, 2] = 0
    assert list(orc.mincut(e)) == [2, 2, 2, 2]


# --------------------------------------------------------------------------
# lattice, path and whole-simulation invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", wl.WORKLOADS)
def test_lattice_is_minimal_cover(orc, name):
    p = dict(_params_only(name))
    from oracle.oracle import SimParams
    sp = SimParams(**{k: p[k] for k in ("ti", "grid", "tmpl", "overlap", "level", "top_k")})
    geo = orc.geometry(sp)
    for a in range(len(p["ti"])):
        n = bf.lattice_count(p["grid"][a], p["tmpl"][a], p["overlap"][a])
        assert geo["lattice"][a] == n
        assert geo["padded"][a] == n * (p["tmpl"][a] - p["overlap"][a]) + p["overlap"][a]
        assert geo["padded"][a] >= p["grid"][a]


def _params_only(name):
    table = {
        "c1_plain2d": dict(ti=(150, 150), grid=(100, 100), tmpl=(24, 24), overlap=(6, 6), level=1, top_k=5),
        "c2_scale2d": dict(ti=(500, 500), grid=(1000, 1000), tmpl=(40, 40), overlap=(10, 10), level=2, top_k=10),
        "c3_split3d": dict(ti=(180, 150, 60), grid=(300, 300, 80), tmpl=(30, 30, 10), overlap=(6, 6, 3),
                           level=2, top_k=10),
        "c4_batched": dict(ti=(400, 400), grid=(256, 256), tmpl=(32, 32), overlap=(8, 8), level=2, top_k=10),
        "c5_learned": dict(ti=(1000, 1000), grid=(2000, 2000), tmpl=(48, 48), overlap=(12, 12), level=2,
                           top_k=10),
    }
    return table[name]


def _sp(p, **over):
    from oracle.oracle import SimParams
    keys = ("ti", "grid", "tmpl", "overlap", "level", "top_k", "n_real", "n_facies", "seed",
            "path_mode", "score_mode", "nc_margin", "cut")
    d = {k: p[k] for k in keys}
    d["wavelet"] = p.get("wavelet", 0)
    d.update(over)
    return SimParams(**d)


TINY_CASES = [
    # (name, params overrides, hd count per realization)
    ("fixed_2d_j1", dict(ti=(20, 18), grid=(22, 19), tmpl=(6, 6), overlap=(2, 2), level=1, top_k=3,
                         path_mode=0, n_real=1, cut=1), 0),
    ("seeded_2d_j1_hd", dict(ti=(18, 20), grid=(20, 21), tmpl=(6, 5), overlap=(2, 2), level=1, top_k=4,
                             path_mode=1, n_real=3, cut=1), 12),
    ("fixed_2d_j2_partial", dict(ti=(22, 22), grid=(20, 17), tmpl=(7, 6), overlap=(3, 2), level=2,
                                 top_k=2, path_mode=0, n_real=1, cut=1), 6),
    ("fixed_2d_j0_nocut", dict(ti=(14, 12), grid=(16, 15), tmpl=(5, 5), overlap=(2, 2), level=0,
                               top_k=3, path_mode=1, n_real=2, cut=0), 5),
    ("seeded_3d_j1", dict(ti=(10, 10, 8), grid=(11, 10, 8), tmpl=(5, 5, 4), overlap=(2, 2, 1), level=1,
                          top_k=2, path_mode=1, n_real=2, cut=1), 4),
]


@pytest.mark.parametrize("case", TINY_CASES, ids=[c[0] for c in TINY_CASES])
def test_simulate_matches_bruteforce(orc, case):
    name, over, nhd = case
    p = dict(nc_margin=(-1, -1, -1), n_facies=3, seed=11, score_mode=0)
    p.update(over)
    nd = len(p["ti"])
    if nd == 2:
        ti = syn.channel_image_2d(p["ti"][0], p["ti"][1], 3, 3, seed=21)
        ref = syn.channel_image_2d(p["grid"][0], p["grid"][1], 3, 3, seed=22)
    else:
        ti = syn.tube_image_3d(*p["ti"], 3, seed=21)
        ref = syn.tube_image_3d(*p["grid"], 3, seed=22)
        p["n_facies"] = 2
    hd = syn.sample_hard_data(ref, [nhd] * p["n_real"], seed=23) if nhd else None
    out, chosen = orc.simulate(_sp(p), ti, hd)
    bout, bchosen = bf.simulate(p, ti, hd, orc.rng, orc.perm20)
    assert np.array_equal(chosen, bchosen)
    assert np.array_equal(out, bout)


@pytest.mark.parametrize("case", TINY_CASES, ids=[c[0] for c in TINY_CASES])
def test_simulate_53_matches_bruteforce(orc, case):
    # the LeGall 5/3 path: transform-domain scores against the brute force's
    # direct sum of squared coefficient differences, patterns by crop
    name, over, nhd = case
    p = dict(nc_margin=(-1, -1, -1), n_facies=3, seed=11, score_mode=0, wavelet=1)
    p.update(over)
    nd = len(p["ti"])
    if nd == 2:
        ti = syn.channel_image_2d(p["ti"][0], p["ti"][1], 3, 3, seed=21)
        ref = syn.channel_image_2d(p["grid"][0], p["grid"][1], 3, 3, seed=22)
    else:
        ti = syn.tube_image_3d(*p["ti"], 3, seed=21)
        ref = syn.tube_image_3d(*p["grid"], 3, seed=22)
        p["n_facies"] = 2
    hd = syn.sample_hard_data(ref, [nhd] * p["n_real"], seed=23) if nhd else None
    out, chosen = orc.simulate(_sp(p), ti, hd)
    bout, bchosen = bf.simulate(p, ti, hd, orc.rng, orc.perm20)
    assert np.array_equal(chosen, bchosen)
    assert np.array_equal(out, bout)
    # a different wavelet gives a different search (same inputs)
    hout, hchosen = orc.simulate(_sp(dict(p, wavelet=0)), ti, hd)
    if p["level"] > 0:
        assert not np.array_equal(chosen, hchosen)


@pytest.mark.parametrize("name", ["c1_plain2d", "c2_scale2d", "c4_batched", "c3_split3d"])
def test_simulate_invariants(orc, name):
    scale = {"c1_plain2d": 1.0, "c2_scale2d": 0.16, "c4_batched": 0.3, "c3_split3d": 0.25}[name]
    p, ti, hd = wl.make(name, scale=scale, n_real=2 if name == "c4_batched" else None)
    out, chosen = orc.simulate(_sp(p), ti, hd)
    # every cell simulated, codes drawn from the TI's codes
    assert out.min() >= 0
    assert set(np.unique(out)) <= set(np.unique(ti))
    # conditioning data honoured (Sec. 5.2)
    if hd is not None:
        for r, pos, v in zip(*hd):
            assert out[(r,) + tuple(pos[::-1])] == v
    geo = orc.geometry(_sp(p))
    assert chosen.shape == (p["n_real"], geo["nsteps"])
    assert chosen.min() >= 0 and chosen.max() < geo["ncand"]


def test_first_patch_is_a_ti_crop(orc):
    # Algorithm 1: the first patch is a random TI patch; with FIXED path and
    # no cut beyond the first window, the first window's non-overlapped part
    # is the TI crop at the chosen candidate
    p, ti, _ = wl.make("c1_plain2d")
    sp = _sp(p)
    out, chosen = orc.simulate(sp, ti, None)
    geo = orc.geometry(sp)
    b = geo["b"][0]
    c = int(chosen[0, 0])
    cx, cy = c % geo["cand"][0], c // geo["cand"][0]
    s = 24 - 6
    crop = ti[b * cy: b * cy + s, b * cx: b * cx + s]
    assert np.array_equal(out[0, :s, :s], crop)


# --------------------------------------------------------------------------
# realization statistics (Sec. 5.2, 5.3, 5.8)
# --------------------------------------------------------------------------
from oracle import stats as ost   # noqa: E402


def test_histogram_counts_closed_form():
    y, x = np.mgrid[0:6, 0:9]
    img = ((x + y) % 3).astype(np.int8)
    img[0, 0] = 7                                   # a code outside 0..2 counts nowhere
    stack = np.stack([img, np.full_like(img, 1)])
    per_image, per_cell = ost.histogram(stack, 3)
    assert per_image.tolist() == [[17, 18, 18], [0, 54, 0]]
    assert per_cell.sum() == 2 * 54 - 1
    assert per_cell[1].min() >= 1                   # image 1 holds facies 1 everywhere
    assert per_cell[:, 0, 0].tolist() == [0, 1, 0]


def test_variogram_alternating_columns_and_step_edge():
    ny, nx = 5, 12
    cols = np.tile((np.arange(nx) % 2).astype(np.int8), (ny, 1))
    d = ost.variogram(cols[None], 2, 0, nx - 1)[0]
    for h in range(1, nx):
        n = ost.pair_count(cols.shape, 0, h)
        assert n == ny * (nx - h)
        assert d[1, h - 1] == (n if h % 2 else 0) and d[0, h - 1] == d[1, h - 1]
    assert not ost.variogram(cols[None], 2, 1, ny - 1).any()   # constant along y
    a = 6
    edge = np.zeros((ny, 2 * a), dtype=np.int8)
    edge[:, :a] = 1
    d = ost.variogram(edge[None], 2, 0, 2 * a - 1)[0, 1]
    assert d.tolist() == [ny * min(h, 2 * a - h) for h in range(1, 2 * a)]


def test_variogram_3d_layers_and_iid_sill():
    z = np.arange(7)[:, None, None]
    layers = np.broadcast_to((z % 2).astype(np.int8), (7, 4, 5)).copy()
    d = ost.variogram(layers[None], 2, 2, 6)[0, 0]
    assert d.tolist() == [ost.pair_count(layers.shape, 2, h) * (h % 2) for h in range(1, 7)]
    # independent cells with P(f) = p: gamma(h) = p (1 - p) at every lag
    rng = np.random.default_rng(5)
    p = 0.3
    img = (rng.random((400, 400)) < p).astype(np.int8)
    d = ost.variogram(img[None], 2, 0, 5)[0, 1]
    gam = [d[h - 1] / (2 * ost.pair_count(img.shape, 0, h)) for h in range(1, 6)]
    assert np.allclose(gam, p * (1 - p), atol=0.005)


def _canon(lab):
    out = np.full(lab.shape, -1, dtype=np.int64)
    seen = {}
    for i, v in enumerate(lab.reshape(-1)):
        if v >= 0:
            out.reshape(-1)[i] = seen.setdefault(v, len(seen))
    return out


@pytest.mark.parametrize("shape,p", [((23, 31), 0.55), ((9, 10, 11), 0.35), ((1, 40), 0.5)])
def test_components_equal_library_labelling(shape, p):
    from scipy import ndimage
    rng = np.random.default_rng(sum(shape))
    mask = rng.random(shape) < p
    ref, _ = ndimage.label(mask)          # face connectivity is the default structure
    assert np.array_equal(_canon(ost.components(mask)), _canon(ref - 1))


def test_connectivity_closed_forms():
    ny, nx = 6, 10
    full = np.ones((ny, nx), dtype=np.int8)
    both, conn = ost.connectivity(full[None], 2, 0, nx - 1)
    assert np.array_equal(both[0, 1], conn[0, 1])
    assert both[0, 1].tolist() == [ny * (nx - h) for h in range(1, nx)] and not both[0, 0].any()
    y, x = np.mgrid[0:ny, 0:nx]
    checker = ((x + y) % 2).astype(np.int8)          # every cell of a facies is isolated
    both, conn = ost.connectivity(checker[None], 2, 0, nx - 1)
    assert not conn.any() and both[0, :, 1].min() > 0
    stripes = (y % 2).astype(np.int8)                # rows alternate: one component per row
    both, conn = ost.connectivity(stripes[None], 2, 0, nx - 1)
    assert conn[0, 1].tolist() == [(ny // 2) * (nx - h) for h in range(1, nx)]
    both, conn = ost.connectivity(stripes[None], 2, 1, ny - 1)
    assert not conn.any()
    assert both[0, 1].tolist() == [nx * len([r for r in range(ny - h) if r % 2 and (r + h) % 2])
                                   for h in range(1, ny)]


def test_connectivity_follows_paths_not_lines():
    # two vertical bars 5 cells apart: joined by a bottom bar they form one
    # component, without it two
    u = np.zeros((8, 9), dtype=np.int8)
    u[:, 1] = 1
    u[:, 6] = 1
    both, conn = ost.connectivity(u[None], 2, 0, 8)
    assert both[0, 1, 4] == 8 and conn[0, 1, 4] == 0
    u[7, 1:7] = 1
    both, conn = ost.connectivity(u[None], 2, 0, 8)
    assert both[0, 1, 4] == 8 and conn[0, 1, 4] == 8


# --------------------------------------------------------------------------
# LeGall 5/3 integer lifting (another mother wavelet than Haar)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 4, 6, 10, 64, 130])
def test_lift53_perfect_reconstruction(orc, n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        x = rng.integers(-300, 300, size=n)
        s, d = orc.lift53_forward(x)
        assert np.array_equal(orc.lift53_inverse(s, d), x)


def test_lift53_constant_and_ramp():
    from oracle import oracle as o
    s, d = o.lift53_forward(np.full(16, 7))
    assert (s == 7).all() and (d == 0).all()
    # the predictor is linear interpolation: a ramp has no detail except
    # where the mirror at the right end breaks it (the last odd sample)
    x = 3 * np.arange(20) + 5
    s, d = o.lift53_forward(x)
    assert (d[:-1] == 0).all() and d[-1] != 0
    assert np.array_equal(s[1:-1], x[2:-2:2])


def test_lift53_hand_example():
    # x = [1, 4, 2, 8, 5, 7]: d0 = 4 - floor((1 + 2) / 2) = 3,
    # d1 = 8 - floor((2 + 5) / 2) = 5, d2 = 7 - floor((5 + 5) / 2) = 2 (x6 mirrors
    # to x4); s0 = 1 + floor((d0 + d0 + 2) / 4) = 3, s1 = 2 + floor((3 + 5 + 2) / 4) = 4,
    # s2 = 5 + floor((5 + 2 + 2) / 4) = 7
    from oracle import oracle as o
    s, d = o.lift53_forward(np.array([1, 4, 2, 8, 5, 7]))
    assert d.tolist() == [3, 5, 2] and s.tolist() == [3, 4, 7]


def test_approx53_is_separable_lifting():
    # the level-J image approximation equals lifting every row, then every
    # column, level after level (checked against the 1D routine)
    from oracle import oracle as o
    rng = np.random.default_rng(3)
    img = rng.integers(0, 3, size=(16, 24))
    cur = img.astype(np.int64)
    for _ in range(2):
        cur = np.stack([o.lift53_forward(r)[0] for r in cur])
        cur = np.stack([o.lift53_forward(c)[0] for c in cur.T]).T
    assert np.array_equal(o.approx53(img, 2), cur)
    img3 = rng.integers(0, 2, size=(4, 8, 8))
    a3 = o.approx53(img3, 1)
    ref = img3.astype(np.int64)
    ref = np.apply_along_axis(lambda v: o.lift53_forward(v)[0], 2, ref)
    ref = np.apply_along_axis(lambda v: o.lift53_forward(v)[0], 1, ref)
    ref = np.apply_along_axis(lambda v: o.lift53_forward(v)[0], 0, ref)
    assert np.array_equal(a3, ref)


# --------------------------------------------------------------------------
# The full LeGall 5/3 transform (approximation and every detail sub-band)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape,J", [((37, 22), 2), ((16, 16), 3), ((9, 12, 10), 1), ((20, 18, 12), 2), ((5, 7), 0)])
def test_dwt53_perfect_reconstruction(orc, shape, J):
    # the integer lifting is exactly invertible: the inverse returns the
    # edge-replicated image
    x = np.random.default_rng(sum(shape) + J).integers(0, 3, size=shape).astype(np.int8)
    a, d = orc.dwt53(x, J)
    assert np.array_equal(orc.idwt53(a, d), orc._pad_edge(x, J))
    assert len(d) == J


@pytest.mark.parametrize("shape,J", [((37, 22), 2), ((20, 18, 12), 2), ((32, 24), 3)])
def test_dwt53_approximation_equals_approx53(orc, shape, J):
    # the approximation band agrees with the level-J approximation routine
    # (written separately in C)
    x = np.random.default_rng(7 + J).integers(0, 3, size=shape).astype(np.int8)
    a, _ = orc.dwt53(x, J)
    assert np.array_equal(a, orc.approx53(orc._pad_edge(x, J), J))


def test_dwt53_constant_and_ramp(orc):
    # a constant has no detail and keeps its value; a ramp along x has zero
    # detail except where the mirror at the far edge bends it, and nothing in
    # the sub-bands that took the high-pass along y
    a, d = orc.dwt53(np.full((8, 12), 2, np.int8), 2)
    assert (a == 2).all() and all((dd == 0).all() for dd in d)
    x = np.tile(np.arange(16, dtype=np.int8), (6, 1))   # [y][x], ramp along x
    a, d = orc.dwt53(x, 1)
    q1, q2, q3 = d[0]
    assert (q2 == 0).all() and (q3 == 0).all()
    assert (q1[:, :-1] == 0).all() and (q1[:, -1] == 1).all()
