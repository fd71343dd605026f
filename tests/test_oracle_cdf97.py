"""Pins of the float64 CDF 9/7 oracle (oracle/cdf97.py) against what the
mathematics and the published filter fix: perfect reconstruction, the
closed form for constants, the four vanishing moments of the analysis
high-pass, the published 9/7 analysis taps (tests/golden/cdf97_taps.txt) on
interior impulses and on explicitly mirrored signals (whole-sample
symmetric extension), and the scores against a sliding-window SSD and
brute force."""
import os

import numpy as np
import pytest

from oracle import cdf97 as c97

GOLD = os.path.join(os.path.dirname(__file__), "golden")
SQ2 = np.sqrt(2.0)


def _taps():
    t = {"low": {}, "high": {}}
    with open(os.path.join(GOLD, "cdf97_taps.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                band, off, val = line.split()
                t[band][int(off)] = float(val)
    return t


def _filter_bank(x, taps):
    """The published analysis filters applied to the whole-sample mirrored
    signal (np.pad 'reflect'), with this module's scaling: low times sqrt 2
    (gain sqrt 2 at DC), high over sqrt 2.  An independent route to the
    same coefficients as the lifting."""
    n = x.shape[0]
    xp = np.pad(x, 8, mode="reflect")
    lo = np.zeros(n // 2)
    hi = np.zeros(n // 2)
    for k in range(n // 2):
        c = 2 * k + 8
        lo[k] = sum(taps["low"][abs(o)] * xp[c + o] for o in range(-4, 5))
        hi[k] = sum(taps["high"][abs(o)] * xp[c + 1 + o] for o in range(-3, 4))
    return lo * SQ2, hi / SQ2


def test_published_taps_sum_rules():
    t = _taps()
    lo = t["low"][0] + 2 * sum(t["low"][o] for o in range(1, 5))
    hi = t["high"][0] + 2 * sum(t["high"][o] for o in range(1, 4))
    assert abs(lo - 1.0) < 1e-12 and abs(hi) < 1e-12


@pytest.mark.parametrize("n", [8, 10, 16, 34])
def test_lifting_equals_filter_bank_on_mirrored_signal(n):
    x = np.random.default_rng(n).normal(size=n)
    s, d = c97.lift97_forward(x)
    lo, hi = _filter_bank(x, _taps())
    assert np.abs(s - lo).max() < 1e-9 and np.abs(d - hi).max() < 1e-9


def test_lifting_impulse_responses_are_the_published_taps():
    t = _taps()
    n, k0 = 64, 16
    for p in range(2 * k0 - 6, 2 * k0 + 7):
        x = np.zeros(n)
        x[p] = 1.0
        s, d = c97.lift97_forward(x)
        off_lo, off_hi = p - 2 * k0, p - (2 * k0 + 1)
        want_lo = t["low"].get(abs(off_lo), 0.0) * SQ2
        want_hi = t["high"].get(abs(off_hi), 0.0) / SQ2
        assert abs(s[k0] - want_lo) < 1e-9, p
        assert abs(d[k0] - want_hi) < 1e-9, p


@pytest.mark.parametrize("n", [2, 4, 6, 12, 40])
def test_perfect_reconstruction_1d(n):
    x = np.random.default_rng(n).normal(size=n) * 50
    s, d = c97.lift97_forward(x)
    assert np.abs(c97.lift97_inverse(s, d) - x).max() < 1e-11


@pytest.mark.parametrize("shape,level", [((16, 24), 2), ((13, 9), 1), ((8, 12, 20), 2), ((37, 50), 3)])
def test_perfect_reconstruction_nd(shape, level):
    img = np.random.default_rng(sum(shape)).integers(0, 3, size=shape)
    approx, det = c97.dwt97(img, level)
    rec = c97.idwt97(approx, det)
    assert rec.shape == c97.pad_edge(img, level).shape
    assert np.abs(rec - c97.pad_edge(img, level)).max() < 1e-10
    b = 2 ** level
    assert approx.shape == tuple(-(-n // b) for n in shape)
    for j, dj in enumerate(det, start=1):
        assert dj.shape == (2 ** len(shape) - 1,) + tuple(-(-n // b) * b >> j for n in shape)


@pytest.mark.parametrize("shape,level", [((16, 16), 2), ((8, 8, 8), 1), ((32, 16), 3)])
def test_constant_closed_form(shape, level):
    # the low-pass has gain sqrt 2 at DC and the high-pass kills constants:
    # a constant c becomes c * sqrt(2)^(d J), every detail zero
    c = 1.75
    approx, det = c97.dwt97(np.full(shape, c), level)
    assert np.abs(approx - c * SQ2 ** (len(shape) * level)).max() < 1e-11
    assert max(np.abs(d).max() for d in det) < 1e-11


def test_vanishing_moments():
    # the analysis high-pass has four vanishing moments: the interior
    # details of any cubic are zero, those of a quartic are not
    n = 64
    t = np.arange(n, dtype=np.float64) / n
    cubic = 3 - 2 * t + 5 * t ** 2 - 7 * t ** 3
    _, d = c97.lift97_forward(cubic)
    assert np.abs(d[3:-3]).max() < 1e-12
    _, d4 = c97.lift97_forward(t ** 4)
    assert np.abs(d4[3:-3]).max() > 1e-8


def test_scores_against_sliding_window_ssd():
    rng = np.random.default_rng(5)
    K = rng.normal(size=(20, 23))
    tc = (5, 6)
    n = (rng.random(tc) < 0.5).astype(np.int32)
    n[0, 0] = 1
    A = K[7:12, 3:9].copy()   # the event is the grid's own window at (7, 3)
    A[n == 0] = 99.0           # values outside the mask must not matter
    cand = (20 - tc[0] + 1, 23 - tc[1] + 1)
    S = c97.scores97(K, cand, n, A)
    from numpy.lib.stride_tricks import sliding_window_view
    win = sliding_window_view(K, tc)                 # [cy][cx][by][bx]
    want = ((win - np.where(n == 1, A, 0.0)) ** 2 * n).sum(axis=(2, 3))
    assert S.shape == cand
    assert np.abs(S - want).max() < 1e-9
    assert S[7, 3] == 0.0 and c97.topk97(S, 1)[0] == 7 * cand[1] + 3


def test_scores_brute_force_3d():
    rng = np.random.default_rng(8)
    K = rng.normal(size=(4, 5, 6))
    tc = (2, 3, 2)
    n = rng.integers(0, 2, size=tc)
    A = rng.normal(size=tc)
    cand = (3, 3, 5)
    S = c97.scores97(K, cand, n, A)
    for cz in range(3):
        for cy in range(3):
            for cx in range(5):
                s = 0.0
                for bz in range(2):
                    for by in range(3):
                        for bx in range(2):
                            if n[bz, by, bx]:
                                s += (K[cz + bz, cy + by, cx + bx] - A[bz, by, bx]) ** 2
                assert abs(S[cz, cy, cx] - s) < 1e-12


def test_topk_ties_to_smaller_index():
    S = np.array([3.0, 1.0, 2.0, 1.0, 0.5, 2.0])
    assert list(c97.topk97(S, 4)) == [4, 1, 3, 2]


def test_band_layout_separable_image():
    # an image varying along x only: the y pass multiplies by sqrt 2 (low)
    # and gives zero (high), so band 1 (x high, y low) is sqrt 2 times the
    # line's detail, bands 2 and 3 (y high) vanish, and the approximation is
    # sqrt 2 times the line's low band
    f = np.random.default_rng(3).normal(size=24)
    img = np.tile(f, (10, 1))            # [y][x]
    approx, det = c97.dwt97(img, 1)
    s, d = c97.lift97_forward(f)
    assert np.abs(approx - SQ2 * s[None, :]).max() < 1e-11
    assert np.abs(det[0][0] - SQ2 * d[None, :]).max() < 1e-11
    assert np.abs(det[0][1:]).max() < 1e-11


def test_band_layout_separable_volume():
    # a volume varying along z only: the x and y passes multiply by sqrt 2
    # (low) or give zero (high), so only band 4 (z high, x and y low) of the
    # details is non-zero, equal to 2 times the line's detail, and the
    # approximation is 2 times the line's low band
    f = np.random.default_rng(4).normal(size=16)
    vol = np.broadcast_to(f[:, None, None], (16, 6, 8)).copy()   # [z][y][x]
    approx, det = c97.dwt97(vol, 1)
    s, d = c97.lift97_forward(f)
    assert np.abs(approx - 2.0 * s[:, None, None]).max() < 1e-11
    for q in range(1, 8):
        want = 2.0 * d[:, None, None] if q == 4 else 0.0
        assert np.abs(det[0][q - 1] - want).max() < 1e-11, q
