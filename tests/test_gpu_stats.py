"""Realization statistics on the GPU against the oracle (Sec. 5.2, 5.3, 5.8).

Every count is an integer and must match exactly.
"""
import numpy as np
import pytest
import torch

from oracle import stats as ost
from paper_2404_00441_amd import synthetic as syn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_00441_amd import ccwsim
    ccwsim.load()
    return ccwsim


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int8)).cuda()


def _iid(shape, nf, seed, other=0.0):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, nf, size=shape).astype(np.int8)
    if other:
        a[rng.random(shape) < other] = nf + 2          # codes outside 0..nf-1
    return a


def _serpentine(ny, nx):
    # one winding component: full rows joined alternately at the right and
    # left ends (the longest union chains a row-run start can form)
    a = np.zeros((ny, nx), dtype=np.int8)
    a[0::2, :] = 1
    for k, y in enumerate(range(1, ny, 2)):
        a[y, nx - 1 if k % 2 == 0 else 0] = 1
    return a


def _channels(n_img, nx, ny, nf, seed):
    return np.stack([syn.channel_image_2d(nx, ny, 12, nf, seed=seed + i) for i in range(n_img)])


CASES = [
    ("iid_2d_ragged", lambda: _iid((5, 37, 45), 3, 1), 3),
    ("iid_2d_other_codes", lambda: _iid((4, 33, 70), 4, 2, other=0.1), 4),
    ("iid_3d", lambda: _iid((3, 9, 11, 13), 2, 3), 2),
    ("channels_2d", lambda: _channels(3, 150, 120, 3, 10), 3),
    ("tubes_3d", lambda: np.stack([syn.tube_image_3d(40, 30, 20, 6, seed=s) for s in (4, 5)]), 2),
    ("serpentine", lambda: _serpentine(65, 97)[None], 2),
    ("one_facies", lambda: _iid((2, 20, 33), 1, 6, other=0.3), 1),
    ("wide_row", lambda: _iid((2, 1, 300), 2, 7), 2),
    ("tall_column", lambda: _iid((2, 64, 1), 2, 8), 2),
    ("word_edges", lambda: _iid((2, 5, 64), 2, 9), 2),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_histogram_matches_oracle(cc, case):
    name, make, nf = case
    imgs = make()
    _say("histogram", name, imgs.shape)
    pi, pc = cc.stats_histogram(_dev(imgs), nf)
    want_i, want_c = ost.histogram(imgs, nf)
    assert np.array_equal(pi.cpu().numpy(), want_i)
    assert np.array_equal(pc.cpu().numpy(), want_c)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_variogram_matches_oracle(cc, case):
    name, make, nf = case
    imgs = make()
    d = _dev(imgs)
    for axis in range(imgs.ndim - 1):
        n = imgs.shape[imgs.ndim - 1 - axis]
        if n < 2:
            continue
        for lag in sorted({1, min(7, n - 1), n - 1}):
            _say("variogram", name, axis, lag)
            got = cc.stats_variogram(d, nf, axis, lag).cpu().numpy()
            assert np.array_equal(got, ost.variogram(imgs, nf, axis, lag)), (axis, lag)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_connectivity_matches_oracle(cc, case):
    name, make, nf = case
    imgs = make()
    d = _dev(imgs)
    for axis in range(imgs.ndim - 1):
        n = imgs.shape[imgs.ndim - 1 - axis]
        if n < 2:
            continue
        lag = n - 1
        _say("connectivity", name, axis, lag)
        both, conn = cc.stats_connectivity(d, nf, axis, lag)
        wb, wc = ost.connectivity(imgs, nf, axis, lag)
        assert np.array_equal(both.cpu().numpy(), wb), axis
        assert np.array_equal(conn.cpu().numpy(), wc), axis


def test_connectivity_is_repeatable(cc):
    # the union order differs from run to run; the counts may not
    imgs = _channels(4, 200, 160, 3, 40)
    d = _dev(imgs)
    a = [t.cpu().numpy() for t in cc.stats_connectivity(d, 3, 0, 120)]
    for _ in range(3):
        b = [t.cpu().numpy() for t in cc.stats_connectivity(d, 3, 0, 120)]
        assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_statistics_of_a_realization_at_full_size(cc):
    # a 1000^2 channel image, the grid size of the benchmark workload:
    # histogram and variograms in full, connectivity of the channel facies
    img = syn.channel_image_2d(1000, 1000, 50, 3, seed=77)[None]
    _say("full size")
    d = _dev(img)
    pi, pc = cc.stats_histogram(d, 3)
    wi, wc = ost.histogram(img, 3)
    assert np.array_equal(pi.cpu().numpy(), wi) and np.array_equal(pc.cpu().numpy(), wc)
    for axis in (0, 1):
        got = cc.stats_variogram(d, 3, axis, 250).cpu().numpy()
        assert np.array_equal(got, ost.variogram(img, 3, axis, 250))
    both, conn = cc.stats_connectivity(d, 3, 0, 250)
    lab = ost.components(img[0] == 1)
    for h in (1, 17, 64, 250):
        lo, hi = lab[:, :-h], lab[:, h:]
        inb = (lo >= 0) & (hi >= 0)
        assert both[0, 1, h - 1].item() == np.count_nonzero(inb)
        assert conn[0, 1, h - 1].item() == np.count_nonzero(inb & (lo == hi))
