"""CPU checks of the float64 reference of the learned proposer: its
analytic gradient against central finite differences of its loss, and the
receptive field covering the template window."""
import numpy as np

from tests import lp_ref


def _setup(seed=0):
    rng = np.random.default_rng(seed)
    nw = sum(co * ci * t + co for cin0 in (1, 2) for (co, ci, t) in lp_ref.layer_shapes(cin0))
    w = rng.normal(0, 0.2, size=nw)
    K = rng.integers(0, 9, size=(8, 9))          # level-J grid [y][x]
    tc = (4, 3)                                  # template blocks (x, y)
    cand = (9 - tc[0] + 1, 8 - tc[1] + 1)
    ev = rng.random((3, 2, tc[1], tc[0]))
    labels = rng.integers(0, cand[0] * cand[1], size=3)
    return w, K, ev, labels, cand, tc


def test_reference_gradient_matches_finite_differences():
    w, K, ev, labels, cand, tc = _setup()
    loss, g = lp_ref.loss_and_grad(w, K, 4, ev, labels, cand, tc)
    rng = np.random.default_rng(1)
    f = lambda ww: lp_ref.loss_and_grad(ww, K, 4, ev, labels, cand, tc)[0].mean()
    for i in rng.choice(w.size, size=40, replace=False):
        h = 1e-5
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        num = (f(wp) - f(wm)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-4 * abs(num), (i, num, g[i])


def test_reference_receptive_field_covers_the_window():
    # the key of a candidate changes when any block of its template window
    # changes (dilations 1, 2, 4 reach 7 blocks each way)
    w, _, ev, _, _, _ = _setup(2)
    K = np.zeros((20, 20))
    tc = (12, 12)
    cand = (9, 9)
    ev = np.zeros((1, 2, 12, 12))
    k0, _, _, _ = lp_ref.forward(w, K, 16, ev, cand, tc)
    for (y, x) in [(0, 0), (11, 11), (0, 11), (11, 0)]:
        K2 = K.copy()
        K2[y, x] = 5.0
        k1, _, _, _ = lp_ref.forward(w, K2, 16, ev, cand, tc)
        assert not np.allclose(k1[0], k0[0])   # candidate (0, 0)


def test_reference_set_loss_gradient_and_special_case():
    # several positives: finite differences again; one positive: the
    # single-label loss, log(sum exp S) - S_label
    w, K, ev, labels, cand, tc = _setup(3)
    rng = np.random.default_rng(4)
    sets = np.stack([rng.choice(cand[0] * cand[1], size=3, replace=False) for _ in range(3)])
    loss, g = lp_ref.loss_and_grad(w, K, 4, ev, sets, cand, tc)
    f = lambda ww: lp_ref.loss_and_grad(ww, K, 4, ev, sets, cand, tc)[0].mean()
    for i in rng.choice(w.size, size=30, replace=False):
        h = 1e-5
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        num = (f(wp) - f(wm)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-4 * abs(num), (i, num, g[i])
    l1, _ = lp_ref.loss_and_grad(w, K, 4, ev, labels, cand, tc)
    _, _, S, _ = lp_ref.forward(w, K, 4, ev, cand, tc)
    direct = np.log(np.exp(S).sum(axis=1)) - S[np.arange(3), labels]
    assert np.allclose(l1, direct, rtol=1e-12, atol=1e-12)
