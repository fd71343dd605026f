"""GPU checks of the learned proposer's kernels against the float64 numpy
reference in tests/lp_ref.py: encoder forward (keys, queries, scores), the
loss and every weight gradient of one training step, the Adam update, and
the top-k shortlist against a sort.

Tolerance: every value is a sum of at most a few thousand fp32 products
of O(1) terms, so a relative error of 1e-4 of the largest magnitude of the
compared quantity bounds fp32 rounding with a wide margin; the shortlist
is integer work and compared exactly."""
import sys

import numpy as np
import pytest

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


def _t(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a.astype(dtype))).cuda()


def _close(got, want, rel=1e-4, what=""):
    got = np.asarray(got, dtype=np.float64)
    scale = max(np.abs(want).max(), 1e-30)
    err = np.abs(got - want).max()
    assert err <= rel * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


# (TI extent, level, template, batch)
GEOMS = [((64, 56), 1, (16, 16), 5), ((90, 70), 2, (24, 20), 3), ((120, 120), 2, (48, 48), 4)]


def _inputs(ti, level, tmpl, B, seed):
    rng = np.random.default_rng(seed)
    b = 2 ** level
    G = (-(-ti[0] // b), -(-ti[1] // b))          # the level-J grid covers the TI
    K = rng.integers(0, 2 * b * b + 1, size=(G[1], G[0]))
    tc = ((tmpl[0] + b - 1) // b, (tmpl[1] + b - 1) // b)
    on = np.zeros((B, tc[1], tc[0]), np.int32)
    om = np.zeros((B, tc[1], tc[0]), np.int32)
    # L-shaped overlaps of random width (some blocks partly known), zero
    # elsewhere, like a data event
    for i in range(B):
        wx, wy = rng.integers(1, tc[0] // 2 + 1), rng.integers(1, tc[1] // 2 + 1)
        mask = np.zeros((tc[1], tc[0]), bool)
        mask[:, :wx] = True
        mask[:wy, :] = True
        on[i][mask] = rng.integers(1, b * b + 1, size=mask.sum())
        om[i][mask] = rng.integers(0, 2 * on[i][mask] + 1)
    ev = np.stack([om, on], axis=1) / float(b * b)   # the encoder's input channels
    cand = ((ti[0] - tmpl[0]) // b + 1, (ti[1] - tmpl[1]) // b + 1)
    return K, (on.reshape(B, -1), om.reshape(B, -1)), ev, cand, tc


@pytest.mark.parametrize("geom", GEOMS, ids=[f"{g[0][0]}x{g[0][1]}_J{g[1]}_T{g[2][0]}" for g in GEOMS])
def test_encode_matches_reference(cc, geom):
    ti, level, tmpl, B = geom
    _say("lp encode", geom)
    K, (on, om), ev, cand, tc = _inputs(ti, level, tmpl, B, 3)
    w = cc.lp_init(7)
    wn = w.cpu().numpy().astype(np.float64)
    ws = cc.LpWorkspace(ti, level, tmpl, B)
    assert ws.ncand == cand[0] * cand[1]
    keys, q, S = cc.lp_encode(w, _t(K, np.int32), ws, _t(on, np.int32), _t(om, np.int32), want_keys=True,
                              want_queries=True, want_scores=True)
    k_ref, q_ref, S_ref, _ = lp_ref.forward(wn, K, (2 ** level) ** 2, ev, cand, tc)
    _close(keys.cpu().numpy(), k_ref, what="keys")
    _close(q.cpu().numpy(), q_ref, what="queries")
    _close(S.cpu().numpy(), S_ref, what="scores")


def test_init_is_he_uniform_and_seeded(cc):
    w1, w2, w3 = cc.lp_init(7).cpu().numpy(), cc.lp_init(7).cpu().numpy(), cc.lp_init(8).cpu().numpy()
    assert np.array_equal(w1, w2) and not np.array_equal(w1, w3)
    o = 0
    for cin0 in (1, 2):
        for (co, ci, t) in lp_ref.layer_shapes(cin0):
            W = w1[o: o + co * ci * t]
            o += co * ci * t
            bound = np.sqrt(6.0 / (ci * t))
            assert np.all(np.abs(W) <= bound) and np.abs(W).max() > 0.9 * bound
            assert abs(W.mean()) < 0.1 * bound
            assert np.all(w1[o: o + co] == 0)
            o += co
    assert o == w1.size


TRAIN_CASES = [(GEOMS[0], 1), (GEOMS[1], 1), (GEOMS[0], 4), (GEOMS[1], 10)]


@pytest.mark.parametrize("geom,n_pos", TRAIN_CASES, ids=[f"{g[0][0]}x{g[0][1]}_J{g[1]}_L{L}" for g, L in TRAIN_CASES])
def test_train_step_matches_reference(cc, geom, n_pos):
    import torch
    ti, level, tmpl, B = geom
    _say("lp train step", geom, n_pos)
    K, (on, om), ev, cand, tc = _inputs(ti, level, tmpl, B, 5)
    rng = np.random.default_rng(9)
    if n_pos == 1:
        labels = rng.integers(0, cand[0] * cand[1], size=B)
    else:
        labels = np.stack([rng.choice(cand[0] * cand[1], size=n_pos, replace=False) for _ in range(B)])
    w = cc.lp_init(11)
    w0 = w.cpu().numpy().astype(np.float64)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    ws = cc.LpWorkspace(ti, level, tmpl, B)
    Kt, lt = _t(K, np.int32), _t(labels, np.int32)
    ont, omt = _t(on, np.int32), _t(om, np.int32)
    loss, g = cc.lp_train_step(w, m, v, 1, 1e-3, Kt, ws, ont, omt, lt, want_grad=True)
    loss_ref, g_ref = lp_ref.loss_and_grad(w0, K, (2 ** level) ** 2, ev, labels, cand, tc)
    _close(loss.cpu().numpy(), loss_ref, what="loss")
    gn = g.cpu().numpy()
    # per layer, relative to that layer's largest gradient
    o = 0
    for e, cin0 in enumerate((1, 2)):
        for l, (co, ci, t) in enumerate(lp_ref.layer_shapes(cin0)):
            n = co * ci * t + co
            _close(gn[o: o + n], g_ref[o: o + n], rel=1e-3, what=f"grad enc {e} layer {l}")
            o += n
    # the Adam update from the reference gradient (first step)
    w_ref, m_ref, v_ref = lp_ref.adam(w0, gn.astype(np.float64), 0 * w0, 0 * w0, 1, 1e-3)
    # (1 - 0.999 in fp32 is 1.3e-5 off in relative terms)
    _close(m.cpu().numpy(), m_ref, rel=1e-4, what="adam m")
    _close(v.cpu().numpy(), v_ref, rel=1e-4, what="adam v")
    _close(w.cpu().numpy() - w0, w_ref - w0, rel=1e-3, what="adam update")
    # a second step runs on the updated weights and moments
    loss2, _ = cc.lp_train_step(w, m, v, 2, 1e-3, Kt, ws, ont, omt, lt)
    assert np.isfinite(loss2.cpu().numpy()).all()


SHORTLIST_CASES = [(3, 1000, 256), (2, 57121, 256), (4, 300, 1), (1, 256, 256), (2, 5000, 100)]


@pytest.mark.parametrize("B,n,k", SHORTLIST_CASES, ids=[f"B{b}_n{n}_k{k}" for b, n, k in SHORTLIST_CASES])
def test_shortlist_matches_a_sort(cc, B, n, k):
    _say("lp shortlist", B, n, k)
    rng = np.random.default_rng(n + k)
    S = rng.normal(size=(B, n)).astype(np.float32)
    # heavy ties and both signs of zero
    S[:, ::7] = np.round(S[:, ::7], 1)
    S[0, :50] = 0.0
    S[0, 50:60] = -0.0
    idx = cc.lp_shortlist(_t(S), k).cpu().numpy()
    for b in range(B):
        # the k largest, ties to the smaller index: a stable sort of -S
        # (-0.0 and 0.0 compare equal to numpy, but not as float bit
        # patterns: take the order of the kernel's key, 0.0 above -0.0)
        key = S[b].astype(np.float64) + np.where(np.signbit(S[b]) & (S[b] == 0), -1e-300, 0.0)
        want = np.sort(np.argsort(-key, kind="stable")[:k])
        assert np.array_equal(idx[b], want), b   # ascending order


@pytest.mark.parametrize("B,n,k", [(3, 1000, 10), (2, 57121, 10), (1, 300, 256)])
def test_labels_match_a_sort(cc, B, n, k):
    # the k smallest exact scores, ties to the smaller index
    rng = np.random.default_rng(n)
    S = rng.integers(-5000, 5000, size=(B, n)).astype(np.int32)
    S[0, ::3] = S[0, 0]
    S[-1, :20] = np.iinfo(np.int32).min
    idx = cc.lp_labels(_t(S, np.int32), k).cpu().numpy()
    for b in range(B):
        want = np.sort(np.argsort(S[b].astype(np.int64), kind="stable")[:k])
        assert np.array_equal(idx[b], want), b   # ascending order


def test_shortlist_validation(cc):
    import torch
    S = torch.zeros((2, 100), device="cuda")
    with pytest.raises(cc.CcwsimError):
        cc.lp_shortlist(S, 0)
    with pytest.raises(cc.CcwsimError):
        cc.lp_shortlist(S, 101)
    with pytest.raises(cc.CcwsimError):
        cc.lp_shortlist(torch.zeros((2, 1000), device="cuda"), 257)
