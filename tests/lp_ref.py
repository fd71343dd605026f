"""Float64 numpy reference of the learned proposer's networks (test
infrastructure): the two 4-layer convolutional encoders, the scores, the
softmax cross-entropy against the best position, their gradients and one
Adam step, written out with plain array operations from the definitions.
Nothing here is shared with the HIP path."""
from __future__ import annotations

import numpy as np

C, D = 32, 64
LAYERS = [(9, 1), (9, 2), (9, 4), (1, 1)]   # (taps, dilation)


def layer_shapes(cin0):
    return [(C, cin0, 9), (C, C, 9), (C, C, 9), (D, C, 1)]


def unpack(w):
    """Weights buffer -> [(W, b)] for the key encoder, then the query's."""
    w = np.asarray(w, dtype=np.float64)
    out, o = [], 0
    for cin0 in (1, 2):
        enc = []
        for (co, ci, t) in layer_shapes(cin0):
            W = w[o: o + co * ci * t].reshape(co, ci, t)
            o += co * ci * t
            b = w[o: o + co]
            o += co
            enc.append((W, b))
        out.append(enc)
    assert o == w.size
    return out


def pack(grads):
    return np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for enc in grads for g in enc])


def _shift(x, dy, dx):
    """out[..., y, x] = x[..., y + dy, x + dx], zero outside."""
    out = np.zeros_like(x)
    H, W = x.shape[-2:]
    if abs(dy) >= H or abs(dx) >= W:
        return out
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    out[..., yd, xd] = x[..., ys, xs]
    return out


def _offsets(taps, dil):
    if taps == 1:
        return [(0, 0)]
    return [(dil * (t // 3 - 1), dil * (t % 3 - 1)) for t in range(9)]


def conv(x, W, b, taps, dil):
    out = np.zeros((x.shape[0], W.shape[0]) + x.shape[2:])
    for t, (dy, dx) in enumerate(_offsets(taps, dil)):
        out += np.einsum("oc,nchw->nohw", W[:, :, t], _shift(x, dy, dx))
    return out + b[None, :, None, None]


def encoder(enc, x):
    acts, h = [], x
    for l, ((W, b), (taps, dil)) in enumerate(zip(enc, LAYERS)):
        h = conv(h, W, b, taps, dil)
        if l < 3:
            h = np.maximum(h, 0.0)
            acts.append(h)
    return acts, h


def encoder_backward(enc, x, acts, dout):
    grads = [None] * 4
    d = dout
    for l in range(3, -1, -1):
        W, b = enc[l]
        taps, dil = LAYERS[l]
        lin = x if l == 0 else acts[l - 1]
        gW = np.zeros_like(W)
        for t, (dy, dx) in enumerate(_offsets(taps, dil)):
            gW[:, :, t] = np.einsum("nohw,nchw->oc", d, _shift(lin, dy, dx))
        grads[l] = (gW, d.sum(axis=(0, 2, 3)))
        if l == 0:
            break
        din = np.zeros_like(lin)
        for t, (dy, dx) in enumerate(_offsets(taps, dil)):
            din += _shift(np.einsum("oc,nohw->nchw", W[:, :, t], d), -dy, -dx)
        d = din * (lin > 0)
    return grads


def forward(w, K, beta, events, cand, tc):
    """keys [ncand, 64], queries [B, 64], scores [B, ncand] and the
    intermediate values for the backward pass."""
    kenc, qenc = unpack(w)
    kin = (np.asarray(K, dtype=np.float64) / beta)[None, None]
    kacts, kmap = encoder(kenc, kin)
    hy, hx = tc[1] // 2, tc[0] // 2
    keys = kmap[0][:, hy: hy + cand[1], hx: hx + cand[0]].reshape(D, -1).T
    ev = np.asarray(events, dtype=np.float64)
    qacts, qmap = encoder(qenc, ev)
    q = qmap[:, :, hy, hx]
    return keys, q, q @ keys.T, (kin, kacts, kmap, ev, qacts, qmap)


def loss_and_grad(w, K, beta, events, labels, cand, tc):
    """labels: [B] (the best candidate) or [B, L] (a set of distinct
    positives): loss = -log of the softmax mass on the set."""
    keys, q, S, (kin, kacts, kmap, ev, qacts, qmap) = forward(w, K, beta, events, cand, tc)
    B = S.shape[0]
    lab = np.asarray(labels).reshape(B, -1)
    m = S.max(axis=1, keepdims=True)
    e = np.exp(S - m)
    z = e.sum(axis=1, keepdims=True)
    rows = np.arange(B)[:, None]
    zt = e[rows, lab].sum(axis=1)
    loss = np.log(z[:, 0]) - np.log(zt)
    dS = e / z / B
    dS[rows, lab] -= e[rows, lab] / zt[:, None] / B
    dq = dS @ keys
    dkeys = dS.T @ q
    kenc, qenc = unpack(w)
    hy, hx = tc[1] // 2, tc[0] // 2
    dkmap = np.zeros_like(kmap)
    dkmap[0][:, hy: hy + cand[1], hx: hx + cand[0]] = dkeys.T.reshape(D, cand[1], cand[0])
    dqmap = np.zeros_like(qmap)
    dqmap[:, :, hy, hx] = dq
    gk = encoder_backward(kenc, kin, kacts, dkmap)
    gq = encoder_backward(qenc, ev, qacts, dqmap)
    return loss, pack([gk, gq])


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh, vh = m / (1 - b1 ** t), v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
