"""Brute-force restatement of the simulation for tiny inputs (test helper).

Written independently of the C oracle so that the oracle can be pinned to
something other than itself:

* the score of a candidate is computed in the SPATIAL domain as the sum of
  squared differences between the level-J block means of the TI window and of
  the known overlap cells (exact rationals), which is what the CCW of Haar
  approximations measures (Haar scaling function = box, Sec. 4.2; CCW, Sec.
  4.3) -- no wavelet transform and no block-sum grid are used;
* the chosen pattern is the TI crop itself (perfect reconstruction, Sec. 3.1),
  not an inverse transform;
* the boundary cut enumerates every 8-connected seam instead of running a
  dynamic programme;
* candidates are ordered by a plain tuple sort, not by packed keys.

With the LeGall 5/3 wavelet (p["wavelet"] = 1) the score is the sum of
squared differences between the TI's level-J approximation at the
candidate's blocks and the approximation of the zero-filled overlap window,
over the blocks holding a known cell (exact integers), minus the constant
sum of the window approximation's squares; the lifting is written out here
with plain integer loops.

Only the random inputs (the counter-based generator and the tie-break
bijection, pinned on their own by known-answer and bijection tests) are taken
from the oracle.
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def lattice_count(n_grid: int, T: int, OV: int) -> int:
    """Smallest number of patches n >= 1 with n*(T-OV) + OV >= n_grid."""
    n = 1
    while n * (T - OV) + OV < n_grid:
        n += 1
    return n


def enumerate_seams(rows: int, cols: int):
    """All 8-connected seams: one column per row, moving by at most 1."""
    def rec(prefix):
        if len(prefix) == rows:
            yield tuple(prefix)
            return
        last = prefix[-1]
        for w in (last - 1, last, last + 1):
            if 0 <= w < cols:
                yield from rec(prefix + [w])
    for w0 in range(cols):
        yield from rec([w0])


_MOVE_RANK = {0: 0, -1: 1, 1: 2}


def best_seam(e: np.ndarray):
    """Minimal-error seam by enumeration, ties resolved like the DP reading:
    the smallest final column first, then, walking back up, the predecessor
    at the same column, then one to the left, then one to the right."""
    rows, cols = e.shape
    best = None
    for s in enumerate_seams(rows, cols):
        cost = sum(int(e[y, s[y]]) for y in range(rows))
        tie = [s[rows - 1]] + [_MOVE_RANK[s[y] - s[y + 1]] for y in range(rows - 2, -1, -1)]
        key = (cost, tie)
        if best is None or key < best[0]:
            best = (key, s)
    return np.array(best[1], dtype=np.int32), best[0][0]


def _lift_low(line):
    """Low-pass half of one 5/3 integer lifting level (mirror extension)."""
    n = len(line)

    def x(i):
        while i < 0 or i >= n:
            i = -i if i < 0 else 2 * (n - 1) - i
        return line[i]

    def d(k):
        return x(2 * k + 1) - (x(2 * k) + x(2 * k + 2)) // 2

    return [x(2 * k) + (d(k - 1) + d(k) + 2) // 4 for k in range(n // 2)]


def _approx53(arr, J):
    """Level-J approximation of an integer array indexed [x][y][z]."""
    a = np.asarray(arr, dtype=object)
    for _ in range(J):
        for ax in range(a.ndim):
            a = np.apply_along_axis(lambda v: np.array(_lift_low(list(v)), dtype=object), ax, a)
    return a


def simulate(p: dict, ti: np.ndarray, hd, rng, perm20):
    """Brute-force realizations; p is a workload dict (extents (x, y[, z]))."""
    ndim = len(p["ti"])
    J = p["level"]
    b = 2 ** J
    T = list(p["tmpl"])
    OV = list(p["overlap"])
    Nti = list(p["ti"])
    Nsg = list(p["grid"])
    margin = [OV[a] if (p["nc_margin"][a] if a < len(p["nc_margin"]) else -1) < 0 else p["nc_margin"][a]
              for a in range(ndim)]
    lat = [lattice_count(Nsg[a], T[a], OV[a]) for a in range(ndim)]
    pad = [lat[a] * (T[a] - OV[a]) + OV[a] for a in range(ndim)]
    cand = [(Nti[a] - T[a]) // b + 1 for a in range(ndim)]
    ncand = int(np.prod(cand))
    beta = b ** ndim
    # numpy arrays are indexed [z][y][x]; helpers take (x, y[, z]) tuples
    tiT = np.asarray(ti).transpose()          # now indexed [x][y][z]

    def ti_at(pt):
        return int(tiT[tuple(pt)])

    wav = p.get("wavelet", 0)
    if wav == 1:
        npad = [-(-Nti[a] // b) * b for a in range(ndim)]
        rep_ti = np.empty(npad, dtype=object)
        for pt in itertools.product(*[range(npad[a]) for a in range(ndim)]):
            rep_ti[pt] = ti_at([min(pt[a], Nti[a] - 1) for a in range(ndim)])
        K53 = _approx53(rep_ti, J)
    tcb = [-(-T[a] // b) for a in range(ndim)]

    def ti_block_mean(fine_lo):
        # mean of the b^d TI cells of a block, edge-replicated past the border
        s = 0
        for off in itertools.product(range(b), repeat=ndim):
            pt = [min(fine_lo[a] + off[a], Nti[a] - 1) for a in range(ndim)]
            s += ti_at(pt)
        return Fraction(s, beta)

    outs, chosen_all = [], []
    nsteps = int(np.prod(lat))
    for r in range(p["n_real"]):
        sg = np.full(pad, -1, dtype=np.int64)      # indexed [x][y][z]
        hdv = {}
        if hd is not None:
            for i in range(len(hd[0])):
                if int(hd[0][i]) == r:
                    pos = tuple(int(v) for v in hd[1][i])
                    sg[pos] = int(hd[2][i])
                    hdv[pos] = int(hd[2][i])
        perm = list(range(ndim))
        flip = [0] * ndim
        if p["path_mode"] == 1:
            u = rng(p["seed"], 1, r, 0)
            flip = [(u >> a) & 1 for a in range(ndim)]
            if ndim == 2 and (u >> 3) & 1:
                perm = [1, 0]
        plen = [lat[perm[k]] for k in range(ndim)]
        chosen = []
        for step in range(nsteps):
            q, rem = [], step
            for k in range(ndim):
                q.append(rem % plen[k])
                rem //= plen[k]
            li = [0] * ndim
            band = [False] * ndim
            for k in range(ndim):
                a = perm[k]
                li[a] = lat[a] - 1 - q[k] if flip[a] else q[k]
                band[a] = q[k] > 0
            org = [li[a] * (T[a] - OV[a]) for a in range(ndim)]

            def w_of(a, ua):
                return T[a] - 1 - ua if flip[a] else ua

            cells = list(itertools.product(*[range(T[a]) for a in range(ndim)]))
            M = [u for u in cells if any(band[a] and w_of(a, u[a]) < OV[a] for a in range(ndim))]
            # block means of the known overlap cells
            blk_n, blk_m = {}, {}
            for u in M:
                bk = tuple(u[a] // b for a in range(ndim))
                v = int(sg[tuple(org[a] + u[a] for a in range(ndim))])
                assert v >= 0
                blk_n[bk] = blk_n.get(bk, 0) + 1
                blk_m[bk] = blk_m.get(bk, 0) + v
            const = sum(Fraction(blk_m[k] ** 2, blk_n[k]) for k in blk_n) * beta * beta
            if wav == 1:
                win = np.zeros([tcb[a] * b for a in range(ndim)], dtype=object)
                for u in M:
                    win[u] = int(sg[tuple(org[a] + u[a] for a in range(ndim))])
                A = _approx53(win, J)
                const53 = sum(int(A[k]) ** 2 for k in blk_n)
            # hard data in the virtual template
            vlo = [(-margin[a] if flip[a] else 0) for a in range(ndim)]
            vhi = [(T[a] if flip[a] else T[a] + margin[a]) for a in range(ndim)]
            hd_in = [(tuple(pos[a] - org[a] for a in range(ndim)), v) for pos, v in hdv.items()
                     if all(vlo[a] <= pos[a] - org[a] < vhi[a] for a in range(ndim))]
            tkey = rng(p["seed"], 2, r, step)
            order = []
            for idx in range(ncand):
                c, rem = [], idx
                for a in range(ndim):
                    c.append(rem % cand[a])
                    rem //= cand[a]
                if wav == 1:
                    S = Fraction(sum((int(K53[tuple(c[a] + k[a] for a in range(ndim))]) - int(A[k])) ** 2
                                     for k in blk_n) - const53)
                else:
                    ssd = Fraction(0)
                    for u in M:
                        bk = tuple(u[a] // b for a in range(ndim))
                        pti = ti_block_mean([b * c[a] + b * bk[a] for a in range(ndim)])
                        por = Fraction(blk_m[bk], blk_n[bk])
                        ssd += (pti - por) ** 2
                    S = ssd * beta * beta - const
                assert S.denominator == 1
                mis = 0
                for uu, v in hd_in:
                    pt = [b * c[a] + uu[a] for a in range(ndim)]
                    if all(0 <= pt[a] < Nti[a] for a in range(ndim)) and ti_at(pt) != v:
                        mis += 1
                order.append((min(mis, 4095), int(S), perm20(idx, tkey), idx))
            order.sort()
            kk = min(p["top_k"], ncand)
            j = ((rng(p["seed"], 3, r, step) >> 32) * kk) >> 32
            pick = order[j][3]
            chosen.append(pick)
            c, rem = [], pick
            for a in range(ndim):
                c.append(rem % cand[a])
                rem //= cand[a]
            patch = {u: ti_at([b * c[a] + u[a] for a in range(ndim)]) for u in cells}
            keep_old = set()
            if p["cut"]:
                for a in range(ndim):
                    if not band[a]:
                        continue
                    ra = 1 if a == 0 else 0
                    others = [x for x in range(ndim) if x not in (a, ra)]
                    sa = others[0] if others else None
                    nsl = T[sa] if sa is not None else 1
                    for sl in range(nsl):
                        e = np.zeros((T[ra], OV[a]), dtype=np.int64)
                        for y in range(T[ra]):
                            for w in range(OV[a]):
                                u = [0] * ndim
                                u[a] = T[a] - 1 - w if flip[a] else w
                                u[ra] = y
                                if sa is not None:
                                    u[sa] = sl
                                sv = int(sg[tuple(org[x] + u[x] for x in range(ndim))])
                                e[y, w] = (sv - patch[tuple(u)]) ** 2
                        seam, _ = best_seam(e)
                        for y in range(T[ra]):
                            for w in range(int(seam[y])):
                                u = [0] * ndim
                                u[a] = T[a] - 1 - w if flip[a] else w
                                u[ra] = y
                                if sa is not None:
                                    u[sa] = sl
                                keep_old.add(tuple(u))
            for u in cells:
                at = tuple(org[a] + u[a] for a in range(ndim))
                if at in hdv or u in keep_old:
                    continue
                sg[at] = patch[u]
        crop = sg[tuple(slice(0, Nsg[a]) for a in range(ndim))]
        outs.append(crop.transpose().astype(np.int8))
        chosen_all.append(chosen)
    return np.stack(outs), np.array(chosen_all, dtype=np.int32)
