"""The five synthetic workloads (sizes, seeds and input recipes).

Each workload is a plain dict of simulation parameters (extents as (x, y[, z]))
plus its seeded inputs.  The training images stand in for the paper's
images (Sec. 5): binary or 3-facies sinuous channels in 2D, elliptic tubes in
3D.  Hard data are samples of a reference image drawn by the same generator
with its own seed.

``scale`` < 1 shrinks a workload for parity tests: the TI and grid extents and
the hard-data counts shrink, template/overlap/level stay as they are (so the
method's geometry -- partial blocks, band shapes, wavefront concurrency -- is
the one of the full workload).
"""
from __future__ import annotations

import numpy as np

from . import synthetic as syn

WORKLOADS = ("c1_plain2d", "c2_scale2d", "c3_split3d", "c4_batched", "c5_learned")


def _base(**kw):
    d = dict(n_real=1, n_facies=2, seed=1, path_mode=0, score_mode=0,
             nc_margin=(-1, -1, -1), cut=1, shortlist=0)
    d.update(kw)
    return d


def _scaled(n, scale, minimum):
    return max(minimum, int(round(n * scale)))


def make(name: str, scale: float = 1.0, n_real: int | None = None):
    """Return (params, ti, hd) for a workload; hd is (real, pos, val) or None."""
    if name == "c1_plain2d":
        ti_n = (_scaled(150, scale, 40), _scaled(150, scale, 40))
        p = _base(ti=ti_n, grid=(_scaled(100, scale, 30),) * 2, tmpl=(24, 24), overlap=(6, 6),
                  level=1, top_k=5, n_facies=2, seed=1, path_mode=0)
        ti = syn.channel_image_2d(ti_n[0], ti_n[1], 6, 2, seed=101)
        hd = None
    elif name == "c2_scale2d":
        ti_n = (_scaled(500, scale, 60),) * 2
        g = (_scaled(1000, scale, 60),) * 2
        p = _base(ti=ti_n, grid=g, tmpl=(40, 40), overlap=(10, 10), level=2, top_k=10,
                  n_facies=3, seed=1, path_mode=1)
        ti = syn.channel_image_2d(ti_n[0], ti_n[1], max(3, int(round(25 * scale))), 3, seed=102)
        ref = syn.channel_image_2d(g[0], g[1], max(3, int(round(50 * scale))), 3, seed=202)
        hd = syn.sample_hard_data(ref, [max(1, int(round(300 * scale * scale)))], seed=302)
    elif name == "c3_split3d":
        ti_n = (_scaled(180, scale, 40), _scaled(150, scale, 40), _scaled(60, scale, 14))
        g = (_scaled(300, scale, 40), _scaled(300, scale, 40), _scaled(80, scale, 14))
        p = _base(ti=ti_n, grid=g, tmpl=(30, 30, 10), overlap=(6, 6, 3), level=2, top_k=10,
                  n_facies=2, seed=1, path_mode=1, shortlist=32)
        ti = syn.tube_image_3d(ti_n[0], ti_n[1], ti_n[2], max(4, int(round(40 * scale))), seed=103)
        hd = None
    elif name == "c4_batched":
        nr = 64 if n_real is None else n_real
        ti_n = (_scaled(400, scale, 60),) * 2
        g = (_scaled(256, scale, 50),) * 2
        p = _base(ti=ti_n, grid=g, tmpl=(32, 32), overlap=(8, 8), level=2, top_k=10,
                  n_facies=3, seed=1, path_mode=1, n_real=nr)
        ti = syn.channel_image_2d(ti_n[0], ti_n[1], max(3, int(round(20 * scale))), 3, seed=104)
        ref = syn.channel_image_2d(g[0], g[1], max(3, int(round(13 * scale))), 3, seed=204)
        counts = np.random.default_rng(404).integers(0, 501, size=nr)
        counts = np.maximum(0, np.round(counts * scale * scale)).astype(int)
        hd = syn.sample_hard_data(ref, counts, seed=304)
    elif name == "c5_learned":
        nr = 16 if n_real is None else n_real
        ti_n = (_scaled(1000, scale, 80),) * 2
        g = (_scaled(2000, scale, 80),) * 2
        p = _base(ti=ti_n, grid=g, tmpl=(48, 48), overlap=(12, 12), level=2, top_k=10,
                  n_facies=3, seed=1, path_mode=1, n_real=nr)
        ti = syn.channel_image_2d(ti_n[0], ti_n[1], max(3, int(round(50 * scale))), 3, seed=105)
        hd = None
    else:
        raise KeyError(name)
    if n_real is not None:
        p["n_real"] = n_real
    p["name"] = name
    p["max_hard_data"] = 0 if hd is None else int(len(hd[0]))
    return p, ti, hd


def dense_conditioning(n_hd: int, scale: float = 1.0):
    """The C2 workload with n_hd hard data instead of 300 (dense conditioning:
    4000 or 8000 at full size, the count scaled with the grid area)."""
    p, ti, _ = make("c2_scale2d", scale=scale)
    g = p["grid"]
    ref = syn.channel_image_2d(g[0], g[1], max(3, int(round(50 * scale))), 3, seed=202)
    hd = syn.sample_hard_data(ref, [max(1, int(round(n_hd * scale * scale)))], seed=303)
    p["name"] = f"c2_dense{n_hd}"
    p["max_hard_data"] = int(len(hd[0]))
    return p, ti, hd


def ensemble(n_real: int = 100, scale: float = 1.0):
    """The C2 workload as an ensemble: n_real realizations in one call, all
    conditioned by the same 300 hard data (the set-up of the ensemble map
    and of the variogram and connection checks)."""
    p, ti, hd = make("c2_scale2d", scale=scale)
    real, pos, val = hd
    m = len(real)
    hd = (np.repeat(np.arange(n_real, dtype=np.int32), m), np.tile(pos, (n_real, 1)), np.tile(val, n_real))
    p["n_real"] = n_real
    p["name"] = f"c2_ensemble{n_real}"
    p["max_hard_data"] = int(len(hd[0]))
    return p, ti, hd


def level_grid_case(level: int, grid_n: int, hd_per_512: int = 1000):
    """Level x grid-size sweep: the C2 training image (500^2, 3 facies),
    template 32, overlap 8, level J, a grid_n^2 grid conditioned by
    hd_per_512 * (grid_n / 512)^2 hard data, seeded path."""
    ti = syn.channel_image_2d(500, 500, 25, 3, seed=102)
    n_hd = max(1, int(round(hd_per_512 * (grid_n / 512.0) ** 2)))
    ref = syn.channel_image_2d(grid_n, grid_n, max(3, int(round(25 * grid_n / 500))), 3, seed=206)
    hd = syn.sample_hard_data(ref, [n_hd], seed=306)
    p = _base(ti=(500, 500), grid=(grid_n, grid_n), tmpl=(32, 32), overlap=(8, 8), level=level, top_k=10,
              n_facies=3, seed=1, path_mode=1)
    p["name"] = f"sweep_J{level}_n{grid_n}"
    p["max_hard_data"] = int(len(hd[0]))
    return p, ti, hd


def describe(p) -> str:
    return (f"{p['name']}: TI {'x'.join(map(str, p['ti']))}, grid {'x'.join(map(str, p['grid']))}"
            f" x{p['n_real']}, T {'x'.join(map(str, p['tmpl']))}, OV {'x'.join(map(str, p['overlap']))},"
            f" J={p['level']}, k={p['top_k']}")
