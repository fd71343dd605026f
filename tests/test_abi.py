"""CPU-side checks of the C ABI: the library builds, loads and exports every
function declared in include/ccwsim.h; host-side argument validation
returns the documented status codes without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ccwsim.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccwsim_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2404_00441_amd import ccwsim
    if not os.path.exists(ccwsim.LIB_PATH):
        from paper_2404_00441_amd import build
        build.build()
    return ccwsim.load()


def test_header_declares_the_five_entry_points():
    names = _declared()
    for n in ("ccwsim_dwt", "ccwsim_ccf_scan", "ccwsim_select", "ccwsim_idwt", "ccwsim_simulate"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2404_00441_amd import ccwsim
    names = _declared()
    assert set(names) == set(ccwsim.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    assert lib.ccwsim_status_string(0) == b"ok"
    assert lib.ccwsim_status_string(5) == b"unsupported"
    assert lib.ccwsim_status_string(99) == b"unknown status"


def test_dwt_sizes_host_only(lib):
    from paper_2404_00441_amd import ccwsim
    na, nd, _ = ccwsim.dwt_sizes((500, 500), 2)
    assert na == 125 * 125
    assert nd == 3 * 250 * 250 + 3 * 125 * 125
    na, nd, _ = ccwsim.dwt_sizes((180, 150, 60), 2)
    assert na == 45 * 38 * 15
    assert nd == 7 * (90 * 76 * 30) + 7 * (45 * 38 * 15)
    with pytest.raises(ccwsim.CcwsimError):
        ccwsim.dwt_sizes((10, 10), 7)


@pytest.mark.parametrize("bad", [
    dict(overlap=(24, 24)),            # T > OV violated
    dict(overlap=(0, 6)),              # OV >= 1 violated
    dict(tmpl=(200, 24)),              # template larger than the TI
    dict(top_k=0),
    dict(top_k=17),
    dict(n_real=0),
    dict(n_facies=0),
    dict(path_mode=2),
    dict(score_mode=3),
    dict(level=7),
    dict(shortlist=3),                 # below top_k
    dict(shortlist=33),                # above the longest shortlist
    dict(precision=5),
    dict(proposer_dim=7),
    dict(proposer_dim=16, shortlist=8),
    dict(proposer_dim=16, score_mode=1),
    dict(hd_direct=2),
    dict(wavelet=2),
    dict(wavelet=1, shortlist=8),
    dict(wavelet=1, proposer_dim=16),
    dict(proposer_dim=64, lp_probe=4),            # no proposer index
    dict(proposer_dim=65),
])
def test_simulate_validation_errors(lib, bad):
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    p, _, _ = wl.make("c1_plain2d")
    p.update(bad)
    q = ccwsim.params_of(p)
    assert lib.ccwsim_simulate_workspace_size(ctypes.byref(q)) == -1
    assert lib.ccwsim_last_error() != b""
    st = lib.ccwsim_simulate(ctypes.byref(q), ctypes.c_void_p(1), 0, None, None, None, ctypes.c_void_p(1),
                             None, ctypes.c_void_p(256), 1 << 30, None)
    assert st in (1, 2, 5)


def test_inexact_range_is_rejected(lib):
    # 3 facies at J = 3 in 2D: block sums up to 2 * 64 = 128 are fine, but a
    # level-4 grid of |beta| = 256 gives 512 -> still fine; codes up to 126 at
    # J = 3 give 8064 > 2048 and must be rejected before any launch
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    p, _, _ = wl.make("c1_plain2d")
    p.update(level=3, n_facies=127)
    q = ccwsim.params_of(p)
    assert lib.ccwsim_simulate_workspace_size(ctypes.byref(q)) == -1
    assert b"fp16" in lib.ccwsim_last_error()


def test_bf16_range_is_rejected(lib):
    # 3 facies at J = 3 in 2D: block sums up to 2 * 64 = 128 fit bf16, at
    # J = 4 (256 cells) they reach 512 and must be refused for bf16
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    p, _, _ = wl.make("c1_plain2d")
    p.update(level=4, n_facies=3, precision=1, tmpl=(48, 48), overlap=(12, 12))
    q = ccwsim.params_of(p)
    assert lib.ccwsim_simulate_workspace_size(ctypes.byref(q)) == -1
    assert b"bf16" in lib.ccwsim_last_error()


@pytest.mark.parametrize("name", ["c1_plain2d", "c2_scale2d", "c3_split3d", "c4_batched", "c5_learned"])
def test_every_workload_fits_the_kernel_limits(lib, name):
    # the plan checks LDS budgets and operand ranges; building it and sizing
    # the workspace are host work (no device is touched)
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    p, _, _ = wl.make(name)
    q = ccwsim.params_of(p)
    v = lib.ccwsim_simulate_workspace_size(ctypes.byref(q))
    assert v > 0, lib.ccwsim_last_error().decode()


def test_simulate_stats_host_only(lib):
    # the work accounting of a call needs no device
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    p, _, _ = wl.make("c2_scale2d")
    st = ccwsim.simulate_stats(p)
    assert st["patches"] == 33 * 33
    assert st["candidates"] == 116 * 116
    assert st["cells"] == 1000 * 1000
    assert st["scan_flops"] == 2.0 * st["or_blocks"] * st["candidates"]


def test_plan_cache_is_bounded(lib):
    # a caller sweeping seeds gets a new plan per seed; the cache keeps at
    # most 16 of them (least recently used dropped first)
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    ccwsim.release_caches()
    p, _, _ = wl.make("c1_plain2d", scale=0.3)
    for seed in range(200):
        p["seed"] = seed + 1
        assert ccwsim.simulate_workspace_size(p) > 0
        plans, graphs = ccwsim.cache_counts()
        assert plans <= 16
    assert ccwsim.cache_counts()[0] == 16
    ccwsim.release_caches()
    assert ccwsim.cache_counts() == (0, 0)


def test_scan_group_validation(lib):
    assert lib.ccwsim_set_scan_group(3) == 1
    assert b"tiles per scan workgroup" in lib.ccwsim_last_error()
    assert lib.ccwsim_set_scan_group(0) == 0


def test_stats_validation_errors(lib):
    from paper_2404_00441_amd import ccwsim
    sh = ccwsim.shape_of((40, 30))
    assert lib.ccwsim_stats_workspace_size(sh, 3) > 0
    assert lib.ccwsim_stats_workspace_size(ccwsim.shape_of((40, 0)), 3) == -1
    assert lib.ccwsim_stats_workspace_size(sh, -1) == -1
    fake = ctypes.c_void_p(256)
    # (n_img, n_facies, axis, max_lag): rejected before anything is launched
    for args in [(2, 0, 0, 5), (2, 128, 0, 5), (-1, 3, 0, 5), (2, 3, 2, 5), (2, 3, -1, 5), (2, 3, 0, 0),
                 (2, 3, 0, 40), (2, 3, 1, 30)]:
        n, nf, axis, lag = args
        st = lib.ccwsim_stats_variogram(fake, sh, n, nf, axis, lag, fake, fake, 1 << 30, None)
        assert st == 1, args
        st = lib.ccwsim_stats_connectivity(fake, sh, n, nf, axis, lag, fake, fake, fake, 1 << 30, None)
        assert st == 1, args
    assert lib.ccwsim_stats_variogram(fake, sh, 2, 3, 0, 39, fake, None, 0, None) == 3      # no workspace
    assert lib.ccwsim_stats_variogram(fake, sh, 2, 3, 1, 29, fake, ctypes.c_void_p(257), 1 << 30, None) == 3
    assert lib.ccwsim_stats_connectivity(fake, sh, 2, 3, 0, 39, fake, fake, fake, 16, None) == 3
    assert lib.ccwsim_stats_histogram(fake, ccwsim.shape_of((4, 4, 4, )), 1, 0, fake, None, None) == 1
    assert lib.ccwsim_stats_histogram(fake, sh, 1, 3, None, None, None) == 1
    # no images: nothing to do
    assert lib.ccwsim_stats_histogram(None, sh, 0, 3, fake, None, None) == 0
    assert lib.ccwsim_stats_variogram(None, sh, 0, 3, 0, 5, fake, None, 0, None) == 0


def test_selection_switch_validation(lib):
    assert lib.ccwsim_set_selection(4) == 1
    assert lib.ccwsim_set_selection(-1) == 1
    assert lib.ccwsim_set_selection(0) == 0


def test_learned_plan_fits(lib):
    # the learned proposer's plan (LDS of the proposal, packed scan tiles) is
    # host work; a stand-in index address is never read when sizing
    from paper_2404_00441_amd import ccwsim
    from paper_2404_00441_amd import workloads as wl
    p, _, _ = wl.make("c5_learned")
    q = ccwsim.params_of(p)
    q.proposer_dim, q.lp_probe, q.lp_gate, q.proposer = 64, 8, 0.5, 256
    v = lib.ccwsim_simulate_workspace_size(ctypes.byref(q))
    assert v > 0, lib.ccwsim_last_error().decode()
    for bad in [dict(lp_probe=0), dict(lp_probe=65), dict(lp_gate=float("nan"))]:
        q2 = ccwsim.params_of(p)
        q2.proposer_dim, q2.lp_probe, q2.lp_gate, q2.proposer = 64, 8, 0.5, 256
        for k, v2 in bad.items():
            setattr(q2, k, v2)
        assert lib.ccwsim_simulate_workspace_size(ctypes.byref(q2)) == -1


def test_proposer_skew_validation(lib):
    assert lib.ccwsim_set_proposer_skew(ctypes.c_float(-1.0)) == 1
    assert lib.ccwsim_set_proposer_skew(ctypes.c_float(float("nan"))) == 1
    assert lib.ccwsim_set_proposer_skew(ctypes.c_float(0.0)) == 0


def test_cdf97_sizes_and_validation(lib):
    from paper_2404_00441_amd import ccwsim
    sh = ccwsim.shape_of((120, 100))
    assert lib.ccwsim_dwt97_workspace_size(sh, 2) == 3 * (-(-120 * 100 * 4 // 256) * 256)   # three 256-aligned buffers
    assert lib.ccwsim_dwt97_workspace_size(ccwsim.shape_of((0, 100)), 2) == -1
    t = ccwsim._i3((24, 24), 1)
    ws = lib.ccwsim_ccf_scan97_workspace_size
    assert ws(sh, 2, 0, t, 8, 10, 0, 1, 1) > 0          # exact keys and the map
    assert ws(sh, 2, 0, t, 8, 10, 64, 0, 1) > 0         # bulk shortlist
    assert ws(sh, 2, 1, t, 8, 10, 64, 0, 1) > 0
    assert ws(sh, 2, 2, t, 8, 10, 64, 0, 1) == -1       # precision
    assert ws(sh, 2, 0, t, 8, 10, 4, 0, 1) == -1        # shortlist below top_k
    assert ws(sh, 2, 0, t, 8, 10, 129, 0, 1) == -1      # shortlist above 128
    assert ws(sh, 2, 0, t, 8, 17, 0, 0, 1) == -1        # top_k above 16
    assert ws(sh, 2, 0, t, 0, 10, 0, 0, 1) == -1        # no events
    assert ws(sh, 2, 0, t, 8, 10, 0, 0, 0) == -1        # no output
    big = ccwsim._i3((68, 68), 1)                       # 17 x 17 blocks > 256
    assert ws(sh, 2, 0, big, 8, 10, 0, 1, 0) == -1
    tall = ccwsim.shape_of((4, 1000))                   # 250 block rows of one block at J = 0
    assert ws(tall, 0, 0, ccwsim._i3((1, 250), 1), 8, 10, 0, 1, 0) == -1
    assert ws(tall, 0, 0, ccwsim._i3((1, 200), 1), 8, 10, 0, 1, 0) > 0
