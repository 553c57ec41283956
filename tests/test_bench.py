"""Host-side parts of bench.py: the byte models its roofline uses and the refusal of
more than one GPU (no GPU needed).

The algorithmic bytes per voxel-iteration are pinned against the sweep counts of
the method (forward sweep, backward sweep, direction, further line-search
passes), written out here term by term for MIX and F64, and against the three
values the roofline is quoted with (L = 3 MIX: 168 B, L = 3 F64: 320 B,
L = 6 MIX: 240 B).
"""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("L", [2, 3, 4, 6])
@pytest.mark.parametrize("nmls", [1, 2, 3, 5])
def test_alg_bytes_by_sweep(bench, L, nmls):
    # MIX: echo data 8L (complex64), f/z/g/D/x 4 B, pivots 8 B
    fwd = 8 * L + 4 + 4 + (4 + 4 + 4 + 8 + 4)          # in: echoes, f, z_prev; out: f, g, D, pivot, x
    bwd = 4 + 8 + 4 + 4 + 4 + 4                          # in: x, pivot, g, g_prev, z_prev; out: p
    dirn = 4 + 4 + 4 + 4 + 4                             # in: p, z_prev, f, D; out: z
    mls = 8 * L + 4 + 4                                  # in: echoes, f, z
    assert bench.alg_bytes_per_voxel("mix", L, nmls) == fwd + bwd + dirn + (nmls - 1) * mls
    # F64: every per-voxel value 8 B, echoes 16L
    fwd = 16 * L + 8 + 8 + (8 + 8 + 8 + 8 + 8)
    bwd = 6 * 8
    dirn = 5 * 8
    mls = 16 * L + 16
    assert bench.alg_bytes_per_voxel("f64", L, nmls) == fwd + bwd + dirn + (nmls - 1) * mls


def test_alg_bytes_quoted_values(bench):
    assert bench.alg_bytes_per_voxel("mix", 3, 3) == 168
    assert bench.alg_bytes_per_voxel("f64", 3, 3) == 320
    assert bench.alg_bytes_per_voxel("mix", 6, 3) == 240


def test_pass_model_of_the_red_black_iteration(bench):
    # gradient 49 (code, echoes, f, z_prev / f, g, D, 1/h of red voxels), black 17, red + direction 23,
    # two line-search passes 33 each
    assert bench.bytes_per_voxel("grad", "mix", 3, "redblack", "ic0") == 49
    assert bench.bytes_per_voxel("precond_a", "mix", 3, "redblack", "ic0") == 17
    assert bench.bytes_per_voxel("precond_b", "mix", 3, "redblack", "ic0") == 23
    assert bench.bytes_per_voxel("mls", "mix", 3, "redblack", "ic0") == 33
    assert bench.iteration_bytes_per_voxel("mix", 3, "redblack", "ic0", 3) == 155
    # the direction pass is separate for the other preconditioners
    assert bench.iteration_bytes_per_voxel("mix", 3, "natural", "diag", 3) == \
        45 + bench.bytes_per_voxel("precond_a", "mix", 3, "natural", "diag") + 21 + 2 * 33


def test_second_order_model(bench):
    for prec in ("mix", "f64"):
        vals = {k: bench.order2_bytes_per_voxel(k, prec, 3) for k in ("grad", "precond_a", "precond_b", "dir", "mls")}
        assert all(v > 0 for v in vals.values())
    # MIX, t = 4: forward passes (22 + 20) / 2, backward (10.33 + 9) / 2
    assert abs(bench.order2_bytes_per_voxel("precond_a", "mix", 3) - 21.0) < 1e-9
    assert abs(bench.order2_bytes_per_voxel("precond_b", "mix", 3) - (31 / 3 + 9) / 2) < 1e-9


def test_kernel_symbols(bench):
    assert bench.kernel_symbol("precond_a", "redblack", "ic0", 64) == "k_rb_black_pair"
    assert bench.kernel_symbol("precond_b", "redblack", "ic0", 63) == "k_rb_red_dir"
    assert bench.kernel_symbol("precond_a", "natural", "ic0", 64) == "k_ic_fwd_wave"
    assert bench.kernel_symbol("grad", "redblack", "ic0", 64) == "k_grad"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr or "single" in r.stderr
    assert r.stdout.strip() == ""


def test_source_hash_ignores_comments_only():
    from paper_2005_08661_amd.prof_summary import _code_only
    a = 'int a = 1; // one\n/* block\n comment */ const char *s = "x // not a comment /* nor this */";\n\n'
    b = 'int a = 1;\n const char *s = "x // not a comment /* nor this */";'
    assert _code_only(a) == _code_only(b)
    assert _code_only("char q = '\"'; int b; // tail") == "char q = '\"'; int b;"
    assert _code_only("int a = 1;") != _code_only("int a = 2;")


def test_flip_threshold_and_map_diff(bench):
    # TE 0 / 2.2 / 4.4 ms: the closest pair is 2.2 ms apart, half its wrap period is 1/(2 * 2.2 ms)
    assert bench.flip_threshold([0.0, 2.2e-3, 4.4e-3]) == pytest.approx(1.0 / 4.4e-3)
    a = [[0.0, 1.0], [2.0, 300.0]]
    b = [[0.0, 0.0], [2.0, 0.0]]
    m = [[True, True], [True, False]]
    import numpy as np
    d = bench.map_diff(np.array(a), np.array(b), np.array(m), 227.0)
    assert d["max_abs_hz"] == 1.0 and d["basin_flips"] == 0
    assert d["rms_hz"] == pytest.approx(np.sqrt(1.0 / 3.0))
    d = bench.map_diff(np.array(a), np.array(b), np.ones((2, 2), bool), 227.0)
    assert d["basin_flips"] == 1


def test_host_threads_respects_environment(bench, monkeypatch):
    n = len(os.sched_getaffinity(0))
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    assert bench.host_threads() == 1
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.host_threads() == n


def test_roofline_limiter_from_measured_traffic(bench):
    kinfo = {"resident": {"gbs": 3500.0, "avg_us": 5000.0}}
    e = bench.roofline_entry(kinfo, "resident", None)
    assert e["bound"] == "hbm" and e["frac"] == pytest.approx(3500.0 / 8000.0) and e["limiter"] is None
    e = bench.roofline_entry(kinfo, "resident", 8.3e9)  # 8.3 GB in 5 ms: 1.66 TB/s
    assert e["measured_frac"] == pytest.approx(8.3e9 / 5e-3 / 8e12)
    assert e["limiter"].startswith("latency")
    e = bench.roofline_entry(kinfo, "resident", 25e9)
    assert e["limiter"] == "hbm bandwidth"


def test_pass_model_of_the_block_red_black_sweeps(bench):
    """Block red-black sweeps move the arrays of the natural-order sweeps (one tile at a time): forward
    code, D, g in and 1/P (8 bytes), x out; backward code, x, 1/P, g, g_prev in and p out.  The profile
    names the block kernels."""
    for prec, t in (("mix", 4), ("f64", 8)):
        assert bench.bytes_per_voxel("precond_a", prec, 3, "blockrb", "ic0") == 1 + 3 * t + 8
        assert bench.bytes_per_voxel("precond_b", prec, 3, "blockrb", "ic0") == 1 + 4 * t + 8
        for kc in ("precond_a", "precond_b"):
            assert (bench.bytes_per_voxel(kc, prec, 3, "blockrb", "ic0")
                    == bench.bytes_per_voxel(kc, prec, 3, "natural", "ic0"))
    assert bench.kernel_symbol("precond_a", "blockrb", "ic0", 64) == "k_icb_fwd"
    assert bench.kernel_symbol("precond_b", "blockrb", "ic0", 64) == "k_icb_bwd"
    assert bench.kernel_symbol("precond_a", "natural", "ic0", 64) == "k_ic_fwd_wave"
