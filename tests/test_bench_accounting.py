"""The bench's byte accounting (CPU): the window lags a step applies, sum
over pairs of min(W_ij, n + 1), averaged over the timed steps, against a
brute-force sum; the counted HBM traffic from the committed counter data and
its calibration, reported only for the kernel sources it was measured
on."""
import numpy as np

import bench


def test_near_lags_mean_equals_brute_force():
    rng = np.random.Generator(np.random.PCG64(11))
    W = rng.integers(1, 600, size=2000)
    for n0, n1 in ((0, 0), (0, 50), (100, 700), (599, 620), (1000, 1010)):
        ref = np.mean([np.minimum(W, n + 1).sum() for n in range(n0, n1 + 1)])
        assert bench.near_lags_mean(W, n0, n1) == ref


def test_near_lags_mean_at_full_history_is_the_window_sum():
    W = np.array([5, 17, 64, 128, 3])
    assert bench.near_lags_mean(W, 200, 300) == W.sum()


def _committed_traffic():
    import json
    import os

    with open(os.path.join(os.path.dirname(bench.__file__), "profiles", "k_near_fdph_fp64_n4096_m2048_traffic.json")) as f:
        return json.load(f)


def test_committed_counter_bytes_follow_from_the_calibration():
    """HBM bytes of a kernel = FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by what the counter read for a kernel of known traffic: the
    streaming-read probe for FETCH_SIZE (when the run holds it), a plain copy
    for WRITE_SIZE."""
    d = _committed_traffic()
    cal = d["copy_calibration"]
    pc = d.get("probe_calibration")
    if pc:
        sf = pc["bytes_read"] / (pc["fetch_kib"] * 1024.0)
    else:
        sf = cal["bytes_read"] / (cal["fetch_kib"] * 1024.0)
    sw = cal["bytes_written"] / (cal["write_kib"] * 1024.0)
    assert abs(d["scale_fetch"] - sf) <= 1e-9 * sf and abs(d["scale_write"] - sw) <= 1e-9 * sw
    for k in d["kernels"].values():
        ref = (k["fetch_kib"] * sf + k["write_kib"] * sw) * 1024.0
        assert abs(k["hbm_bytes"] - ref) <= 1e-9 * ref


def test_traffic_is_reported_only_for_the_measured_kernel_sources(tmp_path):
    import json

    d = _committed_traffic()
    good = dict(d, source_hash=bench._kernel_source_hash())
    stale = dict(d, source_hash="0" * 16)
    pg, ps = tmp_path / "good.json", tmp_path / "stale.json"
    pg.write_text(json.dumps(good))
    ps.write_text(json.dumps(stale))
    assert bench._traffic(str(pg), "k_near") == d["kernels"]["k_near"]["hbm_bytes"]
    assert bench._traffic(str(ps), "k_near") is None
    assert bench._traffic(str(pg), "no_such_kernel") is None
    assert bench._traffic(str(tmp_path / "missing.json"), "k_near") is None


def test_bench_refuses_more_than_one_gpu():
    """One GPU only: --gpus N > 1 (or a multi-rank launch) exits with a message
    before anything touches a device."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *argv], capture_output=True, text=True,
                           timeout=120, env=dict(os.environ, **env))
        assert r.returncode != 0
        assert "one GPU" in (r.stdout + r.stderr)
