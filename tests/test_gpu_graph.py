"""Captured steps (bie_run_graph) against eager launches (bie_run).

Up to 32 steps are captured as a HIP graph and launched once per 32 steps;
the step index comes from a device counter.  A graph call runs the same
kernels in the same order as a bie_run call over the same steps (time blocks
at the same steps), so the tractions must be bit-identical to eager launches
cut into the same calls, across several graph calls with eager steps in
between (each call captures a new graph after the previous one finished).
Calls cut elsewhere put the time blocks of the near field at other steps,
whose matrix-core sums agree to rounding.
"""
import numpy as np
import pytest

from synth import smooth_slip_rate, straight_fault, curved_fault

pytestmark = pytest.mark.gpu


def _eager(op, Dd, torch):
    s = torch.cuda.current_stream()
    T = torch.zeros_like(Dd)
    op.reset(stream=s)
    op.run(Dd, T, stream=s)
    torch.cuda.synchronize()
    return T.cpu().numpy()


def _mixed(op, Dd, torch, cuts, graph=True):
    """Graph for [0, c0), eager for [c0, c1), graph for [c1, c2), ... (with
    graph=False every call eager)."""
    s = torch.cuda.current_stream()
    T = torch.zeros_like(Dd)
    op.reset(stream=s)
    bounds = [0, *cuts, Dd.shape[0]]
    for k in range(len(bounds) - 1):
        a, b = bounds[k], bounds[k + 1]
        if b <= a:
            continue
        if k % 2 == 0 and graph:
            op.run_graph(Dd[a:b], T[a:b], stream=s)
        else:
            op.run(Dd[a:b], T[a:b], stream=s)
        torch.cuda.synchronize()
    assert op.stats()["steps_done"] == Dd.shape[0]
    return T.cpu().numpy()


@pytest.mark.parametrize("kind", ["dense", "fdph", "fdph_mixed", "batched"])
def test_graph_steps_equal_eager_steps(gpu_lib, kind):
    import torch

    from paper_1903_02118_amd.binding import BIE_MIXED_FP32, Operator, make_params

    if kind == "dense":
        N, M = 96, 60
        xa, xb = straight_fault(N)
        op = Operator.build_kernel(xa, xb, M)
    elif kind == "batched":
        faults = [(*straight_fault(130), 200), (*curved_fault(96), 150)]
        op = Operator.compress_fdph_batched(faults, params=make_params())
        N, M = 226, 200
    else:
        N, M = 256, 300
        xa, xb = straight_fault(N)
        prec = BIE_MIXED_FP32 if kind == "fdph_mixed" else 0
        op = Operator.compress_fdph(xa, xb, M, params=make_params(precision=prec))
    D = smooth_slip_rate(N, M, 10, 20, 9)
    Dd = torch.from_numpy(D).to("cuda")
    print(f"graph {kind} N={N} M={M}", flush=True)
    Te = _eager(op, Dd, torch)
    for cuts in ([M // 3, M // 2], [1, 2, M - 1], [32, 64]):
        Tg = _mixed(op, Dd, torch, cuts)
        Tc = _mixed(op, Dd, torch, cuts, graph=False)
        assert np.array_equal(Tg, Tc), (kind, cuts, float(np.abs(Tg - Tc).max()))
        tol = 1e-5 if kind == "fdph_mixed" else 1e-12
        assert np.abs(Tg - Te).max() <= tol * np.abs(Te).max(), (kind, cuts)
    op.close()


def test_autotuned_near_kernel_gives_identical_steps(gpu_lib):
    """Near-kernel configurations of one load width perform the same
    arithmetic per work item: after the autotuner picks one, the tractions
    are bit-identical.  A different load width sums each receiver's lags in
    another order, so the tractions then agree to rounding."""
    import torch

    from paper_1903_02118_amd.binding import Operator, make_params

    faults = [(*straight_fault(300), 400), (*curved_fault(200), 300)]
    op = Operator.compress_fdph_batched(faults, params=make_params())
    N, M = 500, 400
    D = smooth_slip_rate(N, M, 10, 20, 13)
    Dd = torch.from_numpy(D).to("cuda")
    Te = _eager(op, Dd, torch)
    s = torch.cuda.current_stream()
    T = torch.zeros_like(Dd)
    # cut after whole time blocks, so that both runs put them at the same steps
    op.reset(stream=s)
    op.run(Dd[:144], T[:144], stream=s)
    res = op.autotune(reps=2, stream=s)
    print("autotune", res, flush=True)
    assert res["candidates"] >= 4 and res["best_ms"] <= res["default_ms"]
    op.run(Dd[144:], T[144:], stream=s)
    torch.cuda.synchronize()
    Tg = T.cpu().numpy()
    # the default configuration of an FP64 operator: 16-byte loads per step,
    # the matrix-core kernel for time blocks
    if res["load_bytes"] == 16 and res["mfma"] == 1:
        assert np.array_equal(Tg, Te)
    else:
        assert np.allclose(Tg, Te, rtol=1e-12, atol=1e-12 * np.abs(Te).max())
    op.close()


def test_cached_graph_replays_after_reset(gpu_lib):
    """A second graph run with the same buffers from step 0 replays the cached
    graph; its tractions equal the eager ones."""
    import torch

    from paper_1903_02118_amd.binding import Operator, make_params

    N, M = 200, 160
    xa, xb = straight_fault(N)
    op = Operator.compress_fdph(xa, xb, M, params=make_params())
    Dd = torch.from_numpy(smooth_slip_rate(N, M, 10, 20, 17)).to("cuda")
    Te = _eager(op, Dd, torch)
    s = torch.cuda.current_stream()
    T = torch.zeros_like(Dd)
    for _ in range(3):
        op.reset(stream=s)
        T.zero_()
        op.run_graph(Dd, T, stream=s)
        torch.cuda.synchronize()
        assert np.array_equal(T.cpu().numpy(), Te)
    op.close()


def test_autotune_drops_the_cached_graph(gpu_lib, monkeypatch):
    """A graph captured before the autotuner ran holds the old near-kernel
    configuration; after bie_autotune the same run_graph call recaptures, so
    it equals eager steps with the tuned configuration (here the narrow
    8-byte loads at first, so that the tuned load width may differ)."""
    import torch

    from paper_1903_02118_amd.binding import Operator, make_params

    monkeypatch.setenv("BIE_NEAR_WIDE", "0")
    N, M = 200, 160
    xa, xb = straight_fault(N)
    op = Operator.compress_fdph(xa, xb, M, params=make_params())
    Dd = torch.from_numpy(smooth_slip_rate(N, M, 10, 20, 18)).to("cuda")
    s = torch.cuda.current_stream()
    T = torch.zeros_like(Dd)
    op.reset(stream=s)
    op.run_graph(Dd, T, stream=s)
    torch.cuda.synchronize()
    tune = op.autotune(reps=2, stream=s)
    print("autotune", tune, flush=True)
    Te = _eager(op, Dd, torch)
    op.reset(stream=s)
    T.zero_()
    op.run_graph(Dd, T, stream=s)
    torch.cuda.synchronize()
    assert np.array_equal(T.cpu().numpy(), Te)
    op.close()
