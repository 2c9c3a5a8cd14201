"""Time blocks of prescribed-slip runs: the near field of BIE_TIME_BLOCK consecutive steps
in one pass over the windows (bie_run, bie_run_graph) against the same
operator stepped one step at a time (bie_step), and against an operator
built without time blocks.

Two kernels take a block's near field.  The matrix-core kernel (the default;
BIE_NEAR_MFMA=2 its work items of up to four lag chunks of a tile) adds the
same products as the single-step kernel in another order (16 x 16 MFMA tiles;
FP32 windows multiply the history rounded to FP32 and accumulate in FP32
within a work item), so the tractions agree to rounding: 1e-12 of their norm
with FP64 windows, 1e-5 in the mixed modes.  The lane-per-lag kernel adds
them in the single-step kernel's order, so its tractions are bit-identical.
The far-field scatter of a block's 16 steps in one launch is bit-identical to
one launch per step.  The runs include a remainder shorter than a block,
blocks that start before the first history reaches a chunk, and batched
faults whose runs end inside a block (tiles of fewer than 16 receivers).
"""
import numpy as np
import pytest

from synth import curved_fault, smooth_slip_rate, straight_fault

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "mixed": 1e-5}


def _run(op, D, mode):
    import torch

    s = torch.cuda.current_stream()
    Dd = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    Td = torch.full_like(Dd, np.nan)
    op.reset(stream=s)
    if mode == "run":
        op.run(Dd, Td, stream=s)
    elif mode == "graph":
        op.run_graph(Dd, Td, stream=s)
    else:
        for n in range(D.shape[0]):
            op.step(Dd[n], Td[n], stream=s)
    torch.cuda.synchronize()
    return Td.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("mfma", ["1", "2"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("geom", ["planar", "curved"])
def test_time_blocks_agree_with_single_steps(gpu_lib, monkeypatch, prec, geom, mfma):
    """mfma 2: work items of up to four consecutive lag chunks of a tile, one
    partial sum per receiver and step for the group."""
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32, BIE_TIME_BLOCK, Operator, make_params

    monkeypatch.setenv("BIE_NEAR_MFMA", mfma)
    N, M = (600, 403) if geom == "planar" else (384, 251)
    xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 33)
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32
    print(f"time blocks {geom} {prec} N={N} M={M} mfma {mfma}", flush=True)
    opb = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, precision=code,
                                                               time_block=BIE_TIME_BLOCK))
    op1 = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, precision=code, time_block=1))
    T_run = _run(opb, D, "run")
    T_graph = _run(opb, D, "graph")
    T_step = _run(opb, D, "step")
    T_one = _run(op1, D, "run")
    assert opb.stats()["time_block"] == BIE_TIME_BLOCK
    opb.close()
    op1.close()
    assert np.isfinite(T_run).all()
    # the same launches in a graph: the same sums
    assert np.array_equal(T_graph, T_run)
    err_step = _rel(T_run, T_step)
    # another operator (ring lengths differ, windows and factors the same up
    # to ACA+'s random references)
    err_one = _rel(T_run, T_one)
    print(f"  blocked vs single steps {err_step:.2e}, vs operator without blocks {err_one:.2e}", flush=True)
    assert err_step <= TOL[prec] and err_one <= TOL[prec]
    # element-wise too: no traction off by more than 10x that of the largest
    assert np.abs(T_run - T_step).max() <= 10 * TOL[prec] * np.abs(T_step).max()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_lane_per_lag_time_blocks_equal_single_steps(gpu_lib, monkeypatch, prec):
    """The lane-per-lag kernel of time blocks (BIE_NEAR_MFMA=0) keeps the
    single-step kernel's order of operations: bit-identical tractions."""
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32, BIE_TIME_BLOCK, Operator, make_params

    monkeypatch.setenv("BIE_NEAR_MFMA", "0")
    N, M = 600, 403
    xa, xb = straight_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 34)
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32
    print(f"lane-per-lag time blocks {prec} N={N} M={M}", flush=True)
    op = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, precision=code,
                                                              time_block=BIE_TIME_BLOCK))
    T_run = _run(op, D, "run")
    T_step = _run(op, D, "step")
    T_graph = _run(op, D, "graph")
    op.close()
    assert np.isfinite(T_run).all()
    assert np.array_equal(T_run, T_step)
    assert np.array_equal(T_graph, T_run)


@pytest.mark.parametrize("mfma", ["2", "1", "0"])
def test_time_blocks_of_a_batch_whose_runs_end_inside_a_block(gpu_lib, monkeypatch, mfma):
    from paper_1903_02118_amd.binding import BIE_TIME_BLOCK, Operator, make_params

    monkeypatch.setenv("BIE_NEAR_MFMA", mfma)
    sizes, lags = [96, 200, 45], [130, 158, 97]
    faults = [(*straight_fault(n), m) for n, m in zip(sizes, lags)]
    D = np.concatenate([smooth_slip_rate(n, max(lags), 10, 20, 40 + k) for k, n in enumerate(sizes)], axis=1)
    print("time blocks, batch", sizes, lags, "mfma", mfma, flush=True)
    op = Operator.compress_fdph_batched(faults, params=make_params(eps_aca=1e-8, time_block=BIE_TIME_BLOCK))
    T_run = _run(op, D, "run")
    T_step = _run(op, D, "step")
    op.close()
    if mfma != "0":
        err = _rel(T_run, T_step)
        print(f"  blocked vs single steps {err:.2e}", flush=True)
        assert err <= TOL["fp64"]
    else:
        assert np.array_equal(T_run, T_step)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for k, m in enumerate(lags):
        assert np.all(T_run[m:, off[k]:off[k + 1]] == 0.0)


@pytest.mark.parametrize("case", ["planar-fp64", "curved-fp64-staircase", "curved-bf16", "batch-mixed"])
def test_one_launch_scatter_equals_per_step_scatters(gpu_lib, monkeypatch, case):
    """The scatter of a time block in one launch (slots summing their
    contributions in step order) against one launch per step in step order
    (BIE_FAR_SCATTER_TB=0): the same operations on every ring slot, so
    bit-identical tractions.  Covers the transient's rings (curved), the
    staircase sums, BF16 factors with hi + lo columns and faults whose runs end
    inside a block."""
    from paper_1903_02118_amd.binding import (BIE_FP64, BIE_MIXED_BF16, BIE_MIXED_FP32, BIE_TIME_BLOCK, Operator,
                                              make_params)

    geom, prec = case.split("-")[:2]
    code = {"fp64": BIE_FP64, "mixed": BIE_MIXED_FP32, "bf16": BIE_MIXED_BF16}[prec]
    par = dict(eps_aca=1e-8 if prec == "fp64" else 1e-4, precision=code, time_block=BIE_TIME_BLOCK,
               quantize_tr=case.endswith("staircase"))
    print("one-launch scatter", case, flush=True)

    def build():
        if geom == "batch":
            sizes, lags = [96, 200, 45], [130, 158, 97]
            faults = [(*straight_fault(n), m) for n, m in zip(sizes, lags)]
            return Operator.compress_fdph_batched(faults, params=make_params(**par))
        N, M = (600, 403) if geom == "planar" else (384, 251)
        xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
        return Operator.compress_fdph(xa, xb, M, params=make_params(**par))

    if geom == "batch":
        D = np.concatenate([smooth_slip_rate(n, 158, 10, 20, 50 + k) for k, n in enumerate([96, 200, 45])], axis=1)
    elif geom == "planar":
        D = smooth_slip_rate(600, 403, 20, 40, 35)
    else:
        D = smooth_slip_rate(384, 251, 20, 40, 36)
    monkeypatch.setenv("BIE_FAR_SCATTER_TB", "1")
    op1 = build()
    monkeypatch.setenv("BIE_FAR_SCATTER_TB", "0")
    op0 = build()
    T1 = _run(op1, D, "run")
    T1g = _run(op1, D, "graph")
    T0 = _run(op0, D, "run")
    op1.close()
    op0.close()
    assert np.isfinite(T1).all() and np.abs(T1).max() > 0
    assert np.array_equal(T1, T0)
    assert np.array_equal(T1g, T1)
