"""Time blocks of prescribed-slip runs: the near field of BIE_TIME_BLOCK consecutive steps
in one pass over the windows (bie_run, bie_run_graph) against the same
operator stepped one step at a time (bie_step), and against an operator
built without time blocks.  The time-blocked kernel adds the same products
in the same order as the single-step kernel, so the tractions must be
bit-identical; the runs include a remainder shorter than a block, blocks
that start before the first history reaches a chunk, and batched faults
whose runs end inside a block."""
import numpy as np
import pytest

from synth import curved_fault, smooth_slip_rate, straight_fault

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("geom", ["planar", "curved"])
def test_time_blocks_equal_single_steps(gpu_lib, prec, geom):
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32, BIE_TIME_BLOCK, Operator, make_params

    N, M = (600, 403) if geom == "planar" else (384, 251)
    xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 33)
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32
    print(f"time blocks {geom} {prec} N={N} M={M}", flush=True)
    op4 = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, precision=code,
                                                               time_block=BIE_TIME_BLOCK))
    op1 = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, precision=code, time_block=1))
    T_run = _run(op4, D, "run")
    T_graph = _run(op4, D, "graph")
    T_step = _run(op4, D, "step")
    T_one = _run(op1, D, "run")
    op4.close()
    op1.close()
    assert np.isfinite(T_run).all()
    assert np.array_equal(T_run, T_step)
    assert np.array_equal(T_graph, T_run)
    # another operator (ring lengths differ, windows and factors the same
    # up to ACA+'s random references): equal to rounding
    err = float(np.linalg.norm(T_run - T_one) / np.linalg.norm(T_one))
    print(f"  blocked vs operator without blocks: {err:.2e}", flush=True)
    assert err <= 1e-12 if prec == "fp64" else err <= 1e-6


def test_time_blocks_of_a_batch_whose_runs_end_inside_a_block(gpu_lib):
    from paper_1903_02118_amd.binding import BIE_TIME_BLOCK, Operator, make_params

    sizes, lags = [96, 200, 45], [130, 158, 97]
    faults = [(*straight_fault(n), m) for n, m in zip(sizes, lags)]
    D = np.concatenate([smooth_slip_rate(n, max(lags), 10, 20, 40 + k) for k, n in enumerate(sizes)], axis=1)
    print("time blocks, batch", sizes, lags, flush=True)
    op = Operator.compress_fdph_batched(faults, params=make_params(eps_aca=1e-8, time_block=BIE_TIME_BLOCK))
    T_run = _run(op, D, "run")
    T_step = _run(op, D, "step")
    op.close()
    assert np.array_equal(T_run, T_step)
    off = np.concatenate([[0], np.cumsum(sizes)])
    for k, m in enumerate(lags):
        assert np.all(T_run[m:, off[k]:off[k + 1]] == 0.0)
