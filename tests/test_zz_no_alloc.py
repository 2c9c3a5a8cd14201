"""bie_run_static: the run whose per-step partial sums live in the library's
static device array (for callers that cannot allocate), through the C ABI,
against bie_run on the same operator.  bie_run_static takes one step per
pass, so the FDP=H operators here are built without time blocks; then the
same kernels run in the same order on the same inputs, and the tractions
must be bit-identical: two calls
in a row, the second on a smaller operator and input, then an FDP=H run
again, so that stale contents of the shared array from a larger call would
show.
"""
import numpy as np
import pytest

from synth import curved_fault, smooth_slip_rate, straight_fault

pytestmark = pytest.mark.gpu


def _both(op, D):
    import torch

    s = torch.cuda.current_stream()
    Dd = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    Tr = torch.full_like(Dd, np.nan)
    Ts = torch.full_like(Dd, np.nan)
    op.reset(stream=s)
    op.run(Dd, Tr, stream=s)
    op.reset(stream=s)
    op.run_static(Dd, Ts, stream=s)
    torch.cuda.synchronize()
    return Tr.cpu().numpy(), Ts.cpu().numpy()


def test_static_scratch_run_equals_run(gpu_lib):
    from paper_1903_02118_amd.binding import Operator, make_params

    cases = [("fdph", straight_fault(512), 400), ("dense", straight_fault(200), 150),
             ("fdph", curved_fault(256), 120)]
    for kind, (xa, xb), M in cases:
        N = xa.shape[0]
        print(f"run_static {kind} N={N} M={M}", flush=True)
        op = Operator.build_kernel(xa, xb, M) if kind == "dense" else \
            Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, time_block=1))
        D = smooth_slip_rate(N, M, 20, 40, 70 + N)
        Tr, Ts = _both(op, D)
        op.close()
        assert np.isfinite(Tr).all()
        assert np.array_equal(Tr, Ts)


def test_static_scratch_refuses_an_operator_beyond_its_size(gpu_lib):
    """Four scenarios on N = 16384, M = 8192: their per-step partial sums
    exceed the 32 MiB array; the call is refused with a message, nothing run."""
    import torch

    from paper_1903_02118_amd.binding import BIE_EINVAL, BIE_MIXED_FP32, BieError, Operator, Plan, make_params

    N, M = 16384, 8192
    xa, xb = straight_fault(N)
    print(f"run_static refusal N={N} M={M} n_rhs=4", flush=True)
    plan = Plan.fdph([(xa, xb, M)], params=make_params(precision=BIE_MIXED_FP32, n_rhs=4))
    plan.windows()
    need = plan.stats()["scratch_bytes"]
    print(f"per-step partial sums: {need} bytes", flush=True)
    assert need > 32 << 20
    op = Operator.from_plan(plan)
    plan.close()
    D = torch.zeros((2, 4 * N), dtype=torch.float64, device="cuda")
    T = torch.zeros_like(D)
    with pytest.raises(BieError) as e:
        op.run_static(D, T, stream=torch.cuda.current_stream())
    assert e.value.code == BIE_EINVAL and "static scratch" in str(e.value)
    assert op.stats()["steps_done"] == 0
    op.close()
