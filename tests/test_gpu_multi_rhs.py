"""GPU: several slip-rate histories (scenarios) sharing one FDP=H operator.

An operator built with n_rhs = R carries R independent histories through the
same windows and factors: every step row holds R blocks of N values.  Each
scenario's arithmetic is the single-scenario one in the same order (its own
accumulators in the near kernel, its own state in the far field), so the
tractions equal, bit for bit, those of R single-scenario operators built from
the same geometry and seed with the same lag chunks (64 lags, the default
with several scenarios; the single-scenario default is 128, which sums in
another order) and without time blocks (several scenarios take one step per
pass), and those are parity-tested against the oracle.  Checked on
ragged planar and curved faults (windows spanning several lag chunks), FP64
and mixed precision, eager and graph launches, after the autotuner, and for
a batch of faults.
"""
import numpy as np
import pytest

from synth import curved_fault, smooth_slip_rate, straight_fault

pytestmark = pytest.mark.gpu


def _run(op, D, graph=False):
    import torch

    Dd = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    Td = torch.full_like(Dd, np.nan)
    s = torch.cuda.current_stream()
    op.reset(stream=s)
    (op.run_graph if graph else op.run)(Dd, Td, stream=s)
    torch.cuda.synchronize()
    return Td.cpu().numpy()


@pytest.mark.parametrize("R,prec,geom", [(2, "fp64", "planar"), (4, "fp64", "planar"), (2, "fp32", "curved"),
                                         (4, "fp32", "planar"), (4, "fp64", "planar4k")])
def test_scenarios_equal_single_operators(gpu_lib, monkeypatch, R, prec, geom):
    """planar4k: the bench's fault at full size (N = 4096, M = 2048)."""
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32, Operator, make_params

    N, M = {"planar": (333, 300), "curved": (256, 260), "planar4k": (4096, 2048)}[geom]
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32
    xa, xb = curved_fault(N) if geom == "curved" else straight_fault(N)
    print(f"multi-rhs R={R} {prec} {geom} N={N} M={M}", flush=True)
    Ds = [smooth_slip_rate(N, M, 20, 40, 30 + r) for r in range(R)]
    opR = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-6, seed=7, precision=code, n_rhs=R))
    TR = _run(opR, np.concatenate(Ds, axis=1))
    st = opR.stats()
    opR.close()
    assert st["n_elem"] == N
    monkeypatch.setenv("BIE_NEAR_CHUNK", "64")
    for r in range(R):
        op1 = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-6, seed=7, precision=code,
                                                                   time_block=1))
        T1 = _run(op1, Ds[r])
        op1.close()
        assert np.array_equal(TR[:, r * N:(r + 1) * N], T1), r


def test_scenarios_graph_autotune_and_batch(gpu_lib, monkeypatch):
    import torch

    from paper_1903_02118_amd.binding import BieError, Operator, make_params

    R, M = 2, 200
    faults = [(*straight_fault(150), M), (*curved_fault(130), 180)]
    Ntot = 150 + 130
    print(f"multi-rhs batch R={R}", flush=True)
    Ds = [np.concatenate([smooth_slip_rate(n, M, 10, 20, 40 + 2 * r + k) for k, n in enumerate((150, 130))], axis=1)
          for r in range(R)]
    q = make_params(eps_aca=1e-6, seed=7, n_rhs=R)
    op = Operator.compress_fdph_batched(faults, params=q)
    DR = np.concatenate(Ds, axis=1)
    Te = _run(op, DR)
    Tg = _run(op, DR, graph=True)
    assert np.array_equal(Tg, Te)
    # after the autotuner (at most a change of load width: rounding)
    s = torch.cuda.current_stream()
    Dd = torch.from_numpy(DR).cuda()
    T = torch.zeros_like(Dd)
    op.reset(stream=s)
    op.run(Dd[:100], T[:100], stream=s)
    op.autotune(reps=2, stream=s)
    op.run(Dd[100:], T[100:], stream=s)
    torch.cuda.synchronize()
    assert np.allclose(T.cpu().numpy(), Te, rtol=1e-12, atol=1e-12 * np.abs(Te).max())
    # the coupled step is for one scenario
    with pytest.raises(BieError):
        op.step_predict(T[0], stream=s)
    op.close()
    monkeypatch.setenv("BIE_NEAR_CHUNK", "64")
    for r in range(R):
        o1 = Operator.compress_fdph_batched(faults, params=make_params(eps_aca=1e-6, seed=7, time_block=1))
        T1 = _run(o1, Ds[r])
        o1.close()
        assert np.array_equal(Te[:, r * Ntot:(r + 1) * Ntot], T1), r


@pytest.mark.parametrize("geom,prec", [("planar", "fp64"), ("curved", "fp64"), ("planar", "fp32")])
def test_four_scenarios_match_the_oracle(gpu_lib, geom, prec):
    """n_rhs = 4 against the oracle directly: each of the four histories
    carried by one operator equals the FDP=H-approximated convolution (Tier-B)
    of that history, within 1e-6 in FP64 and 1e-4 in mixed precision."""
    from oracle.dense import convolve_rows
    from oracle.fdph import FdphOracle, FdphParams
    from oracle.kernel2d import Problem
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32, Operator, make_params

    N, M, R = (256, 300, 4)
    xa, xb = curved_fault(N) if geom == "curved" else straight_fault(N)
    Ds = [smooth_slip_rate(N, M, 20, 40, 60 + r) for r in range(R)]
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32
    print(f"multi-rhs R=4 vs oracle {geom} {prec}", flush=True)
    op = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-8, seed=7, precision=code, n_rhs=R))
    TR = _run(op, np.concatenate(Ds, axis=1))
    op.close()
    o = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams())
    rec = np.arange(0, N, 2)
    rows = o.rows(rec)
    for r in range(R):
        Tb = convolve_rows(rows, Ds[r])
        Tg = TR[:, r * N + rec].T
        err = float(np.linalg.norm(Tg - Tb) / np.linalg.norm(Tb))
        print(f"  scenario {r} rel err {err:.3e}", flush=True)
        assert err <= (1e-6 if prec == "fp64" else 1e-4)
