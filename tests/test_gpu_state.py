"""GPU: checkpoint and resume of a time-marching run through the C ABI.

A state saved at step k and loaded again (into the same operator, or into a
fresh one built from the same problem and parameters) gives the steps after k
bit for bit as the run that saved it went on to give (and, to rounding, as
one uninterrupted run, whose time blocks fall at other steps): the plain form, the FDP=H form in FP64
and in mixed precision with the staircase transient (every kind of ring and
running sum), several scenarios, and a rupture run (the caller keeps its own
slip and rupture state beside the operator's).  Bad buffers and states of
other operators are refused before anything is copied into the operator.
"""
import numpy as np
import pytest

from synth import curved_fault, smooth_slip_rate, straight_fault, uniform_slip_rate

pytestmark = pytest.mark.gpu


def _build(kind, N, M, **kw):
    from paper_1903_02118_amd.binding import Operator, make_params

    geom = kw.pop("geom", "planar")
    xa, xb = curved_fault(N) if geom == "curved" else straight_fault(N)
    if kind == "dense":
        return Operator.build_kernel(xa, xb, M)
    return Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-6, seed=7, **kw))


def _state_buf(op, extra=0):
    import torch

    return torch.zeros(op.state_bytes() + extra, dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("case", ["dense", "fdph_fp64", "fdph_mixed_quant_curved", "fdph_2_scenarios"])
def test_resume_from_a_saved_state_is_bit_identical(gpu_lib, case):
    import torch

    from paper_1903_02118_amd.binding import BIE_MIXED_FP32

    N, M, k = {"dense": (130, 70, 37), "fdph_fp64": (333, 300, 150), "fdph_mixed_quant_curved": (256, 260, 131),
               "fdph_2_scenarios": (200, 220, 101)}[case]
    kw = {"dense": {}, "fdph_fp64": {}, "fdph_mixed_quant_curved": {"geom": "curved", "precision": BIE_MIXED_FP32,
                                                                    "quantize_tr": True},
          "fdph_2_scenarios": {"n_rhs": 2}}[case]
    kind = "dense" if case == "dense" else "fdph"
    R = kw.get("n_rhs", 1)
    print(f"state {case} N={N} M={M} k={k}", flush=True)
    D = (uniform_slip_rate(N * R, M, 21) if kind == "dense"
         else np.concatenate([smooth_slip_rate(N, M, 10, 20, 22 + r) for r in range(R)], axis=1))
    Dd = torch.from_numpy(np.ascontiguousarray(D)).cuda()
    s = torch.cuda.current_stream()
    op = _build(kind, N, M, **dict(kw))
    T_full = torch.zeros_like(Dd)
    op.reset(stream=s)
    op.run(Dd, T_full, stream=s)
    # run to step k, save, run on; load, run again
    buf = _state_buf(op)
    T1 = torch.zeros_like(Dd)
    op.reset(stream=s)
    op.run(Dd[:k], T1[:k], stream=s)
    op.save_state(buf, stream=s)
    assert op.stats()["steps_done"] == k
    op.run(Dd[k:], T1[k:], stream=s)
    T2 = torch.full_like(Dd, np.nan)
    op.load_state(buf, stream=s)
    assert op.stats()["steps_done"] == k
    op.run(Dd[k:], T2[k:], stream=s)
    # a fresh operator of the same problem and parameters resumes the run too
    op2 = _build(kind, N, M, **dict(kw))
    T3 = torch.full_like(Dd, np.nan)
    op2.load_state(buf, stream=s)
    op2.run(Dd[k:], T3[k:], stream=s)
    torch.cuda.synchronize()
    a, b = T_full.cpu().numpy(), T1.cpu().numpy()
    # the uninterrupted run puts its time blocks at other steps than the run
    # cut at k (matrix-core sums: equal to rounding)
    tol = 1e-5 if kw.get("precision") else 1e-12
    assert np.abs(a - b).max() <= tol * np.abs(a).max()
    assert np.array_equal(T2.cpu().numpy()[k:], b[k:])
    assert np.array_equal(T3.cpu().numpy()[k:], b[k:])
    op.close()
    op2.close()


def test_rupture_run_resumes_from_a_checkpoint(gpu_lib):
    """Coupled steps (predict, friction, commit) on the FDP=H form: save the
    operator's state with the caller's slip and rupture flags, run on, then
    restore both and run again."""
    import torch

    from paper_1903_02118_amd.binding import BIE_LAW_EXP_WEAKENING, make_friction

    N, M, k, steps = 256, 200, 60, 120
    print(f"state rupture N={N} k={k}", flush=True)
    op = _build("fdph", N, M)
    s = torch.cuda.current_stream()
    x = np.arange(N) + 0.5
    T0 = torch.from_numpy(np.where(np.abs(x - N / 2) < 10, 1.01, 0.35)).cuda()
    fr = make_friction(BIE_LAW_EXP_WEAKENING, 1.0, 0.0, 0.05)
    slip = torch.zeros(N, dtype=torch.float64, device="cuda")
    state = torch.zeros(N, dtype=torch.int32, device="cuda")
    D = torch.zeros(steps, N, dtype=torch.float64, device="cuda")
    T = torch.zeros_like(D)
    op.reset(stream=s)
    op.rupture_run(fr, T0, slip, state, D[:k], T[:k], stream=s)
    buf = _state_buf(op)
    op.save_state(buf, stream=s)
    slip_k, state_k = slip.clone(), state.clone()
    op.rupture_run(fr, T0, slip, state, D[k:], T[k:], stream=s)
    D2, T2 = torch.full_like(D, np.nan), torch.full_like(T, np.nan)
    op.load_state(buf, stream=s)
    slip.copy_(slip_k)
    state.copy_(state_k)
    op.rupture_run(fr, T0, slip, state, D2[k:], T2[k:], stream=s)
    torch.cuda.synchronize()
    assert int((state != 0).sum()) >= 20  # the nucleation patch ruptured
    assert torch.equal(D2[k:], D[k:]) and torch.equal(T2[k:], T[k:])
    op.close()


def test_bad_state_buffers_are_refused(gpu_lib):
    import torch

    from paper_1903_02118_amd.binding import BieError

    print("state errors", flush=True)
    s = torch.cuda.current_stream()
    a = _build("fdph", 150, 120)
    b = _build("fdph", 170, 120)
    d = _build("dense", 150, 120)
    big = max(a.state_bytes(), b.state_bytes(), d.state_bytes())
    buf = torch.zeros(big + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(BieError):  # no saved state in the buffer
        a.load_state(buf, stream=s)
    with pytest.raises(BieError):  # too small
        a.save_state(buf[: a.state_bytes() - 256], stream=s)
    with pytest.raises(BieError):  # not 256-byte aligned
        a.save_state(buf[8:], stream=s)
    a.save_state(buf, stream=s)
    with pytest.raises(BieError):  # another fault size
        b.load_state(buf, stream=s)
    with pytest.raises(BieError):  # another operator kind
        d.load_state(buf, stream=s)
    # a predicted step must be committed before a save
    Z = torch.zeros(150, dtype=torch.float64, device="cuda")
    P = torch.zeros_like(Z)
    a.reset(stream=s)
    a.step_predict(P, stream=s)
    with pytest.raises(BieError):
        a.save_state(buf, stream=s)
    a.step_commit(Z, stream=s)
    a.save_state(buf, stream=s)
    a.load_state(buf, stream=s)
    torch.cuda.synchronize()
    assert a.stats()["steps_done"] == 1
    for o in (a, b, d):
        o.close()
