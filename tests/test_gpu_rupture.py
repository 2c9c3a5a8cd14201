"""GPU: the coupled step and dynamic rupture, through the C ABI.

  * predict + commit reproduces the plain step: T_n = P_n + K_ii,0 D_n, with
    K_ii,0 = -mu/(2 beta) on a planar fault (plain and FDP=H forms, FP64 and
    mixed precision);
  * rupture runs against the oracle's coupled time marching (oracle.rupture)
    on the same kernel: the exact tensor for the plain form (Tier-A), the
    FDP=H-approximated one for the compressed form (Tier-B);
  * the FDP=H rupture against the plain-form rupture on the GPU (the paper's
    own accuracy check of Sec. 6.2, there below 0.4% at eta = 1/2).
Initial stress: the single-asperity model (App. A.2.3) with a small
overstress on the patch; friction: the exponential slip-weakening law of
Sec. 6.2 with its parameter ratios (T_bg/T_th = 0.35, T_dy = 0,
D_c = 0.05 dx), and the static-dynamic law.
"""
import numpy as np
import pytest

import oracle.rupture as rp
from oracle.fdph import FdphOracle, FdphParams
from oracle.kernel2d import Problem
from synth import curved_fault, smooth_slip_rate, straight_fault

pytestmark = pytest.mark.gpu

T_TH, T_BG, T_DY, D_C, OVER = 1e-2, 0.35e-2, 0.0, 0.05, 0.01


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _op(kind, N, M, precision=None, eta=None, geom="planar"):
    from paper_1903_02118_amd.binding import BIE_FP64, Operator, make_params

    xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
    if kind == "dense":
        return Operator.build_kernel(xa, xb, M), xa, xb
    kw = {} if eta is None else {"eta": eta}
    # coupled steps take one step per pass: references from bie_run use the
    # same single-step arithmetic (no time blocks)
    q = make_params(eps_aca=1e-6, seed=7, precision=BIE_FP64 if precision is None else precision, time_block=1,
                    **kw)
    return Operator.compress_fdph(xa, xb, M, params=q), xa, xb


@pytest.mark.parametrize("kind,prec,geom", [("dense", None, "planar"), ("fdph", "fp64", "planar"),
                                            ("fdph", "fp32", "planar"), ("fdph", "fp64", "curved")])
def test_predict_and_commit_reproduce_the_step(gpu_lib, kind, prec, geom):
    """On the curved trace the neighbours' first-lag entries (grazing fronts,
    below 1e-9) are left out of the coupled step: the step then differs by
    that much."""
    import torch

    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32

    N, M = (96, 120) if kind == "dense" else (200, 260)
    code = None if prec is None else (BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32)
    tol = 1e-12 if geom == "planar" else 1e-8
    print(f"predict/commit {kind} {prec} {geom} N={N} M={M}", flush=True)
    D = torch.from_numpy(smooth_slip_rate(N, M, 10, 20, 21)).cuda()
    s = torch.cuda.current_stream()
    a, _, _ = _op(kind, N, M, code, geom=geom)
    Tref = torch.zeros_like(D)
    a.reset(stream=s)
    a.run(D, Tref, stream=s)
    b, _, _ = _op(kind, N, M, code, geom=geom)
    k0 = torch.zeros(N, dtype=torch.float64, device="cuda")
    b.first_lag(k0, stream=s)
    P = torch.zeros_like(D)
    b.reset(stream=s)
    for n in range(M):
        b.step_predict(P[n], stream=s)
        b.step_commit(D[n], stream=s)
    torch.cuda.synchronize()
    k0h = k0.cpu().numpy()
    assert np.allclose(k0h, -0.5, rtol=1e-13, atol=0)  # -mu/(2 beta)
    T = (P + k0[None, :] * D).cpu().numpy()
    Tr = Tref.cpu().numpy()
    assert np.abs(T - Tr).max() <= tol * np.abs(Tr).max()
    # a predict without its commit blocks a plain step; past the lag count
    # (FDP=H) a predict is refused
    from paper_1903_02118_amd.binding import BieError

    if kind == "fdph":
        with pytest.raises(BieError):
            b.step_predict(P[0], stream=s)
    b.reset(stream=s)
    b.step_predict(P[0], stream=s)
    with pytest.raises(BieError):
        b.step(D[0], P[1], stream=s)
    b.step_commit(D[0], stream=s)
    a.close()
    b.close()


def _initial(N):
    x = np.arange(N) + 0.5
    half = 10.0
    return rp.single_asperity_stress(x, T_BG, T_TH * (1 + OVER), N / 2 - half, N / 2 + half)


def _gpu_rupture(op, T0, law, steps):
    import torch

    from paper_1903_02118_amd.binding import BIE_LAW_EXP_WEAKENING, BIE_LAW_STATIC_DYNAMIC, make_friction

    N = len(T0)
    code = BIE_LAW_EXP_WEAKENING if law == "exp" else BIE_LAW_STATIC_DYNAMIC
    fr = make_friction(code, T_TH, T_DY, D_C)
    t0 = torch.from_numpy(T0).cuda()
    slip = torch.zeros(N, dtype=torch.float64, device="cuda")
    state = torch.zeros(N, dtype=torch.int32, device="cuda")
    D = torch.full((steps, N), np.nan, dtype=torch.float64, device="cuda")
    T = torch.full_like(D, np.nan)
    s = torch.cuda.current_stream()
    op.reset(stream=s)
    op.rupture_run(fr, t0, slip, state, D, T, stream=s)
    torch.cuda.synchronize()
    return D.cpu().numpy(), T.cpu().numpy(), slip.cpu().numpy(), state.cpu().numpy().astype(bool)


@pytest.mark.parametrize("law", ["exp", "static_dynamic"])
def test_dense_rupture_matches_oracle(gpu_lib, law):
    N, M = 96, 150
    print(f"rupture dense {law} N={N} M={M}", flush=True)
    op, xa, xb = _op("dense", N, M)
    T0 = _initial(N)
    D, T, slip, rup = _gpu_rupture(op, T0, law, M)
    op.close()
    K = Problem(xa, xb).kernel_tensor(M)
    Do, To, so, ro = rp.simulate(np.transpose(K, (1, 2, 0)), T0, rp.Friction(law, T_TH, T_DY, D_C, 0.5), M)
    err = _relerr(D, Do)
    print("rupture dense rel err", law, err, "ruptured", int(rup.sum()), flush=True)
    assert np.array_equal(rup, ro) and rup.sum() > 20
    assert err <= 1e-10
    assert np.abs(T - To).max() <= 1e-10 * np.abs(To).max()
    assert np.allclose(slip, so, rtol=1e-9, atol=1e-15)


def test_fdph_rupture_matches_tier_b(gpu_lib):
    """The FDP=H operator (FP64, ACA+ at 1e-6) against the oracle's dense
    FDP=H-approximated kernel: the difference is the ACA+ error of the
    far-field blocks, carried through the rupture (measured 2e-10)."""
    N, M = 256, 300
    print(f"rupture fdph N={N} M={M}", flush=True)
    op, xa, xb = _op("fdph", N, M)
    T0 = _initial(N)
    D, T, slip, rup = _gpu_rupture(op, T0, "exp", M)
    op.close()
    Kt = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams()).rows(np.arange(N))
    Do, To, so, ro = rp.simulate(Kt, T0, rp.Friction("exp", T_TH, T_DY, D_C, 0.5), M)
    err = _relerr(D, Do)
    print("rupture fdph vs tier-b rel err", err, "ruptured", int(rup.sum()), flush=True)
    assert np.array_equal(rup, ro) and rup.sum() > 40
    assert err <= 1e-8


@pytest.mark.parametrize("kind", ["dense", "fdph"])
def test_curved_rupture_matches_oracle(gpu_lib, kind):
    """Rupture on the sinusoidal fault (the nonplanar case of Sec. 6.2):
    plain form vs Tier-A, FDP=H vs Tier-B (stress components projected on
    each element's normal).  On the curved trace, S fronts reach element
    ends at collocation times up to rounding; those grazing entries are the
    square root of a rounding-size argument, so the two sides' kernels
    differ there at ~1e-10 relative (measured 1.9e-10 on the rupture run),
    hence 1e-8 rather than the planar 1e-10.  The FDP=H run carries the
    ACA+ error of the far-field blocks (eps_aca = 1e-6, the FP64 target of
    the prescribed-slip parity); measured 5.8e-9, gated at 1e-7."""
    N, M = (128, 160) if kind == "dense" else (256, 240)
    print(f"rupture curved {kind} N={N} M={M}", flush=True)
    op, xa, xb = _op(kind, N, M, geom="curved")
    T0 = _initial(N)
    D, T, slip, rup = _gpu_rupture(op, T0, "exp", M)
    op.close()
    if kind == "dense":
        Kr = np.transpose(Problem(xa, xb).kernel_tensor(M), (1, 2, 0))
    else:
        Kr = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams()).rows(np.arange(N))
    Do, To, so, ro = rp.simulate(Kr, T0, rp.Friction("exp", T_TH, T_DY, D_C, 0.5), M)
    err = _relerr(D, Do)
    print("rupture curved rel err", kind, err, "ruptured", int(rup.sum()), flush=True)
    assert np.array_equal(rup, ro) and rup.sum() > 20
    assert err <= (1e-8 if kind == "dense" else 1e-7)


def test_fdph_rupture_close_to_plain_form(gpu_lib):
    """The paper's accuracy check (Sec. 6.2): the FDP=H solution against the
    plain ST-BIEM one, per step, relative L2 of the slip rate over the
    fault; eta = 1/2 as there, and the paper's bound of 0.4% (measured here:
    at most 0.25% over 500 steps)."""
    N, M, steps = 512, 500, 500
    print(f"rupture fdph vs dense N={N} steps={steps}", flush=True)
    T0 = _initial(N)
    opd, _, _ = _op("dense", N, M)
    Dd, _, _, rd = _gpu_rupture(opd, T0, "exp", steps)
    opd.close()
    opf, _, _ = _op("fdph", N, M, eta=0.5)
    Df, _, _, rf = _gpu_rupture(opf, T0, "exp", steps)
    opf.close()
    per_step = [_relerr(Df[n], Dd[n]) for n in range(steps) if np.linalg.norm(Dd[n]) > 0]
    print("rupture fdph vs dense: max per-step rel err", max(per_step), "final", per_step[-1],
          "ruptured", int(rd.sum()), int(rf.sum()), flush=True)
    assert rd.sum() > 100
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")) as f:
        paper = json.load(f)["rupture_error_planar_eta_half"]
    assert paper["eta"] == 0.5
    assert max(per_step) <= paper["max_rel_err"]


def test_batched_rupture_equals_each_fault_alone(gpu_lib):
    """Independent faults in one batched operator rupture as each does alone
    (the coupled step and the friction solve per element keep the faults
    apart; the run is limited by the shortest lag count).  The batch draws
    its own ACA+ pivots, so its far-field factors differ from a lone fault's
    within eps_aca: the slip rates agree to 1e-8 (measured 3e-10), the
    ruptured sets exactly."""
    import torch

    from paper_1903_02118_amd.binding import BIE_LAW_EXP_WEAKENING, Operator, make_friction, make_params

    sizes, lags, steps = [96, 160], [200, 150], 150
    print(f"rupture batched sizes={sizes} steps={steps}", flush=True)
    q = make_params(eps_aca=1e-6, seed=7)
    faults = [(*straight_fault(n), m) for n, m in zip(sizes, lags)]
    T0 = np.concatenate([_initial(n) for n in sizes])
    fr = make_friction(BIE_LAW_EXP_WEAKENING, T_TH, T_DY, D_C)

    def run(op, t0):
        N = len(t0)
        s = torch.cuda.current_stream()
        args = [torch.from_numpy(t0).cuda(), torch.zeros(N, dtype=torch.float64, device="cuda"),
                torch.zeros(N, dtype=torch.int32, device="cuda"),
                torch.zeros((steps, N), dtype=torch.float64, device="cuda"),
                torch.zeros((steps, N), dtype=torch.float64, device="cuda")]
        op.reset(stream=s)
        op.rupture_run(fr, *args, stream=s)
        torch.cuda.synchronize()
        return args[3].cpu().numpy(), args[2].cpu().numpy()

    ob = Operator.compress_fdph_batched(faults, params=q)
    Db, rb = run(ob, T0)
    # past the shortest lag count the batch refuses further coupled steps
    from paper_1903_02118_amd.binding import BieError

    with pytest.raises(BieError):
        import torch as _t

        tmp = _t.zeros(sum(sizes), dtype=_t.float64, device="cuda")
        ob.step_predict(tmp)
    ob.close()
    c = 0
    for (xa, xb, m), n in zip(faults, sizes):
        oa = Operator.compress_fdph(xa, xb, m, params=q)
        Da, ra = run(oa, T0[c:c + n])
        oa.close()
        assert np.array_equal(rb[c:c + n], ra) and ra.sum() > 20
        assert np.abs(Db[:, c:c + n] - Da).max() <= 1e-8 * np.abs(Da).max()
        c += n
