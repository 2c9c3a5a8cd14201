"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Dense form vs Tier-A (exact convolution, Eq. 4); FDP=H form vs Tier-B (the
FDP=H-approximated operator applied densely).  Tolerances:
  * dense FP64: relative L2 <= 1e-12 and max |dT| <= 1e-11 max|T|.  Both sides
    evaluate K_m = S(t_m) - S(t_{m-1}) in FP64 with different libm/ocml
    asin/sqrt (<= 1 ulp); the difference of two O(m) step responses loses up
    to log10(m) digits, so entries agree to ~1e-14 and sums of N*M of them to
    ~1e-13 relative.
  * FDP=H FP64: relative L2 <= 1e-6 (the FP64 target for this form); the
    difference is the ACA+ error (eps_aca) of the far-field blocks plus
    rounding.
"""
import numpy as np
import pytest

from oracle.dense import convolve_dense, convolve_rows, convolve_rows_fft
from oracle.fdph import FdphOracle, FdphParams
from oracle.kernel2d import Problem
from synth import curved_fault, impulse_slip_rate, smooth_slip_rate, straight_fault, uniform_slip_rate

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def _run(op, D):
    torch = _torch()
    Dd = torch.from_numpy(np.ascontiguousarray(D)).to("cuda")
    Td = torch.zeros_like(Dd)
    s = torch.cuda.current_stream()
    op.reset(stream=s)
    op.run(Dd, Td, stream=s)
    torch.cuda.synchronize()
    return Td.cpu().numpy()


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ dense ---
def test_dense_matches_tier_a_small_config(gpu_lib):
    """N=256, M=128, i.i.d. U(0,1) slip rate (seed 1), every receiver and step."""
    from paper_1903_02118_amd.binding import Operator

    N, M = 256, 128
    xa, xb = straight_fault(N)
    D = uniform_slip_rate(N, M, 1)
    print(f"dense N={N} M={M} seed=1", flush=True)
    op = Operator.build_kernel(xa, xb, M, mu=1.0, beta=1.0, dt=0.5)
    T = _run(op, D)
    K = Problem(xa, xb, dt=0.5).kernel_tensor(M)
    Tref = convolve_dense(K, D)
    assert _relerr(T, Tref) <= 1e-12
    assert np.abs(T - Tref).max() <= 1e-11 * np.abs(Tref).max()
    op.close()


@pytest.mark.parametrize("N,M", [(1, 5), (37, 19), (130, 70)])
def test_dense_ragged_and_degenerate_sizes(gpu_lib, N, M):
    from paper_1903_02118_amd.binding import Operator

    xa, xb = curved_fault(N) if N > 1 else straight_fault(N)
    D = uniform_slip_rate(N, M + 7, 11)  # run past M: lags beyond M are dropped
    print(f"dense ragged N={N} M={M}", flush=True)
    op = Operator.build_kernel(xa, xb, M, mu=1.3, beta=0.8, dt=0.4, eps_t=0.7)
    T = _run(op, D)
    K = Problem(xa, xb, mu=1.3, beta=0.8, dt=0.4, eps_t=0.7).kernel_tensor(M)
    Tref = convolve_dense(K, D)
    assert _relerr(T, Tref) <= 1e-12
    op.close()


def test_dense_impulse_response_is_the_kernel(gpu_lib):
    from paper_1903_02118_amd.binding import Operator

    N, M = 64, 40
    xa, xb = straight_fault(N)
    op = Operator.build_kernel(xa, xb, M)
    K = Problem(xa, xb).kernel_tensor(M)
    for j0, n0 in [(0, 0), (31, 5)]:
        T = _run(op, impulse_slip_rate(N, M, j0, n0))
        for n in range(M):
            ref = K[n - n0][:, j0] if n >= n0 else np.zeros(N)
            assert np.allclose(T[n], ref, rtol=0, atol=1e-14)
    op.close()


# ------------------------------------------------------------------ FDP=H ---
def _fdph_case(xa, xb, M, D, receivers, eps_aca=1e-6, seed=7, fft=False, **kw):
    from paper_1903_02118_amd.binding import Operator, make_params

    q = make_params(eps_aca=eps_aca, seed=seed, **kw)
    op = Operator.compress_fdph(xa, xb, M, params=q)
    T = _run(op, D)
    okw = {k: v for k, v in kw.items() if k in ("eta", "leaf_size", "eps_q", "eps_st", "n_c", "quantize_tr")}
    if "eps_qtr" in kw:
        okw["eps_q_tr"] = kw["eps_qtr"]
    o = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams(**okw))
    rows = o.rows(receivers)
    Tb = (convolve_rows_fft if fft else convolve_rows)(rows, D)
    st = op.stats()
    return op, o, T[:, receivers].T, Tb, st


@pytest.mark.parametrize("N,M", [(256, 512), (333, 300)])
def test_fdph_matches_tier_b_planar(gpu_lib, N, M):
    """Every receiver and step; N=333 leaves ragged clusters and tiles."""
    xa, xb = straight_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 2)
    rec = np.arange(N)
    print(f"fdph planar N={N} M={M}", flush=True)
    op, o, T, Tb, st = _fdph_case(xa, xb, M, D, rec)
    assert st["n_adm"] == o.stats()["n_adm"] and st["near_pairs"] == o.stats()["near_pairs"]
    err = _relerr(T, Tb)
    print("fdph planar rel err", err, st, flush=True)
    assert err <= 1e-6
    op.close()


_NEAR_REF = {}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("chunk", [64, 128, 256])
@pytest.mark.parametrize("wide", [0, 1])
@pytest.mark.parametrize("mfma", [2, 1, 0])
def test_fdph_near_kernel_variants_match_tier_b(gpu_lib, monkeypatch, prec, chunk, wide, mfma):
    """Every near-kernel variant the launcher can pick (64-, 128- or 256-lag
    chunks; narrow or wide window loads, the latter on two sources per load
    where a wave-wide load would pass the chunk; FP64 or FP32 windows; for
    the time blocks of the run, the matrix-core kernel on single lag chunks
    or on groups of consecutive chunks, or the lane-per-lag kernel),
    on a ragged planar fault (odd source counts at tile ends) whose windows
    span several chunks."""
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_FP32, Operator, make_params

    monkeypatch.setenv("BIE_NEAR_CHUNK", str(chunk))
    monkeypatch.setenv("BIE_NEAR_WIDE", str(wide))
    monkeypatch.setenv("BIE_NEAR_MFMA", str(mfma))
    N, M = 203, 300
    xa, xb = straight_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 6)
    if "Tb" not in _NEAR_REF:
        o = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams())
        _NEAR_REF["Tb"] = convolve_rows(o.rows(np.arange(N)), D)
    Tb = _NEAR_REF["Tb"]
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_FP32
    print(f"near variant {prec} chunk={chunk} wide={wide} mfma={mfma}", flush=True)
    op = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-6, seed=7, precision=code))
    T = _run(op, D).T
    err = _relerr(T, Tb)
    print("near variant rel err", err, flush=True)
    assert err <= (1e-6 if prec == "fp64" else 1e-4)
    op.close()


@pytest.mark.parametrize("N,M", [(1, 1), (1, 7), (2, 3), (40, 90), (65, 1)])
def test_fdph_degenerate_sizes(gpu_lib, N, M):
    """One element, a single lag, and faults too small for any admissible
    leaf (every pair in the near field): FDP=H equals Tier-B, which there is
    the exact convolution with static tails past each window."""
    xa, xb = straight_fault(N)
    D = uniform_slip_rate(N, M, 3)
    print(f"fdph degenerate N={N} M={M}", flush=True)
    op, o, T, Tb, st = _fdph_case(xa, xb, M, D, np.arange(N))
    assert st["n_adm"] == 0
    assert np.abs(T - Tb).max() <= 1e-12 * max(np.abs(Tb).max(), 1e-300)
    op.close()


def test_fdph_integers_match_oracle(gpu_lib):
    """Windows W_ij, ART integers and transient lengths agree exactly."""
    from paper_1903_02118_amd.binding import BIE_EXPORT_ART, BIE_EXPORT_NEAR, BIE_EXPORT_TRANS, Operator, make_params

    N, M = 256, 600
    xa, xb = straight_fault(N)
    op = Operator.compress_fdph(xa, xb, M, params=make_params())
    o = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams())
    near = op.export(BIE_EXPORT_NEAR)
    ref = {}
    for lf in o.leaves:
        if lf.admissible:
            continue
        for i in lf.tau.idx:
            W, _, _ = o.near_window(int(i), lf.sigma.idx)
            for j, w in zip(lf.sigma.idx, W):
                ref[(int(i), int(j))] = int(w)
    got = {(int(r[0]), int(r[1])): int(r[2]) for r in near}
    assert got == ref
    art = op.export(BIE_EXPORT_ART)
    # map (receiver-cluster min, source-cluster min) -> oracle leaf
    src_rows = {}
    rec_rows = {}
    for la, j, mb, dm, i, dmi in art:
        if j >= 0:
            src_rows.setdefault(int(la), {})[int(j)] = (int(mb), int(dm))
        else:
            rec_rows.setdefault(int(la), {})[int(i)] = int(dmi)
    ref_src, ref_rec = [], []
    for lf in o.leaves:
        if not lf.admissible:
            continue
        mb, dm = o.art_source(lf)
        ref_src.append({int(j): (int(a), int(b)) for j, a, b in zip(lf.sigma.idx, mb, dm)})
        dmi = o.art_delta_m(lf, lf.tau.idx)
        ref_rec.append({int(i): int(d) for i, d in zip(lf.tau.idx, dmi)})
    key = lambda d: tuple(sorted(d.items()))
    assert sorted(map(key, src_rows.values())) == sorted(map(key, ref_src))
    assert sorted(map(key, rec_rows.values())) == sorted(map(key, ref_rec))
    tr = op.export(BIE_EXPORT_TRANS)
    ref_tr = []
    for lf in o.leaves:
        if lf.admissible:
            htr, ntr = o.transient(lf)
            ref_tr.append((lf.jpiv, ntr[0]))
    assert sorted((int(a), int(b)) for _, a, b, _ in tr) == sorted(ref_tr)
    assert (tr[:, 3] == 0).all()
    op.close()


@pytest.mark.parametrize("geom", ["planar", "curved"])
def test_fdph_quantized_transient_matches_oracle(gpu_lib, geom):
    """Staircase transient: same runs as the oracle and the same stresses."""
    from paper_1903_02118_amd.binding import BIE_EXPORT_TRANS

    N, M = (256, 640) if geom == "planar" else (256, 400)
    xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 5)
    rec = np.arange(0, N, 2)
    print(f"fdph quantized {geom} N={N} M={M}", flush=True)
    op, o, T, Tb, st = _fdph_case(xa, xb, M, D, rec, eps_aca=1e-8, quantize_tr=True, eps_qtr=0.1)
    tr = op.export(BIE_EXPORT_TRANS)
    ref = []
    for lf in o.leaves:
        if lf.admissible:
            o.transient(lf)
            ref.append((lf.jpiv, lf.ntr[0], lf.nq_tr[0]))
    ref.sort()
    got = sorted((int(a), int(b), int(c)) for _, a, b, c in tr)
    assert got == ref
    assert any(c > 0 for _, _, c in got)
    err = _relerr(T, Tb)
    print("fdph quantized rel err", err, flush=True)
    assert err <= 1e-6
    op.close()


def test_fdph_impulse_response_is_a_tier_b_column(gpu_lib):
    from paper_1903_02118_amd.binding import Operator, make_params

    N, M = 128, 400
    xa, xb = straight_fault(N)
    op = Operator.compress_fdph(xa, xb, M, params=make_params(eps_aca=1e-10))
    o = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams())
    j0 = 77
    T = _run(op, impulse_slip_rate(N, M, j0, 0))
    rows = o.rows(np.arange(N))  # [i][j][m]
    col = rows[:, j0, :].T       # [m][i]
    assert np.abs(T - col).max() <= 1e-8 * np.abs(col).max()
    op.close()


def test_fdph_curved_matches_tier_b(gpu_lib):
    """Nonplanar trace: stress components, then projection on the normals."""
    N, M = 256, 300
    xa, xb = curved_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 3)
    rec = np.arange(0, N, 3)
    print(f"fdph curved N={N} M={M}", flush=True)
    op, o, T, Tb, st = _fdph_case(xa, xb, M, D, rec, eps_aca=1e-8)
    err = _relerr(T, Tb)
    print("fdph curved rel err", err, st, flush=True)
    assert err <= 1e-6
    op.close()


@pytest.mark.parametrize("kind", ["dense", "fdph"])
def test_advance_equals_zero_slip_steps(gpu_lib, kind):
    """bie_advance(k) == a run of k steps with zero slip rate (then the same
    continuation, bit for bit); and == one run over all steps, whose time
    blocks fall at other steps (FDP=H: equal to rounding)."""
    torch = _torch()
    from paper_1903_02118_amd.binding import Operator, make_params

    N, M, k = 96, 160, 37
    xa, xb = straight_fault(N)
    D = smooth_slip_rate(N, M, 10, 20, 5)
    D[:k] = 0.0
    op = Operator.build_kernel(xa, xb, M) if kind == "dense" else Operator.compress_fdph(xa, xb, M, params=make_params())
    Tfull = _run(op, D)
    Dd = torch.from_numpy(np.ascontiguousarray(D)).to("cuda")
    s = torch.cuda.current_stream()
    Tz = torch.zeros_like(Dd)
    op.reset(stream=s)
    op.run(Dd[:k], Tz[:k], stream=s)
    op.run(Dd[k:], Tz[k:], stream=s)
    Td = torch.zeros_like(Dd[k:])
    op.reset(stream=s)
    op.advance(k, stream=s)
    op.run(Dd[k:], Td, stream=s)
    torch.cuda.synchronize()
    assert np.array_equal(Td.cpu().numpy(), Tz[k:].cpu().numpy())
    assert np.abs(Td.cpu().numpy() - Tfull[k:]).max() <= 1e-12 * np.abs(Tfull).max()
    op.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("geom", ["planar", "curved"])
def test_fdph_mixed_precision_within_1e4(gpu_lib, geom, prec):
    """FP32 near windows, FP32 or BF16 factors (leading cross terms as hi + lo
    BF16 pairs), FP64 sums, self terms and accumulators: within 1e-4 of
    Tier-B (the mixed-precision target)."""
    from paper_1903_02118_amd.binding import BIE_MIXED_BF16, BIE_MIXED_FP32

    code = BIE_MIXED_FP32 if prec == "fp32" else BIE_MIXED_BF16
    N, M = 256, 400
    xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
    D = smooth_slip_rate(N, M, 20, 40, 4)
    rec = np.arange(0, N, 2)
    print(f"fdph mixed {geom} {prec} N={N} M={M}", flush=True)
    op, o, T, Tb, st = _fdph_case(xa, xb, M, D, rec, eps_aca=1e-6, precision=code)
    err = _relerr(T, Tb)
    print("fdph mixed rel err", geom, prec, err, flush=True)
    assert st["precision"] == code
    assert err <= 1e-4
    op.close()


def test_fdph_runs_end_at_the_lag_count(gpu_lib):
    """An FDP=H operator refuses steps past its lag count (its tractions would
    be zero there) and reports it; the plain form keeps convolving."""
    torch = _torch()
    from paper_1903_02118_amd.binding import BIE_EINVAL, BieError, Operator, make_params

    N, M = 64, 40
    xa, xb = straight_fault(N)
    D = torch.zeros((M + 1, N), dtype=torch.float64, device="cuda")
    T = torch.zeros_like(D)
    s = torch.cuda.current_stream()
    op = Operator.compress_fdph(xa, xb, M, params=make_params())
    with pytest.raises(BieError) as e:
        op.run(D, T, stream=s)
    assert e.value.code == BIE_EINVAL and op.stats()["steps_done"] == 0
    op.run(D[:M], T[:M], stream=s)
    with pytest.raises(BieError):
        op.step(D[M], T[M], stream=s)
    op.reset(stream=s)
    op.run(D[:M], T[:M], stream=s)
    torch.cuda.synchronize()
    op.close()
    dop = Operator.build_kernel(xa, xb, M)
    dop.run(D, T, stream=s)
    torch.cuda.synchronize()
    dop.close()


@pytest.mark.parametrize("kind", ["dense", "fdph"])
def test_nonfinite_scan_reports_the_first_bad_traction(gpu_lib, kind):
    """Debug scan (bie_set_debug): clean runs report -1; a NaN slip rate of
    source 17 at step 3 reaches the tractions of step 3 (no earlier step) at
    the receivers whose lag-0 kernel entries with source 17 are stored (the
    plain form's causal band around it, the FDP=H form's whole near tile), and
    the scan reports the first of them."""
    torch = _torch()
    from paper_1903_02118_amd.binding import Operator, make_params

    N, M = 96, 40
    xa, xb = straight_fault(N)
    D = uniform_slip_rate(N, M, 5)
    op = Operator.build_kernel(xa, xb, M) if kind == "dense" else Operator.compress_fdph(xa, xb, M, params=make_params())
    s = torch.cuda.current_stream()
    op.set_debug(stream=s)
    _run(op, D)
    assert op.debug_status(stream=s) == -1
    D[3, 17] = np.nan
    op.set_debug(stream=s)
    _run(op, D)
    bad = op.debug_status(stream=s)
    print(f"{kind}: first non-finite traction at step {bad // N}, receiver {bad % N}", flush=True)
    assert bad // N == 3
    assert (15 <= bad % N <= 17) if kind == "dense" else bad % N == 0
    op.close()
