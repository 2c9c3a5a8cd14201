"""GPU parity of the batched FDP=H form: independent faults in one operator.

Each fault of the batch is checked against the oracle's FDP=H-approximated
operator of that fault alone (Tier-B, its own cluster tree and lag count):
the batch must neither couple faults nor change any of them.  Steps past a
fault's own lag count must leave its tractions at zero.
"""
import numpy as np
import pytest

from oracle.dense import convolve_rows
from oracle.fdph import FdphOracle, FdphParams
from oracle.kernel2d import Problem
from synth import curved_fault, smooth_slip_rate, straight_fault

pytestmark = pytest.mark.gpu

# BF16 factors keep 8 mantissa bits; the leading cross terms of every block
# are stored as hi + lo BF16 pairs until the rounding bound of the rest is
# 2^-12 of the block, so the target of the mixed form holds.
BF16_TOL = 1e-4


def _relerr(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _batch_run(faults, D, params):
    import torch

    from paper_1903_02118_amd.binding import Operator

    op = Operator.compress_fdph_batched(faults, params=params)
    Dd = torch.from_numpy(np.ascontiguousarray(D)).to("cuda")
    Td = torch.full_like(Dd, np.nan)
    s = torch.cuda.current_stream()
    op.reset(stream=s)
    op.run(Dd, Td, stream=s)
    torch.cuda.synchronize()
    st = op.stats()
    op.close()
    return Td.cpu().numpy(), st


def _union_input(sizes, lags, seed0):
    """Concatenated slip rate [max M][sum N]; fault k's data at its columns.
    Steps past a fault's lag count carry data too, which must be ignored."""
    Mx = max(lags)
    D = np.concatenate([smooth_slip_rate(n, Mx, 10, 20, seed0 + k) for k, n in enumerate(sizes)], axis=1)
    return np.ascontiguousarray(D)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_batched_matches_each_fault_alone(gpu_lib, prec):
    from paper_1903_02118_amd.binding import BIE_FP64, BIE_MIXED_BF16, make_params

    sizes = [96, 200, 45, 333, 128]
    lags = [192, 150, 300, 260, 64]
    faults = [(*straight_fault(n), m) for n, m in zip(sizes, lags)]
    D = _union_input(sizes, lags, 11)
    code = BIE_FP64 if prec == "fp64" else BIE_MIXED_BF16
    print(f"batched {prec} sizes={sizes} lags={lags}", flush=True)
    T, st = _batch_run(faults, D, make_params(eps_aca=1e-8, precision=code))
    assert st["n_elem"] == sum(sizes) and st["n_lags"] == max(lags)
    off = np.concatenate([[0], np.cumsum(sizes)])
    n_adm = near = 0
    for k, (n, m) in enumerate(zip(sizes, lags)):
        xa, xb, _ = faults[k]
        o = FdphOracle(Problem(xa, xb, dt=0.5), m, FdphParams())
        n_adm += o.stats()["n_adm"]
        near += o.stats()["near_pairs"]
        Tb = convolve_rows(o.rows(np.arange(n)), D[:m, off[k]:off[k + 1]])
        Tg = T[:m, off[k]:off[k + 1]].T
        err = _relerr(Tg, Tb)
        print(f"  fault {k} N={n} M={m} rel err {err:.3e}", flush=True)
        assert err <= (1e-6 if prec == "fp64" else BF16_TOL)
        assert np.all(T[m:, off[k]:off[k + 1]] == 0.0)
    assert st["n_adm"] == n_adm and st["near_pairs"] == near


def test_batched_planar_and_curved(gpu_lib):
    """A curved fault in the batch makes every fault use both stress
    components (projected at the receivers); the planar ones must not change."""
    from paper_1903_02118_amd.binding import make_params

    faults = [(*straight_fault(150), 200), (*curved_fault(256), 240), (*straight_fault(70), 120)]
    sizes = [150, 256, 70]
    lags = [200, 240, 120]
    D = _union_input(sizes, lags, 21)
    print("batched planar+curved", flush=True)
    T, st = _batch_run(faults, D, make_params(eps_aca=1e-8))
    off = np.concatenate([[0], np.cumsum(sizes)])
    for k, (n, m) in enumerate(zip(sizes, lags)):
        xa, xb, _ = faults[k]
        o = FdphOracle(Problem(xa, xb, dt=0.5), m, FdphParams())
        rec = np.arange(0, n, 3)
        Tb = convolve_rows(o.rows(rec), D[:m, off[k]:off[k + 1]])
        err = _relerr(T[:m, off[k] + rec].T, Tb)
        print(f"  fault {k} N={n} M={m} rel err {err:.3e}", flush=True)
        assert err <= 1e-6
        assert np.all(T[m:, off[k]:off[k + 1]] == 0.0)


def test_batched_windows_match_oracle(gpu_lib):
    """Near windows W_ij of every fault of a batch equal the oracle's (exact
    integers), with the lag count of each fault capping its own windows.  On
    the curved fault the deviation from the static value changes sign after
    the fronts, so the windows end after short late runs of violations."""
    from paper_1903_02118_amd.binding import BIE_EXPORT_NEAR, Operator, make_params

    sizes = [256, 100, 256]
    lags = [600, 1500, 240]
    faults = [(*straight_fault(256), 600), (*straight_fault(100), 1500), (*curved_fault(256), 240)]
    op = Operator.compress_fdph_batched(faults, params=make_params())
    near = op.export(BIE_EXPORT_NEAR)
    op.close()
    off = np.concatenate([[0], np.cumsum(sizes)])
    got = {(int(r[0]), int(r[1])): int(r[2]) for r in near}
    ref = {}
    for k, (n, m) in enumerate(zip(sizes, lags)):
        xa, xb, _ = faults[k]
        o = FdphOracle(Problem(xa, xb, dt=0.5), m, FdphParams())
        for lf in o.leaves:
            if lf.admissible:
                continue
            for i in lf.tau.idx:
                W, _, _ = o.near_window(int(i), lf.sigma.idx)
                for j, w in zip(lf.sigma.idx, W):
                    ref[(int(i) + off[k], int(j) + off[k])] = int(w)
    assert got == ref
