#!/usr/bin/env python3
"""Benchmark of the per-step space-time BIEM convolution on one MI355X.

Workload (default): the FDP=H form in FP64 on the planar anti-plane fault,
N = 4096 elements, M = 2048 steps, eta = 2, leaf 32, eps_ACA = 1e-6,
n_c = 20, eps_Q = 1e-3, eps_st = 1e-6, slip rate a Gaussian-smoothed random
field (correlation 20 elements / 40 steps, seed 2).  A step is one pass of
the whole FDP=H per-step path (history update, near-field windows, far-field
FIR and ring scatter, 2D transient, per-receiver gather) for one time step.

The M-step run is the real one: the first M - W - K steps fill the history
(untimed), then W warm-up steps, then K timed steps at full history, all on
inputs resident in HBM.  The near-field kernel is autotuned first
(bie_autotune); the run is timed twice, with eager launches (the near-kernel
time per launch comes from HIP events on its stream) and with every step a
launch of one captured HIP graph (bie_run_graph), and the faster of the two
identical runs is the reported value.  The dense FP64 plain form on the same
problem is timed at full history as the comparator (after bie_advance over a
quiescent prefix, since a dense step's cost depends only on the step index).
The oracle (CPU, FP64) computes the FDP=H-approximated convolution on sampled
receivers: its result is the parity check (relative error) and its wall time
the CPU baseline.

Other workloads: --workload curved16k (sinusoidal fault, N = 16384,
M = 8192, mixed precision, staircase transient), --workload ensemble64
(64 independent planar faults in one batched operator), dense256 (the plain
form, N = 256, M = 128, whole runs), inplane2k (the plain form of the
in-plane problem, N = 2048, M = 2048) and rupture4k (dynamic rupture with
exponential slip weakening on the default fault: coupled steps).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published
PREC_NAMES = {"fp64": "FP64", "mixed": "mixed (FP32 windows and factors, FP64 sums and accumulators)",
              "bf16": "mixed (FP32 windows, BF16 factors, FP64 sums and accumulators)"}
N_DEF, M_DEF = 4096, 2048


def _kernel_source_hash():
    from paper_1903_02118_amd.profsum import source_hash

    return source_hash()


def _traffic(path, kernel_name):
    """HBM bytes per launch of `kernel_name` from committed counter data, or None.

    The file holds FETCH_SIZE and WRITE_SIZE of the kernel (rocprofv3 --pmc,
    KiB per dispatch), the same counters read for a plain copy kernel of
    known size, and the source hash of the kernels at measurement time; the
    figure is dropped when the kernels changed since.
    """
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    k = d.get("kernels", {}).get(kernel_name)
    if not k or d.get("source_hash") != _kernel_source_hash():
        return None
    return k["hbm_bytes"]


def hbm_probe(gib, dev, stream):
    """Best of three streaming reads of a gib-GiB device buffer (bie_hbm_read_probe)."""
    if not gib:
        return None
    import torch

    from paper_1903_02118_amd.binding import hbm_read_probe

    nb = int(gib * (1 << 30)) // 16 * 16
    buf = torch.ones(nb // 8, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    ms = min(hbm_read_probe(buf, stream) for _ in range(3))
    del buf
    torch.cuda.empty_cache()
    rate = nb / (ms / 1e3) / 1e9
    print(f"[bench] HBM read probe: {nb / 1e9:.1f} GB in {ms:.3f} ms -> {rate:.0f} GB/s", file=sys.stderr, flush=True)
    return {"bytes": nb, "GB/s": rate, "frac_of_peak": rate / HBM_PEAK_GBPS}


def near_lags_mean(W, n0, n1):
    """Mean over steps n0..n1 of sum over near pairs of min(W_ij, n + 1): the
    window lags a step applies (a pair's window is cut by the history)."""
    import numpy as np

    W = np.sort(np.asarray(W, dtype=np.int64))
    cs = np.concatenate([[0], np.cumsum(W)])
    tot = 0
    for n in range(n0, n1 + 1):
        k = int(np.searchsorted(W, n + 1, side="right"))  # pairs whose whole window has history
        tot += int(cs[k]) + (len(W) - k) * (n + 1)
    return tot / (n1 - n0 + 1)


# ---- CPU baseline: the oracle on the host cores, in a process pool --------------
CPU_WORKERS = 16   # the host cores one GPU's box provides
_CPU = {}          # inputs the pool's workers inherit (fork), set before the pool starts


def _one_thread():
    from threadpoolctl import threadpool_limits

    threadpool_limits(limits=1)


def cpu_pool(fn, items):
    """Map fn over items on min(16, cpu_count, len(items)) forked worker
    processes, one BLAS thread each.  Must run before anything initializes the
    GPU in this process (the workers are forks of it).  Returns (results,
    wall seconds, workers)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    if "torch" in sys.modules and sys.modules["torch"].cuda.is_initialized():
        raise RuntimeError("the oracle pool must start before the GPU is initialized")
    workers = max(1, min(CPU_WORKERS, os.cpu_count() or 1, len(items)))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork"), initializer=_one_thread) as ex:
        res = list(ex.map(fn, items))
    return res, time.perf_counter() - t0, workers


def _tierb_rows_convolved(recs):
    """Tier-B rows of some receivers, convolved over every step (oracle)."""
    from oracle.dense import convolve_rows_fft

    return convolve_rows_fft(_CPU["oracle"].rows(recs), _CPU["D"])


def _tierb_at(i):
    """Tier-B of one receiver at the sampled steps, leaf by leaf (oracle)."""
    return _CPU["oracle"].apply_at(int(i), _CPU["D"], _CPU["steps"])


def _exact_rows_convolved(recs):
    """The exact convolution (Tier-A) of some receivers over every step (oracle)."""
    import numpy as np

    from oracle.dense import convolve_rows_fft

    pr, N, M = _CPU["problem"], _CPU["N"], _CPU["M"]
    js = np.arange(N)
    K = np.stack([pr.kernel(int(i), js[:, None], np.arange(M)[None, :]) for i in recs])
    return convolve_rows_fft(K, _CPU["D"])


def _inplane_last_step(i):
    """Both traction components of receiver i at the last step with data (the
    exact in-plane convolution, oracle)."""
    import numpy as np

    pr, D2, N = _CPU["inplane"], _CPU["D2"], _CPU["N"]
    L = D2.shape[0]
    ks, kn = pr.kernel(int(i), np.arange(N)[None, :], np.arange(L)[:, None])  # [lag][j]
    n = L - 1
    return np.array([sum(kk[m] @ D2[n - m, :, c] for m in range(n + 1)) for c, kk in ((0, ks), (1, kn))])


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=208, help="timed steps K")
    ap.add_argument("--warmup", type=int, default=20, help="untimed warm-up steps W")
    ap.add_argument("--workload", choices=["planar4k", "curved16k", "ensemble64", "dense256", "inplane2k", "rupture4k"],
                    default="planar4k",
                    help="planar4k: planar fault N=4096 M=2048 eps_aca=1e-6 (FP64 by default); "
                         "curved16k: sinusoidal fault N=16384 M=8192 eps_aca=1e-5 (mixed by default); "
                         "ensemble64: 64 independent planar faults, N log-uniform in [1024, 16384], M=2N, "
                         "one batched operator, eps_aca=1e-4 (mixed by default); "
                         "dense256: plain dense form, planar fault N=256, M=128, i.i.d. U(0,1) slip rate; "
                         "inplane2k: plain dense form of the in-plane (P-SV) problem, N=2048, M=2048, two components; "
                         "rupture4k: dynamic rupture (coupled steps with exponential slip weakening) on the planar "
                         "fault N=4096, M=2048, FDP=H")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--dense-steps", type=int, default=5, help="timed steps of the dense comparator")
    ap.add_argument("--precision", choices=["fp64", "mixed", "bf16"], default=None,
                    help="fp64: everything FP64; mixed: FP32 near windows and factors, FP64 sums/accumulators; "
                         "bf16: as mixed with BF16 factors")
    ap.add_argument("--prefix", type=int, default=None,
                    help="ensemble64: quiescent steps run before the data (through bie_advance), default 4000; "
                         "faults whose runs (2N steps) have ended by then do no work")
    ap.add_argument("--eps-aca", type=float, default=None, help="ACA+ tolerance (default: the workload's)")
    ap.add_argument("--quantize-tr", choices=["auto", "on", "off"], default="auto",
                    help="staircase-quantized 2D Domain-S transient (running sums instead of the FIR); "
                         "auto: on for the curved fault and the ensemble (whose transients last most of the run), "
                         "off for planar4k")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the run with graph-launched steps")
    ap.add_argument("--no-autotune", action="store_true", help="keep the near kernel's default launch configuration")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-receivers", type=int, default=None, help="receivers of the oracle sample (16 planar, 2 curved)")
    ap.add_argument("--traffic-file", default=None,
                    help="counted-traffic summary (default: the committed one of the planar workload's precision)")
    ap.add_argument("--rhs", type=int, choices=[1, 2, 4], default=1,
                    help="planar4k/curved16k: slip-rate histories (scenarios) sharing the operator; the near field "
                         "reads each window value once for all of them")
    ap.add_argument("--hbm-probe", type=float, default=8.0, metavar="GIB",
                    help="size of the streaming-read probe (a plain 16-byte non-temporal read kernel) whose rate "
                         "puts the near kernel's next to what the HBM delivers to such a kernel; 0: skip")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB between two device buffers (a plain copy kernel of known size, "
                         "used to scale HBM counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (one process, one device).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "ensemble64":
        return run_ensemble(args)
    if args.workload == "dense256":
        return run_dense_small(args)
    if args.workload == "inplane2k":
        return run_inplane_dense(args)
    if args.workload == "rupture4k":
        return run_rupture(args)

    import numpy as np
    import torch

    from paper_1903_02118_amd.binding import (BIE_EXPORT_NEAR, BIE_FP64, BIE_MIXED_BF16, BIE_MIXED_FP32, Operator,
                                              make_params)
    from synth import curved_fault, smooth_slip_rate, straight_fault

    curved = args.workload == "curved16k"
    args.quantize_tr = args.quantize_tr == "on" or (args.quantize_tr == "auto" and curved)
    if args.n is None:
        args.n = 16384 if curved else N_DEF
    if args.m is None:
        args.m = 8192 if curved else M_DEF
    if args.precision is None:
        args.precision = "bf16" if curved else "fp64"
    eps_aca = args.eps_aca if args.eps_aca is not None else (1e-4 if curved else 1e-6)
    if args.cpu_receivers is None:
        args.cpu_receivers = 1 if curved else 32
    seed = 3 if curved else 2
    N, M, K, W = args.n, args.m, args.steps, args.warmup
    prefix = M - K - W
    if prefix < 0:
        sys.exit(f"--steps + --warmup must not exceed M={M}")
    xa, xb = curved_fault(N) if curved else straight_fault(N)
    D = smooth_slip_rate(N, M, 20.0, 40.0, seed)

    # ---- oracle on the host cores (before the GPU is touched) -------------------
    oracle = None
    if not args.no_cpu:
        from oracle.fdph import FdphOracle, FdphParams
        from oracle.kernel2d import Problem

        rng = np.random.Generator(np.random.PCG64(102))
        rec = np.sort(rng.choice(N, size=args.cpu_receivers, replace=False))
        fp = FdphParams(eta=2.0, leaf_size=32, eps_q=1e-3, eps_st=1e-6, n_c=20, quantize_tr=args.quantize_tr)
        t0 = time.perf_counter()
        _CPU.update(oracle=FdphOracle(Problem(xa, xb, dt=0.5), M, fp), D=D, N=N, M=M,
                    problem=Problem(xa, xb, dt=0.5))
        if curved:
            # sampled steps of the timed region, leaf by leaf (a full row is N x M)
            smp = sorted({prefix + W, prefix + W + K // 2, M - 1})
            _CPU["steps"] = smp
            Tb, wall, workers = cpu_pool(_tierb_at, list(rec))
            Tb = np.stack(Tb)
            units = len(rec) * len(smp)
        else:
            smp = None
            Tb, wall, workers = cpu_pool(_tierb_rows_convolved, [rec[k:k + 1] for k in range(len(rec))])
            Tb = np.concatenate(Tb)
            units = len(rec) * M
        oracle = {"rec": rec, "steps": smp, "Tb": Tb, "wall": wall, "workers": workers, "units": units}
        print(f"[bench] oracle {wall:.1f}s on {workers} cores for {len(rec)} receivers", file=sys.stderr, flush=True)
        if not curved:
            # the approximation's own error (reported, not gated): the exact
            # convolution of Eq. 4 with the closed-form kernel, first four receivers
            ra = rec[:4]
            t1 = time.perf_counter()
            Ta, _, _ = cpu_pool(_exact_rows_convolved, [ra[k:k + 1] for k in range(len(ra))])
            oracle["exact"] = (ra, np.concatenate(Ta), time.perf_counter() - t1)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    if args.calibrate_copy:
        nb = args.calibrate_copy * (1 << 20)
        a = torch.ones(nb // 8, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {nb} bytes", file=sys.stderr, flush=True)
        del a, b

    probe = hbm_probe(args.hbm_probe, dev, stream)
    R = args.rhs
    # scenario r > 0: another smoothed random field (seed + 100 r); rows hold the R scenarios
    DR = D if R == 1 else np.concatenate([D] + [smooth_slip_rate(N, M, 20.0, 40.0, seed + 100 * r)
                                                for r in range(1, R)], axis=1)
    Dd = torch.from_numpy(DR).to(dev)
    Td = torch.zeros_like(Dd)
    prec = {"fp64": BIE_FP64, "mixed": BIE_MIXED_FP32, "bf16": BIE_MIXED_BF16}[args.precision]
    params = make_params(eta=2.0, leaf_size=32, n_c=20, eps_aca=eps_aca, eps_q=1e-3, eps_st=1e-6, seed=12345,
                         precision=prec, quantize_tr=args.quantize_tr, n_rhs=R)
    op, setup = build_fdph_timed([(xa, xb, M)], params, stream, torch)
    setup_s = setup["total_s"]
    st = op.stats()
    print(f"[bench] FDP=H N={N} M={M} built in {setup_s:.1f}s ({_setup_text(setup)}): adm={st['n_adm']} "
          f"inadm={st['n_inadm']} near_pairs={st['near_pairs']} near_lags={st['near_lags']} ranks={st['rank_sum']}, "
          f"{st['aca_host_blocks']} ACA+ blocks on the host", file=sys.stderr, flush=True)

    tune = None
    if not args.no_autotune:
        tune = op.autotune(reps=3, stream=stream)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    op.reset(stream=stream)
    if prefix:
        op.run(Dd[:prefix], Td[:prefix], stream=stream)
    if W:
        op.run(Dd[prefix:prefix + W], Td[prefix:prefix + W], stream=stream)
    torch.cuda.synchronize()
    op.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    op.run(Dd[prefix + W:], Td[prefix + W:], stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    near_ms, near_launches = op.timing_read()
    op.timing(False)
    tb = st["time_block"]
    if tb > 1 and K % tb and K >= tb:
        # the timed steps end in single steps: time the near kernel of whole
        # blocks alone (same steps, untimed otherwise) so that its average
        # launch is one block's
        Tb = torch.zeros_like(Dd)
        op.reset(stream=stream)
        op.run(Dd[:prefix + W], Tb[:prefix + W], stream=stream)
        torch.cuda.synchronize()
        op.timing(True)
        op.run(Dd[prefix + W:prefix + W + K - K % tb], Tb[prefix + W:prefix + W + K - K % tb], stream=stream)
        torch.cuda.synchronize()
        near_ms, near_launches = op.timing_read()
        op.timing(False)
        del Tb
    T = Td.cpu().numpy()
    steps_per_s = K / elapsed
    ms_per_step = 1e3 * elapsed / K
    near_avg_s = near_ms / 1e3 / max(near_launches, 1)
    # algorithmic near-field bytes of the timed steps: lags m <= min(n, W_ij - 1) of every pair
    kb = 8.0 if args.precision == "fp64" else 4.0
    near_bytes = kb * near_lags_mean(op.export(BIE_EXPORT_NEAR)[:, 2], prefix + W, M - 1)
    achieved = near_bytes / near_avg_s / 1e9
    step_gbps = (st["bytes_per_step"] - st["near_bytes_per_step"] + near_bytes) * steps_per_s / 1e9
    print(f"[bench] FDP=H {steps_per_s:.1f} steps/s ({ms_per_step:.3f} ms/step), near kernel {1e3*near_avg_s:.3f} ms "
          f"-> {achieved:.0f} GB/s algorithmic", file=sys.stderr, flush=True)

    # ---- the same run with every step a launch of one captured graph ---------------
    graph = None
    if not args.no_graph:
        # capture (and instantiate) the timed slice's graph once, untimed; the
        # timed call then replays it: same buffers, same first step
        Tg = torch.zeros_like(Dd)
        for timed_pass in (False, True):
            # the eager run's calls before the timed steps (time blocks at the same steps)
            op.reset(stream=stream)
            if prefix:
                op.run(Dd[:prefix], Tg[:prefix], stream=stream)
            if W:
                op.run(Dd[prefix:prefix + W], Tg[prefix:prefix + W], stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            op.run_graph(Dd[prefix + W:], Tg[prefix + W:], stream=stream)
            torch.cuda.synchronize()
            eg = time.perf_counter() - t0
        same = bool(torch.equal(Tg, Td))
        graph = {"steps_per_s": K / eg, "ms_per_step": 1e3 * eg / K, "identical_to_eager": same}
        print(f"[bench] FDP=H graph launches {K / eg:.1f} steps/s ({1e3 * eg / K:.3f} ms/step), "
              f"identical to eager: {same}", file=sys.stderr, flush=True)
        del Tg
        if same and K / eg > steps_per_s:
            steps_per_s, ms_per_step = K / eg, 1e3 * eg / K
            step_gbps = (st["bytes_per_step"] - st["near_bytes_per_step"] + near_bytes) * steps_per_s / 1e9

    # ---- the same steps one at a time (bie_step: the single-step kernels) -----------
    per_step = None
    if st["time_block"] > 1:
        Ts = torch.zeros_like(Dd)
        op.reset(stream=stream)
        op.run(Dd[:prefix + W], Ts[:prefix + W], stream=stream)
        torch.cuda.synchronize()
        op.timing(True)
        t0 = time.perf_counter()
        for k in range(prefix + W, prefix + W + K):
            op.step(Dd[k], Ts[k], stream=stream)
        torch.cuda.synchronize()
        es = time.perf_counter() - t0
        sn_ms, sn_n = op.timing_read()
        op.timing(False)
        sn_s = sn_ms / 1e3 / max(sn_n, 1)
        per_step = {"steps_per_s": K / es, "ms_per_step": 1e3 * es / K, "near_kernel_ms": 1e3 * sn_s,
                    "near_gbps_algorithmic": near_bytes / sn_s / 1e9, "near_frac": near_bytes / sn_s / 1e9 / HBM_PEAK_GBPS,
                    # time blocks sum the same terms in another order (matrix cores)
                    "rel_diff_vs_time_blocks": float(torch.linalg.norm(Ts - Td) / torch.linalg.norm(Ts))}
        print(f"[bench] FDP=H one step per call {K / es:.1f} steps/s ({1e3 * es / K:.3f} ms/step), near kernel "
              f"{1e3 * sn_s:.3f} ms -> {near_bytes / sn_s / 1e9:.0f} GB/s; rel diff vs blocks "
              f"{per_step['rel_diff_vs_time_blocks']:.2e}", file=sys.stderr, flush=True)
        del Ts
    op.close()
    del Td

    # ---- plain form (FP64, causal band of the dense tensor) at full history ------
    dense = None
    if not args.no_dense:
        from paper_1903_02118_amd.binding import Plan

        t0 = time.perf_counter()
        dplan = Plan.dense(xa, xb, M)
        need = dplan.workspace_size()
        free, _ = torch.cuda.mem_get_info(dev)
        if free < need + 2e9:
            dense = {"skipped": f"needs {need / 1e9:.0f} GB, {free / 1e9:.0f} GB free"}
            dplan.close()
        else:
            dop = Operator.from_plan(dplan, stream=stream)
            dplan.close()
            dsetup = time.perf_counter() - t0
            Kd, Wd = args.dense_steps, 2
            Td2 = torch.zeros((Kd + Wd, N), dtype=torch.float64, device=dev)
            Dd1 = Dd[:, :N].contiguous()
            # steps n >= M read every lag of the band: steady state
            dop.reset(stream=stream)
            dop.advance(M, stream=stream)
            dop.run(Dd1[:Wd], Td2[:Wd], stream=stream)
            torch.cuda.synchronize()
            dop.timing(True)
            t0 = time.perf_counter()
            dop.run(Dd1[Wd:Wd + Kd], Td2[Wd:], stream=stream)
            torch.cuda.synchronize()
            de = time.perf_counter() - t0
            dk_ms, dk_n = dop.timing_read()
            dst = dop.stats()
            dbytes = dst["bytes_per_step"]
            dense = {
                "form": "plain dense convolution of Eq. 4, causal band of the kernel tensor (the exact zeros outside "
                        "the S-wave cone skipped), FP64",
                "steps_per_s": Kd / de,
                "ms_per_step": 1e3 * de / Kd,
                "hbm_gbps_algorithmic": dbytes * Kd / de / 1e9,
                "kernel_ms": dk_ms / max(dk_n, 1),
                "kernel_gbps": dbytes / (dk_ms / max(dk_n, 1) / 1e3) / 1e9 if dk_n else None,
                "bytes_per_step": dbytes,
                "full_tensor_bytes_per_step": 8.0 * M * N * N,
                "setup_s": dsetup,
                "steps_timed": Kd,
                "timed_steps_at": [M + Wd, M + Wd + Kd - 1],
            }
            dop.close()
            del Td2, dop
            torch.cuda.empty_cache()
            print(f"[bench] dense FP64 (causal band, {dbytes / 1e9:.1f} GB/step) {dense['steps_per_s']:.2f} steps/s "
                  f"({dense['ms_per_step']:.1f} ms/step, {dense['hbm_gbps_algorithmic']:.0f} GB/s)",
                  file=sys.stderr, flush=True)

    # ---- oracle: parity on sampled receivers and the CPU baseline -----------------
    cpu = None
    rel_err = None
    method_err = None
    if oracle is not None:
        rec, Tb = oracle["rec"], oracle["Tb"]
        Tg = T[oracle["steps"]][:, rec].T if curved else T[:, rec].T  # scenario 0
        rel_err = float(np.linalg.norm(Tg - Tb) / np.linalg.norm(Tb))
        cpu = {
            "value": oracle["units"] / (N * oracle["wall"]),
            "unit": "steps/s",
            "cores": oracle["workers"],
            "kind": "oracle",
            "sample": (f"FDP=H-approximated operator applied by the oracle (FP64, one process per core) to "
                       f"{len(rec)} seeded receiver{'s' if len(rec) > 1 else ''} at "
                       + (f"{len(oracle['steps'])} sampled steps" if curved else f"all {M} steps")
                       + f"; {oracle['wall']:.1f} s wall on {oracle['workers']} cores, extrapolated to {N} "
                       f"receivers per step"),
        }
        print(f"[bench] GPU vs oracle rel err {rel_err:.2e}", file=sys.stderr, flush=True)
        if "exact" in oracle:
            ra, Ta, t_exact = oracle["exact"]
            method_err = {
                "value": float(np.linalg.norm(T[:, ra].T - Ta) / np.linalg.norm(Ta)),
                "sample": f"{len(ra)} seeded receivers at all {M} steps against the exact convolution (Tier-A)",
            }
            print(f"[bench] FDP=H vs exact convolution {method_err['value']:.2e} ({t_exact:.1f}s)",
                  file=sys.stderr, flush=True)

    # counted HBM bytes per launch, from the committed counter runs of this
    # workload (planar N=4096, M=2048, one scenario) in this precision
    tfile = args.traffic_file or os.path.join(
        ROOT, "profiles", f"k_near_fdph_{'fp64' if args.precision == 'fp64' else 'mixed'}_n4096_m2048_traffic.json")
    planar_std = not curved and N == 4096 and M == 2048 and R == 1 and args.precision in ("fp64", "mixed")
    # the near kernel the run used: the matrix-core one for time blocks (16
    # steps per pass; on single lag chunks or chunk groups), unless the
    # autotuner or BIE_NEAR_MFMA=0 chose the lane-per-lag one (8 steps per launch)
    mf = tb > 1 and (tune["mfma"] >= 1 if tune else os.environ.get("BIE_NEAR_MFMA", "1") != "0")
    kname, spp = ("k_near_mfma", tb) if mf else (("k_near_tb", 8) if tb > 1 else ("k_near", 1))
    traffic = _traffic(tfile, kname) if planar_std else None
    line = {
        "metric": "time steps/sec and HBM GB/s of per-step H-matvec vs dense FP64, at rel err <=1e-4",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"FDP=H {PREC_NAMES[args.precision]}, 2D anti-plane "
                        f"{'curved (sinusoidal, amplitude 0.05L, wavelength L/4)' if curved else 'planar'} fault, "
                        f"N={N}, M={M}, eta=2, leaf 32, eps_aca={eps_aca:g}, "
                        f"n_c=20, eps_q=1e-3, eps_st=1e-6, "
                        f"{'staircase transient (eps 0.1), ' if args.quantize_tr else ''}"
                        f"smoothed random slip rate (20 el, seed {seed})"
                        + (f"; {R} scenarios sharing the operator (seeds {seed} + 100 r)" if R > 1 else ""),
            "N": N,
            "M": M,
            "n_rhs": R,
            "history_steps_untimed": prefix,
            "timed_steps_at": [prefix + W, M - 1],
            "time_block": st["time_block"],
        },
        "hbm_gbps_algorithmic": step_gbps,
        "step_launch": ("graph" if graph and graph["identical_to_eager"] and graph["steps_per_s"] >= K / elapsed
                        else "eager"),
        "eager": {"steps_per_s": K / elapsed, "ms_per_step": 1e3 * elapsed / K},
        "graph": graph,
        "rel_err_vs_oracle": rel_err,
        "method_error_vs_exact": method_err,
        "dense_fp64": dense,
        # the causal-band plain form runs one step per pass over its band
        "speedup_vs_dense_fp64": (steps_per_s / dense["steps_per_s"]) if dense and "steps_per_s" in dense else None,
        "speedup_vs_dense_fp64_one_step_per_pass": (per_step["steps_per_s"] / dense["steps_per_s"])
        if dense and "steps_per_s" in dense and per_step else None,
        "per_step": per_step,
        "roofline": {
            "bound": "hbm",
            "kernel": (f"{kname}<{'double' if args.precision == 'fp64' else 'float'}> "
                       f"(near-field window convolution{', %d steps per pass' % spp if spp > 1 else ''})"),
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": near_bytes,
            "avg_launch_ms": 1e3 * near_avg_s,
        },
        "hbm_read_probe": dict(probe, near_frac_of_probe=achieved / probe["GB/s"]) if probe else None,
        "scenarios": {"n_rhs": R, "scenario_steps_per_s": R * steps_per_s} if R > 1 else None,
        "cpu_baseline": cpu,
        "operator": {k: st[k] for k in ("n_adm", "n_inadm", "near_pairs", "near_lags", "rank_sum", "rank_max", "aca_fallbacks",
                                        "aca_host_blocks", "aca_seconds", "device_bytes", "bytes_per_step", "flops_per_step")},
        "near_autotune": tune,
        "setup_s": setup_s,
        "setup": setup,
    }
    print(json.dumps(line))


def build_fdph_timed(faults, params, stream, torch):
    """FDP=H operator through the plan calls, each phase timed: the host plan
    (trees, ART integers, transients, near tiles), the device stage (near
    windows and ACA+, then the far-field and near-field layouts), and the
    build inside the workspace (uploads, window fill, zeroed state)."""
    from paper_1903_02118_amd.binding import Operator, Plan

    t0 = time.perf_counter()
    plan = Plan.fdph(faults, params=params)
    t1 = time.perf_counter()
    plan.windows(stream=stream)
    torch.cuda.empty_cache()  # the scratch of the device stage is free again
    t2 = time.perf_counter()
    op = Operator.from_plan(plan, stream=stream)
    t3 = time.perf_counter()
    aca = plan.stats()["aca_seconds"]
    plan.close()
    return op, {"total_s": t3 - t0, "host_plan_s": t1 - t0, "device_stage_s": t2 - t1, "aca_s": aca,
                "build_s": t3 - t2}


def _setup_text(setup):
    return (f"host plan {setup['host_plan_s']:.2f}s, device stage {setup['device_stage_s']:.2f}s with ACA+ "
            f"{setup['aca_s']:.2f}s, build {setup['build_s']:.2f}s")


def run_dense_small(args):
    """The plain dense form on its own small configuration: planar fault, N = 256, M = 128,
    slip rate i.i.d. U(0,1) (seed 1).  A step is one step of the 128-step run; the whole run is
    repeated (reset, then 128 steps) and the mean over the run is reported, once with eager launches
    and once with every step a launch of one captured graph (a step moves at most 34 MB, so launch
    overhead matters).  The kernel tensor (67 MB) stays in the GPU's caches between steps."""
    import numpy as np
    import torch

    from paper_1903_02118_amd.binding import Operator
    from synth import straight_fault, uniform_slip_rate

    N, M = 256, 128
    reps = max(10, args.steps // M)
    xa, xb = straight_fault(N)
    D = uniform_slip_rate(N, M, 1)
    oracle = None
    if not args.no_cpu:
        # the exact convolution of every receiver over the whole run, receivers
        # split over the host cores (before the GPU is touched)
        from oracle.kernel2d import Problem

        _CPU.update(problem=Problem(xa, xb, dt=0.5), D=D, N=N, M=M)
        parts = [np.arange(k, N, 16) for k in range(16)]
        res, wall, workers = cpu_pool(_exact_rows_convolved, parts)
        Tref = np.zeros((M, N))
        for idx, r in zip(parts, res):
            Tref[:, idx] = r.T
        oracle = {"T": Tref, "wall": wall, "workers": workers}
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    op = Operator.build_kernel(xa, xb, M, stream=stream)
    st = op.stats()
    Dd = torch.from_numpy(D).to(dev)
    Te = torch.zeros_like(Dd)
    Tg = torch.zeros_like(Dd)

    def timed(fn, T):
        for _ in range(2):  # warm-up runs
            op.reset(stream=stream)
            fn(Dd, T, stream=stream)
        torch.cuda.synchronize()
        op.timing(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            op.reset(stream=stream)
            fn(Dd, T, stream=stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        k_ms, k_n = op.timing_read()
        op.timing(False)
        return el, (k_ms / k_n if k_n else None)

    el_e, kern_ms = timed(op.run, Te)
    el_g, _ = timed(op.run_graph, Tg)
    same = bool(torch.equal(Te, Tg))
    T = Te.cpu().numpy()
    op.close()
    steps = reps * M
    sps_e, sps_g = steps / el_e, steps / el_g
    best = sps_g if (same and sps_g > sps_e) else sps_e
    # algorithmic bytes of the run: step n reads the causal bands of lags 0..n
    # (8 B per kernel value), the history row of each of those lags (N values)
    # and the band rows' metadata (12 B per row)
    from paper_1903_02118_amd.binding import Plan

    pl = Plan.dense(xa, xb, M)
    lag_e = pl.lag_entries(M)
    pl.close()
    cum = np.cumsum(lag_e)
    run_bytes = float(sum(8.0 * cum[n] + 20.0 * N * (n + 1) for n in range(M)))
    print(f"[bench] dense N={N} M={M}: eager {sps_e:.0f} steps/s, graph {sps_g:.0f} steps/s (identical: {same})",
          file=sys.stderr, flush=True)
    cpu = None
    rel_err = None
    if oracle is not None:
        rel_err = float(np.linalg.norm(T - oracle["T"]) / np.linalg.norm(oracle["T"]))
        cpu = {"value": M / oracle["wall"], "unit": "steps/s", "cores": oracle["workers"], "kind": "oracle",
               "sample": f"the whole {M}-step run of all {N} receivers (kernel rows from the closed form, then the "
                         f"convolution of Eq. 4), {oracle['wall']:.2f} s wall on {oracle['workers']} cores"}
        print(f"[bench] oracle {oracle['wall']:.2f}s; GPU vs oracle rel err {rel_err:.2e}", file=sys.stderr, flush=True)
    line = {
        "metric": "time steps/sec and HBM GB/s of per-step H-matvec vs dense FP64, at rel err <=1e-4",
        "value": best,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 2 * M,
        "ms_per_step": 1e3 / best,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain dense form FP64, planar anti-plane fault, N={N}, M={M}, full {M}-step run "
                               f"repeated {reps} times, slip rate i.i.d. U(0,1) (seed 1)", "N": N, "M": M},
        "eager": {"steps_per_s": sps_e},
        "graph": {"steps_per_s": sps_g, "identical_to_eager": same},
        "hbm_gbps_algorithmic": run_bytes / M * best / 1e9,
        "rel_err_vs_oracle": rel_err,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_dense_step (lag-chunked dense sum)",
            "achieved": (run_bytes / M) / (kern_ms / 1e3) / 1e9 if kern_ms else None,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": ((run_bytes / M) / (kern_ms / 1e3) / 1e9 / HBM_PEAK_GBPS) if kern_ms else None,
            "traffic": None,
            "algorithmic_bytes_per_launch": run_bytes / M,
            "avg_launch_ms": kern_ms,
            "note": "the 67 MB kernel tensor is cache-resident between steps, so the rate can exceed HBM peak",
        },
        "cpu_baseline": cpu,
        "operator": {"device_bytes": st["device_bytes"]},
    }
    print(json.dumps(line))


def run_inplane_dense(args):
    """Plain dense form of the in-plane (P-SV) problem on a straight fault: N = 2048, M = 2048,
    alpha = 1, beta = alpha/sqrt(3), alpha dt/dx = 1/2, shear slip and opening rates from two
    smoothed random fields (seeds 4, 5).  Steps are timed at full history (the kernel tensors of
    both components' causal bands are read every step, the timed steps lying past step M); the
    history before the data is quiescent (bie_advance), which changes no cost."""
    import numpy as np
    import torch

    from paper_1903_02118_amd.binding import BIE_MODE_INPLANE, Operator
    from synth import smooth_slip_rate, straight_fault

    N, M = args.n or 2048, args.m or 2048
    K, W = min(args.steps, 10), min(args.warmup, 2)
    alpha, beta, dt = 1.0, 1.0 / np.sqrt(3.0), 0.5
    xa, xb = straight_fault(N)
    D2 = np.stack([smooth_slip_rate(N, K + W, 50, 50, 4), smooth_slip_rate(N, K + W, 50, 50, 5)], axis=2)
    oracle = None
    if not args.no_cpu:
        # exact rows of 16 seeded receivers, both components, at the last timed
        # step, on the host cores (before the GPU is touched)
        from oracle.inplane2d import InplaneProblem

        rng = np.random.Generator(np.random.PCG64(104))
        rec = np.sort(rng.choice(N, size=16, replace=False))
        _CPU.update(inplane=InplaneProblem(xa[:, 0], xb[:, 0], alpha=alpha, beta=beta, dt=dt), D2=D2, N=N)
        ref, wall, workers = cpu_pool(_inplane_last_step, list(rec))
        oracle = {"rec": rec, "ref": np.array(ref), "wall": wall, "workers": workers}
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    op = Operator.build_kernel(xa, xb, M, stream=stream, mode=BIE_MODE_INPLANE, alpha=alpha, beta=beta, dt=dt)
    setup_s = time.perf_counter() - t0
    st = op.stats()
    Dd = torch.from_numpy(D2.reshape(K + W, 2 * N)).to(dev)
    Td = torch.zeros_like(Dd)
    op.reset(stream=stream)
    op.advance(M, stream=stream)  # steps n >= M read every lag of the bands: steady state
    op.run(Dd[:W], Td[:W], stream=stream)
    torch.cuda.synchronize()
    op.timing(True)
    t0 = time.perf_counter()
    op.run(Dd[W:], Td[W:], stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    k_ms, k_n = op.timing_read()
    op.close()
    T = Td.cpu().numpy().reshape(K + W, N, 2)
    sps = K / el
    step_bytes = st["bytes_per_step"]  # every lag of both components' causal bands
    print(f"[bench] in-plane dense N={N} M={M}: {sps:.2f} steps/s ({1e3 * el / K:.1f} ms/step), built in "
          f"{setup_s:.1f}s", file=sys.stderr, flush=True)
    rel_err = None
    cpu = None
    if oracle is not None:
        n_loc = K + W - 1  # local row of the last step
        got = np.stack([T[n_loc, i, :] for i in oracle["rec"]])
        rel_err = float(np.linalg.norm(got - oracle["ref"]) / np.linalg.norm(oracle["ref"]))
        nr = len(oracle["rec"])
        # nr receivers over K + W lags -> N receivers over M lags (both components in both)
        cpu_per_step = oracle["wall"] * (N / float(nr)) * (M / float(K + W))
        cpu = {"value": 1.0 / cpu_per_step, "unit": "steps/s", "cores": oracle["workers"], "kind": "oracle",
               "sample": f"exact rows of {nr} receivers x 2 components over the {K + W} lags with data, "
                         f"{oracle['wall']:.2f} s wall on {oracle['workers']} cores, extrapolated to {N} receivers "
                         f"x 2 components x {M} lags per step"}
        print(f"[bench] oracle {oracle['wall']:.2f}s; GPU vs oracle rel err {rel_err:.2e}", file=sys.stderr, flush=True)
    line = {
        "metric": "time steps/sec and HBM GB/s of per-step H-matvec vs dense FP64, at rel err <=1e-4",
        "value": sps,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"plain dense form FP64, in-plane (P-SV) straight fault, N={N}, M={M}, two "
                               f"components, alpha=1, beta=1/sqrt(3), alpha dt/dx=1/2, full history",
                   "N": N, "M": M},
        "hbm_gbps_algorithmic": step_bytes * sps / 1e9,
        "rel_err_vs_oracle": rel_err,
        "roofline": {"bound": "hbm", "kernel": "k_dense_step (both components per timed interval)",
                     "achieved": (step_bytes / (k_ms / k_n / 1e3) / 1e9) if k_n else None,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": (step_bytes / (k_ms / k_n / 1e3) / 1e9 / HBM_PEAK_GBPS) if k_n else None,
                     "traffic": None, "algorithmic_bytes_per_launch": step_bytes,
                     "avg_launch_ms": (k_ms / k_n) if k_n else None},
        "cpu_baseline": cpu,
        "operator": {"device_bytes": st["device_bytes"], "bytes_per_step": st["bytes_per_step"]},
        "setup_s": setup_s,
    }
    print(json.dumps(line))


def _ensemble_oracle(item):
    """Tier-B of some receivers of one fault of the ensemble at the sampled steps (oracle)."""
    import numpy as np

    from oracle.fdph import FdphOracle, FdphParams
    from oracle.kernel2d import Problem

    k, recs = item
    xa, xb, m = _CPU["faults"][k]
    P, data = _CPU["P"], _CPU["data"][k]
    Dk = np.zeros((P + data.shape[0], data.shape[1]))
    Dk[P:] = data
    o = FdphOracle(Problem(xa, xb, dt=0.5), m, FdphParams(eta=2.0, leaf_size=32, eps_q=1e-3, eps_st=1e-6, n_c=20,
                                                         quantize_tr=_CPU["quant"]))
    return np.stack([o.apply_at(int(i), Dk, _CPU["steps"]) for i in recs])


def _ensemble_timed(op, Dd, Td, P, W, K, stream, torch):
    """Quiescent prefix (bie_advance), W warm-up and K timed steps; returns the
    wall seconds of the K steps and the near kernel's average launch time."""
    op.reset(stream=stream)
    t0 = time.perf_counter()
    op.advance(P, stream=stream)
    torch.cuda.synchronize()
    print(f"[bench] {P} quiescent steps in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if W:
        op.run(Dd[:W], Td[:W], stream=stream)
    torch.cuda.synchronize()
    op.timing(True)
    t0 = time.perf_counter()
    op.run(Dd[W:], Td[W:], stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    near_ms, near_launches = op.timing_read()
    op.timing(False)
    return elapsed, near_ms / 1e3 / max(near_launches, 1)


def run_ensemble(args):
    """64 independent planar faults in one batched FDP=H operator (the batched
    configuration): N_k log-uniform in [1024, 16384] (seed 5), M_k = 2 N_k,
    eta = 2, leaf 32, eps_ACA = 1e-4, n_c = 20, eps_Q = 1e-3, eps_st = 1e-6,
    BF16 factors, FP32 near windows, FP64 sums and accumulators.  A step
    advances every fault by one time step with one set of launches.  The run
    starts from rest: `--prefix` steps of zero slip rate go through
    bie_advance (the same kernels and memory traffic as any other step), then
    W warm-up and K timed steps consume a Gaussian-smoothed random field per
    fault (20 elements / 40 steps, seed 5000 + k).  The default window lies
    past the shortest faults' runs (those have ended: zero tractions, no
    work) and where the long faults' near windows are mostly filled; the line
    reports the active faults and the share of near-window lags applied.  The
    same window is then timed on the FP64 operator of the same faults (the
    speed-up of the mixed batched form over FP64), when it fits in HBM."""
    import numpy as np
    import torch

    from paper_1903_02118_amd.binding import BIE_EXPORT_NEAR, BIE_FP64, BIE_MIXED_BF16, BIE_MIXED_FP32, Operator, \
        Plan, make_params
    from synth import ensemble_sizes, smooth_slip_rate, straight_fault

    args.quantize_tr = args.quantize_tr != "off"  # auto: on (runs of 2N steps keep long transients)
    prec_name = args.precision or "bf16"
    codes = {"fp64": BIE_FP64, "mixed": BIE_MIXED_FP32, "bf16": BIE_MIXED_BF16}
    eps_aca = args.eps_aca if args.eps_aca is not None else 1e-4
    sizes = ensemble_sizes(64, 1024, 16384, 5)
    lags = 2 * sizes
    K, W = args.steps, args.warmup
    P = args.prefix if args.prefix is not None else 4000
    S = W + K
    if P + S > int(lags.max()):
        sys.exit(f"--prefix + --warmup + --steps must not exceed the longest run ({int(lags.max())} steps)")
    faults = [(*straight_fault(int(n)), int(m)) for n, m in zip(sizes, lags)]
    off = np.concatenate([[0], np.cumsum(sizes)])
    Ntot = int(off[-1])
    data = [smooth_slip_rate(int(n), S, 20.0, 40.0, 5000 + k) for k, n in enumerate(sizes)]
    D = np.ascontiguousarray(np.concatenate(data, axis=1))
    steps = [P + W, P + S - 1]
    active = int(np.sum(lags > P + W))

    # ---- oracle on the host cores (before the GPU is touched) ----------------------
    oracle = None
    if not args.no_cpu:
        rng = np.random.Generator(np.random.PCG64(105))
        live = [k for k in range(64) if lags[k] > P + S - 1]
        pick = sorted({min(live, key=lambda k: sizes[k]), max(live, key=lambda k: sizes[k]),
                       *rng.choice(live, size=2, replace=False).tolist()})
        recs = {k: np.sort(np.random.Generator(np.random.PCG64(500 + k)).choice(int(sizes[k]), size=2, replace=False))
                for k in pick}
        _CPU.update(faults=faults, data=data, P=P, steps=steps, quant=args.quantize_tr)
        items = [(k, recs[k][q:q + 1]) for k in pick for q in range(2)]
        res, wall, workers = cpu_pool(_ensemble_oracle, items)
        oracle = {"items": items, "Tb": res, "wall": wall, "workers": workers}
        print(f"[bench] oracle {wall:.1f}s on {workers} cores for {len(items)} receivers", file=sys.stderr, flush=True)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    def params(code):
        return make_params(eta=2.0, leaf_size=32, n_c=20, eps_aca=eps_aca, eps_q=1e-3, eps_st=1e-6, seed=12345,
                           precision=code, quantize_tr=args.quantize_tr)

    op, setup = build_fdph_timed(faults, params(codes[prec_name]), stream, torch)
    setup_s = setup["total_s"]
    st = op.stats()
    print(f"[bench] ensemble of 64 faults, sum N={Ntot}, max M={int(lags.max())}, built in {setup_s:.1f}s: "
          f"adm={st['n_adm']} inadm={st['n_inadm']} near_pairs={st['near_pairs']} near_lags={st['near_lags']} "
          f"device={st['device_bytes']/1e9:.1f} GB ({_setup_text(setup)}, {st['aca_host_blocks']} ACA+ blocks on the "
          f"host)", file=sys.stderr, flush=True)
    tune = None
    if not args.no_autotune:
        tune = op.autotune(reps=3, stream=stream)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    tb = st["time_block"]
    mf = tb > 1 and (tune["mfma"] >= 1 if tune else os.environ.get("BIE_NEAR_MFMA", "1") != "0")
    kname, spp = ("k_near_mfma", tb) if mf else (("k_near_tb", 8) if tb > 1 else ("k_near", 1))
    # algorithmic near-field bytes of the timed steps: lags m <= min(n, W_ij - 1) of the
    # pairs of every fault still running (a finished fault's kernels skip their work)
    Wp = op.export(BIE_EXPORT_NEAR)
    fault_of = np.searchsorted(off, Wp[:, 0], side="right") - 1
    live_pairs = lags[fault_of] > P + W
    timed = np.arange(P + W, P + S)
    near_lags_timed = near_lags_mean(Wp[live_pairs, 2], int(timed[0]), int(timed[-1]))
    lag_share = near_lags_timed / float(Wp[live_pairs, 2].sum())
    del Wp, fault_of, live_pairs
    kb = 8.0 if prec_name == "fp64" else 4.0
    near_bytes = kb * near_lags_timed
    Dd = torch.from_numpy(D).to(dev)
    Td = torch.zeros_like(Dd)
    elapsed, near_avg_s = _ensemble_timed(op, Dd, Td, P, W, K, stream, torch)
    T = Td.cpu().numpy()
    op.close()
    del op
    torch.cuda.empty_cache()
    steps_per_s = K / elapsed
    achieved = near_bytes / near_avg_s / 1e9
    print(f"[bench] ensemble {steps_per_s:.2f} steps/s ({1e3 * elapsed / K:.2f} ms/step), near kernel "
          f"{1e3 * near_avg_s:.2f} ms -> {achieved:.0f} GB/s algorithmic; {active} faults active, "
          f"{100 * lag_share:.0f}% of their near-window lags applied", file=sys.stderr, flush=True)

    # ---- the same faults and window in FP64 --------------------------------------------
    fp64 = None
    if prec_name != "fp64" and not args.no_dense:
        plan = Plan.fdph(faults, params=params(BIE_FP64))
        plan.windows(stream=stream)
        need = plan.workspace_size()
        free, _ = torch.cuda.mem_get_info(dev)
        if need + 2e9 > free:
            fp64 = {"skipped": f"the FP64 operator needs {need / 1e9:.0f} GB, {free / 1e9:.0f} GB free"}
            plan.close()
        else:
            op64 = Operator.from_plan(plan, stream=stream)
            plan.close()
            if not args.no_autotune:
                op64.autotune(reps=3, stream=stream)
            T64 = torch.zeros_like(Dd)
            e64, n64 = _ensemble_timed(op64, Dd, T64, P, W, K, stream, torch)
            fp64 = {"steps_per_s": K / e64, "ms_per_step": 1e3 * e64 / K, "near_kernel_ms": 1e3 * n64,
                    "device_bytes": op64.stats()["device_bytes"],
                    "rel_diff_of_mixed": float(torch.linalg.norm(Td - T64) / torch.linalg.norm(T64))}
            op64.close()
            del op64, T64
            torch.cuda.empty_cache()
            print(f"[bench] ensemble FP64 {fp64['steps_per_s']:.2f} steps/s; mixed is "
                  f"{steps_per_s / fp64['steps_per_s']:.2f}x", file=sys.stderr, flush=True)

    cpu = None
    rel_err = None
    if oracle is not None:
        num = den = 0.0
        for (k, rr), Tb in zip(oracle["items"], oracle["Tb"]):
            Tg = np.stack([T[[s_ - P for s_ in steps], off[k] + i] for i in rr])
            num += float(np.sum((Tg - Tb) ** 2))
            den += float(np.sum(Tb ** 2))
        rel_err = float(np.sqrt(num / den))
        units = len(oracle["items"]) * len(steps)
        cpu = {
            "value": units / (Ntot * oracle["wall"]),
            "unit": "steps/s",
            "cores": oracle["workers"],
            "kind": "oracle",
            "sample": (f"FDP=H-approximated operator of faults {sorted({k for k, _ in oracle['items']})} applied by "
                       f"the oracle (FP64, one process per core) to 2 seeded receivers each at steps {steps}; "
                       f"{oracle['wall']:.1f} s wall on {oracle['workers']} cores for {units} receiver-steps, "
                       f"extrapolated to {Ntot} receivers per batched step"),
        }
        print(f"[bench] GPU vs oracle rel err {rel_err:.2e}", file=sys.stderr, flush=True)

    line = {
        "metric": "time steps/sec and HBM GB/s of per-step H-matvec vs dense FP64, at rel err <=1e-4",
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * elapsed / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"batched FDP=H ({PREC_NAMES[prec_name]}), 64 independent planar anti-plane faults, N "
                         f"log-uniform in [1024, 16384] (seed 5, sum {Ntot}), M = 2N, eta=2, leaf 32, "
                         f"eps_aca={eps_aca:g}, n_c=20, eps_q=1e-3, eps_st=1e-6, "
                         f"{'staircase transient (eps 0.1), ' if args.quantize_tr else ''}"
                         f"one operator and one set of launches per step; "
                         f"{P} quiescent steps, then smoothed random slip rate (20 el, 40 steps, seed 5000+k)"),
            "N_total": Ntot,
            "faults": 64,
            "active_faults_at_timed_steps": active,
            "near_window_lags_applied_share": lag_share,
            "timed_steps_at": [P + W, P + S - 1],
        },
        "fault_steps_per_s": active * steps_per_s,
        "element_steps_per_s": float(np.sum(sizes[lags > P + W])) * steps_per_s,
        "hbm_gbps_algorithmic": (st["bytes_per_step"] - st["near_bytes_per_step"] + near_bytes) * steps_per_s / 1e9,
        "rel_err_vs_oracle": rel_err,
        "fp64_batched": fp64,
        "speedup_vs_fp64_batched": (steps_per_s / fp64["steps_per_s"]) if fp64 and "steps_per_s" in fp64 else None,
        "dense_fp64": {"skipped": "64 dense kernel tensors would need "
                       f"{float(np.sum(lags * sizes.astype(float) ** 2)) * 8 / 1e12:.0f} TB"},
        "roofline": {
            "bound": "hbm",
            "kernel": f"{kname}<{'double' if prec_name == 'fp64' else 'float'}> (near-field window convolution"
                      f"{f', {spp} steps per pass' if spp > 1 else ''})",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": None,
            "algorithmic_bytes_per_launch": near_bytes,
            "avg_launch_ms": 1e3 * near_avg_s,
        },
        "cpu_baseline": cpu,
        "operator": {k: st[k] for k in ("n_adm", "n_inadm", "near_pairs", "near_lags", "rank_sum", "rank_max",
                                        "aca_fallbacks", "aca_host_blocks", "aca_seconds", "device_bytes",
                                        "bytes_per_step", "flops_per_step")},
        "near_autotune": tune,
        "setup_s": setup_s,
        "setup": setup,
    }
    print(json.dumps(line))


def run_rupture(args):
    """Dynamic rupture on the planar fault N = 4096, M = 2048 with the FDP=H operator: every step
    is a coupled step (prediction from the history, the friction solve per element, commit).
    Friction and initial stress after the paper's planar rupture problem (Sec. 6.2): exponential
    slip weakening with T_th = 1e-2, T_bg = 0.35 T_th, T_dy = 0, D_c = 0.1 dx/2; a nucleation patch
    of 50 elements at the centre loaded 1% above T_th (the single-asperity model of App. A.2.3 in
    place of the paper's elliptic dislocation).  The first M - K - W coupled steps run untimed, so
    the timed steps have (nearly) full history."""
    import numpy as np
    import torch

    from paper_1903_02118_amd.binding import (BIE_EXPORT_NEAR, BIE_FP64, BIE_LAW_EXP_WEAKENING, BIE_MIXED_FP32,
                                              Operator, make_friction, make_params)
    from synth import straight_fault

    N, M, K, W = args.n or N_DEF, args.m or M_DEF, args.steps, args.warmup
    prec_name = args.precision or "fp64"
    P = M - K - W
    if P < 0:
        sys.exit(f"--steps + --warmup must not exceed M={M}")
    t_th, t_bg, t_dy, d_c, half = 1e-2, 0.35e-2, 0.0, 0.05, 25.0
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    xa, xb = straight_fault(N)
    x = 0.5 * (xa[:, 0] + xb[:, 0])
    T0 = np.where(np.abs(x - N / 2) < half, 1.01 * t_th, t_bg)
    prec = BIE_FP64 if prec_name == "fp64" else BIE_MIXED_FP32
    params = make_params(eta=2.0, leaf_size=32, n_c=20, eps_aca=args.eps_aca or 1e-6, eps_q=1e-3, eps_st=1e-6,
                         seed=12345, precision=prec)
    op, setup = build_fdph_timed([(xa, xb, M)], params, stream, torch)
    setup_s = setup["total_s"]
    st = op.stats()
    tune = None
    if not args.no_autotune:
        tune = op.autotune(reps=3, stream=stream)
    fr = make_friction(BIE_LAW_EXP_WEAKENING, t_th, t_dy, d_c)
    t0d = torch.from_numpy(T0).to(dev)
    slip = torch.zeros(N, dtype=torch.float64, device=dev)
    state = torch.zeros(N, dtype=torch.int32, device=dev)
    D = torch.zeros((M, N), dtype=torch.float64, device=dev)
    T = torch.zeros_like(D)
    op.reset(stream=stream)
    op.rupture_run(fr, t0d, slip, state, D[:P + W], T[:P + W], stream=stream)
    torch.cuda.synchronize()
    op.timing(True)
    t0 = time.perf_counter()
    op.rupture_run(fr, t0d, slip, state, D[P + W:], T[P + W:], stream=stream)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    near_ms, near_n = op.timing_read()
    op.timing(False)
    kb = 8.0 if prec_name == "fp64" else 4.0
    near_bytes = kb * near_lags_mean(op.export(BIE_EXPORT_NEAR)[:, 2], P + W, M - 1)
    op.close()
    near_avg_s = near_ms / 1e3 / max(near_n, 1)
    achieved = near_bytes / near_avg_s / 1e9
    sps = K / el
    rup = int(state.sum().item())
    Dh = D.cpu().numpy()
    front = np.nonzero(Dh[M - 1] > 0)[0]
    print(f"[bench] rupture N={N} M={M}: {sps:.1f} coupled steps/s ({1e3 * el / K:.3f} ms/step), near kernel "
          f"{1e3 * near_avg_s:.3f} ms -> {achieved:.0f} GB/s; ruptured {rup} of {N}", file=sys.stderr, flush=True)
    line = {
        "metric": "coupled (dynamic rupture) time steps/sec of the FDP=H operator",
        "value": sps,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * el / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_name == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"dynamic rupture, FDP=H {'FP64' if prec_name == 'fp64' else 'mixed'}, planar fault "
                               f"N={N}, M={M}, eta=2, leaf 32, exponential slip weakening (T_th=1e-2, T_bg=0.35 T_th, "
                               f"T_dy=0, D_c=0.05), 50-element nucleation patch at 1.01 T_th",
                   "N": N, "M": M, "untimed_coupled_steps": P + W, "timed_steps_at": [P + W, M - 1]},
        "rupture": {"ruptured_elements": rup,
                    "slipping_span_at_last_step": [int(front.min()), int(front.max())] if len(front) else None,
                    "max_slip_rate": float(Dh.max())},
        "roofline": {"bound": "hbm",
                     "kernel": f"k_near<{'double' if prec_name == 'fp64' else 'float'}> (near-field window convolution)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": None, "algorithmic_bytes_per_launch": near_bytes, "avg_launch_ms": 1e3 * near_avg_s},
        "cpu_baseline": None,
        "near_autotune": tune,
        "setup_s": setup_s,
        "setup": setup,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
