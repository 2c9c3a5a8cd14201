"""Writes the stored expected values of the full-size GPU parity tests.

Test infrastructure: calls only the CPU oracle (`oracle/`, FP64) and the
seeded input generators (`synth/`).  For each case it applies the
FDP=H-approximated operator (Tier-B: the dense assembly of the kernel the
method approximates, Secs. 3-5, Apps. B.1, B.3, C.2, E, H) to seeded
receivers at sampled steps and stores the tractions as JSON next to this
file, so that the GPU tests compare element by element without recomputing
the oracle on the GPU host.

Cases (inputs fully determined by the seeds below):
  planar4k    straight fault, N = 4096, M = 2048, eta = 2, leaf 32, n_c = 20,
              eps_Q = 1e-3, eps_st = 1e-6; slip rate a smoothed random field
              (20 elements, 40 steps, seed 2); 64 receivers (PCG64 seed 102);
              every 16th step.
  curved16k   sinusoidal trace (amplitude 0.05 L, wavelength L/4), N = 16384,
              M = 8192, same parameters with the staircase transient
              (eps 0.1); slip rate seed 3; 64 receivers (seed 103); 5 steps.
  ensemble64  64 straight faults, N_k log-uniform in [1024, 16384] (seed 5),
              M_k = 2 N_k, staircase transient; per fault a smoothed field
              (seed 5000 + k) over the first 1024 steps and 16 receivers
              (seed 500 + k); 4 steps.

usage: python tests/golden/make_golden.py [case ...] [--jobs J]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

CASES = {
    "planar4k": dict(geom="straight", N=4096, M=2048, seed=2, rec_seed=102, n_rec=64, quantize_tr=False,
                     steps=list(range(15, 2048, 16))),
    "curved16k": dict(geom="curved", N=16384, M=8192, seed=3, rec_seed=103, n_rec=64, quantize_tr=True,
                      steps=[1023, 2047, 4095, 6143, 8191]),
    "ensemble64": dict(count=64, n_lo=1024, n_hi=16384, size_seed=5, S=1024, n_rec=16, quantize_tr=True,
                       steps=[255, 511, 767, 1023]),
}
PARAMS = dict(eta=2.0, leaf_size=32, eps_q=1e-3, eps_st=1e-6, n_c=20, eps_q_tr=0.1)


def receivers(n, count, seed):
    """Sorted seeded sample of `count` distinct receivers among n."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n, size=count, replace=False))


def _fault(geom, n):
    from synth import curved_fault, straight_fault

    return curved_fault(n) if geom == "curved" else straight_fault(n)


def _oracle(xa, xb, M, quantize_tr):
    from oracle.fdph import FdphOracle, FdphParams
    from oracle.kernel2d import Problem

    return FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams(quantize_tr=quantize_tr, **PARAMS))


def _planar_chunk(args):
    """Tier-B rows of a few receivers, convolved over every step, sampled."""
    from oracle.dense import convolve_rows_fft
    from synth import smooth_slip_rate

    c, rec = args
    xa, xb = _fault(c["geom"], c["N"])
    D = smooth_slip_rate(c["N"], c["M"], 20.0, 40.0, c["seed"])
    o = _oracle(xa, xb, c["M"], c["quantize_tr"])
    T = convolve_rows_fft(o.rows(rec), D)
    return T[:, c["steps"]]


def _apply_chunk(args):
    """Tier-B of a few receivers at the sampled steps (leaf by leaf)."""
    from synth import smooth_slip_rate

    c, rec = args
    xa, xb = _fault(c["geom"], c["N"])
    D = smooth_slip_rate(c["N"], c["M"], 20.0, 40.0, c["seed"])
    o = _oracle(xa, xb, c["M"], c["quantize_tr"])
    return np.stack([o.apply_at(int(i), D, c["steps"]) for i in rec])


def _ensemble_fault(args):
    from synth import ensemble_sizes, smooth_slip_rate, straight_fault

    c, k = args
    sizes = ensemble_sizes(c["count"], c["n_lo"], c["n_hi"], c["size_seed"])
    n = int(sizes[k])
    xa, xb = straight_fault(n)
    D = smooth_slip_rate(n, c["S"], 20.0, 40.0, 5000 + k)
    o = _oracle(xa, xb, 2 * n, c["quantize_tr"])
    rec = receivers(n, c["n_rec"], 500 + k)
    return k, rec, np.stack([o.apply_at(int(i), D, c["steps"]) for i in rec])


def make(case, jobs):
    c = CASES[case]
    t0 = time.time()
    out = {"case": case, "generator": "tests/golden/make_golden.py", "params": PARAMS, "dt": 0.5, "mu": 1.0,
           "beta": 1.0, "steps": c["steps"]}
    out.update({k: v for k, v in c.items() if k != "steps"})
    with ProcessPoolExecutor(max_workers=jobs) as ex:
        if case == "ensemble64":
            faults = []
            for k, rec, T in ex.map(_ensemble_fault, [(c, k) for k in range(c["count"])]):
                faults.append({"fault": k, "receivers": rec.tolist(), "T": T.tolist()})
                print(f"[golden] {case} fault {k} done ({time.time() - t0:.0f}s)", flush=True)
            out["faults"] = sorted(faults, key=lambda f: f["fault"])
        else:
            rec = receivers(c["N"], c["n_rec"], c["rec_seed"])
            per = 4 if case == "planar4k" else 2
            parts = [rec[b:b + per] for b in range(0, len(rec), per)]
            fn = _planar_chunk if case == "planar4k" else _apply_chunk
            Ts = []
            for k, T in enumerate(ex.map(fn, [(c, p) for p in parts])):
                Ts.append(T)
                print(f"[golden] {case} part {k + 1}/{len(parts)} ({time.time() - t0:.0f}s)", flush=True)
            out["receivers"] = rec.tolist()
            out["T"] = np.concatenate(Ts).tolist()  # [receiver][sampled step]
    path = os.path.join(HERE, f"tierb_{case}.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print(f"[golden] wrote {path} in {time.time() - t0:.0f}s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*", default=list(CASES))
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    a = ap.parse_args()
    for case in a.cases:
        make(case, a.jobs)


if __name__ == "__main__":
    main()
