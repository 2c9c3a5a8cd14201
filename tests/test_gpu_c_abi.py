"""The C ABI from a plain C program (tests/c_abi/example.c, built with gcc
against libbie.so and the HIP runtime): its tractions match the oracle."""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle.dense import convolve_dense, convolve_rows
from oracle.fdph import FdphOracle, FdphParams
from oracle.kernel2d import Problem
from synth import straight_fault

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _build(tmp_path):
    exe = str(tmp_path / "example")
    lib = os.path.join(ROOT, "paper_1903_02118_amd")
    cmd = ["gcc", "-O2", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "c_abi", "example.c"), "-o", exe, "-L" + lib, "-lbie",
           "-L/opt/rocm/lib", "-lamdhip64", "-lm", "-Wl,-rpath," + lib + ":/opt/rocm/lib"]
    subprocess.run(cmd, check=True, capture_output=True)
    return exe


def test_c_program_matches_oracle(gpu_lib, tmp_path):
    N, M = 200, 150
    exe = _build(tmp_path)
    print("running the C example", flush=True)
    r = subprocess.run([exe, str(N), str(M)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    vals = np.array([float(v) for v in r.stdout.split()])
    assert vals.size == 2 * M * N
    Td, Tf = vals[: M * N].reshape(M, N), vals[M * N:].reshape(M, N)
    j = np.arange(N)[None, :]
    n = np.arange(M)[:, None]
    D = np.sin(0.37 * j + 0.11 * n) + 0.5 * np.cos(0.05 * j * n)
    xa, xb = straight_fault(N)
    pr = Problem(xa, xb, dt=0.5)
    Ta = convolve_dense(pr.kernel_tensor(M), D)
    assert np.linalg.norm(Td - Ta) / np.linalg.norm(Ta) <= 1e-12
    o = FdphOracle(pr, M, FdphParams())
    Tb = convolve_rows(o.rows(np.arange(N)), D).T
    assert np.linalg.norm(Tf - Tb) / np.linalg.norm(Tb) <= 1e-6
    assert math.isfinite(float(np.abs(Tf).max()))


def test_hbm_read_probe_runs(gpu_lib):
    """The streaming-read probe of the bench: a positive time, a rate below
    the HBM peak of 8 TB/s for a buffer far larger than the caches."""
    import torch

    from paper_1903_02118_amd.binding import hbm_read_probe

    buf = torch.ones((1 << 30) // 8, dtype=torch.float64, device="cuda")  # 1 GiB
    ms = min(hbm_read_probe(buf) for _ in range(3))
    rate = buf.numel() * 8 / (ms / 1e3) / 1e9
    print("probe GB/s", rate, flush=True)
    assert ms > 0 and rate < 8000.0
