"""The C ABI from a plain C program (tests/c_abi/example.c, built with gcc
against libbie.so and the HIP runtime): its tractions, those of an operator
carrying two slip-rate histories, and its rupture slip rates match the
oracle."""
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


def _run_c(tmp_path, N, M, mode):
    exe = _build(tmp_path)
    print(f"running the C example ({mode})", flush=True)
    r = subprocess.run([exe, str(N), str(M), mode], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return np.array([float(v) for v in r.stdout.split()])


def test_c_program_two_scenarios_match_oracle(gpu_lib, tmp_path):
    N, M = 160, 120
    vals = _run_c(tmp_path, N, M, "scenarios")
    assert vals.size == 2 * M * N
    T = vals.reshape(M, 2, N)
    j = np.arange(N)[None, :]
    n = np.arange(M)[:, None]
    Ds = [np.sin(0.37 * j + 0.11 * n) + 0.5 * np.cos(0.05 * j * n), np.cos(0.21 * j - 0.07 * n)]
    xa, xb = straight_fault(N)
    rows = FdphOracle(Problem(xa, xb, dt=0.5), M, FdphParams()).rows(np.arange(N))
    for r in range(2):
        Tb = convolve_rows(rows, Ds[r]).T
        assert np.linalg.norm(T[:, r] - Tb) / np.linalg.norm(Tb) <= 1e-6, r


def test_c_program_rupture_matches_oracle(gpu_lib, tmp_path):
    import oracle.rupture as rp

    N, M = 96, 120
    vals = _run_c(tmp_path, N, M, "rupture")
    assert vals.size == M * N
    D = vals.reshape(M, N)
    xa, xb = straight_fault(N)
    K = Problem(xa, xb, dt=0.5).kernel_tensor(M)
    t0 = np.where((np.arange(N) >= N // 2 - 10) & (np.arange(N) < N // 2 + 10), 1.01e-2, 0.35e-2)
    Do, _, _, ro = rp.simulate(np.transpose(K, (1, 2, 0)), t0, rp.Friction("exp", 1e-2, 0.0, 0.05, 0.5), M)
    assert ro.sum() > 20
    assert np.linalg.norm(D - Do) / np.linalg.norm(Do) <= 1e-10


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
