"""The C-ABI library loads and exports every entry point of include/bie.h and
include/bie_diag.h, and its host-side checks and plans run without a GPU."""
import ctypes
import os
import re

import pytest

from paper_1903_02118_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("bie.h", "bie_diag.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(bie_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = binding.load()
    names = _declared()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(binding.EXPORTED) == set(names)


def test_struct_layouts_match_header_sizes():
    # 2 int32 + 2 pointers + 4 doubles + 2 int32 + 1 double
    assert ctypes.sizeof(binding.bie_problem) == 8 + 16 + 32 + 8 + 8
    assert ctypes.sizeof(binding.bie_fdph_params) == 8 + 8 + 24 + 8 + 8 + 8 + 8
    assert ctypes.sizeof(binding.bie_stats) == 16 + 8 * 5 + 8 * 6 + 8 * 2 + 8 * 4 + 8 * 5
    assert ctypes.sizeof(binding.bie_tune) == 24 + 16


def _plan_dense(lib, xa, xb, M, **phys):
    p, keep = binding.make_problem(xa, xb, M, **phys)
    h = ctypes.c_void_p()
    rc = lib.bie_plan_dense(ctypes.byref(p), ctypes.byref(h))
    return rc, h


def _plan_fdph(lib, probs, q):
    arr = (binding.bie_problem * max(len(probs), 1))(*probs)
    h = ctypes.c_void_p()
    rc = lib.bie_plan_fdph(arr, len(probs), ctypes.byref(q), ctypes.byref(h))
    return rc, h


def test_invalid_arguments_are_rejected_without_a_gpu():
    lib = binding.load()
    h = ctypes.c_void_p()
    # null problem: rejected before any device call
    assert lib.bie_plan_dense(None, ctypes.byref(h)) == binding.BIE_EINVAL
    assert b"invalid problem" in lib.bie_last_error()
    assert lib.bie_step(None, None, None, None) == binding.BIE_EINVAL
    assert lib.bie_run(None, None, None, 1, None) == binding.BIE_EINVAL
    assert lib.bie_build_kernel(None, None, 0, None, ctypes.byref(h)) == binding.BIE_EINVAL
    assert lib.bie_set_debug(None, 1, None) == binding.BIE_EINVAL
    rc, _ = _plan_dense(lib, [[0.0, 0.0]], [[0.0, 0.0]], 4)  # zero-length element
    assert rc == binding.BIE_EINVAL
    p, keep = binding.make_problem([[0.0, 0.0]], [[1.0, 0.0]], 4, eps_t=0.5)
    rc, _ = _plan_fdph(lib, [p], binding.make_params())
    assert rc == binding.BIE_EINVAL
    assert b"eps_t" in lib.bie_last_error()


def test_workspace_is_checked_before_any_device_call():
    """A plain plan is host-only; the build refuses a null, misaligned or short
    workspace (BIE_EWORKSPACE) and an FDP=H plan before its window scan
    (BIE_ESTATE), all before touching the device."""
    from synth import straight_fault

    lib = binding.load()
    xa, xb = straight_fault(16)
    rc, pl = _plan_dense(lib, xa, xb, 8)
    assert rc == binding.BIE_OK
    need = ctypes.c_int64()
    assert lib.bie_workspace_size(pl, ctypes.byref(need)) == binding.BIE_OK
    st = binding.bie_stats()
    assert lib.bie_plan_query(pl, ctypes.byref(st)) == binding.BIE_OK
    assert st.kind == binding.BIE_KIND_DENSE and st.device_bytes == need.value
    # the causal band of K is part of it (16 x 16 x 8 doubles at most)
    E = st.flops_per_step / 2
    assert E * 8 <= need.value and E <= 16 * 16 * 8
    op = ctypes.c_void_p()
    assert lib.bie_build_kernel(pl, None, need.value, None, ctypes.byref(op)) == binding.BIE_EWORKSPACE
    assert lib.bie_build_kernel(pl, ctypes.c_void_p(4096 + 8), need.value, None, ctypes.byref(op)) == binding.BIE_EWORKSPACE
    assert lib.bie_build_kernel(pl, ctypes.c_void_p(4096), need.value - 1, None, ctypes.byref(op)) == binding.BIE_EWORKSPACE
    assert b"needs" in lib.bie_last_error()
    assert lib.bie_compress_fdph(pl, ctypes.c_void_p(4096), need.value, None, ctypes.byref(op)) == binding.BIE_EINVAL
    assert not op.value
    lib.bie_plan_free(pl)
    p, keep = binding.make_problem(*straight_fault(256), 64)
    rc, pf = _plan_fdph(lib, [p], binding.make_params())
    assert rc == binding.BIE_OK
    assert lib.bie_workspace_size(pf, ctypes.byref(need)) == binding.BIE_ESTATE
    assert lib.bie_compress_fdph(pf, ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(op)) == binding.BIE_ESTATE
    scratch = ctypes.c_int64()
    assert lib.bie_plan_scratch_size(pf, ctypes.byref(scratch)) == binding.BIE_OK and scratch.value > 0
    assert lib.bie_plan_windows(pf, None, scratch.value, None) == binding.BIE_EWORKSPACE
    lib.bie_plan_free(pf)


def test_batched_arguments_are_checked_without_a_gpu():
    lib = binding.load()
    q = binding.make_params()
    p1, k1 = binding.make_problem([[0.0, 0.0]], [[1.0, 0.0]], 4)
    p2, k2 = binding.make_problem([[0.0, 0.0]], [[1.0, 0.0]], 4, mu=2.0)
    rc, _ = _plan_fdph(lib, [], q)
    assert rc == binding.BIE_EINVAL
    rc, _ = _plan_fdph(lib, [p1, p2], q)
    assert rc == binding.BIE_EINVAL
    assert b"share mu" in lib.bie_last_error()
    q.precision = 7
    rc, _ = _plan_fdph(lib, [p1], q)
    assert rc == binding.BIE_EINVAL
    assert b"precision" in lib.bie_last_error()


def test_aca_stall_sweeps_the_residual():
    """A block whose only nonzero entry the random references miss: ACA+
    sweeps the true residual instead of stopping at rank 0, and recovers the
    exact rank-1 block (a zero block stays at rank 0)."""
    import numpy as np

    A = np.zeros((300, 200))
    A[137, 71] = 2.5  # off every random reference row and column but 1 in 300 and 1 in 200
    swept = 0
    for seed in range(1, 6):
        rank, fb, sweeps, err = binding.diag_aca(A, 1e-8, seed)
        assert rank == 1 and not fb and err < 1e-14
        swept += sweeps > 0
    assert swept >= 4
    assert binding.diag_aca(np.zeros((40, 30)), 1e-8, 1)[0] == 0
    assert binding.diag_aca(np.zeros((40, 30)), 1e-8, 1)[3] == 0.0


def test_aca_meets_its_tolerance_on_smooth_kernels():
    """ACA+ of 1/r between two separated point clouds (an elastostatic-like
    kernel): the exact relative Frobenius error stays below eps_aca."""
    import numpy as np

    rng = np.random.default_rng(3)
    x = rng.random((120, 2))
    y = rng.random((90, 2)) + np.array([3.0, 0.5])
    A = 1.0 / np.linalg.norm(x[:, None, :] - y[None, :, :], axis=2)
    for eps in (1e-4, 1e-8):
        rank, fb, sweeps, err = binding.diag_aca(A, eps, 7)
        assert not fb and rank < 30 and err <= eps


def test_aca_full_rank_is_refused_when_the_fallback_is_disabled():
    """Blocks that cannot reach eps_aca before their full rank are kept exactly
    (Sec. 6.2) unless BIE_FLAG_NO_ACA_FALLBACK asks for BIE_ENOTCONV."""
    from synth import straight_fault

    lib = binding.load()
    p, keep = binding.make_problem(*straight_fault(128), 64)
    q = binding.make_params(leaf_size=8, eps_aca=1e-17, host_aca=True)
    rc, pl = _plan_fdph(lib, [p], q)
    assert rc == binding.BIE_OK
    lib.bie_plan_free(pl)
    q.flags |= binding.BIE_FLAG_NO_ACA_FALLBACK
    rc, pl = _plan_fdph(lib, [p], q)
    assert rc == binding.BIE_ENOTCONV
    assert b"fallback" in lib.bie_last_error()


@pytest.mark.parametrize("geom", ["planar", "curved"])
def test_plan_blocks_meet_eps_aca(geom):
    """Exact errors of every low-rank block of a plan (host ACA+, evaluated
    entry by entry on the host): below eps_aca in FP64, and with the BF16 storage of
    the factors (leading cross terms as hi + lo pairs) below 2.5e-4; the 2D
    transient blocks stay low-rank on the curved fault."""
    from synth import curved_fault, straight_fault

    xa, xb = straight_fault(1024) if geom == "planar" else curved_fault(1024)
    for prec in (binding.BIE_FP64, binding.BIE_MIXED_BF16):
        pl = binding.Plan.fdph([(xa, xb, 1024)], binding.make_params(eps_aca=1e-4, precision=prec, host_aca=True))
        E = pl.block_errors()
        pl.close()
        assert len(E) > 100
        assert E[:, 6].max() <= 1e-4
        if prec == binding.BIE_MIXED_BF16:
            assert E[:, 7].max() <= 2.5e-4
        else:
            assert E[E[:, 1] == 2, 5].max() <= 16


def test_autotune_rejects_bad_arguments_without_a_gpu():
    lib = binding.load()
    t = binding.bie_tune()
    assert lib.bie_autotune(None, 3, ctypes.byref(t), None) == binding.BIE_EINVAL
    assert b"FDP=H" in lib.bie_last_error()


def test_inplane_mode_arguments_are_checked_without_a_gpu():
    from synth import curved_fault, straight_fault

    lib = binding.load()
    xa, xb = straight_fault(8)
    rc, _ = _plan_dense(lib, xa, xb, 4, mode=binding.BIE_MODE_INPLANE, alpha=0.5)
    assert rc == binding.BIE_EINVAL
    assert b"alpha > beta" in lib.bie_last_error()
    xa, xb = curved_fault(16)
    rc, _ = _plan_dense(lib, xa, xb, 4, mode=binding.BIE_MODE_INPLANE, alpha=3 ** 0.5)
    assert rc == binding.BIE_EINVAL
    assert b"straight fault" in lib.bie_last_error()
    xa, xb = straight_fault(8)
    p, keep = binding.make_problem(xa, xb, 4, mode=binding.BIE_MODE_INPLANE, alpha=3 ** 0.5)
    rc, _ = _plan_fdph(lib, [p], binding.make_params())
    assert rc == binding.BIE_EINVAL
    assert b"anti-plane problem only" in lib.bie_last_error()


def test_coupled_step_entry_points_reject_bad_arguments_without_a_gpu():
    lib = binding.load()
    assert ctypes.sizeof(binding.bie_friction) == 8 + 24
    assert lib.bie_step_predict(None, None, None) == binding.BIE_EINVAL
    assert lib.bie_step_commit(None, None, None) == binding.BIE_EINVAL
    assert lib.bie_first_lag(None, None, None) == binding.BIE_EINVAL
    fr = binding.make_friction(binding.BIE_LAW_EXP_WEAKENING, 1.0, 0.2, 0.1)
    assert lib.bie_rupture_run(None, ctypes.byref(fr), None, None, None, None, None, 1, None) == binding.BIE_EINVAL
    assert b"bie_rupture_run" in lib.bie_last_error()


def test_hbm_probe_rejects_bad_arguments_without_a_gpu():
    lib = binding.load()
    ms = ctypes.c_double()
    assert lib.bie_hbm_read_probe(None, 16, ctypes.byref(ms), None) == binding.BIE_EINVAL
    assert lib.bie_hbm_read_probe(ctypes.c_void_p(16), 15, ctypes.byref(ms), None) == binding.BIE_EINVAL


def test_state_entry_points_reject_bad_arguments_without_a_gpu():
    lib = binding.load()
    n = ctypes.c_int64()
    assert lib.bie_state_bytes(None, ctypes.byref(n)) == binding.BIE_EINVAL
    assert lib.bie_save_state(None, ctypes.c_void_p(256), 1 << 20, None) == binding.BIE_EINVAL
    assert lib.bie_load_state(None, None, 1 << 20, None) == binding.BIE_EINVAL
    assert b"bie_load_state" in lib.bie_last_error()


def test_causality_violation_is_reported_without_a_gpu():
    """The FDP=H plan checks discretized causality (min dm_i + mbar_j >= 1
    in every admissible leaf, App. D.1) on the host before it touches the
    device: a step that carries the wave past a whole admissible gap (beta dt
    = 100 dx on a 256-element line; the oracle flags the same case) is
    refused with BIE_ECAUSALITY."""
    from synth import straight_fault

    lib = binding.load()
    xa, xb = straight_fault(256)
    p, keep = binding.make_problem(xa, xb, 16, dt=100.0)
    rc, pl = _plan_fdph(lib, [p], binding.make_params())
    assert rc == binding.BIE_ECAUSALITY
    assert b"causality" in lib.bie_last_error()
    assert not pl.value


class _FakeDeviceTensor:
    """Stands in for a device tensor on a machine without one (never dereferenced)."""

    def __init__(self, n=8, dtype="torch.float64", contiguous=True):
        self.is_cuda = True
        self.dtype = dtype
        self._n, self._c = n, contiguous

    def is_contiguous(self):
        return self._c

    def numel(self):
        return self._n

    def data_ptr(self):
        return 4096


def test_binding_refuses_tensors_the_kernels_cannot_read_without_a_gpu():
    import torch

    binding.load()

    good = _FakeDeviceTensor(8)
    assert binding._ptr(good, "D", 8).value == 4096
    assert binding._ptr(_FakeDeviceTensor(8, "torch.uint8"), "buf", dtype=None).value == 4096
    assert binding._ptr(_FakeDeviceTensor(8, "torch.int32"), "state", 8, "int32").value == 4096
    assert binding._ptr(12288).value == 12288  # a raw device address is taken as is
    bad = [
        (torch.zeros(8, dtype=torch.float64), 8, "float64"),          # host memory
        (_FakeDeviceTensor(8, contiguous=False), 8, "float64"),       # strided
        (_FakeDeviceTensor(8, "torch.float32"), 8, "float64"),        # element type
        (_FakeDeviceTensor(7), 8, "float64"),                         # too short
        (_FakeDeviceTensor(8, "torch.float64"), 8, "int32"),          # state flags are int32
    ]
    for x, n, dt in bad:
        with pytest.raises(ValueError):
            binding._ptr(x, "x", n, dt)
    # an operator method checks before it calls the library
    op = binding.Operator.__new__(binding.Operator)
    op.h, op.row = None, 4
    with pytest.raises(ValueError):
        op.run(torch.zeros((3, 4), dtype=torch.float64), torch.zeros((3, 4), dtype=torch.float64))
    with pytest.raises(ValueError):
        op.step(_FakeDeviceTensor(3), _FakeDeviceTensor(4))


@pytest.mark.parametrize("geom", ["planar", "curved"])
def test_dense_plan_band_holds_every_nonzero_of_the_kernel(geom):
    """The plain form stores, per lag and receiver, the hull of the sources the
    wave has reached (plus one lag against rounding): its entry count is at
    least the number of nonzero entries of the oracle's exact tensor and at
    most that plus the hull's inner zeros, and far below N^2 M at small lags."""
    import numpy as np

    from oracle.kernel2d import Problem
    from synth import curved_fault, straight_fault

    N, M = 64, 40
    xa, xb = straight_fault(N) if geom == "planar" else curved_fault(N)
    pl = binding.Plan.dense(xa, xb, M, dt=0.5)
    E = pl.stats()["flops_per_step"] / 2
    pl.close()
    K = Problem(xa, xb, dt=0.5).kernel_tensor(M)
    nnz = int(np.count_nonzero(K))
    hull = 0
    for m in range(M):
        for i in range(N):
            nz = np.nonzero(np.abs(K[: m + 2 if m + 2 <= M else M, i, :]).max(axis=0))[0]
            if len(nz):
                hull += nz.max() - nz.min() + 1
    assert nnz <= E <= hull + 2 * N * M
    assert E < 0.6 * N * N * M



def test_library_and_torch_share_one_hip_runtime():
    """torch ships its own HIP runtime: the binding loads torch before the
    library, so that a process that loads the library first still maps one
    runtime (two would leave the library's kernels without torch's memory)."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("from paper_1903_02118_amd import binding; binding.load(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=600)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_library_sources_allocate_no_device_memory():
    """Every device array lives in caller memory or in a static device array:
    no allocating HIP call appears in the library's sources."""
    import os
    import re

    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1903_02118_amd", "csrc")
    pat = re.compile(r"\bhip(Malloc|MallocAsync|MallocManaged|ExtMallocWithFlags|MallocPitch|Free|FreeAsync)\b")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name)) as f:
            code = "\n".join(line.split("//")[0] for line in f)
        assert not pat.search(code), name


def test_time_block_arguments_are_checked_without_a_gpu():
    from synth import straight_fault

    lib = binding.load()
    p, keep = binding.make_problem(*straight_fault(64), 32)
    q = binding.make_params(time_block=3)
    rc, _ = _plan_fdph(lib, [p], q)
    assert rc == binding.BIE_EINVAL and b"time_block" in lib.bie_last_error()
    q = binding.make_params(n_rhs=2, time_block=binding.BIE_TIME_BLOCK)
    rc, _ = _plan_fdph(lib, [p], q)
    assert rc == binding.BIE_EINVAL and b"one scenario" in lib.bie_last_error()
    for tb in (0, 1, binding.BIE_TIME_BLOCK):
        rc, pl = _plan_fdph(lib, [p], binding.make_params(time_block=tb))
        assert rc == binding.BIE_OK
        lib.bie_plan_free(pl)
