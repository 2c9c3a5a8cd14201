"""Thin ctypes binding of libbie.so (argument marshalling only).

Every name mirrors a C entry point of include/bie.h.  Device buffers are
passed as raw pointers (e.g. torch.Tensor.data_ptr() of a CUDA/HIP tensor)
and streams as raw hipStream_t handles (torch.cuda.current_stream().cuda_stream).
No computation happens here; if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbie.so")

BIE_OK = 0
BIE_EINVAL = -1
BIE_ECAUSALITY = -2
BIE_ENOMEM = -3
BIE_EHIP = -4
BIE_ESTATE = -5
BIE_EWORKSPACE = -6
BIE_ENOTCONV = -7
BIE_KIND_DENSE = 1
BIE_KIND_FDPH = 2
BIE_FP64 = 0
BIE_MIXED_FP32 = 1
BIE_MIXED_BF16 = 2
BIE_MODE_ANTIPLANE = 0
BIE_MODE_INPLANE = 1
BIE_EXPORT_NEAR = 1
BIE_EXPORT_LEAVES = 2
BIE_EXPORT_ART = 3
BIE_EXPORT_TRANS = 4
BIE_FLAG_QUANTIZE_TRANSIENT = 1
BIE_FLAG_NO_ACA_FALLBACK = 2
BIE_FLAG_HOST_ACA = 4
BIE_TIME_BLOCK = 16
BIE_DEBUG_SCAN_FINITE = 1
BIE_LAW_STATIC_DYNAMIC = 0
BIE_LAW_EXP_WEAKENING = 1

EXPORTED = [
    "bie_plan_dense",
    "bie_plan_fdph",
    "bie_plan_scratch_size",
    "bie_plan_windows",
    "bie_workspace_size",
    "bie_plan_query",
    "bie_plan_free",
    "bie_build_kernel",
    "bie_compress_fdph",
    "bie_step",
    "bie_run",
    "bie_run_graph",
    "bie_run_static",
    "bie_advance",
    "bie_autotune",
    "bie_reset",
    "bie_query",
    "bie_state_bytes",
    "bie_save_state",
    "bie_load_state",
    "bie_step_predict",
    "bie_step_commit",
    "bie_first_lag",
    "bie_rupture_run",
    "bie_destroy",
    "bie_last_error",
    # diagnostics (include/bie_diag.h)
    "bie_timing",
    "bie_timing_read",
    "bie_hbm_read_probe",
    "bie_fdph_export",
    "bie_set_debug",
    "bie_debug_status",
    "bie_diag_aca",
    "bie_plan_block_errors",
    "bie_plan_dense_lag_entries",
]


class bie_problem(ctypes.Structure):
    _fields_ = [
        ("n_elem", ctypes.c_int32),
        ("n_lags", ctypes.c_int32),
        ("xa_host", ctypes.POINTER(ctypes.c_double)),
        ("xb_host", ctypes.POINTER(ctypes.c_double)),
        ("mu", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("eps_t", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("alpha", ctypes.c_double),
    ]


class bie_fdph_params(ctypes.Structure):
    _fields_ = [
        ("eta", ctypes.c_double),
        ("leaf_size", ctypes.c_int32),
        ("n_c", ctypes.c_int32),
        ("eps_aca", ctypes.c_double),
        ("eps_q", ctypes.c_double),
        ("eps_st", ctypes.c_double),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("eps_qtr", ctypes.c_double),
        ("n_rhs", ctypes.c_int32),
        ("time_block", ctypes.c_int32),
    ]


class bie_stats(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("n_elem", ctypes.c_int32),
        ("n_lags", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("steps_done", ctypes.c_int64),
        ("n_adm", ctypes.c_int64),
        ("n_inadm", ctypes.c_int64),
        ("near_pairs", ctypes.c_int64),
        ("near_lags", ctypes.c_int64),
        ("rank_sum", ctypes.c_int64 * 3),
        ("rank_max", ctypes.c_int64 * 3),
        ("aca_fallbacks", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("bytes_per_step", ctypes.c_double),
        ("near_bytes_per_step", ctypes.c_double),
        ("flops_per_step", ctypes.c_double),
        ("setup_seconds", ctypes.c_double),
        ("aca_sweeps", ctypes.c_int64),
        ("scratch_bytes", ctypes.c_int64),
        ("aca_host_blocks", ctypes.c_int64),
        ("aca_seconds", ctypes.c_double),
        ("time_block", ctypes.c_int64),
    ]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        return d


class bie_tune(ctypes.Structure):
    _fields_ = [
        ("unroll", ctypes.c_int32),
        ("lds_pad", ctypes.c_int32),
        ("item_order", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("load_bytes", ctypes.c_int32),
        ("mfma", ctypes.c_int32),
        ("best_ms", ctypes.c_double),
        ("default_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class bie_friction(ctypes.Structure):
    _fields_ = [
        ("law", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("t_th", ctypes.c_double),
        ("t_dy", ctypes.c_double),
        ("d_c", ctypes.c_double),
    ]


def make_friction(law, t_th, t_dy, d_c=0.0):
    """bie_friction: law BIE_LAW_EXP_WEAKENING or BIE_LAW_STATIC_DYNAMIC."""
    f = bie_friction()
    f.law = int(law)
    f.t_th = float(t_th)
    f.t_dy = float(t_dy)
    f.d_c = float(d_c)
    return f


class BieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libbie error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libbie.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1903_02118_amd.build`")
    # torch ships its own HIP runtime; loading it first makes the library bind
    # to that same runtime (one HIP runtime per process), so that the device
    # memory and streams torch hands over are valid for its kernels.  Loaded
    # the other way round, the process maps two runtimes and the library's
    # kernels do not see torch's memory.
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    i64, i32, pi64 = ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.bie_plan_dense.argtypes = [ctypes.POINTER(bie_problem), ctypes.POINTER(vp)]
    lib.bie_plan_fdph.argtypes = [ctypes.POINTER(bie_problem), i32, ctypes.POINTER(bie_fdph_params), ctypes.POINTER(vp)]
    lib.bie_plan_scratch_size.argtypes = [vp, pi64]
    lib.bie_plan_windows.argtypes = [vp, vp, i64, vp]
    lib.bie_workspace_size.argtypes = [vp, pi64]
    lib.bie_plan_query.argtypes = [vp, ctypes.POINTER(bie_stats)]
    lib.bie_plan_free.argtypes = [vp]
    lib.bie_plan_free.restype = None
    lib.bie_build_kernel.argtypes = [vp, vp, i64, vp, ctypes.POINTER(vp)]
    lib.bie_compress_fdph.argtypes = [vp, vp, i64, vp, ctypes.POINTER(vp)]
    lib.bie_step.argtypes = [vp, vp, vp, vp]
    lib.bie_run.argtypes = [vp, vp, vp, i64, vp]
    lib.bie_run_graph.argtypes = [vp, vp, vp, i64, vp]
    lib.bie_run_static.argtypes = [vp, vp, vp, i64, vp]
    lib.bie_reset.argtypes = [vp, vp]
    lib.bie_advance.argtypes = [vp, i64, vp]
    lib.bie_autotune.argtypes = [vp, i32, ctypes.POINTER(bie_tune), vp]
    lib.bie_query.argtypes = [vp, ctypes.POINTER(bie_stats)]
    lib.bie_state_bytes.argtypes = [vp, pi64]
    lib.bie_save_state.argtypes = [vp, vp, i64, vp]
    lib.bie_load_state.argtypes = [vp, vp, i64, vp]
    lib.bie_fdph_export.argtypes = [vp, i32, pi64, i64, pi64]
    lib.bie_timing.argtypes = [vp, i32]
    lib.bie_timing_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), pi64]
    lib.bie_step_predict.argtypes = [vp, vp, vp]
    lib.bie_step_commit.argtypes = [vp, vp, vp]
    lib.bie_first_lag.argtypes = [vp, vp, vp]
    lib.bie_rupture_run.argtypes = [vp, ctypes.POINTER(bie_friction), vp, vp, vp, vp, vp, i64, vp]
    lib.bie_hbm_read_probe.argtypes = [vp, i64, ctypes.POINTER(ctypes.c_double), vp]
    lib.bie_set_debug.argtypes = [vp, i32, vp]
    lib.bie_debug_status.argtypes = [vp, pi64, vp]
    lib.bie_diag_aca.argtypes = [i32, i32, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.c_uint64,
                                 ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                 ctypes.POINTER(ctypes.c_double)]
    lib.bie_plan_block_errors.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64, pi64]
    lib.bie_plan_dense_lag_entries.argtypes = [vp, pi64, i64]
    lib.bie_destroy.argtypes = [vp]
    lib.bie_destroy.restype = None
    lib.bie_last_error.restype = ctypes.c_char_p
    for f in EXPORTED:
        if f not in ("bie_destroy", "bie_plan_free", "bie_last_error"):
            getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != BIE_OK:
        raise BieError(rc, _lib.bie_last_error().decode())


def _ptr(x, what="buffer", n=None, dtype="float64"):
    """Device pointer of a tensor handed to the library, after the checks the
    library cannot make on a raw pointer: a contiguous device (cuda) tensor
    of the element type the library reads (dtype None: any) holding at least
    n elements.  A host tensor or a short one would otherwise be read or
    written by the kernels out of bounds.  An int is taken as a device
    address as is."""
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    if not getattr(x, "is_cuda", False):
        raise ValueError(f"{what}: needs a device (cuda) tensor")
    if not x.is_contiguous():
        raise ValueError(f"{what}: needs a contiguous tensor")
    if dtype is not None and str(x.dtype) != "torch." + dtype:
        raise ValueError(f"{what}: element type {x.dtype}, the library reads {dtype}")
    if n is not None and x.numel() < n:
        raise ValueError(f"{what}: {x.numel()} elements, the call needs {n}")
    return ctypes.c_void_p(x.data_ptr())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def hbm_read_probe(buf, stream=None):
    """Milliseconds of one 16-byte non-temporal streaming read of the device
    tensor `buf` (bie_hbm_read_probe)."""
    lib = load()
    ms = ctypes.c_double()
    _check(lib.bie_hbm_read_probe(_ptr(buf, "buf", dtype=None), int(buf.numel() * buf.element_size()), ctypes.byref(ms),
                                  _stream(stream)))
    return ms.value


def make_problem(xa, xb, n_lags, mu=1.0, beta=1.0, dt=0.5, eps_t=1.0, mode=0, alpha=0.0):
    """bie_problem plus the host arrays it points to (kept alive together)."""
    xa = np.ascontiguousarray(xa, dtype=np.float64)
    xb = np.ascontiguousarray(xb, dtype=np.float64)
    p = bie_problem()
    p.n_elem = xa.shape[0]
    p.n_lags = int(n_lags)
    p.xa_host = xa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.xb_host = xb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.mu, p.beta, p.dt, p.eps_t = mu, beta, dt, eps_t
    p.mode, p.reserved, p.alpha = int(mode), 0, float(alpha)
    return p, (xa, xb)


def make_params(eta=2.0, leaf_size=32, n_c=20, eps_aca=1e-6, eps_q=1e-3, eps_st=1e-6, precision=BIE_FP64, seed=12345,
                quantize_tr=False, eps_qtr=0.1, n_rhs=1, host_aca=False, time_block=None):
    q = bie_fdph_params()
    q.eta, q.leaf_size, q.n_c = eta, leaf_size, n_c
    q.eps_aca, q.eps_q, q.eps_st = eps_aca, eps_q, eps_st
    q.precision, q.seed = precision, seed
    q.flags = (BIE_FLAG_QUANTIZE_TRANSIENT if quantize_tr else 0) | (BIE_FLAG_HOST_ACA if host_aca else 0)
    q.eps_qtr = eps_qtr
    q.n_rhs = int(n_rhs)
    # prescribed-slip runs share each pass over the near windows among
    # BIE_TIME_BLOCK steps unless several scenarios already share it
    q.time_block = (BIE_TIME_BLOCK if int(n_rhs) <= 1 else 1) if time_block is None else int(time_block)
    return q


def _device_bytes(nbytes):
    """A device buffer of at least nbytes bytes (a torch uint8 tensor; the
    caching allocator returns 512-byte aligned blocks)."""
    import torch

    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
    if t.data_ptr() % 256:
        raise RuntimeError("device buffer not 256-byte aligned")
    return t


def diag_aca(A, eps, seed=1):
    """ACA+ of the library on a host matrix (bie_diag_aca): (rank, fallback, sweeps, rel err)."""
    lib = load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    r, f, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    e = ctypes.c_double()
    _check(lib.bie_diag_aca(A.shape[0], A.shape[1], A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(eps),
                            int(seed), ctypes.byref(r), ctypes.byref(f), ctypes.byref(w), ctypes.byref(e)))
    return r.value, bool(f.value), w.value, e.value


class Plan:
    """Owner of a bie_plan handle: the host setup of an operator (bie_plan_dense,
    bie_plan_fdph), its window scan and its workspace size."""

    def __init__(self, handle, keep, row_mult):
        self.h = handle
        self._keep = keep
        self.row_mult = row_mult

    @classmethod
    def dense(cls, xa, xb, n_lags, **phys):
        lib = load()
        p, keep = make_problem(xa, xb, n_lags, **phys)
        h = ctypes.c_void_p()
        _check(lib.bie_plan_dense(ctypes.byref(p), ctypes.byref(h)))
        return cls(h, keep, 2 if phys.get("mode", 0) == BIE_MODE_INPLANE else 1)

    @classmethod
    def fdph(cls, faults, params=None, **phys):
        """faults: list of (xa, xb, n_lags); rows of D and T concatenate them in order."""
        lib = load()
        arr = (bie_problem * len(faults))()
        keep = []
        for k, (xa, xb, n_lags) in enumerate(faults):
            p, kp = make_problem(xa, xb, n_lags, **phys)
            arr[k] = p
            keep.append(kp)
        q = params if params is not None else make_params()
        h = ctypes.c_void_p()
        _check(lib.bie_plan_fdph(arr, len(faults), ctypes.byref(q), ctypes.byref(h)))
        return cls(h, keep, max(1, q.n_rhs))

    def scratch_size(self):
        n = ctypes.c_int64()
        _check(_lib.bie_plan_scratch_size(self.h, ctypes.byref(n)))
        return n.value

    def windows(self, scratch=None, stream=None):
        """The plan's device stage (bie_plan_windows): the near-field window
        scan and, unless the plan ran ACA+ on the host, ACA+ of every
        admissible block; with no scratch tensor given, a temporary one of the
        needed size is used."""
        need = self.scratch_size()
        if need == 0:
            _check(_lib.bie_plan_windows(self.h, None, 0, _stream(stream)))
            return
        buf = _device_bytes(need) if scratch is None else scratch
        _check(_lib.bie_plan_windows(self.h, _ptr(buf, "scratch", dtype=None), int(buf.numel() * buf.element_size()),
                                     _stream(stream)))

    def workspace_size(self):
        n = ctypes.c_int64()
        _check(_lib.bie_workspace_size(self.h, ctypes.byref(n)))
        return n.value

    def stats(self):
        s = bie_stats()
        _check(_lib.bie_plan_query(self.h, ctypes.byref(s)))
        return s.as_dict()

    def lag_entries(self, M):
        """Causal-band entries of each lag of a plain-form plan (bie_plan_dense_lag_entries)."""
        buf = np.zeros(int(M), dtype=np.int64)
        _check(_lib.bie_plan_dense_lag_entries(self.h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(M)))
        return buf

    def block_errors(self):
        """Exact relative errors of every low-rank block (bie_plan_block_errors):
        [blocks][8] = leaf, piece, component, rows, columns, rank, FP64 error, BF16 error."""
        rows = ctypes.c_int64()
        _check(_lib.bie_plan_block_errors(self.h, None, 0, ctypes.byref(rows)))
        buf = np.zeros((rows.value, 8))
        if rows.value:
            _check(_lib.bie_plan_block_errors(self.h, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), rows.value,
                                              ctypes.byref(rows)))
        return buf

    def close(self):
        if self.h:
            _lib.bie_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Operator:
    """Owner of a bie_op handle and of the device workspace it lives in."""

    def __init__(self, handle, keep, row_mult=1, ws=None):
        self.h = handle
        self._keep = keep
        self._ws = ws
        self.N = self.stats()["n_elem"]
        # values per step row of D and T: N, 2N (in-plane pairs) or n_rhs * N
        self.row = self.N * row_mult

    @classmethod
    def from_plan(cls, plan, ws=None, stream=None):
        """Build the operator of a plan (windows scanned for FDP=H) inside the
        device tensor ws (a new one of the workspace size if None)."""
        need = plan.workspace_size()
        ws = _device_bytes(need) if ws is None else ws
        st = bie_stats()
        _check(_lib.bie_plan_query(plan.h, ctypes.byref(st)))
        fn = _lib.bie_build_kernel if st.kind == BIE_KIND_DENSE else _lib.bie_compress_fdph
        h = ctypes.c_void_p()
        _check(fn(plan.h, _ptr(ws, "workspace", dtype=None), int(ws.numel() * ws.element_size()), _stream(stream),
                  ctypes.byref(h)))
        return cls(h, plan._keep, plan.row_mult, ws)

    @classmethod
    def build_kernel(cls, xa, xb, n_lags, stream=None, **phys):
        plan = Plan.dense(xa, xb, n_lags, **phys)
        try:
            return cls.from_plan(plan, stream=stream)
        finally:
            plan.close()

    @classmethod
    def compress_fdph(cls, xa, xb, n_lags, params=None, stream=None, **phys):
        return cls.compress_fdph_batched([(xa, xb, n_lags)], params=params, stream=stream, **phys)

    @classmethod
    def compress_fdph_batched(cls, faults, params=None, stream=None, **phys):
        """faults: list of (xa, xb, n_lags); rows of D and T concatenate them in order."""
        plan = Plan.fdph(faults, params=params, **phys)
        try:
            plan.windows(stream=stream)
            return cls.from_plan(plan, stream=stream)
        finally:
            plan.close()

    def step(self, d_n, t_n, stream=None):
        _check(_lib.bie_step(self.h, _ptr(d_n, "d_n", self.row), _ptr(t_n, "t_n", self.row), _stream(stream)))

    def run(self, D, T, steps=None, stream=None):
        steps = D.shape[0] if steps is None else steps
        n = int(steps) * self.row
        _check(_lib.bie_run(self.h, _ptr(D, "D", n), _ptr(T, "T", n), int(steps), _stream(stream)))

    def run_graph(self, D, T, steps=None, stream=None):
        steps = D.shape[0] if steps is None else steps
        n = int(steps) * self.row
        _check(_lib.bie_run_graph(self.h, _ptr(D, "D", n), _ptr(T, "T", n), int(steps), _stream(stream)))

    def run_static(self, D, T, steps=None, stream=None):
        """bie_run with the per-step partial sums in the library's static
        device array (allocates nothing)."""
        steps = D.shape[0] if steps is None else steps
        n = int(steps) * self.row
        _check(_lib.bie_run_static(self.h, _ptr(D, "D", n), _ptr(T, "T", n), int(steps), _stream(stream)))

    def autotune(self, reps=5, stream=None):
        """Time the near-kernel configurations and keep the fastest (blocks)."""
        t = bie_tune()
        _check(_lib.bie_autotune(self.h, int(reps), ctypes.byref(t), _stream(stream)))
        return t.as_dict()

    def step_predict(self, p_n, stream=None):
        """P_n = sum_{m>=1} K_m D_{n-m} of the current step (no advance)."""
        _check(_lib.bie_step_predict(self.h, _ptr(p_n, "p_n", self.row), _stream(stream)))

    def step_commit(self, d_n, stream=None):
        """Take the predicted step's slip rate into the history; advance."""
        _check(_lib.bie_step_commit(self.h, _ptr(d_n, "d_n", self.row), _stream(stream)))

    def first_lag(self, k0, stream=None):
        """K_ii,0 of every element into the device buffer k0 ([N])."""
        _check(_lib.bie_first_lag(self.h, _ptr(k0, "k0", self.row), _stream(stream)))

    def rupture_run(self, friction, t0, slip, state, D, T, steps=None, stream=None):
        """Coupled steps with the friction law (bie_friction): D, T [steps][N] out;
        slip (float64) and state (int32) [N] are read and updated."""
        steps = D.shape[0] if steps is None else steps
        r, n = self.row, int(steps) * self.row
        _check(_lib.bie_rupture_run(self.h, ctypes.byref(friction), _ptr(t0, "t0", r), _ptr(slip, "slip", r),
                                    _ptr(state, "state", r, "int32"), _ptr(D, "D", n), _ptr(T, "T", n), int(steps),
                                    _stream(stream)))

    def advance(self, steps, stream=None):
        _check(_lib.bie_advance(self.h, int(steps), _stream(stream)))

    def reset(self, stream=None):
        _check(_lib.bie_reset(self.h, _stream(stream)))

    def state_bytes(self):
        """Bytes of a saved time-marching state (bie_state_bytes)."""
        n = ctypes.c_int64()
        _check(_lib.bie_state_bytes(self.h, ctypes.byref(n)))
        return n.value

    def save_state(self, buf, stream=None):
        """Checkpoint into the device tensor `buf` (bie_save_state; 256-byte
        aligned, at least state_bytes() bytes).  Returns when done."""
        _check(_lib.bie_save_state(self.h, _ptr(buf, "buf", dtype=None), int(buf.numel() * buf.element_size()),
                                   _stream(stream)))

    def load_state(self, buf, stream=None):
        """Resume from a state saved by an operator of the same problem and
        parameters (bie_load_state).  Returns when done."""
        _check(_lib.bie_load_state(self.h, _ptr(buf, "buf", dtype=None), int(buf.numel() * buf.element_size()),
                                   _stream(stream)))

    def stats(self):
        s = bie_stats()
        _check(_lib.bie_query(self.h, ctypes.byref(s)))
        return s.as_dict()

    def export(self, what):
        width = {BIE_EXPORT_NEAR: 3, BIE_EXPORT_LEAVES: 5, BIE_EXPORT_ART: 6, BIE_EXPORT_TRANS: 4}[what]
        rows = ctypes.c_int64()
        _check(_lib.bie_fdph_export(self.h, what, None, 0, ctypes.byref(rows)))
        buf = np.zeros((rows.value, width), dtype=np.int64)
        if rows.value:
            _check(_lib.bie_fdph_export(self.h, what, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows.value, ctypes.byref(rows)))
        return buf

    def timing(self, enable=True):
        _check(_lib.bie_timing(self.h, 1 if enable else 0))

    def timing_read(self):
        """(total ms, launches) of the dominant kernel since timing(True)."""
        ms = ctypes.c_double()
        k = ctypes.c_int64()
        _check(_lib.bie_timing_read(self.h, ctypes.byref(ms), ctypes.byref(k)))
        return ms.value, k.value

    def set_debug(self, flags=BIE_DEBUG_SCAN_FINITE, stream=None):
        """Scan every step's tractions for NaN/Inf (bie_set_debug)."""
        _check(_lib.bie_set_debug(self.h, int(flags), _stream(stream)))

    def debug_status(self, stream=None):
        """First (step * row + index) of a non-finite traction, or -1 (bie_debug_status)."""
        v = ctypes.c_int64()
        _check(_lib.bie_debug_status(self.h, ctypes.byref(v), _stream(stream)))
        return v.value

    def close(self):
        if self.h:
            _lib.bie_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
