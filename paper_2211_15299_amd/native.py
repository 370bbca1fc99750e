"""ctypes binding of the C ABI in include/hidft.h (argument marshalling only).

Every step of the transform runs in the HIP library; this module only converts
Python values and torch tensors into the pointers, sizes and stream handles
the C functions take.  There is no fallback: if the library is missing, every
call raises.

torch is imported (when installed) before the library is loaded, so the
library binds to the same HIP runtime instance as torch's tensors and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

try:  # load torch's HIP runtime first: one runtime instance per process
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - the planner still works without torch
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhidft.so")

HIDFT_PLAN_HOST_ONLY = 0x1
HIDFT_SAS_TWO_PASS = 0x2
HIDFT_SAS_WEIGHTS_ONLY = 0x4
SAS_MAX_REL_ERR = 1e-5
MAX_LOG2_K_DEVICE = 14
MAX_LOG2_K_LARGE = 22
SAS_SCRATCH_BYTES = 16 << 20  # hidft_sas_execute_noalloc: one signal's workspace at most

# Execution variants (hidft_exec_config)
PREC_FP32, PREC_F16X2, PREC_BF16X3 = 0, 1, 2
PRECISIONS = {"fp32": PREC_FP32, "f16x2": PREC_F16X2, "bf16x3": PREC_BF16X3}
SCHED_DEFAULT, SCHED_SHORT_FIRST, SCHED_SHORT_LAST, SCHED_TUNED = 0, 1, 2, 3

STATUS_NAMES = {
    0: "HIDFT_OK", 1: "HIDFT_ERR_INVALID_ARGUMENT", 2: "HIDFT_ERR_INDEX_OUT_OF_RANGE",
    3: "HIDFT_ERR_DUPLICATE_INDEX", 4: "HIDFT_ERR_SIZE_NOT_POW2",
    5: "HIDFT_ERR_NOT_HOMOGENEOUS", 6: "HIDFT_ERR_OUT_OF_MEMORY", 7: "HIDFT_ERR_DEVICE",
    8: "HIDFT_ERR_UNSUPPORTED",
}

# (name, restype, argtypes) of every function declared in include/hidft.h
_u32, _u64, _i32, _i64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
_vp, _pp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = [
    ("hidft_analyze", ctypes.c_int, [_u32, ctypes.POINTER(_u64), _u64, ctypes.POINTER(_u32),
                                     ctypes.POINTER(_u32), ctypes.POINTER(_i32)]),
    ("hidft_plan_create", ctypes.c_int, [_u32, ctypes.POINTER(_u64), _u64, _u32, _vp, _pp]),
    ("hidft_plan_destroy", ctypes.c_int, [_vp]),
    ("hidft_plan_get_info", ctypes.c_int, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u64),
                                           ctypes.POINTER(_u32)]),
    ("hidft_plan_get_pivots", ctypes.c_int, [_vp, ctypes.POINTER(_u32)]),
    ("hidft_plan_get_samples", ctypes.c_int, [_vp, ctypes.POINTER(_u64)]),
    ("hidft_plan_get_schedule", ctypes.c_int, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u64),
                                               ctypes.POINTER(ctypes.c_uint8)]),
    ("hidft_plan_get_twiddles", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float)]),
    ("hidft_plan_device_bytes", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    ("hidft_execute", ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _u64, _vp]),
    ("hidft_plan_workspace_bytes", ctypes.c_int, [_vp, _u64, ctypes.POINTER(ctypes.c_size_t)]),
    ("hidft_execute_ws", ctypes.c_int,
     [_vp, _vp, _i64, _vp, _i64, _u64, _vp, ctypes.c_size_t, _vp]),
    ("hidft_execute_config", ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _u64, _vp]),
    ("hidft_autotune", ctypes.c_int, [_vp, _u32, _vp, _i64, _vp, _i64, _u64, _u32, _vp, _vp,
                                      ctypes.POINTER(ctypes.c_double)]),
    ("hidft_tune_lookup", ctypes.c_int, [_vp, _u32, _u64, _vp, ctypes.POINTER(_i32)]),
    ("hidft_tune_clear", ctypes.c_int, []),
    ("hidft_tune_save", ctypes.c_int, [ctypes.c_char_p]),
    ("hidft_tune_load", ctypes.c_int, [ctypes.c_char_p]),
    ("hidft_execute_plain", ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _u64, _vp]),
    ("hidft_execute_inverse", ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _u64, _vp]),
    ("hidft_execute_inverse_ws", ctypes.c_int,
     [_vp, _vp, _i64, _vp, _i64, _u64, _vp, ctypes.c_size_t, _vp]),
    ("hidft_group_create", ctypes.c_int, [_vp, _u64, _vp, _pp]),
    ("hidft_group_execute", ctypes.c_int, [_vp, _vp]),
    ("hidft_group_destroy", ctypes.c_int, [_vp]),
    ("hidft_group_set_config", ctypes.c_int, [_vp, _vp, _vp]),
    ("hidft_group_get_config", ctypes.c_int, [_vp, _vp]),
    ("hidft_group_autotune", ctypes.c_int, [_vp, _u32, _vp, _vp, ctypes.POINTER(ctypes.c_double)]),
    ("hidft_group_get_info", ctypes.c_int, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                            ctypes.POINTER(ctypes.c_size_t)]),
    ("hidft_server_create", ctypes.c_int, [_vp, _pp]),
    ("hidft_server_submit", ctypes.c_int, [_vp, _u32, ctypes.POINTER(_u64), _u64, _vp, _vp,
                                           ctypes.POINTER(_u64)]),
    ("hidft_server_submit_many", ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, ctypes.POINTER(_u64)]),
    ("hidft_server_poll", ctypes.c_int, [_vp, _vp, _u32, ctypes.POINTER(_u32), _i32]),
    ("hidft_server_drain", ctypes.c_int, [_vp]),
    ("hidft_server_get_stats", ctypes.c_int, [_vp, _vp]),
    ("hidft_server_destroy", ctypes.c_int, [_vp]),
    ("hidft_sas_create", ctypes.c_int, [_u32, ctypes.POINTER(_u64), _u64, ctypes.POINTER(_u32),
                                        _u32, _u32, _vp, _pp]),
    ("hidft_sas_destroy", ctypes.c_int, [_vp]),
    ("hidft_sas_get_info", ctypes.c_int, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32),
                                          ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                          ctypes.POINTER(ctypes.c_double)]),
    ("hidft_sas_get_accuracy", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
    ("hidft_sas_get_pivots", ctypes.c_int, [_vp, ctypes.POINTER(_u32)]),
    ("hidft_sas_get_samples", ctypes.c_int, [_vp, ctypes.POINTER(_u64)]),
    ("hidft_sas_get_nodes", ctypes.c_int, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u32)]),
    ("hidft_sas_workspace_bytes", ctypes.c_int, [_vp, _u64, ctypes.POINTER(ctypes.c_size_t)]),
    ("hidft_sas_execute", ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _u64, _vp, _vp]),
    ("hidft_sas_weights", ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _u64, _vp]),
    ("hidft_sas_execute_noalloc", ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _u64, _vp]),
    ("hidft_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("hidft_last_error", ctypes.c_char_p, []),
]

_LIB: Optional[ctypes.CDLL] = None


class HiDFTError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, f"status {status}")
        super().__init__(f"{self.status_name}: {message}")


def lib() -> ctypes.CDLL:
    """The loaded C library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"HIP library {LIB_PATH} is missing: build it with "
                "`python -m paper_2211_15299_amd.build` (there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(status: int) -> None:
    if status != 0:
        msg = lib().hidft_last_error().decode(errors="replace")
        raise HiDFTError(status, msg)


def _u64_array(J: Sequence[int]) -> np.ndarray:
    arr = np.ascontiguousarray(np.asarray(J, dtype=np.uint64))
    return arr


def _ptr(arr: np.ndarray, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def analyze(log2_n: int, J: Sequence[int]):
    """(pivots, is_homogeneous) of J subset of Z_{2^log2_n} (hidft_analyze)."""
    arr = _u64_array(J)
    piv = np.zeros(64, dtype=np.uint32)
    n = _u32(0)
    hom = _i32(0)
    _check(lib().hidft_analyze(log2_n, _ptr(arr, _u64), len(arr), _ptr(piv, _u32),
                               ctypes.byref(n), ctypes.byref(hom)))
    return [int(x) for x in piv[: n.value]], bool(hom.value)


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class GroupConfig(ctypes.Structure):
    """hidft_group_config: schedule and pack order of a grouped launch."""
    _fields_ = [("schedule", ctypes.c_uint32), ("order", ctypes.c_uint32)]

    def __repr__(self):
        return f"GroupConfig(schedule={self.schedule}, order={self.order})"


GROUP_ORDER_LARGEST_FIRST = 0
GROUP_ORDER_ALTERNATE = 1


class ExecConfig(ctypes.Structure):
    """hidft_exec_config: precision, schedule and launch shape of a transform."""
    _fields_ = [("precision", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("radix", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32)]

    def __repr__(self):
        return (f"ExecConfig(precision={self.precision}, schedule={self.schedule}, "
                f"radix={self.radix}, blocks_per_cu={self.blocks_per_cu})")

    def as_tuple(self):
        return (self.precision, self.schedule, self.radix, self.blocks_per_cu)


class Plan:
    """Owning wrapper of a hidft_plan (hidft_plan_create / hidft_plan_destroy)."""

    def __init__(self, log2_n: int, J: Sequence[int], host_only: bool = False, stream=None):
        arr = _u64_array(J)
        self._h = ctypes.c_void_p(None)
        flags = HIDFT_PLAN_HOST_ONLY if host_only else 0
        st = None if host_only else _stream_handle(stream)
        _check(lib().hidft_plan_create(log2_n, _ptr(arr, _u64), len(arr), flags, st,
                                       ctypes.byref(self._h)))
        self.host_only = host_only
        M, k, s = _u32(0), _u64(0), _u32(0)
        _check(lib().hidft_plan_get_info(self._h, ctypes.byref(M), ctypes.byref(k),
                                         ctypes.byref(s)))
        self.log2_n, self.k, self.s = M.value, k.value, s.value

    # -- lifecycle
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().hidft_plan_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h.value:
            raise HiDFTError(1, "plan has been destroyed")
        return self._h

    # -- getters
    def pivots(self) -> list:
        out = np.zeros(max(self.s, 1), dtype=np.uint32)
        _check(lib().hidft_plan_get_pivots(self.handle, _ptr(out, _u32)))
        return [int(x) for x in out[: self.s]]

    def samples(self) -> np.ndarray:
        out = np.zeros(self.k, dtype=np.uint64)
        _check(lib().hidft_plan_get_samples(self.handle, _ptr(out, _u64)))
        return out

    def schedule(self):
        """(freq_pos[k], tw_num[k-1], tw_log2den[k-1]) as numpy arrays."""
        fp = np.zeros(self.k, dtype=np.uint32)
        n = max(self.k - 1, 1)
        num = np.zeros(n, dtype=np.uint64)
        den = np.zeros(n, dtype=np.uint8)
        _check(lib().hidft_plan_get_schedule(self.handle, _ptr(fp, _u32), _ptr(num, _u64),
                                             _ptr(den, ctypes.c_uint8)))
        return fp, num[: self.k - 1], den[: self.k - 1]

    def twiddles(self) -> np.ndarray:
        out = np.zeros(2 * max(self.k - 1, 1), dtype=np.float32)
        _check(lib().hidft_plan_get_twiddles(self.handle, _ptr(out, ctypes.c_float)))
        return (out[0::2] + 1j * out[1::2]).astype(np.complex64)[: self.k - 1]

    def device_bytes(self) -> int:
        b = ctypes.c_size_t(0)
        _check(lib().hidft_plan_device_bytes(self.handle, ctypes.byref(b)))
        return b.value

    def workspace_bytes(self, batch: int) -> int:
        """hidft_plan_workspace_bytes: 0 up to 2^14 points, else batch * k * 8."""
        b = ctypes.c_size_t(0)
        _check(lib().hidft_plan_workspace_bytes(self.handle, batch, ctypes.byref(b)))
        return b.value

    # -- execution on raw device pointers
    def execute_ws_ptr(self, d_in: int, ld_in: int, d_out: int, ld_out: int, batch: int,
                       d_work: int, work_bytes: int, stream=None) -> None:
        _check(lib().hidft_execute_ws(self.handle, d_in, ld_in, d_out, ld_out, batch, d_work,
                                      work_bytes, _stream_handle(stream)))

    def execute_ptr(self, d_in: int, ld_in: int, d_out: int, ld_out: int, batch: int,
                    stream=None, plain: bool = False,
                    config: Optional[ExecConfig] = None) -> None:
        if config is not None:
            if plain:
                raise HiDFTError(1, "the plain method has no execution variants")
            _check(lib().hidft_execute_config(self.handle, ctypes.byref(config), d_in, ld_in,
                                              d_out, ld_out, batch, _stream_handle(stream)))
            return
        fn = lib().hidft_execute_plain if plain else lib().hidft_execute
        _check(fn(self.handle, d_in, ld_in, d_out, ld_out, batch, _stream_handle(stream)))

    def autotune_ptr(self, d_in: int, ld_in: int, d_out: int, ld_out: int, batch: int,
                     precision: int = PREC_FP32, reps: int = 10, stream=None):
        """hidft_autotune: (best ExecConfig, its mean launch time in us)."""
        best = ExecConfig()
        us = ctypes.c_double(0.0)
        _check(lib().hidft_autotune(self.handle, precision, d_in, ld_in, d_out, ld_out, batch,
                                    reps, _stream_handle(stream), ctypes.byref(best),
                                    ctypes.byref(us)))
        return best, us.value

    def tune_lookup(self, batch: int, precision: int = PREC_FP32) -> Optional[ExecConfig]:
        cfg = ExecConfig()
        found = _i32(0)
        _check(lib().hidft_tune_lookup(self.handle, precision, batch, ctypes.byref(cfg),
                                       ctypes.byref(found)))
        return cfg if found.value else None

    def inverse_ptr(self, d_coefs: int, ld_in: int, d_samples: int, ld_out: int, batch: int,
                    stream=None) -> None:
        _check(lib().hidft_execute_inverse(self.handle, d_coefs, ld_in, d_samples, ld_out, batch,
                                           _stream_handle(stream)))

    def inverse_ws_ptr(self, d_coefs: int, ld_in: int, d_samples: int, ld_out: int, batch: int,
                       d_work: int, work_bytes: int, stream=None) -> None:
        _check(lib().hidft_execute_inverse_ws(self.handle, d_coefs, ld_in, d_samples, ld_out,
                                              batch, d_work, work_bytes, _stream_handle(stream)))

    # -- execution on torch tensors
    def execute(self, samples, out=None, stream=None, plain: bool = False,
                config: Optional[ExecConfig] = None):
        """Coefficients (batch, k) complex64 of samples (batch, k) or (k,) on the device."""
        if torch is None:
            raise RuntimeError("torch is required for tensor execution")
        squeeze = samples.dim() == 1
        x = samples.unsqueeze(0) if squeeze else samples
        if x.dtype != torch.complex64 or not x.is_cuda:
            raise HiDFTError(1, "samples must be a complex64 CUDA/HIP tensor")
        if x.dim() != 2 or x.shape[1] != self.k or x.stride(1) != 1:
            raise HiDFTError(1, f"samples must be (batch, {self.k}) with unit inner stride")
        if out is None:
            out = torch.empty((x.shape[0], self.k), dtype=torch.complex64, device=x.device)
        y = out.unsqueeze(0) if out.dim() == 1 else out
        if y.dtype != torch.complex64 or y.dim() != 2 or y.shape != x.shape or y.stride(1) != 1:
            raise HiDFTError(1, "out must match samples' shape, complex64, unit inner stride")
        ld_in = x.stride(0) if x.shape[0] > 1 else self.k
        ld_out = y.stride(0) if y.shape[0] > 1 else self.k
        wb = self.workspace_bytes(x.shape[0])
        if wb and not plain and config is None:
            # k > 2^14: the passes' workspace from torch's allocator
            work = torch.empty(wb // 8, dtype=torch.complex64, device=x.device)
            self.execute_ws_ptr(x.data_ptr(), ld_in, y.data_ptr(), ld_out, x.shape[0],
                                work.data_ptr(), wb, stream)
        else:
            self.execute_ptr(x.data_ptr(), ld_in, y.data_ptr(), ld_out, x.shape[0], stream,
                             plain, config)
        return out


def tune_clear() -> None:
    _check(lib().hidft_tune_clear())


def tune_save(path: str) -> None:
    _check(lib().hidft_tune_save(os.fsencode(path)))


def tune_load(path: str) -> None:
    _check(lib().hidft_tune_load(os.fsencode(path)))


class Work(ctypes.Structure):
    """hidft_work: a plan and `batch` rows of samples / coefficients."""
    _fields_ = [("plan", ctypes.c_void_p), ("d_samples", ctypes.c_void_p), ("ld_in", ctypes.c_int64),
                ("d_coefs", ctypes.c_void_p), ("ld_out", ctypes.c_int64), ("batch", ctypes.c_uint64)]


class Group:
    """Owning wrapper of a hidft_group (one persistent launch over uneven work).

    items: sequence of (plan, d_samples, ld_in, d_coefs, ld_out, batch); the
    plans and buffers must outlive the group.
    """

    def __init__(self, items, stream=None):
        arr = (Work * len(items))()
        self._keep = []
        for i, (plan, d_in, ld_in, d_out, ld_out, batch) in enumerate(items):
            arr[i] = Work(plan.handle.value, d_in, ld_in, d_out, ld_out, batch)
            self._keep.append(plan)
        self._h = ctypes.c_void_p(None)
        _check(lib().hidft_group_create(ctypes.cast(arr, ctypes.c_void_p), len(items),
                                        _stream_handle(stream), ctypes.byref(self._h)))
        n_inst, n_packs, nbytes = _u64(0), _u64(0), ctypes.c_size_t(0)
        _check(lib().hidft_group_get_info(self._h, ctypes.byref(n_inst), ctypes.byref(n_packs),
                                          ctypes.byref(nbytes)))
        self.n_instances, self.n_packs, self.device_bytes = n_inst.value, n_packs.value, nbytes.value

    def execute(self, stream=None) -> None:
        _check(lib().hidft_group_execute(self._h, _stream_handle(stream)))

    def set_config(self, schedule: int, order: int, stream=None) -> None:
        cfg = GroupConfig(schedule, order)
        _check(lib().hidft_group_set_config(self._h, ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p),
                                            _stream_handle(stream)))

    def config(self) -> GroupConfig:
        cfg = GroupConfig(0, 0)
        _check(lib().hidft_group_get_config(self._h, ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p)))
        return cfg

    def autotune(self, reps: int = 10, stream=None):
        """Times every launch configuration, keeps the fastest; returns it and
        its mean launch time in microseconds."""
        cfg = GroupConfig(0, 0)
        us = ctypes.c_double(0.0)
        _check(lib().hidft_group_autotune(self._h, reps, _stream_handle(stream),
                                          ctypes.cast(ctypes.byref(cfg), ctypes.c_void_p),
                                          ctypes.byref(us)))
        return cfg, us.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().hidft_group_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ServerConfig(ctypes.Structure):
    _fields_ = [("data_bytes", ctypes.c_size_t), ("plan_bytes", ctypes.c_size_t),
                ("slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32)]


RESULT_DTYPE = np.dtype([("id", np.uint64), ("status", np.int32), ("batch_size", np.uint32),
                         ("latency_us", np.float64)])


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("submitted", "completed", "rejected", "batches", "plan_hits", "plan_misses",
                 "plan_evictions", "max_inflight_batches", "plans_resident")] + \
               [("plan_bytes_resident", ctypes.c_size_t), ("slot_bytes", ctypes.c_size_t),
                ("plan_bytes_peak", ctypes.c_size_t)] + \
               [(n, ctypes.c_uint64) for n in ("waiting_for_plan", "plan_waits", "failed")]


# hidft_server_request, as a numpy record (one call submits many)
REQUEST_DTYPE = np.dtype([("log2_n", np.uint32), ("J", np.uint64), ("k", np.uint64),
                          ("host_samples", np.uint64), ("host_coefs", np.uint64)], align=True)


class Server:
    """Continuous-batching request server (hidft_server_*).

    submit() takes host numpy arrays; the caller keeps `samples` and `out`
    alive until the request's result has been polled.
    """

    def __init__(self, data_bytes=256 << 20, plan_bytes=64 << 20, slots=3, max_batch=512):
        cfg = ServerConfig(data_bytes, plan_bytes, slots, max_batch)
        self._h = ctypes.c_void_p(None)
        _check(lib().hidft_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._res = np.zeros(4096, dtype=RESULT_DTYPE)

    def submit(self, log2_n: int, J: np.ndarray, samples: np.ndarray, out: np.ndarray) -> int:
        rid = _u64(0)
        _check(lib().hidft_server_submit(self._h, log2_n, J.ctypes.data_as(ctypes.POINTER(_u64)),
                                         J.shape[0], samples.ctypes.data, out.ctypes.data,
                                         ctypes.byref(rid)))
        return rid.value

    def submit_many(self, reqs: np.ndarray):
        """Submits the REQUEST_DTYPE records `reqs` (pointers as integers; the
        arrays they point to must stay alive) in one call; returns (ids,
        statuses) per request (id 0 where refused)."""
        n = len(reqs)
        ids = np.zeros(max(n, 1), dtype=np.uint64)
        sts = np.zeros(max(n, 1), dtype=np.int32)
        acc = _u64(0)
        _check(lib().hidft_server_submit_many(self._h, reqs.ctypes.data, n, ids.ctypes.data,
                                              sts.ctypes.data, ctypes.byref(acc)))
        return ids[:n], sts[:n]

    def poll(self, wait_us: int = 0) -> np.ndarray:
        n = _u32(0)
        _check(lib().hidft_server_poll(self._h, self._res.ctypes.data, len(self._res),
                                       ctypes.byref(n), wait_us))
        return self._res[: n.value].copy()

    def drain(self) -> None:
        _check(lib().hidft_server_drain(self._h))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().hidft_server_get_stats(self._h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in ServerStats._fields_}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().hidft_server_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SASPlan:
    """Shift-and-Sample plan of a part-homogeneous support (hidft_sas_*).

    pivots=None lets the planner choose r (Lemma 4's cost within the accuracy
    bound).  two_pass=True keeps the shifted Hi-DFTs and the leaf solves in
    two launches through a workspace even where the plan could run as one
    kernel.  weights_only=True makes a plan for the induced weights alone.
    """

    def __init__(self, log2_n: int, J: Sequence[int], pivots=None, host_only: bool = False,
                 stream=None, two_pass: bool = False, weights_only: bool = False):
        arr = _u64_array(J)
        self._h = ctypes.c_void_p(None)
        if pivots is None:
            rp, nr = None, 0
        else:  # an explicit vector, possibly empty: always a non-NULL pointer
            self._r = np.zeros(max(len(pivots), 1), dtype=np.uint32)
            self._r[: len(pivots)] = pivots
            rp, nr = _ptr(self._r, _u32), len(pivots)
        flags = ((HIDFT_PLAN_HOST_ONLY if host_only else 0) | (HIDFT_SAS_TWO_PASS if two_pass else 0)
                 | (HIDFT_SAS_WEIGHTS_ONLY if weights_only else 0))
        _check(lib().hidft_sas_create(log2_n, _ptr(arr, _u64), len(arr), rp, nr, flags,
                                      None if host_only else _stream_handle(stream),
                                      ctypes.byref(self._h)))
        s, mu, nn, sp = _u32(0), _u32(0), _u64(0), _u64(0)
        cost = ctypes.c_double(0)
        _check(lib().hidft_sas_get_info(self._h, ctypes.byref(s), ctypes.byref(mu),
                                        ctypes.byref(nn), ctypes.byref(sp), ctypes.byref(cost)))
        self.log2_n, self.k = log2_n, len(arr)
        self.s, self.mu_max, self.n_nodes = s.value, mu.value, nn.value
        self.samples_per_signal, self.cost = sp.value, cost.value
        cond, amp, bound = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        _check(lib().hidft_sas_get_accuracy(self._h, ctypes.byref(cond), ctypes.byref(amp),
                                            ctypes.byref(bound)))
        self.leaf_cond, self.amplification, self.err_bound = cond.value, amp.value, bound.value

    def pivots(self):
        out = np.zeros(max(self.s, 1), dtype=np.uint32)
        _check(lib().hidft_sas_get_pivots(self._h, _ptr(out, _u32)))
        return [int(x) for x in out[: self.s]]

    def samples(self) -> np.ndarray:
        out = np.zeros(self.samples_per_signal, dtype=np.uint64)
        _check(lib().hidft_sas_get_samples(self._h, _ptr(out, _u64)))
        return out

    def nodes(self):
        """(node index of each J[t], slot of each node)."""
        nt = np.zeros(self.k, dtype=np.uint32)
        sl = np.zeros(max(self.n_nodes, 1), dtype=np.uint32)
        _check(lib().hidft_sas_get_nodes(self._h, _ptr(nt, _u32), _ptr(sl, _u32)))
        return nt, sl[: self.n_nodes]

    def workspace_bytes(self, batch: int) -> int:
        b = ctypes.c_size_t(0)
        _check(lib().hidft_sas_workspace_bytes(self._h, batch, ctypes.byref(b)))
        return b.value

    def execute_ptr(self, d_in, ld_in, d_out, ld_out, batch, d_work, stream=None):
        _check(lib().hidft_sas_execute(self._h, d_in, ld_in, d_out, ld_out, batch, d_work,
                                       _stream_handle(stream)))

    def execute_noalloc_ptr(self, d_in, ld_in, d_out, ld_out, batch, stream=None):
        _check(lib().hidft_sas_execute_noalloc(self._h, d_in, ld_in, d_out, ld_out, batch,
                                               _stream_handle(stream)))

    def weights_ptr(self, d_in, ld_in, d_out, ld_out, batch, stream=None):
        _check(lib().hidft_sas_weights(self._h, d_in, ld_in, d_out, ld_out, batch,
                                       _stream_handle(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(lib().hidft_sas_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def status_string(status: int) -> str:
    return lib().hidft_status_string(status).decode()
