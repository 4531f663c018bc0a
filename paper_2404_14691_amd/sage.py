"""Python binding of libsage (include/sage.h): argument marshalling only.

Every function has the name of the C entry point it calls and raises
``SageError`` when that call returns a status other than SAGE_OK.  Host
buffers are numpy arrays (or anything exposing the buffer protocol); device
buffers are plain integer addresses (e.g. ``torch.Tensor.data_ptr()``).
The shared library is built in-tree by ``paper_2404_14691_amd.build``; when it
is missing this module raises on import instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib")
LIB_PATH = os.path.join(LIB_DIR, "libsage.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2404_14691_amd.build`")

_lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)

# ------------------------------------------------------------------ constants
SAGE_OK, SAGE_EINVAL, SAGE_ENOMEM, SAGE_EBUSY, SAGE_ENOTFOUND, SAGE_ESTATE, SAGE_EHIP, SAGE_EIO = range(8)
STATUS_NAMES = ["SAGE_OK", "SAGE_EINVAL", "SAGE_ENOMEM", "SAGE_EBUSY", "SAGE_ENOTFOUND",
                "SAGE_ESTATE", "SAGE_EHIP", "SAGE_EIO"]
SAGE_RO, SAGE_RW = 0, 1
SAGE_SRC_HOST, SAGE_SRC_DEVICE = 0, 1
SAGE_MLP_F32, SAGE_MLP_BF16, SAGE_STENCIL7_F32, SAGE_RELAX7_F32 = 1, 2, 3, 4
SAGE_IO_DEVICE_IN, SAGE_IO_DEVICE_OUT = 1, 2
SAGE_OP_COPY, SAGE_OP_VERIFY = 0, 1
BLOCK = 65536


class SageError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}: {msg}")


# ------------------------------------------------------------------ structs
class sage_blob(C.Structure):
    _fields_ = [("src", C.c_void_p), ("nbytes", C.c_size_t), ("access", C.c_uint32),
                ("where", C.c_uint32), ("key", C.c_uint64)]


class sage_fn_desc(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("layers", C.c_uint32), ("width", C.c_uint32),
                ("nx", C.c_uint32), ("ny", C.c_uint32), ("nz", C.c_uint32), ("sweeps", C.c_uint32),
                ("coef", C.c_float)]


class sage_config(C.Structure):
    _fields_ = [("ring_slots", C.c_size_t), ("chunk_bytes", C.c_size_t), ("streams", C.c_uint32),
                ("fill_threads", C.c_uint32), ("inflight_groups", C.c_uint32), ("share", C.c_uint32),
                ("batch", C.c_uint32), ("serial_setup", C.c_uint32), ("pool_budget_bytes", C.c_size_t),
                ("tune_cache", C.c_char_p), ("exit_stage_ms", C.c_double), ("host_cache_bytes", C.c_size_t),
                ("progressive", C.c_uint32)]


class sage_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "logical_bytes", "unique_bytes", "shared_bytes", "private_bytes", "resident_bytes",
        "resident_slots", "budget_slots", "classes", "h2d_bytes", "refcount_sum", "live_setups",
        "evictions", "reloads", "registrations", "invocations", "verify_mismatches", "workspace_bytes")] + \
        [(n, C.c_double) for n in ("t_register_ms", "t_code_ms", "t_fp_wait_ms", "t_dedup_ms", "t_verify_ms",
                                   "t_setup_ms", "t_invoke_ms")] + \
        [(n, C.c_uint64) for n in ("host_cached_bytes", "demotions", "host_reloads", "module_loads",
                                   "module_unloads")] + \
        [(n, C.c_double) for n in ("t_module_ms", "t_reload_ms", "t_release_ms", "t_unregister_ms")]

    def as_dict(self) -> dict:
        return {n: (int(getattr(self, n)) if t is C.c_uint64 else float(getattr(self, n)))
                for n, t in self._fields_}

    def counters(self) -> dict:
        """The integer counters only (timers excluded)."""
        return {n: int(getattr(self, n)) for n, t in self._fields_ if t is C.c_uint64}


class sage_req_info(C.Structure):
    _fields_ = [("setup_ms", C.c_double), ("e2e_ms", C.c_double), ("status", C.c_uint32)]


class sage_serve_report(C.Structure):
    _fields_ = [("completed", C.c_uint64), ("failed", C.c_uint64), ("launches", C.c_uint64), ("rows", C.c_uint64),
                ("setup_p50_ms", C.c_double), ("setup_p99_ms", C.c_double), ("e2e_p50_ms", C.c_double),
                ("e2e_p99_ms", C.c_double), ("span_ms", C.c_double), ("throughput", C.c_double)]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class sage_blk_op(C.Structure):
    _fields_ = [("src", C.c_uint64), ("dst", C.c_uint64), ("len", C.c_uint32), ("op", C.c_uint32)]


# ------------------------------------------------------------------ signatures
_P = C.c_void_p
_sigs = {
    "sage_config_default": (None, [C.POINTER(sage_config)]),
    "sage_open": (C.c_int, [C.c_int, C.POINTER(sage_config), C.POINTER(_P)]),
    "sage_close": (C.c_int, [_P]),
    "sage_last_error": (C.c_char_p, []),
    "sage_host_alloc": (_P, [_P, C.c_size_t]),
    "sage_host_free": (None, [_P, _P]),
    "fn_register": (C.c_int, [_P, C.POINTER(sage_fn_desc), C.POINTER(sage_blob), C.c_size_t,
                              C.POINTER(C.c_uint64)]),
    "fn_register_batch": (C.c_int, [_P, C.c_size_t, C.POINTER(sage_fn_desc), C.POINTER(C.POINTER(sage_blob)),
                                    C.POINTER(C.c_size_t), C.POINTER(C.c_uint64), C.POINTER(C.c_double)]),
    "fn_unregister": (C.c_int, [_P, C.c_uint64]),
    "fn_setup": (C.c_int, [_P, C.c_uint64, C.c_uint32, C.POINTER(C.c_uint64)]),
    "fn_invoke": (C.c_int, [_P, C.c_uint64, _P, C.c_size_t, _P, C.c_size_t, C.c_uint32]),
    "fn_invoke_batch": (C.c_int, [_P, C.c_size_t, C.POINTER(C.c_uint64), C.POINTER(_P), C.POINTER(C.c_size_t),
                                  C.POINTER(_P), C.POINTER(C.c_size_t), C.c_uint32]),
    "fn_invoke_noalloc": (C.c_int, [_P, C.c_uint64, _P, C.c_size_t, _P, C.c_size_t]),
    "fn_release": (C.c_int, [_P, C.c_uint64]),
    "fn_setup_batch": (C.c_int, [_P, C.c_size_t, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32),
                                 C.POINTER(C.c_uint64), C.POINTER(C.c_size_t), C.POINTER(C.c_double)]),
    "fn_release_batch": (C.c_int, [_P, C.c_size_t, C.POINTER(C.c_uint64)]),
    "sage_get_stats": (C.c_int, [_P, C.POINTER(sage_stats)]),
    "sage_fn_fingerprints": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_uint64), C.c_size_t]),
    "sage_fn_block_info": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                     C.POINTER(C.c_uint32), C.c_size_t]),
    "sage_fn_block_count": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_size_t)]),
    "sage_read_slot": (C.c_int, [_P, C.c_uint32, _P]),
    "sage_fingerprint": (C.c_int, [_P, _P, C.c_size_t, _P, _P]),
    "sage_blkcopy": (C.c_int, [_P, _P, C.c_size_t, _P, _P]),
    "sage_timing_enable": (C.c_int, [_P, C.c_int]),
    "sage_timing_get": (C.c_int, [_P, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]),
    "sage_mfma_ceiling": (C.c_int, [_P, C.c_uint32, C.c_uint32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "sage_timing_reset": (C.c_int, [_P]),
    "sage_timing_only": (C.c_int, [_P, C.c_char_p]),
    "sage_last_launch": (C.c_int, [_P, C.c_char_p, C.c_size_t]),
    "sage_tick": (C.c_int, [_P]),
    "sage_selftest_segments": (C.c_int, [C.POINTER(C.c_uint32), C.c_size_t, C.c_uint32, C.c_uint64,
                                         C.POINTER(C.c_size_t)]),
    "sage_selftest_plan": (C.c_int, [C.c_uint32, C.POINTER(C.c_uint32), C.c_size_t, C.POINTER(C.c_char_p),
                                     C.POINTER(C.c_double), C.c_size_t, C.c_uint32, C.c_char_p, C.c_size_t]),
    "sage_selftest_setup_overlap": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_int,
                                              C.POINTER(C.c_double)]),
    "sage_selftest_pool": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, C.POINTER(C.c_uint32)]),
    "sage_serve_start": (C.c_int, [_P, C.c_uint32]),
    "sage_serve_stop": (C.c_int, [_P]),
    "sage_submit": (C.c_int, [_P, C.c_uint64, C.c_uint32, _P, C.c_size_t, _P, C.c_size_t, C.c_uint32,
                              C.POINTER(C.c_uint64)]),
    "sage_wait": (C.c_int, [_P, C.c_uint64, C.c_double, C.POINTER(sage_req_info)]),
    "sage_serve_stats": (C.c_int, [_P, C.POINTER(sage_serve_report)]),
    "sage_serve_reset_stats": (C.c_int, [_P]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sigs)


def _check(st: int, where: str):
    if st != SAGE_OK:
        msg = _lib.sage_last_error()
        raise SageError(st, where, msg.decode() if msg else "")


def _host_ptr(a) -> int:
    arr = np.asarray(a)
    if not arr.flags["C_CONTIGUOUS"]:
        raise ValueError("host buffers must be C-contiguous")
    return arr.ctypes.data


def _nbytes(a) -> int:
    return np.asarray(a).nbytes


# ------------------------------------------------------------------ context
def sage_config_default() -> sage_config:
    cfg = sage_config()
    _lib.sage_config_default(C.byref(cfg))
    return cfg


def sage_open(device: int = 0, cfg: sage_config | None = None) -> int:
    h = _P()
    _check(_lib.sage_open(device, C.byref(cfg) if cfg is not None else None, C.byref(h)), "sage_open")
    return h.value


def sage_close(ctx: int) -> None:
    _check(_lib.sage_close(ctx), "sage_close")


def sage_last_error() -> str:
    m = _lib.sage_last_error()
    return m.decode() if m else ""


def sage_host_alloc(ctx: int, nbytes: int) -> int:
    p = _lib.sage_host_alloc(ctx, nbytes)
    if not p:
        raise SageError(SAGE_ENOMEM, "sage_host_alloc", sage_last_error())
    return p


def sage_host_free(ctx: int, p: int) -> None:
    _lib.sage_host_free(ctx, p)


def pinned_array(ctx: int, shape, dtype) -> np.ndarray:
    """numpy view of a sage_host_alloc buffer (freed with sage_host_free of
    ``arr.ctypes.data`` by the caller)."""
    dtype = np.dtype(dtype)
    n = int(np.prod(shape)) * dtype.itemsize
    p = sage_host_alloc(ctx, n)
    buf = (C.c_uint8 * n).from_address(p)
    return np.frombuffer(buf, dtype=dtype).reshape(shape)


# ------------------------------------------------------------------ functions
def make_blob(src, nbytes: int | None = None, where: int = SAGE_SRC_HOST, access: int = SAGE_RO,
              key: int = 0) -> sage_blob:
    """A blob from a host array (``where`` = host) or a device address (int)."""
    if where == SAGE_SRC_HOST and not isinstance(src, int):
        return sage_blob(_host_ptr(src), _nbytes(src) if nbytes is None else nbytes, access, where, key)
    return sage_blob(src, nbytes, access, where, key)


def fn_register(ctx: int, desc: sage_fn_desc, blobs) -> int:
    arr = (sage_blob * len(blobs))(*blobs)
    out = C.c_uint64()
    _check(_lib.fn_register(ctx, C.byref(desc), arr, len(blobs), C.byref(out)), "fn_register")
    return out.value


def fn_register_batch(ctx: int, descs, blob_lists):
    """Register len(descs) functions in one pipelined call; returns (handles,
    per-function registration ms)."""
    n = len(descs)
    if n != len(blob_lists):
        raise ValueError("one blob list per descriptor")
    darr = (sage_fn_desc * n)(*descs)
    barrs = [(sage_blob * len(b))(*b) for b in blob_lists]
    ptrs = (C.POINTER(sage_blob) * n)(*[C.cast(a, C.POINTER(sage_blob)) for a in barrs])
    counts = (C.c_size_t * n)(*[len(b) for b in blob_lists])
    out = (C.c_uint64 * n)()
    ms = (C.c_double * n)()
    _check(_lib.fn_register_batch(ctx, n, darr, ptrs, counts, out, ms), "fn_register_batch")
    return list(out), list(ms)


def fn_unregister(ctx: int, fn: int) -> None:
    _check(_lib.fn_unregister(ctx, fn), "fn_unregister")


def fn_setup(ctx: int, fn: int, batch: int) -> int:
    out = C.c_uint64()
    _check(_lib.fn_setup(ctx, fn, batch, C.byref(out)), "fn_setup")
    return out.value


def _io_ptr(x, device: bool) -> tuple:
    if device:
        if not isinstance(x, tuple):
            raise ValueError("device buffers are (address, nbytes) tuples")
        return int(x[0]), int(x[1])
    return _host_ptr(x), _nbytes(x)


def fn_invoke(ctx: int, inv: int, inp, out, io_flags: int = 0) -> None:
    """inp/out: numpy arrays for host I/O, or (address, nbytes) for device I/O."""
    ip, ib = _io_ptr(inp, bool(io_flags & SAGE_IO_DEVICE_IN))
    op, ob = _io_ptr(out, bool(io_flags & SAGE_IO_DEVICE_OUT))
    _check(_lib.fn_invoke(ctx, inv, ip, ib, op, ob, io_flags), "fn_invoke")


def fn_invoke_batch(ctx: int, invs, inputs, outputs, io_flags: int = 0) -> None:
    """invs: handles (a list, or a uint64 array); inputs/outputs: one entry per
    handle as for fn_invoke, or, for device I/O, a uint64 array of shape
    (n, 2) holding (address, nbytes) rows, marshalled without a Python loop."""
    n = len(invs)
    keep = []

    def u64(a):
        a = np.ascontiguousarray(a, dtype=np.uint64)
        keep.append(a)
        return a

    ids = u64(invs).ctypes.data_as(C.POINTER(C.c_uint64)) if isinstance(invs, np.ndarray) \
        else (C.c_uint64 * n)(*invs)

    def side(xs, device):
        if device and isinstance(xs, np.ndarray):
            if xs.shape != (n, 2):
                raise ValueError("device I/O array must have shape (n, 2)")
            return (u64(xs[:, 0]).ctypes.data_as(C.POINTER(_P)),
                    u64(xs[:, 1]).ctypes.data_as(C.POINTER(C.c_size_t)))
        pairs = [_io_ptr(x, device) for x in xs]
        return (_P * n)(*[p for p, _ in pairs]), (C.c_size_t * n)(*[b for _, b in pairs])

    ip, ib = side(inputs, bool(io_flags & SAGE_IO_DEVICE_IN))
    op, ob = side(outputs, bool(io_flags & SAGE_IO_DEVICE_OUT))
    _check(_lib.fn_invoke_batch(ctx, n, ids, ip, ib, op, ob, io_flags), "fn_invoke_batch")


def fn_invoke_noalloc(ctx: int, inv: int, inp, out) -> None:
    """inp/out: (device address, nbytes) tuples."""
    ip, ib = _io_ptr(inp, True)
    op, ob = _io_ptr(out, True)
    _check(_lib.fn_invoke_noalloc(ctx, inv, ip, ib, op, ob), "fn_invoke_noalloc")


def fn_release(ctx: int, inv: int) -> None:
    _check(_lib.fn_release(ctx, inv), "fn_release")


def fn_setup_batch(ctx: int, fns, batches, timed: bool = False):
    """Invocation handles; with timed=True also each request's own setup time
    (ms).  Given numpy arrays, returns numpy arrays (no Python loop)."""
    n = len(fns)
    if isinstance(fns, np.ndarray):
        f = np.ascontiguousarray(fns, dtype=np.uint64)
        b = np.ascontiguousarray(batches, dtype=np.uint32)
        out = np.zeros(n, dtype=np.uint64)
        ms = np.zeros(n, dtype=np.float64) if timed else None
        done = C.c_size_t()
        st = _lib.fn_setup_batch(ctx, n, f.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 b.ctypes.data_as(C.POINTER(C.c_uint32)), out.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 C.byref(done), ms.ctypes.data_as(C.POINTER(C.c_double)) if timed else None)
        _check(st, "fn_setup_batch")
        return (out, ms) if timed else out
    out = (C.c_uint64 * n)()
    done = C.c_size_t()
    ms = (C.c_double * n)() if timed else None
    st = _lib.fn_setup_batch(ctx, n, (C.c_uint64 * n)(*fns), (C.c_uint32 * n)(*batches), out, C.byref(done), ms)
    _check(st, "fn_setup_batch")
    return (list(out), list(ms)) if timed else list(out)


def fn_release_batch(ctx: int, invs) -> None:
    n = len(invs)
    if isinstance(invs, np.ndarray):
        a = np.ascontiguousarray(invs, dtype=np.uint64)
        _check(_lib.fn_release_batch(ctx, n, a.ctypes.data_as(C.POINTER(C.c_uint64))), "fn_release_batch")
        return
    _check(_lib.fn_release_batch(ctx, n, (C.c_uint64 * n)(*invs)), "fn_release_batch")


# ------------------------------------------------------------------ introspection
def sage_get_stats(ctx: int) -> dict:
    s = sage_stats()
    _check(_lib.sage_get_stats(ctx, C.byref(s)), "sage_get_stats")
    return s.as_dict()


def sage_fn_block_count(ctx: int, fn: int) -> int:
    n = C.c_size_t()
    _check(_lib.sage_fn_block_count(ctx, fn, C.byref(n)), "sage_fn_block_count")
    return n.value


def sage_fn_fingerprints(ctx: int, fn: int) -> np.ndarray:
    n = sage_fn_block_count(ctx, fn)
    out = np.zeros(n, dtype=np.uint64)
    _check(_lib.sage_fn_fingerprints(ctx, fn, out.ctypes.data_as(C.POINTER(C.c_uint64)), n),
           "sage_fn_fingerprints")
    return out


def sage_fn_block_info(ctx: int, fn: int):
    n = sage_fn_block_count(ctx, fn)
    cls = np.zeros(n, dtype=np.uint32)
    slot = np.zeros(n, dtype=np.uint32)
    refs = np.zeros(n, dtype=np.uint32)
    u32p = C.POINTER(C.c_uint32)
    _check(_lib.sage_fn_block_info(ctx, fn, cls.ctypes.data_as(u32p), slot.ctypes.data_as(u32p),
                                   refs.ctypes.data_as(u32p), n), "sage_fn_block_info")
    return cls, slot, refs


def sage_read_slot(ctx: int, slot: int) -> np.ndarray:
    out = np.zeros(BLOCK, dtype=np.uint8)
    _check(_lib.sage_read_slot(ctx, slot, out.ctypes.data), "sage_read_slot")
    return out


# ------------------------------------------------------------------ kernel entry points
def sage_fingerprint(ctx: int, dev: int, nbytes: int, dev_out: int, stream: int = 0) -> None:
    _check(_lib.sage_fingerprint(ctx, dev, nbytes, dev_out, stream or None), "sage_fingerprint")


def sage_blkcopy(ctx: int, dev_ops: int, n_ops: int, dev_result: int, stream: int = 0) -> None:
    _check(_lib.sage_blkcopy(ctx, dev_ops, n_ops, dev_result, stream or None), "sage_blkcopy")


# ------------------------------------------------------------------ timing
def sage_timing_enable(ctx: int, on: bool = True) -> None:
    _check(_lib.sage_timing_enable(ctx, 1 if on else 0), "sage_timing_enable")


def sage_timing_only(ctx: int, kernel: str | None = None) -> None:
    """Time only the launches of `kernel` (None: every kernel again)."""
    _check(_lib.sage_timing_only(ctx, kernel.encode() if kernel else None), "sage_timing_only")


def sage_timing_get(ctx: int, kernel: str):
    ms = C.c_double()
    n = C.c_uint64()
    _check(_lib.sage_timing_get(ctx, kernel.encode(), C.byref(ms), C.byref(n)), "sage_timing_get")
    return ms.value, n.value



def sage_mfma_ceiling(ctx: int, k: int, reps: int = 20):
    """(us per launch, shader GHz) of the main GEMM tile shape without its global loads."""
    us, ghz = C.c_double(), C.c_double()
    _check(_lib.sage_mfma_ceiling(ctx, k, reps, C.byref(us), C.byref(ghz)), "sage_mfma_ceiling")
    return us.value, ghz.value

def sage_timing_reset(ctx: int) -> None:
    _check(_lib.sage_timing_reset(ctx), "sage_timing_reset")


def sage_selftest_segments(first, layers: int, layer_bytes: int) -> list:
    """Per layer, the number of leading reload classes (ordered by first
    block) that layer's launch waits for; host only."""
    n = len(first)
    f = (C.c_uint32 * max(n, 1))(*first)
    out = (C.c_size_t * layers)()
    _check(_lib.sage_selftest_segments(f, n, layers, layer_bytes, out), "sage_selftest_segments")
    return list(out)


def sage_selftest_plan(width: int, rows, wave_ms: dict, cus: int = 256):
    """(plan text, predicted ms) of the BF16 launch planner for groups of
    `rows` under full-wave times `wave_ms` {shape: ms}; host only."""
    names = list(wave_ms)
    r = (C.c_uint32 * len(rows))(*rows)
    sh = (C.c_char_p * len(names))(*[n.encode() for n in names])
    ms = (C.c_double * len(names))(*[wave_ms[n] for n in names])
    buf = C.create_string_buffer(512)
    _check(_lib.sage_selftest_plan(width, r, len(rows), sh, ms, len(names), cus, buf, 512), "sage_selftest_plan")
    plan, cost = buf.value.decode().rsplit(" ", 1)
    return plan, float(cost)


def sage_tick(ctx: int) -> None:
    _check(_lib.sage_tick(ctx), "sage_tick")


def sage_last_launch(ctx: int) -> str:
    buf = C.create_string_buffer(512)
    _check(_lib.sage_last_launch(ctx, buf, 512), "sage_last_launch")
    return buf.value.decode()


def sage_selftest_setup_overlap(load_ms: float, host_ms: float, copy_ms: float, serial: bool) -> float:
    out = C.c_double()
    _check(_lib.sage_selftest_setup_overlap(load_ms, host_ms, copy_ms, 1 if serial else 0, C.byref(out)),
           "sage_selftest_setup_overlap")
    return out.value


# ------------------------------------------------------------------ serving
def sage_selftest_pool(seed: int, n_ops: int, budget_slots: int) -> int:
    """Operations run before the first failed invariant (n_ops: none failed);
    raises SageError with the reason on a failure."""
    at = C.c_uint32()
    _check(_lib.sage_selftest_pool(seed, n_ops, budget_slots, C.byref(at)), "sage_selftest_pool")
    return at.value


def sage_serve_start(ctx: int, max_rows: int = 0) -> None:
    _check(_lib.sage_serve_start(ctx, max_rows), "sage_serve_start")


def sage_serve_stop(ctx: int) -> None:
    _check(_lib.sage_serve_stop(ctx), "sage_serve_stop")


def sage_submit(ctx: int, fn: int, batch: int, inp, out, io_flags: int = 0) -> int:
    """Queue a request; host arrays must stay alive until sage_wait returns."""
    ip, ib = _io_ptr(inp, bool(io_flags & SAGE_IO_DEVICE_IN))
    op, ob = _io_ptr(out, bool(io_flags & SAGE_IO_DEVICE_OUT))
    rid = C.c_uint64()
    _check(_lib.sage_submit(ctx, fn, batch, ip, ib, op, ob, io_flags, C.byref(rid)), "sage_submit")
    return rid.value


def sage_wait(ctx: int, req_id: int, timeout_ms: float = -1.0) -> dict:
    info = sage_req_info()
    _check(_lib.sage_wait(ctx, req_id, timeout_ms, C.byref(info)), "sage_wait")
    return {"setup_ms": info.setup_ms, "e2e_ms": info.e2e_ms, "status": info.status}


def sage_serve_stats(ctx: int) -> dict:
    r = sage_serve_report()
    _check(_lib.sage_serve_stats(ctx, C.byref(r)), "sage_serve_stats")
    return r.as_dict()


def sage_serve_reset_stats(ctx: int) -> None:
    _check(_lib.sage_serve_reset_stats(ctx), "sage_serve_reset_stats")


# ------------------------------------------------------------------ descriptors
def mlp_desc(kind: int, layers: int, width: int) -> sage_fn_desc:
    return sage_fn_desc(kind=kind, layers=layers, width=width)


def stencil_desc(nx: int, ny: int, nz: int, sweeps: int) -> sage_fn_desc:
    return sage_fn_desc(kind=SAGE_STENCIL7_F32, nx=nx, ny=ny, nz=nz, sweeps=sweeps)


def relax_desc(nx: int, ny: int, nz: int, sweeps: int, coef: float) -> sage_fn_desc:
    return sage_fn_desc(kind=SAGE_RELAX7_F32, nx=nx, ny=ny, nz=nz, sweeps=sweeps, coef=coef)
