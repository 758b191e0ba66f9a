"""Python binding of libhx (include/hx.h): argument marshalling only.

Every function keeps the C name and signature shape; handles are plain ints,
argument structs are ctypes mirrors of the C structs, and a negative status
raises HxError carrying the context's last error message.  All computation
runs in the HIP kernels of libhx.so; importing this module without a built
library raises ImportError (there is no fallback).

torch is imported first: libhx links the HIP runtime that torch ships, and
loading torch first makes both use that one runtime instance.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import threading

import torch  # noqa: F401  (loads the HIP runtime libhx links against)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhx.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1810_11482_amd/build.py`")
lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants
HX_OK = 0
HX_PENDING = 1
HX_ERR_INVALID = -1
HX_ERR_ARG = -2
HX_ERR_NO_DEVICE = -3
HX_ERR_HIP = -4
HX_ERR_OOM = -5
HX_ERR_DEP_FAILED = -6
HX_ERR_TIMEOUT = -7
HX_ERR_INJECTED = -8
HX_ERR_HAZARD = -9
HX_ERR_UNSUPPORTED = -10
HX_ERR_RANGE = -11

HX_F32, HX_F64 = 0, 1
HX_H2D, HX_D2H, HX_D2D = 0, 1, 2
HX_BC_PERIODIC, HX_BC_DIRICHLET0, HX_BC_GHOST = 0, 1, 2

_u64 = ctypes.c_uint64
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
_vp = ctypes.c_void_p


# -------------------------------------------------------------------- structs
class hx_device_info_t(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("arch", ctypes.c_char * 64),
                ("compute_units", ctypes.c_int), ("wavefront_size", ctypes.c_int),
                ("clock_khz", ctypes.c_int), ("memory_clock_khz", ctypes.c_int),
                ("memory_bus_bits", ctypes.c_int), ("hbm_bytes", _sz),
                ("lds_bytes_per_cu", _sz), ("l2_bytes", _sz)]


class hx_ctx_opts(ctypes.Structure):
    _fields_ = [("compute_streams", ctypes.c_int), ("external_stream", _vp),
                ("check", ctypes.c_int), ("timing", ctypes.c_int)]


class hx_copy_desc(ctypes.Structure):
    _fields_ = [("dir", ctypes.c_int), ("host", _vp), ("buf", _u64), ("offset", _sz),
                ("src_buf", _u64), ("src_offset", _sz), ("bytes", _sz)]


class hx_stencil_args(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int), ("dtype", ctypes.c_int), ("nx", _i64), ("ny", _i64),
                ("steps", ctypes.c_int), ("r", ctypes.c_double),
                ("in_", _u64), ("in_offset", _sz), ("out", _u64), ("out_offset", _sz),
                ("tmp", _u64), ("tmp_offset", _sz),
                ("bc_lo", ctypes.c_int), ("bc_hi", ctypes.c_int),
                ("halo_lo", _u64), ("halo_lo_offset", _sz),
                ("halo_hi", _u64), ("halo_hi_offset", _sz),
                ("halo_width", ctypes.c_int),
                ("cells_per_lane", ctypes.c_int), ("time_block", ctypes.c_int),
                ("waves_per_group", ctypes.c_int), ("rows_per_block", ctypes.c_int)]


class hx_partitioned_desc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("parts", ctypes.c_int),
                ("sizes", ctypes.POINTER(_i64)), ("bufs_a", ctypes.POINTER(_u64)),
                ("bufs_b", ctypes.POINTER(_u64)), ("periodic", ctypes.c_int),
                ("steps", ctypes.c_int), ("r", ctypes.c_double), ("mode", ctypes.c_int),
                ("time_block", ctypes.c_int), ("cells_per_lane", ctypes.c_int),
                ("waves_per_group", ctypes.c_int), ("dims", ctypes.c_int), ("nx", _i64),
                ("rows_per_block", ctypes.c_int)]


class hx_pipeline_desc(ctypes.Structure):
    _fields_ = [("part", hx_partitioned_desc), ("host_in", _vp), ("host_out", _vp)]


HX_PART_GRAPH, HX_PART_PLAIN, HX_PART_BATCHED = 0, 1, 2
HX_BATCH_PERSISTENT, HX_BATCH_GRAPH, HX_BATCH_PLAIN = 0, 1, 2
HX_FORM_DIRECT, HX_FORM_PROPAGATOR, HX_FORM_AUTO = 0, 1, 2


class hx_segment(ctypes.Structure):
    _fields_ = [("in_", _u64), ("in_offset", _sz), ("out", _u64), ("out_offset", _sz),
                ("tmp", _u64), ("tmp_offset", _sz), ("n", _i64), ("r", ctypes.c_double),
                ("bc_lo", ctypes.c_int), ("bc_hi", ctypes.c_int),
                ("halo_lo", _u64), ("halo_lo_offset", _sz),
                ("halo_hi", _u64), ("halo_hi_offset", _sz), ("halo_width", ctypes.c_int)]


class hx_batch_desc(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("steps", ctypes.c_int), ("count", ctypes.c_int),
                ("segs", ctypes.POINTER(hx_segment)), ("mode", ctypes.c_int),
                ("cells_per_lane", ctypes.c_int), ("waves_per_group", ctypes.c_int),
                ("grid_waves_per_cu", ctypes.c_int), ("form", ctypes.c_int),
                ("span_blocks", ctypes.c_int)]


class hx_vc_args(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("nx", _i64), ("ny", _i64), ("dt", ctypes.c_double),
                ("steps", ctypes.c_int), ("ckpt", ctypes.c_int),
                ("u0", _u64), ("kappa", _u64), ("uT", _u64), ("ckpts", _u64), ("work", _u64),
                ("seg", _u64), ("lamT", _u64), ("lam0", _u64), ("gk64", _u64), ("gacc", _u64),
                ("rows_per_block", ctypes.c_int)]


class hx_kernel_arg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("access", ctypes.c_int32), ("buffer", ctypes.c_uint64),
                ("offset", ctypes.c_uint64), ("size", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("value", ctypes.c_uint8 * 16)]


class hx_halo_desc(ctypes.Structure):
    _fields_ = [("src", _u64), ("src_offset", _sz), ("dst", _u64), ("dst_offset", _sz),
                ("rows", _i64), ("row_bytes", _i64), ("src_pitch", _i64), ("dst_pitch", _i64)]


# ----------------------------------------------------------------- prototypes
_PROTOS = {
    "hx_status_string": (ctypes.c_char_p, [_i32]),
    "hx_device_count": (_i32, [ctypes.POINTER(ctypes.c_int)]),
    "hx_device_info": (_i32, [ctypes.c_int, ctypes.POINTER(hx_device_info_t)]),
    "hx_ctx_create": (_i32, [ctypes.c_int, ctypes.POINTER(hx_ctx_opts), ctypes.POINTER(_vp)]),
    "hx_ctx_destroy": (_i32, [_vp]),
    "hx_ctx_synchronize": (_i32, [_vp]),
    "hx_last_error": (_i32, [_vp, ctypes.c_char_p, _sz]),
    "hx_buffer_create": (_i32, [_vp, _sz, ctypes.POINTER(_u64)]),
    "hx_buffer_wrap": (_i32, [_vp, _vp, _sz, ctypes.POINTER(_u64)]),
    "hx_buffer_destroy": (_i32, [_vp, _u64]),
    "hx_buffer_ptr": (_i32, [_vp, _u64, ctypes.POINTER(_vp), ctypes.POINTER(_sz)]),
    "hx_host_alloc": (_i32, [_vp, _sz, ctypes.POINTER(_vp)]),
    "hx_host_free": (_i32, [_vp, _vp]),
    "hx_copy_async": (_i32, [_vp, ctypes.POINTER(hx_copy_desc), ctypes.POINTER(_u64),
                             ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_launch_stencil": (_i32, [_vp, ctypes.POINTER(hx_stencil_args), ctypes.POINTER(_u64),
                                 ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_when_all": (_i32, [_vp, ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_plan_create_batched": (_i32, [_vp, ctypes.POINTER(hx_batch_desc), ctypes.POINTER(_u64)]),
    "hx_propagator_coefficients": (_i32, [ctypes.c_double, ctypes.c_int,
                                          ctypes.POINTER(ctypes.c_double)]),
    "hx_launch_batched": (_i32, [_vp, _u64, ctypes.POINTER(_u64), ctypes.c_int,
                                 ctypes.POINTER(_u64)]),
    "hx_plan_destroy": (_i32, [_vp, _u64]),
    "hx_graph_begin": (_i32, [_vp]),
    "hx_graph_end": (_i32, [_vp, ctypes.POINTER(_u64)]),
    "hx_graph_launch": (_i32, [_vp, _u64, ctypes.POINTER(_u64), ctypes.c_int,
                               ctypes.POINTER(_u64)]),
    "hx_graph_info": (_i32, [_vp, _u64, ctypes.POINTER(ctypes.c_int64)]),
    "hx_plan_create_halo": (_i32, [_vp, ctypes.POINTER(hx_halo_desc), ctypes.c_int,
                                   ctypes.POINTER(_u64)]),
    "hx_launch_halo": (_i32, [_vp, _u64, ctypes.POINTER(_u64), ctypes.c_int,
                              ctypes.POINTER(_u64)]),
    "hx_heat_vc_step": (_i32, [_vp, ctypes.c_int, _i64, _i64, ctypes.c_double, _u64, _u64, _u64,
                               ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_heat_vc_adjoint_step": (_i32, [_vp, ctypes.c_int, _i64, _i64, ctypes.c_double, _u64,
                                       _u64, _u64, _u64, _u64, ctypes.POINTER(_u64),
                                       ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_vc_schedule": (_i32, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int)]),
    "hx_heat_vc_forward": (_i32, [_vp, ctypes.POINTER(hx_vc_args), ctypes.POINTER(_u64),
                                  ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_heat_vc_backward": (_i32, [_vp, ctypes.POINTER(hx_vc_args), ctypes.POINTER(_u64),
                                   ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_launch_loss": (_i32, [_vp, ctypes.c_int, _i64, _u64, _u64, _u64, _u64, _u64,
                              ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_launch_loss_noalloc": (_i32, [_vp, ctypes.c_int, _i64, _u64, _u64, _u64, _u64,
                                      ctypes.POINTER(_u64), ctypes.c_int,
                                      ctypes.POINTER(_u64)]),
    "hx_launch_dot": (_i32, [_vp, ctypes.c_int, _i64, _u64, _u64, _u64, _u64,
                             ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_launch_scale": (_i32, [_vp, ctypes.c_int, _i64, _u64, _u64, _u64,
                               ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_launch_cast64": (_i32, [_vp, ctypes.c_int, _i64, _u64, _u64,
                                ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_run_partitioned": (_i32, [_vp, ctypes.POINTER(hx_partitioned_desc), ctypes.POINTER(_u64),
                                  ctypes.c_int, ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(_u64)]),
    "hx_run_pipeline": (_i32, [_vp, ctypes.POINTER(hx_pipeline_desc), ctypes.POINTER(_u64),
                               ctypes.c_int, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "hx_wait": (_i32, [_vp, _u64, _i64]),
    "hx_event_query": (_i32, [_vp, _u64, ctypes.POINTER(_i32)]),
    "hx_event_release": (_i32, [_vp, _u64]),
    "hx_event_elapsed": (_i32, [_vp, _u64, _u64, ctypes.POINTER(ctypes.c_double)]),
    "hx_event_span": (_i32, [_vp, _u64, _u64, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)]),
    "hx_user_event_create": (_i32, [_vp, ctypes.POINTER(_u64)]),
    "hx_user_event_set": (_i32, [_vp, _u64, _i32]),
    "hx_event_record_stream": (_i32, [_vp, _vp, ctypes.POINTER(_u64)]),
    "hx_host_task": (_i32, [_vp, ctypes.c_void_p, _vp, ctypes.POINTER(_u64), ctypes.c_int,
                            ctypes.POINTER(_u64)]),
    "hx_stream_wait_event": (_i32, [_vp, _vp, _u64]),
    "hx_debug_next_seq": (_i32, [_vp, ctypes.POINTER(_u64)]),
    "hx_debug_inject": (_i32, [_vp, _u64]),
    "hx_hazard_count": (_i32, [_vp, ctypes.POINTER(_i64)]),
    "hx_hazard_report": (_i32, [_vp, ctypes.c_char_p, _sz]),
    "hx_tune_cache_save": (_i32, [ctypes.c_char_p]),
    "hx_tune_stencil": (_i32, [_vp, ctypes.POINTER(hx_stencil_args), ctypes.c_int,
                               ctypes.POINTER(hx_stencil_args)]),
    "hx_tune_batched": (_i32, [_vp, ctypes.POINTER(hx_batch_desc), ctypes.c_int,
                               ctypes.POINTER(hx_batch_desc)]),
    "hx_tune_cache_clear": (_i32, []),
    "hx_program_create": (_i32, [_vp, ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_u64)]),
    "hx_program_build": (_i32, [_vp, _u64, ctypes.POINTER(ctypes.c_char_p), ctypes.c_int]),
    "hx_program_log": (_i32, [_vp, _u64, ctypes.c_char_p, _sz, ctypes.POINTER(_sz)]),
    "hx_program_run": (_i32, [_vp, _u64, ctypes.c_char_p, ctypes.POINTER(hx_kernel_arg),
                              ctypes.c_int, ctypes.POINTER(ctypes.c_uint32),
                              ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32,
                              ctypes.POINTER(_u64), ctypes.c_int, ctypes.POINTER(_u64)]),
    "hx_program_function": (_i32, [_vp, _u64, ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "hx_program_destroy": (_i32, [_vp, _u64]),
}
for _name, (_res, _args) in _PROTOS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class HxError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{hx_status_string(status)}: {msg}" if msg else hx_status_string(status))


def hx_status_string(s: int) -> str:
    return lib.hx_status_string(s).decode()


def _err(ctx, s: int):
    msg = ""
    if ctx:
        buf = ctypes.create_string_buffer(1024)
        if lib.hx_last_error(ctx, buf, 1024) == 0:
            msg = buf.value.decode(errors="replace")
    raise HxError(s, msg)


def _ok(ctx, s: int) -> None:
    if s < 0:
        _err(ctx, s)


def _deps(deps):
    deps = [int(d) for d in (deps or []) if d]
    arr = (_u64 * max(1, len(deps)))(*deps)
    return arr, len(deps)


# ------------------------------------------------------------------ functions
def hx_device_count() -> int:
    n = ctypes.c_int()
    _ok(None, lib.hx_device_count(ctypes.byref(n)))
    return n.value


def hx_device_info(dev: int = 0) -> hx_device_info_t:
    info = hx_device_info_t()
    _ok(None, lib.hx_device_info(dev, ctypes.byref(info)))
    return info


def hx_ctx_create(dev: int = 0, compute_streams: int = 0, external_stream=None, check=False,
                  timing=False):
    opts = hx_ctx_opts(compute_streams, external_stream, int(bool(check)), int(bool(timing)))
    ctx = _vp()
    _ok(None, lib.hx_ctx_create(dev, ctypes.byref(opts), ctypes.byref(ctx)))
    return ctx


def hx_ctx_destroy(ctx) -> None:
    _ok(None, lib.hx_ctx_destroy(ctx))


def hx_ctx_synchronize(ctx) -> None:
    _ok(ctx, lib.hx_ctx_synchronize(ctx))


def hx_last_error(ctx) -> str:
    buf = ctypes.create_string_buffer(4096)
    _ok(None, lib.hx_last_error(ctx, buf, 4096))
    return buf.value.decode(errors="replace")


def hx_buffer_create(ctx, nbytes: int) -> int:
    h = _u64()
    _ok(ctx, lib.hx_buffer_create(ctx, nbytes, ctypes.byref(h)))
    return h.value


def hx_buffer_wrap(ctx, dev_ptr: int, nbytes: int) -> int:
    h = _u64()
    _ok(ctx, lib.hx_buffer_wrap(ctx, dev_ptr, nbytes, ctypes.byref(h)))
    return h.value


def hx_buffer_destroy(ctx, buf: int) -> None:
    _ok(ctx, lib.hx_buffer_destroy(ctx, buf))


def hx_buffer_ptr(ctx, buf: int):
    p, n = _vp(), _sz()
    _ok(ctx, lib.hx_buffer_ptr(ctx, buf, ctypes.byref(p), ctypes.byref(n)))
    return p.value or 0, n.value


def hx_host_alloc(ctx, nbytes: int) -> int:
    p = _vp()
    _ok(ctx, lib.hx_host_alloc(ctx, nbytes, ctypes.byref(p)))
    return p.value


def hx_host_free(ctx, ptr: int) -> None:
    _ok(ctx, lib.hx_host_free(ctx, ptr))


def hx_copy_async(ctx, desc: hx_copy_desc, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_copy_async(ctx, ctypes.byref(desc), arr, n, ctypes.byref(ev)))
    return ev.value


def hx_launch_stencil(ctx, args: hx_stencil_args, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_launch_stencil(ctx, ctypes.byref(args), arr, n, ctypes.byref(ev)))
    return ev.value


def partitioned_desc(dtype, sizes, bufs_a, bufs_b, steps, r, periodic=True,
                     mode=HX_PART_GRAPH, time_block=0, cells_per_lane=0, waves_per_group=0,
                     dims=1, nx=0, rows_per_block=0):
    """hx_partitioned_desc; the host arrays are kept alive on the returned struct.
    2D: dims=2, nx = row length, sizes = rows per band, periodic must be False."""
    P = len(sizes)
    sz = (_i64 * P)(*[int(x) for x in sizes])
    ba = (_u64 * P)(*[int(x) for x in bufs_a])
    bb = (_u64 * P)(*[int(x) for x in bufs_b])
    d = hx_partitioned_desc(dtype, P, sz, ba, bb, int(bool(periodic)), steps, r, mode,
                            time_block, cells_per_lane, waves_per_group, dims, nx, rows_per_block)
    d._keep = (sz, ba, bb)
    return d


def hx_run_partitioned(ctx, desc: hx_partitioned_desc, deps=(), node_events=False):
    """Returns (event, final_in_b, node_event_list or None)."""
    arr, n = _deps(deps)
    ev = _u64()
    fb = ctypes.c_int()
    nodes = None
    if node_events:
        D = desc.time_block or min(desc.steps, 8 if desc.dims == 2 else 32)
        if desc.mode == HX_PART_PLAIN:
            D = 1
        passes = 0 if desc.steps == 0 else -(-desc.steps // D)
        nodes = (_u64 * max(1, passes * desc.parts))()
    _ok(ctx, lib.hx_run_partitioned(ctx, ctypes.byref(desc), arr, n, ctypes.byref(ev),
                                    ctypes.byref(fb), nodes))
    return ev.value, bool(fb.value), (list(nodes) if nodes is not None else None)


def hx_run_pipeline(ctx, desc: hx_pipeline_desc, deps=(), op_events=False):
    """Returns (event, [h2d events], [kernel events], [d2h events]) (lists None
    unless op_events)."""
    arr, n = _deps(deps)
    ev = _u64()
    P = desc.part.parts
    ops = (_u64 * (3 * P))() if op_events else None
    _ok(ctx, lib.hx_run_pipeline(ctx, ctypes.byref(desc), arr, n, ctypes.byref(ev), ops))
    if ops is None:
        return ev.value, None, None, None
    o = list(ops)
    return ev.value, o[:P], o[P:2 * P], o[2 * P:]


def hx_plan_create_batched(ctx, dtype, steps, segs, mode=HX_BATCH_PERSISTENT,
                           cells_per_lane=0, waves_per_group=0, grid_waves_per_cu=0,
                           form=HX_FORM_DIRECT, span_blocks=0) -> int:
    """segs: a list of hx_segment."""
    arr = (hx_segment * len(segs))(*segs)
    d = hx_batch_desc(dtype, steps, len(segs), arr, mode, cells_per_lane, waves_per_group,
                      grid_waves_per_cu, form, span_blocks)
    h = _u64()
    _ok(ctx, lib.hx_plan_create_batched(ctx, ctypes.byref(d), ctypes.byref(h)))
    return h.value


def hx_launch_batched(ctx, plan: int, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_launch_batched(ctx, plan, arr, n, ctypes.byref(ev)))
    return ev.value


def hx_plan_destroy(ctx, plan: int) -> None:
    _ok(ctx, lib.hx_plan_destroy(ctx, plan))


def hx_graph_begin(ctx) -> None:
    _ok(ctx, lib.hx_graph_begin(ctx))


def hx_graph_end(ctx) -> int:
    g = _u64()
    _ok(ctx, lib.hx_graph_end(ctx, ctypes.byref(g)))
    return g.value


def hx_graph_launch(ctx, graph: int, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_graph_launch(ctx, graph, arr, n, ctypes.byref(ev)))
    return ev.value


def hx_graph_info(ctx, graph: int) -> int:
    n = ctypes.c_int64()
    _ok(ctx, lib.hx_graph_info(ctx, graph, ctypes.byref(n)))
    return n.value


def hx_plan_create_halo(ctx, descs) -> int:
    arr = (hx_halo_desc * len(descs))(*descs)
    h = _u64()
    _ok(ctx, lib.hx_plan_create_halo(ctx, arr, len(descs), ctypes.byref(h)))
    return h.value


def hx_launch_halo(ctx, plan: int, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_launch_halo(ctx, plan, arr, n, ctypes.byref(ev)))
    return ev.value


HX_ARG_BUFFER, HX_ARG_VALUE = 0, 1
HX_ACCESS_READ, HX_ACCESS_WRITE = 1, 2


def karg_buffer(buf: int, offset: int = 0, access: int = HX_ACCESS_READ | HX_ACCESS_WRITE):
    """A buffer kernel argument: the device address of buf + offset."""
    a = hx_kernel_arg()
    a.kind, a.access, a.buffer, a.offset = HX_ARG_BUFFER, access, buf, offset
    return a


def karg_value(x):
    """A value kernel argument from a numpy scalar (its dtype is the parameter's type)."""
    import numpy as np
    x = np.asarray(x)
    if x.ndim != 0 or x.nbytes > 16:
        raise ValueError("a value argument is a numpy scalar of at most 16 bytes")
    a = hx_kernel_arg()
    a.kind, a.size = HX_ARG_VALUE, x.nbytes
    ctypes.memmove(a.value, x.tobytes(), x.nbytes)
    return a


def hx_program_create(ctx, source: str, name: str = "program.hip") -> int:
    h = _u64()
    _ok(ctx, lib.hx_program_create(ctx, source.encode(), name.encode(), ctypes.byref(h)))
    return h.value


def hx_program_log(ctx, prog: int) -> str:
    need = _sz()
    _ok(ctx, lib.hx_program_log(ctx, prog, None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(max(1, need.value))
    _ok(ctx, lib.hx_program_log(ctx, prog, buf, need.value, None))
    return buf.value.decode(errors="replace")


def hx_program_build(ctx, prog: int, options=()) -> None:
    opts = [o.encode() for o in options]
    arr = (ctypes.c_char_p * max(1, len(opts)))(*opts)
    s = lib.hx_program_build(ctx, prog, arr, len(opts))
    if s < 0:
        raise HxError(s, hx_program_log(ctx, prog))


def hx_program_run(ctx, prog: int, kernel: str, args, grid, block, shared_bytes: int = 0,
                   deps=()) -> int:
    """args: hx_kernel_arg values (karg_buffer / karg_value); grid, block: 1-3 ints."""
    a = (hx_kernel_arg * max(1, len(args)))(*args)
    g = (ctypes.c_uint32 * 3)(*(list(grid) + [1, 1, 1])[:3])
    b = (ctypes.c_uint32 * 3)(*(list(block) + [1, 1, 1])[:3])
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_program_run(ctx, prog, kernel.encode(), a, len(args), g, b, shared_bytes, arr,
                                n, ctypes.byref(ev)))
    return ev.value


def hx_program_function(ctx, prog: int, kernel: str) -> int:
    f = _vp()
    _ok(ctx, lib.hx_program_function(ctx, prog, kernel.encode(), ctypes.byref(f)))
    return f.value or 0


def hx_program_destroy(ctx, prog: int) -> None:
    _ok(ctx, lib.hx_program_destroy(ctx, prog))


def segment(**kw) -> hx_segment:
    if "inp" in kw:
        kw["in_"] = kw.pop("inp")
    s = hx_segment()
    for k, v in kw.items():
        if not hasattr(s, k):
            raise TypeError(f"hx_segment has no field {k}")
        setattr(s, k, v)
    return s


def _op(ctx, fn, *args, deps=()):
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, fn(ctx, *args, arr, n, ctypes.byref(ev)))
    return ev.value


def hx_heat_vc_step(ctx, dtype, nx, ny, dt, u, kappa, out_buf, deps=()) -> int:
    return _op(ctx, lib.hx_heat_vc_step, dtype, nx, ny, dt, u, kappa, out_buf, deps=deps)


def hx_heat_vc_adjoint_step(ctx, dtype, nx, ny, dt, u_t, lam_next, kappa, lam_out, gacc,
                            deps=()) -> int:
    return _op(ctx, lib.hx_heat_vc_adjoint_step, dtype, nx, ny, dt, u_t, lam_next, kappa,
               lam_out, gacc, deps=deps)


def hx_vc_schedule(steps: int, ckpt: int = 0):
    S, n = ctypes.c_int(), ctypes.c_int()
    _ok(None, lib.hx_vc_schedule(steps, ckpt, ctypes.byref(S), ctypes.byref(n)))
    return S.value, n.value


def hx_heat_vc_forward(ctx, args: hx_vc_args, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_heat_vc_forward(ctx, ctypes.byref(args), arr, n, ctypes.byref(ev)))
    return ev.value


def hx_heat_vc_backward(ctx, args: hx_vc_args, deps=()) -> int:
    arr, n = _deps(deps)
    ev = _u64()
    _ok(ctx, lib.hx_heat_vc_backward(ctx, ctypes.byref(args), arr, n, ctypes.byref(ev)))
    return ev.value


def hx_launch_loss(ctx, dtype, n, u, y, resid, out64, work, deps=()) -> int:
    return _op(ctx, lib.hx_launch_loss, dtype, n, u, y, resid, out64, work, deps=deps)


def hx_launch_loss_noalloc(ctx, dtype, n, u, y, resid, out64, deps=()) -> int:
    return _op(ctx, lib.hx_launch_loss_noalloc, dtype, n, u, y, resid, out64, deps=deps)


def hx_launch_dot(ctx, dtype, n, a, b, out64, work, deps=()) -> int:
    return _op(ctx, lib.hx_launch_dot, dtype, n, a, b, out64, work, deps=deps)


def hx_launch_scale(ctx, dtype, n, x, s64, y, deps=()) -> int:
    return _op(ctx, lib.hx_launch_scale, dtype, n, x, s64, y, deps=deps)


def hx_launch_cast64(ctx, dtype, n, src64, dst, deps=()) -> int:
    return _op(ctx, lib.hx_launch_cast64, dtype, n, src64, dst, deps=deps)


def hx_when_all(ctx, events) -> int:
    evs = [int(e) for e in events]
    arr = (_u64 * max(1, len(evs)))(*evs)
    ev = _u64()
    _ok(ctx, lib.hx_when_all(ctx, arr, len(evs), ctypes.byref(ev)))
    return ev.value


def hx_wait(ctx, ev: int, timeout_ns: int = -1) -> int:
    """Returns the event's final status (or HX_ERR_TIMEOUT); raises only for an
    invalid handle."""
    s = lib.hx_wait(ctx, ev, timeout_ns)
    if s == HX_ERR_INVALID:
        _err(ctx, s)
    return s


def hx_event_query(ctx, ev: int) -> int:
    st = _i32()
    _ok(ctx, lib.hx_event_query(ctx, ev, ctypes.byref(st)))
    return st.value


def hx_event_release(ctx, ev: int) -> None:
    _ok(ctx, lib.hx_event_release(ctx, ev))


def hx_event_elapsed(ctx, start: int, stop: int) -> float:
    ms = ctypes.c_double()
    _ok(ctx, lib.hx_event_elapsed(ctx, start, stop, ctypes.byref(ms)))
    return ms.value


def hx_event_span(ctx, ev: int, ref: int):
    a, b = ctypes.c_double(), ctypes.c_double()
    _ok(ctx, lib.hx_event_span(ctx, ev, ref, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def hx_user_event_create(ctx) -> int:
    ev = _u64()
    _ok(ctx, lib.hx_user_event_create(ctx, ctypes.byref(ev)))
    return ev.value


def hx_user_event_set(ctx, ev: int, status: int = HX_OK) -> None:
    _ok(ctx, lib.hx_user_event_set(ctx, ev, status))


_HOST_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p)
_host_live = {}      # callback objects of tasks that have not run yet
_host_done = []      # callbacks that have returned (freed on a later call)
_host_lock = threading.Lock()
_host_ids = itertools.count(1)


def hx_host_task(ctx, fn, deps=()) -> int:
    """Run the Python callable `fn()` on the context's host worker once `deps`
    complete; its return value (None = HX_OK, or an hx status) completes the
    event; an exception completes it with HX_ERR_ARG."""
    key = next(_host_ids)

    def trampoline(_user):
        try:
            r = fn()
            return HX_OK if r is None else int(r)
        except Exception:  # noqa: BLE001 - the status carries the failure
            return HX_ERR_ARG
        finally:
            with _host_lock:
                cb = _host_live.pop(key, None)
                if cb is not None:
                    _host_done.append(cb)

    cb = _HOST_FN(trampoline)
    with _host_lock:
        _host_live[key] = cb
        del _host_done[:-64]  # keep the most recent ones: they may still be returning
    arr, n = _deps(deps)
    ev = _u64()
    st = lib.hx_host_task(ctx, ctypes.cast(cb, ctypes.c_void_p), None, arr, n, ctypes.byref(ev))
    if st < 0:
        with _host_lock:
            _host_live.pop(key, None)
        _err(ctx, st)
    return ev.value


def hx_event_record_stream(ctx, hip_stream: int) -> int:
    ev = _u64()
    _ok(ctx, lib.hx_event_record_stream(ctx, hip_stream, ctypes.byref(ev)))
    return ev.value


def hx_stream_wait_event(ctx, hip_stream: int, ev: int) -> None:
    _ok(ctx, lib.hx_stream_wait_event(ctx, hip_stream, ev))


def hx_debug_next_seq(ctx) -> int:
    s = _u64()
    _ok(ctx, lib.hx_debug_next_seq(ctx, ctypes.byref(s)))
    return s.value


def hx_debug_inject(ctx, seq: int) -> None:
    _ok(ctx, lib.hx_debug_inject(ctx, seq))


def hx_hazard_count(ctx) -> int:
    n = _i64()
    _ok(ctx, lib.hx_hazard_count(ctx, ctypes.byref(n)))
    return n.value


def hx_hazard_report(ctx) -> str:
    buf = ctypes.create_string_buffer(65536)
    _ok(ctx, lib.hx_hazard_report(ctx, buf, 65536))
    return buf.value.decode(errors="replace")


def hx_tune_stencil(ctx, args: hx_stencil_args, budget_ms: int = 2000) -> hx_stencil_args:
    best = hx_stencil_args()
    _ok(ctx, lib.hx_tune_stencil(ctx, ctypes.byref(args), budget_ms, ctypes.byref(best)))
    return best


def hx_tune_batched(ctx, dtype, steps, segs, budget_ms: int = 2000) -> hx_batch_desc:
    arr = (hx_segment * len(segs))(*segs)
    d = hx_batch_desc(dtype, steps, len(segs), arr, HX_BATCH_PERSISTENT, 0, 0, 0)
    best = hx_batch_desc()
    _ok(ctx, lib.hx_tune_batched(ctx, ctypes.byref(d), budget_ms, ctypes.byref(best)))
    best._keep = arr
    return best


def hx_propagator_coefficients(r: float, steps: int) -> "np.ndarray":
    """The steps-step propagator taps p_{-steps}..p_{steps} (FP64)."""
    import numpy as np
    if int(steps) < 0:
        raise HxError(HX_ERR_ARG, "steps must be >= 0")
    out = np.empty(2 * steps + 1, dtype=np.float64)
    st = lib.hx_propagator_coefficients(float(r), int(steps),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _ok(None, st)
    return out


def hx_tune_cache_save(path: str) -> None:
    _ok(None, lib.hx_tune_cache_save(path.encode()))


def hx_tune_cache_clear() -> None:
    _ok(None, lib.hx_tune_cache_clear())


def stencil_args(**kw) -> hx_stencil_args:
    """hx_stencil_args with keyword fields (`in_` may be given as `inp`)."""
    if "inp" in kw:
        kw["in_"] = kw.pop("inp")
    a = hx_stencil_args()
    a.dims = 1
    a.ny = 1
    for k, v in kw.items():
        if not hasattr(a, k):
            raise TypeError(f"hx_stencil_args has no field {k}")
        setattr(a, k, v)
    return a
