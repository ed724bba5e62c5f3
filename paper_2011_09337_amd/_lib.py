"""ctypes binding of libvit.so, the C ABI declared in include/vit.h.

Argument marshalling only: every step of the decode runs in the HIP kernels.
The functions keep the C names; `vit_decode` and `vit_decode_ex` take raw
device addresses (ints) exactly like the C ABI.  If the library is missing
this module raises on import: there is no fallback.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvit.so")

VIT_OK = 0
VIT_EINVAL = -1
VIT_EUNSUPPORTED = -2
VIT_ENOMEM = -3
VIT_EDEVICE = -4
VIT_EBUSY = -5
VIT_ETIMEDOUT = -6
VIT_TIE_LOWER_PRED = 0
VIT_SUBFRAME_STORED = 0
VIT_SUBFRAME_RANDOM = 1
VIT_LLR_F32 = 0
VIT_LLR_I8 = 1
VIT_LLR_HARD = 2
VIT_STATIC_BATCH_MAX_ITEMS = 262144
VIT_STATIC_BATCH_MAX_FRAMES = 65536
VIT_STATIC_BATCH_MAX_STAGES = 65536

STATUS_NAMES = {VIT_OK: "VIT_OK", VIT_EINVAL: "VIT_EINVAL", VIT_EUNSUPPORTED: "VIT_EUNSUPPORTED",
                VIT_ENOMEM: "VIT_ENOMEM", VIT_EDEVICE: "VIT_EDEVICE", VIT_EBUSY: "VIT_EBUSY",
                VIT_ETIMEDOUT: "VIT_ETIMEDOUT"}


class vit_code(C.Structure):
    _fields_ = [("k", C.c_int32), ("beta", C.c_int32), ("gen", C.c_uint32 * 4)]


class vit_opts(C.Structure):
    _fields_ = [("size", C.c_uint32), ("llr_type", C.c_int32), ("terminated", C.c_int32),
                ("v1", C.c_int32), ("check_finite", C.c_int32), ("reserved", C.c_int32),
                ("stream", C.c_void_p), ("subframe_bits", C.c_int32), ("subframe_overlap", C.c_int32),
                ("subframe_start", C.c_int32), ("metric_bits", C.c_int32), ("subframe_seed", C.c_uint64)]


class vit_tuning_entry(C.Structure):
    _fields_ = [("code", vit_code), ("llr_type", C.c_int32), ("length_bucket", C.c_int32),
                ("L", C.c_int32), ("v", C.c_int32), ("v1", C.c_int32), ("waves_per_block", C.c_int32)]


class vit_geometry(C.Structure):
    _fields_ = [("n_stages", C.c_int64), ("n_blocks", C.c_int64), ("v1", C.c_int64), ("v2", C.c_int64),
                ("stages_total", C.c_int64), ("max_block_stages", C.c_int64),
                ("lds_bytes_per_block", C.c_int64)]


class vit_frame(C.Structure):
    _fields_ = [("code_id", C.c_int32), ("terminated", C.c_int32), ("n", C.c_int64), ("llr_off", C.c_int64),
                ("out_off", C.c_int64)]


class vit_tuning(C.Structure):
    _fields_ = [("L", C.c_int32), ("v", C.c_int32), ("v1", C.c_int32), ("waves_per_block", C.c_int32)]


class vit_server_config(C.Structure):
    _fields_ = [("size", C.c_uint32), ("llr_type", C.c_int32), ("max_frames", C.c_int32),
                ("max_items", C.c_int32), ("max_pending", C.c_int32), ("max_wait_ms", C.c_int32),
                ("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("host", C.c_void_p), ("host_bytes", C.c_size_t),
                ("stream", C.c_void_p), ("metric_bits", C.c_int32), ("reserved", C.c_int32)]


class vit_request(C.Structure):
    _fields_ = [("code_id", C.c_int32), ("terminated", C.c_int32), ("n", C.c_int64), ("llr", C.c_void_p),
                ("out", C.c_void_p), ("tag", C.c_uint64), ("arrival_ns", C.c_int64)]


class vit_completion(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("reserved", C.c_int32), ("arrival_ns", C.c_int64),
                ("done_ns", C.c_int64)]


class vit_serve_stats(C.Structure):
    _fields_ = [(name, C.c_int64) for name in (
        "submitted", "completed", "failed", "bits_completed", "iterations", "items_launched", "pending",
        "frames_on_device", "peak_frames_on_device", "peak_arena_bytes", "first_arrival_ns", "last_done_ns",
        "p50_ns", "p99_ns", "max_ns", "iter_ingest_ns", "iter_decode_ns", "iter_max_ns", "admit_wait_ns",
        "admit_wait_max_ns", "submit_lag_ns", "submit_lag_max_ns", "submit_lag_count", "engine_host_ns")]


class VitError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")

lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
lib.vit_decode.argtypes = [C.POINTER(vit_code), _P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _P]
lib.vit_decode.restype = C.c_int
lib.vit_decode_ex.argtypes = [C.POINTER(vit_code), _P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _P,
                              C.POINTER(vit_opts)]
lib.vit_decode_ex.restype = C.c_int
lib.vit_opts_default.argtypes = []
lib.vit_opts_default.restype = vit_opts
lib.vit_query_geometry.argtypes = [C.POINTER(vit_code), C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.POINTER(vit_geometry)]
lib.vit_query_geometry.restype = C.c_int
lib.vit_quantize_i8.argtypes = [_P, C.c_int64, C.c_float, _P, _P]
lib.vit_depuncture.argtypes = [_P, C.c_int64, C.c_int32, _P, C.c_int32, C.c_int32, C.c_int64, _P, _P]
lib.vit_depuncture.restype = C.c_int
lib.vit_quantize_i8.restype = C.c_int
_PC = C.POINTER(vit_code)
_PF = C.POINTER(vit_frame)
_PT = C.POINTER(vit_tuning)
lib.vit_plan_create.argtypes = [C.POINTER(C.c_void_p)]
lib.vit_plan_create.restype = C.c_int
lib.vit_plan_set_metric_bits.argtypes = [C.c_void_p, C.c_int32]
lib.vit_plan_set_metric_bits.restype = C.c_int
lib.vit_plan_set_tune_tolerance.argtypes = [C.c_void_p, C.c_double]
lib.vit_plan_set_tune_tolerance.restype = C.c_int
lib.vit_plan_destroy.argtypes = [C.c_void_p]
lib.vit_plan_destroy.restype = None
lib.vit_batch_workspace_size.argtypes = [_PC, C.c_int32, _PF, C.c_int32, _PT, C.POINTER(C.c_size_t)]
lib.vit_batch_workspace_size.restype = C.c_int
lib.vit_decode_batch.argtypes = [C.c_void_p, _PC, C.c_int32, _PF, C.c_int32, _P, C.c_int64, C.c_int32, _P,
                                 C.c_int64, _PT, _P, C.c_size_t, _P]
lib.vit_decode_batch.restype = C.c_int
lib.vit_decode_batch_static.argtypes = [_PC, C.c_int32, _PF, C.c_int32, _P, C.c_int64, C.c_int32, _P, C.c_int64,
                                        _PT, _P]
lib.vit_decode_batch_static.restype = C.c_int
lib.vit_plan_autotune.argtypes = [C.c_void_p, _PC, C.c_int32, _PF, C.c_int32, _P, C.c_int64, C.c_int32, _P,
                                  C.c_int64, _P, C.c_size_t, _P, _PT]
lib.vit_plan_autotune.restype = C.c_int
_PS = C.POINTER(vit_server_config)
lib.vit_server_workspace_size.argtypes = [_PS, C.POINTER(C.c_size_t)]
lib.vit_server_workspace_size.restype = C.c_int
lib.vit_server_create.argtypes = [_PC, C.c_int32, _PT, _PS, C.POINTER(C.c_void_p)]
lib.vit_server_create.restype = C.c_int
lib.vit_server_submit.argtypes = [C.c_void_p, _P, C.c_int32, C.POINTER(C.c_int32)]
lib.vit_server_submit.restype = C.c_int
lib.vit_server_submit_paced.argtypes = [C.c_void_p, _P, C.c_int32, C.POINTER(C.c_int32)]
lib.vit_server_submit_paced.restype = C.c_int
lib.vit_server_poll.argtypes = [C.c_void_p, _P, C.c_int32, C.POINTER(C.c_int32)]
lib.vit_server_poll.restype = C.c_int
lib.vit_server_drain.argtypes = [C.c_void_p, C.c_int64]
lib.vit_server_drain.restype = C.c_int
lib.vit_server_stats.argtypes = [C.c_void_p, C.POINTER(vit_serve_stats), C.c_int32]
lib.vit_server_stats.restype = C.c_int
lib.vit_server_destroy.argtypes = [C.c_void_p]
lib.vit_server_destroy.restype = None
lib.vit_last_error.argtypes = []
lib.vit_last_error.restype = C.c_char_p
lib.vit_abi_version.argtypes = []
lib.vit_abi_version.restype = C.c_int
lib.vit_debug_fail_allocations.argtypes = [C.c_int32]
lib.vit_debug_fail_allocations.restype = C.c_int
lib.vit_plan_get_tuning.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
lib.vit_plan_get_tuning.restype = C.c_int
lib.vit_plan_set_tuning.argtypes = [C.c_void_p, C.c_void_p, C.c_int32]
lib.vit_plan_set_tuning.restype = C.c_int


def make_code(k, gens):
    c = vit_code()
    c.k = int(k)
    c.beta = len(gens)
    for b, g in enumerate(gens):
        c.gen[b] = int(g)
    return c


def _check(status):
    if status != VIT_OK:
        raise VitError(status, vit_last_error())
    return status


def vit_last_error():
    return lib.vit_last_error().decode()


def vit_abi_version():
    return lib.vit_abi_version()


def vit_opts_default():
    return lib.vit_opts_default()


def vit_decode(code, llr_ptr, n, L, v, tie_rule, out_ptr):
    return _check(lib.vit_decode(C.byref(code), llr_ptr, n, L, v, tie_rule, out_ptr))


def vit_decode_ex(code, llr_ptr, n, L, v, tie_rule, out_ptr, opts=None):
    return _check(lib.vit_decode_ex(C.byref(code), llr_ptr, n, L, v, tie_rule, out_ptr,
                                    C.byref(opts) if opts is not None else None))


def vit_quantize_i8(llr_ptr, count, scale, q_ptr, stream=None):
    return _check(lib.vit_quantize_i8(llr_ptr, count, scale, q_ptr, stream))


def vit_depuncture(received_ptr, received_count, llr_type, mask, period, beta, stages, out_ptr, stream=None):
    m = (C.c_uint8 * (period * beta))(*[1 if x else 0 for x in mask])
    return _check(lib.vit_depuncture(received_ptr, received_count, llr_type, m, period, beta, stages, out_ptr,
                                     stream))


def vit_query_geometry(code, n, L, v, v1=-1, terminated=1):
    g = vit_geometry()
    _check(lib.vit_query_geometry(C.byref(code), n, L, v, v1, terminated, C.byref(g)))
    return g


def codes_array(codes):
    arr = (vit_code * len(codes))()
    for i, c in enumerate(codes):
        arr[i] = c
    return arr


import numpy as _np

# numpy layout of vit_frame: a frame list passes to the C ABI without copying
FRAME_DTYPE = _np.dtype([("code_id", "<i4"), ("terminated", "<i4"), ("n", "<i8"), ("llr_off", "<i8"),
                         ("out_off", "<i8")])


def frames_array(frames):
    """A contiguous FRAME_DTYPE array from an iterable of (code_id,
    terminated, n, llr_off, out_off) or from such an array (returned as is)."""
    if isinstance(frames, _np.ndarray) and frames.dtype == FRAME_DTYPE and frames.flags.c_contiguous:
        return frames
    if isinstance(frames, _np.ndarray):
        return _np.ascontiguousarray(frames, dtype=FRAME_DTYPE)
    return _np.array([tuple(f) for f in frames], dtype=FRAME_DTYPE)


def _fp(arr):
    return arr.ctypes.data_as(_PF)


def tunings_array(tunings):
    arr = (vit_tuning * len(tunings))()
    for i, t in enumerate(tunings):
        arr[i].L, arr[i].v, arr[i].v1, arr[i].waves_per_block = t
    return arr


def vit_plan_create():
    p = C.c_void_p()
    _check(lib.vit_plan_create(C.byref(p)))
    return p


def vit_plan_set_metric_bits(plan, bits):
    return _check(lib.vit_plan_set_metric_bits(plan, int(bits)))


def vit_plan_set_tune_tolerance(plan, max_diff_fraction):
    return _check(lib.vit_plan_set_tune_tolerance(plan, float(max_diff_fraction)))


def vit_plan_destroy(plan):
    lib.vit_plan_destroy(plan)


def vit_plan_get_tuning(plan):
    """The plan's autotuned shapes as a vit_tuning_entry array."""
    n = C.c_int32()
    _check(lib.vit_plan_get_tuning(plan, None, 0, C.byref(n)))
    arr = (vit_tuning_entry * max(1, n.value))()
    _check(lib.vit_plan_get_tuning(plan, arr, n.value, C.byref(n)))
    return arr[:n.value]


def vit_plan_set_tuning(plan, entries):
    arr = (vit_tuning_entry * max(1, len(entries)))(*entries)
    return _check(lib.vit_plan_set_tuning(plan, arr, len(entries)))


def vit_batch_workspace_size(codes_arr, frames_arr, tune_arr=None):
    b = C.c_size_t()
    _check(lib.vit_batch_workspace_size(codes_arr, len(codes_arr), _fp(frames_arr), len(frames_arr), tune_arr,
                                        C.byref(b)))
    return b.value


def vit_decode_batch(plan, codes_arr, frames_arr, llr_ptr, llr_count, llr_type, out_ptr, out_bytes, tune_arr,
                     ws_ptr, ws_bytes, stream=None):
    return _check(lib.vit_decode_batch(plan, codes_arr, len(codes_arr), _fp(frames_arr), len(frames_arr), llr_ptr,
                                       llr_count, llr_type, out_ptr, out_bytes, tune_arr, ws_ptr, ws_bytes,
                                       stream))


def vit_decode_batch_static(codes_arr, frames_arr, llr_ptr, llr_count, llr_type, out_ptr, out_bytes, tune_arr=None,
                            stream=None):
    return _check(lib.vit_decode_batch_static(codes_arr, len(codes_arr), _fp(frames_arr), len(frames_arr), llr_ptr,
                                              llr_count, llr_type, out_ptr, out_bytes, tune_arr, stream))


def vit_plan_autotune(plan, codes_arr, frames_arr, llr_ptr, llr_count, llr_type, out_ptr, out_bytes, ws_ptr,
                      ws_bytes, stream=None):
    chosen = (vit_tuning * len(codes_arr))()
    _check(lib.vit_plan_autotune(plan, codes_arr, len(codes_arr), _fp(frames_arr), len(frames_arr), llr_ptr, llr_count,
                                 llr_type, out_ptr, out_bytes, ws_ptr, ws_bytes, stream, chosen))
    return [(t.L, t.v, t.v1, t.waves_per_block) for t in chosen]


def vit_server_workspace_size(cfg):
    b = C.c_size_t()
    _check(lib.vit_server_workspace_size(C.byref(cfg), C.byref(b)))
    return b.value


def vit_server_create(codes_arr, tune_arr, cfg):
    p = C.c_void_p()
    _check(lib.vit_server_create(codes_arr, len(codes_arr), tune_arr, C.byref(cfg), C.byref(p)))
    return p


def vit_server_submit(server, reqs_ptr, count):
    """reqs_ptr: address of `count` packed vit_request records.  Returns
    (status, accepted); VIT_EBUSY is returned, not raised."""
    acc = C.c_int32()
    st = lib.vit_server_submit(server, reqs_ptr, count, C.byref(acc))
    if st not in (VIT_OK, VIT_EBUSY):
        raise VitError(st, vit_last_error())
    return st, acc.value


def vit_server_submit_paced(server, reqs_ptr, count):
    acc = C.c_int32()
    _check(lib.vit_server_submit_paced(server, reqs_ptr, count, C.byref(acc)))
    return acc.value


def vit_server_poll(server, out_ptr, max_count):
    n = C.c_int32()
    _check(lib.vit_server_poll(server, out_ptr, max_count, C.byref(n)))
    return n.value


def vit_server_drain(server, timeout_ms=-1):
    return _check(lib.vit_server_drain(server, timeout_ms))


def vit_server_stats(server, reset=False):
    st = vit_serve_stats()
    _check(lib.vit_server_stats(server, C.byref(st), 1 if reset else 0))
    return {name: getattr(st, name) for name, _ in vit_serve_stats._fields_}


def vit_server_destroy(server):
    lib.vit_server_destroy(server)
