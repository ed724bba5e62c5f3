"""ctypes front end of the CPU oracle (oracle/libvref.so).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU decoder never imports this module.

All functions take and return numpy arrays.  Decoded bits come back unpacked,
one uint8 (0 or 1) per bit.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvref.so")


class VrefCode(C.Structure):
    _fields_ = [("k", C.c_int32), ("beta", C.c_int32), ("gen", C.c_uint32 * 4)]


try:
    _lib = C.CDLL(LIB_PATH)
except OSError:
    _lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location("vref_build", os.path.join(HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _lib = C.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_P = C.c_void_p


def _declare(L):
    i64, i32 = C.c_int64, C.c_int32
    L.vref_encode.argtypes = [C.POINTER(VrefCode), _P, i64, i32, _P]
    for nm in ("vref_decode_full_f32", "vref_decode_full_f64", "vref_decode_full_i8"):
        getattr(L, nm).argtypes = [C.POINTER(VrefCode), _P, i64, i32, _P, _P]
    for nm in ("vref_decode_blocked_f32", "vref_decode_blocked_f64", "vref_decode_blocked_i8"):
        getattr(L, nm).argtypes = [C.POINTER(VrefCode), _P, i64, i32, i64, i64, i64, _P, i32]
    L.vref_window_f64.argtypes = [C.POINTER(VrefCode), _P, i64, i64, i32, i32, i64, i64, _P, _P]
    L.vref_quantize_i8.argtypes = [_P, i64, C.c_float, _P]
    L.vref_bruteforce_window.argtypes = [C.POINTER(VrefCode), _P, i64, i64, i32, i32, _P, _P]
    L.vref_depuncture_f32.argtypes = [_P, i64, _P, i32, i32, i64, _P]
    L.vref_depuncture_i8.argtypes = [_P, i64, _P, i32, i32, i64, _P]
    L.vref_decode_full_i16mod.argtypes = [C.POINTER(VrefCode), _P, i64, i32, _P, _P]
    L.vref_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.vref_splitmix64.restype = C.c_uint64
    for nm in ("vref_decode_blocked_pt_f32", "vref_decode_blocked_pt_i8"):
        getattr(L, nm).argtypes = [C.POINTER(VrefCode), _P, i64, i32, i64, i64, i64, i64, i64, i32, C.c_uint64,
                                   _P, i32]
    L.vref_bruteforce_window_to.argtypes = [C.POINTER(VrefCode), _P, i64, i64, i32, i32, _P, _P]
    for fn in (L.vref_encode, L.vref_decode_full_f32, L.vref_decode_full_f64, L.vref_decode_full_i8,
               L.vref_decode_blocked_f32, L.vref_decode_blocked_f64, L.vref_decode_blocked_i8,
               L.vref_window_f64, L.vref_quantize_i8, L.vref_bruteforce_window, L.vref_depuncture_f32,
               L.vref_depuncture_i8,
               L.vref_decode_full_i16mod, L.vref_decode_blocked_pt_f32, L.vref_decode_blocked_pt_i8,
               L.vref_bruteforce_window_to):
        fn.restype = C.c_int


if _lib is not None:
    _declare(_lib)


def make_code(k, gens):
    """Code (k, beta = len(gens), generators).  gens are ints (write octal as 0o171)."""
    c = VrefCode()
    c.k = int(k)
    c.beta = len(gens)
    for b, g in enumerate(gens):
        c.gen[b] = int(g)
    return c


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def n_stages(code, n, terminated):
    return int(n) + (code.k - 1 if terminated else 0)


def encode(code, bits, terminated=True):
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    n = bits.size
    out = np.zeros(n_stages(code, n, terminated) * code.beta, dtype=np.uint8)
    _check(lib().vref_encode(C.byref(code), _ptr(bits), n, int(bool(terminated)), _ptr(out)), "vref_encode")
    return out


def decode_full(code, llr, n, terminated=True, want_metric=False):
    """Full-frame ML decode.  dtype of llr selects the arithmetic: float32, float64, int8."""
    llr = np.ascontiguousarray(llr)
    assert llr.size == n_stages(code, n, terminated) * code.beta, "llr size"
    out = np.zeros(n, dtype=np.uint8)
    if llr.dtype == np.float32:
        met = C.c_float()
        fn = lib().vref_decode_full_f32
    elif llr.dtype == np.float64:
        met = C.c_double()
        fn = lib().vref_decode_full_f64
    elif llr.dtype == np.int8:
        met = C.c_int64()
        fn = lib().vref_decode_full_i8
    else:
        raise TypeError(llr.dtype)
    _check(fn(C.byref(code), _ptr(llr), n, int(bool(terminated)), _ptr(out), C.byref(met)), fn.__name__)
    return (out, met.value) if want_metric else out


def decode_full_i16mod(code, llr, n, terminated=True):
    """Full-frame decode of int8 LLRs with 16-bit path metrics modulo 2^16
    (compared by the sign of the wrapped difference).  Returns (bits, the
    traced path's metric as a signed 16-bit value)."""
    llr = np.ascontiguousarray(llr, dtype=np.int8)
    assert llr.size == n_stages(code, n, terminated) * code.beta, "llr size"
    out = np.zeros(n, dtype=np.uint8)
    met = C.c_int16()
    _check(lib().vref_decode_full_i16mod(C.byref(code), _ptr(llr), n, int(bool(terminated)), _ptr(out),
                                         C.byref(met)), "vref_decode_full_i16mod")
    return out, met.value


def split_overlap(v, v1=None):
    """Default split of the overlap v into left v1 = floor(v/2) and right v2 = v - v1."""
    if v1 is None or v1 < 0:
        v1 = v // 2
    return int(v1), int(v - v1)


def decode_blocked(code, llr, n, L, v1, v2, terminated=True, nthreads=1):
    """Blocked decode with overlap (left v1, right v2 stages) and cores of L bits."""
    llr = np.ascontiguousarray(llr)
    assert llr.size == n_stages(code, n, terminated) * code.beta, "llr size"
    out = np.zeros(n, dtype=np.uint8)
    fn = {np.dtype(np.float32): lib().vref_decode_blocked_f32,
          np.dtype(np.float64): lib().vref_decode_blocked_f64,
          np.dtype(np.int8): lib().vref_decode_blocked_i8}[llr.dtype]
    _check(fn(C.byref(code), _ptr(llr), n, int(bool(terminated)), int(L), int(v1), int(v2), _ptr(out),
              int(nthreads)), fn.__name__)
    return out


def window_f64(code, llr, s, e, start_known, end_zero, emit_lo, emit_hi):
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    out = np.zeros(max(emit_hi - emit_lo, 1), dtype=np.uint8)
    met = C.c_double()
    _check(lib().vref_window_f64(C.byref(code), _ptr(llr), s, e, int(start_known), int(end_zero),
                                 emit_lo, emit_hi, _ptr(out), C.byref(met)), "vref_window_f64")
    return out[: emit_hi - emit_lo], met.value


def quantize_i8(llr, scale):
    llr = np.ascontiguousarray(llr, dtype=np.float32)
    q = np.zeros(llr.size, dtype=np.int8)
    _check(lib().vref_quantize_i8(_ptr(llr), llr.size, C.c_float(scale), _ptr(q)), "vref_quantize_i8")
    return q


def bruteforce_window(code, llr, s, e, start_known, end_zero):
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    out = np.zeros(e - s, dtype=np.uint8)
    met = C.c_double()
    _check(lib().vref_bruteforce_window(C.byref(code), _ptr(llr), s, e, int(start_known), int(end_zero),
                                        _ptr(out), C.byref(met)), "vref_bruteforce_window")
    return out, met.value


def depuncture(received, mask, stages):
    """De-puncturing (Sec. IV-E): mask is a (period, beta) 0/1 array; returns
    stages*beta values with zeros in the punctured slots."""
    received = np.ascontiguousarray(received)
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    period, beta = mask.shape
    out = np.zeros(stages * beta, dtype=received.dtype)
    fn = {np.dtype(np.float32): lib().vref_depuncture_f32, np.dtype(np.int8): lib().vref_depuncture_i8}[received.dtype]
    _check(fn(_ptr(received), received.size, _ptr(mask), period, beta, stages, _ptr(out)), fn.__name__)
    return out


PT_STORED, PT_RANDOM = 0, 1


def splitmix64(seed, i):
    """Output i of SplitMix64 seeded with `seed` (the random start states of
    the parallel traceback)."""
    return int(lib().vref_splitmix64(C.c_uint64(seed & (2 ** 64 - 1)), C.c_uint64(i & (2 ** 64 - 1))))


def decode_blocked_pt(code, llr, n, L, v1, v2, f0, w, start_rule=PT_STORED, seed=0, terminated=True, nthreads=1):
    """Blocked decode with the parallel traceback of Sec. IV-D: subframes of
    f0 core bits, w stages of inner overlap, inner chains started from the
    stored best state (PT_STORED) or a random one (PT_RANDOM, from seed)."""
    llr = np.ascontiguousarray(llr)
    assert llr.size == n_stages(code, n, terminated) * code.beta, "llr size"
    out = np.zeros(n, dtype=np.uint8)
    fn = {np.dtype(np.float32): lib().vref_decode_blocked_pt_f32,
          np.dtype(np.int8): lib().vref_decode_blocked_pt_i8}[llr.dtype]
    _check(fn(C.byref(code), _ptr(llr), n, int(bool(terminated)), int(L), int(v1), int(v2), int(f0), int(w),
              int(start_rule), C.c_uint64(seed & (2 ** 64 - 1)), _ptr(out), int(nthreads)), fn.__name__)
    return out


def bruteforce_window_to(code, llr, s, e, start_known, end_state):
    """Exhaustive search over a window with the final state fixed (-1: free)."""
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    out = np.zeros(e - s, dtype=np.uint8)
    met = C.c_double()
    _check(lib().vref_bruteforce_window_to(C.byref(code), _ptr(llr), s, e, int(start_known), int(end_state),
                                           _ptr(out), C.byref(met)), "vref_bruteforce_window_to")
    return out, met.value
