"""MI355X (gfx950) soft-decision Viterbi decoder for (beta,1,k) convolutional codes.

Blocked decoding with overlap (Mohammadidoost & Hashemi, arXiv 2011.09337,
Sec. III-IV): every step runs in HIP kernels behind the C ABI of
include/vit.h.  This package only marshals torch device tensors into that ABI;
PyTorch provides device memory and streams.
"""
from . import _lib
from ._lib import (FRAME_DTYPE, codes_array, frames_array, tunings_array, vit_batch_workspace_size, vit_decode_batch,
                   vit_decode_batch_static,
                   vit_plan_autotune, vit_plan_create, vit_plan_destroy, vit_plan_get_tuning, vit_plan_set_tuning,
                   vit_plan_set_tune_tolerance,
                   vit_tuning_entry)
from ._lib import (VIT_EBUSY, VIT_ETIMEDOUT, vit_server_config, vit_server_create, vit_server_destroy, vit_server_drain,
                   vit_server_poll, vit_server_stats, vit_server_submit, vit_server_submit_paced,
                   vit_server_workspace_size)
from ._lib import (VIT_SUBFRAME_RANDOM, VIT_SUBFRAME_STORED)
from ._lib import (VIT_EDEVICE, VIT_EINVAL, VIT_ENOMEM, VIT_EUNSUPPORTED, VIT_LLR_F32, VIT_LLR_HARD, VIT_LLR_I8, VIT_OK,
                   VIT_TIE_LOWER_PRED, VitError, make_code, vit_abi_version, vit_decode, vit_decode_ex,
                   vit_last_error, vit_opts_default, vit_quantize_i8, vit_query_geometry, vit_depuncture)

__all__ = ["decode", "quantize", "depuncture", "vit_depuncture", "Batch", "Server", "FRAME_DTYPE", "REQUEST_DTYPE", "COMPLETION_DTYPE", "VIT_EBUSY", "VIT_ETIMEDOUT", "codes_array", "frames_array", "tunings_array",
           "vit_batch_workspace_size", "vit_decode_batch", "vit_decode_batch_static", "vit_plan_autotune", "vit_plan_create",
           "vit_plan_destroy", "vit_plan_get_tuning", "vit_plan_set_tuning", "vit_tuning_entry", "make_code", "vit_quantize_i8", "VitError", "vit_decode", "vit_decode_ex", "vit_query_geometry",
           "vit_last_error", "vit_abi_version", "vit_opts_default", "VIT_OK", "VIT_EINVAL",
           "VIT_EUNSUPPORTED", "VIT_ENOMEM", "VIT_EDEVICE", "VIT_LLR_F32", "VIT_LLR_I8", "VIT_LLR_HARD",
           "VIT_TIE_LOWER_PRED", "VIT_SUBFRAME_STORED", "VIT_SUBFRAME_RANDOM"]


def decode(code, llr, n, L, v, *, v1=None, terminated=True, subframe_bits=0, subframe_overlap=0,
           subframe_start=None, subframe_seed=0, check_finite=False, metric_bits=0, out=None, stream=None):
    """Decode n bits from a device tensor of LLRs (float32 or int8, N*beta
    values, time-major; uint8 = hard decisions, 0 / nonzero per coded bit).
    subframe_bits f0 > 0 runs the parallel traceback of Sec. IV-D: subframes
    of f0 core bits, subframe_overlap stages of inner overlap, inner chains
    started from the stored best state (subframe_start VIT_SUBFRAME_STORED,
    the default) or a random one (VIT_SUBFRAME_RANDOM, seeded by
    subframe_seed); see vit_opts.  0 traces each block back once.  check_finite scans FP32 LLRs
    first and raises VitError(VIT_EINVAL) on a NaN or infinity (the call then
    waits for the scan).  metric_bits picks the integer inputs' path metrics
    (16: modulo 2^16, 32: exact in fp32, 0: 32 where the blocks fit; see
    vit_opts).  Returns (or fills) a uint8 device
    tensor of ceil(n/8) packed bytes.  Asynchronous on `stream` (default:
    torch's current stream)."""
    import torch

    if not llr.is_cuda or not llr.is_contiguous():
        raise ValueError("llr must be a contiguous device tensor")
    if llr.dtype == torch.float32:
        llr_type = VIT_LLR_F32
    elif llr.dtype == torch.int8:
        llr_type = VIT_LLR_I8
    elif llr.dtype == torch.uint8:
        llr_type = VIT_LLR_HARD
    else:
        raise TypeError(f"llr dtype {llr.dtype} (float32, int8 or uint8 hard decisions expected)")
    nbytes = (int(n) + 7) // 8
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device=llr.device)
    elif out.numel() < nbytes or out.dtype != torch.uint8 or not out.is_cuda:
        raise ValueError("out must be a uint8 device tensor of ceil(n/8) bytes")
    N = int(n) + (code.k - 1 if terminated else 0)
    if llr.numel() != N * code.beta:
        raise ValueError(f"llr holds {llr.numel()} values, expected {N * code.beta}")
    opts = vit_opts_default()
    opts.llr_type = llr_type
    opts.terminated = 1 if terminated else 0
    opts.v1 = -1 if v1 is None else int(v1)
    opts.check_finite = 1 if check_finite else 0
    opts.subframe_bits = int(subframe_bits)
    opts.subframe_overlap = int(subframe_overlap)
    opts.subframe_start = VIT_SUBFRAME_STORED if subframe_start is None else int(subframe_start)
    opts.subframe_seed = int(subframe_seed)
    opts.metric_bits = int(metric_bits)
    if stream is None:
        stream = torch.cuda.current_stream(llr.device)
    opts.stream = stream.cuda_stream
    vit_decode_ex(code, llr.data_ptr(), int(n), int(L), int(v), VIT_TIE_LOWER_PRED, out.data_ptr(), opts)
    return out


def quantize(llr, scale, *, out=None, stream=None):
    """int8 quantisation of a float32 device tensor (see vit_quantize_i8)."""
    import torch

    if not llr.is_cuda or not llr.is_contiguous() or llr.dtype != torch.float32:
        raise ValueError("llr must be a contiguous float32 device tensor")
    if out is None:
        out = torch.empty(llr.numel(), dtype=torch.int8, device=llr.device)
    if stream is None:
        stream = torch.cuda.current_stream(llr.device)
    vit_quantize_i8(llr.data_ptr(), llr.numel(), float(scale), out.data_ptr(), stream.cuda_stream)
    return out


def depuncture(received, mask, stages, *, out=None, stream=None):
    """De-puncture a device tensor (float32 or int8) of transmitted values with
    a (period, beta) 0/1 pattern (see vit_depuncture); returns stages*beta
    values with zeros in the punctured slots."""
    import numpy as np
    import torch

    mask = np.asarray(mask, dtype=np.uint8)
    period, beta = mask.shape
    if not received.is_cuda or not received.is_contiguous():
        raise ValueError("received must be a contiguous device tensor")
    llr_type = VIT_LLR_F32 if received.dtype == torch.float32 else VIT_LLR_I8
    if received.dtype not in (torch.float32, torch.int8):
        raise TypeError(f"received dtype {received.dtype} (float32 or int8 expected)")
    if out is None:
        out = torch.empty(int(stages) * beta, dtype=received.dtype, device=received.device)
    if stream is None:
        stream = torch.cuda.current_stream(received.device)
    vit_depuncture(received.data_ptr(), received.numel(), llr_type, mask.reshape(-1).tolist(), period, beta,
                   int(stages), out.data_ptr(), stream.cuda_stream)
    return out


class Batch:
    """A plan plus a device workspace for batched decoding (vit_decode_batch).

    codes: list of vit_code; frames: a FRAME_DTYPE array (passed to the C ABI
    without copying) or a list of (code_id, terminated, n, llr_off, out_off).
    The workspace is a torch uint8 tensor sized by vit_batch_workspace_size
    for the largest frame list seen."""

    def __init__(self, device="cuda", metric_bits=0, tune_tolerance=None):
        self.plan = vit_plan_create()
        self.device = device
        self.ws = None
        if metric_bits:
            _lib.vit_plan_set_metric_bits(self.plan, metric_bits)
        if tune_tolerance is not None:
            _lib.vit_plan_set_tune_tolerance(self.plan, tune_tolerance)

    def close(self):
        if self.plan is not None:
            vit_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _workspace(self, codes_arr, frames_arr, tune_arr):
        import torch
        need = vit_batch_workspace_size(codes_arr, frames_arr, tune_arr)
        if self.ws is None or self.ws.numel() < need + 256:
            self.ws = torch.empty(max(need, 4096) * 2 + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        return aligned, self.ws.numel() - (aligned - base)

    def decode(self, codes, frames, llr, out, tune=None, stream=None):
        import torch
        codes_arr, frames_arr = codes_array(codes), frames_array(frames)
        tune_arr = tunings_array(tune) if tune is not None else None
        ws, ws_bytes = self._workspace(codes_arr, frames_arr, tune_arr)
        llr_type = {torch.int8: VIT_LLR_I8, torch.uint8: VIT_LLR_HARD}.get(llr.dtype, VIT_LLR_F32)
        if stream is None:
            stream = torch.cuda.current_stream(llr.device)
        vit_decode_batch(self.plan, codes_arr, frames_arr, llr.data_ptr(), llr.numel(), llr_type, out.data_ptr(),
                         out.numel(), tune_arr, ws, ws_bytes, stream.cuda_stream)
        return out

    def tuning(self):
        """The plan's autotuned shapes: dicts with the code (k, gens), llr_type,
        length_bucket and the shape (L, v, v1, waves_per_block)."""
        return [{"k": e.code.k, "gens": [int(g) for g in e.code.gen[:e.code.beta]], "llr_type": e.llr_type,
                 "length_bucket": e.length_bucket, "L": e.L, "v": e.v, "v1": e.v1,
                 "waves_per_block": e.waves_per_block} for e in vit_plan_get_tuning(self.plan)]

    def set_tuning(self, entries):
        """Add autotuned shapes (dicts as returned by `tuning`) to the plan."""
        arr = []
        for d in entries:
            e = vit_tuning_entry()
            e.code = make_code(d["k"], d["gens"])
            e.llr_type, e.length_bucket = int(d["llr_type"]), int(d["length_bucket"])
            e.L, e.v, e.v1, e.waves_per_block = int(d["L"]), int(d["v"]), int(d["v1"]), int(d["waves_per_block"])
            arr.append(e)
        vit_plan_set_tuning(self.plan, arr)

    @staticmethod
    def _device_name(device_name):
        if device_name is not None:
            return device_name
        import torch
        return torch.cuda.get_device_name()

    def save_tuning(self, path, device_name=None):
        """Write the plan's autotuned shapes to a JSON file, keyed by the GPU
        model (torch's device name unless `device_name` is given)."""
        import json
        with open(path, "w") as f:
            json.dump({"device": self._device_name(device_name), "entries": self.tuning()}, f, indent=1)

    def load_tuning(self, path, device_name=None):
        """Take the shapes of a file written by `save_tuning` if it was tuned on
        the same GPU model; returns how many were taken (0 for another GPU)."""
        import json
        with open(path) as f:
            data = json.load(f)
        if data.get("device") != self._device_name(device_name):
            return 0
        self.set_tuning(data["entries"])
        return len(data["entries"])

    def autotune(self, codes, frames, llr, out, stream=None):
        import torch
        codes_arr, frames_arr = codes_array(codes), frames_array(frames)
        ws, ws_bytes = self._workspace(codes_arr, frames_arr, None)
        llr_type = {torch.int8: VIT_LLR_I8, torch.uint8: VIT_LLR_HARD}.get(llr.dtype, VIT_LLR_F32)
        if stream is None:
            stream = torch.cuda.current_stream(llr.device)
        return vit_plan_autotune(self.plan, codes_arr, frames_arr, llr.data_ptr(), llr.numel(), llr_type,
                                 out.data_ptr(), out.numel(), ws, ws_bytes, stream.cuda_stream)


# numpy layouts of vit_request and vit_completion (include/vit.h)
try:
    import numpy as _np

    REQUEST_DTYPE = _np.dtype([("code_id", "<i4"), ("terminated", "<i4"), ("n", "<i8"), ("llr", "<u8"),
                               ("out", "<u8"), ("tag", "<u8"), ("arrival_ns", "<i8")])
    COMPLETION_DTYPE = _np.dtype([("tag", "<u8"), ("status", "<i4"), ("reserved", "<i4"), ("arrival_ns", "<i8"),
                                  ("done_ns", "<i8")])
except ImportError:  # pragma: no cover
    REQUEST_DTYPE = COMPLETION_DTYPE = None


class Server:
    """The serving loop of include/vit.h (vit_server_*), with its device arena
    and workspace held as torch tensors.

    codes: list of vit_code; tune: one (L, v, v1, waves_per_block) per code or
    None; host: a pinned uint8 torch tensor holding every request's LLRs and
    output bytes (requests address it by byte offset, see `requests`)."""

    def __init__(self, codes, host, *, tune=None, llr_type=VIT_LLR_I8, arena_bytes=64 << 20, max_frames=4096,
                 max_items=65536, max_pending=1 << 20, max_wait_ms=0, metric_bits=0, device="cuda", stream=None):
        import torch

        if not host.is_pinned() or host.dtype != torch.uint8:
            raise ValueError("host must be a pinned uint8 tensor")
        self.host = host
        self.codes = list(codes)
        cfg = vit_server_config()
        cfg.size = C_sizeof(vit_server_config)
        cfg.llr_type = llr_type
        cfg.max_frames = max_frames
        cfg.max_items = max_items
        cfg.max_pending = max_pending
        cfg.max_wait_ms = max_wait_ms
        cfg.metric_bits = metric_bits
        ws_bytes = vit_server_workspace_size(cfg)
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=device)
        self.ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=device)
        cfg.arena = (self.arena.data_ptr() + 255) // 256 * 256
        cfg.arena_bytes = arena_bytes
        cfg.workspace = (self.ws.data_ptr() + 255) // 256 * 256
        cfg.workspace_bytes = ws_bytes
        cfg.host = host.data_ptr()
        cfg.host_bytes = host.numel()
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        cfg.stream = self.stream.cuda_stream
        self.cfg = cfg
        self.server = vit_server_create(codes_array(self.codes), tunings_array(tune) if tune is not None else None,
                                        cfg)
        self.host_base = host.data_ptr()

    def requests(self, count):
        """A zeroed request array of `count` records."""
        return _np.zeros(count, dtype=REQUEST_DTYPE)

    def submit(self, reqs):
        """Queue a REQUEST_DTYPE array (llr/out as absolute host addresses).
        Returns (status, accepted): VIT_OK, or VIT_EBUSY with a partial count."""
        reqs = _np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        if len(reqs) == 0:
            return VIT_OK, 0
        return vit_server_submit(self.server, reqs.ctypes.data, len(reqs))

    def submit_paced(self, reqs):
        """Submit each request of a REQUEST_DTYPE array at its arrival_ns
        (time.monotonic_ns clock), from the calling thread; returns when all
        are queued.  The GIL is released meanwhile."""
        reqs = _np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        if len(reqs) == 0:
            return 0
        return vit_server_submit_paced(self.server, reqs.ctypes.data, len(reqs))

    def poll(self, max_count=65536):
        """Completions so far (up to max_count), as a COMPLETION_DTYPE array."""
        buf = getattr(self, "_poll_buf", None)
        if buf is None or len(buf) < max_count:
            buf = self._poll_buf = _np.empty(max_count, dtype=COMPLETION_DTYPE)
        n = vit_server_poll(self.server, buf.ctypes.data, max_count)
        return buf[:n].copy()

    def drain(self, timeout_ms=-1):
        return vit_server_drain(self.server, timeout_ms)

    def stats(self, reset=False):
        return vit_server_stats(self.server, reset)

    def close(self):
        if getattr(self, "server", None) is not None:
            vit_server_destroy(self.server)
            self.server = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def C_sizeof(t):
    import ctypes
    return ctypes.sizeof(t)
