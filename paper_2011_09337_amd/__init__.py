"""MI355X (gfx950) soft-decision Viterbi decoder for (beta,1,k) convolutional codes.

Blocked decoding with overlap (Mohammadidoost & Hashemi, arXiv 2011.09337,
Sec. III-IV): every step runs in HIP kernels behind the C ABI of
include/vit.h.  This package only marshals torch device tensors into that ABI;
PyTorch provides device memory and streams.
"""
from . import _lib
from ._lib import (codes_array, frames_array, tunings_array, vit_batch_workspace_size, vit_decode_batch,
                   vit_plan_autotune, vit_plan_create, vit_plan_destroy)
from ._lib import (VIT_EDEVICE, VIT_EINVAL, VIT_ENOMEM, VIT_EUNSUPPORTED, VIT_LLR_F32, VIT_LLR_I8, VIT_OK,
                   VIT_TIE_LOWER_PRED, VitError, make_code, vit_abi_version, vit_decode, vit_decode_ex,
                   vit_last_error, vit_opts_default, vit_quantize_i8, vit_query_geometry)

__all__ = ["decode", "quantize", "Batch", "codes_array", "frames_array", "tunings_array",
           "vit_batch_workspace_size", "vit_decode_batch", "vit_plan_autotune", "vit_plan_create",
           "vit_plan_destroy", "make_code", "vit_quantize_i8", "VitError", "vit_decode", "vit_decode_ex", "vit_query_geometry",
           "vit_last_error", "vit_abi_version", "vit_opts_default", "VIT_OK", "VIT_EINVAL",
           "VIT_EUNSUPPORTED", "VIT_ENOMEM", "VIT_EDEVICE", "VIT_LLR_F32", "VIT_LLR_I8",
           "VIT_TIE_LOWER_PRED"]


def decode(code, llr, n, L, v, *, v1=None, terminated=True, out=None, stream=None):
    """Decode n bits from a device tensor of LLRs (float32 or int8, N*beta
    values, time-major).  Returns (or fills) a uint8 device tensor of
    ceil(n/8) packed bytes.  Asynchronous on `stream` (default: torch's
    current stream)."""
    import torch

    if not llr.is_cuda or not llr.is_contiguous():
        raise ValueError("llr must be a contiguous device tensor")
    if llr.dtype == torch.float32:
        llr_type = VIT_LLR_F32
    elif llr.dtype == torch.int8:
        llr_type = VIT_LLR_I8
    else:
        raise TypeError(f"llr dtype {llr.dtype} (float32 or int8 expected)")
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


class Batch:
    """A plan plus a device workspace for batched decoding (vit_decode_batch).

    codes: list of vit_code; frames: list of (code_id, terminated, n,
    llr_off, out_off).  The workspace is a torch uint8 tensor sized by
    vit_batch_workspace_size for the largest frame list seen."""

    def __init__(self, device="cuda"):
        self.plan = vit_plan_create()
        self.device = device
        self.ws = None

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
        llr_type = VIT_LLR_I8 if llr.dtype == torch.int8 else VIT_LLR_F32
        if stream is None:
            stream = torch.cuda.current_stream(llr.device)
        vit_decode_batch(self.plan, codes_arr, frames_arr, llr.data_ptr(), llr.numel(), llr_type, out.data_ptr(),
                         out.numel(), tune_arr, ws, ws_bytes, stream.cuda_stream)
        return out

    def autotune(self, codes, frames, llr, out, stream=None):
        import torch
        codes_arr, frames_arr = codes_array(codes), frames_array(frames)
        ws, ws_bytes = self._workspace(codes_arr, frames_arr, None)
        llr_type = VIT_LLR_I8 if llr.dtype == torch.int8 else VIT_LLR_F32
        if stream is None:
            stream = torch.cuda.current_stream(llr.device)
        return vit_plan_autotune(self.plan, codes_arr, frames_arr, llr.data_ptr(), llr.numel(), llr_type,
                                 out.data_ptr(), out.numel(), ws, ws_bytes, stream.cuda_stream)
