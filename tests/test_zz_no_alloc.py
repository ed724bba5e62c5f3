"""The allocation-free batch entry point (vit_decode_batch_static) through the
C ABI, against vit_decode_batch (plan + workspace) on the same frames: bit
for bit, on two calls in a row, the second with a smaller batch, and against
the CPU oracle on a sample of frames."""
import numpy as np
import pytest

from test_gpu_batch import CODES, check_frames, make_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def _both(dev, frames, llr, out_bytes, tune):
    torch, vit = dev
    codes = [vit.make_code(*c) for c in CODES]
    codes_arr = vit.codes_array(codes)
    frames_arr = vit.frames_array(frames)
    tune_arr = vit.tunings_array(tune) if tune is not None else None
    t_llr = torch.from_numpy(llr).cuda()
    llr_type = vit.VIT_LLR_I8 if llr.dtype == np.int8 else vit.VIT_LLR_F32
    stream = torch.cuda.current_stream()
    got = torch.full((out_bytes,), 0xAB, dtype=torch.uint8, device="cuda")
    print(f"[gpu] static batch: {len(frames)} frames, tune={tune}", flush=True)
    vit.vit_decode_batch_static(codes_arr, frames_arr, t_llr.data_ptr(), t_llr.numel(), llr_type, got.data_ptr(),
                                got.numel(), tune_arr, stream.cuda_stream)
    want = torch.full((out_bytes,), 0xAB, dtype=torch.uint8, device="cuda")
    b = vit.Batch()
    b.decode(codes, frames, t_llr, want, tune=tune, stream=stream)
    torch.cuda.synchronize()
    b.close()
    return got.cpu().numpy(), want.cpu().numpy()


TUNE = [(256, 35, -1, 1), (128, 35, 10, 2), (64, 45, -1, 1), (64, 25, -1, 1), (32, 20, -1, 4)]


@pytest.mark.parametrize("int8", [False, True])
def test_static_batch_equals_plan_batch_twice(dev, int8):
    rng = np.random.default_rng(71 + int8)
    frames, llr, out_bytes, _ = make_batch(rng, 400, [0, 1, 2, 3, 4], 1, 3000, int8=int8)
    got, want = _both(dev, frames, llr, out_bytes, TUNE)
    np.testing.assert_array_equal(got, want)
    check_frames(got, frames[::25], llr, TUNE)
    # second call, smaller batch, default shapes: the array keeps the first
    # call's longer work list beyond the new one, which must not matter
    frames2, llr2, out_bytes2, _ = make_batch(rng, 37, [0, 1, 2], 40, 900, int8=int8)
    got2, want2 = _both(dev, frames2, llr2, out_bytes2, None)
    np.testing.assert_array_equal(got2, want2)
    check_frames(got2, frames2[::6], llr2, [(256, 35, -1, 1), (256, 35, -1, 1), (256, 64, -1, 1)])


def test_static_batch_full_size_mixed_int8(dev):
    """The 8192-frame mixed-code int8 configuration (lengths 40-6144), the
    largest batch the benchmark runs, at the default shapes."""
    rng = np.random.default_rng(5)
    frames, llr, out_bytes, _ = make_batch(rng, 8192, [0, 1, 2], 40, 6144, int8=True)
    got, want = _both(dev, frames, llr, out_bytes, None)
    np.testing.assert_array_equal(got, want)
