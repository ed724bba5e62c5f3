"""GPU int8 quantiser against the CPU oracle's quantiser, byte for byte."""
import numpy as np
import pytest

from oracle import vref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def _values(rng, n):
    x = (rng.standard_normal(n) * 20).astype(np.float32)
    x[: n // 8] = (rng.integers(-300, 300, n // 8) / 2.0).astype(np.float32)   # exact halves: ties
    x[n // 8: n // 8 + 4] = np.array([-0.0, 0.0, 1e30, -1e30], np.float32)
    x[n // 8 + 4: n // 8 + 8] = np.array([126.5, 127.5, -126.5, -127.5], np.float32)
    return x


@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000, 65536 + 5, 1 << 22])
@pytest.mark.parametrize("scale", [1.0, 0.37, 8.0, 25.0])
def test_quantize_matches_oracle(dev, n, scale):
    torch, vit = dev
    rng = np.random.default_rng(n)
    x = _values(rng, max(n, 16))[:n]
    print(f"[gpu] quantize n={n} scale={scale}", flush=True)
    q = vit.quantize(torch.from_numpy(x).cuda(), scale)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(q.cpu().numpy(), vref.quantize_i8(x, scale))


def test_quantize_unaligned_views(dev):
    torch, vit = dev
    rng = np.random.default_rng(3)
    x = _values(rng, 4099)
    t = torch.from_numpy(x).cuda()
    for off in (1, 3, 5):
        src = t[off:]
        out = torch.empty(src.numel() + 3, dtype=torch.int8, device="cuda")[3:]
        vit.vit_quantize_i8(src.data_ptr(), src.numel(), 3.0, out.data_ptr(), None)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), vref.quantize_i8(x[off:], 3.0))


def test_quantize_then_decode_int8(dev):
    # the int8 path end to end: quantise on the GPU, decode int8 on the GPU,
    # against the oracle quantiser followed by the exact integer oracle decoder
    torch, vit = dev
    import synth
    k, gens = synth.CODES["k7r13"]
    n = 20000
    bits, llr = synth.make_stream("k7r13", n, 2.0, seed=5)
    scale = 16.0 * synth.noise_sigma(2.0, 3) ** 2 / 2.0
    q = vit.quantize(torch.from_numpy(llr).cuda(), scale)
    out = vit.decode(vit.make_code(k, gens), q, n, 256, 35)
    torch.cuda.synchronize()
    qc = vref.quantize_i8(llr, scale)
    np.testing.assert_array_equal(q.cpu().numpy(), qc)
    want = vref.decode_blocked(vref.make_code(k, list(gens)), qc, n, 256, 17, 18, True, nthreads=8)
    np.testing.assert_array_equal(out.cpu().numpy(), synth.pack_bits(want))
