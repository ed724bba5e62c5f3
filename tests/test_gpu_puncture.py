"""De-puncturing on the GPU (Sec. IV-E) against the oracle, and decoding of
punctured streams end to end."""
import numpy as np
import pytest

import synth
from oracle import vref

pytestmark = pytest.mark.gpu

R23 = np.array([[1, 1], [1, 0]], dtype=np.uint8)
R34 = np.array([[1, 1], [1, 0], [0, 1]], dtype=np.uint8)
B3 = np.array([[1, 0, 1], [0, 1, 1], [1, 1, 0]], dtype=np.uint8)


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


@pytest.mark.parametrize("dtype", [np.float32, np.int8])
@pytest.mark.parametrize("mask,stages", [(R23, 1), (R23, 1001), (R34, 100003), (B3, 1 << 20), (R34, 2)])
def test_depuncture_matches_oracle(dev, dtype, mask, stages):
    torch, vit = dev
    period, beta = mask.shape
    rng = np.random.default_rng(stages)
    full = rng.integers(-100, 100, size=stages * beta).astype(dtype)
    sent = np.ascontiguousarray(synth.puncture(full, mask))
    want = vref.depuncture(sent, mask, stages)
    print(f"[gpu] depuncture {mask.tolist()} stages={stages} dtype={np.dtype(dtype).name}", flush=True)
    got = vit.depuncture(torch.from_numpy(sent).cuda(), mask, stages)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), want)


@pytest.mark.parametrize("mask", [R23, R34])
def test_punctured_stream_decodes_like_the_oracle(dev, mask):
    torch, vit = dev
    k, gens = synth.CODES["k7r12"]
    n = 40000
    bits, sent = synth.make_punctured_stream("k7r12", n, 5.0, 9, mask)
    N = n + k - 1
    d = vit.depuncture(torch.from_numpy(sent).cuda(), mask, N)
    out = vit.decode(vit.make_code(k, gens), d, n, 256, 60)
    torch.cuda.synchronize()
    want = vref.decode_blocked(vref.make_code(k, list(gens)), vref.depuncture(sent, mask, N), n, 256, 30, 30, True)
    np.testing.assert_array_equal(out.cpu().numpy(), synth.pack_bits(want))
    assert np.mean(synth.unpack_bits(out.cpu().numpy(), n) != bits) < 1e-2
