"""The subframe traceback (Sec. IV-D) on the GPU against the oracle's
subframe decoder, bit for bit: each block's trace cut into subframes of F
survivor words, each traced by its own chain from the best state W words
above its subframe.  The survivor word length is (k-1)*floor(32/(k-1))
stages, as the decoder's ABI documents."""
import os

import numpy as np
import pytest

import synth
from oracle import vref

pytestmark = pytest.mark.gpu

CODES = {
    "k7r12": (7, (0o171, 0o133)),
    "k7r13": (7, (0o133, 0o171, 0o165)),
    "k9r12": (9, (0o561, 0o753)),
    "k3r12": (3, (0o7, 0o5)),
    "k4r14": (4, (0o13, 0o15, 0o17, 0o11)),
    "k5r12x": (5, (0o22, 0o35)),
    "k6r12": (6, (0o53, 0o75)),
    "k8r12": (8, (0o247, 0o371)),
}
NCPU = max(1, min(16, len(os.sched_getaffinity(0))))


def word_stages(k):
    return (k - 1) * (32 // (k - 1))


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def _check(dev, k, gens, llr, n, L, v, F, W, v1=None, terminated=True, plain_equal=False):
    torch, vit = dev
    print(f"[gpu] k={k} gens={[oct(g) for g in gens]} n={n} L={L} v={v} v1={v1} F={F} W={W} term={terminated} "
          f"dtype={llr.dtype}", flush=True)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    got = vit.decode(vit.make_code(k, gens), t, n, L, v, v1=v1, terminated=terminated, subframe_words=F,
                     subframe_overlap=W)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    e1 = v // 2 if v1 is None else v1
    code = vref.make_code(k, list(gens))
    ol = llr
    if llr.dtype == np.uint8:  # hard decisions: coded bit 0 -> LLR +1, 1 -> -1
        ol = np.where(llr == 0, 1, -1).astype(np.int8)
    Lb, e2 = L, v - e1
    if L == 0:  # the full frame is one block reaching the last stage (tail included)
        Lb, e1, e2 = n, 0, k - 1 if terminated else 0
    want = synth.pack_bits(vref.decode_blocked_split(code, ol, n, Lb, e1, e2, word_stages(k), F, W, terminated,
                                                     nthreads=NCPU))
    if not np.array_equal(got, want):
        gb, wb = synth.unpack_bits(got, n), synth.unpack_bits(want, n)
        bad = np.nonzero(gb != wb)[0]
        raise AssertionError(f"{bad.size} of {n} bits differ; first at {bad[:8]}")
    if plain_equal:
        plain = synth.pack_bits(vref.decode_blocked(code, ol, n, Lb, e1, e2, terminated, nthreads=NCPU))
        np.testing.assert_array_equal(got, plain)
    return synth.unpack_bits(got, n)


def _awgn(k, gens, n, ebn0, seed, terminated=True):
    rng = np.random.default_rng(seed)
    bits = synth.info_bits(n, rng)
    return bits, synth.awgn_llr(synth.encode(k, gens, bits, terminated), ebn0, len(gens), rng)


GEOMS = [
    # n, L, v, v1, terminated
    (1, 8, 0, None, True), (40, 8, 35, None, True), (255, 32, 7, 3, True), (257, 256, 42, None, False),
    (1000, 0, 0, None, True), (1000, 0, 0, None, False), (1001, 128, 35, 30, True), (3333, 64, 12, 12, False),
    (6144, 256, 35, None, True), (6144, 1024, 45, None, True), (777, 8, 60, None, True), (5000, 512, 64, 20, True),
]
SPLITS = [(1, 0), (1, 2), (2, 1), (3, 5)]


@pytest.mark.parametrize("name", list(CODES))
@pytest.mark.parametrize("n,L,v,v1,terminated", GEOMS)
@pytest.mark.parametrize("F,W", SPLITS)
def test_geometry_sweep_awgn(dev, name, n, L, v, v1, terminated, F, W):
    k, gens = CODES[name]
    _, llr = _awgn(k, gens, n, 1.0, seed=n * 17 + L + v + 7 * F + W, terminated=terminated)
    _check(dev, k, gens, llr, n, L, v, F, W, v1, terminated)


@pytest.mark.parametrize("name", list(CODES))
def test_integer_llrs_with_ties(dev, name):
    # ties in the survivor choices and in the best states at subframe starts
    k, gens = CODES[name]
    rng = np.random.default_rng(15)
    for (n, L, v, F, W, terminated) in ((900, 256, 10, 1, 0, True), (900, 0, 0, 2, 1, False),
                                        (600, 128, 40, 1, 1, True)):
        N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * len(gens), -2, 2, rng)
        _check(dev, k, gens, llr, n, L, v, F, W, None, terminated)


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k5r12x"])
def test_all_zero_llrs(dev, name):
    # every metric ties: every chain starts from state 0 by the tie rule
    k, gens = CODES[name]
    n = 2000
    llr = np.zeros((n + k - 1) * len(gens), dtype=np.float32)
    _check(dev, k, gens, llr, n, 512, 40, 1, 0)
    _check(dev, k, gens, llr, n, 0, 0, 40, 1)


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k4r14"])
def test_int8_and_hard_inputs(dev, name):
    k, gens = CODES[name]
    bits, llr = _awgn(k, gens, 20000, 2.0, seed=23)
    q = vref.quantize_i8(llr, 4.0)
    _check(dev, k, gens, q, 20000, 512, 40, 2, 1)
    hard = (llr < 0).astype(np.uint8)
    _check(dev, k, gens, hard, 20000, 256, 42, 1, 2)


def test_one_subframe_is_the_plain_decoder(dev):
    # F so large that every block has one subframe: identical to the one-trace decode
    k, gens = CODES["k7r12"]
    _, llr = _awgn(k, gens, 30000, 1.5, seed=3)
    _check(dev, k, gens, llr, 30000, 512, 35, 1000, 2, plain_equal=True)


def test_most_subframes(dev):
    # 64 subframes of one word: a full frame of 1914 bits + 6 tail stages
    k, gens = CODES["k7r12"]
    _, llr = _awgn(k, gens, 1914, 2.0, seed=5)
    _check(dev, k, gens, llr, 1914, 0, 0, 1, 1)


@pytest.mark.parametrize("F,W", [(1, 1), (4, 2)])
def test_full_size_stream_k7(dev, F, W):
    # the 2^24-bit throughput stream in the benchmark's launch configuration
    # (L = 512, v = 35); the oracle decodes it completely (all host cores)
    k, gens = CODES["k7r12"]
    n = 1 << 24
    bits, llr = synth.make_stream("k7r12", n, 3.0, seed=1 + 3)
    got = _check(dev, k, gens, llr, n, 512, 35, F, W)
    print(f"full size F={F} W={W}: BER {np.mean(got != bits):.3e}")
