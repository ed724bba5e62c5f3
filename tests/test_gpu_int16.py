"""The 16-bit modulo-metric decoder (int8 and hard-decision inputs, two
blocks per wave) against the CPU oracle's exact integer decoders, bit for
bit: vref_decode_blocked_i8 (int64 metrics) for blocked decodes and
vref_decode_full_i8 / vref_decode_full_i16mod for full frames.

The 16-bit metrics wrap modulo 2^16 and decisions come from the sign of the
wrapped difference (eq. 3 in 16 bits); the cases below make the metrics wrap
many times (saturated runs of +-127 and -128), force ties (small integer
LLRs), pair blocks of different lengths in one wave (the first block of a
stream, the last, odd block counts, batches of mixed lengths) and run every
constraint length and rate the library supports."""
import os
import zlib

import numpy as np
import pytest

import synth
from oracle import vref
from test_gpu_parity import CODES

pytestmark = pytest.mark.gpu
NCPU = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def _gpu(dev, k, gens, q, n, L, v, v1=None, terminated=True, metric_bits=16):
    torch, vit = dev
    t = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    print(f"[gpu] int16 k={k} gens={[oct(g) for g in gens]} n={n} L={L} v={v} v1={v1} term={terminated} "
          f"bits={metric_bits} dtype={q.dtype}", flush=True)
    nb = (n + 7) // 8
    buf = torch.full((nb + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    vit.decode(vit.make_code(k, gens), t, n, L, v, v1=v1, terminated=terminated, metric_bits=metric_bits, out=buf)
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    assert (got[nb:] == 0xAB).all(), "the decode wrote past ceil(n/8) bytes"
    return got[:nb]


def _oracle(k, gens, q, n, L, v, v1=None, terminated=True):
    code = vref.make_code(k, list(gens))
    if L == 0:
        return synth.pack_bits(vref.decode_full(code, q, n, terminated))
    e1 = v // 2 if v1 is None else v1
    return synth.pack_bits(vref.decode_blocked(code, q, n, L, e1, v - e1, terminated, nthreads=NCPU))


def _same(got, want, n, what=""):
    if not np.array_equal(got, want):
        gb, wb = synth.unpack_bits(got, n), synth.unpack_bits(want, n)
        bad = np.nonzero(gb != wb)[0]
        raise AssertionError(f"{what}: {bad.size} of {n} bits differ; first at {bad[:8]}")


def _check(dev, k, gens, q, n, L, v, v1=None, terminated=True, bits=(16,)):
    want = _oracle(k, gens, q, n, L, v, v1, terminated)
    for mb in bits:
        _same(_gpu(dev, k, gens, q, n, L, v, v1, terminated, mb), want, n, f"metric_bits={mb}")


def _qawgn(k, gens, n, ebn0, seed, terminated=True, scale=8.0):
    rng = np.random.default_rng(seed)
    bits = synth.info_bits(n, rng)
    llr = synth.awgn_llr(synth.encode(k, gens, bits, terminated), ebn0, len(gens), rng)
    return vref.quantize_i8(llr, scale * synth.noise_sigma(ebn0, len(gens)) ** 2 / 2.0)


# geometries: odd and even block counts, a first block shorter than the
# second (paired in one wave), ragged last blocks, explicit v1, open ends
GEOMS = [
    # n, L, v, v1, terminated
    (1, 8, 0, None, True), (9, 8, 5, 0, True), (40, 8, 35, None, True), (41, 16, 0, None, False),
    (255, 32, 7, 3, True), (257, 256, 42, None, False), (1000, 0, 0, None, True), (1000, 0, 0, None, False),
    (1001, 128, 35, 30, True), (3333, 64, 12, 12, False), (6144, 256, 35, None, True), (6145, 1024, 45, None, True),
    (777, 8, 60, None, True), (2048, 512, 64, 64, False),
]


@pytest.mark.parametrize("name", list(CODES))
@pytest.mark.parametrize("n,L,v,v1,terminated", GEOMS)
def test_int16_geometry_sweep(dev, name, n, L, v, v1, terminated):
    k, gens = CODES[name]
    q = _qawgn(k, gens, n, 1.5, seed=n * 7 + L + v, terminated=terminated)
    _check(dev, k, gens, q, n, L, v, v1, terminated)


@pytest.mark.parametrize("terminated", [True, False])
@pytest.mark.parametrize("name", list(CODES))
def test_int16_edge_lengths_per_code(dev, name, terminated):
    # lengths at this code's own edges and at the block edges, overlaps 0, 1,
    # odd and 5k, the overlap split at both extremes and at the default; one
    # to three blocks, so a wave pairs a block with an empty partner or with
    # the ragged last one
    k, gens = CODES[name]
    L = 16
    for n in sorted({1, k - 1, k, k + 1, L - 1, L, L + 1, 2 * L + 1}):
        q = _qawgn(k, gens, n, 1.0, seed=2000 * k + 10 * n + terminated, terminated=terminated)
        for v in (0, 1, 2 * k + 1, 5 * k):
            for v1 in sorted({None, 0, v}, key=lambda x: -1 if x is None else x):
                _check(dev, k, gens, q, n, L, v, v1, terminated)


@pytest.mark.parametrize("name", list(CODES))
def test_int16_full_range_int8_and_ties(dev, name):
    # uniform int8 over the whole range (-128 included), and integer LLRs in
    # [-2, 2] (ties everywhere), with both metric widths
    k, gens = CODES[name]
    rng = np.random.default_rng(21)
    for (n, L, v, term) in ((2000, 128, 35, True), (600, 0, 0, False), (999, 8, 45, True), (513, 16, 10, False)):
        N = n + (k - 1 if term else 0)
        q = rng.integers(-128, 128, size=N * len(gens)).astype(np.int8)
        _check(dev, k, gens, q, n, L, v, None, term, bits=(16, 32, 0))
        t = rng.integers(-2, 3, size=N * len(gens)).astype(np.int8)
        _check(dev, k, gens, t, n, L, v, None, term, bits=(16, 32))


def _saturated(k, gens, n, kind, rng, terminated=True):
    N = n + (k - 1 if terminated else 0)
    m = N * len(gens)
    if kind == "codeword":      # noiseless codeword at full scale: one path gains 254 per stage
        bits = synth.info_bits(n, rng)
        c = synth.encode(k, gens, bits, terminated)
        return np.where(c == 0, 127, -127).astype(np.int8)
    if kind == "minus128":      # -128 everywhere
        return np.full(m, -128, dtype=np.int8)
    if kind == "signs":         # random signs at full scale, -128 for negatives
        return np.where(rng.random(m) < 0.5, 127, -128).astype(np.int8)
    if kind == "runs":          # long constant runs of either sign
        out = np.empty(m, dtype=np.int8)
        i = 0
        while i < m:
            ln = int(rng.integers(1, 400))
            out[i:i + ln] = 127 if rng.random() < 0.5 else -128
            i += ln
        return out
    raise ValueError(kind)


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k3r12", "k4r14"])
@pytest.mark.parametrize("kind", ["codeword", "minus128", "signs", "runs"])
def test_int16_saturated_wrapping(dev, name, kind):
    # blocks of ~4000 stages gaining up to 127*beta per stage: the 16-bit
    # metrics wrap dozens of times per block
    k, gens = CODES[name]
    rng = np.random.default_rng(zlib.crc32(f"{name}/{kind}".encode()))
    n = 20000
    q = _saturated(k, gens, n, kind, rng)
    Lw = 2048 if k >= 8 else 4000   # two K=9 blocks of 2112 stages fill 132 KiB of LDS
    _check(dev, k, gens, q, n, Lw, 64, bits=(16, 32))
    _check(dev, k, gens, q, n, 256, 35, bits=(16,))


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k5r12x"])
@pytest.mark.parametrize("kind", ["codeword", "signs", "runs"])
def test_int16_full_frame_vs_exact_and_modulo_oracles(dev, name, kind):
    # one full frame as long as the survivor storage of two blocks allows:
    # equal to the exact int64 full-frame decoder and to the oracle's own
    # 16-bit modulo decoder
    k, gens = CODES[name]
    rng = np.random.default_rng(len(kind) + k)
    n = 2400 if k >= 8 else 6000   # two K=9 blocks of 2408 stages: 151 KiB of survivors
    for term in (True, False):
        q = _saturated(k, gens, n, kind, rng, term)
        code = vref.make_code(k, list(gens))
        exact = synth.pack_bits(vref.decode_full(code, q, n, term))
        mod16 = synth.pack_bits(vref.decode_full_i16mod(code, q, n, term)[0])
        np.testing.assert_array_equal(mod16, exact)
        _same(_gpu(dev, k, gens, q, n, 0, 0, None, term, 16), exact, n, f"full frame {kind} term={term}")


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k4r14", "k5r12x"])
def test_int16_hard_decisions(dev, name):
    k, gens = CODES[name]
    n = 2400 if k >= 8 else 3000   # the full frame within two blocks' survivor storage
    rng = np.random.default_rng(17)
    coded = synth.encode(k, gens, synth.info_bits(n, rng), True)
    llr = synth.awgn_llr(coded, 3.0, len(gens), rng)
    hard = synth.hard_bits(llr)
    hard[hard != 0] = rng.integers(1, 256, size=int(np.sum(hard != 0)), dtype=np.uint8)
    q = np.where(hard != 0, -1, 1).astype(np.int8)
    for L, v in ((0, 0), (64, 35), (256, 45), (8, 3)):
        want = _oracle(k, gens, q, n, L, v)
        _same(_gpu(dev, k, gens, hard, n, L, v), want, n, f"hard L={L}")


@pytest.mark.parametrize("L", [128, 256, 512, 1024])
def test_int16_many_pairs(dev, L):
    # 2^21 bits: more pairs than resident waves (XCD-contiguous pair mapping)
    k, gens = CODES["k7r12"]
    n = (1 << 21) + 8 * 3   # an odd block count at every L
    q = _qawgn(k, gens, n, 2.0, seed=L)
    _check(dev, k, gens, q, n, L, 35)


CONFIG3 = [("k7r12", 512, 35), ("k7r13", 512, 35), ("k9r12", 256, 64)]


@pytest.mark.parametrize("name,L,v", CONFIG3)
def test_int16_full_size_three_codes(dev, name, L, v):
    # the three-code configuration: the same 2^24 information bits per code,
    # quantised to int8 on the GPU, decoded at the benchmark's block shapes;
    # the oracle decodes the same bytes completely (all host cores)
    torch, vit = dev
    k, gens = CODES[name]
    n = 1 << 24
    ebn0 = 3.0
    bits, llr = synth.make_stream(name, n, ebn0, seed=1 + 3)
    scale = 8.0 * synth.noise_sigma(ebn0, len(gens)) ** 2 / 2.0
    q = vit.quantize(torch.from_numpy(llr).cuda(), scale)
    torch.cuda.synchronize()
    qh = q.cpu().numpy()
    np.testing.assert_array_equal(qh, vref.quantize_i8(llr, scale))
    want = _oracle(k, gens, qh, n, L, v)
    for mb in (16, 32):
        print(f"[gpu] full size {name} L={L} v={v} bits={mb}", flush=True)
        got = vit.decode(vit.make_code(k, gens), q, n, L, v, metric_bits=mb)
        torch.cuda.synchronize()
        _same(got.cpu().numpy(), want, n, f"{name} metric_bits={mb}")
