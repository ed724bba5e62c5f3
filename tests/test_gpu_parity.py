"""GPU decoder (HIP, through the C ABI) against the CPU oracle, bit for bit.

Every case runs the same seeded input through both and compares the packed
decoded bits exactly: decisions are exact in both (fp32 sums rounded once in
the same order, or exact integers for int8 LLRs), so any difference is a bug.
"""
import os
import sys

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
    "k5r12x": (5, (0o22, 0o35)),        # generator without the newest-input tap
    "k6r12": (6, (0o53, 0o75)),
    "k8r12": (8, (0o247, 0o371)),
    "k5r13x": (5, (0o25, 0o33, 0o16)),  # generator without the oldest-input tap
}
NCPU = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def _gpu(dev, k, gens, llr, n, L, v, v1=None, terminated=True, stream=None):
    torch, vit = dev
    code = vit.make_code(k, gens)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    print(f"[gpu] k={k} gens={[oct(g) for g in gens]} n={n} L={L} v={v} v1={v1} term={terminated} "
          f"dtype={llr.dtype}", flush=True)
    nb = (n + 7) // 8
    buf = torch.full((nb + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()  # the fill is on torch's stream, the decode may be on another
    vit.decode(code, t, n, L, v, v1=v1, terminated=terminated, stream=stream, out=buf)
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    assert (got[nb:] == 0xAB).all(), "the decode wrote past ceil(n/8) bytes"
    return got[:nb]


def _oracle(k, gens, llr, n, L, v, v1=None, terminated=True):
    code = vref.make_code(k, list(gens))
    if L == 0:
        bits = vref.decode_full(code, llr, n, terminated)
    else:
        e1 = v // 2 if v1 is None else v1
        bits = vref.decode_blocked(code, llr, n, L, e1, v - e1, terminated, nthreads=NCPU)
    return synth.pack_bits(bits)


def _check(dev, k, gens, llr, n, L, v, v1=None, terminated=True):
    got = _gpu(dev, k, gens, llr, n, L, v, v1, terminated)
    want = _oracle(k, gens, llr, n, L, v, v1, terminated)
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        gb, wb = synth.unpack_bits(got, n), synth.unpack_bits(want, n)
        bad = np.nonzero(gb != wb)[0]
        raise AssertionError(f"{bad.size} of {n} bits differ; first at {bad[:8]}")


def _awgn(k, gens, n, ebn0, seed, terminated=True):
    rng = np.random.default_rng(seed)
    bits = synth.info_bits(n, rng)
    return synth.awgn_llr(synth.encode(k, gens, bits, terminated), ebn0, len(gens), rng)


# ----------------------------------------------------------------------------- config 1

def test_config1_full_and_blocked(dev):
    # K=7 r1/2, n = 4096, Eb/N0 = 3 dB, seed 0; full frame and L = 256, v = 42
    k, gens = CODES["k7r12"]
    bits, llr = synth.make_stream("k7r12", 4096, 3.0, seed=0)
    for L, v in ((0, 0), (256, 42)):
        _check(dev, k, gens, llr, 4096, L, v)
    got = synth.unpack_bits(_gpu(dev, k, gens, llr, 4096, 256, 42), 4096)
    ml = vref.decode_full(vref.make_code(k, list(gens)), llr, 4096, True)
    print(f"config1: BER blocked {np.mean(got != bits):.5f}, ML {np.mean(ml != bits):.5f}, "
          f"blocked vs ML {np.mean(got != ml):.5f}")


# ----------------------------------------------------------------------------- geometry sweep

GEOMS = [
    # n, L, v, v1, terminated
    (1, 8, 0, None, True), (6, 8, 3, None, True), (7, 8, 1, None, False), (8, 8, 0, None, True),
    (9, 8, 5, 0, True), (40, 8, 35, None, True), (40, 16, 0, None, False), (255, 32, 7, 3, True),
    (256, 256, 42, None, True), (257, 256, 42, None, False), (1000, 0, 0, None, True),
    (1000, 0, 0, None, False), (1001, 128, 35, 30, True), (3333, 64, 12, 12, False),
    (6144, 256, 35, None, True), (6144, 1024, 45, None, True), (777, 8, 60, None, True),
]


@pytest.mark.parametrize("name", list(CODES))
@pytest.mark.parametrize("n,L,v,v1,terminated", GEOMS)
def test_geometry_sweep_awgn(dev, name, n, L, v, v1, terminated):
    k, gens = CODES[name]
    llr = _awgn(k, gens, n, 1.5, seed=n * 31 + L + v, terminated=terminated)
    _check(dev, k, gens, llr, n, L, v, v1, terminated)


@pytest.mark.parametrize("terminated", [True, False])
@pytest.mark.parametrize("name", list(CODES))
def test_edge_lengths_per_code(dev, name, terminated):
    # lengths at this code's own edges (1, k-1, k, k+1) and at the block
    # edges (L-1, L, L+1, 2L+1), overlaps 0, 1, odd and 5k, with the
    # overlap split at both extremes as well as the default
    k, gens = CODES[name]
    L = 16
    for n in sorted({1, k - 1, k, k + 1, L - 1, L, L + 1, 2 * L + 1}):
        llr = _awgn(k, gens, n, 1.0, seed=1000 * k + 10 * n + terminated, terminated=terminated)
        for v in (0, 1, 2 * k + 1, 5 * k):
            for v1 in sorted({None, 0, v}, key=lambda x: -1 if x is None else x):
                _check(dev, k, gens, llr, n, L, v, v1, terminated)


# ----------------------------------------------------------------------------- ties and special values

@pytest.mark.parametrize("name", list(CODES))
def test_integer_llrs_with_ties(dev, name):
    k, gens = CODES[name]
    rng = np.random.default_rng(5)
    for (n, L, v, terminated) in ((500, 16, 10, True), (500, 0, 0, False), (300, 8, 3, True)):
        N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * len(gens), -2, 2, rng)
        _check(dev, k, gens, llr, n, L, v, None, terminated)


@pytest.mark.parametrize("name", ["k7r12", "k9r12", "k7r13", "k5r12x"])
def test_all_zero_llrs(dev, name):
    k, gens = CODES[name]
    n = 700
    llr = np.zeros((n + k - 1) * len(gens), dtype=np.float32)
    _check(dev, k, gens, llr, n, 64, 20)
    _check(dev, k, gens, llr, n, 0, 0)


@pytest.mark.parametrize("name", ["k7r12", "k9r12", "k7r13"])
def test_extreme_values(dev, name):
    k, gens = CODES[name]
    n = 600
    N = n + k - 1
    rng = np.random.default_rng(8)
    base = _awgn(k, gens, n, 2.0, seed=3)
    # huge magnitudes, denormals, signed zeros mixed in
    for scale in (1e30, 1e-41, 1.0):
        llr = (base * np.float32(scale)).astype(np.float32)
        llr[rng.integers(0, llr.size, 50)] = -0.0
        llr[rng.integers(0, llr.size, 50)] = 0.0
        _check(dev, k, gens, llr, n, 32, 12)
    assert N * len(gens) == base.size


# ----------------------------------------------------------------------------- int8 LLRs

@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k4r14", "k5r12x"])
def test_int8_llrs_exact(dev, name):
    k, gens = CODES[name]
    rng = np.random.default_rng(12)
    for (n, L, v) in ((2000, 128, 35), (600, 0, 0), (999, 8, 45)):
        N = n + k - 1
        q = rng.integers(-128, 128, size=N * len(gens)).astype(np.int8)
        _check(dev, k, gens, q, n, L, v)
        qs = vref.quantize_i8(_awgn(k, gens, n, 2.0, seed=n), 8.0)
        _check(dev, k, gens, qs, n, L, v)


# ----------------------------------------------------------------------------- many blocks

@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k4r14", "k5r12x"])
def test_hard_decisions_exact(dev, name):
    # hard-decision input (one byte per coded bit, 0 / nonzero) against the
    # oracle on the integer LLRs +1 / -1; nonzero bytes other than 1 included
    k, gens = CODES[name]
    n = 3000
    bits, llr = synth.make_stream(name, n, 3.0, seed=17) if name in synth.CODES else (None, None)
    if llr is None:
        rng = np.random.default_rng(17)
        coded = synth.encode(k, gens, synth.info_bits(n, rng), True)
        llr = synth.awgn_llr(coded, 3.0, len(gens), rng)
    hard = synth.hard_bits(llr)
    hard[hard != 0] = np.random.default_rng(3).integers(1, 256, size=int(np.sum(hard != 0)), dtype=np.uint8)
    q = np.where(hard != 0, -1, 1).astype(np.int8)
    for L, v in ((0, 0), (64, 35), (256, 45)):
        got = _gpu(dev, k, gens, hard, n, L, v)
        want = _oracle(k, gens, q, n, L, v)
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("L", [128, 256, 512, 1024])
def test_many_blocks_k7(dev, L):
    # 2^21 bits: more blocks than resident waves, so each wave loops over
    # blocks and the XCD-contiguous block mapping is exercised.
    k, gens = CODES["k7r12"]
    n = 1 << 21
    llr = _awgn(k, gens, n, 2.0, seed=L)
    _check(dev, k, gens, llr, n, L, 35)


def test_many_blocks_k9_and_r13(dev):
    for name, n, L, v in (("k9r12", 1 << 18, 256, 45), ("k7r13", 1 << 19, 256, 35)):
        k, gens = CODES[name]
        _check(dev, k, gens, _awgn(k, gens, n, 2.0, seed=9), n, L, v)


# ----------------------------------------------------------------------------- streams and determinism

def test_nondefault_stream_and_repeatability(dev):
    torch, vit = dev
    k, gens = CODES["k7r12"]
    n = 50000
    llr = _awgn(k, gens, n, 1.0, seed=77)
    s = torch.cuda.Stream()
    a = _gpu(dev, k, gens, llr, n, 256, 35, stream=s)
    b = _gpu(dev, k, gens, llr, n, 256, 35)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, _oracle(k, gens, llr, n, 256, 35))


def test_synchronous_entry_point(dev):
    torch, vit = dev
    k, gens = CODES["k7r12"]
    n = 3000
    llr = _awgn(k, gens, n, 3.0, seed=1)
    t = torch.from_numpy(llr).cuda()
    out = torch.zeros((n + 7) // 8, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    vit.vit_decode(vit.make_code(k, gens), t.data_ptr(), n, 256, 42, 0, out.data_ptr())
    np.testing.assert_array_equal(out.cpu().numpy(), _oracle(k, gens, llr, n, 256, 42))


# ----------------------------------------------------------------------------- full size

@pytest.mark.parametrize("L", [128, 512, 1024])
def test_full_size_stream_k7(dev, L):
    # the 2^24-bit stream of the throughput workload, in the benchmark's launch
    # configuration; the oracle decodes it completely (all host cores)
    k, gens = CODES["k7r12"]
    n = 1 << 24
    bits, llr = synth.make_stream("k7r12", n, 3.0, seed=1 + 3)
    _check(dev, k, gens, llr, n, L, 35)


# ----------------------------------------------------------------------------- maximum likelihood, exhaustively

@pytest.mark.parametrize("name", ["k3r12", "k7r12", "k7r13", "k9r12"])
def test_full_frame_gpu_is_ml_over_all_2_16_messages(dev, name):
    # the GPU's full-frame decode (L = 0) of a terminated 16-bit frame is the
    # best of all 2^16 messages, scored with the independent numpy
    # transmitter's codewords (no oracle involved); frames whose two best
    # scores lie within 1e-3 are redrawn, so that fp32 rounding cannot decide
    torch, vit = dev
    k, gens = CODES[name]
    beta = len(gens)
    n = 16
    G = np.stack([synth.encode(k, gens, np.eye(n, dtype=np.uint8)[i], True) for i in range(n)]).astype(np.int64)
    msgs = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)
    sign = 1.0 - 2.0 * ((msgs @ G) & 1)
    rng = np.random.default_rng(316)
    done = 0
    while done < 4:
        bits = synth.info_bits(n, rng)
        llr = synth.awgn_llr(synth.encode(k, gens, bits, True), 0.0, beta, rng)
        metrics = sign @ llr.astype(np.float64)
        top = np.sort(metrics)[-2:]
        if top[1] - top[0] < 1e-3:
            continue
        want = synth.pack_bits(msgs[int(np.argmax(metrics))].astype(np.uint8))
        got = _gpu(dev, k, gens, llr, n, 0, 0)
        np.testing.assert_array_equal(got, want, err_msg=f"{name} frame {done}")
        done += 1


# ----------------------------------------------------------------------------- maximum size

@pytest.mark.parametrize("kind", ["i8", "i8m16", "f32"])
def test_maximum_stream_size_sampled(dev, kind):
    # a K=7 r1/2 stream just under the library's limits (2^32 LLR bytes and
    # 2^31 stages), where the kernels' 32-bit byte offsets are at their
    # largest: integer-valued LLRs drawn on the device (so that the oracle's
    # window decoder in float64 is exact), sampled blocks, the last ones
    # included, against the oracle's decode of each block's window
    torch, vit = dev
    k, gens = CODES["k7r12"]
    code = vit.make_code(k, gens)
    ocode = vref.make_code(k, list(gens))
    L, v = 512, 35
    v1, v2 = v // 2, v - v // 2
    elem = 4 if kind == "f32" else 1
    N = ((1 << 32) - 64) // (2 * elem)
    N = min(N, (1 << 31) - 64)
    n = N - (k - 1)
    print(f"[gpu] maximum size {kind}: n={n} N={N} LLR bytes={2 * N * elem}", flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(2024)
    if kind != "f32":
        llr = torch.randint(-127, 128, (2 * N,), dtype=torch.int8, device="cuda", generator=g)
    else:
        llr = torch.randint(-40, 41, (2 * N,), dtype=torch.int32, device="cuda", generator=g).to(torch.float32)
    # i8m16: the 16-bit modulo-metric kernels (two blocks per wave)
    out = vit.decode(code, llr, n, L, v, metric_bits=16 if kind == "i8m16" else 0)
    torch.cuda.synchronize()
    nblocks = -(-n // L)
    rng = np.random.default_rng(5)
    picks = sorted(set([0, 1, nblocks // 2] + rng.integers(2, nblocks - 3, size=8).tolist()
                       + [nblocks - 3, nblocks - 2, nblocks - 1]))
    for b in picks:
        cs, ce = b * L, min(b * L + L, n)
        s, e = max(0, cs - v1), min(N, ce + v2)
        w = llr[2 * s:2 * e].cpu().numpy().astype(np.float64)
        want, _ = vref.window_f64(ocode, w, 0, e - s, s == 0, e == N, cs - s, ce - s)
        got = synth.unpack_bits(out[cs // 8:(ce + 7) // 8].cpu().numpy(), ce - cs)
        np.testing.assert_array_equal(got, want, err_msg=f"block {b} of {nblocks} ({kind})")
    del llr, out
    torch.cuda.empty_cache()


# ----------------------------------------------------------------------------- BER-gap reference

@pytest.mark.parametrize("ebn0", [2.5, 3.5, 4.5])
def test_ber_gap_ml_reference_is_ml(dev, ebn0):
    # bench.py's BER-gap grids take the blocked decoder with v1 = v2 = 128 as
    # the maximum-likelihood reference; on the first 2^18 bits of each of its
    # streams (same seeds) it agrees with the oracle's full-frame ML decode of
    # that prefix as an open stream, except where the prefix end is unknown
    # (the last 64 bits) and for a handful of bits at the lowest Eb/N0
    torch, vit = dev
    k, gens = CODES["k7r12"]
    n = 1 << 24
    bits, llr = synth.make_stream("k7r12", n, ebn0, seed=100 + int(ebn0 * 10))
    got = synth.unpack_bits(_gpu(dev, k, gens, llr, n, 512, 256, v1=128), n)
    m = 1 << 18
    ref = vref.decode_full(vref.make_code(k, list(gens)), llr[: m * 2], m, terminated=False)
    diff = int(np.sum(ref[: m - 64] != got[: m - 64]))
    print(f"Eb/N0 {ebn0}: {diff} bits differ from full-frame ML")
    assert diff <= (64 if ebn0 < 3.0 else 0)


# ----------------------------------------------------------------------------- finiteness pre-pass

def test_check_finite(dev):
    # vit_opts.check_finite: finite input decodes exactly as without the check;
    # a NaN or an infinity anywhere (vector and scalar paths of the scan,
    # aligned and unaligned buffers) is refused with VIT_EINVAL
    torch, vit = dev
    k, gens = CODES["k7r12"]
    code = vit.make_code(k, gens)
    n = 5000
    llr = _awgn(k, gens, n, 2.0, seed=77)
    N2 = llr.size
    for off in (0, 1):
        buf = torch.zeros(N2 + 1, dtype=torch.float32, device="cuda")
        t = buf[off:off + N2]
        t.copy_(torch.from_numpy(llr))
        plain = vit.decode(code, t, n, 256, 35).cpu().numpy()
        checked = vit.decode(code, t, n, 256, 35, check_finite=True).cpu().numpy()
        np.testing.assert_array_equal(checked, plain)
        for bad, pos in ((float("nan"), 0), (float("inf"), N2 - 1), (float("-inf"), N2 // 2 + 3)):
            t.copy_(torch.from_numpy(llr))
            t[pos] = bad
            print(f"[gpu] check_finite off={off} value={bad} at {pos}", flush=True)
            with pytest.raises(vit.VitError) as ei:
                vit.decode(code, t, n, 256, 35, check_finite=True)
            assert ei.value.status == vit.VIT_EINVAL
    q = vit.quantize(torch.from_numpy(llr).cuda(), 4.0)
    np.testing.assert_array_equal(vit.decode(code, q, n, 256, 35, check_finite=True).cpu().numpy(),
                                  vit.decode(code, q, n, 256, 35).cpu().numpy())
