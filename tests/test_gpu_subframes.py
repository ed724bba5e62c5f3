"""The parallel traceback of Sec. IV-D on the GPU against the oracle's
decoder of the same scheme (vref_decode_blocked_pt), bit for bit: each
block's core cut into subframes of f0 bits, subframe c traced by its own
chain from w stages above its end (the last one from the block end), inner
chains started from the best state after their start stage (the forward
pass keeps it) or from a random state drawn by SplitMix64."""
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


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def _check(dev, k, gens, llr, n, L, v, f0, w, rule=0, seed=0, v1=None, terminated=True, plain_equal=False):
    torch, vit = dev
    print(f"[gpu] k={k} gens={[oct(g) for g in gens]} n={n} L={L} v={v} v1={v1} f0={f0} w={w} rule={rule} "
          f"seed={seed} term={terminated} dtype={llr.dtype}", flush=True)
    t = torch.from_numpy(np.ascontiguousarray(llr)).cuda()
    nb = (n + 7) // 8
    buf = torch.full((nb + 64,), 0xAB, dtype=torch.uint8, device="cuda")
    vit.decode(vit.make_code(k, gens), t, n, L, v, v1=v1, terminated=terminated, subframe_bits=f0,
               subframe_overlap=w, subframe_start=rule, subframe_seed=seed, out=buf)
    torch.cuda.synchronize()
    got = buf.cpu().numpy()
    assert (got[nb:] == 0xAB).all(), "the decode wrote past ceil(n/8) bytes"
    got = got[:nb]
    e1 = v // 2 if v1 is None else v1
    code = vref.make_code(k, list(gens))
    ol = llr
    if llr.dtype == np.uint8:  # hard decisions: coded bit 0 -> LLR +1, 1 -> -1
        ol = np.where(llr == 0, 1, -1).astype(np.int8)
    Lb, e2 = L, v - e1
    if L == 0:  # the full frame is one block reaching the last stage (tail included)
        Lb, e1, e2 = n, 0, k - 1 if terminated else 0
    want = synth.pack_bits(vref.decode_blocked_pt(code, ol, n, Lb, e1, e2, f0, w, rule, seed, terminated,
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
    (3000, 296, 50, 25, True),
]
SPLITS = [(1, 0, 0), (3, 2, 0), (8, 25, 1), (24, 7, 0), (31, 0, 1), (56, 45, 0), (40, 30, 1), (2000, 3, 0)]


# every geometry with every split that leaves at most 64 subframes per block
# (more are refused before any device work: test_too_many_subframes)
SWEEP = [g + s for g in GEOMS for s in SPLITS if -(-(g[0] if g[1] == 0 else g[1]) // s[0]) <= 64]


@pytest.mark.parametrize("name", list(CODES))
@pytest.mark.parametrize("n,L,v,v1,terminated,f0,w,rule", SWEEP)
def test_geometry_sweep_awgn(dev, name, n, L, v, v1, terminated, f0, w, rule):
    k, gens = CODES[name]
    _, llr = _awgn(k, gens, n, 1.0, seed=n * 17 + L + v + 7 * f0 + w, terminated=terminated)
    _check(dev, k, gens, llr, n, L, v, f0, w, rule, seed=n + f0, v1=v1, terminated=terminated)


@pytest.mark.parametrize("name", list(CODES))
def test_integer_llrs_with_ties(dev, name):
    # ties in the survivor choices and in the best states at the chains' starts
    k, gens = CODES[name]
    rng = np.random.default_rng(15)
    for (n, L, v, f0, w, terminated) in ((900, 256, 10, 8, 0, True), (900, 0, 0, 16, 5, False),
                                         (600, 128, 40, 3, 1, True), (600, 128, 40, 24, 25, True)):
        N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * len(gens), -2, 2, rng)
        for rule in (0, 1):
            _check(dev, k, gens, llr, n, L, v, f0, w, rule, seed=5, terminated=terminated)


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k5r12x"])
def test_all_zero_llrs(dev, name):
    # every metric ties: every stored start is state 0 by the tie rule
    k, gens = CODES[name]
    n = 2000
    llr = np.zeros((n + k - 1) * len(gens), dtype=np.float32)
    _check(dev, k, gens, llr, n, 512, 40, 8, 0)
    _check(dev, k, gens, llr, n, 0, 0, 40, 10)
    _check(dev, k, gens, llr, n, 512, 40, 8, 3, rule=1, seed=99)


@pytest.mark.parametrize("name", ["k7r12", "k7r13", "k9r12", "k4r14"])
def test_int8_and_hard_inputs(dev, name):
    k, gens = CODES[name]
    bits, llr = _awgn(k, gens, 20000, 2.0, seed=23)
    q = vref.quantize_i8(llr, 4.0)
    _check(dev, k, gens, q, 20000, 512, 40, 24, 30)
    _check(dev, k, gens, q, 20000, 512, 40, 16, 20, rule=1, seed=3)
    hard = (llr < 0).astype(np.uint8)
    _check(dev, k, gens, hard, 20000, 256, 42, 8, 35)


@pytest.mark.parametrize("rule", [0, 1])
def test_one_subframe_is_the_plain_decoder(dev, rule):
    # f0 >= L: one subframe per block, traced from the block end
    k, gens = CODES["k7r12"]
    _, llr = _awgn(k, gens, 30000, 1.5, seed=3)
    _check(dev, k, gens, llr, 30000, 512, 35, 512, 20, rule, seed=1, plain_equal=True)


def test_overlap_reaching_the_block_end(dev):
    # w so large that every chain starts at the block end: the plain decoder
    k, gens = CODES["k7r12"]
    _, llr = _awgn(k, gens, 20000, 1.5, seed=4)
    _check(dev, k, gens, llr, 20000, 256, 42, 16, 1000, plain_equal=True)


def test_most_subframes(dev):
    # 64 subframes of one bit: a full frame of 64 bits, and blocks of 512 in
    # subframes of 8
    k, gens = CODES["k7r12"]
    _, llr = _awgn(k, gens, 64, 2.0, seed=5)
    _check(dev, k, gens, llr, 64, 0, 0, 1, 0)
    _, llr = _awgn(k, gens, 8192, 2.0, seed=6)
    for rule in (0, 1):
        _check(dev, k, gens, llr, 8192, 512, 35, 8, 25, rule, seed=11)


def test_too_many_subframes(dev):
    torch, vit = dev
    k, gens = CODES["k7r12"]
    llr = torch.zeros((1000 + 6) * 2, dtype=torch.float32, device="cuda")
    with pytest.raises(vit.VitError) as ei:
        vit.decode(vit.make_code(k, gens), llr, 1000, 520, 35, subframe_bits=8)
    assert ei.value.status == vit.VIT_EUNSUPPORTED


def test_random_starts_depend_on_the_seed(dev):
    # different seeds draw different start states; with w = 0 the errors they
    # leave differ
    k, gens = CODES["k7r12"]
    bits, llr = _awgn(k, gens, 20000, 3.0, seed=8)
    a = _check(dev, k, gens, llr, 20000, 256, 42, 8, 0, rule=1, seed=1)
    b = _check(dev, k, gens, llr, 20000, 256, 42, 8, 0, rule=1, seed=2)
    assert not np.array_equal(a, b)


@pytest.mark.parametrize("f0,w,rule", [(24, 25, 0), (56, 45, 0), (24, 25, 1)])
def test_full_size_stream_k7(dev, f0, w, rule):
    # the 2^24-bit throughput stream with the paper's frame of f = 296 bits
    # (a multiple of 8 near its 300) and v2 = 18; the oracle decodes it
    # completely (all host cores)
    k, gens = CODES["k7r12"]
    n = 1 << 24
    bits, llr = synth.make_stream("k7r12", n, 3.0, seed=1 + 3)
    got = _check(dev, k, gens, llr, n, 296, 35, f0, w, rule, seed=7)
    print(f"full size f0={f0} w={w} rule={rule}: BER {np.mean(got != bits):.3e}")
