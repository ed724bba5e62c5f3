"""Pins of the oracle's parallel traceback in the paper's geometry (Sec. IV-D):
vref_decode_blocked_pt_{f32,i8}.

Each block's core is cut into subframes of f0 bits; subframe c is traced from
x_c = min(e, end_c + w) (the last one from the block end e) and keeps only its
own bits.  Its start state is the block's own at the block end, else the best
state after stage x_c - 1 (stored) or a random state (SplitMix64 of the seed,
the block and the subframe).  The geometry is recomputed here from that
definition, and each subframe is checked against exhaustive search over the
stages its chain saw; the generator against its published first outputs;
noiseless recovery against a bound derived from the trellis; the paper's BER
claims (the stored start beats the random one, errors fall with the inner
overlap and with longer subframes) as trends.
"""
import os
from functools import lru_cache

import numpy as np
import pytest

import synth
from oracle import vref

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = 2 ** 64 - 1
NTHREADS = max(1, min(16, len(os.sched_getaffinity(0))))


def _code(k, gens):
    return vref.make_code(k, list(gens))


def _splitmix64(seed, i):
    """SplitMix64 output i for `seed`, restated from its published definition."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def test_splitmix64_published_outputs():
    rows = [ln.strip() for ln in open(os.path.join(HERE, "golden", "splitmix64_seed0.txt"))
            if ln.strip() and not ln.startswith("#")]
    want = [int(r, 16) for r in rows]
    assert [vref.splitmix64(0, i) for i in range(len(want))] == want
    assert [_splitmix64(0, i) for i in range(len(want))] == want
    rng = np.random.default_rng(0)
    for _ in range(200):
        seed, i = int(rng.integers(0, 2 ** 63)) * 2 + 1, int(rng.integers(0, 2 ** 62))
        assert vref.splitmix64(seed, i) == _splitmix64(seed, i)


def _blocks(n, N, L, v1, v2):
    for b, cs in enumerate(range(0, n, L)):
        ce = min(cs + L, n)
        yield b, cs, ce, max(0, cs - v1), min(N, ce + v2)


def _subframes(cs, ce, e, f0, w):
    """(c, a, b, x): subframe c keeps bits [a, b) and is traced from stage x."""
    C = -(-(ce - cs) // f0)
    for c in range(C):
        a, b = cs + c * f0, min(cs + (c + 1) * f0, ce)
        x = e if c == C - 1 else min(e, b + w)
        yield c, a, b, x


GEOMS = [  # n, L, v1, v2, f0, w
    (17, 8, 2, 3, 3, 2), (13, 13, 0, 0, 4, 1), (16, 6, 4, 2, 1, 3), (12, 12, 0, 4, 5, 0),
    (11, 5, 1, 5, 2, 1), (10, 10, 3, 3, 9, 0), (14, 14, 0, 2, 3, 4), (15, 7, 3, 0, 2, 2),
]


@pytest.mark.parametrize("k,gens", [(3, (0o7, 0o5)), (4, (0o17, 0o13)), (5, (0o23, 0o35)),
                                    (4, (0o13, 0o15, 0o17, 0o11))])
@pytest.mark.parametrize("terminated", [True, False])
@pytest.mark.parametrize("rule", [vref.PT_STORED, vref.PT_RANDOM])
def test_pt_equals_bruteforce_per_subframe(k, gens, terminated, rule):
    # A chain from the block end gives the ML bits of the block window (end
    # state known only at the end of a terminated stream); a stored start
    # gives those of [s, x) with a free end; a random start j gives those of
    # [s, x) ending in state j.  Integer LLRs make ties, which must break as
    # in the full-frame case.
    c = _code(k, gens)
    beta = len(gens)
    rng = np.random.default_rng(400 + k + 10 * terminated + 100 * rule)
    seed = 0x1234_5678_9ABC_DEF1
    inner = 0
    for (n, L, v1, v2, f0, w) in GEOMS:
        N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * beta, -2, 2, rng)
        want = np.zeros(n, dtype=np.uint8)
        mask = np.zeros(n, dtype=bool)
        for (blk, cs, ce, s, e) in _blocks(n, N, L, v1, v2):
            if (k - 1) + (e - s) > 22:
                pytest.skip("window too long for exhaustive search")
            for (ch, a, b, x) in _subframes(cs, ce, e, f0, w):
                if x == e:
                    end_state = 0 if (terminated and e == N) else -1
                elif rule == vref.PT_STORED:
                    end_state = -1
                else:
                    end_state = _splitmix64(seed, (blk << 32) | ch) >> (65 - k)
                    if s == 0 and x < k - 1:
                        continue  # that state may be unreachable from the known start
                bf, _ = vref.bruteforce_window_to(c, llr.astype(np.float64), s, x, s == 0, end_state)
                want[a:b] = bf[a - s:b - s]
                mask[a:b] = True
                inner += x < e
        for dt in (np.float32, np.int8):
            got = vref.decode_blocked_pt(c, llr.astype(dt), n, L, v1, v2, f0, w, rule, seed, terminated)
            np.testing.assert_array_equal(got[mask], want[mask],
                                          err_msg=f"n={n} L={L} v1={v1} v2={v2} f0={f0} w={w} {dt}")
    assert inner >= 10


def test_pt_random_start_uses_the_seed():
    # different seeds pick different inner start states, so some bits change
    # (short overlap, noisy input); the stored rule ignores the seed
    k, gens = synth.CODES["k7r12"]
    c = _code(k, gens)
    bits, llr = synth.make_stream("k7r12", 20000, 1.0, seed=3)
    a = vref.decode_blocked_pt(c, llr, bits.size, 256, 20, 20, 16, 2, vref.PT_RANDOM, 1)
    b = vref.decode_blocked_pt(c, llr, bits.size, 256, 20, 20, 16, 2, vref.PT_RANDOM, 2)
    assert (a != b).sum() > 10
    s1 = vref.decode_blocked_pt(c, llr, bits.size, 256, 20, 20, 16, 2, vref.PT_STORED, 1)
    s2 = vref.decode_blocked_pt(c, llr, bits.size, 256, 20, 20, 16, 2, vref.PT_STORED, 2)
    np.testing.assert_array_equal(s1, s2)


@pytest.mark.parametrize("name", list(synth.CODES))
def test_pt_single_trace_cases_are_the_plain_blocked_decoder(name):
    # f0 >= L: one subframe per block, traced from the block end.  w >= L + v2:
    # every chain starts at the block end from the same state and follows the
    # same survivors, so the bits are those of one trace.  Either start rule.
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    bits, llr = synth.make_stream(name, 5000, 1.5, seed=8)
    want = vref.decode_blocked(c, llr, bits.size, 128, 20, 20, True)
    for (f0, w) in [(128, 0), (500, 3), (8, 148), (1, 200), (37, 150)]:
        for rule in (vref.PT_STORED, vref.PT_RANDOM):
            got = vref.decode_blocked_pt(c, llr, bits.size, 128, 20, 20, f0, w, rule, 5)
            np.testing.assert_array_equal(got, want, err_msg=f"f0={f0} w={w} rule={rule}")


def _longest_zero_output_run(k, gens):
    """Longest run of zero-output trellis branches starting in a nonzero state
    (a graph search on the encoder FSM; finite for non-catastrophic codes)."""
    S = 1 << (k - 1)

    def out(i, u):
        r = (u << (k - 1)) | i
        return any(bin(g & r).count("1") & 1 for g in gens)

    @lru_cache(None)
    def run(i):
        if i == 0:
            return 0
        nxt = [((u << (k - 2)) | (i >> 1)) for u in (0, 1) if not out(i, u)]
        return max([0] + [1 + run(j) for j in nxt])

    return max(run(i) for i in range(1, S))


@pytest.mark.parametrize("name", list(synth.CODES))
def test_pt_noiseless_recovery(name):
    # Noiseless input: the metric of a path is A times (beta*stages - 2 x its
    # Hamming distance to the codeword).  Stored start: the best state after
    # any stage is the transmitted one once v1 >= D (as for the plain decoder),
    # so every split recovers the bits.  Random start j: the best path into j
    # leaves the transmitted path at most m stages before x, where m stages of
    # a non-remerging difference excursion weigh at least floor(m / (D+1)) and
    # must not exceed the (k-1)*beta of the direct detour; so with
    # w >= (D+1)*((k-1)*beta+1) every kept bit is exact.
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    D = _longest_zero_output_run(k, gens)
    beta = len(gens)
    wr = (D + 1) * ((k - 1) * beta + 1)
    bits = synth.info_bits(1500, np.random.default_rng(12))
    for terminated in (True, False):
        llr = synth.noiseless_llr(vref.encode(c, bits, terminated))
        for (L, f0, w) in [(64, 8, 0), (200, 24, 3), (1500, 56, 25), (5, 1, 0), (300, 16, 45)]:
            got = vref.decode_blocked_pt(c, llr, bits.size, L, D, 0, f0, w, vref.PT_STORED, 0, terminated)
            np.testing.assert_array_equal(got, bits, err_msg=f"stored L={L} f0={f0} w={w}")
        for (L, f0) in [(256, 8), (300, 32), (1500, 56)]:
            got = vref.decode_blocked_pt(c, llr, bits.size, L, D, 0, f0, wr, vref.PT_RANDOM, 9, terminated)
            np.testing.assert_array_equal(got, bits, err_msg=f"random L={L} f0={f0} w={wr}")


def test_pt_error_trends_of_the_paper():
    # Sec. IV-D and its BER table: a chain's start is a guess that its inner
    # overlap corrects, so errors fall as w grows and as f0 grows (fewer
    # guesses), and a random start costs more than the stored best state (the
    # start-state figure: f = 256, v1 = v2 = 20).
    k, gens = synth.CODES["k7r12"]
    c = _code(k, gens)
    bits, llr = synth.make_stream("k7r12", 200000, 2.5, seed=9)
    plain = int((vref.decode_blocked(c, llr, bits.size, 256, 20, 20, True, nthreads=4) != bits).sum())

    def errs(f0, w, rule=vref.PT_STORED):
        return int((vref.decode_blocked_pt(c, llr, bits.size, 256, 20, 20, f0, w, rule, 77, True, nthreads=4)
                    != bits).sum())

    s8_5, s8_20, s8_40 = errs(8, 5), errs(8, 20), errs(8, 40)
    s32_5 = errs(32, 5)
    r8_20, r32_20 = errs(8, 20, vref.PT_RANDOM), errs(32, 20, vref.PT_RANDOM)
    assert s8_5 > s8_20 > plain * 0.9
    assert s8_40 <= 1.05 * plain + 5
    assert s8_5 > s32_5
    assert r8_20 > 1.2 * s8_20 + 10
    assert r32_20 > errs(32, 20) + 5
    assert r8_20 > r32_20


def test_pt_rejects_bad_arguments():
    c = _code(7, (0o171, 0o133))
    llr = np.zeros(2 * 16, dtype=np.float32)
    with pytest.raises(ValueError):
        vref.decode_blocked_pt(c, llr, 10, 4, 1, 1, 0, 1)
    with pytest.raises(ValueError):
        vref.decode_blocked_pt(c, llr, 10, 4, 1, 1, 2, -1)
    with pytest.raises(ValueError):
        vref.decode_blocked_pt(c, llr, 10, 4, 1, 1, 2, 1, start_rule=2)


def test_pt_random_start_reproduces_the_papers_ber_gaps():
    # The paper's BER-gap table of the parallel traceback (Table III: Eb/N0
    # gap at BER 1e-4 to the theoretical curve, K=7 r1/2, f = 300) against
    # this decoder with random chain starts (frames of 300 bits, v1 = 20,
    # right overlap v2 = w), the gap taken to the full-frame ML decode of the
    # same streams.  Two cells, 2^22 bits per Eb/N0 point (about 400 errors at
    # BER 1e-4, so about +-0.04 dB of estimate noise).
    k, gens = synth.CODES["k7r12"]
    c = _code(k, gens)
    n = 1 << 22
    grid = [3.0, 3.5, 4.0, 4.5, 5.0]
    cells = {(30, 24): 1.09, (40, 8): 0.43}
    errs = {"ml": []}
    for key in cells:
        errs[key] = []
    for e in grid:
        bits, llr = synth.make_stream("k7r12", n, e, seed=500 + int(e * 10))
        errs["ml"].append(int((vref.decode_full(c, llr.astype(np.float64), n) != bits).sum()))
        for (w, f0) in cells:
            got = vref.decode_blocked_pt(c, llr, n, 300, 20, w, f0, w, vref.PT_RANDOM, 99, True,
                                         nthreads=NTHREADS)
            errs[(w, f0)].append(int((got != bits).sum()))

    def at_1e4(es):
        bers = [max(x, 0.5) / n for x in es]
        for i in range(len(grid) - 1):
            if bers[i] >= 1e-4 > bers[i + 1]:
                y0, y1 = np.log(bers[i]), np.log(bers[i + 1])
                return grid[i] + (np.log(1e-4) - y0) * (grid[i + 1] - grid[i]) / (y1 - y0)
        raise AssertionError(f"BER 1e-4 not bracketed: {es}")

    ml = at_1e4(errs["ml"])
    for key, paper in cells.items():
        gap = at_1e4(errs[key]) - ml
        print(f"v2={key[0]} f0={key[1]}: gap {gap:.3f} dB (paper {paper})")
        assert abs(gap - paper) < 0.12, (key, gap, paper)
