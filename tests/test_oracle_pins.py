"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the paper's
generator strings (encoder figure, Sec. II-A) and eq. (1) worked by hand, an
independent numpy transmitter, algebraic identities (GF(2) linearity, the
complement identity eq. 8), exhaustive search over every input sequence, a
structural bound computed from the trellis graph, and closed forms.
"""
import os
from functools import lru_cache

import numpy as np
import pytest

import synth
from oracle import vref

HERE = os.path.dirname(os.path.abspath(__file__))

SMALL_CODES = [
    (3, (0o7, 0o5)),
    (4, (0o17, 0o13)),
    (5, (0o23, 0o35)),
    (5, (0o27, 0o31, 0o35)),
    (6, (0o53, 0o75)),
    (4, (0o13, 0o15, 0o17, 0o11)),
]


def _code(k, gens):
    return vref.make_code(k, list(gens))


# --------------------------------------------------------------------------- encoder, eq. (1)

def test_generator_strings_are_171_133():
    # Sec. II-A prints the example generators as 1111001 and 1011011 = octal 171, 133.
    assert int("1111001", 2) == 0o171
    assert int("1011011", 2) == 0o133


def test_encoder_impulse_response_golden():
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(HERE, "golden", "encoder_171_133_impulse.txt"))
            if ln.strip() and not ln.startswith("#")]
    want = np.array(rows, dtype=np.uint8)
    c = _code(7, (0o171, 0o133))
    got = vref.encode(c, np.array([1], dtype=np.uint8), terminated=True).reshape(-1, 2)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("name", list(synth.CODES))
def test_encoder_matches_independent_transmitter(name):
    k, gens = synth.CODES[name]
    rng = np.random.default_rng(5)
    for terminated in (True, False):
        bits = synth.info_bits(777, rng)
        np.testing.assert_array_equal(vref.encode(_code(k, gens), bits, terminated),
                                      synth.encode(k, gens, bits, terminated))


@pytest.mark.parametrize("name", list(synth.CODES))
def test_encoder_linear_over_gf2(name):
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    rng = np.random.default_rng(2)
    a, b = synth.info_bits(500, rng), synth.info_bits(500, rng)
    np.testing.assert_array_equal(vref.encode(c, a ^ b), vref.encode(c, a) ^ vref.encode(c, b))


@pytest.mark.parametrize("name,dfree", [("k7r12", 10), ("k7r13", 15), ("k9r12", 12)])
def test_free_distance(name, dfree):
    # Textbook free distances of these standard codes; the minimum weight of a
    # nonzero terminated codeword, found by exhaustive search over short inputs.
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    best = 10 ** 9
    for n in range(1, 11):
        for v in range(1, 1 << n):
            if not (v >> (n - 1)) & 1:
                continue  # leading input must be 1 (shifts are equivalent)
            bits = np.array([(v >> i) & 1 for i in range(n)], dtype=np.uint8)
            best = min(best, int(vref.encode(c, bits, True).sum()))
    assert best == dfree


# --------------------------------------------------------------------------- branch metric, eqs. (2) and (8)

def test_branch_metric_complement_identity_exact_fp32():
    # eq. (8): the complemented output pattern gives exactly the negated metric,
    # also after float32 rounding of the left-to-right sum.
    rng = np.random.default_rng(3)
    l = (rng.standard_normal((10000, 3)) * 7).astype(np.float32)
    for beta in (2, 3):
        for a in range(1 << beta):
            abar = (~a) & ((1 << beta) - 1)
            d = np.where((a & 1), -l[:, 0], l[:, 0]).astype(np.float32)
            e = np.where((abar & 1), -l[:, 0], l[:, 0]).astype(np.float32)
            for b in range(1, beta):
                d = (d + np.where((a >> b) & 1, -l[:, b], l[:, b])).astype(np.float32)
                e = (e + np.where((abar >> b) & 1, -l[:, b], l[:, b])).astype(np.float32)
            np.testing.assert_array_equal(e, -d)


@pytest.mark.parametrize("name", list(synth.CODES))
def test_noiseless_full_frame_metric_is_maximal(name):
    # On a noiseless stream every branch of the transmitted path matches, so the
    # decoded path is the transmitted one and its metric is beta per stage.
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    bits = synth.info_bits(300, np.random.default_rng(9))
    llr = synth.noiseless_llr(vref.encode(c, bits))
    out, met = vref.decode_full(c, llr.astype(np.float64), bits.size, True, want_metric=True)
    np.testing.assert_array_equal(out, bits)
    assert met == (bits.size + k - 1) * len(gens)


@pytest.mark.parametrize("k,gens", SMALL_CODES + [(7, (0o171, 0o133))])
def test_reported_metric_equals_independent_path_metric(k, gens):
    # Re-encode the decoded bits with the independent transmitter and sum
    # eq. (2) along that path in numpy (integer LLRs: every sum exact).
    c = _code(k, gens)
    rng = np.random.default_rng(k)
    for terminated in (True, False):
        n = 200
        N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * len(gens), -9, 9, rng).astype(np.float64)
        out, met = vref.decode_full(c, llr, n, terminated, want_metric=True)
        cw = synth.encode(k, gens, out, terminated).astype(np.float64)
        if not terminated:
            cw = cw[: N * len(gens)]
        assert met == float(np.sum(llr * (1.0 - 2.0 * cw)))


# --------------------------------------------------------------------------- full-frame ML vs exhaustive search

@pytest.mark.parametrize("k,gens", SMALL_CODES + [(7, (0o171, 0o133))])
@pytest.mark.parametrize("terminated", [True, False])
def test_full_frame_equals_bruteforce_integer_llrs_with_ties(k, gens, terminated):
    # Integer LLRs in [-2, 2] make many paths tie.  The oracle must return the
    # maximum metric and, among the maximisers, the sequence that is smallest
    # as an integer whose top bit is the latest input (lower predecessor wins
    # ACS ties, lowest state wins the final argmax).
    c = _code(k, gens)
    rng = np.random.default_rng(100 + k)
    beta = len(gens)
    for trial in range(6):
        n = int(rng.integers(1, 11))
        N = n + (k - 1 if terminated else 0)
        if n + 2 * (k - 1) > 22:
            n = 22 - 2 * (k - 1)
            N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * beta, -2, 2, rng).astype(np.float64)
        bf, bfm = vref.bruteforce_window(c, llr, 0, N, start_known=True, end_zero=terminated)
        for dt in (np.float64, np.float32, np.int8):
            out, met = vref.decode_full(c, llr.astype(dt), n, terminated, want_metric=True)
            np.testing.assert_array_equal(out, bf[:n], err_msg=f"dtype {dt} trial {trial}")
            assert float(met) == bfm


@pytest.mark.parametrize("k,gens", [(3, (0o7, 0o5)), (7, (0o171, 0o133)), (7, (0o133, 0o171, 0o165)),
                                    (9, (0o561, 0o753))])
def test_full_frame_is_ml_over_all_2_16_messages(k, gens):
    # terminated frames of n = 16 information bits: the full-frame decoder
    # returns the message, among all 2^16, whose codeword (the independent
    # numpy transmitter's) correlates best with the LLRs (eq. 2 summed over
    # the frame: sum of llr * (1 - 2c)); every codeword is built from the 16
    # impulse responses by GF(2) linearity of eq. 1
    c = _code(k, gens)
    rng = np.random.default_rng(216)
    beta = len(gens)
    n = 16
    G = np.stack([synth.encode(k, gens, np.eye(n, dtype=np.uint8)[i], True) for i in range(n)]).astype(np.int64)
    msgs = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)  # bit i = message bit i
    words = (msgs @ G) & 1                                                            # 2^16 codewords
    sign = 1.0 - 2.0 * words
    for trial in range(3):
        bits = synth.info_bits(n, rng)
        llr = synth.awgn_llr(synth.encode(k, gens, bits, True), 0.5, beta, rng).astype(np.float64)
        metrics = sign @ llr
        best = int(np.argmax(metrics))
        assert np.sum(metrics == metrics[best]) == 1  # real-valued LLRs: no tie
        out, met = vref.decode_full(c, llr, n, True, want_metric=True)
        np.testing.assert_array_equal(out, msgs[best].astype(np.uint8), err_msg=f"trial {trial}")
        assert met == pytest.approx(metrics[best], rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("k,gens", [(3, (0o7, 0o5)), (5, (0o23, 0o35)), (7, (0o171, 0o133)),
                                    (7, (0o133, 0o171, 0o165))])
def test_full_frame_equals_bruteforce_real_llrs(k, gens):
    c = _code(k, gens)
    rng = np.random.default_rng(7)
    beta = len(gens)
    for trial in range(4):
        n = 22 - 2 * (k - 1) if k > 3 else 12
        bits = synth.info_bits(n, rng)
        llr = synth.awgn_llr(synth.encode(k, gens, bits), 1.0, beta, rng).astype(np.float64)
        bf, bfm = vref.bruteforce_window(c, llr, 0, n + k - 1, start_known=True, end_zero=True)
        out, met = vref.decode_full(c, llr, n, True, want_metric=True)
        np.testing.assert_array_equal(out, bf[:n])
        assert met == pytest.approx(bfm, rel=1e-12, abs=1e-9)
        out32 = vref.decode_full(c, llr.astype(np.float32), n, True)
        np.testing.assert_array_equal(out32, bf[:n])


# --------------------------------------------------------------------------- blocked variant, Sec. III

def _geometry(n, N, L, v1, v2):
    blocks = []
    for cs in range(0, n, L):
        ce = min(cs + L, n)
        blocks.append((cs, ce, max(0, cs - v1), min(N, ce + v2)))
    return blocks


@pytest.mark.parametrize("k,gens", [(3, (0o7, 0o5)), (4, (0o17, 0o13)), (5, (0o23, 0o35)),
                                    (4, (0o13, 0o15, 0o17, 0o11))])
@pytest.mark.parametrize("terminated", [True, False])
def test_blocked_equals_bruteforce_per_window(k, gens, terminated):
    # Each block is, by definition, the ML sequence of its own window: known
    # start state only at stage 0, known end state only at the end of a
    # terminated stream, ties as in the full-frame case.  Window geometry is
    # recomputed here from the definition (cores of L, overlaps v1 / v2).
    c = _code(k, gens)
    beta = len(gens)
    rng = np.random.default_rng(200 + k)
    for (n, L, v1, v2) in [(17, 4, 2, 3), (13, 5, 0, 0), (10, 3, 4, 1), (9, 9, 0, 2), (11, 2, 1, 5)]:
        N = n + (k - 1 if terminated else 0)
        llr = synth.integer_llr(N * beta, -2, 2, rng)
        want = np.zeros(n, dtype=np.uint8)
        for (cs, ce, s, e) in _geometry(n, N, L, v1, v2):
            if (k - 1) + (e - s) > 22:
                pytest.skip("window too long for exhaustive search")
            bf, _ = vref.bruteforce_window(c, llr.astype(np.float64), s, e, start_known=(s == 0),
                                           end_zero=(terminated and e == N))
            want[cs:ce] = bf[cs - s:ce - s]
        for dt in (np.float32, np.float64, np.int8):
            got = vref.decode_blocked(c, llr.astype(dt), n, L, v1, v2, terminated)
            np.testing.assert_array_equal(got, want, err_msg=f"n={n} L={L} v1={v1} v2={v2} {dt}")


@pytest.mark.parametrize("k,gens", [(3, (0o7, 0o5)), (4, (0o17, 0o13)), (5, (0o23, 0o35)),
                                    (4, (0o13, 0o15, 0o17, 0o11))])
def test_window_is_ml_over_every_path_of_the_window(k, gens):
    # One window of the blocked decoder (Sec. III) is the best path over the
    # window's stages: from state 0 when the start is known, else from any
    # state at no cost; into state 0 when the end is fixed, else into any
    # state.  Every candidate path is enumerated here as k-1 history bits (the
    # start state) followed by the window's inputs and encoded by the
    # independent numpy transmitter (by GF(2) linearity of eq. 1), the history
    # stages' outputs dropped; its score is eq. 2 summed over the window.
    c = _code(k, gens)
    beta = len(gens)
    P = k - 1
    rng = np.random.default_rng(300 + 10 * k + beta)
    N = 40
    ties = 0
    for trial in range(12):
        W = int(rng.integers(1, 19 - P))
        s = int(rng.integers(0, N - W + 1))
        e = s + W
        start_known, end_zero = bool(trial & 1), bool(trial & 2) and W > P
        lo = int(rng.integers(s, e))
        hi = int(rng.integers(lo + 1, e + 1))
        llr = rng.normal(0.0, 2.0, N * beta)
        nin = P + W
        G = np.stack([synth.encode(k, gens, np.eye(nin, dtype=np.uint8)[i], False)
                      for i in range(nin)]).astype(np.int64)[:, P * beta:]
        seqs = ((np.arange(1 << nin)[:, None] >> np.arange(nin)[None, :]) & 1).astype(np.int64)
        keep = np.ones(len(seqs), dtype=bool)
        if start_known:
            keep &= ~seqs[:, :P].any(axis=1)
        if end_zero:
            keep &= ~seqs[:, nin - P:].any(axis=1)
        seqs = seqs[keep]
        metrics = (1.0 - 2.0 * ((seqs @ G) & 1)) @ llr[s * beta:e * beta]
        top = metrics.max()
        # paths with the same outputs tie exactly (a free start in a window
        # shorter than the register); any of the best is then a valid answer
        best = seqs[metrics == top][:, P + lo - s:P + hi - s].astype(np.uint8)
        got, met = vref.window_f64(c, llr, s, e, start_known, end_zero, lo, hi)
        what = f"s={s} e={e} known={start_known} end0={end_zero} emit=[{lo},{hi})"
        assert (best == got[None, :]).all(axis=1).any(), f"{what}: {got} not among {best}"
        assert met == pytest.approx(top, rel=1e-12, abs=1e-9), what
        ties += len(best) > 1
        # the oracle's own exhaustive search (the reference of other pins)
        # against the same enumeration: the whole window's bits, free or
        # fixed end state (state = last k-1 inputs, newest in the top bit)
        whole = seqs[metrics == top][:, P:].astype(np.uint8)
        bf, bfm = vref.bruteforce_window(c, llr, s, e, start_known, end_zero)
        assert (whole == bf[None, :]).all(axis=1).any() and bfm == pytest.approx(top, rel=1e-12, abs=1e-9), what
        endst = sum(seqs[:, nin - 1 - m] << (P - 1 - m) for m in range(P))
        j = int(rng.integers(0, 1 << P))
        mj = np.where(endst == j, metrics, -np.inf)
        if np.isfinite(mj).any():
            topj = mj.max()
            bfj, bfjm = vref.bruteforce_window_to(c, llr, s, e, start_known, j)
            wj = seqs[mj == topj][:, P:].astype(np.uint8)
            assert (wj == bfj[None, :]).all(axis=1).any() and bfjm == pytest.approx(topj, rel=1e-12, abs=1e-9), \
                f"{what} end state {j}"
    assert ties < 12


def _longest_zero_output_run(k, gens):
    """Longest run of zero-output trellis branches that starts in a nonzero state
    (a graph search on the encoder FSM, independent of any decoder)."""
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
def test_blocked_noiseless_recovery(name):
    # Two paths that match a noiseless window equally well differ by a
    # zero-output path.  Such a path can only start in a nonzero state (the
    # unknown start of an interior window) and reaches state 0 within D stages,
    # D = longest zero-output run.  So with v1 >= D every core bit is exact, for
    # every L and every v2 (including 0).
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    D = _longest_zero_output_run(k, gens)
    assert 1 <= D < 2 * k
    bits = synth.info_bits(1500, np.random.default_rng(11))
    for terminated in (True, False):
        llr = synth.noiseless_llr(vref.encode(c, bits, terminated))
        for L in (1, 7, 64, 1500):
            for v2 in (0, 1, 5):
                for v1 in (D, D + 3):
                    got = vref.decode_blocked(c, llr, bits.size, L, v1, v2, terminated)
                    np.testing.assert_array_equal(got, bits, err_msg=f"L={L} v1={v1} v2={v2}")


@pytest.mark.parametrize("name", list(synth.CODES))
def test_blocked_single_block_equals_full_frame(name):
    k, gens = synth.CODES[name]
    c = _code(k, gens)
    bits, llr = synth.make_stream(name, 1000, 2.0, seed=4)
    full = vref.decode_full(c, llr, 1000, True)
    for L in (1000, 5000):
        np.testing.assert_array_equal(vref.decode_blocked(c, llr, 1000, L, 0, k - 1, True), full)
    # open-ended stream: the single block ends at the last stage either way
    bits2 = bits
    llr2 = synth.awgn_llr(synth.encode(k, gens, bits2, False), 2.0, len(gens), np.random.default_rng(1))
    np.testing.assert_array_equal(vref.decode_blocked(c, llr2, 1000, 1000, 0, 0, False),
                                  vref.decode_full(c, llr2, 1000, False))


def test_blocked_result_independent_of_threads():
    k, gens = synth.CODES["k7r12"]
    c = _code(k, gens)
    bits, llr = synth.make_stream("k7r12", 20000, 1.0, seed=6)
    a = vref.decode_blocked(c, llr, bits.size, 128, 17, 18, True, nthreads=1)
    b = vref.decode_blocked(c, llr, bits.size, 128, 17, 18, True, nthreads=4)
    np.testing.assert_array_equal(a, b)


def test_blocked_rejects_bad_geometry():
    c = _code(7, (0o171, 0o133))
    llr = np.zeros(2 * 16, dtype=np.float32)
    with pytest.raises(ValueError):
        vref.decode_blocked(c, llr, 10, 0, 1, 1, True)
    with pytest.raises(ValueError):
        vref.decode_blocked(c, llr, 10, 4, -1, 1, True)


# --------------------------------------------------------------------------- int8 quantiser

def test_quantize_round_half_even_and_saturation():
    x = np.array([0.5, 1.5, 2.5, -0.5, -1.5, -2.5, 0.49999997, 126.5, 127.5, 300.0, -300.0, -127.5, 3.25],
                 dtype=np.float32)
    want = np.array([0, 2, 2, 0, -2, -2, 0, 126, 127, 127, -127, -127, 3], dtype=np.int8)
    np.testing.assert_array_equal(vref.quantize_i8(x, 1.0), want)
    # the product is rounded to float32 first, then to the nearest integer
    np.testing.assert_array_equal(vref.quantize_i8(np.array([0.1], np.float32), 25.0), np.array([2], np.int8))
    assert vref.quantize_i8(np.array([-200.0, 200.0], np.float32), 1.0).min() == -127


def _adversarial_i8(code, nst, rng):
    """Saturated int8 LLRs over nst stages, in runs of random kind and length:
    random signs at +-127, a noiseless codeword at +-127 (the best path pulls
    away from the rest as fast as it can), all zeros (every compare a tie),
    and constant +127 or -127."""
    beta = code.beta
    parts, left = [], nst
    while left > 0:
        m = min(left, int(rng.integers(64, 4097)))
        kind = int(rng.integers(0, 5))
        if kind == 0:
            x = np.where(rng.random(m * beta) < 0.5, -127, 127)
        elif kind == 1:
            coded = vref.encode(code, rng.integers(0, 2, m, dtype=np.uint8), terminated=False)
            x = np.where(coded != 0, -127, 127)
        elif kind == 2:
            x = np.zeros(m * beta)
        else:
            x = np.full(m * beta, 127 if kind == 3 else -127)
        parts.append(x.astype(np.int8))
        left -= m
    return np.concatenate(parts)


@pytest.mark.parametrize("k,gens,log2_stages", [(7, (0o171, 0o133), 20), (7, (0o133, 0o171, 0o165), 18),
                                                (9, (0o561, 0o753), 18)])
@pytest.mark.parametrize("terminated", [True, False])
def test_int16_modulo_metrics_decide_like_exact_integers(k, gens, log2_stages, terminated):
    # 16-bit metrics modulo 2^16, compared by the sign of the wrapped
    # difference, take the exact integer decisions as long as compared metrics
    # differ by less than 2^15: path metrics of one stage differ by at most
    # (k-1)*2*127*beta (any state reaches any other in k-1 steps), 9144 /
    # 13716 / 12192 here, plus the 2^14 start offset of unreachable states in
    # the first k-1 stages.  Over 2^18-2^20 saturated stages the metrics wrap
    # hundreds of times or more, so a plain compare of the stored values would
    # fail.
    code = _code(k, gens)
    rng = np.random.default_rng(1000 + k + 10 * len(gens) + int(terminated))
    nst = 1 << log2_stages
    n = nst - (k - 1 if terminated else 0)
    q = _adversarial_i8(code, nst, rng)
    exact, m_exact = vref.decode_full(code, q, n, terminated, want_metric=True)
    mod, m_mod = vref.decode_full_i16mod(code, q, n, terminated)
    assert abs(m_exact) > (1 << 16) * 500, "the metrics must wrap many times"
    np.testing.assert_array_equal(mod, exact)
    assert (m_mod - m_exact) % (1 << 16) == 0


