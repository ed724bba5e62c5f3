"""The synthetic input chain (Sec. V-B verification system) against closed forms,
and statistical trends of the paper's method (Sec. V-B, BER discussion)."""
import math

import numpy as np
import pytest

import synth
from oracle import vref


def _q(x):
    return 0.5 * math.erfc(x / math.sqrt(2.0))


@pytest.mark.parametrize("beta,ebn0", [(2, 0.0), (2, 3.0), (2, 6.0), (3, 0.0), (3, 3.0)])
def test_raw_bit_error_rate_matches_q_function(beta, ebn0):
    # Hard decisions on the channel output err with probability Q(sqrt(2 R Eb/N0)).
    rng = np.random.default_rng(17)
    n = 400000
    coded = rng.integers(0, 2, n, dtype=np.uint8)
    llr = synth.awgn_llr(coded, ebn0, beta, rng)
    p = _q(math.sqrt(2.0 * (1.0 / beta) * 10 ** (ebn0 / 10.0)))
    err = np.mean((llr < 0) != (coded == 1))
    sd = math.sqrt(p * (1 - p) / n)
    assert abs(err - p) < 5 * sd + 1e-6


def test_q_function_reference_values():
    # r1/2: 0.0789 at 3 dB, 0.0230 at 6 dB; r1/3: 0.2071 at 0 dB.
    assert _q(math.sqrt(10 ** 0.3)) == pytest.approx(0.0789, abs=2e-4)
    assert _q(math.sqrt(10 ** 0.6)) == pytest.approx(0.0230, abs=2e-4)
    assert _q(math.sqrt(2 / 3)) == pytest.approx(0.2071, abs=2e-4)


def test_llr_sign_convention():
    # positive LLR = bit 0 more likely (Sec. II-C)
    llr = synth.noiseless_llr(np.array([0, 1], dtype=np.uint8))
    assert llr[0] > 0 > llr[1]


def test_make_stream_is_seeded():
    a = synth.make_stream("k7r12", 100, 3.0, seed=0)
    b = synth.make_stream("k7r12", 100, 3.0, seed=0)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert a[1].dtype == np.float32 and a[1].size == 2 * 106


def test_pack_bits_lsb_first():
    bits = np.array([1, 0, 0, 0, 0, 0, 0, 0, 0, 1], dtype=np.uint8)
    np.testing.assert_array_equal(synth.pack_bits(bits), np.array([1, 2], dtype=np.uint8))
    np.testing.assert_array_equal(synth.unpack_bits(synth.pack_bits(bits), 10), bits)


def test_ber_falls_with_ebn0_and_blocked_gap_shrinks_with_v2():
    # Trends the paper reports: BER decreases with Eb/N0; the right overlap v2
    # drives convergence, so the disagreement with full-frame ML shrinks as v2
    # grows (Sec. V-B).  Statistical, on 2^16 bits.
    k, gens = synth.CODES["k7r12"]
    c = vref.make_code(k, list(gens))
    n = 1 << 16
    bers = []
    for ebn0 in (1.0, 2.0, 3.0):
        bits, llr = synth.make_stream("k7r12", n, ebn0, seed=21)
        ml = vref.decode_full(c, llr, n, True)
        bers.append(np.mean(ml != bits))
        if ebn0 == 2.0:
            outs = [vref.decode_blocked(c, llr, n, 64, 20, v2, True, nthreads=4) for v2 in (2, 6, 12, 24)]
            diffs = [np.mean(o != ml) for o in outs]
            assert diffs[0] > diffs[1] > diffs[2] > diffs[3]
            # with v2 = 24 the blocked decoder's BER is within 25% of ML's
            assert np.mean(outs[3] != bits) < 1.25 * bers[-1]
    assert bers[0] > bers[1] > bers[2]
    assert bers[1] < _q(math.sqrt(10 ** 0.2))  # coding gain over the raw channel


def test_hard_decision_costs_about_two_db():
    # Soft inputs are worth about 2 dB over hard decisions for this code
    # (Sec. I and II-C).  The hard-decision decoder is the same decoder on
    # integer LLRs +1 / -1 (coded bit 0 / 1).  Statistical, on 2^17 bits: find
    # the Eb/N0 at which hard decisions reach the soft-input BER at 2 dB, by
    # log-linear interpolation.
    k, gens = synth.CODES["k7r12"]
    c = vref.make_code(k, list(gens))
    n = 1 << 17

    def ber(ebn0, hard):
        bits, llr = synth.make_stream("k7r12", n, ebn0, seed=31)
        if hard:
            llr = np.where(synth.hard_bits(llr) != 0, -1, 1).astype(np.int8)
        return float(np.mean(vref.decode_full(c, llr, n, True) != bits))

    target = ber(2.0, False)
    grid = (3.5, 4.0, 4.5)
    hard = [ber(e, True) for e in grid]
    assert hard[0] > hard[1] > hard[2]
    assert hard[0] > target > hard[2]
    i = 0 if hard[1] < target else 1
    x0, x1 = grid[i], grid[i + 1]
    y0, y1 = math.log(hard[i]), math.log(hard[i + 1])
    gap = x0 + (math.log(target) - y0) * (x1 - x0) / (y1 - y0) - 2.0
    assert 1.5 < gap < 3.0, gap
