"""De-puncturing (Sec. IV-E): the oracle's expansion against its definition,
noiseless recovery of punctured codes, the rate/BER ordering, and the C ABI's
argument checks (no GPU needed)."""
import numpy as np
import pytest

import synth
from oracle import vref

# Puncturing patterns are not given in the paper; these are common ones for the
# rate-1/2 mother code (keep = 1), rows = stages of one period, columns = outputs.
R23 = np.array([[1, 1], [1, 0]], dtype=np.uint8)
R34 = np.array([[1, 1], [1, 0], [0, 1]], dtype=np.uint8)


@pytest.mark.parametrize("dtype", [np.float32, np.int8])
@pytest.mark.parametrize("mask", [R23, R34, np.array([[1, 0, 1], [0, 1, 1]], dtype=np.uint8)])
def test_depuncture_inverts_puncture(dtype, mask):
    period, beta = mask.shape
    stages = 7 * period + 2  # a partial last period
    rng = np.random.default_rng(1)
    full = rng.integers(1, 100, size=stages * beta).astype(dtype)
    got = vref.depuncture(synth.puncture(full, mask), mask, stages)
    keep = np.tile(mask.astype(bool), (stages // period + 1, 1))[:stages].reshape(-1)
    np.testing.assert_array_equal(got[keep], full[keep])
    assert np.all(got[~keep] == 0)


def test_depuncture_rejects_wrong_count():
    with pytest.raises(ValueError):
        vref.depuncture(np.ones(5, dtype=np.float32), R23, 4)  # 4 stages keep 6


@pytest.mark.parametrize("mask", [R23, R34])
def test_noiseless_punctured_stream_decodes_exactly(mask):
    k, gens = synth.CODES["k7r12"]
    c = vref.make_code(k, list(gens))
    n = 2000
    rng = np.random.default_rng(5)
    bits = synth.info_bits(n, rng)
    coded = synth.encode(k, gens, bits, True)
    sent = synth.puncture(1.0 - 2.0 * coded.astype(np.float32), mask).astype(np.float32)
    llr = vref.depuncture(sent, mask, n + k - 1)
    np.testing.assert_array_equal(vref.decode_full(c, llr, n, True), bits)
    np.testing.assert_array_equal(vref.decode_blocked(c, llr, n, 64, 60, 60, True), bits)


def test_higher_punctured_rates_cost_more():
    # same Eb/N0, rate 1/2 < 2/3 < 3/4 in BER (statistical, 2^15 bits)
    k, gens = synth.CODES["k7r12"]
    c = vref.make_code(k, list(gens))
    n = 1 << 15
    bers = []
    for mask in (np.ones((1, 2), dtype=np.uint8), R23, R34):
        bits, sent = synth.make_punctured_stream("k7r12", n, 4.0, 7, mask)
        llr = vref.depuncture(sent, mask, n + k - 1)
        bers.append(np.mean(vref.decode_full(c, llr, n, True) != bits))
    assert bers[0] < bers[1] < bers[2]


def test_abi_depuncture_argument_errors():
    import paper_2011_09337_amd as vit
    FAKE = 0x1000
    bad = [
        (FAKE, 6, 7, R23, 4),     # unknown llr_type
        (FAKE, 5, 0, R23, 4),     # wrong count (4 stages keep 6)
        (FAKE, 0, 0, np.zeros((2, 2), np.uint8), 4),  # keeps nothing
        (None, 6, 0, R23, 4),     # NULL input
        (FAKE, 6, 0, np.ones((17, 4), np.uint8), 4),  # pattern longer than 64 slots
    ]
    for ptr, cnt, lt, mask, stages in bad:
        with pytest.raises(vit.VitError) as ei:
            vit.vit_depuncture(ptr, cnt, lt, mask.reshape(-1).tolist(), mask.shape[0], mask.shape[1], stages, FAKE)
        assert ei.value.status == vit.VIT_EINVAL
