"""The stream and batch kernels' setup computes, for codes whose generators
all tap both ends of the register, each slot's partner-branch metric address
from the generators rotated by the phase (scalar work) instead of from the
rotated slot index (vector work).  The two formulas agree for every phase and
slot: a check of that algebra (eq. 1 is linear over GF(2)), with both
formulas restated here; the GPU parity tests check the kernels themselves."""
import numpy as np


def _parity(x):
    return bin(x).count("1") & 1


def _general(gens, k, q, st):
    # partner predecessor of slot st at phase q: register (u << (k-1)) | rotr(st, q), low bit flipped;
    # the pattern is complemented when u = 1 (the slot keeps its metric negated)
    P, S, M = k - 1, 1 << (k - 1), (1 << len(gens)) - 1
    up = (st >> q) & 1
    iown = ((st >> q) | (st << (P - q))) & (S - 1)
    rb = ((up << (k - 1)) | iown) ^ 1
    c = sum(_parity(g & rb) << b for b, g in enumerate(gens))
    return (c ^ (M if up else 0)) << 2


def _both_taps(gens, k, q, st):
    # the same address from the generators' low k-1 bits rotated left by q
    P, S, M = k - 1, 1 << (k - 1), (1 << len(gens)) - 1
    c = 0
    for b, g in enumerate(gens):
        gl = g & (S - 1)
        c |= _parity((((gl << q) | (gl >> ((P - q) % P))) & (S - 1)) & st) << b
    return (c ^ M) << 2


def test_partner_address_of_codes_with_both_end_taps():
    rng = np.random.default_rng(5)
    codes = [(7, (0o171, 0o133)), (7, (0o133, 0o171, 0o165)), (9, (0o561, 0o753))]
    for k in range(3, 10):
        for _ in range(12):
            beta = int(rng.integers(2, 5))
            codes.append((k, tuple(int(rng.integers(0, 1 << k)) | (1 << (k - 1)) | 1 for _ in range(beta))))
    for k, gens in codes:
        for q in range(k - 1):
            for st in range(1 << (k - 1)):
                assert _general(gens, k, q, st) == _both_taps(gens, k, q, st), (k, gens, q, st)


def test_a_code_without_both_taps_needs_the_general_formula():
    # the reduction uses both end taps: without the oldest tap it fails somewhere
    k, gens = 5, (0o22, 0o35)
    assert any(_general(gens, k, q, st) != _both_taps(gens, k, q, st) for q in range(k - 1) for st in range(16))
