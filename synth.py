"""Seeded synthetic inputs for the Viterbi decoder: the paper's verification
chain (Sec. V-B): uniform random bits -> convolutional encoder (eq. 1) ->
BPSK over AWGN at a given Eb/N0 -> soft LLRs.

This module holds no decoder arithmetic.  It serves both the GPU path and the
CPU oracle as their common source of inputs (tests, smoke check, benchmark).
Its encoder is an independent numpy model of the transmitter; the tests check
it against the oracle's encoder.

Channel model:
  x = 1 - 2c                       (bit 0 -> +1, so a positive LLR means "0")
  sigma = sqrt(1 / (2 R Eb/N0))    (R = 1/beta; tail rate loss ignored)
  y = x + sigma * z,  z ~ N(0, 1)
  llr = 2 y / sigma^2              (computed in float64, rounded once to float32)
The paper prints the noise deviation in a garbled form; the reading above is
the standard one and is pinned by the raw bit-error-rate test Q(sqrt(2R Eb/N0)).
"""
import math

import numpy as np

# Codes of the workloads: (k, generators in octal, listed in output order).
CODES = {
    "k7r12": (7, (0o171, 0o133)),        # the paper's (2,1,7) code, Sec. V-A
    "k7r13": (7, (0o133, 0o171, 0o165)),
    "k9r12": (9, (0o561, 0o753)),
}


def info_bits(n, rng):
    return rng.integers(0, 2, size=int(n), dtype=np.uint8)


def encode(k, gens, bits, terminated=True):
    """Transmitter model of eq. (1): register bit k-1 holds in_t, bit 0 in_{t-k+1};
    output b = parity(gens[b] & register).  Returns N*beta uint8, time-major."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = bits.size
    N = n + (k - 1 if terminated else 0)
    x = np.zeros(N + k - 1, dtype=np.uint8)          # k-1 leading zeros: the initial state
    x[k - 1:k - 1 + n] = bits
    out = np.zeros((N, len(gens)), dtype=np.uint8)
    for b, g in enumerate(gens):
        acc = np.zeros(N, dtype=np.uint8)
        for m in range(k):                           # tap m multiplies in_{t-m}
            if (g >> (k - 1 - m)) & 1:
                acc ^= x[k - 1 - m:k - 1 - m + N]
        out[:, b] = acc
    return out.reshape(-1)


def noise_sigma(ebn0_db, beta):
    rate = 1.0 / beta
    return float(np.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0))))


def awgn_llr(coded, ebn0_db, beta, rng):
    """BPSK + AWGN + LLR (float32), noise drawn from rng after whatever it already drew."""
    coded = np.asarray(coded, dtype=np.uint8)
    sigma = noise_sigma(ebn0_db, beta)
    x = 1.0 - 2.0 * coded.astype(np.float64)
    y = x + sigma * rng.standard_normal(coded.size)
    return (2.0 * y / sigma ** 2).astype(np.float32)


def noiseless_llr(coded, amplitude=1.0):
    return (amplitude * (1.0 - 2.0 * np.asarray(coded, dtype=np.float64))).astype(np.float32)


def make_stream(code_name, n, ebn0_db, seed, terminated=True):
    """One stream: bits from default_rng(seed), then the noise from the same generator."""
    k, gens = CODES[code_name]
    rng = np.random.default_rng(seed)
    bits = info_bits(n, rng)
    coded = encode(k, gens, bits, terminated)
    llr = awgn_llr(coded, ebn0_db, len(gens), rng)
    return bits, llr


def puncture(values, mask):
    """Transmitter side of puncturing: keep the values (time-major, beta per
    stage) whose slot the (period, beta) 0/1 pattern marks."""
    mask = np.asarray(mask, dtype=bool)
    period, beta = mask.shape
    v = np.asarray(values).reshape(-1, beta)
    keep = np.tile(mask, (v.shape[0] // period + 1, 1))[: v.shape[0]]
    return v[keep]


def make_punctured_stream(code_name, n, ebn0_db, seed, mask, terminated=True):
    """Bits, then the punctured coded bits sent over BPSK/AWGN at the punctured
    rate (LLR = 2y/sigma^2, float64 rounded once to float32)."""
    k, gens = CODES[code_name]
    rng = np.random.default_rng(seed)
    bits = info_bits(n, rng)
    sent = puncture(encode(k, gens, bits, terminated), mask)
    mask = np.asarray(mask, dtype=bool)
    rate = mask.shape[0] / mask.sum()
    sigma = math.sqrt(1.0 / (2.0 * rate * 10.0 ** (ebn0_db / 10.0)))
    y = (1.0 - 2.0 * sent.astype(np.float64)) + sigma * rng.standard_normal(sent.size)
    return bits, (2.0 * y / sigma ** 2).astype(np.float32)


def hard_bits(llr):
    """Hard decisions of soft inputs: coded bit 1 where the LLR is negative."""
    return (np.asarray(llr) < 0).astype(np.uint8)


def integer_llr(num, lo, hi, rng):
    """Small integer-valued LLRs (float32): exact sums, many ties."""
    return rng.integers(lo, hi + 1, size=int(num)).astype(np.float32)


def pack_bits(bits):
    """Bit t -> byte t >> 3, bit position t & 7 (LSB first); pad bits zero."""
    return np.packbits(np.asarray(bits, dtype=np.uint8), bitorder="little")


def unpack_bits(packed, n):
    return np.unpackbits(np.asarray(packed, dtype=np.uint8), bitorder="little")[:n]
