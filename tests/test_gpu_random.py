"""Randomised parity: seeded random codes (k 3..9, beta 2..4, any generators
with both end taps or not), lengths, block shapes, overlaps, termination,
input kinds (FP32, int8, hard bytes) and subframe settings, each decoded on
the GPU and by the CPU oracle and compared bit for bit."""
import os

import numpy as np
import pytest

import synth
from oracle import vref

pytestmark = pytest.mark.gpu
NCPU = max(1, min(16, len(os.sched_getaffinity(0))))


def random_case(rng):
    k = int(rng.integers(3, 10))
    beta = int(rng.integers(2, 5))
    gens = tuple(int(rng.integers(1, 1 << k)) for _ in range(beta))
    n = int(rng.integers(1, 3001))
    L = 0 if rng.random() < 0.1 else 8 * int(rng.integers(1, 129))
    v = int(rng.integers(0, 81))
    v1 = None if rng.random() < 0.5 else int(rng.integers(0, v + 1))
    term = bool(rng.random() < 0.7)
    kind = ("f32", "i8", "hard")[int(rng.integers(0, 3))]
    sub = (0, 0, 0, 0) if rng.random() < 0.6 else (int(rng.integers(1, 65)), int(rng.integers(0, 50)),
                                                     int(rng.integers(0, 2)), int(rng.integers(0, 1 << 62)))
    if sub[0]:  # at most 64 subframes per block
        sub = (max(sub[0], -(-(n if L == 0 else L) // 64)),) + sub[1:]
    return k, gens, n, L, v, v1, term, kind, sub


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_random_cases(dev, seed):
    torch, vit = dev
    rng = np.random.default_rng(1000 + seed)
    ran = 0
    for case in range(40):
        k, gens, n, L, v, v1, term, kind, (f0, w, rule, sseed) = random_case(rng)
        N = n + (k - 1 if term else 0)
        llr = synth.awgn_llr(synth.encode(k, gens, synth.info_bits(n, rng), term), float(rng.uniform(0.0, 4.0)),
                             len(gens), rng)
        if kind == "i8":
            x = vref.quantize_i8(llr, float(rng.choice([2.0, 4.0, 16.0])))
            ol = x
        elif kind == "hard":
            x = (llr < 0).astype(np.uint8)
            ol = np.where(x == 0, 1, -1).astype(np.int8)
        else:
            x = llr
            ol = llr
        print(f"[gpu] seed={seed} case={case} k={k} gens={[oct(g) for g in gens]} n={n} L={L} v={v} v1={v1} "
              f"term={term} {kind} f0={f0} w={w} rule={rule} seed={sseed}", flush=True)
        try:
            got = vit.decode(vit.make_code(k, gens), torch.from_numpy(np.ascontiguousarray(x)).cuda(), n, L, v,
                             v1=v1, terminated=term, subframe_bits=f0, subframe_overlap=w, subframe_start=rule,
                             subframe_seed=sseed)
            torch.cuda.synchronize()
        except vit.VitError as err:
            # only shapes the device cannot hold may be refused
            assert err.status == vit.VIT_EUNSUPPORTED, str(err)
            continue
        got = got.cpu().numpy()
        e1 = v // 2 if v1 is None else v1
        Lb, e2 = L, v - e1
        if L == 0:
            Lb, e1, e2 = n, 0, k - 1 if term else 0
        c = vref.make_code(k, list(gens))
        if f0 > 0:
            want = vref.decode_blocked_pt(c, ol, n, Lb, e1, e2, f0, w, rule, sseed, term, nthreads=NCPU)
        else:
            want = vref.decode_blocked(c, ol, n, Lb, e1, e2, term, nthreads=NCPU)
        want = synth.pack_bits(want)
        if not np.array_equal(got, want):
            gb, wb = synth.unpack_bits(got, n), synth.unpack_bits(want, n)
            bad = np.nonzero(gb != wb)[0]
            raise AssertionError(f"case {case}: {bad.size} of {n} bits differ; first at {bad[:8]}")
        ran += 1
    assert ran >= 30


@pytest.mark.parametrize("seed", [1, 2])
def test_random_batches(dev, seed):
    # a batch of frames over up to four random codes, random lengths and
    # termination, one input kind per batch, random shapes per code; every
    # frame equals the oracle's blocked decode of that frame alone
    torch, vit = dev
    rng = np.random.default_rng(2000 + seed)
    for trial in range(3):
        ncodes = int(rng.integers(1, 5))
        codes = []
        for _ in range(ncodes):
            k = int(rng.integers(3, 10))
            beta = int(rng.integers(2, 5))
            codes.append((k, tuple(int(rng.integers(1, 1 << k)) for _ in range(beta))))
        tunes = []
        for k, _ in codes:
            v = int(rng.integers(0, 70))
            tunes.append((8 * int(rng.integers(2, 65)), v, -1 if rng.random() < 0.5 else int(rng.integers(0, v + 1)),
                          int(rng.integers(1, 3))))
        kind = ("f32", "i8", "hard")[int(rng.integers(0, 3))]
        frames, chunks, olls = [], [], []
        llr_off = out_off = 0
        for f in range(int(rng.integers(20, 120))):
            cid = int(rng.integers(0, ncodes))
            k, gens = codes[cid]
            n = int(rng.integers(1, 4000))
            term = int(rng.random() < 0.7)
            llr = synth.awgn_llr(synth.encode(k, gens, synth.info_bits(n, rng), bool(term)),
                                 float(rng.uniform(0.5, 4.0)), len(gens), rng)
            if kind == "i8":
                x = vref.quantize_i8(llr, 4.0)
                ol = x
            elif kind == "hard":
                x = (llr < 0).astype(np.uint8)
                ol = np.where(x == 0, 1, -1).astype(np.int8)
            else:
                x = ol = llr
            gap = int(rng.integers(0, 4))
            chunks.append(np.zeros(gap, dtype=x.dtype))
            llr_off += gap
            frames.append((cid, term, n, llr_off, out_off))
            chunks.append(x)
            olls.append(ol)
            llr_off += x.size
            out_off += (n + 7) // 8 + int(rng.integers(0, 3))
        allx = np.concatenate(chunks)
        vcodes = [vit.make_code(k, g) for k, g in codes]
        print(f"[gpu] random batch seed={seed} trial={trial} codes={codes} tunes={tunes} {kind} "
              f"frames={len(frames)}", flush=True)
        out = torch.full((out_off + 1,), 0xAB, dtype=torch.uint8, device="cuda")
        b = vit.Batch()
        try:
            b.decode(vcodes, frames, torch.from_numpy(allx).cuda(), out, tune=tunes)
            torch.cuda.synchronize()
        except vit.VitError as err:
            assert err.status == vit.VIT_EUNSUPPORTED, str(err)
            b.close()
            continue
        b.close()
        got = out.cpu().numpy()
        for (cid, term, n, lo, oo), ol in zip(frames, olls):
            k, gens = codes[cid]
            L, v, v1, _ = tunes[cid]
            v1 = v // 2 if v1 < 0 else v1
            want = synth.pack_bits(vref.decode_blocked(vref.make_code(k, list(gens)), ol, n, L, v1, v - v1,
                                                       bool(term), nthreads=NCPU))
            np.testing.assert_array_equal(got[oo:oo + want.size], want,
                                          err_msg=f"trial {trial} frame code {cid} n={n} term={term}")
