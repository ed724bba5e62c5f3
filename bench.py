"""Throughput benchmark of the blocked soft-decision Viterbi decoder on one MI355X.

Workload (the throughput configuration): the K=7 rate-1/2 code (171/133), one
continuous terminated stream of 2^24 uniform information bits, BPSK over AWGN
at Eb/N0 = 3 dB, FP32 LLRs resident in HBM; blocked decoding with cores of
L bits and overlap v = 5k = 35 (v1 = 17, v2 = 18).  One step = one decode of
the whole stream (one kernel launch).  The headline uses L = 256; every
L in {128, 256, 512, 1024} is also timed and reported under "sweep".

Prints one JSON line:  value = decoded information Mbps; roofline = the
decode kernel against the VALU (plain ALU) peak, work = 4 lane-ops (2 adds,
1 compare, 1 select) per state per trellis stage processed, overlap
included; cpu_baseline = the CPU oracle on a bounded sample of the same stream.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded info Mbps on 1 MI355X (K=7 r1/2 and batched mixed) + % roofline, p99 latency"

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 32-bit VALU lane-ops/s
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--ebn0", type=float, default=3.0)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-frames", type=int, default=8192)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def traffic_from_profiles(kernel_tag):
    """HBM bytes per launch measured by rocprofv3 counters, if recorded for the
    current kernel sources (profiles/<tag>_traffic.json carries a source hash)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("source_hash") != source_hash():
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2011_09337_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def time_decode(vit, torch, code, llr_d, out_d, n, L, v, steps, warmup):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        vit.decode(code, llr_d, n, L, v, out=out_d, stream=stream)
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        vit.decode(code, llr_d, n, L, v, out=out_d, stream=stream)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def cpu_baseline(code_np, llr, n, L, v):
    """The oracle as it stands, on the host cores: all-core blocked decode of
    the first 2^22 bits (terminated sample), and single-core on 2^19."""
    from oracle import vref
    import synth
    threads = len(os.sched_getaffinity(0))
    k, gens = synth.CODES["k7r12"]
    c = vref.make_code(k, list(gens))
    res = {}
    for tag, nb, th in (("all", 1 << 22, threads), ("one", 1 << 19, 1)):
        nb = min(nb, n)
        sub = llr[: (nb + k - 1) * 2]  # the first nb stages plus k-1 more as a tail
        t0 = time.perf_counter()
        vref.decode_blocked(c, sub, nb, L, v // 2, v - v // 2, True, nthreads=th)
        dt = time.perf_counter() - t0
        res[tag] = (nb / dt / 1e6, nb, dt, th)
    return res


BATCH_CODES = ("k7r12", "k7r13", "k9r12")


def batched_workload(nframes, seed=0):
    """Batched configuration: terminated frames, lengths uniform in [40, 6144],
    code uniform over K=7 r1/2, K=7 r1/3, K=9 r1/2, Eb/N0 uniform in [1, 5] dB."""
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    frames, chunks, bits, scales = [], [], [], []
    llr_off = out_off = 0
    for _ in range(nframes):
        cid = int(rng.integers(0, len(BATCH_CODES)))
        k, gens = synth.CODES[BATCH_CODES[cid]]
        n = int(rng.integers(40, 6145))
        ebn0 = float(rng.uniform(1.0, 5.0))
        b = synth.info_bits(n, rng)
        llr = synth.awgn_llr(synth.encode(k, gens, b, True), ebn0, len(gens), rng)
        frames.append((cid, 1, n, llr_off, out_off))
        chunks.append(llr)
        bits.append(b)
        # int8 scale: a noiseless symbol (|llr| = 2/sigma^2) maps to amplitude 8
        scales.append(8.0 * synth.noise_sigma(ebn0, len(gens)) ** 2 / 2.0)
        llr_off += llr.size
        out_off += (n + 7) // 8
    return frames, np.concatenate(chunks), out_off, bits, scales


def batch_stages(frames, tunes):
    """Trellis stages x states processed by a batch (the algorithmic ACS work is 4 lane-ops each)."""
    import synth
    work = 0
    for cid, term, n, _, _ in frames:
        k, _ = synth.CODES[BATCH_CODES[cid]]
        L, v, v1, _ = tunes[cid]
        v1 = v // 2 if v1 < 0 else v1
        v2 = v - v1
        N = n + (k - 1 if term else 0)
        for cs in range(0, n, L):
            ce = min(cs + L, n)
            work += (min(N, ce + v2) - max(0, cs - v1)) * (1 << (k - 1))
    return work


def bench_batched(vit, torch, args):
    import numpy as np
    import synth
    frames, llr, out_bytes, bits, scales = batched_workload(args.batched_frames)
    codes = [vit.make_code(*synth.CODES[c]) for c in BATCH_CODES]
    llr_d = torch.from_numpy(llr).cuda()
    q_d = torch.empty(llr.size, dtype=torch.int8, device="cuda")
    for (cid, term, n, lo, oo), sc in zip(frames, scales):
        k, gens = synth.CODES[BATCH_CODES[cid]]
        cnt = (n + (k - 1 if term else 0)) * len(gens)
        vit.vit_quantize_i8(llr_d.data_ptr() + 4 * lo, cnt, sc, q_d.data_ptr() + lo, None)
    out = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    b = vit.Batch()
    tunes = b.autotune(codes, frames, q_d, out)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        b.decode(codes, frames, q_d, out, stream=stream)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 2)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(steps):
        b.decode(codes, frames, q_d, out, stream=stream)
    s1.record(stream)
    torch.cuda.synchronize()
    ms = s0.elapsed_time(s1) / steps
    got = out.cpu().numpy()
    nbits = sum(f[2] for f in frames)
    err8 = sum(int(np.sum(synth.unpack_bits(got[f[4]:f[4] + (f[2] + 7) // 8], f[2]) != bt))
               for f, bt in zip(frames, bits))
    # the same frames and shapes with the fp32 LLRs, for the int8 BER cost
    out32 = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    b.decode(codes, frames, llr_d, out32, tune=tunes)
    torch.cuda.synchronize()
    g32 = out32.cpu().numpy()
    err32 = sum(int(np.sum(synth.unpack_bits(g32[f[4]:f[4] + (f[2] + 7) // 8], f[2]) != bt))
                for f, bt in zip(frames, bits))
    work = 4.0 * batch_stages(frames, tunes)
    b.close()
    return {
        "workload": f"{len(frames)} terminated frames, n uniform in [40, 6144] ({nbits} bits), code uniform over "
                    f"{'/'.join(BATCH_CODES)}, Eb/N0 uniform in [1, 5] dB, int8 LLRs (noiseless amplitude 8); "
                    f"one graph launch per step, autotuned shapes",
        "mbps": round(nbits / (ms * 1e-3) / 1e6, 2),
        "ms_per_step": round(ms, 4),
        "valu_frac": round(work / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS, 4),
        "tuning": {BATCH_CODES[i]: {"L": t[0], "v": t[1], "waves_per_block": t[3]} for i, t in enumerate(tunes)},
        "ber_int8": err8 / nbits,
        "ber_fp32_same_shapes": err32 / nbits,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the decoder has no multi-GPU path "
              f"in this build.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2011_09337_amd as vit
    import synth

    k, gens = synth.CODES["k7r12"]
    v = 5 * k
    n = 1 << args.n_log2
    bits, llr = synth.make_stream("k7r12", n, args.ebn0, seed=1 + int(args.ebn0))
    code = vit.make_code(k, gens)
    llr_d = torch.from_numpy(llr).cuda()
    out_d = torch.empty((n + 7) // 8, dtype=torch.uint8, device="cuda")

    Ls = [args.L] if args.no_sweep else sorted(set([128, 256, 512, 1024, args.L]))
    sweep = {}
    for L in Ls:
        ms, wall = time_decode(vit, torch, code, llr_d, out_d, n, L, v,
                               args.steps if L == args.L else max(3, args.steps // 4), args.warmup)
        g = vit.vit_query_geometry(code, n, L, v)
        ops = 4.0 * (1 << (k - 1)) * g.stages_total
        sweep[L] = {"ms": ms, "mbps": n / (ms * 1e-3) / 1e6, "tops": ops / (ms * 1e-3) / 1e12,
                    "stages": g.stages_total, "wall_s": wall}
        if L == args.L:
            head_wall = wall
    head = sweep[args.L]
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # decode once more for the BER of the headline configuration
    vit.decode(code, llr_d, n, args.L, v, out=out_d)
    torch.cuda.synchronize()
    got = synth.unpack_bits(out_d.cpu().numpy(), n)
    ber = float(np.mean(got != bits))

    llr_bytes = llr.nbytes
    hbm_alg_bytes = llr_bytes + (n + 7) // 8  # LLRs read once + packed output
    traffic = traffic_from_profiles(f"vit_blocked_k7r12_f32_L{args.L}")
    roofline = {
        "bound": "alu",
        "achieved": round(head["tops"], 3),
        "peak": round(VALU_PEAK_TOPS, 2),
        "unit": "T lane-op/s",
        "frac": round(head["tops"] / VALU_PEAK_TOPS, 4),
        "traffic": traffic,
        "hbm_achieved_GBps": round(hbm_alg_bytes / (head["ms"] * 1e-3) / 1e9, 1),
        "hbm_frac": round(hbm_alg_bytes / (head["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
    }
    cpu = None
    if not args.no_cpu:
        res = cpu_baseline(None, llr, n, args.L, v)
        mbps, nb, dt, th = res["all"]
        cpu = {"value": round(mbps, 3), "unit": "Mbps", "cores": th, "kind": "oracle",
               "sample": f"first {nb} bits of the stream, blocked L={args.L} v={v}, {dt:.2f} s",
               "single_core_mbps": round(res["one"][0], 3)}
    batched = None if args.no_batched else bench_batched(vit, torch, args)
    if batched:
        batched["vs_stream_fp32"] = round(batched["mbps"] / head["mbps"], 3)
    line = {
        "metric": METRIC,
        "value": round(head["mbps"], 2),
        "unit": "Mbps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"K=7 r1/2 (171/133) terminated stream of 2^{args.n_log2} info bits, FP32 LLRs, "
                               f"BPSK/AWGN Eb/N0={args.ebn0} dB; blocked L={args.L}, v={v} (v1={v // 2}, "
                               f"v2={v - v // 2})",
                   "n_bits": n, "L": args.L, "v": v, "ebn0_db": args.ebn0},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ber": ber,
        "batched": batched,
        "sweep": {str(L): {"mbps": round(s["mbps"], 1), "ms": round(s["ms"], 4),
                           "valu_frac": round(s["tops"] / VALU_PEAK_TOPS, 4)} for L, s in sweep.items()},
        "wall_s_timed": round(head_wall, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
