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
        "sweep": {str(L): {"mbps": round(s["mbps"], 1), "ms": round(s["ms"], 4),
                           "valu_frac": round(s["tops"] / VALU_PEAK_TOPS, 4)} for L, s in sweep.items()},
        "wall_s_timed": round(head_wall, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
