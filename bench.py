"""Throughput benchmark of the blocked soft-decision Viterbi decoder on one MI355X.

Workload (the throughput configuration): the K=7 rate-1/2 code (171/133), one
continuous terminated stream of 2^24 uniform information bits, BPSK over AWGN
at Eb/N0 = 3 dB, FP32 LLRs resident in HBM; blocked decoding with cores of
L bits and overlap v = 5k = 35 (v1 = 17, v2 = 18).  One step = one decode of
the whole stream (one kernel launch).  The headline uses L = 512; every
L in {128, 256, 512, 1024} is also timed and reported under "sweep".

Prints one JSON line:  value = decoded information Mbps; roofline = the
decode kernel against MI355X's published vector ALU peak, work = 4
operations (2 adds, 1 compare, 1 select) per state per trellis stage
processed, overlap included; cpu_baseline = the CPU oracle on a bounded
sample of the same stream.
"""
import argparse
import json
import os
import queue
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded info Mbps on 1 MI355X (K=7 r1/2 and batched mixed) + % roofline, p99 latency"

# MI355X's published fp32 vector peak: 157.3 TFLOP/s = 256 CUs x 2.4 GHz x
# 128 FMA lanes per CU per clock x 2 flops.  Each algorithmic operation of
# the decoder (an add, a compare or a select on one state) counts as one
# operation against it, as an fp32 add counts as one flop; the 16-bit integer
# path's packed instructions do two such operations per lane, which is the
# same 157.3 T operations/s at the FMA issue rate.
ALU_PEAK_TOPS = 157.3
# Secondary, labelled separately: the peak of this operation mix at the issue
# rates gfx950 shows for its forms (adds at the FMA rate, 2 cycles per wave64
# instruction; compares and max/min/med3 at 4 cycles, as measured with timing
# probes): 256 lane-ops per 12 cycles per SIMD.
MIX_PEAK_TOPS = 256 * 4 * 2.4e9 * (4 * 64) / (2 * 2 + 4 + 4) / 1e12
HBM_PEAK_GBPS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=512,
                    help="headline block length (the fastest of the configured sweep 128..1024)")
    ap.add_argument("--n-log2", type=int, default=24)
    ap.add_argument("--ebn0", type=float, default=3.0)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--subframes", default=None, metavar="F0:W",
                    help="headline decode with the parallel traceback: subframes of F0 bits, W stages of overlap")
    ap.add_argument("--no-ml-check", action="store_true",
                    help="skip the headline's comparison with the ML reference decode")
    ap.add_argument("--no-subframe-probe", action="store_true",
                    help="skip the side measurement of the parallel traceback")
    ap.add_argument("--precision", action="store_true",
                    help="print the int8-vs-FP32 BER sweep (three codes, 0..6 dB) and exit")
    ap.add_argument("--table3", action="store_true",
                    help="print the parallel traceback's grid (f0 x inner overlap): BER gap to ML and throughput, "
                         "stored and random chain starts, and exit")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-frames", type=int, default=8192)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--table2", action="store_true",
                    help="only the BER-gap sweep over f (=L) x v2 (the paper's Table II grid), then exit")
    ap.add_argument("--batched-tune", default=None,
                    help="fixed batched shapes 'L:v:waves,...' per code instead of autotuning")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="seconds per serving load point (the serving configuration runs 60 s)")
    ap.add_argument("--serve-pool", type=int, default=4096)
    ap.add_argument("--serve-arena-mb", type=int, default=256)
    ap.add_argument("--serve-max-items", type=int, default=1 << 16,
                    help="blocks per serving iteration at most")
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
    """Hash of the sources that define the blocked decode kernel and its launch."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2011_09337_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f in ("vit_decoder.h", "vit_internal.h", "vit_launch.hip") or f.startswith("vit_kernels_k"):
            # (the subframe instances, vit_kernels_sub_k*, are other kernels)
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def subframe_kw(sub):
    """decode() keywords of an (f0, w[, start rule]) parallel-traceback
    setting (None = one trace per block)."""
    if sub is None:
        return {}
    kw = dict(subframe_bits=sub[0], subframe_overlap=sub[1])
    if len(sub) > 2:
        kw["subframe_start"] = sub[2]
    return kw


def time_decode(vit, torch, code, llr_d, out_d, n, L, v, steps, warmup, sub=None):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        vit.decode(code, llr_d, n, L, v, out=out_d, stream=stream, **subframe_kw(sub))
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        vit.decode(code, llr_d, n, L, v, out=out_d, stream=stream, **subframe_kw(sub))
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def cpu_baseline(code_np, llr, n, L, v, ml=True):
    """The oracle as it stands, on the host cores: all-core blocked decode of
    the whole stream (best of 3 passes, about 10-30 core-seconds), and
    single-core on its first 2^21 bits.  With ml, also the full-frame
    maximum-likelihood decode of the whole stream (Algorithms 1-2 over every
    stage, float64 metrics, one core), returned as res["ml_bits"]."""
    import numpy as np
    from oracle import vref
    import synth
    threads = len(os.sched_getaffinity(0))
    k, gens = synth.CODES["k7r12"]
    c = vref.make_code(k, list(gens))
    res = {}
    if ml:
        t0 = time.perf_counter()
        res["ml_bits"] = vref.decode_full(c, llr.astype(np.float64), n, True)
        res["ml_s"] = time.perf_counter() - t0
    for tag, nb, th, reps in (("all", n, threads, 3), ("one", 1 << 21, 1, 1)):
        nb = min(nb, n)
        sub = llr[: (nb + k - 1) * 2]  # the first nb stages plus k-1 more as a tail
        best = None
        for _ in range(reps):
            t0 = time.perf_counter()
            vref.decode_blocked(c, sub, nb, L, v // 2, v - v // 2, True, nthreads=th)
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        res[tag] = (nb / best / 1e6, nb, best, th)
    return res


BATCH_CODES = ("k7r12", "k7r13", "k9r12")


def default_overlap(k):
    """The library's default overlap of the batch and serving paths."""
    return 5 * k if k <= 7 else 8 * (k - 1)


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
    frames_np = vit.frames_array(frames)  # the frame list as the C ABI reads it
    b = vit.Batch()
    if args.batched_tune:
        tunes = []
        for t in args.batched_tune.split(","):
            L_, v_, w_ = (int(x) for x in t.split(":"))
            tunes.append((L_, v_, -1, w_))
    else:
        tunes = b.autotune(codes, frames_np, q_d, out)
    stream = torch.cuda.current_stream()
    steps = max(3, args.steps // 2)

    def time_batch(plan, fr, tu=None):
        tu = tunes if tu is None else tu
        for _ in range(2):
            plan.decode(codes, fr, q_d, out, tune=tu, stream=stream)
        torch.cuda.synchronize()
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        for _ in range(steps):
            plan.decode(codes, fr, q_d, out, tune=tu, stream=stream)
        s1.record(stream)
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / steps

    # each code's frames alone (one kernel per launch): that kernel's rate
    per_code = {}
    for cid, name in enumerate(BATCH_CODES):
        sub = frames_np[frames_np["code_id"] == cid]
        if len(sub) == 0:
            continue
        ms_c = time_batch(b, sub)
        fl = [f for f in frames if f[0] == cid]
        bits_c = sum(f[2] for f in fl)
        work_c = 4.0 * batch_stages(fl, tunes)
        per_code[name] = {"frames": len(fl), "mbps": round(bits_c / (ms_c * 1e-3) / 1e6, 1),
                          "ms": round(ms_c, 4), "alu_frac": round(work_c / (ms_c * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4)}
    # the same batch and shapes with 16-bit modulo path metrics, then with
    # shapes autotuned for them (a 16-bit wave holds two blocks, so its best
    # shapes differ)
    b16 = vit.Batch(metric_bits=16)
    ms16 = time_batch(b16, frames_np)
    out16 = out.cpu().numpy()
    int16_tuned = None
    if not args.batched_tune:
        tunes16 = b16.autotune(codes, frames_np, q_d, out)
        ms16t = time_batch(b16, frames_np, tunes16)
        int16_tuned = {"mbps": round(sum(f[2] for f in frames) / (ms16t * 1e-3) / 1e6, 2),
                       "ms_per_step": round(ms16t, 4),
                       "alu_frac": round(4.0 * batch_stages(frames, tunes16) / (ms16t * 1e-3) / 1e12 / ALU_PEAK_TOPS,
                                         4),
                       "tuning": {BATCH_CODES[i]: {"L": t[0], "v": t[1], "waves_per_block": t[3]}
                                  for i, t in enumerate(tunes16)}}
    b16.close()
    ms = time_batch(b, frames_np)
    got = out.cpu().numpy()
    nbits = sum(f[2] for f in frames)
    err8 = sum(int(np.sum(synth.unpack_bits(got[f[4]:f[4] + (f[2] + 7) // 8], f[2]) != bt))
               for f, bt in zip(frames, bits))
    # the same frames and shapes with the fp32 LLRs, for the int8 BER cost
    out32 = torch.zeros(out_bytes, dtype=torch.uint8, device="cuda")
    b.decode(codes, frames_np, llr_d, out32, tune=tunes)
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
        "metric_bits": 32,
        "mbps": round(nbits / (ms * 1e-3) / 1e6, 2),
        "ms_per_step": round(ms, 4),
        "alu_frac": round(work / (ms * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4),
        "mix_frac": round(work / (ms * 1e-3) / 1e12 / MIX_PEAK_TOPS, 4),
        "per_code": per_code,
        "int16": {"mbps": round(nbits / (ms16 * 1e-3) / 1e6, 2), "ms_per_step": round(ms16, 4),
                  "alu_frac": round(work / (ms16 * 1e-3) / 1e12 / ALU_PEAK_TOPS, 4),
                  "bits_equal_to_32": bool(np.array_equal(out16, got)), "own_tuning": int16_tuned},
        "tuning": {BATCH_CODES[i]: {"L": t[0], "v": t[1], "waves_per_block": t[3]} for i, t in enumerate(tunes)},
        "ber_int8": err8 / nbits,
        "ber_fp32_same_shapes": err32 / nbits,
        "tuning_tuples": [tuple(t) for t in tunes],
    }


def serving_pool(vit, torch, count, seed=7):
    """Serving configuration's frame pool: lengths lognormal (median 1024,
    sigma_ln = 1) clipped to [40, 16384], code uniform over the three codes,
    terminated, Eb/N0 uniform in [1, 5] dB, int8 LLRs quantised on the GPU.
    Returns (frames [(cid, n, llr_off, out_off)], pinned host region)."""
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    frames, chunks, scales = [], [], []
    pos = 0
    for _ in range(count):
        cid = int(rng.integers(0, len(BATCH_CODES)))
        k, gens = synth.CODES[BATCH_CODES[cid]]
        n = int(np.clip(np.round(rng.lognormal(np.log(1024.0), 1.0)), 40, 16384))
        ebn0 = float(rng.uniform(1.0, 5.0))
        llr = synth.awgn_llr(synth.encode(k, gens, synth.info_bits(n, rng), True), ebn0, len(gens), rng)
        lo = pos
        oo = (lo + llr.size + 15) // 16 * 16
        pos = (oo + (n + 7) // 8 + 15) // 16 * 16
        frames.append((cid, n, lo, oo))
        chunks.append(llr)
        scales.append(8.0 * synth.noise_sigma(ebn0, len(gens)) ** 2 / 2.0)
    f32 = torch.zeros(pos, dtype=torch.float32, device="cuda")
    q = torch.zeros(pos, dtype=torch.int8, device="cuda")
    for (cid, n, lo, oo), llr, sc in zip(frames, chunks, scales):
        f32[lo:lo + llr.size] = torch.from_numpy(llr).cuda()
        vit.vit_quantize_i8(f32.data_ptr() + 4 * lo, llr.size, sc, q.data_ptr() + lo, None)
    torch.cuda.synchronize()
    host = torch.empty(pos, dtype=torch.uint8).pin_memory()
    host.copy_(q.view(torch.uint8).cpu())
    return frames, host


def bench_serving(vit, torch, args, tunes):
    """Serving configuration: Poisson arrivals at fractions of the measured
    capacity, each load point args.serve_seconds long; latency from arrival to
    the host seeing the frame's last iteration finish."""
    import numpy as np
    import synth
    frames, host = serving_pool(vit, torch, args.serve_pool)
    codes = [vit.make_code(*synth.CODES[c]) for c in BATCH_CODES]
    srv = vit.Server(codes, host, tune=tunes, llr_type=vit.VIT_LLR_I8, arena_bytes=args.serve_arena_mb << 20,
                     max_frames=1 << 16, max_items=args.serve_max_items, max_pending=1 << 24)
    base = host.data_ptr()
    P = len(frames)
    pool = np.zeros(P, dtype=vit.REQUEST_DTYPE)
    for i, (cid, n, lo, oo) in enumerate(frames):
        pool[i] = (cid, 1, n, base + lo, base + oo, i, 0)
    mean_bits = float(np.mean(pool["n"]))
    # algorithmic work of a mean pool frame under the shapes (the arrivals
    # cycle through the pool, so a point's completed frames carry about this
    # much each): 4 operations per state per trellis stage
    mean_work = 4.0 * batch_stages([(cid, 1, n, 0, 0) for cid, n, _, _ in frames], tunes) / P

    def requests(first, count, arrivals=None):
        idx = (first + np.arange(count)) % P
        r = pool[idx].copy()
        r["tag"] = first + np.arange(count)
        if arrivals is not None:
            r["arrival_ns"] = arrivals
        return r

    def submit_all(r):
        off = 0
        while off < len(r):
            st, acc = srv.submit(r[off:])
            off += acc
            if st == vit.VIT_EBUSY:
                time.sleep(0.0005)

    try:
        # capacity: a closed backlog of the pool, repeated
        srv.stats(reset=True)
        cap = None
        for rep in range(3):
            # a backlog long enough that filling and draining the pipeline
            # (a few ms) is small beside the run (about 60 ms)
            nreq = P * (4 if rep == 0 else 64)
            t0 = time.monotonic_ns()
            submit_all(requests(0, nreq))
            srv.drain(timeout_ms=120000)
            while len(srv.poll(1 << 16)):
                pass
            st = srv.stats(reset=True)
            dt = (st["last_done_ns"] - t0) * 1e-9
            fps = st["completed"] / dt
            cap = fps if cap is None else max(cap, fps)
        points = []
        rng = np.random.default_rng(3)
        tag = 0
        for load in (0.25, 0.5, 0.75, 1.0):
            # a native thread replays the arrival process chunk by chunk while
            # this one builds the next chunk and drains completions
            rate = load * cap
            chunk_s = 0.25
            nchunks = max(1, int(round(args.serve_seconds / chunk_s)))
            per = max(1, int(rate * chunk_s))
            todo = queue.Queue(maxsize=2)
            errs = []

            def replay():
                try:
                    while True:
                        r = todo.get()
                        if r is None:
                            return
                        srv.submit_paced(r)
                except Exception as e:  # surfaced below
                    errs.append(e)

            th = threading.Thread(target=replay, daemon=True)
            th.start()
            t_next = None
            for c in range(nchunks):
                offs = np.cumsum(rng.exponential(1e9 / rate, size=per))
                r = requests(tag, per)
                tag += per
                if t_next is None:
                    t_next = time.monotonic_ns() + 2_000_000
                r["arrival_ns"] = (t_next + offs).astype(np.int64)
                t_next = int(r["arrival_ns"][-1])
                while True:
                    try:
                        todo.put(r, timeout=0.005)
                        break
                    except queue.Full:
                        srv.poll(1 << 16)
                srv.poll(1 << 16)
            todo.put(None)
            while th.is_alive():
                srv.poll(1 << 16)
                th.join(timeout=0.005)
            if errs:
                raise errs[0]
            srv.drain(timeout_ms=120000)
            while len(srv.poll(1 << 16)):
                pass
            st = srv.stats(reset=True)
            span = (st["last_done_ns"] - st["first_arrival_ns"]) * 1e-9
            points.append({
                "load": load, "offered_fps": round(rate, 1), "frames": st["completed"],
                "mbps": round(st["bits_completed"] / span / 1e6, 2),
                "alu_frac": round(st["completed"] * mean_work / span / 1e12 / ALU_PEAK_TOPS, 4),
                "p50_ms": round(st["p50_ns"] * 1e-6, 3), "p99_ms": round(st["p99_ns"] * 1e-6, 3),
                "max_ms": round(st["max_ns"] * 1e-6, 3), "iterations": st["iterations"],
                "mean_items_per_iteration": round(st["items_launched"] / max(1, st["iterations"]), 1),
                "peak_frames_on_device": st["peak_frames_on_device"],
                "peak_arena_MiB": round(st["peak_arena_bytes"] / 2 ** 20, 2),
                # where the time goes (device events per iteration, host clocks per frame)
                "ingest_busy": round(st["iter_ingest_ns"] * 1e-9 / span, 3),
                "decode_busy": round(st["iter_decode_ns"] * 1e-9 / span, 3),
                "mean_ingest_ms": round(st["iter_ingest_ns"] * 1e-6 / max(1, st["iterations"]), 4),
                "mean_decode_ms": round(st["iter_decode_ns"] * 1e-6 / max(1, st["iterations"]), 4),
                "max_iteration_ms": round(st["iter_max_ns"] * 1e-6, 3),
                "engine_host_busy": round(st["engine_host_ns"] * 1e-9 / span, 3),
                "mean_admit_wait_ms": round(st["admit_wait_ns"] * 1e-6 / max(1, st["completed"]), 4),
                "max_admit_wait_ms": round(st["admit_wait_max_ns"] * 1e-6, 3),
                "mean_submit_lag_ms": round(st["submit_lag_ns"] * 1e-6 / max(1, st["submit_lag_count"]), 4),
                "max_submit_lag_ms": round(st["submit_lag_max_ns"] * 1e-6, 3)})
            print(f"serving: load {load:g} done ({st['completed']} frames, p99 {points[-1]['p99_ms']} ms)",
                  file=sys.stderr, flush=True)
    finally:
        srv.close()
    return {
        "workload": f"Poisson arrivals at 0.25-1.0 x measured capacity, {args.serve_seconds:g} s per load point; "
                    f"pool of {P} terminated frames, n lognormal (median 1024, sigma_ln 1) clipped to [40, 16384] "
                    f"(mean {mean_bits:.0f} bits), code uniform over {'/'.join(BATCH_CODES)}, Eb/N0 uniform in "
                    f"[1, 5] dB, int8 LLRs in pinned host memory; arrivals replayed by a native thread "
                    f"(vit_server_submit_paced); latency from arrival to completion seen by the host",
        "capacity_fps": round(cap, 1),
        "capacity_mbps": round(cap * mean_bits / 1e6, 2),
        "capacity_alu_frac": round(cap * mean_work / 1e12 / ALU_PEAK_TOPS, 4),
        "arena_MiB": args.serve_arena_mb,
        "max_items": args.serve_max_items,
        "tuning": {BATCH_CODES[i]: {"L": t[0], "v": t[1], "waves_per_block": t[3]} for i, t in enumerate(tunes)},
        "points": points,
    }


def ber_gaps(vit, torch, configs, log2n=24, time_at=None, grid=(2.5, 3.0, 3.5, 4.0, 4.5, 5.0)):
    """Eb/N0 gap at BER 1e-4 between decoder configurations and maximum-
    likelihood decoding, K=7 r1/2, FP32 LLRs, 2^log2n bits per Eb/N0 point.
    configs: label -> decode keyword arguments (L, v1, v2 and any options).
    The ML reference is the blocked decoder with v1 = v2 = 128, a traceback
    depth far beyond convergence (tests check it against full-frame ML; on the
    2^24-bit 3 dB headline stream the benchmark's CPU leg compares it with the
    oracle's full-frame decode).  time_at: also time every configuration at
    that Eb/N0 (information Mbps)."""
    import numpy as np
    import synth
    k, gens = synth.CODES["k7r12"]
    code = vit.make_code(k, gens)
    n = 1 << log2n
    grid = list(grid)
    errs = {}
    mbps = {}
    out = torch.empty((n + 7) // 8, dtype=torch.uint8, device="cuda")
    for e in grid:
        bits, llr = synth.make_stream("k7r12", n, e, seed=100 + int(e * 10))
        d = torch.from_numpy(llr).cuda()

        def nerr(L, v1, v2, **kw):
            vit.decode(code, d, n, L, v1 + v2, v1=v1, out=out, **kw)
            got = synth.unpack_bits(out.cpu().numpy(), n)
            return int(np.sum(got != bits))

        errs[("ml", e)] = nerr(512, 128, 128)
        for label, kw in configs.items():
            errs[(label, e)] = nerr(**kw)
            if time_at is not None and e == time_at:
                kk = dict(kw)
                L, v1, v2 = kk.pop("L"), kk.pop("v1"), kk.pop("v2")
                stream = torch.cuda.current_stream()
                for _ in range(2):
                    vit.decode(code, d, n, L, v1 + v2, v1=v1, out=out, stream=stream, **kk)
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                for _ in range(5):
                    vit.decode(code, d, n, L, v1 + v2, v1=v1, out=out, stream=stream, **kk)
                s1.record(stream)
                torch.cuda.synchronize()
                mbps[label] = round(n / (s0.elapsed_time(s1) / 5 * 1e-3) / 1e6, 1)
        print(f"[ber] Eb/N0 {e} dB done", file=sys.stderr, flush=True)

    def ebn0_at(label):
        bers = [max(errs[(label, e)], 0.5) / n for e in grid]
        for i in range(len(grid) - 1):
            if bers[i] >= 1e-4 > bers[i + 1]:
                y0, y1 = np.log(bers[i]), np.log(bers[i + 1])
                return grid[i] + (np.log(1e-4) - y0) * (grid[i + 1] - grid[i]) / (y1 - y0)
        return None

    ml_at = ebn0_at("ml")
    table = {}
    for label in configs:
        at = ebn0_at(label)
        table[label] = None if at is None or ml_at is None else round(float(at - ml_at), 4)
    return {
        "workload": f"K=7 r1/2, FP32 LLRs, 2^{log2n} bits per point, Eb/N0 {grid[0]}..{grid[-1]} dB; "
                    f"gap = Eb/N0 at BER 1e-4 minus that of the ML reference (blocked, v1 = v2 = 128)",
        "ml_ebn0_at_1e-4": None if ml_at is None else round(float(ml_at), 4),
        "ml_errors": {str(e): errs[("ml", e)] for e in grid},
        "gap_db": table,
        "mbps": mbps if time_at is not None else None,
    }


def precision_sweep(vit, torch, log2n=24):
    """The integer path's cost: the same 2^log2n-bit stream for K=7 r1/2, K=7
    r1/3 and K=9 r1/2 at Eb/N0 0..6 dB, decoded from FP32 LLRs and from int8
    LLRs (quantised on the GPU with the per-Eb/N0 scale: a noiseless symbol
    maps to 8), BER of each, the Eb/N0 each needs for BER 1e-4 (log-linear
    interpolation) and their difference, and both paths' stream throughput at
    3 dB.  Block shapes: L=512, v=35 for K=7; L=256, v=64 for K=9 (the library's
    default overlaps).  The ML reference is the blocked decoder with v1 = v2 =
    128."""
    import numpy as np
    import synth
    n = 1 << log2n
    grid = list(range(7))
    res = {}
    out = torch.empty((n + 7) // 8, dtype=torch.uint8, device="cuda")
    for name, (L, v) in (("k7r12", (512, 35)), ("k7r13", (512, 35)), ("k9r12", (256, default_overlap(9)))):
        k, gens = synth.CODES[name]
        code = vit.make_code(k, gens)
        rows = {"fp32": [], "int8": [], "ml": []}
        mbps = {}
        for e in grid:
            bits, llr = synth.make_stream(name, n, float(e), seed=1 + e)
            d = torch.from_numpy(llr).cuda()
            q = vit.quantize(d, 8.0 * synth.noise_sigma(float(e), len(gens)) ** 2 / 2.0)
            # the ML reference: FP32, blocks with v1 = v2 = 128 (far beyond convergence)
            vit.decode(code, d, n, 512, 256, v1=128, out=out)
            rows["ml"].append(int(np.sum(synth.unpack_bits(out.cpu().numpy(), n) != bits)))
            for tag, x in (("fp32", d), ("int8", q)):
                vit.decode(code, x, n, L, v, out=out)
                got = synth.unpack_bits(out.cpu().numpy(), n)
                rows[tag].append(int(np.sum(got != bits)))
                if e == 3:
                    ms, _ = time_decode(vit, torch, code, x, out, n, L, v, 10, 2)
                    mbps[tag] = round(n / (ms * 1e-3) / 1e6, 1)
            print(f"[precision] {name} {e} dB done", file=sys.stderr, flush=True)

        def at_1e4(errs):
            bers = [max(x, 0.5) / n for x in errs]
            for i in range(len(grid) - 1):
                if bers[i] >= 1e-4 > bers[i + 1]:
                    y0, y1 = np.log(bers[i]), np.log(bers[i + 1])
                    return grid[i] + (np.log(1e-4) - y0) * (grid[i + 1] - grid[i]) / (y1 - y0)
            return None

        af, aq, am = at_1e4(rows["fp32"]), at_1e4(rows["int8"]), at_1e4(rows["ml"])

        def ml_gap(errs):
            """Per grid point: the Eb/N0 shift at which the ML curve reaches this BER."""
            mb = [max(x, 0.5) / n for x in rows["ml"]]
            out_g = []
            for e, x in zip(grid, errs):
                b = max(x, 0.5) / n
                at = None
                for i in range(len(grid) - 1):
                    if mb[i] >= b > mb[i + 1]:
                        y0, y1 = np.log(mb[i]), np.log(mb[i + 1])
                        at = grid[i] + (np.log(b) - y0) * (grid[i + 1] - grid[i]) / (y1 - y0)
                out_g.append(None if at is None or x == 0 else round(float(e - at), 4))
            return out_g

        res[name] = {"L": L, "v": v, "ebn0_db": grid,
                     "ber_fp32": [x / n for x in rows["fp32"]], "ber_int8": [x / n for x in rows["int8"]],
                     "ber_ml": [x / n for x in rows["ml"]],
                     "ebn0_at_1e-4_fp32": None if af is None else round(float(af), 4),
                     "ebn0_at_1e-4_int8": None if aq is None else round(float(aq), 4),
                     "ebn0_at_1e-4_ml": None if am is None else round(float(am), 4),
                     "int8_loss_db": None if af is None or aq is None else round(float(aq - af), 4),
                     "int8_loss_vs_ml_db": None if am is None or aq is None else round(float(aq - am), 4),
                     "gap_to_ml_per_point_fp32": ml_gap(rows["fp32"]),
                     "gap_to_ml_per_point_int8": ml_gap(rows["int8"]),
                     "mbps_at_3db": mbps}
    return {"workload": f"2^{log2n}-bit terminated streams, BPSK/AWGN, seed 1 + Eb/N0; int8 scale 8 sigma^2 / 2",
            "codes": res}


def table2_configs():
    """The paper's Table II grid: f = L in {32..512}, v2 in {10..40}, v1 = v2."""
    return {f"v2={v2},f={f}": dict(L=f, v1=v2, v2=v2) for v2 in (10, 20, 30, 40) for f in (32, 64, 128, 256, 512)}


TABLE3_F = 304  # the paper's frame of about 300 bits, rounded up to a multiple of 8


def table3_configs():
    """The parallel traceback's grid (Sec. IV-D; the paper's BER-gap and
    throughput tables): frames of f = 304 bits with v1 = 20, subframes of f0
    in {8, ..., 56} bits with w in {25, ..., 45} stages of inner overlap and
    the same right overlap v2 = w, inner chains started from the stored best
    state or from a random state; and the one-trace decoder at each v2 = w."""
    c = {}
    for w in (25, 30, 35, 40, 45):
        c[f"one trace,v2={w}"] = dict(L=TABLE3_F, v1=20, v2=w)
        for f0 in (8, 16, 24, 32, 40, 48, 56):
            c[f"v2={w},f0={f0}"] = dict(L=TABLE3_F, v1=20, v2=w, subframe_bits=f0, subframe_overlap=w)
            c[f"v2={w},f0={f0},random"] = dict(L=TABLE3_F, v1=20, v2=w, subframe_bits=f0, subframe_overlap=w,
                                               subframe_start=1, subframe_seed=12345)
    return c


TABLE3_GRID = tuple(2.5 + 0.5 * i for i in range(12))  # 2.5 .. 8.0 dB: the random starts need the high end


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the decoder has no multi-GPU path "
              f"in this library.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2011_09337_amd as vit
    import synth

    if args.table2:
        print(json.dumps({"table2": ber_gaps(vit, torch, table2_configs())}), flush=True)
        return
    if args.table3:
        print(json.dumps({"table3": ber_gaps(vit, torch, table3_configs(), time_at=3.0, grid=TABLE3_GRID)}),
              flush=True)
        return
    if args.precision:
        print(json.dumps({"precision": precision_sweep(vit, torch)}), flush=True)
        return

    head_sub = None if args.subframes is None else tuple(int(x) for x in args.subframes.split(":"))
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
                               args.steps if L == args.L else max(3, args.steps // 4), args.warmup,
                               sub=head_sub)
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
    vit.decode(code, llr_d, n, args.L, v, out=out_d, **subframe_kw(head_sub))
    torch.cuda.synchronize()
    got = synth.unpack_bits(out_d.cpu().numpy(), n)
    ber = float(np.mean(got != bits))
    # a long-overlap proxy of maximum likelihood on the GPU: the blocked
    # decoder with v1 = v2 = 128 (the exact full-frame figure comes from the
    # CPU leg below)
    vs_long = None
    long_bits = None
    if not args.no_ml_check:
        vit.decode(code, llr_d, n, 512, 256, v1=128, out=out_d)
        torch.cuda.synchronize()
        long_bits = synth.unpack_bits(out_d.cpu().numpy(), n)
        vs_long = int(np.sum(long_bits != got))
    # side measurement: one trace per block vs the parallel traceback of
    # Sec. IV-D (subframes of f0 bits, w stages of inner overlap)
    subframe = None
    if not args.no_subframe_probe:
        subframe = {}
        for sub in (None, (24, 25), (56, 45), (32, 18), (64, 18), (128, 18), (24, 25, 1)):
            ms_w, _ = time_decode(vit, torch, code, llr_d, out_d, n, args.L, v, max(3, args.steps // 2),
                                  args.warmup, sub=sub)
            vit.decode(code, llr_d, n, args.L, v, out=out_d, **subframe_kw(sub))
            torch.cuda.synchronize()
            ber_w = float(np.mean(synth.unpack_bits(out_d.cpu().numpy(), n) != bits))
            tag = "one" if sub is None else f"f0={sub[0]},w={sub[1]}" + (",random" if len(sub) > 2 else "")
            subframe[tag] = {"mbps": round(n / (ms_w * 1e-3) / 1e6, 1), "ber": ber_w}

    llr_bytes = llr.nbytes
    hbm_alg_bytes = llr_bytes + (n + 7) // 8  # LLRs read once + packed output
    traffic = traffic_from_profiles(f"vit_blocked_k7r12_f32_L{args.L}")
    roofline = {
        "bound": "alu",
        "achieved": round(head["tops"], 3),
        "peak": ALU_PEAK_TOPS,
        "unit": "TFLOP/s",  # fp32 adds, compares and selects, one flop each
        "frac": round(head["tops"] / ALU_PEAK_TOPS, 4),
        "mix_peak": round(MIX_PEAK_TOPS, 2),
        "mix_frac": round(head["tops"] / MIX_PEAK_TOPS, 4),
        "traffic": traffic,
        "hbm_achieved_GBps": round(hbm_alg_bytes / (head["ms"] * 1e-3) / 1e9, 1),
        "hbm_frac": round(hbm_alg_bytes / (head["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
    }
    cpu = None
    vs_ml = None
    ml_ber = None
    long_vs_ml = None
    if not args.no_cpu:
        res = cpu_baseline(None, llr, n, args.L, v, ml=not args.no_ml_check)
        if "ml_bits" in res:
            vs_ml = int(np.sum(res["ml_bits"] != got))
            ml_ber = float(np.mean(res["ml_bits"] != bits))
            long_vs_ml = None if long_bits is None else int(np.sum(res["ml_bits"] != long_bits))
        mbps, nb, dt, th = res["all"]
        cpu = {"value": round(mbps, 3), "unit": "Mbps", "cores": th, "kind": "oracle",
               "sample": f"the whole {nb}-bit stream, blocked L={args.L} v={v}, best of 3 passes: {dt:.2f} s "
                         f"on {th} threads; single-core figure on the first 2^21 bits",
               "single_core_mbps": round(res["one"][0], 3)}
    batched = None if args.no_batched else bench_batched(vit, torch, args)
    if batched:
        batched["vs_stream_fp32"] = round(batched["mbps"] / head["mbps"], 3)
        batched["int16"]["vs_stream_fp32"] = round(batched["int16"]["mbps"] / head["mbps"], 3)
    serving = None
    if not args.no_serving:
        tunes = batched["tuning_tuples"] if batched else [(256, default_overlap(synth.CODES[c][0]), -1, 1)
                                                          for c in BATCH_CODES]
        serving = bench_serving(vit, torch, args, tunes)
    if batched:
        batched.pop("tuning_tuples", None)
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
                               f"v2={v - v // 2})" + ("" if head_sub is None else
                                                      f"; parallel traceback in subframes of {head_sub[0]} bits, "
                                                      f"inner overlap {head_sub[1]} stages"),
                   "n_bits": n, "L": args.L, "v": v, "ebn0_db": args.ebn0,
                   "subframes": None if head_sub is None else list(head_sub)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ber": ber,
        "bits_differing_from_ml": vs_ml,
        "ml_reference": None if vs_ml is None else
        {"decoder": "full-frame ML over the whole stream (CPU oracle, float64 metrics)", "ber": ml_ber,
         "long_overlap_bits_differing": long_vs_ml},
        "bits_differing_from_long_overlap": vs_long,
        "subframe_traceback": subframe,
        "batched": batched,
        "serving": serving,
        "sweep": {str(L): {"mbps": round(s["mbps"], 1), "ms": round(s["ms"], 4),
                           "alu_frac": round(s["tops"] / ALU_PEAK_TOPS, 4)} for L, s in sweep.items()},
        "wall_s_timed": round(head_wall, 4),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
