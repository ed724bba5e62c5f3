"""The serving loop on the GPU: frames submitted in waves while earlier ones
are on the device come back identical to the same frames decoded alone on
the GPU and by the CPU oracle; late short frames overtake a long one; queue
limits and request validation."""
import time

import numpy as np
import pytest

import synth
from oracle import vref

pytestmark = pytest.mark.gpu

CODES = [(7, (0o171, 0o133)), (7, (0o133, 0o171, 0o165)), (9, (0o561, 0o753))]
TUNE = [(64, 35, -1, 1), (128, 35, 10, 2), (64, 45, -1, 1)]


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_09337_amd as vit
    return torch, vit


def make_frames(rng, count, nmin, nmax, int8, code=None):
    """(code_id, terminated, n, llr ndarray) for random (or the given) codes
    and random lengths."""
    out = []
    for _ in range(count):
        cid = int(rng.integers(0, len(CODES))) if code is None else code
        k, gens = CODES[cid]
        n = int(rng.integers(nmin, nmax + 1))
        term = int(rng.random() < 0.8)
        e = float(rng.uniform(1.0, 5.0))
        llr = synth.awgn_llr(synth.encode(k, gens, synth.info_bits(n, rng), bool(term)), e, len(gens), rng)
        if int8:
            llr = vref.quantize_i8(llr, 8.0 * synth.noise_sigma(e, len(gens)) ** 2 / 2.0)
        out.append((cid, term, n, llr))
    return out


def place(torch, frames, rng):
    """Lay the frames' LLRs and output areas into one pinned host region (some
    LLR offsets deliberately not 16-byte aligned).  Returns (host tensor,
    [(llr_off, out_off)])."""
    offs, pos = [], 0
    for (_, _, n, llr) in frames:
        pos += int(rng.integers(0, 3)) * 5
        lo = pos
        pos += llr.nbytes
        oo = pos + 1
        pos = oo + (n + 7) // 8
        offs.append((lo, oo))
    host = torch.zeros(pos + 64, dtype=torch.uint8).pin_memory()
    h = host.numpy()
    for (_, _, _, llr), (lo, _) in zip(frames, offs):
        h[lo:lo + llr.nbytes] = llr.view(np.uint8)
    return host, offs


def requests(vit, host, frames, offs, tags):
    r = np.zeros(len(tags), dtype=vit.REQUEST_DTYPE)
    base = host.data_ptr()
    for j, t in enumerate(tags):
        cid, term, n, _ = frames[t]
        lo, oo = offs[t]
        r[j] = (cid, term, n, base + lo, base + oo, t, 0)
    return r


def expected_alone(torch, vit, frame, tune):
    cid, term, n, llr = frame
    k, gens = CODES[cid]
    L, v, v1, _ = tune[cid]
    out = vit.decode(vit.make_code(k, gens), torch.from_numpy(llr).cuda(), n, L, v, v1=None if v1 < 0 else v1,
                     terminated=bool(term))
    return out.cpu().numpy()


def expected_oracle(frame, tune):
    cid, term, n, llr = frame
    k, gens = CODES[cid]
    L, v, v1, _ = tune[cid]
    v1 = v // 2 if v1 < 0 else v1
    return synth.pack_bits(vref.decode_blocked(vref.make_code(k, list(gens)), llr, n, L, v1, v - v1, bool(term)))


@pytest.mark.parametrize("int8,metric_bits", [(True, 0), (True, 16), (False, 0)])
def test_mix_equals_alone_and_oracle(dev, int8, metric_bits):
    torch, vit = dev
    rng = np.random.default_rng(11 if int8 else 12)
    frames = make_frames(rng, 120, 20, 2500, int8)
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    # a small arena and few slots and items, so that admission waits for
    # memory and long frames span several iterations
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8 if int8 else vit.VIT_LLR_F32,
                     arena_bytes=96 << 10, max_frames=10, max_items=48, metric_bits=metric_bits)
    before = host.numpy().copy()
    try:
        order = rng.permutation(len(frames))
        for wave in np.array_split(order, 8):
            st, acc = srv.submit(requests(vit, host, frames, offs, [int(t) for t in wave]))
            assert st == vit.VIT_OK and acc == len(wave)
            time.sleep(0.002)
        srv.drain(timeout_ms=60000)
        comps = srv.poll()
        stats = srv.stats()
    finally:
        srv.close()
    assert sorted(comps["tag"].tolist()) == list(range(len(frames)))
    assert (comps["status"] == 0).all()
    assert (comps["done_ns"] >= comps["arrival_ns"]).all()
    assert stats["completed"] == len(frames) and stats["failed"] == 0
    assert stats["bits_completed"] == sum(f[2] for f in frames)
    assert stats["iterations"] > 1
    assert 1 <= stats["peak_frames_on_device"] <= 10
    assert stats["peak_arena_bytes"] <= 96 << 10
    assert 0 < stats["p50_ns"] <= stats["p99_ns"] <= stats["max_ns"]
    h = host.numpy()
    # the decode writes into the host region only the requests' output bytes
    outside = np.ones(h.size, dtype=bool)
    for t, fr in enumerate(frames):
        outside[offs[t][1]:offs[t][1] + (fr[2] + 7) // 8] = False
    np.testing.assert_array_equal(h[outside], before[outside], err_msg="bytes outside the outputs changed")
    for t, fr in enumerate(frames):
        lo, oo = offs[t]
        got = h[oo:oo + (fr[2] + 7) // 8]
        alone = expected_alone(torch, vit, fr, TUNE)
        np.testing.assert_array_equal(got, alone, err_msg=f"frame {t} differs from its decode alone")
        if t % 3 == 0:  # the oracle on a third of the frames keeps the test short
            np.testing.assert_array_equal(got, expected_oracle(fr, TUNE), err_msg=f"frame {t} vs oracle")


def test_mix_hard_decisions(dev):
    # hard-decision requests (one byte per coded bit) through the serving loop:
    # each frame equals its decode alone and the oracle's on +1 / -1 LLRs
    torch, vit = dev
    rng = np.random.default_rng(13)
    soft = make_frames(rng, 60, 20, 2000, False)
    frames = [(cid, term, n, synth.hard_bits(llr)) for cid, term, n, llr in soft]
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_HARD, arena_bytes=96 << 10, max_frames=10,
                     max_items=48)
    try:
        st, acc = srv.submit(requests(vit, host, frames, offs, list(range(len(frames)))))
        assert st == vit.VIT_OK and acc == len(frames)
        srv.drain(timeout_ms=60000)
        comps = srv.poll()
    finally:
        srv.close()
    assert sorted(comps["tag"].tolist()) == list(range(len(frames)))
    assert (comps["status"] == 0).all()
    h = host.numpy()
    for t, (cid, term, n, hard) in enumerate(frames):
        oo = offs[t][1]
        got = h[oo:oo + (n + 7) // 8]
        np.testing.assert_array_equal(got, expected_alone(torch, vit, frames[t], TUNE), err_msg=f"frame {t} alone")
        pm1 = np.where(hard != 0, -1, 1).astype(np.int8)
        np.testing.assert_array_equal(got, expected_oracle((cid, term, n, pm1), TUNE), err_msg=f"frame {t} oracle")


def test_requests_beyond_4gib_in_the_host_region(dev):
    # requests whose LLRs and outputs sit beyond 2^31 and 2^32 bytes into a
    # 4.3 GB pinned host region (ranges straddling both): the ingest copies'
    # and the direct output writes' 64-bit addresses
    torch, vit = dev
    rng = np.random.default_rng(17)
    frames = make_frames(rng, 5, 500, 4000, True)
    offs_llr = [0, (1 << 31) - 5001, (1 << 31) + 40013, (1 << 32) - 7001, (1 << 32) + 20011]
    offs = []
    for (_, _, n, llr), lo in zip(frames, offs_llr):
        offs.append((lo, lo + llr.nbytes + 3))  # the output right after the LLRs
    size = max(oo + (f[2] + 7) // 8 for f, (_, oo) in zip(frames, offs)) + 64
    print(f"[gpu] host region of {size} bytes", flush=True)
    host = torch.empty(size, dtype=torch.uint8, pin_memory=True)
    h = host.numpy()
    for (_, _, n, llr), (lo, oo) in zip(frames, offs):
        h[lo:lo + llr.nbytes] = llr.view(np.uint8)
        h[oo:oo + (n + 7) // 8] = 0xAB
    codes = [vit.make_code(k, g) for k, g in CODES]
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=8,
                     max_items=256)
    try:
        st, acc = srv.submit(requests(vit, host, frames, offs, list(range(len(frames)))))
        assert st == vit.VIT_OK and acc == len(frames)
        srv.drain(timeout_ms=30000)
        comps = srv.poll()
    finally:
        srv.close()
    assert sorted(comps["tag"].tolist()) == list(range(len(frames))) and (comps["status"] == 0).all()
    for t, fr in enumerate(frames):
        oo = offs[t][1]
        got = h[oo:oo + (fr[2] + 7) // 8]
        np.testing.assert_array_equal(got, expected_oracle(fr, TUNE), err_msg=f"request at host offset {offs[t]}")
    del host


# codes beside the benchmark's three: K=3, a K=5 code without the newest-input
# tap, K=8 (two registers of states per lane) and K=4 at rate 1/4
EDGE_CODES = [(3, (0o7, 0o5)), (5, (0o22, 0o35)), (8, (0o247, 0o371)), (4, (0o13, 0o15, 0o17, 0o11))]
EDGE_TUNE = [(16, 15, -1, 1), (16, 0, -1, 1), (32, 40, 0, 2), (16, 7, 7, 1)]


@pytest.mark.parametrize("int8", [False, True])
def test_edge_lengths_and_other_codes(dev, int8):
    # every frame length at its code's own edges (1, 2, k-1, k, k+1) and at
    # the block edges (L-1, L, L+1, 2L+1), terminated and open, through the
    # scheduler with a small arena and few slots and items (so frames wait
    # for memory and span iterations); each result equals the oracle's
    torch, vit = dev
    rng = np.random.default_rng(31 + int(int8))
    frames = []
    for cid, (k, gens) in enumerate(EDGE_CODES):
        L = EDGE_TUNE[cid][0]
        for n in sorted({1, 2, k - 1, k, k + 1, L - 1, L, L + 1, 2 * L + 1}):
            for term in (1, 0):
                e = float(rng.uniform(0.5, 4.0))
                llr = synth.awgn_llr(synth.encode(k, gens, synth.info_bits(n, rng), bool(term)), e, len(gens), rng)
                if int8:
                    llr = vref.quantize_i8(llr, 8.0 * synth.noise_sigma(e, len(gens)) ** 2 / 2.0)
                frames.append((cid, term, n, llr))
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in EDGE_CODES]
    srv = vit.Server(codes, host, tune=EDGE_TUNE, llr_type=vit.VIT_LLR_I8 if int8 else vit.VIT_LLR_F32,
                     arena_bytes=16 << 10, max_frames=6, max_items=20)
    before = host.numpy().copy()
    try:
        order = rng.permutation(len(frames))
        for wave in np.array_split(order, 4):
            st, acc = srv.submit(requests(vit, host, frames, offs, [int(t) for t in wave]))
            assert st == vit.VIT_OK and acc == len(wave)
        srv.drain(timeout_ms=60000)
        comps = srv.poll()
        stats = srv.stats()
    finally:
        srv.close()
    assert sorted(comps["tag"].tolist()) == list(range(len(frames)))
    assert (comps["status"] == 0).all()
    assert stats["completed"] == len(frames) and stats["iterations"] > 1
    h = host.numpy()
    outside = np.ones(h.size, dtype=bool)
    for t, fr in enumerate(frames):
        outside[offs[t][1]:offs[t][1] + (fr[2] + 7) // 8] = False
    np.testing.assert_array_equal(h[outside], before[outside], err_msg="bytes outside the outputs changed")
    for t, (cid, term, n, llr) in enumerate(frames):
        k, gens = EDGE_CODES[cid]
        L, v, v1, _ = EDGE_TUNE[cid]
        v1 = v // 2 if v1 < 0 else v1
        want = synth.pack_bits(vref.decode_blocked(vref.make_code(k, list(gens)), llr, n, L, v1, v - v1, bool(term)))
        oo = offs[t][1]
        np.testing.assert_array_equal(h[oo:oo + want.size], want, err_msg=f"code {cid} n={n} term={term}")


def test_late_short_frames_overtake_a_long_one(dev):
    torch, vit = dev
    rng = np.random.default_rng(5)
    long = make_frames(rng, 1, 16000, 16000, True, code=2)  # 250 blocks of 64 bits
    short = make_frames(rng, 12, 40, 200, True)
    frames = long + short
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=64,
                     max_items=16)
    try:
        assert srv.submit(requests(vit, host, frames, offs, [0])) == (vit.VIT_OK, 1)
        assert srv.submit(requests(vit, host, frames, offs, list(range(1, len(frames))))) == (vit.VIT_OK,
                                                                                             len(frames) - 1)
        srv.drain(timeout_ms=60000)
        comps = srv.poll()
    finally:
        srv.close()
    done = {int(c["tag"]): int(c["done_ns"]) for c in comps}
    assert len(done) == len(frames)
    # the long frame needs 16 iterations; each short one (at most 4 blocks)
    # gets a block in every iteration from the third at the latest
    assert max(done[t] for t in range(1, len(frames))) < done[0]
    h = host.numpy()
    for t, fr in enumerate(frames):
        lo, oo = offs[t]
        np.testing.assert_array_equal(h[oo:oo + (fr[2] + 7) // 8], expected_alone(torch, vit, fr, TUNE))


def test_queue_limit_and_bad_requests(dev):
    torch, vit = dev
    rng = np.random.default_rng(6)
    frames = make_frames(rng, 20, 40, 300, True)
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=64,
                     max_items=1024, max_pending=5)
    try:
        st, acc = srv.submit(requests(vit, host, frames, offs, list(range(20))))
        assert st == vit.VIT_EBUSY and acc == 5
        srv.drain(timeout_ms=30000)
        bad = requests(vit, host, frames, offs, [5])
        bad["llr"] = host.data_ptr() + host.numel() - 3  # runs past the host region
        with pytest.raises(vit.VitError) as ei:
            srv.submit(bad)
        assert ei.value.status == vit.VIT_EINVAL
        bad = requests(vit, host, frames, offs, [5])
        bad["code_id"] = 3
        with pytest.raises(vit.VitError):
            srv.submit(bad)
        st, acc = srv.submit(requests(vit, host, frames, offs, list(range(5, 10))))
        assert st == vit.VIT_OK and acc == 5
        srv.drain(timeout_ms=30000)
        comps = srv.poll()
        assert sorted(comps["tag"].tolist()) == list(range(10))
        s = srv.stats(reset=True)
        assert s["completed"] == 10 and srv.stats()["completed"] == 0
    finally:
        srv.close()
    h = host.numpy()
    for t in range(10):
        lo, oo = offs[t]
        np.testing.assert_array_equal(h[oo:oo + (frames[t][2] + 7) // 8], expected_alone(torch, vit, frames[t], TUNE))


def test_paced_submission_replays_arrival_times(dev):
    torch, vit = dev
    rng = np.random.default_rng(8)
    frames = make_frames(rng, 40, 40, 800, True)
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=64,
                     max_items=256)
    try:
        reqs = requests(vit, host, frames, offs, list(range(len(frames))))
        t0 = time.monotonic_ns() + 5_000_000
        reqs["arrival_ns"] = t0 + np.sort(rng.integers(0, 30_000_000, size=len(frames)))
        c0 = time.monotonic_ns()
        assert srv.submit_paced(reqs) == len(frames)
        c1 = time.monotonic_ns()
        srv.drain(timeout_ms=30000)
        comps = srv.poll()
    finally:
        srv.close()
    # the call returns no earlier than the last arrival
    assert c1 >= int(reqs["arrival_ns"][-1]) and c0 < t0
    by_tag = {int(c["tag"]): c for c in comps}
    assert sorted(by_tag) == list(range(len(frames)))
    for t in range(len(frames)):
        assert int(by_tag[t]["arrival_ns"]) == int(reqs["arrival_ns"][t])
        assert int(by_tag[t]["done_ns"]) > int(reqs["arrival_ns"][t])
    h = host.numpy()
    for t, fr in enumerate(frames):
        lo, oo = offs[t]
        np.testing.assert_array_equal(h[oo:oo + (fr[2] + 7) // 8], expected_alone(torch, vit, fr, TUNE))


def test_forced_allocation_failures(dev):
    # host allocation failures forced with vit_debug_fail_allocations: server
    # creation and a statistics snapshot return VIT_ENOMEM (no exception
    # leaves the C ABI), and a server created afterwards decodes as usual
    torch, vit = dev
    rng = np.random.default_rng(13)
    frames = make_frames(rng, 20, 40, 600, True)
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    lib = vit._lib.lib
    kw = dict(tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=64, max_items=256)
    try:
        assert lib.vit_debug_fail_allocations(1) == vit.VIT_OK
        with pytest.raises(vit.VitError) as ei:
            vit.Server(codes, host, **kw)
        assert ei.value.status == vit.VIT_ENOMEM
        srv = vit.Server(codes, host, **kw)
        try:
            st, acc = srv.submit(requests(vit, host, frames, offs, list(range(len(frames)))))
            assert st == vit.VIT_OK and acc == len(frames)
            srv.drain(timeout_ms=30000)
            comps = srv.poll()
            assert lib.vit_debug_fail_allocations(1) == vit.VIT_OK
            with pytest.raises(vit.VitError) as ei:
                srv.stats()
            assert ei.value.status == vit.VIT_ENOMEM
            stats = srv.stats()
        finally:
            srv.close()
    finally:
        assert lib.vit_debug_fail_allocations(0) == vit.VIT_OK
    assert sorted(comps["tag"].tolist()) == list(range(len(frames))) and (comps["status"] == 0).all()
    assert stats["completed"] == len(frames)
    h = host.numpy()
    for t, fr in enumerate(frames):
        lo, oo = offs[t]
        np.testing.assert_array_equal(h[oo:oo + (fr[2] + 7) // 8], expected_alone(torch, vit, fr, TUNE))


def test_engine_allocation_failure_fails_the_server(dev):
    # a host allocation failure inside the engine's scheduling step (after
    # admission): the server fails with VIT_ENOMEM, every frame is reported
    # exactly once, and drain returns the failure instead of waiting forever
    torch, vit = dev
    rng = np.random.default_rng(17)
    frames = make_frames(rng, 30, 40, 600, True)
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    lib = vit._lib.lib
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=64,
                     max_items=256)
    try:
        assert lib.vit_debug_fail_allocations(1) == vit.VIT_OK
        st, acc = srv.submit(requests(vit, host, frames, offs, list(range(len(frames)))))
        assert st == vit.VIT_OK and acc == len(frames)
        with pytest.raises(vit.VitError) as ei:
            srv.drain(timeout_ms=30000)
        assert ei.value.status == vit.VIT_ENOMEM
        comps = srv.poll()
    finally:
        assert lib.vit_debug_fail_allocations(0) == vit.VIT_OK
        srv.close()
    assert sorted(comps["tag"].tolist()) == list(range(len(frames)))
    assert (comps["status"] == vit.VIT_ENOMEM).all()


def test_queue_timeout(dev):
    # requests still queued max_wait_ms after their arrival complete with
    # VIT_ETIMEDOUT and are not decoded (their output bytes stay as they
    # were); the requests behind them decode as usual
    torch, vit = dev
    rng = np.random.default_rng(14)
    frames = make_frames(rng, 30, 40, 600, True)
    host, offs = place(torch, frames, rng)
    codes = [vit.make_code(k, g) for k, g in CODES]
    srv = vit.Server(codes, host, tune=TUNE, llr_type=vit.VIT_LLR_I8, arena_bytes=1 << 20, max_frames=64,
                     max_items=256, max_wait_ms=1000)
    try:
        reqs = requests(vit, host, frames, offs, list(range(len(frames))))
        reqs["arrival_ns"][:10] = time.monotonic_ns() - 5_000_000_000  # at the front, already 5 s old
        before = host.numpy().copy()
        st, acc = srv.submit(reqs)
        assert st == vit.VIT_OK and acc == len(frames)
        srv.drain(timeout_ms=30000)
        comps = srv.poll()
        stats = srv.stats()
    finally:
        srv.close()
    by_tag = {int(c["tag"]): int(c["status"]) for c in comps}
    assert sorted(by_tag) == list(range(len(frames)))
    assert all(by_tag[t] == vit.VIT_ETIMEDOUT for t in range(10))
    assert all(by_tag[t] == vit.VIT_OK for t in range(10, len(frames)))
    assert stats["completed"] == len(frames) - 10 and stats["failed"] == 10
    h = host.numpy()
    for t, fr in enumerate(frames):
        lo, oo = offs[t]
        nb = (fr[2] + 7) // 8
        if t < 10:
            np.testing.assert_array_equal(h[oo:oo + nb], before[oo:oo + nb])
        else:
            np.testing.assert_array_equal(h[oo:oo + nb], expected_alone(torch, vit, fr, TUNE))
