"""The serving loop on the host, without a GPU: the scheduler against a fake
device (tests/server_core_check.cpp, built here with g++ and the sanitizers)
and the server ABI's argument validation, which happens before any device
call."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_09337_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("scc") / "server_core_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, os.path.join(ROOT, "tests", "server_core_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    return exe


@pytest.mark.parametrize("seed", range(1, 13))
def test_scheduler_against_fake_device(checker, seed):
    r = subprocess.run([checker, str(seed)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")


@pytest.fixture(scope="module")
def vit():
    import paper_2011_09337_amd as v
    return v


def _cfg(vit, **kw):
    c = vit.vit_server_config()
    c.size = vit.C_sizeof(vit.vit_server_config)
    c.llr_type = vit.VIT_LLR_I8
    c.max_frames = 16
    c.max_items = 100
    c.max_pending = 10
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def test_workspace_size(vit):
    # two iteration slots of: 256-byte header, 40-byte items (the copy ranges
    # stay in pinned host memory)
    b = vit.vit_server_workspace_size(_cfg(vit))
    one = 256 + 100 * 40
    assert b == 2 * ((one + 255) // 256 * 256)


@pytest.mark.parametrize("kw", [dict(size=12), dict(llr_type=5), dict(max_frames=0), dict(max_items=0),
                                dict(max_pending=0), dict(max_frames=1 << 21), dict(max_wait_ms=-1)])
def test_bad_config(vit, kw):
    with pytest.raises(vit.VitError) as ei:
        vit.vit_server_workspace_size(_cfg(vit, **kw))
    assert ei.value.status == vit.VIT_EINVAL


def test_create_validates_before_the_device(vit):
    K7 = vit.make_code(7, (0o171, 0o133))
    codes = vit.codes_array([K7])
    ws = vit.vit_server_workspace_size(_cfg(vit))

    def create(tune=None, codes=codes, **kw):
        base = dict(arena=0x100000, arena_bytes=1 << 20, workspace=0x200000, workspace_bytes=ws, host=0x300000,
                    host_bytes=1 << 20)
        base.update(kw)
        return vit.vit_server_create(codes, vit.tunings_array(tune) if tune else None, _cfg(vit, **base))

    cases = [dict(arena=None), dict(workspace=None), dict(host=None), dict(arena=0x100010),
             dict(workspace_bytes=ws - 1), dict(arena_bytes=100), dict(tune=[(12, 35, -1, 1)]),
             dict(tune=[(64, -1, -1, 1)]), dict(tune=[(64, 35, 36, 1)]), dict(tune=[(64, 35, -1, 5)]),
             dict(codes=vit.codes_array([vit.make_code(7, (0, 0o133))]))]
    for kw in cases:
        with pytest.raises(vit.VitError) as ei:
            create(**kw)
        assert ei.value.status == vit.VIT_EINVAL, kw
    # int8 metrics exact in fp32: a block of 2^16 stages is refused
    with pytest.raises(vit.VitError) as ei:
        create(tune=[(1 << 16, 35, -1, 1)])
    assert ei.value.status == vit.VIT_EUNSUPPORTED


def test_request_layouts(vit):
    import ctypes
    assert vit.REQUEST_DTYPE.itemsize == ctypes.sizeof(vit._lib.vit_request) == 48
    assert vit.COMPLETION_DTYPE.itemsize == ctypes.sizeof(vit._lib.vit_completion) == 32
    for name, _ in vit._lib.vit_request._fields_:
        assert vit.REQUEST_DTYPE.fields[name][1] == getattr(vit._lib.vit_request, name).offset
    for name, _ in vit._lib.vit_completion._fields_:
        assert vit.COMPLETION_DTYPE.fields[name][1] == getattr(vit._lib.vit_completion, name).offset


def test_launch_rules(tmp_path):
    # default overlaps and the batch kernel's grid rule (vit_shapes.h), built
    # with g++ and the sanitizers
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "shapes_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", CSRC, os.path.join(ROOT, "tests", "shapes_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
