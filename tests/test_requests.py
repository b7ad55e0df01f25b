"""Generalized requests (Generalized Requests section, with the poll and wait
callbacks of its extension) and the completion calls they share with the
library's own requests.  The host-side semantics run on the CPU (a plain C
client and the Python binding); the GPU test mixes device requests with a
generalized request that wraps a caller's own stream work."""
import os
import subprocess
import tempfile
import threading
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2402_12274_amd", "libmdt.so")


def test_c_client_grequests():
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "grequest_check")
        subprocess.check_call(["gcc", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-Wall", "-Werror", "-I",
                               os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "native", "grequest_check.c"),
                               "-o", exe, LIB, "-lpthread", f"-Wl,-rpath,{os.path.dirname(LIB)}"])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "grequest ok" in r.stdout


def test_c_client_general_progress():
    # mdt_stream_progress / progress threads driving generalized requests
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "progress_check")
        subprocess.check_call(["gcc", "-std=c11", "-D_POSIX_C_SOURCE=200809L", "-Wall", "-Werror", "-I",
                               os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "native", "progress_check.c"),
                               "-o", exe, LIB, "-lpthread", f"-Wl,-rpath,{os.path.dirname(LIB)}"])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "progress ok" in r.stdout


def test_binding_progress_thread_completes_in_background():
    from paper_2402_12274_amd import mdt

    def poll(g):
        g.state["polls"] += 1
        if g.state["polls"] == 50:
            g.complete()

    g = mdt.GRequest(poll=poll, state={"polls": 0})
    assert not g.status()
    mdt.start_progress_thread()
    try:
        t0 = time.time()
        while not g.status() and time.time() - t0 < 30:
            time.sleep(0.001)
    finally:
        mdt.stop_progress_thread()
    assert g.status() and g.state["polls"] == 50
    assert g.test() is True  # completed by the thread: freed by this test


def test_binding_poll_and_query():
    from paper_2402_12274_amd import mdt

    log = []

    def poll(g):
        g.state["polls"] += 1
        if g.state["polls"] == 4:
            g.complete()

    g = mdt.GRequest(poll=poll, query=lambda g: log.append("query"), free=lambda g: log.append("free"),
                     state={"polls": 0})
    assert [g.test() for _ in range(3)] == [False, False, False]
    assert log == []
    assert g.test() is True
    assert log == ["query", "free"] and g.handle.value is None
    assert g.key not in mdt._GREQS


def test_binding_wait_groups_and_errors():
    from paper_2402_12274_amd import mdt

    calls = []

    def wait(gs, timeout):
        calls.append(([x.state for x in gs], timeout))
        for x in gs:
            x.complete()

    gs = [mdt.GRequest(wait=wait, state=i) for i in range(5)]
    other = mdt.GRequest(state="thread")
    th = threading.Timer(0.02, other.complete)
    th.start()
    mdt.waitall(gs[:2] + [None, other] + gs[2:])
    th.join()
    # one call for the group, bounded while the plain request was pending
    assert calls[0][0] == [0, 1, 2, 3, 4] and calls[0][1] > 0
    assert all(x.handle.value is None for x in gs + [other])

    bad = mdt.GRequest(poll=lambda g: 91)
    with pytest.raises(mdt.MdtError) as e:
        bad.wait()
    assert e.value.code == 91 and bad.handle.value is not None
    bad.complete()
    bad.wait()

    c = mdt.GRequest(cancel=lambda g, done: calls.append(("cancel", done)))
    c.cancel()
    c.complete()
    c.cancel()
    assert calls[-2:] == [("cancel", False), ("cancel", True)]
    with pytest.raises(mdt.MdtError) as e:
        c.complete()
    assert e.value.code == mdt.ERR_STATE
    c.wait()


@pytest.mark.gpu
def test_grequest_wraps_stream_work_beside_device_requests():
    """A generalized request polls a torch event recorded after the caller's
    own kernel; mdt_waitall completes it together with pack requests, and
    every result is the same as when each runs alone."""
    import torch

    from paper_2402_12274_amd import inputs, mdt
    from gpu_util import note

    note("grequest beside device requests")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ms = mdt.Stream(stream.cuda_stream)
    t = mdt.build_type(inputs.vector_small())
    src = torch.from_numpy(inputs.random_bytes(16384, seed=7)).to(dev)
    outs = [torch.empty(t.size(), dtype=torch.uint8, device=dev) for _ in range(3)]
    reqs = [mdt.mdt_pack_enqueue(src.data_ptr(), 1, t, 0, o.data_ptr(), -1, ms, want_request=True)[1] for o in outs]
    x = torch.arange(1 << 20, dtype=torch.float32, device=dev)
    y = x * 2 + 1
    ev = torch.cuda.Event()
    ev.record(stream)

    def poll(g):
        if ev.query():
            g.complete()

    g = mdt.GRequest(poll=poll)
    mdt.waitall(reqs[:2] + [g] + reqs[2:])
    assert ev.query()
    assert torch.equal(y, x * 2 + 1)
    ref = torch.empty_like(outs[0])
    mdt.mdt_pack(src.data_ptr(), 1, t, 0, ref.data_ptr(), -1)
    for o in outs:
        assert torch.equal(o, ref)


@pytest.mark.gpu
def test_stream_progress_thread_completes_gpu_requests():
    """A progress thread on a plain stream records the completion of packs
    enqueued there (no test or wait in between); a general progress thread
    completes a generalized request that polls a torch event recorded after
    work on another stream.  The packed bytes equal the oracle's."""
    import numpy as np
    import torch

    from gpu_util import note
    from oracle import build_type as obuild
    from paper_2402_12274_amd import inputs, mdt

    note("stream progress thread")
    dev = torch.device("cuda:0")
    side = torch.cuda.Stream()
    ms = mdt.Stream(side.cuda_stream)
    spec = inputs.halo_face(128, 2, 2, "hi")
    t = mdt.build_type(spec)
    host = inputs.random_bytes(128 ** 3 * 8, seed=13)
    src = torch.from_numpy(host).to(dev)
    torch.cuda.synchronize()
    outs = [torch.zeros(t.size(), dtype=torch.uint8, device=dev) for _ in range(4)]
    mdt.start_progress_thread(ms)
    try:
        reqs = [mdt.mdt_pack_enqueue(src.data_ptr(), 1, t, 0, o.data_ptr(), -1, ms, want_request=True)[1]
                for o in outs]
        t0 = time.time()
        while not all(r.status() for r in reqs) and time.time() - t0 < 30:
            time.sleep(0.0005)
        assert all(r.status() for r in reqs)
    finally:
        mdt.stop_progress_thread(ms)
    ref = obuild(spec).pack(host, 0, 1)
    for r, o in zip(reqs, outs):
        assert r.test() is True
        assert np.array_equal(o.cpu().numpy(), ref)

    note("general progress thread with a generalized request over a torch event")
    other = torch.cuda.Stream()
    out2 = torch.zeros(t.size(), dtype=torch.uint8, device=dev)
    ms2 = mdt.Stream(other.cuda_stream)
    mdt.mdt_pack_enqueue(src.data_ptr(), 1, t, 0, out2.data_ptr(), -1, ms2)
    ev = torch.cuda.Event()
    ev.record(other)

    def poll(g):
        if ev.query():
            g.complete()

    g = mdt.GRequest(poll=poll)
    mdt.start_progress_thread()
    try:
        t0 = time.time()
        while not g.status() and time.time() - t0 < 30:
            time.sleep(0.0005)
    finally:
        mdt.stop_progress_thread()
    assert g.status() and g.test() is True
    assert np.array_equal(out2.cpu().numpy(), ref)
