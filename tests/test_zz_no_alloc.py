"""The entry point that allocates nothing (mdt_batch_launch_noalloc),
through the C ABI: its output equals mdt_batch_launch's on the same batch
(bit for bit), on two calls in a row, the second with a smaller batch, in
every launch configuration; a batch that never ran through mdt_batch_launch
(its own device buffers never allocated) works; more than 1024 requests is
rejected."""
import numpy as np
import pytest

from gpu_util import note
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs

pytestmark = pytest.mark.gpu


def _requests(torch, mdt, seed, nface, vec_count, nrec, nh):
    """Mixed pack and unpack requests (chunk, record and run-table bodies)
    with their device buffers."""
    dev = torch.device("cuda:0")
    lens, disps = inputs.hindexed_blocks(nblocks=nh, span=1 << 22, seed=seed)
    specs = [(inputs.halo_face(nface, 1, 2, "lo"), 1), (inputs.halo_face(nface, 4, 0, "hi"), 1),
             (("vector", vec_count, 1, 5, inputs.DOUBLE), 1), (inputs.particle_struct(), nrec),
             (inputs.hindexed_type(lens, disps), 1)]
    out = []
    for k, (spec, count) in enumerate(specs):
        t = mdt.build_type(spec)
        a = obuild(spec).attrs()
        nb = (count - 1) * a["extent"] + a["true_ub"] + 64
        src = torch.from_numpy(inputs.random_bytes(nb, seed=seed + k)).to(dev)
        n = t.size() * count
        pk = torch.from_numpy(inputs.random_bytes(n, seed=seed + 50 + k)).to(dev)
        out.append((t, count, src, pk, n, nb))
    return out


def _batch(torch, mdt, reqs, cfg):
    b = mdt.Batch()
    bufs = []
    for t, count, src, pk, n, nb in reqs:
        o = torch.zeros(n + 16, dtype=torch.uint8, device="cuda")
        d = torch.full((nb,), 0x5A, dtype=torch.uint8, device="cuda")
        b.add_pack(src.data_ptr(), count, t, 0, o.data_ptr() + 3, -1)
        b.add_unpack(pk.data_ptr(), n, d.data_ptr(), count, t, 0)
        bufs.append((o, d))
    b.set_config(cfg)
    return b, bufs


def _reset(bufs):
    for o, d in bufs:
        o.zero_()
        d.fill_(0x5A)


def test_noalloc_matches_batch_launch():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    big = _requests(torch, mdt, 11, 80, 30000, 20001, 20000)
    small = _requests(torch, mdt, 23, 40, 3001, 999, 3000)[:3]
    for cfg in [mdt.BatchConfig(1024, 0, 2, 0, 0), mdt.BatchConfig(256, 4, 0, 0, 0), mdt.BatchConfig(4096, 2, 1, 0, 0),
                mdt.BatchConfig(1024, 0, 3, 0, 0), mdt.BatchConfig(1024, 0, 0, 1, 1)]:
        note(f"noalloc batch config {mdt.config_dict(cfg)}")
        results = []
        for reqs in (big, small):  # two calls in a row, the second smaller
            b_ref, ref_bufs = _batch(torch, mdt, reqs, cfg)
            b_ref.launch(ms)
            torch.cuda.synchronize()
            expect = [(o.cpu().numpy(), d.cpu().numpy()) for o, d in ref_bufs]
            b, bufs = _batch(torch, mdt, reqs, cfg)  # never launched through mdt_batch_launch
            _reset(bufs)
            b.launch_noalloc(ms)
            torch.cuda.synchronize()
            results.append((bufs, expect))
        for bufs, expect in results:
            for (o, d), (eo, ed) in zip(bufs, expect):
                assert np.array_equal(o.cpu().numpy(), eo)
                assert np.array_equal(d.cpu().numpy(), ed)
    # the second call reran the small batch after the big one: its outputs
    # above were checked; a relaunch of the big batch still matches
    b, bufs = _batch(torch, mdt, big, mdt.BatchConfig(1024, 0, 2, 0, 0))
    for rep in range(2):
        _reset(bufs)
        b.launch_noalloc(ms)
        torch.cuda.synchronize()
    b_ref, ref_bufs = _batch(torch, mdt, big, mdt.BatchConfig(1024, 0, 2, 0, 0))
    b_ref.launch(ms)
    torch.cuda.synchronize()
    for (o, d), (ro, rd) in zip(bufs, ref_bufs):
        assert torch.equal(o, ro) and torch.equal(d, rd)


def test_noalloc_rejects_too_many_requests():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    t = mdt.build_type(("vector", 16, 1, 2, inputs.DOUBLE))
    src = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    out = torch.zeros(1025 * 128, dtype=torch.uint8, device="cuda")
    b = mdt.Batch()
    for i in range(1025):
        b.add_pack(src.data_ptr(), 1, t, 0, out.data_ptr() + 128 * i, -1)
    with pytest.raises(mdt.MdtError) as e:
        b.launch_noalloc(ms)
    assert e.value.code == mdt.ERR_NO_MEM
