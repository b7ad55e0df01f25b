"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (one kernel launch per request, default tiling).

- 3-D halo faces: 512^3 float64 (1 GiB), 6 faces x ghost widths 1 and 4,
  packed and compared byte for byte with the oracle, then unpacked into a
  zeroed copy that must equal the oracle's unpack (faces set, rest zero);
- hindexed: 1,000,000 blocks (geometric lengths, mean 24 B) at seeded random
  non-overlapping displacements in a 2 GiB buffer, full pack, 1 MiB partial
  packs and unpack;
- particle records: struct {int32, float64[3], char[5]} x 4,000,000, full
  pack, 1 MiB partial packs (126 chunks, the last 928,000 B) and unpack.
"""
import numpy as np
import pytest

from gpu_util import first_diff, note, to_dev, to_host, zeros_dev
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs

pytestmark = pytest.mark.gpu

MiB = 1 << 20


@pytest.fixture(scope="module")
def mdt():
    from gpu_util import torch_cuda

    torch_cuda()
    from paper_2402_12274_amd import mdt as m

    return m


def _dev_equal(dev_tensor, host_expected: np.ndarray) -> bool:
    import torch

    exp = torch.from_numpy(host_expected).to("cuda")
    ok = bool(torch.equal(dev_tensor[: host_expected.size], exp))
    del exp
    return ok


def test_halo_faces_full(mdt):
    n = 512
    host = inputs.random_bytes(n ** 3 * 8, seed=inputs.DEFAULT_SEED)
    src = to_dev(host)
    dst = zeros_dev(n ** 3 * 8, 0)
    expect = np.zeros(n ** 3 * 8, np.uint8)
    total = 0
    for label, spec in inputs.halo_faces(n):
        note(f"full halo face {label}")
        t = mdt.build_type(spec)
        o = obuild(spec)
        ref = o.pack(host, 0, 1)
        out = zeros_dev(ref.size, 0)
        assert mdt.mdt_pack(src.data_ptr(), 1, t, 0, out.data_ptr(), -1) == ref.size
        got = to_host(out)[: ref.size]
        assert first_diff(got, ref) is None, (label, first_diff(got, ref))
        assert mdt.mdt_unpack(out.data_ptr(), ref.size, dst.data_ptr(), 1, t, 0) == ref.size
        o.unpack(ref, expect, 0, 1)
        total += ref.size
    assert total == 6 * (510 ** 2 * 8 + 504 ** 2 * 32)
    assert _dev_equal(dst, expect)


def test_hindexed_full(mdt):
    span = 1 << 31
    lens, disps = inputs.hindexed_blocks(nblocks=1_000_000, span=span, seed=inputs.DEFAULT_SEED)
    spec = inputs.hindexed_type(lens, disps)
    note("full hindexed: build")
    t = mdt.build_type(spec)
    o = obuild(spec)
    host = inputs.random_bytes(span, seed=inputs.DEFAULT_SEED + 1)
    ref = o.pack(host, 0, 1)
    assert ref.size == int(lens.sum())
    src = to_dev(host)
    out = zeros_dev(ref.size, 0)
    note("full hindexed: pack")
    assert mdt.mdt_pack(src.data_ptr(), 1, t, 0, out.data_ptr(), -1) == ref.size
    assert first_diff(to_host(out)[: ref.size], ref) is None
    note("full hindexed: 1 MiB partial packs")
    part = zeros_dev(MiB, 0)
    nchunks = 0
    for off in range(0, ref.size, MiB):
        k = mdt.mdt_pack(src.data_ptr(), 1, t, off, part.data_ptr(), MiB)
        assert k == min(MiB, ref.size - off)
        assert first_diff(to_host(part)[:k], ref[off:off + k]) is None, off
        nchunks += 1
    assert nchunks == (ref.size + MiB - 1) // MiB
    note("full hindexed: unpack")
    del src
    dst = zeros_dev(span, 0)
    assert mdt.mdt_unpack(out.data_ptr(), ref.size, dst.data_ptr(), 1, t, 0) == ref.size
    expect = np.zeros(span, np.uint8)
    o.unpack(ref, expect, 0, 1)
    assert _dev_equal(dst, expect)


def test_particle_records_full(mdt):
    count = 4_000_000
    spec = inputs.particle_struct()
    t = mdt.build_type(spec)
    o = obuild(spec)
    host = inputs.random_bytes(count * 40, seed=inputs.DEFAULT_SEED + 2)
    src = to_dev(host)
    ref = o.pack(host, 0, count)
    assert ref.size == 132_000_000
    note("full particle records: pack")
    out = zeros_dev(ref.size, 0)
    assert mdt.mdt_pack(src.data_ptr(), count, t, 0, out.data_ptr(), -1) == ref.size
    assert _dev_equal(out, ref)
    note("full particle records: partial packs")
    part = zeros_dev(MiB, 0)
    sizes = []
    for off in range(0, ref.size, MiB):
        k = mdt.mdt_pack(src.data_ptr(), count, t, off, part.data_ptr(), MiB)
        sizes.append(k)
        assert _dev_equal(part[:k], ref[off:off + k]), off
    assert len(sizes) == 126 and sizes[-1] == 928_000
    note("full particle records: unpack")
    dst = zeros_dev(count * 40, 0)
    assert mdt.mdt_unpack(out.data_ptr(), ref.size, dst.data_ptr(), count, t, 0) == ref.size
    expect = np.zeros(count * 40, np.uint8)
    o.unpack(ref, expect, 0, count)
    assert _dev_equal(dst, expect)
