"""Relay requests of a batch (pack into a staging buffer, then unpack the
same bytes into a second layout, one workgroup per tile doing both) against
the oracle: the staging buffer must hold the oracle's pack of the range and
the destination its unpack, byte for byte, with every byte outside the
destination's typemap left as it was (canary-filled buffers) -- for random
type pairs at odd alignments and partial ranges, for the workload layouts of
every tile body (chunk, record, run table), mixed with plain packs and
copies, in every launch configuration (split policy, tile order, graph
replay, the no-allocation launch)."""
import numpy as np
import pytest

import bruteforce as bf
from gpu_util import first_diff, note, to_dev, to_host
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs
from typegen import buffer_for, tiny_specs

pytestmark = pytest.mark.gpu

CONFIGS = [(1024, 0, 2, 0, 0), (1024, 0, 2, 0, 1), (256, 4, 0, 1, 0), (4096, 2, 1, 0, 1), (1024, 0, 3, 0, 0),
           (1024, 0, 0, 1, 1)]


@pytest.fixture(scope="module")
def env():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    return torch, mdt


def _pairs(seed, n):
    g = np.random.Generator(np.random.PCG64(seed))
    specs = tiny_specs(seed, 3 * n, allow_overlap=False)
    out, i = [], 0
    while len(out) < n and i + 1 < len(specs):
        sa, sb = specs[i], specs[i + 1]
        i += 2
        za, zb = bf.typemap(sa).size, bf.typemap(sb).size
        if za == 0 or zb == 0:
            continue
        ca = int(g.integers(1, 4))
        cb = -(-ca * za // zb) + int(g.integers(0, 2))
        if bf.overlaps(bf.typemap(sb), cb):
            continue
        out.append((sa, ca, sb, cb))
    return out


class Case:
    """One relay request with its device buffers and expected results."""

    def __init__(self, torch, mdt, sa, ca, sb, cb, off, mx, seed, src_host=None, src_org=0, nd=None, dst_org=0):
        self.ta, self.tb = mdt.build_type(sa), mdt.build_type(sb)
        if src_host is None:
            ns, src_org = buffer_for(bf.typemap(sa), ca, pad=19)
            src_host = inputs.random_bytes(ns, seed=seed)
        if nd is None:
            nd, dst_org = buffer_for(bf.typemap(sb), cb, pad=23)
        self.src_host, self.org_s, self.org_d = src_host, src_org, dst_org
        oa, ob = obuild(sa), obuild(sb)
        self.packed_exp = oa.pack(src_host, src_org, ca, off, mx)
        self.dst_host = np.full(nd, 0xA5, np.uint8)
        self.dst_exp = self.dst_host.copy()
        if self.packed_exp.size:
            ob.unpack(self.packed_exp, self.dst_exp, dst_org, cb, off)
        self.src = to_dev(src_host)
        self.dst = to_dev(self.dst_host)
        self.packed = torch.zeros(self.packed_exp.size + 32, dtype=torch.uint8, device="cuda")
        self.shift = 5 + seed % 11  # odd staging alignment
        self.args = (self.src.data_ptr() + src_org, ca, self.ta, self.packed.data_ptr() + self.shift,
                     self.dst.data_ptr() + dst_org, cb, self.tb, off, mx)

    def reset(self):
        self.dst.copy_(to_dev(self.dst_host))
        self.packed.fill_(0)

    def check(self, what):
        n = self.packed_exp.size
        got = to_host(self.packed)[self.shift:self.shift + n]
        assert first_diff(got, self.packed_exp) is None, (what, "packed", first_diff(got, self.packed_exp))
        h = to_host(self.packed)
        assert not h[:self.shift].any() and not h[self.shift + n:].any(), (what, "staging written outside")
        assert first_diff(to_host(self.dst), self.dst_exp) is None, (what, "dst", first_diff(to_host(self.dst),
                                                                                             self.dst_exp))


def _run(torch, mdt, cases, extra=None, noalloc=False):
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    for cfg in CONFIGS:
        note(f"relay batch cfg={cfg} cases={len(cases)}")
        b = mdt.Batch()
        for c in cases:
            assert b.add_relay(*c.args) == c.packed_exp.size
        if extra:
            extra(b)
        b.set_config(mdt.BatchConfig(*cfg))
        for rep in range(2):
            for c in cases:
                c.reset()
            if noalloc:
                b.launch_noalloc(ms)
            else:
                b.launch(ms)
            torch.cuda.synchronize()
            for c in cases:
                c.check((cfg, rep))


PAIRS = _pairs(91, 24)


def test_relay_random_pairs(env):
    torch, mdt = env
    cases = []
    for i, (sa, ca, sb, cb) in enumerate(PAIRS):
        total = ca * bf.typemap(sa).size
        off, mx = [(0, -1), (3, 17), (total // 2, -1), (1, total)][i % 4]
        cases.append(Case(torch, mdt, sa, ca, sb, cb, off, mx, seed=400 + i))
    _run(torch, mdt, cases)
    _run(torch, mdt, cases[:9], noalloc=True)


def test_relay_workload_layouts_with_packs_and_copies(env):
    torch, mdt = env
    D = inputs.DOUBLE
    lens, disps = inputs.hindexed_blocks(nblocks=20000, span=1 << 22, seed=17)
    hspec = inputs.hindexed_type(lens, disps)
    n = 96
    face_host = inputs.random_bytes(n ** 3 * 8, seed=41)
    cases = [
        # halo faces into a second array (chunk body), whole and partial
        Case(torch, mdt, inputs.halo_face(n, 1, 2, "lo"), 1, inputs.halo_face(n, 1, 2, "lo"), 1, 0, -1, 1,
             src_host=face_host, nd=n ** 3 * 8),
        Case(torch, mdt, inputs.halo_face(n, 4, 0, "hi"), 1, inputs.halo_face(n, 4, 0, "hi"), 1, 1000, 70001, 2,
             src_host=face_host, nd=n ** 3 * 8),
        # particle records (record body) into another record layout of equal size
        Case(torch, mdt, inputs.particle_struct(), 20001, ("contiguous", 33, ("basic", "BYTE")), 20001, 0, -1, 3),
        # hindexed (run-table body) into a strided vector
        Case(torch, mdt, hspec, 1, ("vector", int(lens.sum()), 1, 3, ("basic", "BYTE")), 1, 7, -1, 4),
        # a face into records, odd offset
        Case(torch, mdt, inputs.halo_face(n, 2, 1, "lo"), 1, ("vector", 30000, 3, 5, D), 1, 11, 190000, 5,
             src_host=face_host),
    ]
    # plain packs and copies in the same batch keep their own results
    spec = inputs.halo_face(n, 2, 2, "hi")
    t = mdt.build_type(spec)
    src = to_dev(face_host)
    ref = obuild(spec).pack(face_host, 0, 1)
    out = torch.zeros(ref.size, dtype=torch.uint8, device="cuda")
    cdst = torch.zeros(n ** 3 * 8, dtype=torch.uint8, device="cuda")
    cexp = np.zeros(n ** 3 * 8, np.uint8)
    obuild(spec).unpack(ref, cexp, 0, 1)

    def extra(b):
        b.add_pack(src.data_ptr(), 1, t, 0, out.data_ptr(), -1)
        b.add_copy(src.data_ptr(), 1, t, cdst.data_ptr(), 1, t, 0, -1)

    _run(torch, mdt, cases, extra)
    assert first_diff(to_host(out), ref) is None
    assert first_diff(to_host(cdst), cexp) is None
