"""Parity sweep over many seeded random nested types (every constructor,
negative strides and displacements, zero block lengths, resized and
overlapping types; tests/typegen.py): each type packed on the GPU at counts
1, 37 and 1000 over its whole stream and over random byte ranges, into
guard-filled outputs; unpacked into canary-filled buffers when its typemap
does not overlap; and each seed's count-37 packs run as one batch in six
launch configurations.  Every byte is compared with the oracle.  150 types
per seed; MDT_SWEEP_SEEDS (default 4) sets how many seeds run."""
import os

import numpy as np
import pytest

import bruteforce as bf
from gpu_util import first_diff, note, to_dev, to_host, zeros_dev
from oracle import build_type as obuild
from paper_2402_12274_amd import inputs
from typegen import buffer_for, tiny_specs

pytestmark = pytest.mark.gpu

SEEDS = int(os.environ.get("MDT_SWEEP_SEEDS", "4"))
CFGS = [(1024, 0, 2, 0, 0), (256, 4, 0, 0, 1), (4096, 2, 1, 0, 0), (1024, 0, 3, 0, 0), (512, 8, 0, 1, 1),
        (2048, 0, 2, 0, 1)]


@pytest.fixture(scope="module")
def env():
    from gpu_util import torch_cuda

    torch = torch_cuda()
    from paper_2402_12274_amd import mdt

    return torch, mdt


@pytest.mark.parametrize("seed", range(SEEDS))
def test_random_types_sweep(env, seed):
    torch, mdt = env
    ms = mdt.Stream(torch.cuda.current_stream().cuda_stream)
    specs = tiny_specs(5000 + seed, 150)
    g = np.random.Generator(np.random.PCG64(seed))
    batch_cases = []
    for i, spec in enumerate(specs):
        note(f"sweep seed {seed} type {i}: {str(spec)[:100]}")
        tm = bf.typemap(spec)
        t = mdt.build_type(spec)
        o = obuild(spec)
        for count in (1, 37, 1000):
            size, origin = buffer_for(tm, count, pad=32)
            host = inputs.random_bytes(size, seed=seed * 1000 + i)
            src = to_dev(host)
            total = count * tm.size
            for off, mx in [(0, -1), (int(g.integers(0, total + 1)), int(g.integers(-1, total + 1))),
                            (int(g.integers(0, total + 1)), 1 + int(g.integers(0, 64)))]:
                n = max(0, total - off)
                if mx >= 0:
                    n = min(n, mx)
                out = zeros_dev(n + 48, 0xEE)
                got = mdt.mdt_pack(src.data_ptr() + origin, count, t, off, out.data_ptr() + 7, mx)
                h = to_host(out)
                exp = o.pack(host, origin, count, off, mx)
                assert got == n, (spec, count, off, mx)
                assert first_diff(h[7:7 + n], exp) is None, (spec, count, off, mx, first_diff(h[7:7 + n], exp))
                assert (h[:7] == 0xEE).all() and (h[7 + n:] == 0xEE).all(), (spec, count, "wrote outside")
            if total > 0 and not bf.overlaps(tm, count):
                full = o.pack(host, origin, count)
                dexp = np.full(size, 0x5A, np.uint8)
                o.unpack(full, dexp, origin, count)
                dst = zeros_dev(size, 0x5A)
                fin = to_dev(full)
                mdt.mdt_unpack(fin.data_ptr(), total, dst.data_ptr() + origin, count, t, 0)
                assert first_diff(to_host(dst), dexp) is None, (spec, count, first_diff(to_host(dst), dexp))
                if count == 37:
                    batch_cases.append((t, src, origin, count, total, full))
    outs = [zeros_dev(c[4] + 32, 0xEE) for c in batch_cases]
    b = mdt.Batch()
    for (t, src, origin, count, total, full), out in zip(batch_cases, outs):
        b.add_pack(src.data_ptr() + origin, count, t, 0, out.data_ptr() + 5, -1)
    for cfg in CFGS:
        note(f"sweep seed {seed} batch {cfg}")
        for out in outs:
            out.fill_(0xEE)
        b.set_config(mdt.BatchConfig(*cfg))
        b.launch(ms)
        torch.cuda.synchronize()
        for k, ((t, src, origin, count, total, full), out) in enumerate(zip(batch_cases, outs)):
            h = to_host(out)
            assert first_diff(h[5:5 + total], full) is None, (cfg, k, first_diff(h[5:5 + total], full))
            assert (h[:5] == 0xEE).all() and (h[5 + total:] == 0xEE).all(), (cfg, k, "wrote outside")
