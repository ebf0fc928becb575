"""GPU parity at the full measured sizes, in the launch shape the benchmark
times (one batch, one job per block, seven decoder wavefronts per block),
and for the Zipf text also with one decoder wavefront per block:

* 256 MiB of Zipf text, 1 MiB blocks of 64 x 16 KiB sub-blocks, 32 KiB
  window, matches 3..258, code lengths <= 12; ordinary and DE streams;
* 1 GiB of CSV-like rows, 2 MiB blocks of 32 KiB sub-blocks; both modes.

The whole output is compared with the source bytes (the oracle's round trip
of them is pinned by the CPU suite), and sampled blocks with the oracle's
own decode of those blocks."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import decode_stream_batched

pytestmark = pytest.mark.gpu

CASES = {
    "zipf256": ("text", 256 << 20, dict(block_size=1 << 20, sub_target_raw=16384)),
    "csv1g": ("csv", 1 << 30, dict(block_size=2 << 20, sub_target_raw=32768)),
}


@pytest.fixture(scope="module")
def ctx(hip_lib_built):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1606_00519_amd as gmp
    c = gmp.Context(0)
    yield c
    c.close()


_data = {}


def corpus(name):
    if name not in _data:
        kind, n, _ = CASES[name]
        gen = synth.zipf_text if kind == "text" else synth.csv_rows
        _data.clear()
        _data[name] = gen(n, threads=16).tobytes()
    return _data[name]


@pytest.mark.parametrize("name,de,waves", [(n, d, 7) for n in CASES for d in (0, 1)] +
                         [("zipf256", d, 1) for d in (0, 1)])
def test_full_size(ctx, name, de, waves):
    data = corpus(name)
    p = oracle.CompressParams(window=32768, max_match=258, lmax=12, de=de, group=64, **CASES[name][2])
    s = oracle.compress(data, p, threads=16)
    flags = 2 if de else 1
    st, out = decode_stream_batched(ctx, s, flags=flags, waves=waves, persistent=False)
    assert np.all(st == 0), st[st != 0][:8]
    ref = np.frombuffer(data, np.uint8)
    bad = np.flatnonzero(out != ref)
    assert bad.size == 0, f"first mismatch at byte {bad[0]} of {len(ref)}"
    blocks, bs, total = oracle.stream_blocks(s)
    rng = np.random.default_rng(7 + de)
    for b in sorted(set(rng.choice(len(blocks), size=6, replace=False).tolist()) | {len(blocks) - 1}):
        blk, off = blocks[b]
        rc, want = oracle.decompress_block(blk)
        assert rc == 0
        assert out[off:off + len(want)].tobytes() == want, f"block {b}"
