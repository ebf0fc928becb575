"""GPU compression into byte-level blocks (gmp_compress_batch), with and
without Dependency Elimination.  Several compressed forms of a block are
valid, so the compressed bytes are not compared with the CPU compressor's:
every block must pass the CPU reference's format check (which includes the
DE rule for DE blocks and zero padding), decode on the CPU reference to the
input, and decode on the GPU to the input; its size stays within the bound,
and its ratio is compared with the CPU compressor's."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import decode_stream

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip_lib_built):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1606_00519_amd as gmp
    c = gmp.Context(0)
    yield c
    c.close()


def gpu_compress(ctx, data: bytes, block: int, de: int, window: int = 32768, max_match: int = 258):
    """Compress `data` in blocks of `block` bytes on the GPU; returns the blocks."""
    import torch

    import paper_1606_00519_amd as gmp
    chunks = [data[i:i + block] for i in range(0, len(data), block)] or [b""]
    print(f"[gpu] compress {len(data)} bytes in {len(chunks)} blocks de={de}", flush=True)
    d_in = torch.frombuffer(bytearray(data + bytes(16)), dtype=torch.uint8).cuda()
    caps = [(gmp.compress_bound(len(c)) + 255) & ~255 for c in chunks]
    outs = torch.zeros(sum(caps), dtype=torch.uint8, device="cuda")
    lens = torch.zeros(len(chunks), dtype=torch.int64, device="cuda")
    status = torch.full((len(chunks),), 99, dtype=torch.int32, device="cuda")
    jobs, off = [], 0
    for k, c in enumerate(chunks):
        jobs.append(gmp.CompressJob(d_in.data_ptr() + k * block, len(c), outs.data_ptr() + off, caps[k],
                                    lens.data_ptr() + 8 * k, status.data_ptr() + 4 * k))
        off += caps[k]
    ctx.compress_batch(jobs, window=window, max_match=max_match, de=de)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert np.all(st == 0), st
    ln = lens.cpu().numpy()
    o = outs.cpu().numpy()
    res, off = [], 0
    for k, c in enumerate(chunks):
        assert 48 <= ln[k] <= gmp.compress_bound(len(c))
        res.append(o[off:off + int(ln[k])].tobytes())
        off += caps[k]
    return res


def _inputs():
    rng = np.random.default_rng(5)
    return {
        "text": synth.zipf_text(3 << 20).tobytes(),
        "csv": synth.csv_rows(3 << 20).tobytes(),
        "random": rng.integers(0, 256, 200_000, dtype=np.uint8).tobytes(),
        "zeros": bytes(500_000),
        "period17": bytes(range(17)) * 30_000,
        "farmatch": rng.integers(0, 256, 32768, dtype=np.uint8).tobytes() * 4,
        "one": b"Q",
        "tiny": b"abcabcabcab",
        "empty": b"",
    }


INPUTS = _inputs()


@pytest.mark.parametrize("name", sorted(INPUTS))
@pytest.mark.parametrize("de", [0, 1])
def test_round_trip(ctx, name, de):
    data = INPUTS[name]
    block = 1 << 20
    blocks = gpu_compress(ctx, data, block, de)
    for k, blk in enumerate(blocks):
        raw = data[k * block:(k + 1) * block]
        info = oracle.block_info(blk)
        assert info["format"] == 1 and info["mode"] == de and info["raw_len"] == len(raw)
        assert oracle.validate_block(blk) == 0                      # includes the DE rule when de = 1
        assert oracle.decompress_block(blk) == (0, raw)
        if de and len(raw):
            rc, seqs, _ = oracle.block_tokens(blk)
            assert oracle.de_holds(seqs, 64)
            r, _ = oracle.mrr_rounds(seqs, 64)
            assert set(r.tolist()) <= {0, 1}                        # one pass per group
    if data:                                                        # (an empty input is a stream of no blocks)
        s = oracle.assemble_stream(blocks, block, len(data))
        st, got = decode_stream(ctx, s)                             # the GPU decoder reads them too
        assert np.all(st == 0) and got == data


@pytest.mark.parametrize("kind", ["text", "csv"])
@pytest.mark.parametrize("de", [0, 1])
def test_ratio_against_cpu_compressor(ctx, kind, de):
    data = INPUTS[kind]
    gpu = sum(len(b) for b in gpu_compress(ctx, data, 1 << 20, de))
    cpu = len(oracle.compress(data, oracle.CompressParams(block_size=1 << 20, de=de, format=1), threads=8))
    print(f"[gpu] {kind} de={de}: GPU ratio {len(data) / gpu:.3f}, CPU ratio {len(data) / cpu:.3f}", flush=True)
    assert gpu <= 1.25 * cpu


@pytest.mark.parametrize("name,period,max_lits", [("zeros", 1, 1), ("period17", 17, 64)])
def test_matches_reach_max_match(ctx, name, period, max_lits):
    # A run of one byte and a period of 17.  The greedy parse takes literals
    # until the first match (a run: from position 1, at distance 1, from the
    # bytes beside p; the period: once the hash walk, which links a position
    # only to positions of earlier groups of 64, offers one, so within the
    # first 64), then matches of max_match bytes at a multiple of the period
    # until the last, which the block's end cuts: every candidate is extended
    # to the cap.  The block stays under 64 KiB, which the GPU parses in one
    # part (larger blocks are parsed in parts that no match crosses).
    data = INPUTS[name][:60000]
    (blk,) = gpu_compress(ctx, data, 1 << 20, 0)
    rc, seqs, _ = oracle.block_tokens(blk)
    assert rc == 0
    lits = int(seqs[0, 0])
    assert period <= lits <= max_lits and np.all(seqs[1:, 0] == 0)
    m = seqs[:, 1] > 0
    assert np.all(seqs[m, 2] % period == 0)
    assert np.all(seqs[m, 1][:-1] == 258) and 3 <= seqs[m, 1][-1] <= 258
    assert lits + int(seqs[m, 1].sum()) == len(data)


def test_window_and_match_limits(ctx):
    data = INPUTS["text"][:1 << 20]
    for window, max_match in ((8192, 64), (1024, 16), (32768, 3)):
        for blk in gpu_compress(ctx, data, 1 << 19, 0, window=window, max_match=max_match):
            rc, seqs, _ = oracle.block_tokens(blk)
            assert rc == 0
            m = seqs[:, 1] > 0
            assert seqs[m, 2].max() <= window and seqs[m, 1].max() <= max_match
            assert oracle.validate_block(blk) == 0


def test_rejects_bad_arguments(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    d = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    lens = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    small = gmp.CompressJob(d.data_ptr(), 1000, d.data_ptr() + 2048, 100, lens.data_ptr(), st.data_ptr())
    misaligned = gmp.CompressJob(d.data_ptr(), 100, d.data_ptr() + 2049, 2000, lens.data_ptr(), st.data_ptr())
    for job, kw in ((small, {}), (misaligned, {}), (gmp.CompressJob(d.data_ptr(), 100, d.data_ptr() + 2048, 2000,
                                                                     lens.data_ptr(), st.data_ptr()),
                                                    {"window": 40000})):
        with pytest.raises(gmp.GmpError) as e:
            ctx.compress_batch([job], **kw)
        assert e.value.status == gmp.EINVAL
