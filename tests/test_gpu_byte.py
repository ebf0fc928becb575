"""GPU parity of Gompresso/Byte blocks (section "Parallel Decompression": the
byte-level records are read straight from the compressed block, so the
decoder goes from the records to the LZ77 stage in one pass): every decoded
byte equals the CPU oracle's decode, every malformed block gets the oracle's
error class, and the per-group round counts equal the oracle's simulator.
Byte and Bit blocks mix freely in one stream, batch or request."""
import struct

import numpy as np
import pytest

import oracle
import synth
from gpu_util import decode_batch, decode_block, decode_stream, decode_stream_batched

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip_lib_built):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1606_00519_amd as gmp
    c = gmp.Context(0)
    yield c
    c.close()


def P(**kw):
    kw.setdefault("format", 1)
    return oracle.CompressParams(**kw)


def _inputs():
    rng = np.random.default_rng(11)
    return {
        "text": synth.zipf_text(3 << 20).tobytes(),
        "csv": synth.csv_rows(3 << 20).tobytes(),
        "random": rng.integers(0, 256, 300_000, dtype=np.uint8).tobytes(),
        "zeros": bytes(700_000),
        "period17": bytes(range(17)) * 20_000,
        "farmatch": bytes(rng.integers(0, 256, 32768, dtype=np.uint8)) * 5,
        "one": b"x",
        "empty": b"",
    }


INPUTS = _inputs()


@pytest.mark.parametrize("name", sorted(INPUTS))
@pytest.mark.parametrize("de", [0, 1])
def test_byte_stream_parity(ctx, name, de):
    data = INPUTS[name]
    s = oracle.compress(data, P(block_size=1 << 20, de=de), threads=8)
    rc, want = oracle.decompress(s)
    assert rc == 0 and want == data
    st, got = decode_stream(ctx, s)
    assert np.all(st == 0), st
    assert got == want


@pytest.mark.parametrize("waves,persistent", [(1, False), (7, False), (7, True), (4, False)])
def test_byte_launch_shapes(ctx, waves, persistent):
    data = INPUTS["text"] + INPUTS["csv"][:(1 << 20) + 12345]
    s = oracle.compress(data, P(block_size=1 << 20, de=0), threads=8)
    blocks = [b for b, _ in oracle.stream_blocks(s)[0]]
    st, outs, _ = decode_batch(ctx, blocks, waves=waves, persistent=persistent, workgroups=3)
    assert np.all(st == 0)
    assert b"".join(outs) == data


@pytest.mark.parametrize("kind,size", [("text", 4 << 20), ("csv", 4 << 20)])
@pytest.mark.parametrize("de", [0, 1])
def test_byte_measured_shape(ctx, kind, size, de):
    # the benchmark's shape: 1 MiB (text) / 2 MiB (CSV) blocks, 32 KiB window, matches 3-258
    data = synth.zipf_text(size).tobytes() if kind == "text" else synth.csv_rows(size).tobytes()
    bs = 1 << 20 if kind == "text" else 2 << 20
    s = oracle.compress(data, P(block_size=bs, window=32768, max_match=258, de=de), threads=8)
    st, out = decode_stream_batched(ctx, s, flags=2 if de else 1, waves=7)
    assert np.all(st == 0)
    assert out.tobytes() == data


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("overlap", [0.0, 0.3, 0.9])
def test_byte_random_tokens(ctx, seed, overlap):
    seqs, lits = synth.random_tokens(6000, seed, overlap_frac=overlap)
    out_seqs = []
    for lit, m, d in np.asarray(seqs).tolist():
        while lit > 255:
            out_seqs.append([255, 0, 0])
            lit -= 255
        out_seqs.append([lit, m, d])
    blk = oracle.encode_byte_block(out_seqs, lits, P())
    rc, want = oracle.decompress_block(blk)
    assert rc == 0
    st, got = decode_block(ctx, blk, len(want))
    assert st == 0 and got == want


@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("waves", [1, 7])
@pytest.mark.parametrize("plain", [True, False])
def test_byte_nesting_rounds(ctx, k, waves, plain):
    # k interleaved chains of 16-byte back-references: 64/k rounds in every
    # group by the paper's rule, a third of that with sources moved twice
    import paper_1606_00519_amd as gmp
    seqs, lits = synth.nesting_tokens(64 * 16, k, str_len=16)
    blk = oracle.encode_byte_block(seqs, lits, P())
    rc, want = oracle.decompress_block(blk)
    assert rc == 0
    cnt = []
    st, outs, rounds = decode_batch(ctx, [blk], flags=1 | (gmp.FLAG_PLAIN_MRR if plain else 0), stats=True,
                                    waves=waves, counters=cnt)
    assert st[0] == 0 and outs[0] == want
    want_rounds, bpr = (oracle.mrr_rounds if plain else oracle.mrr_rounds_redirect)(seqs, 64)
    assert rounds[0].tolist() == want_rounds.tolist() == [64 // k if plain else -(-(64 // k) // 3)] * 16
    assert cnt[0][0] == 3                                   # no Huffman stage
    assert cnt[0][16:16 + 64].tolist() == bpr[:64].tolist()


@pytest.mark.parametrize("waves", [1, 7])
@pytest.mark.parametrize("plain", [True, False])
def test_byte_real_data_rounds(ctx, waves, plain):
    import paper_1606_00519_amd as gmp
    data = synth.zipf_text(2 << 20).tobytes()
    blocks = [oracle.compress_block(data[i:i + (1 << 20)], P(block_size=1 << 20)) for i in (0, 1 << 20)]
    cnt = []
    st, outs, rounds = decode_batch(ctx, blocks, flags=1 | (gmp.FLAG_PLAIN_MRR if plain else 0), stats=True,
                                    waves=waves, counters=cnt)
    assert np.all(st == 0) and b"".join(outs) == data
    for b, r, c in zip(blocks, rounds, cnt):
        rc, seqs, _ = oracle.block_tokens(b)
        want, bpr = (oracle.mrr_rounds if plain else oracle.mrr_rounds_redirect)(seqs, 64)
        assert (r & 0x7F).tolist() == want.tolist()
        assert c[16:80].tolist() == bpr[:64].tolist()


def test_byte_de_one_pass_and_sc(ctx):
    import paper_1606_00519_amd as gmp
    data = synth.csv_rows(1 << 20).tobytes()
    blk = oracle.compress_block(data, P(block_size=1 << 20, de=1))
    rc, seqs, _ = oracle.block_tokens(blk)
    st, outs, rounds = decode_batch(ctx, [blk], flags=gmp.MODE_DE, stats=True, waves=7)
    assert st[0] == 0 and outs[0] == data
    assert set((rounds[0] & 0x7F).tolist()) <= {0, 1}
    st, outs, rounds = decode_batch(ctx, [blk], flags=gmp.MODE_SC, stats=True, waves=7)
    assert st[0] == 0 and outs[0] == data
    m = (seqs[:, 1] > 0).astype(np.int64)
    assert (rounds[0] & 0x7F).tolist() == np.add.reduceat(m, np.arange(0, len(m), 64)).tolist()


def test_byte_and_bit_blocks_mix(ctx):
    data = synth.zipf_text(3 << 20).tobytes()
    blocks = []
    for i, off in enumerate(range(0, len(data), 1 << 19)):
        chunk = data[off:off + (1 << 19)]
        fmt = i % 2
        blocks.append(oracle.compress_block(chunk, oracle.CompressParams(block_size=1 << 19, de=(i // 2) % 2,
                                                                         format=fmt)))
    st, outs, _ = decode_batch(ctx, blocks, waves=7)
    assert np.all(st == 0) and b"".join(outs) == data
    # one stream whose blocks alternate between the two formats
    s = oracle.assemble_stream(blocks, 1 << 19, len(data))
    st, got = decode_stream(ctx, s)
    assert np.all(st == 0) and got == data


# --------------------------------------------------------------------------- error classes

def _byte_corrupt_cases():
    lits = bytes(range(40))
    enc = lambda seqs, **kw: oracle.encode_byte_block(seqs, lits, P(**kw))
    good = [[10, 4, 5], [10, 0, 0], [10, 5, 20], [10, 3, 1]]

    def with_record(blk, i, lit, mfield, dist):
        b = bytearray(blk)
        struct.pack_into("<I", b, 32 + 4 * i, lit | (mfield << 8) | (dist << 16))
        return bytes(b)

    blk = enc(good)
    cases = {
        "good": (blk, 52),
        "lit_total": (with_record(blk, 1, 11, 0, 0), 52),
        "raw_total": (with_record(blk, 3, 10, 4, 1), 52),
        "mfield_without_dist": (with_record(blk, 1, 10, 2, 0), 52),
        "too_long": (enc([[10, 4, 5], [10, 0, 0], [10, 73, 20], [10, 3, 1]], max_match=64), 120),
        "before_start_first": (enc([[10, 4, 15], [10, 0, 0], [10, 73, 20], [10, 3, 1]], max_match=64), 120),
        "beyond_window": (enc([[10, 4, 5], [10, 0, 0], [10, 5, 20], [10, 3, 1]], window=8), 52),
    }
    b = bytearray(blk)
    b[0] ^= 1
    cases["magic"] = (bytes(b), 52)
    b = bytearray(blk)
    b[4] = 2
    cases["version"] = (bytes(b), 52)
    b = bytearray(blk)
    b[5] = 2
    cases["mode"] = (bytes(b), 52)
    b = bytearray(blk)
    struct.pack_into("<I", b, 20, 1 << 20)                      # more records than the block holds
    cases["n_seq"] = (bytes(b), 52)
    # records of a real block with random bit flips
    data = synth.zipf_text(300_000).tobytes()
    real = oracle.compress_block(data, P(block_size=1 << 20))
    info = oracle.block_info(real)
    rng = np.random.default_rng(17)
    for k in range(20):
        b = bytearray(real)
        pos = int(rng.integers(32, 32 + 4 * info["n_seq"]))
        b[pos] ^= 1 << int(rng.integers(0, 8))
        cases[f"flip{k}"] = (bytes(b), len(data))
    return cases


BYTE_CORRUPT = _byte_corrupt_cases()


@pytest.mark.parametrize("name", sorted(BYTE_CORRUPT))
def test_byte_error_classes(ctx, name):
    import paper_1606_00519_amd as gmp
    blk, n = BYTE_CORRUPT[name]
    rc, want = oracle.decompress_block(blk, n)
    try:
        st, got = decode_block(ctx, blk, n)
    except gmp.GmpError as e:          # caught on the host (header fields)
        st, got = e.status, None
    print(f"[gpu] byte {name}: oracle {rc} gpu {st}", flush=True)
    assert st == rc
    if rc == 0:
        assert got == want


def test_byte_server(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    data = synth.zipf_text(3 << 20).tobytes()
    s = oracle.compress(data, P(block_size=1 << 20, de=1), threads=8)
    srv = gmp.Server(ctx, budget_bytes=1 << 30, slots=2)
    d_s = torch.frombuffer(bytearray(s), dtype=torch.uint8).cuda()
    o2 = torch.zeros(len(data), dtype=torch.uint8, device="cuda")
    st2 = torch.full((3,), 99, dtype=torch.int32, device="cuda")
    srv.submit(d_s, s, o2, st2, gmp.MODE_AUTO, tag=7)
    srv.drain(60000)
    done = srv.poll(16)
    srv.close()
    assert len(done) == 1 and done[0]["status"] == 0
    assert np.all(st2.cpu().numpy() == 0) and o2.cpu().numpy().tobytes() == data
