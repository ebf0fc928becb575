"""GPU checks of the boundary and of paths the parity suite does not name:
resolution modes (Sequential Copying, the DE-rule check), error classes of
malformed blocks against the oracle's, the first-error word (gmp_poll),
argument checks that never reach the device, which Huffman-stage path a
block took, and batched items of the largest configured sizes."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import decode_batch, decode_block, decode_stream

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
    return oracle.CompressParams(**kw)


# --------------------------------------------------------------------------- a bad distance in a long group

def test_bad_distance_after_long_literal_run(ctx):
    # one sequence: 32600 literals, then a 258-byte copy reaching 100 bytes
    # before the block's start.  Its group's output (32858 bytes) exceeds the
    # on-chip span, so it takes the piece-wise path; the copy is dropped and
    # the block must end with EDIST, writing nothing outside its output.
    rng = np.random.default_rng(5)
    lits = rng.integers(0, 256, 32600, dtype=np.uint8).tobytes()
    seqs = [[32600, 258, 32700]]
    blk = oracle.encode_block(seqs, lits, [1], P())
    rc, _ = oracle.decompress_block(blk, 32600 + 258)
    assert rc == oracle.EDIST
    for waves in (1, 7):
        st, _, _ = decode_batch(ctx, [blk], waves=waves)
        assert st[0] == oracle.EDIST
    st, _ = decode_block(ctx, blk, 32600 + 258)
    assert st == oracle.EDIST


# --------------------------------------------------------------------------- DE rule

def _de_breaking_block():
    # nested back-references (each reads the previous one's output) in a block
    # whose header claims DE: the rule fails in every group
    seqs, lits = synth.nesting_tokens(64 * 12, 2, str_len=16)
    blk = oracle.encode_block(seqs, lits, [len(seqs)], P(de=1))
    assert oracle.block_info(blk)["mode"] == 1
    return blk, seqs


def test_de_rule_broken_is_resolved_by_rounds(ctx):
    blk, seqs = _de_breaking_block()
    rc, want = oracle.decompress_block(blk)
    assert rc == 0
    assert oracle.validate_block(blk) == oracle.EDIST   # the CPU format check rejects it
    cnt = []
    st, outs, rounds = decode_batch(ctx, [blk], stats=True, counters=cnt)
    assert st[0] == 0 and outs[0] == want
    want_rounds, _ = oracle.mrr_rounds(seqs, 64)
    assert rounds[0].tolist() == want_rounds.tolist()
    assert cnt[0][4] == len(want_rounds)          # every group fell back to rounds
    for waves in (1, 7):
        st, outs, _ = decode_batch(ctx, [blk], flags=2, waves=waves)   # explicit DE mode: same
        assert st[0] == 0 and outs[0] == want


def test_verify_de_flag(ctx):
    import paper_1606_00519_amd as gmp
    blk, _ = _de_breaking_block()
    rc, want = oracle.decompress_block(blk)
    st, _ = decode_block(ctx, blk, len(want), flags=gmp.FLAG_VERIFY_DE)
    assert st == oracle.validate_block(blk) == gmp.EDIST
    # a DE stream that keeps the rule passes the check
    data = synth.zipf_text(3 << 20).tobytes()
    s = oracle.compress(data, P(de=1), threads=8)
    st, got = decode_stream(ctx, s, flags=gmp.FLAG_VERIFY_DE)
    assert np.all(st == 0) and got == data


# --------------------------------------------------------------------------- Sequential Copying

@pytest.mark.parametrize("kind,de", [("text", 0), ("csv", 0), ("text", 1)])
def test_sequential_copying(ctx, kind, de):
    import paper_1606_00519_amd as gmp
    data = synth.slice_of(kind, 1 << 20, 2 << 20).tobytes()
    blocks = [oracle.compress_block(data[i:i + (1 << 20)], P(de=de)) for i in range(0, len(data), 1 << 20)]
    cnt = []
    st, outs, rounds = decode_batch(ctx, blocks, flags=gmp.MODE_SC, stats=True, waves=7, counters=cnt)
    assert np.all(st == 0)
    for b, o, r, c in zip(blocks, outs, rounds, cnt):
        rc, seqs, _ = oracle.block_tokens(b)
        assert o == oracle.decompress_block(b)[1]
        # one back-reference per round: rounds = back-references of the group
        m = (seqs[:, 1] > 0).astype(np.int64)
        per_group = np.add.reduceat(m, np.arange(0, len(m), 64))
        assert (r & 0x7F).tolist() == per_group.tolist()
        assert int(c[16:80].sum()) == int(seqs[:, 1].sum())


def test_sequential_copying_nested(ctx):
    import paper_1606_00519_amd as gmp
    seqs, lits = synth.nesting_tokens(64 * 20, 1, str_len=16)
    blk = oracle.encode_block(seqs, lits, [len(seqs)], P())
    st, outs, rounds = decode_batch(ctx, [blk], flags=gmp.MODE_SC, stats=True)
    assert st[0] == 0 and outs[0] == oracle.decompress_block(blk)[1]
    assert rounds[0].tolist() == [64] * 20


# --------------------------------------------------------------------------- error classes

def _de_corrupt_cases():
    data = synth.csv_rows(400_000).tobytes()
    blk = bytes(oracle.compress_block(data, P(sub_target_raw=8192, de=1)))
    info = oracle.block_info(blk)
    rng = np.random.default_rng(3)
    pay0 = 192 + 16 * info["n_sub"] + 16
    cases = {}
    for k in range(16):
        pos = int(rng.integers(pay0, len(blk)))
        bit = int(rng.integers(0, 8))
        b = bytearray(blk)
        b[pos] ^= 1 << bit
        cases[f"de_flip{k}"] = bytes(b)
    return cases, len(data)


DE_CORRUPT, DE_CORRUPT_N = _de_corrupt_cases()


@pytest.mark.parametrize("name", sorted(DE_CORRUPT))
def test_corrupt_de_blocks(ctx, name):
    blk = DE_CORRUPT[name]
    rc, want = oracle.decompress_block(blk, DE_CORRUPT_N)
    st, got = decode_block(ctx, blk, DE_CORRUPT_N)
    print(f"[gpu] {name}: oracle {rc} gpu {st}", flush=True)
    assert st == rc
    if rc == 0:
        assert got == want


# --------------------------------------------------------------------------- first error, argument checks

def test_poll_reports_first_device_error(ctx):
    import paper_1606_00519_amd as gmp
    ctx.poll()                                       # clear what earlier tests left
    assert ctx.poll() == 0
    data = synth.zipf_text(1 << 18).tobytes()
    good = oracle.compress_block(data, P())
    st, _ = decode_block(ctx, good, len(data))
    assert st == 0 and ctx.poll() == 0
    bad = oracle.compress_block(data, P(lmax=15))    # valid format, codes longer than the tables
    st, _ = decode_block(ctx, bad, len(data))
    assert st == gmp.ENOSYS
    assert ctx.poll() == gmp.ENOSYS
    assert ctx.poll() == 0                            # cleared by the previous poll


def test_misaligned_device_pointers_rejected_on_host(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    data = synth.zipf_text(1 << 16).tobytes()
    blk = oracle.compress_block(data, P())
    s = oracle.compress(data, P())
    buf = torch.zeros(len(s) + 64, dtype=torch.uint8, device="cuda")
    out = torch.zeros(len(data), dtype=torch.uint8, device="cuda")
    status = torch.zeros(4, dtype=torch.int32, device="cuda")
    for off in (1, 4, 8):
        with pytest.raises(gmp.GmpError) as e:
            ctx.decompress_block(buf[off:off + len(blk)], blk, out, status)
        assert e.value.status == gmp.EINVAL
        with pytest.raises(gmp.GmpError) as e:
            ctx.decompress_stream(buf[off:off + len(s)], s, out, status)
        assert e.value.status == gmp.EINVAL
        job = gmp.Job(buf.data_ptr() + off, len(blk), out.data_ptr(), len(data), 0, 0, None)
        with pytest.raises(gmp.GmpError) as e:
            ctx.batch_create([job], status)
        assert e.value.status == gmp.EINVAL
        srv = gmp.Server(ctx, budget_bytes=1 << 28, slots=1)
        with pytest.raises(gmp.GmpError) as e:
            srv.submit(buf[off:off + len(s)], s, out, status)
        assert e.value.status == gmp.EINVAL
        srv.close()
    torch.cuda.synchronize()
    assert ctx.poll() == 0


# --------------------------------------------------------------------------- Huffman-stage paths

def test_huffman_stage_paths(ctx):
    # segmented decoding (with and without repaired lanes) and the one lane per
    # sub-block decoder each occur, and each decodes exactly what the oracle does
    text = synth.zipf_text(4 << 20).tobytes()
    csv = synth.csv_rows(2 << 20).tobytes()
    blocks = [oracle.compress_block(text[i:i + (1 << 20)], P()) for i in range(0, 4 << 20, 1 << 20)]
    blocks.append(oracle.compress_block(csv[:1 << 20], P(sub_target_raw=1024)))     # > 512 sub-blocks
    blocks.append(oracle.compress_block(text[:4000], P(sub_target_raw=1024)))       # payload too small to cut
    blocks.append(oracle.compress_block(csv[1 << 20:], P(de=1)))
    want = [oracle.decompress_block(b)[1] for b in blocks]
    paths = {}
    for waves in (1, 7):
        cnt = []
        st, outs, _ = decode_batch(ctx, blocks, stats=True, waves=waves, counters=cnt)
        assert np.all(st == 0) and outs == want
        for c in cnt:
            key = ("segmented" if c[0] == 1 else "per-sub-block", bool(c[1]))
            paths[key] = paths.get(key, 0) + 1
        assert cnt[4][0] == 2 and cnt[5][0] == 2
    print(f"[gpu] Huffman-stage paths: {paths}", flush=True)
    assert paths.get(("segmented", True), 0) > 0
    assert paths.get(("per-sub-block", False), 0) > 0


# --------------------------------------------------------------------------- largest batched items

def test_batched_items_up_to_4mib(ctx):
    # single-block items of the batched mix's largest sizes (1-4 MiB), text and
    # CSV, ordinary and DE, in one persistent launch and in plain launches
    text = synth.zipf_text(6 << 20).tobytes()
    csv = synth.csv_rows(6 << 20).tobytes()
    rng = np.random.default_rng(31)
    blocks, raws = [], []
    for k, size in enumerate((1 << 20, 3 << 19, 2 << 20, 3 << 20, 4 << 20, (4 << 20) - 12345)):
        src = text if k % 2 == 0 else csv
        off = int(rng.integers(0, len(src) - size))
        raw = src[off:off + size]
        blocks.append(oracle.compress_block(raw, P(block_size=size, sub_target_raw=16384, de=(k // 2) % 2)))
        raws.append(raw)
    for waves, persistent in ((7, False), (7, True), (4, False)):
        st, outs, _ = decode_batch(ctx, blocks, waves=waves, persistent=persistent, workgroups=2)
        assert np.all(st == 0)
        assert outs == raws


# --------------------------------------------------------------------------- hand-over order

@pytest.mark.parametrize("waves", [2, 4, 7])
def test_piecewise_group_keeps_done_mark_monotonic(ctx, waves):
    # A first group larger than the on-chip span (32 KiB of literal runs, then
    # 258-byte copies at distance 32768) is resolved in pieces; its last piece
    # publishes the group's end, after which the next group, on another
    # resolver wavefront, moves the finished-output mark on.  The piece-wise
    # path must not store its end again afterwards: later groups would then
    # wait on a mark that went backwards.  Repeated launches give the other
    # wavefronts every chance to run ahead.
    rng = np.random.default_rng(7)
    data = rng.integers(0, 256, 32768, dtype=np.uint8).tobytes() * 6
    blk = oracle.compress_block(data, P(block_size=1 << 18, sub_target_raw=4096))
    st, outs, _ = decode_batch(ctx, [blk] * 64, waves=waves, runs=3)
    assert np.all(st == 0)
    assert all(o == data for o in outs)


def test_slow_sync_blocks_decode_in_segments(ctx):
    # DE streams of the CSV rows hold codes that fall into step slowly: in
    # these 2 MiB blocks some decoder lanes (of 448) stay out of step for
    # 6-8 kbit past their segment's start, beyond what the first attempt's
    # boundary log covers.  The blocks are then decoded in segments a second
    # time, each lane starting 8 kbit before its segment, rather than one lane
    # per sub-block.
    n = 2 << 20
    blocks, raws = [], []
    for b in (47, 55):
        raw = synth.csv_rows(n, b * n).tobytes()
        blocks.append(oracle.compress_block(raw, P(block_size=n, sub_target_raw=32768, de=1)))
        raws.append(raw)
    cnt = []
    st, outs, _ = decode_batch(ctx, blocks, stats=True, waves=7, counters=cnt)
    assert np.all(st == 0) and outs == raws
    print(f"[gpu] paths {[int(c[0]) for c in cnt]}, further attempts {[int(c[7]) for c in cnt]}, "
          f"rejections {[int(c[6]) for c in cnt]}", flush=True)
    assert all(c[0] == 1 for c in cnt)
    assert any(c[7] >= 1 for c in cnt)


def test_out_of_step_lanes_restart_exactly(ctx):
    # In these 2 MiB CSV DE blocks a decoder lane stays out of step for more
    # than 11 kbit, longer than its whole segment and than the second
    # attempt's warm-up.  The second attempt restarts such a lane exactly at
    # the exit of the lane before it (which is in step), so the block is
    # still decoded in segments, not one lane per sub-block.
    n = 2 << 20
    blocks, raws = [], []
    for b in (484, 491):
        raw = synth.csv_rows(n, b * n).tobytes()
        blocks.append(oracle.compress_block(raw, P(block_size=n, sub_target_raw=32768, de=1)))
        raws.append(raw)
    cnt = []
    st, outs, _ = decode_batch(ctx, blocks, stats=True, waves=7, counters=cnt)
    print(f"[gpu] paths {[int(c[0]) for c in cnt]}, further attempts {[int(c[7]) for c in cnt]}, "
          f"rejections {[int(c[6]) for c in cnt]}", flush=True)
    assert np.all(st == 0) and outs == raws
    assert all(c[0] == 1 for c in cnt)
    assert all(c[7] >= 1 for c in cnt)


def test_runs_of_slow_lanes_restart_in_turn(ctx):
    # Here two neighbouring lanes at a block's start both stay out of step for
    # longer than a segment (the second for more than 12 kbit): the second
    # attempt restarts the first exactly, the third restarts the second at the
    # first's new exit.
    n = 2 << 20
    blocks, raws = [], []
    for b in (167, 255):
        raw = synth.csv_rows(n, b * n).tobytes()
        blocks.append(oracle.compress_block(raw, P(block_size=n, sub_target_raw=32768, de=1)))
        raws.append(raw)
    cnt = []
    st, outs, _ = decode_batch(ctx, blocks, stats=True, waves=7, counters=cnt)
    print(f"[gpu] paths {[int(c[0]) for c in cnt]}, further attempts {[int(c[7]) for c in cnt]}, "
          f"rejections {[int(c[6]) for c in cnt]}", flush=True)
    assert np.all(st == 0) and outs == raws
    assert all(c[0] == 1 for c in cnt)
