"""Multi-Round Resolution over several launches (the variant of section
"Performance Impact of Nested back-references" that writes the still
unresolved back-references to device memory and resolves them in later
kernels): output equal to the CPU oracle's at R = 1, 4, 16 rounds per launch
and with every round in one launch, through plain, persistent and
graph-captured launches, with the spill counts the nesting construction
fixes in closed form."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import CANARY, GUARD

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip_lib_built):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1606_00519_amd as gmp
    c = gmp.Context(0)
    yield c
    c.close()


def run(ctx, blocks, rounds, waves=7, persistent=False, graph=False, stats=False, runs=1, plain=False):
    """Decode `blocks` with one batch at `rounds` rounds per launch; returns
    (status, outputs, per-block counters)."""
    import torch

    import paper_1606_00519_amd as gmp
    infos = [gmp.block_info(b) for b in blocks]
    offs, pos = [], 0
    for b in blocks:
        offs.append(pos)
        pos += (len(b) + 255) & ~255
    host = bytearray(max(pos, 16))
    for o, b in zip(offs, blocks):
        host[o:o + len(b)] = b
    d_in = torch.frombuffer(host, dtype=torch.uint8).cuda()
    outs, oo = [], GUARD
    for i in infos:
        outs.append(oo)
        oo += (i["raw_len"] + GUARD + 255) & ~255
    buf = torch.full((oo + GUARD,), CANARY, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros((len(blocks), gmp.STATS_WORDS), dtype=torch.int32, device="cuda")
    status = torch.full((len(blocks),), 12345, dtype=torch.int32, device="cuda")
    jobs = [gmp.Job(d_in.data_ptr() + offs[k], len(b), buf.data_ptr() + outs[k], i["raw_len"], i["n_seq"], i["n_lit"],
                    None, None, cnt.data_ptr() + 4 * gmp.STATS_WORDS * k if stats else None, i["format"])
            for k, (b, i) in enumerate(zip(blocks, infos))]
    print(f"[gpu] multi-launch blocks={len(blocks)} rounds={rounds} waves={waves} persistent={persistent} "
          f"graph={graph}", flush=True)
    batch = ctx.batch_create(jobs, status)
    flags = gmp.MODE_MRR | (gmp.FLAG_STATS if stats else 0) | (gmp.FLAG_PLAIN_MRR if plain else 0)
    if graph:
        batch.graph_create(flags, waves=waves, persistent=persistent, workgroups=0, rounds_per_launch=rounds)
        for _ in range(runs):
            batch.graph_launch()
            torch.cuda.synchronize()
    else:
        for _ in range(runs):
            batch.run(flags, waves=waves, persistent=persistent, rounds_per_launch=rounds)
    torch.cuda.synchronize()
    batch.close()
    o = buf.cpu().numpy()
    res = [o[outs[k]:outs[k] + i["raw_len"]].tobytes() for k, i in enumerate(infos)]
    ends = [outs[k] + i["raw_len"] for k, i in enumerate(infos)]
    starts = outs[1:] + [len(o) - GUARD]
    for e, s_ in zip(ends, starts):
        assert np.all(o[e:s_] == CANARY), "write outside a block's output"
    assert np.all(o[:GUARD] == CANARY)
    return status.cpu().numpy(), res, cnt.cpu().numpy()


@pytest.mark.parametrize("fmt", [0, 1])
@pytest.mark.parametrize("k", [1, 4, 16])
@pytest.mark.parametrize("rounds", [1, 4, 16, 0])
@pytest.mark.parametrize("plain", [True, False])
def test_nesting_spill_counts(ctx, fmt, k, rounds, plain):
    # k interleaved chains: every group of 64 takes 64/k rounds by the paper's
    # rule.  With R < 64/k rounds per launch the first group resolves R*k
    # back-references and every later one reads bytes left pending, so exactly
    # n - R*k are spilled.  With sources moved twice through each chain a
    # group takes ceil(64/k / 3) rounds and its first 3 R k copies resolve.
    n = 64 * 12
    seqs, lits = synth.nesting_tokens(n, k, str_len=16)
    if fmt:
        head, rest = divmod(int(seqs[0, 0]), 255)
        seqs = np.concatenate([np.tile(np.array([[255, 0, 0]], np.uint32), (head, 1)),
                               np.array([[rest, seqs[0, 1], seqs[0, 2]]], np.uint32), seqs[1:]])
        blk = oracle.encode_byte_block(seqs, lits, oracle.CompressParams(format=1))
    else:
        blk = oracle.encode_block(seqs, lits, [len(seqs)], oracle.CompressParams())
    rc, want = oracle.decompress_block(blk)
    assert rc == 0
    st, outs, cnt = run(ctx, [blk], rounds, stats=True, plain=plain)
    assert st[0] == 0 and outs[0] == want
    if fmt == 0:
        spilled = int(cnt[0][8])
        per_group, done = (64 // k, rounds * k) if plain else (-(-(64 // k) // 3), 3 * rounds * k)
        expect = n - done if 0 < rounds < per_group else 0
        assert spilled == expect


@pytest.mark.parametrize("rounds", [1, 4, 16])
@pytest.mark.parametrize("waves,persistent", [(1, False), (7, False), (7, True)])
def test_real_data(ctx, rounds, waves, persistent):
    text = synth.zipf_text(2 << 20).tobytes()
    csv = synth.csv_rows(2 << 20).tobytes()
    blocks = [oracle.compress_block(text[:1 << 20], oracle.CompressParams(block_size=1 << 20)),
              oracle.compress_block(text[1 << 20:], oracle.CompressParams(block_size=1 << 20, format=1)),
              oracle.compress_block(csv, oracle.CompressParams(block_size=2 << 20, sub_target_raw=32768)),
              oracle.compress_block(text[:300_000], oracle.CompressParams(de=1))]
    st, outs, cnt = run(ctx, blocks, rounds, waves=waves, persistent=persistent, stats=True, runs=2)
    assert np.all(st == 0)
    assert outs == [text[:1 << 20], text[1 << 20:], csv, text[:300_000]]
    # a block leaves back-references to later launches exactly when one of its
    # groups needs more rounds than one launch does (the oracle's simulator)
    for b, c in zip(blocks, cnt):
        rc, seqs, _ = oracle.block_tokens(b)
        max_r = int(oracle.mrr_rounds_redirect(seqs, 64)[0].max())
        assert (c[8] > 0) == (max_r > rounds), (max_r, int(c[8]))


def test_graph_replays(ctx):
    text = synth.zipf_text(3 << 20).tobytes()
    blocks = [oracle.compress_block(text[i:i + (1 << 20)], oracle.CompressParams(block_size=1 << 20))
              for i in range(0, 3 << 20, 1 << 20)]
    st, outs, _ = run(ctx, blocks, 4, graph=True, persistent=True, runs=3)
    assert np.all(st == 0) and b"".join(outs) == text


def test_autotune_picks_rounds(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    text = synth.zipf_text(4 << 20).tobytes()
    blocks = [oracle.compress_block(text[i:i + (1 << 20)], oracle.CompressParams(block_size=1 << 20))
              for i in range(0, 4 << 20, 1 << 20)]
    infos = [gmp.block_info(b) for b in blocks]
    d_in = torch.frombuffer(bytearray(b"".join(b + bytes((-len(b)) % 256) for b in blocks)),
                            dtype=torch.uint8).cuda()
    out = torch.zeros(len(text), dtype=torch.uint8, device="cuda")
    status = torch.full((4,), 99, dtype=torch.int32, device="cuda")
    offs = np.concatenate([[0], np.cumsum([len(b) + ((-len(b)) % 256) for b in blocks])])
    jobs = [gmp.Job(d_in.data_ptr() + int(offs[k]), len(b), out.data_ptr() + (k << 20), 1 << 20, i["n_seq"],
                    i["n_lit"], None, None, None, 0) for k, (b, i) in enumerate(zip(blocks, infos))]
    batch = ctx.batch_create(jobs, status)
    tun, ms = batch.autotune(gmp.MODE_MRR, reps=2)
    print(f"[gpu] autotune: {tun}, {ms:.3f} ms", flush=True)
    assert tun["rounds_per_launch"] in (0, 1, 4, 16)
    out.zero_()
    batch.run(gmp.MODE_MRR, waves=tun["waves"], persistent=tun["persistent"], workgroups=tun["workgroups"],
              rounds_per_launch=tun["rounds_per_launch"])
    torch.cuda.synchronize()
    batch.close()
    assert np.all(status.cpu().numpy() == 0) and out.cpu().numpy().tobytes() == text
