"""Helpers of the GPU tests: run the HIP library through its C ABI on
oracle-produced inputs, with guard bands around every output."""
from __future__ import annotations

import numpy as np

GUARD = 4096
CANARY = 0xA5


def _torch():
    import torch
    return torch


def to_device(b: bytes):
    torch = _torch()
    if len(b) == 0:
        return torch.zeros(16, dtype=torch.uint8, device="cuda")
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).cuda()


def decode_stream(ctx, stream: bytes, flags: int = 0):
    """(per-block status array, output bytes) of gmp_decompress_stream; checks the guard bands."""
    import paper_1606_00519_amd as gmp
    torch = _torch()
    nb, bs, total = gmp.stream_info(stream)
    print(f"[gpu] decode_stream blocks={nb} block_size={bs} raw={total} flags={flags:#x}", flush=True)
    d_in = to_device(stream)
    buf = torch.full((total + 2 * GUARD,), CANARY, dtype=torch.uint8, device="cuda")
    status = torch.full((max(nb, 1),), 12345, dtype=torch.int32, device="cuda")
    ctx.decompress_stream(d_in, stream, buf[GUARD:GUARD + total], status, flags)
    torch.cuda.synchronize()
    o = buf.cpu().numpy()
    assert np.all(o[:GUARD] == CANARY) and np.all(o[GUARD + total:] == CANARY), "write outside the output"
    return status.cpu().numpy()[:nb], o[GUARD:GUARD + total].tobytes()


def decode_block(ctx, blk: bytes, out_len: int, flags: int = 0):
    import paper_1606_00519_amd as gmp
    torch = _torch()
    print(f"[gpu] decode_block bytes={len(blk)} raw={out_len} flags={flags:#x}", flush=True)
    d_in = to_device(blk)
    buf = torch.full((out_len + 2 * GUARD,), CANARY, dtype=torch.uint8, device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    ctx.decompress_block(d_in[:len(blk)] if len(blk) else d_in, blk, buf[GUARD:GUARD + out_len], status, flags)
    torch.cuda.synchronize()
    o = buf.cpu().numpy()
    assert np.all(o[:GUARD] == CANARY) and np.all(o[GUARD + out_len:] == CANARY), "write outside the output"
    return int(status.cpu()[0]), o[GUARD:GUARD + out_len].tobytes()


def decode_batch(ctx, blocks: list[bytes], flags: int = 0, waves: int = 1, persistent: bool = False,
                 workgroups: int = 0, stats: bool = False, runs: int = 1, counters: list | None = None):
    """Decode independent blocks with one batch (gmp_batch_create / gmp_batch_run).
    Returns (status array, list of outputs, list of per-group round arrays or None).
    With stats and a `counters` list, each block's GMP_STATS_WORDS counters are appended to it."""
    import paper_1606_00519_amd as gmp
    torch = _torch()
    infos = [gmp.block_info(b) for b in blocks]
    offs, pos = [], 0
    for b in blocks:
        offs.append(pos)
        pos += (len(b) + 255) & ~255
    host = bytearray(max(pos, 16))
    for o, b in zip(offs, blocks):
        host[o:o + len(b)] = b
    d_in = torch.frombuffer(host, dtype=torch.uint8).cuda()
    outs, oo = [], 0
    for i in infos:
        outs.append(oo)
        oo += (i["raw_len"] + GUARD + 255) & ~255
    buf = torch.full((oo + GUARD,), CANARY, dtype=torch.uint8, device="cuda")
    ng = [(i["n_seq"] + 63) // 64 for i in infos]
    goff = np.concatenate([[0], np.cumsum(ng)]).astype(np.int64)
    rounds = torch.zeros((max(int(goff[-1]), 1),), dtype=torch.uint8, device="cuda")
    cnt = torch.zeros((max(len(blocks), 1), gmp.STATS_WORDS), dtype=torch.int32, device="cuda")
    status = torch.full((max(len(blocks), 1),), 12345, dtype=torch.int32, device="cuda")
    jobs = []
    for k, (b, i) in enumerate(zip(blocks, infos)):
        jobs.append(gmp.Job(d_in.data_ptr() + offs[k], len(b), buf.data_ptr() + GUARD + outs[k], i["raw_len"],
                            i["n_seq"], i["n_lit"], rounds.data_ptr() + int(goff[k]) if stats else None, None,
                            cnt.data_ptr() + 4 * gmp.STATS_WORDS * k if stats else None, i["format"]))
    print(f"[gpu] decode_batch blocks={len(blocks)} flags={flags:#x} waves={waves} persistent={persistent}",
          flush=True)
    batch = ctx.batch_create(jobs, status)
    for _ in range(runs):
        batch.run(flags | (gmp.FLAG_STATS if stats else 0), waves=waves, persistent=persistent,
                  workgroups=workgroups)
    torch.cuda.synchronize()
    batch.close()
    o = buf.cpu().numpy()
    res = []
    prev_end = 0
    for k, i in enumerate(infos):
        s, n = GUARD + outs[k], i["raw_len"]
        assert np.all(o[prev_end:s] == CANARY), f"write outside block {k}'s output"
        res.append(o[s:s + n].tobytes())
        prev_end = s + n
    assert np.all(o[prev_end:] == CANARY)
    r = rounds.cpu().numpy()
    rr = [r[goff[k]:goff[k + 1]].copy() for k in range(len(blocks))] if stats else None
    if stats and counters is not None:
        c = cnt.cpu().numpy().astype(np.int64)
        counters.extend(c[k].copy() for k in range(len(blocks)))
    return status.cpu().numpy()[:len(blocks)], res, rr


def decode_stream_batched(ctx, stream: bytes, flags: int = 0, waves: int = 1, persistent: bool = False):
    """Decode a whole stream with one batch over its blocks, the launch shape the
    benchmark times (one job per block, outputs contiguous).  Returns
    (status array, output bytes); checks the guard bands."""
    import struct

    import paper_1606_00519_amd as gmp
    torch = _torch()
    nb, bs, total = gmp.stream_info(stream)
    offs = struct.unpack_from(f"<{nb + 1}Q", stream, 32)
    print(f"[gpu] decode_stream_batched blocks={nb} raw={total} flags={flags:#x} waves={waves} "
          f"persistent={persistent}", flush=True)
    d_in = to_device(stream)
    buf = torch.full((total + 2 * GUARD,), CANARY, dtype=torch.uint8, device="cuda")
    status = torch.full((max(nb, 1),), 12345, dtype=torch.int32, device="cuda")
    jobs = []
    for b in range(nb):
        blk = stream[offs[b]:offs[b + 1]]
        info = gmp.block_info(blk)
        jobs.append(gmp.Job(d_in.data_ptr() + offs[b], len(blk), buf.data_ptr() + GUARD + b * bs, info["raw_len"],
                            info["n_seq"], info["n_lit"], None, None, None, info["format"]))
    batch = ctx.batch_create(jobs, status)
    batch.run(flags, waves=waves, persistent=persistent)
    torch.cuda.synchronize()
    batch.close()
    o = buf.cpu().numpy()
    assert np.all(o[:GUARD] == CANARY) and np.all(o[GUARD + total:] == CANARY), "write outside the output"
    return status.cpu().numpy()[:nb], o[GUARD:GUARD + total]
