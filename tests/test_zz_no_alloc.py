"""The allocation-free single-block call (gmp_decompress_block_noalloc) against
gmp_decompress_block, through the C ABI: identical output and status on two
calls in a row, the second with a smaller block; blocks beyond the fixed
workspace refused on the host."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from gpu_util import CANARY, GUARD, decode_block

pytestmark = pytest.mark.gpu


def _noalloc(blk: bytes, out_len: int, flags: int = 0):
    import torch

    import paper_1606_00519_amd as gmp
    print(f"[gpu] noalloc bytes={len(blk)} raw={out_len} flags={flags:#x}", flush=True)
    d_in = torch.frombuffer(bytearray(blk), dtype=torch.uint8).cuda()
    buf = torch.full((out_len + 2 * GUARD,), CANARY, dtype=torch.uint8, device="cuda")
    status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    h = C.create_string_buffer(bytes(blk), len(blk))
    st = gmp.lib.gmp_decompress_block_noalloc(C.c_void_p(d_in.data_ptr()), len(blk), h, len(blk),
                                              C.c_void_p(buf.data_ptr() + GUARD), out_len,
                                              C.c_void_p(status.data_ptr()), flags,
                                              C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    torch.cuda.synchronize()
    o = buf.cpu().numpy()
    assert np.all(o[:GUARD] == CANARY) and np.all(o[GUARD + out_len:] == CANARY), "write outside the output"
    return int(status.cpu()[0]), o[GUARD:GUARD + out_len].tobytes()


def test_noalloc_matches_block_call_twice():
    import paper_1606_00519_amd as gmp
    ctx = gmp.Context(0)
    text = synth.zipf_text(3 << 20).tobytes()
    big = oracle.compress_block(text[:2 << 20], oracle.CompressParams(block_size=2 << 20))
    small = oracle.compress_block(text[2 << 20:(2 << 20) + 300_000], oracle.CompressParams(de=1))
    for blk, n in ((big, 2 << 20), (small, 300_000)):
        want = decode_block(ctx, blk, n)
        got = _noalloc(blk, n)
        assert got == want and got[0] == 0
        assert got[1] == oracle.decompress_block(blk)[1]
    # a corrupt block: the same error class as the context's call
    b = bytearray(small)
    b[len(b) // 2] ^= 0x10
    assert _noalloc(bytes(b), 300_000)[0] == decode_block(ctx, bytes(b), 300_000)[0]
    ctx.close()


def test_noalloc_refuses_blocks_beyond_its_workspace():
    import torch

    import paper_1606_00519_amd as gmp
    data = synth.csv_rows(12 << 20).tobytes()
    blk = oracle.compress_block(data, oracle.CompressParams(block_size=12 << 20))
    i = gmp.block_info(blk)
    assert gmp.workspace_bytes(i["n_seq"], i["n_lit"], len(blk)) > 32 << 20
    d_in = torch.frombuffer(bytearray(blk), dtype=torch.uint8).cuda()
    out = torch.empty(len(data), dtype=torch.uint8, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    h = C.create_string_buffer(bytes(blk), len(blk))
    st = gmp.lib.gmp_decompress_block_noalloc(C.c_void_p(d_in.data_ptr()), len(blk), h, len(blk),
                                              C.c_void_p(out.data_ptr()), len(data), C.c_void_p(status.data_ptr()),
                                              0, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == gmp.ERANGE
