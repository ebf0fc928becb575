"""The C-ABI library loads and exports every entry point include/gompresso.h
declares; the host-only header parsers agree with the oracle.  No GPU needed
(no decode call is made)."""
import ctypes
import os
import re

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gompresso.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(hip_lib_built):
    lib = ctypes.CDLL(hip_lib_built)
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    import paper_1606_00519_amd as gmp
    assert set(gmp.EXPORTS) == set(names)


def test_host_parsers_agree_with_oracle(hip_lib_built):
    import paper_1606_00519_amd as gmp
    data = synth.zipf_text(700_000).tobytes()
    s = oracle.compress(data, oracle.CompressParams(block_size=1 << 18, de=1))
    assert gmp.stream_info(s) == (3, 1 << 18, len(data))
    for blk, _ in oracle.stream_blocks(s)[0]:
        mine, ref = gmp.block_info(blk), oracle.block_info(blk)
        for k in ("mode", "group", "lmax", "raw_len", "window", "max_match", "n_sub", "n_seq", "n_lit",
                  "payload_bytes", "block_bytes"):
            assert mine[k] == ref[k], k


def test_host_parser_rejects_bad_headers(hip_lib_built):
    import pytest
    import paper_1606_00519_amd as gmp
    blk = bytearray(oracle.compress_block(b"hello hello hello", oracle.CompressParams()))
    for off, val in ((0, 0), (4, 2), (5, 7), (7, 0), (18, 1)):
        b = bytearray(blk)
        b[off] = val
        with pytest.raises(gmp.GmpError) as e:
            gmp.block_info(bytes(b))
        assert e.value.status == gmp.EFORMAT
    assert gmp.strerror(gmp.ESUB)


def test_stream_info_long_block_table(hip_lib_built):
    # 768 blocks: the block table alone is longer than 4 KiB
    import paper_1606_00519_amd as gmp
    data = synth.csv_rows(3 << 20).tobytes()
    s = oracle.compress(data, oracle.CompressParams(block_size=4096, sub_target_raw=1024))
    assert gmp.stream_info(s) == (768, 4096, len(data))


def test_workspace_bytes_covers_token_stream(hip_lib_built):
    import paper_1606_00519_amd as gmp
    for n_seq, n_lit, comp in ((0, 0, 256), (1, 0, 300), (130000, 260000, 360000), (5, 1 << 20, 1 << 20)):
        ws = gmp.workspace_bytes(n_seq, n_lit, comp)
        assert ws >= 8 * n_seq + n_lit + 64 and ws % 256 == 0


def test_host_parser_reads_byte_blocks(hip_lib_built):
    import paper_1606_00519_amd as gmp
    data = synth.zipf_text(300_000).tobytes()
    for de in (0, 1):
        blk = oracle.compress_block(data, oracle.CompressParams(block_size=1 << 20, de=de, format=1))
        mine, ref = gmp.block_info(blk), oracle.block_info(blk)
        assert mine["format"] == ref["format"] == 1
        for k in ("mode", "group", "raw_len", "window", "max_match", "n_seq", "n_lit", "payload_bytes",
                  "block_bytes"):
            assert mine[k] == ref[k], k


def test_compress_bound_covers_worst_cases(hip_lib_built):
    # the largest byte-level blocks: incompressible data (literal-only records
    # of 255) and 3-byte matches back to back
    import numpy as np

    import paper_1606_00519_amd as gmp
    rng = np.random.default_rng(3)
    for data in (rng.integers(0, 256, 100_000, dtype=np.uint8).tobytes(), b"abc" * 30_000, b"", b"x"):
        blk = oracle.compress_block(data, oracle.CompressParams(block_size=1 << 20, format=1))
        assert len(blk) <= gmp.compress_bound(len(data))
    # a record per 3 bytes, each a match
    n = 30_000
    seqs = [[3, 0, 0]] + [[0, 3, 3]] * (n // 3 - 1)
    blk = oracle.encode_byte_block(seqs, b"abc", oracle.CompressParams())
    assert len(blk) <= gmp.compress_bound(n)
