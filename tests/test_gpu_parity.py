"""GPU parity: the HIP decoder (through the C ABI) against the CPU oracle,
byte for byte, on the same seeded inputs; the per-group MRR round counts
against the oracle's simulator; corrupt inputs rejected without writes
outside the output."""
import struct

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


def check_stream(ctx, data: bytes, params, flags=0):
    s = oracle.compress(data, params, threads=8)
    rc, want = oracle.decompress(s)
    assert rc == 0 and want == data
    st, got = decode_stream(ctx, s, flags)
    assert np.all(st == 0), st
    assert got == want
    return s


# --------------------------------------------------------------------------- the paper-shaped configs

def test_plain_single_block_cpu_scale(ctx):
    # 1 MiB Zipf text as 4 x 256 KiB blocks, 16 KiB sub-blocks, 8 KiB window,
    # matches 3..64, code lengths <= 12, multi-round resolution
    data = synth.zipf_text(1 << 20).tobytes()
    check_stream(ctx, data, P(block_size=256 << 10, window=8192, max_match=64, lmax=12, sub_target_raw=16384))


@pytest.mark.parametrize("de", [0, 1])
def test_zipf_text_1mib_blocks(ctx, de):
    data = synth.zipf_text(12 << 20).tobytes()
    s = check_stream(ctx, data, P(block_size=1 << 20, sub_target_raw=16384, de=de))
    if de:
        st, got = decode_stream(ctx, s, flags=1)    # MRR over a DE stream gives the same bytes
        assert np.all(st == 0) and got == data


@pytest.mark.parametrize("de", [0, 1])
def test_csv_2mib_blocks(ctx, de):
    data = synth.csv_rows(12 << 20).tobytes()
    check_stream(ctx, data, P(block_size=2 << 20, sub_target_raw=32768, de=de))


def test_paper_parameters(ctx):
    # the paper's settings: 256 KB blocks, 8 KB window, 64-byte lookahead,
    # sub-blocks of 16 sequences, 10-bit code lengths
    data = synth.zipf_text(3 << 20).tobytes()
    check_stream(ctx, data, P(block_size=256 << 10, window=8192, max_match=64, lmax=10, sub_target_raw=0,
                              sub_target_seq=16))


@pytest.mark.parametrize("sub", [1024, 4096, 65536])
def test_sub_block_sizes(ctx, sub):
    # 1024-byte sub-blocks give ~1000 lanes per block: several decode passes per workgroup
    data = synth.csv_rows(3 << 20).tobytes()
    check_stream(ctx, data, P(block_size=1 << 20, sub_target_raw=sub, de=1))


@pytest.mark.parametrize("lmax", [9, 10, 11, 13])
def test_code_length_limits(ctx, lmax):
    data = synth.zipf_text(2 << 20).tobytes()
    check_stream(ctx, data, P(block_size=1 << 20, lmax=lmax))


def test_code_length_beyond_tables_rejected(ctx):
    data = synth.zipf_text(1 << 18).tobytes()
    blk = oracle.compress_block(data, P(lmax=15))
    assert oracle.decompress_block(blk)[0] == 0
    st, _ = decode_block(ctx, blk, len(data))
    assert st == -11   # ENOSYS: this decoder's tables hold codes up to 13 bits


# --------------------------------------------------------------------------- adversarial inputs

@pytest.mark.parametrize("name", ["random", "zeros", "period3", "period17", "one", "two", "tiny3", "maxmatch",
                                  "farmatch", "lit_run"])
@pytest.mark.parametrize("de", [0, 1])
def test_edge_inputs(ctx, name, de):
    rng = np.random.default_rng(7)
    data = {
        "random": lambda: rng.integers(0, 256, 300_000, dtype=np.uint8).tobytes(),
        "zeros": lambda: bytes(400_000),
        "period3": lambda: b"xyz" * 90_000,
        "period17": lambda: bytes(range(17)) * 20_000,
        "one": lambda: b"Q",
        "two": lambda: b"QQ",
        "tiny3": lambda: b"abc",
        "maxmatch": lambda: (b"a" * 20_000 + bytes(rng.integers(0, 256, 300, dtype=np.uint8))) * 8,
        "farmatch": lambda: rng.integers(0, 256, 32768, dtype=np.uint8).tobytes() * 6,
        "lit_run": lambda: rng.integers(0, 256, 200_000, dtype=np.uint8).tobytes() + b"z" * 1000,
    }[name]()
    # large sub-blocks: incompressible input becomes literal runs far longer than the on-chip window
    check_stream(ctx, data, P(block_size=1 << 20, sub_target_raw=1 << 20, de=de))
    check_stream(ctx, data, P(block_size=1 << 18, sub_target_raw=4096, de=de))


def test_empty_stream(ctx):
    s = oracle.compress(b"", P())
    st, got = decode_stream(ctx, s)
    assert got == b"" and len(st) == 0


@pytest.mark.parametrize("seed", range(8))
def test_random_token_streams(ctx, seed):
    # overlapping copies (distance < length), long matches, distances up to the window
    seqs, lits = synth.random_tokens(6000, seed, overlap_frac=0.25, window=32768, max_match=258)
    n = len(seqs)
    subs = [n // 5] * 4 + [n - 4 * (n // 5)]
    blk = oracle.encode_block(seqs, lits, subs, P())
    rc, want = oracle.decompress_block(blk)
    assert rc == 0
    st, got = decode_block(ctx, blk, len(want))
    assert st == 0 and got == want


@pytest.mark.parametrize("dist", [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32768])
def test_overlap_distances(ctx, dist):
    rng = np.random.default_rng(dist)
    first = dist + 5 if dist < 32768 else 32768
    lits = rng.integers(0, 256, first + 200, dtype=np.uint8).tobytes()
    seqs = [[first, 258, dist]] + [[1, int(rng.integers(3, 259)), dist] for _ in range(200)]
    blk = oracle.encode_block(seqs, lits, [len(seqs)], P())
    rc, want = oracle.decompress_block(blk)
    assert rc == 0
    st, got = decode_block(ctx, blk, len(want))
    assert st == 0 and got == want


# --------------------------------------------------------------------------- MRR rounds against the simulator

@pytest.mark.parametrize("waves", [1, 7])
@pytest.mark.parametrize("k", [1, 2, 4, 8])
@pytest.mark.parametrize("plain", [True, False])
def test_mrr_rounds_nesting(ctx, k, waves, plain):
    import paper_1606_00519_amd as gmp
    seqs, lits = synth.nesting_tokens(64 * 40, k, str_len=16)
    blk = oracle.encode_block(seqs, lits, [len(seqs) // 2, len(seqs) - len(seqs) // 2], P())
    if plain:       # the paper's rule: 64/k rounds
        want_rounds, want_bytes = oracle.mrr_rounds(seqs, 64)
        per_group = 64 // k
    else:           # sources moved through the chain twice: a third of them
        want_rounds, want_bytes = oracle.mrr_rounds_redirect(seqs, 64)
        per_group = -(-(64 // k) // 3)
    cnt = []
    st, outs, rounds = decode_batch(ctx, [blk], flags=1 | (gmp.FLAG_PLAIN_MRR if plain else 0), stats=True,
                                    waves=waves, counters=cnt)
    assert st[0] == 0 and outs[0] == oracle.decompress_block(blk)[1]
    assert rounds[0].tolist() == want_rounds.tolist() == [per_group] * 40
    # bytes copied per round, summed over groups: the simulator's
    assert cnt[0][16:80].tolist() == want_bytes.tolist()
    if plain:       # and 16 k bytes per round per group
        assert want_bytes[:64 // k].tolist() == [40 * 16 * k] * (64 // k)


@pytest.mark.parametrize("waves", [1, 7])
@pytest.mark.parametrize("kind", ["text", "csv"])
@pytest.mark.parametrize("plain", [True, False])
def test_mrr_rounds_real_data(ctx, kind, waves, plain):
    import paper_1606_00519_amd as gmp
    data = synth.slice_of(kind, 0, 4 << 20).tobytes()
    blocks = [oracle.compress_block(data[i:i + (1 << 20)], P()) for i in range(0, len(data), 1 << 20)]
    cnt = []
    st, outs, rounds = decode_batch(ctx, blocks, flags=gmp.FLAG_PLAIN_MRR if plain else 0, stats=True,
                                    waves=waves, counters=cnt)
    assert np.all(st == 0)
    for b, o, r, c in zip(blocks, outs, rounds, cnt):
        rc, seqs, lits = oracle.block_tokens(b)
        want, want_bytes = (oracle.mrr_rounds if plain else oracle.mrr_rounds_redirect)(seqs, 64)
        assert o == oracle.decompress_block(b)[1]
        assert not np.any(r & 0x80)   # no group was split
        assert r.tolist() == want.tolist()
        assert c[16:80].tolist() == want_bytes.tolist()
        assert c[2] == len(want) and c[3] == 0


@pytest.mark.parametrize("waves", [1, 7])
def test_de_single_pass_rounds(ctx, waves):
    data = synth.zipf_text(2 << 20).tobytes()
    blocks = [oracle.compress_block(data[i:i + (1 << 20)], P(de=1)) for i in range(0, len(data), 1 << 20)]
    cnt = []
    st, outs, rounds = decode_batch(ctx, blocks, flags=0, stats=True, waves=waves, counters=cnt)
    assert np.all(st == 0)
    for b, o, r, c in zip(blocks, outs, rounds, cnt):
        assert o == oracle.decompress_block(b)[1]
        assert set(r.tolist()) <= {0, 1}
        rc, seqs, _ = oracle.block_tokens(b)
        assert c[16] == int(seqs[:, 1].sum()) and not np.any(c[17:80])   # every copy in the one pass
        assert c[4] == 0                                                  # no group broke the DE rule


# --------------------------------------------------------------------------- launch shapes

@pytest.mark.parametrize("waves,persistent", [(w, p) for p in (False, True) for w in (1, 2, 4, 7)])
def test_launch_shapes_agree(ctx, waves, persistent):
    data = synth.csv_rows(6 << 20).tobytes()
    blocks = []
    for i, off in enumerate(range(0, len(data), 1 << 20)):
        blocks.append(oracle.compress_block(data[off:off + (1 << 20)], P(sub_target_raw=[4096, 16384][i % 2],
                                                                          de=i % 2)))
    want = [oracle.decompress_block(b)[1] for b in blocks]
    st, outs, _ = decode_batch(ctx, blocks, waves=waves, persistent=persistent, workgroups=3, runs=2)
    assert np.all(st == 0)
    assert outs == want


# --------------------------------------------------------------------------- errors

def _corrupt_cases():
    data = synth.zipf_text(300_000).tobytes()
    blk = bytes(oracle.compress_block(data, P(sub_target_raw=8192)))
    info = oracle.block_info(blk)
    cases = {}

    def mod(name, fn):
        b = bytearray(blk)
        fn(b)
        cases[name] = bytes(b)

    mod("magic", lambda b: struct.pack_into("<I", b, 0, 0x11223344))
    mod("kraft_over", lambda b: b.__setitem__(32 + 128, (b[32 + 128] & 0xF0) | 1))
    mod("len_over_lmax", lambda b: b.__setitem__(32 + 140, 0xFF))
    mod("index_nseq", lambda b: struct.pack_into("<I", b, 196, struct.unpack_from("<I", b, 196)[0] + 1))
    mod("index_bits", lambda b: struct.pack_into("<I", b, 192, struct.unpack_from("<I", b, 192)[0] - 1))
    mod("index_raw", lambda b: struct.pack_into("<I", b, 204, struct.unpack_from("<I", b, 204)[0] + 3))
    rng = np.random.default_rng(1)
    pay0 = 192 + 16 * info["n_sub"] + 16
    for k in range(24):
        pos = int(rng.integers(pay0, len(blk)))
        bit = int(rng.integers(0, 8))
        mod(f"flip{k}", lambda b, pos=pos, bit=bit: b.__setitem__(pos, b[pos] ^ (1 << bit)))
    return cases, len(data)


CORRUPT, CORRUPT_N = _corrupt_cases()


@pytest.mark.parametrize("name", sorted(CORRUPT))
def test_corrupt_blocks(ctx, name):
    blk = CORRUPT[name]
    rc, want = oracle.decompress_block(blk, CORRUPT_N)
    try:
        st, got = decode_block(ctx, blk, CORRUPT_N)
    except Exception as e:  # the host parser may reject the header synchronously
        import paper_1606_00519_amd as gmp
        assert isinstance(e, gmp.GmpError) and rc != 0
        return
    print(f"[gpu] {name}: oracle {rc} gpu {st}", flush=True)
    # the same error class as the oracle: a single corruption damages one
    # sub-block, whose symbols both decoders check in the same order
    assert st == rc
    if rc == 0:
        assert got == want
    if name in ("kraft_over", "len_over_lmax"):
        assert st == rc == -3


def test_de_flag_on_ordinary_stream_rejected(ctx):
    data = synth.zipf_text(1 << 19).tobytes()
    blk = oracle.compress_block(data, P(de=0))
    st, _ = decode_block(ctx, blk, len(data), flags=2)
    assert st == -1


def test_wrong_out_len_rejected(ctx):
    import paper_1606_00519_amd as gmp
    data = synth.zipf_text(1 << 16).tobytes()
    blk = oracle.compress_block(data, P())
    with pytest.raises(gmp.GmpError) as e:
        decode_block(ctx, blk, len(data) - 1)
    assert e.value.status == gmp.ESIZE


def test_repeated_runs_identical(ctx):
    data = synth.zipf_text(4 << 20).tobytes()
    s = oracle.compress(data, P(), threads=4)
    outs = {decode_stream(ctx, s)[1] for _ in range(3)}
    assert outs == {data}
