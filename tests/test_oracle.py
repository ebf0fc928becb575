"""Pins of the CPU oracle against facts that do not come from the oracle itself:
the paper's worked examples, RFC 1951's canonical-code example, closed forms,
brute force on tiny inputs, an independent textbook expander, round trips to
the original bytes, and the MRR round counts of the paper's nesting
construction."""
import itertools
import json
import os
import struct
import zlib

import numpy as np
import pytest

import oracle
import synth
from lz77_textbook import all_parses, expand, tokens_to_sequences

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def P(**kw):
    return oracle.CompressParams(**kw)


# ----------------------------------------------------------------------------- worked examples

def test_lz77_worked_example_decodes():
    g = golden("lz77_worked_example.json")
    rc, out = oracle.lz77_expand(g["sequences"], g["literals"].encode())
    assert rc == 0 and out == g["output"].encode()
    assert expand(g["sequences"], g["literals"].encode()) == g["output"].encode()


def test_lz77_worked_example_parse():
    # the greedy parser finds exactly the paper's literal 'c' and back-reference 'aac'
    g = golden("lz77_worked_example.json")
    seqs, lits, subs = oracle.parse_block(g["input"].encode(), P(sub_target_raw=1 << 20))
    assert seqs.tolist() == g["sequences"]
    assert lits == g["literals"].encode()


def test_rfc1951_canonical_example():
    g = golden("rfc1951_canonical_example.json")
    codes = oracle.canonical_codes(g["lengths"])
    got = [format(int(c), f"0{l}b") for c, l in zip(codes, g["lengths"])]
    assert got == g["codes"]


def test_mrr_nested_example_two_rounds():
    g = golden("mrr_nested_example.json")
    rounds, bpr = oracle.mrr_rounds(g["sequences"], g["group"])
    assert rounds.tolist() == g["rounds"]
    assert bpr[:2].tolist() == g["bytes_per_round"]
    rc, out = oracle.lz77_expand(g["sequences"], g["literals"].encode())
    assert rc == 0 and out == expand(g["sequences"], g["literals"].encode())


@pytest.mark.parametrize("case", golden("mrr_nesting_depth.json")["cases"])
def test_mrr_nesting_depth(case):
    G, k = case["group"], case["k"]
    seqs, lits = synth.nesting_tokens(G * 6, k, str_len=16)
    rounds, bpr = oracle.mrr_rounds(seqs, G)
    assert rounds.tolist() == [case["rounds_per_group"]] * 6
    r = case["rounds_per_group"]
    assert bpr[:r].tolist() == [case["bytes_per_round"] * 6] * r
    assert bpr[r:].sum() == 0


# ----------------------------------------------------------------------------- closed forms

def test_length_distance_tables_closed_form():
    lb, le = oracle.length_table()
    assert lb[0] == 3 and lb[28] == 258 and le[28] == 0
    covered = []
    for i in range(28):
        covered += list(range(int(lb[i]), int(lb[i]) + (1 << int(le[i]))))
    # codes 257..284 cover 3..258 contiguously (code 284 stops at 257 + its top
    # extra value 258 overlaps code 285, which RFC 1951 reserves for 258)
    assert covered[:255] == list(range(3, 258))
    db, de = oracle.dist_table()
    covered = []
    for i in range(30):
        covered += list(range(int(db[i]), int(db[i]) + (1 << int(de[i]))))
    assert covered == list(range(1, 32769))
    assert de.tolist() == [0, 0, 0, 0] + [i // 2 - 1 for i in range(4, 30)]


# ----------------------------------------------------------------------------- Huffman

def _brute_best(w, lmax):
    n = len(w)
    best = None
    for lens in itertools.product(range(1, lmax + 1), repeat=n):
        if sum(2.0 ** -l for l in lens) <= 1.0 + 1e-12:
            c = sum(a * b for a, b in zip(w, lens))
            best = c if best is None else min(best, c)
    return best


@pytest.mark.parametrize("seed", range(40))
def test_package_merge_optimal_vs_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    lmax = int(rng.integers(max(1, int(np.ceil(np.log2(n)))), 6))
    w = (rng.integers(1, 100, n) ** rng.integers(1, 3)).tolist()
    lens = oracle.limited_lengths(w, lmax)
    assert max(lens) <= lmax
    assert abs(sum(2.0 ** -int(l) for l in lens) - 1.0) < 1e-12  # complete code
    assert int(np.dot(w, lens)) == _brute_best(w, lmax)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8])
def test_equiprobable_symbols_get_equal_lengths(k):
    lens = oracle.limited_lengths([7] * (1 << k), 15)
    assert lens.tolist() == [k] * (1 << k)


def test_length_limit_binds():
    # Fibonacci weights want a deep tree; the limit caps it and stays complete
    w = [1, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 610, 987, 1597, 2584, 4181, 6765]
    for lmax in (5, 6, 8, 12):
        lens = oracle.limited_lengths(w, lmax)
        assert lens.max() <= lmax
        assert abs(sum(2.0 ** -int(l) for l in lens) - 1.0) < 1e-12
    # unlimited, the optimal tree for 20 Fibonacci weights is a chain of depth 19
    assert oracle.limited_lengths(w, 15).max() == 15


def test_degenerate_alphabets():
    assert oracle.limited_lengths([0, 0, 0], 12).tolist() == [0, 0, 0]
    assert oracle.limited_lengths([0, 0, 9, 0], 12).tolist() == [1, 0, 1, 0]
    assert oracle.limited_lengths([9, 0, 0, 0], 12).tolist() == [1, 1, 0, 0]


def test_canonical_prefix_free_and_ordered():
    rng = np.random.default_rng(3)
    w = rng.integers(0, 1000, 286)
    lens = oracle.limited_lengths(w, 12)
    codes = oracle.canonical_codes(lens)
    words = [format(int(c), f"0{int(l)}b") for c, l in zip(codes, lens) if l]
    for a, b in itertools.combinations(words, 2):
        assert not a.startswith(b) and not b.startswith(a)
    # within one length, codes increase with the symbol number
    for L in range(1, 13):
        cs = [int(c) for c, l in zip(codes, lens) if l == L]
        assert cs == sorted(cs) and len(set(cs)) == len(cs)


# ----------------------------------------------------------------------------- LZ77 expander pins

@pytest.mark.parametrize("seed", range(12))
def test_expander_matches_textbook(seed):
    seqs, lits = synth.random_tokens(400, seed, window=32768, max_match=258, overlap_frac=0.3)
    rc, out = oracle.lz77_expand(seqs, lits)
    assert rc == 0
    assert out == expand(seqs.tolist(), lits)


def test_expander_overlap_semantics():
    # dist 1 repeats one byte; dist 3 with length 7 repeats a 3-byte period
    rc, out = oracle.lz77_expand([[1, 5, 1]], b"z")
    assert out == b"z" * 6
    rc, out = oracle.lz77_expand([[3, 7, 3]], b"abc")
    assert out == b"abcabcabca"


def test_expander_rejects_bad_tokens():
    assert oracle.lz77_expand([[2, 3, 3]], b"ab")[0] == oracle.EDIST     # beyond produced
    assert oracle.lz77_expand([[2, 3, 0]], b"ab")[0] == oracle.EDIST     # distance 0
    assert oracle.lz77_expand([[5, 3, 5]], b"abcde", window=4)[0] == oracle.EDIST
    assert oracle.lz77_expand([[5, 65, 5]], b"abcde", max_match=64)[0] == oracle.ELEN


# ----------------------------------------------------------------------------- brute force on tiny inputs

def _tiny_inputs():
    out = []
    for n in range(1, 8):
        for t in itertools.product(b"abc", repeat=n):
            if n >= 6 and hash(t) % 7:
                continue
            out.append(bytes(t))
    return out


def test_brute_force_every_parse_decodes_and_parser_is_greedy():
    checked = 0
    for data in _tiny_inputs():
        parses = all_parses(data, max_match=258, window=32768)
        for toks in parses[:50]:
            seqs, lits = tokens_to_sequences(toks)
            # every valid parse, encoded and decoded by the oracle, reproduces data
            blk = oracle.encode_block(seqs, lits, [len(seqs)], P())
            rc, out = oracle.decompress_block(blk)
            assert rc == 0 and out == data
        seqs, lits, subs = oracle.parse_block(data, P(chain=1 << 20))
        toks = []
        li = 0
        for L, M, D in seqs.tolist():
            toks += [("lit", lits[li + q]) for q in range(L)]
            li += L
            if M:
                toks.append(("copy", D, M))
        assert toks in parses
        # greedy: at each copy the length is the longest available; at each literal none of length >= 3 exists
        pos = 0
        for t in toks:
            longest = 0
            for d in range(1, pos + 1):
                L = 0
                while pos + L < len(data) and data[pos + L] == data[pos + L - d]:
                    L += 1
                longest = max(longest, L)
            if t[0] == "lit":
                assert longest < 3
                pos += 1
            else:
                assert t[2] == min(longest, 258)
                pos += t[2]
        checked += 1
    assert checked > 300


# ----------------------------------------------------------------------------- round trips

def _cases():
    rng = np.random.default_rng(11)
    text = synth.zipf_text(300_000)
    csv = synth.csv_rows(300_000)
    return {
        "text": text.tobytes(),
        "csv": csv.tobytes(),
        "random": rng.integers(0, 256, 70_000, dtype=np.uint8).tobytes(),
        "zeros": bytes(100_000),
        "period3": (b"xyz" * 40_000),
        "period17": bytes(range(17)) * 5_000,
        "one": b"Q",
        "two": b"QQ",
        "empty": b"",
        "maxmatch": b"a" * 10_000 + bytes(rng.integers(0, 256, 300, dtype=np.uint8)) + b"a" * 300,
        "farmatch": bytes(rng.integers(0, 256, 32768, dtype=np.uint8)) * 3,
    }


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("de", [0, 1])
def test_round_trip(name, de):
    data = CASES[name]
    p = P(block_size=65536, de=de, sub_target_raw=8192)
    s = oracle.compress(data, p)
    rc, out = oracle.decompress(s)
    assert rc == 0 and out == data
    blocks, bs, total = oracle.stream_blocks(s)
    assert total == len(data) and len(blocks) == (len(data) + bs - 1) // bs
    for blk, off in blocks:
        assert oracle.validate_block(blk) == 0
        rc, seqs, lits = oracle.block_tokens(blk)
        info = oracle.block_info(blk)
        assert rc == 0 and len(seqs) == info["n_seq"] and len(lits) == info["n_lit"]
        # every distance is within the bytes produced and the window; lengths in range
        pos = np.cumsum(seqs[:, 0].astype(np.int64) + seqs[:, 1]) - seqs[:, 1]
        m = seqs[:, 1] > 0
        assert np.all(seqs[m, 2] <= np.minimum(pos[m], 32768))
        assert np.all((seqs[m, 1] >= 3) & (seqs[m, 1] <= 258))
        if de:
            assert oracle.de_holds(seqs, 64)
            rounds, _ = oracle.mrr_rounds(seqs, 64)
            has_match = np.add.reduceat(m.astype(np.int64), np.arange(0, len(seqs), 64)) > 0 if len(seqs) else []
            assert np.all(rounds[has_match] == 1) and np.all(rounds[~np.asarray(has_match, bool)] == 0)


def test_round_trip_paper_parameters():
    # the paper's own settings: 256 KB blocks, 8 KB window, 64-byte lookahead,
    # sub-blocks of 16 sequences, 10-bit code length limit
    data = synth.zipf_text(600_000).tobytes()
    p = P(block_size=256 * 1024, window=8192, max_match=64, lmax=10, sub_target_raw=0, sub_target_seq=16)
    s = oracle.compress(data, p)
    assert oracle.decompress(s) == (0, data)
    blk = oracle.stream_blocks(s)[0][0][0]
    info = oracle.block_info(blk)
    assert info["lmax"] == 10 and info["window"] == 8192
    idx = np.frombuffer(blk[192:192 + 16 * info["n_sub"]], np.uint32).reshape(-1, 4)
    assert np.all(idx[:-1, 1] == 16)


def test_round_trip_staleness_hash():
    data = synth.zipf_text(200_000).tobytes()
    for de in (0, 1):
        s = oracle.compress(data, P(hash_mode=1, staleness=1024, de=de, block_size=1 << 17))
        assert oracle.decompress(s) == (0, data)


def test_threaded_compress_identical():
    data = synth.csv_rows(3 << 20).tobytes()
    p = P(block_size=1 << 20)
    assert oracle.compress(data, p, threads=4) == oracle.compress(data, p)


def test_sub_block_cut_rule():
    data = synth.zipf_text(1 << 20).tobytes()
    seqs, lits, subs = oracle.parse_block(data, P(sub_target_raw=16384))
    raw = seqs[:, 0].astype(np.int64) + seqs[:, 1]
    ends = np.cumsum(raw)[np.cumsum(subs) - 1]
    sizes = np.diff(np.concatenate([[0], ends]))
    assert np.all(sizes[:-1] >= 16384) and np.all(sizes[:-1] < 16384 + 258)


def test_de_group_rule_and_cost():
    data = synth.zipf_text(1 << 20).tobytes()
    s0 = oracle.compress(data, P(de=0))
    s1 = oracle.compress(data, P(de=1))
    seqs = oracle.block_tokens(oracle.stream_blocks(s1)[0][0][0])[1]
    assert oracle.de_holds(seqs, 64) and oracle.de_holds(seqs, 32)   # any divisor of G
    seqs0 = oracle.block_tokens(oracle.stream_blocks(s0)[0][0][0])[1]
    assert not oracle.de_holds(seqs0, 64)
    assert len(s1) >= len(s0)   # eliminating dependencies never helps the ratio here


# ----------------------------------------------------------------------------- MRR properties

@pytest.mark.parametrize("seed", range(6))
def test_mrr_bounds_and_independent_groups(seed):
    seqs, lits = synth.random_tokens(640, seed, overlap_frac=0.2)
    for G in (32, 64):
        rounds, bpr = oracle.mrr_rounds(seqs, G)
        assert np.all(rounds >= 1) and np.all(rounds <= G)
        assert bpr.sum() == seqs[:, 1].sum()
    # back-references that only read data older than the group resolve in one round
    far = np.array([[8, 4, 4000 + 8 * i] for i in range(64)], np.uint32)
    far[0] = [5000, 4, 4000]
    assert oracle.mrr_rounds(far, 64)[0].tolist() == [1]


# ----------------------------------------------------------------------------- MRR with redirected sources

def _check_redirect_schedule(seqs, lits, G=64, jumps=2, span_limit=32768):
    """The redirected schedule against facts outside the simulator: every
    copy, read at its redirected distance, holds the bytes the sequential
    decode puts there; every byte a copy reads is final before its round
    (literals and earlier groups, or copies of earlier rounds); the rounds
    never exceed the paper's rule's."""
    seqs = np.asarray(seqs, np.int64)
    rc, out = oracle.lz77_expand(seqs.astype(np.uint32), lits)
    assert rc == 0
    out = np.frombuffer(out, np.uint8)
    rounds, bpr, sr, sd = oracle.mrr_rounds_redirect(seqs, G, jumps, span_limit, per_seq=True)
    plain, _ = oracle.mrr_rounds(seqs, G)
    assert np.all(rounds <= plain)
    assert bpr.sum() == seqs[:, 1].sum()
    L, M, D = seqs[:, 0], seqs[:, 1], seqs[:, 2]
    dst = np.cumsum(L + M) - M
    has = M > 0
    assert np.all(sd[has] >= D[has])
    moved = has & (sd != D)
    assert np.all(D[moved] >= M[moved])                       # only copies that do not overlap themselves move
    assert np.all((sr > 0) == has)
    final = np.zeros(len(out), bool)
    for g0 in range(0, len(seqs), G):
        g1 = min(len(seqs), g0 + G)
        g_start = int(dst[g0] - L[g0])
        for i in range(g0, g1):                               # the group's literals
            final[dst[i] - L[i]:dst[i]] = True
        assert int(rounds[g0 // G]) == int(sr[g0:g1].max(initial=0))
        for r in range(1, int(rounds[g0 // G]) + 1):
            now = [i for i in range(g0, g1) if sr[i] == r]
            for i in now:
                d, m, p = int(sd[i]), int(M[i]), int(dst[i])
                src = p - d
                assert final[src:src + min(m, d)].all(), (i, r)
                idx = src + np.arange(m) % d if d < m else src + np.arange(m)
                assert np.array_equal(out[idx], out[p:p + m]), i
            for i in now:
                final[dst[i]:dst[i] + M[i]] = True
        assert final[g_start:int(dst[g1 - 1] + M[g1 - 1])].all()


def test_redirect_hand_example():
    # "abcd", then three 4-byte copies at distance 4: each reads the previous
    # one's output.  The paper's rule takes three rounds; one move sends the
    # third copy to the first copy's source (two rounds), two moves send every
    # copy to the literals (one round).
    seqs = [[4, 4, 4], [0, 4, 4], [0, 4, 4]]
    assert oracle.mrr_rounds(seqs, 64)[0].tolist() == [3]
    assert oracle.mrr_rounds_redirect(seqs, 64, jumps=1)[0].tolist() == [2]
    r, bpr, sr, sd = oracle.mrr_rounds_redirect(seqs, 64, jumps=2, per_seq=True)
    assert r.tolist() == [1] and sr.tolist() == [1, 1, 1] and sd.tolist() == [4, 8, 12]
    assert bpr[:2].tolist() == [12, 0]
    # an overlapping copy (distance < length) is never moved, nor read through
    seqs = [[4, 8, 2], [0, 4, 8]]
    r, _, sr, sd = oracle.mrr_rounds_redirect(seqs, 64, per_seq=True)
    assert sd.tolist() == [2, 8] and r.tolist() == [2]
    # a copy reading past the end of the earlier destination stays where it is
    seqs = [[8, 4, 8], [0, 4, 5]]
    r, _, sr, sd = oracle.mrr_rounds_redirect(seqs, 64, per_seq=True)
    assert sd.tolist() == [8, 5] and r.tolist() == [2]
    _check_redirect_schedule([[4, 4, 4], [0, 4, 4], [0, 4, 4]], b"abcd")


@pytest.mark.parametrize("seed", range(4))
def test_redirect_without_moves_is_the_paper_rule(seed):
    seqs, _ = synth.random_tokens(900, seed, overlap_frac=0.3)
    for G in (32, 64):
        a = oracle.mrr_rounds(seqs, G)
        for b in (oracle.mrr_rounds_redirect(seqs, G, jumps=0),
                  oracle.mrr_rounds_redirect(seqs, G, jumps=2, span_limit=1)):   # no group is small enough
            assert a[0].tolist() == b[0].tolist() and a[1].tolist() == b[1].tolist()


@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("jumps", [1, 2, 3])
def test_redirect_nesting_closed_form(k, jumps):
    # chain element c of a group reads element c-1's output; after j moves it
    # reads element c-1-j's, so ceil((64/k)/(j+1)) rounds per group
    seqs, lits = synth.nesting_tokens(64 * 6, k, str_len=16)
    r, bpr = oracle.mrr_rounds_redirect(seqs, 64, jumps=jumps)
    want = -(-(64 // k) // (jumps + 1))
    assert r.tolist() == [want] * 6
    _check_redirect_schedule(seqs, lits, jumps=jumps)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("overlap", [0.0, 0.3])
def test_redirect_schedule_random(seed, overlap):
    seqs, lits = synth.random_tokens(1500, seed, overlap_frac=overlap, window=2048)
    _check_redirect_schedule(seqs, lits)


@pytest.mark.parametrize("kind", ["text", "csv"])
def test_redirect_schedule_real_data(kind):
    data = synth.slice_of(kind, 0, 300_000).tobytes()
    rc, seqs, lits = oracle.block_tokens(oracle.compress_block(data, P()))
    assert rc == 0
    _check_redirect_schedule(seqs, lits)
    r, _ = oracle.mrr_rounds_redirect(seqs, 64)
    plain, _ = oracle.mrr_rounds(seqs, 64)
    assert r.sum() < plain.sum()


# ----------------------------------------------------------------------------- corruption

def _block(de=0, n=200_000):
    data = synth.zipf_text(n).tobytes()
    return bytearray(oracle.compress_block(data, P(de=de, sub_target_raw=8192))), data


def _set32(b, off, v):
    struct.pack_into("<I", b, off, v)


def test_corruption_header_fields():
    blk, data = _block()
    for off, val, want in [(0, 0x12345678, oracle.EFORMAT),          # magic
                           (20, 0xFFFF, oracle.EFORMAT),             # n_sub beyond the block
                           (12, 0, oracle.EFORMAT)]:                 # window 0
        b = bytearray(blk)
        _set32(b, off, val)
        assert oracle.decompress_block(bytes(b), len(data))[0] == want
    b = bytearray(blk)
    b[7] = 0  # lmax 0
    assert oracle.decompress_block(bytes(b), len(data))[0] == oracle.EFORMAT
    assert oracle.decompress_block(bytes(blk), len(data) - 1)[0] == oracle.ESIZE


def test_corruption_code_lengths():
    blk, data = _block()
    b = bytearray(blk)
    b[32 + 128] = (b[32 + 128] & 0xF0) | 1   # literal 256 (end) gets a length-1 code: over-subscribed
    assert oracle.decompress_block(bytes(b), len(data))[0] == oracle.ECODE
    b = bytearray(blk)
    b[32 + 140] = 0xFF                       # two lengths of 15 > lmax 12
    assert oracle.decompress_block(bytes(b), len(data))[0] == oracle.ECODE


def test_corruption_index_and_payload():
    blk, data = _block()
    info = oracle.block_info(bytes(blk))
    b = bytearray(blk)
    _set32(b, 192 + 4, struct.unpack_from("<I", b, 192 + 4)[0] + 1)   # n_seq of sub-block 0
    assert oracle.decompress_block(bytes(b), len(data))[0] == oracle.EFORMAT
    b = bytearray(blk)
    _set32(b, 192, struct.unpack_from("<I", b, 192)[0] - 1)            # bit_len of sub-block 0
    assert oracle.decompress_block(bytes(b), len(data))[0] != 0
    trunc = bytes(blk[:len(blk) - 100])
    assert oracle.decompress_block(trunc, len(data))[0] == oracle.EFORMAT
    rng = np.random.default_rng(0)
    bad = 0
    pay0 = 192 + 16 * info["n_sub"] + 16
    for _ in range(60):
        b = bytearray(blk)
        pos = int(rng.integers(pay0, len(b)))
        b[pos] ^= 1 << int(rng.integers(0, 8))
        rc, out = oracle.decompress_block(bytes(b), len(data))
        bad += rc != 0
        assert rc != 0 or len(out) == len(data)
    assert bad > 10   # many flips break a count, a code or a distance; others only change a value


def test_token_level_errors():
    p = P()
    lits = b"abcdef"
    # distance beyond the bytes produced
    blk = oracle.encode_block([[2, 3, 5], [4, 0, 0]], lits, [2], p)
    assert oracle.decompress_block(blk)[0] == oracle.EDIST
    # distance beyond the window written in the header
    blk = oracle.encode_block([[6, 3, 6]], lits, [1], P(window=4))
    assert oracle.decompress_block(blk)[0] == oracle.EDIST
    # match longer than the header's max_match
    blk = oracle.encode_block([[6, 100, 6]], lits, [1], P(max_match=64))
    assert oracle.decompress_block(blk)[0] == oracle.ELEN


def test_validator_rejects_de_violation():
    # a stream marked DE whose second back-reference reads the first one's output
    seqs = [[4, 4, 4], [0, 4, 4]]
    blk = oracle.encode_block(seqs, b"abcd", [2], P(de=1))
    assert oracle.decompress_block(blk) == (0, b"abcd" * 3)
    assert oracle.validate_block(blk) == oracle.EDIST
    assert oracle.validate_block(oracle.encode_block(seqs, b"abcd", [2], P(de=0))) == 0


def test_stream_errors():
    data = synth.zipf_text(300_000).tobytes()
    s = bytearray(oracle.compress(data, P(block_size=100_000)))
    assert oracle.decompress(bytes(s), len(data) + 1)[0] == oracle.ESIZE
    b = bytearray(s)
    b[0] ^= 1
    assert oracle.decompress(bytes(b), len(data))[0] == oracle.EFORMAT
    b = bytearray(s)
    struct.pack_into("<Q", b, 16, len(data) + 5)      # raw_total disagrees with the blocks
    assert oracle.decompress(bytes(b), len(data) + 5)[0] != 0


# ----------------------------------------------------------------------------- generators

def test_generators_deterministic_and_sliceable():
    a = synth.zipf_text(3 << 20)
    assert np.array_equal(synth.zipf_text(5000, off=(2 << 20) - 1000), a[(2 << 20) - 1000:(2 << 20) + 4000])
    c = synth.csv_rows(2 << 20)
    assert np.array_equal(synth.csv_rows(100, off=12345), c[12345:12445])
    assert synth.sha256(synth.zipf_text(1 << 16)) == synth.sha256(a[:1 << 16])
    text = a[:1 << 20].tobytes()
    words = text.split(b" ")[1:-1]
    assert all(3 <= len(w) <= 9 and w.isalpha() and w.islower() for w in words)
    assert len(set(words)) <= 10_000
    rows = c[:1 << 20].tobytes().split(b"\n")[1:-1]
    assert all(len(r.split(b",")) == 8 for r in rows)
    assert all(0 <= int(v) < 1_000_000 for r in rows[:500] for v in r.split(b","))


def test_batch_mix_shape():
    items = synth.batch_mix()
    assert len(items) == 4096
    assert sum(i["kind"] == "text" for i in items) == 2048
    sizes = np.array([i["size"] for i in items])
    assert sizes.min() >= 4096 and sizes.max() <= 4 << 20
    assert 0.4 < np.mean([i["de"] for i in items]) < 0.6


def test_generators_match_stored_digests():
    # tests/golden/generator_digests.json is written by make_generator_digests.py
    import importlib.util
    spec = importlib.util.spec_from_file_location("mkdig", os.path.join(GOLDEN, "make_generator_digests.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    assert m.digests() == golden("generator_digests.json")


# ----------------------------------------------------------------------------- validator rules

def test_validator_rejects_nonzero_padding_bits():
    # the bits between a sub-block's end and its 128-bit boundary must be zero;
    # the decoder ignores them, the format check does not
    data = synth.zipf_text(100_000).tobytes()
    blk = bytearray(oracle.compress_block(data, P(sub_target_raw=8192)))
    info = oracle.block_info(bytes(blk))
    assert oracle.validate_block(bytes(blk)) == 0
    pay0 = 192 + 16 * info["n_sub"] + 16
    byte_off, hit = 0, 0
    for s in range(info["n_sub"]):
        bit_len = struct.unpack_from("<I", blk, 192 + 16 * s)[0]
        padded = 128 * ((bit_len + 127) // 128)
        if padded > bit_len:
            b = bytearray(blk)
            pos = bit_len + (padded - bit_len) // 2
            b[pay0 + byte_off + pos // 8] |= 1 << (pos % 8)
            assert oracle.validate_block(bytes(b)) == oracle.ESUB
            assert oracle.decompress_block(bytes(b)) == (0, data)
            hit += 1
        byte_off += padded // 8
    assert hit > 0


def test_literal_only_sequence_must_end_its_sub_block():
    # a literal-only sequence in the middle of a sub-block cannot be told apart
    # from the next sequence's literals: the decoder sees one sequence fewer
    # than the index says and rejects the block
    lits = b"abcdefgh"
    bad = oracle.encode_block([[3, 0, 0], [2, 4, 3], [3, 0, 0]], lits, [3], P())
    assert oracle.decompress_block(bad)[0] == oracle.ESUB
    good = oracle.encode_block([[3, 0, 0], [2, 4, 3], [3, 0, 0]], lits, [1, 2], P())
    assert oracle.decompress_block(good) == (0, b"abc" + b"de" + b"cdec" + b"fgh")


@pytest.mark.parametrize("kind", ["text", "csv"])
def test_decoded_literal_only_sequences_end_their_sub_blocks(kind):
    data = synth.slice_of(kind, 0, 600_000).tobytes()
    blk = oracle.compress_block(data, P(sub_target_raw=4096))
    rc, seqs, _ = oracle.block_tokens(blk)
    assert rc == 0
    info = oracle.block_info(blk)
    ends = np.cumsum([struct.unpack_from("<I", blk, 192 + 16 * s + 4)[0] for s in range(info["n_sub"])]) - 1
    zero = np.nonzero(seqs[:, 1] == 0)[0]
    assert set(zero.tolist()) <= set(ends.tolist())
    assert np.all(seqs[zero, 0] > 0)


# ----------------------------------------------------------------------------- RFC 1951 packing, by zlib

def _deflate_dynamic_header(lens, final: bool) -> tuple[int, int]:
    """(bits, count) of a DEFLATE dynamic-block header (RFC 1951 section 3.2.7)
    that declares the given 286 + 30 code lengths.  The code-length alphabet
    uses a 4-bit code for the lengths 0-15 (symbol v has code v) and none for
    the repeat codes 16-18."""
    bits, n = 0, 0

    def put(v, k):  # k bits of v, least significant first
        nonlocal bits, n
        bits |= (v & ((1 << k) - 1)) << n
        n += k

    put(1 if final else 0, 1)
    put(2, 2)                      # BTYPE 10: dynamic Huffman codes
    put(286 - 257, 5)
    put(30 - 1, 5)
    put(19 - 4, 4)
    for _ in (16, 17, 18):
        put(0, 3)
    for _ in range(16):            # code-length code lengths of 0, 8, 7, 9, ... 15: all 4
        put(4, 3)
    for ln in lens:                # each length as its 4-bit code, most significant bit first
        put(int("{:04b}".format(int(ln))[::-1], 2), 4)
    return bits, n


@pytest.mark.parametrize("kind,de", [("text", 0), ("csv", 1)])
def test_sub_block_bitstreams_inflate_with_zlib(kind, de):
    # Every sub-block of a block, given a DEFLATE dynamic header carrying the
    # block's code lengths, is a DEFLATE block; their concatenation inflates
    # with the standard library's zlib to the block's original bytes.  This
    # pins the bit packing, the canonical code assignment, the alphabets and
    # their extra bits against an implementation that shares nothing with the
    # oracle.
    data = synth.slice_of(kind, 0, 200_000).tobytes()
    blk = oracle.compress_block(data, P(block_size=len(data), sub_target_raw=16384, de=de))
    info = oracle.block_info(blk)
    lens = [(blk[32 + i // 2] >> ((i & 1) * 4)) & 15 for i in range(316)]
    pay0 = 192 + 16 * info["n_sub"] + 16
    acc, n, off = 0, 0, 0
    for s in range(info["n_sub"]):
        bit_len = struct.unpack_from("<I", blk, 192 + 16 * s)[0]
        hb, hn = _deflate_dynamic_header(lens, s + 1 == info["n_sub"])
        acc |= hb << n
        n += hn
        nbytes = (bit_len + 7) // 8
        body = int.from_bytes(blk[pay0 + off:pay0 + off + nbytes], "little") & ((1 << bit_len) - 1)
        acc |= body << n
        n += bit_len
        off += 16 * ((bit_len + 127) // 128)
    raw = acc.to_bytes((n + 7) // 8, "little")
    assert zlib.decompress(raw, -15) == data


# ----------------------------------------------------------------------------- Gompresso/Byte

def test_byte_worked_example():
    g = golden("byte_worked_example.json")
    blk = oracle.encode_byte_block(g["sequences"], g["literals"].encode(), P())
    # header: 'GMPY', version 1, mode 0, G 64, raw 7, window 32768, max 258, 2 sequences, 4 literal bytes
    want = (b"GMPY" + bytes([1, 0, 64, 0]) + struct.pack("<IIHHIII", 7, 32768, 258, 0, 2, 4, 0) +
            struct.pack("<II", 3 | (0 << 8) | (3 << 16), 1) + bytes(8) + b"aacb" + bytes(12) + bytes(16))
    assert blk == want == bytes.fromhex(g["block_hex"])
    assert oracle.decompress_block(blk) == (0, g["decoded"].encode())
    info = oracle.block_info(blk)
    assert info["format"] == 1 and info["block_bytes"] == len(blk) and info["n_sub"] == 0


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("de", [0, 1])
def test_byte_round_trip(name, de):
    data = CASES[name]
    s = oracle.compress(data, P(block_size=1 << 18, format=1, de=de), threads=4)
    assert oracle.decompress(s) == (0, data)
    for blk, _ in oracle.stream_blocks(s)[0]:
        assert oracle.validate_block(blk) == 0
        rc, seqs, lits = oracle.block_tokens(blk)
        assert rc == 0
        if len(seqs):
            assert seqs[:, 0].max() <= 255
            # literal-only sequences: only where a run reached 255 bytes, or at the block's end
            lo = np.nonzero(seqs[:, 1] == 0)[0]
            assert all(seqs[i, 0] == 255 or i == len(seqs) - 1 for i in lo)
        if de:
            assert oracle.de_holds(seqs, 64)
            r, _ = oracle.mrr_rounds(seqs, 64)
            assert set(r.tolist()) <= {0, 1}


@pytest.mark.parametrize("seed", range(6))
def test_byte_blocks_decode_like_the_textbook_expander(seed):
    seqs, lits = synth.random_tokens(3000, seed, overlap_frac=0.3)
    seqs = np.asarray(seqs)
    # split literal runs longer than a record holds into literal-only sequences
    out_seqs, li = [], 0
    for lit, m, d in seqs.tolist():
        while lit > 255:
            out_seqs.append([255, 0, 0])
            lit -= 255
        out_seqs.append([lit, m, d])
    blk = oracle.encode_byte_block(out_seqs, lits, P())
    want = expand(out_seqs, lits)
    assert oracle.decompress_block(blk) == (0, want)


def test_byte_error_classes_follow_record_order():
    lits = bytes(range(40))
    enc = lambda seqs, **kw: oracle.encode_byte_block(seqs, lits, P(**kw))
    good = [[10, 4, 5], [10, 0, 0], [10, 5, 20], [10, 3, 1]]
    assert oracle.decompress_block(enc(good))[0] == 0

    def with_record(blk, i, lit, mfield, dist):
        b = bytearray(blk)
        struct.pack_into("<I", b, 32 + 4 * i, lit | (mfield << 8) | (dist << 16))
        return bytes(b)

    blk = enc(good)
    # totals are checked first: a literal count that disagrees with the header
    assert oracle.decompress_block(with_record(blk, 1, 11, 0, 0), 52)[0] == oracle.ESUB
    # a distance of 0 with a match field (the totals ignore the field of a record without a match)
    b = with_record(blk, 1, 10, 2, 0)
    assert oracle.decompress_block(b)[0] == oracle.EFORMAT
    # a match longer than the header's max_match: ELEN
    assert oracle.decompress_block(enc([[10, 4, 5], [10, 0, 0], [10, 73, 20], [10, 3, 1]], max_match=64))[0] \
        == oracle.ELEN
    # ... unless an earlier record fails first: record 0 reaches before the block's start
    assert oracle.decompress_block(enc([[10, 4, 15], [10, 0, 0], [10, 73, 20], [10, 3, 1]], max_match=64))[0] \
        == oracle.EDIST
    # a distance beyond the window
    blk4 = enc([[10, 4, 5], [10, 0, 0], [10, 5, 20], [10, 3, 1]], window=8)
    assert oracle.decompress_block(blk4)[0] == oracle.EDIST
    assert oracle.validate_block(blk4) == oracle.EDIST
    # nonzero padding after the literals (40 of them, from offset 48): only the format check rejects it
    b = bytearray(blk)
    b[48 + 40] = 1
    assert oracle.decompress_block(bytes(b))[0] == 0 and oracle.validate_block(bytes(b)) == oracle.ESUB


def test_byte_and_bit_streams_decode_alike():
    data = synth.zipf_text(2 << 20).tobytes()
    for de in (0, 1):
        bit = oracle.compress(data, P(de=de), threads=4)
        byt = oracle.compress(data, P(de=de, format=1), threads=4)
        assert oracle.decompress(bit)[1] == oracle.decompress(byt)[1] == data
        assert len(byt) > len(bit)   # no entropy stage: a lower compression ratio
