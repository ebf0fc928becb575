"""A second, independent LZ77 expander written straight from the textbook
definition (arXiv 1606.00519, section 'LZ77 Compression'): a back-reference
(distance d, length L) appends, one byte at a time, the byte found d positions
before the current end of the output.  Pure Python; used only to pin the C
oracle's expander."""


def expand(sequences, literals: bytes) -> bytes:
    out = bytearray()
    li = 0
    for lit_len, match_len, dist in sequences:
        out += literals[li:li + lit_len]
        li += lit_len
        for _ in range(match_len):
            out.append(out[len(out) - dist])
    assert li == len(literals)
    return bytes(out)


def all_parses(data: bytes, max_match: int, window: int, min_match: int = 3):
    """Every token sequence (literal or (dist, len) copy) that reproduces data."""
    n = len(data)
    results = []

    def rec(pos, toks):
        if pos == n:
            results.append(list(toks))
            return
        toks.append(("lit", data[pos]))
        rec(pos + 1, toks)
        toks.pop()
        for d in range(1, min(pos, window) + 1):
            for L in range(min_match, min(max_match, n - pos) + 1):
                if all(data[pos + k] == data[pos + k - d] for k in range(L)):
                    toks.append(("copy", d, L))
                    rec(pos + L, toks)
                    toks.pop()
    rec(0, [])
    return results


def tokens_to_sequences(toks):
    seqs, lits, run = [], bytearray(), 0
    for t in toks:
        if t[0] == "lit":
            lits.append(t[1])
            run += 1
        else:
            seqs.append((run, t[2], t[1]))
            run = 0
    if run:
        seqs.append((run, 0, 0))
    return seqs, bytes(lits)
