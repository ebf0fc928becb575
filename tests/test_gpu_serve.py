"""GPU tests of the request loop (gmp_server_*): requests of mixed sizes,
generators and resolution modes decode to the same bytes alone (one
gmp_decompress_stream call each) and in the mix (admitted as they arrive,
overlapping on the device); a small HBM budget holds requests back without
ever exceeding it; a request larger than the budget is refused."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(hip_lib_built):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1606_00519_amd as gmp
    c = gmp.Context(0)
    yield c
    c.close()


def make_requests(n=16, hi=4 << 20, seed=21):
    reqs = synth.request_mix(n, seed=seed, lo=64 << 10, hi=hi, text_corpus=16 << 20, csv_corpus=16 << 20)
    text, csv = synth.zipf_text(16 << 20), synth.csv_rows(16 << 20)
    out = []
    for r in reqs:
        src = text if r["kind"] == "text" else csv
        raw = src[r["off"]:r["off"] + r["size"]].tobytes()
        p = (oracle.CompressParams(block_size=1 << 20, sub_target_raw=16384, de=r["de"]) if r["kind"] == "text"
             else oracle.CompressParams(block_size=2 << 20, sub_target_raw=32768, de=r["de"]))
        out.append((raw, oracle.compress(raw, p, threads=8)))
    return out


class Resident:
    """A request's device buffers."""

    def __init__(self, raw, stream):
        import torch

        import paper_1606_00519_amd as gmp
        self.raw, self.stream = raw, stream
        self.nb, _, total = gmp.stream_info(stream)
        self.d_in = torch.frombuffer(bytearray(stream), dtype=torch.uint8).cuda()
        self.out = torch.zeros(max(total, 1), dtype=torch.uint8, device="cuda")[:total]
        self.status = torch.full((max(self.nb, 1),), 999, dtype=torch.int32, device="cuda")

    def reset(self):
        self.out.zero_()
        self.status.fill_(999)

    def result(self):
        return self.status.cpu().numpy()[:self.nb], self.out.cpu().numpy().tobytes()


def test_alone_equals_mix(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    reqs = [Resident(raw, s) for raw, s in make_requests()]
    alone = []
    for r in reqs:
        r.reset()
        ctx.decompress_stream(r.d_in, r.stream, r.out, r.status)
        torch.cuda.synchronize()
        st, got = r.result()
        assert np.all(st == 0) and got == r.raw
        alone.append(got)
    for r in reqs:
        r.reset()
    torch.cuda.synchronize()
    srv = gmp.Server(ctx, budget_bytes=1 << 30, slots=4)
    print(f"[gpu] server mix of {len(reqs)} requests", flush=True)
    for k, r in enumerate(reqs):
        srv.submit(r.d_in, r.stream, r.out, r.status, gmp.MODE_AUTO, tag=k)
    srv.drain(60000)
    done = srv.poll(1024)
    info = srv.stats()
    srv.close()
    assert sorted(c["tag"] for c in done) == list(range(len(reqs)))
    assert all(c["status"] == 0 for c in done)
    assert all(c["t_submit_ns"] <= c["t_admit_ns"] <= c["t_done_ns"] for c in done)
    assert info["finished"] == len(reqs) and 1 <= info["launches"] <= len(reqs)
    for k, r in enumerate(reqs):
        st, got = r.result()
        assert np.all(st == 0), k
        assert got == alone[k], k


def test_small_budget_back_pressure(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    reqs = [Resident(raw, s) for raw, s in make_requests(n=12, hi=2 << 20, seed=22)]
    torch.cuda.synchronize()  # buffers are filled on torch's stream, requests run on the server's
    sizes = []
    for r in reqs:
        ws = 0
        for blk, _ in oracle.stream_blocks(r.stream)[0]:
            i = gmp.block_info(blk)
            ws += gmp.workspace_bytes(i["n_seq"], i["n_lit"], len(blk))
        sizes.append(len(r.stream) + len(r.raw) + ws)
    budget = int(max(sizes) * 1.5)
    srv = gmp.Server(ctx, budget_bytes=budget, workspace_bytes=budget, slots=4)
    for k, r in enumerate(reqs):
        srv.submit(r.d_in, r.stream, r.out, r.status, gmp.MODE_AUTO, tag=k)
    srv.drain(60000)
    info = srv.stats()
    done = srv.poll(1024)
    srv.close()
    torch.cuda.synchronize()
    assert len(done) == len(reqs) and all(c["status"] == 0 for c in done)
    assert info["peak_in_flight_bytes"] <= budget
    for r in reqs:
        st, got = r.result()
        assert np.all(st == 0) and got == r.raw


def test_oversized_request_refused(ctx):
    import paper_1606_00519_amd as gmp
    raw, s = make_requests(n=1, hi=1 << 20, seed=23)[0]
    r = Resident(raw, s)
    srv = gmp.Server(ctx, budget_bytes=len(raw) // 2, slots=2)
    with pytest.raises(gmp.GmpError) as e:
        srv.submit(r.d_in, r.stream, r.out, r.status)
    assert e.value.status == gmp.EBUSY
    srv.close()


def test_request_larger_than_default_arena_refused(ctx):
    # the budget admits the request's bytes, but its token workspace exceeds the
    # default arena (half the budget): refused at submission, never queued
    import paper_1606_00519_amd as gmp
    raw, s = make_requests(n=1, hi=2 << 20, seed=24)[0]
    r = Resident(raw, s)
    ws = 0
    for blk, _ in oracle.stream_blocks(s)[0]:
        i = gmp.block_info(blk)
        ws += gmp.workspace_bytes(i["n_seq"], i["n_lit"], len(blk))
    total = len(s) + len(raw) + ws
    budget = total + 1024
    assert ws > budget // 2
    srv = gmp.Server(ctx, budget_bytes=budget, slots=2)
    with pytest.raises(gmp.GmpError) as e:
        srv.submit(r.d_in, r.stream, r.out, r.status)
    assert e.value.status == gmp.EBUSY
    srv.drain(1000)
    srv.close()


def test_request_flags_are_kept(ctx):
    # requests with different resolution modes in one mix: each is decoded with
    # its own flags (MRR over a DE stream, Sequential Copying, auto)
    import torch

    import paper_1606_00519_amd as gmp
    reqs = [Resident(raw, s) for raw, s in make_requests(n=9, hi=3 << 20, seed=25)]
    torch.cuda.synchronize()
    modes = [gmp.MODE_AUTO, gmp.MODE_MRR, gmp.MODE_SC] * 3
    srv = gmp.Server(ctx, budget_bytes=1 << 31, slots=2)
    for k, (r, m) in enumerate(zip(reqs, modes)):
        srv.submit(r.d_in, r.stream, r.out, r.status, m, tag=k)
    srv.drain(60000)
    done = srv.poll(64)
    srv.close()
    torch.cuda.synchronize()
    assert sorted(c["tag"] for c in done) == list(range(len(reqs)))
    assert all(c["status"] == 0 for c in done)
    for r in reqs:
        st, got = r.result()
        assert np.all(st == 0) and got == r.raw


def test_completions_are_per_request(ctx):
    # a small request submitted together with large ones completes on its own,
    # before the launch that carries it has finished the large ones
    import torch

    import paper_1606_00519_amd as gmp
    text = synth.zipf_text(24 << 20).tobytes()
    big = [text[i:i + (8 << 20)] for i in (0, 8 << 20)]
    small = text[16 << 20:(16 << 20) + (64 << 10)]
    items = []
    for raw in big + [small]:
        s = oracle.compress(raw, oracle.CompressParams(block_size=1 << 20, sub_target_raw=16384), threads=8)
        items.append(Resident(raw, s))
    torch.cuda.synchronize()
    srv = gmp.Server(ctx, budget_bytes=1 << 31, slots=1)
    for k, r in enumerate(items):
        srv.submit(r.d_in, r.stream, r.out, r.status, gmp.MODE_SC, tag=k)   # slow mode: long launches
    srv.drain(60000)
    done = {c["tag"]: c for c in srv.poll(16)}
    info = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    assert set(done) == {0, 1, 2} and all(c["status"] == 0 for c in done.values())
    for r in items:
        st, got = r.result()
        assert np.all(st == 0) and got == r.raw
    if done[2]["t_admit_ns"] == done[0]["t_admit_ns"]:   # they shared a launch
        assert done[2]["t_done_ns"] < max(done[0]["t_done_ns"], done[1]["t_done_ns"])
    print(f"[gpu] launches {info['launches']}, small done after "
          f"{(done[2]['t_done_ns'] - done[2]['t_submit_ns']) / 1e6:.2f} ms, large after "
          f"{(done[0]['t_done_ns'] - done[0]['t_submit_ns']) / 1e6:.2f} ms", flush=True)
