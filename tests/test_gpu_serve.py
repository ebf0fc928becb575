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
