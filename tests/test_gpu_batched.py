"""GPU tests of the batched form: a mixed batch of independent blocks (uneven
sizes, text and CSV, ordinary and DE) decoded by one graph-captured persistent
launch, replayed several times with eager work in between, each replay checked
against the oracle; the autotuner's choice; per-job status mapping under the
largest-first dispatch order."""
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


def mixed_blocks(n_items=48, hi=1 << 20, sub=16384, seed=11):
    items = synth.batch_mix(n_items, seed=seed, lo=4096, hi=hi, text_corpus=8 << 20, csv_corpus=8 << 20)
    text = synth.zipf_text(8 << 20)
    csv = synth.csv_rows(8 << 20)
    blocks, raws = [], []
    for it in items:
        src = text if it["kind"] == "text" else csv
        raw = src[it["off"]:it["off"] + it["size"]].tobytes()
        p = oracle.CompressParams(block_size=max(len(raw), 1), sub_target_raw=sub, de=it["de"])
        blocks.append(oracle.compress_block(raw, p))
        raws.append(raw)
    return blocks, raws


class DeviceBatch:
    """Device buffers of a batch: blocks packed 256-aligned, outputs separated by guard bands."""

    def __init__(self, ctx, blocks):
        import torch

        import paper_1606_00519_amd as gmp
        self.infos = [gmp.block_info(b) for b in blocks]
        offs, pos = [], 0
        for b in blocks:
            offs.append(pos)
            pos += (len(b) + 255) & ~255
        host = bytearray(max(pos, 16))
        for o, b in zip(offs, blocks):
            host[o:o + len(b)] = b
        self.d_in = torch.frombuffer(host, dtype=torch.uint8).cuda()
        self.outs, oo = [], GUARD
        for i in self.infos:
            self.outs.append(oo)
            oo += (i["raw_len"] + GUARD + 255) & ~255
        self.buf = torch.full((oo,), CANARY, dtype=torch.uint8, device="cuda")
        self.status = torch.full((len(blocks),), 12345, dtype=torch.int32, device="cuda")
        jobs = [gmp.Job(self.d_in.data_ptr() + offs[k], len(b), self.buf.data_ptr() + self.outs[k],
                        i["raw_len"], i["n_seq"], i["n_lit"], None) for k, (b, i) in enumerate(zip(blocks, self.infos))]
        self.batch = ctx.batch_create(jobs, self.status)

    def results(self):
        o = self.buf.cpu().numpy()
        res, prev = [], 0
        for k, i in enumerate(self.infos):
            s, n = self.outs[k], i["raw_len"]
            assert np.all(o[prev:s] == CANARY), f"write outside job {k}'s output"
            res.append(o[s:s + n].tobytes())
            prev = s + n
        assert np.all(o[prev:] == CANARY)
        return self.status.cpu().numpy(), res


def test_graph_replays_match_oracle(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    blocks, raws = mixed_blocks()
    want = [oracle.decompress_block(b)[1] for b in blocks]
    assert want == raws
    db = DeviceBatch(ctx, blocks)
    db.batch.graph_create(gmp.MODE_AUTO, waves=4, persistent=True)
    for rep in range(4):
        print(f"[gpu] graph replay {rep}", flush=True)
        # eager work between replays: clear outputs and statuses with fill kernels
        for k, i in enumerate(db.infos):
            db.buf[db.outs[k]:db.outs[k] + i["raw_len"]].zero_()
        db.status.fill_(777)
        torch.cuda.synchronize()
        db.batch.graph_launch()
        torch.cuda.synchronize()
        st, outs = db.results()
        assert np.all(st == 0), st
        assert outs == want, f"replay {rep}"
    db.batch.close()


def test_graph_plain_launch_shape(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    blocks, raws = mixed_blocks(n_items=20, seed=12)
    db = DeviceBatch(ctx, blocks)
    db.batch.graph_create(gmp.MODE_AUTO, waves=1, persistent=False)
    for rep in range(2):
        db.status.fill_(777)
        db.batch.graph_launch()
        torch.cuda.synchronize()
        st, outs = db.results()
        assert np.all(st == 0) and outs == raws
    db.batch.close()


def test_autotune_choice_decodes(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    blocks, raws = mixed_blocks(n_items=40, seed=13)
    db = DeviceBatch(ctx, blocks)
    tuning, ms = db.batch.autotune(gmp.MODE_AUTO, reps=2)
    assert tuning["waves"] in (1, 2, 4, 7) and ms > 0
    if tuning["persistent"]:
        assert tuning["workgroups"] > 0
    torch.cuda.synchronize()
    st, outs = db.results()
    assert np.all(st == 0) and outs == raws
    db.status.fill_(777)
    db.batch.run(gmp.MODE_AUTO, waves=tuning["waves"], persistent=tuning["persistent"],
                 workgroups=tuning["workgroups"])
    torch.cuda.synchronize()
    st, outs = db.results()
    assert np.all(st == 0) and outs == raws
    db.batch.close()


def test_status_follows_job_index(ctx):
    import torch

    import paper_1606_00519_amd as gmp
    blocks, raws = mixed_blocks(n_items=24, seed=14)
    bad = 5
    b = bytearray(blocks[bad])
    b[32 + 128] = (b[32 + 128] & 0xF0) | 1  # code lengths no longer fill the code space
    blocks[bad] = bytes(b)
    rc, _ = oracle.decompress_block(blocks[bad])
    assert rc != 0
    db = DeviceBatch(ctx, blocks)
    db.batch.run(gmp.MODE_AUTO, waves=2, persistent=True)
    torch.cuda.synchronize()
    st, outs = db.results()
    assert st[bad] == rc
    for k in range(len(blocks)):
        if k != bad:
            assert st[k] == 0 and outs[k] == raws[k], k
    db.batch.close()
