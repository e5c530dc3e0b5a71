"""Prepared batches and their hipGraph replay (sft_batch_*), through the C ABI:
the same results as sft_execute_many bit for bit, on every replay, with the
program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest

import siggen
from tests.test_gpu_parity import dev, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _same(outs_a, counts_a, outs_b, counts_b):
    assert torch.equal(counts_a, counts_b)
    for (wa, ca), (wb, cb) in zip(outs_a, outs_b):
        assert torch.equal(wa, wb) and torch.equal(ca, cb)


def test_prepared_batch_equals_execute_many(gpu):
    """Mixed N, s, presets and identifications in one prepared batch."""
    shapes = [(2 ** 14, 8, {}), (100_003, 20, {"ident": "phase"}), (2 ** 16, 40, {"preset": 1}),
              (2 ** 14, 8, {}), (3 * 2 ** 15, 12, {"dft_path": 2}), (31, 1, {})]
    plans = [gpu.Plan(N, s, **kw) for N, s, kw in shapes]
    fs = [dev(siggen.sparse_signal(N, s, seed=90 + i, snr_db=30.0).f32) for i, (N, s, _) in enumerate(shapes)]
    say("prepared batch", len(shapes))
    ref = gpu.execute_many(plans, fs)
    batch = gpu.Batch(plans, fs)
    outs, counts = batch.launch()
    torch.cuda.synchronize()
    _same(outs, counts, *ref)
    batch.close()


def test_graph_replays_equal_eager(gpu):
    """One batch captured once and replayed four times on new inputs written in
    place; eager execute_many calls run between the replays, and every replay
    equals the eager result of the same inputs."""
    N, s = 2 ** 18, 32
    plan_a = gpu.Plan(N, s)
    plan_b = gpu.Plan(2 ** 16, 16, ident="phase")
    plans = [plan_a] * 6 + [plan_b] * 2
    sets = []
    for r in range(4):
        sets.append([dev(siggen.sparse_signal(p.N, p.s, seed=1000 * r + i, snr_db=25.0).f32)
                     for i, p in enumerate(plans)])
    bufs = [torch.empty_like(f) for f in sets[0]]
    batch = gpu.Batch(plans, bufs)
    st = torch.cuda.Stream()   # default priority
    for r in range(4):
        say("graph replay", r)
        for b, f in zip(bufs, sets[r]):
            b.copy_(f)
        torch.cuda.synchronize()
        ref_outs, ref_counts = gpu.execute_many(plans, sets[r])   # eager, on the current stream
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            outs, counts = batch.graph_launch(st)
        st.synchronize()
        _same(outs, counts, ref_outs, ref_counts)
        # eager work on other inputs between the replays
        gpu.execute_many(plans, sets[(r + 1) % 4])
        torch.cuda.synchronize()
    batch.close()


def test_graph_replay_of_split_launches(gpu):
    """A one-plan batch large enough for the moduli split of the matrix-core
    short DFTs (32 transforms at N = 2^22, s = 64: two launches), captured once
    and replayed on two input sets: every replay equals the plain calls (one
    short-DFT launch each) bit for bit."""
    N, s, B = 2 ** 22, 64, 32
    plan = gpu.Plan(N, s)
    assert plan.info["dft_split"] > 0
    sigs = [dev(siggen.workload("plain_n2e22_s64_20db", i).f32) for i in range(4)]
    bufs = [torch.empty_like(sigs[0]) for _ in range(B)]
    batch = gpu.Batch([plan] * B, bufs)
    st = torch.cuda.Stream()   # default priority
    for r in range(2):
        say("split graph replay", r)
        for i, b in enumerate(bufs):
            b.copy_(sigs[(i + r) % 4])
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            outs, counts = batch.graph_launch(st)
        st.synchronize()
        plain = []
        for f in sigs:
            w, c, n = plan.execute(f)
            torch.cuda.synchronize()
            plain.append((w.clone(), c.clone(), int(n.item())))
        for i in range(B):
            w, c, n = plain[(i + r) % 4]
            assert int(counts[i].item()) == n, i
            assert torch.equal(outs[i][0], w) and torch.equal(outs[i][1], c), i
    batch.close()
