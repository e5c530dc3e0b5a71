"""GPU parity of the phase-shift identification against the FP64 oracle
(same seeded complex64 inputs, through the C ABI), with the tolerances of
test_gpu_parity: the shifted samples and bins are checked like the unshifted
ones, supports bit-equal, coefficients rel-l2 <= 1e-3."""
import numpy as np
import pytest

import oracle
import siggen
from tests.test_gpu_parity import (BIN_TOL, SAMPLE_TOL, assert_same_result, dev, gpu_run, say)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _oplan(N, s, kw):
    return oracle.make_plan(N, s, oracle.Params(ident=1, **{k: v for k, v in kw.items() if k != "dft_path"}))


CASES = [
    ("plain_n2e14_s8", 2 ** 14, 8, None, {}, 0),
    ("prime_n100003_s20_30db", 100_003, 20, 30.0, {}, 1),
    ("mx_n2e16_s40_10db", 2 ** 16, 40, 10.0, {"dft_path": 3}, 6),
    ("valu_n2e16_s40_10db", 2 ** 16, 40, 10.0, {"dft_path": 1}, 6),
    ("split_prime_n100003_s20_30db", 100_003, 20, 30.0, {"dft_path": 2}, 1),
    ("splitmx_n2e16_s40_10db", 2 ** 16, 40, 10.0, {"dft_path": 4}, 6),
    ("kappa12_n3001_s5_40db", 3001, 5, 40.0, {"kappa": 12}, 2),
    ("n31_s1", 31, 1, None, {}, 4),
]


@pytest.mark.parametrize("name,N,s,snr,kw,seed", CASES, ids=[c[0] for c in CASES])
def test_phase_intermediates_match_oracle(gpu, name, N, s, snr, kw, seed):
    say("phase case", name)
    sig = siggen.sparse_signal(N, s, seed=seed, snr_db=snr)
    f32 = sig.f32
    plan = gpu.Plan(N, s, ident="phase", **kw)
    op = _oplan(N, s, kw)
    wg, cg = gpu_run(plan, f32)
    got = {k: plan.fetch(k) for k in (gpu.FETCH_SAMPLES, gpu.FETCH_BINS, gpu.FETCH_SAMPLES_SHIFTED,
                                      gpu.FETCH_BINS_SHIFTED)}
    in_scale = float(np.max(np.abs(f32))) / np.sqrt(2 * np.pi)
    for b in range(op.Q):
        for j in range(op.K):
            for shift, ks, kb in ((0, gpu.FETCH_SAMPLES, gpu.FETCH_BINS),
                                  (1, gpu.FETCH_SAMPLES_SHIFTED, gpu.FETCH_BINS_SHIFTED)):
                So = oracle.filtered_samples(op, f32, b, j, shift=shift)
                Sg = gpu.samples_natural(plan, got[ks], b, j)
                scale = max(np.max(np.abs(So)), in_scale, 1e-30)
                assert np.max(np.abs(Sg - So)) <= SAMPLE_TOL * scale, (shift, b, j)
                Eo = oracle.short_dft(So)
                Eg = gpu.bins_natural(plan, got[kb], b, j)
                escale = max(np.max(np.abs(Eo)), scale)
                assert np.max(np.abs(Eg - Eo)) <= BIN_TOL * escale, (shift, b, j)
    wo, co = oracle.sft(op, f32)
    assert_same_result(wg, cg, wo, co)
    if snr is None or snr >= 30:
        assert set(wg.tolist()) == set(sig.freqs.tolist())


@pytest.mark.parametrize("snr", [20.0, 40.0])
def test_phase_headline_n2e22_s64(gpu, snr):
    """The headline shape with phase identification: plain path against the
    oracle, batched path equal to the plain path bit for bit (a batch of 16,
    whose short DFTs run as the two launches of the moduli split, while a
    single transform's run as one)."""
    N, s, B = 2 ** 22, 64, 16
    plan = gpu.Plan(N, s, ident="phase")
    assert plan.info["dft_split"] > 0
    op = _oplan(N, s, {})
    sigs = [siggen.sparse_signal(N, s, seed=seed, snr_db=snr) for seed in (0, 1)]
    fs = [dev(sg.f32) for sg in sigs]
    outs, counts = gpu.execute_many([plan] * B, [fs[i % 2] for i in range(B)])
    torch.cuda.synchronize()
    for seed, sg in enumerate(sigs):
        say("phase headline", snr, "dB seed", seed)
        wg, cg = gpu_run(plan, sg.f32)
        wo, co = oracle.sft(op, sg.f32)
        assert_same_result(wg, cg, wo, co)
        assert set(wo.tolist()) == set(sg.freqs.tolist())
        for i in range(seed, B, 2):
            k = int(counts[i].item())
            assert np.array_equal(outs[i][0].cpu().numpy()[:k], wg)
            assert np.array_equal(outs[i][1].cpu().numpy()[:k], cg)


def test_phase_split_path_equals_in_lds_path(gpu):
    """Split and in-LDS VALU short DFTs agree bit for bit on both sample sets."""
    N, s = 100_003, 20
    sg = siggen.sparse_signal(N, s, seed=13, snr_db=20.0)
    f = dev(sg.f32)
    res = []
    for path in (1, 2):
        say("phase split vs lds", path)
        plan = gpu.Plan(N, s, dft_path=path, ident="phase")
        w, c, n = plan.execute(f)
        torch.cuda.synchronize()
        res.append((w.cpu().numpy(), c.cpu().numpy(), plan.fetch(gpu.FETCH_BINS),
                    plan.fetch(gpu.FETCH_BINS_SHIFTED), plan.fetch(gpu.FETCH_HEAVY)))
    for x, y in zip(res[0], res[1]):
        assert np.array_equal(x, y)


def test_batched_phase_and_residue_plans_equal_plain(gpu):
    """One execute_many holding phase and residue plans of different shapes
    (the identify kernel then takes the identification per transform) equals
    the single calls bit for bit."""
    shapes = [(2 ** 14, 8, 1), (2 ** 14, 8, 0), (100_003, 20, 1), (2 ** 16, 40, 0), (2 ** 16, 40, 1),
              (31, 1, 1), (3 * 2 ** 15, 12, 0)]
    plans = {sh: gpu.Plan(sh[0], sh[1], ident=sh[2]) for sh in set(shapes)}
    sigs = [siggen.sparse_signal(N, s, seed=70 + i, snr_db=30.0) for i, (N, s, _) in enumerate(shapes)]
    fs = [dev(sg.f32) for sg in sigs]
    pl = [plans[sh] for sh in shapes]
    say("batched phase + residue", len(shapes))
    outs, counts = gpu.execute_many(pl, fs)
    torch.cuda.synchronize()
    for i, (p, f) in enumerate(zip(pl, fs)):
        w, c, n = p.execute(f)
        torch.cuda.synchronize()
        assert int(counts[i].item()) == int(n.item()), i
        assert np.array_equal(outs[i][0].cpu().numpy(), w.cpu().numpy()), i
        assert np.array_equal(outs[i][1].cpu().numpy(), c.cpu().numpy()), i


def test_phase_fetch_rejected_for_residue_plans(gpu):
    plan = gpu.Plan(2 ** 14, 8)
    with pytest.raises(gpu.SftError):          # no sft_execute has run: no workspace yet
        plan.fetch(gpu.FETCH_BINS)
    plan.execute(torch.from_numpy(siggen.sparse_signal(2 ** 14, 8, seed=1).f32).cuda())
    torch.cuda.synchronize()
    assert plan.fetch(gpu.FETCH_BINS).size == plan.info["Q"] * plan.info["M"]
    with pytest.raises(gpu.SftError):
        plan.fetch(gpu.FETCH_BINS_SHIFTED)
