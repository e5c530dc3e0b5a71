"""End-to-end checks of the oracle: exact support recovery on exactly sparse
inputs, Theorem 5's error bound against the dense DFT on small N, metamorphic
relations (frequency shift, time shift, linearity), band-edge frequencies, and
the inner algorithm's candidate and vote steps against brute force."""
import math

import numpy as np
import pytest

import oracle
import siggen
from oracle import Params, make_plan, PRESET_THEORY


def _truth(sig):
    return dict(zip((int(w) for w in sig.freqs), sig.coefs))


def test_exact_support_plain_n2e14_s8_100_seeds():
    """The plain workload (N = 2^14, s = 8, noiseless): the paper's acceptance
    bar is >= 0.9 exact-support probability per trial (Section 5.1); the CRT-vote
    inner algorithm recovers every one of 100 seeds, each coefficient within
    the filter error divided by tau (the bound after Lemma 13)."""
    plan = make_plan(2 ** 14, 8)
    worst = 0.0
    for seed in range(100):
        sig = siggen.workload("plain_n2e14_s8", seed)
        fr, co = oracle.sft(plan, sig.f)
        truth = _truth(sig)
        assert set(fr.tolist()) == set(truth), seed
        worst = max(worst, max(abs(c - truth[int(w)]) for w, c in zip(fr, co)))
    assert worst < 1e-4


def test_exact_support_theory_and_dmsft4():
    for preset in (PRESET_THEORY, 1):
        plan = make_plan(2 ** 14, 8, Params(preset=preset))
        for seed in range(5):
            sig = siggen.workload("plain_n2e14_s8", seed)
            fr, co = oracle.sft(plan, sig.f)
            assert set(fr.tolist()) == set(_truth(sig))


def test_output_order_and_no_duplicates():
    sig = siggen.sparse_signal(5000, 20, seed=7, snr_db=30)
    plan = make_plan(sig.N, sig.s)
    fr, co = oracle.sft(plan, sig.f)
    assert len(set(fr.tolist())) == len(fr) <= sig.s
    keys = [(-abs(c), int(w)) for w, c in zip(fr, co)]
    assert keys == sorted(keys)
    lo, hi = siggen.band_limits(sig.N)
    assert all(lo <= w <= hi for w in fr)


def _dense_truth(f):
    N = f.shape[0]
    c = np.fft.fft(f) / N
    lo, hi = siggen.band_limits(N)
    w = np.arange(lo, hi + 1)
    return w, c[np.mod(w, N)]


@pytest.mark.parametrize("N,s,snr", [(1024, 4, 20.0), (2048, 8, 10.0), (4096, 6, 30.0), (3001, 5, 15.0)])
def test_theorem5_bound_against_dense_dft(N, s, snr):
    """Theorem 5: ||c - v||_2 <= ||c - c_s^opt||_2 + 33/sqrt(s) ||c - c_s^opt||_1
    + 198 sqrt(s) ||f||_inf N^-r with c the dense DFT of the (noisy) input."""
    plan = make_plan(N, s, Params(preset=PRESET_THEORY, r=1.0))
    for seed in range(3):
        sig = siggen.sparse_signal(N, s, seed=100 + seed, snr_db=snr)
        fr, co = oracle.sft(plan, sig.f)
        w, c = _dense_truth(sig.f)
        v = np.zeros_like(c)
        lo = siggen.band_limits(N)[0]
        v[fr - lo] = co
        order = np.lexsort((w, -np.abs(c)))
        tail = np.ones(N, bool)
        tail[order[:s]] = False
        bound = (np.linalg.norm(c[tail]) + 33 / math.sqrt(s) * np.sum(np.abs(c[tail]))
                 + 198 * math.sqrt(s) * np.max(np.abs(sig.f)) * N ** -1.0)
        assert np.linalg.norm(c - v) <= bound


def test_frequency_shift_moves_support():
    sig = siggen.sparse_signal(2 ** 14, 8, seed=21)
    plan = make_plan(sig.N, sig.s)
    fr0, co0 = oracle.sft(plan, sig.f)
    lo, hi = siggen.band_limits(sig.N)
    j = np.arange(sig.N)
    for delta in (1, 137, -4000, 8191):
        g = sig.f * np.exp(2j * math.pi * delta * j / sig.N)
        fr, co = oracle.sft(plan, g)
        shifted = {((int(w) + delta - lo) % sig.N) + lo: c for w, c in zip(fr0, co0)}
        assert set(fr.tolist()) == set(shifted)
        for w, c in zip(fr, co):
            assert abs(c - shifted[int(w)]) < 2e-4


def test_time_shift_rotates_coefficients():
    sig = siggen.sparse_signal(2 ** 14, 8, seed=22)
    plan = make_plan(sig.N, sig.s)
    fr0, co0 = oracle.sft(plan, sig.f)
    for m in (1, 1000, -77):
        g = np.roll(sig.f, m)                       # g_j = f_{j - m}
        fr, co = oracle.sft(plan, g)
        assert set(fr.tolist()) == set(fr0.tolist())
        ref = {int(w): c * np.exp(-2j * math.pi * int(w) * m / sig.N) for w, c in zip(fr0, co0)}
        for w, c in zip(fr, co):
            assert abs(c - ref[int(w)]) < 2e-4


def test_linearity_disjoint_supports():
    a = siggen.sparse_signal(2 ** 14, 4, seed=31)
    b = siggen.sparse_signal(2 ** 14, 4, seed=32)
    assert not set(a.freqs.tolist()) & set(b.freqs.tolist())
    plan = make_plan(a.N, 8)
    fr, co = oracle.sft(plan, a.f + 2 * b.f)
    ref = {**{int(w): c for w, c in zip(a.freqs, a.coefs)},
           **{int(w): 2 * c for w, c in zip(b.freqs, b.coefs)}}
    assert set(fr.tolist()) == set(ref)
    for w, c in zip(fr, co):
        assert abs(c - ref[int(w)]) < 2e-4


def test_band_edge_frequencies():
    """Frequencies on the edges of the bands [q_b - L, q_b + L) and of B are
    found exactly once (Algorithm 1's band test, with B's convention)."""
    N = 2 ** 14
    plan = make_plan(N, 12)
    lo, hi = siggen.band_limits(N)
    freqs = [lo, hi, plan.q[3] - plan.L, plan.q[3] + plan.L - 1, plan.q[8] + plan.L,
             plan.q[0], plan.q[-1] - plan.L, plan.q[-1] - plan.L - 1, 0, 1, -1, plan.q[5] + plan.L - 1]
    freqs = np.array(sorted(set(freqs))[:12], dtype=np.int64)
    rng = np.random.default_rng(4)
    coefs = np.exp(2j * math.pi * rng.random(len(freqs)))
    f = siggen.synthesize(N, freqs, coefs)
    fr, co = oracle.sft(make_plan(N, len(freqs)), f)
    assert sorted(fr.tolist()) == sorted(freqs.tolist())
    ref = dict(zip(freqs.tolist(), coefs))
    for w, c in zip(fr, co):
        assert abs(c - ref[int(w)]) < 1e-4


def test_candidates_equal_bruteforce_definition():
    """A candidate is exactly a w in B whose residue bin, in every modulus of some
    CRT tuple, is heavy and among the class_depth(G) heaviest of its residue
    class mod s1 (brute force over all of B); the vote, R_temp and band test
    follow their definitions."""
    sig = siggen.sparse_signal(2 ** 14, 8, seed=41, snr_db=10)
    plan = make_plan(sig.N, sig.s)
    lo, hi = plan.band_lo, plan.band_hi
    w_all = np.arange(lo, hi + 1)
    depth = oracle.class_depth(plan.G)
    _, _, infos = oracle.sft_trace(plan, sig.f, bands={0, 6, 15})
    for b, info in infos.items():
        heavy_sets = [set(int(h) for h in H) for H in info["heavy"]]
        kept = []
        for j in range(plan.K):
            m2 = np.abs(info["E"][j]) ** 2
            top = set()
            for a in range(plan.s1):
                cls = [h for h in heavy_sets[j] if h % plan.s1 == a]
                cls.sort(key=lambda h: (-m2[h], h))
                top |= set(cls[:depth])
            kept.append(np.array(sorted(top)))
        brute = {}
        for t, tup in enumerate(plan.tuples):
            ok = np.ones(w_all.shape, bool)
            for j in tup:
                ok &= np.isin(np.mod(w_all, plan.P[j]), kept[j])
            for w in w_all[ok].tolist():
                brute.setdefault(w, set()).add(t)
        assert brute == info["candidates"]
        # vote: accepted iff, for a producing tuple, more than half of the K - G
        # other moduli have a heavy bin at w
        acc = {w for w, _ in info["accepted"]}
        for w, tups in info["candidates"].items():
            ok = False
            for t in tups:
                others = [j for j in range(plan.K) if j not in plan.tuples[t]]
                votes = sum((w % plan.P[j]) in heavy_sets[j] for j in others)
                ok |= votes > len(others) / 2
            assert (w in acc) == ok
        # R_temp is the s largest |z| (ties to the smaller w); kept = R_temp inside the band
        ranked = sorted(info["accepted"], key=lambda wz: (-abs(wz[1]), wz[0]))[: plan.s]
        assert ranked == info["r_temp"]
        q = plan.q[b]
        assert [w for w, _ in info["kept"]] == [w for w, _ in ranked if q - plan.L <= w < q + plan.L and lo <= w <= hi]


def test_ghost_combinations_are_rejected():
    """Two strong frequencies in one residue class mod s1 give CRT combinations
    that mix their bins across a tuple's moduli.  Such a ghost has heavy bins in
    its own tuple by construction; the vote over the other moduli rejects it,
    so weak true frequencies are not displaced (log-uniform magnitudes, 40 dB)."""
    plan = make_plan(1_000_003, 64)
    sig = siggen.sparse_signal(1_000_003, 64, seed=0, snr_db=40.0, magnitude="loguniform")
    fr, co = oracle.sft(plan, sig.f32)
    assert set(fr.tolist()) == set(sig.freqs.tolist())


def test_class_depth():
    assert [oracle.class_depth(G) for G in (1, 2, 3, 4, 5, 6)] == [64, 8, 4, 2, 2, 2]
