"""Pins of the oracle's phase-shift identification (CPU only).

The shifted samples are checked against the convolution theorem and against
the time-shift identity; the phase-to-frequency step against worked examples
(worked by hand below, wrap-around and tie included) and against an exactly
1-sparse input, whose bins carry exp(2 pi i w / N) in closed form; the whole
transform against exact support recovery on exactly sparse inputs, against
the residue identification (same bins, same median: the same output where
both find the support) and against Theorem 5's bound on the dense DFT."""
import math

import numpy as np
import pytest

import oracle
import siggen
import tests.test_oracle_pins as pins
from oracle import IDENT_PHASE, Params, make_plan, PRESET_THEORY


def _phase_plan(N, s, **kw):
    return make_plan(N, s, Params(ident=IDENT_PHASE, **kw))


def _ghat(c1, n):
    """Lemma 2, written out."""
    return math.exp(-c1 * c1 * n * n / 2.0) / math.sqrt(2.0 * math.pi)


# ----------------------------------------------------- shifted samples ----

@pytest.mark.parametrize("N,s", [(4096, 6), (3001, 5)])
def test_shifted_samples_closed_form(N, s):
    """(g~_q * f)(theta + 2 pi / N) = sum_n c_n ghat_{n - q} exp(i n (theta + 2 pi / N))
    (convolution theorem, modulation shift), up to the window's truncation."""
    sig = siggen.sparse_signal(N, s, seed=5)
    plan = _phase_plan(N, s)
    tol = pins.gaussian_tail(plan, np.max(np.abs(sig.f)))
    for b in (0, plan.Q // 2, plan.Q - 1):
        for j in (0, plan.K - 1):
            P = plan.P[j]
            theta = 2 * math.pi * np.arange(P) / P + 2 * math.pi / N
            ref = np.zeros(P, dtype=complex)
            for w, c in zip(sig.freqs, sig.coefs):
                for m in (-1, 0, 1):
                    n = int(w) + m * N
                    ref += c * _ghat(plan.c1, n - plan.q[b]) * np.exp(1j * n * theta)
            S2 = oracle.filtered_samples(plan, sig.f, b, j, shift=1)
            assert np.max(np.abs(S2 - ref)) <= tol, (b, j)


def test_shift_is_the_time_shift_of_f():
    """Moving every node one grid step equals sampling f[n + 1] at the old nodes."""
    sig = siggen.sparse_signal(2000, 7, seed=2, snr_db=10.0)
    plan = _phase_plan(2000, 7)
    for b in (0, plan.Q - 1):
        for j in range(plan.K):
            a = oracle.filtered_samples(plan, sig.f, b, j, shift=1)
            r = oracle.filtered_samples(plan, np.roll(sig.f, -1), b, j)
            assert np.array_equal(a, r)


# ------------------------------------------------------ phase -> w --------

class _Tiny:
    """Just the fields phase_frequency reads."""

    def __init__(self, N, P):
        self.N = N
        self.P = (P,)
        self.band_lo = -((N + 1) // 2) + 1
        self.band_hi = N // 2


@pytest.mark.parametrize("N,P,h,angle_turns,expected", [
    # N = 100, B = -49..50.  Class 5 mod 12: -43, -31, -19, -7, 5, 17, 29, 41.
    (100, 12, 5, 0.29, 29),        # x = 29 is a member
    (100, 12, 5, 0.31, 29),        # x = 31: 29 is 2 away, 41 is 10
    (100, 12, 5, 0.499, -43),      # x = 49.9: 41 is 8.9 away, -43 is 7.1 away round the circle
    (100, 12, 5, -0.499, -43),     # x = -49.9
    # class 21 mod 8 in B: ..., 13, 21, 29, ...; x = 25 exactly (angle pi/2) is
    # 4 from 21 and from 29: the tie goes to the smaller frequency
    (100, 8, 21, 0.25, 21),
    # N = 10, B = -4..5, class 10 mod 24: 10 and -14 are both outside B
    (10, 24, 10, 0.1, None),
])
def test_phase_frequency_worked_examples(N, P, h, angle_turns, expected):
    plan = _Tiny(N, P)
    e = 2.0 + 0j
    e2 = e * (np.exp(2j * math.pi * angle_turns) if angle_turns != 0.25 else 1j)
    assert oracle.phase_frequency(plan, 0, h, e, e2) == expected


@pytest.mark.parametrize("N,s", [(2 ** 14, 8), (10_007, 4), (3001, 3)])
def test_one_sparse_bins_carry_the_frequency(N, s):
    """A single frequency w: every bin h = w mod P_j has E'[h] / E[h] =
    exp(2 pi i w / N) (up to the filter error) and phase_frequency returns w,
    also at the two ends of B."""
    lo, hi = siggen.band_limits(N)
    plan = _phase_plan(N, s)
    for w in (lo, lo + 1, -1, 0, 1, hi - 1, hi, 1234 % hi):
        f = np.exp(2j * math.pi * w * np.arange(N) / N)
        b = min(range(plan.Q), key=lambda bb: abs(plan.q[bb] - w))
        for j in range(plan.K):
            E = oracle.short_dft(oracle.filtered_samples(plan, f, b, j))
            E2 = oracle.short_dft(oracle.filtered_samples(plan, f, b, j, shift=1))
            h = w % plan.P[j]
            ratio = E2[h] / E[h]
            assert abs(ratio - np.exp(2j * math.pi * w / N)) < 1e-6, (w, j)
            assert oracle.phase_frequency(plan, j, h, E[h], E2[h]) == w


def test_phase_frequency_equals_rounding_formula():
    """Brute force over the residue class (the oracle) against the closed
    form: nearest member of h + P Z to x, x - N and x + N, kept if in B."""
    rng = np.random.Generator(np.random.PCG64(11))
    for N, P in [(100, 12), (1000, 37 * 8), (2 ** 14, 16 * 41), (997, 24), (50, 64)]:
        plan = _Tiny(N, P)
        for _ in range(300):
            h = int(rng.integers(0, P))
            ang = float(rng.uniform(-math.pi, math.pi))
            x = ang * N / (2 * math.pi)
            best = None
            for xs in (x - N, x, x + N):
                m0 = math.floor((xs - h) / P + 0.5)
                for m in (m0 - 1, m0, m0 + 1):
                    w = h + m * P
                    if plan.band_lo <= w <= plan.band_hi:
                        key = (abs(w - xs), w)
                        if best is None or key < best:
                            best = key
            want = None if best is None else best[1]
            got = oracle.phase_frequency(plan, 0, h, 1.0 + 0j, complex(np.exp(1j * ang)))
            assert got == want, (N, P, h, ang)


# ---------------------------------------------------------- end to end ----

def test_phase_exact_support_plain_n2e14_s8():
    plan = _phase_plan(2 ** 14, 8)
    for seed in range(30):
        sig = siggen.workload("plain_n2e14_s8", seed)
        fr, co = oracle.sft(plan, sig.f)
        truth = dict(zip((int(w) for w in sig.freqs), sig.coefs))
        assert set(fr.tolist()) == set(truth), seed
        assert max(abs(c - truth[int(w)]) for w, c in zip(fr, co)) < 1e-4


@pytest.mark.parametrize("N,s,snr", [(2 ** 14, 8, None), (100_003, 20, 40.0), (3001, 5, 30.0)])
def test_phase_and_residue_identification_agree(N, s, snr):
    """Both identifications read the same bins and take the same median: where
    both recover the support, the outputs are equal."""
    for seed in range(3):
        sig = siggen.sparse_signal(N, s, seed=seed, snr_db=snr)
        f1, c1 = oracle.sft(make_plan(N, s), sig.f)
        f2, c2 = oracle.sft(_phase_plan(N, s), sig.f)
        assert set(f1.tolist()) == set(f2.tolist()) == set(int(w) for w in sig.freqs)
        assert np.array_equal(f1, f2) and np.array_equal(c1, c2)


def test_phase_vote_uses_all_moduli():
    """A candidate needs heavy bins in more than half of all K moduli: the
    producing modulus counts too."""
    sig = siggen.sparse_signal(4096, 6, seed=9, snr_db=20.0)
    plan = _phase_plan(4096, 6)
    _, _, infos = oracle.sft_trace(plan, sig.f, bands=[0, plan.Q // 2])
    for info in infos.values():
        hs = [set(int(h) for h in H) for H in info["heavy"]]
        acc = {w for w, _ in info["accepted"]}
        for w in info["candidates"]:
            votes = sum((w % plan.P[j]) in hs[j] for j in range(plan.K))
            assert (w in acc) == (2 * votes > plan.K)


@pytest.mark.parametrize("N,s,snr", [(1024, 4, 40.0), (4096, 6, 50.0)])
def test_phase_theorem5_bound_against_dense_dft(N, s, snr):
    """Theorem 5's bound with the theory preset's filter; the phase step is
    the identification being bounded (the paper proves the bound for its
    deterministic inner algorithm; here it is checked empirically)."""
    plan = make_plan(N, s, Params(preset=PRESET_THEORY, r=1.0, ident=IDENT_PHASE))
    lo = siggen.band_limits(N)[0]
    for seed in range(3):
        sig = siggen.sparse_signal(N, s, seed=200 + seed, snr_db=snr)
        fr, co = oracle.sft(plan, sig.f)
        c = np.fft.fft(sig.f) / N
        w = np.arange(lo, lo + N)
        c = c[np.mod(w, N)]
        v = np.zeros_like(c)
        v[fr - lo] = co
        order = np.lexsort((w, -np.abs(c)))
        tail = np.ones(N, bool)
        tail[order[:s]] = False
        bound = (np.linalg.norm(c[tail]) + 33 / math.sqrt(s) * np.sum(np.abs(c[tail]))
                 + 198 * math.sqrt(s) * np.max(np.abs(sig.f)) / N)
        assert np.linalg.norm(c - v) <= bound
