"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own formula: each compares an oracle step
with a closed form (Lemma 2, the convolution theorem, the modulation shift of
Section 4), a brute-force computation (the untruncated sum of eq.
UntruncatedFiniteSum, direct DFT, exhaustive CRT, exact rational node
geometry), or an invariant (Parseval, band tiling, Lemma 3's passband).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import siggen
from oracle import Params, make_plan, PRESET_DMSFT4, PRESET_DMSFT6, PRESET_THEORY


def periodized_gaussian(x, c1, images=4):
    """g(x) = (1/c1) sum_n exp(-(x - 2 pi n)^2 / (2 c1^2)) (eq. Def_Periodic_Gaussian)."""
    tot = np.zeros_like(np.asarray(x, dtype=float))
    for n in range(-images, images + 1):
        tot = tot + np.exp(-((x - 2 * math.pi * n) ** 2) / (2 * c1 * c1))
    return tot / c1


def lemma2(c1, n):
    return np.exp(-(c1 ** 2) * np.asarray(n, float) ** 2 / 2) / math.sqrt(2 * math.pi)


def gaussian_tail(plan, fmax):
    """Bound on |truncated - untruncated sum|: fmax * sum_{|i| > kappa} W(u - i)
    over the worst u, from the n = 0 image (Lemma 10's setting)."""
    sig = plan.sigma_t
    tail = 0.0
    for m in range(0, 200):
        d = plan.kappa + 0.5 + m
        tail += math.exp(-d * d / (2 * sig * sig))
    return 2.0 * fmax * tail / (2 * math.pi * sig) * 1.0001 + 1e-14


# ---------------------------------------------------------------- Lemma 2 --

@pytest.mark.parametrize("N", [64, 100, 257])
def test_ghat_matches_numerical_fourier_coefficients(N):
    """Lemma 2: the Fourier coefficients of the periodized Gaussian, computed
    numerically from its definition on a fine grid, equal the closed form."""
    plan = make_plan(N, 2)
    grid = 8192
    x = -math.pi + 2 * math.pi * np.arange(grid) / grid
    g = periodized_gaussian(x, plan.c1)
    coef = np.fft.fft(g) / grid * np.exp(1j * np.arange(grid) * math.pi)  # shift origin to -pi
    for w in range(0, 60):
        num = coef[w].real
        assert abs(num - float(oracle.ghat(plan, w))) < 1e-12
        assert abs(coef[w].imag) < 1e-12
    # the maximum is 1/sqrt(2 pi) at w = 0 and it decreases with |w|
    assert abs(float(oracle.ghat(plan, 0)) - 1 / math.sqrt(2 * math.pi)) < 1e-15
    assert np.all(np.diff(oracle.ghat(plan, np.arange(50))) < 0)


@pytest.mark.parametrize("N,t", [(64, 3.3), (64, 63.7), (97, 48.5), (128, 0.25)])
def test_window_weight_is_g_over_N(N, t):
    """W(v) = g(2 pi v / N) / N: summed over ALL grid points against a pure tone
    it reproduces ghat_w exp(i w theta) up to aliasing (convolution theorem)."""
    plan = make_plan(N, 2)
    j = np.arange(N)
    v = t - j
    W = oracle.window_weight(plan, v)
    assert np.allclose(W, periodized_gaussian(2 * math.pi * v / N, plan.c1) / N, rtol=1e-13, atol=0)
    for w in (-N // 2 + 1, -5, 0, 1, 7, N // 2):
        lhs = np.sum(np.exp(2j * math.pi * w * j / N) * W)
        rhs = sum(lemma2(plan.c1, w + m * N) * np.exp(2j * math.pi * (w + m * N) * t / N)
                  for m in range(-3, 4))
        assert abs(lhs - rhs) < 1e-13


# ------------------------------------------------------- node geometry ----

@pytest.mark.parametrize("N,s", [(2 ** 14, 8), (10_000_019, 128), (1000, 5), (97, 3)])
def test_node_geometry_exact_rationals(N, s):
    plan = make_plan(N, s)
    rng = np.random.default_rng(0)
    for j in range(plan.K):
        P = plan.P[j]
        jp, delta = oracle.node_geometry(plan, j)
        ks = list(range(min(P, 50))) + list(rng.integers(0, P, 200)) + [P - 1]
        for k in ks:
            t = Fraction(k * N, P)
            nearest = math.floor(t + Fraction(1, 2))     # ties rounded up
            assert jp[k] == nearest
            assert Fraction(int(delta[k]), P) == t - nearest
            assert -Fraction(1, 2) <= t - nearest < Fraction(1, 2)


# ------------------------------------------------- filtered samples -------

def _expected_samples(plan, sig, b, j, periodic=True):
    """Convolution theorem + modulation shift: for the discrete (untruncated)
    sum the coefficient of exp(i n theta) is c_{n mod N} * ghat_{n - q_b} for every
    integer n; for the continuous g~_q * f only n in B survive."""
    P = plan.P[j]
    theta = 2 * math.pi * np.arange(P) / P
    q = plan.q[b]
    out = np.zeros(P, dtype=complex)
    ms = (-1, 0, 1) if periodic else (0,)
    for w, c in zip(sig.freqs, sig.coefs):
        for m in ms:
            n = int(w) + m * plan.N
            out += c * lemma2(plan.c1, n - q) * np.exp(1j * n * theta)
    return out


@pytest.mark.parametrize("preset", [PRESET_DMSFT6, PRESET_DMSFT4, PRESET_THEORY])
def test_filtered_samples_closed_form(preset):
    sig = siggen.sparse_signal(4096, 6, seed=3)
    plan = make_plan(sig.N, sig.s, Params(preset=preset))
    fmax = np.max(np.abs(sig.f))
    tol = gaussian_tail(plan, fmax)
    for b in (0, plan.Q // 2, plan.Q - 1):
        for j in (0, plan.K - 1):
            S = oracle.filtered_samples(plan, sig.f, b, j)
            ref = _expected_samples(plan, sig, b, j, periodic=True)
            assert np.max(np.abs(S - ref)) <= tol, (b, j, np.max(np.abs(S - ref)), tol)


def test_filtered_samples_theorem4_bound():
    """Theorem 4 (p = infinity): |(g * f)(x) - truncated sum| <= 3 ||f||_inf N^-r,
    for the unmodulated filter of the theory preset."""
    for r in (1.0, 2.0):
        sig = siggen.sparse_signal(2048, 5, seed=11)
        plan = make_plan(sig.N, sig.s, Params(preset=PRESET_THEORY, r=r))
        import dataclasses
        plan0 = dataclasses.replace(plan, q=(0,), Q=1)
        bound = 3 * np.max(np.abs(sig.f)) * sig.N ** (-r)
        for j in range(plan.K):
            S = oracle.filtered_samples(plan0, sig.f, 0, j)
            ref = _expected_samples(plan0, sig, 0, j, periodic=False)
            assert np.max(np.abs(S - ref)) <= bound


def test_truncated_vs_untruncated_sum():
    """Lemma 10: the 2 kappa + 1 nearest terms of eq. UntruncatedFiniteSum
    versus all N terms (brute force), for random (dense) f."""
    rng = np.random.default_rng(5)
    for N in (64, 500, 4096):
        f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        plan = make_plan(N, 3)
        j_all = np.arange(N)
        for b in (0, plan.Q - 1):
            q = plan.q[b]
            for j in (0, plan.K - 1):
                P = plan.P[j]
                S = oracle.filtered_samples(plan, f, b, j)
                ks = rng.integers(0, P, 40)
                for k in ks:
                    t = k * N / P
                    v = t - j_all
                    v = v - N * np.round(v / N)          # nearest image, |v| <= N/2
                    full = np.sum(f * oracle.window_weight(plan, v) * np.exp(2j * math.pi * q * v / N))
                    assert abs(full - S[k]) <= gaussian_tail(plan, np.max(np.abs(f)))


def test_window_extent_with_a_unit_impulse():
    """f = e_{j0}: a node sees the impulse iff j0 is among its 2 kappa + 1 nearest
    grid points (indices mod N), and then S = W(t - j0) exp(2 pi i q (t - j0)/N).
    The impulse is swept over enough positions that every tap offset occurs."""
    N = 1000
    plan = make_plan(N, 4)
    b = 2
    q = plan.q[b]
    seen_offsets = set()
    for j0 in list(range(0, 12)) + [N - 1, N - 3]:
        f = np.zeros(N, dtype=complex)
        f[j0] = 1.0
        for j in range(plan.K):
            P = plan.P[j]
            S = oracle.filtered_samples(plan, f, b, j)
            for k in range(P):
                t = Fraction(k * N, P)
                jn = math.floor(t + Fraction(1, 2))
                hits = [i for i in range(-plan.kappa, plan.kappa + 1) if (jn + i) % N == j0]
                if hits:
                    seen_offsets.add(hits[0])
                    v = float(t - (jn + hits[0]))
                    ref = float(periodized_gaussian(2 * math.pi * v / N, plan.c1)) / N * np.exp(2j * math.pi * q * v / N)
                    assert abs(S[k] - ref) < 1e-15 + 1e-13 * abs(ref)
                else:
                    assert S[k] == 0
    assert seen_offsets == set(range(-plan.kappa, plan.kappa + 1))


# ---------------------------------------------------------- short DFTs ----

def test_short_dft_direct_and_parseval():
    rng = np.random.default_rng(1)
    for P in (37 * 4, 41 * 16, 53 * 8, 1, 2):
        S = rng.standard_normal(P) + 1j * rng.standard_normal(P)
        E = oracle.short_dft(S)
        k = np.arange(P)
        for h in range(P):
            direct = np.sum(S * np.exp(-2j * math.pi * k * h / P)) / P
            assert abs(E[h] - direct) < 1e-12
        assert abs(np.sum(np.abs(E) ** 2) - np.sum(np.abs(S) ** 2) / P) < 1e-10


def test_dft_bins_aliasing_identity():
    """For an s-sparse f, E_b[j][h] = sum over n = h (mod P_j) of c_{n mod N} ghat_{n - q_b},
    up to the window-truncation error."""
    sig = siggen.sparse_signal(2 ** 14, 8, seed=4)
    plan = make_plan(sig.N, sig.s)
    tol = gaussian_tail(plan, np.max(np.abs(sig.f)))
    for b in (0, 7, plan.Q - 1):
        for j in range(plan.K):
            P = plan.P[j]
            E = oracle.short_dft(oracle.filtered_samples(plan, sig.f, b, j))
            ref = np.zeros(P, dtype=complex)
            for w, c in zip(sig.freqs, sig.coefs):
                for m in (-1, 0, 1):
                    n = int(w) + m * plan.N
                    ref[n % P] += c * lemma2(plan.c1, n - plan.q[b])
            assert np.max(np.abs(E - ref)) <= tol


# ------------------------------------------------------- heavy bins -------

def test_heavy_bins_ties_go_to_lower_index():
    E = np.array([1, 3, 3, 2, 3, 0, 2, 1j * 3, -3, 2], dtype=complex)
    for T in range(0, 11):
        ranked = sorted(range(len(E)), key=lambda h: (-(abs(E[h]) ** 2), h))
        assert list(oracle.heavy_bins(E, T)) == sorted(ranked[:T])
    rng = np.random.default_rng(2)
    for _ in range(50):
        E = rng.integers(-2, 3, 60) + 1j * rng.integers(-2, 3, 60)
        T = int(rng.integers(0, 60))
        ranked = sorted(range(60), key=lambda h: (-(abs(E[h]) ** 2), h))
        assert list(oracle.heavy_bins(E, T)) == sorted(ranked[:T])


# ------------------------------------------------------------- CRT --------

def test_crt_bruteforce():
    rng = np.random.default_rng(3)
    for moduli in ([4, 3, 5], [8, 37, 41], [16, 3, 7, 11], [2, 9, 25, 7]):
        M = int(np.prod(moduli))
        for _ in range(60):
            x = int(rng.integers(0, M))
            res = [x % m for m in moduli]
            assert oracle.crt(res, moduli) == x
        # exhaustive for the smallest
    moduli = [4, 3, 5]
    for x in range(60):
        assert oracle.crt([x % m for m in moduli], moduli) == x


def test_representative_in_band_bruteforce():
    for N in (7, 8, 9, 16):
        lo, hi = siggen.band_limits(N)
        for M in (N, N + 1, N + 5, 2 * N + 3):
            for r in range(M):
                reps = [w for w in range(lo, hi + 1) if (w - r) % M == 0]
                got = oracle.representative_in_band(r, M, N)
                assert (got is None and not reps) or [got] == reps


# ----------------------------------------------------------- median -------

def test_median_estimate_componentwise():
    plan = make_plan(2 ** 14, 8)
    rng = np.random.default_rng(9)
    E = [rng.standard_normal(P) + 1j * rng.standard_normal(P) for P in plan.P]
    for w in (-5, 0, 77, plan.band_hi, plan.band_lo):
        re = sorted(E[j][w % plan.P[j]].real for j in range(plan.K))
        im = sorted(E[j][w % plan.P[j]].imag for j in range(plan.K))
        z = oracle.median_estimate(plan, E, w)
        assert z == complex(re[plan.K // 2], im[plan.K // 2])
    # a single huge outlier bin does not move the median
    E2 = [np.full(P, 1 + 1j) for P in plan.P]
    E2[0][5 % plan.P[0]] = 1e6
    assert oracle.median_estimate(plan, E2, 5) == 1 + 1j


# ------------------------------------------------------ plan rules --------

def test_plan_values_headline_and_theory():
    p = make_plan(2 ** 22, 64)
    assert (p.kappa, p.Q, p.L, p.s1, p.G, p.K) == (6, 16, 139_100, 128, 3, 7)
    assert p.primes == (37, 41, 43, 47, 53, 59, 61)
    assert sum(p.P) == 43_648 and p.T == 128
    p1 = make_plan(2 ** 14, 8)
    assert p1.primes == (37, 41, 43, 47, 53) and p1.L == 544 and p1.s1 == 16
    th = make_plan(2 ** 22, 64, Params(preset=PRESET_THEORY))
    assert th.kappa == 22 and th.beta == 6.0
    # the corrected form of the alpha condition (after Lemma 13): 6 sqrt(2r) / sqrt(ln(1/(tau sqrt(2 pi))))
    assert abs(th.alpha - 6 * math.sqrt(2) / math.sqrt(math.log(3 / math.sqrt(2 * math.pi)))) < 1e-9
    assert abs(th.alpha - 20.02) < 0.01
    d4 = make_plan(2 ** 20, 50, Params(preset=PRESET_DMSFT4))
    assert d4.kappa == 4


@pytest.mark.parametrize("N,s,preset", [(2 ** 14, 8, 0), (2 ** 22, 64, 0), (10_000_019, 128, 0),
                                        (5 * 2 ** 19 + 1, 200, 0), (2 ** 26, 1024, 0), (4096, 3, 2),
                                        (2 ** 22, 50, 1), (31, 1, 0), (31, 31, 0)])
def test_plan_invariants(N, s, preset):
    p = make_plan(N, s, Params(preset=preset))
    # Lemma 3: the passband |w| <= L keeps ghat >= tau
    assert float(oracle.ghat(p, p.L)) >= p.tau
    # bands [q_b - L, q_b + L) are disjoint and cover B (Algorithm 1's band centres and band test)
    edges = [(q - p.L, q + p.L) for q in p.q]
    assert edges[0][0] == p.band_lo
    for a, b in zip(edges, edges[1:]):
        assert a[1] == b[0]
    assert edges[-1][1] > p.band_hi
    # moduli: s1 a power of two >= 2s, odd primes, each tuple's product >= N
    assert p.s1 >= 2 * s and p.s1 & (p.s1 - 1) == 0
    assert len(set(p.primes)) == p.K == 2 * p.G + 1
    for t in p.tuples:
        assert p.s1 * math.prod(p.primes[j] for j in t) >= N
    assert p.T <= min(p.P)


def test_plan_rejects_invalid():
    for N, s, prm in [(12, 2, Params()), (100, 0, Params()), (100, 101, Params()),
                      (100, 5, Params(tau=0.5)), (30, 2, Params(preset=PRESET_THEORY, r=1.0)),
                      (100, 5, Params(preset=9)), (30, 1, Params())]:
        with pytest.raises(ValueError):
            make_plan(N, s, prm)
