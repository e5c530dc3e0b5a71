"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch each one: a flipped modulation sign, a dropped window tap, a shifted
node rounding, a missing DFT normalisation, a wrong tie rule, a mean in place
of the median, a transposed CRT pairing, a wrong exponent in ghat, an
inclusive band edge, a shift in the wrong direction, a phase read without
wrap-around, a tie sent to the larger frequency."""
import math

import numpy as np
import pytest

import oracle
import oracle.transform as osft
import tests.test_oracle_pins as pins
import tests.test_oracle_end_to_end as e2e
import tests.test_oracle_phase as phase


def _bad_samples_sign(plan, f, b, j):
    f = np.asarray(f, dtype=np.complex128)
    jp, delta = osft.node_geometry(plan, j)
    u = delta / plan.P[j]
    S = np.zeros(plan.P[j], dtype=np.complex128)
    for i in range(-plan.kappa, plan.kappa + 1):
        v = u - i
        S += f[np.mod(jp + i, plan.N)] * osft.window_weight(plan, v) * np.exp(-2j * math.pi * plan.q[b] * v / plan.N)
    return S


def _bad_samples_short_window(plan, f, b, j):
    f = np.asarray(f, dtype=np.complex128)
    jp, delta = osft.node_geometry(plan, j)
    u = delta / plan.P[j]
    S = np.zeros(plan.P[j], dtype=np.complex128)
    for i in range(-plan.kappa, plan.kappa):
        v = u - i
        S += f[np.mod(jp + i, plan.N)] * osft.window_weight(plan, v) * np.exp(2j * math.pi * plan.q[b] * v / plan.N)
    return S


def _bad_nodes(plan, j):
    P, N = plan.P[j], plan.N
    k = np.arange(P, dtype=np.int64)
    jp = (2 * k * N + P - 1) // (2 * P)          # ties rounded down
    return jp, k * N - jp * P


def _bad_dft(S):
    return np.fft.fft(S)


def _bad_heavy(E, T):
    mag2 = np.abs(E) ** 2
    h = np.arange(E.shape[0])
    order = np.lexsort((-h, -mag2))
    return np.sort(order[:T])


def _bad_median(plan, E, w):
    vals = np.array([E[j][w % plan.P[j]] for j in range(plan.K)])
    return complex(np.mean(vals.real), np.mean(vals.imag))


def _bad_crt(residues, moduli):
    M = math.prod(moduli)
    x = 0
    for r, m in zip(residues, list(moduli)[::-1]):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def _bad_ghat(plan, n):
    n = np.asarray(n, dtype=np.float64)
    return np.exp(-(plan.c1 ** 2) * n * n) / math.sqrt(2.0 * math.pi)


def _bad_window(plan, v):
    x = 2.0 * math.pi * np.asarray(v, dtype=np.float64) / plan.N
    return np.exp(-(x ** 2) / (2.0 * plan.c1 * plan.c1)) / (plan.c1 * plan.N * math.sqrt(2 * math.pi))


def _bad_vote_all_moduli(plan, heavy_sets, w, tuples):
    return 2 * sum((w % plan.P[j]) in heavy_sets[j] for j in range(plan.K)) > plan.K


_orig_samples = osft.filtered_samples
_orig_phase = osft.phase_frequency


def _bad_shift_sign(plan, f, b, j, shift=0):
    return _orig_samples(plan, f, b, j, shift=-shift)


def _bad_phase_no_wrap(plan, j, h, e, e_shift):
    """Linear instead of circular distance to the phase's frequency."""
    N, P = plan.N, plan.P[j]
    x = float(np.angle(complex(e_shift) * complex(e).conjugate())) * N / (2.0 * math.pi)
    best = None
    for m in range(-((h - plan.band_lo) // P), (plan.band_hi - h) // P + 1):
        w = h + m * P
        if best is None or (abs(w - x), w) < best:
            best = (abs(w - x), w)
    return None if best is None else best[1]


def _bad_phase_ties_up(plan, j, h, e, e_shift):
    w = _orig_phase(plan, j, h, e, e_shift)
    if w is None:
        return None
    x = float(np.angle(complex(e_shift) * complex(e).conjugate())) * plan.N / (2.0 * math.pi)
    up = w + plan.P[j]
    if up <= plan.band_hi and abs(up - x) == abs(w - x):
        return up
    return w


MUTATIONS = [
    ("filtered_samples", _bad_samples_sign, lambda: pins.test_filtered_samples_closed_form(0)),
    ("filtered_samples", _bad_samples_short_window, pins.test_window_extent_with_a_unit_impulse),
    ("node_geometry", _bad_nodes, lambda: pins.test_node_geometry_exact_rationals(1000, 5)),
    ("short_dft", _bad_dft, pins.test_dft_bins_aliasing_identity),
    ("heavy_bins", _bad_heavy, pins.test_heavy_bins_ties_go_to_lower_index),
    ("median_estimate", _bad_median, pins.test_median_estimate_componentwise),
    ("crt", _bad_crt, pins.test_crt_bruteforce),
    ("ghat", _bad_ghat, lambda: pins.test_ghat_matches_numerical_fourier_coefficients(64)),
    ("window_weight", _bad_window, lambda: pins.test_window_weight_is_g_over_N(64, 3.3)),
    ("ghat", _bad_ghat, e2e.test_band_edge_frequencies),
    ("accepted_by_vote", _bad_vote_all_moduli, e2e.test_candidates_equal_bruteforce_definition),
    ("accepted_by_vote", _bad_vote_all_moduli, e2e.test_ghost_combinations_are_rejected),
    ("filtered_samples", _bad_shift_sign, lambda: phase.test_shifted_samples_closed_form(4096, 6)),
    ("filtered_samples", _bad_shift_sign, lambda: phase.test_one_sparse_bins_carry_the_frequency(3001, 3)),
    ("phase_frequency", _bad_phase_no_wrap, lambda: phase.test_phase_frequency_worked_examples(100, 12, 5, 0.499, -43)),
    ("phase_frequency", _bad_phase_ties_up, lambda: phase.test_phase_frequency_worked_examples(100, 8, 21, 0.25, 21)),
]


@pytest.mark.parametrize("name,bad,pin", MUTATIONS, ids=[f"{m[0]}-{m[1].__name__}" for m in MUTATIONS])
def test_pin_catches_planted_mistake(monkeypatch, name, bad, pin):
    monkeypatch.setattr(osft, name, bad)
    monkeypatch.setattr(oracle, name, bad)
    with pytest.raises(AssertionError):
        pin()


def test_inclusive_band_edge_is_caught(monkeypatch):
    """A band test closed on the right would report an edge frequency twice."""
    orig = osft._band

    def _band_inclusive(plan, f, b, keep):
        out, info = orig(plan, f, b, True)
        q = plan.q[b]
        extra = [(w, z / float(osft.ghat(plan, w - q))) for w, z in info["r_temp"]
                 if w == q + plan.L and plan.band_lo <= w <= plan.band_hi]
        return out + extra, info

    monkeypatch.setattr(osft, "_band", _band_inclusive)
    with pytest.raises(AssertionError):
        e2e.test_band_edge_frequencies()
