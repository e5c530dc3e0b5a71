"""The oracle transform (test infrastructure; see the package docstring).

Algorithm 1 (Section 3), step by step, in FP64 and exact integers:

for each band b = 1..Q (Algorithm 1's loop over the band centres):
  1. filtered samples (Algorithm 1's convolution step): at every node theta = 2 pi k / P_j of every
     modulus j, evaluate the truncated semi-discrete convolution of Lemma 10,
         S_b(theta) = sum_{i=-kappa..kappa} f[(j'+i) mod N] * W(u - i)
                                          * exp(2 pi i q_b (u - i) / N),
     where t = k N / P_j is the node in grid steps, j' the nearest grid index
     (ties rounded up), u = t - j', and W(v) = g(2 pi v / N) / N is the
     periodized Gaussian of eq. (Def_Periodic_Gaussian) with c1 from the plan.
     The modulation is g~_q(x) = exp(+i q x) g(x), whose Fourier coefficients
     are ghat_{w-q}; this is the sign under which Algorithm 1's band test and
     its division keep and rescale the frequencies near +q.
  2. short DFTs (Appendix B, eq. DFT_GKlam_Comp):
         E_b[j][h] = (1/P_j) sum_k S_b(2 pi k / P_j) exp(-2 pi i k h / P_j).
  3. heavy bins: the T bins of largest |E_b[j][h]|^2, ties to the lower h.
  4. candidates: in each CRT tuple and residue class a mod s1, keep in every
     modulus of the tuple the c heaviest bins of the class (c^G <= 64), combine
     one kept bin per modulus, solve w = a (mod s1), w = h_g (mod p_g) by the
     CRT and keep the representative of w in B, if there is one.
  5. majority vote ("more than half" of the moduli, Appendix B): the G moduli
     of the tuple that produced w hold heavy bins at w by construction, so the
     vote is taken over the other K - G moduli: keep w if more than half of
     them have (w mod P_j) among their heavy bins (for some producing tuple).
  6. estimate: z_w = median_j Re E_b[j][w mod P_j] + i median_j Im(...).
  7. the inner algorithm's output: the s largest |z_w| (ties to the smaller w) form R_temp.
  8. band test and division: keep w in [q_b - L, q_b + L) and B; divide by
     ghat_{w - q_b} = exp(-c1^2 (w - q_b)^2 / 2) / sqrt(2 pi) (Lemma 2).
then (Algorithm 1's last step) return the s largest |v_w| over all bands, ties to the smaller w.

Phase identification (plan.ident == IDENT_PHASE) replaces steps 4-5:
  1'. the samples of step 1 are also taken at every node moved one grid step,
      theta + 2 pi / N: the same window and weights over f[(j'+1+i) mod N];
  2'. their short DFTs E'_b[j].  A bin h of modulus j that holds one
      frequency w (ghat-weighted) has E'[h] / E[h] = exp(2 pi i w / N), and
      w = h (mod P_j) is known, so the phase only has to single out one member
      of that residue class (a tolerance of pi P_j / N radians);
  4'. candidates: for every heavy bin, the w in B with w = h (mod P_j) whose
      angle 2 pi w / N lies circularly nearest to arg(E'[h] conj(E[h]))
      (ties to the smaller w), over all moduli, duplicates merged;
  5'. vote: keep w if more than half of all K moduli have (w mod P_j) among
      their heavy bins.

Frequencies are integers in B = (-ceil(N/2), floor(N/2)]; coefficients are
those of f_j = sum_w c_w exp(2 pi i w j / N).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .plan import IDENT_PHASE, Plan

COMBO_CAP = 64


def node_geometry(plan: Plan, j: int):
    """Nodes of modulus j: theta_k = 2 pi k / P_j, k = 0..P_j-1.

    Returns (jp, delta): jp[k] = the grid index nearest to t = k N / P_j
    (Lemma 10's j'; a tie is rounded up) and delta[k] = k N - jp[k] P_j, so that
    u = t - j' = delta / P_j lies in [-1/2, 1/2).  Exact integers.
    """
    P = plan.P[j]
    N = plan.N
    k = np.arange(P, dtype=np.int64)
    jp = (2 * k * N + P) // (2 * P)
    delta = k * N - jp * P
    return jp, delta


def window_weight(plan: Plan, v: np.ndarray) -> np.ndarray:
    """W(v) = g(2 pi v / N) / N for an offset of v grid steps.

    g is the periodized Gaussian of eq. (Def_Periodic_Gaussian),
    g(x) = (1/c1) sum_n exp(-(x - 2 pi n)^2 / (2 c1^2)).  The images n = -1, 0, 1
    are summed; every farther image lies at least 2N - kappa - 1 grid steps
    away and underflows to zero for every accepted plan.
    """
    N = plan.N
    c1 = plan.c1
    x = 2.0 * math.pi * np.asarray(v, dtype=np.float64) / N
    tot = np.zeros_like(x)
    for n in (-1, 0, 1):
        tot += np.exp(-((x - 2.0 * math.pi * n) ** 2) / (2.0 * c1 * c1))
    return tot / (c1 * N)


def ghat(plan: Plan, n) -> np.ndarray:
    """Fourier coefficients of g (Lemma 2): exp(-c1^2 n^2 / 2) / sqrt(2 pi)."""
    n = np.asarray(n, dtype=np.float64)
    return np.exp(-(plan.c1 ** 2) * n * n / 2.0) / math.sqrt(2.0 * math.pi)


def filtered_samples(plan: Plan, f: np.ndarray, b: int, j: int, shift: int = 0) -> np.ndarray:
    """S_b at the nodes of modulus j (Algorithm 1's convolution step; Lemma 10's window).

    shift moves every node by that many grid steps (theta + 2 pi shift / N):
    the nearest grid index moves with it and the offset u does not, so the
    weights stay those of the unshifted node."""
    f = np.asarray(f, dtype=np.complex128)
    N = plan.N
    P = plan.P[j]
    q = plan.q[b]
    jp, delta = node_geometry(plan, j)
    u = delta / P
    S = np.zeros(P, dtype=np.complex128)
    for i in range(-plan.kappa, plan.kappa + 1):
        v = u - i
        S += f[np.mod(jp + shift + i, N)] * window_weight(plan, v) * np.exp(2j * math.pi * q * v / N)
    return S


def short_dft(S: np.ndarray) -> np.ndarray:
    """E[h] = (1/P) sum_k S[k] exp(-2 pi i k h / P)  (Appendix B)."""
    return np.fft.fft(S) / S.shape[0]


def heavy_bins(E: np.ndarray, T: int) -> np.ndarray:
    """Indices of the T largest |E[h]|^2, ties to the lower h; sorted by h."""
    mag2 = E.real * E.real + E.imag * E.imag
    h = np.arange(E.shape[0])
    order = np.lexsort((h, -mag2))
    return np.sort(order[:T])


def crt(residues, moduli) -> int:
    """The x in [0, prod(moduli)) with x = r_i (mod m_i), moduli pairwise coprime."""
    M = 1
    for m in moduli:
        M *= m
    x = 0
    for r, m in zip(residues, moduli):
        Mi = M // m
        x += int(r) * Mi * pow(Mi, -1, m)
    return x % M


def representative_in_band(r: int, M: int, N: int):
    """The w in B = (-ceil(N/2), floor(N/2)] with w = r (mod M), or None (M >= N)."""
    lo = -((N + 1) // 2) + 1
    hi = N // 2
    if r <= hi:
        return r
    if r - M >= lo:
        return r - M
    return None


def class_depth(G: int) -> int:
    """Heaviest bins kept per residue class and modulus: the largest c with
    c^G <= 64, so that one class yields at most 64 combinations."""
    c = 1
    while (c + 1) ** G <= COMBO_CAP:
        c += 1
    return c


def candidates(plan: Plan, heavy, E) -> dict:
    """Candidate frequencies of one band from the heavy bins of its K DFTs,
    mapped to the indices of the CRT tuples that produce them.

    In each CRT tuple and residue class a mod s1, the heavy bins of every
    modulus of the tuple that lie in class a are ranked by |E|^2 (ties to the
    lower h) and the class_depth(G) heaviest are kept; every combination of one
    kept bin per modulus is solved by the CRT and mapped into B.
    """
    s1 = plan.s1
    depth = class_depth(plan.G)
    found = {}
    for t, tup in enumerate(plan.tuples):
        moduli = [s1] + [plan.primes[j] for j in tup]
        M = 1
        for m in moduli:
            M *= m
        buckets = []
        for j in tup:
            bk = {}
            for h in heavy[j]:
                bk.setdefault(int(h) % s1, []).append(int(h))
            mag2 = E[j].real ** 2 + E[j].imag ** 2
            for a in bk:
                bk[a] = sorted(bk[a], key=lambda h: (-mag2[h], h))[:depth]
            buckets.append(bk)
        for a in range(s1):
            lists = [bk.get(a, []) for bk in buckets]
            for combo in itertools.product(*lists):
                residues = [a] + [h % plan.primes[j] for h, j in zip(combo, tup)]
                w = representative_in_band(crt(residues, moduli), M, plan.N)
                if w is not None:
                    found.setdefault(w, set()).add(t)
    return dict(sorted(found.items()))


def phase_frequency(plan: Plan, j: int, h: int, e: complex, e_shift: complex):
    """The w in B with w = h (mod P_j) whose angle 2 pi w / N is circularly
    nearest to arg(e_shift conj(e)), ties to the smaller w; None if B holds no
    member of the class.  Every member of the class is tried."""
    N = plan.N
    P = plan.P[j]
    x = float(np.angle(complex(e_shift) * complex(e).conjugate())) * N / (2.0 * math.pi)
    lo, hi = plan.band_lo, plan.band_hi
    m_lo = -((h - lo) // P)          # least m with h + m P >= lo
    m_hi = (hi - h) // P             # largest m with h + m P <= hi
    if m_hi < m_lo:
        return None
    ws = h + P * np.arange(m_lo, m_hi + 1, dtype=np.int64)
    d = ws.astype(np.float64) - x
    dist = np.minimum(np.abs(d), np.minimum(np.abs(d - N), np.abs(d + N)))
    best = np.lexsort((ws, dist))[0]
    return int(ws[best])


def phase_candidates(plan: Plan, heavy, E, E_shift) -> list:
    """Candidate frequencies of one band: phase_frequency of every heavy bin of
    every modulus, duplicates merged, ascending."""
    found = set()
    for j in range(plan.K):
        for h in heavy[j]:
            w = phase_frequency(plan, j, int(h), E[j][h], E_shift[j][h])
            if w is not None:
                found.add(w)
    return sorted(found)


def vote_count(plan: Plan, heavy_sets, w: int, exclude=()) -> int:
    """Number of moduli j (outside `exclude`) whose heavy bins contain w mod P_j."""
    return sum(1 for j in range(plan.K) if j not in exclude and (w % plan.P[j]) in heavy_sets[j])


def accepted_by_vote(plan: Plan, heavy_sets, w: int, tuples) -> bool:
    """More than half of the moduli outside a producing tuple agree."""
    outside = plan.K - plan.G
    return any(2 * vote_count(plan, heavy_sets, w, plan.tuples[t]) > outside for t in tuples)


def median_estimate(plan: Plan, E, w: int) -> complex:
    vals = np.array([E[j][w % plan.P[j]] for j in range(plan.K)])
    return complex(np.median(vals.real), np.median(vals.imag))


def _band(plan: Plan, f: np.ndarray, b: int, keep: bool):
    S = [filtered_samples(plan, f, b, j) for j in range(plan.K)]
    E = [short_dft(Sj) for Sj in S]
    heavy = [heavy_bins(Ej, plan.T) for Ej in E]
    heavy_sets = [set(int(h) for h in Hj) for Hj in heavy]
    accepted = []
    S2 = E2 = None
    if plan.ident == IDENT_PHASE:
        S2 = [filtered_samples(plan, f, b, j, shift=1) for j in range(plan.K)]
        E2 = [short_dft(Sj) for Sj in S2]
        cands = phase_candidates(plan, heavy, E, E2)
        for w in cands:
            if 2 * vote_count(plan, heavy_sets, w) > plan.K:
                accepted.append((w, median_estimate(plan, E, w)))
    else:
        cands = candidates(plan, heavy, E)
        for w, tuples in cands.items():
            if accepted_by_vote(plan, heavy_sets, w, tuples):
                accepted.append((w, median_estimate(plan, E, w)))
    # the s-sparse output of the inner algorithm (Algorithm 1)
    r_temp = sorted(accepted, key=lambda wz: (-abs(wz[1]), wz[0]))[: plan.s]
    # band test and division by the modulated filter's coefficient (Algorithm 1)
    q = plan.q[b]
    out = []
    for w, z in r_temp:
        if q - plan.L <= w < q + plan.L and plan.band_lo <= w <= plan.band_hi:
            out.append((w, z / float(ghat(plan, w - q))))
    info = None
    if keep:
        info = dict(S=S, E=E, heavy=heavy, candidates=cands, accepted=accepted,
                    r_temp=r_temp, kept=out, S_shift=S2, E_shift=E2)
    return out, info


def sft_trace(plan: Plan, f: np.ndarray, bands=None):
    """Run Algorithm 1 and return (freqs, coefs, per-band intermediates)."""
    f = np.asarray(f, dtype=np.complex128)
    if f.shape != (plan.N,):
        raise ValueError("f must have N entries")
    R = []
    infos = {}
    for b in range(plan.Q):
        if bands is not None and b not in bands:
            continue
        kept, info = _band(plan, f, b, keep=True)
        R.extend(kept)
        infos[b] = info
    top = sorted(R, key=lambda wv: (-abs(wv[1]), wv[0]))[: plan.s]
    freqs = np.array([w for w, _ in top], dtype=np.int64)
    coefs = np.array([v for _, v in top], dtype=np.complex128)
    return freqs, coefs, infos


def sft(plan: Plan, f: np.ndarray):
    """Algorithm 1: the s-term output (freqs ordered by |v| desc, w asc; coefs)."""
    f = np.asarray(f, dtype=np.complex128)
    if f.shape != (plan.N,):
        raise ValueError("f must have N entries")
    R = []
    for b in range(plan.Q):
        kept, _ = _band(plan, f, b, keep=False)
        R.extend(kept)
    top = sorted(R, key=lambda wv: (-abs(wv[1]), wv[0]))[: plan.s]
    freqs = np.array([w for w, _ in top], dtype=np.int64)
    coefs = np.array([v for _, v in top], dtype=np.complex128)
    return freqs, coefs
