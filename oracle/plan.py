"""Plan rules of the oracle (test infrastructure; see the package docstring).

Every quantity is derived here from the paper's statements, in FP64 for the
real constants and with exact integer loops for the integers.  The GPU library
derives the same plan with its own, separately written code; tests compare the
two field by field.

Readings where the paper is silent (they are the same on both sides):

* presets ``dmsft6`` / ``dmsft4``: window half-width kappa = 6 / 4 (the two
  DMSFT variants of Section 5); the paper does not give their beta, so the
  Gaussian width in grid steps is sigma_t = sqrt((kappa + 1/2) / pi), which
  makes the window-truncation loss exp(-(kappa+1/2)^2 / (2 sigma_t^2)) equal
  to the aliasing loss exp(-(pi sigma_t)^2 / 2); then beta = 2 pi sigma_t /
  sqrt(ln N) so that c1 = beta sqrt(ln N) / N (Algorithm 1's parameters).
* preset ``theory``: beta = 6 sqrt(r), c1 = 6 sqrt(ln N^r) / N and the window
  half-width kappa = ceil(6 r ln N / (sqrt(2) pi)) + 1 of Theorem 4.
* tau = 1/3 (the choice made after Lemma 13) and alpha taken at equality in
  Lemma 3: alpha = beta / sqrt(ln(1 / (tau sqrt(2 pi))) / 2).  Lemma 3 also
  needs alpha in [1, N / sqrt(ln N)]; plans outside that range are rejected
  (for dmsft6 this means N >= 31).
* c2 = alpha sqrt(ln N) / 2, Q = ceil(c2) bands, L = ceil(N / (alpha sqrt(ln N)))
  and q_b = -ceil(N/2) + 1 + (2b - 1) L (Algorithm 1's parameters and band centres).
* inner algorithm: moduli P_j = s1 * p_j with s1 the least power of two
  >= 2 s (times an optional multiplier), G = max(2, ceil(log2(N / s1) / 6)),
  p_min the least integer with p_min^G * s1 >= N, and p_1 < ... < p_K the
  K = 2G + 1 smallest odd primes >= max(3, p_min).  Two CRT tuples of G
  moduli each: (1..G) and (G+1..2G).  T = min(2 s, P_1) heavy bins per DFT.
* identification (the inner sparse FFT of Algorithm 1): ``IDENT_RESIDUE`` combines heavy
  bins of several moduli by the CRT; ``IDENT_PHASE`` reads each heavy bin's
  frequency from the phase between the bin and the same bin of samples taken
  one grid step later (the phase-shift family the paper pairs with CLW-DSFT in
  Section 5, whose inner algorithm it does not print).  Both use the same
  moduli, heavy bins, majority vote and median.
"""
from __future__ import annotations

import dataclasses
import math

PRESET_DMSFT6 = 0
PRESET_DMSFT4 = 1
PRESET_THEORY = 2

IDENT_RESIDUE = 0
IDENT_PHASE = 1


@dataclasses.dataclass(frozen=True)
class Params:
    """Zero in a field means "the preset's default"."""
    preset: int = PRESET_DMSFT6
    kappa: int = 0
    sigma_t: float = 0.0
    tau: float = 0.0
    r: float = 0.0
    s1_mult: int = 0
    group: int = 0
    heavy_T: int = 0
    ident: int = IDENT_RESIDUE


@dataclasses.dataclass(frozen=True)
class Plan:
    N: int
    s: int
    preset: int
    kappa: int
    sigma_t: float
    beta: float
    c1: float
    tau: float
    alpha: float
    c2: float
    Q: int
    L: int
    q: tuple
    s1: int
    G: int
    K: int
    primes: tuple
    P: tuple
    T: int
    tuples: tuple
    r: float
    ident: int = IDENT_RESIDUE

    @property
    def band_lo(self) -> int:
        return -((self.N + 1) // 2) + 1

    @property
    def band_hi(self) -> int:
        return self.N // 2

    @property
    def M(self) -> int:
        return sum(self.P)


def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def make_plan(N: int, s: int, params: Params = Params()) -> Plan:
    N = int(N)
    s = int(s)
    if N < 2:
        raise ValueError("N must be at least 2")
    if s < 1 or s > N:
        raise ValueError("s must satisfy 1 <= s <= N")
    preset = params.preset
    if params.ident not in (IDENT_RESIDUE, IDENT_PHASE):
        raise ValueError("unknown identification")
    lnN = math.log(N)
    r = 0.0
    if preset in (PRESET_DMSFT6, PRESET_DMSFT4):
        kappa = params.kappa if params.kappa > 0 else (6 if preset == PRESET_DMSFT6 else 4)
        sigma_t = params.sigma_t if params.sigma_t > 0 else math.sqrt((kappa + 0.5) / math.pi)
        beta = 2.0 * math.pi * sigma_t / math.sqrt(lnN)
    elif preset == PRESET_THEORY:
        r = params.r if params.r > 0 else 1.0
        if r < 1.0 or 36.0 * r > N:
            raise ValueError("theory preset needs 1 <= r <= N/36 (Theorem 4)")
        beta = 6.0 * math.sqrt(r)
        sigma_t = beta * math.sqrt(lnN) / (2.0 * math.pi)
        kappa = params.kappa if params.kappa > 0 else (
            math.ceil(6.0 * r * lnN / (math.sqrt(2.0) * math.pi)) + 1)
    else:
        raise ValueError("unknown preset")
    if N < 2 * kappa + 1:
        raise ValueError("N must be at least 2*kappa+1")
    c1 = beta * math.sqrt(lnN) / N
    tau = params.tau if params.tau > 0 else 1.0 / 3.0
    if not (0.0 < tau < 1.0 / math.sqrt(2.0 * math.pi)):
        raise ValueError("tau must lie in (0, 1/sqrt(2 pi)) (Lemma 3)")
    alpha = beta / math.sqrt(math.log(1.0 / (tau * math.sqrt(2.0 * math.pi))) / 2.0)
    if alpha < 1.0 or alpha * math.sqrt(lnN) > N:
        raise ValueError("alpha must lie in [1, N/sqrt(ln N)] (Lemma 3)")
    c2 = alpha * math.sqrt(lnN) / 2.0
    Q = math.ceil(c2)
    L = math.ceil(N / (alpha * math.sqrt(lnN)))
    half_up = (N + 1) // 2
    q = tuple(-half_up + 1 + (2 * b - 1) * L for b in range(1, Q + 1))

    mult = params.s1_mult if params.s1_mult > 0 else 1
    s1 = 1
    while s1 < 2 * s * mult:
        s1 *= 2
    if params.group > 0:
        G = params.group
    else:
        e = 0
        while s1 * 2 ** e < N:
            e += 1
        G = max(2, -(-e // 6))
    p_min = 1
    while p_min ** G * s1 < N:
        p_min += 1
    K = 2 * G + 1
    primes = []
    cand = max(3, p_min)
    while len(primes) < K:
        if cand % 2 == 1 and _is_prime(cand):
            primes.append(cand)
        cand += 1
    P = tuple(s1 * p for p in primes)
    T0 = params.heavy_T if params.heavy_T > 0 else 2 * s
    T = min(T0, min(P))
    tuples = (tuple(range(0, G)), tuple(range(G, 2 * G)))
    return Plan(N=N, s=s, preset=preset, kappa=int(kappa), sigma_t=float(sigma_t),
                beta=float(beta), c1=float(c1), tau=float(tau), alpha=float(alpha),
                c2=float(c2), Q=int(Q), L=int(L), q=q, s1=s1, G=G, K=K,
                primes=tuple(primes), P=P, T=int(T), tuples=tuples, r=float(r),
                ident=int(params.ident))
