"""FP64 CPU oracle of the fully discrete sparse Fourier transform.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or execute anything in
this package.  The GPU library (``paper_1706_02740_amd``) never does, and this
package imports nothing from it: the two share no code, tables or constants.
Inputs come from ``siggen``, which holds none of the method's arithmetic.

The oracle is deliberately plain and slow: it follows the steps of
Algorithm 1 (Section 3) in the paper's order, evaluates the filtered samples
with the truncated convolution sum of Lemma 10, runs the short DFTs of
Appendix B with ``numpy.fft`` as the library primitive, and identifies and
estimates frequencies with the residue/CRT (or phase-shift), majority-vote and
median reading of the inner algorithm (see ``oracle.sft``).  Everything is FP64 / exact
integers.

Modules:
  plan  -- parameter rules (Lemma 3, Algorithm 1's parameters and band centres, Theorem 4)
  transform -- the transform itself, with every intermediate exposed
"""
from .plan import (Params, Plan, make_plan, PRESET_DMSFT6, PRESET_DMSFT4,
                   PRESET_THEORY, IDENT_RESIDUE, IDENT_PHASE)
from .transform import (node_geometry, window_weight, ghat, filtered_samples,
                  short_dft, heavy_bins, crt, representative_in_band,
                  class_depth, candidates, vote_count, accepted_by_vote, median_estimate,
                  phase_frequency, phase_candidates, sft, sft_trace)

__all__ = [
    "Params", "Plan", "make_plan", "PRESET_DMSFT6", "PRESET_DMSFT4",
    "PRESET_THEORY", "IDENT_RESIDUE", "IDENT_PHASE", "node_geometry", "window_weight", "ghat",
    "filtered_samples", "short_dft", "heavy_bins", "crt",
    "representative_in_band", "class_depth", "candidates", "vote_count", "accepted_by_vote",
    "median_estimate", "phase_frequency", "phase_candidates",
    "sft", "sft_trace",
]
