// Host-side plan rules: FP64 constants and exact integer searches.
//
//   c1 = beta sqrt(ln N) / N, c2 = alpha sqrt(ln N) / 2           (Algorithm 1, parameters)
//   q_b = -ceil(N/2) + 1 + (2b - 1) ceil(N / (alpha sqrt(ln N)))    (Algorithm 1, band centres)
//   alpha at equality in Lemma 3, tau = 1/3 by default (after Lemma 13)
//   theory preset: beta = 6 sqrt(r), kappa = ceil(6 r ln N / (sqrt(2) pi)) + 1 (Theorem 4)
//   dmsft presets: kappa = 6 or 4 (Section 5), sigma_t = sqrt((kappa + 1/2) / pi) in grid
//   steps, which balances the window-truncation and aliasing losses.
//   Inner algorithm: s1 = least power of two >= 2 s, G = max(2, ceil(log2(N/s1)/6)),
//   p_min^G s1 >= N, K = 2G + 1 odd primes >= max(3, p_min), P_j = s1 p_j.
#include <algorithm>
#include <math.h>
#include <string.h>

#include "sft_internal.h"

namespace sft {

static bool is_odd_prime(int64_t n) {
    if (n < 3 || (n & 1) == 0) return false;
    for (int64_t d = 3; d * d <= n; d += 2)
        if (n % d == 0) return false;
    return true;
}

static int64_t inv_mod(int64_t a, int64_t m) {  // a^{-1} mod m, gcd(a, m) = 1
    int64_t t = 0, nt = 1, r = m, nr = a % m;
    if (nr < 0) nr += m;
    while (nr != 0) {
        int64_t qq = r / nr, tmp;
        tmp = t - qq * nt; t = nt; nt = tmp;
        tmp = r - qq * nr; r = nr; nr = tmp;
    }
    if (t < 0) t += m;
    return m == 1 ? 0 : t;
}

int derive_plan(int64_t N, int32_t s, const sft_params* prm, sft_plan_info* out, const char** why) {
    sft_params P0;
    memset(&P0, 0, sizeof(P0));
    const sft_params& p = prm ? *prm : P0;
    memset(out, 0, sizeof(*out));
    if (N < 2) { *why = "N must be at least 2"; return SFT_EINVAL; }
    if (N > ((int64_t)1 << 31) - 1) { *why = "N above 2^31 - 1 is not supported"; return SFT_EUNSUPPORTED; }
    if (s < 1 || (int64_t)s > N) { *why = "s must satisfy 1 <= s <= N"; return SFT_EINVAL; }
    if (p.ident != SFT_IDENT_RESIDUE && p.ident != SFT_IDENT_PHASE) { *why = "unknown identification"; return SFT_EINVAL; }
    const double lnN = log((double)N);
    int32_t kappa;
    double sigma_t, beta, r = 0.0;
    if (p.preset == SFT_PRESET_DMSFT6 || p.preset == SFT_PRESET_DMSFT4) {
        kappa = p.kappa > 0 ? p.kappa : (p.preset == SFT_PRESET_DMSFT6 ? 6 : 4);
        sigma_t = p.sigma_t > 0 ? p.sigma_t : sqrt((kappa + 0.5) / M_PI);
        beta = 2.0 * M_PI * sigma_t / sqrt(lnN);
    } else if (p.preset == SFT_PRESET_THEORY) {
        r = p.r > 0 ? p.r : 1.0;
        if (r < 1.0 || 36.0 * r > (double)N) { *why = "theory preset needs 1 <= r <= N/36 (Theorem 4)"; return SFT_EINVAL; }
        beta = 6.0 * sqrt(r);
        sigma_t = beta * sqrt(lnN) / (2.0 * M_PI);
        kappa = p.kappa > 0 ? p.kappa : (int32_t)ceil(6.0 * r * lnN / (sqrt(2.0) * M_PI)) + 1;
    } else {
        *why = "unknown preset"; return SFT_EINVAL;
    }
    if (N < 2 * (int64_t)kappa + 1) { *why = "N must be at least 2*kappa+1"; return SFT_EINVAL; }
    const double c1 = beta * sqrt(lnN) / (double)N;
    const double tau = p.tau > 0 ? p.tau : 1.0 / 3.0;
    if (!(tau > 0.0 && tau < 1.0 / sqrt(2.0 * M_PI))) { *why = "tau must lie in (0, 1/sqrt(2 pi)) (Lemma 3)"; return SFT_EINVAL; }
    const double alpha = beta / sqrt(log(1.0 / (tau * sqrt(2.0 * M_PI))) / 2.0);
    if (alpha < 1.0 || alpha * sqrt(lnN) > (double)N) { *why = "alpha must lie in [1, N/sqrt(ln N)] (Lemma 3)"; return SFT_EINVAL; }
    const double c2 = alpha * sqrt(lnN) / 2.0;
    const int64_t Q = (int64_t)ceil(c2);
    const int64_t L = (int64_t)ceil((double)N / (alpha * sqrt(lnN)));
    if (Q > SFT_MAX_BANDS) { *why = "more than SFT_MAX_BANDS bands"; return SFT_EUNSUPPORTED; }

    const int64_t mult = p.s1_mult > 0 ? p.s1_mult : 1;
    int64_t s1 = 1;
    while (s1 < 2 * (int64_t)s * mult) s1 *= 2;
    int32_t G;
    if (p.group > 0) {
        G = p.group;
    } else {
        int32_t e = 0;
        while ((s1 << e) < N) ++e;
        G = (e + 5) / 6;
        if (G < 2) G = 2;
    }
    if (G > kMaxG) { *why = "more than 7 primes per CRT tuple"; return SFT_EUNSUPPORTED; }
    int64_t pmin = 1;
    for (;;) {
        unsigned __int128 v = (unsigned __int128)s1;
        for (int g = 0; g < G; ++g) v *= (unsigned __int128)pmin;
        if (v >= (unsigned __int128)N) break;
        ++pmin;
    }
    const int32_t K = 2 * G + 1;
    int64_t cand = pmin < 3 ? 3 : pmin;
    int32_t found = 0;
    while (found < K) {
        if (is_odd_prime(cand)) out->primes[found++] = (int32_t)cand;
        ++cand;
    }
    int64_t Pmin = INT64_MAX, M = 0;
    for (int j = 0; j < K; ++j) {
        out->P[j] = s1 * out->primes[j];
        if (out->P[j] < Pmin) Pmin = out->P[j];
        M += out->P[j];
    }
    if (M > ((int64_t)1 << 31) - 1 || s1 > ((int64_t)1 << 24)) { *why = "too many nodes"; return SFT_EUNSUPPORTED; }
    int64_t Pmax = 0;
    for (int j = 0; j < K; ++j) Pmax = out->P[j] > Pmax ? out->P[j] : Pmax;
    if ((uint64_t)s1 * (uint64_t)Pmax >= ((uint64_t)1 << 32)) { *why = "s1 * P_j must stay below 2^32"; return SFT_EUNSUPPORTED; }
    const int64_t T0 = p.heavy_T > 0 ? p.heavy_T : 2 * (int64_t)s;
    const int64_t T = T0 < Pmin ? T0 : Pmin;
    int32_t depth = 1;
    for (;;) {
        int64_t v = 1;
        for (int g = 0; g < G; ++g) v *= depth + 1;
        if (v > 64) break;
        ++depth;
    }
    out->N = N;
    out->s = s;
    out->preset = p.preset;
    out->kappa = kappa;
    out->Q = (int32_t)Q;
    out->L = L;
    out->q_first = -((N + 1) / 2) + 1 + L;
    out->s1 = (int32_t)s1;
    out->G = G;
    out->K = K;
    out->T = (int32_t)T;
    out->depth = depth;
    out->ident = p.ident;
    out->sigma_t = sigma_t;
    out->beta = beta;
    out->c1 = c1;
    out->tau = tau;
    out->alpha = alpha;
    out->c2 = c2;
    out->r = r;
    out->M = M;
    return SFT_OK;
}

void fill_desc(const sft_plan_info& in, SigDesc* d) {
    memset(d, 0, sizeof(*d));
    d->N = in.N;
    d->L = in.L;
    d->q_first = in.q_first;
    d->lo = -((in.N + 1) / 2) + 1;
    d->hi = in.N / 2;
    d->s = in.s;
    d->kappa = in.kappa;
    d->taps = 2 * in.kappa + 1;
    d->Q = in.Q;
    d->K = in.K;
    d->G = in.G;
    d->s1 = in.s1;
    int lg = 0;
    while ((1 << lg) < in.s1) ++lg;
    d->log2s1 = lg;
    d->T = in.T;
    int tp = 1;
    while (tp < in.T) tp *= 2;
    d->Tpow2 = tp;
    d->depth = in.depth;
    d->phase = in.ident == SFT_IDENT_PHASE ? 1 : 0;
    int sc = 1024;
    while (sc < 4 * in.T && sc < 4096) sc *= 2;
    d->sel_cap = sc;
    d->M = (int32_t)in.M;
    int ac = 256;
    while (ac < 8 * in.s && ac < kAcceptCap) ac *= 2;
    d->accept_cap = ac;
    d->inv2sig2 = (float)(1.0 / (2.0 * in.sigma_t * in.sigma_t));
    d->wnorm = (float)(1.0 / (2.0 * M_PI * in.sigma_t));
    for (int i = 0; i < kFastTaps; ++i) {
        const double o = (double)(i - in.kappa);
        d->gtap[i] = i < 2 * in.kappa + 1 ? (float)exp(-o * o / (2.0 * in.sigma_t * in.sigma_t)) : 0.f;
    }
    d->a_first = (float)((double)in.q_first / (double)in.N);
    d->a_step = (float)(2.0 * (double)in.L / (double)in.N);
    d->c1sq_half = in.c1 * in.c1 / 2.0;
    d->ghat0 = 1.0 / sqrt(2.0 * M_PI);
    int32_t off = 0, twoff = 0, trigoff = 0;
    for (int j = 0; j < in.K; ++j) {
        d->p[j] = in.primes[j];
        d->P[j] = (int32_t)in.P[j];
        d->Moff[j] = off;
        off += (int32_t)in.P[j];
        d->pinv_s1[j] = (int32_t)inv_mod(in.primes[j], in.s1);
        d->s1inv_p[j] = (int32_t)inv_mod(in.s1, in.primes[j]);
        d->tw_off[j] = twoff;
        twoff += in.primes[j];
        d->trig_off[j] = trigoff;
        trigoff += ((in.primes[j] - 1) / 2) * ((in.primes[j] - 1) / 2);
        d->magic_p[j] = UINT64_MAX / (uint64_t)in.primes[j] + 1;
        d->magic_P[j] = UINT64_MAX / (uint64_t)in.P[j] + 1;
        d->lo_mod_P[j] = (int32_t)(((d->lo % in.P[j]) + in.P[j]) % in.P[j]);
    }
    d->Moff[in.K] = off;
    for (int t = 0; t < 2; ++t) {
        int64_t Mt = in.s1;
        d->tup_mod[t][0] = in.s1;
        for (int g = 0; g < in.G; ++g) {
            const int j = t * in.G + g;
            d->tup_j[t][g] = j;
            d->tup_mod[t][g + 1] = in.primes[j];
            Mt *= in.primes[j];
        }
        d->tup_M[t] = Mt;
        for (int c = 0; c <= in.G; ++c) {
            const int64_t m = d->tup_mod[t][c];
            d->tup_Mi[t][c] = Mt / m;
            d->tup_inv[t][c] = (int32_t)inv_mod((Mt / m) % m, m);
        }
    }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

WorkspaceLayout workspace_layout(const sft_plan_info& in) {
    WorkspaceLayout w;
    const size_t QM = (size_t)in.Q * (size_t)in.M;
    w.S = align256(QM * 8);
    w.E = align256(QM * 8);
    w.S2 = in.ident == SFT_IDENT_PHASE ? align256(QM * 8) : 0;
    w.E2 = w.S2;
    w.H = align256((size_t)in.K * in.Q * in.T * 4);
    w.thr = align256((size_t)in.K * in.Q * 8);
    w.CL = align256((size_t)in.K * in.Q * in.s1 * in.depth * 4);
    w.Rw = align256((size_t)in.Q * in.s * 8);
    w.Rv = align256((size_t)in.Q * in.s * 16);
    w.Rn = align256((size_t)in.Q * 4);
    w.status = 256;
    w.SH = 0;   // set by sft_plan_create for plans whose column kernel fills the selection's histograms
    w.total = w.S + w.E + w.S2 + w.E2 + w.H + w.thr + w.CL + w.Rw + w.Rv + w.Rn + w.status + w.SH;
    return w;
}

size_t dft_lds_bytes(const SigDesc& d) {
    int32_t Pmax = 0;
    for (int j = 0; j < d.K; ++j)
        if (d.P[j] > Pmax) Pmax = d.P[j];
    const size_t h = (size_t)(d.p[d.K - 1] - 1) / 2;
    // data (8 B per bin) + s1 twiddles + the cosine/sine table + histogram +
    // scan partials + the T heavy keys + the class lists (the VALU step B;
    // dft_mx_lds_bytes gives the matrix-core kernel's)
    const size_t ntrig = h * h;
    return (size_t)Pmax * 8 + (size_t)d.s1 * 8 + ntrig * 8 + (size_t)kSelBins * 4 + 64 + (size_t)d.T * 8 +
           (size_t)d.s1 * d.depth * 4 + 64;
}

size_t dft_mx_lds_bytes(const SigDesc& d, int jhi) {
    // the block (8 B per bin) and the s1 twiddles, over which the selection's
    // scan partials, T heavy keys and class lists go once step B has read the
    // block (past it when they need more); then the selection's first
    // histogram, formed as the bins are
    const size_t block = (size_t)d.P[jhi - 1] * 8 + (size_t)d.s1 * 8;
    const size_t scratch = 64 + (size_t)d.T * 8 + (size_t)d.s1 * d.depth * 4;
    return std::max(block, scratch) + (size_t)kSelBins * 4 + 64;
}

int dft_pairs_per_thread(const SigDesc& d) {
    if (d.s1 > kDftThreads) return 1 << 30;
    const int ng = kDftThreads / d.s1;
    const int h = (d.p[d.K - 1] - 1) / 2;
    return (h + ng - 1) / ng;
}

bool dft_fits_one_workgroup(const SigDesc& d) { return dft_pairs_per_thread(d) <= kDftKBMax; }

int dft_mfma_variant(const SigDesc& d) {
    static_assert(kDftThreads == 512, "the matrix-core step B assumes 8 waves");
    const int ntw = d.s1 == 64 ? 1 : d.s1 == 128 ? 2 : 0;
    const int rows = (d.p[d.K - 1] - 1) / 2 + 1;   // k = 0..h of the largest prime
    const int mt = rows <= 16 ? 1 : rows <= 32 ? 2 : 0;
    return ntw && mt ? mt * 4 + ntw : 0;
}

}  // namespace sft
