// HIP kernels of the sparse Fourier transform hot path (gfx950, wave64).
//
//   k_gather    filtered samples S_b(x_k) for every node and band  (Algorithm 1, line 7;
//               Section 3.1, Lemma 10's 2 kappa + 1 nearest grid values)
//   k_dft       short DFTs of length P_j = s1 p_j (Appendix B) by Good-Thomas:
//               radix-2 over s1 in LDS, direct p-point over the prime, then the
//               top-T bins by |E|^2 (radix select), bucketed by residue class mod s1
//   k_identify  CRT candidates per residue class, majority vote over the K moduli,
//               componentwise median, per-band s-term, band test, division by ghat
//               (Algorithm 1, lines 9-11; Appendix B)
//   k_merge     global s-term over the bands (Algorithm 1, line 16)
//
// Every kernel runs 256-thread workgroups.  A launch covers one transform
// (BatchArgs::descs_many == nullptr) or a batch, where a per-signal block
// prefix maps blockIdx.x to (signal, local block).
#include <algorithm>

#include "sft_internal.h"

namespace sft {

// ----------------------------------------------------------------- helpers --

struct Where {
    int sig;
    int blk;
};

__device__ __forceinline__ Where locate(const BatchArgs& a) {
    Where w;
    const int b = (int)blockIdx.x;
    if (a.descs_many == nullptr) {
        w.sig = 0;
        w.blk = b;
        return w;
    }
    int lo = 0, hi = a.nsig - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.prefix[mid] <= b) lo = mid; else hi = mid - 1;
    }
    w.sig = lo;
    w.blk = b - a.prefix[lo];
    return w;
}

__device__ __forceinline__ const SigDesc* desc_of(const BatchArgs& a, int sig) {
    return a.descs_many ? a.descs_many[sig] : a.desc_one;
}

__device__ __forceinline__ IoDesc io_of(const BatchArgs& a, int sig) {
    return a.descs_many ? a.io_many[sig] : a.io_one;
}

__device__ __forceinline__ int64_t pos_mod(int64_t x, int64_t m) {
    int64_t r = x % m;
    return r < 0 ? r + m : r;
}

// Exclusive scan of data[0..n) (LDS) in place; returns the total.  scratch: int32[256].
__device__ int block_exclusive_scan(int32_t* data, int n, int32_t* scratch) {
    const int tid = threadIdx.x;
    const int chunk = (n + kThreads - 1) / kThreads;
    const int beg = min(n, tid * chunk);
    const int end = min(n, beg + chunk);
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += data[i];
    scratch[tid] = sum;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const int v = tid >= off ? scratch[tid - off] : 0;
        __syncthreads();
        scratch[tid] += v;
        __syncthreads();
    }
    int run = tid > 0 ? scratch[tid - 1] : 0;
    const int total = scratch[kThreads - 1];
    for (int i = beg; i < end; ++i) {
        const int v = data[i];
        data[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

// ------------------------------------------------------------ k_gather ----
// One thread per node (modulus j, PFA position n2 * s1 + n1); all Q bands.
// Node k = (n1 p + n2 s1) mod P_j sits at t = k N / P_j grid steps; its nearest
// grid index j' = floor((2 k N + P_j) / (2 P_j)) and offset u = (k N - j' P_j) / P_j
// are exact integer arithmetic with one rounding of u to FP32.
//   S_b = exp(2 pi i q_b u / N) * sum_i f[(j' + i) mod N] W(u - i) exp(-2 pi i q_b i / N)
// with W(v) = exp(-v^2 / (2 sigma_t^2)) / (2 pi sigma_t) (the periodized Gaussian
// divided by N, eq. Def_Periodic_Gaussian) and the second phasor from the plan's
// exact table.

__global__ void __launch_bounds__(kThreads) k_gather(BatchArgs a) {
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    if (at.blk == 0 && threadIdx.x == 0) io.status[0] = 0;
    const int g = at.blk * kThreads + (int)threadIdx.x;
    const int M = d->M;
    if (g >= M) return;
    const int K = d->K;
    int j = 0;
    while (j + 1 < K && g >= d->Moff[j + 1]) ++j;
    const int l = g - d->Moff[j];
    const int p = d->p[j];
    const int P = d->P[j];
    const int s1 = d->s1;
    const int n1 = l & (s1 - 1);
    const int n2 = l >> d->log2s1;
    const int n = (int)(((int64_t)n1 * p + (int64_t)n2 * s1) % P);
    const int64_t N = d->N;
    const int64_t nN = (int64_t)n * N;
    const int64_t jp = (2 * nN + P) / (2 * (int64_t)P);
    const int32_t delta = (int32_t)(nN - jp * P);
    const float Pf = (float)P;
    const float u = (float)delta / Pf;
    const int kappa = d->kappa;
    const int taps = d->taps;
    const int Q = d->Q;
    const float inv2sig2 = d->inv2sig2;
    const float wnorm = d->wnorm;
    const float2* __restrict__ f = io.f;
    float2* __restrict__ S = io.S + (size_t)Q * d->Moff[j] + l;
    const float* __restrict__ rate = d->rate;
    const bool interior = (jp - kappa >= 0) && (jp + kappa < N);

    for (int b0 = 0; b0 < Q; b0 += kBandChunk) {
        const int nb = min(kBandChunk, Q - b0);
        float2 acc[kBandChunk];
#pragma unroll
        for (int bb = 0; bb < kBandChunk; ++bb) acc[bb] = make_float2(0.f, 0.f);
        const float2* __restrict__ tab = d->bandtab + (size_t)b0 * taps;
        for (int i = 0; i < taps; ++i) {
            int64_t idx = jp - kappa + i;
            if (!interior) {
                if (idx < 0) idx += N;
                else if (idx >= N) idx -= N;
            }
            const float v = (float)(delta - (i - kappa) * P) / Pf;
            const float w = wnorm * expf(-v * v * inv2sig2);
            const float2 fv = f[idx];
            const float xr = fv.x * w;
            const float xi = fv.y * w;
#pragma unroll
            for (int bb = 0; bb < kBandChunk; ++bb) {
                if (bb < nb) {
                    const float2 t = tab[bb * taps + i];
                    acc[bb].x = fmaf(xr, t.x, fmaf(-xi, t.y, acc[bb].x));
                    acc[bb].y = fmaf(xr, t.y, fmaf(xi, t.x, acc[bb].y));
                }
            }
        }
#pragma unroll
        for (int bb = 0; bb < kBandChunk; ++bb) {
            if (bb < nb) {
                float sn, cs;
                sincospif(2.0f * u * rate[b0 + bb], &sn, &cs);
                const float2 r = make_float2(acc[bb].x * cs - acc[bb].y * sn,
                                             acc[bb].x * sn + acc[bb].y * cs);
                S[(size_t)(b0 + bb) * P] = r;
            }
        }
    }
}

// --------------------------------------------------------------- k_dft ----
// Short DFTs of length P = s1 p (Appendix B) by Good-Thomas.  The samples of
// block (modulus j, band b) arrive in Good-Thomas input order: row n2 holds the
// nodes (n1 p + n2 s1) mod P for n1 = 0..s1-1.  Then
//   step A: radix-2 FFT of length s1 along every row,
//   step B: direct p-point DFT along every column k1,
// give the bin h with h = k1 (mod s1), h = k2 (mod p) at k1 + s1 k2, scaled by 1/P.
// The T largest |E|^2 (ties to the lower h) are found by a radix select on
// distinct 64-bit keys (bits(|E|^2) << 32 | (2^32 - 1 - h)) and written sorted by
// (h mod s1, |E|^2 desc, h asc), with the offset of every residue class.
//
// k_dft holds a whole block in LDS.  Blocks too large for LDS take the split
// path: k_dft_rows (step A on a few rows), k_dft_cols (step B on 64 columns),
// k_select (the selection, reading E from global memory).

// Bit reversal and butterflies over `rows` rows of s1 complex values in LDS.
__device__ void fft_rows_lds(float2* buf, int rows, int s1, int lg, const float2* __restrict__ tw) {
    const int tid = (int)threadIdx.x;
    const int n = rows << lg;
    if (lg == 0) return;
    for (int i = tid; i < n; i += kThreads) {
        const int n1 = i & (s1 - 1);
        const int r = (int)(__brev((unsigned)n1) >> (32 - lg));
        if (n1 < r) {
            const int row = i - n1;
            const float2 t0 = buf[row + n1];
            buf[row + n1] = buf[row + r];
            buf[row + r] = t0;
        }
    }
    __syncthreads();
    const int half_n = n >> 1;
    for (int len = 2, ls = 1; len <= s1; len <<= 1, ++ls) {
        const int half = len >> 1;
        const int twstride = s1 >> ls;
        for (int i = tid; i < half_n; i += kThreads) {
            const int row = i >> (lg - 1);
            const int rr = i & ((s1 >> 1) - 1);
            const int grp = rr >> (ls - 1);
            const int pos = rr & (half - 1);
            const int i0 = (row << lg) + grp * len + pos;
            const int i1 = i0 + half;
            const float2 w = tw[pos * twstride];
            const float2 x0 = buf[i0];
            const float2 x1 = buf[i1];
            const float2 y = make_float2(x1.x * w.x - x1.y * w.y, x1.x * w.y + x1.y * w.x);
            buf[i0] = make_float2(x0.x + y.x, x0.y + y.y);
            buf[i1] = make_float2(x0.x - y.x, x0.y - y.y);
        }
        __syncthreads();
    }
}

// p-point DFT of column k1 at output row k2: sum_n2 col[n2 * stride] W_p^(n2 k2).
__device__ __forceinline__ float2 dft_p_point(const float2* col, int stride, int p, int k2,
                                              const float2* __restrict__ twp) {
    float ar = 0.f, ai = 0.f;
    int m = 0;
    for (int n2 = 0; n2 < p; ++n2) {
        const float2 x = col[n2 * stride];
        const float2 w = twp[m];
        ar = fmaf(x.x, w.x, fmaf(-x.y, w.y, ar));
        ai = fmaf(x.x, w.y, fmaf(x.y, w.x, ai));
        m += k2;
        if (m >= p) m -= p;
    }
    return make_float2(ar, ai);
}

__device__ __forceinline__ uint64_t bin_key(float2 e, int i, int lg, int s1, int P, int64_t cA, int64_t cB) {
    const float m2 = fmaf(e.x, e.x, e.y * e.y);
    const int k2 = i >> lg;
    const int k1 = i & (s1 - 1);
    const uint32_t h = (uint32_t)(((int64_t)k1 * cA + (int64_t)k2 * cB) % P);
    return ((uint64_t)__float_as_uint(m2) << 32) | (uint64_t)(0xffffffffu - h);
}

__device__ __forceinline__ bool cls_key_less(int32_t ca, uint64_t ka, int32_t cb, uint64_t kb) {
    return ca < cb || (ca == cb && ka > kb);
}

// Top-T of the P distinct keys key(i), written to H[T] sorted by (class, key
// desc) and Hoff[s1 + 1].  skey/scls: LDS [Tp]; hist: LDS [256].
template <class KeyF>
__device__ void select_heavy(KeyF key, int P, int T, int Tp, int s1, uint64_t* skey, int32_t* scls,
                             int32_t* hist, int32_t* __restrict__ H, int32_t* __restrict__ Hoff) {
    __shared__ int32_t sh_digit, sh_need, sh_count, sh_done;
    const int tid = (int)threadIdx.x;
    if (tid == 0) {
        sh_need = T;
        sh_done = 0;
        sh_count = 0;
    }
    __syncthreads();
    uint64_t prefix = 0, pmask = 0;
    for (int shift = 56; shift >= 0 && T > 0 && T < P; shift -= 8) {
        for (int i = tid; i < 256; i += kThreads) hist[i] = 0;
        __syncthreads();
        for (int i = tid; i < P; i += kThreads) {
            const uint64_t k = key(i);
            if ((k & pmask) == prefix) atomicAdd(&hist[(int)((k >> shift) & 255u)], 1);
        }
        __syncthreads();
        if (tid == 0) {
            int need = sh_need, cum = 0, dsel = 0;
            for (int dg = 255; dg >= 0; --dg) {
                if (cum + hist[dg] >= need) {
                    dsel = dg;
                    break;
                }
                cum += hist[dg];
            }
            sh_digit = dsel;
            sh_need = need - cum;
            sh_done = (hist[dsel] == need - cum) ? 1 : 0;
        }
        __syncthreads();
        prefix |= (uint64_t)sh_digit << shift;
        pmask |= (uint64_t)255u << shift;
        const int done = sh_done;
        __syncthreads();
        if (done) break;
    }
    const uint64_t thr = (T >= P) ? 0ull : prefix;   // the selected keys are those >= thr
    if (T > 0) {
        for (int i = tid; i < P; i += kThreads) {
            const uint64_t k = key(i);
            if (k >= thr) {
                const int pos = atomicAdd(&sh_count, 1);
                if (pos < Tp) {
                    const uint32_t h = 0xffffffffu - (uint32_t)(k & 0xffffffffu);
                    skey[pos] = k;
                    scls[pos] = (int32_t)(h & (uint32_t)(s1 - 1));
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < Tp; i += kThreads) {
        if (i >= T) {
            skey[i] = 0;
            scls[i] = 0x7fffffff;
        }
    }
    __syncthreads();
    for (int kk = 2; kk <= Tp; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int i = tid; i < Tp; i += kThreads) {
                const int ixj = i ^ jj;
                if (ixj > i) {
                    const bool up = (i & kk) == 0;
                    const int32_t ci = scls[i], cx = scls[ixj];
                    const uint64_t ki = skey[i], kx = skey[ixj];
                    const bool sw = up ? cls_key_less(cx, kx, ci, ki) : cls_key_less(ci, ki, cx, kx);
                    if (sw) {
                        scls[i] = cx;
                        scls[ixj] = ci;
                        skey[i] = kx;
                        skey[ixj] = ki;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < T; i += kThreads) H[i] = (int32_t)(0xffffffffu - (uint32_t)(skey[i] & 0xffffffffu));
    for (int c = tid; c <= s1; c += kThreads) {
        int lo = 0, hi = T;   // first index with class >= c
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (scls[mid] < c) lo = mid + 1; else hi = mid;
        }
        Hoff[c] = lo;
    }
}

// One workgroup per (modulus j, band b); the whole block in LDS.
__global__ void __launch_bounds__(kThreads) k_dft(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int K = d->K;
    const int j = at.blk / Q;
    const int b = at.blk - j * Q;
    const int p = d->p[j];
    const int P = d->P[j];
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int Tp = d->Tpow2;
    const int Pmax = d->P[K - 1];
    const size_t base = (size_t)Q * d->Moff[j] + (size_t)b * P;

    float2* buf = reinterpret_cast<float2*>(smem);
    uint64_t* keys = reinterpret_cast<uint64_t*>(smem);
    uint64_t* skey = reinterpret_cast<uint64_t*>(smem + (size_t)Pmax * 8);
    int32_t* scls = reinterpret_cast<int32_t*>(smem + (size_t)Pmax * 8 + (size_t)Tp * 8);
    int32_t* hist = reinterpret_cast<int32_t*>(smem + (size_t)Pmax * 8 + (size_t)Tp * 12);

    const float2* __restrict__ S = io.S + base;
    for (int i = tid; i < P; i += kThreads) buf[i] = S[i];
    __syncthreads();
    fft_rows_lds(buf, p, s1, lg, d->tw_s1);

    // step B; the keys below re-read E: same workgroup, ordered by the barrier
    float2* __restrict__ E = io.E + base;
    const float2* __restrict__ twp = d->tw_p + d->tw_off[j];
    const float invP = 1.0f / (float)P;
    for (int i = tid; i < P; i += kThreads) {
        const int k2 = i >> lg;
        const int k1 = i & (s1 - 1);
        const float2 e = dft_p_point(buf + k1, s1, p, k2, twp);
        E[i] = make_float2(e.x * invP, e.y * invP);
    }
    __syncthreads();
    const int64_t cA = (int64_t)p * d->pinv_s1[j];
    const int64_t cB = (int64_t)s1 * d->s1inv_p[j];
    for (int i = tid; i < P; i += kThreads) keys[i] = bin_key(E[i], i, lg, s1, P, cA, cB);
    __syncthreads();
    select_heavy([&](int i) { return keys[i]; }, P, d->T, Tp, s1, skey, scls, hist,
                 io.H + (size_t)(j * Q + b) * d->T, io.Hoff + (size_t)(j * Q + b) * (s1 + 1));
}

// Split path, step A: block -> (modulus j, band b, chunk of rows_per rows).
__device__ __forceinline__ void split_rows_where(const SigDesc* d, int blk, int rows_per, int& j, int& b, int& chunk) {
    const int Q = d->Q;
    j = 0;
    for (;;) {
        const int nch = (d->p[j] + rows_per - 1) / rows_per;
        if (blk < Q * nch || j + 1 >= d->K) {
            b = blk / nch;
            chunk = blk - b * nch;
            return;
        }
        blk -= Q * nch;
        ++j;
    }
}

__global__ void __launch_bounds__(kThreads) k_dft_rows(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int rows_per = max(1, kRowElems >> lg);
    int j, b, chunk;
    split_rows_where(d, at.blk, rows_per, j, b, chunk);
    const int p = d->p[j];
    const int r0 = chunk * rows_per;
    const int rows = min(rows_per, p - r0);
    const size_t base = (size_t)d->Q * d->Moff[j] + (size_t)b * d->P[j] + ((size_t)r0 << lg);
    float2* buf = reinterpret_cast<float2*>(smem);
    const int n = rows << lg;
    const float2* __restrict__ S = io.S + base;
    for (int i = tid; i < n; i += kThreads) buf[i] = S[i];
    __syncthreads();
    fft_rows_lds(buf, rows, s1, lg, d->tw_s1);
    float2* __restrict__ X = io.E + base;   // the bins' buffer holds the step-A result
    for (int i = tid; i < n; i += kThreads) X[i] = buf[i];
}

// Split path, step B: block -> (modulus j, band b, 64 columns); in place on E.
__global__ void __launch_bounds__(kThreads) k_dft_cols(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int C = min(kColChunk, s1);
    const int nc = s1 / C;
    int blk = at.blk;
    const int j = blk / (Q * nc);
    blk -= j * Q * nc;
    const int b = blk / nc;
    const int c0 = (blk - b * nc) * C;
    const int p = d->p[j];
    const int P = d->P[j];
    const size_t base = (size_t)Q * d->Moff[j] + (size_t)b * P;
    float2* tile = reinterpret_cast<float2*>(smem);   // [p][C]
    float2* __restrict__ E = io.E + base;
    for (int i = tid; i < p * C; i += kThreads) {
        const int n2 = i / C;
        const int k1 = c0 + (i - n2 * C);
        tile[i] = E[((size_t)n2 << lg) + k1];
    }
    __syncthreads();
    const float2* __restrict__ twp = d->tw_p + d->tw_off[j];
    const float invP = 1.0f / (float)P;
    for (int i = tid; i < p * C; i += kThreads) {
        const int k2 = i / C;
        const int kc = i - k2 * C;
        const float2 e = dft_p_point(tile + kc, C, p, k2, twp);
        E[((size_t)k2 << lg) + c0 + kc] = make_float2(e.x * invP, e.y * invP);
    }
}

// Split path, selection: one workgroup per (modulus j, band b), E in global memory.
__global__ void __launch_bounds__(kThreads) k_select(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int Q = d->Q;
    const int j = at.blk / Q;
    const int b = at.blk - j * Q;
    const int p = d->p[j];
    const int P = d->P[j];
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int Tp = d->Tpow2;
    uint64_t* skey = reinterpret_cast<uint64_t*>(smem);
    int32_t* scls = reinterpret_cast<int32_t*>(smem + (size_t)Tp * 8);
    int32_t* hist = reinterpret_cast<int32_t*>(smem + (size_t)Tp * 12);
    const float2* __restrict__ E = io.E + (size_t)Q * d->Moff[j] + (size_t)b * P;
    const int64_t cA = (int64_t)p * d->pinv_s1[j];
    const int64_t cB = (int64_t)s1 * d->s1inv_p[j];
    select_heavy([&](int i) { return bin_key(E[i], i, lg, s1, P, cA, cB); }, P, d->T, Tp, s1, skey, scls, hist,
                 io.H + (size_t)(j * Q + b) * d->T, io.Hoff + (size_t)(j * Q + b) * (s1 + 1));
}

// ---------------------------------------------------------- k_identify ----
// One workgroup per band b.  Candidates: in CRT tuple t and residue class a,
// one of the `depth` heaviest class-a bins of every modulus of the tuple;
// w = a (mod s1), w = h_g (mod p_g) by the CRT in int64, mapped into B.
// Vote ("more than half", Appendix B): the tuple's own G moduli hold heavy bins
// at w by construction, so (w mod P_j) must be a heavy bin for more than half of
// the other K - G moduli.  A w produced by both tuples is accepted if either
// tuple's vote passes (the two entries are equal and merged later).  Estimate:
// componentwise median of E_b[j][w mod P_j] over all K moduli.  Then the s
// largest |z| (ties to the smaller w), the band test w in [q_b - L, q_b + L),
// and v = z / ghat_{w - q_b} in FP64.

__device__ __forceinline__ float median_of(const float* v, int K) {
    float med = 0.f;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) {
        if (i < K) {
            int rank = 0;
#pragma unroll
            for (int k = 0; k < kMaxK; ++k) {
                if (k < K) rank += (v[k] < v[i]) || (v[k] == v[i] && k < i);
            }
            if (rank == (K >> 1)) med = v[i];
        }
    }
    return med;
}

__global__ void __launch_bounds__(kThreads) k_identify(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int b = at.blk;
    const int Q = d->Q;
    const int K = d->K;
    const int G = d->G;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int T = d->T;
    const int depth = d->depth;
    const int64_t lo = d->lo, hi = d->hi;
    const int nslots = 2 * s1;

    uint64_t* akey = reinterpret_cast<uint64_t*>(smem);
    float2* az = reinterpret_cast<float2*>(smem + (size_t)kAcceptCap * 8);
    int32_t* flag = reinterpret_cast<int32_t*>(smem + (size_t)kAcceptCap * 16);
    int32_t* scratch = flag + kAcceptCap;
    int32_t* pre = scratch + kThreads;
    __shared__ int32_t sh_cnt;

    const int32_t* __restrict__ Hall = io.H;
    const int32_t* __restrict__ Hoffall = io.Hoff;
    const float2* __restrict__ Eall = io.E;

    // 1. combinations per (tuple, class) slot
    for (int slot = tid; slot < nslots; slot += kThreads) {
        const int t = slot >> lg;
        const int ac = slot & (s1 - 1);
        int cnt = 1;
        for (int g = 0; g < G; ++g) {
            const int jj = d->tup_j[t][g];
            const int32_t* hb = Hoffall + (size_t)(jj * Q + b) * (s1 + 1);
            cnt *= min(depth, hb[ac + 1] - hb[ac]);
        }
        pre[slot] = cnt;
    }
    if (tid == 0) sh_cnt = 0;
    __syncthreads();
    const int total = block_exclusive_scan(pre, nslots, scratch);
    if (tid == 0) pre[nslots] = total;
    __syncthreads();

    // 2. candidates -> vote -> median
    for (int c = tid; c < total; c += kThreads) {
        int l0 = 0, h0 = nslots - 1;   // last slot with pre[slot] <= c
        while (l0 < h0) {
            const int mid = (l0 + h0 + 1) >> 1;
            if (pre[mid] <= c) l0 = mid; else h0 = mid - 1;
        }
        const int slot = l0;
        int r = c - pre[slot];
        const int t = slot >> lg;
        const int ac = slot & (s1 - 1);
        int64_t x = (int64_t)((ac * (int64_t)d->tup_inv[t][0]) % s1) * d->tup_Mi[t][0];
        for (int g = 0; g < G; ++g) {
            const int jj = d->tup_j[t][g];
            const int32_t* hb = Hoffall + (size_t)(jj * Q + b) * (s1 + 1);
            const int cg = min(depth, hb[ac + 1] - hb[ac]);
            const int ch = r % cg;
            r /= cg;
            const int32_t h = Hall[(size_t)(jj * Q + b) * T + hb[ac] + ch];
            const int pm = d->tup_mod[t][g + 1];
            const int64_t res = h % pm;
            x += ((res * d->tup_inv[t][g + 1]) % pm) * d->tup_Mi[t][g + 1];
        }
        const int64_t Mt = d->tup_M[t];
        x %= Mt;
        int64_t w;
        if (x <= hi) w = x;
        else if (x - Mt >= lo) w = x - Mt;
        else continue;

        float er[kMaxK], ei[kMaxK];
        int votes = 0;                 // heavy bins among the moduli outside tuple t
        const int t_lo = t * G, t_hi = t_lo + G;
#pragma unroll
        for (int jj = 0; jj < kMaxK; ++jj) {
            if (jj < K) {
                const int Pj = d->P[jj];
                const int hh = (int)pos_mod(w, Pj);
                const int cls = hh & (s1 - 1);
                const int32_t* hb = Hoffall + (size_t)(jj * Q + b) * (s1 + 1);
                const int32_t* Hb = Hall + (size_t)(jj * Q + b) * T;
                const int e0 = hb[cls], e1 = hb[cls + 1];
                bool hit = false;
                for (int e = e0; e < e1; ++e) hit |= (Hb[e] == hh);
                votes += (hit && (jj < t_lo || jj >= t_hi)) ? 1 : 0;
                const int k2 = hh % d->p[jj];
                const float2 ev = Eall[(size_t)Q * d->Moff[jj] + (size_t)b * Pj + ((size_t)k2 << lg) + cls];
                er[jj] = ev.x;
                ei[jj] = ev.y;
            }
        }
        if (2 * votes > K - G) {
            const float zr = median_of(er, K);
            const float zi = median_of(ei, K);
            const float m2 = fmaf(zr, zr, zi * zi);
            const int pos = atomicAdd(&sh_cnt, 1);
            if (pos < kAcceptCap) {
                akey[pos] = ((uint64_t)__float_as_uint(m2) << 32) |
                            (uint64_t)(0xffffffffu - (uint32_t)(w - lo));
                az[pos] = make_float2(zr, zi);
            } else {
                atomicOr(io.status, kStatusAcceptOverflow);
            }
        }
    }
    __syncthreads();
    const int nacc = min(sh_cnt, kAcceptCap);
    int np2 = 1;
    while (np2 < nacc) np2 <<= 1;
    for (int i = nacc + tid; i < np2; i += kThreads) {
        akey[i] = 0;
        az[i] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    // 3. sort accepted by key descending (|z|^2 desc, w asc)
    for (int kk = 2; kk <= np2; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int i = tid; i < np2; i += kThreads) {
                const int ixj = i ^ jj;
                if (ixj > i) {
                    const bool desc = (i & kk) == 0;
                    const uint64_t ki = akey[i], kx = akey[ixj];
                    if (desc ? (kx > ki) : (kx < ki)) {
                        akey[i] = kx;
                        akey[ixj] = ki;
                        const float2 zt = az[i];
                        az[i] = az[ixj];
                        az[ixj] = zt;
                    }
                }
            }
            __syncthreads();
        }
    }
    // 4. distinct entries, the first s of them (R_temp), then the band test
    for (int i = tid; i < nacc; i += kThreads) flag[i] = (i == 0 || akey[i] != akey[i - 1]) ? 1 : 0;
    __syncthreads();
    block_exclusive_scan(flag, nacc, scratch);   // for a distinct entry: its rank among distinct ones
    const int64_t q = d->q_first + 2 * (int64_t)b * d->L;
    const int s = d->s;
    int64_t* __restrict__ Rw = io.Rw + (size_t)b * s;
    double2* __restrict__ Rv = io.Rv + (size_t)b * s;
    // in-band results are written in sorted order by a serial pass of wave 0
    if (tid < 64) {
        int outc = 0;
        for (int base = 0; base < nacc; base += 64) {
            const int i = base + tid;
            bool take = false;
            int64_t w = 0;
            if (i < nacc) {
                const bool distinct = (i == 0 || akey[i] != akey[i - 1]);
                if (distinct && flag[i] < s) {
                    w = lo + (int64_t)(0xffffffffu - (uint32_t)(akey[i] & 0xffffffffu));
                    take = (w >= q - d->L) && (w < q + d->L) && (w >= lo) && (w <= hi);
                }
            }
            const uint64_t ballot = __ballot(take);
            const int before = __popcll(ballot & ((1ull << tid) - 1ull));
            if (take) {
                const int o = outc + before;
                const double n = (double)(w - q);
                const double gh = d->ghat0 * exp(-d->c1sq_half * n * n);
                const float2 z = az[i];
                Rw[o] = w;
                Rv[o] = make_double2((double)z.x / gh, (double)z.y / gh);
            }
            outc += __popcll(ballot);
        }
        if (tid == 0) io.Rn[b] = outc;
    }
}

// ------------------------------------------------------------- k_merge ----
// One workgroup per transform: the s largest |v| over all bands (ties to the
// smaller w), written in that order; unfilled slots get w = 0, c = 0.

__device__ __forceinline__ bool merge_before(double ma, int64_t wa, double mb, int64_t wb) {
    return ma > mb || (ma == mb && wa < wb);
}

__global__ void __launch_bounds__(kThreads) k_merge(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const SigDesc* __restrict__ d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int s = d->s;
    double* mm = reinterpret_cast<double*>(smem);
    int64_t* ww = reinterpret_cast<int64_t*>(smem + (size_t)kMergeCap * 8);
    int32_t* src = reinterpret_cast<int32_t*>(smem + (size_t)kMergeCap * 16);
    int32_t* off = src + kMergeCap;
    int32_t* scratch = off + SFT_MAX_BANDS + 1;

    for (int bb = tid; bb < Q; bb += kThreads) off[bb] = io.Rn[bb];
    __syncthreads();
    const int total = block_exclusive_scan(off, Q, scratch);
    const int n = min(total, kMergeCap);
    if (tid == 0 && total > kMergeCap) atomicOr(io.status, kStatusMergeOverflow);
    for (int bb = 0; bb < Q; ++bb) {
        const int cnt = io.Rn[bb];
        const int o = off[bb];
        for (int k = tid; k < cnt; k += kThreads) {
            const int dst = o + k;
            if (dst < n) {
                const double2 v = io.Rv[(size_t)bb * s + k];
                mm[dst] = v.x * v.x + v.y * v.y;
                ww[dst] = io.Rw[(size_t)bb * s + k];
                src[dst] = bb * s + k;
            }
        }
    }
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int i = n + tid; i < np2; i += kThreads) {
        mm[i] = -1.0;
        ww[i] = 0;
        src[i] = -1;
    }
    __syncthreads();
    for (int kk = 2; kk <= np2; kk <<= 1) {
        for (int jj = kk >> 1; jj > 0; jj >>= 1) {
            for (int i = tid; i < np2; i += kThreads) {
                const int ixj = i ^ jj;
                if (ixj > i) {
                    const bool up = (i & kk) == 0;
                    const double mi = mm[i], mx = mm[ixj];
                    const int64_t wi = ww[i], wx = ww[ixj];
                    const bool sw = up ? merge_before(mx, wx, mi, wi) : merge_before(mi, wi, mx, wx);
                    if (sw) {
                        mm[i] = mx;
                        mm[ixj] = mi;
                        ww[i] = wx;
                        ww[ixj] = wi;
                        const int32_t t = src[i];
                        src[i] = src[ixj];
                        src[ixj] = t;
                    }
                }
            }
            __syncthreads();
        }
    }
    const int nout = min(n, s);
    for (int r = tid; r < s; r += kThreads) {
        if (r < nout) {
            const double2 v = io.Rv[src[r]];
            io.out_w[r] = ww[r];
            io.out_c[r] = make_float2((float)v.x, (float)v.y);
        } else {
            io.out_w[r] = 0;
            io.out_c[r] = make_float2(0.f, 0.f);
        }
    }
    if (tid == 0 && io.out_n) io.out_n[0] = nout;
}

// ------------------------------------------------------------ launchers ---

size_t identify_lds_bytes(const SigDesc& d) {
    return (size_t)kAcceptCap * 20 + (size_t)kThreads * 4 + (size_t)(2 * d.s1 + 1) * 4 + 64;
}

size_t merge_lds_bytes() {
    return (size_t)kMergeCap * 20 + (SFT_MAX_BANDS + 1) * 4 + kThreads * 4 + 64;
}

int gather_blocks(const SigDesc& d) { return (d.M + kThreads - 1) / kThreads; }
int dft_blocks(const SigDesc& d) { return d.K * d.Q; }
int identify_blocks(const SigDesc& d) { return d.Q; }
int merge_blocks(const SigDesc&) { return 1; }

int rows_blocks(const SigDesc& d) {
    const int rows_per = std::max(1, kRowElems >> d.log2s1);
    int n = 0;
    for (int j = 0; j < d.K; ++j) n += d.Q * ((d.p[j] + rows_per - 1) / rows_per);
    return n;
}
int cols_blocks(const SigDesc& d) { return d.K * d.Q * (d.s1 / std::min(kColChunk, d.s1)); }
int select_blocks(const SigDesc& d) { return d.K * d.Q; }

size_t rows_lds_bytes(const SigDesc& d) {
    const int rows_per = std::max(1, kRowElems >> d.log2s1);
    return (size_t)rows_per * d.s1 * 8;
}
size_t cols_lds_bytes(const SigDesc& d) {
    int pmax = 0;
    for (int j = 0; j < d.K; ++j) pmax = std::max(pmax, d.p[j]);
    return (size_t)pmax * std::min(kColChunk, d.s1) * 8;
}
size_t select_lds_bytes(const SigDesc& d) { return (size_t)d.Tpow2 * 12 + 256 * 4 + 64; }

// Dynamic LDS above 64 KiB: raise each kernel's limit where the runtime asks
// for an opt-in.  A rejected request is not an error here: the launch itself
// reports a size the device cannot hold.
hipError_t configure_kernels(int max_lds) {
    const void* ks[6] = {(const void*)k_dft, (const void*)k_identify, (const void*)k_merge,
                         (const void*)k_dft_rows, (const void*)k_dft_cols, (const void*)k_select};
    for (const void* k : ks) {
        hipFuncAttributes fa;
        int static_lds = 0;
        if (hipFuncGetAttributes(&fa, k) == hipSuccess) static_lds = (int)fa.sharedSizeBytes;
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - static_lds) != hipSuccess)
            (void)hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_gather(const BatchArgs& a, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(blocks), dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_dft(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_dft, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dft_rows(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_dft_rows, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dft_cols(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_dft_cols, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_select(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_select, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_identify(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_identify, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_merge(const BatchArgs& a, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_merge, dim3(blocks), dim3(kThreads), merge_lds_bytes(), st, a);
    return hipGetLastError();
}

}  // namespace sft
