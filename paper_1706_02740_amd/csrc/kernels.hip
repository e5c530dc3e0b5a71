// HIP kernels of the sparse Fourier transform hot path (gfx950, wave64).
//
//   k_gather    filtered samples S_b(x_k) for every node and band  (Algorithm 1, convolution step;
//               Section 3.1, Lemma 10's 2 kappa + 1 nearest grid values)
//   k_dft       short DFTs of length P_j = s1 p_j (Appendix B) by Good-Thomas, a
//               whole block in LDS: s1-point row FFTs, the p-point step on the
//               matrix cores (k_dft<0, true>) or the vector ALUs, then the top-T
//               bins by |E|^2 (radix select), bucketed by residue class mod s1
//   k_dft_rows, k_dft_cols, k_dft_cols_mx, k_select
//               the same for blocks larger than the LDS, in three steps over HBM
//   k_identify  candidates per residue class (CRT) or from bin phases, majority
//               vote, componentwise median, per-band s-term, band test, division
//               by ghat (Algorithm 1: inner sparse FFT, band test, division; Appendix B)
//   k_merge     global s-term over the bands (Algorithm 1, last step)
//
// Workgroups have 256 threads, except k_dft and k_dft_cols_mx (512), the
// LDS-key form of k_select and k_identify in launches of few bands (1024).  A launch covers one transform
// (BatchArgs::io_many == nullptr) or a batch, where a per-signal block prefix
// (or, for a batch of one plan, a division) maps blockIdx.x to (signal, local
// block).  A k_dft launch may cover a range of the moduli only.
#include <algorithm>
#include <mutex>

#include "sft_internal.h"

namespace sft {

// ----------------------------------------------------------------- helpers --

// Pointers read out of descriptors are generic; these casts restore their
// address space so that wave-uniform reads become scalar (constant) loads and
// data accesses use global (not flat) instructions.
#define GLOBAL __attribute__((address_space(1)))
#define CONSTANT __attribute__((address_space(4)))

template <class T>
__device__ __forceinline__ const CONSTANT T* cst(const T* p) { return (const CONSTANT T*)(p); }
template <class T>
__device__ __forceinline__ const GLOBAL T* glb(const T* p) { return (const GLOBAL T*)(p); }
template <class T>
__device__ __forceinline__ GLOBAL T* glb(T* p) { return (GLOBAL T*)(p); }

// float2 / double2 are classes whose copies take generic references: address-
// space-qualified element accesses go through these POD vector loads/stores.
typedef float pod_f2 __attribute__((ext_vector_type(2)));
typedef double pod_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld2(const GLOBAL float2* p) {
    const pod_f2 v = *(const GLOBAL pod_f2*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ float2 ld2(const CONSTANT float2* p) {
    const pod_f2 v = *(const CONSTANT pod_f2*)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2(GLOBAL float2* p, float2 v) {
    pod_f2 w;
    w.x = v.x;
    w.y = v.y;
    *(GLOBAL pod_f2*)p = w;
}
// Streaming store: data written once and read once later by another kernel
// (samples, bins), kept from displacing reusable lines in the caches.
__device__ __forceinline__ void st2s(GLOBAL float2* p, float2 v) {
    pod_f2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (GLOBAL pod_f2*)p);
}
// a * b with both multiply-adds spelled out: every kernel that inlines it
// rounds the same way (no contraction left to the compiler's choice), which
// keeps the kernels that must agree bit for bit in agreement.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}

typedef float pod_f4 __attribute__((ext_vector_type(4)));
typedef int pod_i4 __attribute__((ext_vector_type(4)));

// Copies n float2 (n even, both ends 16-byte aligned) from global memory into
// LDS, 16 bytes per access, with U accesses of a thread in flight before its
// first LDS write (a plain loop would wait for each load in turn).
template <int NT, int U>
__device__ __forceinline__ void copy_to_lds(float2* dst, const GLOBAL float2* src, int n) {
    const int n4 = n >> 1;
    const GLOBAL pod_f4* s4 = (const GLOBAL pod_f4*)src;
    pod_f4* d4 = (pod_f4*)dst;
    for (int i0 = (int)threadIdx.x; i0 < n4; i0 += U * NT) {
        pod_f4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * NT;
            if (i < n4) v[u] = __builtin_nontemporal_load(s4 + i);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * NT;
            if (i < n4) d4[i] = v[u];
        }
    }
}

__device__ __forceinline__ double2 ldd2(const GLOBAL double2* p) {
    const pod_d2 v = *(const GLOBAL pod_d2*)p;
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void std2(GLOBAL double2* p, double2 v) {
    pod_d2 w;
    w.x = v.x;
    w.y = v.y;
    *(GLOBAL pod_d2*)p = w;
}

struct Where {
    int sig;
    int blk;
};

__device__ __forceinline__ Where locate(const BatchArgs& a) {
    Where w;
    const int b = (int)blockIdx.x;
    if (a.io_many == nullptr) {
        w.sig = 0;
        w.blk = b;
        return w;
    }
    if (a.bps > 0) {
        w.sig = b / a.bps;
        w.blk = b - w.sig * a.bps;
        return w;
    }
    const CONSTANT int32_t* pre = cst(a.prefix);
    int lo = 0, hi = a.nsig - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= b) lo = mid; else hi = mid - 1;
    }
    w.sig = lo;
    w.blk = b - pre[lo];
    return w;
}

__device__ __forceinline__ const CONSTANT SigDesc* desc_of(const BatchArgs& a, int sig) {
    return cst(a.descs_many ? cst(a.descs_many)[sig] : a.desc_one);
}

__device__ __forceinline__ IoDesc io_of(const BatchArgs& a, int sig) {
    if (a.io_many == nullptr) return a.io_one;
    IoDesc io;
    __builtin_memcpy(&io, (const IoDesc*)(cst(a.io_many) + sig), sizeof(IoDesc));
    return io;
}

__device__ __forceinline__ int64_t pos_mod(int64_t x, int64_t m) {
    int64_t r = x % m;
    return r < 0 ? r + m : r;
}

// Sum of the wave totals part[0..wid) (NT / 64 LDS values, read together).
template <int NT>
__device__ __forceinline__ int waves_before(const int32_t* part, int wid) {
    int base = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int v = part[w];
        base += w < wid ? v : 0;
    }
    return base;
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP: shifts by 1, 2,
// 4, 8 within each row of 16 lanes, then the row totals broadcast to the
// following rows (lane 15 to rows 1 and 3, lane 31 to rows 2 and 3).  Every
// lane of the wave must be active.
__device__ __forceinline__ int wave_inclusive_sum(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return x;
}

// Exclusive scan of data[0..n) (LDS) in place for a kThreads workgroup;
// returns the total.  Each thread scans a contiguous chunk; the chunk sums are
// scanned by wave shuffles and one exchange of the wave totals.
// scratch: int32[kThreads / 64].
template <int NT = kThreads>
__device__ int block_exclusive_scan(int32_t* data, int n, int32_t* scratch) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int chunk = (n + NT - 1) / NT;
    const int beg = min(n, tid * chunk);
    const int end = min(n, beg + chunk);
    int sum = 0;
    for (int i = beg; i < end; ++i) sum += data[i];
    const int x = wave_inclusive_sum(sum);
    if (lane == 63) scratch[wid] = x;
    __syncthreads();
    int base = 0, total = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int v = scratch[w];
        base += w < wid ? v : 0;
        total += v;
    }
    int run = base + x - sum;
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
// exact table.  The phasors of taps i and -i are conjugate, so the sum takes
// the taps in pairs (four FMAs per pair and band instead of eight; the
// table's entries for i < 0 are not read).  The node phasors
// exp(2 pi i q_b u / N) follow q_{b+1} - q_b = 2L:
// evaluated directly every kPhaseAnchor bands and by one complex product per
// band in between.  TAPS > 0 fixes 2 kappa + 1 at compile time (the window is
// loaded before any arithmetic); TAPS == 0 reads it from the plan.  Both forms
// perform the same operations in the same order, so their results are equal.
// Phase identification also needs the samples at the node moved one grid step
// (t + 1): the window centre moves to j' + 1 and u stays, so a second pass
// with the same weights writes them to S2.

constexpr int kPhaseAnchor = 8;

typedef float mf4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_bands(GLOBAL float2* __restrict__ S, int P, int b0, int nb, const float2* acc,
                                            float u, const CONSTANT float* rate, float step_rate) {
    float sn, cs;
    sincospif(2.0f * u * step_rate, &sn, &cs);
    const float2 step = make_float2(cs, sn);
    float2 ph = make_float2(1.f, 0.f);
#pragma unroll
    for (int bb = 0; bb < kBandChunk; ++bb) {
        if (bb < nb) {
            if (((b0 + bb) % kPhaseAnchor) == 0) {
                sincospif(2.0f * u * rate[b0 + bb], &sn, &cs);
                ph = make_float2(cs, sn);
            } else {
                ph = cmul(ph, step);
            }
            st2s(S + (size_t)(b0 + bb) * P, cmul(acc[bb], ph));
        }
    }
}

template <int TAPS>
__global__ void __launch_bounds__(kThreads) k_gather(BatchArgs a) {
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    if (at.blk == 0 && threadIdx.x == 0) glb(io.status)[0] = 0;
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
    int n = n1 * p + n2 * s1;   // < 2 P
    if (n >= P) n -= P;
    const int64_t N = d->N;
    const int64_t nN = (int64_t)n * N;
    // jp = floor((2 n N + P) / (2 P)): a double quotient, corrected to the exact floor
    const int64_t num = 2 * nN + P, den = 2 * (int64_t)P;
    int64_t jp = (int64_t)((double)num / (double)den);
    const int64_t rem = num - jp * den;
    if (rem < 0) --jp;
    else if (rem >= den) ++jp;
    const int32_t delta = (int32_t)(nN - jp * P);
    const float Pf = (float)P;
    const float u = (float)delta / Pf;
    const int kappa = TAPS > 0 ? (TAPS - 1) / 2 : d->kappa;
    const int taps = TAPS > 0 ? TAPS : d->taps;
    const int Q = d->Q;
    const float inv2sig2 = d->inv2sig2;
    const float wnorm = d->wnorm;
    const GLOBAL float2* __restrict__ f = glb(io.f);
    const size_t soff = (size_t)Q * d->Moff[j] + l;
    const CONSTANT float* rate = cst(d->rate);
    const float step_rate = d->a_step;
    const int nshift = d->phase;   // 0, or 1: also the node moved one grid step

    if constexpr (TAPS > 0) {
        static_assert(TAPS <= kFastTaps, "tap table");
        constexpr int KP = (TAPS - 1) / 2;
        // W((delta - o P) / P) = wnorm exp(-(u - o)^2 c), o = i - kappa, c = inv2sig2,
        //   = [wnorm exp(-u^2 c)] [exp(-o^2 c)] r^o,  r = exp(2 u c)
        const float e0 = wnorm * expf(-u * u * inv2sig2);
        const float r = expf(2.0f * u * inv2sig2);
        const float ri = expf(-2.0f * u * inv2sig2);
        float w[TAPS];
        w[KP] = e0 * d->gtap[KP];
        float rp = 1.0f, rn = 1.0f;
#pragma unroll
        for (int o = 1; o <= KP; ++o) {
            rp *= r;
            rn *= ri;
            w[KP + o] = e0 * d->gtap[KP + o] * rp;
            w[KP - o] = e0 * d->gtap[KP - o] * rn;
        }
        // f is 8-byte aligned; ab = 1 when it is not 16-byte aligned (element
        // e then starts a 16-byte piece iff e is odd)
        const int64_t ab = (int64_t)(((uintptr_t)io.f >> 3) & 1);
        for (int sh = 0;; ++sh) {
        const int64_t jc = jp + sh;   // window centre
        GLOBAL float2* __restrict__ S = glb(sh ? io.S2 : io.S) + soff;
        float2 x[TAPS];
        const int64_t st0 = jc - kappa;
        const int64_t par = (st0 + ab) & 1;   // the window's first element is the upper half of its piece
        if ((st0 - par >= 0) && (st0 + TAPS < N)) {
            // the window in 16-byte-aligned pieces from the piece holding its
            // first element: (TAPS + 1) / 2 loads, none crossing a 16-byte
            // boundary, all within the window's lines (the extra value shares a
            // piece with the first or the last tap); then a shift by the start's parity
            const GLOBAL pod_f4* w4 = (const GLOBAL pod_f4*)(f + (st0 - par));
            static_assert(TAPS & 1, "2 kappa + 1 taps");
            float2 c[TAPS + 1];
#pragma unroll
            for (int i = 0; i < TAPS + 1; i += 2) {
                const pod_f4 v = w4[i >> 1];   // plain loads: a thread's next load reads the same line
                c[i] = make_float2(v.x, v.y);
                c[i + 1] = make_float2(v.z, v.w);
            }
            // select by bit masks (a conditional select of c[i] and c[i + 1]
            // may become an indexed access that puts c in scratch memory)
            const uint32_t m = 0u - (uint32_t)par;
#pragma unroll
            for (int i = 0; i < TAPS; ++i) {   // in place: c[i + 1] is read before it is replaced
                c[i].x = __uint_as_float((__float_as_uint(c[i].x) & ~m) | (__float_as_uint(c[i + 1].x) & m));
                c[i].y = __uint_as_float((__float_as_uint(c[i].y) & ~m) | (__float_as_uint(c[i + 1].y) & m));
                x[i] = c[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < TAPS; ++i) {
                int64_t idx = jc - kappa + i;
                if (idx < 0) idx += N;
                else if (idx >= N) idx -= N;
                x[i] = ld2(f + idx);
            }
        }
#pragma unroll
        for (int i = 0; i < TAPS; ++i) x[i] = make_float2(x[i].x * w[i], x[i].y * w[i]);
        // the taps folded in pairs: the phasors of offsets o and -o are
        // conjugate, so y_o T_o + y_-o conj(T_o) = (Re T A.x - Im T B.y,
        // Re T A.y + Im T B.x) with A = y_o + y_-o, B = y_o - y_-o, and T_0 = 1
        float2 fa[KP], fb[KP];
#pragma unroll
        for (int o = 1; o <= KP; ++o) {
            fa[o - 1] = make_float2(x[KP + o].x + x[KP - o].x, x[KP + o].y + x[KP - o].y);
            fb[o - 1] = make_float2(x[KP + o].x - x[KP - o].x, x[KP + o].y - x[KP - o].y);
        }
        // two bands per pass (their 2 kappa table values fit the scalar registers);
        // band phasor exp(2 pi i u q_b / N): anchored every kPhaseAnchor bands,
        // rotated by exp(2 pi i u 2L / N) in between
        float sn, cs;
        sincospif(2.0f * u * step_rate, &sn, &cs);
        const float2 step = make_float2(cs, sn);
        float2 ph = make_float2(1.f, 0.f);
        for (int b0 = 0; b0 < Q; b0 += 2) {
            const CONSTANT float2* tab = cst(d->bandtab) + (size_t)b0 * TAPS + KP;   // zero-padded past Q
            float2 acc[2];
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                acc[bb] = x[KP];
#pragma unroll
                for (int o = KP; o >= 1; --o) {   // the outer taps first
                    const float2 t = ld2(tab + bb * TAPS + o);
                    acc[bb].x = fmaf(t.x, fa[o - 1].x, fmaf(-t.y, fb[o - 1].y, acc[bb].x));
                    acc[bb].y = fmaf(t.x, fa[o - 1].y, fmaf(t.y, fb[o - 1].x, acc[bb].y));
                }
            }
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) {
                const int b = b0 + bb;
                if (b < Q) {
                    if ((b % kPhaseAnchor) == 0) {
                        sincospif(2.0f * u * rate[b], &sn, &cs);
                        ph = make_float2(cs, sn);
                    } else {
                        ph = cmul(ph, step);
                    }
                    st2s(S + (size_t)b * P, cmul(acc[bb], ph));
                }
            }
        }
        if (sh >= nshift) break;
        }
    } else {
        // the same weights as the compile-time kernels, bit for bit: r^|o| by
        // |o| multiplications from 1 in the same order, e0 times the Gaussian
        // factor first
        const float e0 = wnorm * expf(-u * u * inv2sig2);
        const float r = expf(2.0f * u * inv2sig2);
        const float ri = expf(-2.0f * u * inv2sig2);
        auto weight = [&](int o) {
            const float gt = taps <= kFastTaps ? d->gtap[kappa + o] : expf(-(float)(o * o) * inv2sig2);
            if (o == 0) return e0 * gt;
            const float rr = o > 0 ? r : ri;
            float pw = 1.0f;
            for (int k = 0; k < (o > 0 ? o : -o); ++k) pw *= rr;
            return e0 * gt * pw;
        };
        for (int sh = 0; sh <= nshift; ++sh) {
        const int64_t jc = jp + sh;   // window centre
        const bool interior = (jc - kappa >= 0) && (jc + kappa < N);
        GLOBAL float2* __restrict__ S = glb(sh ? io.S2 : io.S) + soff;
        auto yv = [&](int o) {   // the windowed value at offset o of the window
            int64_t idx = jc + o;
            if (!interior) {
                if (idx < 0) idx += N;
                else if (idx >= N) idx -= N;
            }
            const float w = weight(o);
            const float2 fv = ld2(f + idx);
            return make_float2(fv.x * w, fv.y * w);
        };
        for (int b0 = 0; b0 < Q; b0 += kBandChunk) {
            const int nb = min(kBandChunk, Q - b0);
            float2 acc[kBandChunk];
            if (taps <= kFastTaps) {
                const float2 y0 = yv(0);
#pragma unroll
                for (int bb = 0; bb < kBandChunk; ++bb) acc[bb] = y0;
            }
            // the transposed table: a tap's kBandChunk bands are one 128-byte piece
            const int qpad = d->qpad;
            const CONSTANT float2* tab = cst(d->bandtab_t) + (size_t)kappa * qpad + b0;
            if (taps <= kFastTaps) {
                // taps folded in conjugate pairs, the outer ones first, as in the
                // compile-time forms (a batch of several widths runs this kernel)
                for (int o = kappa; o >= 1; --o) {
                    const float2 yp = yv(o), ym = yv(-o);
                    const float2 fa = make_float2(yp.x + ym.x, yp.y + ym.y);
                    const float2 fb = make_float2(yp.x - ym.x, yp.y - ym.y);
#pragma unroll
                    for (int bb = 0; bb < kBandChunk; ++bb) {   // zero-padded table: no guard
                        const float2 t = ld2(tab + o * qpad + bb);
                        acc[bb].x = fmaf(t.x, fa.x, fmaf(-t.y, fb.y, acc[bb].x));
                        acc[bb].y = fmaf(t.x, fa.y, fmaf(t.y, fb.x, acc[bb].y));
                    }
                }
            } else {
                // wider windows (no compile-time form): every tap with its own
                // table entry, the window read in order (measured: the folded
                // pairs, read from both ends, took twice as long at 45 taps)
#pragma unroll
                for (int bb = 0; bb < kBandChunk; ++bb) acc[bb] = make_float2(0.f, 0.f);
                for (int o = -kappa; o <= kappa; ++o) {
                    const float2 y = yv(o);
#pragma unroll
                    for (int bb = 0; bb < kBandChunk; ++bb) {
                        const float2 t = ld2(tab + o * qpad + bb);
                        acc[bb].x = fmaf(y.x, t.x, fmaf(-y.y, t.y, acc[bb].x));
                        acc[bb].y = fmaf(y.x, t.y, fmaf(y.y, t.x, acc[bb].y));
                    }
                }
            }
            store_bands(S, P, b0, nb, acc, u, rate, step_rate);
        }
        }
    }
}

// --------------------------------------------------------- k_gather_mx ----
// The same filtered samples with the band sums on the matrix cores.  One lane
// per node, as in k_gather: node geometry, window, weights
// W(u - o) = [wnorm exp(-u^2 c - 2 u c kappa) r^(o + kappa)] exp(-o^2 c),
// r = exp(2 u c), c = inv2sig2 (the bracket by one exponential and a product
// per tap, the last factor from the plan's gmx_g), y_i = f[(j' + i - kappa) mod N] W.
// The band sums S'_b = sum_i y_i T[b][i] of the wave's 64 nodes are four real
// products D = A B (tiles of 16 nodes): B[k][n] = y_{k/2}(node n) (k even:
// real part, odd: imaginary part), A[2 b + e][k] the real form of T[b][k/2]
// (e = 0: Re, 1: Im; gmx_a, in lane order), so that
// D[2 b][n] + i D[2 b + 1][n] = S'_b(node n).  FP32 16x16x4 MFMAs: M = 16 rows
// (8 bands), K = 4 (2 taps), N = 16 nodes.  A 4 x 4 transpose of (register,
// 16-lane row) turns the lane-per-node values of a K-step into the operands of
// the four tiles (lane l of tile t supplies B[4 st + l / 16][l % 16]), and the
// same transpose of the accumulators returns every node's rows to its lane.
// Then S_b = exp(2 pi i q_b u / N) S'_b, the phasor anchored every
// kPhaseAnchor bands and rotated by exp(2 pi i u 2L / N) in between, as in
// k_gather.  MTMAX M-tiles (8 bands each) are accumulated per pass over the
// window.  TAPSMAX <= 16: the window in registers whole, loaded once; else
// in chunks of 8 taps per pass, the next chunk's loads issued before the
// current chunk's products.

// 4 x 4 transpose of (register, row of 16 lanes): on return v[j] in row k
// holds what v[k] held in row j (v_permlane32_swap, then v_permlane16_swap).
__device__ __forceinline__ void transpose4(float (&v)[4]) {
    const auto s02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[0]), __float_as_uint(v[2]), false, false);
    const auto s13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[1]), __float_as_uint(v[3]), false, false);
    const auto t01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
    const auto t23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
    v[0] = __uint_as_float(t01[0]);
    v[1] = __uint_as_float(t01[1]);
    v[2] = __uint_as_float(t23[0]);
    v[3] = __uint_as_float(t23[1]);
}

template <int TAPSMAX, int MTMAX>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MTMAX > 2 ? 2 : 4))) k_gather_mx(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    if (at.blk == 0 && tid == 0) glb(io.status)[0] = 0;
    const int lane = tid & 63;
    const int M = d->M;
    // every lane of a wave takes part in the transposes and products; lanes
    // past the last node work on it again and store nothing (a wave wholly
    // past it still takes part in the table's staging)
    const int g0 = at.blk * kThreads + tid;
    const bool mine = g0 < M;
    const int g = mine ? g0 : M - 1;
    const int K = d->K;
    int j = 0;
    while (j + 1 < K && g >= d->Moff[j + 1]) ++j;
    const int l = g - d->Moff[j];
    const int p = d->p[j];
    const int P = d->P[j];
    const int s1 = d->s1;
    int n = (l & (s1 - 1)) * p + (l >> d->log2s1) * s1;   // node (n1 p + n2 s1) mod P
    if (n >= P) n -= P;
    const int64_t N = d->N;
    const int64_t nN = (int64_t)n * N;
    const int64_t num = 2 * nN + P, den = 2 * (int64_t)P;
    int64_t jp = (int64_t)((double)num / (double)den);
    const int64_t rem = num - jp * den;
    if (rem < 0) --jp;
    else if (rem >= den) ++jp;
    const int32_t delta = (int32_t)(nN - jp * P);
    const float u = (float)delta / (float)P;
    const int kappa = d->kappa, taps = d->taps, Q = d->Q;
    const GLOBAL float2* __restrict__ f = glb(io.f);
    // window value i of the window starting at st0 (zero past the last tap)
    auto tap = [&](int64_t st0, int i) -> float2 {
        if (i >= taps) return make_float2(0.f, 0.f);
        int64_t idx = st0 + i;
        if (idx < 0) idx += N;
        else if (idx >= N) idx -= N;
        return ld2(f + idx);
    };
    // narrow windows (at most 16 taps), loaded whole before the table's staging:
    // inside [0, N) as 16-byte pieces from the even index at or below the
    // start, then shifted by the start's parity (as in k_gather)
    const int64_t ab = (int64_t)(((uintptr_t)io.f >> 3) & 1);
    auto load_window = [&](int64_t st0, float2 (&xw)[16]) {
        const int64_t par = (st0 + ab) & 1;
        if (st0 - par >= 0 && st0 + 18 <= N) {
            const GLOBAL pod_f4* w4 = (const GLOBAL pod_f4*)(f + (st0 - par));
            float2 cc[18];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                pod_f4 v = {0.f, 0.f, 0.f, 0.f};
                if (2 * q <= taps) v = w4[q];   // the pieces that hold taps (uniform)
                cc[2 * q] = make_float2(v.x, v.y);
                cc[2 * q + 1] = make_float2(v.z, v.w);
            }
            const uint32_t mk = 0u - (uint32_t)par;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const float2 lo = cc[i], hi = cc[i + 1];
                const float2 v = make_float2(__uint_as_float((__float_as_uint(lo.x) & ~mk) | (__float_as_uint(hi.x) & mk)),
                                             __uint_as_float((__float_as_uint(lo.y) & ~mk) | (__float_as_uint(hi.y) & mk)));
                xw[i] = i < taps ? v : make_float2(0.f, 0.f);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 16; ++i) xw[i] = tap(st0, i);
        }
    };
    float2 xw[TAPSMAX <= 16 ? 16 : 1];
    float2 x0[TAPSMAX <= 16 ? 1 : 8];
    if constexpr (TAPSMAX <= 16) load_window(jp - kappa, xw);
    else {
#pragma unroll
        for (int q = 0; q < 8; ++q) x0[q] = tap(jp - kappa, q);
    }
    const int MT = d->gmx_mt, KS = d->gmx_ks;
    float* As = reinterpret_cast<float*>(smem);   // [MT][KS][64]
    float* Gs = As + MT * KS * 64;                // [2 KS]
    {
        const int na = MT * KS * 64, ng = 2 * KS;
        const GLOBAL float* ga = glb(d->gmx_a);
        const GLOBAL float* gg = glb(d->gmx_g);
        for (int i = tid; i < na; i += kThreads) As[i] = ga[i];
        for (int i = tid; i < ng; i += kThreads) Gs[i] = gg[i];
    }
    __syncthreads();
    if (g0 - lane >= M) return;   // the whole wave is past the last node
    const float c = d->inv2sig2;
    const float e_first = d->wnorm * expf(-u * u * c - 2.0f * u * c * (float)kappa);   // o = -kappa
    const float r = expf(2.0f * u * c);
    const CONSTANT float* rate = cst(d->rate);
    float sn, cs;
    sincospif(2.0f * u * d->a_step, &sn, &cs);
    const float2 step = make_float2(cs, sn);
    const size_t soff = (size_t)Q * d->Moff[j] + l;
    const int nshift = d->phase;   // 0, or 1: also the node moved one grid step
    for (int sh = 0; sh <= nshift; ++sh) {
        const int64_t st0 = jp - kappa + sh;   // index of the window's first tap
        if (sh > 0) {
            if constexpr (TAPSMAX <= 16) load_window(st0, xw);
            else {
#pragma unroll
                for (int q = 0; q < 8; ++q) x0[q] = tap(st0, q);
            }
        }
        GLOBAL float2* __restrict__ S = glb(sh ? io.S2 : io.S) + soff;
        // MTMAX M-tiles (8 bands each) per pass over the window
        for (int m0 = 0; m0 < MT; m0 += MTMAX) {
            mf4 acc[4][MTMAX];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int mm = 0; mm < MTMAX; ++mm) acc[t][mm] = mf4{0.f, 0.f, 0.f, 0.f};
            float ew = e_first;
            // K-steps c0 .. c0 + 3 (taps 2 c0 .. 2 c0 + 7) from their window values x
            auto chunk = [&](int c0, const float2 (&x)[8]) {
#pragma unroll
                for (int u4 = 0; u4 < 4; ++u4) {
                    const int st = c0 + u4;
                    if (st >= KS) break;
                    float b4[4];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const float w = ew * Gs[2 * st + h];
                        ew *= r;
                        b4[2 * h] = x[2 * u4 + h].x * w;
                        b4[2 * h + 1] = x[2 * u4 + h].y * w;
                    }
                    transpose4(b4);   // b4[t]: this lane's operand for tile t
#pragma unroll
                    for (int mm = 0; mm < MTMAX; ++mm) {
                        if (m0 + mm >= MT) break;
                        const float av = As[((m0 + mm) * KS + st) * 64 + lane];
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            acc[t][mm] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b4[t], acc[t][mm], 0, 0, 0);
                    }
                }
            };
            if constexpr (TAPSMAX <= 16) {
#pragma unroll
                for (int c0 = 0; c0 < 8; c0 += 4) {
                    if (c0 >= KS) break;
                    float2 x[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) x[q] = xw[2 * c0 + q];
                    chunk(c0, x);
                }
            } else {
                // a window inside [0, N) for the whole wave: fixed offsets from its first tap
                const bool inner = __all(st0 >= 0 && st0 + 2 * KS <= N);
                const GLOBAL float2* __restrict__ fw = f + st0;
                auto tapw = [&](int i) -> float2 {
                    if (!inner) return tap(st0, i);
                    return i < taps ? ld2(fw + i) : make_float2(0.f, 0.f);
                };
                float2 x[8], nx[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) x[q] = m0 == 0 ? x0[q] : tapw(q);
                for (int c0 = 0; c0 < KS; c0 += 4) {
                    if (c0 + 4 < KS) {
#pragma unroll
                        for (int q = 0; q < 8; ++q) nx[q] = tapw(2 * (c0 + 4) + q);
                    }
                    chunk(c0, x);
#pragma unroll
                    for (int q = 0; q < 8; ++q) x[q] = nx[q];
                }
            }
            // rows back to the node's lane: after the transposes o[jj][rr] is
            // row 4 jj + rr of M-tile m, i.e. band 8 m + 2 jj + rr / 2, part rr % 2
#pragma unroll
            for (int mm = 0; mm < MTMAX; ++mm) {
                const int m = m0 + mm;
                if (m >= MT) break;
                float o[4][4];
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    float v4[4] = {acc[0][mm][rr], acc[1][mm][rr], acc[2][mm][rr], acc[3][mm][rr]};
                    transpose4(v4);
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) o[jj][rr] = v4[jj];
                }
                float2 ph = make_float2(1.f, 0.f);
#pragma unroll
                for (int bb = 0; bb < 8; ++bb) {   // band b = 8 m + bb, the phasor anchored at bb = 0
                    const int b = 8 * m + bb;
                    if (b >= Q) break;
                    if (bb == 0) {
                        sincospif(2.0f * u * rate[b], &sn, &cs);
                        ph = make_float2(cs, sn);
                    } else {
                        ph = cmul(ph, step);
                    }
                    const float2 v = make_float2(o[bb >> 1][2 * (bb & 1)], o[bb >> 1][2 * (bb & 1) + 1]);
                    if (mine) st2s(S + (size_t)b * P, cmul(v, ph));
                }
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

// Bit reversal, then the radix-2 DIT stages of length-s1 FFTs over `rows`
// rows in LDS.  Stages are fused in pairs: each thread loads four values,
// applies two radix-2 stages in registers and stores them back (a leading
// single stage when log2 s1 is odd).  tw: LDS copy of exp(-2 pi i k / s1).
template <int NT>
__device__ void fft_rows_lds(float2* buf, int rows, int s1, int lg, const float2* tw) {
    const int tid = (int)threadIdx.x;
    const int n = rows << lg;
    if (lg == 0) return;
    for (int i = tid; i < n; i += NT) {
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
    int ls = 1;
    if (lg & 1) {   // stage of length 2: twiddle 1
        for (int i = tid; i < (n >> 1); i += NT) {
            const float2 x0 = buf[2 * i];
            const float2 x1 = buf[2 * i + 1];
            buf[2 * i] = make_float2(x0.x + x1.x, x0.y + x1.y);
            buf[2 * i + 1] = make_float2(x0.x - x1.x, x0.y - x1.y);
        }
        __syncthreads();
        ls = 2;
    }
    for (; ls + 1 <= lg; ls += 2) {
        const int h = 1 << (ls - 1);   // half length of stage ls
        const int quarter = n >> 2;
        for (int i = tid; i < quarter; i += NT) {
            const int row = i >> (lg - 2);
            const int rr = i & ((s1 >> 2) - 1);
            const int blk = rr >> (ls - 1);
            const int pos = rr & (h - 1);
            const int b0 = (row << lg) + blk * (4 * h) + pos;
            float2 x0 = buf[b0], x1 = buf[b0 + h], x2 = buf[b0 + 2 * h], x3 = buf[b0 + 3 * h];
            const float2 w1 = tw[pos << (lg - ls)];
            float2 y = cmul(x1, w1);
            x1 = make_float2(x0.x - y.x, x0.y - y.y);
            x0 = make_float2(x0.x + y.x, x0.y + y.y);
            y = cmul(x3, w1);
            x3 = make_float2(x2.x - y.x, x2.y - y.y);
            x2 = make_float2(x2.x + y.x, x2.y + y.y);
            const float2 w2 = tw[pos << (lg - ls - 1)];
            const float2 w3 = tw[(pos + h) << (lg - ls - 1)];
            y = cmul(x2, w2);
            buf[b0 + 2 * h] = make_float2(x0.x - y.x, x0.y - y.y);
            buf[b0] = make_float2(x0.x + y.x, x0.y + y.y);
            y = cmul(x3, w3);
            buf[b0 + 3 * h] = make_float2(x1.x - y.x, x1.y - y.y);
            buf[b0 + h] = make_float2(x1.x + y.x, x1.y + y.y);
        }
        __syncthreads();
    }
}

// ---- in-register DFTs of length R <= 16 (natural order in and out)
// cos and sin of 2 pi k / 16
__constant__ const float kCos16[16] = {1.000000000f, 0.923879533f, 0.707106781f, 0.382683432f, 0.000000000f, -0.382683432f, -0.707106781f, -0.923879533f, -1.000000000f, -0.923879533f, -0.707106781f, -0.382683432f, -0.000000000f, 0.382683432f, 0.707106781f, 0.923879533f};
__constant__ const float kSin16[16] = {0.000000000f, 0.382683432f, 0.707106781f, 0.923879533f, 1.000000000f, 0.923879533f, 0.707106781f, 0.382683432f, 0.000000000f, -0.382683432f, -0.707106781f, -0.923879533f, -1.000000000f, -0.923879533f, -0.707106781f, -0.382683432f};

constexpr int brev_const(int i, int bits) {
    int r = 0;
    for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
    return r;
}
constexpr int log2_const(int r) { return r <= 1 ? 0 : 1 + log2_const(r / 2); }

// Column swizzle of the matrix-core kernel's block in LDS: complex value c of
// row r sits at c ^ swz_col(r).  Rows a multiple of 4 apart keep their
// columns, rows 1, 2, 3 apart move by 8, 16, 24 complex values (64 to 192
// bytes), so the p-point step's B operands (four consecutive rows, the same
// 16 floats in each) fall in four different groups of 16 banks, and so do the
// row FFT's stores (eight consecutive rows, the same 8 complex values in each).
__device__ __forceinline__ int swz_col(int row) { return (row & 3) << 3; }

// v <- DFT_R(v): X_k = sum_n v_n exp(-2 pi i n k / R), radix-2 decimation in
// time with compile-time twiddles (the bit reversal is a register renaming).
template <int R>
__device__ __forceinline__ void dft_reg(float2 (&v)[R]) {
    static_assert(R >= 2 && R <= 16 && (R & (R - 1)) == 0, "radix");
    constexpr int LG = log2_const(R);
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[brev_const(i, LG)] = v[i];
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int s0 = 0; s0 < R; s0 += len)
#pragma unroll
            for (int k = 0; k < half; ++k) {
                const int e = k * (16 / len);   // W_len^k = W_16^e
                float2 b = t[s0 + k + half];
                if (e == 4) {
                    b = make_float2(b.y, -b.x);
                } else if (e != 0) {
                    const float c = kCos16[e], sn = kSin16[e];
                    b = make_float2(fmaf(b.x, c, b.y * sn), fmaf(b.y, c, -b.x * sn));
                }
                const float2 a0 = t[s0 + k];
                t[s0 + k] = make_float2(a0.x + b.x, a0.y + b.y);
                t[s0 + k + half] = make_float2(a0.x - b.x, a0.y - b.y);
            }
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
}

// Length-S FFTs (S = R1 R2) of `rows` <= ROWSMAX rows in LDS, two passes
// through registers with n = n1 + R1 n2 and k = R2 k1 + k2:
//   Z[n1][k2]     = W_S^(n1 k2) sum_n2 x[n1 + R1 n2] W_R2^(n2 k2)
//   X[R2 k1 + k2] = sum_n1 Z[n1][k2] W_R1^(n1 k1)
// Z sits in the row at k2 R1 + (n1 ^ f), f = (k2 + R2 (row & 1)) mod R1, so
// that pass 2 reads R1 values per thread without LDS bank conflicts.
// SWZ: the result X[k] of a row goes to position k ^ swz_col(row) instead of k
// (the layout the matrix-core p-point step reads without bank conflicts).
// tw: LDS exp(-2 pi i m / (S TWS)), m < S TWS (TWS > 1: a longer transform's
// table, read at every TWS-th entry).
template <int NT, int R1, int R2, int ROWSMAX, bool SWZ = false, int TWS = 1>
__device__ void fft_rows_2pass(float2* buf, int rows, const float2* tw) {
    constexpr int S = R1 * R2;
    constexpr int IT1 = (ROWSMAX * R1 + NT - 1) / NT;
    constexpr int IT2 = (ROWSMAX * R2 + NT - 1) / NT;
    constexpr int L1 = log2_const(R1), L2 = log2_const(R2);
    const int tid = (int)threadIdx.x;
    float2 z[IT1][R2];
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
        const int item = tid + it * NT;
        if (item < rows * R1) {
            const int row = item >> L1;
            const int n1 = item & (R1 - 1);
            const float2* x = buf + row * S + n1;
#pragma unroll
            for (int n2 = 0; n2 < R2; ++n2) z[it][n2] = x[n2 * R1];
            dft_reg<R2>(z[it]);
#pragma unroll
            for (int k2 = 1; k2 < R2; ++k2) {
                const float2 w = tw[n1 * k2 * TWS];
                const float2 b = z[it][k2];
                z[it][k2] = cmul(b, w);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT1; ++it) {
        const int item = tid + it * NT;
        if (item < rows * R1) {
            const int row = item >> L1;
            const int n1 = item & (R1 - 1);
            float2* zr = buf + row * S;
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) zr[k2 * R1 + (n1 ^ ((k2 + R2 * (row & 1)) & (R1 - 1)))] = z[it][k2];
        }
    }
    __syncthreads();
    float2 y[IT2][R1];
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
        const int item = tid + it * NT;
        if (item < rows * R2) {
            const int row = item >> L2;
            const int k2 = item & (R2 - 1);
            const int f = (k2 + R2 * (row & 1)) & (R1 - 1);
            const float2* zr = buf + row * S + k2 * R1;
#pragma unroll
            for (int n1 = 0; n1 < R1; ++n1) y[it][n1] = zr[n1 ^ f];
            dft_reg<R1>(y[it]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT2; ++it) {
        const int item = tid + it * NT;
        if (item < rows * R2) {
            const int row = item >> L2;
            const int k2 = item & (R2 - 1);
            float2* xr = buf + row * S;
            const int sw = SWZ ? swz_col(row) : 0;
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) xr[(k1 * R2 + k2) ^ sw] = y[it][k1];
        }
    }
    __syncthreads();
}

// Length-S row FFTs for S = 8 A (A = 64, 128, 256: s1 = 512, 1024, 2048) in
// register passes.  With n = m + A n3 and k = 8 k' + k3,
//   X[8 k' + k3] = sum_m W_A^(m k') [W_S^(m k3) sum_n3 x[m + A n3] W_8^(n3 k3)]:
// an 8-point DFT and twiddles per (row, m), written to sub-row k3 of the row
// (position k3 A + m); the A-point transforms of the 8 sub-rows by the two
// register passes (their twiddles every 8th entry of the S-point table); then
// the permutation to natural order through registers.  At most ROWS rows.
template <int NT, int A, int ROWS>
__device__ void fft_rows_3pass(float2* buf, int rows, const float2* tw) {
    constexpr int S = 8 * A;
    constexpr int IT0 = (ROWS * A + NT - 1) / NT;
    constexpr int IT3 = (ROWS * S + NT - 1) / NT;
    constexpr int R1 = A == 64 ? 8 : 16, R2 = A == 256 ? 16 : 8;
    static_assert(R1 * R2 == A, "sub-row length");
    const int tid = (int)threadIdx.x;
    float2 z[IT0][8];
#pragma unroll
    for (int it = 0; it < IT0; ++it) {
        const int item = tid + it * NT;
        if (item < rows * A) {
            const int row = item / A, m = item % A;
            const float2* x = buf + row * S + m;
#pragma unroll
            for (int n3 = 0; n3 < 8; ++n3) z[it][n3] = x[n3 * A];
            dft_reg<8>(z[it]);
#pragma unroll
            for (int k3 = 1; k3 < 8; ++k3) z[it][k3] = cmul(z[it][k3], tw[m * k3]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT0; ++it) {
        const int item = tid + it * NT;
        if (item < rows * A) {
            const int row = item / A, m = item % A;
#pragma unroll
            for (int k3 = 0; k3 < 8; ++k3) buf[row * S + k3 * A + m] = z[it][k3];
        }
    }
    __syncthreads();
    fft_rows_2pass<NT, R1, R2, ROWS * 8, false, 8>(buf, rows * 8, tw);
    float2 v[IT3];
#pragma unroll
    for (int it = 0; it < IT3; ++it) {
        const int idx = tid + it * NT;
        if (idx < rows * S) {
            const int row = idx / S, k = idx % S;
            v[it] = buf[row * S + (k & 7) * A + (k >> 3)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT3; ++it) {
        const int idx = tid + it * NT;
        if (idx < rows * S) buf[idx] = v[it];
    }
    __syncthreads();
}

// Row FFTs: two register passes for s1 = 64, 128 and 256 (ROWS256 = 0: no
// such branch compiled), three for s1 = 512 ... 2048 where BIGELEMS > 0
// (BIGELEMS / s1 rows at a time), else the radix-2/4 LDS passes.  Without
// CHUNKED the rows are at most ROWS64, ROWS128 or ROWS256; with it they are
// taken in chunks of that many (multiples of 4).  A row's arithmetic does not
// depend on the chunk it is in, so the in-LDS kernels (a whole block) and the
// split path's row kernel (a few rows) give bitwise equal rows up to s1 = 256.
// Only the row kernel takes the three passes (compiled into the in-LDS VALU
// kernel they raised it from 116 to 169 VGPRs): for s1 >= 512 the in-LDS
// VALU kernel keeps the LDS passes and the two paths agree to rounding.
template <int NT, int ROWS128, int ROWS64, bool SWZ = false, int ROWS256 = 0, bool CHUNKED = false, int BIGELEMS = 0>
__device__ __forceinline__ void fft_rows(float2* buf, int rows, int s1, int lg, const float2* tw) {
    static_assert(!SWZ || (ROWS128 >= 64 && ROWS64 >= 64), "the swizzled layout needs the register passes");
    static_assert(ROWS128 % 4 == 0 && ROWS64 % 4 == 0 && ROWS256 % 4 == 0, "chunks keep the row swizzle");
    if constexpr (BIGELEMS > 0) {   // s1 = 512, 1024, 2048: three register passes, BIGELEMS / s1 rows at a time
        if (s1 >= 512 && s1 <= 2048) {
            const int per = BIGELEMS >> lg;
#pragma unroll 1
            for (int r0 = 0; r0 < rows; r0 += per) {
                float2* b = buf + ((size_t)r0 << lg);
                const int n = min(per, rows - r0);
                if (s1 == 512) fft_rows_3pass<NT, 64, BIGELEMS / 512>(b, n, tw);
                else if (s1 == 1024) fft_rows_3pass<NT, 128, BIGELEMS / 1024>(b, n, tw);
                else fft_rows_3pass<NT, 256, BIGELEMS / 2048>(b, n, tw);
                if (!CHUNKED) break;
            }
            return;
        }
    }
    if constexpr (ROWS256 > 0) {
        if (s1 == 256) {
            if constexpr (CHUNKED) {
                for (int r0 = 0; r0 < rows; r0 += ROWS256)
                    fft_rows_2pass<NT, 16, 16, ROWS256, SWZ>(buf + ((size_t)r0 << 8), min(ROWS256, rows - r0), tw);
            } else {
                fft_rows_2pass<NT, 16, 16, ROWS256, SWZ>(buf, rows, tw);
            }
            return;
        }
    }
    if (s1 == 128) {
        if constexpr (CHUNKED) {
            for (int r0 = 0; r0 < rows; r0 += ROWS128)
                fft_rows_2pass<NT, 16, 8, ROWS128, SWZ>(buf + ((size_t)r0 << 7), min(ROWS128, rows - r0), tw);
        } else {
            fft_rows_2pass<NT, 16, 8, ROWS128, SWZ>(buf, rows, tw);
        }
    } else if (s1 == 64) {
        if constexpr (CHUNKED) {
            for (int r0 = 0; r0 < rows; r0 += ROWS64)
                fft_rows_2pass<NT, 8, 8, ROWS64, SWZ>(buf + ((size_t)r0 << 6), min(ROWS64, rows - r0), tw);
        } else {
            fft_rows_2pass<NT, 8, 8, ROWS64, SWZ>(buf, rows, tw);
        }
    } else {
        fft_rows_lds<NT>(buf, rows, s1, lg, tw);
    }
}

// Cosine/sine table of a p-point step (host-computed per modulus), copied to
// LDS: trig[(n - 1) h + (k - 1)] = (cos, sin)(2 pi (n k mod p) / p), n, k in [1, h].
template <int NT>
__device__ void load_trig(float2* trig, int h, const GLOBAL float2* __restrict__ src) {
    for (int i = (int)threadIdx.x; i < h * h; i += NT) trig[i] = ld2(src + i);
}

constexpr int kDftKB = 8;       // output pairs per work item, split path

// One p-point output group of column c: with h = (p - 1) / 2, a_n = x_n + x_{p-n},
// b_n = x_n - x_{p-n}, C_k = sum_n a_n cos(2 pi n k / p), D_k = sum_n b_n sin(...),
//   X_k = x_0 + C_k - i D_k,  X_{p-k} = x_0 + C_k + i D_k,  X_0 = x_0 + sum_n a_n.
// Accumulates C, D for k = k0 .. k0 + KB - 1 (k <= h) and sa = sum_n a_n.
template <int KBMAX>
__device__ __forceinline__ void pfa_column_sums(const float2* blk, int stride, int c, int p, int h, int k0, int KB,
                                                const float2* trig, float2* C, float2* D, float2& sa) {
#pragma unroll
    for (int kk = 0; kk < KBMAX; ++kk) {
        C[kk] = make_float2(0.f, 0.f);
        D[kk] = make_float2(0.f, 0.f);
    }
    sa = make_float2(0.f, 0.f);
    for (int n = 1; n <= h; ++n) {
        const float2 xa = blk[n * stride + c];
        const float2 xb = blk[(p - n) * stride + c];
        const float2 av = make_float2(xa.x + xb.x, xa.y + xb.y);
        const float2 bv = make_float2(xa.x - xb.x, xa.y - xb.y);
        sa.x += av.x;
        sa.y += av.y;
        const float2* tr = trig + (n - 1) * h + (k0 - 1);
#pragma unroll
        for (int kk = 0; kk < KBMAX; ++kk) {
            if (kk < KB && k0 + kk <= h) {
                const float2 t = tr[kk];
                C[kk].x = fmaf(av.x, t.x, C[kk].x);
                C[kk].y = fmaf(av.y, t.x, C[kk].y);
                D[kk].x = fmaf(bv.x, t.y, D[kk].x);
                D[kk].y = fmaf(bv.y, t.y, D[kk].y);
            }
        }
    }
}

// Split path: p-point DFTs of the columns of a [p][stride] LDS block, one work
// item per (column, group of kDftKB output pairs), written to out[k * out_stride + c].
template <int NT>
__device__ void dft_cols_lds(const float2* blk, int stride, int ncols, int p, const float2* trig,
                             GLOBAL float2* __restrict__ out, int out_stride, float scale) {
    const int h = (p - 1) >> 1;
    const int ng = (h + kDftKB - 1) / kDftKB;
    const int groups = ng > 0 ? ng : 1;
    for (int item = (int)threadIdx.x; item < ncols * groups; item += NT) {
        const int g = item / ncols;
        const int c = item - g * ncols;
        const int k0 = 1 + g * kDftKB;
        const float2 x0 = blk[c];
        float2 C[kDftKB], D[kDftKB], sa;
        pfa_column_sums<kDftKB>(blk, stride, c, p, h, k0, kDftKB, trig, C, D, sa);
#pragma unroll
        for (int kk = 0; kk < kDftKB; ++kk) {
            const int k = k0 + kk;
            if (k <= h) {
                st2s(out + (size_t)k * out_stride + c,
                    make_float2((x0.x + C[kk].x + D[kk].y) * scale, (x0.y + C[kk].y - D[kk].x) * scale));
                st2s(out + (size_t)(p - k) * out_stride + c,
                    make_float2((x0.x + C[kk].x - D[kk].y) * scale, (x0.y + C[kk].y + D[kk].x) * scale));
            }
        }
        if (g == 0) st2s(out + c, make_float2((x0.x + sa.x) * scale, (x0.y + sa.y) * scale));
    }
}

// Selection key of bin h with value e: (bits(|E|^2) << 32) | (2^32 - 1 - h).
__device__ __forceinline__ uint64_t value_key(float2 e, uint32_t h) {
    const float m2 = fmaf(e.x, e.x, e.y * e.y);
    return ((uint64_t)__float_as_uint(m2) << 32) | (uint64_t)(0xffffffffu - h);
}

// Bin index h of Good-Thomas position i = k2 s1 + k1: h = k1 (mod s1), h = k2 (mod p).
__device__ __forceinline__ uint32_t pfa_bin(int i, int lg, int s1, uint32_t P, uint32_t cA, uint32_t cB) {
    const uint32_t k2 = (uint32_t)(i >> lg);
    const uint32_t k1 = (uint32_t)(i & (s1 - 1));
    return (k1 * cA + k2 * cB) % P;
}

// The T-th largest of the P distinct keys key(i), 1 <= T: a radix select over
// 10-bit digits from bit 62 down (bit 63 is the sign of |E|^2, always 0), which
// stops as soon as the chosen digit's bucket holds exactly the keys still
// needed.  The keys >= the returned value are exactly the T largest.  The
// digit search is a block scan of the buckets in descending order.
// hist: LDS int32[kSelBins]; part: LDS int32[NT / 64].
constexpr int kSelBits = 10;
static_assert(kSelBins == 1 << kSelBits, "bucket count");

// each(f) calls f(hi, full) for every key k this thread holds, with hi = k >> 32
// and full() returning k (which may cost more: it is called only in passes
// whose digit reaches below bit 32, and only for keys whose hi matches).
// FILLED: hist already holds the first digit's histogram of every key with
// bit 63 clear (the caller formed it and passed a barrier since).
template <int NT, bool FILLED = false, class EachKey>
__device__ uint64_t kth_largest(EachKey each, int P, int T, int32_t* hist, int32_t* part) {
    __shared__ int32_t sh_digit, sh_need, sh_done;
    constexpr int BPT = kSelBins / NT;   // buckets per thread
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    if (T >= P) return 0;
    uint64_t prefix = 0, pmask = (uint64_t)1 << 63;
    int need = T;
    int top = 63;   // bits [shift, top) form the next digit
    for (;;) {
        const int width = top < kSelBits ? top : kSelBits;
        const int shift = top - width;
        const uint64_t dmask = ((uint64_t)1 << width) - 1;
        if (!FILLED || top != 63) {
        for (int i = tid; i < kSelBins; i += NT) hist[i] = 0;
        __syncthreads();
        const uint32_t pm_hi = (uint32_t)(pmask >> 32), pre_hi = (uint32_t)(prefix >> 32);
        if (shift >= 32) {
            const int sh = shift - 32;
            const uint32_t dm = (uint32_t)dmask;
            each([&](uint32_t hi, auto) {
                if ((hi & pm_hi) == pre_hi) atomicAdd(&hist[(int)((hi >> sh) & dm)], 1);
            });
        } else {
            each([&](uint32_t hi, auto full) {
                if ((hi & pm_hi) == pre_hi) {
                    const uint64_t k = full();
                    if ((k & pmask) == prefix) atomicAdd(&hist[(int)((k >> shift) & dmask)], 1);
                }
            });
        }
        __syncthreads();
        }
        const int nb = 1 << width;
        int cnt[BPT];
        int loc = 0;
#pragma unroll
        for (int q = 0; q < BPT; ++q) {   // descending rank r <-> digit nb - 1 - r
            const int r = tid * BPT + q;
            cnt[q] = r < nb ? hist[nb - 1 - r] : 0;
            loc += cnt[q];
        }
        const int x = wave_inclusive_sum(loc);
        if (lane == 63) part[wid] = x;
        __syncthreads();
        int base = 0;
        base = waves_before<NT>(part, wid);
        const int incl = base + x;
        int run = incl - loc;
        if (run < need && incl >= need) {
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                if (run < need && run + cnt[q] >= need) {
                    sh_digit = nb - 1 - (tid * BPT + q);
                    sh_need = need - run;
                    sh_done = (cnt[q] == need - run) ? 1 : 0;
                }
                run += cnt[q];
            }
        }
        __syncthreads();
        prefix |= (uint64_t)sh_digit << shift;
        pmask |= dmask << shift;
        need = sh_need;
        if (sh_done || shift == 0) break;   // sh_* change again only after the next pass's third barrier
        top = shift;
    }
    return prefix;
}

// Exclusive block-wide prefix sum of one value per thread.  part: LDS
// int32[NT/64].  Without the trailing barrier part must not be rewritten
// before every thread has returned (the caller's next barrier).
template <int NT, bool TAIL_BARRIER = true>
__device__ int block_exclusive_sum(int v, int32_t* part) {
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int x = wave_inclusive_sum(v);
    if (lane == 63) part[wid] = x;
    __syncthreads();
    const int base = waves_before<NT>(part, wid);
    if (TAIL_BARRIER) __syncthreads();
    return base + x - v;
}

// Heavy bins among the keys key(0..P-1) of one block (keys >= thr, at most T
// of them; the keys are those of every bin, or a candidate list that holds
// the heavy ones).  Writes the threshold, the heavy bins in the order of the
// index i (H), and for every residue class c mod s1 (the bin mod s1, column c
// of the [p][s1] layout) the `depth` heaviest heavy bins of the class in
// descending key order (CL[c * depth + e], -1 where fewer).  Wave w walks the
// contiguous indices [w seg, (w + 1) seg) 64 at a time; a ballot per step
// gives each heavy bin its rank within the wave, a scan of the per-wave
// counts its rank in the block, so H comes out in index order without
// sorting.  Class ranks come from key comparisons within each class: for a
// few heavy bins all pairs, split over all threads; else per class list.
// scr: LDS int32[kSelBins]; part: LDS int32[NT / 64]; hk: LDS uint64[2 T];
// cl: LDS int32[s1 * depth].
template <int NT, class KeyF>
__device__ void emit_heavy(KeyF key, int P, int T, int s1, int depth, uint64_t thr, uint64_t* hk, int32_t* scr,
                           int32_t* part, int32_t* cl, GLOBAL int32_t* __restrict__ H,
                           GLOBAL uint64_t* __restrict__ thr_out, GLOBAL int32_t* __restrict__ CL) {
    constexpr int W = NT / 64;
    __shared__ int32_t sh_n;
    const int tid = (int)threadIdx.x;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const uint64_t lt = ((uint64_t)1 << lane) - 1;
    // residue class of a key: its bin mod s1 (the Good-Thomas column)
    auto class_of = [s1](uint64_t k) { return (int)((0xffffffffu - (uint32_t)(k & 0xffffffffu)) & (uint32_t)(s1 - 1)); };
    const int seg = ((P + NT - 1) / NT) * 64;   // positions per wave, a multiple of 64
    const int p0 = wid * seg;
    const int p1 = min(P, p0 + seg);
    if (tid == 0) *thr_out = thr;
    for (int i = tid; i < s1 * depth; i += NT) cl[i] = -1;

    int cnt = 0;   // heavy bins in this wave's segment (wave-uniform)
    for (int i0 = p0; i0 < p1; i0 += 64) {
        const int i = i0 + lane;
        cnt += __popcll(__ballot(i < p1 && key(i) >= thr));
    }
    if (lane == 0) part[wid] = cnt;
    __syncthreads();
    int run = 0;
    for (int w = 0; w < wid; ++w) run += part[w];
    if (tid == NT - 1) sh_n = run + cnt;
    for (int i0 = p0; i0 < p1; i0 += 64) {
        const int i = i0 + lane;
        uint64_t k = 0;
        const bool hv = i < p1 && (k = key(i)) >= thr;
        const uint64_t m = __ballot(hv);
        if (hv) {
            const int e = run + __popcll(m & lt);
            if (e < T) {
                hk[2 * e] = k;
                hk[2 * e + 1] = (uint64_t)i;
                H[e] = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
            }
        }
        run += __popcll(m);
    }
    __syncthreads();
    const int n = min(sh_n, T);

    // class ranks: heavier[e] = number of heavy bins of e's class with a larger key
    const int parts = n > 0 ? min(64, NT / n) : 1;
    int32_t* heavier = scr;
    if (parts > 1) {   // n <= NT / 2 <= kSelBins
        for (int e = tid; e < n; e += NT) heavier[e] = 0;
        __syncthreads();
        const int span = (n + parts - 1) / parts;
        for (int it = tid; it < n * parts; it += NT) {
            const int q = it / n;          // lanes of a wave share q: the hk reads are broadcasts
            const int e = it - q * n;
            const uint64_t k = hk[2 * e];
            const int cls = class_of(k);
            const int f1 = min(n, (q + 1) * span);
            int c = 0;
            for (int f = q * span; f < f1; ++f) c += (class_of(hk[2 * f]) == cls && hk[2 * f] > k) ? 1 : 0;
            if (c) atomicAdd(&heavier[e], c);
        }
        __syncthreads();
        for (int e = tid; e < n; e += NT) {
            const int r = heavier[e];
            if (r < depth) {
                const uint64_t k = hk[2 * e];
                cl[class_of(k) * depth + r] = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
            }
        }
    } else {
        // Rank each entry within its own class only: the entries of a class
        // are linked into a list (head in the class's first CL slot, next in
        // the low word of hk[2 e + 1]; the rank goes to its high word).  An
        // entry whose class list runs past kWalk entries compares against
        // all n instead.
        constexpr int kWalk = 32;
        for (int e = tid; e < n; e += NT)
            hk[2 * e + 1] = (uint32_t)atomicExch(&cl[class_of(hk[2 * e]) * depth], e);
        __syncthreads();
        for (int e = tid; e < n; e += NT) {
            const uint64_t k = hk[2 * e];
            const int cls = class_of(k);
            int r = 0;
            int f = cl[cls * depth];
            for (int st = 0; f >= 0 && st < kWalk; ++st) {
                r += hk[2 * f] > k ? 1 : 0;
                f = (int)(uint32_t)hk[2 * f + 1];
            }
            if (f >= 0) {
                r = 0;
                for (f = 0; f < n; ++f) r += (class_of(hk[2 * f]) == cls && hk[2 * f] > k) ? 1 : 0;
            }
            hk[2 * e + 1] = ((uint64_t)(uint32_t)r << 32) | (uint32_t)hk[2 * e + 1];   // the low word stays
        }
        __syncthreads();
        for (int c = tid; c < s1; c += NT) cl[c * depth] = -1;
        __syncthreads();
        for (int e = tid; e < n; e += NT) {
            const int r = (int)(hk[2 * e + 1] >> 32);
            const uint64_t k = hk[2 * e];
            if (r < depth) cl[class_of(k) * depth + r] = (int32_t)(0xffffffffu - (uint32_t)(k & 0xffffffffu));
        }
    }
    __syncthreads();
    for (int i = tid; i < s1 * depth; i += NT) CL[i] = cl[i];
}

// emit_heavy for keys held in registers: each thread holds up to NK keys
// (slot q valid when bit q of `valid` is set) as hi[q] = key >> 32; the low
// half lo(q, th) of slot q of thread th is computed on demand (q may be a
// run-time value there).  The class of a key is its bin mod s1, and
// ct.count threads ct(c, i) hold every key of class c (they may hold keys of
// other classes too).  Same outputs as emit_heavy, except that H holds the
// heavy bins in an unspecified order.  Each thread's heavy slots go to hk at
// its exclusive-sum offset as (hi, thread, slot); thread e then completes
// entry e (its bin) and ranks it within its class against the entries of
// the threads of that class.
// offs: LDS int32[2 NT]; part: LDS int32[NT / 64]; hk: LDS uint64[T];
// cl: LDS int32[s1 * depth].
template <int NT, int NK, class LoF, class ClassThreads>
__device__ void emit_heavy_regs(const uint32_t (&hi)[NK], uint64_t valid, LoF lo, ClassThreads ct, int lg, int T,
                                int depth, uint64_t thr, uint64_t* hk, int32_t* offs, int32_t* part, int32_t* cl,
                                GLOBAL int32_t* __restrict__ H, GLOBAL uint64_t* __restrict__ thr_out,
                                GLOBAL int32_t* __restrict__ CL) {
    static_assert(NK <= 64 && NT <= (1 << 24), "slot and thread fields");
    const int tid = (int)threadIdx.x;
    const int s1 = 1 << lg;
    if (tid == 0) *thr_out = thr;
    for (int i = tid; i < s1 * depth; i += NT) cl[i] = -1;
    const uint32_t thi = (uint32_t)(thr >> 32), tlo = (uint32_t)thr;
    uint64_t hm = 0;
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        if ((valid >> q) & 1) {
            if (hi[q] > thi) hm |= (uint64_t)1 << q;
            else if (hi[q] == thi && lo(q, tid) >= tlo) hm |= (uint64_t)1 << q;   // ties on |E|^2: rare
        }
    }
    const int cnt = __popcll(hm);
    const int ex = block_exclusive_sum<NT, false>(cnt, part);   // part is not reused in this block
    offs[tid] = ex;
    offs[NT + tid] = cnt;
#pragma unroll
    for (int q = 0; q < NK; ++q) {
        if ((hm >> q) & 1) {
            const int e = ex + __popcll(hm & (((uint64_t)1 << q) - 1));
            if (e < T) hk[e] = ((uint64_t)hi[q] << 32) | (uint32_t)((tid << 6) | q);
        }
    }
    __syncthreads();
    const int n = min(offs[NT - 1] + offs[2 * NT - 1], T);
    for (int e = tid; e < n; e += NT) {   // entry e is read and rewritten by this thread only
        const uint64_t v = hk[e];
        const uint32_t l = lo((int)(v & 63), (int)((uint32_t)v >> 6));
        hk[e] = (v & 0xffffffff00000000ull) | l;
        H[e] = (int32_t)(0xffffffffu - l);
    }
    __syncthreads();
    const uint32_t cmask = (uint32_t)s1 - 1;
    for (int e = tid; e < n; e += NT) {
        const uint64_t mine = hk[e];
        const uint32_t hb = 0xffffffffu - (uint32_t)(mine & 0xffffffffu);
        const int c = (int)(hb & cmask);
        int r = 0;
        for (int i0 = 0; i0 < ct.count; i0 += 8) {   // the entry ranges of 8 class threads at a time
            int o2[8], o3[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                o2[u] = o3[u] = 0;
                if (i0 + u < ct.count) {
                    const int t2 = ct(c, i0 + u);
                    o2[u] = offs[t2];
                    o3[u] = offs[NT + t2];
                }
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int end = min(o2[u] + o3[u], T);
                for (int e2 = o2[u]; e2 < end; ++e2) {
                    const uint64_t k2 = hk[e2];
                    r += (k2 > mine && ((0xffffffffu - (uint32_t)(k2 & 0xffffffffu)) & cmask) == (uint32_t)c) ? 1 : 0;
                }
            }
        }
        if (r < depth) cl[c * depth + r] = (int32_t)hb;
    }
    __syncthreads();
    for (int i = tid; i < s1 * depth; i += NT) CL[i] = cl[i];
}

static_assert(2 * kDftThreads <= kSelBins, "emit_heavy_regs offsets live in the histogram");


// The value held by lane l ^ 1 (DPP quad permutation 1, 0, 3, 2); every lane
// of the wave must be active.
__device__ __forceinline__ float lane_pair(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// The value held by lane l ^ 8 within each row of 16 lanes (DPP row rotation
// by 8); every lane of the wave must be active.
__device__ __forceinline__ float lane_half(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xF, 0xF, false));
}

// Column layout of k_dft's matrix-core step: wave w owns the N-tiles of the
// 16 complex columns 16 w .. 16 w + 15 (tiles 2 w and 2 w + 1, s1 = 128) or
// the 8 columns 8 w .. 8 w + 7 (s1 = 64), and lane l of an N-tile reads the
// real part (l % 16 < 8) or the imaginary part (l % 16 >= 8) of the tile's
// column l % 8, so that after the combine lanes 0-7 of a row hold X_k and
// lanes 8-15 X_{p-k} of eight consecutive columns.
__device__ __forceinline__ int mx_tile(int w, int t, int ntw) { return ntw == 2 ? 2 * w + t : w; }
__device__ __forceinline__ int mx_fcol(int li) { return ((li & 7) << 1) | (li >> 3); }

// Step B on the matrix cores.  Real form of the p-point step: N = 2 c + part
// indexes the real (part 0) and imaginary (part 1) planes of the [p][s1]
// block, a_n = x_n + x_{p-n}, b_n = x_n - x_{p-n}, and for k = 0..h
//   Cm[k][N] = sum_{n=1..h} cos(2 pi n k / p) a_n[N],
//   Dm[k][N] = sum_{n=1..h} sin(2 pi n k / p) b_n[N]
// (row k = 0 of the cosine matrix is all ones: Cm[0] = sum_n a_n).  Tiles are
// FP32 16x16x4 MFMAs: M = 16 values of k, N = 16 floats (8 columns), K = 4
// values of n.  Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and
// receives D[4 (l / 16) + r][l % 16] in register r.  Wave w owns the N-tiles
// mx_tile(w, t), t < NTW = s1 / 64 (lane l reading float mx_fcol(l % 16) of
// the tile), and the M-tiles m < MT = ceil((h + 1) / 16).
// bf: the block as floats, columns swizzled by swz_col.  At: the A operands in
// lane order ((st ATILES + m) 64 + lane, as the plan's mxa and mxc tables), in
// LDS or global memory; an: on entry the operands of step 0
// (At[m 64 + lane]); each step's A operands and the B operands (four LDS
// reads per N-tile) are loaded one step ahead.  A lane's rows n and p - n
// move by 4 per step, so their swizzle stays the same and the reads of the
// steps before the last are fixed offsets from two addresses.
__device__ __forceinline__ float2 load_a(const float2* p) { return *p; }
__device__ __forceinline__ float2 load_a(const GLOBAL float2* p) { return ld2(p); }

template <int MT, int NTW, int ATILES = kMxTiles, class AP>
__device__ __forceinline__ void pfa_mfma(const float* bf, int p, int h, AP At, float2 (&an)[kMxTiles],
                                         mf4 (&Cm)[2][kMxTiles], mf4 (&Dm)[2][kMxTiles]) {
    static_assert(MT <= ATILES && MT <= kMxTiles && NTW <= 2, "A operand tiles");
    constexpr int RS = 128 * NTW;   // floats per row: s1 = 64 NTW
    const int lane = (int)threadIdx.x & 63;
    const int wid = (int)threadIdx.x >> 6;
    const int li = lane & 15;
    const int lk = lane >> 4;
#pragma unroll
    for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            Cm[t][m] = mf4{0.f, 0.f, 0.f, 0.f};
            Dm[t][m] = mf4{0.f, 0.f, 0.f, 0.f};
        }
    const int steps = (h + 3) >> 2;   // <= kMxSteps
    int col[NTW];                     // the lane's float column in each N-tile
#pragma unroll
    for (int t = 0; t < NTW; ++t) col[t] = 16 * mx_tile(wid, t, NTW) + mx_fcol(li);
    auto at = [&](int row, int t) { return row * RS + (col[t] ^ (2 * swz_col(row))); };
    const int ra = 1 + lk, rb = p - 1 - lk;   // the lane's rows n and p - n at step 0
    int oa[NTW], ob[NTW];
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
        oa[t] = at(ra, t);
        ob[t] = at(rb, t);
    }
    // B operands of step st: rows n = 1 + 4 st + lk and p - n; in the last
    // step rows past h are clamped into the block (their values are not used)
    auto fetch = [&](int st, float (&va)[NTW], float (&vb)[NTW]) {
        if (4 * st + 4 <= h) {   // every lane's n <= h (uniform)
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                va[t] = bf[oa[t] + st * 4 * RS];
                vb[t] = bf[ob[t] - st * 4 * RS];
            }
        } else {
            const int n = 1 + 4 * st + lk;
            const int r1 = min(n, p - 1), r2 = max(p - n, 0);
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                va[t] = bf[at(r1, t)];
                vb[t] = bf[at(r2, t)];
            }
        }
    };
    float xa[NTW], xb[NTW];
    fetch(0, xa, xb);
#pragma unroll
    for (int st = 0; st < kMxSteps; ++st) {
        if (st >= steps) break;
        float2 av[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) av[m] = an[m];
        float ya[NTW], yb[NTW];
        if (st + 1 < steps) {
#pragma unroll
            for (int m = 0; m < MT; ++m) an[m] = load_a(At + ((st + 1) * ATILES + m) * 64 + lane);
            fetch(st + 1, ya, yb);
        }
        const bool nin = 1 + 4 * st + lk <= h;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const float a_n = nin ? xa[t] + xb[t] : 0.f;
            const float b_n = nin ? xa[t] - xb[t] : 0.f;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                Cm[t][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m].x, a_n, Cm[t][m], 0, 0, 0);
                Dm[t][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m].y, b_n, Dm[t][m], 0, 0, 0);
            }
        }
        if (st + 1 < steps) {
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                xa[t] = ya[t];
                xb[t] = yb[t];
            }
        }
    }
}

// pfa_mfma for the split path's column tiles (no swizzle, run-time tile counts).
template <int MT, int NTW, int ATILES = kMxTiles, class AP>
__device__ __forceinline__ void pfa_mfma_cols(const float* bf, int s1, int p, int h, int mt, int ntw, AP At,
                                         float2 (&an)[MT], mf4 (&Cm)[NTW][MT], mf4 (&Dm)[NTW][MT]) {
    static_assert(MT <= ATILES, "A operand tiles");
    const int lane = (int)threadIdx.x & 63;
    const int wid = (int)threadIdx.x >> 6;
    const int li = lane & 15;
    const int lk = lane >> 4;
    const int rs = 2 * s1;   // floats per row
#pragma unroll
    for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            Cm[t][m] = mf4{0.f, 0.f, 0.f, 0.f};
            Dm[t][m] = mf4{0.f, 0.f, 0.f, 0.f};
        }
    const int steps = (h + 3) >> 2;
    for (int st = 0; st < steps; ++st) {
        const int n = 1 + 4 * st + lk;   // the K index this lane supplies
        const bool nin = n <= h;
        float2 av[MT];
#pragma unroll
        for (int m = 0; m < MT; ++m) av[m] = an[m];
        if (st + 1 < steps) {
#pragma unroll
            for (int m = 0; m < MT; ++m) an[m] = load_a(At + ((st + 1) * ATILES + m) * 64 + lane);
        }
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            if (t >= ntw) break;
            const int N = 16 * (wid + 8 * t) + li;
            float a_n = 0.f, b_n = 0.f;
            if (nin) {
                const float xa = bf[n * rs + N];
                const float xb = bf[(p - n) * rs + N];
                a_n = xa + xb;
                b_n = xa - xb;
            }
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                if (m >= mt) break;
                Cm[t][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m].x, a_n, Cm[t][m], 0, 0, 0);
                Dm[t][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[m].y, b_n, Dm[t][m], 0, 0, 0);
            }
        }
    }
}

// Threads of the VALU step B holding residue class c: (i << lg) + c.
struct ValuClassThreads {
    int count, lg;
    __device__ int operator()(int c, int i) const { return (i << lg) + c; }
};
// Threads of the MFMA step B holding residue class c (column c): the wave
// of its N-tile (mx_tile), lanes 16 lk + 8 part + c mod 8.
struct MfmaClassThreads {
    int count;   // 8
    int sh;      // wave of column c: c >> sh (4: s1 = 128, 3: s1 = 64)
    __device__ int operator()(int c, int i) const { return 64 * (c >> sh) + 16 * (i >> 1) + 8 * (i & 1) + (c & 7); }
};

// One workgroup per (modulus j, band b); the whole block in LDS.
// MT == 0: step B on the vector ALUs.  Requires s1 <= kDftThreads and
// ceil(h / (kDftThreads / s1)) <= KBMAX, h = (p-1)/2 (KBMAX = 8 keeps two
// workgroups per CU; 16 serves s1 = 256).  One work item per thread (output
// group g = tid / s1 of column c = tid mod s1); the results are written to E
// and their selection keys stay in registers (slots 2 kk and 2 kk + 1: rows
// k0 + kk and p - k0 - kk; slot 2 KBMAX: row 0, group 0 only).
// MX: step B on the matrix cores (pfa_mfma, up to MT = NTW = 2).  Requires
// s1 = 64 or 128 and h + 1 <= 32 for every modulus.  Slot (t MT + m) 4 + r
// holds the key of row k = 16 m + 4 r + l / 16 of N-tile mx_tile(w, t): X_k
// in lanes l % 16 < 8, X_{p-k} in the others (row 0 in the first only); the
// rows of a register are consecutive, so registers whose rows all exceed h
// are skipped.  The bins go to E as whole 128-byte lines (s1 = 128).  LDS: the block
// and the s1 twiddles only (the A operands come from the plan's table in
// global memory); the selection's scratch reuses the block's space, so a
// launch over the smaller moduli (BatchArgs::jn) needs less LDS per
// workgroup and fits more workgroups per CU.
template <int KBMAX, bool MX>
__global__ void __launch_bounds__(kDftThreads) k_dft(BatchArgs a) {
    constexpr int MT = MX ? 2 : 0;
    constexpr int NTW = 2;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NT = kDftThreads;
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int K = d->K;
    // A launch may cover the moduli [jlo, jlo + nj) only (jn > 0), so that
    // the smaller blocks get a smaller LDS allocation and more workgroups per CU.
    const int jlo = a.jn > 0 ? a.jlo : 0;
    const int nj = a.jn > 0 ? a.jn : K;
    // blocks nj Q .. 2 nj Q - 1 (phase identification): the bins of the samples
    // at the nodes moved one grid step, transformed and stored only
    const bool shifted = at.blk >= nj * Q;
    const int blk0 = shifted ? at.blk - nj * Q : at.blk;
    const int j = jlo + blk0 / Q;
    const int b = blk0 - (j - jlo) * Q;
    const int p = d->p[j];
    const int P = d->P[j];
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int Pmax = d->P[jlo + nj - 1];   // the moduli ascend
    const int hmax = (d->p[jlo + nj - 1] - 1) >> 1;
    const int h = (p - 1) >> 1;
    const size_t base = (size_t)Q * d->Moff[j] + (size_t)b * P;

    float2* buf = reinterpret_cast<float2*>(smem);
    float2* tw = reinterpret_cast<float2*>(smem + (size_t)Pmax * 8);   // [s1]
    float2* trig = tw + s1;   // VALU step B: the cosine/sine table [hmax^2]
    // selection scratch: after the table (VALU step B), or over the block
    // once step B has read it (MX)
    // MX: the first digit's histogram is formed as the bins are, past the
    // block and twiddles and past the rest of the scratch, which overlays them
    const size_t mx_ovl = 64 + (size_t)d->T * 8 + (size_t)s1 * d->depth * 4;
    int32_t* hist = MX ? reinterpret_cast<int32_t*>(smem + max((size_t)Pmax * 8 + (size_t)s1 * 8, mx_ovl))
                       : reinterpret_cast<int32_t*>(trig + hmax * hmax);
    int32_t* part = MX ? reinterpret_cast<int32_t*>(smem) : hist + kSelBins;
    uint64_t* hk = reinterpret_cast<uint64_t*>(part + 16);   // [T]
    int32_t* cl = reinterpret_cast<int32_t*>(hk + d->T);        // [s1 depth]

    const GLOBAL float2* __restrict__ S = glb(shifted ? io.S2 : io.S) + base;
    constexpr int MTA = MX ? 2 : 1;
    const GLOBAL float2* A = glb(d->mxa) + (size_t)j * kMxSteps * kMxTiles * 64;   // MX: [step][tile][lane]
    float2 a0[MTA];   // MX: the A operands of step B's first K-step
    if constexpr (MX) {
        // every load of the block in flight at once: samples, twiddles, the
        // first A operands of the p-point step (the others are read from the
        // plan's table, one K-step ahead, as the step runs)
        float2 w = make_float2(0.f, 0.f);
        if (tid < (s1 >> 1)) w = ld2(glb(d->tw_s1) + tid);
#pragma unroll
        for (int m = 0; m < MTA; ++m) a0[m] = ld2(A + m * 64 + (tid & 63));
        copy_to_lds<NT, 8>(buf, S, P);
        if (tid < (s1 >> 1)) {   // the full circle: W^(m + s1/2) = -W^m
            tw[tid] = w;
            tw[tid + (s1 >> 1)] = make_float2(-w.x, -w.y);
        }
        for (int i = tid; i < kSelBins; i += NT) hist[i] = 0;
    } else {
        copy_to_lds<NT, 8>(buf, S, P);
        for (int i = tid; i < (s1 >> 1); i += NT) {   // the full circle: W^(m + s1/2) = -W^m
            const float2 w = ld2(glb(d->tw_s1) + i);
            tw[i] = w;
            tw[i + (s1 >> 1)] = make_float2(-w.x, -w.y);
        }
        load_trig<NT>(trig, h, glb(d->trig) + d->trig_off[j]);
    }
    __syncthreads();
    // MX: p <= 63 rows in one pass; VALU: whole blocks of any height, in chunks
    fft_rows<NT, 64, 64, MX, MX ? 0 : 64, !MX>(buf, p, s1, lg, tw);

    // step B
    GLOBAL float2* __restrict__ E = glb(shifted ? io.E2 : io.E) + base;
    const float scale = 1.0f / (float)P;
    const uint32_t cA = (uint32_t)p * (uint32_t)d->pinv_s1[j];
    const uint32_t cB = (uint32_t)s1 * (uint32_t)d->s1inv_p[j];
    constexpr int NK = MT > 0 ? NTW * MT * 4 : 2 * KBMAX + 1;
    uint32_t hi[NK];   // selection keys: |E|^2 bits; the low halves (2^32 - 1 - h) come from pos_of
    uint64_t valid = 0;
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int li = lane & 15;
    const int lk = lane >> 4;
    const int plane = li >> 3;   // MFMA step B: 0 real plane / X_k, 1 imaginary plane / X_{p-k}
    if constexpr (MT > 0) {
        mf4 Cm[NTW][MT], Dm[NTW][MT];
        const float* bf = reinterpret_cast<const float*>(buf);
        const int mt = (h + 16) >> 4;
        const int ntw = s1 >> 6;
        static_assert(MT == MTA && MT == kMxTiles && NTW == 2, "first A operands");
        if (mt == 2) {
            if (ntw == 2) pfa_mfma<2, 2>(bf, p, h, A, a0, Cm, Dm);
            else pfa_mfma<2, 1>(bf, p, h, A, a0, Cm, Dm);
        } else {
            if (ntw == 2) pfa_mfma<1, 2>(bf, p, h, A, a0, Cm, Dm);
            else pfa_mfma<1, 1>(bf, p, h, A, a0, Cm, Dm);
        }
        const float sgn = plane ? -1.f : 1.f;
#pragma unroll
        for (int q = 0; q < NK; ++q) hi[q] = 0;
        float x0v[NTW];
#pragma unroll
        for (int t = 0; t < NTW; ++t) x0v[t] = t < ntw ? bf[16 * mx_tile(wid, t, ntw) + mx_fcol(li)] : 0.f;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
            if (m >= mt) break;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (16 * m + 4 * r > h) break;   // rows 16 m + 4 r .. + 3: all padding (uniform)
                const int k = 16 * m + 4 * r + lk;
                float2 x[NTW];
#pragma unroll
                for (int t = 0; t < NTW; ++t) {
                    if (t >= ntw) break;
                    const int q = (t * MT + m) * 4 + r;
                    const float cv = Cm[t][m][r];
                    const float dp = lane_half(Dm[t][m][r]);
                    const float xk = (x0v[t] + cv + sgn * dp) * scale;
                    const float xm = (x0v[t] + cv - sgn * dp) * scale;
                    const float xk2 = lane_half(xk);
                    const float xm2 = lane_half(xm);
                    // lanes 0-7 hold X_k = (xk, xk2), lanes 8-15 X_{p-k} = (xm2, xm)
                    x[t] = make_float2(plane ? xm2 : xk, plane ? xm : xk2);
                    hi[q] = __float_as_uint(fmaf(x[t].x, x[t].x, x[t].y * x[t].y));
                    if (k <= h && (plane == 0 || k >= 1)) {   // X_0 once
                        valid |= (uint64_t)1 << q;
                        if (!shifted && (int32_t)hi[q] >= 0) atomicAdd(&hist[hi[q] >> (31 - kSelBits)], 1);
                    }
                }
                if (ntw == 2) {
                    // rows k and p - k of the wave's 16 columns, one full 128-byte line per
                    // 16 lanes: lanes 0-7 of tile 2w with lanes 0-7 of tile 2w + 1 (row k),
                    // lanes 8-15 of both (row p - k); streamed, as the lines are whole
                    const float2 y0 = make_float2(lane_half(x[0].x), lane_half(x[0].y));
                    const float2 y1 = make_float2(lane_half(x[1].x), lane_half(x[1].y));
                    const uint32_t col = (uint32_t)(16 * wid + li);
                    if (k <= h) st2s(E + ((uint32_t)k << lg) + col, plane ? y1 : x[0]);
                    if (k >= 1 && k <= h) st2s(E + ((uint32_t)(p - k) << lg) + col, plane ? x[1] : y0);
                } else if (k <= h && (plane == 0 || k >= 1)) {
                    const uint32_t row = plane ? (uint32_t)(p - k) : (uint32_t)k;
                    st2s(E + (row << lg) + (uint32_t)(8 * wid + (li & 7)), x[0]);
                }
            }
        }
    } else {
    const int ng = NT >> lg;
    const int KB = (h + ng - 1) / ng;
    const int g = tid >> lg;
    const int c = tid & (s1 - 1);
    const int k0 = 1 + g * KB;
    const float2 x0 = buf[c];
    float2 C[KBMAX], D[KBMAX], sa;
    pfa_column_sums<KBMAX>(buf, s1, c, p, h, k0, KB, trig, C, D, sa);
#pragma unroll
    for (int kk = 0; kk < KBMAX; ++kk) {
        const int k = k0 + kk;
        hi[2 * kk] = hi[2 * kk + 1] = 0;
        if (kk < KB && k <= h) {
            const float2 xk = make_float2((x0.x + C[kk].x + D[kk].y) * scale, (x0.y + C[kk].y - D[kk].x) * scale);
            const float2 xm = make_float2((x0.x + C[kk].x - D[kk].y) * scale, (x0.y + C[kk].y + D[kk].x) * scale);
            st2s(E + (k << lg) + c, xk);
            st2s(E + ((p - k) << lg) + c, xm);
            hi[2 * kk] = __float_as_uint(fmaf(xk.x, xk.x, xk.y * xk.y));
            hi[2 * kk + 1] = __float_as_uint(fmaf(xm.x, xm.x, xm.y * xm.y));
            valid |= (uint64_t)3 << (2 * kk);
        }
    }
    hi[NK - 1] = 0;
    if (g == 0) {
        const float2 xz = make_float2((x0.x + sa.x) * scale, (x0.y + sa.y) * scale);
        st2s(E + c, xz);
        hi[NK - 1] = __float_as_uint(fmaf(xz.x, xz.x, xz.y * xz.y));
        valid |= (uint64_t)1 << (NK - 1);
    }
    }
    if (shifted) return;   // uniform over the block
    if constexpr (MX) __syncthreads();   // the selection's scratch overlays the block, which step B has read
    // Good-Thomas position of slot q of thread th
    auto pos_of = [&](int q, int th) -> int {
        if constexpr (MT > 0) {
            const int t = q / (MT * 4);
            const int k = 16 * ((q >> 2) % MT) + 4 * (q & 3) + ((th >> 4) & 3);
            const int c = 8 * mx_tile(th >> 6, t, s1 >> 6) + (th & 7);
            return (((th >> 3) & 1 ? p - k : k) << lg) + c;
        } else {
            const int c = th & (s1 - 1);
            if (q == NK - 1) return c;
            const int ng = NT >> lg;
            const int k = 1 + (th >> lg) * ((h + ng - 1) / ng) + (q >> 1);
            return (((q & 1) ? p - k : k) << lg) + c;
        }
    };
    // The thread index passes through an empty asm so that the position
    // arithmetic stays where a low half is needed (rarely) instead of being
    // hoisted or speculated and held in registers for every slot.
    auto lo_of = [&](int q, int th) -> uint32_t {
        asm volatile("" : "+v"(th));
        return 0xffffffffu - pfa_bin(pos_of(q, th), lg, s1, (uint32_t)P, cA, cB);
    };
    // MX: the slots that hold a key in some lane (the register's rows are not
    // all padding), wave-uniform, so that the passes branch over the others
    // (NK <= 32 there; the VALU form has up to 33 slots and no padding slots)
    uint32_t live = 0xffffffffu;
    if constexpr (MT > 0) {
        static_assert(NK <= 32, "one bit per slot");
        live = 0;
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            const int t = q / (MT * 4), m = (q >> 2) % MT, r = q & 3;
            if (t < (s1 >> 6) && 16 * m + 4 * r <= h) live |= 1u << q;
        }
        live = __builtin_amdgcn_readfirstlane(live);
    }
    auto each = [&](auto f) {
#pragma unroll
        for (int q = 0; q < NK; ++q) {
            if constexpr (MT > 0) {
                if (!((live >> q) & 1)) continue;
            }
            if ((valid >> q) & 1) f(hi[q], [&] { return ((uint64_t)hi[q] << 32) | lo_of(q, tid); });
        }
    };
    const uint64_t thr = kth_largest<NT, MX>(each, P, d->T, hist, part);
    const size_t blk = (size_t)(j * Q + b);
    auto emit = [&](auto ct) {
        emit_heavy_regs<NT, NK>(hi, valid, lo_of, ct, lg, d->T, d->depth, thr, hk, hist, part, cl,
                                glb(io.H) + blk * d->T, glb(io.thr) + blk, glb(io.CL) + blk * (size_t)s1 * d->depth);
    };
    if constexpr (MT > 0) emit(MfmaClassThreads{8, lg == 7 ? 4 : 3});
    else emit(ValuClassThreads{NT >> lg, lg});
}

// Split path, step A: block -> (modulus j, band b, chunk of rows_per rows).
__device__ __forceinline__ void split_rows_where(const CONSTANT SigDesc* d, int blk, int rows_per, int& j, int& b, int& chunk) {
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
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int rows_per = max(1, kRowElems >> lg);
    // blocks past the first set (phase identification): the samples at the
    // nodes moved one grid step
    int nrows1 = 0;
    for (int jj = 0; jj < d->K; ++jj) nrows1 += d->Q * ((d->p[jj] + rows_per - 1) / rows_per);
    const bool shifted = at.blk >= nrows1;
    int j, b, chunk;
    split_rows_where(d, shifted ? at.blk - nrows1 : at.blk, rows_per, j, b, chunk);
    const int p = d->p[j];
    const int r0 = chunk * rows_per;
    const int rows = min(rows_per, p - r0);
    const size_t base = (size_t)d->Q * d->Moff[j] + (size_t)b * d->P[j] + ((size_t)r0 << lg);
    if (io.SH && chunk == 0 && !shifted) {   // the block's top-digit histogram, filled by the column kernel
        GLOBAL int32_t* sh = glb(io.SH) + (size_t)(j * d->Q + b) * kSelBins;
        for (int i = tid; i < kSelBins; i += kThreads) sh[i] = 0;
    }
    float2* buf = reinterpret_cast<float2*>(smem);
    float2* tw = buf + ((size_t)rows_per << lg);
    const int n = rows << lg;
    const GLOBAL float2* __restrict__ S = glb(shifted ? io.S2 : io.S) + base;
    copy_to_lds<kThreads, 8>(buf, S, n);
    for (int i = tid; i < (s1 >> 1); i += kThreads) {   // the full circle: W^(m + s1/2) = -W^m
        const float2 w = ld2(glb(d->tw_s1) + i);
        tw[i] = w;
        tw[i + (s1 >> 1)] = make_float2(-w.x, -w.y);
    }
    __syncthreads();
    // rows are transformed independently, as in the in-LDS kernels
    fft_rows<kThreads, kRowElems / 128, kRowElems / 64, false, kRowElems / 256, false, kRowElems>(buf, rows, s1, lg, tw);
    GLOBAL float2* __restrict__ X = glb(shifted ? io.E2 : io.E) + base;   // the bins' buffer holds the step-A result
    for (int i = tid; i < n; i += kThreads) st2s(X + i, buf[i]);
}

// Split path, step B: block -> (modulus j, band b, 64 columns); in place on E.
__global__ void __launch_bounds__(kThreads) k_dft_cols(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int C = min(kColChunk, s1);
    const int nc = s1 / C;
    int blk = at.blk;
    const bool shifted = blk >= d->K * Q * nc;   // phase identification: the shifted samples' bins
    if (shifted) blk -= d->K * Q * nc;
    const int j = blk / (Q * nc);
    blk -= j * Q * nc;
    const int b = blk / nc;
    const int c0 = (blk - b * nc) * C;
    const int p = d->p[j];
    const int P = d->P[j];
    int pmax = 0;
    for (int jj = 0; jj < d->K; ++jj) pmax = max(pmax, d->p[jj]);
    const size_t base = (size_t)Q * d->Moff[j] + (size_t)b * P;
    float2* tile = reinterpret_cast<float2*>(smem);   // [p][C]
    float2* trig = tile + (size_t)pmax * C;
    GLOBAL float2* __restrict__ E = glb(shifted ? io.E2 : io.E) + base;
    constexpr int U = 8;   // loads of a thread in flight before its LDS writes
    for (int i0 = tid; i0 < p * C; i0 += U * kThreads) {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kThreads;
            if (i < p * C) {
                const int n2 = i / C;
                v[u] = ld2(E + ((size_t)n2 << lg) + c0 + (i - n2 * C));
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kThreads;
            if (i < p * C) tile[i] = v[u];
        }
    }
    load_trig<kThreads>(trig, (p - 1) >> 1, glb(d->trig) + d->trig_off[j]);
    __syncthreads();
    dft_cols_lds<kThreads>(tile, C, C, p, trig, E + c0, s1, 1.0f / (float)P);
}

// Split path, step B on the matrix cores: block -> (modulus j, band b, 64
// columns), 8 waves; in place on E.  The 64 columns of the tile are the
// 128 real columns of pfa_mfma with one N-tile per wave (its s1 is the tile
// width), the A operands come from the plan's larger table (h <= 47), and
// the outputs are combined and stored exactly as in k_dft's matrix-core path,
// so both give the same bins bit for bit.
__global__ void __launch_bounds__(kDftThreads) k_dft_cols_mx(BatchArgs a) {
    constexpr int NT = kDftThreads;
    constexpr int C = 64;
    static_assert(NT / 64 * 16 == 2 * C, "one N-tile per wave");
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int nc = s1 / C;
    int blk = at.blk;
    const bool shifted = blk >= d->K * Q * nc;   // phase identification: the shifted samples' bins
    if (shifted) blk -= d->K * Q * nc;
    const int j = blk / (Q * nc);
    blk -= j * Q * nc;
    const int b = blk / nc;
    const int c0 = (blk - b * nc) * C;
    const int p = d->p[j];
    const int P = d->P[j];
    const int h = (p - 1) >> 1;
    const size_t base = (size_t)Q * d->Moff[j] + (size_t)b * P;
    float2* tile = reinterpret_cast<float2*>(smem);   // [p][C]
    // the top key digit (bits 30..21 of |E|^2) of the tile's bins, added to the
    // block's histogram for the selection (not for the shifted bins)
    const bool hist_on = io.SH != nullptr && !shifted;
    int32_t* hist = reinterpret_cast<int32_t*>(smem + (size_t)p * C * 8 + 64);   // [kSelBins], past the tile
    if (hist_on)
        for (int i = tid; i < kSelBins; i += kDftThreads) hist[i] = 0;   // ordered by the barrier below
    GLOBAL float2* __restrict__ E = glb(shifted ? io.E2 : io.E) + base;
    // the A operands [kMxcSteps][kMxcTiles][64] come from the plan's table
    // (L2-resident), one K-step ahead, as in k_dft
    const GLOBAL float2* __restrict__ A = glb(d->mxc) + (size_t)j * kMxcSteps * kMxcTiles * 64;
    constexpr int MT = kMxcTiles;
    float2 a0[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) a0[m] = ld2(A + m * 64 + (tid & 63));
    constexpr int U = 8;   // loads of a thread in flight before its LDS writes
    for (int i0 = tid; i0 < p * C; i0 += U * NT) {
        float2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * NT;
            if (i < p * C) v[u] = ld2(E + ((size_t)(i / C) << lg) + c0 + (i % C));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * NT;
            if (i < p * C) tile[i] = v[u];
        }
    }
    __syncthreads();
    mf4 Cm[1][MT], Dm[1][MT];
    const float* bf = reinterpret_cast<const float*>(tile);
    const int mt = (h + 16) >> 4;
    pfa_mfma_cols<MT, 1, kMxcTiles>(bf, C, p, h, mt, 1, A, a0, Cm, Dm);
    const int lane = tid & 63;
    const int wid = tid >> 6;
    const int li = lane & 15;
    const int lk = lane >> 4;
    const int plane = li & 1;
    const float sgn = plane ? -1.f : 1.f;
    const float scale = 1.0f / (float)P;
    const int N = 16 * wid + li;
    const int c = c0 + (N >> 1);
    const float x0v = bf[N];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        if (m >= mt) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int k = 16 * m + 4 * lk + r;
            const float cv = Cm[0][m][r];
            const float dp = lane_pair(Dm[0][m][r]);
            const float xk = (x0v + cv + sgn * dp) * scale;
            const float xm = (x0v + cv - sgn * dp) * scale;
            const float xk2 = lane_pair(xk);
            const float xm2 = lane_pair(xm);
            const float re = plane ? xm2 : xk;
            const float im = plane ? xm : xk2;
            if (k <= h && (plane == 0 || k >= 1)) {
                const uint32_t row = plane ? (uint32_t)(p - k) : (uint32_t)k;
                st2(E + (row << lg) + (uint32_t)c, make_float2(re, im));   // two waves per line: plain
                if (hist_on)
                    atomicAdd(&hist[(__float_as_uint(fmaf(re, re, im * im)) >> (31 - kSelBits)) & (kSelBins - 1)], 1);
            }
        }
    }
    if (hist_on) {
        __syncthreads();
        int32_t* sh = io.SH + (size_t)(j * Q + b) * kSelBins;
        for (int i = tid; i < kSelBins; i += kDftThreads) {
            const int v = hist[i];
            if (v) atomicAdd(sh + i, v);
        }
    }
}

// Split path, selection: one workgroup per (modulus j, band b), E in global
// memory.  LDSKEYS: the |E|^2 bits of the block are read once into LDS and
// every pass reads them there (blocks whose keys fit the LDS); otherwise each
// pass reads E.  The keys and the outputs are the same either way.
template <int NT, bool LDSKEYS>
__global__ void __launch_bounds__(NT) k_select(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int Q = d->Q;
    const int j = at.blk / Q;
    const int b = at.blk - j * Q;
    const int p = d->p[j];
    const int P = d->P[j];
    const int s1 = d->s1;
    const int lg = d->log2s1;
    int32_t* hist = reinterpret_cast<int32_t*>(smem);
    int32_t* part = hist + kSelBins;
    uint64_t* hk = reinterpret_cast<uint64_t*>(part + 16);   // [2 T]
    int32_t* cl = reinterpret_cast<int32_t*>(hk + 2 * d->T);   // [s1 depth]
    uint32_t* keys = reinterpret_cast<uint32_t*>(cl + ((s1 * d->depth + 3) & ~3));   // [P] (LDSKEYS)
    const GLOBAL float2* __restrict__ E = glb(io.E) + (size_t)Q * d->Moff[j] + (size_t)b * P;
    const uint32_t cA = (uint32_t)p * (uint32_t)d->pinv_s1[j];
    const uint32_t cB = (uint32_t)s1 * (uint32_t)d->s1inv_p[j];
    if constexpr (LDSKEYS) {
        constexpr int U = 8;   // loads of a thread in flight at once
        for (int i0 = (int)threadIdx.x; i0 < P; i0 += U * NT) {
            float2 ev[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * NT;
                ev[u] = i < P ? ld2(E + i) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = i0 + u * NT;
                if (i < P) keys[i] = __float_as_uint(fmaf(ev[u].x, ev[u].x, ev[u].y * ev[u].y));
            }
        }
        __syncthreads();
    }
    const size_t blk = (size_t)(j * Q + b);
    GLOBAL int32_t* __restrict__ Hout = glb(io.H) + blk * d->T;
    GLOBAL uint64_t* __restrict__ thr_out = glb(io.thr) + blk;
    GLOBAL int32_t* __restrict__ CLout = glb(io.CL) + blk * (size_t)s1 * d->depth;
    if constexpr (!LDSKEYS) {
        // Two reads of E instead of one per radix pass and two more for the
        // emission: the first pass finds the bucket (key bits 62..53) of the
        // T-th largest key; every key in it or above goes to a candidate list
        // in LDS (keys[] as uint64), which holds the T largest; selection and
        // emission run on the list.  A list longer than its capacity leaves
        // the block to the passes over E below.
        uint64_t* cand = reinterpret_cast<uint64_t*>(keys);
        const int cap = d->sel_cap;
        const int tid = (int)threadIdx.x;
        const int lane = tid & 63;
        const int wid = tid >> 6;
        __shared__ int32_t sh_nc, sh_dig;
        __shared__ unsigned long long sh_min;
        constexpr int U = 16;  // loads of a thread in flight at once
        auto hi_of = [](float2 e) { return __float_as_uint(fmaf(e.x, e.x, e.y * e.y)); };
        if (tid == 0) {
            sh_nc = 0;
            sh_dig = 0;
            sh_min = ~0ull;
        }
        const bool all = d->T >= P;
        if (!all) {
            if (io.SH) {   // the histogram the column kernel formed with the bins
                const GLOBAL int32_t* sh = glb(io.SH) + blk * kSelBins;
                for (int i = tid; i < kSelBins; i += NT) hist[i] = sh[i];
            } else {
                for (int i = tid; i < kSelBins; i += NT) hist[i] = 0;
                __syncthreads();
                for (int base = 0; base < P; base += U * NT) {
                    float2 ev[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int i = base + u * NT + tid;
                        ev[u] = i < P ? ld2(E + i) : make_float2(0.f, 0.f);
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (base + u * NT + tid < P) atomicAdd(&hist[(hi_of(ev[u]) >> 21) & (kSelBins - 1)], 1);
                }
            }
            __syncthreads();
            // the bucket holding rank T, scanning the buckets in descending order
            constexpr int BPT = kSelBins / NT;
            int cnt[BPT];
            int loc = 0;
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                cnt[q] = hist[kSelBins - 1 - (tid * BPT + q)];
                loc += cnt[q];
            }
            const int x = wave_inclusive_sum(loc);
            if (lane == 63) part[wid] = x;
            __syncthreads();
            int run = waves_before<NT>(part, wid) + x - loc;
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                if (run < d->T && run + cnt[q] >= d->T) sh_dig = kSelBins - 1 - (tid * BPT + q);
                run += cnt[q];
            }
        }
        __syncthreads();
        const uint32_t dig = (uint32_t)sh_dig;
        const uint64_t ltm = ((uint64_t)1 << lane) - 1;
        for (int base = 0; base < P; base += U * NT) {   // wave-uniform trip count
            float2 ev[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = base + u * NT + tid;
                ev[u] = i < P ? ld2(E + i) : make_float2(0.f, 0.f);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int i = base + u * NT + tid;
                const uint32_t h = hi_of(ev[u]);
                const bool take = i < P && ((h >> 21) & (kSelBins - 1)) >= dig;
                const uint64_t m = __ballot(take);
                if (m) {   // wave-uniform: most bins are below the bucket
                    int wb = 0;
                    if (lane == 0) wb = atomicAdd(&sh_nc, __popcll(m));
                    wb = __builtin_amdgcn_readfirstlane(wb);   // lane 0's (every lane is active here)
                    if (take) {
                        const int pos = wb + __popcll(m & ltm);
                        if (pos < cap)
                            cand[pos] = ((uint64_t)h << 32) |
                                        (uint64_t)(0xffffffffu - pfa_bin(i, lg, s1, (uint32_t)P, cA, cB));
                    }
                }
            }
        }
        __syncthreads();
        const int nc = sh_nc;
        if (nc <= cap) {   // uniform over the block
            uint64_t thr = 0;
            if (!all) {
                if (nc > d->T) {
                    auto each_c = [&](auto f) {
                        for (int i = tid; i < nc; i += NT) {
                            const uint64_t k = cand[i];
                            f((uint32_t)(k >> 32), [k] { return k; });
                        }
                    };
                    thr = kth_largest<NT>(each_c, nc, d->T, hist, part);
                } else {   // exactly the T largest: the threshold is the least of them
                    for (int i = tid; i < nc; i += NT) atomicMin(&sh_min, (unsigned long long)cand[i]);
                    __syncthreads();
                    thr = sh_min;
                }
            }
            emit_heavy<NT>([&](int i) { return cand[i]; }, nc, d->T, s1, d->depth, thr, hk, hist, part, cl, Hout,
                           thr_out, CLout);
            return;
        }
    }
    auto kf = [&](int i) {
        const uint32_t bin = pfa_bin(i, lg, s1, (uint32_t)P, cA, cB);
        if constexpr (LDSKEYS) return ((uint64_t)keys[i] << 32) | (uint64_t)(0xffffffffu - bin);
        else return value_key(ld2(E + i), bin);
    };
    auto each = [&](auto f) {
        for (int i = (int)threadIdx.x; i < P; i += NT) {
            if constexpr (LDSKEYS) {
                const uint32_t h = keys[i];
                f(h, [&] { return kf(i); });
            } else {
                const uint64_t k = kf(i);
                f((uint32_t)(k >> 32), [k] { return k; });
            }
        }
    };
    const uint64_t thr = kth_largest<NT>(each, P, d->T, hist, part);
    emit_heavy<NT>(kf, P, d->T, s1, d->depth, thr, hk, hist, part, cl, Hout, thr_out, CLout);
}

// a mod d for a 32-bit a, from magic = floor((2^64 - 1) / d) + 1 (Lemire,
// Kaser and Kurz 2019): the bits [64, 96) of (magic a mod 2^64) d, formed
// from two 32 x 32-bit products.
__device__ __forceinline__ uint32_t fastmod_u32(uint32_t a, uint64_t magic, uint32_t d) {
    const uint64_t low = magic * (uint64_t)a;
    const uint64_t lo_d = (uint64_t)(uint32_t)low * d;
    const uint64_t hi_d = (uint64_t)(uint32_t)(low >> 32) * d;
    return (uint32_t)((hi_d + (lo_d >> 32)) >> 32);
}

// ---------------------------------------------------------- k_identify ----
// One workgroup of NT threads per band b.  Candidates: in CRT tuple t and residue class a,
// one of the `depth` heaviest heavy class-a bins of every modulus of the tuple
// (the class lists written with the heavy bins);
// w = a (mod s1), w = h_g (mod p_g) by the CRT in int64, mapped into B.
// Vote ("more than half", Appendix B): the tuple's own G moduli hold heavy bins
// at w by construction, so (w mod P_j) must be a heavy bin for more than half of
// the other K - G moduli; a bin is heavy when it is in its block's heavy set
// (key >= threshold), tested against an LDS bitmap built from the heavy bins,
// so that E is read only for accepted candidates.  A w produced by both tuples
// is accepted if either tuple's vote passes (the two entries are equal and
// merged later).  Estimate: componentwise median of E_b[j][w mod P_j] over all
// K moduli.  Then the s
// largest |z| (ties to the smaller w), the band test w in [q_b - L, q_b + L),
// and v = z / ghat_{w - q_b} in FP64.

// Median of v[0..K), K odd: the value whose rank (the values below it, and
// the equal ones at a lower index) is K / 2.  Compiled for each K the plans
// use (K = 2 G + 1), so that no comparison is guarded at run time.
template <int KK>
__device__ __forceinline__ float median_k(const float* v) {
    float med = 0.f;
#pragma unroll
    for (int i = 0; i < KK; ++i) {
        int rank = 0;
#pragma unroll
        for (int k = 0; k < KK; ++k) rank += (v[k] < v[i]) || (v[k] == v[i] && k < i);
        if (rank == (KK >> 1)) med = v[i];
    }
    return med;
}

__device__ __forceinline__ float median_of(const float* v, int K) {
    static_assert(kMaxK == 15, "median cases");
    switch (K) {
        case 5: return median_k<5>(v);
        case 7: return median_k<7>(v);
        case 9: return median_k<9>(v);
        case 11: return median_k<11>(v);
        case 13: return median_k<13>(v);
        case 15: return median_k<15>(v);
        default: return median_k<3>(v);   // K = 2 G + 1 >= 5; 3 for completeness
    }
}

// Phase identification: bin h of a modulus of length P holds e (samples at the
// nodes) and e2 (the nodes moved one grid step); for one dominant frequency w,
// e2 / e = exp(2 pi i w / N).  Returns the w in B = [lo, hi] with w = h (mod P)
// whose angle 2 pi w / N is circularly nearest to arg(e2 conj(e)), ties to the
// smaller w, in FP64; false if B holds no member of the class.  The nearest
// member lies next to the rounded quotient for x, x - N or x + N.
__device__ bool phase_frequency(float2 e, float2 e2, int h, int P, int64_t N, int64_t lo, int64_t hi, int64_t& w) {
    constexpr double kTwoPi = 6.283185307179586;
    const double re = (double)e2.x * (double)e.x + (double)e2.y * (double)e.y;
    const double im = (double)e2.y * (double)e.x - (double)e2.x * (double)e.y;
    const double x = atan2(im, re) * (double)N / kTwoPi;
    bool found = false;
    double best = 0.0;
    for (int sh = -1; sh <= 1; ++sh) {
        const double xs = x + (double)sh * (double)N;
        const int64_t m0 = (int64_t)floor((xs - (double)h) / (double)P + 0.5);
        for (int dm = -1; dm <= 1; ++dm) {
            const int64_t c = (int64_t)h + (m0 + dm) * (int64_t)P;
            if (c < lo || c > hi) continue;
            const double dist = fabs((double)c - xs);
            if (!found || dist < best || (dist == best && c < w)) {
                found = true;
                best = dist;
                w = c;
            }
        }
    }
    return found;
}

// KEYVOTE: the vote compares bin keys with the thresholds (plans whose
// bitmaps exceed the LDS, or batches that contain one); otherwise it tests the
// heavy-bin bitmaps.  Both decide the same way.  PHASE: the launch may hold
// plans with phase identification (taken per transform).
template <bool KEYVOTE, bool PHASE, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu((KEYVOTE || PHASE) ? 1 : 6))) k_identify(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int b = at.blk;
    const int Q = d->Q;
    const int K = d->K;
    const int G = d->G;
    const int s1 = d->s1;
    const int lg = d->log2s1;
    const int depth = d->depth;
    const int64_t lo = d->lo, hi = d->hi;
    const int nslots = 2 * s1;
    const bool phase = PHASE && d->phase != 0;
    const int T = d->T;

    const int acap = d->accept_cap;
    uint64_t* akey = reinterpret_cast<uint64_t*>(smem);
    float2* az = reinterpret_cast<float2*>(smem + (size_t)acap * 8);
    int32_t* flag = reinterpret_cast<int32_t*>(smem + (size_t)acap * 16);
    int32_t* scratch = flag + acap;
    int32_t* pre = scratch + NT;
    uint8_t* ccount = reinterpret_cast<uint8_t*>(pre + ((nslots + 2) & ~1));   // [K * s1]
    uint8_t* ccount2 = ccount + (((size_t)K * s1 + 3) & ~(size_t)3);            // [K * s1]: depth 8, second halves
    // heavy-bin bitmaps of the band's K blocks (when they fit the LDS): bit h of
    // block jj at word woff[jj] + h / 32; otherwise the vote compares keys
    constexpr bool use_bm = !KEYVOTE;
    uint32_t* bm = reinterpret_cast<uint32_t*>(ccount2 + (((size_t)K * s1 + 3) & ~(size_t)3));
    int woff[kMaxK + 1];
    woff[0] = 0;
#pragma unroll
    for (int jj = 0; jj < kMaxK; ++jj) woff[jj + 1] = woff[jj] + (jj < K && use_bm ? (d->P[jj] + 31) >> 5 : 0);
    // slot of every combination (residue identification, at most kSlotMap of them)
    uint16_t* cmap = reinterpret_cast<uint16_t*>(bm + woff[kMaxK]);
    __shared__ int32_t sh_cnt;
    __shared__ uint64_t sh_thr[kMaxK];   // the blocks' thresholds (key vote)

    const GLOBAL int32_t* __restrict__ CLall = glb(io.CL);
    const GLOBAL int32_t* __restrict__ Hall = glb(io.H);
    const GLOBAL float2* __restrict__ Eall = glb(io.E);
    const size_t cl_stride = (size_t)s1 * depth;   // one (modulus, band) block of class lists

    // 0. class-list lengths and heavy-bin bitmaps of this band's K blocks, into LDS
    for (int i = tid; i < woff[kMaxK]; i += NT) bm[i] = 0;
    if (!use_bm)
        for (int jj = tid; jj < K; jj += NT) sh_thr[jj] = glb(io.thr)[jj * Q + b];
    __syncthreads();   // bitmaps cleared
    {
        // class-list lengths (lists are -1 padded) and the heavy bins of block
        // (jj, b) (its min(T, P_jj) entries of H, unordered), read as 16-byte
        // pieces: a class list of depth 4 or 8 is one or two pieces, of depth
        // 1 or 2 a piece holds 4 or 2 lists; a thread's loads are all issued
        // before their first use
        const int nh = use_bm ? K * T : 0;
        const int ncl = phase ? 0 : K * s1;   // class lists: residue identification only
        // the pieces' layout (uniform): T and s1 depth multiples of 4 (each
        // block's lists and heavy bins then start at 16-byte boundaries)
        const bool wide = (T & 3) == 0 && ((s1 * depth) & 3) == 0;
        if (wide) {
            constexpr int U = 4;
            const int hq = T >> 2;                         // pieces of heavy bins per block
            const int cq = (s1 * depth) >> 2;              // pieces of class lists per block
            const int nhq = use_bm ? K * hq : 0, ncq = phase ? 0 : K * cq;
            for (int i0 = tid; i0 < ncq || i0 < nhq; i0 += U * NT) {
                pod_i4 hv[U], lv[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * NT;
                    hv[u] = pod_i4{-1, -1, -1, -1};
                    lv[u] = pod_i4{-1, -1, -1, -1};
                    if (i < nhq) {
                        const int jj = i / hq;
                        hv[u] = *(const GLOBAL pod_i4*)(Hall + (size_t)(jj * Q + b) * T + 4 * (i - jj * hq));
                    }
                    if (i < ncq) {
                        const int jj = i / cq;
                        lv[u] = *(const GLOBAL pod_i4*)(CLall + (size_t)(jj * Q + b) * cl_stride + 4 * (i - jj * cq));
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * NT;
                    if (i < nhq) {
                        const int jj = i / hq;
                        const int hs[4] = {hv[u].x, hv[u].y, hv[u].z, hv[u].w};
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (hs[e] >= 0) atomicOr(&bm[woff[jj] + (hs[e] >> 5)], 1u << (hs[e] & 31));
                    }
                    if (i < ncq) {
                        // entries 4 i .. 4 i + 3 of the band's lists (block jj = i / cq)
                        const int jj = i / cq;
                        const int e0 = 4 * (i - jj * cq);   // entry index within the block
                        const int ls[4] = {lv[u].x, lv[u].y, lv[u].z, lv[u].w};
                        if (depth >= 4) {   // whole piece in class e0 / depth; depth 8: two pieces
                            int n = 0;
#pragma unroll
                            for (int e = 0; e < 4; ++e) n += ls[e] >= 0 ? 1 : 0;
                            const int cidx = (jj << lg) + e0 / depth;
                            if (depth == 4 || (e0 & 7) == 0) ccount[cidx] = (uint8_t)n;   // (first half)
                            else ccount2[cidx] = (uint8_t)n;                                // second half
                        } else if (depth == 2) {   // two classes per piece
#pragma unroll
                            for (int e = 0; e < 4; e += 2)
                                ccount[(jj << lg) + ((e0 + e) >> 1)] =
                                    (uint8_t)((ls[e] >= 0 ? 1 : 0) + (ls[e + 1] >= 0 ? 1 : 0));
                        } else {                   // depth 1: four classes per piece
#pragma unroll
                            for (int e = 0; e < 4; ++e) ccount[(jj << lg) + e0 + e] = (uint8_t)(ls[e] >= 0 ? 1 : 0);
                        }
                    }
                }
            }
        } else {
            constexpr int U = 4;
            for (int i0 = tid; i0 < ncl || i0 < nh; i0 += U * NT) {
                int32_t hv[U];
                int32_t lv[U][kMaxDepth];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * NT;
                    hv[u] = -1;
                    if (i < nh) {
                        const int jj = i / T;
                        const int e = i - jj * T;
                        if (e < d->P[jj]) hv[u] = Hall[(size_t)(jj * Q + b) * T + e];
                    }
#pragma unroll
                    for (int e = 0; e < kMaxDepth; ++e) lv[u][e] = -1;
                    if (i < ncl) {
                        const GLOBAL int32_t* cl =
                            CLall + (size_t)((i >> lg) * Q + b) * cl_stride + (size_t)(i & (s1 - 1)) * depth;
#pragma unroll
                        for (int e = 0; e < kMaxDepth; ++e)
                            if (e < depth) lv[u][e] = cl[e];
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int i = i0 + u * NT;
                    if (hv[u] >= 0) {
                        const int jj = i / T;
                        atomicOr(&bm[woff[jj] + (hv[u] >> 5)], 1u << (hv[u] & 31));
                    }
                    if (i < ncl) {
                        int n = 0;
#pragma unroll
                        for (int e = 0; e < kMaxDepth; ++e) n += lv[u][e] >= 0 ? 1 : 0;
                        ccount[i] = (uint8_t)n;
                    }
                }
            }
        }
    }
    __syncthreads();
    if (!phase && depth == 8 && ((T & 3) == 0) && ((s1 * depth) & 3) == 0) {
        // depth 8 in pieces: a list's length is the sum of its halves' counts
        for (int i = tid; i < K * s1; i += NT) ccount[i] = (uint8_t)(ccount[i] + ccount2[i]);
    }
    __syncthreads();

    // 1. combinations per (tuple, class) slot: product of the class-list lengths
    // (phase identification: one candidate per heavy bin, K T of them)
    for (int slot = tid; slot < nslots && !phase; slot += NT) {
        const int t = slot >> lg;
        const int ac = slot & (s1 - 1);
        int cnt = 1;
        for (int g = 0; g < G; ++g) cnt *= ccount[(d->tup_j[t][g] << lg) + ac];
        pre[slot] = cnt;
    }
    if (tid == 0) sh_cnt = 0;
    __syncthreads();
    const int total = phase ? K * T : block_exclusive_scan<NT>(pre, nslots, scratch);
    if (tid == 0) pre[nslots] = total;
    __syncthreads();
    const bool use_map = !phase && total <= kSlotMap;
    if (use_map) {   // instead of a binary search over the slots per combination
        for (int slot = tid; slot < nslots; slot += NT)
            for (int i = pre[slot]; i < pre[slot + 1]; ++i) cmap[i] = (uint16_t)slot;
        __syncthreads();
    }

    // 2. candidates -> vote -> median
    const bool small_n = d->N <= ((int64_t)1 << 31);   // then B lies in the int32 range
    // a combination's tuple t, class ac and bin of every modulus of the tuple
    // (residue identification); the class-list loads of a thread's next
    // candidate are issued before its current one is processed
    struct Combo {
        int t, ac;
        int32_t hg[kMaxG];
    };
    auto prep = [&](int c, Combo& cb) {
        int slot;
        if (use_map) {
            slot = cmap[c];
        } else {
            int l0 = 0, h0 = nslots - 1;   // last slot with pre[slot] <= c
            while (l0 < h0) {
                const int mid = (l0 + h0 + 1) >> 1;
                if (pre[mid] <= c) l0 = mid; else h0 = mid - 1;
            }
            slot = l0;
        }
        int r = c - pre[slot];
        cb.t = slot >> lg;
        cb.ac = slot & (s1 - 1);
#pragma unroll
        for (int g = 0; g < kMaxG; ++g) {
            if (g < G) {
                const int jj = d->tup_j[cb.t][g];
                const int cg = ccount[(jj << lg) + cb.ac];
                // r < 64 and cg <= kMaxDepth: (r + 1/2) / cg lies at least 1/16
                // from an integer, far beyond the reciprocal's rounding
                const int qd = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)cg));
                const int ch = r - qd * cg;
                r = qd;
                cb.hg[g] = CLall[(size_t)(jj * Q + b) * cl_stride + (size_t)cb.ac * depth + ch];
            }
        }
    };
    // (the kernel that may also run phase identification loads each
    // combination where it is used: it keeps fewer registers that way)
    constexpr bool prefetch = !PHASE;
    Combo cur, nxt;
    if (prefetch && tid < total) prep(tid, cur);
    for (int c = tid; c < total; c += NT) {
        if (prefetch && c + NT < total) prep(c + NT, nxt);
        {   // candidate c; a dropped candidate jumps to the end of the iteration
            int64_t w;
            int t = 0, jp = 0;   // CRT tuple (residue identification); producing modulus (phase)
            if (PHASE && phase) {
                jp = c / T;
                const int e = c - jp * T;
                const int h0 = Hall[(size_t)(jp * Q + b) * T + e];
                const size_t at0 = (size_t)Q * d->Moff[jp] + (size_t)b * d->P[jp] +
                                   ((size_t)(h0 % d->p[jp]) << lg) + (size_t)(h0 & (s1 - 1));
                if (!phase_frequency(ld2(Eall + at0), ld2(glb(io.E2) + at0), h0, d->P[jp], d->N, lo, hi, w)) goto next_candidate;
            } else {
            if constexpr (!prefetch) prep(c, cur);
            t = cur.t;
            const int ac = cur.ac;
            // CRT without 64-bit divisions: every term is below M_t (a residue < m
            // times M_t / m), so the sum is reduced by at most G subtractions
            int64_t x = (int64_t)((ac * d->tup_inv[t][0]) & (s1 - 1)) * d->tup_Mi[t][0];
#pragma unroll
            for (int g = 0; g < kMaxG; ++g) {
                if (g < G) {
                    const uint32_t pm = (uint32_t)d->tup_mod[t][g + 1];
                    const uint64_t mg = d->magic_p[d->tup_j[t][g]];   // pm = p of that modulus
                    const uint32_t res = fastmod_u32((uint32_t)cur.hg[g], mg, pm);
                    x += (int64_t)fastmod_u32(res * (uint32_t)d->tup_inv[t][g + 1], mg, pm) * d->tup_Mi[t][g + 1];
                }
            }
            const int64_t Mt = d->tup_M[t];
            while (x >= Mt) x -= Mt;
            if (x <= hi) w = x;
            else if (x - Mt >= lo) w = x - Mt;
            else goto next_candidate;
            }

            // the bin of w in every modulus; the vote counts heavy bins among the
            // moduli outside tuple t (a bin is heavy iff its key >= the block's
            // threshold, i.e. iff it is in the block's heavy set)
            int hh[kMaxK];
            int votes = 0;
            // residue identification: the vote is over the moduli outside tuple t;
            // phase identification: over all K moduli
            const int t_lo = (PHASE && phase) ? 0 : t * G, t_hi = (PHASE && phase) ? 0 : t_lo + G;
            const int need = (PHASE && phase) ? K : K - G;
            auto read_bins = [&](float* er, float* ei) {
#pragma unroll
                for (int jj = 0; jj < kMaxK; ++jj) {
                    if (jj < K) {
                        const int Pj = d->P[jj];
                        const int k2 = (int)fastmod_u32((uint32_t)hh[jj], d->magic_p[jj], (uint32_t)d->p[jj]);
                        const float2 ev = ld2(Eall + (size_t)Q * d->Moff[jj] + (size_t)b * Pj + ((size_t)k2 << lg) +
                                              (hh[jj] & (s1 - 1)));
                        er[jj] = ev.x;
                        ei[jj] = ev.y;
                    }
                }
            };
#pragma unroll
            for (int jj = 0; jj < kMaxK; ++jj) {
                if (jj < K) {
                    if (small_n) {   // w - lo fits 32 bits: w mod P = ((w - lo) mod P + lo mod P) mod P
                        const int Pj = d->P[jj];
                        const int r = (int)fastmod_u32((uint32_t)(w - lo), d->magic_P[jj], (uint32_t)Pj) + d->lo_mod_P[jj];
                        hh[jj] = r >= Pj ? r - Pj : r;
                    } else {
                        hh[jj] = (int)pos_mod(w, d->P[jj]);
                    }
                }
            }
            float er[kMaxK], ei[kMaxK];   // the K bin values, for the median
            if constexpr (use_bm) {
#pragma unroll
                for (int jj = 0; jj < kMaxK; ++jj) {
                    if (jj < K) {
                        const bool heavy = (bm[woff[jj] + (hh[jj] >> 5)] >> (hh[jj] & 31)) & 1u;
                        votes += (heavy && (jj < t_lo || jj >= t_hi)) ? 1 : 0;
                    }
                }
            } else {   // the same heavy test from the bin values: key >= the block's threshold
                read_bins(er, ei);
#pragma unroll
                for (int jj = 0; jj < kMaxK; ++jj) {
                    if (jj < K) {
                        const bool heavy = value_key(make_float2(er[jj], ei[jj]), (uint32_t)hh[jj]) >= sh_thr[jj];
                        votes += (heavy && (jj < t_lo || jj >= t_hi)) ? 1 : 0;
                    }
                }
            }
            if (2 * votes > need) {
                if constexpr (use_bm && !PHASE) {
                    // the bitmap-vote residue kernel keeps only w here; the bins and
                    // the median follow for all accepted candidates at once after the
                    // loop, so that no wave waits on bin loads in it (the kernel that
                    // may also run phase identification reads them here: deferring
                    // there too multiplied its registers)
                    const int pos = atomicAdd(&sh_cnt, 1);
                    if (pos < acap) akey[pos] = (uint64_t)(0xffffffffu - (uint32_t)(w - lo));
                    else atomicOr(io.status, kStatusAcceptOverflow);
                    goto next_candidate;
                }
                if constexpr (use_bm) read_bins(er, ei);
                if (PHASE && phase) {
                    // one entry per frequency: an earlier modulus whose heavy bin at w
                    // gives w as well produces (and keeps) it
                    bool dup = false;
#pragma unroll
                    for (int jj = 0; jj < kMaxK; ++jj) {   // compile-time indices: er, ei, hh stay in registers
                        if (jj < jp && !dup) {
                            const float2 ev = make_float2(er[jj], ei[jj]);
                            bool heavy;
                            if constexpr (use_bm) heavy = (bm[woff[jj] + (hh[jj] >> 5)] >> (hh[jj] & 31)) & 1u;
                            else heavy = value_key(ev, (uint32_t)hh[jj]) >= sh_thr[jj];
                            if (heavy) {
                                const size_t atj = (size_t)Q * d->Moff[jj] + (size_t)b * d->P[jj] +
                                                   ((size_t)(hh[jj] % d->p[jj]) << lg) + (size_t)(hh[jj] & (s1 - 1));
                                int64_t w2;
                                dup = phase_frequency(ev, ld2(glb(io.E2) + atj), hh[jj], d->P[jj], d->N, lo, hi, w2) &&
                                      w2 == w;
                            }
                        }
                    }
                    if (dup) goto next_candidate;
                }
                const float zr = median_of(er, K);
                const float zi = median_of(ei, K);
                const float m2 = fmaf(zr, zr, zi * zi);
                const int pos = atomicAdd(&sh_cnt, 1);
                if (pos < acap) {
                    akey[pos] = ((uint64_t)__float_as_uint(m2) << 32) |
                                (uint64_t)(0xffffffffu - (uint32_t)(w - lo));
                    az[pos] = make_float2(zr, zi);
                } else {
                    atomicOr(io.status, kStatusAcceptOverflow);
                }
            }
        }
    next_candidate:
        if constexpr (prefetch) cur = nxt;
    }
    __syncthreads();
    int nacc = min(sh_cnt, acap);
    if constexpr (use_bm && !PHASE) {
        // the accepted candidates' bins in every modulus (all loads of a thread
        // issued together) and their componentwise median
        for (int i = tid; i < nacc; i += NT) {
            const int64_t w = lo + (int64_t)(0xffffffffu - (uint32_t)(akey[i] & 0xffffffffu));
            float er[kMaxK], ei[kMaxK];
            float2 ev[kMaxK];
#pragma unroll
            for (int jj = 0; jj < kMaxK; ++jj) {
                if (jj < K) {
                    const int Pj = d->P[jj];
                    int h;
                    if (small_n) {
                        const int r = (int)fastmod_u32((uint32_t)(w - lo), d->magic_P[jj], (uint32_t)Pj) + d->lo_mod_P[jj];
                        h = r >= Pj ? r - Pj : r;
                    } else {
                        h = (int)pos_mod(w, Pj);
                    }
                    const int k2 = (int)fastmod_u32((uint32_t)h, d->magic_p[jj], (uint32_t)d->p[jj]);
                    ev[jj] = ld2(Eall + (size_t)Q * d->Moff[jj] + (size_t)b * Pj + ((size_t)k2 << lg) + (h & (s1 - 1)));
                }
            }
#pragma unroll
            for (int jj = 0; jj < kMaxK; ++jj) {
                if (jj < K) {
                    er[jj] = ev[jj].x;
                    ei[jj] = ev[jj].y;
                }
            }
            const float zr = median_of(er, K);
            const float zi = median_of(ei, K);
            const float m2 = fmaf(zr, zr, zi * zi);
            akey[i] |= (uint64_t)__float_as_uint(m2) << 32;
            az[i] = make_float2(zr, zi);
        }
        __syncthreads();
    }
    // 3. sort accepted by key descending (|z|^2 desc, w asc)
    if (nacc > 512) {
        // Many accepted entries, of which only the s largest distinct keys are
        // kept: the copies of one frequency w (equal keys and medians) are
        // dropped through a hash table of w over flag, the s-th largest of the
        // remaining keys is selected, and only the kept entries (distinct
        // keys) are sorted below.  The result is the sorted list's first s
        // distinct entries, as without this step.
        __shared__ int32_t sh_d, sh_k;
        int32_t* table = flag;   // [acap], acap a power of two >= nacc: every insert finds a slot
        for (int i = tid; i < acap; i += NT) table[i] = -1;
        if (tid == 0) {
            sh_d = 0;
            sh_k = 0;
        }
        __syncthreads();
        const int lgc = 31 - __clz(acap);
        int dl = 0;   // entries this thread keeps as first copies
        for (int i = tid; i < nacc; i += NT) {
            const uint32_t wk = (uint32_t)akey[i];
            uint32_t slot = (wk * 2654435761u) >> (32 - lgc);
            for (int probe = 0; probe < acap; ++probe) {
                const int prev = atomicCAS(&table[slot], -1, i);
                if (prev < 0) {   // the first copy of w
                    ++dl;
                    break;
                }
                if ((uint32_t)akey[prev] == wk) {   // a later copy (entries in the table stay)
                    akey[i] = 0;
                    break;
                }
                slot = (slot + 1) & (uint32_t)(acap - 1);
            }
        }
        dl = wave_inclusive_sum(dl);
        if ((tid & 63) == 63) atomicAdd(&sh_d, dl);
        __syncthreads();
        const int dn = sh_d;
        uint64_t kthr = 1;   // every remaining (nonzero) key
        if (dn > d->s) {
            // the histogram over the slot map, free after the combinations
            static_assert(kSlotMap * 2 >= kSelBins * 4, "selection histogram in the slot map");
            auto each = [&](auto f) {
                for (int i = tid; i < nacc; i += NT) {
                    const uint64_t k = akey[i];
                    if (k != 0) f((uint32_t)(k >> 32), [k] { return k; });
                }
            };
            kthr = kth_largest<NT>(each, dn, d->s, reinterpret_cast<int32_t*>(cmap), scratch);
        }
        // the kept entries (at most s) to the slot prefix sums' space, free
        // now ((2 s1 + 2) * 4 >= 16 s bytes as s1 >= 2 s; 8-byte aligned)
        uint64_t* kk = reinterpret_cast<uint64_t*>(pre);
        float2* kz = reinterpret_cast<float2*>(kk + d->s);
        for (int i = tid; i < nacc; i += NT) {
            const uint64_t k = akey[i];
            if (k != 0 && k >= kthr) {
                const int pos = atomicAdd(&sh_k, 1);
                if (pos < d->s) {   // exactly min(dn, s) entries pass; the bound only guards the space
                    kk[pos] = k;
                    kz[pos] = az[i];
                }
            }
        }
        __syncthreads();
        const int kn = min(sh_k, d->s);
        for (int i = tid; i < kn; i += NT) {
            akey[i] = kk[i];
            az[i] = kz[i];
        }
        __syncthreads();
        nacc = kn;
    }
    if (nacc <= 512) {
        // by rank: an entry's position is the number of entries ahead of it
        // (a larger key, or an equal key at a lower index)
        uint64_t kk[2];
        float2 zz[2];
        int rk[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = tid + u * NT;
            rk[u] = -1;
            if (i < nacc) {
                const uint64_t k = akey[i];
                int r = 0;
                for (int jn = 0; jn < nacc; ++jn) {
                    const uint64_t kj = akey[jn];
                    r += (kj > k || (kj == k && jn < i)) ? 1 : 0;
                }
                kk[u] = k;
                zz[u] = az[i];
                rk[u] = r;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rk[u] >= 0) {
                akey[rk[u]] = kk[u];
                az[rk[u]] = zz[u];
            }
        }
        __syncthreads();
    } else {   // bitonic sort of the entries padded with zero keys to a power of two
        int np2 = 1;
        while (np2 < nacc) np2 <<= 1;
        for (int i = nacc + tid; i < np2; i += NT) {
            akey[i] = 0;
            az[i] = make_float2(0.f, 0.f);
        }
        __syncthreads();
        for (int kk = 2; kk <= np2; kk <<= 1) {
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int i = tid; i < np2; i += NT) {
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
    }
    // 4. distinct entries, the first s of them (R_temp), then the band test
    for (int i = tid; i < nacc; i += NT) flag[i] = (i == 0 || akey[i] != akey[i - 1]) ? 1 : 0;
    __syncthreads();
    block_exclusive_scan<NT>(flag, nacc, scratch);   // for a distinct entry: its rank among distinct ones
    const int64_t q = d->q_first + 2 * (int64_t)b * d->L;
    const int s = d->s;
    GLOBAL int64_t* __restrict__ Rw = glb(io.Rw) + (size_t)b * s;
    GLOBAL double2* __restrict__ Rv = glb(io.Rv) + (size_t)b * s;
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
                std2(Rv + o, make_double2((double)z.x / gh, (double)z.y / gh));
            }
            outc += __popcll(ballot);
        }
        if (tid == 0) glb(io.Rn)[b] = outc;
    }
}

// ------------------------------------------------------------- k_merge ----
// One workgroup per transform: the s largest |v| over all bands (ties to the
// smaller w), written in that order; unfilled slots get w = 0, c = 0.

__device__ __forceinline__ bool merge_before(double ma, int64_t wa, double mb, int64_t wb) {
    return ma > mb || (ma == mb && wa < wb);
}

template <int NT>
__global__ void __launch_bounds__(NT) k_merge(BatchArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Where at = locate(a);
    const CONSTANT SigDesc* d = desc_of(a, at.sig);
    const IoDesc io = io_of(a, at.sig);
    const int tid = (int)threadIdx.x;
    const int Q = d->Q;
    const int s = d->s;
    double* mm = reinterpret_cast<double*>(smem);
    int64_t* ww = reinterpret_cast<int64_t*>(smem + (size_t)kMergeCap * 8);
    int32_t* src = reinterpret_cast<int32_t*>(smem + (size_t)kMergeCap * 16);
    int32_t* off = src + kMergeCap;
    int32_t* scratch = off + SFT_MAX_BANDS + 1;

    for (int bb = tid; bb < Q; bb += NT) off[bb] = glb(io.Rn)[bb];
    __syncthreads();
    const int total = block_exclusive_scan<NT>(off, Q, scratch);
    const int n = min(total, kMergeCap);
    if (tid == 0 && total > kMergeCap) atomicOr(io.status, kStatusMergeOverflow);
    // entry e of the concatenation belongs to the last band bb with off[bb] <= e
    // (a band with off[bb] <= e < off[bb + 1] is not empty); all loads at once
    for (int e = tid; e < n; e += NT) {
        int lo = 0, hi = Q - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (off[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int k = e - off[lo];
        const double2 v = ldd2(glb(io.Rv) + (size_t)lo * s + k);
        mm[e] = v.x * v.x + v.y * v.y;
        ww[e] = glb(io.Rw)[(size_t)lo * s + k];
        src[e] = lo * s + k;
    }
    __syncthreads();
    if (n <= 512) {
        // by rank: an entry's position is the number of entries ordered before
        // it (the frequencies of a transform are distinct, so the ranks are);
        // n compares per entry, fewer steps than the sort's up to 512 entries
        double mv[2];
        int64_t wv[2];
        int32_t sv[2];
        int rk[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = tid + u * NT;
            rk[u] = -1;
            if (i < n) {
                mv[u] = mm[i];
                wv[u] = ww[i];
                sv[u] = src[i];
                int r = 0;
                for (int j = 0; j < n; ++j) r += merge_before(mm[j], ww[j], mv[u], wv[u]) ? 1 : 0;
                rk[u] = r;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (rk[u] >= 0) {
                mm[rk[u]] = mv[u];
                ww[rk[u]] = wv[u];
                src[rk[u]] = sv[u];
            }
        }
        __syncthreads();
    } else {   // bitonic sort of the entries padded to a power of two
        int np2 = 1;
        while (np2 < n) np2 <<= 1;
        for (int i = n + tid; i < np2; i += NT) {
            mm[i] = -1.0;
            ww[i] = 0;
            src[i] = -1;
        }
        __syncthreads();
        for (int kk = 2; kk <= np2; kk <<= 1) {
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int i = tid; i < np2; i += NT) {
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
    }
    const int nout = min(n, s);
    for (int r = tid; r < s; r += NT) {
        if (r < nout) {
            const double2 v = ldd2(glb(io.Rv) + src[r]);
            glb(io.out_w)[r] = ww[r];
            st2(glb(io.out_c) + r, make_float2((float)v.x, (float)v.y));
        } else {
            glb(io.out_w)[r] = 0;
            st2(glb(io.out_c) + r, make_float2(0.f, 0.f));
        }
    }
    if (tid == 0 && io.out_n) glb(io.out_n)[0] = nout;
}

// ------------------------------------------------------------ launchers ---

size_t identify_lds_bytes(const SigDesc& d, bool bitmap) {
    const int nslots = 2 * d.s1;
    size_t words = 0;   // heavy-bin bitmaps
    if (bitmap)
        for (int j = 0; j < d.K; ++j) words += (size_t)(d.P[j] + 31) / 32;
    return (size_t)d.accept_cap * 20 + (size_t)kThreads * 4 + (size_t)((nslots + 2) & ~1) * 4 +
           2 * (((size_t)d.K * d.s1 + 3) & ~(size_t)3) + words * 4 + (size_t)kSlotMap * 2 + 64;
}

size_t merge_lds_bytes() {
    return (size_t)kMergeCap * 20 + (SFT_MAX_BANDS + 1) * 4 + kMergeWide * 4 + 64;
}

int gather_blocks(const SigDesc& d) { return (d.M + kThreads - 1) / kThreads; }
int dft_blocks(const SigDesc& d) { return d.K * d.Q * (1 + d.phase); }
int identify_blocks(const SigDesc& d) { return d.Q; }
int merge_blocks(const SigDesc&) { return 1; }

int rows_blocks(const SigDesc& d) {
    const int rows_per = std::max(1, kRowElems >> d.log2s1);
    int n = 0;
    for (int j = 0; j < d.K; ++j) n += d.Q * ((d.p[j] + rows_per - 1) / rows_per);
    return n * (1 + d.phase);
}
int cols_blocks(const SigDesc& d) { return d.K * d.Q * (d.s1 / std::min(kColChunk, d.s1)) * (1 + d.phase); }
int cols_mx_blocks(const SigDesc& d) { return d.K * d.Q * (d.s1 / 64) * (1 + d.phase); }
bool cols_mx_covers(const SigDesc& d) {
    int pmax = 0;
    for (int j = 0; j < d.K; ++j) pmax = std::max(pmax, d.p[j]);
    return d.s1 >= 64 && (pmax - 1) / 2 <= 4 * kMxcSteps && (pmax - 1) / 2 + 1 <= 16 * kMxcTiles;
}
size_t cols_mx_lds_bytes(const SigDesc& d) {
    int pmax = 0;
    for (int j = 0; j < d.K; ++j) pmax = std::max(pmax, d.p[j]);
    return (size_t)pmax * 64 * 8 + 64 + (size_t)kSelBins * 4;   // the tile, then the selection's histogram
}
int select_blocks(const SigDesc& d) { return d.K * d.Q; }

size_t rows_lds_bytes(const SigDesc& d) {
    const int rows_per = std::max(1, kRowElems >> d.log2s1);
    return (size_t)rows_per * d.s1 * 8 + (size_t)d.s1 * 8 + 64;
}
size_t cols_lds_bytes(const SigDesc& d) {
    int pmax = 0;
    for (int j = 0; j < d.K; ++j) pmax = std::max(pmax, d.p[j]);
    const size_t h = (size_t)(pmax - 1) / 2;
    return (size_t)pmax * std::min(kColChunk, d.s1) * 8 + h * h * 8 + 64;
}
size_t select_lds_bytes(const SigDesc& d, bool lds_keys) {
    int32_t Pmax = 0;
    for (int j = 0; j < d.K; ++j) Pmax = d.P[j] > Pmax ? d.P[j] : Pmax;
    return kSelBins * 4 + 64 + (size_t)d.T * 16 + (((size_t)d.s1 * d.depth + 3) & ~(size_t)3) * 4 +
           (lds_keys ? (size_t)Pmax * 4 : (size_t)d.sel_cap * 8) + 64;
}

// Dynamic LDS above 64 KiB: raise each kernel's limit where the runtime asks
// for an opt-in.  A rejected request is not an error here: the launch itself
// reports a size the device cannot hold.
static int g_max_lds = 0;   // the smallest per-workgroup LDS limit of the configured devices

hipError_t configure_kernels(int max_lds) {
    if (g_max_lds == 0 || max_lds < g_max_lds) g_max_lds = max_lds;
    const void* ks[] = {(const void*)k_dft<8, false>, (const void*)k_dft<16, false>, (const void*)k_dft<0, true>,
                         (const void*)k_identify<false, false, kThreads>, (const void*)k_identify<true, false, kThreads>,
                         (const void*)k_identify<false, true, kThreads>, (const void*)k_identify<true, true, kThreads>,
                         (const void*)k_identify<false, false, kIdentifyWide>,
                         (const void*)k_identify<true, false, kIdentifyWide>,
                         (const void*)k_gather_mx<16, 2>, (const void*)k_gather_mx<64, 6>,
                         (const void*)k_gather_mx<64, 8>,
                         (const void*)k_merge<kThreads>, (const void*)k_merge<kMergeWide>, (const void*)k_dft_rows,
                         (const void*)k_dft_cols, (const void*)k_dft_cols_mx, (const void*)k_select<kThreads, false>,
                         (const void*)k_select<kSelLdsThreads, false>, (const void*)k_select<kSelLdsThreads, true>};
    for (const void* k : ks) {
        hipFuncAttributes fa;
        int static_lds = 0;
        if (hipFuncGetAttributes(&fa, k) == hipSuccess) static_lds = (int)fa.sharedSizeBytes;
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds - static_lds) != hipSuccess)
            (void)hipGetLastError();
    }
    return hipSuccess;
}

// Workspace of sft_execute_noalloc, for callers that cannot allocate device
// memory: a fixed array in every device's copy of the code object, held until
// the process ends.  Host code never passes the array's name to a kernel (on
// the host it is only a stand-in for the symbol); it passes the device address
// that hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_gather(const BatchArgs& a, int blocks, int taps, hipStream_t st) {
    switch (taps) {
        case 9: hipLaunchKernelGGL(k_gather<9>, dim3(blocks), dim3(kThreads), 0, st, a); break;
        case 13: hipLaunchKernelGGL(k_gather<13>, dim3(blocks), dim3(kThreads), 0, st, a); break;
        default: hipLaunchKernelGGL(k_gather<0>, dim3(blocks), dim3(kThreads), 0, st, a); break;
    }
    return hipGetLastError();
}

int gather_mx_blocks(const SigDesc& d) { return (d.M + kThreads - 1) / kThreads; }

size_t gather_mx_lds_bytes(const SigDesc& d) { return (size_t)d.gmx_mt * d.gmx_ks * 64 * 4 + (size_t)d.gmx_ks * 8; }

hipError_t launch_gather_mx(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    // bits 32..39: the largest M-tile count of the launch's plans; bit 40:
    // some plan has more than 16 taps.  Wide windows: every M-tile in one pass
    // over the window (up to 8; 6 when that covers the launch).
    const size_t bytes = lds & 0xffffffffu;
    const int mt = (int)((lds >> 32) & 0xff);
    const dim3 gr(blocks), th(kThreads);
    if (!((lds >> 40) & 1)) hipLaunchKernelGGL((k_gather_mx<16, 2>), gr, th, bytes, st, a);
    else if (mt <= 6) hipLaunchKernelGGL((k_gather_mx<64, 6>), gr, th, bytes, st, a);
    else hipLaunchKernelGGL((k_gather_mx<64, 8>), gr, th, bytes, st, a);
    return hipGetLastError();
}

hipError_t launch_dft(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    // lds carries the byte count in its low 32 bits and the output-pair bound above them
    const size_t bytes = lds & 0xffffffffu;
    const int pairs = (int)(lds >> 32);
    const dim3 g(blocks), t(kDftThreads);
    if (pairs > 8) hipLaunchKernelGGL((k_dft<16, false>), g, t, bytes, st, a);
    else hipLaunchKernelGGL((k_dft<8, false>), g, t, bytes, st, a);
    return hipGetLastError();
}

hipError_t launch_dft_mx(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((k_dft<0, true>), dim3(blocks), dim3(kDftThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dft_rows(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_dft_rows, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dft_cols_mx(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_dft_cols_mx, dim3(blocks), dim3(kDftThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_dft_cols(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL(k_dft_cols, dim3(blocks), dim3(kThreads), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_select(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    // lds: the byte count of the kernel that reads E in every pass (low 32
    // bits) and of the one holding the keys in LDS (above; 0 if some block's
    // keys do not fit).  The LDS-key kernel runs one workgroup per CU: it is
    // taken when the launch has at most one block per CU, where the latency
    // of a block decides; larger launches keep many workgroups per CU, or,
    // where the LDS of a block leaves room for one workgroup per CU only
    // (large T and s1), run it with 16 waves instead of 4.
    const size_t bytes = lds & 0xffffffffu, kbytes = lds >> 32;
    if (kbytes && blocks <= kSelLdsMaxBlocks)
        hipLaunchKernelGGL((k_select<kSelLdsThreads, true>), dim3(blocks), dim3(kSelLdsThreads), kbytes, st, a);
    else if (2 * bytes > (size_t)g_max_lds)
        hipLaunchKernelGGL((k_select<kSelLdsThreads, false>), dim3(blocks), dim3(kSelLdsThreads), bytes, st, a);
    else
        hipLaunchKernelGGL((k_select<kThreads, false>), dim3(blocks), dim3(kThreads), bytes, st, a);
    return hipGetLastError();
}

hipError_t launch_identify(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    // lds carries the byte count in its low 32 bits; bit 32 selects the key
    // vote, bit 33 the kernel that also handles phase identification
    const size_t bytes = lds & 0xffffffffu;
    const int kind = (int)((lds >> 32) & 3);
    const dim3 g(blocks), t(kThreads);
    // a launch of at most one band per CU (a single transform or a small
    // batch), or of bands whose LDS leaves room for one workgroup per CU
    // (large s), runs four waves per CU at 256 threads: give each band a
    // workgroup of kIdentifyWide threads instead (its scan partials take
    // (kIdentifyWide - kThreads) ints more).  Residue identification only
    // (bitmap or key vote): the phase variants need more than the 128 VGPRs
    // such a workgroup allows.
    const size_t wbytes = bytes + (size_t)(kIdentifyWide - kThreads) * 4;
    if (kind <= 1 && (blocks <= kIdentifyWideMaxBlocks || 2 * bytes > (size_t)g_max_lds) &&
        wbytes + 256 <= (size_t)g_max_lds) {
        if (kind == 0)
            hipLaunchKernelGGL((k_identify<false, false, kIdentifyWide>), g, dim3(kIdentifyWide), wbytes, st, a);
        else
            hipLaunchKernelGGL((k_identify<true, false, kIdentifyWide>), g, dim3(kIdentifyWide), wbytes, st, a);
        return hipGetLastError();
    }
    switch (kind) {
        case 0: hipLaunchKernelGGL((k_identify<false, false, kThreads>), g, t, bytes, st, a); break;
        case 1: hipLaunchKernelGGL((k_identify<true, false, kThreads>), g, t, bytes, st, a); break;
        case 2: hipLaunchKernelGGL((k_identify<false, true, kThreads>), g, t, bytes, st, a); break;
        default: hipLaunchKernelGGL((k_identify<true, true, kThreads>), g, t, bytes, st, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_merge(const BatchArgs& a, int blocks, size_t lds, hipStream_t st) {
    // lds: bit 32 set when some transform has s > kMergeWideMinS (its band
    // results take the sort rather than the rank form).  At most one
    // transform per CU: 1024 threads sort each (16 waves instead of 4 per CU)
    if ((lds >> 32) != 0 && blocks <= kMergeWideMaxBlocks)
        hipLaunchKernelGGL((k_merge<kMergeWide>), dim3(blocks), dim3(kMergeWide), merge_lds_bytes(), st, a);
    else
        hipLaunchKernelGGL((k_merge<kThreads>), dim3(blocks), dim3(kThreads), merge_lds_bytes(), st, a);
    return hipGetLastError();
}

}  // namespace sft
