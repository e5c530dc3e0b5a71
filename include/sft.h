/*
 * sft.h -- C ABI of the MI355X sparse Fourier transform library (libsft.so).
 *
 * The library computes a near-best s-term approximation of the DFT of a vector
 * f in C^N with Algorithm 1 of Merhi, Zhang, Iwen and Christlieb, "A New Class
 * of Fully Discrete Sparse Fourier Transforms" (Section 3): for every band
 * q_b it evaluates the modulated, periodized-Gaussian-filtered samples
 * (g~_q * f)(x_k) from the 2 kappa + 1 entries of f nearest each node
 * (Section 3.1, Lemma 10), runs short DFTs over those samples (Appendix B),
 * identifies energetic frequencies by residues, CRT and majority vote, and
 * estimates their coefficients by a median divided by ghat (Lemma 2), keeping
 * the s largest over all bands (Algorithm 1, last step).
 *
 * Conventions
 *   - Frequencies are int64 integers in B = (-ceil(N/2), floor(N/2)]
 *     (Section 2, definition of B).
 *   - Coefficients c_w are those of f_j = sum_w c_w exp(2 pi i w j / N),
 *     j = 0..N-1, i.e. numpy.fft.fft(f)[w mod N] / N.  The paper samples f at
 *     -pi + 2 pi j / N, so its fhat_w equals (-1)^w c_w.
 *   - Complex values are interleaved single precision (complex64: re, im).
 *   - Device buffers passed to the execute calls must be aligned to their
 *     element: f and out_coeffs to 8 bytes (complex64), out_freqs to 8 bytes
 *     (int64), counts to 4 bytes; a misaligned pointer returns SFT_EINVAL
 *     before anything is enqueued.  f need not be 16-byte aligned.
 *   - "stream" is a hipStream_t passed as void*; NULL is the null stream.
 *   - Every function returns an SFT_* status; no exception crosses the ABI.
 *     sft_last_error() gives the message of the calling thread's last failure.
 *
 * Ownership
 *   The caller owns f and the output buffers (device memory).  They must stay
 *   valid until the work enqueued on the stream has completed.  A plan owns its
 *   device tables and its workspace; at most one sft_execute may be in flight
 *   per plan.  sft_execute_many uses a workspace owned by the library and
 *   keyed by stream: calls on one stream are ordered, calls on different
 *   streams use different workspaces.
 */
#ifndef SFT_H
#define SFT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define SFT_API __attribute__((visibility("default")))
#else
#define SFT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SFT_OK            0
#define SFT_EINVAL       -1  /* invalid argument or plan outside the paper's parameter domain */
#define SFT_ENOMEM       -2  /* device or host allocation failed */
#define SFT_EHIP         -3  /* a HIP runtime call failed */
#define SFT_EBUDGET      -4  /* request exceeds a configured memory budget */
#define SFT_EUNSUPPORTED -5  /* valid plan the kernels do not handle (size limits) */
#define SFT_EOVERFLOW    -6  /* a device-side capacity was exceeded (see sft_plan_status) */

/* ---- parameter presets ------------------------------------------------ */
#define SFT_PRESET_DMSFT6 0  /* kappa = 6 (13 taps), sigma_t = sqrt((kappa+1/2)/pi); Section 5's DMSFT-6 window */
#define SFT_PRESET_DMSFT4 1  /* kappa = 4 (9 taps); Section 5's DMSFT-4 window */
#define SFT_PRESET_THEORY 2  /* beta = 6 sqrt(r), kappa = ceil(6 r ln N / (sqrt(2) pi)) + 1 (Theorem 4) */

/* identification of the inner sparse FFT (Algorithm 1) */
#define SFT_IDENT_RESIDUE 0  /* heavy bins of several moduli combined by the CRT, then a majority vote */
#define SFT_IDENT_PHASE   1  /* each heavy bin's frequency from its phase against samples one grid step later */

#define SFT_MAX_MODULI 15    /* K = 2G + 1 <= 15 */
#define SFT_MAX_BANDS  128

/*
 * Filter / window / inner-algorithm parameters.  A zero field means "the
 * preset's default".  tau is Lemma 3's passband floor (default 1/3, the
 * choice made after Lemma 13); r is Theorem 4's accuracy exponent (theory
 * preset only, default 1); s1_mult multiplies the identification modulus s1
 * (default 1: s1 = least power of two >= 2 s); group is G, the number of
 * primes per CRT tuple (default max(2, ceil(log2(N/s1)/6))); heavy_T is the
 * number of heavy bins kept per short DFT (default 2 s).  dft_path chooses the
 * short-DFT kernels: 1 = a whole block in LDS, p-point step on the vector
 * ALUs; 2 = split (row FFTs, p-point columns and selection as separate
 * kernels over HBM); 3 = a whole block in LDS, p-point step on the matrix
 * cores (s1 = 64 or 128, every (p_j - 1)/2 < 32); 4 = split with the p-point
 * step on the matrix cores (s1 >= 64, every (p_j - 1)/2 <= 47); 0 = automatic:
 * 3 when it covers the plan, else 1 when two of its workgroups fit a CU's
 * LDS, else 4 when it covers the plan, else 2 (sft_plan_info.dft_path reports
 * the choice).  Paths 1 and 2 give bitwise equal results for s1 <= 256 (for
 * s1 >= 512 their row FFTs differ in order, results agree to FP32 rounding),
 * and so do paths 3 and 4; the matrix-core paths sum the p-point step in
 * another order.
 * gather_path chooses the filtered-sample kernel: 1 = band sums on the vector
 * ALUs (one node per lane), 2 = band sums as a product on the matrix cores
 * (s1 >= 16, up to 64 bands and 63 taps), 0 = automatic (2 when it covers the plan;
 * sft_plan_info.gather_path reports the choice).  The two sum in different
 * orders (results agree to FP32 rounding).
 * dft_split (dft_path 3 only): 0 = automatic (the moduli whose blocks fit
 * three workgroups per CU run as a launch of their own when the largest do
 * not), -1 = one launch, j >= 1 = the moduli [0, j) in a launch of their own
 * (j < K); every choice gives the same results.
 * ident chooses the identification (SFT_IDENT_*).  SFT_IDENT_PHASE is the
 * phase-shift family that Section 5 pairs with CLW-DSFT (whose inner algorithm
 * the paper does not print): the filtered samples are also taken at every node
 * moved one grid step (x + 2 pi / N), their short DFTs E' are formed too, and a
 * heavy bin h of modulus j yields the w in B with w = h (mod P_j) whose angle
 * 2 pi w / N lies circularly nearest to arg(E'[h] conj(E[h])) (FP64; ties to
 * the smaller w).  Candidates of all moduli are merged and kept if more than
 * half of all K moduli hold a heavy bin at w; the estimate is the same median.
 * It doubles the samples and short DFTs.
 */
typedef struct sft_params {
    int32_t preset;
    int32_t kappa;
    double  sigma_t;   /* Gaussian standard deviation in grid steps (dmsft presets) */
    double  tau;
    double  r;
    int32_t s1_mult;
    int32_t group;
    int32_t heavy_T;
    int32_t dft_path;
    int32_t ident;
    int32_t gather_path;
    int32_t dft_split;
} sft_params;

/*
 * Every derived plan quantity (Algorithm 1's parameters and band centres; Lemma 3;
 * Theorem 4; the inner algorithm's moduli).  Band b = 0..Q-1 has centre
 * q_b = q_first + 2 b L and keeps the frequencies [q_b - L, q_b + L) of B.
 * Modulus j = 0..K-1 has short-DFT length P[j] = s1 * primes[j] and nodes
 * x = 2 pi k / P[j], k = 0..P[j]-1.
 */
typedef struct sft_plan_info {
    int64_t N;
    int32_t s;
    int32_t preset;
    int32_t kappa;
    int32_t Q;
    int64_t L;
    int64_t q_first;
    int32_t s1;
    int32_t G;
    int32_t K;
    int32_t T;
    int32_t depth;      /* heaviest bins per residue class combined by the CRT step */
    int32_t ident;      /* SFT_IDENT_* */
    double  sigma_t;
    double  beta;
    double  c1;
    double  tau;
    double  alpha;
    double  c2;
    double  r;
    int32_t primes[SFT_MAX_MODULI];
    int32_t dft_path;   /* short-DFT path the plan runs (1-4; 0 from sft_plan_describe) */
    int64_t P[SFT_MAX_MODULI];
    int64_t M;          /* sum of P[j]: nodes per band */
    int32_t dft_split;  /* dft_path 3: the moduli [0, dft_split) run as a launch of their own with a
                           smaller LDS allocation per workgroup (more workgroups per CU); 0: one
                           launch (always 0 from sft_plan_describe) */
    int32_t gather_path;  /* filtered-sample kernel the plan runs (1, 2; 0 from sft_plan_describe) */
} sft_plan_info;

typedef struct sft_plan_s* sft_plan_t;

/* Fill *p with the defaults of a preset (all-zero overrides).  Host only. */
SFT_API int sft_params_default(sft_params* p, int32_t preset);

/*
 * Derive the plan for (N, s, params) without touching any device.  Host only.
 * N >= 2 kappa + 1, 1 <= s <= N, tau in (0, 1/sqrt(2 pi)), alpha in
 * [1, N / sqrt(ln N)] (Lemma 3), 1 <= r <= N/36 (theory preset, Theorem 4);
 * otherwise SFT_EINVAL.  p may be NULL (dmsft6 defaults).
 */
SFT_API int sft_plan_describe(int64_t N, int32_t s, const sft_params* p, sft_plan_info* out);

/*
 * Create a plan on the current HIP device: derives the plan and uploads its
 * tables (band phasors exp(-2 pi i (q_b i mod N)/N), DFT twiddles, CRT
 * constants).  Synchronous.  The workspace of sft_execute is allocated by
 * the plan's first sft_execute (a plan used only in batches never holds
 * one).  On failure *out is NULL and nothing is leaked.
 */
SFT_API int sft_plan_create(sft_plan_t* out, int64_t N, int32_t s, const sft_params* p);

SFT_API int sft_plan_get_info(const sft_plan_t plan, sft_plan_info* out);

/* Device bytes the plan holds now: its tables, plus its sft_execute
 * workspace once allocated; excludes f and outputs. */
SFT_API int sft_plan_footprint(const sft_plan_t plan, size_t* bytes_device);

/* Device workspace one transform of this plan needs (filtered samples,
 * bins, heavy-bin tables, band results; for the split path with matrix-core
 * columns also the per-block digit histograms of its selection): the size of its sft_execute
 * workspace and of its slice of a batch's workspace.  Host only. */
SFT_API int sft_plan_workspace_bytes(const sft_plan_t plan, size_t* bytes);

/*
 * One transform, enqueued on stream (asynchronous, no host synchronisation).
 *   f_dev           complex64[N] on the device, read only.
 *   out_freqs_dev   int64[s]: frequencies ordered by |coefficient| descending,
 *                   ties to the smaller frequency (Algorithm 1, last step).
 *   out_coeffs_dev  complex64[s]: the matching coefficients c_w.
 *   out_count_dev   int32[1] or NULL: number of filled slots n <= s; slots
 *                   n..s-1 hold w = 0, c = 0.
 */
SFT_API int sft_execute(sft_plan_t plan, const void* f_dev, int64_t* out_freqs_dev,
                void* out_coeffs_dev, int32_t* out_count_dev, void* stream);

/*
 * sft_execute for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as sft_execute, with the workspace taken from a
 * fixed per-device scratch array of the library (64 MiB; each device the
 * library runs on holds it until the process ends) instead of the plan's own.
 * Calls no hipMalloc, hipFree or other allocating routine, and records no
 * per-kernel timing events.  Arguments as sft_execute; the plan must have been
 * created on the current device.  Returns SFT_EINVAL, before anything is
 * enqueued, when sft_plan_workspace_bytes of the plan exceeds 64 MiB (the
 * headline N = 2^22, s = 64 plan needs 11.5 MB).  Every call on a device
 * shares that device's scratch and leaves its contents behind: calls that
 * overlap on one device (different streams, or host threads, without
 * ordering between them) race and give wrong results; order them on one
 * stream.  sft_plan_status reads the call's flags from the scratch, valid
 * until the next call that uses it; sft_plan_fetch does not see it.
 */
SFT_API int sft_execute_noalloc(sft_plan_t plan, const void* f_dev, int64_t* out_freqs_dev,
                                void* out_coeffs_dev, int32_t* out_count_dev, void* stream);

/*
 * count transforms in one batched launch sequence; plans may differ in N and s
 * and the same plan may appear several times.  Arrays are host arrays of
 * device pointers, one entry per transform; out_counts_dev is a device
 * int32[count] or NULL.  Results are identical to count sft_execute calls.
 */
SFT_API int sft_execute_many(const sft_plan_t* plans, int32_t count, const void* const* f_dev,
                     int64_t* const* out_freqs_dev, void* const* out_coeffs_dev,
                     int32_t* out_counts_dev, void* stream);

/*
 * Device-side status of every transform of the last sft_execute_many on
 * stream (Algorithm 1 per transform; the capacities are those of
 * sft_plan_status).  Synchronises the stream; flags (host int32[count], may
 * be NULL) receives each transform's flags.  count must equal that call's
 * count.  Returns SFT_EOVERFLOW if any flag is set.
 */
SFT_API int sft_execute_many_status(void* stream, int32_t count, int32_t* flags);

/*
 * The workspace of sft_execute_many is owned by the library, one per
 * (device, stream), and grows when a larger batch arrives (after the stream
 * has drained).  reserve sizes it for batches of up to count transforms
 * whose sft_plan_workspace_bytes sum to at most workspace_bytes, so that
 * such calls allocate nothing; release frees the stream's workspace after
 * its work has completed.
 */
SFT_API int sft_execute_many_reserve(void* stream, size_t workspace_bytes, int32_t count);
SFT_API int sft_execute_many_release(void* stream);

/*
 * Prepared batches: the transforms of sft_execute_many with their inputs and
 * outputs fixed once, for callers that run the same batch shape again and
 * again (a serving slot, a pipeline stage).  Same computation and results as
 * sft_execute_many over the same arguments (Algorithm 1 per transform).
 *
 * sft_batch_create (host, synchronous): validates the arguments as
 *   sft_execute_many does, allocates the batch's own workspace and uploads
 *   its descriptor tables.  The plans must stay alive and the device buffers
 *   valid while the batch exists; the caller rewrites the contents of the
 *   input buffers between launches.  out_counts_dev may be NULL.
 * sft_batch_launch: enqueues the kernel sequence on stream: no allocation,
 *   no copies, no host synchronisation (so it may itself be captured).
 * sft_batch_graph_launch: the first call captures that kernel sequence into a
 *   hipGraph (on a stream of the batch's own) and instantiates it; every call
 *   launches the graph on stream.  Launches of one batch share its workspace:
 *   they must not overlap (order them on one stream).
 * sft_batch_destroy: frees the batch; it must be idle.  NULL is a no-op.
 */
typedef struct sft_batch_s* sft_batch_t;
SFT_API int sft_batch_create(sft_batch_t* out, const sft_plan_t* plans, int32_t count, const void* const* f_dev,
                             int64_t* const* out_freqs_dev, void* const* out_coeffs_dev, int32_t* out_counts_dev);
SFT_API int sft_batch_launch(sft_batch_t batch, void* stream);
SFT_API int sft_batch_graph_launch(sft_batch_t batch, void* stream);
SFT_API void sft_batch_destroy(sft_batch_t batch);
/* Status flags of every transform of the batch's last launch (as
 * sft_execute_many_status): synchronises, fills flags (host int32[count],
 * may be NULL), returns SFT_EOVERFLOW if any is set. */
SFT_API int sft_batch_status(sft_batch_t batch, int32_t* flags);

/*
 * Synchronise with the plan's last sft_execute (or sft_execute_noalloc) and return its device-side
 * status flags (0 = fine; bit 0: accepted-candidate list of a band overflowed;
 * bit 1: merge list overflowed).  Returns SFT_EOVERFLOW if any flag is set,
 * SFT_EINVAL if the plan has not run sft_execute.  Batches report through
 * sft_execute_many_status and sft_batch_status.
 */
SFT_API int sft_plan_status(sft_plan_t plan, int32_t* flags);

/*
 * Copy an intermediate of the plan's last sft_execute to host memory
 * (synchronises the device).  what:
 *   SFT_FETCH_SAMPLES  complex64[Q * M]: filtered samples; modulus j, band b
 *                      occupy [Q*Moff_j + b*P_j, +P_j) with Moff_j = sum_{i<j} P_i;
 *                      entry n1 + s1*n2 is the node k = (n1 p_j + n2 s1) mod P_j.
 *   SFT_FETCH_BINS     complex64[Q * M]: short-DFT bins, same blocks; entry
 *                      k1 + s1*k2 is the bin h with h = k1 (mod s1), h = k2 (mod p_j).
 *   SFT_FETCH_HEAVY    int32[K * Q * T]: heavy bins h of block (j, b) at
 *                      (j*Q + b)*T, in ascending Good-Thomas position.
 *   SFT_FETCH_BANDS    per band b: int32 count at [b], then (int64 w, double re,
 *                      double im) records; see the library documentation.
 *   SFT_FETCH_SAMPLES_SHIFTED, SFT_FETCH_BINS_SHIFTED  (SFT_IDENT_PHASE plans)
 *                      as SAMPLES and BINS for the nodes moved one grid step.
 *   SFT_FETCH_CLASSES  int32[K * Q * s1 * depth]: per block (j, b) and residue
 *                      class c (h mod s1), at ((j*Q + b)*s1 + c)*depth + e, the
 *                      e-th heaviest heavy bin of the class (larger |E|^2
 *                      first, the lower h first on equal |E|^2), -1 where the
 *                      class holds fewer than e + 1 heavy bins: the lists
 *                      that the CRT step combines.
 * bytes_needed (may be NULL) receives the size; dst may be NULL to query.
 */
#define SFT_FETCH_SAMPLES 0
#define SFT_FETCH_BINS    1
#define SFT_FETCH_HEAVY   2
#define SFT_FETCH_BANDS   3
#define SFT_FETCH_SAMPLES_SHIFTED 4
#define SFT_FETCH_BINS_SHIFTED    5
#define SFT_FETCH_CLASSES         6
SFT_API int sft_plan_fetch(const sft_plan_t plan, int32_t what, void* dst, size_t bytes,
                   size_t* bytes_needed);

/* Free the plan's device memory.  The plan must be idle.  NULL is a no-op. */
SFT_API void sft_plan_destroy(sft_plan_t plan);

/* Message of the calling thread's last failed call ("" if none). */
SFT_API const char* sft_last_error(void);

/*
 * Per-kernel timing with HIP events recorded around every launch on the
 * launch stream.  Off by default.  kernel: SFT_KERNEL_*.  Reading
 * synchronises on the recorded events; sft_profile_reset clears the totals.
 */
#define SFT_KERNEL_GATHER   0   /* filtered samples */
#define SFT_KERNEL_DFT      1   /* short DFTs + heavy-bin selection, block in LDS */
#define SFT_KERNEL_IDENTIFY 2   /* candidates, vote, median, band test, divide */
#define SFT_KERNEL_MERGE    3   /* global top-s */
#define SFT_KERNEL_DFT_ROWS 4   /* split path for blocks larger than LDS: radix-2 row FFTs */
#define SFT_KERNEL_DFT_COLS 5   /* split path: p-point column DFTs */
#define SFT_KERNEL_SELECT   6   /* split path: heavy-bin selection from global memory */
#define SFT_KERNEL_DFT_MX   7   /* as SFT_KERNEL_DFT, the p-point step on the matrix cores */
#define SFT_KERNEL_DFT_COLS_MX 8   /* as SFT_KERNEL_DFT_COLS, on the matrix cores */
#define SFT_KERNEL_GATHER_MX 9   /* as SFT_KERNEL_GATHER, the band sums on the matrix cores */
#define SFT_KERNEL_COUNT    10
SFT_API int sft_profile_enable(int32_t on);
SFT_API int sft_profile_reset(void);
SFT_API int sft_profile_read(int32_t kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* SFT_H */
