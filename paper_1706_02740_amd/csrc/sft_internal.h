// Internal definitions shared by the host runtime and the HIP kernels.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

#include "sft.h"

namespace sft {

constexpr int kMaxK = SFT_MAX_MODULI;
constexpr int kMaxG = 7;
constexpr int kThreads = 256;          // workgroup size of every kernel but k_dft (4 wave64)
constexpr int kIdentifyWide = 1024;    // k_identify workgroup size for launches of at most
constexpr int kIdentifyWideMaxBlocks = 256;  // this many bands (one per CU at most)
constexpr int kDftThreads = 512;       // k_dft workgroup size (8 wave64)
constexpr int kBandChunk = 16;         // bands accumulated per pass of the generic gather kernel (table padding)
constexpr int kFastTaps = 16;          // window widths with a compile-time gather kernel are at most this
constexpr int kAcceptCap = 4096;       // bound on the accepted candidates per band kept in LDS
constexpr int kMergeCap = 4096;        // band results merged per signal in LDS
constexpr int kMergeWide = 1024;       // k_merge workgroup size for launches of at most
constexpr int kMergeWideMaxBlocks = 256;   // this many transforms (one per CU at most),
constexpr int kMergeWideMinS = 128;    // one of them with s above this
constexpr int kSlotMap = 2048;         // k_identify: combinations whose (tuple, class) slot is tabulated in LDS
constexpr int kRowElems = 4096;        // complex values per workgroup in the split path's row FFTs
constexpr int kColChunk = 64;          // columns per workgroup in the split path's p-point DFTs
constexpr int kMaxDepth = 8;           // class-list length bound (depth^G <= 64 with G >= 2)
constexpr int kSelBins = 1024;         // buckets of one radix-select pass (10-bit digits)
constexpr int kMxSteps = 8;            // K-steps (4 values of n each) of the matrix-core p-point step: h <= 32
constexpr int kMxTiles = 2;            // M-tiles (16 values of k each): h + 1 <= 32
constexpr int kMxcSteps = 12;          // the split path's matrix-core columns: h <= 48
constexpr int kMxcTiles = 3;           // h + 1 <= 48
constexpr int kDftKBMax = 16;          // p-point output pairs per thread in the in-LDS short-DFT kernel
constexpr int kSelLdsThreads = 1024;   // workgroup size of the split path's selection with its keys in LDS
constexpr int kSelLdsMaxBlocks = 256;  // launches up to this many selection blocks (one per CU) take it
constexpr int kGmxMaxMT = 8, kGmxMaxKS = 32;  // k_gather_mx: at most 64 bands and 63 taps

// Status bits written by the device.
constexpr int kStatusAcceptOverflow = 1;
constexpr int kStatusMergeOverflow = 2;

// Per-plan constants, uploaded once at plan creation.  Every kernel reads it
// through a device pointer; all reads are wave-uniform.
struct SigDesc {
    int64_t N;
    int64_t L;
    int64_t q_first;        // q_b = q_first + 2 b L
    int64_t lo, hi;         // B = [lo, hi]
    int32_t s, kappa, taps, Q, K, G, s1, log2s1, T, depth, M, Tpow2;
    int32_t accept_cap;     // accepted candidates one band may hold: min(4096, pow2 >= 8 s)
    int32_t vote_bitmap;    // 1: the heavy-bin bitmaps of identify fit the LDS; 0: identify must vote from bin keys
    int32_t phase;          // 1: phase identification (samples and bins also at the nodes moved one grid step)
    int32_t sel_cap;        // candidate keys the split path's selection keeps in LDS: pow2 >= 4 T in [1024, 4096]
    float   inv2sig2;       // 1 / (2 sigma_t^2)
    float   wnorm;          // 1 / (2 pi sigma_t): W(v) = wnorm exp(-v^2 inv2sig2)
    float   gtap[kFastTaps];  // exp(-(i - kappa)^2 inv2sig2), i < taps (taps <= kFastTaps)
    float   a_first;        // q_first / N    (per-node band phase rate, in turns)
    float   a_step;         // 2 L / N
    double  c1sq_half;      // c1^2 / 2
    double  ghat0;          // 1 / sqrt(2 pi)
    int32_t p[kMaxK];
    int32_t P[kMaxK];
    int32_t Moff[kMaxK + 1];
    int32_t pinv_s1[kMaxK];  // p_j^{-1} mod s1   (Good-Thomas output map)
    int32_t s1inv_p[kMaxK];  // s1^{-1} mod p_j
    int32_t tw_off[kMaxK];   // offset of modulus j's p-point twiddles in tw_p
    // CRT tuples: component 0 is s1, components 1..G are the tuple's primes.
    int32_t tup_j[2][kMaxG];
    int64_t tup_M[2];
    int64_t tup_Mi[2][kMaxG + 1];
    int32_t tup_inv[2][kMaxG + 1];
    int32_t tup_mod[2][kMaxG + 1];
    // exact remainders by multiplication for the identification's divisors
    // (Lemire, Kaser and Kurz, "Faster remainder by direct computation", 2019):
    // magic = floor((2^64 - 1) / d) + 1, valid for every 32-bit dividend
    uint64_t magic_p[kMaxK];   // d = p_j
    uint64_t magic_P[kMaxK];   // d = P_j
    int32_t lo_mod_P[kMaxK];   // lo mod P_j, in [0, P_j)
    // device tables owned by the plan
    const float2* bandtab;   // [Q][taps]: exp(-2 pi i ((q_b (i - kappa)) mod N) / N)
    const float2* bandtab_t; // [taps][Qpad]: the same transposed, zero past Q (Qpad: Q up to whole kBandChunk)
    int32_t qpad;
    const float2* tw_s1;     // [s1/2]: exp(-2 pi i k / s1)
    const float2* tw_p;      // concatenated [p_j]: exp(-2 pi i m / p_j)
    const float* rate;       // [Q]: q_b / N, the per-node band phase rate in turns
    const float2* trig;      // concatenated [h_j^2]: (cos, sin)(2 pi (n k mod p_j) / p_j), n, k in [1, h_j]
    int32_t trig_off[kMaxK];
    // [K][kMxSteps][kMxTiles][64]: the matrix-core step's A operands in lane order;
    // lane l of step st, tile m, i = l % 16: n = 1 + 4 st + l / 16, k = 16 m + 4 (i % 4) + i / 4 ->
    // (cos, sin)(2 pi (n k mod p) / p) for n, k in [1, h]; (1, 0) for k = 0 < n <= h; else 0
    const float2* mxa;
    // [K][kMxcSteps][kMxcTiles][64]: the same operands for the split path's
    // matrix-core column kernel (null when the plan does not use it)
    const float2* mxc;
    // k_gather_mx: the band table as a real matrix, [gmx_mt][gmx_ks][64] in
    // lane order (lane l of M-tile m, K-step st holds A[16 m + l % 16][4 st + l / 16],
    // A[2 b + e][2 i + x]: e = 0: (Re T, -Im T), e = 1: (Im T, Re T) for x = 0, 1),
    // and exp(-(i - kappa)^2 inv2sig2) for i < 2 gmx_ks (zero from taps on)
    int32_t gmx_mt, gmx_ks;
    const float* gmx_a;
    const float* gmx_g;
};

// Per-transform pointers: input, outputs and workspace slices.
struct IoDesc {
    const float2* f;
    int64_t* out_w;
    float2* out_c;
    int32_t* out_n;
    float2* S;        // [Q*M] filtered samples
    float2* E;        // [Q*M] short-DFT bins
    float2* S2;       // [Q*M] samples at the nodes moved one grid step (phase identification), else null
    float2* E2;       // [Q*M] their short-DFT bins
    int32_t* H;       // [K*Q*T] heavy bins, ascending Good-Thomas position (for inspection)
    uint64_t* thr;    // [K*Q] selection threshold: a bin is heavy iff its key >= thr
    int32_t* CL;      // [K*Q*s1*depth] per residue class: heaviest heavy bins, -1 padded
    int64_t* Rw;      // [Q*s] band results: frequencies
    double2* Rv;      // [Q*s] band results: coefficients
    int32_t* Rn;      // [Q] band result counts
    int32_t* status;  // [1]
    int32_t* SH;      // [K*Q*kSelBins] split path with matrix-core columns: per block, the histogram of
                      // the bins' top key digit (filled by the column kernel), else null
};

// Kernel launch argument: one transform (io_many == nullptr), a batch of one
// plan (bps > 0: transform i owns blocks [i bps, (i + 1) bps) and desc_one is
// its descriptor), or a batch of several plans (prefix table + descriptors).
struct BatchArgs {
    const SigDesc* desc_one;
    IoDesc io_one;
    const SigDesc* const* descs_many;  // [nsig] device array of plan descriptors (mixed batches)
    const IoDesc* io_many;             // [nsig]
    const int32_t* prefix;             // [nsig+1] first block of each signal for this kernel (mixed)
    int32_t nsig;
    int32_t bps;                       // blocks per transform of a one-plan batch, else 0
    int32_t jlo, jn;                   // short-DFT launches: the moduli [jlo, jlo + jn) only (jn = 0: all)
};

// The matrix-core short DFTs of a plan in two launches: moduli [0, j1) with
// lds_lo bytes per workgroup, then [j1, K) (j1 = 0: one launch).  qb: blocks
// per modulus of one transform, Q (1 + phase).  Launches of fewer than
// min_blocks blocks stay whole: with a few blocks per CU, occupancy does not
// matter and the second launch would only add its latency.
struct MxSplit {
    int j1 = 0, K = 0, qb = 0, min_blocks = 0;
    size_t lds_lo = 0;
};

// Per-signal workspace sizes in bytes (each slice 256-byte aligned).
struct WorkspaceLayout {
    size_t S, E, S2, E2, H, thr, CL, Rw, Rv, Rn, status, SH, total;
};

// plan.cpp
int derive_plan(int64_t N, int32_t s, const sft_params* p, sft_plan_info* out, const char** why);
void fill_desc(const sft_plan_info& info, SigDesc* d);
WorkspaceLayout workspace_layout(const sft_plan_info& info);
size_t dft_lds_bytes(const SigDesc& d);
// LDS of the matrix-core in-LDS short-DFT kernel for a launch over the moduli [0, jhi) or up to jhi.
size_t dft_mx_lds_bytes(const SigDesc& d, int jhi);
bool dft_fits_one_workgroup(const SigDesc& d);   // the in-LDS short-DFT kernel's shape limits
int dft_pairs_per_thread(const SigDesc& d);
// Whether the in-LDS kernel's matrix-core step B covers the plan (s1 = 64 NTW, h + 1 <= 16 MT, NTW, MT <= 2):
// MT * 4 + NTW, else 0.
int dft_mfma_variant(const SigDesc& d);

// kernels.hip: host-side launchers (enqueue only).  Block counts per signal:
int gather_blocks(const SigDesc& d);
int dft_blocks(const SigDesc& d);
int identify_blocks(const SigDesc& d);
int merge_blocks(const SigDesc& d);
// taps: 2 kappa + 1 shared by every transform of the launch, or 0 (read per transform)
hipError_t launch_gather(const BatchArgs& a, int blocks, int taps, hipStream_t st);
// lds: the byte count (low 32 bits); above: the M-tile count (bits 32..39) and whether some
// plan has more than 16 taps (bit 40), each the maximum over the launch's plans
int gather_mx_blocks(const SigDesc& d);
size_t gather_mx_lds_bytes(const SigDesc& d);
hipError_t launch_gather_mx(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t launch_dft(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t launch_identify(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
// split short-DFT path for blocks larger than one workgroup's LDS
int rows_blocks(const SigDesc& d);
int cols_blocks(const SigDesc& d);
int select_blocks(const SigDesc& d);
size_t rows_lds_bytes(const SigDesc& d);
size_t cols_lds_bytes(const SigDesc& d);
size_t select_lds_bytes(const SigDesc& d, bool lds_keys);   // with the block's keys held in LDS or not
hipError_t launch_dft_rows(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t launch_dft_mx(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t launch_dft_cols(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
// the split path with its p-point step on the matrix cores (s1 >= 64, every h <= 47)
int cols_mx_blocks(const SigDesc& d);
bool cols_mx_covers(const SigDesc& d);
size_t cols_mx_lds_bytes(const SigDesc& d);
hipError_t launch_dft_cols_mx(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t launch_select(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t launch_merge(const BatchArgs& a, int blocks, size_t lds, hipStream_t st);
hipError_t configure_kernels(int max_lds);
// The no-alloc workspace: kScratchBytes per device, its device address on
// device dev (the current device; looked up on the first call per device).
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
hipError_t scratch_address(int dev, void** out);
size_t identify_lds_bytes(const SigDesc& d, bool bitmap);   // with or without the heavy-bin bitmaps
size_t merge_lds_bytes();

}  // namespace sft
