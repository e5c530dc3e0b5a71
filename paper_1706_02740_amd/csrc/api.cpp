// C ABI of libsft: plans, device tables, workspaces, launches, profiling.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "sft_internal.h"

using namespace sft;

// ------------------------------------------------------------- errors ----
static thread_local std::string g_err;

static int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

static int hip_fail(hipError_t e, const char* what) {
    return fail(SFT_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// --------------------------------------------------------------- plans ----
struct sft_plan_s {
    sft_plan_info info;
    SigDesc hdesc;          // host copy (device pointers filled in)
    SigDesc* ddesc = nullptr;
    void* tables = nullptr; // one allocation for every table
    void* ws = nullptr;     // workspace of sft_execute
    WorkspaceLayout wl;
    IoDesc ws_io;           // workspace slices (f and outputs unset)
    size_t footprint = 0;
    size_t lds[SFT_KERNEL_COUNT] = {};
    int blocks[SFT_KERNEL_COUNT] = {};   // per transform; 0 = kernel not used
    bool split = false;     // short DFTs too large for one workgroup's LDS
    MxSplit mxs;            // the matrix-core short DFTs in two launches (mxs.j1 > 0)
    int device = 0;
    hipStream_t last_stream = nullptr;
    int32_t* last_status = nullptr;   // status word of the last single transform (own workspace or scratch)
};

static IoDesc carve(void* base, const WorkspaceLayout& wl) {
    IoDesc io;
    memset(&io, 0, sizeof(io));
    char* p = static_cast<char*>(base);
    io.S = reinterpret_cast<float2*>(p); p += wl.S;
    io.E = reinterpret_cast<float2*>(p); p += wl.E;
    io.S2 = wl.S2 ? reinterpret_cast<float2*>(p) : nullptr; p += wl.S2;
    io.E2 = wl.E2 ? reinterpret_cast<float2*>(p) : nullptr; p += wl.E2;
    io.H = reinterpret_cast<int32_t*>(p); p += wl.H;
    io.thr = reinterpret_cast<uint64_t*>(p); p += wl.thr;
    io.CL = reinterpret_cast<int32_t*>(p); p += wl.CL;
    io.Rw = reinterpret_cast<int64_t*>(p); p += wl.Rw;
    io.Rv = reinterpret_cast<double2*>(p); p += wl.Rv;
    io.Rn = reinterpret_cast<int32_t*>(p); p += wl.Rn;
    io.status = reinterpret_cast<int32_t*>(p); p += wl.status;
    io.SH = wl.SH ? reinterpret_cast<int32_t*>(p) : nullptr;
    return io;
}

static std::mutex g_cfg_mu;
static std::map<int, int> g_max_lds;   // device -> max dynamic LDS per workgroup (configured)

static int device_lds_limit(int dev, int* out) {
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    auto it = g_max_lds.find(dev);
    if (it != g_max_lds.end()) {
        *out = it->second;
        return SFT_OK;
    }
    int v = 0;
    HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev), "hipDeviceGetAttribute");
    HIP_TRY(configure_kernels(v), "hipFuncSetAttribute");
    g_max_lds[dev] = v;
    *out = v;
    return SFT_OK;
}

extern "C" {

int sft_params_default(sft_params* p, int32_t preset) {
    if (!p) return fail(SFT_EINVAL, "params pointer is NULL");
    if (preset < 0 || preset > 2) return fail(SFT_EINVAL, "unknown preset");
    memset(p, 0, sizeof(*p));
    p->preset = preset;
    return SFT_OK;
}

int sft_plan_describe(int64_t N, int32_t s, const sft_params* p, sft_plan_info* out) {
    if (!out) return fail(SFT_EINVAL, "info pointer is NULL");
    const char* why = "";
    const int rc = derive_plan(N, s, p, out, &why);
    if (rc != SFT_OK) return fail(rc, why);
    return SFT_OK;
}

void sft_plan_destroy(sft_plan_t plan) {
    if (!plan) return;
    if (plan->ws) (void)hipFree(plan->ws);
    if (plan->tables) (void)hipFree(plan->tables);
    if (plan->ddesc) (void)hipFree(plan->ddesc);
    delete plan;
}

int sft_plan_create(sft_plan_t* out, int64_t N, int32_t s, const sft_params* p) {
    if (!out) return fail(SFT_EINVAL, "plan pointer is NULL");
    *out = nullptr;
    sft_plan_info info;
    const char* why = "";
    int rc = derive_plan(N, s, p, &info, &why);
    if (rc != SFT_OK) return fail(rc, why);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    int lds_limit = 0;
    if ((rc = device_lds_limit(dev, &lds_limit)) != SFT_OK) return rc;
    int cus = 0;
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "hipDeviceGetAttribute");

    sft_plan_s* pl = new sft_plan_s();
    pl->info = info;
    pl->device = dev;
    fill_desc(info, &pl->hdesc);
    SigDesc& d = pl->hdesc;
    const size_t lds_cap = (size_t)lds_limit - 256;   // room for the kernels' static LDS
    const int path = p ? p->dft_path : 0;
    if (path < 0 || path > 4) {
        delete pl;
        return fail(SFT_EINVAL, "dft_path must be 0, 1, 2, 3 or 4");
    }
    if (p && (p->dft_split < -1 || p->dft_split >= d.K)) {
        delete pl;
        return fail(SFT_EINVAL, "dft_split must be -1, 0 or a modulus count below K");
    }
    const bool fits = dft_fits_one_workgroup(d) && dft_lds_bytes(d) <= lds_cap;
    const int mx = dft_mfma_variant(d);
    const bool mx_fits = mx != 0 && dft_mx_lds_bytes(d, d.K) <= lds_cap;
    if (path == 1 && !fits) {
        delete pl;
        return fail(SFT_EUNSUPPORTED, "the in-LDS short-DFT kernel cannot hold this plan (use dft_path 0 or 2)");
    }
    if (path == 3 && !mx_fits) {
        delete pl;
        return fail(SFT_EUNSUPPORTED, "the matrix-core short-DFT kernel does not cover this plan (use dft_path 0)");
    }
    const bool cmx_fits = cols_mx_covers(d) && cols_mx_lds_bytes(d) <= lds_cap;
    if (path == 4 && !cmx_fits) {
        delete pl;
        return fail(SFT_EUNSUPPORTED, "the matrix-core column kernel does not cover this plan (use dft_path 0 or 2)");
    }
    // automatic: the in-LDS VALU kernel only while two of its workgroups fit
    // a CU (with one, the split kernels are faster: measured by the tuner)
    const bool valu_auto = fits && dft_lds_bytes(d) <= (size_t)lds_limit / 2;
    pl->split = path == 2 || path == 4 || (path == 0 && !mx_fits && !valu_auto);
    const bool cols_mx = pl->split && (path == 4 || (path == 0 && cmx_fits));
    // filtered samples: band sums on the matrix cores when the band table fits
    // the kernel's tiles and its LDS, else on the vector ALUs
    const int gpath = p ? p->gather_path : 0;
    if (gpath < 0 || gpath > 2) {
        delete pl;
        return fail(SFT_EINVAL, "gather_path must be 0, 1 or 2");
    }
    d.gmx_mt = (2 * d.Q + 15) / 16;
    d.gmx_ks = (2 * d.taps + 3) / 4;
    // (tiles of 16 nodes lie within one modulus when 16 divides s1)
    const bool gmx_fits = d.s1 >= 16 && d.gmx_mt <= kGmxMaxMT && d.gmx_ks <= kGmxMaxKS &&
                          gather_mx_lds_bytes(d) <= lds_cap;
    if (gpath == 2 && !gmx_fits) {
        delete pl;
        return fail(SFT_EUNSUPPORTED, "the matrix-core gather does not cover this plan (use gather_path 0 or 1)");
    }
    // automatic: the matrix cores for windows wider than 16 taps; narrower
    // windows are faster on the vector ALUs (measured: N = 2^22, s = 64, 13
    // taps, 0.60 vs 0.72 ms per 256 transforms; 45 taps, 11.4 vs 4.5 ms)
    const bool use_gmx = gpath == 2 || (gpath == 0 && gmx_fits && d.taps > 16);
    pl->info.gather_path = use_gmx ? 2 : 1;
    if (use_gmx) {
        // bits 32..39: M-tiles; bit 40: more than 16 taps (merged over a batch by maximum)
        pl->lds[SFT_KERNEL_GATHER_MX] = gather_mx_lds_bytes(d) | ((size_t)d.gmx_mt << 32) |
                                        ((size_t)(d.taps > 16) << 40);
        pl->blocks[SFT_KERNEL_GATHER_MX] = gather_mx_blocks(d);
    } else {
        d.gmx_mt = d.gmx_ks = 0;
        pl->lds[SFT_KERNEL_GATHER] = (size_t)d.taps;   // the gather launcher's tap count
        pl->blocks[SFT_KERNEL_GATHER] = gather_blocks(d);
    }
    d.vote_bitmap = identify_lds_bytes(d, true) <= lds_cap ? 1 : 0;
    // bit 32: the key vote; bit 33: phase identification (a batch takes each
    // when any of its plans needs it)
    pl->lds[SFT_KERNEL_IDENTIFY] = identify_lds_bytes(d, d.vote_bitmap != 0) | ((size_t)(d.vote_bitmap == 0) << 32) |
                                   ((size_t)d.phase << 33);
    pl->lds[SFT_KERNEL_MERGE] = merge_lds_bytes() | ((size_t)(d.s > kMergeWideMinS) << 32);   // bit 32: a large s
    pl->blocks[SFT_KERNEL_IDENTIFY] = identify_blocks(d);
    pl->blocks[SFT_KERNEL_MERGE] = merge_blocks(d);
    pl->info.dft_path = pl->split ? (cols_mx ? 4 : 2) : (path == 3 || (path == 0 && mx_fits)) ? 3 : 1;
    if (!pl->split) {
        const bool use_mx = path == 3 || (path == 0 && mx_fits);
        if (use_mx) {
            pl->lds[SFT_KERNEL_DFT_MX] = dft_mx_lds_bytes(d, d.K);
            pl->blocks[SFT_KERNEL_DFT_MX] = dft_blocks(d);
            // Two workgroups of the largest blocks fill a CU's LDS; when the
            // smaller moduli's blocks fit three to a CU, they get a launch of
            // their own with that smaller allocation (measured: three
            // workgroups per CU take ~20 % less time per block than two).
            // The margin covers the static LDS and the allocation granularity.
            const size_t third = (size_t)lds_limit / 3 - 512;
            const int want = p ? p->dft_split : 0;   // 0: the rule above; -1: one launch; j: moduli [0, j)
            if (want > 0 || (want == 0 && pl->lds[SFT_KERNEL_DFT_MX] > third)) {
                int j1 = want;
                if (want == 0)
                    while (j1 < d.K && dft_mx_lds_bytes(d, j1 + 1) <= third) ++j1;
                if (j1 > 0 && j1 < d.K) {
                    pl->mxs.min_blocks = 12 * cus;   // four rounds of three workgroups per CU
                    pl->mxs.j1 = j1;
                    pl->mxs.K = d.K;
                    pl->mxs.qb = d.Q * (1 + d.phase);
                    pl->mxs.lds_lo = dft_mx_lds_bytes(d, j1);
                }
            }
            pl->info.dft_split = pl->mxs.j1;
        } else {
            // low 32 bits: LDS bytes; above: output pairs per thread (selects the kernel variant)
            pl->lds[SFT_KERNEL_DFT] = dft_lds_bytes(d) | ((size_t)dft_pairs_per_thread(d) << 32);
            pl->blocks[SFT_KERNEL_DFT] = dft_blocks(d);
        }
    } else {
        pl->lds[SFT_KERNEL_DFT_ROWS] = rows_lds_bytes(d);
        if (cols_mx) pl->lds[SFT_KERNEL_DFT_COLS_MX] = cols_mx_lds_bytes(d);
        else pl->lds[SFT_KERNEL_DFT_COLS] = cols_lds_bytes(d);
        // low 32 bits: the selection that reads E in every pass; above: the
        // one with the block's keys in LDS, 0 when they do not fit
        const size_t kbytes = select_lds_bytes(d, true);
        pl->lds[SFT_KERNEL_SELECT] = select_lds_bytes(d, false) | ((kbytes <= lds_cap ? kbytes : 0) << 32);
        pl->blocks[SFT_KERNEL_DFT_ROWS] = rows_blocks(d);
        if (cols_mx) pl->blocks[SFT_KERNEL_DFT_COLS_MX] = cols_mx_blocks(d);
        else pl->blocks[SFT_KERNEL_DFT_COLS] = cols_blocks(d);
        pl->blocks[SFT_KERNEL_SELECT] = select_blocks(d);
    }
    for (int k = 0; k < SFT_KERNEL_COUNT; ++k) {
        if (k != SFT_KERNEL_GATHER && (pl->lds[k] & 0xffffffffu) > lds_cap) {
            delete pl;
            return fail(SFT_EUNSUPPORTED, "plan needs more LDS per workgroup than the device holds");
        }
    }

    // ---- tables (FP64 on the host, rounded once to FP32)
    const int taps = d.taps;
    const int Qpad = (d.Q + kBandChunk - 1) / kBandChunk * kBandChunk;   // zero rows up to whole chunks
    const size_t n_band = (size_t)Qpad * taps;
    const size_t n_tws1 = d.s1 >= 2 ? (size_t)d.s1 / 2 : 1;
    size_t n_twp = 0;
    for (int j = 0; j < d.K; ++j) n_twp += d.p[j];
    size_t n_trig = 0;
    for (int j = 0; j < d.K; ++j) n_trig += (size_t)((d.p[j] - 1) / 2) * ((d.p[j] - 1) / 2);
    if (n_trig == 0) n_trig = 1;
    std::vector<float2> band(n_band, make_float2(0.f, 0.f)), tws1(n_tws1), twp(n_twp), trig(n_trig);
    std::vector<float> rate(Qpad, 0.f);
    for (int b = 0; b < d.Q; ++b) {
        const int64_t q = info.q_first + 2 * (int64_t)b * info.L;
        rate[b] = (float)((double)q / (double)N);
        for (int i = 0; i < taps; ++i) {
            const int64_t o = i - d.kappa;
            int64_t m = (q % N) * o % N;
            if (m < 0) m += N;
            const double ang = -2.0 * M_PI * ((double)m / (double)N);
            band[(size_t)b * taps + i] = make_float2((float)cos(ang), (float)sin(ang));
        }
    }
    std::vector<float2> bandt(n_band, make_float2(0.f, 0.f));   // [taps][Qpad]
    for (int b = 0; b < d.Q; ++b)
        for (int i = 0; i < taps; ++i) bandt[(size_t)i * Qpad + b] = band[(size_t)b * taps + i];
    d.qpad = Qpad;
    for (size_t k = 0; k < n_tws1; ++k) {
        const double ang = -2.0 * M_PI * (double)k / (double)d.s1;
        tws1[k] = make_float2((float)cos(ang), (float)sin(ang));
    }
    size_t o = 0;
    for (int j = 0; j < d.K; ++j)
        for (int m = 0; m < d.p[j]; ++m, ++o) {
            const double ang = -2.0 * M_PI * (double)m / (double)d.p[j];
            twp[o] = make_float2((float)cos(ang), (float)sin(ang));
        }
    o = 0;
    for (int j = 0; j < d.K; ++j) {
        const int pj = d.p[j], hj = (pj - 1) / 2;
        for (int n = 1; n <= hj; ++n)
            for (int k = 1; k <= hj; ++k, ++o) {
                const double ang = 2.0 * M_PI * (double)((n * k) % pj) / (double)pj;
                trig[o] = make_float2((float)cos(ang), (float)sin(ang));
            }
    }
    const size_t n_mxa = (size_t)d.K * kMxSteps * kMxTiles * 64;
    std::vector<float2> mxa(n_mxa, make_float2(0.f, 0.f));
    for (int j = 0; j < d.K; ++j) {
        const int pj = d.p[j], hj = (pj - 1) / 2;
        for (int st = 0; st < kMxSteps; ++st)
            for (int m = 0; m < kMxTiles; ++m)
                for (int l = 0; l < 64; ++l) {
                    // lane l supplies row i = l % 16 of the tile, which the
                    // in-LDS kernel assigns to k = 16 m + 4 (i % 4) + i / 4 (the
                    // four rows of an output register are consecutive)
                    const int i = l % 16;
                    const int n = 1 + 4 * st + l / 16, k = 16 * m + 4 * (i % 4) + i / 4;
                    float2 v = make_float2(0.f, 0.f);
                    if (n <= hj && k == 0) {
                        v = make_float2(1.f, 0.f);
                    } else if (n <= hj && k <= hj) {
                        const double ang = 2.0 * M_PI * (double)((n * k) % pj) / (double)pj;
                        v = make_float2((float)cos(ang), (float)sin(ang));
                    }
                    mxa[(((size_t)j * kMxSteps + st) * kMxTiles + m) * 64 + l] = v;
                }
    }
    // the split path's matrix-core columns: the same operands for up to
    // kMxcSteps x kMxcTiles tiles (only when the plan uses that kernel)
    const size_t n_mxc = pl->blocks[SFT_KERNEL_DFT_COLS_MX] ? (size_t)d.K * kMxcSteps * kMxcTiles * 64 : 0;
    std::vector<float2> mxc(n_mxc, make_float2(0.f, 0.f));
    for (int j = 0; j < d.K && n_mxc; ++j) {
        const int pj = d.p[j], hj = (pj - 1) / 2;
        for (int st = 0; st < kMxcSteps; ++st)
            for (int m = 0; m < kMxcTiles; ++m)
                for (int l = 0; l < 64; ++l) {
                    const int n = 1 + 4 * st + l / 16, k = 16 * m + l % 16;
                    float2 v = make_float2(0.f, 0.f);
                    if (n <= hj && k == 0) {
                        v = make_float2(1.f, 0.f);
                    } else if (n <= hj && k <= hj) {
                        const double ang = 2.0 * M_PI * (double)((n * k) % pj) / (double)pj;
                        v = make_float2((float)cos(ang), (float)sin(ang));
                    }
                    mxc[(((size_t)j * kMxcSteps + st) * kMxcTiles + m) * 64 + l] = v;
                }
    }
    // the matrix-core gather: the band table as the real matrix A (rows 2 b + e,
    // columns 2 i + x) in lane order, and the window factors exp(-(i - kappa)^2 c)
    const size_t n_gmxa = (size_t)d.gmx_mt * d.gmx_ks * 64, n_gmxg = (size_t)d.gmx_ks * 2;
    std::vector<float> gmxa(n_gmxa, 0.f), gmxg(n_gmxg, 0.f);
    for (int m = 0; m < d.gmx_mt; ++m)
        for (int st = 0; st < d.gmx_ks; ++st)
            for (int l = 0; l < 64; ++l) {
                const int row = 16 * m + l % 16, col = 4 * st + l / 16;
                const int b = row / 2, e = row % 2, i = col / 2, x = col % 2;
                if (b >= d.Q || i >= taps) continue;
                const float2 t = band[(size_t)b * taps + i];
                gmxa[((size_t)m * d.gmx_ks + st) * 64 + l] = e == 0 ? (x == 0 ? t.x : -t.y) : (x == 0 ? t.y : t.x);
            }
    for (size_t i = 0; i < n_gmxg && (int)i < taps; ++i) {
        const double o = (double)((int)i - d.kappa);
        gmxg[i] = (float)exp(-o * o / (2.0 * info.sigma_t * info.sigma_t));
    }
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t b_band = al(n_band * 8), b_tws1 = al(n_tws1 * 8), b_twp = al(n_twp * 8), b_rate = al((size_t)Qpad * 4);
    const size_t b_trig = al(n_trig * 8), b_mxa = al(n_mxa * 8), b_mxc = al(n_mxc * 8);
    const size_t b_gmxa = al(n_gmxa * 4), b_gmxg = al(n_gmxg * 4);
    const size_t tbytes = b_band + b_tws1 + b_twp + b_rate + b_trig + b_mxa + b_mxc + b_gmxa + b_gmxg + b_band;
    hipError_t e = hipMalloc(&pl->tables, tbytes);
    if (e != hipSuccess) { sft_plan_destroy(pl); return fail(SFT_ENOMEM, "hipMalloc(tables) failed"); }
    char* tb = static_cast<char*>(pl->tables);
    d.bandtab = reinterpret_cast<const float2*>(tb);
    d.tw_s1 = reinterpret_cast<const float2*>(tb + b_band);
    d.tw_p = reinterpret_cast<const float2*>(tb + b_band + b_tws1);
    d.rate = reinterpret_cast<const float*>(tb + b_band + b_tws1 + b_twp);
    d.trig = reinterpret_cast<const float2*>(tb + b_band + b_tws1 + b_twp + b_rate);
    d.mxa = reinterpret_cast<const float2*>(tb + b_band + b_tws1 + b_twp + b_rate + b_trig);
    d.mxc = n_mxc ? reinterpret_cast<const float2*>(tb + b_band + b_tws1 + b_twp + b_rate + b_trig + b_mxa) : nullptr;
    const size_t o_gmx = b_band + b_tws1 + b_twp + b_rate + b_trig + b_mxa + b_mxc;
    d.gmx_a = n_gmxa ? reinterpret_cast<const float*>(tb + o_gmx) : nullptr;
    d.gmx_g = n_gmxg ? reinterpret_cast<const float*>(tb + o_gmx + b_gmxa) : nullptr;
    d.bandtab_t = reinterpret_cast<const float2*>(tb + o_gmx + b_gmxa + b_gmxg);
    e = hipMemcpy(tb, band.data(), n_band * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + b_band, tws1.data(), n_tws1 * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + b_band + b_tws1, twp.data(), n_twp * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + b_band + b_tws1 + b_twp, rate.data(), (size_t)Qpad * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(tb + b_band + b_tws1 + b_twp + b_rate, trig.data(), n_trig * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(tb + b_band + b_tws1 + b_twp + b_rate + b_trig, mxa.data(), n_mxa * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_mxc)
        e = hipMemcpy(tb + b_band + b_tws1 + b_twp + b_rate + b_trig + b_mxa, mxc.data(), n_mxc * 8,
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && n_gmxa) e = hipMemcpy(tb + o_gmx, gmxa.data(), n_gmxa * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && n_gmxg) e = hipMemcpy(tb + o_gmx + b_gmxa, gmxg.data(), n_gmxg * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(tb + o_gmx + b_gmxa + b_gmxg, bandt.data(), n_band * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) { sft_plan_destroy(pl); return hip_fail(e, "hipMemcpy(tables)"); }
    e = hipMalloc(&pl->ddesc, sizeof(SigDesc));
    if (e != hipSuccess) { sft_plan_destroy(pl); return fail(SFT_ENOMEM, "hipMalloc(descriptor) failed"); }
    e = hipMemcpy(pl->ddesc, &d, sizeof(SigDesc), hipMemcpyHostToDevice);
    if (e != hipSuccess) { sft_plan_destroy(pl); return hip_fail(e, "hipMemcpy(descriptor)"); }

    // ---- the workspace of sft_execute is allocated by the plan's first sft_execute
    pl->wl = workspace_layout(info);
    if (pl->blocks[SFT_KERNEL_DFT_COLS_MX]) {   // the column kernel's histograms for the selection
        pl->wl.SH = ((size_t)d.K * d.Q * kSelBins * 4 + 255) & ~(size_t)255;
        pl->wl.total += pl->wl.SH;
    }
    pl->footprint = tbytes + sizeof(SigDesc);
    *out = pl;
    return SFT_OK;
}

int sft_plan_workspace_bytes(const sft_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return fail(SFT_EINVAL, "NULL argument");
    *bytes = plan->wl.total;
    return SFT_OK;
}

int sft_plan_get_info(const sft_plan_t plan, sft_plan_info* out) {
    if (!plan || !out) return fail(SFT_EINVAL, "NULL argument");
    *out = plan->info;
    return SFT_OK;
}

int sft_plan_footprint(const sft_plan_t plan, size_t* bytes) {
    if (!plan || !bytes) return fail(SFT_EINVAL, "NULL argument");
    *bytes = plan->footprint;
    return SFT_OK;
}

}  // extern "C"

// ------------------------------------------------------------ profiling ----
namespace {
struct Profiler {
    std::mutex mu;
    bool on = false;
    struct Pending { int kernel; hipEvent_t a, b; };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    int64_t launches[SFT_KERNEL_COUNT] = {};
    double total_ms[SFT_KERNEL_COUNT] = {};

    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    void drain() {
        for (auto& p : pending) {
            (void)hipEventSynchronize(p.b);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                launches[p.kernel] += 1;
                total_ms[p.kernel] += ms;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
};
Profiler g_prof;

template <class F>
hipError_t timed(int kernel, hipStream_t st, F&& launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        on = g_prof.on;
    }
    if (!on) return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        a = g_prof.get();
        b = g_prof.get();
    }
    (void)hipEventRecord(a, st);
    hipError_t e = launch();
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({kernel, a, b});
    if (g_prof.pending.size() > 4096) g_prof.drain();
    return e;
}

using LaunchFn = hipError_t (*)(const BatchArgs&, int, size_t, hipStream_t);

// For the gather kernel the lds argument carries the common tap count (0 = mixed).
hipError_t launch_gather_l(const BatchArgs& a, int b, size_t taps, hipStream_t st) {
    return launch_gather(a, b, (int)taps, st);
}
hipError_t launch_merge_l(const BatchArgs& a, int b, size_t lds, hipStream_t st) { return launch_merge(a, b, lds, st); }

// Launch order of the pipeline and the launcher of each kernel id.
const int kOrder[SFT_KERNEL_COUNT] = {SFT_KERNEL_GATHER,   SFT_KERNEL_GATHER_MX,   SFT_KERNEL_DFT_MX,
                                      SFT_KERNEL_DFT,      SFT_KERNEL_DFT_ROWS,    SFT_KERNEL_DFT_COLS,
                                      SFT_KERNEL_DFT_COLS_MX, SFT_KERNEL_SELECT,   SFT_KERNEL_IDENTIFY,
                                      SFT_KERNEL_MERGE};
const char* kNames[SFT_KERNEL_COUNT] = {"launch(gather)",   "launch(dft)",      "launch(identify)",
                                        "launch(merge)",    "launch(dft_rows)", "launch(dft_cols)",
                                        "launch(select)",   "launch(dft_mx)",   "launch(dft_cols_mx)",
                                        "launch(gather_mx)"};

LaunchFn launcher(int k) {
    switch (k) {
        case SFT_KERNEL_GATHER: return launch_gather_l;
        case SFT_KERNEL_DFT: return launch_dft;
        case SFT_KERNEL_IDENTIFY: return launch_identify;
        case SFT_KERNEL_MERGE: return launch_merge_l;
        case SFT_KERNEL_DFT_ROWS: return launch_dft_rows;
        case SFT_KERNEL_DFT_COLS: return launch_dft_cols;
        case SFT_KERNEL_DFT_MX: return launch_dft_mx;
        case SFT_KERNEL_DFT_COLS_MX: return launch_dft_cols_mx;
        case SFT_KERNEL_GATHER_MX: return launch_gather_mx;
        default: return launch_select;
    }
}

// Enqueue the pipeline.  prefix[k] is the device prefix table of kernel k
// (batch of several plans), bps[k] the blocks per transform of a one-plan
// batch; both null for a single transform.
// timing: per-kernel HIP events when profiling is on (off while a graph is
// captured).
// mxs: the plan's split of the matrix-core short DFTs (single transforms and
// one-plan batches; null for a batch of several plans, whose block prefix
// covers every modulus).
int enqueue(BatchArgs a, const int blocks[SFT_KERNEL_COUNT], const size_t lds[SFT_KERNEL_COUNT],
            const int32_t* const prefix[SFT_KERNEL_COUNT], hipStream_t st, const int* bps, const MxSplit* mxs,
            bool timing = true) {
    for (int o = 0; o < SFT_KERNEL_COUNT; ++o) {
        const int k = kOrder[o];
        if (blocks[k] <= 0) continue;
        a.prefix = prefix ? prefix[k] : nullptr;
        a.bps = bps ? bps[k] : 0;
        LaunchFn fn = launcher(k);
        auto launch = [&]() -> hipError_t {
            if (k != SFT_KERNEL_DFT_MX || !mxs || mxs->j1 <= 0 || prefix || blocks[k] < mxs->min_blocks)
                return fn(a, blocks[k], lds[k], st);
            // moduli [0, j1) with the smaller LDS allocation, then [j1, K)
            const int per = mxs->K * mxs->qb;
            const int count = blocks[k] / per;
            BatchArgs b = a;
            b.jlo = 0;
            b.jn = mxs->j1;
            b.bps = bps ? mxs->j1 * mxs->qb : 0;
            hipError_t e = fn(b, count * mxs->j1 * mxs->qb, mxs->lds_lo, st);
            if (e != hipSuccess) return e;
            b.jlo = mxs->j1;
            b.jn = mxs->K - mxs->j1;
            b.bps = bps ? (mxs->K - mxs->j1) * mxs->qb : 0;
            return fn(b, count * (mxs->K - mxs->j1) * mxs->qb, lds[k], st);
        };
        const hipError_t e = timing ? timed(k, st, launch) : launch();
        if (e != hipSuccess) return hip_fail(e, kNames[k]);
    }
    return SFT_OK;
}

// ------------------------------------------------------------ batches ----
// A batch of transforms: every transform's workspace slice, the launch
// parameters merged over the plans, and the descriptor tables
// ([count] descriptor pointers | [count] IoDesc | one [count+1] block prefix
// per kernel).
struct BatchShape {
    std::vector<size_t> wsoff;
    size_t ws_total = 0;
    size_t lds[SFT_KERNEL_COUNT] = {};
    bool used[SFT_KERNEL_COUNT] = {};   // some plan of the batch launches kernel k
    size_t m_desc = 0, m_io = 0, m_pre = 0, m_status = 0, meta_total = 0;
    bool one_plan = true;
};

// The kernels read f as 8-byte complex values (16-byte pieces where the
// address allows) and write 8-byte frequencies and coefficients.
int check_alignment(const void* f, const void* w, const void* c, const void* n) {
    if (((uintptr_t)f & 7) != 0) return fail(SFT_EINVAL, "f must be 8-byte aligned (complex64)");
    if (((uintptr_t)w & 7) != 0) return fail(SFT_EINVAL, "out_freqs must be 8-byte aligned (int64)");
    if (((uintptr_t)c & 7) != 0) return fail(SFT_EINVAL, "out_coeffs must be 8-byte aligned (complex64)");
    if (((uintptr_t)n & 3) != 0) return fail(SFT_EINVAL, "out_count must be 4-byte aligned (int32)");
    return SFT_OK;
}

int batch_shape(const sft_plan_t* plans, int32_t count, const void* const* f_dev, int64_t* const* out_freqs_dev,
                void* const* out_coeffs_dev, int dev, BatchShape& B) {
    if (!plans || !f_dev || !out_freqs_dev || !out_coeffs_dev) return fail(SFT_EINVAL, "NULL argument");
    B.wsoff.assign(count, 0);
    for (int i = 0; i < count; ++i) {
        const sft_plan_s* p = plans[i];
        if (!p || !f_dev[i] || !out_freqs_dev[i] || !out_coeffs_dev[i]) return fail(SFT_EINVAL, "NULL entry");
        if (const int rc = check_alignment(f_dev[i], out_freqs_dev[i], out_coeffs_dev[i], nullptr)) return rc;
        if (p->device != dev) return fail(SFT_EINVAL, "plan belongs to another device");
        B.one_plan &= p == plans[0];
        B.wsoff[i] = B.ws_total;
        B.ws_total += p->wl.total;
        for (int k = 0; k < SFT_KERNEL_COUNT; ++k)
            if (k != SFT_KERNEL_GATHER) {   // field-wise maximum of (pairs << 32 | bytes); identify's flags: union;
                                            // the selection's LDS-key bytes: 0 if any plan has 0; the
                                            // matrix-core gather: largest M-tile count, any wide window
                if (p->blocks[k] == 0) continue;   // the plan does not use kernel k
                const size_t ph = p->lds[k] >> 32, bh = B.lds[k] >> 32;
                const size_t hi = k == SFT_KERNEL_IDENTIFY ? (ph | bh)
                                  : k == SFT_KERNEL_SELECT ? (!B.used[k] ? ph : (ph && bh ? std::max(ph, bh) : 0))
                                  : k == SFT_KERNEL_GATHER_MX ? (std::max(ph & 0xff, bh & 0xff) | ((ph | bh) & 0x100))
                                                           : std::max(ph, bh);
                B.used[k] = true;
                const size_t lo = std::max(p->lds[k] & 0xffffffffu, B.lds[k] & 0xffffffffu);
                B.lds[k] = (hi << 32) | lo;
            }
        // one compile-time tap count when every transform of the vector-ALU
        // gather shares it, else the generic kernel
        if (p->blocks[SFT_KERNEL_GATHER] > 0) {
            if (!B.used[SFT_KERNEL_GATHER]) B.lds[SFT_KERNEL_GATHER] = p->lds[SFT_KERNEL_GATHER];
            else if (B.lds[SFT_KERNEL_GATHER] != p->lds[SFT_KERNEL_GATHER]) B.lds[SFT_KERNEL_GATHER] = 0;
            B.used[SFT_KERNEL_GATHER] = true;
        }
    }
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    B.m_desc = al(sizeof(void*) * count);
    B.m_io = al(sizeof(IoDesc) * count);
    B.m_pre = al(sizeof(int32_t) * (count + 1));
    B.m_status = al(sizeof(int32_t) * count);
    B.meta_total = B.m_desc + B.m_io + SFT_KERNEL_COUNT * B.m_pre + B.m_status;
    return SFT_OK;
}

// Offset of the per-transform status words (int32[count]) in the descriptor tables.
size_t status_offset(const BatchShape& B) { return B.m_desc + B.m_io + SFT_KERNEL_COUNT * B.m_pre; }

// The host image of the descriptor tables (hs, meta_total bytes) that will
// sit at dm on the device, for the workspace at ws; blocks receives the grid
// size of every kernel.  Each transform's status word is the count-long array
// at status_offset(B) of the tables (zero in the image), not its workspace slice.
void batch_tables(const BatchShape& B, const sft_plan_t* plans, int32_t count, const void* const* f_dev,
                  int64_t* const* out_freqs_dev, void* const* out_coeffs_dev, int32_t* out_counts_dev, char* ws,
                  char* dm, char* hs, int blocks[SFT_KERNEL_COUNT]) {
    memset(hs + status_offset(B), 0, sizeof(int32_t) * (size_t)count);
    const SigDesc** hdesc = reinterpret_cast<const SigDesc**>(hs);
    IoDesc* hio = reinterpret_cast<IoDesc*>(hs + B.m_desc);
    int32_t* hpre[SFT_KERNEL_COUNT];
    for (int k = 0; k < SFT_KERNEL_COUNT; ++k) {
        hpre[k] = reinterpret_cast<int32_t*>(hs + B.m_desc + B.m_io + k * B.m_pre);
        blocks[k] = 0;
    }
    for (int i = 0; i < count; ++i) {
        const sft_plan_s* p = plans[i];
        hdesc[i] = p->ddesc;
        IoDesc io = carve(ws + B.wsoff[i], p->wl);
        io.f = static_cast<const float2*>(f_dev[i]);
        io.out_w = out_freqs_dev[i];
        io.out_c = static_cast<float2*>(out_coeffs_dev[i]);
        io.out_n = out_counts_dev ? out_counts_dev + i : nullptr;
        io.status = reinterpret_cast<int32_t*>(dm + status_offset(B)) + i;
        hio[i] = io;
        for (int k = 0; k < SFT_KERNEL_COUNT; ++k) {
            hpre[k][i] = blocks[k];
            blocks[k] += p->blocks[k];
        }
    }
    for (int k = 0; k < SFT_KERNEL_COUNT; ++k) hpre[k][count] = blocks[k];
}

// Enqueue a batch whose descriptor tables are on the device at dm.
int enqueue_batch(const BatchShape& B, const sft_plan_t* plans, int32_t count, char* dm,
                  const int blocks[SFT_KERNEL_COUNT], hipStream_t st, bool timing) {
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.io_many = reinterpret_cast<const IoDesc*>(dm + B.m_desc);
    a.nsig = count;
    if (B.one_plan) {   // blocks follow from blockIdx by a division; one descriptor
        a.desc_one = plans[0]->ddesc;
        return enqueue(a, blocks, B.lds, nullptr, st, plans[0]->blocks, &plans[0]->mxs, timing);
    }
    a.descs_many = reinterpret_cast<const SigDesc* const*>(dm);
    const int32_t* dpre[SFT_KERNEL_COUNT];
    for (int k = 0; k < SFT_KERNEL_COUNT; ++k)
        dpre[k] = reinterpret_cast<const int32_t*>(dm + B.m_desc + B.m_io + k * B.m_pre);
    return enqueue(a, blocks, B.lds, dpre, st, nullptr, nullptr, timing);
}

// ----------------------------------------------------- batch arenas ----
// One per (device, stream): the workspace of every transform of an
// sft_execute_many call plus its descriptor tables.  Calls on one stream are
// ordered, so the arena is reused; it grows (after a stream synchronisation)
// when a larger batch arrives.
struct Arena {
    void* ws = nullptr;
    size_t ws_bytes = 0;
    void* meta = nullptr;
    size_t meta_bytes = 0;
    void* staging = nullptr;     // pinned host copy of meta
    hipEvent_t staged = nullptr; // the last upload from staging has been consumed
    int32_t last_count = 0;      // transforms of the last call on this stream
    char* last_status = nullptr; // their status words (device)
};
std::mutex g_arena_mu;
std::map<std::pair<int, void*>, Arena*> g_arenas;

Arena* arena_for(int dev, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    auto key = std::make_pair(dev, (void*)st);
    auto it = g_arenas.find(key);
    if (it != g_arenas.end()) return it->second;
    Arena* a = new Arena();
    g_arenas[key] = a;
    return a;
}

Arena* arena_find(int dev, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_arena_mu);
    auto it = g_arenas.find(std::make_pair(dev, (void*)st));
    return it == g_arenas.end() ? nullptr : it->second;
}

Arena* arena_take(int dev, hipStream_t st) {   // removed from the map; the caller frees it
    std::lock_guard<std::mutex> lk(g_arena_mu);
    auto it = g_arenas.find(std::make_pair(dev, (void*)st));
    if (it == g_arenas.end()) return nullptr;
    Arena* a = it->second;
    g_arenas.erase(it);
    return a;
}

// Descriptor-table bytes of a batch of count transforms (as batch_shape lays them out).
size_t meta_bytes_for(int32_t count) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(sizeof(void*) * count) + al(sizeof(IoDesc) * count) + SFT_KERNEL_COUNT * al(sizeof(int32_t) * (count + 1)) +
           al(sizeof(int32_t) * count);
}

// Grow the arena to hold ws_total workspace bytes and meta_total table bytes
// (after the stream has drained, since its buffers are replaced); no-op when
// it already does.  Waits until the previous upload from the staging buffer
// has been consumed.
int arena_fit(Arena* ar, hipStream_t st, size_t ws_total, size_t meta_total) {
    if (ar->staged) HIP_TRY(hipEventSynchronize(ar->staged), "hipEventSynchronize");
    if (ar->ws_bytes >= ws_total && ar->meta_bytes >= meta_total && ar->staged) return SFT_OK;
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (ar->ws_bytes < ws_total) {
        if (ar->ws) (void)hipFree(ar->ws);
        ar->ws = nullptr;
        ar->ws_bytes = 0;
        if (hipMalloc(&ar->ws, ws_total) != hipSuccess) return fail(SFT_ENOMEM, "hipMalloc(batch workspace) failed");
        ar->ws_bytes = ws_total;
    }
    if (ar->meta_bytes < meta_total) {
        if (ar->meta) (void)hipFree(ar->meta);
        if (ar->staging) (void)hipHostFree(ar->staging);
        ar->meta = nullptr;
        ar->staging = nullptr;
        ar->meta_bytes = 0;
        ar->last_status = nullptr;
        if (hipMalloc(&ar->meta, meta_total) != hipSuccess) return fail(SFT_ENOMEM, "hipMalloc(batch meta) failed");
        if (hipHostMalloc(&ar->staging, meta_total, hipHostMallocDefault) != hipSuccess)
            return fail(SFT_ENOMEM, "hipHostMalloc(batch staging) failed");
        ar->meta_bytes = meta_total;
    }
    if (!ar->staged) HIP_TRY(hipEventCreateWithFlags(&ar->staged, hipEventDisableTiming), "hipEventCreate");
    return SFT_OK;
}
}  // namespace

extern "C" {

int sft_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return SFT_OK;
}

int sft_profile_reset(void) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.drain();
    for (int k = 0; k < SFT_KERNEL_COUNT; ++k) {
        g_prof.launches[k] = 0;
        g_prof.total_ms[k] = 0.0;
    }
    return SFT_OK;
}

int sft_profile_read(int32_t kernel, int64_t* launches, double* total_ms) {
    if (kernel < 0 || kernel >= SFT_KERNEL_COUNT) return fail(SFT_EINVAL, "unknown kernel id");
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.drain();
    if (launches) *launches = g_prof.launches[kernel];
    if (total_ms) *total_ms = g_prof.total_ms[kernel];
    return SFT_OK;
}

int sft_execute(sft_plan_t plan, const void* f_dev, int64_t* out_freqs_dev, void* out_coeffs_dev,
                int32_t* out_count_dev, void* stream) {
    if (!plan || !f_dev || !out_freqs_dev || !out_coeffs_dev) return fail(SFT_EINVAL, "NULL argument");
    if (const int rc = check_alignment(f_dev, out_freqs_dev, out_coeffs_dev, out_count_dev)) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (!plan->ws) {   // the plan's first transform: its workspace
        if (hipMalloc(&plan->ws, plan->wl.total) != hipSuccess) {
            plan->ws = nullptr;
            return fail(SFT_ENOMEM, "hipMalloc(workspace) failed");
        }
        plan->ws_io = carve(plan->ws, plan->wl);
        plan->footprint += plan->wl.total;
    }
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.desc_one = plan->ddesc;
    a.io_one = plan->ws_io;
    a.io_one.f = static_cast<const float2*>(f_dev);
    a.io_one.out_w = out_freqs_dev;
    a.io_one.out_c = static_cast<float2*>(out_coeffs_dev);
    a.io_one.out_n = out_count_dev;
    a.nsig = 1;
    plan->last_stream = st;
    plan->last_status = plan->ws_io.status;
    return enqueue(a, plan->blocks, plan->lds, nullptr, st, nullptr, &plan->mxs);
}

int sft_execute_noalloc(sft_plan_t plan, const void* f_dev, int64_t* out_freqs_dev, void* out_coeffs_dev,
                        int32_t* out_count_dev, void* stream) {
    if (!plan || !f_dev || !out_freqs_dev || !out_coeffs_dev) return fail(SFT_EINVAL, "NULL argument");
    if (const int rc = check_alignment(f_dev, out_freqs_dev, out_coeffs_dev, out_count_dev)) return rc;
    if (plan->wl.total > sft::kScratchBytes)
        return fail(SFT_EINVAL, "the plan's workspace (" + std::to_string(plan->wl.total) +
                                    " bytes) exceeds the no-alloc scratch (" + std::to_string(sft::kScratchBytes) +
                                    " bytes); use sft_execute");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev != plan->device) return fail(SFT_EINVAL, "the plan was created on another device");
    void* ws = nullptr;
    HIP_TRY(sft::scratch_address(dev, &ws), "hipGetSymbolAddress(scratch)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.desc_one = plan->ddesc;
    a.io_one = carve(ws, plan->wl);   // the status word is cleared by the first kernel, nothing else is read first
    a.io_one.f = static_cast<const float2*>(f_dev);
    a.io_one.out_w = out_freqs_dev;
    a.io_one.out_c = static_cast<float2*>(out_coeffs_dev);
    a.io_one.out_n = out_count_dev;
    a.nsig = 1;
    plan->last_stream = st;
    plan->last_status = a.io_one.status;
    // no per-kernel timing events: creating them may allocate
    return enqueue(a, plan->blocks, plan->lds, nullptr, st, nullptr, &plan->mxs, false);
}

int sft_execute_many(const sft_plan_t* plans, int32_t count, const void* const* f_dev,
                     int64_t* const* out_freqs_dev, void* const* out_coeffs_dev, int32_t* out_counts_dev,
                     void* stream) {
    if (count < 0) return fail(SFT_EINVAL, "count must be >= 0");
    if (count == 0) return SFT_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    BatchShape B;
    const int rc = batch_shape(plans, count, f_dev, out_freqs_dev, out_coeffs_dev, dev, B);
    if (rc != SFT_OK) return rc;

    Arena* ar = arena_for(dev, st);
    if (const int rc2 = arena_fit(ar, st, B.ws_total, B.meta_total)) return rc2;
    int blocks[SFT_KERNEL_COUNT];
    batch_tables(B, plans, count, f_dev, out_freqs_dev, out_coeffs_dev, out_counts_dev, static_cast<char*>(ar->ws),
                 static_cast<char*>(ar->meta), static_cast<char*>(ar->staging), blocks);
    HIP_TRY(hipMemcpyAsync(ar->meta, ar->staging, B.meta_total, hipMemcpyHostToDevice, st), "hipMemcpyAsync(meta)");
    HIP_TRY(hipEventRecord(ar->staged, st), "hipEventRecord");
    ar->last_count = count;
    ar->last_status = static_cast<char*>(ar->meta) + status_offset(B);
    return enqueue_batch(B, plans, count, static_cast<char*>(ar->meta), blocks, st, true);
}

int sft_execute_many_status(void* stream, int32_t count, int32_t* flags) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    Arena* ar = arena_find(dev, st);
    if (!ar || !ar->last_status) return fail(SFT_EINVAL, "no sft_execute_many has run on this stream");
    if (count != ar->last_count) return fail(SFT_EINVAL, "count differs from the last sft_execute_many on this stream");
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    std::vector<int32_t> v((size_t)count);
    HIP_TRY(hipMemcpy(v.data(), ar->last_status, sizeof(int32_t) * (size_t)count, hipMemcpyDeviceToHost),
            "hipMemcpy(status)");
    bool any = false;
    for (int i = 0; i < count; ++i) {
        if (flags) flags[i] = v[i];
        any |= v[i] != 0;
    }
    if (any) return fail(SFT_EOVERFLOW, "a device-side capacity was exceeded in some transform of the batch");
    return SFT_OK;
}

int sft_execute_many_reserve(void* stream, size_t workspace_bytes, int32_t count) {
    if (count < 0) return fail(SFT_EINVAL, "count must be >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    return arena_fit(arena_for(dev, st), st, workspace_bytes, meta_bytes_for(count));
}

int sft_execute_many_release(void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    Arena* ar = arena_take(dev, st);
    if (!ar) return SFT_OK;
    HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (ar->ws) (void)hipFree(ar->ws);
    if (ar->meta) (void)hipFree(ar->meta);
    if (ar->staging) (void)hipHostFree(ar->staging);
    if (ar->staged) (void)hipEventDestroy(ar->staged);
    delete ar;
    return SFT_OK;
}

// --------------------------------------------------- prepared batches ----
struct sft_batch_s {
    int32_t count = 0;
    std::vector<sft_plan_t> plans;
    BatchShape shape;
    int blocks[SFT_KERNEL_COUNT] = {};
    void* ws = nullptr;
    void* meta = nullptr;
    hipStream_t capture = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;   // stream of the last launch
};

void sft_batch_destroy(sft_batch_t b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->last);   // its memory is freed below
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->meta) (void)hipFree(b->meta);
    if (b->ws) (void)hipFree(b->ws);
    delete b;
}

int sft_batch_create(sft_batch_t* out, const sft_plan_t* plans, int32_t count, const void* const* f_dev,
                     int64_t* const* out_freqs_dev, void* const* out_coeffs_dev, int32_t* out_counts_dev) {
    if (!out) return fail(SFT_EINVAL, "NULL argument");
    *out = nullptr;
    if (count < 1) return fail(SFT_EINVAL, "count must be >= 1");
    if (!plans) return fail(SFT_EINVAL, "NULL argument");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    sft_batch_s* b = new sft_batch_s();
    b->count = count;
    b->plans.assign(plans, plans + count);
    int rc = batch_shape(plans, count, f_dev, out_freqs_dev, out_coeffs_dev, dev, b->shape);
    if (rc != SFT_OK) { sft_batch_destroy(b); return rc; }
    if (hipMalloc(&b->ws, b->shape.ws_total) != hipSuccess || hipMalloc(&b->meta, b->shape.meta_total) != hipSuccess) {
        sft_batch_destroy(b);
        return fail(SFT_ENOMEM, "hipMalloc(batch) failed");
    }
    std::vector<char> hs(b->shape.meta_total, 0);
    batch_tables(b->shape, plans, count, f_dev, out_freqs_dev, out_coeffs_dev, out_counts_dev,
                 static_cast<char*>(b->ws), static_cast<char*>(b->meta), hs.data(), b->blocks);
    const hipError_t e = hipMemcpy(b->meta, hs.data(), b->shape.meta_total, hipMemcpyHostToDevice);
    if (e != hipSuccess) { sft_batch_destroy(b); return hip_fail(e, "hipMemcpy(batch tables)"); }
    *out = b;
    return SFT_OK;
}

int sft_batch_launch(sft_batch_t b, void* stream) {
    if (!b) return fail(SFT_EINVAL, "NULL batch");
    b->last = static_cast<hipStream_t>(stream);
    return enqueue_batch(b->shape, b->plans.data(), b->count, static_cast<char*>(b->meta), b->blocks,
                         static_cast<hipStream_t>(stream), true);
}

int sft_batch_graph_launch(sft_batch_t b, void* stream) {
    if (!b) return fail(SFT_EINVAL, "NULL batch");
    if (!b->exec) {   // capture the launch sequence once, on a stream of the batch's own
        if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "hipStreamCreate");
        HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        const int rc = enqueue_batch(b->shape, b->plans.data(), b->count, static_cast<char*>(b->meta), b->blocks,
                                     b->capture, false);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture, &g);
        if (rc != SFT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    b->last = static_cast<hipStream_t>(stream);
    HIP_TRY(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)), "hipGraphLaunch");
    return SFT_OK;
}

int sft_batch_status(sft_batch_t b, int32_t* flags) {
    if (!b) return fail(SFT_EINVAL, "NULL batch");
    HIP_TRY(hipStreamSynchronize(b->last), "hipStreamSynchronize");
    std::vector<int32_t> v((size_t)b->count);
    HIP_TRY(hipMemcpy(v.data(), static_cast<char*>(b->meta) + status_offset(b->shape), sizeof(int32_t) * v.size(),
                      hipMemcpyDeviceToHost), "hipMemcpy(status)");
    bool any = false;
    for (int i = 0; i < b->count; ++i) {
        if (flags) flags[i] = v[i];
        any |= v[i] != 0;
    }
    if (any) return fail(SFT_EOVERFLOW, "a device-side capacity was exceeded in some transform of the batch");
    return SFT_OK;
}

int sft_plan_status(sft_plan_t plan, int32_t* flags) {
    if (!plan) return fail(SFT_EINVAL, "NULL plan");
    if (!plan->last_status) return fail(SFT_EINVAL, "the plan has not run sft_execute");
    HIP_TRY(hipStreamSynchronize(plan->last_stream), "hipStreamSynchronize");
    int32_t v = 0;
    HIP_TRY(hipMemcpy(&v, plan->last_status, 4, hipMemcpyDeviceToHost), "hipMemcpy(status)");
    if (flags) *flags = v;
    if (v != 0) return fail(SFT_EOVERFLOW, "a device-side capacity was exceeded");
    return SFT_OK;
}

int sft_plan_fetch(const sft_plan_t plan, int32_t what, void* dst, size_t bytes, size_t* bytes_needed) {
    if (!plan) return fail(SFT_EINVAL, "NULL plan");
    if (!plan->ws) return fail(SFT_EINVAL, "the plan has not run sft_execute");
    const sft_plan_info& in = plan->info;
    const void* src = nullptr;
    size_t need = 0;
    switch (what) {
        case SFT_FETCH_SAMPLES: src = plan->ws_io.S; need = (size_t)in.Q * in.M * 8; break;
        case SFT_FETCH_BINS: src = plan->ws_io.E; need = (size_t)in.Q * in.M * 8; break;
        case SFT_FETCH_HEAVY: src = plan->ws_io.H; need = (size_t)in.K * in.Q * in.T * 4; break;
        case SFT_FETCH_BANDS: need = (size_t)in.Q * 4 + (size_t)in.Q * in.s * 24; break;
        case SFT_FETCH_SAMPLES_SHIFTED:
        case SFT_FETCH_BINS_SHIFTED:
            if (in.ident != SFT_IDENT_PHASE) return fail(SFT_EINVAL, "shifted samples exist for phase identification only");
            src = what == SFT_FETCH_SAMPLES_SHIFTED ? plan->ws_io.S2 : plan->ws_io.E2;
            need = (size_t)in.Q * in.M * 8;
            break;
        case SFT_FETCH_CLASSES: src = plan->ws_io.CL; need = (size_t)in.K * in.Q * in.s1 * in.depth * 4; break;
        default: return fail(SFT_EINVAL, "unknown fetch kind");
    }
    if (bytes_needed) *bytes_needed = need;
    if (!dst) return SFT_OK;
    if (bytes < need) return fail(SFT_EINVAL, "destination too small");
    HIP_TRY(hipStreamSynchronize(plan->last_stream), "hipStreamSynchronize");
    if (what != SFT_FETCH_BANDS) {
        HIP_TRY(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost), "hipMemcpy(fetch)");
        if (what == SFT_FETCH_HEAVY) {
            // the device writes each block's heavy bins in any order: sort them
            // by Good-Thomas position (h mod s1) + s1 (h mod p_j)
            int32_t* H = static_cast<int32_t*>(dst);
            const int64_t s1 = in.s1;
            for (int j = 0; j < in.K; ++j) {
                const int64_t pj = in.primes[j];
                for (int b = 0; b < in.Q; ++b) {
                    int32_t* blk = H + ((size_t)j * in.Q + b) * in.T;
                    std::sort(blk, blk + in.T, [&](int32_t x, int32_t y) {
                        return x % s1 + s1 * (x % pj) < y % s1 + s1 * (y % pj);
                    });
                }
            }
        }
        return SFT_OK;
    }
    // counts[Q], then Q*s records {int64 w; double re; double im}, band b's at b*s
    char* o = static_cast<char*>(dst);
    HIP_TRY(hipMemcpy(o, plan->ws_io.Rn, (size_t)in.Q * 4, hipMemcpyDeviceToHost), "hipMemcpy(fetch)");
    std::vector<int64_t> w((size_t)in.Q * in.s);
    std::vector<double2> v((size_t)in.Q * in.s);
    HIP_TRY(hipMemcpy(w.data(), plan->ws_io.Rw, w.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy(fetch)");
    HIP_TRY(hipMemcpy(v.data(), plan->ws_io.Rv, v.size() * 16, hipMemcpyDeviceToHost), "hipMemcpy(fetch)");
    char* rec = o + (size_t)in.Q * 4;
    for (size_t i = 0; i < w.size(); ++i) {
        memcpy(rec + i * 24, &w[i], 8);
        memcpy(rec + i * 24 + 8, &v[i].x, 8);
        memcpy(rec + i * 24 + 16, &v[i].y, 8);
    }
    return SFT_OK;
}

const char* sft_last_error(void) { return g_err.c_str(); }

}  // extern "C"
