// Host runtime of libscs: contexts, device buffers, launch sequencing,
// profiling, tuning, swarms.  Implements the C ABI declared in include/scs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <sstream>
#include <string>
#include <limits>
#include <vector>

#include "../../include/scs.h"
#include "scs_internal.hpp"
#include "scs_math.hpp"

using namespace scs;

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(SCS_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- device setup
static std::mutex g_dev_mu;
static std::map<int, bool> g_dev_ready;


// Chebyshev nodes x_n = cos(pi (2n+1) / (2 kNodes)) and the inverse of the
// Vandermonde matrix V[n][m] = x_n^m (computed in extended precision).
static void cheb_matrix(double* x, double* minv)
{
    long double X[kNodes], V[kNodes][2 * kNodes];
    for (int n = 0; n < kNodes; ++n) {
        X[n] = cosl(3.141592653589793238462643383279502884L * (2 * n + 1) / (2.0L * kNodes));
        x[n] = (double)X[n];
        long double v = 1.0L;
        for (int m = 0; m < kNodes; ++m) {
            V[n][m] = v;
            v *= X[n];
            V[n][kNodes + m] = (n == m) ? 1.0L : 0.0L;
        }
    }
    for (int c = 0; c < kNodes; ++c) {
        int piv = c;
        for (int r = c + 1; r < kNodes; ++r)
            if (fabsl(V[r][c]) > fabsl(V[piv][c])) piv = r;
        for (int k = 0; k < 2 * kNodes; ++k) std::swap(V[c][k], V[piv][k]);
        const long double d = V[c][c];
        for (int k = 0; k < 2 * kNodes; ++k) V[c][k] /= d;
        for (int r = 0; r < kNodes; ++r)
            if (r != c) {
                const long double f = V[r][c];
                for (int k = 0; k < 2 * kNodes; ++k) V[r][k] -= f * V[c][k];
            }
    }
    // V^-1 maps node values to monomial coefficients: coef_m = sum_n Vinv[m][n] val_n
    for (int m = 0; m < kNodes; ++m)
        for (int n = 0; n < kNodes; ++n) minv[m * kNodes + n] = (double)V[m][kNodes + n];
}

// ---------------------------------------------------------------- scratch
// Device memory of scs_evaluate_noalloc: a static array every GPU the library
// runs on holds until the process ends.  Its name is a host-side stand-in in
// host code; the device address of each GPU's copy is taken once, at that
// device's set-up, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[SCS_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 256;
static void* g_scratch[kMaxDevices] = {nullptr};  // written under g_dev_mu before the device is marked ready

static int device_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (device >= 0 && device < kMaxDevices && g_dev_ready[device]) return SCS_OK;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(SCS_EDEVICE, "no HIP device");
    if (device < 0 || device >= count) return fail(SCS_EDEVICE, "device %d out of range (%d devices)", device, count);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SCS_EDEVICE, "device %d is %s; libscs is built for gfx950", device, prop.gcnArchName);
    HIP_TRY(hipSetDevice(device));
    double x[kNodes], m[kNodes * kNodes];
    cheb_matrix(x, m);
    HIP_TRY(upload_cheb(x, m));
    std::vector<double> trig(2 * kTrig);
    for (int i = 0; i < kTrig; ++i) {
        const long double a = 2.0L * 3.141592653589793238462643383279502884L * i / kTrig;
        trig[2 * i] = (double)cosl(a);
        trig[2 * i + 1] = (double)sinl(a);
    }
    HIP_TRY(upload_trig(trig.data()));
    if (device >= kMaxDevices) return fail(SCS_EDEVICE, "device %d: at most %d devices", device, kMaxDevices);
    void* sp = nullptr;
    const hipError_t e = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !sp)
        return fail(SCS_EDEVICE, "device %d: address of the no-allocation scratch: %s", device, hipGetErrorString(e));
    g_scratch[device] = sp;
    g_dev_ready[device] = true;
    return SCS_OK;
}


static PhysConst phys_const()
{
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double c = 299792458.0L;
    const long double tsun = 1.32712440018e20L / (c * c * c);
    const long double pt = pi * tsun;
    const long double k3 = 3.0L / (256.0L * pi);
    PhysConst pc;
    pc.pitsun_hi = (double)pt;
    pc.pitsun_lo = (double)(pt - (long double)pc.pitsun_hi);
    pc.k3_hi = (double)k3;
    pc.k3_lo = (double)(k3 - (long double)pc.k3_hi);
    return pc;
}

// ---------------------------------------------------------------- context
struct Workspace {
    int64_t capP = 0;
    int64_t capBounds = 0;  // int32 entries
    int64_t capRec = 0;     // doubles
    int64_t capZs = 0;      // doubles
    double* coef = nullptr;
    int32_t* klo = nullptr;
    int32_t* khi = nullptr;
    int8_t* lg = nullptr;
    int32_t* bounds = nullptr;
    double* rec = nullptr;
    double* zs = nullptr;  // [P][N][3] per-segment sums (when the caller asks for no segment output)
    int64_t capSpl = 0;     // doubles
    double* spl = nullptr;  // sparse-grid template: node records [capP][nmax][spl_rec]
    // host-pointer staging
    int64_t capStage = 0;
    double* stage = nullptr;
    int64_t P_last = 0;
    int N_last = 0;
    // support-order permutation (counting sort of (k_hi, k_lo) buckets)
    int64_t capSort = 0;
    int32_t* bucket = nullptr;  // [P]
    int32_t* rank = nullptr;    // [P]
    int32_t* perm = nullptr;    // [P]
    unsigned* hist = nullptr;   // [kSortBuckets]
};

// Device descriptors of one fused batched launch: the MainArgs of every
// item, the per-item first tile, the work counter; and the pinned host copy
// they are uploaded from.  A ring of these lets eager batched calls overlap
// without overwriting descriptors a queued launch still reads.
struct BatchSlot {
    int cap = 0;  // items
    MainArgs* d_items = nullptr;
    int64_t* d_start = nullptr;                // [kVariants][cap + 1]
    unsigned long long* d_counter = nullptr;  // [kVariants]
    MainArgs* h_items = nullptr;               // pinned
    int64_t* h_start = nullptr;                // pinned
    hipEvent_t done = nullptr;                 // recorded after the last launch that read the slot
};

// Launch shape of the generate-and-reduce: waves per workgroup (64 particle
// slots each), LDS-staged blocks per chunk, bins per LDS block, and the
// occupancy instantiation (alt: two waves per SIMD for FP64, four for mixed).
struct TuneChoice {
    int waves = 4;
    int CB = 16;
    int L = 512;
    int alt = 0;
};

struct scs_ctx {
    int device = 0;
    bool has_data = false, has_model = false;
    GridArgs g{};
    ModelArgs m{};
    int L = 512;
    int lg_max = 9;
    int N = 1, mode = SCS_SEG_EQUAL_SNR;
    int64_t G = 1024;
    int64_t* d_edges = nullptr;
    int64_t edges_cap = 0;
    double* b64 = nullptr;
    float* b32 = nullptr;
    double* d_dev = nullptr;    // the loaded data [nch][K][2] and PSD [nch][K], kept for the
    double* psd_dev = nullptr;  // fixed-theta streams
    double zscale32 = 1.0, hscale32 = 1.0;  // undo the FP32 table scaling
    double dd = 0.0;                        // <d|d> of the loaded data
    double* gtab = nullptr;  // basis Taylor tables, every sub-block level
    int64_t gtab_cap = 0;
    int64_t gtab_off[kMaxLevel] = {0};
    bool gtab_ok = false;
    unsigned long long* counters = nullptr;  // evals_support, evals_band, unresolved
    std::map<int, Workspace> ws;             // slot -> workspace
    uint64_t gen = 0;  // bumped by every change of data, model or segmentation (graphs built earlier go stale)
    hipStream_t last_stream = nullptr;
    // profiling of the generate-and-reduce kernel
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    int64_t prof_launches = 0;
    double prof_ms = 0.0;
    // tuning
    std::map<std::string, TuneChoice> tune;
    TuneChoice override_choice;
    bool has_override = false;
    // fused batched launches whose first item is this context
    int n_cu = 0;
    static constexpr int kRing = 4;
    BatchSlot ring[kRing];
    int ring_next = 0;
    // side streams (default priority) on which a batch's per-item kernels
    // before and after the fused launch run side by side, forked from and
    // joined back to the caller's stream by events (null: one stream)
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[kSide] = {};
};

static int build_gtab(scs_ctx* c);
static void free_slot(BatchSlot& b);

// Channels each response model produces: none one, low-frequency A and E,
// full A and E, or A, E and T.
static bool model_fits(int response, int nch)
{
    if (response == SCS_RESP_NONE) return nch == 1;
    if (response == SCS_RESP_LISA_LF_AE) return nch == 2;
    if (response == SCS_RESP_LISA_FD_AE) return nch == 2 || nch == 3;
    return false;
}

// Entries per theta row: 7, or 8 with the eccentricity of an eccentric model.
static int theta_dim(const scs_ctx* c) { return c->m.ecc ? kThetaMax : kTheta; }

struct DevScope {
    int prev = -1;
    explicit DevScope(int d)
    {
        hipGetDevice(&prev);
        if (prev != d) hipSetDevice(d);
    }
    ~DevScope()
    {
        int cur = -1;
        hipGetDevice(&cur);
        if (prev >= 0 && cur != prev) hipSetDevice(prev);
    }
};

template <class T>
static int grow(T** p, int64_t* cap, int64_t need)
{
    if (need <= *cap) return SCS_OK;
    if (*p) hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (need <= 0) return SCS_OK;
    if (hipMalloc((void**)p, sizeof(T) * (size_t)need) != hipSuccess) {
        *p = nullptr;
        return fail(SCS_ENOMEM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * need));
    }
    *cap = need;
    return SCS_OK;
}

static void free_ws(Workspace& w)
{
    hipFree(w.coef);
    hipFree(w.klo);
    hipFree(w.khi);
    hipFree(w.lg);
    hipFree(w.bounds);
    hipFree(w.rec);
    hipFree(w.zs);
    hipFree(w.spl);
    hipFree(w.stage);
    hipFree(w.bucket);
    hipFree(w.rank);
    hipFree(w.perm);
    hipFree(w.hist);
    w = Workspace();
}

// Error record for the library's other translation units (the search driver).
int scs_record_error(int code, const char* msg) { return fail(code, "%s", msg); }

extern "C" const char* scs_last_error(void) { return g_last_error.c_str(); }

extern "C" int scs_ctx_create(scs_ctx** out, int device)
{
    if (!out) return fail(SCS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = device_setup(device);
    if (rc) return rc;
    DevScope ds(device);
    scs_ctx* c = new (std::nothrow) scs_ctx();
    if (!c) return fail(SCS_ENOMEM, "host allocation failed");
    c->device = device;
    if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || c->n_cu < 1)
        c->n_cu = 256;
    if (hipMalloc((void**)&c->counters, 3 * sizeof(unsigned long long)) != hipSuccess) {
        delete c;
        return fail(SCS_ENOMEM, "counter allocation failed");
    }
    launch_fill_u64(c->counters, 3, 0ULL, nullptr);
    bool side_ok = hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; i < scs_ctx::kSide && side_ok; ++i)
        side_ok = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&c->join_ev[i], hipEventDisableTiming) == hipSuccess;
    if (!side_ok) {  // the batched form then stays on the caller's stream
        for (int i = 0; i < scs_ctx::kSide; ++i) {
            if (c->side[i]) hipStreamDestroy(c->side[i]);
            if (c->join_ev[i]) hipEventDestroy(c->join_ev[i]);
            c->side[i] = nullptr;
            c->join_ev[i] = nullptr;
        }
        if (c->fork_ev) hipEventDestroy(c->fork_ev);
        c->fork_ev = nullptr;
        (void)hipGetLastError();
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        hipFree(c->counters);
        delete c;
        return fail(SCS_EDEVICE, "device synchronisation failed");
    }
    *out = c;
    return SCS_OK;
}

extern "C" int scs_ctx_destroy(scs_ctx* c)
{
    if (!c) return SCS_OK;
    DevScope ds(c->device);
    hipDeviceSynchronize();
    for (auto& kv : c->ws) free_ws(kv.second);
    for (auto& b : c->ring) free_slot(b);
    for (auto& e : c->ev) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    for (int i = 0; i < scs_ctx::kSide; ++i) {
        if (c->side[i]) hipStreamDestroy(c->side[i]);
        if (c->join_ev[i]) hipEventDestroy(c->join_ev[i]);
    }
    if (c->fork_ev) hipEventDestroy(c->fork_ev);
    hipFree(c->b64);
    hipFree(c->b32);
    hipFree(c->d_dev);
    hipFree(c->psd_dev);
    hipFree(c->gtab);
    hipFree(c->d_edges);
    hipFree(c->counters);
    delete c;
    return SCS_OK;
}

extern "C" int scs_load_data(scs_ctx* c, int32_t n_chan, int64_t K, double f_min, double df, const double* d_ri,
                             const double* psd, int32_t mem_kind)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (n_chan < 1 || n_chan > 3) return fail(SCS_EINVAL, "n_chan must be 1, 2 or 3 (got %d)", n_chan);
    if (K < 1 || K > (int64_t)1 << 30) return fail(SCS_EINVAL, "K out of range (%lld)", (long long)K);
    if (!(df > 0.0) || !std::isfinite(df) || !(f_min >= 0.0) || !std::isfinite(f_min))
        return fail(SCS_EINVAL, "f_min and df must be finite, df > 0");
    const double k0 = std::round(f_min / df);
    if (std::fabs(k0 * df - f_min) > 1e-9 * std::max(f_min, df)) return fail(SCS_EINVAL, "f_min / df is not an integer");
    if (!d_ri || !psd) return fail(SCS_EINVAL, "data or psd is NULL");
    if (mem_kind != SCS_MEM_HOST && mem_kind != SCS_MEM_DEVICE) return fail(SCS_EINVAL, "bad mem_kind");
    DevScope ds(c->device);
    const int64_t nd = (int64_t)n_chan * K;
    std::vector<double> hp;
    if (mem_kind == SCS_MEM_HOST) {
        for (int64_t i = 0; i < nd; ++i)
            if (!(psd[i] > 0.0) || !std::isfinite(psd[i])) return fail(SCS_EINVAL, "psd[%lld] is not finite and > 0", (long long)i);
        for (int64_t i = 0; i < 2 * nd; ++i)
            if (!std::isfinite(d_ri[i])) return fail(SCS_EINVAL, "data[%lld] is not finite", (long long)i);
    } else {
        hp.resize(nd);
        HIP_TRY(hipMemcpy(hp.data(), psd, sizeof(double) * nd, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < nd; ++i)
            if (!(hp[i] > 0.0) || !std::isfinite(hp[i])) return fail(SCS_EINVAL, "psd[%lld] is not finite and > 0", (long long)i);
    }
    double *dd_ = nullptr, *dp = nullptr;
    if (hipMalloc((void**)&dd_, sizeof(double) * 2 * nd) != hipSuccess) return fail(SCS_ENOMEM, "data allocation failed");
    if (hipMalloc((void**)&dp, sizeof(double) * nd) != hipSuccess) {
        hipFree(dd_);
        return fail(SCS_ENOMEM, "psd allocation failed");
    }
    const hipMemcpyKind kind = mem_kind == SCS_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    hipError_t e1 = hipMemcpy(dd_, d_ri, sizeof(double) * 2 * nd, kind);
    hipError_t e2 = hipMemcpy(dp, psd, sizeof(double) * nd, kind);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        hipFree(dd_);
        hipFree(dp);
        return fail(SCS_EDEVICE, "copy of data failed");
    }
    hipFree(c->b64);
    hipFree(c->b32);
    c->b64 = nullptr;
    c->b32 = nullptr;
    if (hipMalloc((void**)&c->b64, sizeof(double) * bin_stride(n_chan) * K) != hipSuccess ||
        hipMalloc((void**)&c->b32, sizeof(float) * bin_stride(n_chan) * K) != hipSuccess) {
        hipFree(dd_);
        hipFree(dp);
        return fail(SCS_ENOMEM, "bin table allocation failed");
    }
    c->g.K = K;
    c->g.k0 = k0;
    c->g.df = df;
    c->g.nch = n_chan;
    // FP32 scale s = 1 / median of q = f^-7/3 / S over 65 sampled bins and the channels
    {
        if (hp.empty()) hp.assign(psd, psd + nd);
        std::vector<double> qs;
        for (int ch = 0; ch < n_chan; ++ch)
            for (int i = 0; i <= 64; ++i) {
                const int64_t k = (K - 1) * i / 64;
                const double f = (k0 + (double)k) * df;
                qs.push_back(std::pow(f, -7.0 / 3.0) / hp[(int64_t)ch * K + k]);
            }
        std::nth_element(qs.begin(), qs.begin() + qs.size() / 2, qs.end());
        double sq = qs[qs.size() / 2];
        sq = (sq > 0.0 && std::isfinite(sq)) ? 1.0 / sq : 1.0;
        sq = std::exp2(std::round(std::log2(sq)));  // a power of two: exact in both directions
        const double su = std::sqrt(sq);
        c->zscale32 = 1.0 / su;
        c->hscale32 = 1.0 / sq;
        launch_bins(c->g, dd_, dp, c->b64, c->b32, su, sq, nullptr);
    }
    // <d|d>: workgroup partials, then their fixed-order total, in the tail of
    // the bin table (overwritten by nothing until the next load)
    double* nrm = nullptr;
    if (hipMalloc((void**)&nrm, sizeof(double) * (kNormBlocks + 1)) != hipSuccess) {
        hipFree(dd_);
        hipFree(dp);
        return fail(SCS_ENOMEM, "norm scratch allocation failed");
    }
    launch_data_norm(c->g, dd_, dp, nrm, nrm + kNormBlocks, nullptr);
    hipError_t e3 = hipDeviceSynchronize();
    if (e3 == hipSuccess) e3 = hipMemcpy(&c->dd, nrm + kNormBlocks, sizeof(double), hipMemcpyDeviceToHost);
    hipFree(nrm);
    hipFree(c->d_dev);
    hipFree(c->psd_dev);
    c->d_dev = dd_;
    c->psd_dev = dp;
    if (e3 != hipSuccess) return fail(SCS_EDEVICE, "bin precompute failed: %s", hipGetErrorString(e3));
    c->has_data = true;
    ++c->gen;
    c->gtab_ok = false;
    if (c->has_model && !model_fits(c->m.response, n_chan)) c->has_model = false;
    if (c->has_model) return build_gtab(c);
    return SCS_OK;
}

extern "C" int scs_set_model(scs_ctx* c, const scs_model* m)
{
    if (!c || !m) return fail(SCS_EINVAL, "NULL argument");
    if (!c->has_data) return fail(SCS_ESTATE, "load data before setting the model");
    if (m->pn_order < 0 || m->pn_order > 7) return fail(SCS_EINVAL, "pn_order must be 0..7");
    if (m->response != SCS_RESP_NONE && m->response != SCS_RESP_LISA_LF_AE && m->response != SCS_RESP_LISA_FD_AE)
        return fail(SCS_EINVAL, "bad response");
    if (!model_fits(m->response, c->g.nch))
        return fail(SCS_EINVAL, "response %d does not match %d loaded channels", m->response, c->g.nch);
    if (m->support != SCS_SUPPORT_FULL && m->support != SCS_SUPPORT_TOBS) return fail(SCS_EINVAL, "bad support");
    const int bl = m->block_len ? m->block_len : 2048;
    if (bl < 16 || bl > 2048 || (bl & (bl - 1))) return fail(SCS_EINVAL, "block_len must be a power of 2 in 16..2048");
    if (m->t_obs < 0.0 || !std::isfinite(m->t_obs)) return fail(SCS_EINVAL, "bad t_obs");
    if (m->eccentric != 0 && m->eccentric != 1) return fail(SCS_EINVAL, "eccentric must be 0 or 1");
    if (m->sparse_stride < 0 || m->sparse_stride > kMaxSparseStride)
        return fail(SCS_EINVAL, "sparse_stride must be 0 (template per bin) or 1..%d", kMaxSparseStride);
    c->m.pn_order = m->pn_order;
    c->m.response = m->response;
    c->m.support = m->support;
    c->m.t_obs = m->t_obs > 0.0 ? m->t_obs : 1.0 / c->g.df;
    double oc = m->orbit_phase0 / (2.0 * M_PI);
    c->m.orb0_cyc = oc - std::floor(oc);
    c->m.cart0 = m->cartwheel_phase0;
    c->m.cart_c = std::cos(m->cartwheel_phase0);
    c->m.cart_s = std::sin(m->cartwheel_phase0);
    c->m.ecc = m->eccentric;
    c->m.sparse = m->sparse_stride;
    c->L = 512;  // bins per LDS-staged block of the generate-and-reduce kernel
    int lg = 0;
    while ((1 << lg) < bl) ++lg;
    c->lg_max = lg;
    c->has_model = true;
    ++c->gen;
    DevScope ds(c->device);
    return build_gtab(c);
}

extern "C" int scs_define_segmentation(scs_ctx* c, int32_t N, int32_t mode, int32_t G, const int64_t* edges)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (N < 1 || N > SCS_MAX_SEGMENTS) return fail(SCS_EINVAL, "N must be in 1..%d (got %d)", SCS_MAX_SEGMENTS, N);
    if (G < 1) return fail(SCS_EINVAL, "G must be >= 1");
    if (mode < 0 || mode > 2) return fail(SCS_EINVAL, "bad segmentation mode");
    if (mode == SCS_SEG_EXPLICIT) {
        if (!edges) return fail(SCS_EINVAL, "EXPLICIT mode needs edges");
        for (int n = 0; n < N; ++n)
            if (edges[n + 1] < edges[n]) return fail(SCS_EINVAL, "edges not monotone at %d", n);
        DevScope ds(c->device);
        int rc = grow(&c->d_edges, &c->edges_cap, (int64_t)N + 1);
        if (rc) return rc;
        HIP_TRY(hipMemcpy(c->d_edges, edges, sizeof(int64_t) * (N + 1), hipMemcpyHostToDevice));
    }
    c->N = N;
    ++c->gen;
    c->mode = mode;
    c->G = G;
    return SCS_OK;
}

// ---------------------------------------------------------------- tiling
static std::string tune_key(const scs_ctx* c, int64_t P, int N, int prec)
{
    auto cls = [](int64_t v) {
        int b = 0;
        while ((int64_t)1 << (b + 1) <= v) ++b;
        return b;
    };
    std::ostringstream o;
    o << "K" << c->g.K << "_c" << c->g.nch << "_r" << c->m.response << "_s" << c->m.sparse << "_p" << prec << "_P"
      << cls(P) << "_N" << cls(N);
    return o.str();
}

// ==== launch shape of the generate-and-reduce (begin)
static TuneChoice default_choice(const scs_ctx* c, int64_t P);
static TuneChoice choose(const scs_ctx* c, int64_t P, int N, int prec)
{
    if (c->has_override) return c->override_choice;
    auto it = c->tune.find(tune_key(c, P, N, prec));
    if (it != c->tune.end()) return it->second;
    return default_choice(c, P);
}

static TuneChoice default_choice(const scs_ctx* c, int64_t P)
{
    TuneChoice t;
    // default: 4 waves (256 particles) per workgroup, fewer when the swarm is
    // small so that the chip still fills; chunks as short as the longest
    // polynomial block (2^lg_max bins, at least one staged block): a tile
    // then lasts a fraction of a millisecond, so the persistent grid drains
    // evenly (with 8192-bin chunks the last tiles ran ~15% of the launch
    // alone), and no block straddles two chunks
    t.waves = P >= 4096 ? 4 : (P >= 1024 ? 2 : 1);
    t.L = c->L;
    t.CB = std::max(1, (1 << c->lg_max) / t.L);
    t.alt = 0;
    return t;
}

struct Plan {
    int waves, CB, L, alt;
    int64_t cbins, n_chunks, n_groups, n_tiles;
};

static Plan make_plan(const scs_ctx* c, int64_t P, const TuneChoice& t)
{
    Plan pl;
    pl.waves = t.waves;
    pl.CB = t.CB;
    pl.L = t.L;
    pl.alt = t.alt;
    pl.cbins = (int64_t)t.L * t.CB;
    pl.n_chunks = (c->g.K + pl.cbins - 1) / pl.cbins;
    pl.n_groups = (P + 64 * t.waves - 1) / (64 * t.waves);
    pl.n_tiles = pl.n_chunks * pl.n_groups;
    return pl;
}

// ==== launch shape of the generate-and-reduce (end)

static int64_t pad64(int64_t v) { return (v + 63) / 64 * 64; }

// Swarms of at least this many particles are evaluated in support order.
static constexpr int64_t kSortMin = 128;

// Node records of the sparse-grid template for Pp particle slots (0 when the
// template is evaluated per bin).
static int64_t spl_doubles(const scs_ctx* c, int64_t Pp)
{
    if (c->m.sparse <= 0) return 0;
    return Pp * spl_max_nodes(c->g.K, c->m.sparse) * spl_rec(c->g.nch);
}

static size_t ws_bytes(const scs_ctx* c, int64_t P, int N, const Plan& pl)
{
    const int64_t Pp = pad64(std::max<int64_t>(P, 1));
    size_t b = 0;
    b += sizeof(double) * (size_t)kCoefStride * Pp;
    b += (sizeof(int32_t) * 2 + 1) * (size_t)Pp;
    b += sizeof(int32_t) * ((size_t)P * (N + 1) + 2);
    b += sizeof(double) * (size_t)pl.n_chunks * kRec * Pp;
    b += sizeof(double) * 3 * (size_t)P * N;
    b += sizeof(double) * (size_t)spl_doubles(c, Pp);
    return b;
}

static int ensure_ws(scs_ctx* c, Workspace& w, int64_t P, int N, const Plan& pl)
{
    const int64_t Pp = pad64(std::max<int64_t>(P, 1));
    int rc;
    if (Pp > w.capP) {
        hipFree(w.coef);
        hipFree(w.klo);
        hipFree(w.khi);
        hipFree(w.lg);
        w.coef = nullptr;
        w.klo = w.khi = nullptr;
        w.lg = nullptr;
        if (hipMalloc((void**)&w.coef, sizeof(double) * kCoefStride * Pp) != hipSuccess ||
            hipMalloc((void**)&w.klo, sizeof(int32_t) * Pp) != hipSuccess ||
            hipMalloc((void**)&w.khi, sizeof(int32_t) * Pp) != hipSuccess ||
            hipMalloc((void**)&w.lg, Pp) != hipSuccess) {
            w.capP = 0;
            return fail(SCS_ENOMEM, "workspace allocation failed (P = %lld)", (long long)P);
        }
        w.capP = Pp;
    }
    // two spare entries after the last row: the generate-and-reduce kernel
    // reads each particle's edges two ahead without a bounds test
    if ((rc = grow(&w.bounds, &w.capBounds, P * (int64_t)(N + 1) + 2))) return rc;
    if ((rc = grow(&w.rec, &w.capRec, pl.n_chunks * kRec * w.capP))) return rc;
    if ((rc = grow(&w.zs, &w.capZs, 3 * P * (int64_t)N))) return rc;
    if (c->m.sparse > 0 && (rc = grow(&w.spl, &w.capSpl, spl_doubles(c, w.capP)))) return rc;
    if (P >= kSortMin && P > w.capSort) {
        int64_t c1 = 0, c2 = 0, c3 = 0, c4 = 0;
        hipFree(w.bucket);
        hipFree(w.rank);
        hipFree(w.perm);
        hipFree(w.hist);
        w.bucket = w.rank = w.perm = nullptr;
        w.hist = nullptr;
        w.capSort = 0;
        if ((rc = grow(&w.bucket, &c1, w.capP)) || (rc = grow(&w.rank, &c2, w.capP)) ||
            (rc = grow(&w.perm, &c3, w.capP)) || (rc = grow(&w.hist, &c4, (int64_t)kSortBuckets)))
            return rc;
        w.capSort = w.capP;
    }
    return SCS_OK;
}

// One evaluation, queued in stages: front (prologue, support sort, edges),
// the generate-and-reduce (solo or inside a fused batched launch), back
// (finalize).  Device pointers throughout.
struct EvalJob {
    scs_ctx* c = nullptr;
    Workspace* w = nullptr;
    int64_t P = 0;
    int N = 1;
    Plan pl{};
    MainArgs ma{};
    FinalArgs fa{};
};

static int eval_front(EvalJob& j, const double* theta, double* ups, double* seg, const TuneChoice& t, hipStream_t s,
                      double* stats = nullptr, bool fixed_ws = false, const int32_t* frozen = nullptr)
{
    scs_ctx* c = j.c;
    Workspace& w = *j.w;
    const int64_t P = j.P;
    const int N = j.N;
    if (c->mode == SCS_SEG_EXPLICIT && N != c->N) return fail(SCS_EINVAL, "EXPLICIT edges were defined for N = %d", c->N);
    j.pl = make_plan(c, P, t);
    // a fixed workspace was laid out by the caller for exactly this P, N and
    // plan (the evaluation without allocations); anything else grows to fit
    int rc = fixed_ws ? SCS_OK : ensure_ws(c, w, P, N, j.pl);
    if (rc) return rc;
    w.P_last = P;
    w.N_last = N;
    if (P == 0) return SCS_OK;
    PrologueArgs pa{};
    pa.g = c->g;
    pa.m = c->m;
    pa.c = phys_const();
    pa.P = P;
    pa.stride = w.capP;
    pa.theta = theta;
    pa.coef = w.coef;
    pa.klo = w.klo;
    pa.khi = w.khi;
    pa.lg = w.lg;
    pa.lg_max = c->lg_max;
    pa.evals = c->counters;
    pa.unresolved = c->counters + 2;
    pa.frozen = frozen;
    launch_prologue(pa, s);
    const int64_t spl_nmax = c->m.sparse > 0 ? spl_max_nodes(c->g.K, c->m.sparse) : 0;
    if (c->m.sparse > 0) {
        SplineArgs sa{};
        sa.g = c->g;
        sa.m = c->m;
        sa.P = P;
        sa.stride = w.capP;
        sa.coef = w.coef;
        sa.klo = w.klo;
        sa.khi = w.khi;
        sa.lg = w.lg;
        sa.nmax = spl_nmax;
        sa.spl = w.spl;
        launch_spline(sa, s);
    }
    const int32_t* perm = nullptr;
    if (P >= kSortMin && w.perm) {
        launch_sort_perm(P, c->g.K, w.klo, w.khi, w.hist, w.bucket, w.rank, w.perm, s);
        perm = w.perm;
    }
    BoundArgs ba{};
    ba.g = c->g;
    ba.m = c->m;
    ba.P = P;
    ba.stride = w.capP;
    ba.N = N;
    ba.mode = c->mode;
    ba.G = c->G;
    ba.coef = w.coef;
    ba.klo = w.klo;
    ba.khi = w.khi;
    ba.lg = w.lg;
    ba.b64 = c->b64;
    ba.edges = c->d_edges;
    ba.bounds = w.bounds;
    // node weights kept in LDS between the two passes of the equal-[h|h]
    // edges: every node of the widest support (K bins), up to 4096 (32 KiB)
    ba.wcache = (int)std::min<int64_t>((c->g.K - 1) / std::max<int64_t>(c->G, 1) + 2, 4096);
    launch_bounds(ba, s);
    MainArgs& ma = j.ma;
    ma = MainArgs{};
    ma.g = c->g;
    ma.m = c->m;
    ma.p0 = 0;
    ma.P_end = P;
    ma.stride = w.capP;
    ma.N = N;
    ma.L = j.pl.L;
    ma.CB = j.pl.CB;
    ma.chunk0 = 0;
    ma.n_groups = j.pl.n_groups;
    ma.n_tiles = j.pl.n_tiles;
    ma.rec_stride = w.capP;
    ma.coef = w.coef;
    ma.klo = w.klo;
    ma.khi = w.khi;
    ma.lg = w.lg;
    ma.bounds = w.bounds;
    ma.b64 = c->b64;
    ma.b32 = c->b32;
    ma.gtab = c->gtab;
    for (int l = 0; l < kMaxLevel; ++l) ma.gtab_off[l] = c->gtab_off[l];
    ma.lg_max = c->lg_max;
    ma.perm = perm;
    ma.rec = w.rec;
    ma.zs = seg ? seg : w.zs;
    ma.zscale32 = c->zscale32;
    ma.hscale32 = c->hscale32;
    ma.spl = c->m.sparse > 0 ? w.spl : nullptr;
    ma.spl_nmax = spl_nmax;
    FinalArgs& fa = j.fa;
    fa = FinalArgs{};
    fa.K = c->g.K;
    fa.df = c->g.df;
    fa.p0 = 0;
    fa.P_end = P;
    fa.N = N;
    fa.cbins = j.pl.cbins;
    fa.chunk0 = 0;
    fa.rec_stride = w.capP;
    fa.klo = w.klo;
    fa.khi = w.khi;
    fa.lg = w.lg;
    fa.bounds = w.bounds;
    fa.perm = perm;
    fa.rec = w.rec;
    fa.zs = seg ? seg : w.zs;
    fa.ups = ups;
    fa.seg = seg;
    fa.stats = stats;
    return SCS_OK;
}

// Launch timing (scs_ctx_profile): an event before and after each main launch.
// Timing is best effort: if an event cannot be created or recorded, that
// launch is left out of the profile and the evaluation goes on.
static void prof_begin(scs_ctx* c, hipStream_t s, hipEvent_t* e0)
{
    *e0 = nullptr;
    if (!c->prof) return;
    if (hipEventCreate(e0) != hipSuccess) {
        *e0 = nullptr;
        return;
    }
    if (hipEventRecord(*e0, s) != hipSuccess) {
        hipEventDestroy(*e0);
        *e0 = nullptr;
    }
}
static void prof_end(scs_ctx* c, hipStream_t s, hipEvent_t e0)
{
    if (!c->prof || !e0) return;
    hipEvent_t e1 = nullptr;
    if (hipEventCreate(&e1) != hipSuccess || hipEventRecord(e1, s) != hipSuccess) {
        if (e1) hipEventDestroy(e1);
        hipEventDestroy(e0);
        return;
    }
    c->ev.emplace_back(e0, e1);
}

static int eval_main(scs_ctx* c, EvalJob& j, int prec, hipStream_t s);

// Queue the whole evaluation on stream s (device pointers).
static int run_eval(scs_ctx* c, Workspace& w, int64_t P, int N, const double* theta, int prec, double* ups,
                    double* seg, hipStream_t s, const TuneChoice* force = nullptr, double* stats = nullptr)
{
    EvalJob j;
    j.c = c;
    j.w = &w;
    j.P = P;
    j.N = N;
    const TuneChoice t = force ? *force : choose(c, P, N, prec);
    int rc = eval_front(j, theta, ups, seg, t, s, stats);
    if (rc || P == 0) return rc;
    if ((rc = eval_main(c, j, prec, s))) return rc;
    launch_finalize(j.fa, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    c->last_stream = s;
    return SCS_OK;
}

// Basis tables for sub-block lengths 2^3 .. 2^lg_max over the loaded grid.
static int build_gtab(scs_ctx* c)
{
    int64_t off = 0;
    for (int lg = 0; lg < kMaxLevel; ++lg) {
        c->gtab_off[lg] = off;
        if (lg >= 3 && lg <= c->lg_max) off += (c->g.K + ((int64_t)1 << lg) - 1) >> lg;
    }
    int rc = grow(&c->gtab, &c->gtab_cap, off * kGStride);
    if (rc) return rc;
    for (int lg = 3; lg <= c->lg_max; ++lg) {
        const int64_t nsub = (c->g.K + ((int64_t)1 << lg) - 1) >> lg;
        launch_gtab(c->g, lg, nsub, c->gtab + c->gtab_off[lg] * kGStride, nullptr);
    }
    HIP_TRY(hipDeviceSynchronize());
    c->gtab_ok = true;
    return SCS_OK;
}

static int check_ready(const scs_ctx* c)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (!c->has_data) return fail(SCS_ESTATE, "no data loaded");
    if (!c->has_model) return fail(SCS_ESTATE, "no model set");
    return SCS_OK;
}

extern "C" int scs_evaluate(scs_ctx* c, int64_t P, const double* theta, int32_t prec, double* ups, double* seg,
                            int32_t mem_kind, void* stream)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 0) return fail(SCS_EINVAL, "P < 0");
    if (P > 0 && (!theta || !ups)) return fail(SCS_EINVAL, "theta or ups is NULL");
    if (prec != SCS_PREC_FP64 && prec != SCS_PREC_MIXED) return fail(SCS_EINVAL, "bad precision");
    if (mem_kind != SCS_MEM_HOST && mem_kind != SCS_MEM_DEVICE) return fail(SCS_EINVAL, "bad mem_kind");
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = c->ws[0];
    const int N = c->N;
    if (mem_kind == SCS_MEM_DEVICE) return run_eval(c, w, P, N, theta, prec, ups, seg, s);
    // host pointers: stage through device memory
    const int td = theta_dim(c);
    const int64_t need = P * td + P + (seg ? P * (int64_t)N * 3 : 0);
    if ((rc = grow(&w.stage, &w.capStage, std::max<int64_t>(need, 1)))) return rc;
    double* dth = w.stage;
    double* dup = dth + P * td;
    double* dseg = seg ? dup + P : nullptr;
    HIP_TRY(hipMemcpyAsync(dth, theta, sizeof(double) * td * P, hipMemcpyHostToDevice, s));
    if ((rc = run_eval(c, w, P, N, dth, prec, dup, dseg, s))) return rc;
    HIP_TRY(hipMemcpyAsync(ups, dup, sizeof(double) * P, hipMemcpyDeviceToHost, s));
    if (seg) HIP_TRY(hipMemcpyAsync(seg, dseg, sizeof(double) * P * N * 3, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SCS_OK;
}

// ---------------------------------------------------------------- no allocation
// The one-item launch descriptor, its tile range and the cleared work counter
// written into device memory by a kernel (the descriptor travels as a kernel
// argument), so that the evaluation needs no pinned staging and no memset.
__global__ void k_put_main_args(MainArgs a, MainArgs* d, int64_t* start, int64_t total, unsigned long long* counter)
{
    *d = a;
    start[0] = 0;
    start[1] = total;
    *counter = 0ULL;
}

// Regions of one evaluation inside the scratch (offsets in bytes, each
// 256-byte aligned); total = bytes needed.
struct NoallocLayout {
    size_t coef, klo, khi, lg, bounds, rec, zs, spl, bucket, rank, perm, hist, items, start, counter, total;
};

static NoallocLayout noalloc_layout(const scs_ctx* c, int64_t P, int N, const Plan& pl, bool own_zs)
{
    const uint64_t Pp = (uint64_t)pad64(std::max<int64_t>(P, 1));
    NoallocLayout l{};
    size_t off = 0;
    auto take = [&](size_t& at, uint64_t bytes) {
        at = off;
        off += (size_t)((bytes + 255) / 256 * 256);
    };
    take(l.coef, sizeof(double) * kCoefStride * Pp);
    take(l.klo, sizeof(int32_t) * Pp);
    take(l.khi, sizeof(int32_t) * Pp);
    take(l.lg, Pp);
    take(l.bounds, sizeof(int32_t) * ((uint64_t)P * (uint64_t)(N + 1) + 2));
    take(l.rec, sizeof(double) * (uint64_t)pl.n_chunks * kRec * Pp);
    take(l.zs, own_zs ? sizeof(double) * 3 * (uint64_t)P * (uint64_t)N : 0);
    take(l.spl, sizeof(double) * (uint64_t)spl_doubles(c, (int64_t)Pp));
    const bool sorted = P >= kSortMin;
    take(l.bucket, sorted ? sizeof(int32_t) * Pp : 0);
    take(l.rank, sorted ? sizeof(int32_t) * Pp : 0);
    take(l.perm, sorted ? sizeof(int32_t) * Pp : 0);
    take(l.hist, sorted ? sizeof(unsigned) * (uint64_t)kSortBuckets : 0);
    take(l.items, sizeof(MainArgs));
    take(l.start, 2 * sizeof(int64_t));
    take(l.counter, sizeof(unsigned long long));
    l.total = off;
    return l;
}

extern "C" int scs_evaluate_noalloc(scs_ctx* c, int64_t P, const double* theta, int32_t prec, double* ups, double* seg,
                                    void* stream)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 0) return fail(SCS_EINVAL, "P < 0");
    if (P > 0 && (!theta || !ups)) return fail(SCS_EINVAL, "theta or ups is NULL");
    if (prec != SCS_PREC_FP64 && prec != SCS_PREC_MIXED) return fail(SCS_EINVAL, "bad precision");
    if (c->device < 0 || c->device >= kMaxDevices || !g_scratch[c->device])
        return fail(SCS_ESTATE, "device %d has no no-allocation scratch", c->device);
    if (P == 0) return SCS_OK;
    const int N = c->N;
    // every particle needs its coefficient record at least: a cheap bound
    // that keeps the layout arithmetic below far from overflow
    if (P > (int64_t)(SCS_NOALLOC_SCRATCH_BYTES / (sizeof(double) * kCoefStride)))
        return fail(SCS_EINVAL, "P = %lld exceeds what the %zu-byte device scratch of scs_evaluate_noalloc holds",
                    (long long)P, (size_t)SCS_NOALLOC_SCRATCH_BYTES);
    // the default launch shape (or the context's forced one); the tuning
    // cache is not consulted, its lookup would allocate host memory
    const TuneChoice t = c->has_override ? c->override_choice : default_choice(c, P);
    const Plan pl = make_plan(c, P, t);
    const NoallocLayout l = noalloc_layout(c, P, N, pl, seg == nullptr);
    if (l.total > (size_t)SCS_NOALLOC_SCRATCH_BYTES)
        return fail(SCS_EINVAL, "P = %lld, N = %d on %lld bins needs %zu bytes of device scratch; "
                    "scs_evaluate_noalloc has %zu", (long long)P, N, (long long)c->g.K, l.total,
                    (size_t)SCS_NOALLOC_SCRATCH_BYTES);
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    unsigned char* base = (unsigned char*)g_scratch[c->device];
    const int64_t Pp = pad64(P);
    Workspace w;  // views into the scratch, freed by no one
    w.capP = Pp;
    w.capBounds = P * (int64_t)(N + 1) + 2;
    w.capRec = pl.n_chunks * kRec * Pp;
    w.capZs = seg ? 0 : 3 * P * (int64_t)N;
    w.coef = (double*)(base + l.coef);
    w.klo = (int32_t*)(base + l.klo);
    w.khi = (int32_t*)(base + l.khi);
    w.lg = (int8_t*)(base + l.lg);
    w.bounds = (int32_t*)(base + l.bounds);
    w.rec = (double*)(base + l.rec);
    w.zs = seg ? nullptr : (double*)(base + l.zs);
    w.capSpl = spl_doubles(c, Pp);
    w.spl = w.capSpl ? (double*)(base + l.spl) : nullptr;
    if (P >= kSortMin) {
        w.capSort = Pp;
        w.bucket = (int32_t*)(base + l.bucket);
        w.rank = (int32_t*)(base + l.rank);
        w.perm = (int32_t*)(base + l.perm);
        w.hist = (unsigned*)(base + l.hist);
    }
    EvalJob j;
    j.c = c;
    j.w = &w;
    j.P = P;
    j.N = N;
    if ((rc = eval_front(j, theta, ups, seg, t, s, nullptr, /*fixed_ws=*/true))) return rc;
    MainArgs* d_items = (MainArgs*)(base + l.items);
    int64_t* d_start = (int64_t*)(base + l.start);
    unsigned long long* d_counter = (unsigned long long*)(base + l.counter);
    hipLaunchKernelGGL(k_put_main_args, dim3(1), dim3(1), 0, s, j.ma, d_items, d_start, j.pl.n_tiles, d_counter);
    const int variant = variant_of(c->m.response, c->g.nch, c->m.sparse);
    const bool mixed = prec == SCS_PREC_MIXED;
    const int per_cu = main_multi_blocks_per_cu(variant, j.pl.L, j.pl.waves, mixed, j.pl.alt != 0);
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(j.pl.n_tiles, (int64_t)c->n_cu * per_cu));
    hipError_t e = launch_main_multi(d_items, d_start, 1, d_counter, variant, j.pl.L, j.pl.waves, mixed,
                                     j.pl.alt != 0, (int)grid, s);
    if (e != hipSuccess) return fail(SCS_EDEVICE, "generate-and-reduce launch failed: %s", hipGetErrorString(e));
    launch_finalize(j.fa, s);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    c->last_stream = s;
    return SCS_OK;
}

extern "C" int scs_evaluate_stats(scs_ctx* c, int64_t P, const double* theta, int32_t prec, double* stats,
                                  int32_t mem_kind, void* stream)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 0) return fail(SCS_EINVAL, "P < 0");
    if (P > 0 && (!theta || !stats)) return fail(SCS_EINVAL, "theta or stats is NULL");
    if (prec != SCS_PREC_FP64 && prec != SCS_PREC_MIXED) return fail(SCS_EINVAL, "bad precision");
    if (mem_kind != SCS_MEM_HOST && mem_kind != SCS_MEM_DEVICE) return fail(SCS_EINVAL, "bad mem_kind");
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = c->ws[0];
    const int N = c->N;
    // staging: theta, Upsilon (also written by the epilogue) and the statistics
    const int td = theta_dim(c);
    const int64_t need = P * (td + 1 + kNStats);
    if ((rc = grow(&w.stage, &w.capStage, std::max<int64_t>(need, 1)))) return rc;
    double* dth = w.stage;
    double* dup = dth + P * td;
    double* dst = dup + P;
    if (mem_kind == SCS_MEM_DEVICE) return run_eval(c, w, P, N, theta, prec, dup, nullptr, s, nullptr, stats);
    HIP_TRY(hipMemcpyAsync(dth, theta, sizeof(double) * td * P, hipMemcpyHostToDevice, s));
    if ((rc = run_eval(c, w, P, N, dth, prec, dup, nullptr, s, nullptr, dst))) return rc;
    HIP_TRY(hipMemcpyAsync(stats, dst, sizeof(double) * kNStats * P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SCS_OK;
}

extern "C" int scs_data_norm(const scs_ctx* c, double* dd)
{
    if (!c || !dd) return fail(SCS_EINVAL, "NULL argument");
    if (!c->has_data) return fail(SCS_ESTATE, "no data loaded");
    *dd = c->dd;
    return SCS_OK;
}

extern "C" int scs_distance_amplitude(scs_ctx* c, int64_t P, const double* theta, const double* dl_mpc, double* amp,
                                      int32_t mem_kind, void* stream)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 0) return fail(SCS_EINVAL, "P < 0");
    if (P > 0 && (!theta || !dl_mpc || !amp)) return fail(SCS_EINVAL, "theta, dl_mpc or amp is NULL");
    if (mem_kind != SCS_MEM_HOST && mem_kind != SCS_MEM_DEVICE) return fail(SCS_EINVAL, "bad mem_kind");
    if (P == 0) return SCS_OK;
    // sqrt(5/24) pi^(-2/3) (G Msun / c^3)^(5/6) c / (1 Mpc): the restricted
    // stationary-phase amplitude of the (2,2) mode per Msun^(5/6) at 1 Mpc
    const double gm_sun = 1.32712440018e20, c_light = 299792458.0, mpc = 3.0856775814913673e22;
    const double k = std::sqrt(5.0 / 24.0) * std::pow(M_PI, -2.0 / 3.0) *
                     std::pow(gm_sun / (c_light * c_light * c_light), 5.0 / 6.0) * c_light / mpc;
    const int td = theta_dim(c);
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (mem_kind == SCS_MEM_DEVICE) {
        launch_distance_amp(P, td, theta, dl_mpc, k, amp, s);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? SCS_OK : fail(SCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    }
    Workspace& w = c->ws[-2];
    if ((rc = grow(&w.stage, &w.capStage, P * (td + 2)))) return rc;
    double* dth = w.stage;
    double* ddl = dth + P * td;
    double* damp = ddl + P;
    HIP_TRY(hipMemcpyAsync(dth, theta, sizeof(double) * td * P, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(ddl, dl_mpc, sizeof(double) * P, hipMemcpyHostToDevice, s));
    launch_distance_amp(P, td, dth, ddl, k, damp, s);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(amp, damp, sizeof(double) * P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SCS_OK;
}

extern "C" int scs_loglike(scs_ctx* c, int64_t P, const double* stats, const double* amp, const double* phase,
                           double* logl_semi, double* logl_coh, int32_t mem_kind, void* stream)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (!c->has_data) return fail(SCS_ESTATE, "no data loaded");
    if (P < 0) return fail(SCS_EINVAL, "P < 0");
    if (P > 0 && (!stats || !amp)) return fail(SCS_EINVAL, "stats or amp is NULL");
    if (mem_kind != SCS_MEM_HOST && mem_kind != SCS_MEM_DEVICE) return fail(SCS_EINVAL, "bad mem_kind");
    if (P == 0 || (!logl_semi && !logl_coh)) return SCS_OK;
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (mem_kind == SCS_MEM_DEVICE) {
        launch_loglike(P, c->dd, stats, amp, phase, logl_semi, logl_coh, s);
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? SCS_OK : fail(SCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    }
    Workspace& w = c->ws[-2];
    const int64_t need = P * (kNStats + 4);
    int rc = grow(&w.stage, &w.capStage, need);
    if (rc) return rc;
    double* dstat = w.stage;
    double* damp = dstat + P * kNStats;
    double* dph = damp + P;
    double* dsemi = dph + P;
    double* dcoh = dsemi + P;
    HIP_TRY(hipMemcpyAsync(dstat, stats, sizeof(double) * kNStats * P, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(damp, amp, sizeof(double) * P, hipMemcpyHostToDevice, s));
    if (phase) HIP_TRY(hipMemcpyAsync(dph, phase, sizeof(double) * P, hipMemcpyHostToDevice, s));
    launch_loglike(P, c->dd, dstat, damp, phase ? dph : nullptr, logl_semi ? dsemi : nullptr,
                   logl_coh ? dcoh : nullptr, s);
    HIP_TRY(hipGetLastError());
    if (logl_semi) HIP_TRY(hipMemcpyAsync(logl_semi, dsemi, sizeof(double) * P, hipMemcpyDeviceToHost, s));
    if (logl_coh) HIP_TRY(hipMemcpyAsync(logl_coh, dcoh, sizeof(double) * P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SCS_OK;
}

extern "C" int scs_last_bounds(scs_ctx* c, int64_t P, int32_t* support, int32_t* bounds)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    auto it = c->ws.find(0);
    if (it == c->ws.end() || it->second.P_last != P) return fail(SCS_ESTATE, "no evaluation of %lld particles to report", (long long)P);
    Workspace& w = it->second;
    DevScope ds(c->device);
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    if (support) {
        std::vector<int32_t> lo(P), hi(P);
        HIP_TRY(hipMemcpy(lo.data(), w.klo, sizeof(int32_t) * P, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hi.data(), w.khi, sizeof(int32_t) * P, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < P; ++i) {
            support[2 * i] = lo[i];
            support[2 * i + 1] = hi[i];
        }
    }
    if (bounds) HIP_TRY(hipMemcpy(bounds, w.bounds, sizeof(int32_t) * P * (w.N_last + 1), hipMemcpyDeviceToHost));
    return SCS_OK;
}

extern "C" int scs_waveform(scs_ctx* c, const double* theta, double* h_ri, int32_t mem_kind, void* stream)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (!theta || !h_ri) return fail(SCS_EINVAL, "NULL argument");
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = c->ws[-1];
    TuneChoice t;
    const Plan pl = make_plan(c, 1, t);
    if ((rc = ensure_ws(c, w, 1, 1, pl))) return rc;
    const int64_t nout = 2 * (int64_t)c->g.nch * c->g.K;
    const int td = theta_dim(c);
    if ((rc = grow(&w.stage, &w.capStage, td + nout))) return rc;
    const double* dth = theta;
    double* dh = h_ri;
    if (mem_kind == SCS_MEM_HOST) {
        HIP_TRY(hipMemcpyAsync(w.stage, theta, sizeof(double) * td, hipMemcpyHostToDevice, s));
        dth = w.stage;
        dh = w.stage + td;
    }
    PrologueArgs pa{};
    pa.g = c->g;
    pa.m = c->m;
    pa.c = phys_const();
    pa.P = 1;
    pa.stride = w.capP;
    pa.theta = dth;
    pa.coef = w.coef;
    pa.klo = w.klo;
    pa.khi = w.khi;
    pa.lg = w.lg;
    pa.lg_max = c->lg_max;
    pa.evals = c->counters + 1;  // not counted as statistic work
    pa.unresolved = c->counters + 2;
    launch_prologue(pa, s);
    MainArgs ma{};
    ma.g = c->g;
    ma.m = c->m;
    ma.stride = w.capP;
    ma.coef = w.coef;
    ma.klo = w.klo;
    ma.khi = w.khi;
    ma.lg = w.lg;
    ma.gtab = c->gtab;
    for (int l = 0; l < kMaxLevel; ++l) ma.gtab_off[l] = c->gtab_off[l];
    ma.lg_max = c->lg_max;
    if (c->m.sparse > 0) {
        SplineArgs sa{};
        sa.g = c->g;
        sa.m = c->m;
        sa.P = 1;
        sa.stride = w.capP;
        sa.coef = w.coef;
        sa.klo = w.klo;
        sa.khi = w.khi;
        sa.lg = w.lg;
        sa.nmax = spl_max_nodes(c->g.K, c->m.sparse);
        sa.spl = w.spl;
        launch_spline(sa, s);
        ma.spl = w.spl;
        ma.spl_nmax = sa.nmax;
    }
    launch_waveform(ma, dh, s);
    if (mem_kind == SCS_MEM_HOST) {
        HIP_TRY(hipMemcpyAsync(h_ri, dh, sizeof(double) * nout, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "waveform launch failed: %s", hipGetErrorString(e));
    return SCS_OK;
}

// ---------------------------------------------------------------- fixed theta, many data streams (Sec 5.1)
extern "C" int scs_make_realisations(scs_ctx* c, int64_t R, uint64_t seed, int64_t r0, double scale, double* streams,
                                     void* stream)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (!c->has_data) return fail(SCS_ESTATE, "no data loaded");
    if (R < 0 || r0 < 0 || r0 + R > ((int64_t)1 << 32)) return fail(SCS_EINVAL, "realisations [r0, r0 + R) must lie in [0, 2^32)");
    if (R > 0 && !streams) return fail(SCS_EINVAL, "streams is NULL");
    if (!std::isfinite(scale)) return fail(SCS_EINVAL, "scale is not finite");
    DevScope ds(c->device);
    StreamGenArgs a{};
    a.K = c->g.K;
    a.R = R;
    a.r0 = r0;
    a.nch = c->g.nch;
    a.df = c->g.df;
    a.scale = scale;
    a.seed = seed;
    a.d = c->d_dev;
    a.psd = c->psd_dev;
    a.streams = streams;
    launch_make_streams(a, c->n_cu, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SCS_OK : fail(SCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
}

extern "C" int scs_evaluate_streams(scs_ctx* c, const double* theta, int64_t R, const double* streams, double* stats,
                                    void* stream)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (!theta) return fail(SCS_EINVAL, "theta is NULL");
    if (R < 0) return fail(SCS_EINVAL, "R < 0");
    if (R > 0 && (!streams || !stats)) return fail(SCS_EINVAL, "streams or stats is NULL");
    if (R == 0) return SCS_OK;
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    Workspace& w = c->ws[-3];
    const int N = c->N;
    const int nch = c->g.nch;
    const int64_t K = c->g.K;
    // edges of theta with the context's segmentation (one-particle evaluation)
    const int td = theta_dim(c);
    if ((rc = grow(&w.stage, &w.capStage, td + 1))) return rc;
    HIP_TRY(hipMemcpyAsync(w.stage, theta, sizeof(double) * td, hipMemcpyHostToDevice, s));
    const bool prof = c->prof;
    c->prof = false;  // with profiling on, only the streamed reduction below is timed
    rc = run_eval(c, w, 1, N, w.stage, SCS_PREC_FP64, w.stage + td, nullptr, s);
    c->prof = prof;
    if (rc) return rc;
    std::vector<int32_t> bo(N + 1);
    int8_t lg = -1;
    HIP_TRY(hipMemcpyAsync(bo.data(), w.bounds, sizeof(int32_t) * (N + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&lg, w.lg, 1, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (lg < 0) {  // invalid or unresolved theta
        launch_fill(stats, R * kNStats, std::numeric_limits<double>::quiet_NaN(), s);
        HIP_TRY(hipGetLastError());
        return SCS_OK;
    }
    // pieces: every segment cut into runs of at most kPieceBins bins, in order
    std::vector<int32_t> pcs;
    for (int n = 0; n < N; ++n)
        for (int32_t k = bo[n]; k < bo[n + 1]; k += kPieceBins) {
            pcs.push_back(k);
            pcs.push_back(std::min<int32_t>(k + kPieceBins, bo[n + 1]));
            pcs.push_back(n);
        }
    const int64_t np = (int64_t)pcs.size() / 3;
    // stage: template [nch][K][2], weights [nch][K][2], hq [K], hpart [np],
    // zpart [np][R][2], pieces [np][3] int32
    const int64_t off_h = 0, off_w = off_h + 2 * nch * K, off_q = off_w + 2 * nch * K, off_hp = off_q + K;
    const int64_t off_z = off_hp + np, off_p = off_z + 2 * np * R;
    if ((rc = grow(&w.stage, &w.capStage, off_p + (3 * np + 1) / 2 + 1))) return rc;
    double* st = w.stage;
    MainArgs ma{};
    ma.g = c->g;
    ma.m = c->m;
    ma.stride = w.capP;
    ma.coef = w.coef;
    ma.klo = w.klo;
    ma.khi = w.khi;
    ma.lg = w.lg;
    ma.gtab = c->gtab;
    for (int l = 0; l < kMaxLevel; ++l) ma.gtab_off[l] = c->gtab_off[l];
    ma.lg_max = c->lg_max;
    ma.spl = w.spl;  // the sparse-grid template's nodes of theta, from the evaluation above
    ma.spl_nmax = c->m.sparse > 0 ? spl_max_nodes(c->g.K, c->m.sparse) : 0;
    launch_waveform(ma, st + off_h, s);
    launch_stream_weights(nch, K, st + off_h, c->psd_dev, st + off_w, st + off_q, s);
    int32_t* dpcs = reinterpret_cast<int32_t*>(st + off_p);
    if (np > 0) {
        HIP_TRY(hipMemcpyAsync(dpcs, pcs.data(), sizeof(int32_t) * pcs.size(), hipMemcpyHostToDevice, s));
    }
    StreamArgs a{};
    a.K = K;
    a.R = R;
    a.nch = nch;
    a.df = c->g.df;
    a.streams = streams;
    a.wts = st + off_w;
    a.hq = st + off_q;
    a.pieces = dpcs;
    a.n_pieces = np;
    a.zpart = st + off_z;
    a.hpart = st + off_hp;
    a.stats = stats;
    hipEvent_t e0;
    prof_begin(c, s, &e0);
    launch_streams(a, s);
    prof_end(c, s, e0);
    launch_streams_final(a, s);
    HIP_TRY(hipGetLastError());
    // the piece table is read from pageable host memory: finish before it goes
    HIP_TRY(hipStreamSynchronize(s));
    return SCS_OK;
}

extern "C" int scs_ctx_stats(scs_ctx* c, int64_t* evals_support, int64_t* evals_band, int64_t* unresolved, int32_t reset)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    DevScope ds(c->device);
    HIP_TRY(hipDeviceSynchronize());
    unsigned long long h[3];
    HIP_TRY(hipMemcpy(h, c->counters, sizeof h, hipMemcpyDeviceToHost));
    if (evals_support) *evals_support = (int64_t)h[0];
    if (evals_band) *evals_band = (int64_t)h[1];
    if (unresolved) *unresolved = (int64_t)h[2];
    if (reset) {
        launch_fill_u64(c->counters, 3, 0ULL, nullptr);
        HIP_TRY(hipDeviceSynchronize());
    }
    return SCS_OK;
}

extern "C" int scs_ctx_profile(scs_ctx* c, int32_t enable, int64_t* launches, double* total_ms)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    DevScope ds(c->device);
    // every recorded pair is read (until the first failure) and released
    int rc = SCS_OK;
    for (auto& e : c->ev) {
        float ms = 0.f;
        if (rc == SCS_OK && (hipEventSynchronize(e.second) != hipSuccess ||
                             hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess))
            rc = fail(SCS_EDEVICE, "reading the launch timing events failed");
        if (rc == SCS_OK) {
            c->prof_ms += ms;
            c->prof_launches += 1;
        }
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    c->ev.clear();
    if (rc) return rc;
    if (launches) *launches = c->prof_launches;
    if (total_ms) *total_ms = c->prof_ms;
    if (enable >= 0) {
        if (enable && !c->prof) {
            c->prof_launches = 0;
            c->prof_ms = 0.0;
        }
        c->prof = enable != 0;
    }
    return SCS_OK;
}

extern "C" int scs_footprint(const scs_ctx* c, int64_t P, int32_t N, int32_t prec, size_t* bytes)
{
    if (!c || !bytes) return fail(SCS_EINVAL, "NULL argument");
    if (!c->has_data) return fail(SCS_ESTATE, "no data loaded");
    if (P < 0 || N < 1 || N > SCS_MAX_SEGMENTS) return fail(SCS_EINVAL, "bad P or N");
    const TuneChoice t = choose(c, P, N, prec);
    *bytes = ws_bytes(c, P, N, make_plan(c, P, t));
    return SCS_OK;
}

// ---------------------------------------------------------------- batched
// Every item owns a workspace slot of its context (slot 1 + its index), so
// items may share a context; calls that share a context must be issued on
// one stream.  The prologues, sorts and edges of the items are queued first,
// then ONE persistent generate-and-reduce launch per channel count covers
// the tiles of all its items (workgroups take tiles from a device counter),
// then the finalizes.

static void free_slot(BatchSlot& b)
{
    if (b.done) hipEventSynchronize(b.done);
    hipFree(b.d_items);
    hipFree(b.d_start);
    hipFree(b.d_counter);
    hipHostFree(b.h_items);
    hipHostFree(b.h_start);
    if (b.done) hipEventDestroy(b.done);
    b = BatchSlot();
}

static int slot_reserve(BatchSlot& b, int n)
{
    if (b.done) HIP_TRY(hipEventSynchronize(b.done));  // the launch that last read it has finished
    if (n <= b.cap) return SCS_OK;
    free_slot(b);
    const int cap = std::max(n, 8);
    if (hipMalloc((void**)&b.d_items, sizeof(MainArgs) * cap) != hipSuccess ||
        hipMalloc((void**)&b.d_start, sizeof(int64_t) * kVariants * (cap + 1)) != hipSuccess ||
        hipMalloc((void**)&b.d_counter, sizeof(unsigned long long) * kVariants) != hipSuccess ||
        hipHostMalloc((void**)&b.h_items, sizeof(MainArgs) * cap) != hipSuccess ||
        hipHostMalloc((void**)&b.h_start, sizeof(int64_t) * kVariants * (cap + 1)) != hipSuccess ||
        hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess) {
        free_slot(b);
        return fail(SCS_ENOMEM, "batch descriptor allocation failed");
    }
    b.cap = cap;
    return SCS_OK;
}

static int check_items(const scs_batch_item* items, int32_t n_items, int32_t prec)
{
    if (!items || n_items < 0) return fail(SCS_EINVAL, "bad items");
    if (prec != SCS_PREC_FP64 && prec != SCS_PREC_MIXED) return fail(SCS_EINVAL, "bad precision");
    for (int i = 0; i < n_items; ++i) {
        const scs_batch_item& it = items[i];
        int rc = check_ready(it.ctx);
        if (rc) return rc;
        if (it.N < 1 || it.N > SCS_MAX_SEGMENTS || it.P < 0 || (it.P > 0 && (!it.theta || !it.ups)))
            return fail(SCS_EINVAL, "item %d: bad N, P or pointers", i);
        if (it.ctx->device != items[0].ctx->device || it.ctx->L != items[0].ctx->L)
            return fail(SCS_EINVAL, "item %d: all items of a batch must share the device", i);
    }
    return SCS_OK;
}

// ==== launch shape of the generate-and-reduce (begin)
// The generate-and-reduce of prepared evaluations: one persistent launch per
// kernel variant (response model and channels) over the tiles of all of
// them (descriptors in slot b; upload: copy them from the pinned host copy
// first).
static int fused_main(std::vector<EvalJob>& jobs, int waves, bool mixed, hipStream_t s, BatchSlot& b, bool upload)
{
    const int n_items = (int)jobs.size();
    scs_ctx* c0 = jobs[0].c;
    int off = 0;
    for (int gi = 0; gi < kVariants; ++gi) {
        int cnt = 0;
        int64_t total = 0;
        int Lmax = 0;           // the launch stages up to the longest LDS block of its items
        int alt = 0;            // and takes the occupancy of its item with the most tiles
        int64_t most = -1;
        int64_t* hs = b.h_start + gi * (b.cap + 1);
        for (int i = 0; i < n_items; ++i) {
            const EvalJob& j = jobs[i];
            if (variant_of(j.c->m.response, j.c->g.nch, j.c->m.sparse) != gi || j.P == 0 || j.pl.n_tiles == 0) continue;
            if (upload) {
                b.h_items[off + cnt] = j.ma;
                hs[cnt] = total;
            }
            total += j.pl.n_tiles;
            Lmax = std::max(Lmax, j.pl.L);
            if (j.pl.n_tiles > most) {
                most = j.pl.n_tiles;
                alt = j.pl.alt;
            }
            ++cnt;
        }
        if (!cnt) continue;
        if (upload) {
            hs[cnt] = total;
            HIP_TRY(hipMemcpyAsync(b.d_items + off, b.h_items + off, sizeof(MainArgs) * cnt, hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(b.d_start + gi * (b.cap + 1), hs, sizeof(int64_t) * (cnt + 1), hipMemcpyHostToDevice, s));
        }
        launch_fill_u64(b.d_counter + gi, 1, 0ULL, s);
        const int per_cu = main_multi_blocks_per_cu(gi, Lmax, waves, mixed, alt != 0);
        const int64_t grid = std::min<int64_t>(total, (int64_t)c0->n_cu * per_cu);
        hipEvent_t e0;
        prof_begin(c0, s, &e0);
        hipError_t e = launch_main_multi(b.d_items + off, b.d_start + gi * (b.cap + 1), cnt, b.d_counter + gi, gi, Lmax,
                                         waves, mixed, alt != 0, (int)grid, s);
        if (e != hipSuccess) return fail(SCS_EDEVICE, "generate-and-reduce launch failed: %s", hipGetErrorString(e));
        prof_end(c0, s, e0);
        off += cnt;
    }
    return SCS_OK;
}

// One evaluation's generate-and-reduce, through the same persistent kernel
// (a device queue spreads its tiles over every XCD), descriptors from the
// context's ring.
static int eval_main(scs_ctx* c, EvalJob& j, int prec, hipStream_t s)
{
    BatchSlot& b = c->ring[c->ring_next];
    c->ring_next = (c->ring_next + 1) % scs_ctx::kRing;
    int rc = slot_reserve(b, 1);
    if (rc) return rc;
    std::vector<EvalJob> one(1, j);
    if ((rc = fused_main(one, j.pl.waves, prec == SCS_PREC_MIXED, s, b, true))) return rc;
    HIP_TRY(hipEventRecord(b.done, s));
    return SCS_OK;
}

// ==== launch shape of the generate-and-reduce (end)

// Queue a batch on s using the descriptors of slot b.  upload: copy the
// descriptors from the pinned host copy (skipped under graph capture, where
// they were uploaded when the graph was built and stay valid).
// wss[i] (nullable) is the workspace of item i; by default slot 1 + i of its
// context.
static int run_batched(const scs_batch_item* items, int n_items, int prec, hipStream_t s, BatchSlot& b, bool upload,
                       Workspace* const* wss = nullptr, const TuneChoice* force = nullptr,
                       const int32_t* const* frozen = nullptr)
{
    const bool mixed = prec == SCS_PREC_MIXED;
    constexpr int kWaves = 4;  // workgroup shape of the fused launch
    // The items' prologues, sorts and edges (and afterwards their
    // finalizes) are independent: item i runs on the caller's stream or on
    // side stream (i - 1) mod kSide of the first item's context, forked from
    // the caller's stream and joined back before the fused launch (and
    // before the call returns), so that small items do not wait for large
    // ones.  Graph capture records the fork and join as dependencies.
    scs_ctx* c0 = items[0].ctx;
    const int n_side = (n_items > 1 && c0->fork_ev) ? std::min(n_items - 1, scs_ctx::kSide) : 0;
    auto stream_of = [&](int i) { return i == 0 || n_side == 0 ? s : c0->side[(i - 1) % n_side]; };
    auto fork = [&]() -> hipError_t {
        hipError_t e = n_side ? hipEventRecord(c0->fork_ev, s) : hipSuccess;
        for (int k = 0; k < n_side && e == hipSuccess; ++k) e = hipStreamWaitEvent(c0->side[k], c0->fork_ev, 0);
        return e;
    };
    auto join = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int k = 0; k < n_side && e == hipSuccess; ++k) {
            e = hipEventRecord(c0->join_ev[k], c0->side[k]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, c0->join_ev[k], 0);
        }
        return e;
    };
    std::vector<EvalJob> jobs(n_items);
    hipError_t e = fork();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "stream fork failed: %s", hipGetErrorString(e));
    int rc = SCS_OK;
    for (int i = 0; i < n_items && rc == SCS_OK; ++i) {
        const scs_batch_item& it = items[i];
        EvalJob& j = jobs[i];
        j.c = it.ctx;
        j.w = (wss && wss[i]) ? wss[i] : &it.ctx->ws[1 + i];
        j.P = it.P;
        j.N = it.N;
        TuneChoice t = force ? force[i] : choose(it.ctx, it.P, it.N, prec);
        t.waves = kWaves;
        rc = eval_front(j, it.theta, it.ups, it.seg, t, stream_of(i), nullptr, false, frozen ? frozen[i] : nullptr);
    }
    // joined even after a failed item, so that no side stream is left
    // waiting apart from the caller's (a capture needs every branch joined)
    e = join();
    if (rc) return rc;
    if (e != hipSuccess) return fail(SCS_EDEVICE, "stream join failed: %s", hipGetErrorString(e));
    rc = fused_main(jobs, kWaves, mixed, s, b, upload);
    if (rc) return rc;
    if ((e = fork()) != hipSuccess) return fail(SCS_EDEVICE, "stream fork failed: %s", hipGetErrorString(e));
    for (int i = 0; i < n_items; ++i)
        if (jobs[i].P > 0) launch_finalize(jobs[i].fa, stream_of(i));
    if ((e = join()) != hipSuccess) return fail(SCS_EDEVICE, "stream join failed: %s", hipGetErrorString(e));
    e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    for (int i = 0; i < n_items; ++i) items[i].ctx->last_stream = s;
    return SCS_OK;
}

extern "C" int scs_evaluate_batched(const scs_batch_item* items, int32_t n_items, int32_t prec, void* stream)
{
    int rc = check_items(items, n_items, prec);
    if (rc || n_items == 0) return rc;
    scs_ctx* c0 = items[0].ctx;
    DevScope ds(c0->device);
    hipStream_t s = (hipStream_t)stream;
    BatchSlot& b = c0->ring[c0->ring_next];
    c0->ring_next = (c0->ring_next + 1) % scs_ctx::kRing;
    if ((rc = slot_reserve(b, n_items))) return rc;
    if ((rc = run_batched(items, n_items, prec, s, b, true))) return rc;
    HIP_TRY(hipEventRecord(b.done, s));
    return SCS_OK;
}

struct scs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    BatchSlot slot;  // descriptors read by the captured fused launches
    // the graph's own workspaces (one per item): the captured kernels hold
    // their addresses, so no later call on the contexts may move them
    std::vector<Workspace> ws;
    std::vector<std::pair<const scs_ctx*, uint64_t>> ctx_gen;  // contexts and their state when captured
};

static void graph_free(scs_graph* g)
{
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    free_slot(g->slot);
    for (auto& w : g->ws) free_ws(w);
    delete g;
}

extern "C" int scs_graph_create(scs_graph** out, const scs_batch_item* items, int32_t n_items, int32_t prec)
{
    if (!out) return fail(SCS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_items(items, n_items, prec);
    if (rc) return rc;
    if (n_items < 1) return fail(SCS_EINVAL, "no items");
    const int dev = items[0].ctx->device;
    DevScope ds(dev);
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    scs_graph* g = new scs_graph();
    g->device = dev;
    g->ws.resize(n_items);
    std::vector<Workspace*> wsp(n_items);
    for (int i = 0; i < n_items; ++i) {
        wsp[i] = &g->ws[i];
        g->ctx_gen.emplace_back(items[i].ctx, items[i].ctx->gen);
    }
    // one eager pass: allocates every workspace and uploads the descriptors
    if ((rc = slot_reserve(g->slot, n_items)) == SCS_OK)
        rc = run_batched(items, n_items, prec, s, g->slot, true, wsp.data());
    hipError_t e = hipStreamSynchronize(s);
    if (rc == SCS_OK && e == hipSuccess) {
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = run_batched(items, n_items, prec, s, g->slot, false, wsp.data());
            e = hipStreamEndCapture(s, &g->graph);
        }
        if (e == hipSuccess && rc == SCS_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    }
    hipStreamDestroy(s);
    if (e != hipSuccess || rc != SCS_OK) {
        graph_free(g);
        return rc ? rc : fail(SCS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return SCS_OK;
}

extern "C" int scs_graph_launch(scs_graph* g, void* stream)
{
    if (!g) return fail(SCS_EINVAL, "graph is NULL");
    for (const auto& cg : g->ctx_gen)
        if (cg.first->gen != cg.second)
            return fail(SCS_ESTATE, "a context of this graph changed its data, model or segmentation after the "
                                    "capture; build a new graph");
    DevScope ds(g->device);
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    HIP_TRY(hipEventRecord(g->slot.done, (hipStream_t)stream));
    return SCS_OK;
}

extern "C" int scs_graph_destroy(scs_graph* g)
{
    if (!g) return SCS_OK;
    DevScope ds(g->device);
    if (g->slot.done) hipEventSynchronize(g->slot.done);
    graph_free(g);
    return SCS_OK;
}

// ---------------------------------------------------------------- serving
namespace {

struct SrvRequest {
    uint64_t id = 0;
    scs_ctx* ctx = nullptr;
    int N = 1;
    int64_t P = 0;
    int prec = SCS_PREC_FP64;
    double* ups_user = nullptr;
    std::vector<double> theta;  // host copy
    uint64_t bytes = 0;
    int slot = -1;
    double t_submit = 0, t_admit = 0, t_launch = 0;
};

// A request slot: device theta / result buffers, a workspace and the pinned
// host buffers of its copies; kept and regrown across requests.
struct SrvSlot {
    bool busy = false;
    int64_t cap = 0;
    double* d_theta = nullptr;
    double* d_ups = nullptr;
    double* h_theta = nullptr;  // pinned
    double* h_ups = nullptr;    // pinned
    Workspace ws;
};

struct SrvBatch {
    std::vector<SrvRequest*> reqs;
    int stream = 0;
    hipEvent_t done = nullptr;
};

}  // namespace

struct scs_server {
    int device = 0;
    int max_inflight = 1;
    uint64_t budget = 0;
    std::chrono::steady_clock::time_point t0;
    std::vector<hipStream_t> streams;
    std::vector<bool> stream_busy;
    std::vector<BatchSlot> bslots;  // descriptors, one per stream and precision
    std::vector<SrvSlot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvRequest*> pending;
    std::deque<scs_request_done> done;
    std::vector<SrvBatch> inflight;
    uint64_t next_id = 1;
    bool stop = false;
    scs_server_counters st{};
    std::thread worker;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
    uint64_t resident() const;  // device bytes held by all request slots
    void run();
    int launch(std::vector<SrvRequest*>& batch, int si);
    void finish(SrvBatch& b, int status);
};

// Device bytes a request slot holds: its workspace (as ensure_ws sized it)
// and its theta and result buffers.
static uint64_t slot_bytes(const SrvSlot& s)
{
    const Workspace& w = s.ws;
    uint64_t b = (uint64_t)w.capP * (sizeof(double) * kCoefStride + 2 * sizeof(int32_t) + 1);
    b += (uint64_t)w.capBounds * sizeof(int32_t) + (uint64_t)(w.capRec + w.capZs + w.capSpl) * sizeof(double);
    if (w.capSort) b += (uint64_t)w.capSort * 3 * sizeof(int32_t) + sizeof(unsigned) * (uint64_t)kSortBuckets;
    b += (uint64_t)s.cap * sizeof(double) * (kThetaMax + 1);
    return b;
}

// The bytes slot s holds after serving P particles with N segments of
// context c: slot_grow and ensure_ws grow each buffer to fit and shrink none.
static uint64_t slot_bytes_after(const SrvSlot& s, const scs_ctx* c, int64_t P, int N, int prec)
{
    TuneChoice t = choose(c, P, N, prec);
    t.waves = 4;  // the workgroup shape of batched launches (the chunk count does not depend on it)
    const Plan pl = make_plan(c, P, t);
    SrvSlot x;
    x.cap = P <= s.cap ? s.cap : std::max<int64_t>(P, 256);
    Workspace& w = x.ws;
    w.capP = std::max(s.ws.capP, pad64(std::max<int64_t>(P, 1)));
    w.capBounds = std::max(s.ws.capBounds, P * (int64_t)(N + 1) + 2);
    w.capRec = std::max(s.ws.capRec, pl.n_chunks * kRec * w.capP);
    w.capZs = std::max(s.ws.capZs, 3 * P * (int64_t)N);
    w.capSpl = std::max(s.ws.capSpl, spl_doubles(c, w.capP));
    w.capSort = (P >= kSortMin && P > s.ws.capSort) ? w.capP : s.ws.capSort;
    return slot_bytes(x);
}

// Device bytes of a request in a slot of its own: what admission must find
// free for it at least.
static uint64_t request_bytes(const scs_ctx* c, int64_t P, int N, int prec)
{
    return slot_bytes_after(SrvSlot(), c, P, N, prec);
}

// Free a slot's device buffers (an idle slot, to make room under the budget).
static void slot_release(SrvSlot& s)
{
    free_ws(s.ws);
    hipFree(s.d_theta);
    hipFree(s.d_ups);
    hipHostFree(s.h_theta);
    hipHostFree(s.h_ups);
    s.d_theta = s.d_ups = s.h_theta = s.h_ups = nullptr;
    s.cap = 0;
}

static int slot_grow(SrvSlot& s, int64_t P)
{
    if (P <= s.cap) return SCS_OK;
    hipFree(s.d_theta);
    hipFree(s.d_ups);
    hipHostFree(s.h_theta);
    hipHostFree(s.h_ups);
    s.d_theta = s.d_ups = s.h_theta = s.h_ups = nullptr;
    s.cap = 0;
    const int64_t cap = std::max<int64_t>(P, 256);
    if (hipMalloc((void**)&s.d_theta, sizeof(double) * kThetaMax * cap) != hipSuccess ||
        hipMalloc((void**)&s.d_ups, sizeof(double) * cap) != hipSuccess ||
        hipHostMalloc((void**)&s.h_theta, sizeof(double) * kThetaMax * cap) != hipSuccess ||
        hipHostMalloc((void**)&s.h_ups, sizeof(double) * cap) != hipSuccess)
        return fail(SCS_ENOMEM, "request buffers of %lld particles", (long long)P);
    s.cap = cap;
    return SCS_OK;
}

uint64_t scs_server::resident() const
{
    uint64_t b = 0;
    for (const SrvSlot& sl : slots) b += slot_bytes(sl);
    return b;
}

// Queue one batched launch of the admitted requests on stream si.
int scs_server::launch(std::vector<SrvRequest*>& batch, int si)
{
    hipStream_t s = streams[si];
    std::vector<scs_batch_item> items(batch.size());
    std::vector<Workspace*> wss(batch.size());
    int rc = SCS_OK;
    for (size_t i = 0; i < batch.size() && rc == SCS_OK; ++i) {
        SrvRequest* r = batch[i];
        SrvSlot& sl = slots[r->slot];
        if ((rc = slot_grow(sl, r->P))) break;
        std::memcpy(sl.h_theta, r->theta.data(), sizeof(double) * r->theta.size());
        if (hipMemcpyAsync(sl.d_theta, sl.h_theta, sizeof(double) * r->theta.size(), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            rc = fail(SCS_EDEVICE, "theta upload failed");
        items[i] = scs_batch_item{r->ctx, r->N, 0, r->P, sl.d_theta, sl.d_ups, nullptr};
        wss[i] = &sl.ws;
    }
    // one precision per launch: split the batch if it mixes them
    for (int prec : {SCS_PREC_FP64, SCS_PREC_MIXED}) {
        if (rc) break;
        std::vector<scs_batch_item> it2;
        std::vector<Workspace*> w2;
        for (size_t i = 0; i < batch.size(); ++i)
            if (batch[i]->prec == prec) {
                it2.push_back(items[i]);
                w2.push_back(wss[i]);
            }
        if (it2.empty()) continue;
        // a slot of its own per precision, so that queuing the second part
        // of a mixed batch does not wait for the first one to finish
        BatchSlot& b = bslots[2 * si + (prec == SCS_PREC_MIXED)];
        if ((rc = slot_reserve(b, (int)it2.size()))) break;
        if ((rc = run_batched(it2.data(), (int)it2.size(), prec, s, b, true, w2.data()))) break;
        if (hipEventRecord(b.done, s) != hipSuccess) rc = fail(SCS_EDEVICE, "event record failed");
    }
    for (size_t i = 0; i < batch.size() && rc == SCS_OK; ++i) {
        SrvSlot& sl = slots[batch[i]->slot];
        if (hipMemcpyAsync(sl.h_ups, sl.d_ups, sizeof(double) * batch[i]->P, hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = fail(SCS_EDEVICE, "result download failed");
    }
    return rc;
}

void scs_server::finish(SrvBatch& b, int status)
{
    const double t = now();
    for (SrvRequest* r : b.reqs) {
        if (status == SCS_OK) std::memcpy(r->ups_user, slots[r->slot].h_ups, sizeof(double) * r->P);
        scs_request_done d{};
        d.id = r->id;
        d.status = status;
        d.t_submit = r->t_submit;
        d.t_admit = r->t_admit;
        d.t_launch = r->t_launch;
        d.t_done = t;
        {
            std::lock_guard<std::mutex> lk(mu);
            slots[r->slot].busy = false;
            if (status == SCS_OK) ++st.completed; else ++st.failed;
            done.push_back(d);
        }
        delete r;
    }
    b.reqs.clear();
    cv_done.notify_all();
}

void scs_server::run()
{
    DevScope ds(device);
    while (true) {
        // ---- completions
        for (size_t k = 0; k < inflight.size();) {
            const hipError_t q = hipEventQuery(inflight[k].done);
            if (q == hipErrorNotReady) {
                ++k;
                continue;
            }
            finish(inflight[k], q == hipSuccess ? SCS_OK : SCS_EDEVICE);
            hipEventDestroy(inflight[k].done);
            stream_busy[inflight[k].stream] = false;
            inflight.erase(inflight.begin() + k);
        }
        // ---- admission: arrival order, while a slot, the memory and a stream are free
        std::vector<SrvRequest*> batch;
        int si = -1;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (stop && pending.empty() && inflight.empty()) break;
            for (int i = 0; i < (int)streams.size(); ++i)
                if (!stream_busy[i]) {
                    si = i;
                    break;
                }
            if (si >= 0) {
                // Memory is charged as the slots hold it: every slot keeps
                // its buffers at the largest size it has served, so the
                // charge is the device bytes of all slots after the chosen
                // one has grown to fit the request.  The free slot that grows
                // least is taken; if the budget would still be exceeded, the
                // buffers of the idle slots are released (the chosen slot
                // then starts from nothing), else the request waits.
                uint64_t held = resident();
                while (!pending.empty()) {
                    SrvRequest* r = pending.front();
                    int pick = -1;
                    uint64_t pick_now = 0, pick_after = 0;
                    for (int i = 0; i < max_inflight; ++i) {
                        if (slots[i].busy) continue;
                        const uint64_t nw = slot_bytes(slots[i]);
                        const uint64_t af = slot_bytes_after(slots[i], r->ctx, r->P, r->N, r->prec);
                        if (pick < 0 || af - nw < pick_after - pick_now) {
                            pick = i;
                            pick_now = nw;
                            pick_after = af;
                        }
                    }
                    if (pick < 0) break;
                    if (held - pick_now + pick_after > budget) {
                        for (SrvSlot& sl : slots)
                            if (!sl.busy && sl.cap + sl.ws.capP > 0) slot_release(sl);
                        held = resident();
                        pick_now = 0;
                        pick_after = slot_bytes_after(slots[pick], r->ctx, r->P, r->N, r->prec);
                        if (held + pick_after > budget) break;
                    }
                    pending.pop_front();
                    slots[pick].busy = true;
                    r->slot = pick;
                    r->t_admit = now();
                    held = held - pick_now + pick_after;
                    st.hbm_in_use = held;
                    st.hbm_peak = std::max(st.hbm_peak, held);
                    batch.push_back(r);
                }
                int64_t busy = 0;
                for (auto& sl : slots) busy += sl.busy;
                st.max_inflight = std::max<int64_t>(st.max_inflight, busy);
            }
            if (batch.empty()) {
                if (inflight.empty()) cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
        if (batch.empty()) {
            if (!inflight.empty()) std::this_thread::sleep_for(std::chrono::microseconds(20));
            continue;
        }
        const double tl = now();
        for (SrvRequest* r : batch) r->t_launch = tl;
        SrvBatch b;
        b.reqs = batch;
        b.stream = si;
        int rc = launch(batch, si);
        if (rc == SCS_OK && hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess &&
            hipEventRecord(b.done, streams[si]) == hipSuccess) {
            stream_busy[si] = true;
            {
                std::lock_guard<std::mutex> lk(mu);
                ++st.launches;
                st.max_batch = std::max<int64_t>(st.max_batch, (int64_t)batch.size());
            }
            inflight.push_back(b);
        } else {
            if (b.done) hipEventDestroy(b.done);
            hipStreamSynchronize(streams[si]);
            finish(b, rc ? rc : SCS_EDEVICE);
        }
    }
}

extern "C" int scs_server_create(scs_server** out, int32_t device, int32_t max_inflight, uint64_t hbm_budget,
                                 int32_t n_streams)
{
    if (!out) return fail(SCS_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > 1024) return fail(SCS_EINVAL, "max_inflight must be in 1..1024");
    if (n_streams < 1 || n_streams > 16) return fail(SCS_EINVAL, "n_streams must be in 1..16");
    if (hbm_budget == 0) return fail(SCS_EINVAL, "hbm_budget must be > 0");
    int rc = device_setup(device);
    if (rc) return rc;
    DevScope ds(device);
    scs_server* s = new (std::nothrow) scs_server();
    if (!s) return fail(SCS_ENOMEM, "host allocation failed");
    s->device = device;
    s->max_inflight = max_inflight;
    s->budget = hbm_budget;
    s->t0 = std::chrono::steady_clock::now();
    s->slots.resize(max_inflight);
    s->bslots.resize(2 * n_streams);
    s->stream_busy.assign(n_streams, false);
    for (int i = 0; i < n_streams; ++i) {
        hipStream_t st;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : s->streams) hipStreamDestroy(x);
            delete s;
            return fail(SCS_EDEVICE, "stream creation failed");
        }
        s->streams.push_back(st);
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return SCS_OK;
}

extern "C" int scs_server_submit(scs_server* srv, scs_ctx* ctx, int32_t N, int64_t P, const double* theta, int32_t prec,
                                 double* ups, uint64_t* id)
{
    if (!srv) return fail(SCS_EINVAL, "server is NULL");
    int rc = check_ready(ctx);
    if (rc) return rc;
    if (ctx->device != srv->device) return fail(SCS_EINVAL, "context is on device %d, server on %d", ctx->device, srv->device);
    if (N < 1 || N > SCS_MAX_SEGMENTS || P < 1 || !theta || !ups) return fail(SCS_EINVAL, "bad N, P or pointers");
    if (prec != SCS_PREC_FP64 && prec != SCS_PREC_MIXED) return fail(SCS_EINVAL, "bad precision");
    if (ctx->mode == SCS_SEG_EXPLICIT && N != ctx->N) return fail(SCS_EINVAL, "EXPLICIT edges were defined for N = %d", ctx->N);
    const uint64_t bytes = request_bytes(ctx, P, N, prec);
    if (bytes > srv->budget)
        return fail(SCS_EBUSY, "request needs %llu bytes, budget is %llu", (unsigned long long)bytes,
                    (unsigned long long)srv->budget);
    SrvRequest* r = new (std::nothrow) SrvRequest();
    if (!r) return fail(SCS_ENOMEM, "host allocation failed");
    r->ctx = ctx;
    r->N = N;
    r->P = P;
    r->prec = prec;
    r->ups_user = ups;
    r->theta.assign(theta, theta + (int64_t)theta_dim(ctx) * P);
    r->bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            delete r;
            return fail(SCS_ESTATE, "server is stopping");
        }
        r->id = srv->next_id++;
        r->t_submit = srv->now();
        srv->pending.push_back(r);
        ++srv->st.submitted;
        if (id) *id = r->id;
    }
    srv->cv_work.notify_one();
    return SCS_OK;
}

extern "C" int scs_server_poll(scs_server* srv, scs_request_done* out, int32_t max_out, int32_t wait_ms, int32_t* n_out)
{
    if (!srv || (!out && max_out > 0) || !n_out) return fail(SCS_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_ms > 0)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [srv] { return !srv->done.empty(); });
    int n = 0;
    while (n < max_out && !srv->done.empty()) {
        out[n++] = srv->done.front();
        srv->done.pop_front();
    }
    *n_out = n;
    return SCS_OK;
}

extern "C" int scs_server_stats(scs_server* srv, scs_server_counters* out)
{
    if (!srv || !out) return fail(SCS_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    return SCS_OK;
}

extern "C" double scs_server_clock(const scs_server* srv) { return srv ? srv->now() : 0.0; }

extern "C" int scs_server_destroy(scs_server* srv)
{
    if (!srv) return SCS_OK;
    std::deque<SrvRequest*> dropped;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        dropped.swap(srv->pending);
    }
    for (SrvRequest* r : dropped) delete r;
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    DevScope ds(srv->device);
    for (auto st : srv->streams) {
        hipStreamSynchronize(st);
        hipStreamDestroy(st);
    }
    for (auto& b : srv->bslots) free_slot(b);
    for (auto& sl : srv->slots) slot_release(sl);
    delete srv;
    return SCS_OK;
}

// ---------------------------------------------------------------- autotuner
// Cache file: one "key waves blocks L alt" line per evaluation class (a line
// of the older "key waves blocks" form reads as L = 512 and alt = 0).
static bool choice_ok(const TuneChoice& t)
{
    return (t.waves == 1 || t.waves == 2 || t.waves == 4) && t.CB >= 1 && t.CB <= 64 &&
           (t.L == 256 || t.L == 512 || t.L == 1024) && (t.alt == 0 || t.alt == 1);
}

static void read_cache(const char* path, std::map<std::string, TuneChoice>& into)
{
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string key;
        TuneChoice t;
        if (!(is >> key >> t.waves >> t.CB)) continue;
        if (!(is >> t.L >> t.alt)) {
            t.L = 512;
            t.alt = 0;
        }
        if (choice_ok(t)) into[key] = t;
    }
}

static void save_cache(const std::map<std::string, TuneChoice>& tune, const char* path)
{
    std::map<std::string, TuneChoice> all;
    read_cache(path, all);
    for (auto& kv : tune) all[kv.first] = kv.second;
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        for (auto& kv : all)
            o << kv.first << " " << kv.second.waves << " " << kv.second.CB << " " << kv.second.L << " "
              << kv.second.alt << "\n";
    }
    std::rename(tmp.c_str(), path);
}

// The candidate values of each coordinate of a shape.  The alternative
// occupancy exists for the per-bin template on one and two channels.
static const int kTuneWaves[] = {1, 2, 4};
static const int kTuneL[] = {256, 512, 1024};
static const int kTuneChunk[] = {1024, 2048, 4096, 8192};  // bins per chunk (L x CB)
static bool has_alt(const scs_ctx* c) { return c->m.sparse == 0 && c->g.nch <= 2; }

// Candidates along one coordinate d (0 waves, 1 LDS block, 2 chunk, 3
// occupancy) of shape t.
static std::vector<TuneChoice> along(const scs_ctx* c, const TuneChoice& t, int d, bool waves_fixed)
{
    std::vector<TuneChoice> v;
    if (d == 0 && !waves_fixed)
        for (int w : kTuneWaves) { TuneChoice x = t; x.waves = w; v.push_back(x); }
    if (d == 1) {
        const int chunk = t.L * t.CB;
        for (int L : kTuneL) { TuneChoice x = t; x.L = L; x.CB = std::max(1, chunk / L); v.push_back(x); }
    }
    if (d == 2)
        for (int ch : kTuneChunk) { TuneChoice x = t; x.CB = std::max(1, ch / t.L); v.push_back(x); }
    if (d == 3 && has_alt(c))
        for (int a = 0; a <= 1; ++a) { TuneChoice x = t; x.alt = a; v.push_back(x); }
    return v;
}

static bool same_shape(const TuneChoice& a, const TuneChoice& b)
{
    return a.waves == b.waves && a.CB == b.CB && a.L == b.L && a.alt == b.alt;
}

// Time fn (which queues one evaluation on s): one untimed run, then the mean
// of `reps`; negative on an error (recorded).
template <class Fn>
static double time_on(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, Fn fn)
{
    if (fn()) return -1.0;
    if (hipEventRecord(e0, s) != hipSuccess) return fail(SCS_EDEVICE, "event record failed"), -1.0;
    for (int r = 0; r < reps; ++r)
        if (fn()) return -1.0;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return fail(SCS_EDEVICE, "timing a candidate failed"), -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(SCS_EDEVICE, "event timing failed"), -1.0;
    return ms / reps;
}

extern "C" int scs_autotune(scs_ctx* c, int64_t P, const double* theta_dev, int32_t N, int32_t prec,
                            const char* cache_path)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 1 || N < 1 || N > SCS_MAX_SEGMENTS) return fail(SCS_EINVAL, "bad P or N");
    const std::string key = tune_key(c, P, N, prec);
    if (cache_path) {
        read_cache(cache_path, c->tune);
        if (c->tune.count(key)) return SCS_OK;
    }
    if (!theta_dev) return fail(SCS_EINVAL, "theta is NULL");
    DevScope ds(c->device);
    double* ups = nullptr;
    HIP_TRY(hipMalloc((void**)&ups, sizeof(double) * P));
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
        hipFree(ups);
        return fail(SCS_EDEVICE, "stream creation failed");
    }
    Workspace tw;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(SCS_EDEVICE, "event creation failed");
    // coordinate descent from the default shape: waves, LDS block, chunk,
    // occupancy, twice over
    TuneChoice best = default_choice(c, P);
    double best_ms = 1e300;
    for (int pass = 0; pass < 2 && !rc; ++pass)
        for (int d = 0; d < 4 && !rc; ++d)
            for (const TuneChoice& t : along(c, best, d, false)) {
                if (pass + d > 0 && same_shape(t, best)) continue;  // timed already
                const double ms = time_on(s, e0, e1, 3, [&] {
                    return run_eval(c, tw, P, N, theta_dev, prec, ups, nullptr, s, &t);
                });
                if (ms < 0.0) {
                    rc = SCS_EDEVICE;
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = t;
                }
            }
    hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipStreamDestroy(s);
    free_ws(tw);
    hipFree(ups);
    if (rc) return rc;
    c->tune[key] = best;
    if (cache_path) save_cache(c->tune, cache_path);
    return SCS_OK;
}

extern "C" int scs_autotune_batch(const scs_batch_item* items, int32_t n_items, int32_t prec, const char* cache_path)
{
    int rc = check_items(items, n_items, prec);
    if (rc || n_items == 0) return rc;
    scs_ctx* c0 = items[0].ctx;
    std::vector<std::string> keys(n_items);
    bool all_cached = cache_path != nullptr;
    for (int i = 0; i < n_items; ++i) {
        keys[i] = tune_key(items[i].ctx, items[i].P, items[i].N, prec);
        if (cache_path) read_cache(cache_path, items[i].ctx->tune);
        all_cached = all_cached && items[i].ctx->tune.count(keys[i]);
    }
    if (all_cached) return SCS_OK;
    DevScope ds(c0->device);
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return fail(SCS_EDEVICE, "stream creation failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        rc = fail(SCS_EDEVICE, "event creation failed");
    BatchSlot& b = c0->ring[c0->ring_next];
    c0->ring_next = (c0->ring_next + 1) % scs_ctx::kRing;
    if (!rc) rc = slot_reserve(b, n_items);
    std::vector<TuneChoice> cur(n_items);
    for (int i = 0; i < n_items; ++i) {
        cur[i] = choose(items[i].ctx, items[i].P, items[i].N, prec);
        cur[i].waves = 4;  // the fused launch's workgroup shape
    }
    auto batch_ms = [&](const std::vector<TuneChoice>& sh) {
        return time_on(s, e0, e1, 2, [&] { return run_batched(items, n_items, prec, s, b, true, nullptr, sh.data()); });
    };
    double best_ms = rc ? -1.0 : batch_ms(cur);
    if (best_ms < 0.0 && !rc) rc = SCS_EDEVICE;
    // the occupancy of the launch, then each item's LDS block and chunk,
    // items with the most tiles first
    if (!rc) {
        bool any_alt = false;
        for (int i = 0; i < n_items; ++i) any_alt = any_alt || has_alt(items[i].ctx);
        if (any_alt) {
            std::vector<TuneChoice> alt = cur;
            for (auto& t : alt) t.alt = 1 - t.alt;
            const double ms = batch_ms(alt);
            if (ms < 0.0) rc = SCS_EDEVICE;
            else if (ms < best_ms) {
                best_ms = ms;
                cur = alt;
            }
        }
    }
    std::vector<int> order(n_items);
    for (int i = 0; i < n_items; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b2) {
        return (double)items[a].P * items[a].N > (double)items[b2].P * items[b2].N;
    });
    for (int oi = 0; oi < n_items && !rc; ++oi) {
        const int i = order[oi];
        if (items[i].P == 0) continue;
        for (int d = 1; d <= 2 && !rc; ++d)
            for (const TuneChoice& t : along(items[i].ctx, cur[i], d, true)) {
                if (same_shape(t, cur[i])) continue;
                std::vector<TuneChoice> trial = cur;
                trial[i] = t;
                const double ms = batch_ms(trial);
                if (ms < 0.0) {
                    rc = SCS_EDEVICE;
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    cur = trial;
                }
            }
    }
    if (b.done) hipEventRecord(b.done, s);
    hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipStreamDestroy(s);
    if (rc) return rc;
    for (int i = 0; i < n_items; ++i) {
        items[i].ctx->tune[keys[i]] = cur[i];
        if (cache_path) save_cache(items[i].ctx->tune, cache_path);
    }
    return SCS_OK;
}

// ---------------------------------------------------------------- swarms
struct scs_swarm {
    scs_ctx* ctx = nullptr;
    int64_t P = 0;
    double *theta = nullptr, *vel = nullptr, *pbest = nullptr, *pbest_val = nullptr;
    double *gbest = nullptr, *ups = nullptr;  // gbest[dim] position, gbest[dim] = value
    int dim = kTheta;                          // entries per theta row (the context's)
    PsoBox box{};
    uint64_t seed = 0;
    uint32_t swarm_id = 0;
    uint32_t iteration = 0;
};

static int make_box(const double* lo, const double* hi, const int32_t* periodic, int dim, PsoBox* box)
{
    if (dim != kTheta && dim != kThetaMax) return fail(SCS_EINVAL, "dim must be 7 or 8");
    box->dim = dim;
    for (int d = 0; d < dim; ++d) {
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || hi[d] < lo[d]) return fail(SCS_EINVAL, "bad box in dimension %d", d);
        box->lo[d] = lo[d];
        box->hi[d] = hi[d];
        box->periodic[d] = periodic ? (periodic[d] != 0) : 0;
        if (box->periodic[d] && !(hi[d] > lo[d])) return fail(SCS_EINVAL, "periodic dimension %d needs hi > lo", d);
    }
    return SCS_OK;
}

extern "C" int scs_swarm_create(scs_ctx* c, scs_swarm** out, int64_t P, const double* lo, const double* hi,
                                const int32_t* periodic, uint64_t seed, uint32_t swarm_id)
{
    if (!out) return fail(SCS_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 1 || !lo || !hi) return fail(SCS_EINVAL, "bad P or box");
    scs_swarm* sw = new scs_swarm();
    const int D = theta_dim(c);
    if ((rc = make_box(lo, hi, periodic, D, &sw->box))) {
        delete sw;
        return rc;
    }
    DevScope ds(c->device);
    sw->ctx = c;
    sw->P = P;
    sw->dim = D;
    sw->seed = seed;
    sw->swarm_id = swarm_id;
    const size_t nb = sizeof(double) * D * P;
    if (hipMalloc((void**)&sw->theta, nb) || hipMalloc((void**)&sw->vel, nb) || hipMalloc((void**)&sw->pbest, nb) ||
        hipMalloc((void**)&sw->pbest_val, sizeof(double) * P) ||
        hipMalloc((void**)&sw->gbest, sizeof(double) * (D + 1)) || hipMalloc((void**)&sw->ups, sizeof(double) * P)) {
        scs_swarm_destroy(sw);
        return fail(SCS_ENOMEM, "swarm allocation failed");
    }
    launch_pso_init(P, sw->box, seed, swarm_id, sw->theta, nullptr);
    launch_fill(sw->vel, D * P, 0.0, nullptr);
    launch_fill(sw->pbest, D * P, 0.0, nullptr);
    launch_fill(sw->pbest_val, P, -INFINITY, nullptr);
    launch_fill(sw->gbest, D, 0.0, nullptr);
    launch_fill(sw->gbest + D, 1, -INFINITY, nullptr);
    if (hipDeviceSynchronize() != hipSuccess) {
        scs_swarm_destroy(sw);
        return fail(SCS_EDEVICE, "swarm initialisation failed");
    }
    *out = sw;
    return SCS_OK;
}

extern "C" int scs_swarm_destroy(scs_swarm* sw)
{
    if (!sw) return SCS_OK;
    DevScope ds(sw->ctx ? sw->ctx->device : 0);
    hipDeviceSynchronize();
    hipFree(sw->theta);
    hipFree(sw->vel);
    hipFree(sw->pbest);
    hipFree(sw->pbest_val);
    hipFree(sw->gbest);
    hipFree(sw->ups);
    delete sw;
    return SCS_OK;
}

static PsoParams to_params(const scs_pso_params* p, int dim)
{
    PsoParams q;
    q.omega = p->omega;
    q.phi_p = p->phi_p;
    q.phi_g = p->phi_g;
    for (int d = 0; d < kThetaMax; ++d) q.eps[d] = d < dim ? p->eps[d] : 0.0;
    return q;
}

static int check_eps(const scs_pso_params* p, int dim)
{
    for (int d = 0; d < dim; ++d)
        if (!(p->eps[d] >= 0.0)) return fail(SCS_EINVAL, "eps[%d] must be >= 0", d);
    return SCS_OK;
}

extern "C" int scs_pso_step(scs_swarm* sw, const scs_pso_params* prm, int32_t prec, void* stream)
{
    if (!sw || !prm) return fail(SCS_EINVAL, "NULL argument");
    int rc0 = check_eps(prm, sw->dim);
    if (rc0) return rc0;
    scs_ctx* c = sw->ctx;
    int rc = check_ready(c);
    if (rc) return rc;
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (sw->iteration > 0)
        launch_pso_move(sw->P, sw->box, to_params(prm, sw->dim), sw->seed, sw->swarm_id, sw->iteration, sw->theta,
                        sw->vel, sw->pbest, sw->gbest, s);
    if ((rc = run_eval(c, c->ws[0], sw->P, c->N, sw->theta, prec, sw->ups, nullptr, s))) return rc;
    launch_pso_best(sw->P, sw->box, sw->theta, sw->ups, sw->pbest, sw->pbest_val, sw->gbest, sw->gbest + sw->dim, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "pso launch failed: %s", hipGetErrorString(e));
    sw->iteration += 1;
    return SCS_OK;
}

extern "C" int scs_pso_step_swarms(scs_swarm* const* sws, int32_t n, const scs_pso_params* prm, int32_t prec,
                                   double* gbest_vals, void* stream)
{
    if (!sws || n < 0 || !prm) return fail(SCS_EINVAL, "bad arguments");
    if (check_eps(prm, kThetaMax)) {
        for (int i = 0; i < n; ++i) {  // eps[7] is read only by eccentric swarms
            int rc = sws[i] ? check_eps(prm, sws[i]->dim) : SCS_OK;
            if (rc) return rc;
        }
    }
    if (n == 0) return SCS_OK;
    std::vector<scs_batch_item> items(n);
    for (int i = 0; i < n; ++i) {
        scs_swarm* sw = sws[i];
        if (!sw) return fail(SCS_EINVAL, "swarm %d is NULL", i);
        for (int j = 0; j < i; ++j)
            if (sws[j] == sw) return fail(SCS_EINVAL, "swarm %d appears twice", i);
        items[i] = scs_batch_item{sw->ctx, sw->ctx ? sw->ctx->N : 0, 0, sw->P, sw->theta, sw->ups, nullptr};
    }
    // items are checked (ready contexts, one device) before anything is queued
    int rc = check_items(items.data(), n, prec);
    if (rc) return rc;
    DevScope ds(sws[0]->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        scs_swarm* sw = sws[i];
        if (sw->iteration > 0)
            launch_pso_move(sw->P, sw->box, to_params(prm, sw->dim), sw->seed, sw->swarm_id, sw->iteration, sw->theta,
                            sw->vel, sw->pbest, sw->gbest, s);
    }
    if ((rc = scs_evaluate_batched(items.data(), n, prec, stream))) return rc;
    for (int i = 0; i < n; ++i) {
        scs_swarm* sw = sws[i];
        launch_pso_best(sw->P, sw->box, sw->theta, sw->ups, sw->pbest, sw->pbest_val, sw->gbest, sw->gbest + sw->dim, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "pso launch failed: %s", hipGetErrorString(e));
    for (int i = 0; i < n; ++i) sws[i]->iteration += 1;
    if (gbest_vals) {
        for (int i = 0; i < n; ++i)
            HIP_TRY(hipMemcpyAsync(gbest_vals + i, sws[i]->gbest + sws[i]->dim, sizeof(double), hipMemcpyDeviceToHost,
                                   s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return SCS_OK;
}

// One iteration of the swarms of a search whose convergence is tracked on the
// device (conv[i], one record per swarm): a swarm whose record says converged
// is left as it is by every kernel of the step (move, evaluation, bests), and
// the swarm best kernel pushes each new best value and applies the rule.
// Queues only; the caller reads the records when it needs them.  Each swarm's
// iteration counter advances here; the caller winds back those that
// converged, so that they count the iterations they took.
int pso_step_swarms_tracked(scs_swarm* const* sws, int n, const scs_pso_params* prm, int prec,
                            const ConvRecord* conv, int32_t rung_it, hipStream_t s)
{
    if (!sws || n < 1 || !prm || !conv) return fail(SCS_EINVAL, "bad arguments");
    std::vector<scs_batch_item> items(n);
    std::vector<const int32_t*> frozen(n);
    for (int i = 0; i < n; ++i) {
        scs_swarm* sw = sws[i];
        if (!sw) return fail(SCS_EINVAL, "swarm %d is NULL", i);
        int rc = check_eps(prm, sw->dim);
        if (rc) return rc;
        items[i] = scs_batch_item{sw->ctx, sw->ctx ? sw->ctx->N : 0, 0, sw->P, sw->theta, sw->ups, nullptr};
        frozen[i] = conv[i].state + 1;
    }
    int rc = check_items(items.data(), n, prec);
    if (rc) return rc;
    scs_ctx* c0 = sws[0]->ctx;
    DevScope ds(c0->device);
    for (int i = 0; i < n; ++i) {
        scs_swarm* sw = sws[i];
        if (sw->iteration > 0)
            launch_pso_move(sw->P, sw->box, to_params(prm, sw->dim), sw->seed, sw->swarm_id, sw->iteration, sw->theta,
                            sw->vel, sw->pbest, sw->gbest, s, frozen[i]);
    }
    BatchSlot& b = c0->ring[c0->ring_next];
    c0->ring_next = (c0->ring_next + 1) % scs_ctx::kRing;
    if ((rc = slot_reserve(b, n))) return rc;
    if ((rc = run_batched(items.data(), n, prec, s, b, true, nullptr, nullptr, frozen.data()))) return rc;
    HIP_TRY(hipEventRecord(b.done, s));
    for (int i = 0; i < n; ++i) {
        scs_swarm* sw = sws[i];
        launch_pso_best(sw->P, sw->box, sw->theta, sw->ups, sw->pbest, sw->pbest_val, sw->gbest, sw->gbest + sw->dim, s,
                        &conv[i], rung_it);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "pso launch failed: %s", hipGetErrorString(e));
    for (int i = 0; i < n; ++i) sws[i]->iteration += 1;
    return SCS_OK;
}

// The iteration counter of a swarm (the tracked step's caller sets it back
// for a swarm that converged part way through the queued iterations).
uint32_t swarm_iteration(const scs_swarm* sw) { return sw->iteration; }
void set_swarm_iteration(scs_swarm* sw, uint32_t it) { sw->iteration = it; }
int ctx_device(const scs_ctx* c) { return c->device; }
// A swarm's device arrays: theta, vel, pbest [P][D], pbest_val [P], gbest [D + 1].
void swarm_arrays(scs_swarm* sw, double** theta, double** vel, double** pbest, double** pbest_val, double** gbest)
{
    *theta = sw->theta;
    *vel = sw->vel;
    *pbest = sw->pbest;
    *pbest_val = sw->pbest_val;
    *gbest = sw->gbest;
}

extern "C" int scs_swarm_read(scs_swarm* sw, double* theta, double* vel, double* pbest, double* pbest_val,
                              double* gbest, double* gbest_val, uint32_t* iteration)
{
    if (!sw) return fail(SCS_EINVAL, "swarm is NULL");
    DevScope ds(sw->ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    const int D = sw->dim;
    const size_t nb = sizeof(double) * D * sw->P;
    if (theta) HIP_TRY(hipMemcpy(theta, sw->theta, nb, hipMemcpyDeviceToHost));
    if (vel) HIP_TRY(hipMemcpy(vel, sw->vel, nb, hipMemcpyDeviceToHost));
    if (pbest) HIP_TRY(hipMemcpy(pbest, sw->pbest, nb, hipMemcpyDeviceToHost));
    if (pbest_val) HIP_TRY(hipMemcpy(pbest_val, sw->pbest_val, sizeof(double) * sw->P, hipMemcpyDeviceToHost));
    double g[kThetaMax + 1];
    HIP_TRY(hipMemcpy(g, sw->gbest, sizeof(double) * (D + 1), hipMemcpyDeviceToHost));
    if (gbest) memcpy(gbest, g, sizeof(double) * D);
    if (gbest_val) *gbest_val = g[D];
    if (iteration) *iteration = sw->iteration;
    return SCS_OK;
}

extern "C" int scs_swarm_write(scs_swarm* sw, const double* theta, const double* vel, const double* pbest,
                               const double* pbest_val, const double* gbest, double gbest_val, uint32_t iteration)
{
    if (!sw || !theta || !vel || !pbest || !pbest_val || !gbest) return fail(SCS_EINVAL, "NULL argument");
    DevScope ds(sw->ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    const int D = sw->dim;
    const size_t nb = sizeof(double) * D * sw->P;
    HIP_TRY(hipMemcpy(sw->theta, theta, nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sw->vel, vel, nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sw->pbest, pbest, nb, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sw->pbest_val, pbest_val, sizeof(double) * sw->P, hipMemcpyHostToDevice));
    double g[kThetaMax + 1];
    memcpy(g, gbest, sizeof(double) * D);
    g[D] = gbest_val;
    HIP_TRY(hipMemcpy(sw->gbest, g, sizeof(double) * (D + 1), hipMemcpyHostToDevice));
    sw->iteration = iteration;
    return SCS_OK;
}

extern "C" int scs_theta_dim(const scs_ctx* c, int32_t* dim)
{
    int rc = check_ready(const_cast<scs_ctx*>(c));
    if (rc) return rc;
    if (!dim) return fail(SCS_EINVAL, "dim is NULL");
    *dim = theta_dim(c);
    return SCS_OK;
}

extern "C" int scs_ctx_info(const scs_ctx* c, int32_t* dim, int32_t* N, int32_t* n_chan, int64_t* K)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (dim) *dim = theta_dim(c);
    if (N) *N = c->N;
    if (n_chan) *n_chan = c->has_data ? c->g.nch : 0;
    if (K) *K = c->has_data ? c->g.K : 0;
    return SCS_OK;
}

extern "C" int scs_swarm_device_ptrs(scs_swarm* sw, double** theta, double** ups)
{
    if (!sw) return fail(SCS_EINVAL, "swarm is NULL");
    if (theta) *theta = sw->theta;
    if (ups) *ups = sw->ups;
    return SCS_OK;
}

extern "C" int scs_pso_move(int64_t P, int32_t dim, double* theta, double* vel, const double* pbest,
                            const double* gbest, const scs_pso_params* prm, const double* lo, const double* hi,
                            const int32_t* periodic, uint64_t seed, uint32_t swarm_id, uint32_t iteration, void* stream)
{
    if (P < 0 || !prm || !lo || !hi) return fail(SCS_EINVAL, "bad arguments");
    if (P == 0) return SCS_OK;
    if (!theta || !vel || !pbest || !gbest) return fail(SCS_EINVAL, "NULL buffer");
    PsoBox box;
    int rc = make_box(lo, hi, periodic, dim, &box);
    if (rc || (rc = check_eps(prm, dim))) return rc;
    launch_pso_move(P, box, to_params(prm, dim), seed, swarm_id, iteration, theta, vel, pbest, gbest,
                    (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    return SCS_OK;
}

extern "C" int scs_pso_best(int64_t P, int32_t dim, const double* theta, const double* vals, const double* lo,
                            const double* hi, const int32_t* periodic, double* pbest, double* pbest_val, double* gbest,
                            double* gbest_val, void* stream)
{
    if (P < 0 || !lo || !hi) return fail(SCS_EINVAL, "bad arguments");
    if (P == 0) return SCS_OK;
    if (!theta || !vals || !pbest || !pbest_val || !gbest || !gbest_val) return fail(SCS_EINVAL, "NULL buffer");
    PsoBox box;
    int rc = make_box(lo, hi, periodic, dim, &box);
    if (rc) return rc;
    launch_pso_best(P, box, theta, vals, pbest, pbest_val, gbest, gbest_val, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    return SCS_OK;
}
