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
#include <mutex>
#include <sstream>
#include <string>
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

static int device_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (g_dev_ready[device]) return SCS_OK;
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
    double* coef = nullptr;
    int32_t* klo = nullptr;
    int32_t* khi = nullptr;
    int8_t* lg = nullptr;
    int32_t* bounds = nullptr;
    double* rec = nullptr;
    // host-pointer staging
    int64_t capStage = 0;
    double* stage = nullptr;
    int64_t P_last = 0;
    int N_last = 0;
    // support-order permutation (radix sort of (k_hi, k_lo))
    int64_t capSort = 0;
    uint64_t* keys = nullptr;  // [2P]
    int32_t* idx = nullptr;    // [P]
    int32_t* perm = nullptr;   // [P]
    int64_t capTemp = 0;
    unsigned char* temp = nullptr;
};

struct TuneChoice {
    int waves = 4;
    int CB = 16;
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
    double zscale32 = 1.0, hscale32 = 1.0;  // undo the FP32 table scaling
    double* gtab = nullptr;  // basis Taylor tables, every sub-block level
    int64_t gtab_cap = 0;
    int64_t gtab_off[kMaxLevel] = {0};
    bool gtab_ok = false;
    unsigned long long* counters = nullptr;  // evals_support, evals_band, unresolved
    std::map<int, Workspace> ws;             // slot -> workspace
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
};

static int build_gtab(scs_ctx* c);

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
    hipFree(w.stage);
    hipFree(w.keys);
    hipFree(w.idx);
    hipFree(w.perm);
    hipFree(w.temp);
    w = Workspace();
}

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
    if (hipMalloc((void**)&c->counters, 3 * sizeof(unsigned long long)) != hipSuccess) {
        delete c;
        return fail(SCS_ENOMEM, "counter allocation failed");
    }
    launch_fill_u64(c->counters, 3, 0ULL, nullptr);
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
    for (auto& e : c->ev) {
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    hipFree(c->b64);
    hipFree(c->b32);
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
    if (n_chan != 1 && n_chan != 2) return fail(SCS_EINVAL, "n_chan must be 1 or 2 (got %d)", n_chan);
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
    if (hipMalloc((void**)&c->b64, sizeof(double) * 3 * nd) != hipSuccess ||
        hipMalloc((void**)&c->b32, sizeof(float) * 3 * nd) != hipSuccess) {
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
    hipError_t e3 = hipDeviceSynchronize();
    hipFree(dd_);
    hipFree(dp);
    if (e3 != hipSuccess) return fail(SCS_EDEVICE, "bin precompute failed: %s", hipGetErrorString(e3));
    c->has_data = true;
    c->gtab_ok = false;
    if (c->has_model && ((c->m.response == 1) != (n_chan == 2))) c->has_model = false;
    if (c->has_model) return build_gtab(c);
    return SCS_OK;
}

extern "C" int scs_set_model(scs_ctx* c, const scs_model* m)
{
    if (!c || !m) return fail(SCS_EINVAL, "NULL argument");
    if (!c->has_data) return fail(SCS_ESTATE, "load data before setting the model");
    if (m->pn_order < 0 || m->pn_order > 7) return fail(SCS_EINVAL, "pn_order must be 0..7");
    if (m->response != SCS_RESP_NONE && m->response != SCS_RESP_LISA_LF_AE) return fail(SCS_EINVAL, "bad response");
    if ((m->response == SCS_RESP_LISA_LF_AE) != (c->g.nch == 2))
        return fail(SCS_EINVAL, "response %d does not match %d loaded channels", m->response, c->g.nch);
    if (m->support != SCS_SUPPORT_FULL && m->support != SCS_SUPPORT_TOBS) return fail(SCS_EINVAL, "bad support");
    int L = m->block_len ? m->block_len : 512;
    if (L < 16 || L > 512 || (L & (L - 1))) return fail(SCS_EINVAL, "block_len must be a power of 2 in 16..512");
    if (m->t_obs < 0.0 || !std::isfinite(m->t_obs)) return fail(SCS_EINVAL, "bad t_obs");
    c->m.pn_order = m->pn_order;
    c->m.response = m->response;
    c->m.support = m->support;
    c->m.t_obs = m->t_obs > 0.0 ? m->t_obs : 1.0 / c->g.df;
    double oc = m->orbit_phase0 / (2.0 * M_PI);
    c->m.orb0_cyc = oc - std::floor(oc);
    c->m.cart0 = m->cartwheel_phase0;
    c->L = L;
    int lg = 0;
    while ((1 << lg) < L) ++lg;
    c->lg_max = lg;
    c->has_model = true;
    DevScope ds(c->device);
    return build_gtab(c);
}

extern "C" int scs_define_segmentation(scs_ctx* c, int32_t N, int32_t mode, int32_t G, const int64_t* edges)
{
    if (!c) return fail(SCS_EINVAL, "ctx is NULL");
    if (N < 1) return fail(SCS_EINVAL, "N must be >= 1");
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
    o << "K" << c->g.K << "_c" << c->g.nch << "_L" << c->L << "_p" << prec << "_P" << cls(P) << "_N" << cls(N);
    return o.str();
}

static TuneChoice choose(const scs_ctx* c, int64_t P, int N, int prec)
{
    if (c->has_override) return c->override_choice;
    auto it = c->tune.find(tune_key(c, P, N, prec));
    if (it != c->tune.end()) return it->second;
    TuneChoice t;
    // default: 4 waves (256 particles) per workgroup; chunks of ~8192 bins,
    // fewer waves when the swarm is small so that the chip still fills
    t.waves = P >= 4096 ? 4 : (P >= 1024 ? 2 : 1);
    t.CB = std::max(1, 8192 / c->L);
    return t;
}

struct Plan {
    int waves, CB;
    int64_t cbins, n_chunks, n_groups, n_tiles;
};

static Plan make_plan(const scs_ctx* c, int64_t P, const TuneChoice& t)
{
    Plan pl;
    pl.waves = t.waves;
    pl.CB = t.CB;
    pl.cbins = (int64_t)c->L * t.CB;
    pl.n_chunks = (c->g.K + pl.cbins - 1) / pl.cbins;
    pl.n_groups = (P + 64 * t.waves - 1) / (64 * t.waves);
    pl.n_tiles = pl.n_chunks * pl.n_groups;
    return pl;
}

static int64_t pad64(int64_t v) { return (v + 63) / 64 * 64; }

// Swarms of at least this many particles are evaluated in support order.
static constexpr int64_t kSortMin = 128;

static size_t ws_bytes(const scs_ctx* c, int64_t P, int N, const Plan& pl)
{
    const int64_t Pp = pad64(std::max<int64_t>(P, 1));
    size_t b = 0;
    b += sizeof(double) * (size_t)kCoefStride * Pp;
    b += (sizeof(int32_t) * 2 + 1) * (size_t)Pp;
    b += sizeof(int32_t) * (size_t)P * (N + 1);
    b += sizeof(double) * (size_t)pl.n_chunks * 7 * Pp;
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
    if ((rc = grow(&w.bounds, &w.capBounds, P * (int64_t)(N + 1)))) return rc;
    if ((rc = grow(&w.rec, &w.capRec, pl.n_chunks * 7 * w.capP))) return rc;
    if (P >= kSortMin && P > w.capSort) {
        int64_t c1 = 0, c2 = 0, c3 = 0;
        hipFree(w.keys);
        hipFree(w.idx);
        hipFree(w.perm);
        w.keys = nullptr;
        w.idx = w.perm = nullptr;
        w.capSort = 0;
        if ((rc = grow(&w.keys, &c1, 2 * w.capP)) || (rc = grow(&w.idx, &c2, w.capP)) || (rc = grow(&w.perm, &c3, w.capP)))
            return rc;
        w.capSort = w.capP;
        if ((rc = grow(&w.temp, &w.capTemp, (int64_t)sort_temp_bytes(w.capP)))) return rc;
    }
    return SCS_OK;
}

// Queue the whole evaluation on stream s (device pointers).
static int run_eval(scs_ctx* c, Workspace& w, int64_t P, int N, const double* theta, int prec, double* ups,
                    double* seg, hipStream_t s, const TuneChoice* force = nullptr)
{
    const TuneChoice t = force ? *force : choose(c, P, N, prec);
    const Plan pl = make_plan(c, P, t);
    int rc = ensure_ws(c, w, P, N, pl);
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
    launch_prologue(pa, s);
    const int32_t* perm = nullptr;
    if (P >= kSortMin && w.perm) {
        int kb = 32;
        while (kb < 64 && ((int64_t)1 << (kb - 32)) <= c->g.K) ++kb;
        hipError_t e = launch_sort_perm(P, w.klo, w.khi, w.keys, w.idx, w.perm, w.temp, (size_t)w.capTemp, kb, s);
        if (e != hipSuccess) return fail(SCS_EDEVICE, "support sort failed: %s", hipGetErrorString(e));
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
    if (c->mode == SCS_SEG_EXPLICIT && N != c->N) return fail(SCS_EINVAL, "EXPLICIT edges were defined for N = %d", c->N);
    launch_bounds(ba, s);
    MainArgs ma{};
    ma.g = c->g;
    ma.m = c->m;
    ma.p0 = 0;
    ma.P_end = P;
    ma.stride = w.capP;
    ma.N = N;
    ma.L = c->L;
    ma.CB = pl.CB;
    ma.chunk0 = 0;
    ma.n_groups = pl.n_groups;
    ma.n_tiles = pl.n_tiles;
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
    ma.perm = perm;
    ma.rec = w.rec;
    ma.seg = seg;
    ma.zscale32 = c->zscale32;
    ma.hscale32 = c->hscale32;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof) {
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        hipEventRecord(e0, s);
    }
    launch_main(ma, pl.waves, prec == SCS_PREC_MIXED, s);
    if (c->prof) {
        hipEventRecord(e1, s);
        c->ev.emplace_back(e0, e1);
    }
    FinalArgs fa{};
    fa.K = c->g.K;
    fa.df = c->g.df;
    fa.p0 = 0;
    fa.P_end = P;
    fa.N = N;
    fa.cbins = pl.cbins;
    fa.chunk0 = 0;
    fa.rec_stride = w.capP;
    fa.klo = w.klo;
    fa.khi = w.khi;
    fa.lg = w.lg;
    fa.bounds = w.bounds;
    fa.perm = perm;
    fa.rec = w.rec;
    fa.ups = ups;
    fa.seg = seg;
    launch_finalize(fa, s);
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
    const int64_t need = P * 8 + P + (seg ? P * (int64_t)N * 3 : 0);
    if ((rc = grow(&w.stage, &w.capStage, std::max<int64_t>(need, 1)))) return rc;
    double* dth = w.stage;
    double* dup = dth + P * 7;
    double* dseg = seg ? dup + P : nullptr;
    HIP_TRY(hipMemcpyAsync(dth, theta, sizeof(double) * 7 * P, hipMemcpyHostToDevice, s));
    if ((rc = run_eval(c, w, P, N, dth, prec, dup, dseg, s))) return rc;
    HIP_TRY(hipMemcpyAsync(ups, dup, sizeof(double) * P, hipMemcpyDeviceToHost, s));
    if (seg) HIP_TRY(hipMemcpyAsync(seg, dseg, sizeof(double) * P * N * 3, hipMemcpyDeviceToHost, s));
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
    if ((rc = grow(&w.stage, &w.capStage, 7 + nout))) return rc;
    const double* dth = theta;
    double* dh = h_ri;
    if (mem_kind == SCS_MEM_HOST) {
        HIP_TRY(hipMemcpyAsync(w.stage, theta, sizeof(double) * 7, hipMemcpyHostToDevice, s));
        dth = w.stage;
        dh = w.stage + 7;
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
    launch_waveform(ma, dh, s);
    if (mem_kind == SCS_MEM_HOST) {
        HIP_TRY(hipMemcpyAsync(h_ri, dh, sizeof(double) * nout, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "waveform launch failed: %s", hipGetErrorString(e));
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
    for (auto& e : c->ev) {
        HIP_TRY(hipEventSynchronize(e.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
        c->prof_ms += ms;
        c->prof_launches += 1;
        hipEventDestroy(e.first);
        hipEventDestroy(e.second);
    }
    c->ev.clear();
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
    if (P < 0 || N < 1) return fail(SCS_EINVAL, "bad P or N");
    const TuneChoice t = choose(c, P, N, prec);
    *bytes = ws_bytes(c, P, N, make_plan(c, P, t));
    return SCS_OK;
}

// ---------------------------------------------------------------- batched
// Items are evaluated back to back on one stream; every item owns a
// workspace slot of its context, so items may share a context.
extern "C" int scs_evaluate_batched(const scs_batch_item* items, int32_t n_items, int32_t prec, void* stream)
{
    if (!items || n_items < 0) return fail(SCS_EINVAL, "bad items");
    if (prec != SCS_PREC_FP64 && prec != SCS_PREC_MIXED) return fail(SCS_EINVAL, "bad precision");
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n_items; ++i) {
        const scs_batch_item& it = items[i];
        int rc = check_ready(it.ctx);
        if (rc) return rc;
        if (it.N < 1 || it.P < 0 || (it.P > 0 && (!it.theta || !it.ups)))
            return fail(SCS_EINVAL, "item %d: bad N, P or pointers", i);
    }
    for (int i = 0; i < n_items; ++i) {
        const scs_batch_item& it = items[i];
        DevScope ds(it.ctx->device);
        int rc = run_eval(it.ctx, it.ctx->ws[1 + i], it.P, it.N, it.theta, prec, it.ups, it.seg, s);
        if (rc) return rc;
    }
    return SCS_OK;
}

struct scs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

extern "C" int scs_graph_create(scs_graph** out, const scs_batch_item* items, int32_t n_items, int32_t prec)
{
    if (!out || !items || n_items < 1) return fail(SCS_EINVAL, "bad arguments");
    *out = nullptr;
    const int dev = items[0].ctx ? items[0].ctx->device : 0;
    DevScope ds(dev);
    // first call outside capture: allocates every workspace
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    int rc = scs_evaluate_batched(items, n_items, prec, s);
    if (rc) {
        hipStreamDestroy(s);
        return rc;
    }
    HIP_TRY(hipStreamSynchronize(s));
    scs_graph* g = new scs_graph();
    g->device = dev;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = scs_evaluate_batched(items, n_items, prec, s);
        e = hipStreamEndCapture(s, &g->graph);
    }
    if (e == hipSuccess && rc == SCS_OK) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    hipStreamDestroy(s);
    if (e != hipSuccess || rc != SCS_OK) {
        if (g->exec) hipGraphExecDestroy(g->exec);
        if (g->graph) hipGraphDestroy(g->graph);
        delete g;
        return rc ? rc : fail(SCS_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return SCS_OK;
}

extern "C" int scs_graph_launch(scs_graph* g, void* stream)
{
    if (!g) return fail(SCS_EINVAL, "graph is NULL");
    DevScope ds(g->device);
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return SCS_OK;
}

extern "C" int scs_graph_destroy(scs_graph* g)
{
    if (!g) return SCS_OK;
    DevScope ds(g->device);
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    delete g;
    return SCS_OK;
}

// ---------------------------------------------------------------- autotuner
static void load_cache(scs_ctx* c, const char* path)
{
    std::ifstream f(path);
    std::string key;
    int w, cb;
    while (f >> key >> w >> cb) {
        if (w == 1 || w == 2 || w == 4) c->tune[key] = TuneChoice{w, std::max(1, cb)};
    }
}

static void save_cache(const scs_ctx* c, const char* path)
{
    std::map<std::string, TuneChoice> all;
    {
        std::ifstream f(path);
        std::string key;
        int w, cb;
        while (f >> key >> w >> cb) all[key] = TuneChoice{w, cb};
    }
    for (auto& kv : c->tune) all[kv.first] = kv.second;
    std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream o(tmp);
        for (auto& kv : all) o << kv.first << " " << kv.second.waves << " " << kv.second.CB << "\n";
    }
    std::rename(tmp.c_str(), path);
}

extern "C" int scs_autotune(scs_ctx* c, int64_t P, const double* theta_dev, int32_t N, int32_t prec,
                            const char* cache_path)
{
    int rc = check_ready(c);
    if (rc) return rc;
    if (P < 1 || N < 1) return fail(SCS_EINVAL, "bad P or N");
    const std::string key = tune_key(c, P, N, prec);
    if (cache_path) {
        load_cache(c, cache_path);
        if (c->tune.count(key)) return SCS_OK;
    }
    if (!theta_dev) return fail(SCS_EINVAL, "theta is NULL");
    DevScope ds(c->device);
    const int64_t Pt = P;
    const double* th = theta_dev;
    double* ups = nullptr;
    HIP_TRY(hipMalloc((void**)&ups, sizeof(double) * Pt));
    hipStream_t s;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    Workspace tw;
    TuneChoice best;
    double best_ms = 1e300;
    const int cbs[] = {4, 8, 16, 32, 64};
    const int wvs[] = {1, 2, 4};
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    for (int wv : wvs)
        for (int cb0 : cbs) {
            TuneChoice t{wv, std::max(1, cb0 * 512 / c->L)};
            if ((rc = run_eval(c, tw, Pt, N, th, prec, ups, nullptr, s, &t))) break;
            hipEventRecord(e0, s);
            for (int r = 0; r < 3; ++r) run_eval(c, tw, Pt, N, th, prec, ups, nullptr, s, &t);
            hipEventRecord(e1, s);
            hipEventSynchronize(e1);
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            if (ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamDestroy(s);
    free_ws(tw);
    hipFree(ups);
    if (rc) return rc;
    c->tune[key] = best;
    if (cache_path) save_cache(c, cache_path);
    return SCS_OK;
}

// ---------------------------------------------------------------- swarms
struct scs_swarm {
    scs_ctx* ctx = nullptr;
    int64_t P = 0;
    double *theta = nullptr, *vel = nullptr, *pbest = nullptr, *pbest_val = nullptr;
    double *gbest = nullptr, *ups = nullptr;  // gbest[7], gbest[7] = value
    PsoBox box{};
    uint64_t seed = 0;
    uint32_t swarm_id = 0;
    uint32_t iteration = 0;
};

static int make_box(const double* lo, const double* hi, const int32_t* periodic, PsoBox* box)
{
    for (int d = 0; d < 7; ++d) {
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
    if ((rc = make_box(lo, hi, periodic, &sw->box))) {
        delete sw;
        return rc;
    }
    DevScope ds(c->device);
    sw->ctx = c;
    sw->P = P;
    sw->seed = seed;
    sw->swarm_id = swarm_id;
    const size_t n7 = sizeof(double) * 7 * P;
    if (hipMalloc((void**)&sw->theta, n7) || hipMalloc((void**)&sw->vel, n7) || hipMalloc((void**)&sw->pbest, n7) ||
        hipMalloc((void**)&sw->pbest_val, sizeof(double) * P) || hipMalloc((void**)&sw->gbest, sizeof(double) * 8) ||
        hipMalloc((void**)&sw->ups, sizeof(double) * P)) {
        scs_swarm_destroy(sw);
        return fail(SCS_ENOMEM, "swarm allocation failed");
    }
    launch_pso_init(P, sw->box, seed, swarm_id, sw->theta, nullptr);
    launch_fill(sw->vel, 7 * P, 0.0, nullptr);
    launch_fill(sw->pbest, 7 * P, 0.0, nullptr);
    launch_fill(sw->pbest_val, P, -INFINITY, nullptr);
    launch_fill(sw->gbest, 7, 0.0, nullptr);
    launch_fill(sw->gbest + 7, 1, -INFINITY, nullptr);
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

static PsoParams to_params(const scs_pso_params* p)
{
    PsoParams q;
    q.omega = p->omega;
    q.phi_p = p->phi_p;
    q.phi_g = p->phi_g;
    for (int d = 0; d < 7; ++d) q.eps[d] = p->eps[d];
    return q;
}

extern "C" int scs_pso_step(scs_swarm* sw, const scs_pso_params* prm, int32_t prec, void* stream)
{
    if (!sw || !prm) return fail(SCS_EINVAL, "NULL argument");
    for (int d = 0; d < 7; ++d)
        if (!(prm->eps[d] >= 0.0)) return fail(SCS_EINVAL, "eps[%d] must be >= 0", d);
    scs_ctx* c = sw->ctx;
    int rc = check_ready(c);
    if (rc) return rc;
    DevScope ds(c->device);
    hipStream_t s = (hipStream_t)stream;
    if (sw->iteration > 0)
        launch_pso_move(sw->P, sw->box, to_params(prm), sw->seed, sw->swarm_id, sw->iteration, sw->theta, sw->vel,
                        sw->pbest, sw->gbest, s);
    if ((rc = run_eval(c, c->ws[0], sw->P, c->N, sw->theta, prec, sw->ups, nullptr, s))) return rc;
    launch_pso_best(sw->P, sw->box, sw->theta, sw->ups, sw->pbest, sw->pbest_val, sw->gbest, sw->gbest + 7, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "pso launch failed: %s", hipGetErrorString(e));
    sw->iteration += 1;
    return SCS_OK;
}

extern "C" int scs_swarm_read(scs_swarm* sw, double* theta, double* vel, double* pbest, double* pbest_val,
                              double* gbest, double* gbest_val, uint32_t* iteration)
{
    if (!sw) return fail(SCS_EINVAL, "swarm is NULL");
    DevScope ds(sw->ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    const size_t n7 = sizeof(double) * 7 * sw->P;
    if (theta) HIP_TRY(hipMemcpy(theta, sw->theta, n7, hipMemcpyDeviceToHost));
    if (vel) HIP_TRY(hipMemcpy(vel, sw->vel, n7, hipMemcpyDeviceToHost));
    if (pbest) HIP_TRY(hipMemcpy(pbest, sw->pbest, n7, hipMemcpyDeviceToHost));
    if (pbest_val) HIP_TRY(hipMemcpy(pbest_val, sw->pbest_val, sizeof(double) * sw->P, hipMemcpyDeviceToHost));
    double g[8];
    HIP_TRY(hipMemcpy(g, sw->gbest, sizeof g, hipMemcpyDeviceToHost));
    if (gbest) memcpy(gbest, g, sizeof(double) * 7);
    if (gbest_val) *gbest_val = g[7];
    if (iteration) *iteration = sw->iteration;
    return SCS_OK;
}

extern "C" int scs_swarm_write(scs_swarm* sw, const double* theta, const double* vel, const double* pbest,
                               const double* pbest_val, const double* gbest, double gbest_val, uint32_t iteration)
{
    if (!sw || !theta || !vel || !pbest || !pbest_val || !gbest) return fail(SCS_EINVAL, "NULL argument");
    DevScope ds(sw->ctx->device);
    HIP_TRY(hipDeviceSynchronize());
    const size_t n7 = sizeof(double) * 7 * sw->P;
    HIP_TRY(hipMemcpy(sw->theta, theta, n7, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sw->vel, vel, n7, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sw->pbest, pbest, n7, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(sw->pbest_val, pbest_val, sizeof(double) * sw->P, hipMemcpyHostToDevice));
    double g[8];
    memcpy(g, gbest, sizeof(double) * 7);
    g[7] = gbest_val;
    HIP_TRY(hipMemcpy(sw->gbest, g, sizeof g, hipMemcpyHostToDevice));
    sw->iteration = iteration;
    return SCS_OK;
}

extern "C" int scs_swarm_device_ptrs(scs_swarm* sw, double** theta, double** ups)
{
    if (!sw) return fail(SCS_EINVAL, "swarm is NULL");
    if (theta) *theta = sw->theta;
    if (ups) *ups = sw->ups;
    return SCS_OK;
}

extern "C" int scs_pso_move(int64_t P, double* theta, double* vel, const double* pbest, const double* gbest,
                            const scs_pso_params* prm, const double* lo, const double* hi, const int32_t* periodic,
                            uint64_t seed, uint32_t swarm_id, uint32_t iteration, void* stream)
{
    if (P < 0 || !prm || !lo || !hi) return fail(SCS_EINVAL, "bad arguments");
    if (P == 0) return SCS_OK;
    if (!theta || !vel || !pbest || !gbest) return fail(SCS_EINVAL, "NULL buffer");
    PsoBox box;
    int rc = make_box(lo, hi, periodic, &box);
    if (rc) return rc;
    launch_pso_move(P, box, to_params(prm), seed, swarm_id, iteration, theta, vel, pbest, gbest, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    return SCS_OK;
}

extern "C" int scs_pso_best(int64_t P, const double* theta, const double* vals, const double* lo, const double* hi,
                            const int32_t* periodic, double* pbest, double* pbest_val, double* gbest, double* gbest_val,
                            void* stream)
{
    if (P < 0 || !lo || !hi) return fail(SCS_EINVAL, "bad arguments");
    if (P == 0) return SCS_OK;
    if (!theta || !vals || !pbest || !pbest_val || !gbest || !gbest_val) return fail(SCS_EINVAL, "NULL buffer");
    PsoBox box;
    int rc = make_box(lo, hi, periodic, &box);
    if (rc) return rc;
    launch_pso_best(P, box, theta, vals, pbest, pbest_val, gbest, gbest_val, (hipStream_t)stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SCS_EDEVICE, "launch failed: %s", hipGetErrorString(e));
    return SCS_OK;
}
