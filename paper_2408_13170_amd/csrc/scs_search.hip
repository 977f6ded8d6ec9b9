// Hierarchical multi-swarm search (arXiv:2408.13170, Sec 3.1 - 3.2 and the PSO
// appendix app:PSO_params).  The swarms live on the device; every iteration
// is one batched step over the swarms still moving (their moves, ONE batched
// generate-and-reduce over all of their particles, their bests), and the
// convergence rule runs on the device too: the swarm best kernel keeps each
// swarm's last window + 1 best values and freezes a swarm that converged, so
// that every kernel of the later iterations leaves it as it is.  The host
// queues kConvBatch iterations at a time and then reads the swarms'
// convergence records (three integers each), instead of reading the best
// values back after every iteration.  It re-groups the particles between
// rungs with k-means.
//
//   rung:      Upsilon_N with the rung's N, equal-[h|h] edges, and the rung's
//              hyper-parameters and minimum speeds (tab:PSO_hyperparams);
//   converged: a swarm's best value gained no more than conv_tol over its
//              last conv_window iterations (2 over 50 in the paper); a
//              converged swarm stops moving until the rung ends;
//   regroup:   before every rung but the first, k-means on the positions of
//              all particles of all swarms (k = the initial number of
//              swarms); every non-empty cluster becomes a swarm; the number of
//              particles is conserved.  Positions, velocities and best
//              positions carry over; best values restart because the
//              objective changed.  A position outside the prior box scores
//              -inf, so best positions lie inside the box, and as attractors
//              they pull a cluster of particles that stand outside back in.
//              The swarm's best position starts at the best position of its
//              particle with the highest earlier best value.
//
// The re-grouping runs on the device too (k_features, k_kmeans: one
// workgroup runs the whole k-means, every sum in a fixed order); the host
// reads back the cluster count, sizes and top members.  scs_kmeans, the same
// k-means on host data, stays available to callers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/scs.h"
#include "scs_internal.hpp"

// scs_host.hip: one iteration of a search's swarms with convergence tracked
// on the device, and the swarms' iteration counters
int pso_step_swarms_tracked(scs_swarm* const* sws, int n, const scs_pso_params* prm, int prec,
                            const scs::ConvRecord* conv, int32_t rung_it, hipStream_t s);
uint32_t swarm_iteration(const scs_swarm* sw);
void set_swarm_iteration(scs_swarm* sw, uint32_t it);
int ctx_device(const scs_ctx* c);
void swarm_arrays(scs_swarm* sw, double** theta, double** vel, double** pbest, double** pbest_val, double** gbest);

// iterations queued between two reads of the convergence records
constexpr int kConvBatch = 8;

namespace {

// splitmix64 (Steele, Lea & Flood 2014): the k-means++ draws.
struct SplitMix {
    uint64_t s;
    uint64_t next()
    {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((double)(next() >> 11) + 0.5) * 0x1p-53; }  // (0, 1)
};

}  // namespace

// The library's error record (scs_last_error), defined beside the other entry points.
int scs_record_error(int code, const char* msg);
static int err(int code, const char* msg) { return scs_record_error(code, msg); }

struct scs_search {
    scs_ctx* ctx = nullptr;
    scs_search_params p{};
    int dim = 7;  // theta entries of the context (7, or 8 with e0)
    double lo[8], hi[8];
    int32_t per[8];
    std::vector<scs_swarm*> swarms;
    std::vector<int64_t> sizes;
    uint32_t next_id = 0;
    int rungs_done = 0;
    // device convergence records, one per swarm slot (at most n_swarms
    // swarms exist at a time): ring [n][window + 1], state [n][3]
    double* d_ring = nullptr;
    int32_t* d_state = nullptr;
    int32_t* h_state = nullptr;  // pinned copy of d_state
    double* h_best = nullptr;    // pinned: the swarms' best values
};

// k-means with k-means++ seeding (Arthur & Vassilvitskii 2007) and Lloyd
// iterations until no label changes (or iters); squared Euclidean distance.
// Ties go to the lower cluster index.  Empty clusters are dropped and the
// labels renumbered in order of first appearance of the kept clusters.
extern "C" int scs_kmeans(const double* x, int64_t n, int32_t dim, int32_t k, int32_t iters, uint64_t seed,
                          int32_t* labels, double* centers, int32_t* k_out)
{
    if (!x || !labels || !k_out || n < 1 || dim < 1 || k < 1 || iters < 1) return err(SCS_EINVAL, "bad k-means arguments");
    k = (int32_t)std::min<int64_t>(k, n);
    std::vector<double> c((size_t)k * dim), d2(n, std::numeric_limits<double>::infinity());
    SplitMix rng{seed};
    auto dist = [&](int64_t i, const double* ctr) {
        double s = 0.0;
        for (int j = 0; j < dim; ++j) {
            const double t = x[i * dim + j] - ctr[j];
            s += t * t;
        }
        return s;
    };
    // seeding: first centre uniform, the others with probability ~ D^2
    int64_t first = (int64_t)(rng.uniform() * (double)n);
    first = std::min<int64_t>(first, n - 1);
    std::copy(x + first * dim, x + (first + 1) * dim, c.begin());
    for (int m = 1; m < k; ++m) {
        double tot = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            d2[i] = std::min(d2[i], dist(i, &c[(size_t)(m - 1) * dim]));
            tot += d2[i];
        }
        int64_t pick = n - 1;
        if (tot > 0.0) {
            const double u = rng.uniform() * tot;
            double acc = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                acc += d2[i];
                if (acc >= u) {
                    pick = i;
                    break;
                }
            }
        } else {
            pick = (int64_t)(rng.uniform() * (double)n);
            pick = std::min<int64_t>(pick, n - 1);
        }
        std::copy(x + pick * dim, x + (pick + 1) * dim, c.begin() + (size_t)m * dim);
    }
    std::vector<int32_t> lab(n, -1);
    std::vector<double> sum((size_t)k * dim);
    std::vector<int64_t> cnt(k);
    for (int it = 0; it < iters; ++it) {
        bool changed = false;
        for (int64_t i = 0; i < n; ++i) {
            int best = 0;
            double bd = dist(i, &c[0]);
            for (int m = 1; m < k; ++m) {
                const double dm = dist(i, &c[(size_t)m * dim]);
                if (dm < bd) {
                    bd = dm;
                    best = m;
                }
            }
            if (lab[i] != best) {
                lab[i] = best;
                changed = true;
            }
        }
        if (!changed && it > 0) break;
        std::fill(sum.begin(), sum.end(), 0.0);
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int64_t i = 0; i < n; ++i) {
            ++cnt[lab[i]];
            for (int j = 0; j < dim; ++j) sum[(size_t)lab[i] * dim + j] += x[i * dim + j];
        }
        for (int m = 0; m < k; ++m)
            if (cnt[m] > 0)
                for (int j = 0; j < dim; ++j) c[(size_t)m * dim + j] = sum[(size_t)m * dim + j] / (double)cnt[m];
    }
    // drop empty clusters, renumber by first appearance
    std::vector<int32_t> map(k, -1);
    int32_t kk = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (map[lab[i]] < 0) map[lab[i]] = kk++;
        labels[i] = map[lab[i]];
    }
    if (centers)
        for (int m = 0; m < k; ++m)
            if (map[m] >= 0) std::copy(&c[(size_t)m * dim], &c[(size_t)(m + 1) * dim], centers + (size_t)map[m] * dim);
    *k_out = kk;
    return SCS_OK;
}

extern "C" int scs_search_create(scs_ctx* ctx, const scs_search_params* p, const double* lo, const double* hi,
                                 const int32_t* periodic, scs_search** out)
{
    if (!ctx || !p || !lo || !hi || !out) return err(SCS_EINVAL, "NULL argument");
    if (p->n_swarms < 1 || p->n_swarms > 1024 || p->particles < 1 || p->G < 1 || p->conv_window < 1 || p->kmeans_iters < 1 ||
        !(p->conv_tol >= 0.0) || (p->prec != SCS_PREC_FP64 && p->prec != SCS_PREC_MIXED))
        return err(SCS_EINVAL, "bad search parameters");
    scs_search* s = new (std::nothrow) scs_search();
    if (!s) return err(SCS_ENOMEM, "host allocation failed");
    s->ctx = ctx;
    s->p = *p;
    int32_t dim = 0;
    int rc0 = scs_theta_dim(ctx, &dim);
    if (rc0) {
        scs_search_destroy(s);
        return rc0;
    }
    s->dim = dim;
    {
        const int n = p->n_swarms;
        const size_t ring = sizeof(double) * (size_t)n * (p->conv_window + 1);
        if (hipSetDevice(ctx_device(ctx)) != hipSuccess || hipMalloc((void**)&s->d_ring, ring) != hipSuccess ||
            hipMalloc((void**)&s->d_state, sizeof(int32_t) * 3 * n) != hipSuccess ||
            hipHostMalloc((void**)&s->h_state, sizeof(int32_t) * 3 * n, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&s->h_best, sizeof(double) * n, hipHostMallocDefault) != hipSuccess) {
            scs_search_destroy(s);
            return err(SCS_ENOMEM, "search: convergence records could not be allocated");
        }
    }
    for (int d = 0; d < dim; ++d) {
        s->lo[d] = lo[d];
        s->hi[d] = hi[d];
        s->per[d] = periodic ? periodic[d] : 0;
    }
    for (int i = 0; i < p->n_swarms; ++i) {
        scs_swarm* sw = nullptr;
        int rc = scs_swarm_create(ctx, &sw, p->particles, s->lo, s->hi, s->per, p->seed, s->next_id++);
        if (rc) {
            scs_search_destroy(s);
            return rc;
        }
        s->swarms.push_back(sw);
        s->sizes.push_back(p->particles);
    }
    *out = s;
    return SCS_OK;
}

namespace {

constexpr int kKmThreads = 1024;  // one workgroup runs a re-grouping's whole k-means
constexpr int kKmWaves = kKmThreads / 64;
constexpr int kMaxFeat = 16;  // features per particle: at most 8 dimensions, 2 each when periodic

struct FeatBox {
    double lo[8], hi[8];
    int32_t per[8];
    int32_t D;
};

// The k-means input: each dimension of a position scaled to the prior box,
// a periodic one as the point (cos, sin) / 2 pi of its angle on the circle,
// so that a full turn spans about as much as the box.
__global__ void k_features(int64_t P, FeatBox b, int F, const double* __restrict__ th, double* __restrict__ f)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    int j = 0;
    for (int d = 0; d < b.D; ++d) {
        const double w = b.hi[d] - b.lo[d];
        const double u = w > 0.0 ? (th[i * b.D + d] - b.lo[d]) / w : 0.0;
        if (b.per[d]) {
            const double a = 2.0 * M_PI * u;
            f[i * F + j++] = cos(a) / (2.0 * M_PI);
            f[i * F + j++] = sin(a) / (2.0 * M_PI);
        } else {
            f[i * F + j++] = u;
        }
    }
}

struct KmArgs {
    int64_t P;
    int32_t F, k, iters;
    const double* x;      // [P][F] features
    const double* draws;  // [k] the k-means++ draws, uniform in (0, 1), in the order they are used
    const double* pv;     // [P] (nullable) the particles' best values so far, for the top members
    double* d2;           // [P] scratch
    int32_t* lab;         // [P] scratch: cluster labels
    double* cen;          // [k][F] scratch: centres
    int32_t* inv;         // [k] scratch: old label of each kept cluster
    int32_t* map;         // [k] scratch: new label of each old one (-1: dropped)
    int32_t* info;        // out: [0] clusters kept kk, [1 + c] size of kept cluster c, [1 + k + c] its top member
    int32_t* labels;      // out (nullable): [P] labels, kept clusters numbered by first appearance
    double* centers;      // out (nullable): [kk][F] their centres
    int32_t* order;       // out (nullable, with pv): [P] particle indices, cluster by cluster, ascending within each
};

// Sums over the workgroup of v[j] for j < n (n <= kMaxFeat) and, with
// count, of v[kMaxFeat], in a fixed order (wave shuffles, then the waves in
// turn), so that a run gives the same totals every time; the totals land in
// out[j] (and out[kMaxFeat]).  Every index is a constant after unrolling, so
// v stays in registers.
__device__ void wg_sums(const double* v, int n, bool count, double* red, double* out)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < kMaxFeat + 1; ++j) {
        if (j < n || (count && j == kMaxFeat)) {
            double x = v[j];
            for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
            if (lane == 0) red[w * (kMaxFeat + 1) + j] = x;
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    if (j < n || (count && j == kMaxFeat)) {
        double t = 0.0;
        for (int q = 0; q < kKmWaves; ++q) t += red[q * (kMaxFeat + 1) + j];
        out[j] = t;
    }
    __syncthreads();
}

// k-means (Arthur & Vassilvitskii 2007 seeding, then Lloyd iterations until
// no label changes, at most iters), then the kept clusters in order of first
// appearance and the particles grouped by cluster: the steps of scs_kmeans
// and of the host re-grouping, on the device.  Each thread takes a run of
// consecutive particles; every sum is formed in a fixed order.
__global__ __launch_bounds__(kKmThreads) void k_kmeans(KmArgs a)
{
    __shared__ double red[kKmWaves * (kMaxFeat + 1)];
    __shared__ double tot[kMaxFeat + 1];
    __shared__ double part[kKmThreads];
    __shared__ int32_t ipart[kKmThreads];
    __shared__ double bvs[kKmThreads];
    __shared__ unsigned long long s_min, s_cnt;
    __shared__ int s_changed;
    const int t = threadIdx.x;
    const int64_t P = a.P;
    const int F = a.F, k = a.k;
    const int64_t C = (P + kKmThreads - 1) / kKmThreads;
    const int64_t i0 = t * C < P ? t * C : P, i1 = i0 + C < P ? i0 + C : P;
    const double* x = a.x;
    auto dist = [&](int64_t i, const double* c) {
        double s = 0.0;
        for (int j = 0; j < F; ++j) {
            const double d = x[i * F + j] - c[j];
            s += d * d;
        }
        return s;
    };
    auto clamp_pick = [&](double u) {
        const int64_t q = (int64_t)(u * (double)P);
        return q < P - 1 ? q : P - 1;
    };
    // ---- seeding: the first centre a uniform pick, each next one a pick
    // with probability proportional to the squared distance to the nearest
    // centre so far
    if (t < F) a.cen[t] = x[clamp_pick(a.draws[0]) * F + t];
    for (int64_t i = i0; i < i1; ++i) a.d2[i] = INFINITY;
    __syncthreads();
    for (int m = 1; m < k; ++m) {
        double pl = 0.0;
        const double* c = a.cen + (int64_t)(m - 1) * F;
        for (int64_t i = i0; i < i1; ++i) {
            const double d = dist(i, c);
            if (d < a.d2[i]) a.d2[i] = d;
            pl += a.d2[i];
        }
        part[t] = pl;
        double v1[kMaxFeat + 1];
#pragma unroll
        for (int j = 0; j < kMaxFeat + 1; ++j) v1[j] = 0.0;
        v1[0] = pl;
        wg_sums(v1, 1, false, red, tot);
        const double total = tot[0];
        int64_t pick;
        if (total > 0.0) {
            const double u = a.draws[m] * total;
            if (t == 0) {  // exclusive prefix sums of the runs, in thread order
                double acc = 0.0;
                for (int q = 0; q < kKmThreads; ++q) {
                    const double v = part[q];
                    part[q] = acc;
                    acc += v;
                }
                s_min = (unsigned long long)P;
            }
            __syncthreads();
            // the first particle whose running sum reaches u
            double acc = part[t];
            for (int64_t i = i0; i < i1; ++i) {
                acc += a.d2[i];
                if (acc >= u) {
                    atomicMin(&s_min, (unsigned long long)i);
                    break;
                }
            }
            __syncthreads();
            pick = (int64_t)s_min < P ? (int64_t)s_min : P - 1;
        } else {
            pick = clamp_pick(a.draws[m]);
        }
        if (t < F) a.cen[(int64_t)m * F + t] = x[pick * F + t];
        __syncthreads();
    }
    // ---- Lloyd iterations: nearest centre (ties to the lower index), then
    // every non-empty cluster's centre to its mean
    for (int64_t i = i0; i < i1; ++i) a.lab[i] = -1;
    for (int it = 0; it < a.iters; ++it) {
        if (t == 0) s_changed = 0;
        __syncthreads();
        int ch = 0;
        for (int64_t i = i0; i < i1; ++i) {
            int best = 0;
            double bd = dist(i, a.cen);
            for (int m = 1; m < k; ++m) {
                const double dm = dist(i, a.cen + (int64_t)m * F);
                if (dm < bd) {
                    bd = dm;
                    best = m;
                }
            }
            if (a.lab[i] != best) {
                a.lab[i] = best;
                ch = 1;
            }
        }
        if (ch) atomicOr(&s_changed, 1);
        __syncthreads();
        const bool changed = s_changed != 0;
        __syncthreads();
        if (!changed && it > 0) break;
        for (int m = 0; m < k; ++m) {
            double v[kMaxFeat + 1];
#pragma unroll
            for (int j = 0; j < kMaxFeat + 1; ++j) v[j] = 0.0;
            for (int64_t i = i0; i < i1; ++i)
                if (a.lab[i] == m) {
#pragma unroll
                    for (int j = 0; j < kMaxFeat; ++j)
                        if (j < F) v[j] += x[i * F + j];
                    v[kMaxFeat] += 1.0;
                }
            wg_sums(v, F, true, red, tot);
            if (tot[kMaxFeat] > 0.0 && t < F) a.cen[(int64_t)m * F + t] = tot[t] / tot[kMaxFeat];
            __syncthreads();
        }
    }
    // ---- the kept clusters in order of first appearance
    for (int m = 0; m < k; ++m) {
        if (t == 0) {
            s_min = (unsigned long long)P;
            s_cnt = 0ULL;
        }
        __syncthreads();
        unsigned long long first = (unsigned long long)P, cnt = 0ULL;
        for (int64_t i = i0; i < i1; ++i)
            if (a.lab[i] == m) {
                if (first == (unsigned long long)P) first = (unsigned long long)i;
                ++cnt;
            }
        if (cnt) {
            atomicMin(&s_min, first);
            atomicAdd(&s_cnt, cnt);
        }
        __syncthreads();
        if (t == 0) {
            a.d2[m] = (double)s_min;  // d2 is free now: cluster m's first particle
            ipart[m] = (int32_t)s_cnt;
        }
        __syncthreads();
    }
    if (t == 0) {  // non-empty clusters, by insertion, in order of their first particle
        int kk = 0;
        for (int m = 0; m < k; ++m)
            if (ipart[m] > 0) {
                int q = kk++;
                while (q > 0 && a.d2[a.inv[q - 1]] > a.d2[m]) {
                    a.inv[q] = a.inv[q - 1];
                    --q;
                }
                a.inv[q] = m;
            }
        a.info[0] = kk;
        for (int m = 0; m < k; ++m) a.map[m] = -1;
        for (int c = 0; c < kk; ++c) {
            a.info[1 + c] = ipart[a.inv[c]];
            a.map[a.inv[c]] = c;
        }
    }
    __syncthreads();
    const int kk = a.info[0];
    if (a.labels)
        for (int64_t i = i0; i < i1; ++i) a.labels[i] = a.map[a.lab[i]];
    if (a.centers && t < F)
        for (int c = 0; c < kk; ++c) a.centers[(int64_t)c * F + t] = a.cen[(int64_t)a.inv[c] * F + t];
    if (!a.order || !a.pv) return;
    // ---- the particles grouped by kept cluster, each cluster's top member
    // (the highest earlier best value, the first among equals)
    int64_t base = 0;
    for (int c = 0; c < kk; ++c) {
        const int m = a.inv[c];
        // the run's count and top member: its first member, then strictly larger values
        int32_t cnt = 0;
        double bv = -INFINITY;
        int64_t bi = P;
        for (int64_t i = i0; i < i1; ++i)
            if (a.lab[i] == m) {
                if (bi == P || a.pv[i] > bv) {
                    bv = a.pv[i];
                    bi = i;
                }
                ++cnt;
            }
        ipart[t] = cnt;
        bvs[t] = bv;
        part[t] = (double)bi;
        __syncthreads();
        if (t == 0) {
            int32_t acc = 0;
            for (int q = 0; q < kKmThreads; ++q) {
                const int32_t v = ipart[q];
                ipart[q] = acc;
                acc += v;
            }
            // the top over the runs: the largest value, the lowest index among equals
            double tv = -INFINITY;
            int64_t ti = P;
            for (int q = 0; q < kKmThreads; ++q) {
                const int64_t qi = (int64_t)part[q];
                if (qi < P && (ti == P || bvs[q] > tv)) {
                    tv = bvs[q];
                    ti = qi;
                }
            }
            a.info[1 + k + c] = (int32_t)ti;
        }
        __syncthreads();
        int64_t pos = base + ipart[t];
        for (int64_t i = i0; i < i1; ++i)
            if (a.lab[i] == m) a.order[pos++] = (int32_t)i;
        base += a.info[1 + c];
        __syncthreads();
    }
}

// dst[r] = src[idx[r]] for rows of D doubles
__global__ void k_gather_rows(int64_t n, int D, const int32_t* __restrict__ idx, const double* __restrict__ src,
                              double* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * D) return;
    const int64_t r = i / D;
    const int d = (int)(i % D);
    dst[i] = src[(int64_t)idx[r] * D + d];
}

}  // namespace

// The k-means of KmArgs on device data x [P][F]: scratch allocated here, the
// draws from seed (splitmix64, in the order the seeding uses them); info
// (host, 1 + 2k entries) receives the kept count, sizes and top members.
// Queued on st; returns once info is on the host.
static int kmeans_dev(const double* x, int64_t P, int F, int k, int iters, uint64_t seed, const double* pv,
                      int32_t* labels, double* centers, int32_t* order, std::vector<int32_t>& info, hipStream_t st)
{
    SplitMix rng{seed};
    std::vector<double> draws(k);
    for (int m = 0; m < k; ++m) draws[m] = rng.uniform();
    double *d2 = nullptr, *cen = nullptr, *dr = nullptr;
    int32_t *lab = nullptr, *inv = nullptr, *map = nullptr, *dinfo = nullptr;
    int rc = SCS_OK;
    if (hipMalloc((void**)&d2, sizeof(double) * std::max<int64_t>(P, k)) != hipSuccess ||
        hipMalloc((void**)&cen, sizeof(double) * (size_t)k * F) != hipSuccess ||
        hipMalloc((void**)&dr, sizeof(double) * k) != hipSuccess ||
        hipMalloc((void**)&lab, sizeof(int32_t) * P) != hipSuccess ||
        hipMalloc((void**)&inv, sizeof(int32_t) * k) != hipSuccess ||
        hipMalloc((void**)&map, sizeof(int32_t) * k) != hipSuccess ||
        hipMalloc((void**)&dinfo, sizeof(int32_t) * (1 + 2 * k)) != hipSuccess)
        rc = err(SCS_ENOMEM, "k-means: device buffers could not be allocated");
    info.assign(1 + 2 * k, 0);
    if (rc == SCS_OK &&
        hipMemcpyAsync(dr, draws.data(), sizeof(double) * k, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = err(SCS_EDEVICE, "k-means: upload failed");
    if (rc == SCS_OK) {
        KmArgs ka{P, F, k, iters, x, dr, pv, d2, lab, cen, inv, map, dinfo, labels, centers, order};
        hipLaunchKernelGGL(k_kmeans, dim3(1), dim3(kKmThreads), 0, st, ka);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(info.data(), dinfo, sizeof(int32_t) * (1 + 2 * k), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            rc = err(SCS_EDEVICE, "k-means on the device failed");
    }
    hipStreamSynchronize(st);
    for (void* q : {(void*)d2, (void*)cen, (void*)dr, (void*)lab, (void*)inv, (void*)map, (void*)dinfo})
        if (q) hipFree(q);
    return rc;
}

extern "C" int scs_kmeans_device(const double* x, int64_t n, int32_t dim, int32_t k, int32_t iters, uint64_t seed,
                                 int32_t* labels, double* centers, int32_t* k_out, void* stream)
{
    if (!x || !labels || !k_out || n < 1 || n > INT32_MAX || dim < 1 || dim > kMaxFeat || k < 1 || k > 1024 ||
        iters < 1)
        return err(SCS_EINVAL, "bad k-means arguments");
    k = (int32_t)std::min<int64_t>(k, n);
    std::vector<int32_t> info;
    int rc = kmeans_dev(x, n, dim, k, iters, seed, nullptr, labels, centers, nullptr, info, (hipStream_t)stream);
    if (rc) return rc;
    *k_out = info[0];
    return SCS_OK;
}

// Re-group all particles into k-means clusters of their positions, on the
// device: the swarms' arrays are gathered into one set, k_features and
// k_kmeans cluster them, and every kept cluster becomes a new swarm whose
// rows are gathered from the set (positions, velocities and best positions
// carry over; best values restart at -inf, the first step of the rung only
// evaluates; the swarm's best position starts at the best position of its
// member with the highest earlier best value).  The host reads back the
// cluster count, sizes and top members only.
static int regroup(scs_search* s, hipStream_t st)
{
    const int nsw = (int)s->swarms.size();
    int64_t P = 0;
    for (int64_t n : s->sizes) P += n;
    const int D = s->dim;
    int F = 0;
    for (int d = 0; d < D; ++d) F += s->per[d] ? 2 : 1;
    const int k = (int)std::min<int64_t>(s->p.n_swarms, P);
    if (P > INT32_MAX) return err(SCS_EINVAL, "search: too many particles to re-group");
    const size_t rows = sizeof(double) * (size_t)P * D;
    double *th = nullptr, *vel = nullptr, *pb = nullptr, *pv = nullptr, *f = nullptr;
    int32_t* order = nullptr;
    auto release = [&]() {
        hipStreamSynchronize(st);
        for (void* q : {(void*)th, (void*)vel, (void*)pb, (void*)pv, (void*)f, (void*)order})
            if (q) hipFree(q);
    };
    if (hipMalloc((void**)&th, rows) != hipSuccess || hipMalloc((void**)&vel, rows) != hipSuccess ||
        hipMalloc((void**)&pb, rows) != hipSuccess || hipMalloc((void**)&pv, sizeof(double) * P) != hipSuccess ||
        hipMalloc((void**)&f, sizeof(double) * (size_t)P * F) != hipSuccess ||
        hipMalloc((void**)&order, sizeof(int32_t) * P) != hipSuccess) {
        release();
        return err(SCS_ENOMEM, "search: re-grouping buffers could not be allocated");
    }
    bool ok = true;
    int64_t off = 0;
    for (int i = 0; i < nsw; ++i) {
        double *sth, *svel, *spb, *spv, *sg;
        swarm_arrays(s->swarms[i], &sth, &svel, &spb, &spv, &sg);
        const size_t nb = sizeof(double) * (size_t)s->sizes[i] * D;
        ok = ok && hipMemcpyAsync(th + off * D, sth, nb, hipMemcpyDeviceToDevice, st) == hipSuccess &&
             hipMemcpyAsync(vel + off * D, svel, nb, hipMemcpyDeviceToDevice, st) == hipSuccess &&
             hipMemcpyAsync(pb + off * D, spb, nb, hipMemcpyDeviceToDevice, st) == hipSuccess &&
             hipMemcpyAsync(pv + off, spv, sizeof(double) * s->sizes[i], hipMemcpyDeviceToDevice, st) == hipSuccess;
        off += s->sizes[i];
    }
    if (!ok) {
        release();
        return err(SCS_EDEVICE, "search: re-grouping copies failed");
    }
    FeatBox fb{};
    fb.D = D;
    for (int d = 0; d < D; ++d) {
        fb.lo[d] = s->lo[d];
        fb.hi[d] = s->hi[d];
        fb.per[d] = s->per[d];
    }
    hipLaunchKernelGGL(k_features, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, P, fb, F, th, f);
    std::vector<int32_t> info;
    int rc = kmeans_dev(f, P, F, k, s->p.kmeans_iters, s->p.seed ^ (0x6b6d65616e73ull + (uint64_t)s->rungs_done), pv,
                        nullptr, nullptr, order, info, st);
    if (rc) {
        release();
        return rc;
    }
    const int kk = info[0];
    std::vector<scs_swarm*> nsws;
    std::vector<int64_t> nsizes;
    int64_t base = 0;
    for (int c = 0; c < kk && rc == SCS_OK; ++c) {
        const int64_t n = info[1 + c];
        const int64_t top = info[1 + k + c];
        scs_swarm* sw = nullptr;
        if ((rc = scs_swarm_create(s->ctx, &sw, n, s->lo, s->hi, s->per, s->p.seed, s->next_id++))) break;
        nsws.push_back(sw);
        nsizes.push_back(n);
        double *sth, *svel, *spb, *spv, *sg;
        swarm_arrays(sw, &sth, &svel, &spb, &spv, &sg);
        const unsigned g = (unsigned)((n * D + 255) / 256);
        hipLaunchKernelGGL(k_gather_rows, dim3(g), dim3(256), 0, st, n, D, order + base, th, sth);
        hipLaunchKernelGGL(k_gather_rows, dim3(g), dim3(256), 0, st, n, D, order + base, vel, svel);
        hipLaunchKernelGGL(k_gather_rows, dim3(g), dim3(256), 0, st, n, D, order + base, pb, spb);
        // best values restart (pbest_val is -inf from creation); the swarm's
        // best position is the top member's best position, its value -inf
        if (hipMemcpyAsync(sg, pb + top * D, sizeof(double) * D, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipGetLastError() != hipSuccess)
            rc = err(SCS_EDEVICE, "search: re-grouping gathers failed");
        base += n;
    }
    release();
    if (rc) {
        for (scs_swarm* sw : nsws) scs_swarm_destroy(sw);
        return rc;
    }
    for (scs_swarm* sw : s->swarms) scs_swarm_destroy(sw);
    s->swarms = nsws;
    s->sizes = nsizes;
    return SCS_OK;
}

extern "C" int scs_search_run_rung(scs_search* s, const scs_rung* r, scs_rung_report* rep, void* stream)
{
    if (!s || !r) return err(SCS_EINVAL, "NULL argument");
    if (r->N < 1 || r->N > SCS_MAX_SEGMENTS || r->max_iters < 1) return err(SCS_EINVAL, "bad rung");
    const auto t0 = std::chrono::steady_clock::now();
    int rc;
    if (s->rungs_done > 0 && (rc = regroup(s, (hipStream_t)stream))) return rc;
    if ((rc = scs_define_segmentation(s->ctx, r->N, SCS_SEG_EQUAL_SNR, s->p.G, nullptr))) return rc;
    const int nsw = (int)s->swarms.size();
    const int W = s->p.conv_window;
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx_device(s->ctx)) != hipSuccess) return err(SCS_EDEVICE, "hipSetDevice failed");
    // fresh records: nothing pushed, nothing converged
    std::fill(s->h_state, s->h_state + 3 * nsw, 0);
    if (hipMemcpyAsync(s->d_state, s->h_state, sizeof(int32_t) * 3 * nsw, hipMemcpyHostToDevice, st) != hipSuccess)
        return err(SCS_EDEVICE, "search: record upload failed");
    std::vector<scs::ConvRecord> conv(nsw);
    std::vector<uint32_t> it0(nsw);
    for (int i = 0; i < nsw; ++i) {
        conv[i] = scs::ConvRecord{s->d_ring + (size_t)i * (W + 1), s->d_state + 3 * i, W, s->p.conv_tol};
        it0[i] = swarm_iteration(s->swarms[i]);
    }
    std::vector<char> done(nsw, 0);
    std::vector<int32_t> done_at(nsw, -1);
    std::vector<scs_swarm*> act;
    std::vector<scs::ConvRecord> cact;
    int it = 0;
    bool all = false;
    while (it < r->max_iters && !all) {
        act.clear();
        cact.clear();
        for (int i = 0; i < nsw; ++i)
            if (!done[i]) {
                act.push_back(s->swarms[i]);
                cact.push_back(conv[i]);
            }
        // a batch of iterations, queued with no read back: a swarm that
        // converges part way through is frozen by its record on the device
        const int nb = std::min(kConvBatch, r->max_iters - it);
        for (int j = 0; j < nb; ++j)
            if ((rc = pso_step_swarms_tracked(act.data(), (int)act.size(), &r->prm, s->p.prec, cact.data(), it + j, st)))
                return rc;
        if (hipMemcpyAsync(s->h_state, s->d_state, sizeof(int32_t) * 3 * nsw, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return err(SCS_EDEVICE, "search: record read failed");
        all = true;
        for (int i = 0; i < nsw; ++i) {
            if (!done[i] && s->h_state[3 * i + 1]) {
                done[i] = 1;
                done_at[i] = s->h_state[3 * i + 2];
                // the swarm took the iterations up to the one it converged in
                set_swarm_iteration(s->swarms[i], it0[i] + (uint32_t)done_at[i] + 1u);
            }
            all = all && done[i];
        }
        it += nb;
    }
    // the rung ends at the iteration in which its last swarm converged
    int iterations = it;
    if (all) iterations = 1 + *std::max_element(done_at.begin(), done_at.end());
    s->rungs_done += 1;
    if (rep) {
        rep->N = r->N;
        rep->n_swarms = nsw;
        rep->iterations = iterations;
        int n_conv = 0;
        double best = -std::numeric_limits<double>::infinity();
        for (int i = 0; i < nsw; ++i) {
            n_conv += done[i];
            // a frozen swarm's best is the last value its record took
            double g = 0.0;
            if ((rc = scs_swarm_read(s->swarms[i], nullptr, nullptr, nullptr, nullptr, nullptr, &g, nullptr))) return rc;
            best = std::max(best, g);
        }
        rep->converged = n_conv;
        rep->best_val = best;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return SCS_OK;
}

extern "C" int scs_search_swarms(scs_search* s, int32_t* n_swarms, int64_t* sizes, double* best)
{
    if (!s || !n_swarms) return err(SCS_EINVAL, "NULL argument");
    *n_swarms = (int32_t)s->swarms.size();
    for (size_t i = 0; i < s->swarms.size(); ++i) {
        if (sizes) sizes[i] = s->sizes[i];
        if (best) {
            int rc = scs_swarm_read(s->swarms[i], nullptr, nullptr, nullptr, nullptr, best + (s->dim + 1) * i,
                                    best + (s->dim + 1) * i + s->dim, nullptr);
            if (rc) return rc;
        }
    }
    return SCS_OK;
}

extern "C" int scs_search_destroy(scs_search* s)
{
    if (!s) return SCS_OK;
    for (scs_swarm* sw : s->swarms) scs_swarm_destroy(sw);
    if (s->d_ring || s->d_state) {
        hipSetDevice(ctx_device(s->ctx));
        hipDeviceSynchronize();
    }
    if (s->d_ring) hipFree(s->d_ring);
    if (s->d_state) hipFree(s->d_state);
    if (s->h_state) hipHostFree(s->h_state);
    if (s->h_best) hipHostFree(s->h_best);
    delete s;
    return SCS_OK;
}
