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
// The re-grouping runs on the device too (k_features, then the k_km_*
// kernels: k-means over many workgroups, every sum in a fixed order); the
// host reads back the cluster count, sizes and top members.  scs_kmeans, the same
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

// k-means (Arthur & Vassilvitskii 2007 seeding, then Lloyd iterations until
// no label changes, at most iters) on the device, with the steps of
// scs_kmeans and of the host re-grouping: each workgroup takes a run of
// kKmBlock consecutive points, one per thread, and every sum is formed in a
// fixed order (within a workgroup by wave shuffles and then the waves in
// turn, across workgroups in workgroup order), so a call gives the same
// result every time.  The sums are ordered differently from the host's
// sequential ones, so labels can differ only where a point lies within
// rounding of two centres or a draw within rounding of a cumulative weight.
constexpr int kKmBlock = 256;
constexpr int kKmBWaves = kKmBlock / 64;

// Workgroup sums of v[j], j < n (n <= kMaxFeat), and with count of
// v[kMaxFeat], in a fixed order (wave shuffles, then the waves in turn); the
// totals land in out[j] (and out[kMaxFeat]).  Every index is a constant after
// unrolling, so v stays in registers.  red: [kKmBWaves][kMaxFeat + 1].
__device__ void blk_sums(const double* v, int n, bool count, double* red, double* out)
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
        for (int q = 0; q < kKmBWaves; ++q) t += red[q * (kMaxFeat + 1) + j];
        out[j] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ double km_dist(const double* __restrict__ x, int64_t i, int F, const double* c)
{
    double s = 0.0;
    for (int j = 0; j < F; ++j) {
        const double d = x[i * F + j] - c[j];
        s += d * d;
    }
    return s;
}

__global__ void k_km_fill(int32_t* p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Seeding, centre m >= 1: each point's squared distance to its nearest centre
// so far (centre m - 1 the newest), and each workgroup's sum of them.
__global__ __launch_bounds__(kKmBlock) void k_km_seed_d2(int64_t P, int F, const double* __restrict__ x,
                                                          const double* __restrict__ c, int first, double* d2,
                                                          double* bsum)
{
    __shared__ double red[kKmBWaves * (kMaxFeat + 1)];
    __shared__ double tot[kMaxFeat + 1];
    const int64_t i = (int64_t)blockIdx.x * kKmBlock + threadIdx.x;
    double v[kMaxFeat + 1];
#pragma unroll
    for (int j = 0; j < kMaxFeat + 1; ++j) v[j] = 0.0;
    if (i < P) {
        const double d = km_dist(x, i, F, c);
        const double o = first ? INFINITY : d2[i];
        const double n = d < o ? d : o;
        d2[i] = n;
        v[0] = n;
    }
    blk_sums(v, 1, false, red, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot[0];
}

// Seeding, centre m: the pick (centre 0: uniform; else the first point whose
// running sum of squared distances reaches draw * total, the runs taken
// workgroup by workgroup and then point by point), copied to centre m.
__global__ void k_km_seed_pick(int64_t P, int F, int m, int64_t nb, const double* __restrict__ x,
                               const double* __restrict__ draws, const double* __restrict__ d2,
                               const double* __restrict__ bsum, double* cen)
{
    __shared__ int64_t s_pick;
    if (threadIdx.x == 0) {
        const double r = draws[m];
        int64_t pick = -1;
        double total = 0.0;
        if (m > 0)
            for (int64_t b = 0; b < nb; ++b) total += bsum[b];
        if (m > 0 && total > 0.0) {
            const double u = r * total;
            double acc = 0.0;
            for (int64_t b = 0; b < nb && pick < 0; ++b) {
                if (acc + bsum[b] >= u) {
                    double a2 = acc;
                    const int64_t e = (b + 1) * kKmBlock < P ? (b + 1) * kKmBlock : P;
                    for (int64_t i = b * kKmBlock; i < e; ++i) {
                        a2 += d2[i];
                        if (a2 >= u) {
                            pick = i;
                            break;
                        }
                    }
                }
                acc += bsum[b];
            }
            if (pick < 0) pick = P - 1;
        } else {
            pick = (int64_t)(r * (double)P);
            pick = pick < P - 1 ? pick : P - 1;
        }
        s_pick = pick;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < F; j += blockDim.x) cen[(int64_t)m * F + j] = x[s_pick * F + j];
}

// Lloyd, one iteration's first half: nearest centre of each point (ties to
// the lower index), whether any label of the workgroup changed, and each
// cluster's sum and count over the workgroup's points.  Nothing once the
// iterations have stopped (state[0]).
__global__ __launch_bounds__(kKmBlock) void k_km_assign(int64_t P, int F, int k, const double* __restrict__ x,
                                                         const double* __restrict__ cen, int32_t* lab,
                                                         double* part, int32_t* chg, const int32_t* state)
{
    __shared__ double red[kKmBWaves * (kMaxFeat + 1)];
    __shared__ double tot[kMaxFeat + 1];
    if (state[0]) return;
    const int64_t i = (int64_t)blockIdx.x * kKmBlock + threadIdx.x;
    int best = -1;
    int changed = 0;
    if (i < P) {
        best = 0;
        double bd = km_dist(x, i, F, cen);
        for (int m = 1; m < k; ++m) {
            const double dm = km_dist(x, i, F, cen + (int64_t)m * F);
            if (dm < bd) {
                bd = dm;
                best = m;
            }
        }
        if (lab[i] != best) {
            lab[i] = best;
            changed = 1;
        }
    }
    const int any = __syncthreads_or(changed);
    if (threadIdx.x == 0) chg[blockIdx.x] = any;
    double* pb = part + (int64_t)blockIdx.x * k * (kMaxFeat + 1);
    for (int m = 0; m < k; ++m) {
        const bool mine = best == m;
        if (!__syncthreads_or(mine)) {
            if ((int)threadIdx.x <= F) pb[(int64_t)m * (kMaxFeat + 1) + (threadIdx.x == (unsigned)F ? kMaxFeat : threadIdx.x)] = 0.0;
            continue;
        }
        double v[kMaxFeat + 1];
#pragma unroll
        for (int j = 0; j < kMaxFeat + 1; ++j) v[j] = 0.0;
        if (mine) {
#pragma unroll
            for (int j = 0; j < kMaxFeat; ++j)
                if (j < F) v[j] = x[i * F + j];
            v[kMaxFeat] = 1.0;
        }
        blk_sums(v, F, true, red, tot);
        if ((int)threadIdx.x < F) pb[(int64_t)m * (kMaxFeat + 1) + threadIdx.x] = tot[threadIdx.x];
        if ((int)threadIdx.x == F) pb[(int64_t)m * (kMaxFeat + 1) + kMaxFeat] = tot[kMaxFeat];
    }
}

// Lloyd, the second half (one workgroup): stop if no label changed (and it
// was not the first iteration); else every non-empty cluster's centre to the
// mean of its points, the workgroups' sums added in workgroup order.
__global__ void k_km_update(int F, int k, int64_t nb, const double* __restrict__ part, const int32_t* __restrict__ chg,
                            double* cen, int32_t* state)
{
    __shared__ int s_stop;
    const int done = state[0], it = state[1];
    if (done) return;
    if (threadIdx.x == 0) {
        int any = 0;
        for (int64_t b = 0; b < nb; ++b) any |= chg[b];
        s_stop = (!any && it > 0);
    }
    __syncthreads();
    if (s_stop) {
        if (threadIdx.x == 0) state[0] = 1;
        return;
    }
    for (int q = threadIdx.x; q < k * F; q += blockDim.x) {
        const int m = q / F, j = q % F;
        double sj = 0.0, cnt = 0.0;
        for (int64_t b = 0; b < nb; ++b) {
            const double* pb = part + (b * k + m) * (kMaxFeat + 1);
            sj += pb[j];
            cnt += pb[kMaxFeat];
        }
        if (cnt > 0.0) cen[(int64_t)m * F + j] = sj / cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) state[1] = it + 1;
}

// Per workgroup and cluster: the count, the first point, and the top member
// (the highest earlier best value, the first among equals; pv may be NULL).
__global__ __launch_bounds__(kKmBlock) void k_km_blockstats(int64_t P, int k, const int32_t* __restrict__ lab,
                                                             const double* __restrict__ pv, int32_t* bcnt,
                                                             int32_t* bfirst, double* btv, int32_t* bti)
{
    __shared__ double sv[kKmBlock];
    __shared__ int32_t si[kKmBlock];
    const int64_t i = (int64_t)blockIdx.x * kKmBlock + threadIdx.x;
    const int l = i < P ? lab[i] : -1;
    for (int m = 0; m < k; ++m) {
        const bool mine = l == m;
        sv[threadIdx.x] = mine ? (pv ? pv[i] : 0.0) : -INFINITY;
        si[threadIdx.x] = mine ? (int32_t)i : INT32_MAX;
        __syncthreads();
        if (threadIdx.x == 0) {
            int32_t cnt = 0, first = INT32_MAX, ti = INT32_MAX;
            double tv = -INFINITY;
            for (int q = 0; q < kKmBlock; ++q)
                if (si[q] != INT32_MAX) {
                    ++cnt;
                    if (first == INT32_MAX) first = si[q];
                    if (ti == INT32_MAX || sv[q] > tv) {
                        tv = sv[q];
                        ti = si[q];
                    }
                }
            const int64_t o = (int64_t)blockIdx.x * k + m;
            bcnt[o] = cnt;
            bfirst[o] = first;
            btv[o] = tv;
            bti[o] = ti;
        }
        __syncthreads();
    }
}

// One workgroup, one thread: the kept clusters in order of their first point,
// their sizes and top members, and where each workgroup's points of each
// kept cluster start in the grouped order.
__global__ void k_km_finish(int k, int64_t nb, const int32_t* __restrict__ bcnt, const int32_t* __restrict__ bfirst,
                            const double* __restrict__ btv, const int32_t* __restrict__ bti, int32_t* inv,
                            int32_t* map, int32_t* info, int64_t* base)
{
    if (threadIdx.x != 0) return;
    // each cluster's first point (INT32_MAX: empty), held in map for now
    for (int m = 0; m < k; ++m) {
        int64_t cnt = 0;
        int32_t first = INT32_MAX;
        for (int64_t b = 0; b < nb; ++b) {
            cnt += bcnt[b * k + m];
            if (bfirst[b * k + m] < first) first = bfirst[b * k + m];
        }
        map[m] = cnt ? first : INT32_MAX;
    }
    int kk = 0;
    for (int m = 0; m < k; ++m) {
        if (map[m] == INT32_MAX) continue;
        int q = kk++;  // insertion by first point
        while (q > 0 && map[inv[q - 1]] > map[m]) {
            inv[q] = inv[q - 1];
            --q;
        }
        inv[q] = m;
    }
    for (int m = 0; m < k; ++m) map[m] = -1;
    info[0] = kk;
    int64_t off = 0;
    for (int c = 0; c < kk; ++c) {
        const int m = inv[c];
        map[m] = c;
        double tv = -INFINITY;
        int32_t ti = INT32_MAX;
        int64_t cnt = 0;
        for (int64_t b = 0; b < nb; ++b) {
            base[(int64_t)c * nb + b] = off + cnt;
            cnt += bcnt[b * k + m];
            const int32_t bi = bti[b * k + m];
            if (bi != INT32_MAX && (ti == INT32_MAX || btv[b * k + m] > tv)) {
                tv = btv[b * k + m];
                ti = bi;
            }
        }
        info[1 + c] = (int32_t)cnt;
        info[1 + k + c] = ti;
        off += cnt;
    }
}

// Each point's new label and its place in the grouped order: its cluster's
// start for the workgroup plus the points of that cluster before it there.
__global__ __launch_bounds__(kKmBlock) void k_km_scatter(int64_t P, int64_t nb, const int32_t* __restrict__ lab,
                                                          const int32_t* __restrict__ map, const int32_t* __restrict__ info,
                                                          const int64_t* __restrict__ base, int32_t* labels,
                                                          int32_t* order)
{
    __shared__ int32_t wc[kKmBWaves];
    const int64_t i = (int64_t)blockIdx.x * kKmBlock + threadIdx.x;
    const int c = i < P ? map[lab[i]] : -1;
    if (labels && i < P) labels[i] = c;
    if (!order) return;
    const int kk = info[0];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int q = 0; q < kk; ++q) {
        const unsigned long long mask = __ballot(c == q);
        if (lane == 0) wc[w] = __popcll(mask);
        __syncthreads();
        if (c == q) {
            int64_t pos = base[(int64_t)q * nb + blockIdx.x];
            for (int v = 0; v < w; ++v) pos += wc[v];
            pos += __popcll(mask & ((1ULL << lane) - 1ULL));
            order[pos] = (int32_t)i;
        }
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

// The k-means above on device data x [P][F]: scratch allocated here, the
// draws from seed (splitmix64, in the order the seeding uses them); info
// (host, 1 + 2k entries) receives the kept count, sizes and top members.
// The Lloyd iterations are queued 16 at a time; after each batch the host
// reads whether they stopped.  Queued on st; returns once info is on the host.
static int kmeans_dev(const double* x, int64_t P, int F, int k, int iters, uint64_t seed, const double* pv,
                      int32_t* labels, double* centers, int32_t* order, std::vector<int32_t>& info, hipStream_t st)
{
    SplitMix rng{seed};
    std::vector<double> draws(k);
    for (int m = 0; m < k; ++m) draws[m] = rng.uniform();
    const int64_t nb = (P + kKmBlock - 1) / kKmBlock;
    double *d2 = nullptr, *cen = nullptr, *dr = nullptr, *bsum = nullptr, *part = nullptr, *btv = nullptr;
    int32_t *lab = nullptr, *chg = nullptr, *state = nullptr, *bcnt = nullptr, *bfirst = nullptr, *bti = nullptr,
            *inv = nullptr, *map = nullptr, *dinfo = nullptr;
    int64_t* base = nullptr;
    int rc = SCS_OK;
    auto al = [&](void** q, size_t bytes) { return hipMalloc(q, bytes) == hipSuccess; };
    if (!al((void**)&d2, sizeof(double) * P) || !al((void**)&cen, sizeof(double) * (size_t)k * F) ||
        !al((void**)&dr, sizeof(double) * k) || !al((void**)&bsum, sizeof(double) * nb) ||
        !al((void**)&part, sizeof(double) * (size_t)nb * k * (kMaxFeat + 1)) ||
        !al((void**)&btv, sizeof(double) * (size_t)nb * k) || !al((void**)&lab, sizeof(int32_t) * P) ||
        !al((void**)&chg, sizeof(int32_t) * nb) || !al((void**)&state, sizeof(int32_t) * 2) ||
        !al((void**)&bcnt, sizeof(int32_t) * (size_t)nb * k) || !al((void**)&bfirst, sizeof(int32_t) * (size_t)nb * k) ||
        !al((void**)&bti, sizeof(int32_t) * (size_t)nb * k) || !al((void**)&inv, sizeof(int32_t) * k) ||
        !al((void**)&map, sizeof(int32_t) * k) || !al((void**)&dinfo, sizeof(int32_t) * (1 + 2 * k)) ||
        !al((void**)&base, sizeof(int64_t) * (size_t)k * nb))
        rc = err(SCS_ENOMEM, "k-means: device buffers could not be allocated");
    info.assign(1 + 2 * k, 0);
    if (rc == SCS_OK &&
        hipMemcpyAsync(dr, draws.data(), sizeof(double) * k, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = err(SCS_EDEVICE, "k-means: upload failed");
    if (rc == SCS_OK) {
        const dim3 g((unsigned)nb), b(kKmBlock);
        hipLaunchKernelGGL(k_km_fill, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, lab, P, -1);
        hipLaunchKernelGGL(k_km_fill, dim3(1), dim3(256), 0, st, state, (int64_t)2, 0);
        hipLaunchKernelGGL(k_km_seed_pick, dim3(1), dim3(64), 0, st, P, F, 0, nb, x, dr, d2, bsum, cen);
        for (int m = 1; m < k; ++m) {
            hipLaunchKernelGGL(k_km_seed_d2, g, b, 0, st, P, F, x, cen + (size_t)(m - 1) * F, m == 1 ? 1 : 0, d2,
                               bsum);
            hipLaunchKernelGGL(k_km_seed_pick, dim3(1), dim3(64), 0, st, P, F, m, nb, x, dr, d2, bsum, cen);
        }
        int32_t hstate[2] = {0, 0};
        for (int it = 0; it < iters && rc == SCS_OK;) {
            const int n = std::min(16, iters - it);
            for (int q = 0; q < n; ++q) {
                hipLaunchKernelGGL(k_km_assign, g, b, 0, st, P, F, k, x, cen, lab, part, chg, state);
                hipLaunchKernelGGL(k_km_update, dim3(1), dim3(256), 0, st, F, k, nb, part, chg, cen, state);
            }
            it += n;
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(hstate, state, sizeof(hstate), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = err(SCS_EDEVICE, "k-means on the device failed");
            if (hstate[0]) break;
        }
        if (rc == SCS_OK) {
            hipLaunchKernelGGL(k_km_blockstats, g, b, 0, st, P, k, lab, pv, bcnt, bfirst, btv, bti);
            hipLaunchKernelGGL(k_km_finish, dim3(1), dim3(64), 0, st, k, nb, bcnt, bfirst, btv, bti, inv, map, dinfo,
                               base);
            hipLaunchKernelGGL(k_km_scatter, g, b, 0, st, P, nb, lab, map, dinfo, base, labels, order);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(info.data(), dinfo, sizeof(int32_t) * (1 + 2 * k), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                rc = err(SCS_EDEVICE, "k-means on the device failed");
        }
        if (rc == SCS_OK && centers) {
            std::vector<int32_t> hinv(k);
            if (hipMemcpy(hinv.data(), inv, sizeof(int32_t) * k, hipMemcpyDeviceToHost) != hipSuccess)
                rc = err(SCS_EDEVICE, "k-means: read failed");
            for (int c = 0; c < info[0] && rc == SCS_OK; ++c)
                if (hipMemcpyAsync(centers + (size_t)c * F, cen + (size_t)hinv[c] * F, sizeof(double) * F,
                                   hipMemcpyDeviceToDevice, st) != hipSuccess)
                    rc = err(SCS_EDEVICE, "k-means: centre copy failed");
        }
    }
    hipStreamSynchronize(st);
    for (void* q : {(void*)d2, (void*)cen, (void*)dr, (void*)bsum, (void*)part, (void*)btv, (void*)lab, (void*)chg,
                    (void*)state, (void*)bcnt, (void*)bfirst, (void*)bti, (void*)inv, (void*)map, (void*)dinfo,
                    (void*)base})
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
// the k_km_* kernels cluster them, and every kept cluster becomes a new swarm whose
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
