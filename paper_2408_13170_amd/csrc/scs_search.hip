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
// k-means runs on the host: once per rung on P x 7 numbers (about 60000 x 7
// for the paper's search), milliseconds against the seconds of a rung.
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
    if (p->n_swarms < 1 || p->particles < 1 || p->G < 1 || p->conv_window < 1 || p->kmeans_iters < 1 ||
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

// Regroup all particles into k-means clusters of their positions (features:
// each dimension scaled to the prior box, periodic ones as the point on the
// circle (cos, sin) / 2 pi, so that a full turn spans about the same as a box).
static int regroup(scs_search* s)
{
    const int nsw = (int)s->swarms.size();
    int64_t P = 0;
    for (int64_t n : s->sizes) P += n;
    const int D = s->dim;
    std::vector<double> th((size_t)P * D), vel((size_t)P * D), pb((size_t)P * D), pv(P);
    int64_t off = 0;
    for (int i = 0; i < nsw; ++i) {
        int rc = scs_swarm_read(s->swarms[i], &th[(size_t)off * D], &vel[(size_t)off * D], &pb[(size_t)off * D],
                                &pv[off], nullptr, nullptr, nullptr);
        if (rc) return rc;
        off += s->sizes[i];
    }
    int dim = 0;
    for (int d = 0; d < D; ++d) dim += s->per[d] ? 2 : 1;
    std::vector<double> f((size_t)P * dim);
    for (int64_t i = 0; i < P; ++i) {
        int j = 0;
        for (int d = 0; d < D; ++d) {
            const double w = s->hi[d] - s->lo[d];
            const double u = w > 0.0 ? (th[(size_t)i * D + d] - s->lo[d]) / w : 0.0;
            if (s->per[d]) {
                const double a = 2.0 * M_PI * u;
                f[(size_t)i * dim + j++] = std::cos(a) / (2.0 * M_PI);
                f[(size_t)i * dim + j++] = std::sin(a) / (2.0 * M_PI);
            } else {
                f[(size_t)i * dim + j++] = u;
            }
        }
    }
    std::vector<int32_t> lab(P);
    int32_t k = 0;
    int rc = scs_kmeans(f.data(), P, dim, s->p.n_swarms, s->p.kmeans_iters,
                        s->p.seed ^ (0x6b6d65616e73ull + (uint64_t)s->rungs_done), lab.data(), nullptr, &k);
    if (rc) return rc;
    std::vector<scs_swarm*> nsws;
    std::vector<int64_t> nsizes;
    const double ninf = -std::numeric_limits<double>::infinity();
    for (int c = 0; c < k; ++c) {
        std::vector<double> tc, vc, bc;
        int64_t top = 0, n = 0;
        double top_val = ninf;
        for (int64_t i = 0; i < P; ++i)
            if (lab[i] == c) {
                tc.insert(tc.end(), &th[(size_t)i * D], &th[(size_t)i * D + D]);
                vc.insert(vc.end(), &vel[(size_t)i * D], &vel[(size_t)i * D + D]);
                bc.insert(bc.end(), &pb[(size_t)i * D], &pb[(size_t)i * D + D]);
                if (pv[i] > top_val) {
                    top_val = pv[i];
                    top = n;
                }
                ++n;
            }
        scs_swarm* sw = nullptr;
        if ((rc = scs_swarm_create(s->ctx, &sw, n, s->lo, s->hi, s->per, s->p.seed, s->next_id++))) break;
        nsws.push_back(sw);
        nsizes.push_back(n);
        // best values restart (the first step of the rung only evaluates);
        // the best positions carry over as attractors
        std::vector<double> bv(n, ninf);
        if ((rc = scs_swarm_write(sw, tc.data(), vc.data(), bc.data(), bv.data(), &bc[(size_t)top * D], ninf, 0u)))
            break;
    }
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
    if (s->rungs_done > 0 && (rc = regroup(s))) return rc;
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
