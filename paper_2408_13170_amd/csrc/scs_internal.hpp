// Internal interface between the host runtime (scs_host.hip) and the kernels
// (scs_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scs {

constexpr int kNodes = 6;  // degree-5 block polynomials (6 coefficients / Chebyshev nodes)
// doubles per basis-table entry: 9 functions x 6 orders (the eighth PN
// function, then f^-34/9 of the eccentric term), the value of f^-5/3 and of
// f^-34/9 at the centre in double-double, padding
constexpr int kGStride = 64;
constexpr int kGHi = 54;
constexpr int kGLo = 55;
constexpr int kGEHi = 56;
constexpr int kGELo = 57;
constexpr int kMaxLevel = 12;  // sub-block lengths 2^3 .. 2^11
constexpr int kTrig = 1024;       // entries of the (cos, sin)(2 pi i / kTrig) table
constexpr int kCoefStride = 56;  // doubles per particle record of the coefficient buffer
constexpr int kRec = 8;          // doubles per (chunk, slot) record: head piece, tail piece, padding

// Values per bin of the precomputed tables: [u_c re, u_c im]_c, [q_c]_c, and
// for three channels three padding values so that every bin starts on a
// 32-byte boundary.
__host__ __device__ constexpr int bin_stride(int nch) { return nch == 3 ? 12 : 3 * nch; }

struct GridArgs {
    int64_t K;
    double k0;  // f_min / df
    double df;
    int nch;
};

struct ModelArgs {
    int pn_order;
    int response;
    int support;
    double t_obs;
    double orb0_cyc;  // orbital phase at t = 0 [cycles]
    double cart0;     // cartwheel phase at t = 0 [rad]
    double cart_c, cart_s;  // cos, sin of cart0
    int ecc;                // 1: eccentric phase, theta rows carry an 8th entry e0
    int sparse;             // 0: template per bin (block polynomials); S > 0: the sparse-grid
                            // template, nodes every S bins, cubic splines onto every bin
};

// ---- sparse-grid template (Sec 4: waveform and response on a coarse grid,
// cubic splines onto the FFT grid).  A particle's nodes are the first bin of
// its support, the multiples of S strictly inside it and its last bin; n is
// the number of intervals (nodes - 1).  Each node has a record
//   [I, phi, R_1 .. R_NR, M_0 .. M_NQ-1, T_0 .. T_NQ-1]
// with the template phase I + phi in cycles (I an integer, |phi| <= 1/2), the
// NR real and imaginary parts of the channel responses, the spline's second
// derivatives M of the NQ = 1 + NR quantities and the solver's work space T.
__host__ __device__ constexpr int spl_nr(int nch) { return nch == 1 ? 0 : 2 * nch; }
__host__ __device__ constexpr int spl_nq(int nch) { return 1 + spl_nr(nch); }
__host__ __device__ constexpr int spl_rec(int nch) { return 2 + spl_nr(nch) + 2 * spl_nq(nch); }
__host__ __device__ constexpr int64_t spl_max_nodes(int64_t K, int64_t S) { return (K + S - 1) / S + 2; }
constexpr int kMaxSparseStride = 65536;
__host__ __device__ inline int64_t spl_intervals(int64_t klo, int64_t khi, int64_t S)
{
    if (khi - 1 <= klo) return 0;
    const int64_t first = (klo / S + 1) * S;  // first multiple of S after klo
    return 1 + (first < khi - 1 ? (khi - 2 - first) / S + 1 : 0);
}
__host__ __device__ inline int64_t spl_node(int64_t j, int64_t n, int64_t klo, int64_t khi, int64_t S)
{
    return j == 0 ? klo : (j == n ? khi - 1 : (klo / S + j) * S);
}

struct SplineArgs {
    GridArgs g;
    ModelArgs m;
    int64_t P;
    int64_t stride;  // coefficient buffer stride
    const double* coef;
    const int32_t* klo;
    const int32_t* khi;
    const int8_t* lg;
    int64_t nmax;  // node records per particle
    double* spl;   // [P][nmax][spl_rec(nch)]
};
void launch_spline(const SplineArgs& a, hipStream_t s);  // node values, then the spline solve

struct PhysConst {
    double pitsun_hi, pitsun_lo;  // pi G Msun / c^3 [s], double-double
    double k3_hi, k3_lo;          // 3 / (256 pi), double-double
};

struct PrologueArgs {
    GridArgs g;
    ModelArgs m;
    PhysConst c;
    int64_t P;
    int64_t stride;  // coefficient buffer stride (particle capacity)
    const double* theta;
    double* coef;
    int32_t* klo;
    int32_t* khi;
    int8_t* lg;  // log2 of the polynomial block length; -1 invalid theta, -2 unresolved
    int lg_max;
    unsigned long long* evals;
    unsigned long long* unresolved;
    const int32_t* frozen;  // nullable; when *frozen != 0 no theta is evaluated (all as invalid)
};

struct BoundArgs {
    GridArgs g;
    ModelArgs m;
    int64_t P;
    int64_t stride;
    int N;
    int mode;
    int64_t G;
    const double* coef;
    const int32_t* klo;
    const int32_t* khi;
    const int8_t* lg;
    const double* b64;
    const int64_t* edges;  // device, EXPLICIT mode
    int32_t* bounds;       // [P][N+1]
    int wcache;            // EQUAL_SNR: node weights kept in LDS between the passes
};

struct MainArgs {
    GridArgs g;
    ModelArgs m;
    int64_t p0, P_end;     // particle range handled by this launch
    int64_t stride;
    int N;
    int L;                 // LDS block length (bins) = largest polynomial block
    int CB;                // LDS blocks per chunk
    int64_t chunk0;        // first chunk index covered by rec
    int64_t n_groups;      // particle groups (64 * waves particles each)
    int64_t n_tiles;       // n_chunks * n_groups
    int64_t rec_stride;    // particle stride in rec
    const double* coef;
    const int32_t* klo;
    const int32_t* khi;
    const int8_t* lg;
    const int32_t* bounds;
    const double* b64;
    const float* b32;
    const double* gtab;            // basis tables of every level
    int64_t gtab_off[kMaxLevel];   // entry offset of level lg
    int32_t lg_max;                // log2 of the longest polynomial block (the basis table's top level)
    const int32_t* perm;   // slot -> particle (relative to p0), or null for identity
    double* rec;           // [chunk][rec_stride][kRec], indexed by slot
    double* zs;            // [P][N][3]: (Z re, Z im, H) of segments closed inside a chunk
    double zscale32;       // FP32 tables hold u * sqrt(s), q * s: Z32 * zscale32 = Z, H32 * hscale32 = H
    double hscale32;
    const double* spl;     // sparse-grid template: node records (SplineArgs), else null
    int64_t spl_nmax;
};

struct FinalArgs {
    int64_t K;
    double df;
    int64_t p0, P_end;
    int N;
    int64_t cbins;
    int64_t chunk0;
    int64_t rec_stride;
    const int32_t* klo;
    const int32_t* khi;
    const int8_t* lg;
    const int32_t* bounds;
    const int32_t* perm;  // as in MainArgs
    const double* rec;
    double* zs;   // as in MainArgs
    double* ups;  // [P_end - p0]
    double* seg;  // non-null: zs is the caller's segment output, completed here
    double* stats;  // non-null: [P_end - p0][kNStats] likelihood statistics
};

struct PsoBox {
    double lo[8], hi[8];
    int periodic[8];
    int dim;  // 7, or 8 with e0
};
struct PsoParams {
    double omega, phi_p, phi_g;
    double eps[8];
};

hipError_t upload_cheb(const double* x, const double* m);
hipError_t upload_trig(const double* cs);
constexpr int kNStats = 5;  // Upsilon_N, hat O_N, <h|h>, Re <d|h>, Im <d|h>

// Fixed-theta evaluation over many data streams (noise realisations).  The
// streams are stored [n_chan][K][R][2]: realisations innermost, so that the
// lanes of a wave (consecutive r) read consecutive memory.
constexpr int kPieceBins = 1024;  // bins per work piece of the streamed reduction
struct StreamGenArgs {
    int64_t K, R, r0;
    int nch;
    double df, scale;
    uint64_t seed;
    const double* d;    // loaded data [nch][K][2]
    const double* psd;  // [nch][K]
    double* streams;    // [nch][K][R][2]
};
struct StreamArgs {
    int64_t K, R;
    int nch;
    double df;
    const double* streams;  // [nch][K][R][2]
    const double* wts;      // [nch][K][2]: conj(h) / S
    const double* hq;       // [K]: sum over channels of |h|^2 / S
    const int32_t* pieces;  // [n_pieces][3]: first bin, end bin, segment (in segment order)
    int64_t n_pieces;
    double* zpart;          // [n_pieces][R][2]
    double* hpart;          // [n_pieces]
    double* stats;          // [R][kNStats]
};
void launch_make_streams(const StreamGenArgs& a, int n_cu, hipStream_t s);
void launch_stream_weights(int nch, int64_t K, const double* h_ri, const double* psd, double* wts, double* hq,
                           hipStream_t s);
void launch_streams(const StreamArgs& a, hipStream_t s);        // the streamed reduction
void launch_streams_final(const StreamArgs& a, hipStream_t s);  // per-stream statistics
constexpr int kNormBlocks = 256;
void launch_data_norm(const GridArgs& g, const double* d_ri, const double* psd, double* part, double* out,
                      hipStream_t s);
void launch_distance_amp(int64_t P, int td, const double* theta, const double* dl, double k, double* amp,
                         hipStream_t s);
void launch_loglike(int64_t P, double dd, const double* stats, const double* amp, const double* phase, double* semi,
                    double* coh, hipStream_t s);
void launch_bins(const GridArgs& g, const double* d_ri, const double* psd, double* b64, float* b32, double su,
                 double sq, hipStream_t s);
void launch_prologue(const PrologueArgs& a, hipStream_t s);
void launch_bounds(const BoundArgs& a, hipStream_t s);
size_t main_lds_bytes(int nch, int L, bool mixed);
// The kernel instantiations of the generate-and-reduce, one per (response
// model, channels, template): 0 = low-frequency A+E, 1 = full A+E, 2 = full
// A+E+T, 3 = one channel without response; 4 .. 7 the same with the
// sparse-grid template.
constexpr int kVariants = 8;
__host__ __device__ constexpr int variant_of(int resp, int nch, int sparse)
{
    return (resp == 1 ? 0 : (resp == 2 ? (nch == 3 ? 2 : 1) : 3)) + (sparse > 0 ? 4 : 0);
}
// alt: the instantiation with the alternative occupancy target (two waves
// per SIMD for FP64, four for mixed; the per-bin template on one and two
// channels), for the autotuner
hipError_t launch_main_multi(const MainArgs* items, const int64_t* tile_start, int n_items, unsigned long long* counter,
                             int variant, int L, int waves, bool mixed, bool alt, int grid, hipStream_t s);
int main_multi_blocks_per_cu(int variant, int L, int waves, bool mixed, bool alt);
void launch_finalize(const FinalArgs& a, hipStream_t s);
void launch_waveform(const MainArgs& a, double* h_ri, hipStream_t s);
void launch_gtab(const GridArgs& g, int lg, int64_t nsub, double* tab, hipStream_t s);
void launch_pso_init(int64_t P, const PsoBox& box, uint64_t seed, uint32_t swarm, double* theta, hipStream_t s);
// Convergence record of one swarm of a search, kept on the device: the last
// window + 1 swarm best values (a ring) and state = [values pushed, converged
// (0 or 1), the rung iteration at which it converged].  A converged swarm is
// frozen: every kernel of a step leaves it as it is.
struct ConvRecord {
    double* ring;
    int32_t* state;
    int32_t window;
    double tol;
};
// frozen (nullable): when *frozen != 0 the kernels return at once.  conv
// (nullable): after the swarm best, push it and apply the convergence rule
// (rung iteration rung_it); its state[1] then serves as the frozen flag.
void launch_pso_move(int64_t P, const PsoBox& box, const PsoParams& prm, uint64_t seed, uint32_t swarm, uint32_t it,
                     double* theta, double* vel, const double* pbest, const double* gbest, hipStream_t s,
                     const int32_t* frozen = nullptr);
void launch_pso_best(int64_t P, const PsoBox& box, const double* theta, const double* vals, double* pbest,
                     double* pbest_val, double* gbest, double* gbest_val, hipStream_t s,
                     const ConvRecord* conv = nullptr, int32_t rung_it = 0);
constexpr int kSortBuckets = 65536;  // 256 levels of k_hi x 256 levels of k_lo
void launch_sort_perm(int64_t P, int64_t K, const int32_t* klo, const int32_t* khi, unsigned* hist, int32_t* bucket,
                      int32_t* rank, int32_t* perm, hipStream_t s);
void launch_fill(double* p, int64_t n, double v, hipStream_t s);
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s);

}  // namespace scs
