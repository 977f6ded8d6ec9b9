/*
 * libscs -- semi-coherent search statistic on MI355X (gfx950).
 *
 * C ABI for evaluating the semi-coherent detection statistic Upsilon_N of
 * Bandopadhyay & Moore (arXiv:2408.13170) for a whole particle swarm at once,
 * and for the particle-swarm update that drives the search.
 *
 * Conventions for every entry point
 *   - Return 0 on success, a negative SCS_E* code on failure; never throws or
 *     aborts across the ABI.  scs_last_error() returns a thread-local message
 *     describing the last failure on the calling thread.
 *   - "dev" pointers are HIP device pointers (for example torch CUDA tensors);
 *     "host" pointers are ordinary host memory.  Where an argument accepts
 *     either, a mem_kind argument says which (SCS_MEM_HOST / SCS_MEM_DEVICE).
 *   - The caller keeps ownership of every buffer it passes.  With device
 *     pointers the work is queued on `stream` (a hipStream_t, NULL = the null
 *     stream) and inputs must stay valid until the stream reaches that point;
 *     with host pointers the call returns after the results are on the host.
 *   - A context (one search: one data set, one model) is used by one host
 *     thread and one stream at a time; different contexts may run
 *     concurrently on different streams of the same device.
 *
 * Parameter vector theta, 7 doubles per particle, in this order:
 *   Mc      chirp mass [solar masses, detector frame]
 *   eta     symmetric mass ratio, 0 < eta <= 1/4
 *   f_low   gravitational-wave frequency at the start of observation [Hz];
 *           it fixes the coalescence time through t(f_low) = 0
 *   lambda  ecliptic longitude [rad]
 *   beta    ecliptic latitude [rad]
 *   iota    inclination [rad]
 *   psi     polarisation angle [rad]
 * and, for an eccentric model (scs_model.eccentric = 1), an 8th entry
 *   e0      orbital eccentricity at GW frequency f_low, 0 <= e0 < 0.5
 * (the searched parameters of Table tab:GW150914-like_injection; distance and
 * phase are maximised out of the statistic, Sec 4).  scs_theta_dim gives
 * the row width of a context.
 */
#ifndef SCS_H
#define SCS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------- */
#define SCS_OK 0
#define SCS_EINVAL (-1)  /* bad argument */
#define SCS_ENOMEM (-2)  /* device or host allocation failed */
#define SCS_EDEVICE (-3) /* HIP runtime error, or no usable gfx950 device */
#define SCS_EBUSY (-4)   /* request exceeds an admitted budget */
#define SCS_ESTATE (-5)  /* call out of order (e.g. evaluate before load_data) */

/* ---- enumerations ---------------------------------------------------- */
#define SCS_MEM_HOST 0
#define SCS_MEM_DEVICE 1

#define SCS_PREC_FP64 0  /* every step in IEEE double */
#define SCS_PREC_MIXED 1 /* FP64 anchors + FP32 residual; FP32 partial sums of at most 32 bins, FP64 segment sums */

#define SCS_RESP_NONE 0       /* one channel, h = f^-7/6 e^{-i Psi} */
#define SCS_RESP_LISA_LF_AE 1 /* two channels A, E, low-frequency LISA response */
/* channels A, E (two loaded) or A, E, T (three loaded), full frequency-domain
 * response (Sec 4 response paragraph): first-generation TDI on a rigid
 * equal-arm constellation
 * (arms 2.5e9 m, the geometry of the low-frequency response) with the
 * finite-arm-length transfer of every link at the stationary-phase time,
 * normalised by 4 (2 pi f L)^2 so that it tends to the low-frequency
 * response as f L -> 0; the PSDs go in the same normalisation */
#define SCS_RESP_LISA_FD_AE 2

#define SCS_SUPPORT_FULL 0 /* every bin of the grid */
#define SCS_SUPPORT_TOBS 1 /* bins with 0 <= t(f_k) < T_obs */

#define SCS_SEG_EQUAL_SNR 0 /* equal [h|h] per segment, per particle (Sec 2.2) */
#define SCS_SEG_UNIFORM 1   /* equal bin counts inside the support */
#define SCS_SEG_EXPLICIT 2  /* caller's bin edges, clamped to the support */
#define SCS_MAX_SEGMENTS (1 << 20) /* largest N accepted by scs_define_segmentation */

typedef struct scs_ctx scs_ctx;
typedef struct scs_swarm scs_swarm;

/* Waveform and response model (Sec 4).  Zero-initialise, then set fields. */
typedef struct scs_model {
    int32_t pn_order;        /* highest PN power of v in the phase, 0..7 (4 = 2PN, 7 = 3.5PN) */
    int32_t response;        /* SCS_RESP_* ; NONE needs 1 channel, LISA_LF_AE 2, LISA_FD_AE 2 or 3 */
    int32_t support;         /* SCS_SUPPORT_* */
    int32_t block_len;       /* longest polynomial block in bins (power of 2, 16..2048); 0 = 2048.
                              * A particle's blocks start at the longest length whose remainder
                              * bounds hold at its support start and double (twice at most, up
                              * to block_len) from the first block_len-aligned run of bins
                              * where the longer length meets the same bounds. */
    double t_obs;            /* observation time [s]; 0 = 1/df */
    double orbit_phase0;     /* orbital angle of the constellation centre at t = 0 [rad] */
    double cartwheel_phase0; /* in-plane angle of spacecraft 0 at t = 0 [rad] */
    int32_t eccentric;       /* 1: the eccentric phase of the TaylorF2Ecc model (Sec 4) at its
                                leading order in e0^2: the Newtonian term times
                                1 - (2355/1462) e0^2 (f_low / f)^(19/9), e0 the 8th theta
                                entry; 0: circular, 7 entries */
    int32_t sparse_stride;   /* 0: the template is evaluated at every bin (per-block polynomials
                                with remainders below 1e-12 cycles); S in 1..65536: the sparse-grid
                                evaluation of Sec 4 (waveform and response paragraphs): the
                                template phase (GW and Doppler terms, in cycles) and the real and
                                imaginary parts of every channel's response are evaluated exactly
                                at nodes, the first bin of the support, every multiple of S inside
                                it and its last bin, and interpolated onto every bin by not-a-knot
                                cubic splines (three nodes: the parabola, two: the line, one: the
                                constant); the amplitude f^-7/6 stays exact and the equal-[h|h]
                                edges keep the exact weights.  Needs about
                                8 ((K + S - 1) / S + 2) (2 + 3 NR + 2) bytes of device memory per
                                particle (NR = 0, 4, 6 for 1, 2, 3 channels; scs_footprint counts
                                it); every theta resolves (no NaN for an unresolved theta) */
} scs_model;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device` (a gfx950 GPU).  *out receives the
 * handle.  Fails with SCS_EDEVICE when the device is missing or not gfx950. */
int scs_ctx_create(scs_ctx** out, int device);

/* Release the context and every device buffer it owns.  NULL is accepted. */
int scs_ctx_destroy(scs_ctx* ctx);

/* Load the data stream d_alpha(f_k) and its one-sided PSD S_alpha(f_k)
 * (eqn:inner_prod) on the grid f_k = f_min + k df, k = 0..K-1.
 *   n_chan  1, 2 (A, E) or 3 (A, E, T; full response only)
 *   d_ri    [n_chan][K][2] real and imaginary parts
 *   psd     [n_chan][K], every value finite and > 0
 * f_min / df must be an integer (to 1e-9 relative): f_k are FFT bins and
 * T_obs = 1/df.  The library copies the arrays (the caller may free them on
 * return) and precomputes the particle-independent products
 * f^-7/6 d / S and f^-7/3 / S in FP64 and FP32.  Synchronous. */
int scs_load_data(scs_ctx* ctx, int32_t n_chan, int64_t K, double f_min, double df, const double* d_ri,
                  const double* psd, int32_t mem_kind);

/* Set the waveform/response model.  Errors: pn_order outside 0..7, response
 * not matching the loaded channel count, block_len not a power of 2 in
 * 16..2048, negative t_obs. */
int scs_set_model(scs_ctx* ctx, const scs_model* model);

/* Define the segmentation used by scs_evaluate (Sec 2.2).
 *   N      number of segments, 1..SCS_MAX_SEGMENTS (EINVAL outside)
 *   mode   SCS_SEG_*; EQUAL_SNR places the edges of every particle so that
 *          each segment holds the same [h|h], re-evaluated for every theta
 *   G      node stride of the EQUAL_SNR cumulative (1 = every bin); >= 1
 *   edges  host [N+1] nondecreasing bin indices for EXPLICIT, else NULL */
int scs_define_segmentation(scs_ctx* ctx, int32_t N, int32_t mode, int32_t G, const int64_t* edges);

/* Evaluate Upsilon_N (Sec 2.2, the statistic's definition) for P particles.
 *   theta  [P][D], D = scs_theta_dim (7, or 8 for an eccentric model)
 *   ups    [P] out: Upsilon_N; NaN for invalid theta (Mc <= 0, eta outside
 *          (0, 1/4], f_low <= 0, non-finite) or a theta the polynomial block
 *          scheme cannot resolve (counted by scs_ctx_stats): one whose SPA
 *          time moves so fast per bin that even 8-bin blocks leave the phase
 *          remainder above 1e-12 cycles or the response's above 1e-11, i.e. a
 *          slowly chirping low-mass source on a coarse grid (on the 2^20-bin
 *          band from 0.016 Hz, chirp times above ~270 yr at the support start;
 *          never with the sparse-grid template); 0 when the support is empty
 *   seg    [P][N][3] out, nullable: (Re Z_n, Im Z_n, H_n) with
 *          Z_n = sum_{k in n} sum_alpha d conj(h) / S and H_n = sum w(k), so that
 *          x_n = 4 df |Z_n| and [h|h]_n = 4 df H_n
 *   prec   SCS_PREC_*
 * theta, ups and seg are all host or all device pointers (mem_kind). */
int scs_evaluate(scs_ctx* ctx, int64_t P, const double* theta, int32_t prec, double* ups, double* seg,
                 int32_t mem_kind, void* stream);

/* ---- likelihood epilogues (Sec 2.1 - 2.2) ---------------------------- */

/* Statistics per row of scs_evaluate_stats. */
#define SCS_NSTATS 5

/* scs_evaluate for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  It calls no
 * hipMalloc, hipFree or other allocating routine: every buffer of the
 * evaluation (particle records, supports, edges, chunk records, per-segment
 * sums, the support sort, the launch descriptor) lives in one static device
 * array of SCS_NOALLOC_SCRATCH_BYTES, which every GPU the library runs on
 * holds from its first context until the process ends.
 *   theta, ups, seg  DEVICE pointers, layouts as for scs_evaluate (seg
 *                    nullable; when given, the per-segment sums use it and
 *                    need no scratch)
 *   stream           HIP stream the work is queued on (asynchronous)
 * The launch shape is the default one (the context's forced shape if a test
 * set one); a tuning cache is not consulted.  Results equal scs_evaluate's
 * with that shape, bit for bit.
 * The scratch is shared by every call on a GPU, from every context, thread
 * and stream, and keeps the last call's contents (what must start at zero is
 * cleared by kernels on the stream, no memset): calls that overlap on one GPU
 * race, and the caller must order them (one stream, or events).
 * Errors: EINVAL (bad arguments, or a request whose buffers exceed the
 * scratch, in which case nothing is launched: a particle takes about
 * 470 + 4 (N + 1) + 64 n_chunks bytes, plus 24 N without seg, with n_chunks
 * = K / 2048 on the default 2048-bin chunks), ESTATE (no data or model),
 * EDEVICE. */
#define SCS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int scs_evaluate_noalloc(scs_ctx* ctx, int64_t P, const double* theta, int32_t prec, double* ups, double* seg,
                         void* stream);

/* The generate-and-reduce of scs_evaluate with the likelihood epilogue.  For
 * the template h at unit amplitude and zero phase offset (the h of
 * scs_waveform), stats [P][SCS_NSTATS] out:
 *   [0] Upsilon_N                              (Sec 2.2)
 *   [1] hat O_N(d, h) = sum_n max_phi_n [d|h e^{i phi_n}]_n  (eq:semi-coherent_O)
 *   [2] <h|h>, the squared optimal SNR         (eqn:SNR_coherent)
 *   [3] Re <d|h>, [4] Im <d|h>, so that <d|h e^{i phi}> = Re(e^{-i phi} <d|h>)
 *                                              (eqn:inner_prod)
 * A row is NaN for an invalid theta and zero for an empty support.  Arguments,
 * memory kinds, stream semantics and errors as for scs_evaluate. */
int scs_evaluate_stats(scs_ctx* ctx, int64_t P, const double* theta, int32_t prec, double* stats, int32_t mem_kind,
                       void* stream);

/* <d|d> of the loaded data (eqn:inner_prod with a = b = d), computed when the
 * data are loaded; *dd is a host double.  Errors: EINVAL, ESTATE (no data). */
int scs_data_norm(const scs_ctx* ctx, double* dd);

/* Log-likelihoods of the templates A h e^{i phi} from scs_evaluate_stats rows,
 * without the normalisation constant (as Sec 2.1 drops it):
 *   logl_semi = -<d|d>/2 - A^2 <h|h>/2 + |A| hat O_N   (log hat L_N, Sec 2.2)
 *   logl_coh  = -<d|d>/2 - A^2 <h|h>/2 + A Re(e^{-i phi} <d|h>)  (eqn:LogL_coherent)
 * amp [P] (A); phase [P] (phi) or NULL, which maximises logl_coh over phi;
 * either output [P] may be NULL.  mem_kind applies to every array; device
 * arrays are read on the stream, host arrays are staged and the call
 * synchronises.  Errors: EINVAL, ESTATE (no data), EDEVICE. */
int scs_loglike(scs_ctx* ctx, int64_t P, const double* stats, const double* amp, const double* phase,
                double* logl_semi, double* logl_coh, int32_t mem_kind, void* stream);

/* Absolute amplitude A of the template (the factor that makes A h the strain
 * the data carry) for a source at luminosity distance D_L: the restricted
 * stationary-phase amplitude of the (2,2) mode,
 *   A = sqrt(5/24) pi^(-2/3) (G Mc / c^3)^(5/6) c / D_L,
 * Mc the detector-frame chirp mass (theta[p][0], solar masses), D_L in Mpc
 * (Sec 4: D_L is a 1/D_L prefactor of the waveform amplitude, cancelled by
 * the search statistic; Sec 3.3 draws it for every walker at the hand-off to
 * inference, whose coherent likelihood, eqn:LogL_coherent, needs it).  Feed
 * amp to scs_loglike.  theta [P][D], dl_mpc [P], amp [P] out; NaN for Mc <= 0,
 * D_L <= 0 or non-finite entries.  mem_kind as scs_loglike.  The amplitude
 * matches data whose noise and PSD are in strain units (the synthetic
 * generator's convention).  Errors: EINVAL, ESTATE, EDEVICE. */
int scs_distance_amplitude(scs_ctx* ctx, int64_t P, const double* theta, const double* dl_mpc, double* amp,
                           int32_t mem_kind, void* stream);

/* ---- one theta against many data streams (Sec 5.1) -------------------- */

/* Fill streams (DEVICE [n_chan][K][R][2], realisations innermost) with
 * d_r = scale * d + n_{r0 + r}, r = 0..R-1: d the loaded data, n Gaussian
 * noise of the loaded PSD in the convention <n|h> ~ N(0, <h|h>)
 * (eqn:inner_prod), n = sqrt(S / (4 df)) (g1 + i g2).  g1, g2 are the
 * Box-Muller normals of two 52-bit uniforms taken from one Philox4x32-10
 * block, counter (k, channel, r0 + r, 0x6e6f6973), key (seed low word, seed
 * high word), so that any realisation can be regenerated on its own.
 * Asynchronous on stream.  Errors: EINVAL (r0 + R > 2^32, NULL streams,
 * non-finite scale), ESTATE (no data), EDEVICE. */
int scs_make_realisations(scs_ctx* ctx, int64_t R, uint64_t seed, int64_t r0, double scale, double* streams,
                          void* stream);

/* For one theta (HOST [D]) and R data streams (DEVICE [n_chan][K][R][2], as
 * made by scs_make_realisations or by the caller), stats (DEVICE
 * [R][SCS_NSTATS]) = the rows of scs_evaluate_stats for each stream in place
 * of the loaded data.  The segment edges are theta's under the context's
 * segmentation (so, for EQUAL_SNR, the same for every stream).  The template
 * weights conj(h)/S are formed once; the reduction then streams every
 * stream's bins from HBM once.  NaN rows for an invalid theta.  The call
 * synchronises the stream (the edges are read back to cut the work).
 * Errors: EINVAL, ESTATE, ENOMEM, EDEVICE. */
int scs_evaluate_streams(scs_ctx* ctx, const double* theta, int64_t R, const double* streams, double* stats,
                         void* stream);

/* Per-particle support [k_lo, k_hi) and segment edges b_0..b_N (int32) from
 * the last scs_evaluate on this context, copied to host arrays
 * support [P][2] and bounds [P][N+1] (either may be NULL).  Synchronises the
 * context's last stream. */
int scs_last_bounds(scs_ctx* ctx, int64_t P, int32_t* support, int32_t* bounds);

/* Template h_alpha(f_k) for one theta, h_ri [n_chan][K][2], zero outside
 * the support, with the FP64 kernels (used to synthesise injections). */
int scs_waveform(scs_ctx* ctx, const double* theta, double* h_ri, int32_t mem_kind, void* stream);

/* Counters accumulated since the last reset: in-support particle-bin
 * evaluations, full-band particle-bin evaluations, and particles the block
 * scheme could not resolve.  Synchronises the device. */
int scs_ctx_stats(scs_ctx* ctx, int64_t* evals_support, int64_t* evals_band, int64_t* unresolved, int32_t reset);

/* Time the dominant kernel with HIP events on the stream it is launched on:
 * the generate-and-reduce, and in scs_evaluate_streams the streamed
 * reduction (its one-particle set-up evaluation is not recorded).
 * enable = 1 starts recording; the query returns the number of launches and
 * the summed milliseconds since enabling. */
int scs_ctx_profile(scs_ctx* ctx, int32_t enable, int64_t* launches, double* total_ms);

/* HBM bytes an evaluation of P particles with N segments needs on this
 * context beyond the loaded data (coefficients, edges, fragments), for
 * admission control. */
int scs_footprint(const scs_ctx* ctx, int64_t P, int32_t N, int32_t prec, size_t* bytes);

/* ---- batched evaluation --------------------------------------------- */

/* One swarm of a batched launch.  Segmentation mode and G come from the
 * item's context, N from the item. */
typedef struct scs_batch_item {
    scs_ctx* ctx;
    int32_t N;
    int32_t pad;
    int64_t P;
    const double* theta; /* dev [P][D] of the item's context */
    double* ups;         /* dev [P] */
    double* seg;         /* dev [P][N][3] or NULL */
} scs_batch_item;

/* Evaluate several swarms (uneven P and N, possibly different contexts on
 * one device) with ONE persistent generate-and-reduce launch per channel
 * count: a fixed grid of workgroups takes (swarm, chunk, particle group)
 * tiles of every item from a device counter.  The per-item prologues, edge
 * searches and finalizes are queued before and after it.  Results equal
 * scs_evaluate on each item alone, bit for bit.  Device pointers only.  Each
 * item uses a workspace of its context (one per item index), so calls whose
 * items share a context must be issued on one stream.  Errors: EINVAL (bad
 * items, items on different devices), ENOMEM, EDEVICE. */
int scs_evaluate_batched(const scs_batch_item* items, int32_t n_items, int32_t prec, void* stream);

/* Capture scs_evaluate_batched for fixed items into a HIP graph; replay it
 * with scs_graph_launch after updating theta in place (the items' theta, ups
 * and seg buffers must stay valid while the graph lives).  The graph owns
 * the workspaces its kernels use, so other calls on the same contexts, of
 * any size, leave it intact.  It reads the contexts' data, model and
 * segmentation as they were at the capture: the contexts must outlive the
 * graph, and after scs_load_data, scs_set_model or scs_define_segmentation
 * on one of them scs_graph_launch fails with SCS_ESTATE (build a new
 * graph).  scs_graph_destroy waits for the graph's last replay. */
typedef struct scs_graph scs_graph;
int scs_graph_create(scs_graph** out, const scs_batch_item* items, int32_t n_items, int32_t prec);
int scs_graph_launch(scs_graph* g, void* stream);
int scs_graph_destroy(scs_graph* g);

/* Tile-shape autotuner.  A launch shape of the generate-and-reduce kernel is
 * (waves per workgroup 1 | 2 | 4, bins per LDS-staged block 256 | 512 | 1024,
 * bins per chunk 1024 .. 8192, occupancy: the default instantiation or the
 * alternative one, two waves per SIMD for FP64 and four for mixed, with the
 * per-bin template on one or two channels).  scs_autotune times candidate
 * shapes for the P particles theta_dev (device [P][D]) and N segments of
 * this context by coordinate descent from the default shape (each
 * coordinate in turn, twice over) and keeps the fastest for later calls of
 * the same (P, N, precision) class, solo or batched.  The shape changes only
 * the order in which segment pieces are joined: results agree to rounding.
 * cache_path (nullable) is a text file of "key waves blocks L alt" lines, read
 * before tuning (a hit skips the timing) and rewritten after. */
int scs_autotune(scs_ctx* ctx, int64_t P, const double* theta_dev, int32_t N, int32_t prec, const char* cache_path);

/* The same for a batch as scs_evaluate_batched runs it (one fused launch,
 * four waves per workgroup): the launch's occupancy, then each item's LDS
 * block and chunk length (items with the most work first), each candidate
 * timed as the whole batched evaluation.  The shapes found are kept per item
 * class like scs_autotune's, so later batched calls, graphs built afterwards
 * and the server use them.  Errors as scs_evaluate_batched. */
int scs_autotune_batch(const scs_batch_item* items, int32_t n_items, int32_t prec, const char* cache_path);

/* ---- serving ------------------------------------------------------- */

/* A request loop for several concurrent searches (Sec 3: every search walks
 * its own hierarchy of swarms and segment counts).  Each search is a context
 * whose data stays on the device.  A worker thread admits submitted requests
 * in arrival order while a request slot is free and the HBM footprint of the
 * admitted requests (scs_footprint plus the request's theta and result
 * buffers) stays within hbm_budget; everything admitted since the last
 * launch goes into one batched launch (scs_evaluate_batched) on a free
 * stream, so requests that arrive while others run join the next launch and
 * their work overlaps on the device (continuous batching).  A request's
 * result equals scs_evaluate of the same particles alone.
 *
 * Contexts given to a server are used by its worker thread: the caller must
 * not use them concurrently until the server is destroyed.  Times are
 * seconds on the server's monotonic clock (scs_server_clock). */
typedef struct scs_server scs_server;

typedef struct scs_request_done {
    uint64_t id;
    int32_t status;   /* SCS_OK or the error code of its launch */
    int32_t pad;
    double t_submit;  /* scs_server_submit returned */
    double t_admit;   /* admitted (slot and memory reserved) */
    double t_launch;  /* its batch was queued on a stream */
    double t_done;    /* result copied to the caller's buffer */
} scs_request_done;

typedef struct scs_server_counters {
    int64_t submitted, completed, failed;
    int64_t launches;          /* batched launches */
    int64_t max_batch;         /* most requests in one launch */
    int64_t max_inflight;      /* most requests admitted at once */
    uint64_t hbm_in_use;       /* device bytes the request slots hold: the buffers of the admitted
                                  requests and those idle slots keep for reuse [bytes] */
    uint64_t hbm_peak;         /* the largest hbm_in_use seen at an admission */
} scs_server_counters;

/* max_inflight: request slots (1..1024); hbm_budget: bytes (> 0); n_streams:
 * HIP streams the launches rotate over (1..16, default priority). */
int scs_server_create(scs_server** out, int32_t device, int32_t max_inflight, uint64_t hbm_budget, int32_t n_streams);

/* Queue an evaluation of P particles (theta, HOST [P][D], copied before the
 * call returns) with N segments on search ctx.  ups (HOST [P]) must stay
 * valid until the request is reported by scs_server_poll.  A request whose
 * footprint alone exceeds the budget is rejected with EBUSY.  Errors:
 * EINVAL, EBUSY, ENOMEM (host copy of theta), ESTATE (server stopping). */
int scs_server_submit(scs_server* srv, scs_ctx* ctx, int32_t N, int64_t P, const double* theta, int32_t prec,
                      double* ups, uint64_t* id);

/* Report up to max_out finished requests (oldest first), waiting up to
 * wait_ms milliseconds for the first one; *n_out = number reported. */
int scs_server_poll(scs_server* srv, scs_request_done* out, int32_t max_out, int32_t wait_ms, int32_t* n_out);

int scs_server_stats(scs_server* srv, scs_server_counters* out);
double scs_server_clock(const scs_server* srv);

/* Finish every admitted request, fail the ones not yet admitted (status
 * ESTATE, reported by no further poll), and free the server. */
int scs_server_destroy(scs_server* srv);

/* ---- particle swarm (Sec 3.1) ---------------------------------------- */

/* Hyper-parameters of one rung (Table tab:PSO_hyperparams). */
typedef struct scs_pso_params {
    double omega;  /* inertia */
    double phi_p;  /* pull to the particle best */
    double phi_g;  /* pull to the swarm best */
    double eps[8]; /* minimum speed per dimension (eqn:PSO_min_velocity); eps[7] (e0) is
                      read by eccentric swarms only */
} scs_pso_params;

/* Create a swarm of P particles bound to ctx (its data, model and
 * segmentation), positions uniform in [lo, hi] (host [D] each, D the context's
 * theta width), zero
 * velocity.  periodic[d] = 1 wraps dimension d into [lo, hi).  Random numbers
 * come from Philox4x32-10 with key (seed low word, seed high word + swarm_id)
 * and counter (iteration, particle, dimension, stream). */
int scs_swarm_create(scs_ctx* ctx, scs_swarm** out, int64_t P, const double* lo, const double* hi,
                     const int32_t* periodic, uint64_t seed, uint32_t swarm_id);
int scs_swarm_destroy(scs_swarm* sw);

/* One iteration: on the first call only evaluate; afterwards move every
 * particle (eqn:PSO_velocity_rule then eqn:PSO_min_velocity, using the bests
 * of the previous iteration), evaluate Upsilon_N at the new positions, and
 * update particle and swarm bests (out-of-box or NaN values count as -inf). */
int scs_pso_step(scs_swarm* sw, const scs_pso_params* params, int32_t prec, void* stream);

/* One iteration of n swarms at once (the swarms of one rung of the
 * hierarchical search, Sec 3.2): each swarm's move as in scs_pso_step, then
 * ONE batched generate-and-reduce over all of them (scs_evaluate_batched:
 * each swarm at its context's current N), then each swarm's best update.
 * Every swarm ends in the state scs_pso_step would leave it in, bit for bit.
 * gbest_vals (host [n], nullable) receives each swarm's best value after the
 * iteration; the call then waits for the stream.  All swarms on one device,
 * each at most once; swarms of one context use its batch workspaces (one per
 * position in sws), so such calls go on one stream.  Errors: EINVAL (NULL or
 * repeated swarm, negative eps, swarms on different devices), ENOMEM,
 * EDEVICE. */
int scs_pso_step_swarms(scs_swarm* const* sws, int32_t n, const scs_pso_params* params, int32_t prec,
                        double* gbest_vals, void* stream);

/* Copy the swarm state to host arrays (any may be NULL): theta, vel, pbest
 * [P][D], pbest_val [P], gbest [D], gbest_val, iteration.  Synchronous. */
int scs_swarm_read(scs_swarm* sw, double* theta, double* vel, double* pbest, double* pbest_val, double* gbest,
                   double* gbest_val, uint32_t* iteration);

/* Restore a swarm state from host arrays (checkpoint / resume). */
int scs_swarm_write(scs_swarm* sw, const double* theta, const double* vel, const double* pbest,
                    const double* pbest_val, const double* gbest, double gbest_val, uint32_t iteration);

/* Device pointers to the swarm's live arrays (theta [P][D], ups [P]). */
int scs_swarm_device_ptrs(scs_swarm* sw, double** theta, double** ups);

/* Raw move kernel on caller buffers (dev): theta, vel [P][dim] updated in
 * place from pbest [P][dim] and gbest [dim]; lo, hi, periodic host [dim];
 * dim 7 or 8. */
int scs_pso_move(int64_t P, int32_t dim, double* theta, double* vel, const double* pbest, const double* gbest,
                 const scs_pso_params* params, const double* lo, const double* hi, const int32_t* periodic,
                 uint64_t seed, uint32_t swarm_id, uint32_t iteration, void* stream);

/* Raw best-update kernel on caller buffers (dev): vals [P]; pbest, pbest_val,
 * gbest [dim], gbest_val [1] updated in place; dim 7 or 8. */
int scs_pso_best(int64_t P, int32_t dim, const double* theta, const double* vals, const double* lo, const double* hi,
                 const int32_t* periodic, double* pbest, double* pbest_val, double* gbest, double* gbest_val,
                 void* stream);

/* Entries per theta row of the context's model: 7, or 8 when eccentric. */
int scs_theta_dim(const scs_ctx* ctx, int32_t* dim);

/* Shapes of a context's arguments, for callers that check their buffers:
 * theta row width (7, or 8 when eccentric), the segment count N of the
 * current segmentation (seg rows are [N][3]), and the channels and bins of
 * the loaded data (0 before any data).  Any output may be NULL.  Errors:
 * EINVAL (NULL ctx). */
int scs_ctx_info(const scs_ctx* ctx, int32_t* theta_dim, int32_t* N, int32_t* n_chan, int64_t* K);

/* ---- hierarchical multi-swarm search (Sec 3.1 - 3.2, app:PSO_params) -- */

typedef struct scs_search scs_search;

typedef struct scs_search_params {
    int32_t n_swarms;     /* swarms at the start, and clusters of every re-grouping (6 in the paper) */
    int32_t G;            /* node stride of the equal-[h|h] edges at every rung */
    int64_t particles;    /* per swarm at the start (10^4 in the paper); the total is conserved */
    double conv_tol;      /* a swarm has converged when its best value gained at most conv_tol ... */
    int32_t conv_window;  /* ... over its last conv_window iterations (2 over 50 in the paper) */
    int32_t kmeans_iters; /* cap on the Lloyd iterations of a re-grouping */
    int32_t prec;         /* SCS_PREC_* of every evaluation */
    int32_t pad;
    uint64_t seed;        /* swarm Philox key and k-means++ draws */
} scs_search_params;

/* One rung of the ladder: Upsilon_N with N segments (equal [h|h]) and the
 * rung's hyper-parameters and minimum speeds (tab:PSO_hyperparams). */
typedef struct scs_rung {
    int32_t N;
    int32_t max_iters;    /* iterations at most, converged or not */
    scs_pso_params prm;
} scs_rung;

typedef struct scs_rung_report {
    int32_t N;
    int32_t n_swarms;     /* swarms during the rung */
    int32_t iterations;   /* iterations run (the rung stops when every swarm converged) */
    int32_t converged;    /* swarms that met the convergence rule */
    double best_val;      /* best Upsilon_N over all swarms at the end of the rung */
    double seconds;       /* wall time of the rung, re-grouping included */
} scs_rung_report;

/* Create a search on ctx: n_swarms swarms of `particles` particles, uniform
 * in [lo, hi] (host [D], D the context's theta width; periodic[d] = 1 wraps
 * dimension d, may be NULL).
 * Errors: EINVAL, ENOMEM, and those of scs_swarm_create. */
int scs_search_create(scs_ctx* ctx, const scs_search_params* params, const double* lo, const double* hi,
                      const int32_t* periodic, scs_search** out);

/* Run one rung: before every rung but the first, re-group all particles by
 * k-means of their positions (features: each dimension scaled to the prior
 * box, periodic ones as the point (cos, sin) / 2 pi on the circle;
 * k = n_swarms; empty clusters dropped) into new swarms: positions,
 * velocities and best positions carry over, best values restart at -inf (a
 * swarm's best position starts at the best position of its particle with the
 * highest earlier best value); then define the rung's segmentation on the
 * context and iterate
 * every swarm that has not converged, all of them in one batched step per
 * iteration (as scs_pso_step_swarms), until each has converged (a converged
 * swarm stops moving) or max_iters.  The convergence rule runs on the device:
 * each swarm's last conv_window + 1 best values stay there, and a swarm that
 * converged is frozen by its record, so that every later kernel leaves it as
 * it is.  The host queues 8 iterations at a time and then reads the records
 * (three integers per swarm): one stream synchronisation per 8 iterations,
 * and the results are those of deciding after every iteration.  report may
 * be NULL. */
int scs_search_run_rung(scs_search* s, const scs_rung* rung, scs_rung_report* report, void* stream);

/* Current swarms: their number, sizes [n] and bests [n][D + 1] (position,
 * value; D the context's theta width); sizes and best may be NULL.
 * Synchronous. */
int scs_search_swarms(scs_search* s, int32_t* n_swarms, int64_t* sizes, double* best);

int scs_search_destroy(scs_search* s);

/* k-means on host data x [n][dim] (squared Euclidean distance): k-means++
 * seeding with splitmix64 draws from seed, then Lloyd iterations until no
 * label changes or iters; ties go to the lower index; empty clusters are
 * dropped and labels [n] renumbered by first appearance; centers [k][dim]
 * (may be NULL); *k_out = clusters kept.  The re-grouping's k-means on host
 * data, for callers that hold their points there.  Errors: EINVAL. */
int scs_kmeans(const double* x, int64_t n, int32_t dim, int32_t k, int32_t iters, uint64_t seed, int32_t* labels,
               double* centers, int32_t* k_out);

/* The same k-means on device data, as the search's re-grouping runs it: each
 * workgroup takes a run of 256 consecutive points, every sum is formed in a
 * fixed order (workgroups' partial sums added in workgroup order), so a call
 * gives the same labels every time.  They equal scs_kmeans's except where a point lies
 * within rounding of two centres or a draw falls within rounding of a
 * cumulative weight (the sums are ordered differently).  x (DEVICE [n][dim],
 * dim <= 16), labels (DEVICE [n], out), centers (DEVICE [k][dim], out, may
 * be NULL), *k_out (HOST) the clusters kept; 1 <= k <= 1024.  Allocates its
 * scratch; synchronises the stream.  Errors: EINVAL, ENOMEM, EDEVICE. */
int scs_kmeans_device(const double* x, int64_t n, int32_t dim, int32_t k, int32_t iters, uint64_t seed,
                      int32_t* labels, double* centers, int32_t* k_out, void* stream);

/* Thread-local description of the last error on this thread ("" if none). */
const char* scs_last_error(void);

/* ---- measurement ---------------------------------------------------- */

/* Peak microbenchmark of device `device`, the measured ceilings beside the
 * published ones that the generate-and-reduce kernels are compared with:
 *   out[0]  FP64 FMA rate, TFLOP/s (eight independent chains per lane)
 *   out[1]  FP32 FMA rate, TFLOP/s (non-packed instructions)
 *   out[2]  FP32 hardware sine rate, 1e12 per second
 *   out[3]  HBM streaming copy, TB/s of bytes read plus written (512 MiB each way)
 *   out[4]  the device clock HIP reports, GHz
 * Allocates 1 GiB of device memory for the copy and frees it.  Synchronous.
 * Errors: SCS_EINVAL (out NULL), SCS_ENOMEM, SCS_EDEVICE. */
int scs_peak_probe(int32_t device, double* out);

#ifdef __cplusplus
}
#endif

#endif /* SCS_H */
