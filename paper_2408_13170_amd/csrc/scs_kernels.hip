// Kernels of the semi-coherent statistic Upsilon_N (arXiv:2408.13170, Sec 2.2)
// for gfx950.  Layering:
//   k_bins        particle-independent per-bin products u = f^-7/6 d / S, q = f^-7/3 / S
//   k_prologue    per particle: PN coefficients (double-double where the phase
//                 is large), coalescence time, support window, response
//                 trig-polynomial, polynomial block length          (Sec 4)
//   k_bounds_*    per particle segment edges: equal [h|h], uniform,
//                 explicit                                          (Sec 2.2)
//   k_main_multi  generate-and-reduce over (chunk, particle group) tiles:
//                 data staged in LDS, one particle per lane, per-lane
//                 segmented accumulation                            (Sec 2.2)
//   k_finalize    term_n = 4 df |Z_n|^2 / H_n with the pieces of segments
//                 that straddle chunks joined, Upsilon = sum_n      (Sec 2.2);
//                 optionally the likelihood sums hat O_N, <h|h>, <d|h>
//   k_data_norm   <d|d>; k_loglike: log hat L_N and log L          (Sec 2.1-2.2)
//   k_waveform    template on the grid for one theta (injections, parity)
//   k_pso_*       particle-swarm move and best update               (Sec 3.1)
#include "scs_internal.hpp"
#include "scs_math.hpp"

// Global-memory qualifier.  Pointers the kernels read from memory (launch
// descriptors) are generic to the compiler, whose flat accesses also count
// against the LDS wait counter; casting them keeps global accesses apart
// from LDS waits.
#define GLOBAL __attribute__((address_space(1)))
// Constant-memory qualifier: read-only data at a wave-uniform address, which
// the compiler then reads with scalar loads into scalar registers.
#define CONSTANT __attribute__((address_space(4)))

namespace scs {

// Chebyshev nodes of the degree-5 block interpolant and the matrix taking
// node values to monomial coefficients in x in [-1, 1].
__constant__ double c_cheb_x[kNodes];
__constant__ double c_cheb_m[kNodes * kNodes];
// (cos, sin) of 2 pi i / kTrig, i = 0..kTrig-1, rounded from extended precision
__device__ double2 g_trig[kTrig];

// ============================================================== per-bin data
// The FP32 copy is scaled (u by su = sqrt(s), q by sq = s, s ~ 1 / median q)
// so that it stays far from FP32 overflow for strain-sized PSDs; the
// statistic is invariant under that scaling and Z, H are unscaled on exit.
__global__ void k_bins(GridArgs g, const double* __restrict__ d_ri, const double* __restrict__ psd,
                       double* __restrict__ b64, float* __restrict__ b32, double su, double sq)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= g.K) return;
    const double f = (g.k0 + (double)k) * g.df;
    const double a76 = pow(f, -7.0 / 6.0);
    const double a73 = a76 * a76;
    const int nv = bin_stride(g.nch);
    for (int c = 3 * g.nch; c < nv; ++c) {  // padding
        b64[k * nv + c] = 0.0;
        b32[k * nv + c] = 0.f;
    }
    for (int c = 0; c < g.nch; ++c) {
        const double S = psd[(int64_t)c * g.K + k];
        const double dr = d_ri[((int64_t)c * g.K + k) * 2];
        const double di = d_ri[((int64_t)c * g.K + k) * 2 + 1];
        const double ur = a76 * dr / S, ui = a76 * di / S, q = a73 / S;
        // per bin: [u0r, u0i, (u1r, u1i,) q0, (q1)]
        b64[k * nv + 2 * c] = ur;
        b64[k * nv + 2 * c + 1] = ui;
        b64[k * nv + 2 * g.nch + c] = q;
        b32[k * nv + 2 * c] = (float)(ur * su);
        b32[k * nv + 2 * c + 1] = (float)(ui * su);
        b32[k * nv + 2 * g.nch + c] = (float)(q * sq);
    }
}

// ============================================================== prologue helpers
struct PN {
    double piM, pref, psi2, psi3, psi4, a5, psi6c, psi7;
    int order;
};

// t(f) - t_c = d/df [PN phase] from the basis coefficients (FP64; used for
// the support window and the boundary weights, not for the phase itself).
__device__ inline double dphase_pn(const double* cf, double f)
{
    const double u = 1.0 / cbrt(f);  // f^-1/3
    const double u2 = u * u, u3 = u2 * u, u4 = u2 * u2, u5 = u4 * u, u6 = u3 * u3, u8 = u4 * u4;
    const double lnf = log(f);
    double s = -(5.0 / 3.0) * cf[0] * u8;
    s += -cf[1] * u6;
    s += -(2.0 / 3.0) * cf[2] * u5;
    s += -(1.0 / 3.0) * cf[3] * u4;
    s += cf[4] * u3;
    s += (1.0 / 3.0) * cf[5] * u2;
    s += cf[6] * u2 * (lnf * (1.0 / 3.0) + 1.0);
    s += (2.0 / 3.0) * cf[7] * u;
    if (cf[8] != 0.0) {
        // eccentric term: d/df [b_e f^-34/9] = -(34/9) b_e f^-43/9, f^-43/9 = u^14 u^(1/3)
        s += -(34.0 / 9.0) * cf[8] * (u8 * u6) * cbrt(u);
    }
    return s;
}

static_assert(C_COUNT <= kCoefStride, "the coefficient record holds every field");
// a bin index beyond any grid: no block length change ahead
constexpr double kNoBin = 0x1p40;

__global__ void k_prologue(PrologueArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.P) return;
    if (a.frozen && *a.frozen) {  // a converged swarm of a search: nothing to evaluate
        a.klo[p] = 0;
        a.khi[p] = 0;
        a.lg[p] = -1;
        return;
    }
    const int64_t S = a.stride;
    double* cf = a.coef;
    const int td = a.m.ecc ? kThetaMax : kTheta;
    const double* th = a.theta + (int64_t)td * p;
    double t[kThetaMax];
    bool ok = true;
    for (int i = 0; i < td; ++i) {
        t[i] = th[i];
        ok = ok && isfinite(t[i]);
    }
    const double Mc = t[0], eta = t[1], flow = t[2];
    const double e0 = a.m.ecc ? t[7] : 0.0;
    ok = ok && Mc > 0.0 && eta > 0.0 && eta <= 0.25 && flow > 0.0 && e0 >= 0.0 && e0 < 0.5;
    if (!ok) {
        a.klo[p] = 0;
        a.khi[p] = 0;
        a.lg[p] = -1;
        return;
    }
    const int J = a.m.pn_order;
    // ---- PN phase as sum_i b_i g_i(f) (cycles): f^-5/3, f^-1, f^-2/3, f^-1/3,
    //      ln f, f^1/3, f^1/3 ln f, f^2/3, plus f t_c and a constant.
    const dd x = dd_mul_d(dd{a.c.pitsun_hi, a.c.pitsun_lo}, Mc);  // pi T_sun Mc [s]
    const dd c0 = dd_mul(dd{a.c.k3_hi, a.c.k3_lo}, dd_pow_m53(x));  // (3/(256 pi)) (pi T_sun Mc)^-5/3
    const double piM = x.hi * pow(eta, -0.6);
    const double mu = cbrt(piM);
    const double lnmu = log(mu);
    const double pref = 3.0 / (256.0 * kPi * eta);
    const double eta2 = eta * eta, eta3 = eta2 * eta;
    const double psi2 = 3715.0 / 756.0 + 55.0 * eta / 9.0;
    const double psi3 = -16.0 * kPi;
    const double psi4 = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta2 / 72.0;
    const double a5 = kPi * (38645.0 / 756.0 - 65.0 * eta / 9.0);
    const double psi6c = 11583231236531.0 / 4694215680.0 - 640.0 * kPi * kPi / 3.0 - 6848.0 * kEulerGamma / 21.0 +
                         (-15737765635.0 / 3048192.0 + 2255.0 * kPi * kPi / 12.0) * eta + 76055.0 * eta2 / 1728.0 -
                         127825.0 * eta3 / 1296.0;
    const double b6 = -6848.0 / 21.0;
    const double psi7 = kPi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta2 / 756.0);
    // eccentric term (TaylorF2Ecc at leading order in e0^2, Newtonian order):
    // the Newtonian phase times -(2355/1462) e0^2 (f_low / f)^(19/9), i.e.
    // b_e f^-34/9 with b_e = -(2355/1462) e0^2 f_low^(19/9) c0, double-double
    dd be{0.0, 0.0};
    if (e0 != 0.0) {
        const dd k = dd_mul(dd_ratio(2355.0, 1462.0), two_prod(e0, e0));
        be = dd_mul(dd_mul(k, dd_pow_ratio(dd{flow, 0.0}, 19, 9)), c0);
        be = dd{-be.hi, -be.lo};
    }
    double b[9];
    b[0] = c0.hi;
    b[8] = be.hi;
    b[1] = J >= 2 ? pref * psi2 / piM : 0.0;
    b[2] = J >= 3 ? pref * psi3 / (mu * mu) : 0.0;
    b[3] = J >= 4 ? pref * psi4 / mu : 0.0;
    b[4] = J >= 5 ? pref * a5 : 0.0;
    b[5] = J >= 6 ? pref * mu * (psi6c + b6 * (1.3862943611198906188 + lnmu)) : 0.0;
    b[6] = J >= 6 ? pref * mu * b6 * (1.0 / 3.0) : 0.0;
    b[7] = J >= 7 ? pref * psi7 * mu * mu : 0.0;
    double phic = -0.125;
    if (J >= 5) phic += pref * a5 * (1.0 + 3.0 * lnmu + 1.5 * 1.7917594692280550008);
    // ---- t_c from t(f_low) = 0: t_c = -dPhi_PN/df(f_low); Newtonian part in double-double
    const dd five3 = dd_ratio(5.0, 3.0);
    const dd tN = dd_mul(dd_mul(five3, c0), dd_pow_m83(dd{flow, 0.0}));
    double cf_rest[9];
    cf_rest[0] = 0.0;
    for (int i = 1; i < 8; ++i) cf_rest[i] = b[i];
    cf_rest[8] = 0.0;
    const double trest = -dphase_pn(cf_rest, flow);
    dd tc = dd_add(tN, dd{trest, 0.0});
    if (e0 != 0.0) {
        // eccentric part of -dPhi/df(f_low): -(157/43) e0^2 times the Newtonian one
        const dd te = dd_mul(dd_mul(dd_ratio(157.0, 43.0), two_prod(e0, e0)), tN);
        tc = dd_add(tc, dd{-te.hi, -te.lo});
    }
    const dd tau = dd_mul_d(tc, a.g.df);  // t_c / T, T = 1/df
    // ---- support window
    int64_t klo = 0, khi = a.g.K;
    const double tcs = tc.hi + tc.lo;
    if (a.m.support == 1) {
        // first bin with f_k >= f_low, compared exactly: (k0 + k) df as double-double
        int64_t k = (int64_t)ceil(flow / a.g.df - a.g.k0);
        k = k < 0 ? 0 : k;
        for (int it = 0; it < 4; ++it) {
            if (k > 0) {
                const dd fm = two_prod(a.g.k0 + (double)(k - 1), a.g.df);
                if (fm.hi > flow || (fm.hi == flow && fm.lo >= 0.0)) { --k; continue; }
            }
            const dd f0 = two_prod(a.g.k0 + (double)k, a.g.df);
            if (f0.hi < flow || (f0.hi == flow && f0.lo < 0.0)) { ++k; continue; }
            break;
        }
        klo = k > a.g.K ? a.g.K : k;
        // first bin at or after klo with t(f_k) >= T_obs (t rises with f)
        int64_t lo = klo, hi = a.g.K;
        while (lo < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            const double fm = (a.g.k0 + (double)mid) * a.g.df;
            const double tm = tcs + dphase_pn(b, fm);
            if (tm >= a.m.t_obs) hi = mid; else lo = mid + 1;
        }
        khi = lo;
    }
    // ---- polynomial block length: the largest power of two (<= block_len)
    //      whose Taylor / Chebyshev remainders stay below 1e-12 cycles
    //      (phase) and 1e-11 relative (response), using the Newtonian scaling
    //      at the fastest-chirping point of the support, its start.
    // Both remainders fall as f rises (the chirp slows), so a length that
    // holds at one bin holds at every later one; blocks that start at or
    // after bin kup[i] may be 2^(i+1) times the support start's length.
    auto block_ok = [&](double fs, int l) {
        double taus = -dphase_pn(b, fs);
        taus = taus > 0.0 ? taus : 0.0;
        const double h = (double)(1 << (l - 1));
        const double r = h * a.g.df / fs;
        const double r2 = r * r, r6 = r2 * r2 * r2;
        // the eccentric term's sixth Taylor coefficient is ~17 times the
        // Newtonian one per unit size, and its size is <= 1.61 e0^2 of it
        const double ephi = 2.4 * taus * fs * r6 * (1.0 + 27.0 * e0 * e0);
        bool good = ephi <= 1e-12;
        if (a.m.response != 0) {
            // fourth orbital harmonic; the full response's arm-length
            // terms add harmonics of small amplitude only (its
            // interpolation error at the block's worst point is within
            // a few percent of the low-frequency response's)
            const double th_h = 4.0 * kTwoPi * kInvYear * (8.0 / 3.0) * (taus / fs) * a.g.df * h;
            const double t2 = th_h * th_h;
            good = good && (t2 * t2 * t2 / 11520.0) <= 1e-11;
        }
        return good;
    };
    int lg = -2;
    double kup[2] = {kNoBin, kNoBin};
    if (khi > klo) {
        const double fs = (a.g.k0 + (double)klo) * a.g.df;
        for (int l = a.lg_max; l >= 3; --l) {
            if (block_ok(fs, l)) { lg = l; break; }
        }
        // the sparse-grid template expands nothing in blocks: every theta resolves
        if (lg < 0 && a.m.sparse > 0) lg = a.lg_max;
        if (lg < 0) atomicAdd(a.unresolved, 1ULL);
        if (lg >= 3 && a.m.sparse == 0) {
            for (int i = 0; i < 2 && lg + 1 + i <= a.lg_max; ++i) {
                const int l = lg + 1 + i;
                int64_t lo = klo, hi = khi;  // first bin of [klo, khi) where l holds, or khi
                while (lo < hi) {
                    const int64_t mid = lo + (hi - lo) / 2;
                    if (block_ok((a.g.k0 + (double)mid) * a.g.df, l)) hi = mid; else lo = mid + 1;
                }
                // the bisection takes the bound as falling with f; where it
                // does not also hold at the support's end, keep the length
                if (lo >= khi || !block_ok((a.g.k0 + (double)(khi - 1)) * a.g.df, l)) break;
                kup[i] = (double)lo;
            }
        }
    } else {
        lg = a.lg_max;  // empty support: nothing to resolve
    }
    // ---- response: trig polynomial of degree 4 in the orbital angle, from
    //      nine samples (exact for degree <= 4)
    if (a.m.response == 1) {
        const Pol pol = polarisation(t[3], t[4], t[6]);
        const double ci = cos(t[5]);
        const double ap = 0.5 * (1.0 + ci * ci), ax = ci;
        double acc[36];
        for (int i = 0; i < 36; ++i) acc[i] = 0.0;
        for (int sIdx = 0; sIdx < 9; ++sIdx) {
            const double Phi = kTwoPi * sIdx / 9.0;
            double F[4];
            antenna_lf(Phi, a.m.cart0, pol, F);
            const double R[4] = {ap * F[0], -ax * F[1], ap * F[2], -ax * F[3]};
            double ch[5], sh[5];
            double s1, c1;
            sincos(Phi, &s1, &c1);
            harmonics(c1, s1, ch, sh);
            for (int f = 0; f < 4; ++f) {
                acc[9 * f] += R[f] * (1.0 / 9.0);
                for (int k = 1; k <= 4; ++k) {
                    acc[9 * f + k] += R[f] * ch[k] * (2.0 / 9.0);
                    acc[9 * f + 4 + k] += R[f] * sh[k] * (2.0 / 9.0);
                }
            }
        }
        for (int i = 0; i < 36; ++i) cf[p * kCoefStride + (C_RESP + i)] = acc[i];
    } else if (a.m.response == 2) {
        const Pol pol = polarisation(t[3], t[4], t[6]);
        double sl, cl, sb, cb;
        sincos(t[3], &sl, &cl);
        sincos(t[4], &sb, &cb);
        const double ci = cos(t[5]);
        double rec[FD_COUNT];
        rec[FD_N + 0] = cb * cl;
        rec[FD_N + 1] = cb * sl;
        rec[FD_N + 2] = sb;
        for (int i = 0; i < 3; ++i) {
            rec[FD_P + i] = pol.P[i];
            rec[FD_Q + i] = pol.Q[i];
        }
        rec[FD_AP] = 0.5 * (1.0 + ci * ci);
        rec[FD_AX] = ci;
        for (int i = 0; i < FD_COUNT; ++i) cf[p * kCoefStride + (C_RESP + i)] = rec[i];
    }
    if (a.m.response != 0) {
        double sl, cl;
        sincos(t[3], &sl, &cl);
        const double cb = cos(t[4]);
        cf[p * kCoefStride + C_DC] = -kAuOverC * cb * cl;
        cf[p * kCoefStride + C_DS] = -kAuOverC * cb * sl;
    }
    cf[p * kCoefStride + C_C0H] = c0.hi;
    cf[p * kCoefStride + C_C0L] = c0.lo;
    for (int i = 1; i < 8; ++i) cf[p * kCoefStride + (C_B1 + i - 1)] = b[i];
    cf[p * kCoefStride + C_PHIC] = phic;
    cf[p * kCoefStride + C_BEH] = be.hi;
    cf[p * kCoefStride + C_BEL] = be.lo;
    cf[p * kCoefStride + C_TAUH] = tau.hi;
    cf[p * kCoefStride + C_TAUL] = tau.lo;
    cf[p * kCoefStride + C_TC] = tcs;
    cf[p * kCoefStride + C_TCL] = tc.lo - (tcs - tc.hi);
    cf[p * kCoefStride + C_LGUP] = kup[0];
    cf[p * kCoefStride + C_LGUP + 1] = kup[1];
    a.klo[p] = (int32_t)klo;
    a.khi[p] = (int32_t)khi;
    a.lg[p] = (int8_t)lg;
    if (lg >= 0 && khi > klo) atomicAdd(a.evals, (unsigned long long)(khi - klo));
}

// ============================================================== block polynomials
// Taylor coefficients in j (bins from a sub-block centre fc = Kc df) of the
// eight PN basis functions f^-5/3, f^-1, f^-2/3, f^-1/3, ln f, f^1/3,
// f^1/3 ln f, f^2/3, m = 0..5.  They depend on the grid only, so one table per
// sub-block length (level lg, Lp = 2^lg) is built once per context; entry
// [i*6 + m], plus G[0][0] as a double-double ([kGHi] = hi, [kGLo] = lo).
__global__ void k_gtab(GridArgs g, int lg, int64_t nsub, double* __restrict__ tab)
{
    const int64_t sidx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sidx >= nsub) return;
    const int64_t Lp = (int64_t)1 << lg;
    const double Kc = g.k0 + (double)(sidx * Lp + Lp / 2);
    const dd fc = two_prod(Kc, g.df);
    const double eps = g.df / fc.hi;
    const double u = rcbrt(fc.hi);  // f^-1/3
    const double u2 = u * u;
    const double lnf = log(fc.hi) + fc.lo / fc.hi;
    // the power functions, the last the eccentric term's f^-34/9 = u^11 u^(1/3)
    const double u11 = u2 * u2 * u2 * u2 * u2 * u;
    const double pw[7] = {u2 * u2 * u, u2 * u, u2, u, 1.0 / u, 1.0 / u2, u11 * cbrt(u)};
    const double sig[7] = {-5.0 / 3.0, -1.0, -2.0 / 3.0, -1.0 / 3.0, 1.0 / 3.0, 2.0 / 3.0, -34.0 / 9.0};
    const int slot[7] = {0, 1, 2, 3, 5, 7, 8};
    double epow[kNodes], lnser[kNodes], f13[kNodes];
    double e = 1.0;
    for (int m = 0; m < kNodes; ++m) {
        epow[m] = e;
        e *= eps;
    }
    lnser[0] = lnf;
    for (int m = 1; m < kNodes; ++m) lnser[m] = ((m & 1) ? 1.0 : -1.0) * epow[m] / m;
    double* out = tab + sidx * kGStride;
    for (int i = 0; i < 7; ++i) {
        double bin = 1.0;
        for (int m = 0; m < kNodes; ++m) {
            const double gim = pw[i] * bin * epow[m];
            out[slot[i] * kNodes + m] = gim;
            if (i == 4) f13[m] = gim;
            bin *= (sig[i] - m) / (m + 1.0);
        }
    }
    for (int m = 0; m < kNodes; ++m) out[4 * kNodes + m] = lnser[m];
    for (int m = 0; m < kNodes; ++m) {
        double s = 0.0;
        for (int q = 0; q <= m; ++q) s = __builtin_fma(f13[q], lnser[m - q], s);
        out[6 * kNodes + m] = s;
    }
    const dd g0 = dd_pow_m53(fc);
    out[kGHi] = g0.hi;
    out[kGLo] = g0.lo;
    const dd ge = dd_pow_ratio(fc, -34, 9);
    out[kGEHi] = ge.hi;
    out[kGELo] = ge.lo;
    for (int q = kGELo + 1; q < kGStride; ++q) out[q] = 0.0;
}

struct PhasePoly {
    double ph[kNodes];  // phase [cycles] (GW + Doppler), monomials in x = j / h; ph[0] in [-0.5, 0.5)
};
template <int NR>
struct RespPolyN {
    double r[NR][kNodes];  // response R_A re, R_A im, R_E re, R_E im (, R_T re, R_T im), monomials in x
};
using RespPoly = RespPolyN<4>;

// Per-lane polynomial set-up for one sub-block of length 2h centred on
// absolute bin Kc: phase Taylor coefficients from the basis table (wave-
// uniform, scalar loads), constant term reduced exactly in double-double;
// for the LISA response, response and Doppler interpolated at the Chebyshev
// nodes.  Returns the GW phase coefficients a[] (x-space) for node times.
template <int RM, int NR = 4>
__device__ inline void block_setup(const GLOBAL double* __restrict__ cf, int64_t S, int64_t p, double Kc, int lg,
                                   const GLOBAL double* __restrict__ G, const GridArgs& g, const ModelArgs& m,
                                   PhasePoly& out, RespPolyN<NR>& resp)
{
    const double h = (double)(1 << (lg - 1));
    const double c0h = cf[p * kCoefStride + C_C0H];
    double ci[8];
    ci[0] = c0h;
#pragma unroll
    for (int i = 1; i < 8; ++i) ci[i] = cf[p * kCoefStride + (C_B1 + i - 1)];
    double a[kNodes];
#pragma unroll
    for (int mm = 0; mm < kNodes; ++mm) a[mm] = 0.0;
    // one basis function at a time, so only six table values are live
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int mm = 0; mm < kNodes; ++mm)
            if (!(i == 0 && mm == 0)) a[mm] = __builtin_fma(ci[i], G[i * kNodes + mm], a[mm]);
    }
    double ecc_c = 0.0;  // the eccentric term's constant, reduced in double-double
    if (m.ecc) {
        const double beh = cf[p * kCoefStride + C_BEH];
        if (beh != 0.0) {
#pragma unroll
            for (int mm = 1; mm < kNodes; ++mm) a[mm] = __builtin_fma(beh, G[8 * kNodes + mm], a[mm]);
            ecc_c = dd_frac(dd_mul(dd{beh, cf[p * kCoefStride + C_BEL]}, dd{G[kGEHi], G[kGELo]}));
        }
    }
    {
        // constant term: frac(Kc tau) + frac(c0 f^-5/3) + frac(rest), cycles
        const double tauh = cf[p * kCoefStride + C_TAUH], taul = cf[p * kCoefStride + C_TAUL];
        dd lin = two_prod(Kc, tauh);
        lin.lo = __builtin_fma(Kc, taul, lin.lo);
        const dd n0 = dd_mul(dd{c0h, cf[p * kCoefStride + C_C0L]}, dd{G[kGHi], G[kGLo]});
        const double rest = a[0] + cf[p * kCoefStride + C_PHIC];
        const double c = dd_frac(lin) + dd_frac(n0) + (rest - rint(rest)) + ecc_c;
        a[0] = c - rint(c);
        a[1] += tauh + taul;
    }
    double hp = 1.0;
#pragma unroll
    for (int mm = 0; mm < kNodes; ++mm) {
        a[mm] *= hp;
        out.ph[mm] = a[mm];
        hp *= h;
    }
    if constexpr (RM != 0) {
#pragma unroll
        for (int f = 0; f < NR; ++f)
#pragma unroll
            for (int mm = 0; mm < kNodes; ++mm) resp.r[f][mm] = 0.0;
        const double dcx = cf[p * kCoefStride + C_DC], dsx = cf[p * kCoefStride + C_DS];
        const double inv_hdf = 1.0 / (h * g.df);
#pragma unroll 1
        for (int n = 0; n < kNodes; ++n) {
            __asm__ volatile("" ::: "memory");  // reload coefficients per node instead of pinning 36 registers
            const double xn = c_cheb_x[n];
            // t = (dPhi/dj) / df ; dPhi/dj = (1/h) sum m a_m x^(m-1)
            double d = 5.0 * a[5];
            d = __builtin_fma(d, xn, 4.0 * a[4]);
            d = __builtin_fma(d, xn, 3.0 * a[3]);
            d = __builtin_fma(d, xn, 2.0 * a[2]);
            d = __builtin_fma(d, xn, a[1]);
            double orb = m.orb0_cyc + d * inv_hdf * kInvYear;  // orbital angle [cycles]
            orb -= rint(orb);
            double s1, c1;
            sincos2pi(orb, &s1, &c1);
            const double fn = (Kc + xn * h) * g.df;
            const double dop = fn * (dcx * c1 + dsx * s1);
            if constexpr (RM == 2) {
                const double cz = __builtin_fma(m.cart_c, c1, m.cart_s * s1);
                const double sz = __builtin_fma(m.cart_s, c1, -(m.cart_c * s1));
                double rv[NR];
                fd_response<NR / 2>(fn, c1, s1, cz, sz, cf + (p * kCoefStride + C_RESP), rv);
#pragma unroll
                for (int f = 0; f < NR; ++f)
#pragma unroll
                    for (int mm = 0; mm < kNodes; ++mm)
                        resp.r[f][mm] = __builtin_fma(c_cheb_m[mm * kNodes + n], rv[f], resp.r[f][mm]);
            } else {
                double ch[5], sh[5];
                harmonics(c1, s1, ch, sh);
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    __asm__ volatile("" ::: "memory");  // nine coefficients live at a time
                    const GLOBAL double* cc = cf + p * kCoefStride + (C_RESP + 9 * f);
                    double rv = cc[0];
#pragma unroll
                    for (int k = 1; k <= 4; ++k)
                        rv = __builtin_fma(cc[k], ch[k], __builtin_fma(cc[4 + k], sh[k], rv));
#pragma unroll
                    for (int mm = 0; mm < kNodes; ++mm)
                        resp.r[f][mm] = __builtin_fma(c_cheb_m[mm * kNodes + n], rv, resp.r[f][mm]);
                }
            }
#pragma unroll
            for (int mm = 0; mm < kNodes; ++mm) out.ph[mm] = __builtin_fma(c_cheb_m[mm * kNodes + n], dop, out.ph[mm]);
        }
        out.ph[0] -= rint(out.ph[0]);
    }
}

// Horner's rule for a polynomial of degree D (D + 1 coefficients, lowest first).
template <int D>
__device__ __forceinline__ double horner(const double* c, double x)
{
    double v = c[D];
#pragma unroll
    for (int i = D - 1; i >= 0; --i) v = __builtin_fma(v, x, c[i]);
    return v;
}
__device__ __forceinline__ double horner5(const double* c, double x)
{
    double v = c[5];
    v = __builtin_fma(v, x, c[4]);
    v = __builtin_fma(v, x, c[3]);
    v = __builtin_fma(v, x, c[2]);
    v = __builtin_fma(v, x, c[1]);
    return __builtin_fma(v, x, c[0]);
}
// The mixed path's phase-residual and response polynomials are cubic (see
// the block set-up).
constexpr int kRespMixed = 4;
__device__ __forceinline__ float horner3f(const float* c, float x)
{
    float v = c[3];
    v = __builtin_fmaf(v, x, c[2]);
    v = __builtin_fmaf(v, x, c[1]);
    return __builtin_fmaf(v, x, c[0]);
}

// ============================================================== boundaries
__device__ __forceinline__ double wave_incl_scan(double v, int lane)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Dense weight w(k) = sum_alpha q_alpha(k) |R_alpha(t(f_k))|^2 (RM: the
// response model, 0 = none, 1 = low-frequency, 2 = full).
template <int RM>
__device__ inline double weight_at(const CONSTANT double* __restrict__ cf, int64_t S, int64_t p, int64_t k, const GridArgs& g,
                                   const ModelArgs& m, const double* __restrict__ b64, const double* bcoef, double tc)
{
    if constexpr (RM == 0) {
        return b64[k * 3 + 2];
    } else {
        const double f = (g.k0 + (double)k) * g.df;
        const double t = tc + dphase_pn(bcoef, f);
        double orb = m.orb0_cyc + t * kInvYear;
        orb -= rint(orb);
        double s1, c1;
        sincos2pi(orb, &s1, &c1);
        if constexpr (RM == 2) {
            const double cz = __builtin_fma(m.cart_c, c1, m.cart_s * s1);
            const double sz = __builtin_fma(m.cart_s, c1, -(m.cart_c * s1));
            if (g.nch == 3) {
                double rv[6];
                fd_response<3>(f, c1, s1, cz, sz, cf + (p * kCoefStride + C_RESP), rv);
                const double* q = b64 + k * bin_stride(3) + 6;
                return q[0] * (rv[0] * rv[0] + rv[1] * rv[1]) + q[1] * (rv[2] * rv[2] + rv[3] * rv[3]) +
                       q[2] * (rv[4] * rv[4] + rv[5] * rv[5]);
            }
            double rv[4];
            fd_response<2>(f, c1, s1, cz, sz, cf + (p * kCoefStride + C_RESP), rv);
            return b64[k * 6 + 4] * (rv[0] * rv[0] + rv[1] * rv[1]) + b64[k * 6 + 5] * (rv[2] * rv[2] + rv[3] * rv[3]);
        }
        double ch[5], sh[5];
        harmonics(c1, s1, ch, sh);
        double rv[4];
        for (int fi = 0; fi < 4; ++fi) {
            double cc[9];
            for (int kk = 0; kk < 9; ++kk) cc[kk] = cf[p * kCoefStride + (C_RESP + 9 * fi + kk)];
            rv[fi] = trig4(cc, ch, sh);
        }
        return b64[k * 6 + 4] * (rv[0] * rv[0] + rv[1] * rv[1]) + b64[k * 6 + 5] * (rv[2] * rv[2] + rv[3] * rv[3]);
    }
}

// Equal-[h|h] edges (rule: nodes k_lo + jG and k_hi - 1, W linear between
// nodes, C(k) = sum_{i<k} W(i), b_n = min{k : C(k) >= (n/N) C(k_hi)}).  One
// wave per particle; 63 node intervals per round; two passes (total, then
// edges), the second reading the first's node weights from LDS as far as
// a.wcache reaches and recomputing the rest.
// Three waves per SIMD fit without spills (168 VGPRs); the kernel is
// latency-bound, so residency is what counts.
template <int RM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void k_bounds_equal(BoundArgs a)
{
    const int64_t p = blockIdx.x;
    const int lane = threadIdx.x;
    if (p >= a.P) return;
    const int N = a.N;
    int32_t* bo = a.bounds + p * (int64_t)(N + 1);
    const int lgp = a.lg[p];
    const int64_t klo = a.klo[p], khi = a.khi[p];
    if (lgp < 0 || khi <= klo) {
        for (int n = lane; n <= N; n += 64) bo[n] = (int32_t)klo;
        return;
    }
    const int64_t S = a.stride;
    // the particle's coefficients are the same in every lane: scalar loads
    // (the kernel writes only the edges, so the scalar cache stays valid)
    const CONSTANT double* cfc = (const CONSTANT double*)a.coef;
    double bcoef[9];
    bcoef[0] = cfc[p * kCoefStride + C_C0H];
    for (int i = 1; i < 8; ++i) bcoef[i] = cfc[p * kCoefStride + (C_B1 + i - 1)];
    bcoef[8] = cfc[p * kCoefStride + C_BEH];
    const double tc = cfc[p * kCoefStride + C_TC];
    const int64_t G = a.G;
    const int64_t len = khi - klo;
    const int64_t nreg = (len - 1) / G + 1;
    const int64_t nn = nreg + ((klo + (nreg - 1) * G != khi - 1) ? 1 : 0);  // nodes
    // node j position; node nn is khi (end of the final single-bin interval)
    auto node = [&](int64_t j) -> int64_t { return j >= nn ? khi : (j == nn - 1 ? khi - 1 : klo + j * G); };
    // interval integral over [node j, node j+1): g w_j + (w_{j+1} - w_j)(g - 1)/2,
    // the last interval being the single bin khi - 1 (w_{j+1} := w_j).
    // LDS: the weights of the first a.wcache nodes, computed in the first
    // pass and read in the second; C(node j0 + l + 1), l < 63, of the
    // current round, which each target lane searches by bisection
    extern __shared__ double s_w[];
    __shared__ double s_c[64];
    double total = 0.0;
    const int passes = N > 1 ? 2 : 1;  // one segment: no inner edges to place
    for (int pass = 0; pass < passes; ++pass) {
        __syncthreads();  // first-pass weights are in LDS
        double C0 = 0.0;
        int n_next = 1;
        for (int64_t j0 = 0; j0 < nn; j0 += 63) {
            const int64_t j = j0 + lane;
            double w = 0.0;
            if (j < nn) {
                if (pass == 1 && j < a.wcache) {
                    w = s_w[j];
                } else {
                    w = weight_at<RM>(cfc, S, p, node(j), a.g, a.m, a.b64, bcoef, tc);
                    if (j < a.wcache) s_w[j] = w;
                }
            }
            double wn = __shfl_down(w, 1, 64);
            if (j + 1 >= nn) wn = w;
            const int64_t xj = node(j), gj = node(j + 1) - xj;
            double I = 0.0;
            const bool live = lane < 63 && j < nn;
            if (live) I = (double)gj * w + (wn - w) * (double)(gj - 1) * 0.5;
            const double incl = wave_incl_scan(I, lane);
            const double chunk = __shfl(incl, 62, 64);
            if (pass == 0) {
                total += chunk;
                continue;
            }
            const double cend = C0 + incl;     // C(node j+1)
            const double cbeg = cend - I;      // C(node j)
            const double chunk_end = C0 + chunk;
            const int last_live = (nn - 1 - j0) < 62 ? (int)(nn - 1 - j0) : 62;
            __syncthreads();  // the previous round's searches are done
            if (lane < 63) s_c[lane] = cend;
            __syncthreads();
            // targets falling in this round
            while (n_next < N) {
                const int n = n_next + lane;
                const double tgt = ((double)n / (double)N) * total;
                const bool mine = n < N && (tgt <= chunk_end || j0 + 63 >= nn);
                // interval: first live lane with C(node j+1) >= tgt, else the
                // last live one (C is non-decreasing: the weights are >= 0)
                int sl = 0, sh = last_live;
                while (sl < sh) {
                    const int mid = (sl + sh) >> 1;
                    if (s_c[mid] >= tgt) sh = mid; else sl = mid + 1;
                }
                const int sel = sl;
                const double cb = __shfl(cbeg, sel, 64);
                const double ws = __shfl(w, sel, 64);
                const double wns = __shfl(wn, sel, 64);
                const int64_t xs = node(j0 + sel);
                const int64_t gs = node(j0 + sel + 1) - xs;
                if (mine) {
                    // min m in [0, g] with cb + S(m) >= tgt, S(m) = m w + (wn - w) m (m-1) / (2 g)
                    const double dlt = (wns - ws) / (2.0 * (double)gs);
                    const double D = tgt - cb;
                    double mst;
                    const double A = dlt, B = ws - dlt;
                    if (fabs(A) * (double)gs < 1e-12 * fabs(B) || A == 0.0) mst = D / B;
                    else {
                        const double disc = B * B + 4.0 * A * D;
                        mst = disc > 0.0 ? (2.0 * D) / (B + sqrt(disc)) : (double)gs;
                    }
                    int64_t mm = (int64_t)ceil(mst);
                    mm = mm < 0 ? 0 : (mm > gs ? gs : mm);
                    auto Sm = [&](int64_t q) {
                        const double qd = (double)q;
                        return cb + (qd * ws + (wns - ws) * (qd * (qd - 1.0)) / (2.0 * (double)gs));
                    };
                    while (mm > 0 && Sm(mm - 1) >= tgt) --mm;
                    while (mm < gs && Sm(mm) < tgt) ++mm;
                    bo[n] = (int32_t)(xs + mm);
                }
                const unsigned long long bal = __ballot(mine);
                const int cnt = __popcll(bal);
                n_next += cnt;
                if (cnt < 64) break;
            }
            C0 = chunk_end;
        }
        if (pass == 1) {
            for (int n = n_next + lane; n < N; n += 64) bo[n] = (int32_t)khi;
        }
    }
    if (lane == 0) {
        bo[0] = (int32_t)klo;
        bo[N] = (int32_t)khi;
    }
}

__global__ void k_bounds_simple(BoundArgs a)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = a.N;
    const int64_t p = idx / (N + 1);
    const int n = (int)(idx % (N + 1));
    if (p >= a.P) return;
    const int64_t klo = a.klo[p], khi = a.khi[p];
    int64_t v;
    if (a.lg[p] < 0 || khi <= klo) v = klo;
    else if (a.mode == 1) v = klo + (int64_t)(((__int128)n * (khi - klo)) / N);
    else {
        const int64_t e = a.edges[n];
        v = e < klo ? klo : (e > khi ? khi : e);
    }
    a.bounds[p * (int64_t)(N + 1) + n] = (int32_t)v;
}

// ============================================================== sparse-grid template
// The paper's way of evaluating the template (Sec 4, waveform and response
// paragraphs): waveform and response on a grid coarser than the FFT grid,
// cubic splines onto every bin.  The nodes of a particle are every S-th bin
// of its support plus the support's ends (spl_node); the quantities are the
// template phase in cycles (GW and Doppler terms, unreduced) and the real and
// imaginary parts of each channel's response; the splines are the not-a-knot
// cubic splines through the nodes.  Node values are exact evaluations (the
// phase reduced in double-double like the block set-up, its whole cycles
// from a plain FP64 evaluation), so the template differs from the per-bin
// one only by the interpolation.

// Node values of the quantities, one thread per (particle, node).
template <int NCH, int RM>
__global__ void k_spline_nodes(SplineArgs a)
{
    constexpr int NR = spl_nr(NCH), REC = spl_rec(NCH);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = i / a.nmax, j = i - p * a.nmax;
    if (p >= a.P || a.lg[p] < 0) return;
    const int64_t klo = a.klo[p], khi = a.khi[p];
    if (khi <= klo) return;
    const int64_t S = a.m.sparse;
    const int64_t n = spl_intervals(klo, khi, S);
    if (j > n) return;
    const double* cf = a.coef + p * kCoefStride;
    const double K = a.g.k0 + (double)spl_node(j, n, klo, khi, S);  // absolute bin, an integer
    const dd fK = two_prod(K, a.g.df);
    const double f = fK.hi;
    // A spline whose end interval is a few bins long multiplies the rounding
    // of the node values by up to ~S / (that length) next to it, so every term
    // of the phase above a few cycles, and the SPA time that sets the
    // Doppler term, is taken in double-double; the terms left in double stay
    // below ~10 cycles (rounding ~1e-15 cycles).
    const double u = 1.0 / cbrt(f), u2 = u * u, lnf = log(f) + fK.lo / fK.hi;
    // f^-1 in double-double: one Newton step from y0 = 1/f, with r = 1 - f y0
    const double y0 = 1.0 / f;
    const dd fy = two_prod(fK.hi, y0);
    const double rr = ((1.0 - fy.hi) - fy.lo) - fK.lo * y0;
    const dd inv = fast_two_sum(y0, y0 * rr);
    const dd t1 = dd_mul_d(inv, cf[C_B1]);
    const dd t2 = dd_mul_d(dd_pow_ratio(fK, -2, 3), cf[C_B2]);
    const dd t3 = dd_mul_d(dd_pow_ratio(fK, -1, 3), cf[C_B3]);
    const double small = cf[C_B4] * lnf + cf[C_B5] / u + cf[C_B6] * (lnf / u) + cf[C_B7] / u2 + cf[C_PHIC];
    const double u5 = u2 * u2 * u;
    const double beh = cf[C_BEH];
    // SPA time: t_c and the Newtonian term in double-double, the rest in double
    double bc[9];
    bc[0] = 0.0;
    for (int q = 1; q < 8; ++q) bc[q] = cf[C_B1 + q - 1];
    bc[8] = beh;
    const dd c0 = dd{cf[C_C0H], cf[C_C0L]};
    const dd tN = dd_mul(dd_mul(dd_ratio(5.0, 3.0), c0), dd_pow_m83(fK));
    const dd tcd = dd_add(dd{cf[C_TC], cf[C_TCL]}, dd{-tN.hi, -tN.lo});
    const double t = tcd.hi + (tcd.lo + dphase_pn(bc, f));  // stationary-phase time [s]
    double s1 = 0.0, c1 = 1.0, dop = 0.0;
    if constexpr (RM != 0) {
        double orb = a.m.orb0_cyc + t * kInvYear;
        orb -= rint(orb);
        sincos2pi(orb, &s1, &c1);
        dop = f * (cf[C_DC] * c1 + cf[C_DS] * s1);
    }
    // the phase modulo one cycle
    dd lin = two_prod(K, cf[C_TAUH]);
    lin.lo = __builtin_fma(K, cf[C_TAUL], lin.lo);
    const dd n0 = dd_mul(c0, dd_pow_m53(fK));
    double ecc = 0.0, ecc_whole = 0.0;
    if (beh != 0.0) {
        const dd fe = dd_pow_ratio(fK, -34, 9);
        ecc = dd_frac(dd_mul(dd{beh, cf[C_BEL]}, fe));
        ecc_whole = beh * fe.hi;
    }
    double phi = dd_frac(lin) + dd_frac(n0) + dd_frac(t1) + dd_frac(t2) + dd_frac(t3) + (small - rint(small)) +
                 ecc + dop;
    phi -= rint(phi);
    // whole cycles from the unreduced phase in double (error far below a cycle)
    const double whole = K * (cf[C_TAUH] + cf[C_TAUL]) + cf[C_C0H] * u5 + t1.hi + t2.hi + t3.hi + small +
                         ecc_whole + dop;
    double* r = a.spl + (p * a.nmax + j) * REC;
    r[0] = rint(whole - phi);
    r[1] = phi;
    if constexpr (RM == 1) {
        double ch[5], sh[5];
        harmonics(c1, s1, ch, sh);
        for (int fi = 0; fi < 4; ++fi) r[2 + fi] = trig4(cf + C_RESP + 9 * fi, ch, sh);
    } else if constexpr (RM == 2) {
        const double cz = __builtin_fma(a.m.cart_c, c1, a.m.cart_s * s1);
        const double sz = __builtin_fma(a.m.cart_s, c1, -(a.m.cart_c * s1));
        double rv[NR];
        fd_response<NCH>(f, c1, s1, cz, sz, cf + C_RESP, rv);
        for (int fi = 0; fi < NR; ++fi) r[2 + fi] = rv[fi];
    }
}

// Second derivatives M of the not-a-knot cubic spline through the nodes, one
// thread per (particle, quantity).  Interior nodes i = 1 .. n-1 make the
// first derivative continuous,
//   h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1} = 6 (s_i - s_{i-1}),
// with h_i the length and s_i the slope of interval i; not-a-knot makes the
// third derivative continuous at nodes 1 and n-1, which expresses M_0 and M_n
// through their neighbours and leaves a tridiagonal system in M_1 .. M_n-1,
// solved by forward elimination (slopes formed on the way) and back
// substitution.  Two intervals: the parabola through the three nodes (one
// M); one interval: the line (M = 0).  The phase enters as whole cycles plus
// fraction, so that differences keep their precision.  Each pass reads its
// node values BLK at a time into registers before using them, so one memory
// latency covers BLK steps of the recurrence.
template <int NCH>
__global__ __launch_bounds__(64) void k_spline_solve(SplineArgs a)
{
    constexpr int NR = spl_nr(NCH), NQ = spl_nq(NCH), REC = spl_rec(NCH);
    constexpr int BLK = 32;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = i / NQ;
    const int q = (int)(i - p * NQ);
    if (p >= a.P || a.lg[p] < 0) return;
    const int64_t klo = a.klo[p], khi = a.khi[p];
    if (khi <= klo) return;
    const int64_t S = a.m.sparse;
    const int64_t n = spl_intervals(klo, khi, S);
    double* base = a.spl + p * a.nmax * REC;
    const int mo = 2 + NR + q, to = 2 + NR + NQ + q;
    if (n <= 1) {
        for (int64_t j = 0; j <= n; ++j) base[j * REC + mo] = 0.0;
        return;
    }
    // the quantity at node j as a pair whose sum is its value: the phase as
    // whole cycles and fraction, a response part as itself and 0
    const int ia = q == 0 ? 0 : 1 + q, ib = q == 0 ? 1 : 1 + q;
    const double wb = q == 0 ? 1.0 : 0.0;
    const int64_t kb = klo / S;
    auto node = [&](int64_t jj) { return jj == 0 ? klo : (jj == n ? khi - 1 : (kb + jj) * S); };  // spl_node
    auto len = [&](int64_t jj) { return (double)(node(jj + 1) - node(jj)); };
    const double h0 = len(0), h1 = len(1);
    double a0 = base[ia], b0 = wb * base[ib];
    double a1 = base[REC + ia], b1 = wb * base[REC + ib];
    double a2 = base[2 * REC + ia], b2 = wb * base[2 * REC + ib];
    const double s0 = ((a1 - a0) + (b1 - b0)) / h0, s1 = ((a2 - a1) + (b2 - b1)) / h1;
    if (n == 2) {
        const double v = 2.0 * (s1 - s0) / (h0 + h1);
        for (int64_t j = 0; j <= 2; ++j) base[j * REC + mo] = v;
        return;
    }
    // forward elimination over rows 1 .. n-1; row 1 with
    // M_0 = ((h0 + h1) M_1 - h0 M_2) / h1 substituted, row n-1 with
    // M_n = ((h_{n-2} + h_{n-1}) M_{n-1} - h_{n-1} M_{n-2}) / h_{n-2}
    double dpv = 2.0 * (h0 + h1) + h0 * (h0 + h1) / h1;
    double upv = h1 - h0 * h0 / h1;
    double rpv = 6.0 * (s1 - s0);
    base[1 * REC + to] = dpv;
    base[1 * REC + mo] = rpv;
    double sp = s1, ap = a2, bp = b2;  // slope of row r's left interval, values at node r
    for (int64_t r0 = 2; r0 <= n - 1; r0 += BLK) {
        double va[BLK], vb[BLK];  // values at nodes r0 + 1 .. r0 + BLK
#pragma unroll
        for (int t = 0; t < BLK; ++t) {
            const int64_t j = r0 + 1 + t <= n ? r0 + 1 + t : n;
            va[t] = base[j * REC + ia];
            vb[t] = wb * base[j * REC + ib];
        }
#pragma unroll
        for (int t = 0; t < BLK; ++t) {
            const int64_t r = r0 + t;
            if (r <= n - 1) {
                const double hl = len(r - 1), hr = len(r);
                const double sr = ((va[t] - ap) + (vb[t] - bp)) / hr;
                double lower = hl, diag = 2.0 * (hl + hr);
                if (r == n - 1) {
                    diag += hr * (hl + hr) / hl;
                    lower -= hr * hr / hl;
                }
                const double w = lower / dpv;
                diag -= w * upv;
                const double rhs = 6.0 * (sr - sp) - w * rpv;
                base[r * REC + to] = diag;
                base[r * REC + mo] = rhs;
                dpv = diag;
                rpv = rhs;
                upv = hr;
                sp = sr;
                ap = va[t];
                bp = vb[t];
            }
        }
    }
    // back substitution, rows n-1 .. 1
    double mnext = rpv / dpv;
    base[(n - 1) * REC + mo] = mnext;
    for (int64_t r0 = n - 2; r0 >= 1; r0 -= BLK) {
        double rr[BLK], dg[BLK];
#pragma unroll
        for (int t = 0; t < BLK; ++t) {
            const int64_t r = r0 - t >= 1 ? r0 - t : 1;
            rr[t] = base[r * REC + mo];
            dg[t] = base[r * REC + to];
        }
#pragma unroll
        for (int t = 0; t < BLK; ++t) {
            const int64_t r = r0 - t;
            if (r >= 1) {
                const double up = r == 1 ? h1 - h0 * h0 / h1 : len(r);
                const double m = (rr[t] - up * mnext) / dg[t];
                base[r * REC + mo] = m;
                mnext = m;
            }
        }
    }
    const double m1 = base[1 * REC + mo], m2 = base[2 * REC + mo];
    base[mo] = ((h0 + h1) * m1 - h0 * m2) / h1;
    const double hl = len(n - 2), hr = len(n - 1);
    const double ma = base[(n - 1) * REC + mo], mb = base[(n - 2) * REC + mo];
    base[n * REC + mo] = ((hl + hr) * ma - hr * mb) / hl;
}

// The cubics of one spline interval [x_j, x_j + h] in u = k - x_j, from the
// node records of its two ends (r0 and the record after it):
// S(u) = y0 + c1 u + (M0 / 2) u^2 + (M1 - M0) / (6 h) u^3 with
// c1 = (y1 - y0) / h - h (2 M0 + M1) / 6; the phase's y1 - y0 is taken as
// (I1 - I0) + (phi1 - phi0) and its constant term is phi0 (cycles).  Without
// a right end (a one-bin support) the cubics are constants.
template <int NCH>
__device__ inline void spline_interval(const GLOBAL double* __restrict__ r0, bool right, double h, double* cph,
                                       double (*crs)[4])
{
    constexpr int NR = spl_nr(NCH), REC = spl_rec(NCH), MO = 2 + NR;
    if (!right) {
        cph[0] = r0[1];
        cph[1] = cph[2] = cph[3] = 0.0;
#pragma unroll
        for (int f = 0; f < NR; ++f) {
            crs[f][0] = r0[2 + f];
            crs[f][1] = crs[f][2] = crs[f][3] = 0.0;
        }
        return;
    }
    const GLOBAL double* r1 = r0 + REC;
    const double ih = 1.0 / h, h6 = h * (1.0 / 6.0), ih6 = ih * (1.0 / 6.0);
    {
        const double m0 = r0[MO], m1 = r1[MO];
        const double dy = (r1[0] - r0[0]) + (r1[1] - r0[1]);
        cph[0] = r0[1];
        cph[1] = dy * ih - h6 * (2.0 * m0 + m1);
        cph[2] = 0.5 * m0;
        cph[3] = (m1 - m0) * ih6;
    }
#pragma unroll
    for (int f = 0; f < NR; ++f) {
        const double m0 = r0[MO + 1 + f], m1 = r1[MO + 1 + f];
        const double y0 = r0[2 + f], y1 = r1[2 + f];
        crs[f][0] = y0;
        crs[f][1] = (y1 - y0) * ih - h6 * (2.0 * m0 + m1);
        crs[f][2] = 0.5 * m0;
        crs[f][3] = (m1 - m0) * ih6;
    }
}

// The sparse-grid template of particle 0 on the grid (injections, parity).
template <int NCH>
__global__ void k_waveform_spline(MainArgs a, double* __restrict__ h_ri)
{
    constexpr int NR = spl_nr(NCH);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.g.K) return;
    for (int c = 0; c < NCH; ++c) {
        h_ri[((int64_t)c * a.g.K + k) * 2] = 0.0;
        h_ri[((int64_t)c * a.g.K + k) * 2 + 1] = 0.0;
    }
    const int64_t klo = a.klo[0], khi = a.khi[0];
    if (a.lg[0] < 0 || k < klo || k >= khi) return;
    const int64_t S = a.m.sparse;
    const int64_t n = spl_intervals(klo, khi, S);
    int64_t j = k / S - klo / S;
    j = j < n - 1 ? j : n - 1;
    j = j > 0 ? j : 0;
    const int64_t xl = spl_node(j, n, klo, khi, S);
    const int64_t xr = spl_node(j < n ? j + 1 : j, n, klo, khi, S);
    double cph[4], crs[NR > 0 ? NR : 1][4];
    spline_interval<NCH>((const GLOBAL double*)a.spl + j * (int64_t)spl_rec(NCH), j < n, (double)(xr - xl), cph, crs);
    const double u = (double)(k - xl);
    double ph = horner<3>(cph, u);
    ph -= rint(ph);
    double sn, cs;
    sincos2pi(ph, &sn, &cs);
    const double amp = pow((a.g.k0 + (double)k) * a.g.df, -7.0 / 6.0);
    if constexpr (NR == 0) {
        h_ri[2 * k] = amp * cs;
        h_ri[2 * k + 1] = -amp * sn;
    } else {
        for (int c = 0; c < NCH; ++c) {
            const double rr = horner<3>(crs[2 * c], u), ri = horner<3>(crs[2 * c + 1], u);
            h_ri[((int64_t)c * a.g.K + k) * 2] = amp * (rr * cs + ri * sn);
            h_ri[((int64_t)c * a.g.K + k) * 2 + 1] = amp * (ri * cs - rr * sn);
        }
    }
}

// ============================================================== main kernel
// Work tile = (chunk of CB LDS blocks of L bins, group of 64 W particles).
// One lane = one particle; all lanes of a workgroup read the same staged bins
// (LDS broadcast).  Each lane accumulates Z and H of its current segment and
// closes it at its own edges; a chunk leaves per (particle, chunk) the sum of
// terms of segments complete inside it and the head / tail pieces of the
// segments that cross its edges, which k_finalize joins.
//
// Each lane keeps the bin of its next event: the start of its support (the
// sums drop the terms that bins of its first polynomial block before the
// support added) or the end of its current segment (the sums go out).  The
// wave adds bin after bin; one wave-wide test per bin sends the lanes whose
// event is due to the event code first.  That test is a compare and a
// branch per bin, so the frequent edges of many-segment swarms (one every
// bin or two across the 64 lanes at N = 4096) stay cheap.
template <class IntPtr>
__device__ __forceinline__ int bsearch_seg(IntPtr bo, int N, int64_t k)
{
    // largest n in [0, N-1] with b_n <= k
    int lo = 0, hi = N - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bo[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// The FP64 phase is carried in units of 1/kTrig cycle.  sin and cos of
// x = 2 pi s / kTrig for |s| <= 1/2 (|x| <= pi / 1024): Taylor polynomials
// in z = s^2 with the powers of the angle unit folded in, sine to degree 3
// and cosine to degree 2.  The remainders, x^5/120 < 3e-15 and x^4/24 <
// 4e-12, change the phasor's length by at most 4e-12 and its angle by less
// than 3e-15 rad, so Upsilon_N moves by at most 8e-12 relative.
constexpr double kPhaseUnits = kTrig;
constexpr double kArg = kTwoPi / kPhaseUnits;
constexpr double kSin1 = kArg;
constexpr double kSin3 = -(kArg * kArg * kArg) / 6.0;
constexpr double kCos2 = -(kArg * kArg) / 2.0;
// Adding 1.5 * 2^52 to a double of magnitude below 2^51 rounds it to the
// nearest integer, which then sits in the low mantissa bits.
constexpr double kRoundShift = 0x1.8p52;
constexpr int kTabMask = kTrig - 1;  // table index of an entry
constexpr int kTabZero = kTrig;      // index of the zero entry

// One bin of the FP64 path: template phase at bin offset j from the block
// centre, in units of 1/kTrig cycle (the block polynomial carries that
// power-of-two scale); e^{2 pi i phase} from the table entry of the nearest
// unit and the polynomials for the remainder; then
// Z += (sum_alpha u_alpha conj(R_alpha)) e^{2 pi i phase},
// H += sum_alpha q_alpha |R_alpha|^2.  bin = [uA re, uA im, uE re, uE im, qA, qE]
// (two channels) or [u re, u im, q]; amp scales the one-channel terms (0 or 1).
// Constants of the remainder polynomials, held in vector registers for the
// whole loop (an FP64 FMA reads at most one scalar register, so constants
// kept in scalar registers would be copied into a vector register per use).
struct SinCosK {
    double s3, s1, c2;
};

// What one bin adds to the running sums, kept apart from the sums so that
// two bins can be evaluated side by side before either is added:
// Z += (sr + i si)(cs + i sn), H += sum_alpha q_alpha w_alpha, where sr + i si
// is the data weighted by the conjugate response, (cs, sn) the phasor and
// w_alpha = |R_alpha|^2 (one channel: the amplitude factor).
template <typename T, int NCH>
struct BinTerms {
    T sr, si, sn, cs;
    T w[NCH], q[NCH];
};
__device__ __forceinline__ double fmx(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmx(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// Keeps terms formed where they are written: without it the compiler sinks
// the second bin's arithmetic past the first bin's event branch, where it no
// longer interleaves with the first bin's.
template <typename T, int NCH>
__device__ __forceinline__ void pin_terms(BinTerms<T, NCH>& b)
{
    __asm__ volatile("" : "+v"(b.sr), "+v"(b.si), "+v"(b.sn), "+v"(b.cs));
#pragma unroll
    for (int c = 0; c < NCH; ++c) __asm__ volatile("" : "+v"(b.w[c]), "+v"(b.q[c]));
}
template <typename T, int NCH>
__device__ __forceinline__ void add_terms(const BinTerms<T, NCH>& b, T& zr, T& zi, T& hh)
{
    zr = fmx(b.sr, b.cs, fmx(-b.si, b.sn, zr));
    zi = fmx(b.sr, b.sn, fmx(b.si, b.cs, zi));
    T h = hh;
#pragma unroll
    for (int c = NCH - 1; c >= 0; --c) h = fmx(b.q[c], b.w[c], h);
    hh = h;
}

template <int NCH, int D = 5>
__device__ __forceinline__ void bin_terms_fp64(double j, const double* __restrict__ bin,
                                               const double2* __restrict__ tab, const SinCosK& kk,
                                               const PhasePoly& poly, const RespPolyN<NCH == 3 ? 6 : 4>& rp,
                                               int tmask, int toff, double amp, BinTerms<double, NCH>& o)
{
    constexpr bool RESP = NCH >= 2;
    // the bin's data first, then the table read, so that both are in flight
    // while the response and the noise weight are evaluated
    double2 uA, uE, uT, qq, qT;
    double ur, ui, q1;
    if constexpr (NCH == 3) {
        uA = *reinterpret_cast<const double2*>(bin);
        uE = *reinterpret_cast<const double2*>(bin + 2);
        uT = *reinterpret_cast<const double2*>(bin + 4);
        qq = *reinterpret_cast<const double2*>(bin + 6);
        qT = *reinterpret_cast<const double2*>(bin + 8);
    } else if constexpr (RESP) {
        uA = *reinterpret_cast<const double2*>(bin);
        uE = *reinterpret_cast<const double2*>(bin + 2);
        qq = *reinterpret_cast<const double2*>(bin + 4);
    } else {
        ur = bin[0];
        ui = bin[1];
        q1 = bin[2];
    }
    const double pc = horner<D>(poly.ph, j);
    const double t = pc + kRoundShift;
    const int iq = ((int)(uint32_t)__double_as_longlong(t) & tmask) | toff;
    const double2 tt = tab[iq];
    // the table read is issued before the response work that hides its latency
    __builtin_amdgcn_sched_barrier(0);
    double sr, si;
    if constexpr (NCH == 3) {
        const double rar = horner<D>(rp.r[0], j), rai = horner<D>(rp.r[1], j);
        const double rer = horner<D>(rp.r[2], j), rei = horner<D>(rp.r[3], j);
        const double rtr = horner<D>(rp.r[4], j), rti = horner<D>(rp.r[5], j);
        sr = uA.x * rar;
        sr = __builtin_fma(uA.y, rai, sr);
        sr = __builtin_fma(uE.x, rer, sr);
        sr = __builtin_fma(uE.y, rei, sr);
        sr = __builtin_fma(uT.x, rtr, sr);
        sr = __builtin_fma(uT.y, rti, sr);
        si = uA.y * rar;
        si = __builtin_fma(-uA.x, rai, si);
        si = __builtin_fma(uE.y, rer, si);
        si = __builtin_fma(-uE.x, rei, si);
        si = __builtin_fma(uT.y, rtr, si);
        si = __builtin_fma(-uT.x, rti, si);
        o.w[0] = __builtin_fma(rar, rar, rai * rai);
        o.w[1] = __builtin_fma(rer, rer, rei * rei);
        o.w[2] = __builtin_fma(rtr, rtr, rti * rti);
        o.q[0] = qq.x;
        o.q[1] = qq.y;
        o.q[2] = qT.x;
    } else if constexpr (RESP) {
        const double rar = horner<D>(rp.r[0], j), rai = horner<D>(rp.r[1], j);
        const double rer = horner<D>(rp.r[2], j), rei = horner<D>(rp.r[3], j);
        sr = uA.x * rar;
        sr = __builtin_fma(uA.y, rai, sr);
        sr = __builtin_fma(uE.x, rer, sr);
        sr = __builtin_fma(uE.y, rei, sr);
        si = uA.y * rar;
        si = __builtin_fma(-uA.x, rai, si);
        si = __builtin_fma(uE.y, rer, si);
        si = __builtin_fma(-uE.x, rei, si);
        o.w[0] = __builtin_fma(rar, rar, rai * rai);
        o.w[1] = __builtin_fma(rer, rer, rei * rei);
        o.q[0] = qq.x;
        o.q[1] = qq.y;
    } else {
        sr = ur;
        si = ui;
        o.w[0] = amp;
        o.q[0] = q1;
    }
    const double s = pc - (t - kRoundShift);  // exact, |s| <= 1/2
    const double z = s * s;
    const double sn = s * __builtin_fma(z, kk.s3, kk.s1);
    const double cn = __builtin_fma(z, kk.c2, 1.0);
    o.sn = __builtin_fma(tt.y, cn, tt.x * sn);
    o.cs = __builtin_fma(tt.x, cn, -(tt.y * sn));
    o.sr = sr;
    o.si = si;
}
template <int NCH, int D = 5>
__device__ __forceinline__ void bin_fp64(double j, const double* __restrict__ bin, const double2* __restrict__ tab,
                                         const SinCosK& kk, const PhasePoly& poly,
                                         const RespPolyN<NCH == 3 ? 6 : 4>& rp, int tmask, int toff, double amp,
                                         double& zr, double& zi, double& hh)
{
    BinTerms<double, NCH> t;
    bin_terms_fp64<NCH, D>(j, bin, tab, kk, poly, rp, tmask, toff, amp, t);
    add_terms(t, zr, zi, hh);
}

// One bin of the mixed path: FP32 phase a0 + frac(a1h j) + residual(j)
// (a1h j exact, see the block set-up), hardware sin / cos of cycles, FP32
// response; plain FP32 partial sums over at most kMixedRun bins, which then
// enter FP64 segment sums.
// PH64: the phase is the FP64 cubic ph64 at ud (cycles), reduced and then
// rounded to FP32 (the sparse-grid template, whose spline intervals are too
// long for an FP32 residual), instead of a0 + frac(a1h j) + residual.
template <int NCH, bool PH64 = false>
__device__ __forceinline__ void bin_terms_mixed(float jf, const float* __restrict__ bin, const float* phf, float a1h,
                                                const float (*rf)[kRespMixed], float amp, BinTerms<float, NCH>& o,
                                                const double* ph64 = nullptr, double ud = 0.0)
{
    constexpr bool RESP = NCH >= 2;
    // the bin's data first, in flight while the phase and sin / cos are formed
    float4 u, tq;  // three channels: (uT re, uT im, qA, qE), then qT
    float2 qq;
    float ur, ui, q1, qt;
    if constexpr (NCH == 3) {
        u = *reinterpret_cast<const float4*>(bin);
        tq = *reinterpret_cast<const float4*>(bin + 4);
        qt = bin[8];
    } else if constexpr (RESP) {
        u = *reinterpret_cast<const float4*>(bin);
        qq = *reinterpret_cast<const float2*>(bin + 4);
    } else {
        ur = bin[0];
        ui = bin[1];
        q1 = bin[2];
    }
    float ph;
    if constexpr (PH64) {
        const double pd = horner<3>(ph64, ud);
        ph = (float)(pd - rint(pd));
    } else {
        const float pl = a1h * jf;
        const float f1 = __builtin_amdgcn_fractf(pl);  // [0, 1): sin and cos take revolutions
        float r = phf[3];
        r = __builtin_fmaf(r, jf, phf[2]);
        r = __builtin_fmaf(r, jf, phf[1]);
        ph = __builtin_fmaf(r, jf, phf[0] + f1);
    }
    const float sn = __builtin_amdgcn_sinf(ph);
    const float cs = __builtin_amdgcn_cosf(ph);
    if constexpr (NCH == 3) {
        const float rar = horner3f(rf[0], jf), rai = horner3f(rf[1], jf);
        const float rer = horner3f(rf[2], jf), rei = horner3f(rf[3], jf);
        const float rtr = horner3f(rf[4], jf), rti = horner3f(rf[5], jf);
        float sr = u.x * rar;
        sr = __builtin_fmaf(u.y, rai, sr);
        sr = __builtin_fmaf(u.z, rer, sr);
        sr = __builtin_fmaf(u.w, rei, sr);
        sr = __builtin_fmaf(tq.x, rtr, sr);
        sr = __builtin_fmaf(tq.y, rti, sr);
        float si = u.y * rar;
        si = __builtin_fmaf(-u.x, rai, si);
        si = __builtin_fmaf(u.w, rer, si);
        si = __builtin_fmaf(-u.z, rei, si);
        si = __builtin_fmaf(tq.y, rtr, si);
        si = __builtin_fmaf(-tq.x, rti, si);
        o.sr = sr;
        o.si = si;
        o.w[0] = __builtin_fmaf(rar, rar, rai * rai);
        o.w[1] = __builtin_fmaf(rer, rer, rei * rei);
        o.w[2] = __builtin_fmaf(rtr, rtr, rti * rti);
        o.q[0] = tq.z;
        o.q[1] = tq.w;
        o.q[2] = qt;
    } else if constexpr (RESP) {
        const float rar = horner3f(rf[0], jf), rai = horner3f(rf[1], jf);
        const float rer = horner3f(rf[2], jf), rei = horner3f(rf[3], jf);
        float sr = u.x * rar;
        sr = __builtin_fmaf(u.y, rai, sr);
        sr = __builtin_fmaf(u.z, rer, sr);
        sr = __builtin_fmaf(u.w, rei, sr);
        float si = u.y * rar;
        si = __builtin_fmaf(-u.x, rai, si);
        si = __builtin_fmaf(u.w, rer, si);
        si = __builtin_fmaf(-u.z, rei, si);
        o.sr = sr;
        o.si = si;
        o.w[0] = __builtin_fmaf(rar, rar, rai * rai);
        o.w[1] = __builtin_fmaf(rer, rer, rei * rei);
        o.q[0] = qq.x;
        o.q[1] = qq.y;
    } else {
        o.sr = ur * amp;
        o.si = ui * amp;
        o.w[0] = amp;
        o.q[0] = q1;
    }
    o.sn = sn;
    o.cs = cs;
}
template <int NCH, bool PH64 = false>
__device__ __forceinline__ void bin_mixed(float jf, const float* __restrict__ bin, const float* phf, float a1h,
                                          const float (*rf)[kRespMixed], float amp, float& pzr, float& pzi, float& phh,
                                          const double* ph64 = nullptr, double ud = 0.0)
{
    BinTerms<float, NCH> t;
    bin_terms_mixed<NCH, PH64>(jf, bin, phf, a1h, rf, amp, t, ph64, ud);
    add_terms(t, pzr, pzi, phh);
}

// Occupancy target (waves per SIMD), measured on MI355X: three for both
// (168 VGPRs; what spills is block set-up code, not the bin loop).  On the
// 2^20-bin step two waves (256 VGPRs, no spills) are within noise of three
// for FP64, and four are no faster for mixed; the autotuner can pick these
// alternatives (ALT) per evaluation class.
#ifndef SCS_WAVES_FP64
#define SCS_WAVES_FP64 3
#endif
#ifndef SCS_WAVES_MIXED
#define SCS_WAVES_MIXED 3
#endif
__host__ __device__ constexpr int main_waves_per_eu(int nch, bool mixed, bool alt)
{
    return mixed ? (alt ? 4 : SCS_WAVES_MIXED) : (nch == 3 ? 2 : (alt ? 2 : SCS_WAVES_FP64));
}
// Plain FP32 partial sums cover the bins between consecutive multiples of
// this (and a lane's own segment edges) before they enter the FP64 sums.
constexpr int kMixedRun = 32;
// The mixed path's polynomial blocks are twice as long as the FP64 bounds
// allow (up to the longest block).  Its response cubics drop the
// interpolant's T4 and T5 terms; the fourth orbital harmonic, at the largest
// amplitude the FP64 bound admits, then spans at most ~0.14 rad per half
// block, whose T4 coefficient is below 2e-6 of |R|: Upsilon moves by at most
// ~4e-6, within the path's 1e-5, and by ~1e-7 on the PSO workloads (the
// harmonic is far weaker than |R|).  Set-ups halve; four times as long would
// allow ~6e-5 at worst.
constexpr int kMixedLgBoost = 1;

// One work tile (chunk, particle group) of the generate-and-reduce.  Called
// by every thread of the workgroup; returns early, uniformly, when no
// particle of the group has support in the chunk.  s_trig holds the table
// and, at kTrig, a zero entry for idle one-channel lanes.
template <int NCH, bool MIXED, int RM, int TM>
__device__ __forceinline__ void main_tile(const MainArgs& a, const double* __restrict__ gtab, int64_t logical,
                                          unsigned char* smem, const double2* __restrict__ s_trig)
{
    constexpr int NV = bin_stride(NCH);  // values per bin
    constexpr bool RESP = NCH >= 2;
    constexpr int NR = NCH == 3 ? 6 : 4;  // response components
    const int64_t chunk = a.chunk0 + logical / a.n_groups;
    const int64_t group = logical % a.n_groups;
    const int tid = threadIdx.x;
    // slot s in the support-sorted order; particle p = perm[s]
    const int64_t s_idx = a.p0 + group * (int64_t)blockDim.x + tid;
    const int64_t p =
        (a.perm && s_idx < a.P_end) ? a.p0 + ((const GLOBAL int32_t*)a.perm)[s_idx - a.p0] : s_idx;
    const int K = (int)a.g.K;
    const int cbins = a.L * a.CB;
    const int Kc = (int)chunk * cbins;
    const int Ke = (Kc + cbins < K) ? Kc + cbins : K;
    // Block level (log2 of the polynomial block length) of the lane at a bin:
    // the prologue's level lgb at the support start, one more from the first
    // super-block (2^lg_max bins, aligned) that starts at or after the bin
    // from which twice the length meets the same bounds (up0), two more from
    // up1 (the chirp slows as f rises).  Levels change only at super-block
    // starts, so every block lies inside one super-block, and the choice
    // does not depend on how the band is cut into chunks.  The mixed path
    // then doubles the length (below lg_max).
    int lo = 0, hi = 0, lgb = -1;
    int up0 = INT32_MAX, up1 = INT32_MAX;
    if (p < a.P_end) {
        lgb = ((const GLOBAL int8_t*)a.lg)[p];
        if (TM == 0 && lgb >= 3 && lgb < a.lg_max) {
            const GLOBAL double* cfp = (const GLOBAL double*)a.coef + p * kCoefStride + C_LGUP;
            const double sup = (double)(1 << a.lg_max);
            const double u0 = ceil(cfp[0] / sup) * sup, u1 = ceil(cfp[1] / sup) * sup;
            up0 = u0 < 2147483647.0 ? (int)u0 : INT32_MAX;
            up1 = (lgb + 2 <= a.lg_max && u1 < 2147483647.0) ? (int)u1 : INT32_MAX;
        }
        if (lgb >= 0) {
            lo = ((const GLOBAL int32_t*)a.klo)[p];
            hi = ((const GLOBAL int32_t*)a.khi)[p];
        }
    }
    auto level_at = [&](int k) {
        int l = lgb + (k >= up0 ? 1 : 0) + (k >= up1 ? 1 : 0);
        if (MIXED && l >= 0 && l < a.lg_max) l += kMixedLgBoost;
        return l;
    };
    const int plo = lo, phi = hi;  // the whole support (the sparse-grid template's nodes)
    lo = lo > Kc ? lo : Kc;
    hi = hi < Ke ? hi : Ke;
    // the lane's level at its first bin in the chunk, the lowest in the chunk
    const int lg = level_at(lo);
    const bool has = lo < hi;
    if (!__syncthreads_or(has)) return;
    const int64_t S = a.stride;
    const int N = a.N;
    const GLOBAL int32_t* __restrict__ bo = (const GLOBAL int32_t*)a.bounds + (p < a.P_end ? p : a.p0) * (int64_t)(N + 1);
    // wave-uniform polynomial block length: the smallest requested in the wave
    int lgw = has ? lg : 30;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int t = __shfl_xor(lgw, o, 64);
        lgw = t < lgw ? t : lgw;
    }
    lgw = __builtin_amdgcn_readfirstlane(lgw);  // uniform: scalar registers and scalar loads downstream
    // segment state: current segment n, its end nb = b_{n+1}, and b_{n+2}
    // loaded ahead so that closing a segment does not wait for memory
    int n = 0, nb = INT32_MAX, nb2 = INT32_MAX;
    bool before = false;  // segment n started in an earlier chunk
    if (has) {
        n = bsearch_seg(bo, N, lo);
        nb = bo[n + 1];
        nb2 = bo[n + 2];  // used only while n + 2 <= N (rows are padded for the read)
        before = bo[n] < Kc;
    }
    // bin of the lane's next event: the support start when it lies inside
    // the chunk (the sums then drop what the lane's first polynomial block
    // added before it), else the end of the current segment
    int nxt = has ? (lo > Kc ? lo : nb) : INT32_MAX;
    double zr = 0.0, zi = 0.0, hh = 0.0;  // FP64 sums (mixed: of the FP32 partial sums)
    // mixed: plain FP32 sums of the bins since the last multiple of kMixedRun
    float qzr = 0.f, qzi = 0.f, qhh = 0.f;
    auto flush32 = [&]() {  // the FP32 partial sums enter the FP64 ones
        zr += (double)qzr;
        zi += (double)qzi;
        hh += (double)qhh;
        qzr = qzi = qhh = 0.f;
    };
    auto clear_sums = [&]() {
        zr = zi = hh = 0.0;
        qzr = qzi = qhh = 0.f;
    };
    // chunk record of this slot: [0..2] head piece (Z re, Z im, H) of the
    // segment open at the chunk start, [3..5] tail piece of the segment open
    // at its end; sums of segments that close inside the chunk go to zs
    GLOBAL double* const recp =
        (GLOBAL double*)a.rec + ((chunk - a.chunk0) * a.rec_stride + (s_idx < a.P_end ? s_idx - a.p0 : 0)) * kRec;
    GLOBAL double* zsp = (GLOBAL double*)a.zs + ((p < a.P_end ? p : a.p0) * (int64_t)N + n) * 3;  // Z, H of segment n
    // where segment n's sums go when it ends: the head record if it started
    // in an earlier chunk, else zs (a pointer rather than a flag, so that the
    // bin loop carries no per-lane condition)
    GLOBAL double* dst = before ? recp : zsp;
    // the mixed path's scales, read once: read at each segment end, the
    // compiler reloads them from the argument record (no alias proof against
    // the stores) and each segment end waits for the scalar load
    const double zscale32 = a.zscale32, hscale32 = a.hscale32;
    auto store_sums = [&](GLOBAL double* dst) {
        if constexpr (MIXED) {
            dst[0] = (zr + (double)qzr) * zscale32;
            dst[1] = (zi + (double)qzi) * zscale32;
            dst[2] = (hh + (double)qhh) * hscale32;
        } else {
            dst[0] = zr;
            dst[1] = zi;
            dst[2] = hh;
        }
    };
    // Event of the lanes with nxt <= k, before bin k is added.  The sums go
    // out and are cleared: at a segment end (reached here, or passed while
    // the wave skipped bins where this lane has none after its support) to
    // dst; at the support start to zs of the first segment, which that
    // segment's own store replaces later (or nothing reads, if it continues
    // into the next chunk).  A segment end moves the lane to the next
    // non-empty segment; after the last one the lane has no more events and
    // nothing reads its sums.
    //
    // The next edge but one is read ahead with no wait: the bounds rows
    // carry two spare entries after the last, and the value is used only
    // while it is an edge of this particle (n + 2 <= N).  Only a run of empty
    // segments needs edges at once: a search finds the segment that holds
    // bin k, or none if the support ended at or before k.
    auto handle = [&](int k) {
        store_sums(dst);
        clear_sums();
        if (nb <= k) {
            ++n;
            zsp += 3;
            nb = (n < N) ? nb2 : INT32_MAX;
            nb2 = bo[n + 2];
            if (nb <= k) {
                n = bsearch_seg(bo, N, k);
                nb = bo[n + 1];
                if (nb <= k) {
                    n = N;
                    nb = INT32_MAX;
                }
                nb2 = bo[n + 2];
                zsp = (GLOBAL double*)a.zs + ((p < a.P_end ? p : a.p0) * (int64_t)N + n) * 3;
            }
            dst = zsp;
        }
        nxt = nb;
    };
    const int L = a.L;
    const int nthreads = blockDim.x;
    PhasePoly poly;
    RespPolyN<NR> rp;
    float phf[kRespMixed], rf[NR][kRespMixed];
    float a1h = 0.f;
    SinCosK kk{kSin3, kSin1, kCos2};
    __asm__ volatile("" : "+v"(kk.s3), "+v"(kk.s1), "+v"(kk.c2));
    // Polynomials are zero until the lane's first block set-up (one-channel
    // lanes also read the table's zero entry, with zero weight), so bins the
    // wave runs before a lane's support add exact zeros.
    int tmask = 0, toff = kTabZero;
    double amp = 0.0;
    if constexpr (MIXED) {
#pragma unroll
        for (int mm = 0; mm < kRespMixed; ++mm) phf[mm] = 0.f;
        if constexpr (RESP) {
#pragma unroll
            for (int f = 0; f < NR; ++f)
#pragma unroll
                for (int mm = 0; mm < kRespMixed; ++mm) rf[f][mm] = 0.f;
        }
    } else {
#pragma unroll
        for (int mm = 0; mm < kNodes; ++mm) poly.ph[mm] = 0.0;
        if constexpr (RESP) {
#pragma unroll
            for (int f = 0; f < NR; ++f)
#pragma unroll
                for (int mm = 0; mm < kNodes; ++mm) rp.r[f][mm] = 0.0;
        }
    }
    // Each lane builds its polynomials on the sub-blocks of its own length
    // 2^lgl (aligned; the wave steps through the shortest in the wave at the
    // chunk start, whose boundaries are boundaries of every lane's blocks in
    // the chunk), so a particle's arithmetic does not depend on the particles
    // that share its wave.  have: first bin of the lane's current sub-block
    // (-1: none yet); kcl its centre.  After its support a lane keeps its
    // last polynomials: what they add is never read.
    const GLOBAL double* __restrict__ coef = (const GLOBAL double*)a.coef;
    int have = -1, kcl = 0;
    // Sparse-grid template: bins are taken in pieces between multiples of
    // the node stride S, inside which every lane stays on one spline
    // interval (the last interval also takes the support's last bin, which
    // lies past the last multiple of S).  On its first piece of an interval a
    // lane forms the interval's cubics from the node records and evaluates
    // them at u = k - (left node): all in FP64 on the FP64 path; on the mixed
    // path the phase cubic in FP64 (an interval of S bins holds far more
    // phase curvature than an FP32 residual can carry) and the response
    // cubics in FP32.
    [[maybe_unused]] int64_t nint = 0;
    [[maybe_unused]] int xl = 0;
    [[maybe_unused]] double cph[4] = {0.0, 0.0, 0.0, 0.0};
    [[maybe_unused]] double crs[NR][4];
    if constexpr (TM == 1) {
#pragma unroll
        for (int f = 0; f < NR; ++f)
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) crs[f][mm] = 0.0;
        if (has) nint = spl_intervals(plo, phi, a.m.sparse);
    }
    auto spline_pieces = [&](int b0, int wlo, int whi, bool act, int llo, int lhi) {
        if constexpr (TM == 1) {
            const int S = a.m.sparse;
#pragma unroll 1
            for (int sb0 = (wlo / S) * S; sb0 < whi; sb0 += S) {
                const int s_lo = sb0 > wlo ? sb0 : wlo;
                const int s_hi = (sb0 + S < whi) ? sb0 + S : whi;
                const bool sact = act && llo < s_hi && lhi > s_lo;
                if (sact) {
                    int64_t jint = (int64_t)(sb0 / S) - (int64_t)(plo / S);
                    jint = jint < nint - 1 ? jint : nint - 1;
                    jint = jint > 0 ? jint : 0;
                    if (have != (int)jint) {
                        have = (int)jint;
                        xl = (int)spl_node(jint, nint, plo, phi, S);
                        const int xr = (int)spl_node(jint < nint ? jint + 1 : jint, nint, plo, phi, S);
                        const GLOBAL double* r0 =
                            (const GLOBAL double*)a.spl + (p * a.spl_nmax + jint) * (int64_t)spl_rec(NCH);
                        spline_interval<NCH>(r0, jint < nint, (double)(xr - xl), cph, crs);
                        if constexpr (MIXED && RESP) {
#pragma unroll
                            for (int f = 0; f < NR; ++f)
#pragma unroll
                                for (int mm = 0; mm < 4; ++mm) rf[f][mm] = (float)crs[f][mm];
                        }
                        if constexpr (!MIXED) {
                            double sc = kPhaseUnits;
#pragma unroll
                            for (int mm = 0; mm < 4; ++mm) poly.ph[mm] = cph[mm] * sc;
                            if constexpr (RESP) {
#pragma unroll
                                for (int f = 0; f < NR; ++f)
#pragma unroll
                                    for (int mm = 0; mm < 4; ++mm) rp.r[f][mm] = crs[f][mm];
                            }
                        }
                    }
                    tmask = kTabMask;
                    toff = 0;
                    amp = 1.0;
                }
                __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): nothing of the set-up pending in the bin loop
                if constexpr (!MIXED) {
                    // one bin at a time: two per pass measured no faster here
                    double jd = (double)(s_lo - xl);
                    const double* binp = reinterpret_cast<const double*>(smem) + (s_lo - b0) * NV;
#pragma unroll 1
                    for (int k = s_lo; k < s_hi; ++k) {
                        if (nxt <= k) handle(k);
                        bin_fp64<NCH, 3>(jd, binp, s_trig, kk, poly, rp, tmask, toff, amp, zr, zi, hh);
                        jd += 1.0;
                        binp += NV;
                    }
                } else {
                    // two bins per pass, as in the block polynomials' loop below
                    // (the same arithmetic per bin, sums and events in bin order)
                    const float ampf = (float)amp;
                    const float* const sb = reinterpret_cast<const float*>(smem);
#pragma unroll 1
                    for (int k0 = s_lo; k0 < s_hi;) {
                        const int kr = (k0 | (kMixedRun - 1)) + 1;
                        const int k1 = kr < s_hi ? kr : s_hi;
                        double ud = (double)(k0 - xl);
                        const float* binp = sb + (k0 - b0) * NV;
#pragma unroll 1
                        for (int k = k0; k < k1; k += 2) {
                            const bool two = k + 1 < k1;  // wave-uniform
                            BinTerms<float, NCH> t0, t1;
                            bin_terms_mixed<NCH, true>((float)ud, binp, phf, a1h, rf, ampf, t0, cph, ud);
                            bin_terms_mixed<NCH, true>((float)(ud + 1.0), binp + NV, phf, a1h, rf, ampf, t1, cph,
                                                       ud + 1.0);
                            pin_terms(t0);
                            pin_terms(t1);
                            if (nxt <= k) handle(k);
                            add_terms(t0, qzr, qzi, qhh);
                            if (two) {
                                if (nxt <= k + 1) handle(k + 1);
                                add_terms(t1, qzr, qzi, qhh);
                            }
                            ud += 2.0;
                            binp += 2 * NV;
                        }
                        if ((k1 & (kMixedRun - 1)) == 0) flush32();
                        k0 = k1;
                    }
                }
            }
        }
    };
    for (int b0 = Kc; b0 < Ke; b0 += L) {
        const int b1 = (b0 + L < Ke) ? b0 + L : Ke;
        const int nbins = b1 - b0;
        // ---- stage bins [b0, b1) into LDS
        __syncthreads();
        if constexpr (!MIXED && NV % 2 == 0) {
            typedef double dbl2 __attribute__((ext_vector_type(2)));
            const GLOBAL dbl2* src = (const GLOBAL dbl2*)(a.b64 + (int64_t)b0 * NV);
            dbl2* dst = reinterpret_cast<dbl2*>(smem);
            const int cnt = nbins * NV / 2;
            for (int i = tid; i < cnt; i += nthreads) dst[i] = src[i];
        } else if constexpr (!MIXED) {
            const GLOBAL double* src = (const GLOBAL double*)(a.b64 + (int64_t)b0 * NV);
            double* dst = reinterpret_cast<double*>(smem);
            const int cnt = nbins * NV;
            for (int i = tid; i < cnt; i += nthreads) dst[i] = src[i];
        } else {
            const GLOBAL float* src = (const GLOBAL float*)(a.b32 + (int64_t)b0 * NV);
            float* dst = reinterpret_cast<float*>(smem);
            const int cnt = nbins * NV;
            for (int i = tid; i < cnt; i += nthreads) dst[i] = src[i];
        }
        if (tid < NV) {  // the spare bin after the staged ones
            if constexpr (MIXED) reinterpret_cast<float*>(smem)[nbins * NV + tid] = 0.f;
            else reinterpret_cast<double*>(smem)[nbins * NV + tid] = 0.0;
        }
        __syncthreads();
        const int llo = lo > b0 ? lo : b0;
        const int lhi = hi < b1 ? hi : b1;
        const bool act = llo < lhi;
        // wave-uniform bin range: the union of the lanes' ranges
        int wlo = act ? llo : INT32_MAX, whi = act ? lhi : INT32_MIN;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int t1 = __shfl_xor(wlo, o, 64);
            const int t2 = __shfl_xor(whi, o, 64);
            wlo = t1 < wlo ? t1 : wlo;
            whi = t2 > whi ? t2 : whi;
        }
        wlo = __builtin_amdgcn_readfirstlane(wlo);
        whi = __builtin_amdgcn_readfirstlane(whi);
        if (wlo >= whi) continue;
        if constexpr (TM == 1) {
            spline_pieces(b0, wlo, whi, act, llo, lhi);
            continue;
        }
        const int Lp = 1 << lgw;
#pragma unroll 1
        for (int sb0 = (wlo >> lgw) << lgw; sb0 < whi; sb0 += Lp) {
            const int s_lo = sb0 > wlo ? sb0 : wlo;
            const int s_hi = (sb0 + Lp < whi) ? sb0 + Lp : whi;
            const bool sact = act && llo < sb0 + Lp && lhi > sb0;
            const int lgl = has ? level_at(sb0) : lgw;
            const int sbl = (sb0 >> lgl) << lgl;
            if (sact && have != sbl) {
                have = sbl;
                kcl = sbl + (1 << (lgl - 1));
                const double inv_h = 1.0 / (double)(1 << (lgl - 1));
                const GLOBAL double* __restrict__ gtl = (const GLOBAL double*)gtab + a.gtab_off[lgl] * kGStride;
                block_setup<RM, NR>(coef, S, p, a.g.k0 + (double)kcl, lgl, gtl + (int64_t)(sbl >> lgl) * kGStride,
                                  a.g, a.m, poly, rp);
                if constexpr (MIXED) {
                    // the FP32 residual phase to degree 3 the same way: off by
                    // |a4|/8 + |a5|/16 cycles, below 1e-6 even where the FP64
                    // bound admits the most curvature, smooth within the block,
                    // so second order in the statistic
                    const double a5 = poly.ph[5], a4 = poly.ph[4];
                    poly.ph[3] += 1.25 * a5;
                    poly.ph[1] -= 0.3125 * a5;
                    poly.ph[2] += a4;
                    poly.ph[0] -= 0.125 * a4;
                }
                if constexpr (MIXED && RESP) {
                    // the FP32 response to degree 3: the interpolant's Chebyshev
                    // series without its T4 and T5 terms (x^5 and x^4 folded into
                    // the lower powers), off by |a4|/8 + |a5|/16 on [-1, 1]: at
                    // most ~2e-7 of |R| on the blocks the FP64 bound selects, the
                    // size of FP32 rounding
#pragma unroll
                    for (int f = 0; f < NR; ++f) {
                        const double a5 = rp.r[f][5], a4 = rp.r[f][4];
                        rp.r[f][3] += 1.25 * a5;
                        rp.r[f][1] -= 0.3125 * a5;
                        rp.r[f][2] += a4;
                        rp.r[f][0] -= 0.125 * a4;
                    }
                }
                // monomials in j = x h (h a power of two: exact rescaling); the
                // FP64 phase also in units of 1/kTrig cycle
                {
                    double sc = 1.0;
#pragma unroll
                    for (int mm = 0; mm < kNodes; ++mm) {
                        poly.ph[mm] *= MIXED ? sc : sc * kPhaseUnits;
                        if constexpr (RESP) {
#pragma unroll
                            for (int f = 0; f < NR; ++f) rp.r[f][mm] *= sc;
                        }
                        sc *= inv_h;
                    }
                }
                tmask = kTabMask;
                toff = 0;
                amp = 1.0;
                if constexpr (MIXED) {
                    // phase = a0 + frac(a1h j) + residual(j): j is an integer and
                    // a1h keeps 12 significant bits, so a1h j is exact in FP32
                    int ex;
                    frexp(poly.ph[1], &ex);
                    const double qd = ldexp(1.0, ex - 12);
                    const double hi1 = rint(poly.ph[1] / qd) * qd;
                    a1h = (float)hi1;
                    phf[0] = (float)poly.ph[0];
                    phf[1] = (float)(poly.ph[1] - hi1);
#pragma unroll
                    for (int mm = 2; mm < kRespMixed; ++mm) phf[mm] = (float)poly.ph[mm];
                    if constexpr (RESP) {
#pragma unroll
                        for (int f = 0; f < NR; ++f)
#pragma unroll
                            for (int mm = 0; mm < kRespMixed; ++mm) rf[f][mm] = (float)rp.r[f][mm];
                    }
                }
            }
            // ---- bins [s_lo, s_hi), one at a time; a wave-wide test per bin
            // sends the lanes whose event is due to handle() first
            // no vector-memory operation of the set-up (spill reloads
            // included) is left pending, so the bin loop needs no wait for one
            __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
            // Two bins per pass: the terms of both are formed before either
            // enters the sums (the lanes' events come between them), so the
            // two bins' arithmetic interleaves.  A pass with one bin left
            // forms its second terms from the next staged bin (at the block's
            // end the spare bin, zero) and drops them.
            if constexpr (!MIXED) {
                double jd = (double)(s_lo - kcl);
                const double* binp = reinterpret_cast<const double*>(smem) + (s_lo - b0) * NV;
#pragma unroll 1
                for (int k = s_lo; k < s_hi; k += 2) {
                    const bool two = k + 1 < s_hi;  // wave-uniform
                    BinTerms<double, NCH> t0, t1;
                    bin_terms_fp64<NCH>(jd, binp, s_trig, kk, poly, rp, tmask, toff, amp, t0);
                    bin_terms_fp64<NCH>(jd + 1.0, binp + NV, s_trig, kk, poly, rp, tmask, toff, amp, t1);
                    pin_terms(t0);
                    pin_terms(t1);
                    if (nxt <= k) handle(k);
                    add_terms(t0, zr, zi, hh);
                    if (two) {
                        if (nxt <= k + 1) handle(k + 1);
                        add_terms(t1, zr, zi, hh);
                    }
                    jd += 2.0;
                    binp += 2 * NV;
                }
            } else {
                const float ampf = (float)amp;
                const float* const sb = reinterpret_cast<const float*>(smem);
                // runs of bins between multiples of kMixedRun, after each of
                // which the plain FP32 sums enter the FP64 ones (a position
                // fixed by the bin index)
#pragma unroll 1
                for (int k0 = s_lo; k0 < s_hi;) {
                    const int kr = (k0 | (kMixedRun - 1)) + 1;
                    const int k1 = kr < s_hi ? kr : s_hi;
                    float jf = (float)(k0 - kcl);
                    const float* binp = sb + (k0 - b0) * NV;
#pragma unroll 1
                    for (int k = k0; k < k1; k += 2) {
                        const bool two = k + 1 < k1;  // wave-uniform
                        BinTerms<float, NCH> t0, t1;
                        bin_terms_mixed<NCH>(jf, binp, phf, a1h, rf, ampf, t0);
                        bin_terms_mixed<NCH>(jf + 1.f, binp + NV, phf, a1h, rf, ampf, t1);
                        pin_terms(t0);
                        pin_terms(t1);
                        if (nxt <= k) handle(k);
                        add_terms(t0, qzr, qzi, qhh);
                        if (two) {
                            if (nxt <= k + 1) handle(k + 1);
                            add_terms(t1, qzr, qzi, qhh);
                        }
                        jf += 2.f;
                        binp += 2 * NV;
                    }
                    if ((k1 & (kMixedRun - 1)) == 0) flush32();
                    k0 = k1;
                }
            }
        }
    }
    // ---- close the chunk: the open segment ends at hi (with the support or
    // exactly at the chunk end), or continues into the next chunk, where the
    // whole-chunk piece of a segment that also started earlier goes to the
    // head record, else the tail
    if (has && n < N) store_sums(nb <= hi ? dst : (dst == recp ? recp : recp + 3));
}

// The generate-and-reduce kernel, persistent, over the tiles of one or
// several evaluations (items): a fixed grid of workgroups takes tiles from a
// device counter until none is left, so swarms of uneven sizes share one
// launch, every XCD gets work wherever the particles' supports lie in the
// band, and the chip stays full to the end.  Consecutive tiles are the
// particle groups of one chunk, so workgroups running together share the
// chunk's data in L2.  tile_start[i] is the first global tile of item i (prefix sums,
// tile_start[n_items] = total); the counter starts at 0.
template <int NCH, bool MIXED, int RM, int TM, bool ALT = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(main_waves_per_eu(NCH, MIXED, ALT)))) void k_main_multi(
    const MainArgs* __restrict__ items, const int64_t* __restrict__ tile_start, int n_items,
    unsigned long long* __restrict__ counter)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double2 s_trig[MIXED ? 1 : kTrig + 1];
    __shared__ unsigned long long s_next;
    if constexpr (!MIXED) {
        for (int i = threadIdx.x; i < kTrig; i += blockDim.x) s_trig[i] = g_trig[i];
        if (threadIdx.x == 0) s_trig[kTrig] = make_double2(0.0, 0.0);
    }
    const int64_t total = tile_start[n_items];
    while (true) {
        if (threadIdx.x == 0) s_next = atomicAdd(counter, 1ULL);
        __syncthreads();
        const int64_t t = (int64_t)s_next;
        __syncthreads();  // every thread has read s_next before the next tile overwrites it
        if (t >= total) break;
        int it = 0;
        while (it + 1 < n_items && tile_start[it + 1] <= t) ++it;
        const MainArgs& a = items[it];
        main_tile<NCH, MIXED, RM, TM>(a, a.gtab, t - tile_start[it], smem, s_trig);
    }
}

// ============================================================== finalize
// Sum of a double over the 64 lanes of a wave (every lane active), result in
// every lane: prefix sums inside each row of 16 lanes by DPP row shifts,
// then the four row totals.
template <int CTRL>
__device__ __forceinline__ double dpp_row_shr_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
    v += dpp_row_shr_f64<0x111>(v);  // row_shr:1
    v += dpp_row_shr_f64<0x112>(v);  // row_shr:2
    v += dpp_row_shr_f64<0x114>(v);  // row_shr:4
    v += dpp_row_shr_f64<0x118>(v);  // row_shr:8
    return (lane_f64(v, 15) + lane_f64(v, 31)) + (lane_f64(v, 47) + lane_f64(v, 63));
}

// One wave per particle (slot of the main kernel): lane l takes segments
// l, l + 64, ...; a segment inside one chunk has its (Z, H) in zs, one that
// crosses chunks is the tail piece of its first chunk plus the head pieces
// of the following ones.  term_n = 4 df |Z_n|^2 / H_n (0 if H_n = 0),
// Upsilon = sum_n term_n.  With seg output, zs is that array and is completed
// here (joined pieces, zeros for empty segments).
__global__ __launch_bounds__(256) void k_finalize(FinalArgs a)
{
    const int lane = threadIdx.x & 63;
    const int64_t s_idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64 + a.p0;
    if (s_idx >= a.P_end) return;  // wave-uniform
    const int64_t p = a.perm ? a.p0 + a.perm[s_idx - a.p0] : s_idx;
    const int N = a.N;
    const int lg = a.lg[p];
    double* const zs = a.zs + p * (int64_t)N * 3;
    const bool out_seg = a.seg != nullptr;
    if (lg == -1 || lg == -2) {
        const double nan = __longlong_as_double(0x7ff8000000000000LL);  // invalid / unresolved theta
        if (lane == 0) a.ups[p - a.p0] = nan;
        if (a.stats && lane < kNStats) a.stats[(p - a.p0) * kNStats + lane] = nan;
        if (out_seg)
            for (int n = lane; n < N; n += 64) zs[3 * n] = zs[3 * n + 1] = zs[3 * n + 2] = nan;
        return;
    }
    const int64_t klo = a.klo[p], khi = a.khi[p];
    const int32_t* __restrict__ bo = a.bounds + p * (int64_t)(N + 1);
    const int64_t cb_len = a.cbins;
    const double* const rec = a.rec + (s_idx - a.p0) * kRec;
    const int64_t cstride = a.rec_stride * kRec;
    const double four_df = 4.0 * a.df;
    double sum = 0.0;
    double ov = 0.0, hs = 0.0, zrs = 0.0, zis = 0.0;  // likelihood sums (stats only)
    for (int n = lane; n < N; n += 64) {
        const int64_t b = bo[n], e = bo[n + 1];
        double zr = 0.0, zi = 0.0, h = 0.0;
        if (khi > klo && e > b) {
            const int64_t c0 = b / cb_len, c1 = (e - 1) / cb_len;
            if (c0 == c1) {
                zr = zs[3 * n];
                zi = zs[3 * n + 1];
                h = zs[3 * n + 2];
            } else {
                const double* r = rec + (c0 - a.chunk0) * cstride;
                zr = r[3];
                zi = r[4];
                h = r[5];
                for (int64_t c = c0 + 1; c <= c1; ++c) {
                    r = rec + (c - a.chunk0) * cstride;
                    zr += r[0];
                    zi += r[1];
                    h += r[2];
                }
                if (out_seg) {
                    zs[3 * n] = zr;
                    zs[3 * n + 1] = zi;
                    zs[3 * n + 2] = h;
                }
            }
            if (h > 0.0) sum += four_df * (zr * zr + zi * zi) / h;
            ov += sqrt(zr * zr + zi * zi);
            hs += h;
            zrs += zr;
            zis += zi;
        } else if (out_seg) {
            zs[3 * n] = zs[3 * n + 1] = zs[3 * n + 2] = 0.0;
        }
    }
    sum = wave_sum_f64(sum);
    if (lane == 0) a.ups[p - a.p0] = sum;
    if (a.stats) {
        // hat O_N = sum_n 4 df |Z_n| (eq:semi-coherent_O), <h|h> = 4 df sum_n H_n,
        // <d|h> = 4 df sum_n Z_n (eqn:inner_prod) for the unit-amplitude template
        ov = wave_sum_f64(ov);
        hs = wave_sum_f64(hs);
        zrs = wave_sum_f64(zrs);
        zis = wave_sum_f64(zis);
        if (lane == 0) {
            double* o = a.stats + (p - a.p0) * kNStats;
            o[0] = sum;
            o[1] = four_df * ov;
            o[2] = four_df * hs;
            o[3] = four_df * zrs;
            o[4] = four_df * zis;
        }
    }
}

// ============================================================== likelihoods
// <d|d> = 4 df sum over channels and bins of |d|^2 / S (eqn:inner_prod with
// a = b = d): every workgroup sums a fixed strided share of the bins and a
// fixed tree adds them, so the value does not depend on timing.
__global__ __launch_bounds__(256) void k_data_norm(GridArgs g, const double* __restrict__ d_ri,
                                                   const double* __restrict__ psd, double* __restrict__ part)
{
    __shared__ double s[256];
    const int64_t n = (int64_t)g.nch * g.K;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double dr = d_ri[2 * i], di = d_ri[2 * i + 1];
        acc += (dr * dr + di * di) / psd[i];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
__global__ __launch_bounds__(kNormBlocks) void k_data_norm_total(const double* __restrict__ part, double df,
                                                                 double* __restrict__ out)
{
    __shared__ double s[kNormBlocks];
    s[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int o = kNormBlocks / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 4.0 * df * s[0];
}

// Log-likelihoods of the templates A h e^{i phi}, without the normalisation
// constant: the semi-coherent log hat L_N = -<d|d>/2 - A^2 <h|h>/2 + |A| hat O_N
// and the coherent log L = -<d|d>/2 - A^2 <h|h>/2 + A Re(e^{-i phi} <d|h>)
// (eqn:LogL_coherent), the latter maximised over phi when phase is null.
__global__ void k_loglike(int64_t P, double dd, const double* __restrict__ stats, const double* __restrict__ amp,
                          const double* __restrict__ phase, double* __restrict__ semi, double* __restrict__ coh)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const double* st = stats + i * kNStats;
    const double A = amp[i];
    const double base = -0.5 * dd - 0.5 * A * A * st[2];
    if (semi) semi[i] = base + fabs(A) * st[1];
    if (coh) {
        double x;
        if (phase) {
            double sp, cp;
            sincos(phase[i], &sp, &cp);
            x = A * (cp * st[3] + sp * st[4]);
        } else {
            x = fabs(A) * sqrt(st[3] * st[3] + st[4] * st[4]);
        }
        coh[i] = base + x;
    }
}

// Absolute template amplitude from the luminosity distance: k Mc^(5/6) / D_L
// (k carries the restricted-amplitude constants and the units, Mc in solar
// masses, D_L in Mpc); NaN for Mc <= 0, D_L <= 0 or a non-finite entry.
__global__ void k_distance_amp(int64_t P, int td, const double* __restrict__ theta, const double* __restrict__ dl,
                               double k, double* __restrict__ amp)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const double mc = theta[i * td], d = dl[i];
    amp[i] = (mc > 0.0 && d > 0.0 && isfinite(mc) && isfinite(d)) ? k * pow(mc, 5.0 / 6.0) / d : __builtin_nan("");
}

// ============================================================== waveform
__global__ void k_waveform(MainArgs a, double* __restrict__ h_ri)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.g.K) return;
    const int nch = a.g.nch;
    for (int c = 0; c < nch; ++c) {
        h_ri[((int64_t)c * a.g.K + k) * 2] = 0.0;
        h_ri[((int64_t)c * a.g.K + k) * 2 + 1] = 0.0;
    }
    const int lg = a.lg[0];
    if (lg < 0 || k < a.klo[0] || k >= a.khi[0]) return;
    const int64_t Lp = (int64_t)1 << lg;
    const int64_t sb = k >> lg;
    const int64_t kc = sb * Lp + (Lp >> 1);
    const double* G = a.gtab + (a.gtab_off[lg] + sb) * kGStride;
    PhasePoly poly;
    RespPoly rp;
    const double x = (double)(k - kc) / (double)(Lp >> 1);
    const double f = (a.g.k0 + (double)k) * a.g.df;
    const double amp = pow(f, -7.0 / 6.0);
    if (nch == 3) {
        RespPolyN<6> rp3;
        block_setup<2, 6>((const GLOBAL double*)a.coef, a.stride, 0, a.g.k0 + (double)kc, lg,
                          (const GLOBAL double*)G, a.g, a.m, poly, rp3);
        double ph = horner5(poly.ph, x);
        ph -= rint(ph);
        double sn, cs;
        sincos2pi(ph, &sn, &cs);
        for (int c = 0; c < 3; ++c) {
            const double rr = horner5(rp3.r[2 * c], x), ri = horner5(rp3.r[2 * c + 1], x);
            h_ri[((int64_t)c * a.g.K + k) * 2] = amp * (rr * cs + ri * sn);
            h_ri[((int64_t)c * a.g.K + k) * 2 + 1] = amp * (ri * cs - rr * sn);
        }
    } else if (nch == 2) {
        if (a.m.response == 2)
            block_setup<2>((const GLOBAL double*)a.coef, a.stride, 0, a.g.k0 + (double)kc, lg, (const GLOBAL double*)G,
                           a.g, a.m, poly, rp);
        else
            block_setup<1>((const GLOBAL double*)a.coef, a.stride, 0, a.g.k0 + (double)kc, lg, (const GLOBAL double*)G,
                           a.g, a.m, poly, rp);
        double ph = horner5(poly.ph, x);
        ph -= rint(ph);
        double sn, cs;
        sincos2pi(ph, &sn, &cs);
        for (int c = 0; c < 2; ++c) {
            const double rr = horner5(rp.r[2 * c], x), ri = horner5(rp.r[2 * c + 1], x);
            // h = amp R e^{-i 2 pi ph}
            h_ri[((int64_t)c * a.g.K + k) * 2] = amp * (rr * cs + ri * sn);
            h_ri[((int64_t)c * a.g.K + k) * 2 + 1] = amp * (ri * cs - rr * sn);
        }
    } else {
        block_setup<0>((const GLOBAL double*)a.coef, a.stride, 0, a.g.k0 + (double)kc, lg, (const GLOBAL double*)G,
                       a.g, a.m, poly, rp);
        double ph = horner5(poly.ph, x);
        ph -= rint(ph);
        double sn, cs;
        sincos2pi(ph, &sn, &cs);
        h_ri[2 * k] = amp * cs;
        h_ri[2 * k + 1] = -amp * sn;
    }
}

// ============================================================== PSO
// Philox4x32-10 (Salmon et al. 2011): 10 rounds of two 32x32 -> 64-bit
// multiplies, Weyl key schedule.
__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}
__device__ __forceinline__ double uniform01(uint64_t seed, uint32_t swarm, uint32_t it, uint32_t pp, uint32_t d,
                                            uint32_t stream)
{
    uint32_t c[4] = {it, pp, d, stream};
    philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32) + swarm);
    const uint64_t x = ((uint64_t)(c[0] >> 6) << 26) | (uint64_t)(c[1] >> 6);
    return ((double)x + 0.5) * 0x1p-52;
}

// ============================================================== noise realisations (Sec 5.1)
// streams[alpha][k][r] = scale d_alpha,k + n_{r0 + r, alpha, k} with
// n = sqrt(S / (4 df)) (g1 + i g2), the convention under which
// <n|h> ~ N(0, <h|h>) (eqn:inner_prod).  g1, g2: Box-Muller (Box & Muller
// 1958) of two 52-bit uniforms from one Philox4x32-10 block with counter
// (k, alpha, r, kNoiseStream) and key (seed low word, seed high word).
constexpr uint32_t kNoiseStream = 0x6e6f6973u;
__global__ void k_make_streams(StreamGenArgs a)
{
    const int64_t n = (int64_t)a.nch * a.K * a.R;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i % a.R;
        const int64_t ak = i / a.R;  // alpha * K + k
        const int64_t k = ak % a.K;
        const int alpha = (int)(ak / a.K);
        uint32_t c[4] = {(uint32_t)k, (uint32_t)alpha, (uint32_t)(a.r0 + r), kNoiseStream};
        philox10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
        const uint64_t x1 = ((uint64_t)(c[0] >> 6) << 26) | (uint64_t)(c[1] >> 6);
        const uint64_t x2 = ((uint64_t)(c[2] >> 6) << 26) | (uint64_t)(c[3] >> 6);
        const double u1 = ((double)x1 + 0.5) * 0x1p-52;
        const double u2 = ((double)x2 + 0.5) * 0x1p-52;
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos(kTwoPi * u2, &sn, &cs);
        const double sig = sqrt(a.psd[ak] / (4.0 * a.df));
        double* o = a.streams + 2 * i;
        o[0] = a.scale * a.d[2 * ak] + sig * (rad * cs);
        o[1] = a.scale * a.d[2 * ak + 1] + sig * (rad * sn);
    }
}

// Template weights of the streamed reduction: w = conj(h) / S per channel and
// bin, and sum over channels of |h|^2 / S per bin.
__global__ void k_stream_weights(int nch, int64_t K, const double* __restrict__ h_ri, const double* __restrict__ psd,
                                 double* __restrict__ wts, double* __restrict__ hq)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double q = 0.0;
    for (int a = 0; a < nch; ++a) {
        const int64_t i = (int64_t)a * K + k;
        const double hr = h_ri[2 * i], hi = h_ri[2 * i + 1];
        const double inv = 1.0 / psd[i];
        wts[2 * i] = hr * inv;
        wts[2 * i + 1] = -hi * inv;
        q += (hr * hr + hi * hi) * inv;
    }
    hq[k] = q;
}

typedef double dbl2v __attribute__((ext_vector_type(2)));
// Streamed reduction, HBM-bound: workgroup (piece, group of 256 streams), one
// stream per lane.  The piece's weights sit in LDS and are read as
// broadcasts; every lane reads its stream's 16 bytes per bin and channel,
// consecutive lanes consecutive addresses.  Z of the piece goes to zpart; the
// piece's share of H (the same for every stream) to hpart.
__global__ __launch_bounds__(256) void k_streams(StreamArgs a)
{
    extern __shared__ double s_w[];  // [len][nch][2] weights, then [len] hq
    const int64_t pc = blockIdx.x;
    const int k0 = a.pieces[3 * pc], k1 = a.pieces[3 * pc + 1];
    const int len = k1 - k0;
    const int nch = a.nch;
    double* s_h = s_w + (int64_t)kPieceBins * nch * 2;
    for (int i = threadIdx.x; i < len * nch; i += blockDim.x) {
        const int kk = i / nch, al = i % nch;
        const int64_t src = ((int64_t)al * a.K + k0 + kk) * 2;
        s_w[2 * i] = a.wts[src];
        s_w[2 * i + 1] = a.wts[src + 1];
    }
    for (int i = threadIdx.x; i < len; i += blockDim.x) s_h[i] = a.hq[k0 + i];
    __syncthreads();
    const int64_t r = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (r < a.R) {
        double zr = 0.0, zi = 0.0;
        const int64_t stride_k = a.R * 2;                 // doubles between consecutive bins
        const int64_t stride_a = a.K * a.R * 2;           // between channels
        const double* base = a.streams + (int64_t)k0 * stride_k + 2 * r;
        for (int al = 0; al < nch; ++al) {
            const double* sp = base + al * stride_a;
#pragma unroll 8
            for (int kk = 0; kk < len; ++kk) {
                // each stream element is read once: non-temporal, so the
                // streams do not evict the weights and each other from the
                // caches (5.8 -> 6.4 TB/s on 1024 realisations of 2^20 bins)
                const dbl2v dv = __builtin_nontemporal_load(reinterpret_cast<const dbl2v*>(sp + (int64_t)kk * stride_k));
                const double wr = s_w[2 * (kk * nch + al)], wi = s_w[2 * (kk * nch + al) + 1];
                zr = __builtin_fma(dv.x, wr, __builtin_fma(-dv.y, wi, zr));
                zi = __builtin_fma(dv.x, wi, __builtin_fma(dv.y, wr, zi));
            }
        }
        a.zpart[(pc * a.R + r) * 2] = zr;
        a.zpart[(pc * a.R + r) * 2 + 1] = zi;
    }
    if (blockIdx.y == 0 && threadIdx.x == 0) {
        double h = 0.0;
        for (int i = 0; i < len; ++i) h += s_h[i];
        a.hpart[pc] = h;
    }
}

// Per stream: join the pieces of every segment and form the statistics of
// scs_evaluate_stats (Upsilon_N, hat O_N, <h|h>, Re and Im <d_r|h>).
__global__ void k_streams_final(StreamArgs a)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    const double four_df = 4.0 * a.df;
    double ups = 0.0, ov = 0.0, hs = 0.0, zrs = 0.0, zis = 0.0;
    double zr = 0.0, zi = 0.0, h = 0.0;
    int cur = -1;
    auto close = [&]() {
        if (h > 0.0) ups += four_df * (zr * zr + zi * zi) / h;
        ov += sqrt(zr * zr + zi * zi);
        hs += h;
        zrs += zr;
        zis += zi;
    };
    for (int64_t i = 0; i < a.n_pieces; ++i) {
        const int n = a.pieces[3 * i + 2];
        if (n != cur) {
            if (cur >= 0) close();
            zr = zi = h = 0.0;
            cur = n;
        }
        zr += a.zpart[(i * a.R + r) * 2];
        zi += a.zpart[(i * a.R + r) * 2 + 1];
        h += a.hpart[i];
    }
    if (cur >= 0) close();
    double* o = a.stats + r * kNStats;
    o[0] = ups;
    o[1] = four_df * ov;
    o[2] = four_df * hs;
    o[3] = four_df * zrs;
    o[4] = four_df * zis;
}

// Every arithmetic step is a single IEEE operation (no contraction) so the
// result is reproducible bit for bit on any IEEE machine.
#pragma clang fp contract(off)
__global__ void k_pso_init(int64_t P, PsoBox box, uint64_t seed, uint32_t swarm, double* __restrict__ theta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * box.dim) return;
    const int64_t pp = i / box.dim;
    const int d = (int)(i % box.dim);
    const double r = uniform01(seed, swarm, 0u, (uint32_t)pp, (uint32_t)d, 3u);
    const double w = box.hi[d] - box.lo[d];
    const double x = r * w;
    theta[i] = box.lo[d] + x;
}

__global__ void k_pso_move(int64_t P, PsoBox box, PsoParams prm, uint64_t seed, uint32_t swarm, uint32_t it,
                           double* __restrict__ theta, double* __restrict__ vel, const double* __restrict__ pbest,
                           const double* __restrict__ gbest, const int32_t* __restrict__ frozen)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * box.dim || (frozen && *frozen)) return;
    const int64_t pp = i / box.dim;
    const int d = (int)(i % box.dim);
    const double x = theta[i];
    const double rp = uniform01(seed, swarm, it, (uint32_t)pp, (uint32_t)d, 0u);
    const double rg = uniform01(seed, swarm, it, (uint32_t)pp, (uint32_t)d, 1u);
    const double t1 = prm.omega * vel[i];
    const double ta = prm.phi_p * rp;
    const double tb = pbest[i] - x;
    const double t2 = ta * tb;
    const double tcg = prm.phi_g * rg;
    const double te = gbest[d] - x;
    const double t3 = tcg * te;
    const double s = t1 + t2;
    const double u = s + t3;
    const double eps = prm.eps[d];
    double v;
    if (fabs(u) >= eps) v = u;
    else if (u != 0.0) v = copysign(eps, u);
    else if (eps == 0.0) v = 0.0;
    else v = uniform01(seed, swarm, it, (uint32_t)pp, (uint32_t)d, 2u) < 0.5 ? -eps : eps;
    double xn = x + v;
    if (box.periodic[d]) {
        const double per = box.hi[d] - box.lo[d];
        double y = xn - box.lo[d];
        const double q = floor(y / per);
        const double z = per * q;
        y = y - z;
        xn = box.lo[d] + y;
    }
    vel[i] = v;
    theta[i] = xn;
}
#pragma clang fp contract(on)

// Particle bests (one thread per particle), then the swarm best by a
// single-workgroup arg-max (first index among equal values).
__global__ void k_pso_pbest(int64_t P, PsoBox box, const double* __restrict__ theta, const double* __restrict__ vals,
                            double* __restrict__ pbest, double* __restrict__ pbest_val, const int32_t* __restrict__ frozen)
{
    const int64_t pp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pp >= P || (frozen && *frozen)) return;
    double v = vals[pp];
    bool inbox = true;
    const int D = box.dim;
    for (int d = 0; d < D; ++d) {
        const double x = theta[pp * D + d];
        if (!box.periodic[d] && !(x >= box.lo[d] && x <= box.hi[d])) inbox = false;
    }
    if (!inbox || isnan(v)) v = -INFINITY;
    if (v > pbest_val[pp]) {
        pbest_val[pp] = v;
        for (int d = 0; d < D; ++d) pbest[pp * D + d] = theta[pp * D + d];
    }
}

__global__ __launch_bounds__(1024) void k_pso_gbest(int64_t P, int D, const double* __restrict__ pbest,
                                                     const double* __restrict__ pbest_val, double* __restrict__ gbest,
                                                     double* __restrict__ gbest_val, ConvRecord conv, int32_t rung_it)
{
    // the flag is read by every thread before thread 0 may set it below
    if (conv.state && conv.state[1]) return;
    __shared__ double sv[1024];
    __shared__ int64_t si[1024];
    const int tid = threadIdx.x;
    double bv = -INFINITY;
    int64_t bi = -1;
    for (int64_t i = tid; i < P; i += blockDim.x) {
        const double v = pbest_val[i];
        if (v > bv) { bv = v; bi = i; }
    }
    sv[tid] = bv;
    si[tid] = bi;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            const double v2 = sv[tid + s];
            const int64_t i2 = si[tid + s];
            if (v2 > sv[tid] || (v2 == sv[tid] && i2 >= 0 && (si[tid] < 0 || i2 < si[tid]))) {
                sv[tid] = v2;
                si[tid] = i2;
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (si[0] >= 0 && sv[0] > *gbest_val) {
            *gbest_val = sv[0];
            for (int d = 0; d < D; ++d) gbest[d] = pbest[si[0] * D + d];
        }
        if (conv.state) {
            // the convergence rule: the best value rose by at most tol over
            // the last window iterations (the value pushed window pushes ago
            // still sits in the ring of window + 1)
            const int32_t W = conv.window;
            const int32_t h = conv.state[0];
            const double v = *gbest_val;
            conv.ring[h % (W + 1)] = v;
            conv.state[0] = h + 1;
            if (h + 1 > W) {
                const double old = conv.ring[(h - W) % (W + 1)];
                if (isfinite(old) && v - old <= conv.tol) {
                    conv.state[1] = 1;
                    conv.state[2] = rung_it;
                }
            }
        }
    }
}

__global__ void k_fill_f64(double* p, int64_t n, double v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ============================================================== launchers
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t upload_cheb(const double* x, const double* m)
{
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_cheb_x), x, sizeof(double) * kNodes);
    if (e != hipSuccess) return e;
    return hipMemcpyToSymbol(HIP_SYMBOL(c_cheb_m), m, sizeof(double) * kNodes * kNodes);
}
hipError_t upload_trig(const double* cs)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(g_trig), cs, sizeof(double) * 2 * kTrig);
}

void launch_data_norm(const GridArgs& g, const double* d_ri, const double* psd, double* part, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_data_norm, dim3(kNormBlocks), dim3(256), 0, s, g, d_ri, psd, part);
    hipLaunchKernelGGL(k_data_norm_total, dim3(1), dim3(kNormBlocks), 0, s, part, g.df, out);
}
void launch_distance_amp(int64_t P, int td, const double* theta, const double* dl, double k, double* amp,
                         hipStream_t s)
{
    if (P > 0) hipLaunchKernelGGL(k_distance_amp, dim3(nblk(P, 256)), dim3(256), 0, s, P, td, theta, dl, k, amp);
}
void launch_loglike(int64_t P, double dd, const double* stats, const double* amp, const double* phase, double* semi,
                    double* coh, hipStream_t s)
{
    if (P > 0) hipLaunchKernelGGL(k_loglike, dim3(nblk(P, 256)), dim3(256), 0, s, P, dd, stats, amp, phase, semi, coh);
}
void launch_make_streams(const StreamGenArgs& a, int n_cu, hipStream_t s)
{
    const int64_t n = (int64_t)a.nch * a.K * a.R;
    const int64_t blocks = std::min<int64_t>(nblk(n, 256), (int64_t)n_cu * 16);
    if (n > 0) hipLaunchKernelGGL(k_make_streams, dim3((unsigned)blocks), dim3(256), 0, s, a);
}
void launch_stream_weights(int nch, int64_t K, const double* h_ri, const double* psd, double* wts, double* hq,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_stream_weights, dim3(nblk(K, 256)), dim3(256), 0, s, nch, K, h_ri, psd, wts, hq);
}
void launch_streams(const StreamArgs& a, hipStream_t s)
{
    if (a.R <= 0 || a.n_pieces <= 0) return;
    const size_t lds = sizeof(double) * (size_t)kPieceBins * (2 * a.nch + 1);
    hipLaunchKernelGGL(k_streams, dim3((unsigned)a.n_pieces, nblk(a.R, 256)), dim3(256), lds, s, a);
}
void launch_streams_final(const StreamArgs& a, hipStream_t s)
{
    if (a.R > 0) hipLaunchKernelGGL(k_streams_final, dim3(nblk(a.R, 256)), dim3(256), 0, s, a);
}
void launch_bins(const GridArgs& g, const double* d_ri, const double* psd, double* b64, float* b32, double su,
                 double sq, hipStream_t s)
{
    hipLaunchKernelGGL(k_bins, dim3(nblk(g.K, 256)), dim3(256), 0, s, g, d_ri, psd, b64, b32, su, sq);
}
void launch_prologue(const PrologueArgs& a, hipStream_t s)
{
    if (a.P > 0) hipLaunchKernelGGL(k_prologue, dim3(nblk(a.P, 64)), dim3(64), 0, s, a);
}
void launch_bounds(const BoundArgs& a, hipStream_t s)
{
    if (a.P <= 0) return;
    if (a.mode == 0) {
        const size_t lds = sizeof(double) * (size_t)a.wcache;
        if (a.m.response == 2) hipLaunchKernelGGL(k_bounds_equal<2>, dim3((unsigned)a.P), dim3(64), lds, s, a);
        else if (a.m.response == 1) hipLaunchKernelGGL(k_bounds_equal<1>, dim3((unsigned)a.P), dim3(64), lds, s, a);
        else hipLaunchKernelGGL(k_bounds_equal<0>, dim3((unsigned)a.P), dim3(64), lds, s, a);
    } else {
        hipLaunchKernelGGL(k_bounds_simple, dim3(nblk(a.P * (a.N + 1), 256)), dim3(256), 0, s, a);
    }
}
// L staged bins and one spare bin after them (read by a two-bin pass that
// has one bin left, whose second terms are dropped)
size_t main_lds_bytes(int nch, int L, bool mixed) { return (size_t)(L + 1) * bin_stride(nch) * (mixed ? 4 : 8); }
// The generate-and-reduce instantiation of a kernel variant (variant_of) and
// precision.
typedef void (*MainKernel)(const MainArgs*, const int64_t*, int, unsigned long long*);
static MainKernel main_kernel(int variant, bool mixed, bool alt)
{
    // the alternative occupancy exists for the per-bin template on one and
    // two channels (three channels already run at two waves)
    if (alt) {
        switch (variant) {
        case 0: return mixed ? k_main_multi<2, true, 1, 0, true> : k_main_multi<2, false, 1, 0, true>;
        case 1: return mixed ? k_main_multi<2, true, 2, 0, true> : k_main_multi<2, false, 2, 0, true>;
        case 3: return mixed ? k_main_multi<1, true, 0, 0, true> : k_main_multi<1, false, 0, 0, true>;
        default: break;
        }
    }
    switch (variant) {
    case 0: return mixed ? k_main_multi<2, true, 1, 0> : k_main_multi<2, false, 1, 0>;
    case 1: return mixed ? k_main_multi<2, true, 2, 0> : k_main_multi<2, false, 2, 0>;
    case 2: return mixed ? k_main_multi<3, true, 2, 0> : k_main_multi<3, false, 2, 0>;
    case 3: return mixed ? k_main_multi<1, true, 0, 0> : k_main_multi<1, false, 0, 0>;
    case 4: return mixed ? k_main_multi<2, true, 1, 1> : k_main_multi<2, false, 1, 1>;
    case 5: return mixed ? k_main_multi<2, true, 2, 1> : k_main_multi<2, false, 2, 1>;
    case 6: return mixed ? k_main_multi<3, true, 2, 1> : k_main_multi<3, false, 2, 1>;
    default: return mixed ? k_main_multi<1, true, 0, 1> : k_main_multi<1, false, 0, 1>;
    }
}
static int variant_channels(int variant)
{
    const int v = variant & 3;
    return v == 2 ? 3 : (v == 3 ? 1 : 2);
}
hipError_t launch_main_multi(const MainArgs* items, const int64_t* tile_start, int n_items, unsigned long long* counter,
                             int variant, int L, int waves, bool mixed, bool alt, int grid, hipStream_t s)
{
    const size_t lds = main_lds_bytes(variant_channels(variant), L, mixed);
    hipLaunchKernelGGL(main_kernel(variant, mixed, alt), dim3(grid), dim3(64 * waves), lds, s, items, tile_start,
                       n_items, counter);
    return hipGetLastError();
}
int main_multi_blocks_per_cu(int variant, int L, int waves, bool mixed, bool alt)
{
    const size_t lds = main_lds_bytes(variant_channels(variant), L, mixed);
    int nb = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, main_kernel(variant, mixed, alt), 64 * waves, lds);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}
void launch_finalize(const FinalArgs& a, hipStream_t s)
{
    const int64_t n = a.P_end - a.p0;  // one wave per slot
    if (n > 0) hipLaunchKernelGGL(k_finalize, dim3(nblk(n, 4)), dim3(256), 0, s, a);
}

// Order particles by support window so that the particles of a workgroup
// cover nearly the same bins: counting sort into kSortBuckets buckets of
// (k_hi, k_lo), each quantised to 256 levels.  The order inside a bucket is
// whatever the atomics give; no result depends on it (every particle's
// arithmetic is independent of its slot).  Made of kernels only, so that it
// can be captured in a graph.
__global__ void k_sort_hist(int64_t P, int64_t K, const int32_t* __restrict__ klo, const int32_t* __restrict__ khi,
                            unsigned* __restrict__ hist, int32_t* __restrict__ bucket, int32_t* __restrict__ rank)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < P;
    const int64_t w = K / 256 + 1;  // level width
    const int b = live ? (int)(((int64_t)khi[i] / w) * 256 + (int64_t)klo[i] / w) : -1;
    if (live) bucket[i] = b;
    // one atomic per distinct bucket of the wave (a converged swarm puts
    // most particles in a few buckets, where per-particle atomics serialise)
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ULL << lane) - 1ULL;
    unsigned long long todo = __ballot(live);
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int bl = __shfl(b, leader, 64);
        const unsigned long long peers = __ballot(live && b == bl);
        unsigned base = 0;
        if (lane == leader) base = atomicAdd(&hist[bl], (unsigned)__popcll(peers));
        base = __shfl(base, leader, 64);
        if (live && b == bl) rank[i] = (int32_t)(base + (unsigned)__popcll(peers & below));
        todo &= ~peers;
    }
}
// Exclusive prefix sums of the histogram, one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_sort_scan(unsigned* __restrict__ hist)
{
    constexpr int per = kSortBuckets / 1024;
    __shared__ unsigned part[1024];
    const int t = threadIdx.x;
    unsigned v[per];
    unsigned sum = 0;
    for (int q = 0; q < per; ++q) {
        v[q] = hist[t * per + q];
        sum += v[q];
    }
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const unsigned x = t >= o ? part[t - o] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    unsigned run = part[t] - sum;  // exclusive prefix of this thread's run
    for (int q = 0; q < per; ++q) {
        hist[t * per + q] = run;
        run += v[q];
    }
}
__global__ void k_sort_scatter(int64_t P, const unsigned* __restrict__ offs, const int32_t* __restrict__ bucket,
                               const int32_t* __restrict__ rank, int32_t* __restrict__ perm)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    perm[offs[bucket[i]] + (unsigned)rank[i]] = (int32_t)i;
}
__global__ void k_fill_u32(unsigned* p, int64_t n, unsigned v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

void launch_sort_perm(int64_t P, int64_t K, const int32_t* klo, const int32_t* khi, unsigned* hist, int32_t* bucket,
                      int32_t* rank, int32_t* perm, hipStream_t s)
{
    if (P <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(nblk(kSortBuckets, 256)), dim3(256), 0, s, hist, (int64_t)kSortBuckets, 0u);
    hipLaunchKernelGGL(k_sort_hist, dim3(nblk(P, 256)), dim3(256), 0, s, P, K, klo, khi, hist, bucket, rank);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, hist);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nblk(P, 256)), dim3(256), 0, s, P, hist, bucket, rank, perm);
}
void launch_gtab(const GridArgs& g, int lg, int64_t nsub, double* tab, hipStream_t s)
{
    if (nsub > 0) hipLaunchKernelGGL(k_gtab, dim3(nblk(nsub, 128)), dim3(128), 0, s, g, lg, nsub, tab);
}
void launch_waveform(const MainArgs& a, double* h_ri, hipStream_t s)
{
    if (a.m.sparse > 0) {
        const dim3 grid(nblk(a.g.K, 128));
        if (a.g.nch == 3) hipLaunchKernelGGL(k_waveform_spline<3>, grid, dim3(128), 0, s, a, h_ri);
        else if (a.g.nch == 2) hipLaunchKernelGGL(k_waveform_spline<2>, grid, dim3(128), 0, s, a, h_ri);
        else hipLaunchKernelGGL(k_waveform_spline<1>, grid, dim3(128), 0, s, a, h_ri);
        return;
    }
    hipLaunchKernelGGL(k_waveform, dim3(nblk(a.g.K, 128)), dim3(128), 0, s, a, h_ri);
}
void launch_spline(const SplineArgs& a, hipStream_t s)
{
    if (a.P <= 0 || a.m.sparse <= 0) return;
    const dim3 gn(nblk(a.P * a.nmax, 256)), b(256);
    const int nq = spl_nq(a.g.nch);
    const dim3 gs(nblk(a.P * nq, 64)), bs(64);
    if (a.m.response == 2 && a.g.nch == 3) {
        hipLaunchKernelGGL((k_spline_nodes<3, 2>), gn, b, 0, s, a);
        hipLaunchKernelGGL(k_spline_solve<3>, gs, bs, 0, s, a);
    } else if (a.m.response == 2) {
        hipLaunchKernelGGL((k_spline_nodes<2, 2>), gn, b, 0, s, a);
        hipLaunchKernelGGL(k_spline_solve<2>, gs, bs, 0, s, a);
    } else if (a.m.response == 1) {
        hipLaunchKernelGGL((k_spline_nodes<2, 1>), gn, b, 0, s, a);
        hipLaunchKernelGGL(k_spline_solve<2>, gs, bs, 0, s, a);
    } else {
        hipLaunchKernelGGL((k_spline_nodes<1, 0>), gn, b, 0, s, a);
        hipLaunchKernelGGL(k_spline_solve<1>, gs, bs, 0, s, a);
    }
}
void launch_pso_init(int64_t P, const PsoBox& box, uint64_t seed, uint32_t swarm, double* theta, hipStream_t s)
{
    hipLaunchKernelGGL(k_pso_init, dim3(nblk(P * box.dim, 256)), dim3(256), 0, s, P, box, seed, swarm, theta);
}
void launch_pso_move(int64_t P, const PsoBox& box, const PsoParams& prm, uint64_t seed, uint32_t swarm, uint32_t it,
                     double* theta, double* vel, const double* pbest, const double* gbest, hipStream_t s,
                     const int32_t* frozen)
{
    hipLaunchKernelGGL(k_pso_move, dim3(nblk(P * box.dim, 256)), dim3(256), 0, s, P, box, prm, seed, swarm, it, theta,
                       vel, pbest, gbest, frozen);
}
void launch_pso_best(int64_t P, const PsoBox& box, const double* theta, const double* vals, double* pbest,
                     double* pbest_val, double* gbest, double* gbest_val, hipStream_t s, const ConvRecord* conv,
                     int32_t rung_it)
{
    const ConvRecord c = conv ? *conv : ConvRecord{nullptr, nullptr, 0, 0.0};
    hipLaunchKernelGGL(k_pso_pbest, dim3(nblk(P, 256)), dim3(256), 0, s, P, box, theta, vals, pbest, pbest_val,
                       c.state ? c.state + 1 : nullptr);
    hipLaunchKernelGGL(k_pso_gbest, dim3(1), dim3(1024), 0, s, P, box.dim, pbest, pbest_val, gbest, gbest_val, c,
                       rung_it);
}
void launch_fill(double* p, int64_t n, double v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_f64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
}
void launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u64, dim3(nblk(n, 256)), dim3(256), 0, s, p, n, v);
}

}  // namespace scs
