// Device arithmetic for the semi-coherent statistic kernels (gfx950).
//
// * double-double helpers (Dekker / Knuth error-free transformations) for the
//   few quantities whose size (~1e6-1e7 cycles of phase) exceeds what one
//   double resolves at the 1e-12-cycle level;
// * sin/cos of 2 pi r for a phase already reduced to cycles;
// * the TaylorF2 phase written as a sum of particle coefficients times
//   particle-independent basis functions of frequency (Sec 4 waveform);
// * the low-frequency LISA A/E antenna patterns and the full frequency-domain
//   TDI response with finite arm length (Sec 4 response).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scs {

// ---------------------------------------------------------------- constants
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279503;
constexpr double kAuOverC = 1.495978707e11 / 299792458.0;  // light travel time of 1 AU [s]
constexpr double kInvYear = 1.0 / 31557600.0;              // Julian year
constexpr double kArmS = 2.5e9 / 299792458.0;              // light time of one constellation arm [s]
constexpr double kEulerGamma = 0.57721566490153286060651209;
constexpr int kTheta = 7;     // theta entries of a circular model
constexpr int kThetaMax = 8;  // with the eccentricity e0

// coefficient-buffer field indices (one record of kCoefStride doubles per particle)
enum Coef : int {
    C_C0H = 0, C_C0L,      // Newtonian coefficient of f^-5/3, double-double
    C_B1, C_B2, C_B3, C_B4, C_B5, C_B6, C_B7,  // coefficients of f^-1, f^-2/3, f^-1/3, ln f, f^1/3, f^1/3 ln f, f^2/3
    C_BEH, C_BEL,          // coefficient of f^-34/9 (eccentric term), double-double
    C_PHIC,                // constant phase [cycles]
    C_TAUH, C_TAUL,        // t_c * df, double-double
    C_TC,                  // t_c [s]
    C_DC, C_DS,            // Doppler [cycles/Hz] = dc cos(Phi_orb) + ds sin(Phi_orb)
    C_RESP,                // 36 response trig-polynomial coefficients: R_A re, R_A im, R_E re, R_E im
                           // (full response: the source record FdSlot instead)
    C_TCL = C_RESP + 36,   // low part of t_c in double-double: t_c = C_TC + C_TCL
    C_LGUP,                // first bins from which blocks of 2 and 4 times the
                           // support start's length meet the same bounds (2 slots)
    C_COUNT = C_LGUP + 2
};

// Source record of the full response, at C_RESP: direction to the source,
// polarisation vectors P, Q (e+ = PP - QQ, ex = PQ + QP) and the (2,2)
// amplitudes of the two polarisations.
enum FdSlot : int { FD_N = 0, FD_P = 3, FD_Q = 6, FD_AP = 9, FD_AX = 10, FD_COUNT = 11 };

// ---------------------------------------------------------------- double-double
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b)
{
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b)
{
    const double s = a + b;
    return {s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b)
{
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_mul(dd a, dd b)
{
    dd p = two_prod(a.hi, b.hi);
    p.lo = __builtin_fma(a.hi, b.lo, __builtin_fma(a.lo, b.hi, p.lo));
    return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b)
{
    dd p = two_prod(a.hi, b);
    p.lo = __builtin_fma(a.lo, b, p.lo);
    return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_add(dd a, dd b)
{
    dd s = two_sum(a.hi, b.hi);
    s.lo += a.lo + b.lo;
    return fast_two_sum(s.hi, s.lo);
}
// exact rational constant p/q as double-double
__device__ __forceinline__ dd dd_ratio(double p, double q)
{
    const double hi = p / q;
    const double lo = __builtin_fma(-hi, q, p) / q;
    return {hi, lo};
}
// fractional part of a double-double in [-0.5, 0.5)
__device__ __forceinline__ double dd_frac(dd a)
{
    const double r = a.hi - rint(a.hi);  // exact
    const double s = r + a.lo;
    return s - rint(s);
}

// x^(-5/3) and x^(-8/3) in double-double for double-double x (one Newton
// step on y^3 x^5 = 1, resp. y^3 x^8 = 1, from the double estimate).
__device__ inline dd dd_pow_m53(dd x)
{
    const double y0 = pow(x.hi, -5.0 / 3.0);
    const dd x2 = dd_mul(x, x);
    const dd x5 = dd_mul(dd_mul(x2, x2), x);
    const dd y3 = dd_mul_d(two_prod(y0, y0), y0);
    const dd pr = dd_mul(y3, x5);
    const double r = (pr.hi - 1.0) + pr.lo;
    return two_sum(y0, -y0 * r * (1.0 / 3.0));
}
__device__ inline dd dd_pow_m83(dd x)
{
    const double y0 = pow(x.hi, -8.0 / 3.0);
    const dd x2 = dd_mul(x, x);
    const dd x4 = dd_mul(x2, x2);
    const dd x8 = dd_mul(x4, x4);
    const dd y3 = dd_mul_d(two_prod(y0, y0), y0);
    const dd pr = dd_mul(y3, x8);
    const double r = (pr.hi - 1.0) + pr.lo;
    return two_sum(y0, -y0 * r * (1.0 / 3.0));
}

// Integer power of a double-double by repeated squaring (n >= 1).
__device__ inline dd dd_powi(dd x, int n)
{
    dd r{1.0, 0.0};
    bool first = true;
    while (n > 0) {
        if (n & 1) {
            r = first ? x : dd_mul(r, x);
            first = false;
        }
        n >>= 1;
        if (n) x = dd_mul(x, x);
    }
    return r;
}
// x^(p/q) in double-double for x > 0 (q > 0, p != 0): one Newton step on
// y^q = x^p from the double estimate.
__device__ inline dd dd_pow_ratio(dd x, int p, int q)
{
    const double y0 = pow(x.hi, (double)p / (double)q);
    const dd yq = dd_powi(dd{y0, 0.0}, q);
    double r;
    if (p < 0) {  // r = y0^q x^|p| - 1
        const dd pr = dd_mul(yq, dd_powi(x, -p));
        r = (pr.hi - 1.0) + pr.lo;
    } else {  // r = (y0^q - x^p) / x^p
        const dd xp = dd_powi(x, p);
        const dd df = dd_add(yq, dd{-xp.hi, -xp.lo});
        r = (df.hi + df.lo) / xp.hi;
    }
    return two_sum(y0, -y0 * r / (double)q);
}

// ---------------------------------------------------------------- sin/cos(2 pi r)
// r in cycles (|r| < 2^40).  Quarter-turn reduction, then Taylor series of
// sin and cos on |x| <= pi/4 truncated after x^15 and x^16 (remainders below
// 1e-16); the quadrant swaps and negates the pair.
__device__ __forceinline__ void sincos2pi(double r, double* s_out, double* c_out)
{
    const double q = rint(4.0 * r);
    const double t = __builtin_fma(q, -0.25, r);
    const double x = t * kTwoPi;
    const double x2 = x * x;
    double ps = -7.6471637318198164759e-13;  // -1/15!
    ps = __builtin_fma(ps, x2, 1.6059043836821614599e-10);   // 1/13!
    ps = __builtin_fma(ps, x2, -2.5052108385441718775e-8);   // -1/11!
    ps = __builtin_fma(ps, x2, 2.7557319223985890653e-6);    // 1/9!
    ps = __builtin_fma(ps, x2, -1.9841269841269841270e-4);   // -1/7!
    ps = __builtin_fma(ps, x2, 8.3333333333333333333e-3);    // 1/5!
    ps = __builtin_fma(ps, x2, -1.6666666666666666667e-1);   // -1/3!
    const double sn = __builtin_fma(x * x2, ps, x);
    double pc = 4.7794773323873852974e-14;  // 1/16!
    pc = __builtin_fma(pc, x2, -1.1470745597729724714e-11);  // -1/14!
    pc = __builtin_fma(pc, x2, 2.0876756987868098979e-9);    // 1/12!
    pc = __builtin_fma(pc, x2, -2.7557319223985890653e-7);   // -1/10!
    pc = __builtin_fma(pc, x2, 2.4801587301587301587e-5);    // 1/8!
    pc = __builtin_fma(pc, x2, -1.3888888888888888889e-3);   // -1/6!
    pc = __builtin_fma(pc, x2, 4.1666666666666666667e-2);    // 1/4!
    pc = __builtin_fma(pc, x2, -0.5);
    const double cs = __builtin_fma(x2, pc, 1.0);
    const int iq = ((int)q) & 3;
    const double s1 = (iq & 1) ? cs : sn;
    const double c1 = (iq & 1) ? sn : cs;
    *s_out = (iq & 2) ? -s1 : s1;
    *c_out = ((iq + 1) & 2) ? -c1 : c1;
}

// ---------------------------------------------------------------- response
// Polarisation vectors for sky direction (lambda, beta) and angle psi.
struct Pol {
    double P[3], Q[3];
};
__device__ inline Pol polarisation(double lam, double bet, double psi)
{
    double sl, cl, sb, cb, sp, cp;
    sincos(lam, &sl, &cl);
    sincos(bet, &sb, &cb);
    sincos(psi, &sp, &cp);
    const double u[3] = {sb * cl, sb * sl, -cb};
    const double v[3] = {sl, -cl, 0.0};
    Pol o;
    for (int i = 0; i < 3; ++i) {
        o.P[i] = cp * u[i] + sp * v[i];
        o.Q[i] = -sp * u[i] + cp * v[i];
    }
    return o;
}

// Antenna patterns at constellation orbital angle Phi.  For an arm with unit
// vector n, n.e+.n = (n.P)^2 - (n.Q)^2 and n.ex.n = 2 (n.P)(n.Q).  With
// q_ab the arm forms, F_X = (q01 - q02)/2 (and cyclic), hence
// F_A = (2 q02 - q01 - q12) / (2 sqrt2) and F_E = 3 (q01 - q12) / (2 sqrt6).
// out[0] = F+_A, out[1] = Fx_A, out[2] = F+_E, out[3] = Fx_E.
__device__ inline void antenna_lf(double Phi, double cart0, const Pol& pol, double out[4])
{
    double sP, cP;
    sincos(Phi, &sP, &cP);
    const double h3 = 0.86602540378443864676;  // sqrt(3)/2
    // in-plane orthonormal pair: e1 = -r/2 - (sqrt3/2) z, e2 = phi-hat
    const double e1[3] = {-0.5 * cP, -0.5 * sP, -h3};
    const double e2[3] = {-sP, cP, 0.0};
    double s[3][3];
    for (int a = 0; a < 3; ++a) {
        double st, ct;
        sincos(cart0 - Phi + kTwoPi * a / 3.0, &st, &ct);
        for (int i = 0; i < 3; ++i) s[a][i] = ct * e1[i] + st * e2[i];
    }
    const double inv_r3 = 0.57735026918962576451;  // 1/sqrt(3): chord between craft
    double qp[3], qx[3];                             // arms 01, 02, 12
    const int A0[3] = {0, 0, 1}, A1[3] = {1, 2, 2};
    for (int k = 0; k < 3; ++k) {
        double n[3];
        for (int i = 0; i < 3; ++i) n[i] = (s[A1[k]][i] - s[A0[k]][i]) * inv_r3;
        const double a = n[0] * pol.P[0] + n[1] * pol.P[1] + n[2] * pol.P[2];
        const double b = n[0] * pol.Q[0] + n[1] * pol.Q[1] + n[2] * pol.Q[2];
        qp[k] = a * a - b * b;
        qx[k] = 2.0 * a * b;
    }
    const double ka = 0.35355339059327376220;  // 1/(2 sqrt2)
    const double ke = 0.61237243569579452455;  // 3/(2 sqrt6)
    out[0] = ka * (2.0 * qp[1] - qp[0] - qp[2]);
    out[1] = ka * (2.0 * qx[1] - qx[0] - qx[2]);
    out[2] = ke * (qp[0] - qp[2]);
    out[3] = ke * (qx[0] - qx[2]);
}

// Full frequency-domain response (A, E) at frequency f [Hz], constellation
// orbital angle Phi (c1, s1 = cos, sin Phi) and cartwheel angle zeta =
// cart0 - Phi (cz, sz), for the source record src (FdSlot; any pointer type).
//
// Link j -> i, n the unit vector from craft j to craft i, craft at the
// centre plus r p_a (r = L / sqrt3, p_a unit): a plane wave along -nhat with
// polarisation content P = a+ e+ - i ax ex gives, per Fourier component
// (delay tau -> e^{-2 pi i f tau}; the centre's delay is the Doppler term of
// the phase),
//     y_ij / h = -i pi f L sinc(pi f L (1 + nhat.n)) e^{-i pi f (L - r nhat.(p_i + p_j))} n.P.n .
// First-generation TDI on equal static arms (z = e^{-2 pi i f L}):
//     X = (1 - z^2) [(y01 + z y10) - (y02 + z y20)], Y and Z cyclic,
//     A = (Z - X) / sqrt2, E = (X - 2Y + Z) / sqrt6, both over 4 (2 pi f L)^2,
// so that they tend to the low-frequency response as f L -> 0.  The common
// factor (1 - z^2)(-i pi f L) / (4 (2 pi f L)^2) equals z sin(x) / (4x) with
// x = 2 pi f L.  Arm (i, j) = (k, k+1) adds y_ij + z y_ji to channel k of
// (X, Y, Z) and subtracts y_ji + z y_ij from channel k+1.  Every vector enters
// through its projections on the plane's basis e1 = -r_hat/2 - (sqrt3/2) z_hat,
// e2 = phi_hat, so an arm costs a few products.  All sines and cosines are of
// arguments below a few turns (sincos2pi), seven per call.  out = {Re A,
// Im A, Re E, Im E} and, for NC = 3, T = (X + Y + Z) / sqrt3 after them.
template <int NC, typename Src>
__device__ inline void fd_response(double f, double c1, double s1, double cz, double sz, Src src, double out[2 * NC])
{
    const double h3 = 0.86602540378443864676;     // sqrt(3)/2
    const double inv_r3 = 0.57735026918962576451;  // 1/sqrt(3)
    double e1n, e2n, e1p, e2p, e1q, e2q;
    {
        const double v0 = src[FD_N], v1 = src[FD_N + 1], v2 = src[FD_N + 2];
        e1n = __builtin_fma(-0.5, __builtin_fma(c1, v0, s1 * v1), -h3 * v2);
        e2n = __builtin_fma(c1, v1, -(s1 * v0));
    }
    {
        const double v0 = src[FD_P], v1 = src[FD_P + 1], v2 = src[FD_P + 2];
        e1p = __builtin_fma(-0.5, __builtin_fma(c1, v0, s1 * v1), -h3 * v2);
        e2p = __builtin_fma(c1, v1, -(s1 * v0));
    }
    {
        const double v0 = src[FD_Q], v1 = src[FD_Q + 1], v2 = src[FD_Q + 2];
        e1q = __builtin_fma(-0.5, __builtin_fma(c1, v0, s1 * v1), -h3 * v2);
        e2q = __builtin_fma(c1, v1, -(s1 * v0));
    }
    const double ap = src[FD_AP], ax = src[FD_AX];
    // craft angles zeta, zeta + 2pi/3, zeta + 4pi/3
    const double ca3[3] = {cz, __builtin_fma(-0.5, cz, -h3 * sz), __builtin_fma(-0.5, cz, h3 * sz)};
    const double sa3[3] = {sz, __builtin_fma(-0.5, sz, h3 * cz), __builtin_fma(-0.5, sz, -h3 * cz)};
    const double fl = f * kArmS;  // one arm in cycles of f
    // a = pi f L: its sine and cosine give z = e^{-2ia} by the double angle,
    // the common factor e^{-ia} of every link phase, and (with those of a g)
    // sin(a (1 +- g)) by angle addition
    double sa, ca;
    sincos2pi(0.5 * fl, &sa, &ca);
    const double sx = 2.0 * sa * ca, cx = __builtin_fma(ca, ca, -(sa * sa));  // z = cx - i sx
    double acc[3][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};  // X, Y, Z
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = k, j = (k + 1) % 3;
        const double dc = (ca3[i] - ca3[j]) * inv_r3, ds = (sa3[i] - sa3[j]) * inv_r3;
        const double a = __builtin_fma(dc, e1p, ds * e2p);  // n.P
        const double b = __builtin_fma(dc, e1q, ds * e2q);  // n.Q
        const double g = __builtin_fma(dc, e1n, ds * e2n);  // nhat.n
        const double sp = __builtin_fma(ca3[i] + ca3[j], e1n, (sa3[i] + sa3[j]) * e2n);
        const double npr = ap * __builtin_fma(a, a, -(b * b)), npi = -2.0 * ax * a * b;  // n.P.n
        // link phase -a + pi f r sp
        double sb, cb;
        sincos2pi(0.5 * f * kArmS * inv_r3 * sp, &sb, &cb);
        const double cs = __builtin_fma(ca, cb, sa * sb), sn = __builtin_fma(sb, ca, -(cb * sa));
        const double cr = __builtin_fma(cs, npr, -(sn * npi)), ci = __builtin_fma(cs, npi, sn * npr);
        // sinc(a (1 +- g)): sin(a +- a g) = sin a cos(a g) +- cos a sin(a g); below
        // 1e-5 turns of argument the series 1 - u^2/6 (remainder u^4/120 < 1e-18)
        double sg, cg;
        sincos2pi(0.5 * fl * g, &sg, &cg);
        const double uf = kPi * fl * (1.0 + g), ub = kPi * fl * (1.0 - g);  // radians
        const double sf = uf < 6.3e-5 ? __builtin_fma(-uf * uf, 1.0 / 6.0, 1.0) : __builtin_fma(sa, cg, ca * sg) / uf;
        const double sbk = ub < 6.3e-5 ? __builtin_fma(-ub * ub, 1.0 / 6.0, 1.0) : __builtin_fma(sa, cg, -(ca * sg)) / ub;
        const double yfr = cr * sf, yfi = ci * sf;    // y_ij
        const double ybr = cr * sbk, ybi = ci * sbk;  // y_ji
        // + (y_ij + z y_ji) into channel k, - (y_ji + z y_ij) into channel k+1
        acc[i][0] += yfr + __builtin_fma(cx, ybr, sx * ybi);
        acc[i][1] += yfi + __builtin_fma(cx, ybi, -(sx * ybr));
        acc[j][0] -= ybr + __builtin_fma(cx, yfr, sx * yfi);
        acc[j][1] -= ybi + __builtin_fma(cx, yfi, -(sx * yfr));
    }
    const double wm = sx / (4.0 * kTwoPi * fl);  // sin(x) / (4x)
    const double wr = wm * cx, wi = -wm * sx;     // z sin(x) / (4x)
    const double ka = 0.70710678118654752440, ke = 0.40824829046386301637;  // 1/sqrt2, 1/sqrt6
    const double Ar = ka * (acc[2][0] - acc[0][0]), Ai = ka * (acc[2][1] - acc[0][1]);
    const double Er = ke * (acc[0][0] - 2.0 * acc[1][0] + acc[2][0]), Ei = ke * (acc[0][1] - 2.0 * acc[1][1] + acc[2][1]);
    out[0] = __builtin_fma(wr, Ar, -(wi * Ai));
    out[1] = __builtin_fma(wr, Ai, wi * Ar);
    out[2] = __builtin_fma(wr, Er, -(wi * Ei));
    out[3] = __builtin_fma(wr, Ei, wi * Er);
    if constexpr (NC == 3) {
        const double kt = 0.57735026918962576451;  // 1/sqrt3
        const double Tr = kt * (acc[0][0] + acc[1][0] + acc[2][0]), Ti = kt * (acc[0][1] + acc[1][1] + acc[2][1]);
        out[4] = __builtin_fma(wr, Tr, -(wi * Ti));
        out[5] = __builtin_fma(wr, Ti, wi * Tr);
    }
}

// Evaluate a degree-4 trigonometric polynomial c[0] + sum_k c[k] cos kPhi + c[4+k] sin kPhi
// given the harmonics (ch[k], sh[k]) = (cos kPhi, sin kPhi), k = 1..4.
__device__ __forceinline__ double trig4(const double* c, const double* ch, const double* sh)
{
    double v = c[0];
#pragma unroll
    for (int k = 1; k <= 4; ++k) v = __builtin_fma(c[k], ch[k], __builtin_fma(c[4 + k], sh[k], v));
    return v;
}

__device__ __forceinline__ void harmonics(double c1, double s1, double* ch, double* sh)
{
    ch[1] = c1;
    sh[1] = s1;
    ch[2] = c1 * c1 - s1 * s1;
    sh[2] = 2.0 * c1 * s1;
    ch[3] = ch[2] * c1 - sh[2] * s1;
    sh[3] = sh[2] * c1 + ch[2] * s1;
    ch[4] = ch[2] * ch[2] - sh[2] * sh[2];
    sh[4] = 2.0 * ch[2] * sh[2];
}

}  // namespace scs
