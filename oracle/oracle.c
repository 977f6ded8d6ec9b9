/*
 * Plain CPU oracle for the semi-coherent search statistic Upsilon_N of
 * Bandopadhyay & Moore, "A GPU-accelerated semi-coherent hierarchical search
 * for stellar-mass binary inspiral signals in LISA" (arXiv:2408.13170).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP library.
 *
 * Everything here is written for obviousness, not speed: every bin of every
 * particle is evaluated directly from the definitions, in the order the paper
 * states them.  Floating point is IEEE double, except the gravitational-wave
 * phase and the SPA time, which are evaluated in x87 extended precision
 * (long double, 64-bit mantissa): the phase reaches ~1e6-1e7 cycles, so
 * double would leave ~1e-9 rad of rounding in every bin, which is the size of
 * the parity tolerance itself.  Segment sums accumulate in long double.
 * The sparse-grid template's node phases and their spline are evaluated in
 * quad precision (__float128): a not-a-knot spline whose end interval is a
 * few bins long multiplies the rounding of the node values by up to ~S/h
 * there (S the node stride, h the end interval), which in extended precision
 * would reach ~1e-10 cycles.
 *
 * Definitions (paper section / equation in brackets):
 *   inner product          <a|b> = sum_alpha 4 Re sum_k df a b* / S      [Sec 2.1, eqn:inner_prod]
 *   segmented product      [a|b]_n over bins of segment n               [Sec 2.2]
 *   statistic              Upsilon_N = sum_n x_n^2 / [h|h]_n,
 *                          x_n = max_phi [d|h e^{i phi}]_n = 4 df |Z_n|  [Sec 2.2, Upsilon_N definition]
 *   equal-SNR boundaries   every segment holds the same [h|h]           [Sec 2.2, boundary choice]
 *   waveform               TaylorF2 (2,2) mode, restricted amplitude     [Sec 4, waveform paragraph]
 *   response               low-frequency LISA A/E channels, or the full   [Sec 4, response paragraph]
 *                          frequency-domain TDI transfer functions A/E/T
 *   PSO update             velocity rule + minimum-velocity clamp       [Sec 3.1, eqn:PSO_velocity_rule,
 *                                                                         eqn:PSO_min_velocity]
 * Where the paper leaves a point open, the reading taken is stated next to
 * the code that takes it.
 *
 * Eccentric models (TaylorF2Ecc, Sec 4) keep the leading-order correction in
 * e0^2 at Newtonian order, pinned against the Peters-Mathews evolution.
 *
 * The PN phase coefficients above the Newtonian term (the paper does not
 * print them; they are the standard TaylorF2 values) are pinned by rebuilding
 * the stationary-phase time from the PN energy and flux functions.
 * Parity unpinned: the low-frequency response beyond its invariants (the
 * paper's full response code is not available).
 * The full response is pinned to its own definition (link light-travel
 * formula and TDI with explicit delays, evaluated in the time domain) and to
 * the low-frequency limit, not to another implementation: its constellation
 * is rigid with equal, static arms, a reading of the response paragraph.
 */
#include <complex.h>
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;
typedef __float128 qd; /* quad precision: the node phases of the sparse-grid template */

/* ---- physical constants (SI) ---------------------------------------- */
#define GM_SUN_SI 1.32712440018e20L /* m^3 s^-2, IAU nominal solar mass parameter */
#define C_SI 299792458.0L           /* m s^-1 */
#define AU_SI 1.495978707e11L       /* m */
#define YEAR_SI 31557600.0L         /* s, Julian year */
#define EULER_GAMMA_L 0.577215664901532860606512090082402431L
#define PI_L 3.141592653589793238462643383279502884L
#define ARM_SI 2.5e9                /* m, arm length of the constellation (full response) */

/* ---- public structures (mirrored by ctypes in oracle/__init__.py) ----- */
typedef struct {
    int64_t K;     /* number of bins */
    int64_t k0;    /* f_min / df, an integer */
    double df;     /* bin width [Hz]; f_k = (k0 + k) df */
    int32_t n_chan;
    int32_t pad;
} orc_grid;

typedef struct {
    int32_t pn_order;        /* highest power j of v kept in the phase series, 0..7 */
    int32_t response;        /* 0: none (one channel), 1: LISA low-frequency A,E,
                                2: LISA full frequency-domain response A,E (,T) */
    int32_t support;         /* 0: whole band, 1: observation window */
    int32_t eccentric;       /* 0: circular, theta has 7 entries; 1: an 8th entry e0 */
    double t_obs;            /* observation time [s] */
    double orbit_phase0;     /* orbital angle of the constellation centre at t = 0 [rad] */
    double cartwheel_phase0; /* in-plane angle of spacecraft 0 at t = 0 [rad] */
    int32_t sparse_stride;   /* 0: template evaluated at every bin; > 0: the sparse-grid
                                evaluation of Sec 4, nodes every sparse_stride bins, cubic
                                spline onto the FFT grid (see sparse_spline below) */
    int32_t pad;
} orc_model;

/* theta layout: Mc [Msun, detector frame], eta, f_low [Hz], lambda, beta, iota, psi
 * (, e0: the eccentricity at GW frequency f_low, eccentric models only) */
enum { TH_MC = 0, TH_ETA, TH_FLOW, TH_LAMBDA, TH_BETA, TH_IOTA, TH_PSI, TH_DIM, TH_E0 = TH_DIM };

static int theta_dim(const orc_model* m) { return m->eccentric ? TH_DIM + 1 : TH_DIM; }

/* ---- per-source derived quantities ------------------------------------ */
typedef struct {
    int valid;
    ld eta;
    ld piM;      /* pi * total mass [s] */
    ld pref;     /* 3 / (256 pi eta): converts sum psi_j v^(j-5) into cycles */
    ld psi[8];   /* PN coefficients; psi5 and psi6 hold their v-independent parts */
    ld a5;       /* multiplies (1 + 3 ln(v / v_lso)) in psi5 */
    ld b6log;    /* multiplies ln(4 v) in psi6 (= -6848/21) */
    int order;
    ld tc;       /* coalescence time [s], fixed by t(f_low) = 0 */
    ld ecc;      /* eccentric term: -(2355/1462) e0^2 v0^(19/3), multiplies v^(-19/3) in the series */
    /* extrinsic */
    double a_plus, a_cross; /* (1 + cos^2 iota)/2, cos iota */
    double eplus[3][3], ecross[3][3];
    double nhat[3];
} src_t;

/* PN phase coefficients of the circular TaylorF2 approximant (Buonanno, Iyer,
 * Ochsner, Pan & Sathyaprakash 2009, eq. 3.18); e0 -> 0 limit of the
 * TaylorF2Ecc model the paper uses (Sec 4). */
static void pn_coefficients(src_t* s)
{
    const ld eta = s->eta, eta2 = eta * eta, eta3 = eta2 * eta;
    const ld pi = PI_L;
    for (int j = 0; j < 8; ++j) s->psi[j] = 0.0L;
    s->psi[0] = 1.0L;
    s->psi[1] = 0.0L;
    s->psi[2] = 3715.0L / 756.0L + 55.0L * eta / 9.0L;
    s->psi[3] = -16.0L * pi;
    s->psi[4] = 15293365.0L / 508032.0L + 27145.0L * eta / 504.0L + 3085.0L * eta2 / 72.0L;
    s->a5 = pi * (38645.0L / 756.0L - 65.0L * eta / 9.0L);
    s->psi[5] = 0.0L; /* handled through a5 */
    s->psi[6] = 11583231236531.0L / 4694215680.0L - 640.0L * pi * pi / 3.0L
              - 6848.0L * EULER_GAMMA_L / 21.0L
              + (-15737765635.0L / 3048192.0L + 2255.0L * pi * pi / 12.0L) * eta
              + 76055.0L * eta2 / 1728.0L - 127825.0L * eta3 / 1296.0L;
    s->b6log = -6848.0L / 21.0L;
    s->psi[7] = pi * (77096675.0L / 254016.0L + 378515.0L * eta / 1512.0L - 74045.0L * eta2 / 756.0L);
}

/* Sum_j psi_j(v) v^(j-5) for j <= order.  The v-dependent parts of psi5
 * (3 ln(v/v_lso)) and psi6 (ln 4v) are included here; v_lso = 1/sqrt(6). */
static ld pn_series(const src_t* s, ld v)
{
    const ld lnv = logl(v);
    ld vp[8];
    vp[0] = 1.0L;
    for (int j = 1; j < 8; ++j) vp[j] = vp[j - 1] * v;
    ld sum = 0.0L;
    for (int j = 0; j <= s->order; ++j) {
        ld c;
        if (j == 5)
            c = s->a5 * (1.0L + 3.0L * (lnv + 0.5L * logl(6.0L)));
        else if (j == 6)
            c = s->psi[6] + s->b6log * (logl(4.0L) + lnv);
        else
            c = s->psi[j];
        sum += c * vp[j];
    }
    if (s->ecc != 0.0L) sum += s->ecc * powl(v, -19.0L / 3.0L);
    return sum / (vp[5]);
}

/* f * d/df [ Sum_j psi_j(v) v^(j-5) ], using dv/df = v / (3 f). */
static ld pn_series_fderiv(const src_t* s, ld v)
{
    const ld lnv = logl(v);
    ld vp[8];
    vp[0] = 1.0L;
    for (int j = 1; j < 8; ++j) vp[j] = vp[j - 1] * v;
    ld sum = 0.0L;
    for (int j = 0; j <= s->order; ++j) {
        if (j == 5) {
            /* d/dv [a5 (1 + 3 ln v)] * v/3 = a5 */
            sum += s->a5 * vp[5];
        } else if (j == 6) {
            /* d/dv [(psi6 + b ln 4v) v] * v/3 = (psi6(v) + b) v / 3 */
            const ld p6 = s->psi[6] + s->b6log * (logl(4.0L) + lnv);
            sum += (p6 + s->b6log) * vp[6] / 3.0L;
        } else {
            sum += s->psi[j] * ((ld)(j - 5) / 3.0L) * vp[j];
        }
    }
    /* f d/df of ecc v^(-34/3) = ecc (-34/9) v^(-34/3) */
    if (s->ecc != 0.0L) sum += s->ecc * (-34.0L / 9.0L) * powl(v, -19.0L / 3.0L);
    return sum / vp[5];
}

/* Phase in cycles, Psi(f)/(2 pi) = f t_c - 1/8 + (3/(256 pi eta)) Sum_j psi_j v^(j-5),
 * phi_c = 0 (a constant phase, maximised away by the statistic). */
static ld phase_cycles(const src_t* s, ld f)
{
    const ld v = cbrtl(s->piM * f);
    return f * s->tc - 0.125L + s->pref * pn_series(s, v);
}

/* The same phase in quad precision (the coefficients as computed above,
 * every operation on them in __float128), for the sparse-grid nodes. */
static qd pn_series_q(const src_t* s, qd v)
{
    const qd lnv = logq(v);
    qd vp[8];
    vp[0] = 1.0Q;
    for (int j = 1; j < 8; ++j) vp[j] = vp[j - 1] * v;
    qd sum = 0.0Q;
    for (int j = 0; j <= s->order; ++j) {
        qd c;
        if (j == 5)
            c = (qd)s->a5 * (1.0Q + 3.0Q * (lnv + 0.5Q * logq(6.0Q)));
        else if (j == 6)
            c = (qd)s->psi[6] + (qd)s->b6log * (logq(4.0Q) + lnv);
        else
            c = (qd)s->psi[j];
        sum += c * vp[j];
    }
    if (s->ecc != 0.0L) sum += (qd)s->ecc * powq(v, -19.0Q / 3.0Q);
    return sum / vp[5];
}

static qd phase_cycles_q(const src_t* s, qd f)
{
    const qd v = cbrtq((qd)s->piM * f);
    return f * (qd)s->tc - 0.125Q + (qd)s->pref * pn_series_q(s, v);
}

/* SPA time t(f) = (1/2pi) dPsi/df [s]. */
static ld spa_time(const src_t* s, ld f)
{
    const ld v = cbrtl(s->piM * f);
    return s->tc + s->pref * pn_series_fderiv(s, v) / f;
}

static void outer_sym(const double a[3], const double b[3], double w, double m[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) m[i][j] += w * a[i] * b[j];
}

/* Polarisation tensors of a wave from sky direction (lambda, beta), rotated by
 * psi: e+ = p p - q q, ex = p q + q p with p = cos(psi) u + sin(psi) v,
 * q = -sin(psi) u + cos(psi) v, u and v orthonormal and perpendicular to n. */
static void polarisation(src_t* s, double lam, double bet, double psi)
{
    const double cl = cos(lam), sl = sin(lam), cb = cos(bet), sb = sin(bet);
    const double n[3] = {cb * cl, cb * sl, sb};
    const double u[3] = {sb * cl, sb * sl, -cb};
    const double v[3] = {sl, -cl, 0.0};
    double p[3], q[3];
    for (int i = 0; i < 3; ++i) {
        p[i] = cos(psi) * u[i] + sin(psi) * v[i];
        q[i] = -sin(psi) * u[i] + cos(psi) * v[i];
        s->nhat[i] = n[i];
    }
    memset(s->eplus, 0, sizeof s->eplus);
    memset(s->ecross, 0, sizeof s->ecross);
    outer_sym(p, p, 1.0, s->eplus);
    outer_sym(q, q, -1.0, s->eplus);
    outer_sym(p, q, 1.0, s->ecross);
    outer_sym(q, p, 1.0, s->ecross);
}

/* Rigid equilateral constellation: centre on a 1 AU circular orbit at
 * angle Phi; plane inclined by 60 degrees to the ecliptic (normal
 * z/2 - (sqrt 3 / 2) r_hat); the spacecraft turn in that plane once per orbit
 * in the opposite sense (cartwheel).  D_X = (a01 a01 - a02 a02)/2 etc.,
 * A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6. */
/* Unit in-plane positions p[a] of the three spacecraft relative to the
 * constellation centre (the craft sit at R0 + (L / sqrt3) p[a]). */
static void constellation(double Phi, double cart0, double p[3][3])
{
    const double cp = cos(Phi), sp = sin(Phi);
    const double er[3] = {cp, sp, 0.0}, ephi[3] = {-sp, cp, 0.0}, ez[3] = {0.0, 0.0, 1.0};
    const double h3 = sqrt(3.0) / 2.0;
    double e1[3];
    for (int i = 0; i < 3; ++i) e1[i] = -0.5 * er[i] - h3 * ez[i];
    const double zeta = cart0 - Phi;
    for (int a = 0; a < 3; ++a) {
        const double th = zeta + 2.0 * M_PI * a / 3.0;
        for (int i = 0; i < 3; ++i) p[a][i] = cos(th) * e1[i] + sin(th) * ephi[i];
    }
}

static void detector_tensors(double Phi, double cart0, double DA[3][3], double DE[3][3])
{
    double p[3][3];
    constellation(Phi, cart0, p);
    double arm[3][3][3]; /* arm[a][b] = unit vector from craft a to craft b */
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int i = 0; i < 3; ++i) arm[a][b][i] = (p[b][i] - p[a][i]) / sqrt(3.0);
    double DX[3][3] = {{0}}, DY[3][3] = {{0}}, DZ[3][3] = {{0}};
    outer_sym(arm[0][1], arm[0][1], 0.5, DX);
    outer_sym(arm[0][2], arm[0][2], -0.5, DX);
    outer_sym(arm[1][2], arm[1][2], 0.5, DY);
    outer_sym(arm[1][0], arm[1][0], -0.5, DY);
    outer_sym(arm[2][0], arm[2][0], 0.5, DZ);
    outer_sym(arm[2][1], arm[2][1], -0.5, DZ);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            DA[i][j] = (DZ[i][j] - DX[i][j]) / sqrt(2.0);
            DE[i][j] = (DX[i][j] - 2.0 * DY[i][j] + DZ[i][j]) / sqrt(6.0);
        }
}

static double contract(const double a[3][3], const double b[3][3])
{
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) s += a[i][j] * b[i][j];
    return s;
}

/* Antenna patterns F[chan][pol] (pol 0 = plus, 1 = cross) at SPA time t. */
static void antenna(const src_t* s, const orc_model* m, double t, double F[2][2])
{
    const double Phi = m->orbit_phase0 + 2.0 * M_PI * t / (double)YEAR_SI;
    double DA[3][3], DE[3][3];
    detector_tensors(Phi, m->cartwheel_phase0, DA, DE);
    F[0][0] = contract(DA, s->eplus);
    F[0][1] = contract(DA, s->ecross);
    F[1][0] = contract(DE, s->eplus);
    F[1][1] = contract(DE, s->ecross);
}

/* Doppler phase in cycles, -f n.R(t)/c, R = 1 AU (cos Phi, sin Phi, 0). */
static double doppler_cycles(const src_t* s, const orc_model* m, double f, double t)
{
    const double Phi = m->orbit_phase0 + 2.0 * M_PI * t / (double)YEAR_SI;
    const double nR = s->nhat[0] * cos(Phi) + s->nhat[1] * sin(Phi);
    return -f * nR * (double)(AU_SI / C_SI);
}

/* Full frequency-domain response (response 2), from the light-travel
 * formula of one link and first-generation TDI on the same rigid equal-arm
 * constellation, at frequency f and stationary-phase time t.
 *
 * Link j -> i (unit vector n from craft j to craft i, light time L): for a
 * plane wave travelling along k = -nhat, H(t - k.x) = h(t - k.x) P, the
 * fractional frequency shift is
 *     y_ij(t) = n.[H(t - L - k.x_j) - H(t - k.x_i)].n / (2 (1 - k.n)).
 * A delay tau multiplies a Fourier component by e^{-2 pi i f tau}, so with
 * the polarisation content P = a+ e+ - i ax ex of the template (the same as
 * the low-frequency response's) and x_i - x_j = L n,
 *     y_ij / h = -i pi f L sinc(pi f L (1 - k.n)) e^{-i pi f (L + k.(x_i + x_j))} n.P.n .
 * The common delay of the constellation centre, e^{-2 pi i f k.R0}, is the
 * Doppler factor already in the phase, so x are taken from the centre.
 * TDI (equal, static arms; one-arm delay z = e^{-2 pi i f L}):
 *     X = (1 - z^2) [(y_01 + z y_10) - (y_02 + z y_20)], Y and Z cyclic,
 *     A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3,
 * each divided by 4 (2 pi f L)^2, so that A and E tend to the low-frequency
 * response (D_A:P, D_E:P) as f L -> 0.  R[c] for c < nch. */
static void fd_transfer(const src_t* s, const orc_model* m, double f, double t, int nch, double complex R[3])
{
    const double Phi = m->orbit_phase0 + 2.0 * M_PI * t / (double)YEAR_SI;
    double p[3][3];
    constellation(Phi, m->cartwheel_phase0, p);
    const double L = ARM_SI / (double)C_SI; /* light time of one arm [s] */
    const double r = L / sqrt(3.0);        /* centre-to-craft light time [s] */
    double complex y[3][3] = {{0}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            if (i == j) continue;
            double n[3];
            for (int c = 0; c < 3; ++c) n[c] = (p[i][c] - p[j][c]) / sqrt(3.0);
            double kn = 0.0, kx = 0.0, npp = 0.0, npx = 0.0;
            for (int c = 0; c < 3; ++c) {
                kn -= s->nhat[c] * n[c];
                kx -= r * s->nhat[c] * (p[i][c] + p[j][c]);
                for (int d = 0; d < 3; ++d) {
                    npp += n[c] * s->eplus[c][d] * n[d];
                    npx += n[c] * s->ecross[c][d] * n[d];
                }
            }
            const double complex nPn = s->a_plus * npp - I * s->a_cross * npx;
            const double arg = M_PI * f * L * (1.0 - kn);
            const double sinc = arg == 0.0 ? 1.0 : sin(arg) / arg;
            y[i][j] = -I * M_PI * f * L * sinc * cexp(-I * M_PI * f * (L + kx)) * nPn;
        }
    const double complex z = cexp(-2.0 * I * M_PI * f * L);
    const double complex w = 1.0 - z * z;
    const double complex X = w * ((y[0][1] + z * y[1][0]) - (y[0][2] + z * y[2][0]));
    const double complex Y = w * ((y[1][2] + z * y[2][1]) - (y[1][0] + z * y[0][1]));
    const double complex Z = w * ((y[2][0] + z * y[0][2]) - (y[2][1] + z * y[1][2]));
    const double x = 2.0 * M_PI * f * L;
    const double norm = 4.0 * x * x;
    R[0] = (Z - X) / sqrt(2.0) / norm;
    R[1] = (X - 2.0 * Y + Z) / sqrt(6.0) / norm;
    if (nch > 2) R[2] = (X + Y + Z) / sqrt(3.0) / norm;
}

/* Derive everything that depends on theta only.  Invalid theta -> valid = 0. */
static void make_source(const double* th, const orc_model* m, src_t* s)
{
    memset(s, 0, sizeof *s);
    const double Mc = th[TH_MC], eta = th[TH_ETA], flow = th[TH_FLOW];
    for (int i = 0; i < theta_dim(m); ++i)
        if (!isfinite(th[i])) return;
    if (!(Mc > 0.0) || !(eta > 0.0) || !(eta <= 0.25) || !(flow > 0.0)) return;
    const double e0 = m->eccentric ? th[TH_E0] : 0.0;
    if (!(e0 >= 0.0) || !(e0 < 0.5)) return; /* a leading-order expansion in e0^2 */
    if (m->pn_order < 0 || m->pn_order > 7) return;
    s->valid = 1;
    s->order = m->pn_order;
    s->eta = eta;
    const ld tsun = GM_SUN_SI / (C_SI * C_SI * C_SI);
    const ld M = (ld)Mc * powl((ld)eta, -0.6L) * tsun; /* total mass [s] */
    s->piM = PI_L * M;
    s->pref = 3.0L / (256.0L * PI_L * (ld)eta);
    pn_coefficients(s);
    /* t(f_low) = 0 fixes t_c: f_low is the GW frequency at the start of the
     * observation (Table tab:GW150914-like_injection lists t_c as derived). */
    const ld fl = (ld)flow;
    const ld v = cbrtl(s->piM * fl);
    /* Eccentric phase (the TaylorF2Ecc model of Sec 4): the leading-order
     * correction in e0^2 to the Newtonian term of the SPA phase, with e0 the
     * eccentricity at GW frequency f_low (v0 = v(f_low)); Yunes & Arun 2009. */
    s->ecc = -(2355.0L / 1462.0L) * (ld)e0 * (ld)e0 * powl(v, 19.0L / 3.0L);
    s->tc = -s->pref * pn_series_fderiv(s, v) / fl;
    const double iota = th[TH_IOTA];
    s->a_plus = 0.5 * (1.0 + cos(iota) * cos(iota));
    s->a_cross = cos(iota);
    polarisation(s, th[TH_LAMBDA], th[TH_BETA], th[TH_PSI]);
}

static ld freq(const orc_grid* g, int64_t k) { return (ld)(g->k0 + k) * (ld)g->df; }

/* Template h_alpha(f_k) (complex, per channel), up to one global complex
 * constant (distance and phase, which the statistic removes).  Returns the
 * number of channels written. */
static int template_bin(const src_t* s, const orc_model* m, const orc_grid* g, int64_t k,
                        double hre[3], double him[3])
{
    const ld f = freq(g, k);
    const ld ph = phase_cycles(s, f);
    const ld phf = ph - floorl(ph); /* reduce before leaving extended precision */
    const double amp = (double)powl(f, -7.0L / 6.0L);
    if (m->response == 0) {
        const double a = -2.0 * M_PI * (double)phf;
        hre[0] = amp * cos(a);
        him[0] = amp * sin(a);
        return 1;
    }
    const double t = (double)spa_time(s, f);
    double tot = (double)phf + doppler_cycles(s, m, (double)f, t);
    tot -= floor(tot);
    const double c = cos(2.0 * M_PI * tot), sn = sin(2.0 * M_PI * tot);
    if (m->response == 2) {
        double complex R[3];
        fd_transfer(s, m, (double)f, t, g->n_chan, R);
        for (int a = 0; a < g->n_chan; ++a) {
            /* h = amp R e^{-i 2 pi tot} */
            const double rr = creal(R[a]), ri = cimag(R[a]);
            hre[a] = amp * (rr * c + ri * sn);
            him[a] = amp * (ri * c - rr * sn);
        }
        return g->n_chan;
    }
    double F[2][2];
    antenna(s, m, t, F);
    for (int a = 0; a < 2; ++a) {
        /* R = F+ A+ - i Fx Ax ; h = amp R e^{-i 2 pi tot} */
        const double rr = F[a][0] * s->a_plus, ri = -F[a][1] * s->a_cross;
        hre[a] = amp * (rr * c + ri * sn);
        him[a] = amp * (ri * c - rr * sn);
    }
    return 2;
}

/* ---- sparse-grid evaluation (Sec 4, waveform and response paragraphs) ----
 * The paper evaluates the waveform and the response on a frequency grid far
 * coarser than the FFT grid (by a factor 1000) and interpolates them onto the
 * FFT grid with cubic splines.  Readings taken where the paper is silent:
 *   - the coarse grid is every S-th FFT bin (S = sparse_stride), a fixed grid
 *     in frequency, restricted to the particle's support; the support's first
 *     and last bins are nodes too, so every support bin lies between nodes;
 *   - the interpolated quantities are the template's phase in cycles (the GW
 *     phase plus the Doppler phase of the response) and the real and
 *     imaginary parts of each channel's response (transfer function); the
 *     amplitude f^-7/6 is exact (it is folded into the data products);
 *   - the spline is the not-a-knot cubic spline (third derivative continuous
 *     at the second and the second-to-last node); with three nodes it is the
 *     parabola through them, with two the line;
 *   - the equal-[h|h] segment edges keep the template's exact weights at
 *     their own nodes (Sec 2.2's rule does not depend on how the template is
 *     evaluated on the dense grid).
 * Node phases and their spline are taken in quad precision (see the file
 * header), the response parts in extended precision like the exact template. */
typedef struct {
    int64_t n;  /* intervals: nodes x[0..n] */
    int nr;     /* response quantities: re / im of each response channel (0 without response) */
    int64_t* x; /* [n + 1] node bins */
    qd* yph;    /* [n + 1] node phases (cycles, unreduced) */
    qd* Mph;    /* [n + 1] second derivatives of the phase spline at the nodes */
    ld* y;      /* [n + 1][nr] node values of the response parts */
    ld* M;      /* [n + 1][nr] second derivatives of their splines */
} sparse_spline;

/* Exact values at bin k of the spline's quantities: the template phase in
 * cycles (GW + Doppler), in quad precision, and the response's real and
 * imaginary parts per channel in r[].  Returns the number of response parts. */
static int exact_quantities(const src_t* s, const orc_model* m, const orc_grid* g, int64_t k, qd* phase, ld* r)
{
    const ld f = freq(g, k);
    const qd fq = (qd)(g->k0 + k) * (qd)g->df;
    *phase = phase_cycles_q(s, fq);
    if (m->response == 0) return 0;
    const double t = (double)spa_time(s, f);
    *phase += (qd)doppler_cycles(s, m, (double)f, t);
    if (m->response == 2) {
        double complex R[3];
        fd_transfer(s, m, (double)f, t, g->n_chan, R);
        for (int a = 0; a < g->n_chan; ++a) {
            r[2 * a] = creal(R[a]);
            r[2 * a + 1] = cimag(R[a]);
        }
        return 2 * g->n_chan;
    }
    double F[2][2];
    antenna(s, m, t, F);
    for (int a = 0; a < 2; ++a) {
        r[2 * a] = F[a][0] * s->a_plus;   /* R = F+ A+ - i Fx Ax */
        r[2 * a + 1] = -F[a][1] * s->a_cross;
    }
    return 4;
}

/* Second derivatives M[0..N] of the not-a-knot cubic spline through
 * (x[j], y[j]), j = 0..N (N >= 1 intervals), in quad precision.
 * Continuity of the first derivative at interior nodes i = 1..N-1:
 *   h[i-1] M[i-1] + 2 (h[i-1] + h[i]) M[i] + h[i] M[i+1] = 6 (s[i] - s[i-1]),
 * s[i] = (y[i+1] - y[i]) / h[i]; not-a-knot at both ends:
 *   (M[1] - M[0]) / h[0] = (M[2] - M[1]) / h[1],
 *   (M[N-1] - M[N-2]) / h[N-2] = (M[N] - M[N-1]) / h[N-1].
 * M[0] and M[N] are eliminated from the first and last interior rows,
 * leaving a tridiagonal system in M[1..N-1] (Thomas algorithm).  With two
 * intervals the spline is the parabola through the three nodes, with one the
 * line (M = 0). */
static void spline_second_derivatives(int64_t N, const int64_t* x, const qd* y, qd* M)
{
    for (int64_t j = 0; j <= N; ++j) M[j] = 0.0Q;
    if (N < 2) return;
    qd* h = (qd*)malloc(sizeof(qd) * N);
    for (int64_t j = 0; j < N; ++j) h[j] = (qd)(x[j + 1] - x[j]);
    if (N == 2) {
        const qd s0 = (y[1] - y[0]) / h[0], s1 = (y[2] - y[1]) / h[1];
        M[0] = M[1] = M[2] = 2.0Q * (s1 - s0) / (h[0] + h[1]);
        free(h);
        return;
    }
    const int64_t R = N - 1;
    qd* a = (qd*)malloc(sizeof(qd) * R);
    qd* b = (qd*)malloc(sizeof(qd) * R);
    qd* cc = (qd*)malloc(sizeof(qd) * R);
    qd* r = (qd*)malloc(sizeof(qd) * R);
    for (int64_t i = 1; i <= R; ++i) {
        const qd sl = (y[i] - y[i - 1]) / h[i - 1], sr = (y[i + 1] - y[i]) / h[i];
        a[i - 1] = h[i - 1];
        b[i - 1] = 2.0Q * (h[i - 1] + h[i]);
        cc[i - 1] = h[i];
        r[i - 1] = 6.0Q * (sr - sl);
    }
    /* M[0] = ((h0 + h1) M[1] - h0 M[2]) / h1 into row 1 */
    b[0] += h[0] * (h[0] + h[1]) / h[1];
    cc[0] -= h[0] * h[0] / h[1];
    /* M[N] = ((h[N-2] + h[N-1]) M[N-1] - h[N-1] M[N-2]) / h[N-2] into row N-1 */
    b[R - 1] += h[N - 1] * (h[N - 2] + h[N - 1]) / h[N - 2];
    a[R - 1] -= h[N - 1] * h[N - 1] / h[N - 2];
    for (int64_t i = 1; i < R; ++i) {
        const qd w = a[i] / b[i - 1];
        b[i] -= w * cc[i - 1];
        r[i] -= w * r[i - 1];
    }
    M[R] = r[R - 1] / b[R - 1];
    for (int64_t i = R - 1; i >= 1; --i) M[i] = (r[i - 1] - cc[i - 1] * M[i + 1]) / b[i - 1];
    M[0] = ((h[0] + h[1]) * M[1] - h[0] * M[2]) / h[1];
    M[N] = ((h[N - 2] + h[N - 1]) * M[N - 1] - h[N - 1] * M[N - 2]) / h[N - 2];
    free(a);
    free(b);
    free(cc);
    free(r);
    free(h);
}

/* Node bins over [klo, khi): klo, the multiples of S strictly inside, khi - 1. */
static void sparse_build(const src_t* s, const orc_model* m, const orc_grid* g, int64_t klo, int64_t khi,
                         sparse_spline* sp)
{
    const int64_t S = m->sparse_stride;
    int64_t n = 0;
    int64_t* x = (int64_t*)malloc(sizeof(int64_t) * ((khi - klo) / S + 3));
    x[n++] = klo;
    for (int64_t k = (klo / S + 1) * S; k < khi - 1; k += S) x[n++] = k;
    if (khi - 1 > klo) x[n++] = khi - 1;
    sp->n = n - 1;
    sp->x = x;
    qd ph;
    ld r[6];
    sp->nr = exact_quantities(s, m, g, klo, &ph, r);
    const int nr = sp->nr;
    sp->yph = (qd*)malloc(sizeof(qd) * n);
    sp->Mph = (qd*)malloc(sizeof(qd) * n);
    sp->y = (ld*)malloc(sizeof(ld) * n * (nr > 0 ? nr : 1));
    sp->M = (ld*)malloc(sizeof(ld) * n * (nr > 0 ? nr : 1));
    for (int64_t j = 0; j < n; ++j) {
        exact_quantities(s, m, g, x[j], &sp->yph[j], r);
        for (int c = 0; c < nr; ++c) sp->y[j * nr + c] = r[c];
    }
    spline_second_derivatives(sp->n, x, sp->yph, sp->Mph);
    qd* yc = (qd*)malloc(sizeof(qd) * n);
    qd* Mc = (qd*)malloc(sizeof(qd) * n);
    for (int c = 0; c < nr; ++c) {
        for (int64_t j = 0; j < n; ++j) yc[j] = (qd)sp->y[j * nr + c];
        spline_second_derivatives(sp->n, x, yc, Mc);
        for (int64_t j = 0; j < n; ++j) sp->M[j * nr + c] = (ld)Mc[j];
    }
    free(yc);
    free(Mc);
}

static void sparse_free(sparse_spline* sp)
{
    free(sp->x);
    free(sp->yph);
    free(sp->Mph);
    free(sp->y);
    free(sp->M);
}

/* The spline's quantities at bin k (inside [x0, xn]): on interval j,
 * S(u) = y_j + b u + (M_j / 2) u^2 + (M_{j+1} - M_j) / (6 h) u^3, u = k - x_j,
 * b = (y_{j+1} - y_j) / h - h (2 M_j + M_{j+1}) / 6.  The phase comes back
 * reduced to [0, 1) cycles (taken in quad precision), the response parts in r[]. */
static double sparse_eval(const sparse_spline* sp, int64_t k, ld* r)
{
    const int nr = sp->nr;
    if (sp->n == 0) {
        for (int c = 0; c < nr; ++c) r[c] = sp->y[c];
        return (double)(sp->yph[0] - floorq(sp->yph[0]));
    }
    int64_t lo = 0, hi = sp->n - 1; /* interval: the last j <= n-1 with x_j <= k */
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (sp->x[mid] <= k) lo = mid; else hi = mid - 1;
    }
    const int64_t j = lo;
    const int64_t hb = sp->x[j + 1] - sp->x[j], ub = k - sp->x[j];
    {
        const qd h = (qd)hb, u = (qd)ub;
        const qd y0 = sp->yph[j], y1 = sp->yph[j + 1], M0 = sp->Mph[j], M1 = sp->Mph[j + 1];
        const qd b = (y1 - y0) / h - h * (2.0Q * M0 + M1) / 6.0Q;
        const qd q = y0 + u * (b + u * (0.5Q * M0 + u * (M1 - M0) / (6.0Q * h)));
        for (int c = 0; c < nr; ++c) {
            const ld hl = (ld)hb, ul = (ld)ub;
            const ld z0 = sp->y[j * nr + c], z1 = sp->y[(j + 1) * nr + c];
            const ld N0 = sp->M[j * nr + c], N1 = sp->M[(j + 1) * nr + c];
            const ld bb = (z1 - z0) / hl - hl * (2.0L * N0 + N1) / 6.0L;
            r[c] = z0 + ul * (bb + ul * (0.5L * N0 + ul * (N1 - N0) / (6.0L * hl)));
        }
        return (double)(q - floorq(q));
    }
}

/* Template at bin k from the spline (the sparse-grid counterpart of
 * template_bin; same conventions). */
static int sparse_template_bin(const sparse_spline* sp, const orc_model* m, const orc_grid* g, int64_t k,
                               double hre[3], double him[3])
{
    ld r[6];
    const double tot = sparse_eval(sp, k, r);
    const ld f = freq(g, k);
    const double amp = (double)powl(f, -7.0L / 6.0L);
    const double c = cos(2.0 * M_PI * tot), sn = sin(2.0 * M_PI * tot);
    if (m->response == 0) {
        hre[0] = amp * c;
        him[0] = -amp * sn;
        return 1;
    }
    const int nc = sp->nr / 2;
    for (int a = 0; a < nc; ++a) {
        const double rr = (double)r[2 * a], ri = (double)r[2 * a + 1];
        hre[a] = amp * (rr * c + ri * sn);
        him[a] = amp * (ri * c - rr * sn);
    }
    return nc;
}

/* Support [k_lo, k_hi): whole band, or the bins whose SPA time lies in the
 * observation window, 0 <= t(f_k) < T_obs.  t(f_low) = 0 and t rises with f,
 * so the lower edge is the first bin with f_k >= f_low (compared exactly in
 * extended precision); the upper edge is the first bin with t >= T_obs. */
static void support(const src_t* s, const orc_model* m, const orc_grid* g, double flow,
                    int64_t* klo, int64_t* khi)
{
    if (m->support == 0) {
        *klo = 0;
        *khi = g->K;
        return;
    }
    int64_t lo = 0;
    while (lo < g->K && freq(g, lo) < (ld)flow) ++lo;
    int64_t hi = lo;
    while (hi < g->K && spa_time(s, freq(g, hi)) < (ld)m->t_obs) ++hi;
    *klo = lo;
    *khi = hi;
}

/* Dense weight w(k) = sum_alpha |h_alpha(f_k)|^2 / S_alpha(f_k). */
static double weight(const src_t* s, const orc_model* m, const orc_grid* g, const double* psd,
                     int64_t k)
{
    double hr[3], hi[3];
    const int nc = template_bin(s, m, g, k, hr, hi);
    double w = 0.0;
    for (int a = 0; a < nc; ++a) w += (hr[a] * hr[a] + hi[a] * hi[a]) / psd[(int64_t)a * g->K + k];
    return w;
}

/* Cumulative of the equal-[h|h] edge rule over a non-empty support:
 * nodes x_j = k_lo + j G and k_hi - 1, W(k) = w(k) at nodes and linear in k
 * between them, C(k) = sum_{i = k_lo}^{k-1} W(i), returned as a malloc'd
 * array C[k - k_lo] for k = k_lo..k_hi, summed bin by bin. */
static double* edge_cumulative(const src_t* s, const orc_model* m, const orc_grid* g, const double* psd,
                               int64_t klo, int64_t khi, int32_t G)
{
    const int64_t len = khi - klo;
    /* node list */
    int64_t nn = (len - 1) / G + 1;
    if (klo + (nn - 1) * (int64_t)G != khi - 1) ++nn;
    int64_t* xs = (int64_t*)malloc(sizeof(int64_t) * nn);
    double* ws = (double*)malloc(sizeof(double) * nn);
    for (int64_t j = 0; j < nn; ++j) {
        xs[j] = (j == nn - 1) ? khi - 1 : klo + j * (int64_t)G;
        ws[j] = weight(s, m, g, psd, xs[j]);
    }
    double* C = (double*)malloc(sizeof(double) * (len + 1));
    C[0] = 0.0;
    int64_t j = 0;
    for (int64_t k = klo; k < khi; ++k) {
        while (j + 1 < nn && xs[j + 1] <= k) ++j;
        double W;
        if (j + 1 < nn) {
            const double frac = (double)(k - xs[j]) / (double)(xs[j + 1] - xs[j]);
            W = ws[j] + (ws[j + 1] - ws[j]) * frac;
        } else {
            W = ws[j];
        }
        C[k - klo + 1] = C[k - klo] + W;
    }
    free(ws);
    free(xs);
    return C;
}

/* Segment boundaries b[0..N].
 * mode 0 (equal [h|h], the paper's choice): nodes x_j = k_lo + j G and
 *   k_hi - 1; W(k) = w(k) at nodes, linear in k between nodes;
 *   C(k) = sum_{i = k_lo}^{k-1} W(i); b_n = min{k : C(k) >= (n/N) C(k_hi)}.
 *   Decided in double, like the GPU.
 * mode 1 (uniform bins): b_n = k_lo + floor(n (k_hi - k_lo) / N).
 * mode 2 (explicit edges e[0..N]): b_n = clamp(e_n, k_lo, k_hi). */
static void boundaries(const src_t* s, const orc_model* m, const orc_grid* g, const double* psd,
                       int64_t klo, int64_t khi, int32_t N, int mode, int32_t G,
                       const int64_t* edges, int64_t* b)
{
    b[0] = klo;
    b[N] = khi;
    if (khi <= klo) {
        for (int n = 0; n <= N; ++n) b[n] = klo;
        return;
    }
    if (mode == 1) {
        for (int n = 1; n < N; ++n) b[n] = klo + (int64_t)((__int128)n * (khi - klo) / N);
        return;
    }
    if (mode == 2) {
        for (int n = 0; n <= N; ++n) {
            int64_t e = edges[n];
            b[n] = e < klo ? klo : (e > khi ? khi : e);
        }
        return;
    }
    const int64_t len = khi - klo;
    double* C = edge_cumulative(s, m, g, psd, klo, khi, G);
    const double tot = C[len];
    int64_t kk = 0;
    for (int n = 1; n < N; ++n) {
        const double target = ((double)n / (double)N) * tot;
        while (kk < len && C[kk] < target) ++kk;
        b[n] = klo + kk;
    }
    free(C);
}

/* Channels each response model produces: none 1, low-frequency 2 (A, E),
 * full 2 (A, E) or 3 (A, E, T). */
static int channels_ok(const orc_model* m, const orc_grid* g)
{
    if (m->response == 0) return g->n_chan == 1;
    if (m->response == 1) return g->n_chan == 2;
    if (m->response == 2) return g->n_chan == 2 || g->n_chan == 3;
    return 0;
}

/* ---- exported: statistic ---------------------------------------------- */

/* Upsilon_N for P particles.
 *   d_ri  [n_chan][K][2]  data (real, imag)
 *   psd   [n_chan][K]     one-sided PSD
 *   theta [P][7]
 *   ups   [P]             output; NaN for invalid theta, 0 for empty support
 *   seg   [P][N][3]       optional (Re Z_n, Im Z_n, H_n)
 *   bnd   [P][N+1]        optional boundaries
 *   sup   [P][2]          optional support (k_lo, k_hi)
 * Z_n = sum_{k in n} sum_alpha d conj(h) / S, H_n = sum_{k in n} w(k);
 * term_n = 4 df |Z_n|^2 / H_n (0 when H_n = 0); Upsilon = sum_n term_n. */
int orc_evaluate(const orc_grid* g, const orc_model* m, const double* d_ri, const double* psd,
                 int64_t P, const double* theta, int32_t N, int32_t mode, int32_t G,
                 const int64_t* edges, double* ups, double* seg, int64_t* bnd, int64_t* sup,
                 int32_t n_threads)
{
    if (N < 1 || G < 1 || P < 0 || m->sparse_stride < 0) return -1;
    if (!channels_ok(m, g)) return -2;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#else
    (void)n_threads;
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < P; ++p) {
        src_t s;
        const double* th = theta + p * theta_dim(m);
        make_source(th, m, &s);
        if (!s.valid) {
            ups[p] = NAN;
            if (seg)
                for (int64_t i = 0; i < (int64_t)N * 3; ++i) seg[p * (int64_t)N * 3 + i] = NAN;
            if (bnd)
                for (int n = 0; n <= N; ++n) bnd[p * (int64_t)(N + 1) + n] = 0;
            if (sup) sup[2 * p] = sup[2 * p + 1] = 0;
            continue;
        }
        int64_t klo, khi;
        support(&s, m, g, th[TH_FLOW], &klo, &khi);
        int64_t* b = (int64_t*)malloc(sizeof(int64_t) * (N + 1));
        boundaries(&s, m, g, psd, klo, khi, N, mode, G, edges, b);
        sparse_spline sp = {0};
        const int sparse = m->sparse_stride > 0 && khi > klo;
        if (sparse) sparse_build(&s, m, g, klo, khi, &sp);
        ld total = 0.0L;
        for (int n = 0; n < N; ++n) {
            ld zr = 0.0L, zi = 0.0L, hh = 0.0L;
            for (int64_t k = b[n]; k < b[n + 1]; ++k) {
                double hr[3], hi[3];
                const int nc = sparse ? sparse_template_bin(&sp, m, g, k, hr, hi) : template_bin(&s, m, g, k, hr, hi);
                for (int a = 0; a < nc; ++a) {
                    const double S = psd[(int64_t)a * g->K + k];
                    const double dr = d_ri[((int64_t)a * g->K + k) * 2];
                    const double di = d_ri[((int64_t)a * g->K + k) * 2 + 1];
                    /* d * conj(h) / S */
                    zr += (ld)((dr * hr[a] + di * hi[a]) / S);
                    zi += (ld)((di * hr[a] - dr * hi[a]) / S);
                    hh += (ld)((hr[a] * hr[a] + hi[a] * hi[a]) / S);
                }
            }
            ld term = 0.0L;
            if (hh > 0.0L) term = 4.0L * (ld)g->df * (zr * zr + zi * zi) / hh;
            total += term;
            if (seg) {
                seg[(p * N + n) * 3 + 0] = (double)zr;
                seg[(p * N + n) * 3 + 1] = (double)zi;
                seg[(p * N + n) * 3 + 2] = (double)hh;
            }
        }
        if (sparse) sparse_free(&sp);
        ups[p] = (double)total;
        if (bnd)
            for (int n = 0; n <= N; ++n) bnd[p * (int64_t)(N + 1) + n] = b[n];
        if (sup) {
            sup[2 * p] = klo;
            sup[2 * p + 1] = khi;
        }
        free(b);
    }
    return 0;
}

/* The edge rule's cumulative for one particle (test support: where an edge
 * computed elsewhere differs from this oracle's, the cumulative shows
 * whether the target sits within rounding of C there).  sup [2] receives
 * the support; C(k) for the nk bins ks[i] (each clamped to [k_lo, k_hi]) goes
 * to Ck, and C(k_hi) to *total.  Returns -1 for invalid theta, -2 for a bad
 * channel count; an empty support gives total 0. */
int orc_edge_cumulative(const orc_grid* g, const orc_model* m, const double* psd, const double* theta, int32_t G,
                        int64_t nk, const int64_t* ks, double* Ck, double* total, int64_t* sup)
{
    if (G < 1) return -1;
    if (!channels_ok(m, g)) return -2;
    src_t s;
    make_source(theta, m, &s);
    if (!s.valid) return -1;
    int64_t klo, khi;
    support(&s, m, g, theta[TH_FLOW], &klo, &khi);
    sup[0] = klo;
    sup[1] = khi;
    if (khi <= klo) {
        *total = 0.0;
        for (int64_t i = 0; i < nk; ++i) Ck[i] = 0.0;
        return 0;
    }
    double* C = edge_cumulative(&s, m, g, psd, klo, khi, G);
    *total = C[khi - klo];
    for (int64_t i = 0; i < nk; ++i) {
        int64_t k = ks[i] < klo ? klo : (ks[i] > khi ? khi : ks[i]);
        Ck[i] = C[k - klo];
    }
    free(C);
    return 0;
}

/* Template over the whole grid, h_ri [n_chan][K][2]; zero outside the support. */
int orc_template(const orc_grid* g, const orc_model* m, const double* theta, double* h_ri)
{
    src_t s;
    if (!channels_ok(m, g)) return -2;
    if (m->sparse_stride < 0) return -1;
    make_source(theta, m, &s);
    memset(h_ri, 0, sizeof(double) * 2 * (size_t)g->n_chan * (size_t)g->K);
    if (!s.valid) return -1;
    int64_t klo, khi;
    support(&s, m, g, theta[TH_FLOW], &klo, &khi);
    sparse_spline sp = {0};
    const int sparse = m->sparse_stride > 0 && khi > klo;
    if (sparse) sparse_build(&s, m, g, klo, khi, &sp);
    for (int64_t k = klo; k < khi; ++k) {
        double hr[3], hi[3];
        const int nc = sparse ? sparse_template_bin(&sp, m, g, k, hr, hi) : template_bin(&s, m, g, k, hr, hi);
        for (int a = 0; a < nc; ++a) {
            h_ri[((int64_t)a * g->K + k) * 2] = hr[a];
            h_ri[((int64_t)a * g->K + k) * 2 + 1] = hi[a];
        }
    }
    if (sparse) sparse_free(&sp);
    return 0;
}

/* Phase, SPA time and t_c at arbitrary frequencies, for pins.
 * phase_frac [n] = Psi/(2 pi) mod 1 in [0,1); phase_int [n] = the integer part;
 * t [n] SPA time [s]; returns t_c through tc_out. */
int orc_phase(const orc_model* m, const double* theta, int64_t n, const double* f_hz,
              double* phase_frac, double* phase_int, double* t, double* tc_out)
{
    src_t s;
    make_source(theta, m, &s);
    if (!s.valid) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const ld ph = phase_cycles(&s, (ld)f_hz[i]);
        const ld fl = floorl(ph);
        if (phase_frac) phase_frac[i] = (double)(ph - fl);
        if (phase_int) phase_int[i] = (double)fl;
        if (t) t[i] = (double)spa_time(&s, (ld)f_hz[i]);
    }
    if (tc_out) *tc_out = (double)s.tc;
    return 0;
}

/* Same as orc_phase but on grid bins (f_k in extended precision). */
int orc_phase_bins(const orc_grid* g, const orc_model* m, const double* theta, int64_t n,
                   const int64_t* bins, double* phase_frac, double* t)
{
    src_t s;
    make_source(theta, m, &s);
    if (!s.valid) return -1;
    for (int64_t i = 0; i < n; ++i) {
        const ld f = freq(g, bins[i]);
        const ld ph = phase_cycles(&s, f);
        if (phase_frac) phase_frac[i] = (double)(ph - floorl(ph));
        if (t) t[i] = (double)spa_time(&s, f);
    }
    return 0;
}

/* Antenna patterns F [2 chan][2 pol], T-channel check value and the Doppler
 * phase per Hz at time t, for pins.  tchan [2] = (F+_T, Fx_T) with
 * D_T = (D_X + D_Y + D_Z)/sqrt3. */
int orc_response(const orc_model* m, const double* theta, double t, double* F, double* doppler_per_hz,
                 double* tchan)
{
    src_t s;
    make_source(theta, m, &s);
    if (!s.valid) return -1;
    double FF[2][2];
    antenna(&s, m, t, FF);
    F[0] = FF[0][0];
    F[1] = FF[0][1];
    F[2] = FF[1][0];
    F[3] = FF[1][1];
    if (doppler_per_hz) *doppler_per_hz = doppler_cycles(&s, m, 1.0, t);
    if (tchan) {
        /* Rebuild X, Y, Z from A and E is not possible; recompute directly. */
        const double Phi = m->orbit_phase0 + 2.0 * M_PI * t / (double)YEAR_SI;
        const double cp = cos(Phi), sp = sin(Phi);
        const double er[3] = {cp, sp, 0.0}, ephi[3] = {-sp, cp, 0.0}, ez[3] = {0.0, 0.0, 1.0};
        double e1[3], p[3][3];
        for (int i = 0; i < 3; ++i) e1[i] = -0.5 * er[i] - sqrt(3.0) / 2.0 * ez[i];
        for (int a = 0; a < 3; ++a) {
            const double th = m->cartwheel_phase0 - Phi + 2.0 * M_PI * a / 3.0;
            for (int i = 0; i < 3; ++i) p[a][i] = cos(th) * e1[i] + sin(th) * ephi[i];
        }
        double D[3][3] = {{0}};
        for (int a = 0; a < 3; ++a) {
            const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
            double u1[3], u2[3];
            for (int i = 0; i < 3; ++i) {
                u1[i] = (p[b1][i] - p[a][i]) / sqrt(3.0);
                u2[i] = (p[b2][i] - p[a][i]) / sqrt(3.0);
            }
            outer_sym(u1, u1, 0.5 / sqrt(3.0), D);
            outer_sym(u2, u2, -0.5 / sqrt(3.0), D);
        }
        tchan[0] = contract(D, s.eplus);
        tchan[1] = contract(D, s.ecross);
    }
    return 0;
}

/* Full-response transfer functions R [3][2] (A, E, T as real, imaginary) at
 * frequency f and time t, for pins. */
int orc_fd_transfer(const orc_model* m, const double* theta, double f, double t, double* R)
{
    src_t s;
    make_source(theta, m, &s);
    if (!s.valid) return -1;
    double complex r[3];
    fd_transfer(&s, m, f, t, 3, r);
    for (int a = 0; a < 3; ++a) {
        R[2 * a] = creal(r[a]);
        R[2 * a + 1] = cimag(r[a]);
    }
    return 0;
}

/* ---- exported: PSO (Sec 3.1) ------------------------------------------ */

/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11), written from its
 * published definition: ten rounds of two 32x32->64 multiplies with a Weyl
 * key schedule. */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Uniform in (0,1): 52 random bits x, (x + 1/2) 2^-52.  Counter =
 * (iteration, particle, dimension, stream); key = (seed low word, seed high
 * word + swarm id).  Streams: 0 r_P, 1 r_G, 2 sign of a zero velocity,
 * 3 initial position. */
double orc_uniform(uint64_t seed, uint32_t swarm, uint32_t iter, uint32_t particle, uint32_t dim,
                   uint32_t stream)
{
    const uint32_t ctr[4] = {iter, particle, dim, stream};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) + swarm};
    uint32_t o[4];
    orc_philox4x32_10(ctr, key, o);
    const uint64_t x = ((uint64_t)(o[0] >> 6) << 26) | (uint64_t)(o[1] >> 6);
    return ((double)x + 0.5) * 0x1p-52;
}

/* Initial positions, uniform in the prior box (Sec 3.1: drawn from the prior). */
void orc_pso_init(int64_t P, int32_t D, const double* lo, const double* hi, uint64_t seed,
                  uint32_t swarm, double* theta)
{
    for (int64_t p = 0; p < P; ++p)
        for (int d = 0; d < D; ++d) {
            const double r = orc_uniform(seed, swarm, 0u, (uint32_t)p, (uint32_t)d, 3u);
            const double w = hi[d] - lo[d];
            const double x = r * w;
            theta[p * D + d] = lo[d] + x;
        }
}

/* One synchronous move: u = Omega v + Phi_P r_P (pbest - x) + Phi_G r_G (gbest - x),
 * v = max(eps, |u|) u/|u|, x += v; periodic dimensions wrap into [lo, hi).
 * Operations are done one at a time in this order (no fused multiply-add), so
 * that any IEEE implementation reproduces them bit for bit. */
void orc_pso_move(int64_t P, int32_t D, double* theta, double* vel, const double* pbest,
                  const double* gbest, double omega, double phi_p, double phi_g, const double* eps,
                  const double* lo, const double* hi, const int32_t* periodic, uint64_t seed,
                  uint32_t swarm, uint32_t iter)
{
    for (int64_t p = 0; p < P; ++p)
        for (int d = 0; d < D; ++d) {
            const int64_t i = p * D + d;
            const double x = theta[i];
            const double rp = orc_uniform(seed, swarm, iter, (uint32_t)p, (uint32_t)d, 0u);
            const double rg = orc_uniform(seed, swarm, iter, (uint32_t)p, (uint32_t)d, 1u);
            volatile double t1 = omega * vel[i];
            volatile double a = phi_p * rp;
            volatile double b = pbest[i] - x;
            volatile double t2 = a * b;
            volatile double c = phi_g * rg;
            volatile double e = gbest[d] - x;
            volatile double t3 = c * e;
            volatile double s = t1 + t2;
            const double u = s + t3;
            double v;
            if (fabs(u) >= eps[d])
                v = u;
            else if (u != 0.0)
                v = copysign(eps[d], u);
            else if (eps[d] == 0.0)
                v = 0.0;
            else
                v = orc_uniform(seed, swarm, iter, (uint32_t)p, (uint32_t)d, 2u) < 0.5 ? -eps[d] : eps[d];
            double xn = x + v;
            if (periodic[d]) {
                const double per = hi[d] - lo[d];
                volatile double y = xn - lo[d];
                volatile double q = floor(y / per);
                volatile double z = per * q;
                y = y - z;
                xn = lo[d] + y;
            }
            vel[i] = v;
            theta[i] = xn;
        }
}

/* Best update: values outside the box (non-periodic dimensions) or NaN count
 * as -inf; a particle best moves on strict improvement; the swarm best is the
 * first particle holding the largest particle best, if that beats it. */
void orc_pso_best(int64_t P, int32_t D, const double* theta, const double* vals, const double* lo,
                  const double* hi, const int32_t* periodic, double* pbest, double* pbest_val,
                  double* gbest, double* gbest_val)
{
    for (int64_t p = 0; p < P; ++p) {
        double v = vals[p];
        int inbox = 1;
        for (int d = 0; d < D; ++d) {
            const double x = theta[p * D + d];
            if (!periodic[d] && !(x >= lo[d] && x <= hi[d])) inbox = 0;
        }
        if (!inbox || isnan(v)) v = -INFINITY;
        if (v > pbest_val[p]) {
            pbest_val[p] = v;
            for (int d = 0; d < D; ++d) pbest[p * D + d] = theta[p * D + d];
        }
    }
    int64_t best = -1;
    double bv = -INFINITY;
    for (int64_t p = 0; p < P; ++p)
        if (pbest_val[p] > bv) {
            bv = pbest_val[p];
            best = p;
        }
    if (best >= 0 && bv > *gbest_val) {
        *gbest_val = bv;
        for (int d = 0; d < D; ++d) gbest[d] = pbest[best * D + d];
    }
}

/* ---------------------------------------------------------------- noise realisations (Sec 5.1)
 * Realisation r of Gaussian noise of one-sided PSD S on the grid, in the
 * convention under which <n|h> ~ N(0, <h|h>) (eqn:inner_prod):
 *     n_{r,alpha,k} = sqrt(S_alpha(f_k) / (4 df)) (g1 + i g2),
 * g1, g2 independent standard normals from the Box-Muller transform (Box &
 * Muller 1958) of two uniforms in (0,1), each made of 52 bits of one
 * Philox4x32-10 block (Salmon et al. 2011) with counter (k, alpha, r,
 * ORC_NOISE_STREAM) and key (seed low word, seed high word):
 *     u1 = ((o0 >> 6) 2^26 + (o1 >> 6) + 1/2) 2^-52, u2 likewise from (o2, o3),
 *     g1 = sqrt(-2 ln u1) cos(2 pi u2),  g2 = sqrt(-2 ln u1) sin(2 pi u2).
 * out [n_chan][K][2]. */
#define ORC_NOISE_STREAM 0x6e6f6973u
void orc_noise(int64_t K, int32_t n_chan, const double* psd, double df, uint64_t seed, uint32_t r, double* out)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int32_t a = 0; a < n_chan; ++a)
        for (int64_t k = 0; k < K; ++k) {
            const uint32_t ctr[4] = {(uint32_t)k, (uint32_t)a, r, ORC_NOISE_STREAM};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            const uint64_t x1 = ((uint64_t)(o[0] >> 6) << 26) | (uint64_t)(o[1] >> 6);
            const uint64_t x2 = ((uint64_t)(o[2] >> 6) << 26) | (uint64_t)(o[3] >> 6);
            const double u1 = ((double)x1 + 0.5) * 0x1p-52;
            const double u2 = ((double)x2 + 0.5) * 0x1p-52;
            const double rad = sqrt(-2.0 * log(u1));
            const double ang = 2.0 * M_PI * u2;
            const double sig = sqrt(psd[a * K + k] / (4.0 * df));
            out[(a * K + k) * 2] = sig * (rad * cos(ang));
            out[(a * K + k) * 2 + 1] = sig * (rad * sin(ang));
        }
}
