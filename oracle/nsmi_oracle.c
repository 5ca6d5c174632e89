/*
 * nsmi oracle: a plain, slow, FP64 CPU definition of the batched
 * acceptance-walk nested sampler and of the frequency-domain
 * gravitational-wave likelihood it drives.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code, header or table with the HIP
 * library; the two meet only through seeded inputs.
 *
 * Every function follows a passage of arXiv:2509.04336 (cited per function)
 * or, where the paper is silent, a textbook definition named inline.  Loops
 * run in natural order, in double precision, with no blocking, fusion or
 * reordering; floating-point contraction is disabled at build time so that
 * the few explicit fma() calls are the only fused operations.
 *
 * Parity status per function is stated in its comment ("pinned by ..." or
 * "parity unpinned").
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Physical constants (SI).  Derived constants are computed, not typed. */
/* ------------------------------------------------------------------ */
#define OR_PI 3.141592653589793238462643383279502884
#define OR_GM_SUN 1.32712440018e20        /* m^3 s^-2 */
#define OR_C_SI 299792458.0               /* m s^-1 (exact) */
#define OR_MPC_SI 3.0856775814913673e22   /* m */
#define OR_EULER_GAMMA 0.5772156649015329

static double or_tsun(void) { return OR_GM_SUN / (OR_C_SI * OR_C_SI * OR_C_SI); }

/* Parameter order used everywhere (physical vector theta[11]):
 *   0 chirp mass Mc [Msun]   1 mass ratio q = m2/m1 <= 1   2 chi1   3 chi2
 *   4 luminosity distance dL [Mpc]   5 inclination theta_JN   6 ra alpha
 *   7 dec delta   8 polarisation psi   9 coalescence phase phi_c
 *  10 coalescence time t_c [s]
 * (Table 1 of the paper lists the priors of these parameters.) */
#define OR_NPAR 11

/* Likelihood kinds. */
#define OR_LIKE_GW 0      /* Whittle log-likelihood ratio, Sec. 3.3 / 4.1 */
#define OR_LIKE_GAUSS 1   /* Gaussian toy in the unit cube (closed-form Z) */
#define OR_LIKE_GW_RB 2   /* Whittle likelihood, data term heterodyned (relative binning) */

typedef struct {
    int32_t n_bins, n_det, ndim, like_kind;
    double f_lo, df;               /* f_k = f_lo + k*df */
    const double *data;            /* [n_det][n_bins][2] complex strain d_d(f_k) */
    const double *psd;             /* [n_det][n_bins] one-sided S_d(f_k) */
    const double *det_tensor;      /* [n_det][9] response tensor, or NULL */
    const double *det_loc;         /* [n_det][3] detector position (m), or NULL */
    const double *fixed_antenna;   /* [n_det][2] (F+, Fx) with zero delay, or NULL */
    const double *prior_lo;        /* [11] */
    const double *prior_hi;        /* [11] */
    const double *fixed_theta;     /* [11] values of parameters that are not sampled */
    double gmst;
    double toy_sigma;              /* width of the Gaussian toy */
    /* relative binning (like_kind OR_LIKE_GW_RB): fiducial parameters and
     * rb_bins + 1 node sample indices, rb_edges[0] = 0 < ... <
     * rb_edges[rb_bins] = n_bins */
    const double *rb_theta0;       /* [11] */
    const int32_t *rb_edges;       /* [rb_bins + 1] */
    int32_t rb_bins, rb_pad;
} or_event;

/* ------------------------------------------------------------------ */
/* Prior transforms (Sec. 3.4, Table 1): unit cube -> physical.        */
/* Pinned by CDF round trips and moments in tests/test_oracle_priors.  */
/* ------------------------------------------------------------------ */

/* Uniform on [a, b]. */
static double or_tr_uniform(double u, double a, double b) { return a + u * (b - a); }

/* Power law p(x) ~ x^2 on [a, b] (luminosity distance): invert the CDF
 * (x^3 - a^3) / (b^3 - a^3) = u. */
static double or_tr_powerlaw2(double u, double a, double b)
{
    double a3 = a * a * a, b3 = b * b * b;
    return cbrt(a3 + u * (b3 - a3));
}

/* Sine prior p(x) ~ sin x on [a, b] (inclination): CDF
 * (cos a - cos x) / (cos a - cos b) = u. */
static double or_tr_sine(double u, double a, double b)
{
    return acos(cos(a) - u * (cos(a) - cos(b)));
}

/* Cosine prior p(x) ~ cos x on [a, b] (declination): CDF
 * (sin x - sin a) / (sin b - sin a) = u. */
static double or_tr_cosine(double u, double a, double b)
{
    return asin(sin(a) + u * (sin(b) - sin(a)));
}

/* Map the sampled coordinates u[0..ndim) to the full physical vector.
 * ndim == 11 samples every parameter; ndim == 4 samples (Mc, q, chi1, chi2)
 * and takes the rest from fixed_theta. */
void or_prior_transform(const or_event *ev, const double *u, double *theta)
{
    for (int i = 0; i < OR_NPAR; ++i) theta[i] = ev->fixed_theta ? ev->fixed_theta[i] : 0.0;
    for (int i = 0; i < ev->ndim; ++i) {
        double a = ev->prior_lo[i], b = ev->prior_hi[i];
        switch (i) {
        case 4: theta[i] = or_tr_powerlaw2(u[i], a, b); break;
        case 5: theta[i] = or_tr_sine(u[i], a, b); break;
        case 7: theta[i] = or_tr_cosine(u[i], a, b); break;
        default: theta[i] = or_tr_uniform(u[i], a, b); break;
        }
    }
}

/* Coordinates that wrap around the unit interval (Sec. 4.1.1): right
 * ascension, polarisation angle and coalescence phase. */
int or_is_periodic(int ndim, int j)
{
    if (ndim != OR_NPAR) return 0;
    return j == 6 || j == 8 || j == 9;
}

/* ------------------------------------------------------------------ */
/* TaylorF2 aligned-spin phase (stationary-phase approximation).       */
/* The paper's approximant (IMRPhenomD, Sec. 3.3) needs coefficient    */
/* tables that are not available; the closed-form 3.5PN TaylorF2 phase */
/* stands in for it.  Non-spinning coefficients: Buonanno, Iyer,        */
/* Ochsner, Pan & Sathyaprakash 2009 (Eq. 3.18).  Aligned-spin terms:  */
/* spin-orbit at 1.5, 2.5, 3, 3.5PN and spin-spin at 2PN as collected  */
/* in the TaylorF2 appendix of Khan et al. 2016.  Pinned in            */
/* tests/test_oracle_waveform.py: the 0PN closed form; every           */
/* non-spinning coefficient through 3.5PN by the stationary-phase      */
/* relation to the TaylorT2 time to coalescence; the spin terms at     */
/* leading order in eta by the test-mass limit (Kerr circular-orbit    */
/* energy and test-mass flux); exchange symmetry; the 1.5PN and 2PN    */
/* spin identities (beta, sigma) at every eta.  The eta-dependent      */
/* parts of the 2.5, 3 and 3.5PN spin-orbit coefficients are parity    */
/* unpinned (no independent source for them is available here).       */
/* ------------------------------------------------------------------ */

/* phi[j], j = 0..7, multiplying v^j inside 3/(128 eta v^5) * sum_j phi_j v^j.
 * x = sqrt(1 - 4 eta) = (m1 - m2)/M.  Ms = total mass in seconds.  The
 * log terms depend on f. */
void or_pn_coeffs(double eta, double x, double chis, double chia, double Ms, double f,
                  double *phi)
{
    const double pi = OR_PI;
    double eta2 = eta * eta, eta3 = eta2 * eta;
    double lnpmf = log(pi * Ms * f);
    phi[0] = 1.0;
    phi[1] = 0.0;
    phi[2] = 3715.0 / 756.0 + 55.0 * eta / 9.0;
    phi[3] = -16.0 * pi + (113.0 / 3.0) * x * chia + (113.0 / 3.0 - 76.0 * eta / 3.0) * chis;
    phi[4] = 15293365.0 / 508032.0 + 27145.0 * eta / 504.0 + 3085.0 * eta2 / 72.0
             + (-405.0 / 8.0 + 200.0 * eta) * chia * chia
             - (405.0 / 4.0) * x * chia * chis
             + (-405.0 / 8.0 + 5.0 * eta / 2.0) * chis * chis;
    phi[5] = (1.0 + lnpmf)
             * (pi * (38645.0 / 756.0 - 65.0 * eta / 9.0)
                + x * (-732985.0 / 2268.0 - 140.0 * eta / 9.0) * chia
                + (-732985.0 / 2268.0 + 24260.0 * eta / 81.0 + 340.0 * eta2 / 9.0) * chis);
    phi[6] = 11583231236531.0 / 4694215680.0 - 6848.0 * OR_EULER_GAMMA / 21.0
             - 640.0 * pi * pi / 3.0
             + (-15737765635.0 / 3048192.0 + 2255.0 * pi * pi / 12.0) * eta
             + 76055.0 * eta2 / 1728.0 - 127825.0 * eta3 / 1296.0
             - (6848.0 / 63.0) * log(64.0 * pi * Ms * f)
             + pi * ((2270.0 / 3.0) * x * chia + (2270.0 / 3.0 - 520.0 * eta) * chis);
    phi[7] = pi * (77096675.0 / 254016.0 + 378515.0 * eta / 1512.0 - 74045.0 * eta2 / 756.0)
             + x * (-25150083775.0 / 3048192.0 + 26804935.0 * eta / 6048.0 - 1985.0 * eta2 / 48.0)
                   * chia
             + (-25150083775.0 / 3048192.0 + 10566655595.0 * eta / 762048.0
                - 1042165.0 * eta2 / 3024.0 + 5345.0 * eta3 / 36.0) * chis;
}

/* Psi(f) = 2 pi f t_c - 2 phi_c - pi/4 + 3/(128 eta v^5) sum_j phi_j v^j,
 * v = (pi M f)^(1/3).  No cut-off at the last stable orbit: every bin of the
 * grid is evaluated. */
double or_phase(const double *th, double f)
{
    double Mc = th[0], q = th[1];
    double eta = q / ((1.0 + q) * (1.0 + q));
    double Ms = Mc * pow(eta, -0.6) * or_tsun();
    double x = (1.0 - q) / (1.0 + q);
    double chis = 0.5 * (th[2] + th[3]), chia = 0.5 * (th[2] - th[3]);
    double phi[8];
    or_pn_coeffs(eta, x, chis, chia, Ms, f, phi);
    double v = cbrt(OR_PI * Ms * f);
    double sum = 0.0, vj = 1.0;
    for (int j = 0; j < 8; ++j) {
        sum += phi[j] * vj;
        vj *= v;
    }
    double v5 = v * v * v * v * v;
    return 2.0 * OR_PI * f * th[10] - 2.0 * th[9] - 0.25 * OR_PI + 3.0 / (128.0 * eta * v5) * sum;
}

/* Newtonian amplitude factor A, so that |h~(f)| = A f^(-7/6) times the
 * inclination factor:  A = sqrt(5/24) pi^(-2/3) (G Mc/c^3)^(5/6) c / dL
 * (leading-order stationary-phase amplitude, e.g. Cutler & Flanagan 1994). */
double or_amplitude(const double *th)
{
    double mcs = th[0] * or_tsun();
    return sqrt(5.0 / 24.0) * pow(OR_PI, -2.0 / 3.0) * pow(mcs, 5.0 / 6.0) * OR_C_SI
           / (th[4] * OR_MPC_SI);
}

/* ------------------------------------------------------------------ */
/* Detector response (standard tensor construction; the paper names    */
/* the three-detector network but prints no formulas).  Pinned by the  */
/* antenna identities in tests/test_oracle_detector.py.                */
/* ------------------------------------------------------------------ */

/* Direction to the source and polarisation basis vectors X, Y. */
static void or_basis(double ra, double dec, double psi, double gmst, double *n, double *X,
                     double *Y)
{
    double phi = ra - gmst;
    double a[3] = {sin(phi), -cos(phi), 0.0};
    double b[3] = {-cos(phi) * sin(dec), -sin(phi) * sin(dec), cos(dec)};
    n[0] = cos(dec) * cos(phi);
    n[1] = cos(dec) * sin(phi);
    n[2] = sin(dec);
    for (int i = 0; i < 3; ++i) {
        X[i] = cos(psi) * a[i] + sin(psi) * b[i];
        Y[i] = -sin(psi) * a[i] + cos(psi) * b[i];
    }
}

/* F+ = D : (X X^T - Y Y^T),  Fx = D : (X Y^T + Y X^T). */
void or_antenna(const double *D, double ra, double dec, double psi, double gmst, double *Fp,
                double *Fx)
{
    double n[3], X[3], Y[3];
    or_basis(ra, dec, psi, gmst, n, X, Y);
    double fp = 0.0, fx = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            fp += D[3 * i + j] * (X[i] * X[j] - Y[i] * Y[j]);
            fx += D[3 * i + j] * (X[i] * Y[j] + Y[i] * X[j]);
        }
    *Fp = fp;
    *Fx = fx;
}

/* Arrival-time offset relative to the geocentre: dt = -(r . n) / c. */
double or_time_delay(const double *r, double ra, double dec, double gmst)
{
    double n[3], X[3], Y[3];
    or_basis(ra, dec, 0.0, gmst, n, X, Y);
    return -(r[0] * n[0] + r[1] * n[1] + r[2] * n[2]) / OR_C_SI;
}

/* Per-detector response (F+, Fx, dt) for detector d. */
static void or_response(const or_event *ev, const double *th, int d, double *Fp, double *Fx,
                        double *dt)
{
    if (ev->fixed_antenna) {
        *Fp = ev->fixed_antenna[2 * d];
        *Fx = ev->fixed_antenna[2 * d + 1];
        *dt = 0.0;
        return;
    }
    or_antenna(ev->det_tensor + 9 * d, th[6], th[7], th[8], ev->gmst, Fp, Fx);
    *dt = or_time_delay(ev->det_loc + 3 * d, th[6], th[7], ev->gmst);
}

/* Detector-frame strain at one frequency:
 *   h+ = A f^(-7/6) (1 + cos^2 i)/2 e^{-i Psi},  hx = -i A f^(-7/6) cos i e^{-i Psi},
 *   h_d = (F+ h+ + Fx hx) e^{-2 pi i f dt}.
 * Fourier convention h~(f) = int h(t) e^{-2 pi i f t} dt. */
static void or_strain(const double *th, double A, double Fp, double Fx, double dt, double f,
                      double *re, double *im)
{
    double ci = cos(th[5]);
    double amp = A * pow(f, -7.0 / 6.0);
    double psi = or_phase(th, f);
    double c = cos(psi), s = sin(psi);
    /* e^{-i Psi} = c - i s */
    double hp_re = amp * 0.5 * (1.0 + ci * ci) * c;
    double hp_im = -amp * 0.5 * (1.0 + ci * ci) * s;
    /* hx = -i amp ci (c - i s) = -amp ci s - i amp ci c */
    double hx_re = -amp * ci * s;
    double hx_im = -amp * ci * c;
    double r_re = Fp * hp_re + Fx * hx_re;
    double r_im = Fp * hp_im + Fx * hx_im;
    double ang = 2.0 * OR_PI * f * dt;
    double cr = cos(ang), sr = -sin(ang); /* e^{-i ang} */
    *re = r_re * cr - r_im * sr;
    *im = r_re * sr + r_im * cr;
}

/* Fill h[d][k][2] with the detector strain for physical parameters th. */
void or_waveform(const or_event *ev, const double *th, double *h)
{
    double A = or_amplitude(th);
    for (int d = 0; d < ev->n_det; ++d) {
        double Fp, Fx, dt;
        or_response(ev, th, d, &Fp, &Fx, &dt);
        for (int k = 0; k < ev->n_bins; ++k) {
            double f = ev->f_lo + k * ev->df;
            double *o = h + 2 * ((size_t)d * ev->n_bins + k);
            or_strain(th, A, Fp, Fx, dt, f, &o[0], &o[1]);
        }
    }
}

/* A physical parameter vector the likelihood can evaluate. */
static int or_theta_valid(const double *th)
{
    for (int i = 0; i < OR_NPAR; ++i)
        if (!isfinite(th[i])) return 0;
    if (!(th[1] > 0.0 && th[1] <= 1.0)) return 0;
    if (!(th[0] > 0.0)) return 0;
    if (!(th[4] > 0.0)) return 0;
    return 1;
}

/* Whittle log-likelihood ratio against the noise-only model (use_ratio,
 * Sec. 4.1.1):  log Lambda = sum_d [ <d|h> - <h|h>/2 ],
 * <a|b> = 4 df Re sum_k conj(a_k) b_k / S_d(f_k).
 * The strain is computed bin by bin from the waveform; no closed form for
 * <h|h> and no precomputed weights are used.  Returns -inf for a parameter
 * vector outside the physical domain. */
double or_loglike_theta(const or_event *ev, const double *th)
{
    if (!or_theta_valid(th)) return -INFINITY;
    double A = or_amplitude(th);
    double total = 0.0;
    for (int d = 0; d < ev->n_det; ++d) {
        double Fp, Fx, dt;
        or_response(ev, th, d, &Fp, &Fx, &dt);
        double dh = 0.0, hh = 0.0;
        for (int k = 0; k < ev->n_bins; ++k) {
            double f = ev->f_lo + k * ev->df;
            double hr, hi;
            or_strain(th, A, Fp, Fx, dt, f, &hr, &hi);
            const double *dd = ev->data + 2 * ((size_t)d * ev->n_bins + k);
            double S = ev->psd[(size_t)d * ev->n_bins + k];
            dh += (dd[0] * hr + dd[1] * hi) / S;   /* Re(conj(d) h) */
            hh += (hr * hr + hi * hi) / S;
        }
        total += 4.0 * ev->df * dh - 0.5 * 4.0 * ev->df * hh;
    }
    return total;
}

/* ------------------------------------------------------------------ */
/* Heterodyned (relative-binning) likelihood.  The paper names           */
/* heterodyning as the way to cut the per-call cost (Sec. 3.3, Sec. 5,   */
/* appendix on likelihood-level parallelisation) without fixing a        */
/* scheme; this follows relative binning (Zackay, Dai & Venumadhav 2018) */
/* applied to the data term.  With Phi_d(f) = Psi(f) + 2 pi f dt_d the   */
/* detector phase of theta and Phi0_d that of the fiducial theta0, the   */
/* strain h_d(f) = a_d f^(-7/6) e^{-i Phi_d(f)} is written               */
/*   h_d(f) = a_d f^(-7/6) e^{-i Phi0_d(f)} e^{-i (Phi_d - Phi0_d)(f)}   */
/* and the slowly varying last factor is replaced, inside bin b, by its  */
/* linear interpolation between the nodes f(edges[b]) and                */
/* f(edges[b+1]) (edges[B] = n_bins: the node one grid step past the     */
/* last sample).  <h|h> is kept exact.  Pinned in                         */
/* tests/test_oracle_rb.py: equal to the exact likelihood at theta0, for */
/* one sample per bin, and for theta that differ from theta0 only in    */
/* phase and distance (the ratio is then constant); the error shrinks    */
/* as the bins get finer.                                                 */
/* ------------------------------------------------------------------ */

/* e^{-i (Phi_d(f) - Phi0_d(f))} */
static void or_rb_ratio_phase(const double *th, double dt, const double *th0, double dt0, double f,
                              double *re, double *im)
{
    double dphi = (or_phase(th, f) + 2.0 * OR_PI * f * dt) - (or_phase(th0, f) + 2.0 * OR_PI * f * dt0);
    *re = cos(dphi);
    *im = -sin(dphi);
}

double or_loglike_rb(const or_event *ev, const double *th)
{
    if (!or_theta_valid(th)) return -INFINITY;
    const double *th0 = ev->rb_theta0;
    const int B = ev->rb_bins;
    double A = or_amplitude(th);
    double ci = cos(th[5]);
    double total = 0.0;
    for (int d = 0; d < ev->n_det; ++d) {
        double Fp, Fx, dt, Fp0, Fx0, dt0;
        or_response(ev, th, d, &Fp, &Fx, &dt);
        or_response(ev, th0, d, &Fp0, &Fx0, &dt0);
        (void)Fp0;
        (void)Fx0;
        /* a_d = A [F+ (1 + cos^2 i)/2 - i Fx cos i] */
        double a_re = A * Fp * 0.5 * (1.0 + ci * ci);
        double a_im = -A * Fx * ci;
        double dh = 0.0, hh = 0.0;
        /* exact <h|h> */
        for (int k = 0; k < ev->n_bins; ++k) {
            double f = ev->f_lo + k * ev->df;
            double hr, hi;
            or_strain(th, A, Fp, Fx, dt, f, &hr, &hi);
            hh += (hr * hr + hi * hi) / ev->psd[(size_t)d * ev->n_bins + k];
        }
        /* heterodyned <d|h> */
        for (int b = 0; b < B; ++b) {
            int k0 = ev->rb_edges[b], k1 = ev->rb_edges[b + 1];
            double f0 = ev->f_lo + k0 * ev->df, f1 = ev->f_lo + k1 * ev->df;
            double e0r, e0i, e1r, e1i;
            or_rb_ratio_phase(th, dt, th0, dt0, f0, &e0r, &e0i);
            or_rb_ratio_phase(th, dt, th0, dt0, f1, &e1r, &e1i);
            for (int k = k0; k < k1; ++k) {
                double f = ev->f_lo + k * ev->df;
                double lam = (f - f0) / (f1 - f0);
                double er = e0r + lam * (e1r - e0r), ei = e0i + lam * (e1i - e0i);
                /* fiducial phase factor e^{-i Phi0_d(f)} */
                double p0 = or_phase(th0, f) + 2.0 * OR_PI * f * dt0;
                double cr = cos(p0), cim = -sin(p0);
                double amp = pow(f, -7.0 / 6.0);
                /* h = a amp (cr + i cim)(er + i ei) */
                double ur = cr * er - cim * ei, ui = cr * ei + cim * er;
                double hr = amp * (a_re * ur - a_im * ui), hi = amp * (a_re * ui + a_im * ur);
                const double *dd = ev->data + 2 * ((size_t)d * ev->n_bins + k);
                dh += (dd[0] * hr + dd[1] * hi) / ev->psd[(size_t)d * ev->n_bins + k];
            }
        }
        total += 4.0 * ev->df * dh - 0.5 * 4.0 * ev->df * hh;
    }
    return total;
}

/* Gaussian toy: log L(u) = -sum_j (u_j - 1/2)^2 / (2 sigma^2) on the unit
 * cube (closed-form evidence; pinned in tests/test_oracle_ns.py). */
static double or_loglike_toy(const or_event *ev, const double *u)
{
    double s = 0.0;
    for (int j = 0; j < ev->ndim; ++j) {
        double z = u[j] - 0.5;
        s += z * z;
    }
    return -s / (2.0 * ev->toy_sigma * ev->toy_sigma);
}

/* Log-likelihood of a unit-cube point (prior transform, then likelihood). */
double or_loglike_u(const or_event *ev, const double *u)
{
    if (ev->like_kind == OR_LIKE_GAUSS) return or_loglike_toy(ev, u);
    double th[OR_NPAR];
    or_prior_transform(ev, u, th);
    if (ev->like_kind == OR_LIKE_GW_RB) return or_loglike_rb(ev, th);
    return or_loglike_theta(ev, th);
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw,  */
/* SC'11).  Pinned bitwise against numpy.random.Philox.                */
/* ------------------------------------------------------------------ */
static uint64_t or_mulhi64(uint64_t a, uint64_t b, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *lo = (uint64_t)p;
    return (uint64_t)(p >> 64);
}

void or_philox4x64(const uint64_t *ctr_in, const uint64_t *key_in, uint64_t *out)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t lo0, lo1;
        uint64_t hi0 = or_mulhi64(M0, c0, &lo0);
        uint64_t hi1 = or_mulhi64(M1, c2, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0, 1). */
double or_u01(uint64_t r) { return (double)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Purposes of the fourth counter word: which part of the method a block feeds. */
#define OR_P_WALK_A 0u
#define OR_P_START 1u
#define OR_P_DA2 2u
#define OR_P_WALK_B 6u
#define OR_P_INIT 7u
#define OR_P_HRSS 8u          /* per slice step: V, donors a and b, offset r */
#define OR_P_HRSS_SHRINK 64u  /* + k: the k-th shrinkage draw of a slice step */
#define OR_HRSS_M 8           /* stepping-out budget (interval widths) */
#define OR_HRSS_K 64          /* shrinkage draws before the step gives up */

static void or_draw(uint64_t seed, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t purpose,
                    double *u4)
{
    uint64_t ctr[4] = {c0, c1, c2, purpose}, key[2] = {seed, 0}, r[4];
    or_philox4x64(ctr, key, r);
    for (int i = 0; i < 4; ++i) u4[i] = or_u01(r[i]);
}

static uint64_t or_chain_id(int event, int slot)
{
    return ((uint64_t)(uint32_t)event << 32) | (uint64_t)(uint32_t)slot;
}

/* ------------------------------------------------------------------ */
/* Acceptance walk (Sec. 3.1): differential-evolution proposals in the  */
/* unit cube, strict acceptance L > L*, a fixed number W of steps.      */
/* Exact per-step parity with the GPU walk is the test of this routine. */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n_acc, n_calls, n_oob;
} or_walk_stats;

/* The DE scale mixture (Sec. 3.1 footnote): 1 with probability 1/2, else
 * 2.38/sqrt(2 d) times a Gamma(shape 4, scale 1/4) variate, drawn as the sum
 * of four exponentials of mean 1/4. */
double or_de_gamma(double u_mode, const double *ug, int ndim)
{
    if (u_mode < 0.5) return 1.0;
    double g = 0.0;
    for (int i = 0; i < 4; ++i) g += -0.25 * log(1.0 - ug[i]);
    return 2.38 / sqrt(2.0 * ndim) * g;
}

/* One chain: start at u (logL *L), W steps against the frozen snapshot S
 * (m rows of ndim), threshold Lstar.  u and *L are updated in place. */
void or_walk(const or_event *ev, const double *S, int32_t m, double Lstar, double *u, double *L,
             int32_t W, uint64_t seed, int32_t event, int32_t slot, int64_t batch,
             or_walk_stats *st)
{
    int d = ev->ndim;
    double prop[OR_NPAR];
    uint64_t cid = or_chain_id(event, slot);
    for (int s = 0; s < W; ++s) {
        double A4[4], B4[4];
        or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_WALK_A, A4);
        or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_WALK_B, B4);
        int a = (int)floor(A4[1] * m);
        int b = (int)floor(A4[2] * (m - 1));
        if (b >= a) b += 1;
        double gam = or_de_gamma(A4[0], B4, d);
        int oob = 0;
        for (int j = 0; j < d; ++j) {
            double diff = S[(size_t)a * d + j] - S[(size_t)b * d + j];
            prop[j] = fma(gam, diff, u[j]);
            if (or_is_periodic(d, j)) {
                prop[j] = prop[j] - floor(prop[j]);
            } else if (prop[j] < 0.0 || prop[j] > 1.0) {
                oob = 1;
            }
        }
        if (oob) {
            st->n_oob++;
            continue;
        }
        double Lp = or_loglike_u(ev, prop);
        st->n_calls++;
        if (Lp > Lstar) {
            for (int j = 0; j < d; ++j) u[j] = prop[j];
            *L = Lp;
            st->n_acc++;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Acceptance walk with delayed acceptance through a learned screen.    */
/* The paper names batched machine-learning models as a companion of   */
/* the batched sampler (Sec. 5) without fixing a scheme; this is the   */
/* two-stage delayed-acceptance Metropolis-Hastings step of Christen &  */
/* Fox (2005), "Markov chain Monte Carlo using an approximation", with  */
/* the walk's target (the prior restricted to L > L*) and a strictly    */
/* positive screen density                                              */
/*   pi(x) = floor + (1 - floor) / (1 + exp(-(s(x) - L* + margin)/temp)) */
/* where s(x) is the surrogate's log-likelihood prediction:             */
/*   stage 1: continue with probability min(1, pi(x')/pi(x)), no exact   */
/*            likelihood call otherwise (a saved call);                  */
/*   stage 2: exact L(x'); accept iff L(x') > L* and a second uniform is */
/*            below min(1, pi(x)/pi(x')).                                */
/* The differential-evolution proposal is symmetric given the frozen    */
/* survivors, so the constrained prior stays invariant.  The uniforms    */
/* of a step are words 0 and 1 of its Philox block with purpose 2.      */
/* Pinned: with a constant screen the chain is or_walk's exactly; with  */
/* an arbitrary screen it keeps the uniform distribution on a           */
/* constrained ball (tests/test_oracle_ns.py).                           */
/* ------------------------------------------------------------------ */
double or_mlp_eval1(const double *p, const double *x);

typedef struct {
    const double *params;  /* FP64 network parameters (or_mlp layout), or NULL: s(x) = const_s */
    double in_mean[OR_NPAR], in_sd[OR_NPAR];  /* input standardisation of the sampled coords */
    double mu, sigma;      /* target de-standardisation */
    double top;            /* log-gap target map when finite: s = top - exp(-z) */
    double const_s;        /* prediction when params is NULL */
    double margin, temp, floor;
} or_screen;

typedef struct {
    int64_t n_acc, n_calls, n_oob, n_saved;
    /* smallest distance of any decision of the chain from its threshold:
     * |log U - log(pi ratio)| over the stage-1 and stage-2 screen tests, and
     * |L' - L*| over the exact tests; a second implementation whose screen
     * or likelihood differs by less than these takes the same decisions */
    double min_gap_screen, min_gap_L;
} or_da_stats;

/* Surrogate log-likelihood prediction s(x) of a unit-cube point. */
double or_screen_predict(const or_screen *sc, int ndim, const double *u)
{
    if (!sc->params) return sc->const_s;
    double x[OR_NPAR];
    for (int j = 0; j < OR_NPAR; ++j) x[j] = j < ndim ? (u[j] - sc->in_mean[j]) / sc->in_sd[j] : 0.0;
    double z = sc->mu + sc->sigma * or_mlp_eval1(sc->params, x);
    return isinf(sc->top) ? z : sc->top - exp(-z);
}

/* Screen density pi(x) given the prediction s(x). */
double or_screen_density(const or_screen *sc, double s_hat, double Lstar)
{
    double z = (s_hat - Lstar + sc->margin) / sc->temp;
    return sc->floor + (1.0 - sc->floor) / (1.0 + exp(-z));
}

void or_walk_da(const or_event *ev, const or_screen *sc, const double *S, int32_t m, double Lstar,
                double *u, double *L, int32_t W, uint64_t seed, int32_t event, int32_t slot,
                int64_t batch, or_da_stats *st)
{
    int d = ev->ndim;
    double prop[OR_NPAR];
    uint64_t cid = or_chain_id(event, slot);
    double pi_cur = or_screen_density(sc, or_screen_predict(sc, d, u), Lstar);
    st->min_gap_screen = INFINITY;
    st->min_gap_L = INFINITY;
    for (int s = 0; s < W; ++s) {
        double A4[4], B4[4], D4[4];
        or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_WALK_A, A4);
        or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_WALK_B, B4);
        int a = (int)floor(A4[1] * m);
        int b = (int)floor(A4[2] * (m - 1));
        if (b >= a) b += 1;
        double gam = or_de_gamma(A4[0], B4, d);
        int oob = 0;
        for (int j = 0; j < d; ++j) {
            double diff = S[(size_t)a * d + j] - S[(size_t)b * d + j];
            prop[j] = fma(gam, diff, u[j]);
            if (or_is_periodic(d, j)) {
                prop[j] = prop[j] - floor(prop[j]);
            } else if (prop[j] < 0.0 || prop[j] > 1.0) {
                oob = 1;
            }
        }
        if (oob) {
            st->n_oob++;
            continue;
        }
        or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_DA2, D4);
        double pi_prop = or_screen_density(sc, or_screen_predict(sc, d, prop), Lstar);
        /* stage 1 */
        double r1 = pi_prop / pi_cur;
        double g1 = fabs(log(D4[0]) - log(r1));
        if (g1 < st->min_gap_screen) st->min_gap_screen = g1;
        if (!(D4[0] < (r1 < 1.0 ? r1 : 1.0))) {
            st->n_saved++;
            continue;
        }
        /* stage 2 */
        double Lp = or_loglike_u(ev, prop);
        st->n_calls++;
        double gL = fabs(Lp - Lstar);
        if (gL < st->min_gap_L) st->min_gap_L = gL;
        if (!(Lp > Lstar)) continue;
        double r2 = pi_cur / pi_prop;
        double g2 = fabs(log(D4[1]) - log(r2));
        if (g2 < st->min_gap_screen) st->min_gap_screen = g2;
        if (D4[1] < (r2 < 1.0 ? r2 : 1.0)) {
            for (int j = 0; j < d; ++j) u[j] = prop[j];
            *L = Lp;
            pi_cur = pi_prop;
            st->n_acc++;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Hit-and-run slice sampling (named in the closing section as the     */
/* alternative inner kernel; the slice sampler is Neal 2003, Sec. 4).   */
/* The target is the prior restricted to L > L*, uniform in the cube,  */
/* so the slice along a line is the constrained set itself.  Each step */
/* picks the line through the current point along a differential-      */
/* evolution direction S_a - S_b (frozen survivors), places a unit     */
/* interval at a random offset, steps it out by whole widths while its */
/* ends are inside (budget M split at random between the two sides),   */
/* then draws uniformly on the interval, shrinking it towards the      */
/* current point after every draw outside, until a draw is inside.     */
/* Out-of-cube points (non-periodic coordinates) are outside without a */
/* likelihood call.  parity unpinned against an external slice-sampler */
/* implementation; pinned by stationarity (uniform in a constrained    */
/* ball) and by the evidence of the Gaussian toy.                      */
/* ------------------------------------------------------------------ */

/* Point of the line at parameter t: p = x + t dir, periodic coordinates
 * wrapped.  Returns 1 when p lies in the cube. */
static int or_line_point(const or_event *ev, const double *x, const double *dir, double t,
                         double *p)
{
    int d = ev->ndim, in = 1;
    for (int j = 0; j < d; ++j) {
        double v = fma(t, dir[j], x[j]);
        if (or_is_periodic(d, j))
            v = v - floor(v);
        else if (v < 0.0 || v > 1.0)
            in = 0;
        p[j] = v;
    }
    return in;
}

/* Inside the slice: in the cube and L(p) > L*.  Counts calls and
 * out-of-cube points; the likelihood of p is left in *Lp. */
static int or_slice_inside(const or_event *ev, const double *x, const double *dir, double t,
                           double Lstar, double *p, double *Lp, or_walk_stats *st)
{
    if (!or_line_point(ev, x, dir, t, p)) {
        st->n_oob++;
        return 0;
    }
    *Lp = or_loglike_u(ev, p);
    st->n_calls++;
    return *Lp > Lstar;
}

/* One chain: W slice steps from u (logL *L) against the snapshot S (m rows);
 * u and *L are updated in place; a step that moves counts as accepted. */
void or_hrss(const or_event *ev, const double *S, int32_t m, double Lstar, double *u, double *L,
             int32_t W, uint64_t seed, int32_t event, int32_t slot, int64_t batch,
             or_walk_stats *st)
{
    int d = ev->ndim;
    double dir[OR_NPAR], p[OR_NPAR], Lp = 0.0;
    uint64_t cid = or_chain_id(event, slot);
    for (int s = 0; s < W; ++s) {
        double A4[4];
        or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_HRSS, A4);
        int a = (int)floor(A4[1] * m);
        int b = (int)floor(A4[2] * (m - 1));
        if (b >= a) b += 1;
        for (int j = 0; j < d; ++j) dir[j] = S[(size_t)a * d + j] - S[(size_t)b * d + j];
        double lo = -A4[3], hi = 1.0 - A4[3];
        int J = (int)floor(OR_HRSS_M * A4[0]);
        int K = OR_HRSS_M - 1 - J;
        while (J > 0 && or_slice_inside(ev, u, dir, lo, Lstar, p, &Lp, st)) {
            lo -= 1.0;
            J--;
        }
        while (K > 0 && or_slice_inside(ev, u, dir, hi, Lstar, p, &Lp, st)) {
            hi += 1.0;
            K--;
        }
        for (int k = 0; k < OR_HRSS_K; ++k) {
            double B4[4];
            or_draw(seed, (uint64_t)s, cid, (uint64_t)batch, OR_P_HRSS_SHRINK + (uint64_t)k, B4);
            double t = lo + B4[0] * (hi - lo);
            if (or_slice_inside(ev, u, dir, t, Lstar, p, &Lp, st)) {
                for (int j = 0; j < d; ++j) u[j] = p[j];
                *L = Lp;
                st->n_acc++;
                break;
            }
            if (t < 0.0)
                lo = t;
            else
                hi = t;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Batched nested sampling (Sec. 2.2.3, 3.2) with per-deletion volume   */
/* accounting and batch-level walk-length tuning.                       */
/* ------------------------------------------------------------------ */
typedef struct {
    const or_event *ev;
    int32_t event_id;
    int32_t n_live, naccept, maxmcmc;
    double delay;
    uint64_t seed;
    int64_t batch;
    int32_t W;
    int32_t ndim;
    double *live_u;   /* [n_live][ndim] */
    double *live_L;   /* [n_live] */
    /* dead points, appended in deletion order */
    int64_t n_dead, cap_dead;
    double *dead_u, *dead_L, *dead_logw, *dead_nlive;
    double logX;      /* log of the remaining prior volume */
    double logZ;      /* log evidence accumulated from dead points */
    double sumH;      /* sum_i p_i log L_i, with p_i = w_i L_i / Z (running) */
    double sum_inv_n, sum_inv_n2;  /* sum over dead points of 1/n_i and 1/n_i^2 */
    int64_t n_calls, n_acc_total, n_oob_total, steps_total;
    /* statistics of the last batch */
    int64_t last_acc, last_calls, last_oob;
    double last_Lstar;
    int32_t last_W, last_k;
    int32_t inner;    /* 0: acceptance walk, 1: hit-and-run slice sampling */
    int32_t capped;   /* consecutive batches whose tuned walk length is maxmcmc */
    const or_screen *screen;  /* delayed acceptance through a screen, or NULL */
    int64_t n_saved;          /* stage-1 rejections (exact calls not made) */
    double *last_gap_s, *last_gap_L;  /* per chain of the last batch (or_da_stats) */
    int64_t *last_chain;              /* per chain of the last batch: accepts, calls, out-of-cube */
    int32_t last_gap_n;
} or_ns;

static double or_logaddexp(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

/* Draw the initial live set from the prior (Sec. 2.2.1): coordinate j of
 * point i uses word j%4 of the block with counter (j/4, chain id(i), 0, INIT). */
or_ns *or_ns_create(const or_event *ev, int32_t event_id, int32_t n_live, int32_t naccept,
                    int32_t maxmcmc, int32_t walk0, double delay, uint64_t seed)
{
    or_ns *ns = (or_ns *)calloc(1, sizeof(or_ns));
    ns->ev = ev;
    ns->event_id = event_id;
    ns->n_live = n_live;
    ns->naccept = naccept;
    ns->maxmcmc = maxmcmc;
    ns->delay = delay;
    ns->seed = seed;
    ns->W = walk0;
    ns->ndim = ev->ndim;
    ns->live_u = (double *)malloc(sizeof(double) * (size_t)n_live * ev->ndim);
    ns->live_L = (double *)malloc(sizeof(double) * (size_t)n_live);
    ns->cap_dead = 0;
    ns->logX = 0.0;
    ns->logZ = -INFINITY;
    ns->sumH = 0.0;
    int d = ev->ndim;
    for (int i = 0; i < n_live; ++i) {
        uint64_t cid = or_chain_id(event_id, i);
        for (int j = 0; j < d; ++j) {
            double u4[4];
            or_draw(seed, (uint64_t)(j / 4), cid, 0, OR_P_INIT, u4);
            ns->live_u[(size_t)i * d + j] = u4[j % 4];
        }
    }
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < n_live; ++i)
        ns->live_L[i] = or_loglike_u(ev, ns->live_u + (size_t)i * d);
    return ns;
}

/* Inner kernel of the chains: 0 acceptance walk (default), 1 hit-and-run
 * slice sampling; the tuned length then counts slice steps. */
int or_ns_set_inner(or_ns *ns, int32_t inner)
{
    if (inner != 0 && inner != 1) return -1;
    ns->inner = inner;
    return 0;
}

/* Delayed acceptance through a screen for the walks of later batches
 * (NULL: the plain walk).  The screen must outlive its use. */
void or_ns_set_screen(or_ns *ns, const or_screen *sc) { ns->screen = sc; }

void or_ns_free(or_ns *ns)
{
    if (!ns) return;
    free(ns->last_gap_s); free(ns->last_gap_L); free(ns->last_chain);
    free(ns->live_u); free(ns->live_L);
    free(ns->dead_u); free(ns->dead_L); free(ns->dead_logw); free(ns->dead_nlive);
    free(ns);
}

/* Replace the live set (tests use this to start both implementations from
 * the same state). */
void or_ns_set_live(or_ns *ns, const double *u, const double *L)
{
    memcpy(ns->live_u, u, sizeof(double) * (size_t)ns->n_live * ns->ndim);
    memcpy(ns->live_L, L, sizeof(double) * (size_t)ns->n_live);
}

/* Ordering of live points: ascending logL, ties by position (stable). */
static const double *or_sort_keys;
static int or_cmp_rows(const void *pa, const void *pb)
{
    int a = *(const int *)pa, b = *(const int *)pb;
    double la = or_sort_keys[a], lb = or_sort_keys[b];
    if (la < lb) return -1;
    if (la > lb) return 1;
    return (a > b) - (a < b);
}

static void or_dead_push(or_ns *ns, const double *u, double L, double logw, double nl)
{
    int d = ns->ndim;
    if (ns->n_dead == ns->cap_dead) {
        int64_t cap = ns->cap_dead ? 2 * ns->cap_dead : 1024;
        ns->dead_u = (double *)realloc(ns->dead_u, sizeof(double) * (size_t)cap * d);
        ns->dead_L = (double *)realloc(ns->dead_L, sizeof(double) * (size_t)cap);
        ns->dead_logw = (double *)realloc(ns->dead_logw, sizeof(double) * (size_t)cap);
        ns->dead_nlive = (double *)realloc(ns->dead_nlive, sizeof(double) * (size_t)cap);
        ns->cap_dead = cap;
    }
    memcpy(ns->dead_u + (size_t)ns->n_dead * d, u, sizeof(double) * d);
    ns->dead_L[ns->n_dead] = L;
    ns->dead_logw[ns->n_dead] = logw;
    ns->dead_nlive[ns->n_dead] = nl;
    ns->n_dead++;
}

/* Walk-length update after a batch (Sec. 3.2): target naccept accepted
 * steps from the batch-mean acceptance rate, smoothed with the sequential
 * delay D applied once per deleted point, i.e. a memory factor
 * r = (D/(D+1))^k, computed by repeated multiplication. */
int32_t or_tune_walk(int32_t W, int64_t sum_acc, int32_t k, double delay, int32_t naccept,
                     int32_t maxmcmc)
{
    double rate = (double)sum_acc / ((double)k * (double)W);
    double floor_rate = 1.0 / ((double)k * (double)W);
    double target = (double)naccept / (rate > floor_rate ? rate : floor_rate);
    double step = delay / (delay + 1.0);
    double r = 1.0;
    for (int i = 0; i < k; ++i) r = r * step;
    double next = round(target + ((double)W - target) * r);
    if (next < 1.0) next = 1.0;
    if (next > (double)maxmcmc) next = (double)maxmcmc;
    return (int32_t)next;
}

/* One batched iteration: delete the k lowest (L* = the largest deleted
 * logL), start each of k chains from a uniformly chosen survivor with
 * logL > L*, walk W steps against the frozen survivor snapshot, account
 * the k deletions with live counts n, n-1, ..., n-k+1, refill, retune.
 * walk <= 0 uses the tuned walk length.  Returns 0, or -1 on bad k. */
int or_ns_step(or_ns *ns, int32_t k, int32_t walk)
{
    int n = ns->n_live, d = ns->ndim;
    if (k < 1 || k >= n) return -1;
    int W = walk > 0 ? walk : ns->W;
    int *ord = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    or_sort_keys = ns->live_L;
    qsort(ord, n, sizeof(int), or_cmp_rows);
    double Lstar = ns->live_L[ord[k - 1]];

    /* survivor snapshot: rows after the deleted block with logL > L*, in
     * sorted order */
    int m = 0;
    double *S = (double *)malloc(sizeof(double) * (size_t)n * d);
    double *SL = (double *)malloc(sizeof(double) * (size_t)n);
    for (int r = k; r < n; ++r) {
        int i = ord[r];
        if (ns->live_L[i] > Lstar) {
            memcpy(S + (size_t)m * d, ns->live_u + (size_t)i * d, sizeof(double) * d);
            SL[m] = ns->live_L[i];
            m++;
        }
    }
    if (m < 2) {
        free(ord); free(S); free(SL);
        return -2;
    }

    /* chains */
    double *cu = (double *)malloc(sizeof(double) * (size_t)k * d);
    double *cL = (double *)malloc(sizeof(double) * (size_t)k);
    or_walk_stats *cst = (or_walk_stats *)calloc((size_t)k, sizeof(or_walk_stats));
    or_da_stats *dst = (or_da_stats *)calloc((size_t)k, sizeof(or_da_stats));
#pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < k; ++c) {
        double u4[4];
        or_draw(ns->seed, 0, or_chain_id(ns->event_id, c), (uint64_t)ns->batch, OR_P_START, u4);
        int j = (int)floor(u4[0] * m);
        memcpy(cu + (size_t)c * d, S + (size_t)j * d, sizeof(double) * d);
        cL[c] = SL[j];
        if (ns->inner == 1) {
            or_hrss(ns->ev, S, m, Lstar, cu + (size_t)c * d, &cL[c], W, ns->seed, ns->event_id, c,
                    ns->batch, &cst[c]);
        } else if (ns->screen) {
            or_walk_da(ns->ev, ns->screen, S, m, Lstar, cu + (size_t)c * d, &cL[c], W, ns->seed,
                       ns->event_id, c, ns->batch, &dst[c]);
            cst[c].n_acc = dst[c].n_acc;
            cst[c].n_calls = dst[c].n_calls;
            cst[c].n_oob = dst[c].n_oob;
        } else {
            or_walk(ns->ev, S, m, Lstar, cu + (size_t)c * d, &cL[c], W, ns->seed, ns->event_id, c,
                    ns->batch, &cst[c]);
        }
    }
    ns->last_gap_s = (double *)realloc(ns->last_gap_s, sizeof(double) * (size_t)k);
    ns->last_gap_L = (double *)realloc(ns->last_gap_L, sizeof(double) * (size_t)k);
    ns->last_chain = (int64_t *)realloc(ns->last_chain, sizeof(int64_t) * 3 * (size_t)k);
    ns->last_gap_n = k;
    for (int c = 0; c < k; ++c) {
        ns->last_chain[3 * c] = cst[c].n_acc;
        ns->last_chain[3 * c + 1] = cst[c].n_calls;
        ns->last_chain[3 * c + 2] = cst[c].n_oob;
        int da = ns->inner != 1 && ns->screen;
        ns->last_gap_s[c] = da ? dst[c].min_gap_screen : INFINITY;
        ns->last_gap_L[c] = da ? dst[c].min_gap_L : INFINITY;
        if (da) ns->n_saved += dst[c].n_saved;
    }
    free(dst);

    /* dead bookkeeping, deleted rows in ascending order */
    for (int i = 0; i < k; ++i) {
        int row = ord[i];
        double nl = (double)(n - i);
        double logX_new = ns->logX - 1.0 / nl;
        double logw = ns->logX + log(-expm1(-1.0 / nl)); /* log(X_prev - X_new) */
        double L = ns->live_L[row];
        double t = L + logw;
        double logZ_new = or_logaddexp(ns->logZ, t);
        /* running information: sumH = sum_i p_i L_i with p_i = e^{t_i - logZ} */
        if (ns->logZ == -INFINITY)
            ns->sumH = L;
        else
            ns->sumH = ns->sumH * exp(ns->logZ - logZ_new) + exp(t - logZ_new) * L;
        ns->logZ = logZ_new;
        ns->logX = logX_new;
        ns->sum_inv_n += 1.0 / nl;
        ns->sum_inv_n2 += 1.0 / (nl * nl);
        or_dead_push(ns, ns->live_u + (size_t)row * d, L, logw, nl);
    }

    /* new live set: survivors in sorted order, then the chain outputs */
    double *nu = (double *)malloc(sizeof(double) * (size_t)n * d);
    double *nL = (double *)malloc(sizeof(double) * (size_t)n);
    for (int r = k; r < n; ++r) {
        int i = ord[r];
        memcpy(nu + (size_t)(r - k) * d, ns->live_u + (size_t)i * d, sizeof(double) * d);
        nL[r - k] = ns->live_L[i];
    }
    int64_t sacc = 0, scalls = 0, soob = 0;
    for (int c = 0; c < k; ++c) {
        memcpy(nu + (size_t)(n - k + c) * d, cu + (size_t)c * d, sizeof(double) * d);
        nL[n - k + c] = cL[c];
        sacc += cst[c].n_acc;
        scalls += cst[c].n_calls;
        soob += cst[c].n_oob;
    }
    memcpy(ns->live_u, nu, sizeof(double) * (size_t)n * d);
    memcpy(ns->live_L, nL, sizeof(double) * (size_t)n);

    ns->last_acc = sacc;
    ns->last_calls = scalls;
    ns->last_oob = soob;
    ns->last_Lstar = Lstar;
    ns->last_W = W;
    ns->last_k = k;
    ns->n_calls += scalls;
    ns->n_acc_total += sacc;
    ns->n_oob_total += soob;
    ns->steps_total += (int64_t)k * W;
    ns->W = or_tune_walk(W, sacc, k, ns->delay, ns->naccept, ns->maxmcmc);
    ns->capped = ns->W >= ns->maxmcmc ? ns->capped + 1 : 0;
    ns->batch++;

    free(ord); free(S); free(SL); free(cu); free(cL); free(cst); free(nu); free(nL);
    return 0;
}

/* Evidence summary (Sec. 3.2.1, and the termination rules of Sec. 4.1.1
 * and 4.2):
 *   out[0] logZ (dead points only)
 *   out[1] logZ_total = logaddexp(logZ, logX + logmeanexp(live logL))
 *   out[2] dlogZ = logaddexp(logZ, logX + max live logL) - logZ
 *   out[3] log fraction remaining = logX + logmeanexp(live logL) - logZ
 *   out[4] information H = sum p_i log L_i - logZ
 *   out[5] logX
 *   out[6] standard error of logZ, sqrt(H sum(1/n_i^2) / sum(1/n_i)).
 * The error follows Skilling's argument (Skilling 2006): the posterior
 * bulk spans about H in log X; a deletion at live count n_i shrinks log X by
 * 1/n_i on average with variance 1/n_i^2, so about H / mean(1/n_i)
 * deletions cross the bulk, each adding mean(1/n_i^2) to the variance of
 * log Z.  With a constant live count this is sqrt(H / n); the batched
 * saw-tooth of live counts (Sec. 3.2.1) makes it larger.  Pinned against
 * the replicate spread of logz_spread on the Gaussian toy. */
void or_ns_evidence(const or_ns *ns, double *out)
{
    int n = ns->n_live;
    double mx = -INFINITY;
    for (int i = 0; i < n; ++i)
        if (ns->live_L[i] > mx) mx = ns->live_L[i];
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += exp(ns->live_L[i] - mx);
    double lme = mx + log(s / n);
    out[0] = ns->logZ;
    out[1] = or_logaddexp(ns->logZ, ns->logX + lme);
    out[2] = or_logaddexp(ns->logZ, ns->logX + mx) - ns->logZ;
    out[3] = ns->logX + lme - ns->logZ;
    out[4] = ns->sumH - ns->logZ;
    out[5] = ns->logX;
    double H = out[4] > 0.0 ? out[4] : 0.0;
    out[6] = ns->sum_inv_n > 0.0 ? sqrt(H * ns->sum_inv_n2 / ns->sum_inv_n) : 0.0;
}

/* Accessors for the ctypes wrapper. */
int64_t or_ns_n_dead(const or_ns *ns) { return ns->n_dead; }
int32_t or_ns_W(const or_ns *ns) { return ns->W; }
int64_t or_ns_batch(const or_ns *ns) { return ns->batch; }
void or_ns_set_W(or_ns *ns, int32_t W) { ns->W = W; }
void or_ns_get_live(const or_ns *ns, double *u, double *L)
{
    memcpy(u, ns->live_u, sizeof(double) * (size_t)ns->n_live * ns->ndim);
    memcpy(L, ns->live_L, sizeof(double) * (size_t)ns->n_live);
}
void or_ns_get_dead(const or_ns *ns, double *u, double *L, double *logw, double *nlive)
{
    int64_t n = ns->n_dead;
    memcpy(u, ns->dead_u, sizeof(double) * (size_t)n * ns->ndim);
    memcpy(L, ns->dead_L, sizeof(double) * (size_t)n);
    memcpy(logw, ns->dead_logw, sizeof(double) * (size_t)n);
    memcpy(nlive, ns->dead_nlive, sizeof(double) * (size_t)n);
}
/* stats: [calls, accepts, oob, steps, last_acc, last_calls, last_oob, last_W, last_k, capped] */
void or_ns_stats(const or_ns *ns, int64_t *out)
{
    out[0] = ns->n_calls; out[1] = ns->n_acc_total; out[2] = ns->n_oob_total;
    out[3] = ns->steps_total; out[4] = ns->last_acc; out[5] = ns->last_calls;
    out[6] = ns->last_oob; out[7] = ns->last_W; out[8] = ns->last_k; out[9] = ns->capped;
}
double or_ns_last_Lstar(const or_ns *ns) { return ns->last_Lstar; }
int64_t or_ns_n_saved(const or_ns *ns) { return ns->n_saved; }
/* Decision gaps (or_da_stats) of each chain of the last batch; returns the
 * number of chains written (at most cap). */
int32_t or_ns_last_gaps(const or_ns *ns, double *gap_s, double *gap_L, int32_t cap)
{
    int32_t n = ns->last_gap_n < cap ? ns->last_gap_n : cap;
    for (int32_t c = 0; c < n; ++c) {
        gap_s[c] = ns->last_gap_s[c];
        gap_L[c] = ns->last_gap_L[c];
    }
    return n;
}

/* Counts (accepts, calls, out-of-cube steps) of each chain of the last
 * batch, three per chain; returns the number of chains written (at most cap). */
int32_t or_ns_last_chains(const or_ns *ns, int64_t *out, int32_t cap)
{
    int32_t n = ns->last_gap_n < cap ? ns->last_gap_n : cap;
    for (int32_t i = 0; i < 3 * n; ++i) out[i] = ns->last_chain[i];
    return n;
}

/* Batched likelihood over n unit-cube points (timing and parity helper). */
void or_loglike_batch_u(const or_event *ev, const double *u, int64_t n, double *out)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i) out[i] = or_loglike_u(ev, u + (size_t)i * ev->ndim);
}

/* Batched likelihood over n physical parameter vectors [n][11]. */
void or_loglike_batch_theta(const or_event *ev, const double *th, int64_t n, double *out)
{
#pragma omp parallel for schedule(dynamic)
    for (int64_t i = 0; i < n; ++i)
        out[i] = ev->like_kind == OR_LIKE_GW_RB ? or_loglike_rb(ev, th + (size_t)i * OR_NPAR)
                                                : or_loglike_theta(ev, th + (size_t)i * OR_NPAR);
}

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
