// Device code of the MI355X acceptance-walk nested sampler: counter-based
// random numbers, prior transform, aligned-spin TaylorF2 phase in basis form,
// detector response and the Whittle inner-product accumulation over bins.
//
// Everything here is written for gfx950 (CDNA4, wave64).  It shares nothing
// with the CPU oracle; the two agree only through the paper's definitions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsmi {

constexpr int NPAR = 11;
constexpr int MAXDET = 3;
constexpr int WAVE = 64;
// Byte layout of one 64-bin table row (see DevEvent).
constexpr int ROW_T = 0, ROW_S = 512, ROW_L = 1024, ROW_W = 1536;
constexpr int ROW_W64 = 1024, ROW_W32 = 512;  // bytes per detector
constexpr int ROW64 = ROW_W + MAXDET * ROW_W64;  // 4608
constexpr int ROW32 = ROW_W + MAXDET * ROW_W32;  // 3072
// Relative-binning table: row r, slot l holds node b = 63 r + l (slot 63
// repeats the first node of the next row) and, for l < 63, bin b (from node
// b to node b + 1).  Per slot: node frequency f, basis f^(-1/3), f^(1/3),
// ln f, the fiducial detector phases r0_d (turns), 1 / (f_{b+1} - f_b), and
// the bin's fiducial sums G0_d = sum_k w_k e^{-2 pi i r0_d(f_k)} and
// G1_d = sum_k w_k e^{-2 pi i r0_d(f_k)} (f_k - f_b) (complex).
constexpr int RB_BINS_PER_ROW = WAVE - 1;
constexpr int RB_F = 0, RB_T = 512, RB_S = 1024, RB_L = 1536, RB_R0 = 2048, RB_IW = 3584;
constexpr int RB_G0 = 4096, RB_G1 = 7168, RB_ROW = 10240;  // G rows: 1024 B per detector
constexpr int RB_MAX_BINS = 4095;

constexpr double PI = 3.141592653589793238462643383279502884;
constexpr double TWO_PI = 6.283185307179586476925286766559005768;
constexpr double INV_TWO_PI = 0.159154943091895335768883763372514362;
constexpr double GM_SUN = 1.32712440018e20;      // m^3 s^-2
constexpr double C_SI = 299792458.0;             // m / s
constexpr double MPC_SI = 3.0856775814913673e22; // m
constexpr double EULER_GAMMA = 0.5772156649015329;

// ---------------------------------------------------------------------------
// Event description as the kernels see it (device memory, one per event).
// ---------------------------------------------------------------------------
struct DevEvent {
    int32_t n_bins, n_det, ndim, likelihood;
    int32_t fixed_antenna, n_live, k;
    int32_t n_pad;  // bins rounded up to a multiple of 64: table row length
    double f_lo, df;
    // Bin tables in rows of 64 bins (bin k = 64 r + l sits in row r, slot l),
    // n_pad / 64 rows.  Per row: the phase basis f^(-1/3), f^(1/3), ln f
    // (FP64, 64 each; the padding continues the frequency grid), then for
    // each of MAXDET detectors the whitened, amplitude-weighted data
    // w_d = 4 df conj(d) f^(-7/6) / S as (re, im) pairs, zero for k >= n_bins
    // and d >= n_det.  rows64 holds FP64 weights, rows32 the same weights
    // scaled by wscale in FP32 (mixed precision).
    const char *rows64, *rows32;
    double wscale;
    double K[MAXDET];        // 4 df sum_k f^(-7/3) / S_d(f_k)
    double D[MAXDET][9];     // symmetrised response tensors
    double loc[MAXDET][3];   // detector positions [m]
    double Fp[MAXDET], Fx[MAXDET];  // fixed antenna (zero delay)
    double lo[NPAR], hi[NPAR], fixed[NPAR];
    // prior-edge trigonometry for the sine (theta_JN) and cosine (dec) priors
    double cos_lo5, cos_hi5, sin_lo7, sin_hi7;
    // trigonometry of fixed (not sampled) angles
    double fixed_cosi, fixed_sindec, fixed_cosdec;
    double gmst, toy_sigma;
    // Relative binning (likelihood 2): rb_bins bins between rb_bins + 1
    // nodes, tabulated in rows of 64 node slots (see RB_* below).
    const char *rb_rows;
    int32_t rb_bins, rb_nrows;
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// ---------------------------------------------------------------------------
struct U4 {
    uint64_t x[4];
};

__device__ __forceinline__ U4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                         uint64_t k0, uint64_t k1)
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    U4 r;
    r.x[0] = c0;
    r.x[1] = c1;
    r.x[2] = c2;
    r.x[3] = c3;
    return r;
}

// 53-bit uniform in [0, 1).
__device__ __forceinline__ double u01(uint64_t r)
{
    return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

// Counter layout: (step or block, chain id = event << 32 | slot, batch, purpose).
enum Purpose : uint64_t { P_WALK_A = 0, P_START = 1, P_DA2 = 2, P_MLP = 5, P_WALK_B = 6, P_INIT = 7,
                          P_REPL = 9 };

__device__ __forceinline__ uint64_t chain_id(int event, int slot)
{
    return ((uint64_t)(uint32_t)event << 32) | (uint64_t)(uint32_t)slot;
}

// ---------------------------------------------------------------------------
// sin and cos of 2 pi r for r given in revolutions.  Reduction to the nearest
// half turn q (exact: r - q/2 is computed without rounding error, |x| <= 1/4),
// then Taylor polynomials of sin(2 pi x) and cos(2 pi x) on |2 pi x| <= pi/2,
// truncated after x^21 and x^22 (first omitted term below 2e-18), and the
// sign (-1)^q applied to both by flipping sign bits.  Coefficients
// (2 pi)^n / n! are formed at compile time.
// ---------------------------------------------------------------------------
constexpr double taylor_2pi(int n)
{
    double v = 1.0;
    for (int i = 1; i <= n; ++i) v = v * TWO_PI / (double)i;
    return v;
}

__device__ __forceinline__ void sincos_rev(double r, double *s, double *c)
{
    double q = rint(2.0 * r);
    double x = fma(-0.5, q, r);
    double z = x * x;
    double ps = taylor_2pi(21);
    ps = fma(ps, z, -taylor_2pi(19));
    ps = fma(ps, z, taylor_2pi(17));
    ps = fma(ps, z, -taylor_2pi(15));
    ps = fma(ps, z, taylor_2pi(13));
    ps = fma(ps, z, -taylor_2pi(11));
    ps = fma(ps, z, taylor_2pi(9));
    ps = fma(ps, z, -taylor_2pi(7));
    ps = fma(ps, z, taylor_2pi(5));
    ps = fma(ps, z, -taylor_2pi(3));
    ps = fma(ps, z, taylor_2pi(1));
    double sx = ps * x;
    double pc = -taylor_2pi(22);
    pc = fma(pc, z, taylor_2pi(20));
    pc = fma(pc, z, -taylor_2pi(18));
    pc = fma(pc, z, taylor_2pi(16));
    pc = fma(pc, z, -taylor_2pi(14));
    pc = fma(pc, z, taylor_2pi(12));
    pc = fma(pc, z, -taylor_2pi(10));
    pc = fma(pc, z, taylor_2pi(8));
    pc = fma(pc, z, -taylor_2pi(6));
    pc = fma(pc, z, taylor_2pi(4));
    pc = fma(pc, z, -taylor_2pi(2));
    double cx = fma(pc, z, 1.0);
    // (-1)^q: q is integral; its low bit flips the sign of both (phases
    // beyond 2^30 revolutions carry no precision anyway)
    const int odd = __double2int_rz(q) & 1;
    const int flip = odd << 31;
    *s = __hiloint2double(__double2hiint(sx) ^ flip, __double2loint(sx));
    *c = __hiloint2double(__double2hiint(cx) ^ flip, __double2loint(cx));
}

// ---------------------------------------------------------------------------
// Table-assisted sin/cos for the bin loop.  The phase is carried in units of
// 1/TAB_N of a turn (R = TAB_N r).  The nearest integer q of R selects the
// table angle 2 pi (q mod TAB_N) / TAB_N, whose (cos, sin) pair is read from
// a TAB_N-entry table in LDS (4 KB); the remainder x = R - q (|x| <= 1/2,
// exact subtraction) gives sin and cos of the angle 2 pi x / TAB_N
// (|angle| <= pi / 256 = 1.2e-2) by Taylor polynomials truncated after the
// angle^5 and angle^6 terms (first omitted terms 8e-18 and 1.3e-20, below
// half an ulp of 1); the angle-addition formulas combine the two.  (A
// 1024-entry table, which drops the angle^6 term, measured no faster.)
// ---------------------------------------------------------------------------
constexpr int TAB_N = 256;

constexpr double taylor_tab(int n)
{
    double v = 1.0;
    for (int i = 1; i <= n; ++i) v = v * (TWO_PI / TAB_N) / (double)i;
    return v;
}

// Entries (cos, sin)(2 pi j / TAB_N), written by the threads of a block (the
// caller synchronises before use).
__device__ __forceinline__ void fill_sincos_tab(double2 *tab)
{
    for (int j = threadIdx.x; j < TAB_N; j += blockDim.x) {
        double s, c;
        sincos_rev((double)j * (1.0 / TAB_N), &s, &c);
        tab[j] = make_double2(c, s);
    }
}

// sin and cos of 2 pi R / TAB_N (phases below 2^31 / TAB_N turns).
__device__ __forceinline__ void sincos_tab(const double2 *tab, double R, double *s, double *c)
{
    const double q = rint(R);
    const double x = R - q;
    const double2 t = tab[__double2int_rz(q) & (TAB_N - 1)];
    const double z = x * x;
    const double sp = x * fma(z, fma(z, taylor_tab(5), -taylor_tab(3)), taylor_tab(1));
    const double cp = fma(z, fma(z, fma(z, -taylor_tab(6), taylor_tab(4)), -taylor_tab(2)), 1.0);
    *c = fma(t.x, cp, -(t.y * sp));
    *s = fma(t.y, cp, t.x * sp);
}

// ---------------------------------------------------------------------------
// Source parameters needed by the likelihood, from the unit cube or from a
// physical parameter vector.  The inclination and declination enter only
// through cos(theta_JN) and (sin, cos)(dec), which the sine and cosine priors
// give without inverse trigonometry.
// ---------------------------------------------------------------------------
struct Src {
    double mc, q, chi1, chi2, dl, cosi, ra, sindec, cosdec, psi, phic, tc;
    // Sampled distance: dl is the cube root of dl3, taken in make_coef (so a
    // wave can share that root with the other transcendental functions).
    double dl3;
    bool dl_pending;
};

__device__ __forceinline__ double lin(double u, double a, double b) { return a + u * (b - a); }

__device__ inline Src src_from_u(const DevEvent &ev, const double *u)
{
    const int nd = ev.ndim;
    Src p;
    p.mc = nd > 0 ? lin(u[0], ev.lo[0], ev.hi[0]) : ev.fixed[0];
    p.q = nd > 1 ? lin(u[1], ev.lo[1], ev.hi[1]) : ev.fixed[1];
    p.chi1 = nd > 2 ? lin(u[2], ev.lo[2], ev.hi[2]) : ev.fixed[2];
    p.chi2 = nd > 3 ? lin(u[3], ev.lo[3], ev.hi[3]) : ev.fixed[3];
    if (nd > 4) {
        // uniform in dL^3 between the prior edges (the cube root is taken later)
        double a3 = ev.lo[4] * ev.lo[4] * ev.lo[4], b3 = ev.hi[4] * ev.hi[4] * ev.hi[4];
        p.dl3 = a3 + u[4] * (b3 - a3);
        p.dl = 0.0;
        p.dl_pending = true;
    } else {
        p.dl3 = 0.0;
        p.dl = ev.fixed[4];
        p.dl_pending = false;
    }
    p.cosi = nd > 5 ? ev.cos_lo5 - u[5] * (ev.cos_lo5 - ev.cos_hi5) : ev.fixed_cosi;
    p.ra = nd > 6 ? lin(u[6], ev.lo[6], ev.hi[6]) : ev.fixed[6];
    if (nd > 7) {
        double y = ev.sin_lo7 + u[7] * (ev.sin_hi7 - ev.sin_lo7);
        p.sindec = y;
        p.cosdec = sqrt((1.0 - y) * (1.0 + y));
    } else {
        p.sindec = ev.fixed_sindec;
        p.cosdec = ev.fixed_cosdec;
    }
    p.psi = nd > 8 ? lin(u[8], ev.lo[8], ev.hi[8]) : ev.fixed[8];
    p.phic = nd > 9 ? lin(u[9], ev.lo[9], ev.hi[9]) : ev.fixed[9];
    p.tc = nd > 10 ? lin(u[10], ev.lo[10], ev.hi[10]) : ev.fixed[10];
    return p;
}

__device__ inline Src src_from_theta(const double *th)
{
    Src p;
    p.mc = th[0];
    p.q = th[1];
    p.chi1 = th[2];
    p.chi2 = th[3];
    p.dl = th[4];
    p.dl3 = 0.0;
    p.dl_pending = false;
    p.cosi = cos(th[5]);
    p.ra = th[6];
    sincos(th[7], &p.sindec, &p.cosdec);
    p.psi = th[8];
    p.phic = th[9];
    p.tc = th[10];
    return p;
}

// ---------------------------------------------------------------------------
// Per-point coefficients.  The TaylorF2 phase Psi(f) = 2 pi f t_c - 2 phi_c -
// pi/4 + 3/(128 eta v^5) sum_j phi_j v^j, v = (pi M f)^(1/3), is linear in the
// eight bin functions f^(-5/3), f^(-1), f^(-2/3), f^(-1/3), ln f, f^(1/3),
// f^(1/3) ln f, f^(2/3) plus a constant and the time term; the coefficients
// below are those of Psi/(2 pi), i.e. the phase in revolutions.  Detector d
// adds f (t_c + dt_d) revolutions.  The complex amplitude alpha_d carries the
// Newtonian amplitude, inclination and antenna factors, so that
// h_d(f) = alpha_d f^(-7/6) exp(-2 pi i r_d(f)).
// ---------------------------------------------------------------------------
struct Coef {
    double c0, ct1, ct2, ct3, ct5, cL, cs1, csL, cs2;
    double tau[MAXDET];
    double ar[MAXDET], ai[MAXDET];
};

__device__ __forceinline__ bool src_valid(const Src &p)
{
    bool fin = isfinite(p.mc) && isfinite(p.q) && isfinite(p.chi1) && isfinite(p.chi2) &&
               isfinite(p.dl) && isfinite(p.cosi) && isfinite(p.ra) && isfinite(p.sindec) &&
               isfinite(p.cosdec) && isfinite(p.psi) && isfinite(p.phic) && isfinite(p.tc);
    return fin && p.q > 0.0 && p.q <= 1.0 && p.mc > 0.0 && p.dl > 0.0;
}

__device__ inline void response(const DevEvent &ev, const Src &p, int d, double s2p, double c2p,
                                double sphi, double cphi, double *Fp, double *Fx, double *dt)
{
    if (ev.fixed_antenna) {
        *Fp = ev.Fp[d];
        *Fx = ev.Fx[d];
        *dt = 0.0;
        return;
    }
    const double *D = ev.D[d];
    double a0 = sphi, a1 = -cphi, a2 = 0.0;
    double b0 = -cphi * p.sindec, b1 = -sphi * p.sindec, b2 = p.cosdec;
    double Da0 = D[0] * a0 + D[1] * a1 + D[2] * a2;
    double Da1 = D[3] * a0 + D[4] * a1 + D[5] * a2;
    double Da2 = D[6] * a0 + D[7] * a1 + D[8] * a2;
    double Db0 = D[0] * b0 + D[1] * b1 + D[2] * b2;
    double Db1 = D[3] * b0 + D[4] * b1 + D[5] * b2;
    double Db2 = D[6] * b0 + D[7] * b1 + D[8] * b2;
    double aDa = a0 * Da0 + a1 * Da1 + a2 * Da2;
    double bDb = b0 * Db0 + b1 * Db1 + b2 * Db2;
    double aDb = a0 * Db0 + a1 * Db1 + a2 * Db2;
    double gp = aDa - bDb, gx = 2.0 * aDb;
    *Fp = c2p * gp + s2p * gx;
    *Fx = c2p * gx - s2p * gp;
    const double *r = ev.loc[d];
    double n0 = p.cosdec * cphi, n1 = p.cosdec * sphi, n2 = p.sindec;
    *dt = -(r[0] * n0 + r[1] * n1 + r[2] * n2) * (1.0 / C_SI);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// Value of x held by lane l, broadcast to the whole wave.
__device__ __forceinline__ double lane_value(double x, int l)
{
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    return __hiloint2double(hi, lo);
}

// Per-point coefficients.  Modes:
//  COEF_LANE  each thread computes everything itself (threads may hold
//             different points);
//  COEF_WAVE  every lane of a full wave holds the same point; the
//             transcendental functions of the point (three logarithms, three
//             exponentials, two sin/cos pairs) are spread over lanes 0-2 and
//             the detector responses over lanes 0..n_det-1, one call each,
//             and their results read back from those lanes;
//  COEF_GROUP the same within each aligned group of COEF_GW lanes (one point
//             per group, all lanes of a group active together).
// All modes give the same values bit for bit.
constexpr int COEF_LANE = 0, COEF_WAVE = 1, COEF_GROUP = 2, COEF_GW = 4;
static_assert(MAXDET <= COEF_GW && 3 <= COEF_GW, "three logarithms and one response per member");

// Value of x held by member j of the calling lane's group (COEF_WAVE: lane j).
template <int MODE>
__device__ __forceinline__ double member_value(double x, int j)
{
    if (MODE == COEF_WAVE) return lane_value(x, j);
    const int src = (lane_id() & ~(COEF_GW - 1)) | j;
    const int hi = __shfl(__double2hiint(x), src, WAVE);
    const int lo = __shfl(__double2loint(x), src, WAVE);
    return __hiloint2double(hi, lo);
}

template <int MODE>
__device__ inline bool make_coef(const DevEvent &ev, const Src &p0, Coef &c)
{
    constexpr bool WAVE_PAR = MODE != COEF_LANE;
    const int lane = MODE == COEF_GROUP ? (lane_id() & (COEF_GW - 1)) : lane_id();
    const double tsun = GM_SUN / (C_SI * C_SI * C_SI);
    Src p = p0;
    double q = p.q;
    double inv_opq = 1.0 / (1.0 + q);
    double eta = q * inv_opq * inv_opq;
    double x = (1.0 - q) * inv_opq;
    double chis = 0.5 * (p.chi1 + p.chi2), chia = 0.5 * (p.chi1 - p.chi2);
    // a = pi M Tsun with M = Mc eta^(-3/5); powers of a from one logarithm.
    // Logarithms: eta, pi Mc Tsun, dL^3; exponentials: a^(1/3),
    // (pi Mc Tsun)^(5/6), dL.
    double l_eta, l_pmc, l_dl3;
    if (WAVE_PAR) {
        double lg = log(lane == 0 ? eta : (lane == 1 ? PI * tsun * p.mc : p.dl3));
        l_eta = member_value<MODE>(lg, 0);
        l_pmc = member_value<MODE>(lg, 1);
        l_dl3 = member_value<MODE>(lg, 2);
    } else {
        l_eta = log(eta);
        l_pmc = log(PI * tsun * p.mc);
        l_dl3 = p.dl_pending ? log(p.dl3) : 0.0;
    }
    double la = l_pmc - 0.6 * l_eta;
    double a13, e56;
    if (WAVE_PAR) {
        double ex = exp(lane == 0 ? la * (1.0 / 3.0)
                                  : (lane == 1 ? (5.0 / 6.0) * l_pmc : l_dl3 * (1.0 / 3.0)));
        a13 = member_value<MODE>(ex, 0);
        e56 = member_value<MODE>(ex, 1);
        if (p.dl_pending) p.dl = member_value<MODE>(ex, 2);
    } else {
        a13 = exp(la * (1.0 / 3.0));
        e56 = exp((5.0 / 6.0) * l_pmc);
        if (p.dl_pending) p.dl = exp(l_dl3 * (1.0 / 3.0));
    }
    if (!src_valid(p)) return false;
    double am13 = 1.0 / a13;
    double a23 = a13 * a13, am23 = am13 * am13;
    double am1 = am23 * am13;
    double am53 = am1 * am23;
    double eta2 = eta * eta, eta3 = eta2 * eta;
    double P = (3.0 / 128.0 * INV_TWO_PI) / eta;

    // PN coefficients with every rational constant folded at compile time
    // (constant / constant), so no division is left for run time
    double phi2 = (3715.0 / 756.0) + (55.0 / 9.0) * eta;
    double phi3 = -16.0 * PI + (113.0 / 3.0) * x * chia + ((113.0 / 3.0) - (76.0 / 3.0) * eta) * chis;
    double phi4 = (15293365.0 / 508032.0) + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * eta2 +
                  ((-405.0 / 8.0) + 200.0 * eta) * chia * chia - (405.0 / 4.0) * x * chia * chis +
                  ((-405.0 / 8.0) + 2.5 * eta) * chis * chis;
    double b5 = PI * ((38645.0 / 756.0) - (65.0 / 9.0) * eta) +
                x * ((-732985.0 / 2268.0) - (140.0 / 9.0) * eta) * chia +
                ((-732985.0 / 2268.0) + (24260.0 / 81.0) * eta + (340.0 / 9.0) * eta2) * chis;
    double a6 = (11583231236531.0 / 4694215680.0 - 6848.0 * EULER_GAMMA / 21.0 -
                 640.0 * PI * PI / 3.0) +
                (-15737765635.0 / 3048192.0 + 2255.0 * PI * PI / 12.0) * eta +
                (76055.0 / 1728.0) * eta2 - (127825.0 / 1296.0) * eta3 +
                PI * ((2270.0 / 3.0) * x * chia + ((2270.0 / 3.0) - 520.0 * eta) * chis);
    double l6 = 6848.0 / 63.0;
    double phi7 = PI * ((77096675.0 / 254016.0) + (378515.0 / 1512.0) * eta - (74045.0 / 756.0) * eta2) +
                  x * ((-25150083775.0 / 3048192.0) + (26804935.0 / 6048.0) * eta - (1985.0 / 48.0) * eta2) *
                      chia +
                  ((-25150083775.0 / 3048192.0) + (10566655595.0 / 762048.0) * eta -
                   (1042165.0 / 3024.0) * eta2 + (5345.0 / 36.0) * eta3) *
                      chis;
    const double ln64 = 4.1588830833596715;  // 6 ln 2

    c.ct5 = P * am53;
    c.ct3 = P * phi2 * am1;
    c.ct2 = P * phi3 * am23;
    c.ct1 = P * phi4 * am13;
    c.cL = P * b5;
    c.cs1 = P * a13 * (a6 - l6 * (ln64 + la));
    c.csL = -P * a13 * l6;
    c.cs2 = P * phi7 * a23;
    c.c0 = (-2.0 * p.phic - 0.25 * PI) * INV_TWO_PI + P * b5 * (1.0 + la);

    // Newtonian amplitude sqrt(5/24) pi^(-2/3) (Mc Tsun)^(5/6) c / dL, with
    // (Mc Tsun)^(5/6) = (pi Mc Tsun)^(5/6) pi^(-5/6)
    const double KA = 0.45643546458763842 /* sqrt(5/24) */ * 0.17958712212516656 /* pi^-(2/3+5/6) = pi^-1.5 */ *
                      C_SI / MPC_SI;
    double A = KA * e56 / p.dl;
    double plus = 0.5 * (1.0 + p.cosi * p.cosi);
    double sphi = 0.0, cphi = 1.0, s2p = 0.0, c2p = 1.0;
    if (!ev.fixed_antenna) {
        if (WAVE_PAR) {
            double sn, cs;
            sincos_rev(lane == 0 ? (p.ra - ev.gmst) * INV_TWO_PI : p.psi * (2.0 * INV_TWO_PI), &sn, &cs);
            sphi = member_value<MODE>(sn, 0);
            cphi = member_value<MODE>(cs, 0);
            s2p = member_value<MODE>(sn, 1);
            c2p = member_value<MODE>(cs, 1);
        } else {
            sincos_rev((p.ra - ev.gmst) * INV_TWO_PI, &sphi, &cphi);
            sincos_rev(p.psi * (2.0 * INV_TWO_PI), &s2p, &c2p);
        }
    }
    double Fp_l = 0.0, Fx_l = 0.0, dt_l = 0.0;
    if (WAVE_PAR) {
        // lane d: detector d
        response(ev, p, lane < ev.n_det ? lane : 0, s2p, c2p, sphi, cphi, &Fp_l, &Fx_l, &dt_l);
    }
#pragma unroll
    for (int d = 0; d < MAXDET; ++d) {
        if (d < ev.n_det) {
            double Fp, Fx, dt;
            if (WAVE_PAR) {
                Fp = member_value<MODE>(Fp_l, d);
                Fx = member_value<MODE>(Fx_l, d);
                dt = member_value<MODE>(dt_l, d);
            } else {
                response(ev, p, d, s2p, c2p, sphi, cphi, &Fp, &Fx, &dt);
            }
            c.tau[d] = p.tc + dt;
            c.ar[d] = A * Fp * plus;
            c.ai[d] = -A * Fx * p.cosi;
        } else {
            c.tau[d] = 0.0;
            c.ar[d] = 0.0;
            c.ai[d] = 0.0;
        }
    }
    return true;
}

// Phase in revolutions at one bin, without the detector time term.
__device__ __forceinline__ double phase_rev(const Coef &c, double t, double s, double L)
{
    double t2 = t * t;
    double pt = fma(t2, c.ct5, c.ct3);
    pt = fma(t, pt, c.ct2);
    pt = fma(t, pt, c.ct1);
    double r = fma(t, pt, c.c0);
    double ps = fma(s, c.cs2, c.cs1);
    r = fma(s, ps, r);
    double pl = fma(s, c.csL, c.cL);
    return fma(L, pl, r);
}

// Global-memory views of the event tables.  The table pointers are read out
// of the event descriptor, so the compiler would otherwise treat them as
// generic pointers (flat loads that cannot be overlapped with computation).
typedef const __attribute__((address_space(1))) double gdouble;
typedef const __attribute__((address_space(1))) float gfloat;

// Tables of one bin held in registers.
template <int ND, typename T>
struct BinRegs {
    double t, s, L;
    T wr[ND], wi[ND];
};

typedef const __attribute__((address_space(1))) char gchar;

// Row r of the tables for this lane: three basis values and ND weight pairs,
// at two addresses (basis stride 8 B, weight stride 16 or 8 B per lane) plus
// constant offsets.  Table sizes stay far below 4 GiB: 32-bit offsets.
template <int ND, typename T, int ROWB>
__device__ __forceinline__ void load_row(BinRegs<ND, T> &b, gchar *base, int r, int lane)
{
    const uint32_t o1 = (uint32_t)r * ROWB + (uint32_t)lane * 8u;
    b.t = *(gdouble *)(base + o1 + ROW_T);
    b.s = *(gdouble *)(base + o1 + ROW_S);
    b.L = *(gdouble *)(base + o1 + ROW_L);
    constexpr int WB = sizeof(T) == 8 ? ROW_W64 : ROW_W32;
    const uint32_t o2 = (uint32_t)r * ROWB + ROW_W + (uint32_t)lane * (2u * sizeof(T));
    typedef const __attribute__((address_space(1))) T gT;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        b.wr[d] = *(gT *)(base + o2 + d * WB);
        b.wi[d] = *(gT *)(base + o2 + d * WB + sizeof(T));
    }
}

// Phase polynomial (revolutions) of one bin without the detector time term.
__device__ __forceinline__ double bin_phase(double t, double s, double L, double c0, double ct1,
                                            double ct2, double ct3, double ct5, double cL,
                                            double cs1, double csL, double cs2)
{
    double t2 = t * t;
    double pt = fma(t2, ct5, ct3);
    pt = fma(t, pt, ct2);
    pt = fma(t, pt, ct1);
    double r = fma(t, pt, c0);
    r = fma(s, fma(s, cs2, cs1), r);
    return fma(L, fma(s, csL, cL), r);
}

// Runs body(regs, row) over rows 0..rows-1 (row r is bin lane + 64 r) with
// the tables of row r + 1 loaded while row r is computed: two register sets
// used alternately, loop count the same for every lane (rows is
// wave-uniform; padded bins carry zero weights).
template <int ND, typename T, int ROWB, typename Body>
__device__ __forceinline__ void for_each_row(gchar *base, int rows, Body body)
{
    const int lane = lane_id();
    BinRegs<ND, T> A, B;
    load_row<ND, T, ROWB>(A, base, 0, lane);
    int r = 0;
    for (; r + 1 < rows; r += 2) {
        load_row<ND, T, ROWB>(B, base, r + 1, lane);
        body(A, r);
        // (re-reads the last row instead of reading past it: no branch in the loop)
        load_row<ND, T, ROWB>(A, base, min(r + 2, rows - 1), lane);
        body(B, r + 1);
    }
    if (r < rows) body(A, r);
}

// The same walk over rows lo..hi-1 (lo < hi, wave-uniform) from the last row
// down to row lo.
template <int ND, typename T, int ROWB, typename Body>
__device__ __forceinline__ void for_rows_desc(gchar *base, int lo, int hi, Body body)
{
    const int lane = lane_id();
    BinRegs<ND, T> A, B;
    int r = hi - 1;
    load_row<ND, T, ROWB>(A, base, r, lane);
    for (; r >= lo + 1; r -= 2) {
        load_row<ND, T, ROWB>(B, base, r - 1, lane);
        body(A, r);
        load_row<ND, T, ROWB>(A, base, max(r - 2, lo), lane);
        body(B, r - 1);
    }
    if (r == lo) body(A, lo);
}


// The exact FP64 sums run over two halves of the rows, lower [0, mid) and
// upper [mid, rows), each reduced over the wave on its own and then added
// lower + upper: the same rounding whether one wave takes both halves or two
// waves take one each.
__device__ __forceinline__ int row_mid(int rows) { return (rows + 1) / 2; }

// Whittle sums Z_d = sum_k w_{d,k} exp(-2 pi i r_d(f_k)), FP64, with one
// sin/cos per bin.  Detector 0 takes e0 = exp(-2 pi i r_0) from the
// polynomial phase.  A detector d > 0 differs by the factor
// exp(-2 pi i f (tau_d - tau_0)) = R_d Q_d^j on the lane's j-th bin
// (f = f_lane + 64 df j; R_d at f_lane, Q_d the constant step), so its sum is
// R_d sum_j (w_{d,j} e0_j) Q_d^j: a Horner recurrence S <- S Q_d + w e0 over
// the rows taken from the last to the first, and one product with R_d at the
// end.  Lane l takes bins l, l + 64, ...  This sums rows lo..hi-1 (lo < hi),
// the recurrence relative to row lo (R_d at the lane's bin of row lo); called
// by all lanes of a full wave with the same point.
template <int ND>
__device__ __forceinline__ void accumulate_fp64_rot(const DevEvent &ev, const Coef &c, int lo,
                                                    int hi, double *Zr, double *Zi,
                                                    const double2 *tab)
{
    gchar *base = (gchar *)ev.rows64;
    const int lane = lane_id();
    const double df = ev.df, flo = ev.f_lo;
    // phase coefficients in 1/TAB_N turns (exact power-of-two scaling)
    constexpr double TS = (double)TAB_N;
    const double c0 = TS * c.c0, ct1 = TS * c.ct1, ct2 = TS * c.ct2, ct3 = TS * c.ct3;
    const double ct5 = TS * c.ct5, cL = TS * c.cL, cs1 = TS * c.cs1, csL = TS * c.csL;
    const double cs2 = TS * c.cs2, tau0 = c.tau[0], tau0s = TS * c.tau[0];
    double Qr[ND], Qi[ND], Sr[ND], Si[ND];
    // the steps are the same for every lane: lane d - 1 evaluates detector
    // d's, one sin/cos for all of them
    double qarg = 0.0;
#pragma unroll
    for (int d = 1; d < ND; ++d)
        if (lane == d - 1) qarg = ((double)WAVE * df) * (c.tau[d] - tau0);
    double qs, qc;
    sincos_rev(qarg, &qs, &qc);
    const double f0 = (double)(lane + WAVE * lo) * df + flo;
#pragma unroll
    for (int d = 1; d < ND; ++d) {
        Qr[d] = lane_value(qc, d - 1);
        Qi[d] = -lane_value(qs, d - 1);
        Sr[d] = Si[d] = 0.0;
    }
    for_rows_desc<ND, double, ROW64>(base, lo, hi, [&](const BinRegs<ND, double> &b, int r) {
        double f = (double)(lane + WAVE * r) * df + flo;
        double ph = fma(f, tau0s, bin_phase(b.t, b.s, b.L, c0, ct1, ct2, ct3, ct5, cL, cs1, csL, cs2));
        double sn, cs;
        sincos_tab(tab, ph, &sn, &cs);
        // w e0 with e0 = cos - i sin
        Zr[0] = fma(b.wr[0], cs, fma(b.wi[0], sn, Zr[0]));
        Zi[0] = fma(b.wi[0], cs, fma(-b.wr[0], sn, Zi[0]));
#pragma unroll
        for (int d = 1; d < ND; ++d) {
            const double pr = fma(b.wr[d], cs, b.wi[d] * sn);
            const double pi = fma(b.wi[d], cs, -(b.wr[d] * sn));
            const double nr = fma(Sr[d], Qr[d], fma(-Si[d], Qi[d], pr));
            const double ni = fma(Sr[d], Qi[d], fma(Si[d], Qr[d], pi));
            Sr[d] = nr;
            Si[d] = ni;
        }
    });
    // R_d = cos - i sin at the lane's bin of row lo, after the loop
#pragma unroll
    for (int d = 1; d < ND; ++d) {
        double Ri, Rr;
        sincos_rev(f0 * (c.tau[d] - tau0), &Ri, &Rr);
        Zr[d] += fma(Rr, Sr[d], Ri * Si[d]);
        Zi[d] += fma(Rr, Si[d], -(Ri * Sr[d]));
    }
}

// Two points at once over rows lo..hi-1: the same sums as accumulate_fp64_rot
// for points cf[0] and cf[1], sharing every table load (half the table
// traffic per point) and giving the scheduler two independent dependency
// chains per bin.  A detector d > 0 takes its Horner recurrence relative to
// row lo, so its end factor is R_d at the lane's bin of row lo.  Adds into
// Zr[x][d], Zi[x][d] for point x; called by all lanes of a full wave.
template <int ND>
__device__ __forceinline__ void accumulate_fp64_pair(const DevEvent &ev, const Coef *const cf[2],
                                                     int lo, int hi, double (&Zr)[2][ND],
                                                     double (&Zi)[2][ND], const double2 *tab)
{
    gchar *base = (gchar *)ev.rows64;
    const int lane = lane_id();
    const double df = ev.df, flo = ev.f_lo;
    constexpr double TS = (double)TAB_N;
    double c0[2], ct1[2], ct2[2], ct3[2], ct5[2], cL[2], cs1[2], csL[2], cs2[2], tau0s[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        const Coef &c = *cf[x];
        c0[x] = TS * c.c0;
        ct1[x] = TS * c.ct1;
        ct2[x] = TS * c.ct2;
        ct3[x] = TS * c.ct3;
        ct5[x] = TS * c.ct5;
        cL[x] = TS * c.cL;
        cs1[x] = TS * c.cs1;
        csL[x] = TS * c.csL;
        cs2[x] = TS * c.cs2;
        tau0s[x] = TS * c.tau[0];
    }
    // row steps: lane x (ND - 1) + d - 1 evaluates point x, detector d
    double qarg = 0.0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int d = 1; d < ND; ++d)
            if (lane == x * (ND - 1) + d - 1)
                qarg = ((double)WAVE * df) * (cf[x]->tau[d] - cf[x]->tau[0]);
    double qs, qc;
    sincos_rev(qarg, &qs, &qc);
    const double fs = (double)(lane + WAVE * lo) * df + flo;
    double Qr[2][ND], Qi[2][ND], Sr[2][ND], Si[2][ND];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int d = 1; d < ND; ++d) {
            Qr[x][d] = lane_value(qc, x * (ND - 1) + d - 1);
            Qi[x][d] = -lane_value(qs, x * (ND - 1) + d - 1);
            Sr[x][d] = Si[x][d] = 0.0;
        }
    for_rows_desc<ND, double, ROW64>(base, lo, hi, [&](const BinRegs<ND, double> &b, int r) {
        const double f = (double)(lane + WAVE * r) * df + flo;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
            const double ph = fma(f, tau0s[x], bin_phase(b.t, b.s, b.L, c0[x], ct1[x], ct2[x], ct3[x],
                                                         ct5[x], cL[x], cs1[x], csL[x], cs2[x]));
            double sn, cs;
            sincos_tab(tab, ph, &sn, &cs);
            Zr[x][0] = fma(b.wr[0], cs, fma(b.wi[0], sn, Zr[x][0]));
            Zi[x][0] = fma(b.wi[0], cs, fma(-b.wr[0], sn, Zi[x][0]));
#pragma unroll
            for (int d = 1; d < ND; ++d) {
                const double pr = fma(b.wr[d], cs, b.wi[d] * sn);
                const double pi = fma(b.wi[d], cs, -(b.wr[d] * sn));
                const double nr = fma(Sr[x][d], Qr[x][d], fma(-Si[x][d], Qi[x][d], pr));
                const double ni = fma(Sr[x][d], Qi[x][d], fma(Si[x][d], Qr[x][d], pi));
                Sr[x][d] = nr;
                Si[x][d] = ni;
            }
        }
    });
    // end factors R_d = cos - i sin at the lane's bin of row lo (after the
    // loop: no registers held across it)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int d = 1; d < ND; ++d) {
            double Ri, Rr;
            sincos_rev(fs * (cf[x]->tau[d] - cf[x]->tau[0]), &Ri, &Rr);
            Zr[x][d] += fma(Rr, Sr[x][d], Ri * Si[x][d]);
            Zi[x][d] += fma(Rr, Si[x][d], -(Ri * Sr[x][d]));
        }
}

// Mixed precision: the phase polynomial and the reduction of the phase to a
// fraction of a turn stay FP64 (exact subtraction of the nearest integer);
// sin and cos of that fraction use the FP32 hardware instructions (argument
// in revolutions), once per bin, for detector 0.  A detector d > 0 differs by
// exp(-2 pi i f (tau_d - tau_0)) = R_d Q_d^j (Q_d the constant step of the
// lane's bins, R_d the factor at a reference row), so its FP32 sum is a
// Horner recurrence S <- S Q_d + w_d e0 over the rows walked downwards,
// restarted at every row r with r % 8 == 0 and at row lo: there S is
// rotated by R_d at the lane's bin of row r (argument f (tau_d - tau_0)
// reduced in FP64, sin/cos in FP32) and flushed into the FP64 sum, as the
// FP32 sums of detector 0 are.  No FP32 sum spans more than 8 rows of a
// lane.  NP points at once over rows lo..hi-1, sharing the table loads;
// adds into Zr[x][d], Zi[x][d] for point x.
template <int ND, int NP>
__device__ __forceinline__ void accumulate_mixed_np(const DevEvent &ev, const Coef *const cf[NP],
                                                    int lo, int hi, double (&Zr)[NP][ND],
                                                    double (&Zi)[NP][ND])
{
    gchar *base = (gchar *)ev.rows32;  // weights scaled by wscale
    const int lane = lane_id();
    const double df = ev.df, flo = ev.f_lo;
    double c0[NP], ct1[NP], ct2[NP], ct3[NP], ct5[NP], cL[NP], cs1[NP], csL[NP], cs2[NP];
    double tau0[NP], dtau[NP][ND];
    float qr[NP][ND], qi[NP][ND], sr[NP][ND], si[NP][ND];
    float zr[NP], zi[NP];
#pragma unroll
    for (int x = 0; x < NP; ++x) {
        const Coef &c = *cf[x];
        c0[x] = c.c0;
        ct1[x] = c.ct1;
        ct2[x] = c.ct2;
        ct3[x] = c.ct3;
        ct5[x] = c.ct5;
        cL[x] = c.cL;
        cs1[x] = c.cs1;
        csL[x] = c.csL;
        cs2[x] = c.cs2;
        tau0[x] = c.tau[0];
        zr[x] = zi[x] = 0.0f;
#pragma unroll
        for (int d = 1; d < ND; ++d) {
            dtau[x][d] = c.tau[d] - c.tau[0];
            // row step: the phase advance over 64 bins, reduced in FP64
            const double a = ((double)WAVE * df) * dtau[x][d];
            const float xr = (float)(a - rint(a));
            qr[x][d] = __builtin_amdgcn_cosf(xr);
            qi[x][d] = -__builtin_amdgcn_sinf(xr);
            sr[x][d] = si[x][d] = 0.0f;
        }
    }
    for_rows_desc<ND, float, ROW32>(base, lo, hi, [&](const BinRegs<ND, float> &b, int r) {
        const double f = (double)(lane + WAVE * r) * df + flo;
#pragma unroll
        for (int x = 0; x < NP; ++x) {
            const double ph = bin_phase(b.t, b.s, b.L, c0[x], ct1[x], ct2[x], ct3[x], ct5[x], cL[x],
                                        cs1[x], csL[x], cs2[x]);
            const double rd = fma(f, tau0[x], ph);
            const float xr = (float)(rd - rint(rd));
            const float sn = __builtin_amdgcn_sinf(xr);
            const float cs = __builtin_amdgcn_cosf(xr);
            // w e0 with e0 = cos - i sin
            zr[x] = fmaf(b.wr[0], cs, fmaf(b.wi[0], sn, zr[x]));
            zi[x] = fmaf(b.wi[0], cs, fmaf(-b.wr[0], sn, zi[x]));
#pragma unroll
            for (int d = 1; d < ND; ++d) {
                const float pr = fmaf(b.wr[d], cs, b.wi[d] * sn);
                const float pi = fmaf(b.wi[d], cs, -(b.wr[d] * sn));
                const float nr = fmaf(sr[x][d], qr[x][d], fmaf(-si[x][d], qi[x][d], pr));
                const float ni = fmaf(sr[x][d], qi[x][d], fmaf(si[x][d], qr[x][d], pi));
                sr[x][d] = nr;
                si[x][d] = ni;
            }
        }
        if ((r & 7) == 0 || r == lo) {
#pragma unroll
            for (int x = 0; x < NP; ++x) {
                Zr[x][0] += (double)zr[x];
                Zi[x][0] += (double)zi[x];
                zr[x] = zi[x] = 0.0f;
#pragma unroll
                for (int d = 1; d < ND; ++d) {
                    // R_d = cos - i sin of f (tau_d - tau_0) at this lane's bin of row r
                    const double a = f * dtau[x][d];
                    const float xr = (float)(a - rint(a));
                    const float Rr = __builtin_amdgcn_cosf(xr), Ri = -__builtin_amdgcn_sinf(xr);
                    Zr[x][d] += (double)fmaf(Rr, sr[x][d], -(Ri * si[x][d]));
                    Zi[x][d] += (double)fmaf(Rr, si[x][d], Ri * sr[x][d]);
                    sr[x][d] = si[x][d] = 0.0f;
                }
            }
        }
    });
}

// Heterodyned data term (relative binning), FP64:
//   Z_d = sum_b G0_{d,b} e_{d,b} + G1_{d,b} (e_{d,b+1} - e_{d,b}) / (f_{b+1} - f_b),
//   e_{d,b} = e^{-2 pi i (r_d(f_b) - r0_d(f_b))},
// the linear interpolation of the ratio to the fiducial phase factor between
// nodes, summed against the fiducial sums of each bin.  Lane l of row r
// evaluates node 63 r + l and takes node 63 r + l + 1 from lane l + 1.
// Called by all lanes of a full wave with the same point.
template <int ND>
__device__ __forceinline__ void accumulate_rb(const DevEvent &ev, const Coef &c, double *Zr,
                                              double *Zi, const double2 *tab)
{
    const int lane = lane_id();
    const int B = ev.rb_bins, rows = ev.rb_nrows;
    gchar *base = (gchar *)ev.rb_rows;
    constexpr double TS = (double)TAB_N;
    const double c0 = TS * c.c0, ct1 = TS * c.ct1, ct2 = TS * c.ct2, ct3 = TS * c.ct3;
    const double ct5 = TS * c.ct5, cL = TS * c.cL, cs1 = TS * c.cs1, csL = TS * c.csL;
    const double cs2 = TS * c.cs2;
    double taus[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) taus[d] = TS * c.tau[d];
    for (int r = 0; r < rows; ++r) {
        const uint32_t o = (uint32_t)r * RB_ROW + (uint32_t)lane * 8u;
        const double f = *(gdouble *)(base + o + RB_F);
        const double ph = bin_phase(*(gdouble *)(base + o + RB_T), *(gdouble *)(base + o + RB_S),
                                    *(gdouble *)(base + o + RB_L), c0, ct1, ct2, ct3, ct5, cL, cs1,
                                    csL, cs2);
        const bool has_bin = lane < RB_BINS_PER_ROW && RB_BINS_PER_ROW * r + lane < B;
        const double iw = *(gdouble *)(base + o + RB_IW);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const double r0 = *(gdouble *)(base + o + RB_R0 + 512 * d);
            double sn, cs;
            sincos_tab(tab, fma(f, taus[d], ph) - TS * r0, &sn, &cs);
            const double er = cs, ei = -sn;
            const double nr = __shfl_down(er, 1, WAVE), ni = __shfl_down(ei, 1, WAVE);
            if (has_bin) {
                const uint32_t og = (uint32_t)r * RB_ROW + (uint32_t)lane * 16u + 1024u * d;
                const double g0r = *(gdouble *)(base + og + RB_G0), g0i = *(gdouble *)(base + og + RB_G0 + 8);
                const double g1r = *(gdouble *)(base + og + RB_G1), g1i = *(gdouble *)(base + og + RB_G1 + 8);
                const double dr = (nr - er) * iw, di = (ni - ei) * iw;
                Zr[d] = fma(g0r, er, fma(-g0i, ei, fma(g1r, dr, fma(-g1i, di, Zr[d]))));
                Zi[d] = fma(g0r, ei, fma(g0i, er, fma(g1r, di, fma(g1i, dr, Zi[d]))));
            }
        }
    }
}

// tab: the LDS sin/cos table (FP64 path only; fill_sincos_tab).
// Relative-binning events (likelihood 2) always take the FP64 heterodyned sum.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = WAVE / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Reduced sums R_d + i I_d of one point over all bins (every lane receives
// them); called by all lanes of a full wave with the same point.  The exact
// likelihood (FP64 or mixed) sums the two row halves apart, as the walk's
// candidate pairs do.
template <int ND, int MIXED>
__device__ __forceinline__ void wave_sums(const DevEvent &ev, const Coef &c, double *R, double *I,
                                          const double2 *tab)
{
    double Zr[1][ND], Zi[1][ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) Zr[0][d] = Zi[0][d] = 0.0;
    if (ev.likelihood == 2) {
        accumulate_rb<ND>(ev, c, Zr[0], Zi[0], tab);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            R[d] = wave_sum(Zr[0][d]);
            I[d] = wave_sum(Zi[0][d]);
        }
        return;
    }
    const int rows = ev.n_pad / WAVE, mid = row_mid(rows);
#pragma unroll
    for (int d = 0; d < ND; ++d) R[d] = I[d] = 0.0;
    // one copy of the row loop for both halves (R + 0 = R for the lower one)
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        const int lo = h ? mid : 0, hi = h ? rows : mid;
        if (lo >= hi) break;
#pragma unroll
        for (int d = 0; d < ND; ++d) Zr[0][d] = Zi[0][d] = 0.0;
        if (MIXED) {
            const Coef *cp[1] = {&c};
            accumulate_mixed_np<ND, 1>(ev, cp, lo, hi, Zr, Zi);
        } else {
            accumulate_fp64_rot<ND>(ev, c, lo, hi, Zr[0], Zi[0], tab);
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            R[d] += wave_sum(Zr[0][d]);
            I[d] += wave_sum(Zi[0][d]);
        }
    }
}

// log Lambda from the reduced sums: sum_d Re(alpha_d Z_d) - |alpha_d|^2 K_d / 2.
// Detectors beyond ev.n_det carry alpha_d = 0 and contribute nothing.
template <int ND, int MIXED = 0>
__device__ __forceinline__ double combine(const DevEvent &ev, const Coef &c, const double *Zr,
                                          const double *Zi)
{
    double tot = 0.0;
    // power of two: exact (the heterodyned sums of relative binning are FP64)
    const double iscale = (MIXED && ev.likelihood != 2) ? 1.0 / ev.wscale : 1.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        double dh = (c.ar[d] * Zr[d] - c.ai[d] * Zi[d]) * iscale;
        double hh = (c.ar[d] * c.ar[d] + c.ai[d] * c.ai[d]) * ev.K[d];
        tot += dh - 0.5 * hh;
    }
    return tot;
}

__device__ __forceinline__ double toy_loglike(const DevEvent &ev, const double *u)
{
    double s = 0.0;
    for (int j = 0; j < ev.ndim; ++j) {
        double z = u[j] - 0.5;
        s += z * z;
    }
    return -s / (2.0 * ev.toy_sigma * ev.toy_sigma);
}

__device__ __forceinline__ bool is_periodic(int ndim, int j)
{
    return ndim == NPAR && (j == 6 || j == 8 || j == 9);
}

}  // namespace nsmi
