// Kernels of the MI355X acceptance-walk nested sampler (gfx950, wave64).
//
//   prep_event   per-bin phase basis, whitened weights, K_d           (init)
//   init_live    prior draws (Philox purpose 7) and their likelihood  (init)
//   loglike_*    one wave per point, bins strided over the lanes
//   select       per event: sort live logL, delete k, L*, survivor
//                snapshot, chain start picks, dead-point evidence update
//   walk         (nsmi_walk.hip) one workgroup per chain: W
//                differential-evolution steps, each a full likelihood
//                evaluation, strict L > L*
//   finish       per event: walk statistics, walk-length retune,
//                termination metrics
#include <hip/hip_runtime.h>

#include "nsmi_kernels.h"
#include "nsmi_mlp.h"

namespace nsmi {

// ---------------------------------------------------------------------------
// init: per-bin tables
// ---------------------------------------------------------------------------
// One thread per padded bin k = 64 r + l: row r, slot l of both row tables.
// Bins N <= k < NP continue the frequency grid in the basis; their weights
// stay zero (the row tables are cleared before this kernel).
__global__ void prep_bins_kernel(int N, int NP, int ND, double f_lo, double df, const double *data,
                                 const double *psd, char *rows64, char *rows32, double wscale)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NP) return;
    const int r = k / WAVE, l = k % WAVE;
    char *R64 = rows64 + (size_t)r * ROW64;
    char *R32 = rows32 + (size_t)r * ROW32;
    double f = (double)k * df + f_lo;
    double s = cbrt(f);
    double t = 1.0 / s, L = log(f);
    reinterpret_cast<double *>(R64 + ROW_T)[l] = t;
    reinterpret_cast<double *>(R64 + ROW_S)[l] = s;
    reinterpret_cast<double *>(R64 + ROW_L)[l] = L;
    reinterpret_cast<double *>(R32 + ROW_T)[l] = t;
    reinterpret_cast<double *>(R32 + ROW_S)[l] = s;
    reinterpret_cast<double *>(R32 + ROW_L)[l] = L;
    if (k >= N) return;
    double fac0 = 4.0 * df * pow(f, -7.0 / 6.0);
    for (int d = 0; d < ND; ++d) {
        double S = psd[(size_t)d * N + k];
        double fac = fac0 / S;
        double dr = data[2 * ((size_t)d * N + k)];
        double di = data[2 * ((size_t)d * N + k) + 1];
        // 4 df conj(d) f^-7/6 / S
        reinterpret_cast<double2 *>(R64 + ROW_W + d * ROW_W64)[l] = make_double2(fac * dr, -fac * di);
        reinterpret_cast<float2 *>(R32 + ROW_W + d * ROW_W32)[l] =
            make_float2((float)(fac * dr * wscale), (float)(-fac * di * wscale));
    }
}

// K_d = 4 df sum_k f_k^(-7/3) / S_d(f_k); one block per detector, fixed
// reduction order.
__global__ void prep_K_kernel(int N, double f_lo, double df, const double *psd, double *K)
{
    __shared__ double part[1024];
    int d = blockIdx.x;
    double acc = 0.0;
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double f = (double)k * df + f_lo;
        acc += pow(f, -7.0 / 3.0) / psd[(size_t)d * N + k];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) K[d] = 4.0 * df * part[0];
}

hipError_t launch_prep_event(const DevEvent &hev, const double *d_data, const double *d_psd,
                             char *rows64, char *rows32, double *K_out, hipStream_t s)
{
    int N = hev.n_bins, NP = hev.n_pad;
    if (NP < N || NP % WAVE != 0 || hev.n_det > MAXDET) return hipErrorInvalidValue;
    prep_bins_kernel<<<(NP + 255) / 256, 256, 0, s>>>(N, NP, hev.n_det, hev.f_lo, hev.df, d_data,
                                                      d_psd, rows64, rows32, hev.wscale);
    prep_K_kernel<<<hev.n_det, 1024, 0, s>>>(N, hev.f_lo, hev.df, d_psd, K_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// init: relative-binning tables (fiducial theta0 and the node indices).
// Nodes: one thread per node b = 0..B, written to its slot (b / 63, b % 63)
// and, for b a positive multiple of 63, also to slot 63 of the previous row.
// ---------------------------------------------------------------------------
__global__ void prep_rb_nodes_kernel(const DevEvent *evp, const int32_t *edges,
                                     const double *theta0, char *rows)
{
    const DevEvent &ev = *evp;
    const int B = ev.rb_bins;
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > B) return;
    double th[NPAR];
    for (int j = 0; j < NPAR; ++j) th[j] = theta0[j];
    Coef c;
    make_coef<COEF_LANE>(ev, src_from_theta(th), c);
    const double f = (double)edges[b] * ev.df + ev.f_lo;
    const double s = cbrt(f), t = 1.0 / s, L = log(f);
    const double iw = b < B ? 1.0 / ((double)(edges[b + 1] - edges[b]) * ev.df) : 0.0;
    for (int slot = 0; slot < 2; ++slot) {
        int r, l;
        if (slot == 0) {
            r = b / RB_BINS_PER_ROW;
            l = b % RB_BINS_PER_ROW;
        } else {
            if (b == 0 || b % RB_BINS_PER_ROW != 0) break;
            r = b / RB_BINS_PER_ROW - 1;
            l = RB_BINS_PER_ROW;
        }
        if (r >= ev.rb_nrows) continue;  // (node B when B is a multiple of 63: slot 1 only)
        char *R = rows + (size_t)r * RB_ROW;
        reinterpret_cast<double *>(R + RB_F)[l] = f;
        reinterpret_cast<double *>(R + RB_T)[l] = t;
        reinterpret_cast<double *>(R + RB_S)[l] = s;
        reinterpret_cast<double *>(R + RB_L)[l] = L;
        for (int d = 0; d < ev.n_det; ++d)
            reinterpret_cast<double *>(R + RB_R0 + 512 * d)[l] = fma(f, c.tau[d], phase_rev(c, t, s, L));
        reinterpret_cast<double *>(R + RB_IW)[l] = slot == 0 ? iw : 0.0;
    }
}

// Fiducial sums of one bin and detector per wave:
// G0 = sum_k w_k e^{-2 pi i r0_d(f_k)}, G1 = sum_k w_k e^{-2 pi i r0_d(f_k)} (f_k - f_b).
__global__ __launch_bounds__(256) void prep_rb_sums_kernel(const DevEvent *evp, const int32_t *edges,
                                                           const double *theta0, char *rows)
{
    const DevEvent &ev = *evp;
    const int wv = (int)((blockIdx.x * blockDim.x + threadIdx.x) / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    if (wv >= ev.rb_bins * ev.n_det) return;
    const int b = wv / ev.n_det, d = wv % ev.n_det;
    double th[NPAR];
    for (int j = 0; j < NPAR; ++j) th[j] = theta0[j];
    Coef c;
    make_coef<COEF_LANE>(ev, src_from_theta(th), c);
    const int k0 = edges[b], k1 = edges[b + 1];
    const double fb = (double)k0 * ev.df + ev.f_lo;
    double g0r = 0.0, g0i = 0.0, g1r = 0.0, g1i = 0.0;
    for (int k = k0 + lane; k < k1; k += WAVE) {
        const char *R = ev.rows64 + (size_t)(k / WAVE) * ROW64;
        const int l = k % WAVE;
        const double t = reinterpret_cast<const double *>(R + ROW_T)[l];
        const double s = reinterpret_cast<const double *>(R + ROW_S)[l];
        const double L = reinterpret_cast<const double *>(R + ROW_L)[l];
        const double wr = reinterpret_cast<const double *>(R + ROW_W + d * ROW_W64)[2 * l];
        const double wi = reinterpret_cast<const double *>(R + ROW_W + d * ROW_W64)[2 * l + 1];
        const double f = (double)k * ev.df + ev.f_lo;
        double sn, cs;
        sincos_rev(fma(f, c.tau[d], phase_rev(c, t, s, L)), &sn, &cs);
        const double gr = wr * cs + wi * sn, gi = wi * cs - wr * sn;  // w (cos - i sin)
        g0r += gr;
        g0i += gi;
        g1r += gr * (f - fb);
        g1i += gi * (f - fb);
    }
    g0r = wave_sum(g0r);
    g0i = wave_sum(g0i);
    g1r = wave_sum(g1r);
    g1i = wave_sum(g1i);
    if (lane == 0) {
        char *R = rows + (size_t)(b / RB_BINS_PER_ROW) * RB_ROW + 16 * (b % RB_BINS_PER_ROW) + 1024 * d;
        reinterpret_cast<double *>(R + RB_G0)[0] = g0r;
        reinterpret_cast<double *>(R + RB_G0)[1] = g0i;
        reinterpret_cast<double *>(R + RB_G1)[0] = g1r;
        reinterpret_cast<double *>(R + RB_G1)[1] = g1i;
    }
}

hipError_t launch_prep_rb(const DevEvent *d_ev, const DevEvent &hev, const int32_t *d_edges,
                          const double *d_theta0, hipStream_t s)
{
    const int B = hev.rb_bins;
    if (B < 1 || hev.rb_nrows * RB_BINS_PER_ROW < B || !hev.rb_rows) return hipErrorInvalidValue;
    char *rows = const_cast<char *>(hev.rb_rows);
    prep_rb_nodes_kernel<<<(B + 1 + 255) / 256, 256, 0, s>>>(d_ev, d_edges, d_theta0, rows);
    const int waves = B * hev.n_det;
    prep_rb_sums_kernel<<<(waves + 3) / 4, 256, 0, s>>>(d_ev, d_edges, d_theta0, rows);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One point's log-likelihood by one wave (all lanes return the same value).
// ---------------------------------------------------------------------------
template <int ND, int MIXED = 0>
__device__ double wave_loglike_gw(const DevEvent &ev, const Src &p, const double2 *tab)
{
    Coef c;
    if (!make_coef<COEF_WAVE>(ev, p, c)) return -INFINITY;
    double R[ND], I[ND];
    wave_sums<ND, MIXED>(ev, c, R, I, tab);
    return combine<ND, MIXED>(ev, c, R, I);
}

template <int ND, int MIXED>
__global__ __launch_bounds__(256) void loglike_theta_kernel(const DevEvent *evp,
                                                            const double *theta, int64_t n,
                                                            double *out)
{
    __shared__ double2 s_tab[TAB_N];
    fill_sincos_tab(s_tab);  // FP64 paths and relative binning
    __syncthreads();
    const DevEvent &ev = *evp;
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;
    double th[NPAR];
    for (int j = 0; j < NPAR; ++j) th[j] = theta[i * NPAR + j];
    Src p = src_from_theta(th);
    double L = wave_loglike_gw<ND, MIXED>(ev, p, s_tab);
    if ((threadIdx.x & (WAVE - 1)) == 0) out[i] = L;
}

template <int ND, int MIXED>
__global__ __launch_bounds__(256) void loglike_u_kernel(const DevEvent *evp, const double *u,
                                                        int64_t n, double *out)
{
    __shared__ double2 s_tab[TAB_N];
    fill_sincos_tab(s_tab);  // FP64 paths and relative binning
    __syncthreads();
    const DevEvent &ev = *evp;
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;
    const int nd = ev.ndim;
    double uu[NPAR];
    for (int j = 0; j < NPAR; ++j) uu[j] = j < nd ? u[i * nd + j] : 0.5;
    double L;
    if (ev.likelihood == 1) {
        L = toy_loglike(ev, uu);
    } else {
        Src p = src_from_u(ev, uu);
        L = wave_loglike_gw<ND, MIXED>(ev, p, s_tab);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) out[i] = L;
}

template <int MIXED>
static void launch_ll_theta(const DevEvent *d_ev, int n_det, const double *theta, int64_t n,
                            double *out, hipStream_t s)
{
    dim3 grid((unsigned)((n + 3) / 4)), block(256);
    switch (n_det) {
    case 1: loglike_theta_kernel<1, MIXED><<<grid, block, 0, s>>>(d_ev, theta, n, out); break;
    case 2: loglike_theta_kernel<2, MIXED><<<grid, block, 0, s>>>(d_ev, theta, n, out); break;
    default: loglike_theta_kernel<3, MIXED><<<grid, block, 0, s>>>(d_ev, theta, n, out); break;
    }
}

template <int MIXED>
static void launch_ll_u(const DevEvent *d_ev, int n_det, const double *u, int64_t n, double *out,
                        hipStream_t s)
{
    dim3 grid((unsigned)((n + 3) / 4)), block(256);
    switch (n_det) {
    case 1: loglike_u_kernel<1, MIXED><<<grid, block, 0, s>>>(d_ev, u, n, out); break;
    case 2: loglike_u_kernel<2, MIXED><<<grid, block, 0, s>>>(d_ev, u, n, out); break;
    default: loglike_u_kernel<3, MIXED><<<grid, block, 0, s>>>(d_ev, u, n, out); break;
    }
}

hipError_t launch_loglike_theta(const DevEvent *d_ev, int n_det, const double *theta, int64_t n,
                                double *out, int mixed, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (mixed)
        launch_ll_theta<1>(d_ev, n_det, theta, n, out, s);
    else
        launch_ll_theta<0>(d_ev, n_det, theta, n, out, s);
    return hipGetLastError();
}

hipError_t launch_loglike_u(const DevEvent *d_ev, int n_det, int ndim, const double *u, int64_t n,
                            double *out, int mixed, hipStream_t s)
{
    (void)ndim;
    if (n <= 0) return hipSuccess;
    if (mixed)
        launch_ll_u<1>(d_ev, n_det, u, n, out, s);
    else
        launch_ll_u<0>(d_ev, n_det, u, n, out, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Physical parameters of unit-cube points through the event's prior
// transforms (Sec. 4, Tab. 1): uniform ranges, d_L uniform in d_L^3 (cube
// root as in the likelihood, exp(ln(d_L^3) / 3)), theta_JN = arccos of a
// uniform cosine, dec = arcsin of a uniform sine; parameters the event does
// not sample take their fixed values.  One thread per point.
// ---------------------------------------------------------------------------
__global__ void theta_from_u_kernel(const DevEvent *evp, const double *u, int64_t n,
                                    double *theta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const DevEvent &ev = *evp;
    const int d = ev.ndim;
    double pr[NPAR];
#pragma unroll
    for (int j = 0; j < NPAR; ++j) pr[j] = j < d ? u[i * d + j] : 0.5;
    const Src p = src_from_u(ev, pr);
    double *t = theta + i * NPAR;
    t[0] = p.mc;
    t[1] = p.q;
    t[2] = p.chi1;
    t[3] = p.chi2;
    t[4] = p.dl_pending ? exp(log(p.dl3) * (1.0 / 3.0)) : p.dl;
    t[5] = acos(p.cosi);
    t[6] = p.ra;
    t[7] = asin(p.sindec);
    t[8] = p.psi;
    t[9] = p.phic;
    t[10] = p.tc;
}

hipError_t launch_theta_from_u(const DevEvent *d_ev, const double *u, int64_t n, double *theta,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    theta_from_u_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(d_ev, u, n, theta);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// init: live points from the prior.  Coordinate j of point i is word j % 4 of
// the Philox block with counter (j / 4, chain id (event, i), 0, INIT).
// One wave per point.
// ---------------------------------------------------------------------------
template <int ND, int MIXED>
__global__ __launch_bounds__(256) void init_live_kernel(const DevEvent *evs, int n_events,
                                                        int n_live, int ndim, uint64_t seed,
                                                        double *live_u, double *live_L)
{
    __shared__ double2 s_tab[TAB_N];
    fill_sincos_tab(s_tab);  // FP64 paths and relative binning
    __syncthreads();
    int64_t gi = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (gi >= (int64_t)n_events * n_live) return;
    int e = (int)(gi / n_live), i = (int)(gi % n_live);
    const DevEvent &ev = evs[e];
    double uu[NPAR];
    uint64_t cid = chain_id(e, i);
    for (int b = 0; b < (NPAR + 3) / 4; ++b) {
        if (4 * b < ndim) {
            U4 r = philox4x64((uint64_t)b, cid, 0, P_INIT, seed, 0);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (4 * b + w < NPAR) uu[4 * b + w] = u01(r.x[w]);
        }
    }
    for (int j = ndim; j < NPAR; ++j) uu[j] = 0.5;
    double L;
    if (ev.likelihood == 1) {
        L = toy_loglike(ev, uu);
    } else {
        Src p = src_from_u(ev, uu);
        L = wave_loglike_gw<ND, MIXED>(ev, p, s_tab);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        for (int j = 0; j < ndim; ++j) live_u[gi * ndim + j] = uu[j];
        live_L[gi] = L;
    }
}

template <int MIXED>
static void launch_init_m(const DevEvent *d_ev, int n_events, int n_live, int ndim, uint64_t seed,
                          double *live_u, double *live_L, int max_det, hipStream_t s)
{
    int64_t n = (int64_t)n_events * n_live;
    dim3 grid((unsigned)((n + 3) / 4)), block(256);
    switch (max_det) {
    case 1: init_live_kernel<1, MIXED><<<grid, block, 0, s>>>(d_ev, n_events, n_live, ndim, seed, live_u, live_L); break;
    case 2: init_live_kernel<2, MIXED><<<grid, block, 0, s>>>(d_ev, n_events, n_live, ndim, seed, live_u, live_L); break;
    default: init_live_kernel<3, MIXED><<<grid, block, 0, s>>>(d_ev, n_events, n_live, ndim, seed, live_u, live_L); break;
    }
}

hipError_t launch_init_live(const DevEvent *d_ev, int n_events, int n_live, int ndim,
                            uint64_t seed, int mixed, double *live_u, double *live_L, int max_det,
                            hipStream_t s)
{
    if (mixed)
        launch_init_m<1>(d_ev, n_events, n_live, ndim, seed, live_u, live_L, max_det, s);
    else
        launch_init_m<0>(d_ev, n_events, n_live, ndim, seed, live_u, live_L, max_det, s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// select: one workgroup per event.
// ---------------------------------------------------------------------------
constexpr int SEL_THREADS = 1024;
constexpr int SEL_MAX = 4096;

__device__ __forceinline__ bool key_less(double ka, int ia, double kb, int ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ double logaddexp(double a, double b)
{
    if (a == -INFINITY) return b;
    if (b == -INFINITY) return a;
    double m = a > b ? a : b;
    return m + log(exp(a - m) + exp(b - m));
}

// Block-wide max / sum of one double per thread (every thread gets the
// result); red holds one slot per wave.  Contains barriers.
__device__ double block_max(double v, double *red)
{
    for (int off = WAVE / 2; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < nw; ++i) r = fmax(r, red[i]);
    return r;
}

__device__ double block_sum(double v, double *red)
{
    for (int off = WAVE / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
    const int w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
    __syncthreads();
    double r = red[0];
    for (int i = 1; i < nw; ++i) r += red[i];
    return r;
}

__global__ __launch_bounds__(SEL_THREADS) void select_kernel(StepArgs A)
{
    __shared__ double key[SEL_MAX];
    __shared__ int idx[SEL_MAX];
    __shared__ double s_lx[SEL_MAX];  // log X before each deletion, then t_i = L_i + log w_i
    __shared__ double s_inv[SEL_MAX], s_inv2[SEL_MAX];  // 1 / n_i and 1 / n_i^2 of each deletion
    __shared__ double s_red[SEL_THREADS / WAVE];
    __shared__ double s_fin[1];
    __shared__ int p0_sh;
    const int e = blockIdx.x;
    const int tid = threadIdx.x;
    const int n = A.n_live, d = A.ndim, k = A.k;
    EvState &st = A.st[e];
    const double *Lc = A.live_L + (size_t)e * n;
    const double *Uc = A.live_u + (size_t)e * n * d;
    double *Ln = A.next_L + (size_t)e * n;
    double *Un = A.next_u + (size_t)e * n * d;

    if (!st.active || st.err) {
        // carry the live set over unchanged so the buffer swap is harmless
        for (int i = tid; i < n; i += blockDim.x) Ln[i] = Lc[i];
        for (int i = tid; i < n * d; i += blockDim.x) Un[i] = Uc[i];
        if (tid == 0) st.k_this = 0;
        return;
    }

    int P = 2;
    while (P < n) P <<= 1;
    for (int i = tid; i < P; i += blockDim.x) {
        key[i] = i < n ? Lc[i] : INFINITY;
        idx[i] = i < n ? i : 0x7fffffff;
    }
    if (tid == 0) p0_sh = n;
    __syncthreads();
    // bitonic sort of (logL, index) pairs, ascending
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = tid; i < P / 2; i += blockDim.x) {
                int lo = 2 * stride * (i / stride) + (i % stride);
                int hi = lo + stride;
                bool up = (lo & size) == 0;
                double ka = key[lo], kb = key[hi];
                int ia = idx[lo], ib = idx[hi];
                bool sw = up ? key_less(kb, ib, ka, ia) : key_less(ka, ia, kb, ib);
                if (sw) {
                    key[lo] = kb; key[hi] = ka;
                    idx[lo] = ib; idx[hi] = ia;
                }
            }
            __syncthreads();
        }
    }
    const double Lstar = key[k - 1];
    for (int r = k + tid; r < n; r += blockDim.x)
        if (key[r] > Lstar && (r == k || !(key[r - 1] > Lstar))) p0_sh = r;
    __syncthreads();
    const int p0 = p0_sh;
    const int m = n - p0;
    if (m < 2) {
        for (int i = tid; i < n; i += blockDim.x) Ln[i] = Lc[i];
        for (int i = tid; i < n * d; i += blockDim.x) Un[i] = Uc[i];
        if (tid == 0) {
            st.err = 1;
            st.k_this = 0;
        }
        return;
    }
    double *S = A.snap_u + (size_t)e * n * d;
    double *SL = A.snap_L + (size_t)e * n;
    for (int i = tid; i < m * d; i += blockDim.x) {
        int r = p0 + i / d, j = i % d;
        S[i] = Uc[(size_t)idx[r] * d + j];
    }
    for (int i = tid; i < m; i += blockDim.x) SL[i] = key[p0 + i];
    // survivors, in sorted order, open the next live set
    for (int i = tid; i < (n - k) * d; i += blockDim.x) {
        int r = k + i / d, j = i % d;
        Un[i] = Uc[(size_t)idx[r] * d + j];
    }
    for (int i = tid; i < n - k; i += blockDim.x) Ln[i] = key[k + i];
    // dead rows
    const int64_t nd0 = st.n_dead;
    double *Du = A.dead_u + ((size_t)e * A.dead_cap + nd0) * d;
    for (int i = tid; i < k * d; i += blockDim.x) {
        int r = i / d, j = i % d;
        Du[i] = Uc[(size_t)idx[r] * d + j];
    }
    // chain starts: a uniformly chosen survivor with logL > L*
    const uint64_t batch = (uint64_t)st.batch;
    double *Cu = A.chain_u + (size_t)e * n * d;
    double *CL = A.chain_L + (size_t)e * n;
    for (int c = tid; c < k; c += blockDim.x) {
        U4 r = philox4x64(0, chain_id(e, c), batch, P_START, A.seed, 0);
        int j = (int)floor(u01(r.x[0]) * m);
        int row = idx[p0 + j];
        for (int q = 0; q < d; ++q) Cu[(size_t)c * d + q] = Uc[(size_t)row * d + q];
        CL[c] = key[p0 + j];
    }
    // Evidence (deleted points in ascending order see n, n-1, ..., n-k+1
    // live points).  log X before each deletion comes from the same
    // sequential subtraction as the definition (thread 0, cheap); the
    // weights, the batch's log-sum-exp and the information sum are then
    // spread over the block.
    // (the quotients first, spread over the block: the serial loop then only
    // adds, in the same order and with the same values)
    for (int i = tid; i < k; i += blockDim.x) {
        const double nl = (double)(n - i);
        s_inv[i] = 1.0 / nl;
        s_inv2[i] = 1.0 / (nl * nl);
    }
    __syncthreads();
    if (tid == 0) {
        double logX = st.logX;
        double si = st.sum_in, si2 = st.sum_in2;
        for (int i = 0; i < k; ++i) {
            s_lx[i] = logX;
            logX -= s_inv[i];
            si += s_inv[i];
            si2 += s_inv2[i];
        }
        s_fin[0] = logX;
        st.sum_in = si;
        st.sum_in2 = si2;
    }
    __syncthreads();
    const int64_t nd_e = (int64_t)e * A.dead_cap + nd0;
    double tmax = -INFINITY;
    for (int i = tid; i < k; i += blockDim.x) {
        double nl = (double)(n - i);
        double logw = s_lx[i] + log(-expm1(-s_inv[i]));  // log(X_{i-1} - X_i)
        double L = key[i];
        double t = L + logw;
        A.dead_L[nd_e + i] = L;
        A.dead_logw[nd_e + i] = logw;
        A.dead_nlive[nd_e + i] = nl;
        s_lx[i] = t;
        tmax = fmax(tmax, t);
    }
    tmax = block_max(tmax, s_red);
    double s0 = 0.0, s1 = 0.0;
    if (tmax > -INFINITY) {
        for (int i = tid; i < k; i += blockDim.x) {
            double t = s_lx[i];
            if (t > -INFINITY) {
                double q = exp(t - tmax);
                s0 += q;
                s1 += q * key[i];
            }
        }
    }
    s0 = block_sum(s0, s_red);
    s1 = block_sum(s1, s_red);
    if (tid == 0) {
        const double logZ = st.logZ;
        const double lz_b = tmax > -INFINITY ? tmax + log(s0) : -INFINITY;
        const double logZ_new = logaddexp(logZ, lz_b);
        // sumH = sum_i p_i L_i with p_i = exp(t_i - logZ): rescale the old sum
        double sumH = logZ == -INFINITY ? 0.0 : st.sumH * exp(logZ - logZ_new);
        if (lz_b > -INFINITY) sumH += s1 * exp(tmax - logZ_new);
        st.logX = s_fin[0];
        st.logZ = logZ_new;
        st.sumH = sumH;
        st.n_dead = nd0 + k;
        st.Lstar = Lstar;
        st.m = m;
        st.k_this = k;
        st.walk_this = A.walk_override > 0 ? A.walk_override : st.W;
    }
}

__global__ __launch_bounds__(256) void order_kernel(StepArgs A, int32_t *order)
{
    const int E = A.n_events;
    auto cost = [&](int f) {
        const EvState &s = A.st[f];
        return (s.active && !s.err && s.k_this > 0) ? (double)s.walk_this * (double)A.ev[f].n_pad : 0.0;
    };
    for (int e = threadIdx.x; e < E; e += blockDim.x) {
        const double ce = cost(e);
        int r = 0;
        for (int f = 0; f < E; ++f) {
            const double cf = cost(f);
            r += (cf > ce || (cf == ce && f < e)) ? 1 : 0;
        }
        order[r] = e;
    }
}

hipError_t launch_order(const StepArgs &a, int32_t *order, hipStream_t s)
{
    order_kernel<<<1, 256, 0, s>>>(a, order);
    return hipGetLastError();
}

// One workgroup per replicate (App. A: the prior-volume shrinkages are
// random, t_i ~ Beta(n_i, 1)): log X runs over the deletions as a prefix sum
// (contiguous chunks per thread, chunk offsets by one thread in order), the
// weights log(X_{i-1} - X_i) = log X_{i-1} + log(-expm1(log t_i)) and the
// log-sum-exp of L_i + log w_i and of the final live term log X_n + log(mean
// exp(L_live)) are reduced over the block.
__global__ __launch_bounds__(256) void replicate_kernel(const double *dL, const double *dn, int64_t n,
                                                        const double *liveL, int n_live,
                                                        const double *U, uint64_t seed, double *out)
{
    __shared__ double s_off[256];
    __shared__ double s_red[256 / WAVE];
    const int r = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int64_t chunk = (n + nt - 1) / nt;
    const int64_t i0 = min((int64_t)tid * chunk, n), i1 = min(i0 + chunk, n);
    auto dlx = [&](int64_t i) {
        const double u = U ? U[(size_t)r * n + i]
                           : 1.0 - u01(philox4x64((uint64_t)i, (uint64_t)r, 0, P_REPL, seed, 0).x[0]);
        return log(u) / dn[i];
    };
    double sum = 0.0;
    for (int64_t i = i0; i < i1; ++i) sum += dlx(i);
    s_off[tid] = sum;
    __syncthreads();
    if (tid == 0) {
        double acc = 0.0;
        for (int t = 0; t < nt; ++t) {
            const double v = s_off[t];
            s_off[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    // per-thread weights: t_i = L_i + log X_{i-1} + log(-expm1(dlx_i))
    double lx = s_off[tid];
    double tmax = -INFINITY;
    for (int64_t i = i0; i < i1; ++i) {
        const double d = dlx(i);
        tmax = fmax(tmax, dL[i] + lx + log(-expm1(d)));
        lx += d;
    }
    // log X after the last deletion, and the live term
    __shared__ double s_lxn, s_lme;
    if (tid == nt - 1) s_lxn = lx;
    if (tid == 0) {
        double mx = -INFINITY;
        for (int j = 0; j < n_live; ++j) mx = fmax(mx, liveL[j]);
        double se = 0.0;
        for (int j = 0; j < n_live; ++j) se += exp(liveL[j] - mx);
        s_lme = mx + log(se / n_live);
    }
    __syncthreads();
    const double tlive = s_lxn + s_lme;
    const double m = fmax(block_max(tmax, s_red), tlive);
    lx = s_off[tid];
    double se = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
        const double d = dlx(i);
        se += exp(dL[i] + lx + log(-expm1(d)) - m);
        lx += d;
    }
    se = block_sum(se, s_red);
    if (tid == 0) out[r] = m + log(se + exp(tlive - m));
}

hipError_t launch_replicates(const double *dead_L, const double *dead_nlive, int64_t n_dead,
                             const double *live_L, int n_live, const double *U, uint64_t seed,
                             int R, double *out, hipStream_t s)
{
    replicate_kernel<<<R, 256, 0, s>>>(dead_L, dead_nlive, n_dead, live_L, n_live, U, seed, out);
    return hipGetLastError();
}

hipError_t launch_select(const StepArgs &a, hipStream_t s)
{
    select_kernel<<<a.n_events, SEL_THREADS, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// finish: one workgroup per event.
// ---------------------------------------------------------------------------
__device__ int32_t tune_walk(int32_t W, int64_t sum_acc, int32_t k, double delay, int32_t naccept,
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

__global__ __launch_bounds__(256) void finish_kernel(StepArgs A)
{
    __shared__ int64_t s_acc[256], s_calls[256], s_oob[256], s_spec[256];
    __shared__ double s_red[256];
    const int e = blockIdx.x, tid = threadIdx.x;
    EvState &st = A.st[e];
    if (!st.active || st.err || st.k_this == 0) return;
    const int n = A.n_live, k = st.k_this;
    int64_t a = 0, c = 0, o = 0, sp = 0;
    for (int i = tid; i < k; i += blockDim.x) {
        const int64_t *cs = A.chain_stats + ((size_t)e * n + i) * 4;
        a += cs[0];
        c += cs[1];
        o += cs[2];
        sp += cs[3];
    }
    s_acc[tid] = a;
    s_calls[tid] = c;
    s_oob[tid] = o;
    s_spec[tid] = sp;
    const double *L = A.next_L + (size_t)e * n;
    double mx = -INFINITY;
    for (int i = tid; i < n; i += blockDim.x) mx = fmax(mx, L[i]);
    s_red[tid] = mx;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) {
            s_acc[tid] += s_acc[tid + off];
            s_calls[tid] += s_calls[tid + off];
            s_oob[tid] += s_oob[tid + off];
            s_spec[tid] += s_spec[tid + off];
            s_red[tid] = fmax(s_red[tid], s_red[tid + off]);
        }
        __syncthreads();
    }
    const double maxL = s_red[0];
    __syncthreads();
    double se = 0.0;
    for (int i = tid; i < n; i += blockDim.x) se += exp(L[i] - maxL);
    s_red[tid] = se;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (tid < off) s_red[tid] += s_red[tid + off];
        __syncthreads();
    }
    if (tid == 0) {
        const int W = st.walk_this;
        const int64_t acc = s_acc[0], calls = s_calls[0], oob = s_oob[0];
        st.n_acc += acc;
        st.n_calls += calls;
        st.n_oob += oob;
        st.n_spec += s_spec[0];
        st.n_steps += (int64_t)k * W;
        st.last_acc = acc;
        st.last_calls = calls;
        st.W = tune_walk(W, acc, k, A.delay, A.naccept, A.maxmcmc);
        st.n_capped = st.W >= A.maxmcmc ? st.n_capped + 1 : 0;
        st.batch += 1;
        const double lme = maxL + log(s_red[0] / (double)n);
        st.maxL = maxL;
        st.lme = lme;
        const double logZ = st.logZ;
        const double dlogZ = logaddexp(logZ, st.logX + maxL) - logZ;
        const double lfrac = st.logX + lme - logZ;
        st.dlogZ = dlogZ;
        st.log_frac = lfrac;
        const bool conv = A.term_kind == 0 ? (dlogZ < A.term_thr) : (lfrac < log(A.term_thr));
        if (conv) {
            st.converged = 1;
            st.active = 0;
        }
    }
}

hipError_t launch_finish(const StepArgs &a, hipStream_t s)
{
    finish_kernel<<<a.n_events, 256, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// signal: h_d(f_k) = alpha_d f^(-7/6) exp(-2 pi i r_d(f_k)) for one theta.
// ---------------------------------------------------------------------------
__global__ void signal_kernel(const DevEvent *evp, const double *theta, double *h)
{
    const DevEvent &ev = *evp;
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ev.n_bins) return;
    double th[NPAR];
    for (int j = 0; j < NPAR; ++j) th[j] = theta[j];
    Src p = src_from_theta(th);
    Coef c;
    bool ok = make_coef<COEF_LANE>(ev, p, c);
    double f = (double)k * ev.df + ev.f_lo;
    double s = cbrt(f);
    double t = 1.0 / s, L = log(f);
    double amp = pow(f, -7.0 / 6.0);
    double r = phase_rev(c, t, s, L);
    for (int d = 0; d < ev.n_det; ++d) {
        double re = 0.0, im = 0.0;
        if (ok) {
            double sn, cs;
            sincos_rev(fma(f, c.tau[d], r), &sn, &cs);
            // alpha (cos - i sin) f^-7/6
            re = amp * (c.ar[d] * cs + c.ai[d] * sn);
            im = amp * (c.ai[d] * cs - c.ar[d] * sn);
        }
        h[2 * ((size_t)d * ev.n_bins + k)] = re;
        h[2 * ((size_t)d * ev.n_bins + k) + 1] = im;
    }
}

hipError_t launch_signal(const DevEvent *d_ev, int n_bins, int n_det, const double *theta,
                         double *h, hipStream_t s)
{
    (void)n_det;
    signal_kernel<<<(n_bins + 255) / 256, 256, 0, s>>>(d_ev, theta, h);
    return hipGetLastError();
}

}  // namespace nsmi
