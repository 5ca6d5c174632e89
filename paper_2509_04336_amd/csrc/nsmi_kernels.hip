// Kernels of the MI355X acceptance-walk nested sampler (gfx950, wave64).
//
//   prep_event   per-bin phase basis, whitened weights, K_d           (init)
//   init_live    prior draws (Philox purpose 7) and their likelihood  (init)
//   loglike_*    one wave per point, bins strided over the lanes
//   select       per event: sort live logL, delete k, L*, survivor
//                snapshot, chain start picks, dead-point evidence update
//   walk         one workgroup per chain: W differential-evolution steps,
//                each a full likelihood evaluation, strict L > L*
//   finish       per event: walk statistics, walk-length retune,
//                termination metrics
#include <hip/hip_runtime.h>

#include "nsmi_kernels.h"
#include "nsmi_mlp.h"

namespace nsmi {

// ---------------------------------------------------------------------------
// init: per-bin tables
// ---------------------------------------------------------------------------
// Bins N <= k < NP continue the frequency grid in the basis tables; their
// weights stay zero (the weight rows are cleared before this kernel).
__global__ void prep_bins_kernel(int N, int NP, int ND, double f_lo, double df, const double *data,
                                 const double *psd, double *tb, double *sb, double *lb,
                                 double2 *w, float2 *w32, double wscale)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= NP) return;
    double f = (double)k * df + f_lo;
    double s = cbrt(f);
    tb[k] = 1.0 / s;
    sb[k] = s;
    lb[k] = log(f);
    if (k >= N) return;
    double fac0 = 4.0 * df * pow(f, -7.0 / 6.0);
    for (int d = 0; d < ND; ++d) {
        double S = psd[(size_t)d * N + k];
        double fac = fac0 / S;
        double dr = data[2 * ((size_t)d * N + k)];
        double di = data[2 * ((size_t)d * N + k) + 1];
        w[(size_t)d * NP + k] = make_double2(fac * dr, -fac * di);  // 4 df conj(d) f^-7/6 / S
        w32[(size_t)d * NP + k] = make_float2((float)(fac * dr * wscale), (float)(-fac * di * wscale));
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
                             double *tb, double *sb, double *lb, double2 *w, float2 *w32,
                             double *K_out, hipStream_t s)
{
    int N = hev.n_bins, NP = hev.n_pad;
    if (NP < N || NP % WAVE != 0) return hipErrorInvalidValue;
    prep_bins_kernel<<<(NP + 255) / 256, 256, 0, s>>>(N, NP, hev.n_det, hev.f_lo, hev.df, d_data,
                                                      d_psd, tb, sb, lb, w, w32, hev.wscale);
    prep_K_kernel<<<hev.n_det, 1024, 0, s>>>(N, hev.f_lo, hev.df, d_psd, K_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One point's log-likelihood by one wave (all lanes return the same value).
// ---------------------------------------------------------------------------
template <int ND, int MIXED = 0>
__device__ double wave_loglike_gw(const DevEvent &ev, const Src &p)
{
    Coef c;
    if (!make_coef<true>(ev, p, c)) return -INFINITY;
    double Zr[ND], Zi[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) Zr[d] = Zi[d] = 0.0;
    accumulate<ND, MIXED>(ev, c, Zr, Zi);
    double R[ND], I[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        R[d] = wave_sum(Zr[d]);
        I[d] = wave_sum(Zi[d]);
    }
    return combine<ND, MIXED>(ev, c, R, I);
}

template <int ND, int MIXED>
__global__ __launch_bounds__(256) void loglike_theta_kernel(const DevEvent *evp,
                                                            const double *theta, int64_t n,
                                                            double *out)
{
    const DevEvent &ev = *evp;
    int64_t i = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (i >= n) return;
    double th[NPAR];
    for (int j = 0; j < NPAR; ++j) th[j] = theta[i * NPAR + j];
    Src p = src_from_theta(th);
    double L = wave_loglike_gw<ND, MIXED>(ev, p);
    if ((threadIdx.x & (WAVE - 1)) == 0) out[i] = L;
}

template <int ND, int MIXED>
__global__ __launch_bounds__(256) void loglike_u_kernel(const DevEvent *evp, const double *u,
                                                        int64_t n, double *out)
{
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
        L = wave_loglike_gw<ND, MIXED>(ev, p);
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
// init: live points from the prior.  Coordinate j of point i is word j % 4 of
// the Philox block with counter (j / 4, chain id (event, i), 0, INIT).
// One wave per point.
// ---------------------------------------------------------------------------
template <int ND, int MIXED>
__global__ __launch_bounds__(256) void init_live_kernel(const DevEvent *evs, int n_events,
                                                        int n_live, int ndim, uint64_t seed,
                                                        double *live_u, double *live_L)
{
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
        L = wave_loglike_gw<ND, MIXED>(ev, p);
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

__global__ __launch_bounds__(SEL_THREADS) void select_kernel(StepArgs A)
{
    __shared__ double key[SEL_MAX];
    __shared__ int idx[SEL_MAX];
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
    // evidence: deleted points in ascending order see n, n-1, ..., n-k+1 live
    if (tid == 0) {
        double logX = st.logX, logZ = st.logZ, sumH = st.sumH;
        double *DL = A.dead_L + (size_t)e * A.dead_cap + nd0;
        double *Dw = A.dead_logw + (size_t)e * A.dead_cap + nd0;
        double *Dn = A.dead_nlive + (size_t)e * A.dead_cap + nd0;
        for (int i = 0; i < k; ++i) {
            double nl = (double)(n - i);
            double logX_new = logX - 1.0 / nl;
            double logw = logX + log(-expm1(-1.0 / nl));
            double L = key[i];
            double t = L + logw;
            double logZ_new = logaddexp(logZ, t);
            if (logZ == -INFINITY)
                sumH = L;
            else
                sumH = sumH * exp(logZ - logZ_new) + exp(t - logZ_new) * L;
            logZ = logZ_new;
            logX = logX_new;
            DL[i] = L;
            Dw[i] = logw;
            Dn[i] = nl;
        }
        st.logX = logX;
        st.logZ = logZ;
        st.sumH = sumH;
        st.n_dead = nd0 + k;
        st.Lstar = Lstar;
        st.m = m;
        st.k_this = k;
        st.walk_this = A.walk_override > 0 ? A.walk_override : st.W;
    }
}

hipError_t launch_select(const StepArgs &a, hipStream_t s)
{
    select_kernel<<<a.n_events, SEL_THREADS, 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// walk: one workgroup (WPC waves) per chain.
//
// Random draws for 64 consecutive steps are generated lane-parallel (lane l
// makes the draws of step s0 + l) and broadcast with readlane, so each wave
// pays one Philox pair and four logarithms per 64 steps.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ double readlane_d(double v, int l)
{
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    return __hiloint2double(hi, lo);
}

// Coefficients of one unit-cube point for the calling wave (results in the
// caller's registers).  Out of line for the same register reason.
__device__ __noinline__ void point_setup_local(const DevEvent *ev, const double *u, Coef *out,
                                               int *flag)
{
    double pr[NPAR];
#pragma unroll
    for (int j = 0; j < NPAR; ++j) pr[j] = u[j];
    Src p = src_from_u(*ev, pr);
    *flag = make_coef<true>(*ev, p, *out) ? 0 : 2;
}

// One workgroup of SPEC waves per chain, evaluating proposals
// speculatively.  Wave 0 owns the chain state and makes the random draws of
// 64 consecutive steps lane-parallel (lane l owns step s0 + l).  While the
// chain's point does not move, the proposals of those steps are independent:
// wave 0 forms them all at once, skips the ones that leave the unit cube
// (rejected without a likelihood call) and hands the next SPEC in-cube
// proposals to the SPEC waves, one each, drawing further windows when one
// window holds fewer than SPEC of them.  Every wave computes its own
// coefficients and the full bin sum of its proposal.  Wave 0 then walks the
// candidates in step order exactly as the sequential chain would: each is one
// likelihood call; the first with L > L* is accepted and the candidates after
// it are discarded (they assumed the earlier steps were rejected).  The chain,
// its counters and its random numbers are those of the one-step-at-a-time
// walk; only discarded evaluations are extra work (counted in n_spec).
template <int SPEC, int ND, int MIXED>
__global__ __launch_bounds__(64 * SPEC) void walk_kernel(StepArgs A)
{
    __shared__ DevEvent s_ev;
    __shared__ double s_u[NPAR];
    __shared__ double s_p[SPEC][NPAR];
    __shared__ double s_L[SPEC];
    __shared__ int s_step[SPEC];
    __shared__ int s_cnt;
    const int chain = blockIdx.x;
    const int k = A.k;
    const int e = chain / k, c = chain % k;
    EvState &st = A.st[e];
    if (!st.active || st.err || st.k_this == 0) return;
    const int n = A.n_live, d = A.ndim;
    const int m = st.m;
    const int W = st.walk_this;
    const double Lstar = st.Lstar;
    const uint64_t batch = (uint64_t)st.batch;
    const uint64_t cid = chain_id(e, c);
    const double *S = A.snap_u + (size_t)e * n * d;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = tid / WAVE;
    const double gscale = 2.38 / sqrt(2.0 * d);

    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(A.ev + e);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_ev);
        for (int i = tid; i < (int)(sizeof(DevEvent) / 4); i += blockDim.x) dst[i] = src[i];
    }
    if (tid < NPAR) s_u[tid] = tid < d ? A.chain_u[((size_t)e * n + c) * d + tid] : 0.5;
    for (int i = tid; i < SPEC * NPAR; i += blockDim.x) s_p[i / NPAR][i % NPAR] = 0.5;
    __syncthreads();
    const int likelihood = s_ev.likelihood;
    double L = A.chain_L[(size_t)e * n + c];
    int64_t n_acc = 0, n_calls = 0, n_oob = 0, n_spec = 0;

    int s = 0;        // next walk step of the sequential chain (wave 0)
    int s0 = -WAVE;   // first step of the current draw window
    int my_a = 0, my_b = 0;
    double my_g = 1.0;
    for (;;) {
        // -- wave 0: the next SPEC in-cube proposals from the current point
        if (wave == 0) {
            int cnt = 0;
            int sp = s;  // scan position: candidates may span several windows
            while (sp < W && cnt < SPEC) {
                if (sp < s0 || sp >= s0 + WAVE) {
                    s0 = sp & ~(WAVE - 1);
                    const int t = s0 + lane;
                    if (t < W) {
                        U4 ra = philox4x64((uint64_t)t, cid, batch, P_WALK_A, A.seed, 0);
                        U4 rb = philox4x64((uint64_t)t, cid, batch, P_WALK_B, A.seed, 0);
                        double umode = u01(ra.x[0]);
                        my_a = (int)floor(u01(ra.x[1]) * m);
                        my_b = (int)floor(u01(ra.x[2]) * (m - 1));
                        if (my_b >= my_a) my_b += 1;
                        if (umode < 0.5) {
                            my_g = 1.0;
                        } else {
                            double g = 0.0;
                            for (int i = 0; i < 4; ++i) g += -0.25 * log(1.0 - u01(rb.x[i]));
                            my_g = gscale * g;
                        }
                    }
                }
                const int t = s0 + lane;
                bool ok = t >= sp && t < W;
                double pv[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) {
                    if (j < d) {
                        double diff = S[(size_t)my_a * d + j] - S[(size_t)my_b * d + j];
                        double v = fma(my_g, diff, s_u[j]);
                        if (is_periodic(d, j)) {
                            v = v - floor(v);
                        } else if (v < 0.0 || v > 1.0) {
                            ok = false;
                        }
                        pv[j] = v;
                    } else {
                        pv[j] = 0.5;
                    }
                }
                uint64_t mask = __ballot(ok);
                const int wend = min(s0 + WAVE, W);
                if (mask != 0) {
                    // rank of this lane among the in-cube proposals found so far
                    const uint64_t below = lane == 0 ? 0ull : (mask & (~0ull >> (WAVE - lane)));
                    const int rank = cnt + __popcll(below);
                    if (ok && rank < SPEC) {
#pragma unroll
                        for (int j = 0; j < NPAR; ++j)
                            if (j < d) s_p[rank][j] = pv[j];
                        s_step[rank] = t;
                    }
                    cnt = min(cnt + __popcll(mask), SPEC);
                } else if (cnt == 0) {
                    // no candidate before this window's end: its steps are
                    // rejected whatever the later candidates decide
                    n_oob += wend - s;
                    s = wend;
                }
                sp = wend;
            }
            if (lane == 0) s_cnt = cnt;
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (cnt == 0) break;
        // -- every wave with a candidate evaluates it
        if (wave < cnt) {
            double Lp;
            if (likelihood == 1) {
                double pr[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) pr[j] = s_p[wave][j];
                Lp = toy_loglike(s_ev, pr);
            } else {
                Coef cf;
                int fl;
                point_setup_local(&s_ev, s_p[wave], &cf, &fl);
                double Zr[ND], Zi[ND];
#pragma unroll
                for (int q = 0; q < ND; ++q) Zr[q] = Zi[q] = 0.0;
                if (fl == 0) accumulate<ND, MIXED>(s_ev, cf, Zr, Zi);
                double R[ND], I[ND];
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    R[q] = wave_sum(Zr[q]);
                    I[q] = wave_sum(Zi[q]);
                }
                Lp = fl == 0 ? combine<ND, MIXED>(s_ev, cf, R, I) : -INFINITY;
            }
            if (lane == 0) {
                s_L[wave] = Lp;
                if (A.hv_count) {
                    unsigned long long slot = atomicAdd(A.hv_count, 1ull);
                    if ((int64_t)slot < A.hv_cap) {
                        for (int j = 0; j < d; ++j) A.hv_u[slot * d + j] = s_p[wave][j];
                        A.hv_L[slot] = Lp;
                    }
                }
            }
        }
        __syncthreads();
        // -- wave 0: resolve the candidates in step order
        if (wave == 0) {
            int i = 0;
            for (; i < cnt; ++i) {
                const int st_i = s_step[i];
                n_oob += st_i - s;
                s = st_i + 1;
                ++n_calls;
                const double Li = s_L[i];
                if (Li > Lstar) {
                    if (lane < d) s_u[lane] = s_p[i][lane];
                    L = Li;
                    ++n_acc;
                    ++i;
                    break;
                }
            }
            n_spec += cnt - i;
        }
        // no barrier here: the other waves next read shared state after the
        // barrier that follows wave 0's next search
    }
    if (tid == 0) {
        const size_t row = (size_t)e * n + (n - k + c);
        for (int j = 0; j < d; ++j) A.next_u[row * d + j] = s_u[j];
        A.next_L[row] = L;
        int64_t *cs = A.chain_stats + ((size_t)e * n + c) * 4;
        cs[0] = n_acc;
        cs[1] = n_calls;
        cs[2] = n_oob;
        cs[3] = n_spec;
    }
}

// ---------------------------------------------------------------------------
// Delayed acceptance with the surrogate (Christen & Fox 2005).  For each
// in-cube proposal u' the screen density pi(x) = sigmoid((s(x) - L* + m)/tau)
// (strictly positive) gives
//   stage 1: continue only if U1 < min(1, pi(u') / pi(u))   (no exact call)
//   stage 2: exact L(u'); accept iff L(u') > L* and U2 < min(1, pi(u) / pi(u'))
// with (U1, U2) the first two words of the Philox block (step, chain, batch,
// DA2).  The DE proposal is symmetric (frozen donors), so the chain keeps the
// constrained prior as its invariant distribution: the exact likelihood still
// decides every accepted point.  With pi constant it is the plain walk.
// ---------------------------------------------------------------------------
constexpr int DA_ROWS = 16;  // MFMA rows: up to 15 candidates + the current point

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// log pi(x) = -log(1 + exp(-z)), z = (s - L* + m) / tau
__device__ __forceinline__ double log_screen(double s_hat, double Lstar, double margin, double temp)
{
    double z = (s_hat - Lstar + margin) / temp;
    return z >= 0.0 ? -log1p(exp(-z)) : z - log1p(exp(z));
}

// Surrogate of DA_ROWS rows held in LDS X[16][32] (bf16): three hidden layers
// with MFMA, column blocks of 16 shared out over the SPEC waves, activations
// in LDS; row outputs mu + sigma y into out[16].  Called by every thread of
// the workgroup (contains barriers).
template <int SPEC>
__device__ void surrogate16(const StepArgs &A, const __bf16 *X, __bf16 *H1, __bf16 *H2,
                            double *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const float *P = A.mP;
    // layer 1: K = 32
    for (int cb = wave; cb < MLP_H / 16; cb += SPEC) {
        bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(X + r * MLP_KIN + 8 * q);
        bf16x8_t b = *reinterpret_cast<const bf16x8_t *>(A.mW1p + (size_t)(cb * 16 + r) * MLP_KIN + 8 * q);
        f32x4_t acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, (f32x4_t){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        const int col = cb * 16 + r;
        const float bias = P[MLP_OFF_B1 + col];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float z = acc[i] + bias;
            H1[(4 * q + i) * MLP_H + col] = (__bf16)(z / (1.0f + __expf(-z)));
        }
    }
    __syncthreads();
    // layers 2 and 3: K = 256
    const __bf16 *Win[2] = {A.mW2, A.mW3};
    const int64_t boff[2] = {MLP_OFF_B2, MLP_OFF_B3};
    __bf16 *src = H1, *dst = H2;
    for (int l = 0; l < 2; ++l) {
        for (int cb = wave; cb < MLP_H / 16; cb += SPEC) {
            f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
            const __bf16 *Wrow = Win[l] + (size_t)(cb * 16 + r) * MLP_H;
#pragma unroll
            for (int k0 = 0; k0 < MLP_H; k0 += 32) {
                bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(src + r * MLP_H + k0 + 8 * q);
                bf16x8_t b = *reinterpret_cast<const bf16x8_t *>(Wrow + k0 + 8 * q);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
            const int col = cb * 16 + r;
            const float bias = P[boff[l] + col];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float z = acc[i] + bias;
                dst[(4 * q + i) * MLP_H + col] = (__bf16)(z / (1.0f + __expf(-z)));
            }
        }
        __syncthreads();
        __bf16 *t = src;
        src = dst;
        dst = t;
    }
    // output layer (src holds h3): row lane / 4, quarter lane % 4
    if (wave == 0) {
        const int row = lane >> 2, part = lane & 3;
        float acc = 0.f;
        for (int j = part * 64; j < part * 64 + 64; ++j) acc += P[MLP_OFF_W4 + j] * (float)src[row * MLP_H + j];
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (part == 0) out[row] = A.m_mu + A.m_sig * (double)(acc + P[MLP_OFF_B4]);
    }
    __syncthreads();
}

template <int SPEC, int ND, int MIXED>
__global__ __launch_bounds__(64 * SPEC) void walk_da_kernel(StepArgs A)
{
    __shared__ DevEvent s_ev;
    __shared__ double s_u[NPAR];
    __shared__ double s_p[DA_ROWS][NPAR];
    __shared__ int s_step[DA_ROWS];
    __shared__ double s_u1[DA_ROWS], s_u2[DA_ROWS];
    __shared__ double s_shat[DA_ROWS];
    __shared__ double s_L[SPEC];
    __shared__ int s_eval[SPEC];     // candidate index evaluated by each wave
    __shared__ int s_cnt, s_neval;
    __shared__ uint32_t s_pass;      // stage-1 outcome per candidate (bit i)
    __shared__ __attribute__((aligned(16))) __bf16 s_X[DA_ROWS * MLP_KIN];
    __shared__ __attribute__((aligned(16))) __bf16 s_H1[DA_ROWS * MLP_H];
    __shared__ __attribute__((aligned(16))) __bf16 s_H2[DA_ROWS * MLP_H];
    const int chain = blockIdx.x;
    const int k = A.k;
    const int e = chain / k, c = chain % k;
    EvState &st = A.st[e];
    if (!st.active || st.err || st.k_this == 0) return;
    const int n = A.n_live, d = A.ndim;
    const int m = st.m;
    const int W = st.walk_this;
    const double Lstar = st.Lstar;
    const uint64_t batch = (uint64_t)st.batch;
    const uint64_t cid = chain_id(e, c);
    const double *S = A.snap_u + (size_t)e * n * d;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int wave = tid / WAVE;
    const double gscale = 2.38 / sqrt(2.0 * d);

    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(A.ev + e);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_ev);
        for (int i = tid; i < (int)(sizeof(DevEvent) / 4); i += blockDim.x) dst[i] = src[i];
    }
    if (tid < NPAR) s_u[tid] = tid < d ? A.chain_u[((size_t)e * n + c) * d + tid] : 0.5;
    for (int i = tid; i < DA_ROWS * NPAR; i += blockDim.x) s_p[i / NPAR][i % NPAR] = 0.5;
    __syncthreads();
    const int likelihood = s_ev.likelihood;
    double L = A.chain_L[(size_t)e * n + c];
    double lpi_cur = 0.0;       // log screen density of the current point (wave 0)
    bool have_cur = false;
    int64_t n_acc = 0, n_calls = 0, n_oob = 0, n_spec = 0, n_saved = 0;

    int s = 0, s0 = -WAVE;
    int my_a = 0, my_b = 0;
    double my_g = 1.0, my_u1 = 0.0, my_u2 = 0.0;
    for (;;) {
        // -- wave 0: up to DA_ROWS - 1 in-cube candidates of the current window
        if (wave == 0) {
            int cnt = 0;
            while (s < W) {
                if (s >= s0 + WAVE) {
                    s0 = s & ~(WAVE - 1);
                    const int t = s0 + lane;
                    if (t < W) {
                        U4 ra = philox4x64((uint64_t)t, cid, batch, P_WALK_A, A.seed, 0);
                        U4 rb = philox4x64((uint64_t)t, cid, batch, P_WALK_B, A.seed, 0);
                        U4 rd = philox4x64((uint64_t)t, cid, batch, P_DA2, A.seed, 0);
                        double umode = u01(ra.x[0]);
                        my_a = (int)floor(u01(ra.x[1]) * m);
                        my_b = (int)floor(u01(ra.x[2]) * (m - 1));
                        if (my_b >= my_a) my_b += 1;
                        if (umode < 0.5) {
                            my_g = 1.0;
                        } else {
                            double g = 0.0;
                            for (int i = 0; i < 4; ++i) g += -0.25 * log(1.0 - u01(rb.x[i]));
                            my_g = gscale * g;
                        }
                        my_u1 = u01(rd.x[0]);
                        my_u2 = u01(rd.x[1]);
                    }
                }
                const int t = s0 + lane;
                bool ok = t >= s && t < W;
                double pv[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) {
                    if (j < d) {
                        double diff = S[(size_t)my_a * d + j] - S[(size_t)my_b * d + j];
                        double v = fma(my_g, diff, s_u[j]);
                        if (is_periodic(d, j)) {
                            v = v - floor(v);
                        } else if (v < 0.0 || v > 1.0) {
                            ok = false;
                        }
                        pv[j] = v;
                    } else {
                        pv[j] = 0.5;
                    }
                }
                uint64_t mask = __ballot(ok);
                const int wend = min(s0 + WAVE, W);
                if (mask == 0) {
                    n_oob += wend - s;
                    s = wend;
                    continue;
                }
                const uint64_t below = lane == 0 ? 0ull : (mask & (~0ull >> (WAVE - lane)));
                const int rank = __popcll(below);
                if (ok && rank < DA_ROWS - 1) {
#pragma unroll
                    for (int j = 0; j < NPAR; ++j)
                        if (j < d) s_p[rank][j] = pv[j];
                    s_step[rank] = t;
                    s_u1[rank] = my_u1;
                    s_u2[rank] = my_u2;
                }
                cnt = min(__popcll(mask), DA_ROWS - 1);
                break;
            }
            if (lane == 0) s_cnt = cnt;
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (cnt == 0) break;
        // -- surrogate on the candidates (rows 0..cnt-1) and the current point (row 15)
        for (int i = tid; i < DA_ROWS * MLP_KIN; i += blockDim.x) {
            const int row = i / MLP_KIN, col = i % MLP_KIN;
            float v = 0.0f;
            if (col < d) {
                double x = row == DA_ROWS - 1 ? s_u[col] : (row < cnt ? s_p[row][col] : 0.0);
                v = ((float)x - A.m_in_mu[col]) * A.m_in_isig[col];
            }
            s_X[i] = (__bf16)v;
        }
        __syncthreads();
        surrogate16<SPEC>(A, s_X, s_H1, s_H2, s_shat);
        // -- wave 0: stage-1 screen in step order, choose up to SPEC exact calls
        if (wave == 0) {
            if (!have_cur) {
                lpi_cur = log_screen(s_shat[DA_ROWS - 1], Lstar, A.da_margin, A.da_temp);
                have_cur = true;
            }
            bool pass = false;
            if (lane < cnt) {
                double lpi = log_screen(s_shat[lane], Lstar, A.da_margin, A.da_temp);
                pass = log(s_u1[lane]) < lpi - lpi_cur;
            }
            const uint64_t pm = __ballot(pass);
            const uint64_t below = lane == 0 ? 0ull : (pm & (~0ull >> (WAVE - lane)));
            const int rank = __popcll(below);
            if (pass && rank < SPEC) s_eval[rank] = lane;
            if (lane == 0) {
                s_neval = min(__popcll(pm), SPEC);
                s_pass = (uint32_t)(pm & 0xffffull);
            }
        }
        __syncthreads();
        const int neval = s_neval;
        // -- exact evaluations of the passing candidates, one per wave
        if (wave < neval) {
            const int ci = s_eval[wave];
            double Lp;
            if (likelihood == 1) {
                double pr[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) pr[j] = s_p[ci][j];
                Lp = toy_loglike(s_ev, pr);
            } else {
                Coef cf;
                int fl;
                point_setup_local(&s_ev, s_p[ci], &cf, &fl);
                double Zr[ND], Zi[ND];
#pragma unroll
                for (int q = 0; q < ND; ++q) Zr[q] = Zi[q] = 0.0;
                if (fl == 0) accumulate<ND, MIXED>(s_ev, cf, Zr, Zi);
                double R[ND], I[ND];
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    R[q] = wave_sum(Zr[q]);
                    I[q] = wave_sum(Zi[q]);
                }
                Lp = fl == 0 ? combine<ND, MIXED>(s_ev, cf, R, I) : -INFINITY;
            }
            if (lane == 0) {
                s_L[wave] = Lp;
                if (A.hv_count) {
                    unsigned long long slot = atomicAdd(A.hv_count, 1ull);
                    if ((int64_t)slot < A.hv_cap) {
                        for (int j = 0; j < d; ++j) A.hv_u[slot * d + j] = s_p[ci][j];
                        A.hv_L[slot] = Lp;
                    }
                }
            }
        }
        __syncthreads();
        // -- wave 0: resolve in step order
        if (wave == 0) {
            const uint32_t pm = s_pass;
            int ev_i = 0;  // next evaluated candidate
            int i = 0;
            for (; i < cnt; ++i) {
                const bool pass = (pm >> i) & 1u;
                if (pass && ev_i >= neval) break;  // not evaluated yet: next round
                const int st_i = s_step[i];
                n_oob += st_i - s;
                s = st_i + 1;
                if (!pass) {
                    ++n_saved;
                    continue;
                }
                const double Li = s_L[ev_i++];
                ++n_calls;
                const double lpi = log_screen(s_shat[i], Lstar, A.da_margin, A.da_temp);
                if (Li > Lstar && log(s_u2[i]) < lpi_cur - lpi) {
                    if (lane < d) s_u[lane] = s_p[i][lane];
                    L = Li;
                    lpi_cur = lpi;
                    ++n_acc;
                    ++i;
                    break;
                }
            }
            n_spec += neval - ev_i;
        }
    }
    if (tid == 0) {
        const size_t row = (size_t)e * n + (n - k + c);
        for (int j = 0; j < d; ++j) A.next_u[row * d + j] = s_u[j];
        A.next_L[row] = L;
        int64_t *cs = A.chain_stats + ((size_t)e * n + c) * 4;
        cs[0] = n_acc;
        cs[1] = n_calls;
        cs[2] = n_oob;
        cs[3] = n_spec;
        atomicAdd((unsigned long long *)&st.n_saved, (unsigned long long)n_saved);
    }
}

template <int WPC, int MIXED>
static void launch_walk_w(const StepArgs &a, int max_det, hipStream_t s)
{
    dim3 grid((unsigned)(a.n_events * a.k)), block(64 * WPC);
    if (a.da_on) {
        switch (max_det) {
        case 1: walk_da_kernel<WPC, 1, MIXED><<<grid, block, 0, s>>>(a); break;
        case 2: walk_da_kernel<WPC, 2, MIXED><<<grid, block, 0, s>>>(a); break;
        default: walk_da_kernel<WPC, 3, MIXED><<<grid, block, 0, s>>>(a); break;
        }
        return;
    }
    switch (max_det) {
    case 1: walk_kernel<WPC, 1, MIXED><<<grid, block, 0, s>>>(a); break;
    case 2: walk_kernel<WPC, 2, MIXED><<<grid, block, 0, s>>>(a); break;
    default: walk_kernel<WPC, 3, MIXED><<<grid, block, 0, s>>>(a); break;
    }
}

template <int MIXED>
static void launch_walk_m(const StepArgs &a, int max_det, int wpc, hipStream_t s)
{
    switch (wpc) {
    case 1: launch_walk_w<1, MIXED>(a, max_det, s); break;
    case 2: launch_walk_w<2, MIXED>(a, max_det, s); break;
    case 4: launch_walk_w<4, MIXED>(a, max_det, s); break;
    default: launch_walk_w<8, MIXED>(a, max_det, s); break;
    }
}

hipError_t launch_walk(const StepArgs &a, int max_det, int wpc, int mixed, hipStream_t s)
{
    if (mixed)
        launch_walk_m<1>(a, max_det, wpc, s);
    else
        launch_walk_m<0>(a, max_det, wpc, s);
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
    bool ok = make_coef<false>(ev, p, c);
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
