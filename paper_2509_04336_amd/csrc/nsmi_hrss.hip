// Hit-and-run slice sampling as the chains' inner kernel, the alternative the
// paper's closing section names for GPU nested sampling; the slice sampler is
// Neal (2003), Sec. 4 (stepping out, shrinkage).  The chain's target is the
// prior restricted to L > L*, uniform in the unit cube, so the slice along a
// line is the constrained set itself.  Each step takes the line through the
// current point along a differential-evolution direction S_a - S_b of the
// frozen survivors, places a unit interval at a random offset, steps it out
// by whole widths while its ends are inside (the budget of HRSS_M widths split
// at random between the two sides), and draws uniformly on the interval,
// shrinking it towards the current point after each draw outside, until a
// draw is inside.  Out-of-cube points (non-periodic coordinates) are outside
// without a likelihood call.  A step that moves counts as an accepted step, so
// the batch tuning of the walk length sets the number of slice steps.
//
// The steps are sequential, so the parallelism is inside each likelihood
// call: the two waves of a chain's workgroup take the lower and upper halves
// of the rows of the same point (the row split of every exact sum), combine
// through LDS and make the same decision.
#include <hip/hip_runtime.h>

#include "nsmi_hrss.h"

namespace nsmi {

// log L of point p for both waves of the workgroup (half = wave index);
// contains barriers, called by every thread with the same point.
template <int ND, int MIXED>
__device__ double pair_loglike(const DevEvent &ev, const double *p, int half, const double2 *tab,
                               double *s_part, double *s_L)
{
    const int lane = lane_id();
    double L = -INFINITY;
    if (ev.likelihood == 1) {
        if (half == 0) L = toy_loglike(ev, p);
    } else {
        const Src src = src_from_u(ev, p);
        Coef c;
        const bool ok = make_coef<COEF_WAVE>(ev, src, c);
        if (ev.likelihood == 2) {
            if (half == 0 && ok) {
                double R[ND], I[ND];
                wave_sums<ND, MIXED>(ev, c, R, I, tab);
                L = combine<ND, MIXED>(ev, c, R, I);
            }
        } else {
            const int rows = ev.n_pad / WAVE, mid = row_mid(rows);
            const int lo = half ? mid : 0, hi = half ? rows : mid;
            double Zr[1][ND], Zi[1][ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) Zr[0][d] = Zi[0][d] = 0.0;
            if (ok && lo < hi) {
                if (MIXED) {
                    const Coef *cp[1] = {&c};
                    accumulate_mixed_np<ND, 1>(ev, cp, lo, hi, Zr, Zi);
                } else {
                    accumulate_fp64_rot<ND>(ev, c, lo, hi, Zr[0], Zi[0], tab);
                }
            }
            double R[ND], I[ND];
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                R[d] = wave_sum(Zr[0][d]);
                I[d] = wave_sum(Zi[0][d]);
            }
            if (half == 1 && lane == 0) {
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    s_part[d] = R[d];
                    s_part[ND + d] = I[d];
                }
            }
            __syncthreads();
            if (half == 0 && ok) {
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    R[d] += s_part[d];
                    I[d] += s_part[ND + d];
                }
                L = combine<ND, MIXED>(ev, c, R, I);
            }
        }
    }
    if (half == 0 && lane == 0) *s_L = L;
    __syncthreads();
    L = *s_L;
    __syncthreads();  // s_part and s_L are reused by the next call
    return L;
}

template <int ND, int MIXED>
__global__ __launch_bounds__(2 * WAVE) void hrss_kernel(StepArgs A)
{
    __shared__ DevEvent s_ev;
    __shared__ double2 s_tab[TAB_N];
    __shared__ double s_part[2 * ND];
    __shared__ double s_L;
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
    const int half = __builtin_amdgcn_readfirstlane(tid / WAVE);
    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(A.ev + e);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_ev);
        for (int i = tid; i < (int)(sizeof(DevEvent) / 4); i += blockDim.x) dst[i] = src[i];
    }
    fill_sincos_tab(s_tab);
    __syncthreads();
    double x[NPAR], dir[NPAR], p[NPAR];
#pragma unroll
    for (int j = 0; j < NPAR; ++j) {
        x[j] = j < d ? A.chain_u[((size_t)e * n + c) * d + j] : 0.5;
        dir[j] = 0.0;
        p[j] = 0.5;
    }
    double L = A.chain_L[(size_t)e * n + c];
    int64_t n_acc = 0, n_calls = 0, n_oob = 0;
    double Lp = 0.0;
    // inside the slice: the line point in the cube and L > L*
    auto inside = [&](double t) -> bool {
        bool in = true;
#pragma unroll
        for (int j = 0; j < NPAR; ++j) {
            if (j < d) {
                double v = fma(t, dir[j], x[j]);
                if (is_periodic(d, j))
                    v = v - floor(v);
                else if (v < 0.0 || v > 1.0)
                    in = false;
                p[j] = v;
            }
        }
        if (!in) {
            ++n_oob;
            return false;
        }
        Lp = pair_loglike<ND, MIXED>(s_ev, p, half, s_tab, s_part, &s_L);
        ++n_calls;
        return Lp > Lstar;
    };
    for (int s = 0; s < W; ++s) {
        const U4 ra = philox4x64((uint64_t)s, cid, batch, HRSS_P_STEP, A.seed, 0);
        const int a = (int)floor(u01(ra.x[1]) * m);
        int b = (int)floor(u01(ra.x[2]) * (m - 1));
        if (b >= a) b += 1;
#pragma unroll
        for (int j = 0; j < NPAR; ++j)
            if (j < d) dir[j] = S[(size_t)a * d + j] - S[(size_t)b * d + j];
        const double r = u01(ra.x[3]);
        double lo = -r, hi = 1.0 - r;
        int J = (int)floor(HRSS_M * u01(ra.x[0]));
        int K = HRSS_M - 1 - J;
        while (J > 0 && inside(lo)) {
            lo -= 1.0;
            --J;
        }
        while (K > 0 && inside(hi)) {
            hi += 1.0;
            --K;
        }
        for (int q = 0; q < HRSS_K; ++q) {
            const U4 rq = philox4x64((uint64_t)s, cid, batch, HRSS_P_SHRINK + (uint64_t)q, A.seed, 0);
            const double t = lo + u01(rq.x[0]) * (hi - lo);
            if (inside(t)) {
#pragma unroll
                for (int j = 0; j < NPAR; ++j) x[j] = p[j];
                L = Lp;
                ++n_acc;
                break;
            }
            if (t < 0.0)
                lo = t;
            else
                hi = t;
        }
    }
    if (tid == 0) {
        const size_t row = (size_t)e * n + (n - k + c);
        for (int j = 0; j < d; ++j) A.next_u[row * d + j] = x[j];
        A.next_L[row] = L;
        int64_t *cs = A.chain_stats + ((size_t)e * n + c) * 4;
        cs[0] = n_acc;
        cs[1] = n_calls;
        cs[2] = n_oob;
        cs[3] = 0;
    }
}

template <int MIXED>
static void launch_hrss_m(const StepArgs &a, int max_det, hipStream_t s)
{
    dim3 grid((unsigned)(a.n_events * a.k)), block(2 * WAVE);
    switch (max_det) {
    case 1: hrss_kernel<1, MIXED><<<grid, block, 0, s>>>(a); break;
    case 2: hrss_kernel<2, MIXED><<<grid, block, 0, s>>>(a); break;
    default: hrss_kernel<3, MIXED><<<grid, block, 0, s>>>(a); break;
    }
}

hipError_t launch_hrss(const StepArgs &a, int max_det, int mixed, hipStream_t s)
{
    if (mixed)
        launch_hrss_m<1>(a, max_det, s);
    else
        launch_hrss_m<0>(a, max_det, s);
    return hipGetLastError();
}

}  // namespace nsmi
