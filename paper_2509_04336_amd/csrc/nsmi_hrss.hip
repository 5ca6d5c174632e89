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
// The steps are sequential, so the parallelism is inside each step.  Every
// round evaluates two points on the chain's two waves: while the interval
// steps out, its lower and upper ends (independent sequences); during
// shrinkage, draw q and draw q + 1 on the interval shrunk as if draw q were
// outside.  The first wave sums both points over the lower half of the rows
// and the second over the upper half (the candidate-pair accumulation of
// the walk, one table load for two points, and the row split of every exact
// sum); they combine through LDS.  Decisions are taken in draw order, so the
// chain, its random numbers and its call count are those of the sequential
// sampler, and an evaluation that draw q makes moot is not counted.
#include <hip/hip_runtime.h>

#include "nsmi_hrss.h"

namespace nsmi {

// Line point at parameter t: p = x + t dir, periodic coordinates wrapped;
// true when p lies in the cube.
__device__ inline bool line_point(int d, const double *x, const double *dir, double t, double *p)
{
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
    return in;
}

// The cube test of line_point alone (same arithmetic, no point written).
__device__ inline bool line_in_cube(int d, const double *x, const double *dir, double t)
{
    bool in = true;
#pragma unroll
    for (int j = 0; j < NPAR; ++j) {
        if (j < d && !is_periodic(d, j)) {
            const double v = fma(t, dir[j], x[j]);
            if (v < 0.0 || v > 1.0) in = false;
        }
    }
    return in;
}

// Per-workgroup LDS of a round's two evaluations.
template <int ND>
struct PairLds {
    Coef cf[2];              // coefficients of points 0 and 1
    int fl[2];               // 0, or 2 for an invalid point
    double part[2][2 * ND];  // upper-half sums of both points
    double L[2];             // the results
};

// log L of the round's points 0 and 1 (live0 / live1: wanted and in the
// cube).  Wave `half` holds point `half` in p and sets up its coefficients;
// for the exact likelihood both waves then sum both points, wave 0 over the
// lower half of the rows and wave 1 over the upper half; the heterodyned
// and toy likelihoods take one point per wave.  Called by every thread (it
// holds its barriers); afterwards s.L[q] is point q's log L (meaningful for
// a live point) until the next call.
template <int ND, int MIXED>
__device__ void pair_loglike2(const DevEvent &ev, const double *p, bool live0, bool live1, int half,
                              const double2 *tab, PairLds<ND> &s)
{
    const int lane = lane_id();
    const int like = ev.likelihood;
    const bool mine = half ? live1 : live0;
    if (mine && like != 1) {
        const Src src = src_from_u(ev, p);
        Coef c;
        const int fl = make_coef<COEF_WAVE>(ev, src, c) ? 0 : 2;
        if (lane == 0) {
            s.cf[half] = c;
            s.fl[half] = fl;
        }
    }
    __syncthreads();
    const bool ok0 = live0 && (like == 1 || s.fl[0] == 0);
    const bool ok1 = live1 && (like == 1 || s.fl[1] == 0);
    double R[2][ND], I[2][ND];
    if (like == 1 || like == 2) {
        double L = -INFINITY;
        if (half ? ok1 : ok0) {
            if (like == 1) {
                L = toy_loglike(ev, p);
            } else {
                wave_sums<ND, MIXED>(ev, s.cf[half], R[0], I[0], tab);
                L = combine<ND, MIXED>(ev, s.cf[half], R[0], I[0]);
            }
        }
        if (lane == 0) s.L[half] = L;
    } else if (ok0 || ok1) {
        const Coef *cf[2] = {&s.cf[ok0 ? 0 : 1], &s.cf[ok1 ? 1 : 0]};
        const int rows = ev.n_pad / WAVE, mid = row_mid(rows);
        const int lo = half ? mid : 0, hi = half ? rows : mid;
        double Zr[2][ND], Zi[2][ND];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int d = 0; d < ND; ++d) Zr[q][d] = Zi[q][d] = 0.0;
        if (lo < hi) {
            if (MIXED)
                accumulate_mixed_np<ND, 2>(ev, cf, lo, hi, Zr, Zi);
            else
                accumulate_fp64_pair<ND>(ev, cf, lo, hi, Zr, Zi, tab);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                R[q][d] = wave_sum(Zr[q][d]);
                I[q][d] = wave_sum(Zi[q][d]);
            }
        if (half == 1 && lane == 0) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    s.part[q][d] = R[q][d];
                    s.part[q][ND + d] = I[q][d];
                }
        }
    }
    __syncthreads();
    if (like != 1 && like != 2 && half == 0 && (ok0 || ok1)) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const bool okq = q ? ok1 : ok0;
            double L = -INFINITY;
            if (okq) {
#pragma unroll
                for (int d = 0; d < ND; ++d) {
                    R[q][d] += s.part[q][d];
                    I[q][d] += s.part[q][ND + d];
                }
                L = combine<ND, MIXED>(ev, s.cf[q], R[q], I[q]);
            }
            if (lane == 0) s.L[q] = L;
        }
    }
    __syncthreads();
}

template <int ND, int MIXED>
__global__ __launch_bounds__(2 * WAVE) void hrss_kernel(StepArgs A)
{
    __shared__ DevEvent s_ev;
    __shared__ double2 s_tab[TAB_N];
    __shared__ PairLds<ND> s_pair;
    int e, c;
    if (!block_chain(A, blockIdx.x, &e, &c)) return;
    const int k = A.k;
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
    // a draw inside the slice moves the chain there
    auto accept = [&](double t, double Lt) {
        line_point(d, x, dir, t, p);
#pragma unroll
        for (int j = 0; j < NPAR; ++j) x[j] = p[j];
        L = Lt;
        ++n_acc;
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
        // one round per iteration: stepping out while either end may move
        // (point 0 the lower end, point 1 the upper end), then shrinkage
        // (point 0 draw q, point 1 draw q + 1 on the interval shrunk at q)
        bool goL = J > 0, goR = K > 0;
        int q = 0;
        while (q < HRSS_K) {
            const bool out = goL || goR;
            double t0, t1 = 0.0, lo1 = lo, hi1 = hi;
            bool in0, in1, has1 = false;
            if (out) {
                t0 = lo;
                t1 = hi;
                in0 = goL && line_in_cube(d, x, dir, lo);
                in1 = goR && line_in_cube(d, x, dir, hi);
            } else {
                const U4 r0 = philox4x64((uint64_t)s, cid, batch, HRSS_P_SHRINK + (uint64_t)q, A.seed, 0);
                t0 = lo + u01(r0.x[0]) * (hi - lo);
                if (t0 < 0.0)
                    lo1 = t0;
                else
                    hi1 = t0;
                has1 = q + 1 < HRSS_K;
                if (has1) {
                    const U4 r1 = philox4x64((uint64_t)s, cid, batch,
                                             HRSS_P_SHRINK + (uint64_t)(q + 1), A.seed, 0);
                    t1 = lo1 + u01(r1.x[0]) * (hi1 - lo1);
                }
                in0 = line_in_cube(d, x, dir, t0);
                in1 = has1 && line_in_cube(d, x, dir, t1);
            }
            double L0 = -INFINITY, L1 = -INFINITY;
            if (in0 || in1) {
                line_point(d, x, dir, half ? t1 : t0, p);
                pair_loglike2<ND, MIXED>(s_ev, p, in0, in1, half, s_tab, s_pair);
                L0 = s_pair.L[0];
                L1 = s_pair.L[1];
            }
            if (out) {
                if (goL) {
                    if (in0) ++n_calls; else ++n_oob;
                    if (in0 && L0 > Lstar) {
                        lo -= 1.0;
                        goL = --J > 0;
                    } else {
                        goL = false;
                    }
                }
                if (goR) {
                    if (in1) ++n_calls; else ++n_oob;
                    if (in1 && L1 > Lstar) {
                        hi += 1.0;
                        goR = --K > 0;
                    } else {
                        goR = false;
                    }
                }
                continue;
            }
            if (in0) ++n_calls; else ++n_oob;
            if (in0 && L0 > Lstar) {
                accept(t0, L0);
                break;
            }
            lo = lo1;
            hi = hi1;
            if (!has1) break;
            if (in1) ++n_calls; else ++n_oob;
            if (in1 && L1 > Lstar) {
                accept(t1, L1);
                break;
            }
            if (t1 < 0.0)
                lo = t1;
            else
                hi = t1;
            q += 2;
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
    dim3 grid((unsigned)chain_blocks(a)), block(2 * WAVE);
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
