// Walk kernels of the MI355X acceptance-walk nested sampler (gfx950, wave64):
// the plain speculative walk and the delayed-acceptance walk with the
// learned surrogate screen.  One workgroup per chain; each chain makes W
// differential-evolution steps, each a full likelihood evaluation, with the
// strict L > L* acceptance (Sec. 3.1, 3.2).
#include <hip/hip_runtime.h>

#include "nsmi_kernels.h"
#include "nsmi_mlp.h"

namespace nsmi {

// ---------------------------------------------------------------------------
// walk: one workgroup (SPEC waves) per chain.
//
// Random draws for 64 consecutive steps are generated lane-parallel (lane l
// makes the draws of step s0 + l), so each wave pays one Philox pair and
// four logarithms per 64 steps.
// ---------------------------------------------------------------------------
// Coefficients of one unit-cube point for the calling wave (all lanes hold
// the same point), written to the wave's slot in LDS; returns 0, or 2 for an
// invalid point.  Out of line so its registers are not held across the bin
// loop; the LDS slot (not a by-reference result, which would live in scratch
// memory and cost 64 lanes x 160 B of write traffic per call) carries them.
__device__ __noinline__ int point_setup_lds(const DevEvent *ev, const double *u, Coef *out)
{
    double pr[NPAR];
#pragma unroll
    for (int j = 0; j < NPAR; ++j) pr[j] = u[j];
    Src p = src_from_u(*ev, pr);
    Coef c;
    const int flag = make_coef<COEF_WAVE>(*ev, p, c) ? 0 : 2;
    if (lane_id() == 0) *out = c;
    return flag;
}

// Coefficients of n <= 16 candidate points at once, one point per group of
// COEF_GW lanes (group g < n takes u[g]) with the point's transcendental
// functions spread over the group, written to out[g] and flags[g] (0, or 2
// for an invalid point).  Wave 0 of the walk sets up all of a round's
// candidates this way: the latency of one point's setup with its independent
// logarithms, exponentials, sin/cos pairs and detector responses side by
// side, for every candidate at once.
__device__ __forceinline__ void point_setup_groups(const DevEvent *ev, const double (*u)[NPAR], int n,
                                                Coef *out, int *flags)
{
    const int g = lane_id() / COEF_GW;
    const int i = g < n ? g : 0;
    double pr[NPAR];
#pragma unroll
    for (int j = 0; j < NPAR; ++j) pr[j] = u[i][j];
    Src p = src_from_u(*ev, pr);
    Coef c;
    const int flag = make_coef<COEF_GROUP>(*ev, p, c) ? 0 : 2;
    if ((lane_id() & (COEF_GW - 1)) == 0 && g < n) {
        out[g] = c;
        flags[g] = flag;
    }
}

// Draw window [s0, s0 + 64) of a chain's walk into LDS slot `slot` (one step
// per lane): the differential-evolution scale gamma and the donor difference
// S_a - S_b of every step.  The draws depend on the step index only (not on
// the chain's current point), so a drawn window stays valid for the whole
// launch.  Lanes past the walk length write gamma = 1 and the differences of
// donors 0 and 1 (never used).  Called by all lanes of one wave; lane 0
// writes the slot's tag last.
__device__ __forceinline__ void draw_window(int s0, int slot, int W, int m, int d, uint64_t cid,
                                            uint64_t batch, uint64_t seed, double gscale,
                                            const double *S, double (*wg)[WAVE],
                                            double (*wdiff)[NPAR][WAVE], int *wtag)
{
    const int lane = lane_id();
    const int t = s0 + lane;
    int a = 0, b = 1;
    double g = 1.0;
    if (t < W) {
        U4 ra = philox4x64((uint64_t)t, cid, batch, P_WALK_A, seed, 0);
        U4 rb = philox4x64((uint64_t)t, cid, batch, P_WALK_B, seed, 0);
        const double umode = u01(ra.x[0]);
        a = (int)floor(u01(ra.x[1]) * m);
        b = (int)floor(u01(ra.x[2]) * (m - 1));
        if (b >= a) b += 1;
        if (umode >= 0.5) {
            double gs = 0.0;
            for (int i = 0; i < 4; ++i) gs += -0.25 * log(1.0 - u01(rb.x[i]));
            g = gscale * gs;
        }
    }
    wg[slot][lane] = g;
#pragma unroll
    for (int j = 0; j < NPAR; ++j)
        if (j < d) wdiff[slot][j][lane] = S[(size_t)a * d + j] - S[(size_t)b * d + j];
    if (lane == 0) wtag[slot] = s0;
}

// One workgroup of SPEC waves per chain, evaluating proposals
// speculatively.  Wave 0 owns the chain state and makes the random draws of
// 64 consecutive steps lane-parallel (lane l owns step s0 + l).  While the
// chain's point does not move, the proposals of those steps are independent:
// wave 0 forms them all at once, skips the ones that leave the unit cube
// (rejected without a likelihood call) and hands the next SPEC in-cube
// proposals to the SPEC waves, drawing further windows when one window holds
// fewer than SPEC of them, and sets up the coefficients of all of them at
// once.  The waves evaluate them (for the exact likelihood, FP64 or mixed,
// two candidates per wave pair, each wave over half of the rows; for the toy
// and the heterodyned likelihoods one candidate per wave over all rows).  Wave 0 then walks the
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
    // one scan prepares several rounds of SPEC candidates (16 at most: one
    // 4-lane group each in the setup); a round is evaluated only if the
    // rounds before it accepted none
    constexpr int NC = (SPEC <= 4 ? 4 : 2) * SPEC;
    __shared__ double s_p[NC][NPAR];
    __shared__ double s_L[NC];
    __shared__ int s_step[NC];
    __shared__ int s_cnt, s_go;
    __shared__ Coef s_cf[NC];
    __shared__ int s_fl[NC];
    __shared__ double2 s_tab[TAB_N];
    // drawn windows of 64 steps (slot = window index mod NSLOT): gamma and
    // donor differences; waves other than wave 0 draw the next ones while
    // wave 0 sets up a round's coefficients
    constexpr int NSLOT = 4, NPRE = SPEC > 2 ? 2 : SPEC - 1;
    __shared__ double s_wg[NSLOT][WAVE];
    __shared__ double s_wdiff[NSLOT][NPAR][WAVE];
    __shared__ int s_wtag[NSLOT];
    __shared__ int s_next;
    static_assert(NC * COEF_GW <= WAVE, "one lane group per candidate in wave 0");
    // pairs of candidates on wave pairs (exact likelihood): partial sums of
    // the upper halves of the rows
    constexpr bool PAIRED = SPEC >= 2 && SPEC % 2 == 0;
    __shared__ double s_part[PAIRED ? SPEC / 2 : 1][2][2 * ND];
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
    const int lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);  // wave-uniform for the compiler
    const double gscale = 2.38 / sqrt(2.0 * d);

    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(A.ev + e);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_ev);
        for (int i = tid; i < (int)(sizeof(DevEvent) / 4); i += blockDim.x) dst[i] = src[i];
    }
    fill_sincos_tab(s_tab);  // FP64 paths and relative binning
    if (tid < NPAR) s_u[tid] = tid < d ? A.chain_u[((size_t)e * n + c) * d + tid] : 0.5;
    for (int i = tid; i < NC * NPAR; i += blockDim.x) s_p[i / NPAR][i % NPAR] = 0.5;
    if (tid < NSLOT) s_wtag[tid] = -1;
    __syncthreads();
    const int likelihood = s_ev.likelihood;
    double L = A.chain_L[(size_t)e * n + c];
    int64_t n_acc = 0, n_calls = 0, n_oob = 0, n_spec = 0;

    int s = 0;        // next walk step of the sequential chain (wave 0)
    for (;;) {
        // -- wave 0: the next NC in-cube proposals from the current point
        if (wave == 0) {
            // the serial phases of the chain (scan, set-up, resolution) issue
            // ahead of the other resident chain's evaluation waves
            __builtin_amdgcn_s_setprio(2);
            int cnt = 0;
            int sp = s;  // scan position: candidates may span several windows
            while (sp < W && cnt < NC) {
                const int s0 = sp & ~(WAVE - 1);
                const int slot = (s0 / WAVE) & (NSLOT - 1);
                if (s_wtag[slot] != s0)
                    draw_window(s0, slot, W, m, d, cid, batch, A.seed, gscale, S, s_wg, s_wdiff, s_wtag);
                const int t = s0 + lane;
                bool ok = t >= sp && t < W;
                const double my_g = s_wg[slot][lane];
                double pv[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) {
                    if (j < d) {
                        double v = fma(my_g, s_wdiff[slot][j][lane], s_u[j]);
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
                    if (ok && rank < NC) {
#pragma unroll
                        for (int j = 0; j < NPAR; ++j)
                            if (j < d) s_p[rank][j] = pv[j];
                        s_step[rank] = t;
                    }
                    cnt = min(cnt + __popcll(mask), NC);
                } else if (cnt == 0) {
                    // no candidate before this window's end: its steps are
                    // rejected whatever the later candidates decide
                    n_oob += wend - s;
                    s = wend;
                }
                sp = wend;
            }
            if (lane == 0) {
                s_cnt = cnt;
                s_next = sp;  // first step past the scanned windows
            }
        }
        __syncthreads();
        const int cnt_all = s_cnt;
        if (cnt_all == 0) break;
        if (wave == 0) {
            // coefficients of every candidate of the round, one per lane group
            if (likelihood != 1) point_setup_groups(&s_ev, s_p, cnt_all, s_cf, s_fl);
            __builtin_amdgcn_s_setprio(0);
        } else if (wave <= NPRE) {
            // meanwhile the next windows past the scan are drawn
            const int s0 = s_next + (wave - 1) * WAVE;
            const int slot = (s0 / WAVE) & (NSLOT - 1);
            // (on the chain's critical path too: the next scan reads them)
            __builtin_amdgcn_s_setprio(2);
            if (s0 < W && s_wtag[slot] != s0)
                draw_window(s0, slot, W, m, d, cid, batch, A.seed, gscale, S, s_wg, s_wdiff, s_wtag);
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        for (int base = 0; base < cnt_all; base += SPEC) {
        const int cnt = min(cnt_all - base, SPEC);  // this round: candidates base .. base + cnt - 1
        if (PAIRED && likelihood == 0) {
            // -- wave pair p evaluates candidates 2p and 2p + 1 together,
            // wave 2p over the lower half of the rows, wave 2p + 1 over the
            // upper half (every wave passes the barrier below)
            const int pr = wave >> 1, half = wave & 1;
            const int ia = base + 2 * pr, ib = ia + 1;
            const bool ok_a = ia < base + cnt && s_fl[ia] == 0, ok_b = ib < base + cnt && s_fl[ib] == 0;
            double Zr[2][ND], Zi[2][ND];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int q = 0; q < ND; ++q) Zr[x][q] = Zi[x][q] = 0.0;
            const int rows = s_ev.n_pad / WAVE, mid = row_mid(rows);
            const int lo = half ? mid : 0, hi = half ? rows : mid;
            if ((ok_a || ok_b) && lo < hi) {
                // a missing or unphysical partner repeats the other point
                const Coef *cf[2] = {&s_cf[ok_a ? ia : ib], &s_cf[ok_b ? ib : ia]};
                if (MIXED)
                    accumulate_mixed_np<ND, 2>(s_ev, cf, lo, hi, Zr, Zi);
                else
                    accumulate_fp64_pair<ND>(s_ev, cf, lo, hi, Zr, Zi, s_tab);
            }
            double R[2][ND], I[2][ND];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int q = 0; q < ND; ++q) {
                    R[x][q] = wave_sum(Zr[x][q]);
                    I[x][q] = wave_sum(Zi[x][q]);
                }
            if (half == 1 && lane == 0) {
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int q = 0; q < ND; ++q) {
                        s_part[pr][x][q] = R[x][q];
                        s_part[pr][x][ND + q] = I[x][q];
                    }
            }
            __syncthreads();
            if (half == 0 && lane == 0) {
#pragma unroll
                for (int x = 0; x < 2; ++x) {
                    const int i = ia + x;
                    if (i >= base + cnt) break;
#pragma unroll
                    for (int q = 0; q < ND; ++q) {
                        R[x][q] += s_part[pr][x][q];
                        I[x][q] += s_part[pr][x][ND + q];
                    }
                    const double Lp = s_fl[i] == 0 ? combine<ND, MIXED>(s_ev, s_cf[i], R[x], I[x])
                                                   : -INFINITY;
                    s_L[i] = Lp;
                    if (A.hv_count) {
                        unsigned long long slot = atomicAdd(A.hv_count, 1ull);
                        if ((int64_t)slot < A.hv_cap) {
                            for (int j = 0; j < d; ++j) A.hv_u[slot * d + j] = s_p[i][j];
                            A.hv_L[slot] = Lp;
                        }
                    }
                }
            }
        } else if (wave < cnt) {
            // -- every wave with a candidate evaluates it
            const int ci = base + wave;
            double Lp;
            if (likelihood == 1) {
                double pr[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) pr[j] = s_p[ci][j];
                Lp = toy_loglike(s_ev, pr);
            } else {
                const int fl = s_fl[ci];
                const Coef &cf = s_cf[ci];
                double R[ND], I[ND];
                if (fl == 0) wave_sums<ND, MIXED>(s_ev, cf, R, I, s_tab);
                Lp = fl == 0 ? combine<ND, MIXED>(s_ev, cf, R, I) : -INFINITY;
            }
            if (lane == 0) {
                s_L[ci] = Lp;
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
        // -- wave 0: resolve this round's candidates in step order; the next
        // prepared round stands only if none of them is accepted
        if (wave == 0) {
            __builtin_amdgcn_s_setprio(2);
            int i = base;
            bool moved = false;
            for (; i < base + cnt; ++i) {
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
                    moved = true;
                    break;
                }
            }
            n_spec += base + cnt - i;
            if (lane == 0) s_go = moved ? 0 : 1;
            __builtin_amdgcn_s_setprio(0);
        }
        if (base + SPEC >= cnt_all) break;  // no prepared round left
        __syncthreads();
        if (!s_go) break;
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
// in-cube proposal u' the screen density
// pi(x) = floor + (1 - floor) sigmoid((s(x) - L* + m)/tau) (strictly positive)
// gives
//   stage 1: continue only if U1 < min(1, pi(u') / pi(u))   (no exact call)
//   stage 2: exact L(u'); accept iff L(u') > L* and U2 < min(1, pi(u) / pi(u'))
// with (U1, U2) the first two words of the Philox block (step, chain, batch,
// DA2).  The DE proposal is symmetric (frozen donors), so the chain keeps the
// constrained prior as its invariant distribution: the exact likelihood still
// decides every accepted point.  With pi constant it is the plain walk.
// ---------------------------------------------------------------------------
constexpr int DA_ROWS = 32;  // MFMA rows: up to 31 candidates + the current point (last row)

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

// log pi(x), pi = floor + (1 - floor) sigmoid(z), z = (s - L* + m) / tau
__device__ __forceinline__ double log_screen(double s_hat, double Lstar, double margin, double temp,
                                             double floor)
{
    const double z = (s_hat - Lstar + margin) / temp;
    if (floor <= 0.0) return z >= 0.0 ? -log1p(exp(-z)) : z - log1p(exp(z));
    const double sig = z >= 0.0 ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z));
    return log(fma(1.0 - floor, sig, floor));
}

// LDS row strides (bf16 elements) of the surrogate's inputs and activations:
// padded by 16 bytes so that the 16 rows of an MFMA fragment read fall on
// different LDS banks.
constexpr int DA_XS = MLP_KIN + 8, DA_HS = MLP_H + 8;

// Weight fragments are read through global-address-space pointers: a
// generic (flat) load also counts against the LDS counter, so every LDS wait
// of a column block would wait for the next block's prefetch as well.
// The block base is wave-uniform (scalar registers) and the lane's offset
// 32-bit, so a load needs no 64-bit address registers per lane.
typedef const __attribute__((address_space(1))) bf16x8_t gbf16x8;
__device__ __forceinline__ bf16x8_t weight_frag(const __bf16 *Wblk, uint32_t off_bytes)
{
    return *(gbf16x8 *)((gchar *)Wblk + off_bytes);
}

// Surrogate of ROWS rows (a multiple of 16) held in LDS X[ROWS][DA_XS]
// (bf16): three hidden layers with MFMA 16x16x32 tiles, column blocks of 16
// shared out over the SPEC waves (each weight fragment is loaded once and
// used for every row tile), activations in LDS H1/H2 [ROWS][DA_HS], biases
// b1, b2, b3, b4 in LDS (bias[3 MLP_H + 1]), so that the only memory loads
// of the layers are weight fragments: a wave's layer-1 fragments and its
// first layer-2 column block are issued before any product, every later
// column block's eight fragments one block ahead.  The output layer (weights
// w4 in LDS) takes 8 rows per wave pass, 8 lanes per row.  Row outputs
// mu + sigma y go to out[ROWS].  Called by every thread of the workgroup
// (contains barriers).
template <int SPEC, int ROWS>
__device__ void surrogate_rows(const StepArgs &A, const __bf16 *X, __bf16 *H1, __bf16 *H2,
                               const float *w4, const float *bias, double *out)
{
    constexpr int RT = ROWS / 16, NCB = MLP_H / 16, NK = MLP_H / 32;
    constexpr int NB1 = (NCB + SPEC - 1) / SPEC;  // layer-1 column blocks per wave
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = lane & 15, q = lane >> 4;
    // lane offsets (bytes) of a fragment within a column block of 16 rows
    const uint32_t off1 = (uint32_t)(r * MLP_KIN + 8 * q) * 2u, offh = (uint32_t)(r * MLP_H + 8 * q) * 2u;
    // every load is issued unconditionally (a step past the end re-reads the
    // last block): a load under a branch leaves the compiler unsure how many
    // are in flight, and it then waits for the prefetch too
    bf16x8_t b1[NB1], bn[NK];
#pragma unroll
    for (int j = 0; j < NB1; ++j)
        b1[j] = weight_frag(A.mW1p + (size_t)min(wave + j * SPEC, NCB - 1) * 16 * MLP_KIN, off1);
    // layer 1 (K = 32): all of the wave's products first, then the first
    // layer-2 column block's loads, which stay in flight during the epilogues
    f32x4_t acc1[NB1][RT];
    {
        bf16x8_t a[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) a[rt] = *reinterpret_cast<const bf16x8_t *>(X + (rt * 16 + r) * DA_XS + 8 * q);
#pragma unroll
        for (int j = 0; j < NB1; ++j)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                acc1[j][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], b1[j], (f32x4_t){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) bn[k] = weight_frag(A.mW2 + (size_t)wave * 16 * MLP_H, offh + 64u * k);
#pragma unroll
    for (int j = 0; j < NB1; ++j) {
        const int cb = wave + j * SPEC;
        if (cb >= NCB) break;
        const int col = cb * 16 + r;
        const float bc = bias[col];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc1[j][rt][i] + bc;
                H1[(rt * 16 + 4 * q + i) * DA_HS + col] = (__bf16)mlp_silu(z);
            }
    }
    __syncthreads();
    // layers 2 and 3: K = 256.  Step t = NBW l + j is column block
    // wave + j SPEC of layer l; two fragment buffers alternate (step t uses
    // buffer t % 2 while step t + 1's fragments load into the other), so a
    // block's loads are in flight during the previous block's products.
    constexpr int NBW = (NCB + SPEC - 1) / SPEC;  // column blocks per wave and layer
    // the layer's input fragments (the same for all of its column blocks)
    // are read from LDS once per layer and held in registers
    const __bf16 *src = H1;
    __bf16 *dst = H2;
    bf16x8_t bq[NK], af[RT][NK];
    auto load_inputs = [&]() {
#pragma unroll
        for (int k = 0; k < NK; ++k)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                af[rt][k] = *reinterpret_cast<const bf16x8_t *>(src + (rt * 16 + r) * DA_HS + 32 * k + 8 * q);
    };
    load_inputs();
    auto load_step = [&](int t, bf16x8_t (&w)[NK]) {
        t = min(t, 2 * NBW - 1);
        const int l = t / NBW, cb = min(wave + (t % NBW) * SPEC, NCB - 1);
        const __bf16 *W = (l == 0 ? A.mW2 : A.mW3) + (size_t)cb * 16 * MLP_H;
#pragma unroll
        for (int k = 0; k < NK; ++k) w[k] = weight_frag(W, offh + 64u * k);
    };
    auto run_step = [&](int t, const bf16x8_t (&w)[NK]) {
        const int l = t / NBW, cb = wave + (t % NBW) * SPEC;
        if (cb < NCB) {
            f32x4_t acc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[rt] = (f32x4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int k = 0; k < NK; ++k)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[rt][k], w[k], acc[rt], 0, 0, 0);
            const int col = cb * 16 + r;
            const float bc = bias[(l + 1) * MLP_H + col];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float z = acc[rt][i] + bc;
                    dst[(rt * 16 + 4 * q + i) * DA_HS + col] = (__bf16)mlp_silu(z);
                }
            }
        }
        if ((t + 1) % NBW == 0) {
            // end of a layer: its output is the next layer's input
            __syncthreads();
            __bf16 *o = dst;
            dst = const_cast<__bf16 *>(src);
            src = o;
            if (t + 1 < 2 * NBW) load_inputs();
        }
    };
#pragma unroll 1
    for (int t = 0; t < 2 * NBW; t += 2) {
        load_step(t + 1, bq);
        run_step(t, bn);
        load_step(t + 2, bn);
        run_step(t + 1, bq);
    }
    // output layer (src holds h3): 8 rows per wave pass, lane -> (row lane / 8,
    // eighth lane % 8 of the 256 inputs)
    for (int rb = wave; rb < ROWS / 8; rb += SPEC) {
        const int row = rb * 8 + (lane >> 3), part = lane & 7;
        float acc = 0.f;
#pragma unroll 8
        for (int j = part * 32; j < part * 32 + 32; ++j) acc += w4[j] * (float)src[row * DA_HS + j];
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        acc += __shfl_xor(acc, 4, 64);
        if (part == 0) out[row] = target_from_z(A.m_mu + A.m_sig * (double)(acc + bias[3 * MLP_H]), A.m_top);
    }
    __syncthreads();
}

template <int SPEC, int ND, int MIXED>
__global__ __launch_bounds__(64 * SPEC) __attribute__((amdgpu_waves_per_eu(2))) void walk_da_kernel(StepArgs A)
{
    // chunk of passing candidates whose coefficients are set up at once (one
    // lane group each in wave 0), evaluated SPEC per round
    constexpr int NCH = WAVE / COEF_GW;
    constexpr bool PAIRED = SPEC >= 2 && SPEC % 2 == 0;
    __shared__ DevEvent s_ev;
    __shared__ double s_u[NPAR];
    __shared__ double s_p[DA_ROWS][NPAR];
    __shared__ int s_step[DA_ROWS];
    __shared__ double s_u1[DA_ROWS], s_u2[DA_ROWS];
    __shared__ double s_shat[DA_ROWS];
    __shared__ int s_plist[DA_ROWS];   // candidates that pass stage 1, in step order
    __shared__ double s_q[NCH][NPAR];  // the current chunk's points
    __shared__ Coef s_cf[NCH];
    __shared__ int s_fl[NCH];
    __shared__ double s_L[NCH];
    __shared__ int s_cnt, s_np, s_go;
    __shared__ uint32_t s_pass;        // stage-1 outcome per candidate (bit i)
    __shared__ double s_part[PAIRED ? SPEC / 2 : 1][2][2 * ND];
    static_assert(DA_ROWS - 1 <= 32 && DA_ROWS % 16 == 0, "candidate mask and MFMA row tiles");
    static_assert(NCH * COEF_GW <= WAVE, "one lane group per candidate of a chunk");
    __shared__ double2 s_tab[TAB_N];
    __shared__ double s_wg[1][WAVE];           // the current draw window: gamma,
    __shared__ double s_wdiff[1][NPAR][WAVE];  // donor differences
    __shared__ int s_wtag[1];
    __shared__ __attribute__((aligned(16))) __bf16 s_X[DA_ROWS * DA_XS];
    __shared__ __attribute__((aligned(16))) __bf16 s_H1[DA_ROWS * DA_HS];
    __shared__ __attribute__((aligned(16))) __bf16 s_H2[DA_ROWS * DA_HS];
    __shared__ float s_w4[MLP_H];
    __shared__ float s_bias[3 * MLP_H + 1];           // b1, b2, b3, b4
    __shared__ float s_inmu[NPAR], s_inis[NPAR];       // input standardisation
    __shared__ double s_lpi[DA_ROWS], s_lu2[DA_ROWS];  // log pi and log U2 of each candidate
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
    const int lane = tid & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / WAVE);
    for (int i = tid; i < MLP_H; i += blockDim.x) {
        s_w4[i] = A.mP[MLP_OFF_W4 + i];
        s_bias[i] = A.mP[MLP_OFF_B1 + i];
        s_bias[MLP_H + i] = A.mP[MLP_OFF_B2 + i];
        s_bias[2 * MLP_H + i] = A.mP[MLP_OFF_B3 + i];
    }
    if (tid == 0) s_bias[3 * MLP_H] = A.mP[MLP_OFF_B4];
    if (tid < NPAR) {
        s_inmu[tid] = tid < A.ndim ? A.m_in_mu[tid] : 0.0f;
        s_inis[tid] = tid < A.ndim ? A.m_in_isig[tid] : 0.0f;
    }
    const double gscale = 2.38 / sqrt(2.0 * d);

    {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(A.ev + e);
        uint32_t *dst = reinterpret_cast<uint32_t *>(&s_ev);
        for (int i = tid; i < (int)(sizeof(DevEvent) / 4); i += blockDim.x) dst[i] = src[i];
    }
    fill_sincos_tab(s_tab);  // FP64 paths and relative binning
    if (tid < NPAR) s_u[tid] = tid < d ? A.chain_u[((size_t)e * n + c) * d + tid] : 0.5;
    for (int i = tid; i < DA_ROWS * NPAR; i += blockDim.x) s_p[i / NPAR][i % NPAR] = 0.5;
    for (int i = tid; i < NCH * NPAR; i += blockDim.x) s_q[i / NPAR][i % NPAR] = 0.5;
    __syncthreads();
    const int likelihood = s_ev.likelihood;
    double L = A.chain_L[(size_t)e * n + c];
    double lpi_cur = 0.0;       // log screen density of the current point (wave 0)
    bool have_cur = false;
    int64_t n_acc = 0, n_calls = 0, n_oob = 0, n_spec = 0, n_saved = 0;

    if (tid == 0) s_wtag[0] = -1;
    int s = 0, s0 = -WAVE;
    double my_u1 = 0.0, my_u2 = 0.0;
    for (;;) {
        // -- wave 0: up to DA_ROWS - 1 in-cube candidates, across draw windows
        // (the serial phases of the chain issue ahead of the other resident
        // chain's evaluation waves)
        if (wave == 0) {
            __builtin_amdgcn_s_setprio(2);
            int cnt = 0;
            int sp = s;  // scan position
            while (sp < W && cnt < DA_ROWS - 1) {
                if (sp < s0 || sp >= s0 + WAVE) {
                    s0 = sp & ~(WAVE - 1);
                    draw_window(s0, 0, W, m, d, cid, batch, A.seed, gscale, S, s_wg, s_wdiff, s_wtag);
                    // and the two screen uniforms of each step
                    const int t = s0 + lane;
                    if (t < W) {
                        U4 rd = philox4x64((uint64_t)t, cid, batch, P_DA2, A.seed, 0);
                        my_u1 = u01(rd.x[0]);
                        my_u2 = u01(rd.x[1]);
                    }
                }
                const int t = s0 + lane;
                const double my_g = s_wg[0][lane];
                bool ok = t >= sp && t < W;
                double pv[NPAR];
#pragma unroll
                for (int j = 0; j < NPAR; ++j) {
                    if (j < d) {
                        double v = fma(my_g, s_wdiff[0][j][lane], s_u[j]);
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
                    const uint64_t below = lane == 0 ? 0ull : (mask & (~0ull >> (WAVE - lane)));
                    const int rank = cnt + __popcll(below);
                    if (ok && rank < DA_ROWS - 1) {
#pragma unroll
                        for (int j = 0; j < NPAR; ++j)
                            if (j < d) s_p[rank][j] = pv[j];
                        s_step[rank] = t;
                        s_u1[rank] = my_u1;
                        s_u2[rank] = my_u2;
                    }
                    cnt = min(cnt + __popcll(mask), DA_ROWS - 1);
                } else if (cnt == 0) {
                    n_oob += wend - s;
                    s = wend;
                }
                sp = wend;
            }
            if (lane == 0) s_cnt = cnt;
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        const int cnt = s_cnt;
        if (cnt == 0) break;
        // -- surrogate on the candidates (rows 0..cnt-1) and the current point (last row)
        for (int i = tid; i < DA_ROWS * MLP_KIN; i += blockDim.x) {
            const int row = i / MLP_KIN, col = i % MLP_KIN;
            float v = 0.0f;
            if (col < d) {
                double x = row == DA_ROWS - 1 ? s_u[col] : (row < cnt ? s_p[row][col] : 0.0);
                v = ((float)x - s_inmu[col]) * s_inis[col];
            }
            s_X[row * DA_XS + col] = (__bf16)v;
        }
        __syncthreads();
        surrogate_rows<SPEC, DA_ROWS>(A, s_X, s_H1, s_H2, s_w4, s_bias, s_shat);
        // -- wave 0: stage-1 screen of every candidate (lane-parallel; the
        // current point's screen value holds until an accept)
        if (wave == 0) {
            __builtin_amdgcn_s_setprio(2);
            if (!have_cur) {
                lpi_cur = log_screen(s_shat[DA_ROWS - 1], Lstar, A.da_margin, A.da_temp, A.da_floor);
                have_cur = true;
            }
            bool pass = false;
            if (lane < cnt) {
                // both screen tests' terms of every candidate, lane-parallel
                const double lpi = log_screen(s_shat[lane], Lstar, A.da_margin, A.da_temp, A.da_floor);
                pass = log(s_u1[lane]) < lpi - lpi_cur;
                s_lpi[lane] = lpi;
                s_lu2[lane] = log(s_u2[lane]);
            }
            const uint64_t pm = __ballot(pass);
            const uint64_t below = lane == 0 ? 0ull : (pm & (~0ull >> (WAVE - lane)));
            if (pass) s_plist[__popcll(below)] = lane;
            if (lane == 0) {
                s_np = __popcll(pm);
                s_pass = (uint32_t)(pm & 0xffffffffull);  // DA_ROWS - 1 <= 32 candidates
            }
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        const int np = s_np;
        // -- exact evaluations of the passing candidates in step order, SPEC
        // per round; wave 0 resolves after every round and the scan's
        // remaining rounds stand only while no candidate is accepted
        int i_res = 0, prank = 0;  // resolve cursor and passing candidates consumed (wave 0)
        const uint32_t pmask = s_pass;
        auto resolve = [&](int ev_hi) {
            bool moved = false;
            for (; i_res < cnt; ++i_res) {
                const bool pass = (pmask >> i_res) & 1u;
                if (pass && prank >= ev_hi) break;  // not evaluated yet: next round
                const int st_i = s_step[i_res];
                n_oob += st_i - s;
                s = st_i + 1;
                if (!pass) {
                    ++n_saved;
                    continue;
                }
                const double Li = s_L[prank % NCH];
                ++prank;
                ++n_calls;
                const double lpi = s_lpi[i_res];
                if (Li > Lstar && s_lu2[i_res] < lpi_cur - lpi) {
                    if (lane < d) s_u[lane] = s_p[i_res][lane];
                    L = Li;
                    lpi_cur = lpi;
                    ++n_acc;
                    ++i_res;
                    moved = true;
                    break;
                }
            }
            if (moved) n_spec += ev_hi - prank;  // evaluated after the accepted one
            return moved;
        };
        if (np == 0) {
            if (wave == 0) (void)resolve(0);  // every candidate screened out
            continue;
        }
        bool stop = false;
        for (int c0 = 0; c0 < np && !stop; c0 += NCH) {
            const int nch = min(np - c0, NCH);
            if (wave == 0) {
                __builtin_amdgcn_s_setprio(2);
                for (int i = lane; i < nch * NPAR; i += WAVE) s_q[i / NPAR][i % NPAR] = s_p[s_plist[c0 + i / NPAR]][i % NPAR];
                if (likelihood != 1) point_setup_groups(&s_ev, s_q, nch, s_cf, s_fl);
                __builtin_amdgcn_s_setprio(0);
            }
            __syncthreads();
            for (int base = 0; base < nch; base += SPEC) {
                const int cr = min(nch - base, SPEC);  // this round: chunk candidates base .. base + cr - 1
                if (PAIRED && likelihood == 0) {
                    // wave pair p: candidates base + 2p and base + 2p + 1, wave 2p
                    // over the lower half of the rows, wave 2p + 1 over the upper
                    const int pr = wave >> 1, half = wave & 1;
                    const int ia = base + 2 * pr, ib = ia + 1;
                    const bool ok_a = ia < base + cr && s_fl[ia] == 0, ok_b = ib < base + cr && s_fl[ib] == 0;
                    double Zr[2][ND], Zi[2][ND];
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int q = 0; q < ND; ++q) Zr[x][q] = Zi[x][q] = 0.0;
                    const int rows = s_ev.n_pad / WAVE, mid = row_mid(rows);
                    const int lo = half ? mid : 0, hi = half ? rows : mid;
                    if ((ok_a || ok_b) && lo < hi) {
                        const Coef *cf[2] = {&s_cf[ok_a ? ia : ib], &s_cf[ok_b ? ib : ia]};
                        if (MIXED)
                            accumulate_mixed_np<ND, 2>(s_ev, cf, lo, hi, Zr, Zi);
                        else
                            accumulate_fp64_pair<ND>(s_ev, cf, lo, hi, Zr, Zi, s_tab);
                    }
                    double R[2][ND], I[2][ND];
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int q = 0; q < ND; ++q) {
                            R[x][q] = wave_sum(Zr[x][q]);
                            I[x][q] = wave_sum(Zi[x][q]);
                        }
                    if (half == 1 && lane == 0) {
#pragma unroll
                        for (int x = 0; x < 2; ++x)
#pragma unroll
                            for (int q = 0; q < ND; ++q) {
                                s_part[pr][x][q] = R[x][q];
                                s_part[pr][x][ND + q] = I[x][q];
                            }
                    }
                    __syncthreads();
                    if (half == 0 && lane == 0) {
#pragma unroll
                        for (int x = 0; x < 2; ++x) {
                            const int i = ia + x;
                            if (i >= base + cr) break;
#pragma unroll
                            for (int q = 0; q < ND; ++q) {
                                R[x][q] += s_part[pr][x][q];
                                I[x][q] += s_part[pr][x][ND + q];
                            }
                            s_L[i] = s_fl[i] == 0 ? combine<ND, MIXED>(s_ev, s_cf[i], R[x], I[x]) : -INFINITY;
                        }
                    }
                } else if (wave < cr) {
                    // one candidate per wave over all rows
                    const int i = base + wave;
                    double Lp;
                    if (likelihood == 1) {
                        double pr[NPAR];
#pragma unroll
                        for (int j = 0; j < NPAR; ++j) pr[j] = s_q[i][j];
                        Lp = toy_loglike(s_ev, pr);
                    } else {
                        double R[ND], I[ND];
                        if (s_fl[i] == 0) wave_sums<ND, MIXED>(s_ev, s_cf[i], R, I, s_tab);
                        Lp = s_fl[i] == 0 ? combine<ND, MIXED>(s_ev, s_cf[i], R, I) : -INFINITY;
                    }
                    if (lane == 0) s_L[i] = Lp;
                }
                __syncthreads();
                if (wave == 0) {
                    __builtin_amdgcn_s_setprio(2);
                    if (A.hv_count && lane < cr) {
                        // record the round's exact evaluations (u, logL)
                        unsigned long long slot = atomicAdd(A.hv_count, 1ull);
                        if ((int64_t)slot < A.hv_cap) {
                            for (int j = 0; j < d; ++j) A.hv_u[slot * d + j] = s_q[base + lane][j];
                            A.hv_L[slot] = s_L[base + lane];
                        }
                    }
                    const bool moved = resolve(c0 + base + cr);
                    if (lane == 0) s_go = moved ? 0 : 1;
                    __builtin_amdgcn_s_setprio(0);
                }
                __syncthreads();
                if (!s_go) {
                    stop = true;
                    break;
                }
            }
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
    dim3 grid((unsigned)chain_blocks(a)), block(64 * WPC);
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
    case 6: launch_walk_w<6, MIXED>(a, max_det, s); break;
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

}  // namespace nsmi
