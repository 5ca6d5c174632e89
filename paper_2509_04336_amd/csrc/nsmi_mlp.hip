// Surrogate network kernels (gfx950): a fully connected 11 -> 256 -> 256 ->
// 256 -> 1 network with SiLU activations, trained on (u, logL) pairs of the
// sampler's own runs with mean squared error and Adam.  Matrix products use
// the BF16 MFMA instruction v_mfma_f32_16x16x32_bf16 with FP32 accumulation;
// FP32 master weights are updated by Adam and re-rounded to BF16 copies.
//
// Every product has the form C[M][N] = A[M][K] B[N][K]^T with K contiguous in
// both operands (the forward pass X W^T, the weight gradient D^T H taken
// from feature-major copies, the activation gradient D W taken from W^T).
#include <hip/hip_runtime.h>

#include "nsmi_mlp.h"

namespace nsmi {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// One wave computes a 16 x 64 tile of C (four 16 x 16 MFMA blocks); a
// workgroup of 4 waves covers 16 x 256.  Lane l of a 16x16x32 block holds
// A[l % 16][8 (l / 16) .. +7], B[8 (l / 16) .. +7][l % 16] and returns
// C[4 (l / 16) .. +3][l % 16].  M is a multiple of 16, N of 256, K of 32
// (callers pad; the drivers below only use N = 256).  With blockIdx.z = z the
// workgroup contracts only over k in [z kc, (z + 1) kc) and stores its
// partial product to C + z M ldc (split K; beta must then be 0).
// Epilogues of the product (element C[row][col] of the lane):
//   EPI_STORE     C = acc (+ beta C)
//   EPI_BIAS_SILU the forward of a hidden layer: z = acc + bias[col] kept in
//                 C (the pre-activation), silu(z) as bf16 in H[row][col] and,
//                 when HT is given, in HT[col][row] (feature-major; M is the
//                 row count of C, a lane's four rows go out as one 8-byte store)
//   EPI_DSILU     the backward through a hidden layer: d = acc silu'(z) with
//                 z = Z[row][col], as bf16 in H[row][col] and HT[col][row]
// (the formulas of the separate elementwise kernels, so the same bits).
enum { EPI_STORE = 0, EPI_BIAS_SILU = 1, EPI_DSILU = 2 };

struct GemmEpi {
    const float *bias = nullptr;  // EPI_BIAS_SILU: [N]
    const float *Z = nullptr;     // EPI_DSILU: [M][ldc] pre-activations
    __bf16 *H = nullptr, *HT = nullptr;
};

// One product's operands and tiling: grid (M / 16, N / 256, S) of 256-thread
// workgroups, K split into slices of kc.
struct GemmArgs {
    int M, N, K;
    const __bf16 *A;
    int lda;
    const __bf16 *B;
    int ldb;
    float *C;
    int ldc;
    float beta;
    int kc;
    GemmEpi ep;
};

// The tile of workgroup (bx, by, bz) of a product.
template <int EPI>
__device__ __forceinline__ void gemm_tile(const GemmArgs &g, int bx, int by, int bz)
{
    const int M = g.M, N = g.N, K = g.K, lda = g.lda, ldb = g.ldb, ldc = g.ldc, kc = g.kc;
    const __bf16 *A = g.A, *B = g.B;
    const float beta = g.beta;
    const GemmEpi &ep = g.ep;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = bx * 16;
    const int col0 = (by * 4 + wave) * 64;
    if (row0 >= M || col0 >= N) return;
    const int kb = bz * kc, ke = min(K, kb + kc);
    float *C = g.C + (size_t)bz * M * ldc;
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int r = lane & 15, q = lane >> 4;
    // K in chunks of KU steps of 32: every fragment of a chunk is loaded
    // before its products, so a chunk costs one memory latency instead of one
    // per step (the products still run in k order: the same sums)
    constexpr int KU = 8;
    const __bf16 *Ar = A + (size_t)(row0 + r) * lda + 8 * q;
    const __bf16 *Br = B + (size_t)(col0 + r) * ldb + 8 * q;
    for (int k0 = kb; k0 < ke; k0 += 32 * KU) {
        const int nk = min(KU, (ke - k0) / 32);
        bf16x8 a[KU], b[KU][4];
        if (nk == KU) {
            // a full chunk: its loads unguarded, so the compiler counts them all
            // in flight and waits for each step's fragments only (loads under a
            // branch make it wait for every load before each step)
#pragma unroll
            for (int t = 0; t < KU; ++t) {
                a[t] = *reinterpret_cast<const bf16x8 *>(Ar + k0 + 32 * t);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    b[t][j] = *reinterpret_cast<const bf16x8 *>(Br + (size_t)(16 * j) * ldb + k0 + 32 * t);
            }
#pragma unroll
            for (int t = 0; t < KU; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[t][j], acc[j], 0, 0, 0);
            continue;
        }
#pragma unroll
        for (int t = 0; t < KU; ++t) {
            if (t < nk) {
                a[t] = *reinterpret_cast<const bf16x8 *>(Ar + k0 + 32 * t);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    b[t][j] = *reinterpret_cast<const bf16x8 *>(Br + (size_t)(16 * j) * ldb + k0 + 32 * t);
            }
        }
#pragma unroll
        for (int t = 0; t < KU; ++t) {
            if (t < nk) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t], b[t][j], acc[j], 0, 0, 0);
            }
        }
    }
    if (EPI == EPI_STORE) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float *c = C + (size_t)(row0 + 4 * q + i) * ldc + col0 + 16 * j + r;
                *c = beta == 0.f ? acc[j][i] : beta * *c + acc[j][i];
            }
        return;
    }
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = col0 + 16 * j + r;
        __bf16 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const size_t o = (size_t)(row0 + 4 * q + i) * ldc + col;
            if (EPI == EPI_BIAS_SILU) {
                const float z = acc[j][i] + ep.bias[col];
                C[o] = z;
                v[i] = (__bf16)mlp_silu(z);
            } else {
                const float z = ep.Z[o], sg = mlp_sigmoid(z);
                v[i] = (__bf16)(acc[j][i] * sg * (1.0f + z * (1.0f - sg)));
            }
            ep.H[o] = v[i];
        }
        if (ep.HT) {
            *reinterpret_cast<bf16x4 *>(ep.HT + (size_t)col * M + row0 + 4 * q) = (bf16x4){v[0], v[1], v[2], v[3]};
        }
    }
}

template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt_bf16_kernel(GemmArgs g)
{
    gemm_tile<EPI>(g, blockIdx.x, blockIdx.y, blockIdx.z);
}

// The three weight-gradient products of a training step (layers 3, 2, 1:
// split over the batch, partial products to their workspaces) in one
// launch; each product's workgroups in gemm_tile's (x, y, z) order.
__global__ __launch_bounds__(256) void gemm_wgrad3_kernel(GemmArgs g3, GemmArgs g2, GemmArgs g1)
{
    int w = blockIdx.x;
    const GemmArgs *gs[3] = {&g3, &g2, &g1};
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const GemmArgs &g = *gs[l];
        const int ax = g.M / 16, n = ax * ((g.K + g.kc - 1) / g.kc);
        if (w < n) {
            gemm_tile<EPI_STORE>(g, w % ax, 0, w / ax);
            return;
        }
        w -= n;
    }
}

// C[M][N] = sum over the S partial products ws[z][M][N], in z order (the
// same bits whatever the launch).
__global__ void splitk_reduce_kernel(int64_t MN, int S, const float *ws, float *C)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= MN) return;
    float acc = 0.f;
    for (int z = 0; z < S; ++z) acc += ws[(size_t)z * MN + i];
    C[i] = acc;
}

// C = A B^T (+ beta C).  A contraction over many rows (the weight gradients,
// K = the batch) is split into slices of at least 256 so that every CU gets
// work: partial products in ws (room for MLP_SPLITK slices of M x N with
// M, N <= MLP_H), then a reduction; ws = nullptr keeps one slice.
// Slices of K (and their length) of a split product C[M][N] (ldc = N).
static int splitk_slices(int M, int N, int K, int *kc_out = nullptr)
{
    int S = 1, kc = K;
    if (K >= 1024 && M <= MLP_H && N <= MLP_H) {
        kc = (K + MLP_SPLITK - 1) / MLP_SPLITK;
        kc = kc < 256 ? 256 : (kc + 31) / 32 * 32;
        S = (K + kc - 1) / kc;
    }
    if (kc_out) *kc_out = kc;
    return S;
}

static void gemm_nt(int M, int N, int K, const __bf16 *A, int lda, const __bf16 *B, int ldb,
                    float *C, int ldc, float beta, hipStream_t s, float *ws = nullptr,
                    int epi = EPI_STORE, GemmEpi ep = GemmEpi())
{
    int S = 1, kc = K;
    if (ws && beta == 0.f && ldc == N) S = splitk_slices(M, N, K, &kc);
    if (epi != EPI_STORE) S = 1, kc = K;  // fused epilogues: one slice
    dim3 grid((unsigned)(M / 16), (unsigned)(N / 256 > 0 ? N / 256 : 1), (unsigned)S);
    const GemmArgs g = {M, N, K, A, lda, B, ldb, S > 1 ? ws : C, ldc, beta, kc, ep};
    if (epi == EPI_BIAS_SILU)
        gemm_nt_bf16_kernel<EPI_BIAS_SILU><<<grid, 256, 0, s>>>(g);
    else if (epi == EPI_DSILU)
        gemm_nt_bf16_kernel<EPI_DSILU><<<grid, 256, 0, s>>>(g);
    else
        gemm_nt_bf16_kernel<EPI_STORE><<<grid, 256, 0, s>>>(g);
    if (S > 1) {
        const int64_t MN = (int64_t)M * N;
        splitk_reduce_kernel<<<(unsigned)((MN + 255) / 256), 256, 0, s>>>(MN, S, ws, C);
    }
}


// Network input rows: the standardised unit-cube point (u - mean) / std,
// zero-padded to 32 columns (bf16).
__global__ void mlp_input_kernel(const double *u, int ndim, int64_t n, int64_t Mp,
                                 const float *in_mu, const float *in_isig, __bf16 *X)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= Mp * MLP_KIN) return;
    int64_t r = i / MLP_KIN;
    int c = (int)(i % MLP_KIN);
    float v = (r < n && c < ndim) ? ((float)u[r * ndim + c] - in_mu[c]) * in_isig[c] : 0.0f;
    X[i] = (__bf16)v;
}

// per-input mean and 1/std of n unit-cube points (one workgroup per column)
__global__ void input_stats_kernel(int64_t n, const double *u, int ndim, float *in_mu, float *in_isig)
{
    __shared__ double s1[256], s2[256];
    const int c = blockIdx.x;
    double a = 0.0, b = 0.0;
    if (c < ndim)
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            double v = u[i * ndim + c];
            a += v;
            b += v * v;
        }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c < ndim) {
            double mu = s1[0] / (double)n;
            double var = s2[0] / (double)n - mu * mu;
            double sd = var > 1e-12 ? sqrt(var) : 1.0;
            in_mu[c] = (float)mu;
            in_isig[c] = (float)(1.0 / sd);
        } else {
            in_mu[c] = 0.0f;
            in_isig[c] = 1.0f;
        }
    }
}

// y[r] = W4 . h3[r] + b4 (fp32), one wave per row
__global__ void mlp_out_kernel(int64_t M, const __bf16 *h3, const float *W4, const float *b4,
                               float *y)
{
    int64_t r = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    if (r >= M) return;
    float s = 0.f;
    for (int j = lane; j < MLP_H; j += 64) s += W4[j] * (float)h3[r * MLP_H + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) y[r] = s + b4[0];
}

// column sums over the batch: bias gradients (rows of a feature-major bf16
// matrix), and the output-layer gradients from dy and h3
// ---------------------------------------------------------------------------
// One training batch's rows, forward and back, 16 rows per workgroup.  Every
// product of the forward pass and of the deltas is C[16][256] = A[16][K] B^T
// for the workgroup's own rows (the 4 waves take 64 columns each, lane l the
// rows 4 (l / 16) + i and the columns 16 j + l % 16 of its wave's part, as in
// gemm_tile), so the whole chain runs in one workgroup with the layer inputs
// in LDS and the pre-activations in registers, and only the sums over the
// batch (weight, bias and output-layer gradients) are left to later
// launches.  The rows, products and epilogues are those of the separate
// kernels (train_rows_kernel, gemm_tile with its bias + SiLU and SiLU'
// epilogues), the same operations in the same order; the output layer's
// row sum W4 . h3 runs over the 16 lanes of a row group and then over the 4
// waves (out_train_kernel sums in another order, so y and dy can differ in
// their last bits between the two paths).  Writes XT, t, h1T, h2T, h3T
// (feature-major, for the weight gradients), dy and sq (output layer,
// loss) and the feature-major deltas dT3, dT2, dT1.
struct SliceArgs {
    int64_t n_src, b, M;  // source pairs, batch rows, padded rows
    const double *u, *y;
    int ndim;
    uint64_t seed, step;
    const float *in_mu, *in_isig;
    double mu, inv_sig, clip, top;
    const float *p;  // fp32 master parameters (biases, W4, b4)
    const __bf16 *W1p, *W2, *W3, *W2T, *W3T;
    __bf16 *XT, *h1T, *h2T, *h3T, *dT3, *dT2, *dT1;
    float *t, *dy;
    double *sq;
};

// A product C[16][64] = A[16][K] B^T of one wave (columns col0 .. col0 + 63
// of B^T: global, N x K, row stride K; A in LDS, row stride lds), in two
// halves so that the weight fragments of the next product can be in
// flight while the current one finishes: slice_weights loads all of the
// wave's fragments (K / 32 k-steps of four 16-column blocks), slice_mfma
// runs the products in k order (as gemm_tile does: the same sums).
template <int K>
__device__ __forceinline__ void slice_weights(const __bf16 *B, int col0, bf16x8 (&b)[K / 32][4])
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const __bf16 *Br = B + (size_t)(col0 + r) * K + 8 * q;
#pragma unroll
    for (int t = 0; t < K / 32; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) b[t][j] = *reinterpret_cast<const bf16x8 *>(Br + (size_t)(16 * j) * K + 32 * t);
}

template <int K>
__device__ __forceinline__ void slice_mfma(const __bf16 *A, int lds, const bf16x8 (&b)[K / 32][4],
                                           f32x4 (&acc)[4])
{
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const __bf16 *Ar = A + r * lds + 8 * q;
    bf16x8 av[K / 32];
#pragma unroll
    for (int t = 0; t < K / 32; ++t) av[t] = *reinterpret_cast<const bf16x8 *>(Ar + 32 * t);
#pragma unroll
    for (int t = 0; t < K / 32; ++t)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[t], b[t][j], acc[j], 0, 0, 0);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void train_slice_kernel(SliceArgs a)
{
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
    constexpr int XS = MLP_KIN + 8, HS = MLP_H + 8;  // LDS row strides (bf16), padded
    __shared__ __attribute__((aligned(16))) __bf16 sX[16 * XS];
    __shared__ __attribute__((aligned(16))) __bf16 sA[16 * HS], sB[16 * HS];
    __shared__ float s_y[4][16];
    __shared__ float s_t[16];
    // biases b1, b2, b3, the output weights W4, b4 and the input
    // standardisation in LDS: read once at the start, before the weight
    // prefetches (a later global load would wait for every load in flight)
    __shared__ float s_b[3][MLP_H], s_w4[MLP_H], s_b4, s_inmu[MLP_KIN], s_inis[MLP_KIN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r = lane & 15, q = lane >> 4;
    const int64_t row0 = (int64_t)blockIdx.x * 16, M = a.M;
    const int col0 = wave * 64;
    bf16x8 w1[1][4], wa[MLP_H / 32][4], wb[MLP_H / 32][4];
    {
        const int i = threadIdx.x;
        const float v1 = a.p[MLP_OFF_B1 + i], v2 = a.p[MLP_OFF_B2 + i], v3 = a.p[MLP_OFF_B3 + i];
        const float v4 = a.p[MLP_OFF_W4 + i];
        const float vm = i < MLP_KIN ? a.in_mu[i] : 0.f, vs = i < MLP_KIN ? a.in_isig[i] : 0.f;
        const float vb = i == 0 ? a.p[MLP_OFF_B4] : 0.f;
        s_b[0][i] = v1, s_b[1][i] = v2, s_b[2][i] = v3, s_w4[i] = v4;
        if (i < MLP_KIN) s_inmu[i] = vm, s_inis[i] = vs;
        if (i == 0) s_b4 = vb;
    }
    __syncthreads();
    // -- the training rows (train_rows_kernel's draws and formulas), 16
    // threads per row, two inputs each; the row's draw is made by all 16
    {
        const int rl = threadIdx.x >> 4, c0 = 2 * (threadIdx.x & 15);
        const int64_t rr = row0 + rl;
        const bool live = rr < a.b;  // padding rows hold zeros
        int64_t j = 0;
        if (live) {
            U4 qq = philox4x64((uint64_t)rr, a.step, 1, P_MLP, a.seed, 0);
            j = (int64_t)(u01(qq.x[0]) * (double)a.n_src);
            if (j >= a.n_src) j = a.n_src - 1;
        }
        // unconditional loads (clamped indices; the values are selected
        // below): a load under a branch would make the compiler wait for
        // every load in flight, the weight prefetch included
        const int ca = min(c0, a.ndim - 1), cb = min(c0 + 1, a.ndim - 1);
        const double yj = a.y[j], u0 = a.u[j * a.ndim + ca], u1 = a.u[j * a.ndim + cb];
        // the weights of the first two products go out after the rows' loads
        // (so the rows wait only for their own) and stay in flight meanwhile;
        // each later product's are loaded while the one before it finishes
        slice_weights<MLP_KIN>(a.W1p, col0, w1);
        slice_weights<MLP_H>(a.W2, col0, wa);
        if (c0 == 0) {
            const float tv = live ? (float)((target_z(yj, a.clip, a.top) - a.mu) * a.inv_sig) : 0.f;
            if (live) a.t[rr] = tv;
            s_t[rl] = tv;
        }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int c = c0 + e;
            const float v = (live && c < a.ndim) ? ((float)(e ? u1 : u0) - s_inmu[c]) * s_inis[c] : 0.0f;
            const __bf16 h = (__bf16)v;
            sX[rl * XS + c] = h;
            a.XT[(size_t)c * M + rr] = h;
        }
    }
    __syncthreads();
    f32x4 acc[4];
    float z1[4][4], z2[4][4];
    // -- layer 1: h1 = silu(X W1^T + b1)
    slice_mfma<MLP_KIN>(sX, XS, w1, acc);
    slice_weights<MLP_H>(a.W3, col0, wb);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = col0 + 16 * j + r;
        const float bc = s_b[0][col];
        __bf16 h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            z1[j][i] = acc[j][i] + bc;
            h[i] = (__bf16)mlp_silu(z1[j][i]);
            sA[(4 * q + i) * HS + col] = h[i];
        }
        *reinterpret_cast<bf16x4 *>(a.h1T + (size_t)col * M + row0 + 4 * q) = (bf16x4){h[0], h[1], h[2], h[3]};
    }
    __syncthreads();
    // -- layer 2: h2 = silu(h1 W2^T + b2)
    slice_mfma<MLP_H>(sA, HS, wa, acc);
    slice_weights<MLP_H>(a.W3T, col0, wa);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = col0 + 16 * j + r;
        const float bc = s_b[1][col];
        __bf16 h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            z2[j][i] = acc[j][i] + bc;
            h[i] = (__bf16)mlp_silu(z2[j][i]);
            sB[(4 * q + i) * HS + col] = h[i];
        }
        *reinterpret_cast<bf16x4 *>(a.h2T + (size_t)col * M + row0 + 4 * q) = (bf16x4){h[0], h[1], h[2], h[3]};
    }
    __syncthreads();
    // -- layer 3 and the output layer: h3 = silu(h2 W3^T + b3), y = W4 . h3 + b4,
    // dy = 2 (y - t) / n, the squared error, d3 = dy W4 silu'(z3)
    slice_mfma<MLP_H>(sB, HS, wb, acc);
    slice_weights<MLP_H>(a.W2T, col0, wb);
    {
        float zz[4][4], py[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = col0 + 16 * j + r;
            const float bc = s_b[2][col], w = s_w4[col];
            __bf16 h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                zz[j][i] = acc[j][i] + bc;
                h[i] = (__bf16)mlp_silu(zz[j][i]);
                py[i] += w * (float)h[i];
            }
            *reinterpret_cast<bf16x4 *>(a.h3T + (size_t)col * M + row0 + 4 * q) = (bf16x4){h[0], h[1], h[2], h[3]};
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) py[i] += __shfl_xor(py[i], o, 64);
        if (r == 0)
#pragma unroll
            for (int i = 0; i < 4; ++i) s_y[wave][4 * q + i] = py[i];
        __syncthreads();  // also: every wave is done reading h1 from sA
        float dyr[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rl = 4 * q + i;
            const int64_t row = row0 + rl;
            const float yr = s_y[0][rl] + s_y[1][rl] + s_y[2][rl] + s_y[3][rl] + s_b4;
            float dv = 0.f;
            double e2 = 0.0;
            if (row < a.b) {
                const float e = yr - s_t[rl];
                e2 = (double)e * e;
                dv = 2.0f * e / (float)a.b;
            }
            dyr[i] = dv;
            if (wave == 0 && r == 0) {
                a.dy[row] = dv;
                a.sq[row] = e2;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = col0 + 16 * j + r;
            const float w = s_w4[col];
            __bf16 dv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = zz[j][i], sg = mlp_sigmoid(z);
                dv[i] = (__bf16)(dyr[i] * w * sg * (1.0f + z * (1.0f - sg)));
                sA[(4 * q + i) * HS + col] = dv[i];
            }
            *reinterpret_cast<bf16x4 *>(a.dT3 + (size_t)col * M + row0 + 4 * q) = (bf16x4){dv[0], dv[1], dv[2], dv[3]};
        }
    }
    __syncthreads();
    // -- d2 = (d3 W3) silu'(z2) (B^T = W3T)
    slice_mfma<MLP_H>(sA, HS, wa, acc);
    __syncthreads();  // every wave is done reading h2 from sB
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = col0 + 16 * j + r;
        __bf16 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = z2[j][i], sg = mlp_sigmoid(z);
            v[i] = (__bf16)(acc[j][i] * sg * (1.0f + z * (1.0f - sg)));
            sB[(4 * q + i) * HS + col] = v[i];
        }
        *reinterpret_cast<bf16x4 *>(a.dT2 + (size_t)col * M + row0 + 4 * q) = (bf16x4){v[0], v[1], v[2], v[3]};
    }
    __syncthreads();
    // -- d1 = (d2 W2) silu'(z1) (B^T = W2T)
    slice_mfma<MLP_H>(sB, HS, wb, acc);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = col0 + 16 * j + r;
        __bf16 v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = z1[j][i], sg = mlp_sigmoid(z);
            v[i] = (__bf16)(acc[j][i] * sg * (1.0f + z * (1.0f - sg)));
        }
        *reinterpret_cast<bf16x4 *>(a.dT1 + (size_t)col * M + row0 + 4 * q) = (bf16x4){v[0], v[1], v[2], v[3]};
    }
}

// Sum of row[0 .. M) by a workgroup of 256 threads in a fixed order (thread
// t adds rows t, t + 256, ...; then a tree over the threads); the result in
// part[0].
__device__ __forceinline__ void block_rowsum(int64_t M, const __bf16 *row, float *part)
{
    float acc = 0.f;
    for (int64_t r = threadIdx.x; r < M; r += 256) acc += (float)row[r];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void rowsum_kernel(int64_t M, const __bf16 *dT, float *out)
{
    __shared__ float part[256];
    block_rowsum(M, dT + (size_t)blockIdx.x * M, part);
    if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// Workgroup c of the output-layer reductions (256 threads, fixed order):
// c < MLP_H: dW4[c] = sum dy h3[., c]; c = MLP_H: db4 = sum dy (returned by
// thread 0); c = MLP_H + 1: the batch loss, the mean of the n squared
// errors sq (padding rows hold 0), written to *loss.
__device__ __forceinline__ float out_grad_block(int c, int64_t n, int64_t M, const float *dy,
                                                const __bf16 *h3T, const double *sq, double *loss)
{
    if (c == MLP_H + 1) {
        __shared__ double lpart[256];
        double acc = 0.0;
        for (int64_t r = threadIdx.x; r < M; r += 256) acc += sq[r];
        lpart[threadIdx.x] = acc;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) lpart[threadIdx.x] += lpart[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) *loss = lpart[0] / (double)n;
        return 0.f;
    }
    __shared__ float part[256];
    float acc = 0.f;
    for (int64_t r = threadIdx.x; r < M; r += 256)
        acc += dy[r] * (c < MLP_H ? (float)h3T[(size_t)c * M + r] : 1.0f);
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    return part[0];
}

// Output-layer gradients and the batch loss (MLP_H + 2 workgroups).
__global__ __launch_bounds__(256) void out_grad_kernel(int64_t n, int64_t M, const float *dy,
                                                       const __bf16 *h3T, const double *sq,
                                                       float *gW4, float *gb4, double *loss)
{
    const int c = blockIdx.x;
    const float v = out_grad_block(c, n, M, dy, h3T, sq, loss);
    if (threadIdx.x == 0 && c < MLP_H) gW4[c] = v;
    if (threadIdx.x == 0 && c == MLP_H) gb4[0] = v;
}

// Output layer of the training rows, one wave per row: y = W4 . h3[r] + b4,
// dy = 2 (y - t) / n (0 on padding rows), the squared error (y - t)^2 into
// sq[r] (0 on padding rows), and the last hidden layer's delta
// d3 = dy W4 silu'(a3) in bf16, row-major (d) and feature-major (dT).
__global__ void out_train_kernel(int64_t n, int64_t M, const __bf16 *h3, const float *W4,
                                 const float *b4, const float *t, const float *a3, float *y,
                                 float *dy, double *sq, __bf16 *d, __bf16 *dT)
{
    const int64_t r = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (r >= M) return;
    float s = 0.f;
    for (int j = lane; j < MLP_H; j += 64) s += W4[j] * (float)h3[r * MLP_H + j];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const float yr = s + b4[0];
    float dyr = 0.f;
    double e2 = 0.0;
    if (r < n) {
        const float e = yr - t[r];
        e2 = (double)e * e;
        dyr = 2.0f * e / (float)n;
    }
    if (lane == 0) {
        y[r] = yr;
        dy[r] = dyr;
        sq[r] = e2;
    }
    for (int c = lane; c < MLP_H; c += 64) {
        const size_t i = (size_t)r * MLP_H + c;
        const float z = a3[i], sg = mlp_sigmoid(z);
        const float v = dyr * W4[c] * sg * (1.0f + z * (1.0f - sg));
        d[i] = (__bf16)v;
        dT[(size_t)c * M + r] = (__bf16)v;
    }
}

// Adam on the fp32 master parameters (bias-corrected; step t from 1) with
// the bf16 working copies written from the updated values: parameter i with
// gradient gi.
struct AdamArgs {
    float *p, *m, *v;
    float lr, b1, b2, eps, c1, c2;
    __bf16 *W1p, *W1T, *W2, *W3, *W2T, *W3T;
};

__device__ __forceinline__ void adam_update(const AdamArgs &a, int64_t i, float gi)
{
    const float mi = a.b1 * a.m[i] + (1.f - a.b1) * gi;
    const float vi = a.b2 * a.v[i] + (1.f - a.b2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    const float pi = a.p[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    a.p[i] = pi;
    const __bf16 h = (__bf16)pi;
    if (i < MLP_OFF_B1) {
        const int j1 = (int)(i / MLP_IN), c1i = (int)(i % MLP_IN);
        a.W1p[j1 * MLP_KIN + c1i] = h;
        a.W1T[(size_t)c1i * MLP_H + j1] = h;
    } else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) {
        const int64_t k = i - MLP_OFF_W2;
        a.W2[k] = h;
        a.W2T[(size_t)(k % MLP_H) * MLP_H + k / MLP_H] = h;
    } else if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) {
        const int64_t k = i - MLP_OFF_W3;
        a.W3[k] = h;
        a.W3T[(size_t)(k % MLP_H) * MLP_H + k / MLP_H] = h;
    }
}

// The gradient of W1 is read from the transposed [32][256] product gW1T,
// the rest from g.
__global__ void adam_weights_kernel(AdamArgs a, const float *g, const float *gW1T)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    const int j1 = (int)(i / MLP_IN), c1i = (int)(i % MLP_IN);
    adam_update(a, i, i < MLP_OFF_B1 ? gW1T[c1i * MLP_H + j1] : g[i]);
}

// One training step's gradient reductions and Adam in one launch (the same
// sums as the separate kernels, in the same order, so the same bits):
// workgroups below nW take 256 parameters each, the weights of layers 1-3
// as the sum of their split-K partial products in slice order (ws1 holds
// the transposed [32][256] product of layer 1); the 3 MLP_H workgroups
// after them each sum one bias gradient of layers 1-3 over the batch rows
// of the feature-major deltas dT_l and update that bias; the last MLP_H + 2
// take the output layer (W4, b4) from dy and h3 and the batch loss.
__global__ __launch_bounds__(256) void adam_reduce_kernel(AdamArgs a, const float *ws3,
                                                          const float *ws2, const float *ws1,
                                                          int S3, int S2, int S1, const __bf16 *dT3,
                                                          const __bf16 *dT2, const __bf16 *dT1,
                                                          int64_t n, int64_t M, const float *dy,
                                                          const __bf16 *h3T, const double *sq,
                                                          double *loss, int nW)
{
    __shared__ float part[256];
    if ((int)blockIdx.x >= nW + 3 * MLP_H) {
        const int c = (int)blockIdx.x - nW - 3 * MLP_H;
        const float v = out_grad_block(c, n, M, dy, h3T, sq, loss);
        if (threadIdx.x == 0 && c <= MLP_H) adam_update(a, c < MLP_H ? MLP_OFF_W4 + c : MLP_OFF_B4, v);
        return;
    }
    if ((int)blockIdx.x >= nW) {
        const int bb = (int)blockIdx.x - nW, layer = bb / MLP_H, c = bb % MLP_H;
        const __bf16 *dT = layer == 0 ? dT1 : (layer == 1 ? dT2 : dT3);
        const int64_t off = layer == 0 ? MLP_OFF_B1 : (layer == 1 ? MLP_OFF_B2 : MLP_OFF_B3);
        block_rowsum(M, dT + (size_t)c * M, part);
        if (threadIdx.x == 0) adam_update(a, off + c, part[0]);
        return;
    }
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    float gi = 0.f;
    if (i < MLP_OFF_B1) {
        const int j1 = (int)(i / MLP_IN), c1i = (int)(i % MLP_IN);
        const size_t o = (size_t)c1i * MLP_H + j1;
        for (int z = 0; z < S1; ++z) gi += ws1[(size_t)z * MLP_KIN * MLP_H + o];
    } else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) {
        const size_t o = (size_t)(i - MLP_OFF_W2);
        for (int z = 0; z < S2; ++z) gi += ws2[(size_t)z * MLP_H * MLP_H + o];
    } else if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) {
        const size_t o = (size_t)(i - MLP_OFF_W3);
        for (int z = 0; z < S3; ++z) gi += ws3[(size_t)z * MLP_H * MLP_H + o];
    } else {
        return;  // biases and the output layer: their own workgroups
    }
    adam_update(a, i, gi);
}

// bf16 working copies of the weights: W1 padded to [256][32], W2, W3 and
// their transposes
__global__ void weights_bf16_kernel(const float *p, __bf16 *W1p, __bf16 *W2, __bf16 *W3,
                                    __bf16 *W2T, __bf16 *W3T, __bf16 *W1T)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float *W1f = p + MLP_OFF_W1, *W2f = p + MLP_OFF_W2, *W3f = p + MLP_OFF_W3;
    if (i < MLP_H * MLP_KIN) {
        int j = i / MLP_KIN, c = i % MLP_KIN;
        __bf16 v = (__bf16)(c < MLP_IN ? W1f[j * MLP_IN + c] : 0.0f);
        W1p[i] = v;
        W1T[(size_t)c * MLP_H + j] = v;
    }
    if (i < MLP_H * MLP_H) {
        int j = i / MLP_H, c = i % MLP_H;
        W2[i] = (__bf16)W2f[i];
        W3[i] = (__bf16)W3f[i];
        W2T[(size_t)c * MLP_H + j] = (__bf16)W2f[i];
        W3T[(size_t)c * MLP_H + j] = (__bf16)W3f[i];
    }
}

// gradient of W1 from the transposed, padded [32][256] product
__global__ void w1_grad_kernel(const float *gT, float *gW1)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= MLP_H * MLP_IN) return;
    int j = i / MLP_IN, c = i % MLP_IN;
    gW1[i] = gT[c * MLP_H + j];
}

// Philox-uniform initial weights: U(-1, 1) / sqrt(fan_in), zero biases
__global__ void mlp_init_kernel(float *p, uint64_t seed)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= MLP_NPARAM) return;
    float fan = 0.f;
    if (i < MLP_OFF_B1) fan = (float)MLP_IN;
    else if (i >= MLP_OFF_W2 && i < MLP_OFF_B2) fan = (float)MLP_H;
    else if (i >= MLP_OFF_W3 && i < MLP_OFF_B3) fan = (float)MLP_H;
    else if (i >= MLP_OFF_W4 && i < MLP_OFF_B4) fan = (float)MLP_H;
    if (fan == 0.f) {
        p[i] = 0.f;
        return;
    }
    U4 r = philox4x64((uint64_t)(i / 4), 0, 0, P_MLP, seed, 0);
    double u = u01(r.x[i % 4]);
    p[i] = (float)((2.0 * u - 1.0) / sqrt((double)fan));
}

// Training rows of one step: row r < b takes pair j, drawn with Philox
// (step, row), its standardised input in bf16 into X[r][0..31] and the
// feature-major XT[c][r], its normalised target into tb[r]; rows b..M-1
// get zero inputs.
__global__ void train_rows_kernel(int64_t n_src, const double *u, const double *y, int ndim,
                                  int64_t b, int64_t M, uint64_t seed, uint64_t step,
                                  const float *in_mu, const float *in_isig, __bf16 *X, __bf16 *XT,
                                  float *tb, double mu, double inv_sig, double clip, double top)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= M) return;
    int64_t j = -1;
    if (r < b) {
        U4 q = philox4x64((uint64_t)r, step, 1, P_MLP, seed, 0);
        j = (int64_t)(u01(q.x[0]) * (double)n_src);
        if (j >= n_src) j = n_src - 1;
        tb[r] = (float)((target_z(y[j], clip, top) - mu) * inv_sig);
    }
    __bf16 row[MLP_KIN];
#pragma unroll
    for (int c = 0; c < MLP_KIN; ++c) {
        const float v = (j >= 0 && c < ndim) ? ((float)u[j * ndim + c] - in_mu[c]) * in_isig[c] : 0.0f;
        row[c] = (__bf16)v;
        XT[(size_t)c * M + r] = row[c];
    }
#pragma unroll
    for (int c = 0; c < MLP_KIN; c += 8)
        *reinterpret_cast<bf16x8 *>(X + r * MLP_KIN + c) =
            (bf16x8){row[c], row[c + 1], row[c + 2], row[c + 3], row[c + 4], row[c + 5], row[c + 6], row[c + 7]};
}

__global__ void to_f32_kernel(int64_t n, const double *src, float *dst, double mu, double inv_sig,
                              double clip, double top)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = (float)((target_z(src[i], clip, top) - mu) * inv_sig);
}

__global__ void to_f64_kernel(int64_t n, const float *src, double *dst, double mu, double sig,
                              double top)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = target_from_z(mu + sig * (double)src[i], top);
}

// mean and standard deviation of the clipped targets (one workgroup)
__global__ void target_stats_kernel(int64_t n, const double *y, double clip, double top,
                                    double *out)
{
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double v = target_z(y[i], clip, top);
        a += v;
        b += v * v;
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s1[threadIdx.x] += s1[threadIdx.x + o];
            s2[threadIdx.x] += s2[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double mu = s1[0] / (double)n;
        double var = s2[0] / (double)n - mu * mu;
        out[0] = mu;
        out[1] = var > 0.0 ? sqrt(var) : 1.0;
    }
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------------------
// host-side drivers (enqueue only)
// ---------------------------------------------------------------------------
hipError_t mlp_refresh_weights(MlpBuffers &B, hipStream_t s)
{
    weights_bf16_kernel<<<nblk(MLP_H * MLP_H, 256), 256, 0, s>>>(B.p, B.W1p, B.W2, B.W3, B.W2T, B.W3T,
                                                               B.W1T);
    return hipGetLastError();
}

hipError_t mlp_init_params(MlpBuffers &B, uint64_t seed, hipStream_t s)
{
    mlp_init_kernel<<<nblk(MLP_NPARAM, 256), 256, 0, s>>>(B.p, seed);
    hipError_t e = hipMemsetAsync(B.m, 0, sizeof(float) * MLP_NPARAM, s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(B.v, 0, sizeof(float) * MLP_NPARAM, s);
    if (e != hipSuccess) return e;
    return mlp_refresh_weights(B, s);
}

// Forward of M (multiple of 16) rows already in B.X through the hidden
// layers, and with `out` the output layer into B.y; keeps activations.
static void forward_rows(MlpBuffers &B, int64_t M, bool keep_T, bool out, hipStream_t s)
{
    const float *p = B.p;
    // each product's epilogue adds the bias and applies SiLU (pre-activation
    // kept for the backward pass, activations row- and feature-major)
    GemmEpi e1, e2, e3;
    e1.bias = p + MLP_OFF_B1, e1.H = B.h1, e1.HT = keep_T ? B.h1T : nullptr;
    e2.bias = p + MLP_OFF_B2, e2.H = B.h2, e2.HT = keep_T ? B.h2T : nullptr;
    e3.bias = p + MLP_OFF_B3, e3.H = B.h3, e3.HT = keep_T ? B.h3T : nullptr;
    gemm_nt((int)M, MLP_H, MLP_KIN, B.X, MLP_KIN, B.W1p, MLP_KIN, B.a1, MLP_H, 0.f, s, nullptr, EPI_BIAS_SILU, e1);
    gemm_nt((int)M, MLP_H, MLP_H, B.h1, MLP_H, B.W2, MLP_H, B.a2, MLP_H, 0.f, s, nullptr, EPI_BIAS_SILU, e2);
    gemm_nt((int)M, MLP_H, MLP_H, B.h2, MLP_H, B.W3, MLP_H, B.a3, MLP_H, 0.f, s, nullptr, EPI_BIAS_SILU, e3);
    if (out) mlp_out_kernel<<<nblk(M, 4), 256, 0, s>>>(M, B.h3, p + MLP_OFF_W4, p + MLP_OFF_B4, B.y);
}

hipError_t mlp_forward(MlpBuffers &B, const double *u, int ndim, int64_t n, double *out,
                       hipStream_t s)
{
    for (int64_t r0 = 0; r0 < n; r0 += B.max_rows) {
        int64_t nr = n - r0 < B.max_rows ? n - r0 : B.max_rows;
        int64_t M = (nr + 31) / 32 * 32;
        mlp_input_kernel<<<nblk(M * MLP_KIN, 256), 256, 0, s>>>(u + r0 * ndim, ndim, nr, M, B.in_mu,
                                                                B.in_isig, B.X);
        forward_rows(B, M, false, true, s);
        to_f64_kernel<<<nblk(nr, 256), 256, 0, s>>>(nr, B.y, out + r0, B.mu, B.sig,
                                                        B.top);
    }
    return hipGetLastError();
}

// Loss and gradient of one batch of n <= max_rows rows with targets t
// (already normalised, fp32): forward, backward, gradient in B.g (the W1
// part only with w1_to_g; B.gtmp holds it transposed either way).
static void loss_grad_rows(MlpBuffers &B, int64_t n, const float *t, bool w1_to_g, hipStream_t s)
{
    const int64_t M = (n + 31) / 32 * 32;
    const float *p = B.p;
    float *g = B.g;
    const size_t RH = (size_t)B.max_rows * MLP_H, WS = (size_t)MLP_SPLITK * MLP_H * MLP_H;
    __bf16 *dT3 = B.dT, *dT2 = B.dT + RH, *dT1 = B.dT + 2 * RH;
    float *ws3 = B.ws, *ws2 = B.ws + WS, *ws1 = B.ws + 2 * WS;
    forward_rows(B, M, true, false, s);
    // output layer: forward, loss terms and the delta of the last hidden layer
    out_train_kernel<<<nblk(M, 4), 256, 0, s>>>(n, M, B.h3, p + MLP_OFF_W4, p + MLP_OFF_B4, t, B.a3,
                                                 B.y, B.dy, B.sq, B.d, dT3);
    out_grad_kernel<<<MLP_H + 2, 256, 0, s>>>(n, M, B.dy, B.h3T, B.sq, g + MLP_OFF_W4, g + MLP_OFF_B4,
                                              B.loss);
    // layer 3: dW3 = d3^T h2, db3 = sum d3, d2 = (d3 W3) silu'(a2)
    gemm_nt(MLP_H, MLP_H, (int)M, dT3, (int)M, B.h2T, (int)M, g + MLP_OFF_W3, MLP_H, 0.f, s, ws3);
    rowsum_kernel<<<MLP_H, 256, 0, s>>>(M, dT3, g + MLP_OFF_B3);
    // (the product reads d3 from B.d while other waves write d2: d2 goes to B.d2)
    GemmEpi b2;
    b2.Z = B.a2, b2.H = B.d2, b2.HT = dT2;
    gemm_nt((int)M, MLP_H, MLP_H, B.d, MLP_H, B.W3T, MLP_H, B.gtmp, MLP_H, 0.f, s, nullptr, EPI_DSILU, b2);
    // layer 2
    gemm_nt(MLP_H, MLP_H, (int)M, dT2, (int)M, B.h1T, (int)M, g + MLP_OFF_W2, MLP_H, 0.f, s, ws2);
    rowsum_kernel<<<MLP_H, 256, 0, s>>>(M, dT2, g + MLP_OFF_B2);
    GemmEpi b1;
    b1.Z = B.a1, b1.H = B.d, b1.HT = dT1;
    gemm_nt((int)M, MLP_H, MLP_H, B.d2, MLP_H, B.W2T, MLP_H, B.gtmp, MLP_H, 0.f, s, nullptr, EPI_DSILU, b1);
    // layer 1: dW1^T = X^T d1 as a [32][256] product (inputs feature-major)
    gemm_nt(MLP_KIN, MLP_H, (int)M, B.XT, (int)M, dT1, (int)M, B.gtmp, MLP_H, 0.f, s, ws1);
    if (w1_to_g) w1_grad_kernel<<<nblk(MLP_H * MLP_IN, 256), 256, 0, s>>>(B.gtmp, g + MLP_OFF_W1);
    rowsum_kernel<<<MLP_H, 256, 0, s>>>(M, dT1, g + MLP_OFF_B1);
}

__global__ void transpose_x_kernel(int64_t M, const __bf16 *X, __bf16 *XT)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= M * MLP_KIN) return;
    int64_t r = i / MLP_KIN;
    int c = (int)(i % MLP_KIN);
    XT[(size_t)c * M + r] = X[i];
}

hipError_t mlp_loss_grad(MlpBuffers &B, const double *u, int ndim, const double *y, int64_t n,
                         hipStream_t s)
{
    const int64_t M = (n + 31) / 32 * 32;
    mlp_input_kernel<<<nblk(M * MLP_KIN, 256), 256, 0, s>>>(u, ndim, n, M, B.in_mu, B.in_isig, B.X);
    transpose_x_kernel<<<nblk(M * MLP_KIN, 256), 256, 0, s>>>(M, B.X, B.XT);
    to_f32_kernel<<<nblk(n, 256), 256, 0, s>>>(n, y, B.t, B.mu, 1.0 / B.sig, B.clip,
                                                 B.top);
    loss_grad_rows(B, n, B.t, true, s);
    return hipGetLastError();
}

hipError_t mlp_input_stats(MlpBuffers &B, const double *u, int ndim, int64_t n, hipStream_t s)
{
    input_stats_kernel<<<MLP_KIN, 256, 0, s>>>(n, u, ndim, B.in_mu, B.in_isig);
    return hipGetLastError();
}

hipError_t mlp_target_stats(MlpBuffers &B, const double *y, int64_t n, hipStream_t s)
{
    target_stats_kernel<<<1, 256, 0, s>>>(n, y, B.clip, B.top, B.stats);
    return hipGetLastError();
}

hipError_t mlp_train_step(MlpBuffers &B, const double *u, const double *y, int ndim, int64_t n_src,
                          int64_t batch, uint64_t seed, int64_t step, float lr, hipStream_t s)
{
    const int64_t M = (batch + 31) / 32 * 32;
    AdamArgs a;
    a.p = B.p, a.m = B.m, a.v = B.v;
    a.lr = lr, a.b1 = 0.9f, a.b2 = 0.999f, a.eps = 1e-8f;
    a.c1 = 1.0f - powf(a.b1, (float)step), a.c2 = 1.0f - powf(a.b2, (float)step);
    a.W1p = B.W1p, a.W1T = B.W1T, a.W2 = B.W2, a.W3 = B.W3, a.W2T = B.W2T, a.W3T = B.W3T;
    int kc3 = 0, kc1 = 0;
    const int S3 = splitk_slices(MLP_H, MLP_H, (int)M, &kc3), S1 = splitk_slices(MLP_KIN, MLP_H, (int)M, &kc1);
    if (S3 > 1 && S1 > 1) {
        // three launches: the rows forward and back, 16 per workgroup; the
        // weight-gradient slices; Adam with every reduction over the batch
        const size_t RH = (size_t)B.max_rows * MLP_H, WS = (size_t)MLP_SPLITK * MLP_H * MLP_H;
        __bf16 *dT3 = B.dT, *dT2 = B.dT + RH, *dT1 = B.dT + 2 * RH;
        SliceArgs sa;
        sa.n_src = n_src, sa.b = batch, sa.M = M, sa.u = u, sa.y = y, sa.ndim = ndim;
        sa.seed = seed, sa.step = (uint64_t)step, sa.in_mu = B.in_mu, sa.in_isig = B.in_isig;
        sa.mu = B.mu, sa.inv_sig = 1.0 / B.sig, sa.clip = B.clip, sa.top = B.top, sa.p = B.p;
        sa.W1p = B.W1p, sa.W2 = B.W2, sa.W3 = B.W3, sa.W2T = B.W2T, sa.W3T = B.W3T;
        sa.XT = B.XT, sa.h1T = B.h1T, sa.h2T = B.h2T, sa.h3T = B.h3T, sa.dT3 = dT3, sa.dT2 = dT2, sa.dT1 = dT1;
        sa.t = B.t, sa.dy = B.dy, sa.sq = B.sq;
        train_slice_kernel<<<(unsigned)(M / 16), 256, 0, s>>>(sa);
        const GemmArgs w3 = {MLP_H, MLP_H, (int)M, dT3, (int)M, B.h2T, (int)M, B.ws, MLP_H, 0.f, kc3, GemmEpi()};
        const GemmArgs w2 = {MLP_H, MLP_H, (int)M, dT2, (int)M, B.h1T, (int)M, B.ws + WS, MLP_H, 0.f, kc3, GemmEpi()};
        const GemmArgs w1 = {MLP_KIN, MLP_H, (int)M, B.XT, (int)M, dT1, (int)M, B.ws + 2 * WS, MLP_H, 0.f, kc1, GemmEpi()};
        gemm_wgrad3_kernel<<<2 * (MLP_H / 16) * S3 + (MLP_KIN / 16) * S1, 256, 0, s>>>(w3, w2, w1);
        const int nW = (int)nblk(MLP_NPARAM, 256);
        adam_reduce_kernel<<<nW + 4 * MLP_H + 2, 256, 0, s>>>(a, B.ws, B.ws + WS, B.ws + 2 * WS, S3, S3, S1,
                                                              B.dT, B.dT + RH, B.dT + 2 * RH, batch, M,
                                                              B.dy, B.h3T, B.sq, B.loss, nW);
    } else {
        train_rows_kernel<<<nblk(M, 256), 256, 0, s>>>(n_src, u, y, ndim, batch, M, seed, (uint64_t)step,
                                                       B.in_mu, B.in_isig, B.X, B.XT, B.t, B.mu,
                                                       1.0 / B.sig, B.clip, B.top);
        loss_grad_rows(B, batch, B.t, false, s);
        adam_weights_kernel<<<nblk(MLP_NPARAM, 256), 256, 0, s>>>(a, B.g, B.gtmp);
    }
    return hipGetLastError();
}

}  // namespace nsmi
