/*
 * Oracle for the learned surrogate: a fully connected network
 * 11 -> 256 -> 256 -> 256 -> 1 with SiLU activations, its mean-squared-error
 * gradient and the Adam update, in FP64 with plain loops.
 *
 * TEST INFRASTRUCTURE ONLY (see nsmi_oracle.c).  The paper names batched
 * machine-learning models as a natural companion of the batched sampler
 * (Sec. 5) without fixing one; the architecture, loss and optimiser follow
 * the workload definition.  Pinned against PyTorch float64 (forward and
 * autograd) and central finite differences in tests/test_oracle_mlp.py.
 *
 * Parameter layout (one flat array): W1[256][11], b1[256], W2[256][256],
 * b2[256], W3[256][256], b3[256], W4[256], b4[1]; weights row-major with the
 * output index first.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MLP_IN 11
#define MLP_H 256

int64_t or_mlp_num_params(void)
{
    return (int64_t)MLP_H * MLP_IN + MLP_H + 2 * ((int64_t)MLP_H * MLP_H + MLP_H) + MLP_H + 1;
}

static void or_mlp_offsets(int64_t *o)
{
    o[0] = 0;                                   /* W1 */
    o[1] = o[0] + (int64_t)MLP_H * MLP_IN;      /* b1 */
    o[2] = o[1] + MLP_H;                        /* W2 */
    o[3] = o[2] + (int64_t)MLP_H * MLP_H;       /* b2 */
    o[4] = o[3] + MLP_H;                        /* W3 */
    o[5] = o[4] + (int64_t)MLP_H * MLP_H;       /* b3 */
    o[6] = o[5] + MLP_H;                        /* W4 */
    o[7] = o[6] + MLP_H;                        /* b4 */
}

static double or_sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }
static double or_silu(double z) { return z * or_sigmoid(z); }
/* d/dz [z sigma(z)] = sigma(z) (1 + z (1 - sigma(z))) */
static double or_dsilu(double z)
{
    double s = or_sigmoid(z);
    return s * (1.0 + z * (1.0 - s));
}

/* One sample: pre-activations a1..a3 and activations h1..h3 (each MLP_H). */
static double or_mlp_one(const double *p, const double *x, double *a, double *h)
{
    int64_t o[8];
    or_mlp_offsets(o);
    const double *W1 = p + o[0], *b1 = p + o[1], *W2 = p + o[2], *b2 = p + o[3];
    const double *W3 = p + o[4], *b3 = p + o[5], *W4 = p + o[6], *b4 = p + o[7];
    double *a1 = a, *a2 = a + MLP_H, *a3 = a + 2 * MLP_H;
    double *h1 = h, *h2 = h + MLP_H, *h3 = h + 2 * MLP_H;
    for (int j = 0; j < MLP_H; ++j) {
        double s = b1[j];
        for (int i = 0; i < MLP_IN; ++i) s += W1[j * MLP_IN + i] * x[i];
        a1[j] = s;
        h1[j] = or_silu(s);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double s = b2[j];
        for (int i = 0; i < MLP_H; ++i) s += W2[j * MLP_H + i] * h1[i];
        a2[j] = s;
        h2[j] = or_silu(s);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double s = b3[j];
        for (int i = 0; i < MLP_H; ++i) s += W3[j * MLP_H + i] * h2[i];
        a3[j] = s;
        h3[j] = or_silu(s);
    }
    double y = b4[0];
    for (int i = 0; i < MLP_H; ++i) y += W4[i] * h3[i];
    return y;
}

/* Network output for one input x[11] (the surrogate screen of the
 * delayed-acceptance walk evaluates it point by point). */
double or_mlp_eval1(const double *p, const double *x)
{
    double a[3 * MLP_H], h[3 * MLP_H];
    return or_mlp_one(p, x, a, h);
}

/* Forward pass of n samples x[n][11] -> y[n]. */
void or_mlp_forward(const double *p, const double *x, int64_t n, double *y)
{
#pragma omp parallel
    {
        double *a = (double *)malloc(sizeof(double) * 3 * MLP_H);
        double *h = (double *)malloc(sizeof(double) * 3 * MLP_H);
#pragma omp for schedule(static)
        for (int64_t b = 0; b < n; ++b) y[b] = or_mlp_one(p, x + b * MLP_IN, a, h);
        free(a);
        free(h);
    }
}

/* Loss (1/n) sum_b (y_b - t_b)^2 and its gradient with respect to every
 * parameter (written to g, same layout as p).  Returns the loss. */
double or_mlp_loss_grad(const double *p, const double *x, const double *t, int64_t n, double *g)
{
    int64_t o[8];
    or_mlp_offsets(o);
    const int64_t P = or_mlp_num_params();
    const double *W2 = p + o[2], *W3 = p + o[4], *W4 = p + o[6];
    memset(g, 0, sizeof(double) * P);
    double *a = (double *)malloc(sizeof(double) * 3 * MLP_H);
    double *h = (double *)malloc(sizeof(double) * 3 * MLP_H);
    double *d3 = (double *)malloc(sizeof(double) * MLP_H);
    double *d2 = (double *)malloc(sizeof(double) * MLP_H);
    double *d1 = (double *)malloc(sizeof(double) * MLP_H);
    double loss = 0.0;
    for (int64_t b = 0; b < n; ++b) {
        const double *xb = x + b * MLP_IN;
        double y = or_mlp_one(p, xb, a, h);
        double r = y - t[b];
        loss += r * r;
        double dy = 2.0 * r / (double)n;
        const double *h1 = h, *h2 = h + MLP_H, *h3 = h + 2 * MLP_H;
        const double *a1 = a, *a2 = a + MLP_H, *a3 = a + 2 * MLP_H;
        /* output layer */
        g[o[7]] += dy;
        for (int i = 0; i < MLP_H; ++i) g[o[6] + i] += dy * h3[i];
        for (int i = 0; i < MLP_H; ++i) d3[i] = dy * W4[i] * or_dsilu(a3[i]);
        /* layer 3 */
        for (int j = 0; j < MLP_H; ++j) {
            g[o[5] + j] += d3[j];
            for (int i = 0; i < MLP_H; ++i) g[o[4] + j * MLP_H + i] += d3[j] * h2[i];
        }
        for (int i = 0; i < MLP_H; ++i) {
            double s = 0.0;
            for (int j = 0; j < MLP_H; ++j) s += W3[j * MLP_H + i] * d3[j];
            d2[i] = s * or_dsilu(a2[i]);
        }
        /* layer 2 */
        for (int j = 0; j < MLP_H; ++j) {
            g[o[3] + j] += d2[j];
            for (int i = 0; i < MLP_H; ++i) g[o[2] + j * MLP_H + i] += d2[j] * h1[i];
        }
        for (int i = 0; i < MLP_H; ++i) {
            double s = 0.0;
            for (int j = 0; j < MLP_H; ++j) s += W2[j * MLP_H + i] * d2[j];
            d1[i] = s * or_dsilu(a1[i]);
        }
        /* layer 1 */
        for (int j = 0; j < MLP_H; ++j) {
            g[o[1] + j] += d1[j];
            for (int i = 0; i < MLP_IN; ++i) g[o[0] + j * MLP_IN + i] += d1[j] * xb[i];
        }
    }
    free(a); free(h); free(d3); free(d2); free(d1);
    return loss / (double)n;
}

/* Adam (Kingma & Ba 2015) with bias correction; step t counts from 1. */
void or_adam_step(double *p, const double *g, double *m, double *v, int64_t n, int64_t t, double lr,
                  double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        p[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
