// Host runtime behind the C ABI of include/nsmi.h: argument checks, device
// buffers, event upload, and the launch sequence of one batched iteration.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/nsmi.h"
#include "nsmi_hrss.h"
#include "nsmi_kernels.h"
#include "nsmi_mlp.h"

using namespace nsmi;

namespace {

thread_local std::string g_init_error;

struct EventBuffers {
    double *data = nullptr, *psd = nullptr;
    char *rows64 = nullptr, *rows32 = nullptr;
    char *rb_rows = nullptr;          // relative-binning table (likelihood NS_LIKE_GW_RB)
    int32_t *rb_edges = nullptr;
    double *rb_theta0 = nullptr;
    double *K = nullptr;
    int n_bins = 0, n_det = 0;
};

}  // namespace

struct ns_ctx {
    ns_config cfg{};
    int n_events = 0, ndim = 0, n_live = 0, max_det = 1;
    double delay = 0.0;
    hipStream_t stream = nullptr;
    std::vector<EventBuffers> evb;
    std::vector<DevEvent> hev;  // host copies of the device descriptors
    DevEvent *d_ev = nullptr;
    EvState *d_st = nullptr;
    double *live_u[2] = {nullptr, nullptr}, *live_L[2] = {nullptr, nullptr};
    int cur = 0;
    double *snap_u = nullptr, *snap_L = nullptr, *chain_u = nullptr, *chain_L = nullptr;
    int64_t *chain_stats = nullptr;
    int32_t *d_order = nullptr;  // events by decreasing walk cost (several events)
    double *dead_u = nullptr, *dead_L = nullptr, *dead_logw = nullptr, *dead_nlive = nullptr;
    int64_t dead_cap = 0;
    int64_t dead_bound = 0;  // upper bound on dead rows per event (host-side count)
    int wpc = 0;             // waves per chain of the walk kernel (0: automatic)
    // iteration graphs (NS_FLAG_GRAPH): one per live-buffer parity
    bool use_graph = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    hipGraph_t graph[2] = {nullptr, nullptr};
    int g_k[2] = {0, 0}, g_walk[2] = {0, 0}, g_wpc[2] = {0, 0};
    int64_t g_cap[2] = {0, 0};
    bool g_da[2] = {false, false}, g_hv[2] = {false, false};
    // kernel timing (NS_FLAG_TIMING): four events per ns_step
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    ns_timing_t acc{};
    // learned surrogate
    bool mlp_ready = false;
    MlpBuffers mlp;
    bool da_on = false;
    int inner = NS_INNER_WALK;  // inner kernel of the chains
    double da_margin = 0.0, da_temp = 1.0, da_floor = 0.0;
    // harvest of exact evaluations
    double *hv_u = nullptr, *hv_L = nullptr;
    unsigned long long *hv_count = nullptr;
    int64_t hv_cap = 0;
    // convergence of each event as last read back by ns_evidence (or
    // restored): ns_step refuses a context whose events have all converged
    std::vector<char> conv_seen;
    uint64_t fingerprint = 0;  // FNV-1a over every event's grid, data and PSD
    std::string err;
};

// FNV-1a (64-bit) over raw bytes, continued from h.
static uint64_t fnv1a(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001b3ULL;
    }
    return h;
}

// Fingerprint of the events a context samples: what a checkpoint must have
// been taken on (likelihood kind, grid, dimension, data and PSD, toy width).
static uint64_t events_fingerprint(const ns_event_desc *ev, int n_events)
{
    uint64_t h = 0xcbf29ce484222325ULL;
    for (int i = 0; i < n_events; ++i) {
        const ns_event_desc &e = ev[i];
        int32_t ints[4] = {e.n_bins, e.n_det, e.ndim, e.likelihood};
        double dbl[3] = {e.f_lo, e.df, e.toy_sigma};
        h = fnv1a(h, ints, sizeof ints);
        h = fnv1a(h, dbl, sizeof dbl);
        if (e.likelihood == NS_LIKE_GW || e.likelihood == NS_LIKE_GW_RB) {
            const size_t N = (size_t)e.n_bins * e.n_det;
            h = fnv1a(h, e.data, sizeof(double) * 2 * N);
            h = fnv1a(h, e.psd, sizeof(double) * N);
        }
    }
    return h;
}

static hipError_t timing_event(ns_ctx *c, hipEvent_t *out)
{
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e;
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) return he;
        c->ev_pool.push_back(e);
    }
    *out = c->ev_pool[c->ev_used++];
    return hipSuccess;
}

// Fold the recorded event quadruples into the accumulated times.
static hipError_t timing_collect(ns_ctx *c)
{
    hipError_t he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return he;
    for (size_t i = 0; i + 3 < c->ev_used; i += 4) {
        float a = 0, b = 0, d = 0;
        if ((he = hipEventElapsedTime(&a, c->ev_pool[i], c->ev_pool[i + 1])) != hipSuccess) return he;
        if ((he = hipEventElapsedTime(&b, c->ev_pool[i + 1], c->ev_pool[i + 2])) != hipSuccess) return he;
        if ((he = hipEventElapsedTime(&d, c->ev_pool[i + 2], c->ev_pool[i + 3])) != hipSuccess) return he;
        c->acc.select_ms += a;
        c->acc.walk_ms += b;
        c->acc.finish_ms += d;
        c->acc.launches += 1;
    }
    c->ev_used = 0;
    return hipSuccess;
}

// Drop captured iteration graphs (their kernel arguments hold surrogate and
// buffer parameters that just changed).
static void invalidate_graphs(ns_ctx *c)
{
    for (int i = 0; i < 2; ++i) {
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
        if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
        c->gexec[i] = nullptr;
        c->graph[i] = nullptr;
    }
}

static ns_status fail(ns_ctx *c, ns_status s, const std::string &msg)
{
    if (c)
        c->err = msg;
    else
        g_init_error = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(ctx, NS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <class T>
static hipError_t dalloc(T **p, size_t n)
{
    return hipMalloc((void **)p, sizeof(T) * (n ? n : 1));
}

static void dfree(void *p)
{
    if (p) (void)hipFree(p);
}

static ns_status check_event(const ns_event_desc &e, int i, std::string &msg)
{
    char b[256];
    if (e.ndim != 4 && e.ndim != 11) {
        snprintf(b, sizeof b, "event %d: ndim must be 4 or 11 (got %d)", i, e.ndim);
        msg = b;
        return NS_EINVAL;
    }
    if (e.likelihood != NS_LIKE_GW && e.likelihood != NS_LIKE_GAUSS && e.likelihood != NS_LIKE_GW_RB) {
        msg = "event " + std::to_string(i) + ": unknown likelihood";
        return NS_EINVAL;
    }
    if (!e.prior_lo || !e.prior_hi || !e.fixed_theta) {
        msg = "event " + std::to_string(i) + ": prior_lo, prior_hi and fixed_theta are required";
        return NS_EINVAL;
    }
    if (e.likelihood == NS_LIKE_GAUSS) {
        if (!(e.toy_sigma > 0.0) || !std::isfinite(e.toy_sigma)) {
            msg = "event " + std::to_string(i) + ": toy_sigma must be positive";
            return NS_EINVAL;
        }
        return NS_OK;
    }
    if (e.n_bins < 1 || e.n_det < 1 || e.n_det > MAXDET) {
        snprintf(b, sizeof b, "event %d: n_bins >= 1 and 1 <= n_det <= 3 required (got %d, %d)", i,
                 e.n_bins, e.n_det);
        msg = b;
        return NS_EINVAL;
    }
    if (!(e.f_lo > 0.0) || !(e.df > 0.0) || !std::isfinite(e.f_lo) || !std::isfinite(e.df)) {
        msg = "event " + std::to_string(i) + ": f_lo and df must be positive and finite";
        return NS_EINVAL;
    }
    if (!e.data || !e.psd) {
        msg = "event " + std::to_string(i) + ": data and psd are required";
        return NS_EINVAL;
    }
    if (!e.fixed_antenna && (!e.det_tensor || !e.det_loc)) {
        msg = "event " + std::to_string(i) + ": det_tensor and det_loc are required without fixed_antenna";
        return NS_EINVAL;
    }
    size_t nb = (size_t)e.n_bins * e.n_det;
    for (size_t j = 0; j < nb; ++j) {
        if (!std::isfinite(e.psd[j]) || !(e.psd[j] > 0.0)) {
            msg = "event " + std::to_string(i) + ": psd must be finite and positive (index " +
                  std::to_string(j) + ")";
            return NS_ENONFINITE;
        }
        if (!std::isfinite(e.data[2 * j]) || !std::isfinite(e.data[2 * j + 1])) {
            msg = "event " + std::to_string(i) + ": data must be finite (index " + std::to_string(j) + ")";
            return NS_ENONFINITE;
        }
    }
    if (e.likelihood == NS_LIKE_GW_RB) {
        if (!e.rb_theta0 || !e.rb_edges || e.rb_bins < 1 || e.rb_bins > RB_MAX_BINS) {
            msg = "event " + std::to_string(i) + ": relative binning needs rb_theta0, rb_edges and 1 <= rb_bins <= 4095";
            return NS_EINVAL;
        }
        if (e.rb_edges[0] != 0 || e.rb_edges[e.rb_bins] != e.n_bins) {
            msg = "event " + std::to_string(i) + ": rb_edges must run from 0 to n_bins";
            return NS_EINVAL;
        }
        for (int b = 0; b < e.rb_bins; ++b)
            if (e.rb_edges[b + 1] <= e.rb_edges[b]) {
                msg = "event " + std::to_string(i) + ": rb_edges must be strictly increasing";
                return NS_EINVAL;
            }
        const double *t0 = e.rb_theta0;
        for (int j = 0; j < NPAR; ++j)
            if (!std::isfinite(t0[j])) {
                msg = "event " + std::to_string(i) + ": rb_theta0 must be finite";
                return NS_ENONFINITE;
            }
        if (!(t0[0] > 0.0) || !(t0[1] > 0.0 && t0[1] <= 1.0) || !(t0[4] > 0.0)) {
            msg = "event " + std::to_string(i) + ": rb_theta0 is not a valid source (Mc > 0, 0 < q <= 1, dL > 0)";
            return NS_EINVAL;
        }
    }
    for (int j = 0; j < NPAR; ++j) {
        if (!std::isfinite(e.prior_lo[j]) || !std::isfinite(e.prior_hi[j]) ||
            !std::isfinite(e.fixed_theta[j])) {
            msg = "event " + std::to_string(i) + ": non-finite prior edge or fixed parameter";
            return NS_ENONFINITE;
        }
    }
    return NS_OK;
}

static void fill_dev_event(DevEvent &d, const ns_event_desc &e)
{
    memset(&d, 0, sizeof d);
    const bool gw = e.likelihood == NS_LIKE_GW || e.likelihood == NS_LIKE_GW_RB;
    d.n_bins = gw ? e.n_bins : 0;
    d.n_pad = (d.n_bins + WAVE - 1) / WAVE * WAVE;
    d.n_det = gw ? e.n_det : 0;
    d.ndim = e.ndim;
    d.likelihood = e.likelihood;
    d.fixed_antenna = e.fixed_antenna ? 1 : 0;
    d.f_lo = e.f_lo;
    d.df = e.df;
    for (int j = 0; j < NPAR; ++j) {
        d.lo[j] = e.prior_lo[j];
        d.hi[j] = e.prior_hi[j];
        d.fixed[j] = e.fixed_theta[j];
    }
    d.cos_lo5 = cos(e.prior_lo[5]);
    d.cos_hi5 = cos(e.prior_hi[5]);
    d.sin_lo7 = sin(e.prior_lo[7]);
    d.sin_hi7 = sin(e.prior_hi[7]);
    d.fixed_cosi = cos(e.fixed_theta[5]);
    d.fixed_sindec = sin(e.fixed_theta[7]);
    d.fixed_cosdec = cos(e.fixed_theta[7]);
    d.gmst = e.gmst;
    d.toy_sigma = e.toy_sigma;
    d.wscale = 1.0;
    if (gw) {
        for (int k = 0; k < e.n_det; ++k) {
            if (e.fixed_antenna) {
                d.Fp[k] = e.fixed_antenna[2 * k];
                d.Fx[k] = e.fixed_antenna[2 * k + 1];
            } else {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b)
                        d.D[k][3 * a + b] = 0.5 * (e.det_tensor[9 * k + 3 * a + b] +
                                                    e.det_tensor[9 * k + 3 * b + a]);
                for (int a = 0; a < 3; ++a) d.loc[k][a] = e.det_loc[3 * k + a];
            }
        }
    }
}

// Upload one event's data and build its device tables.
static ns_status upload_event(ns_ctx *c, const ns_event_desc &e, EventBuffers &b, DevEvent &d)
{
    fill_dev_event(d, e);
    if (e.likelihood != NS_LIKE_GW && e.likelihood != NS_LIKE_GW_RB) return NS_OK;
    size_t N = (size_t)e.n_bins, ND = (size_t)e.n_det;
    b.n_bins = e.n_bins;
    b.n_det = e.n_det;
    HIP_TRY(c, dalloc(&b.data, 2 * N * ND));
    HIP_TRY(c, dalloc(&b.psd, N * ND));
    // tables padded to n_pad bins (a multiple of the wave width) so every
    // lane of a wave walks the same number of rows; weights for all MAXDET
    // detectors, zero beyond n_det and beyond n_bins: kernels built for more
    // detectors than this event has then read zeros, never past the end
    const size_t rows = (size_t)d.n_pad / WAVE;
    HIP_TRY(c, dalloc(&b.rows64, rows * ROW64));
    HIP_TRY(c, dalloc(&b.rows32, rows * ROW32));
    HIP_TRY(c, dalloc(&b.K, MAXDET));
    HIP_TRY(c, hipMemsetAsync(b.rows64, 0, rows * ROW64, c->stream));
    HIP_TRY(c, hipMemsetAsync(b.rows32, 0, rows * ROW32, c->stream));
    // FP32 weights are scaled by a power of two that brings the largest
    // |w| = 4 df |d| f^(-7/6) / S near 1 (exact scaling; undone in FP64)
    {
        double wmax = 0.0;
        for (size_t dd = 0; dd < ND; ++dd)
            for (size_t k = 0; k < N; ++k) {
                double f = (double)k * e.df + e.f_lo;
                double fac = 4.0 * e.df * std::pow(f, -7.0 / 6.0) / e.psd[dd * N + k];
                double a = fac * std::hypot(e.data[2 * (dd * N + k)], e.data[2 * (dd * N + k) + 1]);
                wmax = std::max(wmax, a);
            }
        int ex = 0;
        if (wmax > 0.0 && std::isfinite(wmax)) std::frexp(wmax, &ex);
        d.wscale = std::ldexp(1.0, -ex);
    }
    HIP_TRY(c, hipMemsetAsync(b.K, 0, sizeof(double) * MAXDET, c->stream));
    HIP_TRY(c, hipMemcpyAsync(b.data, e.data, sizeof(double) * 2 * N * ND, hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(b.psd, e.psd, sizeof(double) * N * ND, hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, launch_prep_event(d, b.data, b.psd, b.rows64, b.rows32, b.K, c->stream));
    double K[MAXDET] = {0, 0, 0};
    HIP_TRY(c, hipMemcpyAsync(K, b.K, sizeof(double) * ND, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < ND; ++k) d.K[k] = K[k];
    d.rows64 = b.rows64;
    d.rows32 = b.rows32;
    if (e.likelihood == NS_LIKE_GW_RB) {
        // table filled by launch_prep_rb once the descriptor is on the device
        d.rb_bins = e.rb_bins;
        d.rb_nrows = (e.rb_bins + RB_BINS_PER_ROW - 1) / RB_BINS_PER_ROW;
        HIP_TRY(c, dalloc(&b.rb_rows, (size_t)d.rb_nrows * RB_ROW));
        HIP_TRY(c, dalloc(&b.rb_edges, (size_t)e.rb_bins + 1));
        HIP_TRY(c, dalloc(&b.rb_theta0, NPAR));
        HIP_TRY(c, hipMemsetAsync(b.rb_rows, 0, (size_t)d.rb_nrows * RB_ROW, c->stream));
        HIP_TRY(c, hipMemcpyAsync(b.rb_edges, e.rb_edges, sizeof(int32_t) * ((size_t)e.rb_bins + 1),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipMemcpyAsync(b.rb_theta0, e.rb_theta0, sizeof(double) * NPAR,
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        d.rb_rows = b.rb_rows;
    }
    return NS_OK;
}

static ns_status ensure_dead_capacity(ns_ctx *c, int64_t need)
{
    if (need <= c->dead_cap) return NS_OK;
    int64_t cap = c->dead_cap ? c->dead_cap : 4096;
    while (cap < need) cap *= 2;
    const size_t E = (size_t)c->n_events, d = (size_t)c->ndim;
    double *nu = nullptr, *nL = nullptr, *nw = nullptr, *nn = nullptr;
    HIP_TRY(c, dalloc(&nu, E * cap * d));
    HIP_TRY(c, dalloc(&nL, E * cap));
    HIP_TRY(c, dalloc(&nw, E * cap));
    HIP_TRY(c, dalloc(&nn, E * cap));
    if (c->dead_cap) {
        for (size_t e = 0; e < E; ++e) {
            HIP_TRY(c, hipMemcpyAsync(nu + e * cap * d, c->dead_u + e * c->dead_cap * d,
                                      sizeof(double) * c->dead_cap * d, hipMemcpyDeviceToDevice,
                                      c->stream));
            HIP_TRY(c, hipMemcpyAsync(nL + e * cap, c->dead_L + e * c->dead_cap,
                                      sizeof(double) * c->dead_cap, hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(nw + e * cap, c->dead_logw + e * c->dead_cap,
                                      sizeof(double) * c->dead_cap, hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(nn + e * cap, c->dead_nlive + e * c->dead_cap,
                                      sizeof(double) * c->dead_cap, hipMemcpyDeviceToDevice, c->stream));
        }
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        dfree(c->dead_u);
        dfree(c->dead_L);
        dfree(c->dead_logw);
        dfree(c->dead_nlive);
    }
    c->dead_u = nu;
    c->dead_L = nL;
    c->dead_logw = nw;
    c->dead_nlive = nn;
    c->dead_cap = cap;
    return NS_OK;
}

static StepArgs make_args(ns_ctx *c, int k, int walk)
{
    StepArgs a{};
    a.ev = c->d_ev;
    a.st = c->d_st;
    a.live_u = c->live_u[c->cur];
    a.live_L = c->live_L[c->cur];
    a.next_u = c->live_u[1 - c->cur];
    a.next_L = c->live_L[1 - c->cur];
    a.snap_u = c->snap_u;
    a.snap_L = c->snap_L;
    a.chain_u = c->chain_u;
    a.chain_L = c->chain_L;
    a.chain_stats = c->chain_stats;
    a.ev_order = c->n_events > 1 ? c->d_order : nullptr;
    a.dead_u = c->dead_u;
    a.dead_L = c->dead_L;
    a.dead_logw = c->dead_logw;
    a.dead_nlive = c->dead_nlive;
    a.dead_cap = c->dead_cap;
    a.seed = c->cfg.seed;
    a.n_live = c->n_live;
    a.ndim = c->ndim;
    a.k = k;
    a.walk_override = walk;
    a.naccept = c->cfg.naccept;
    a.maxmcmc = c->cfg.maxmcmc;
    a.term_kind = c->cfg.term_kind;
    a.n_events = c->n_events;
    a.delay = c->delay;
    a.term_thr = c->cfg.term_thr;
    a.hv_u = c->hv_u;
    a.hv_L = c->hv_L;
    a.hv_count = c->hv_count;
    a.hv_cap = c->hv_cap;
    a.da_on = c->da_on ? 1 : 0;
    a.mW1p = c->mlp.W1p;
    a.mW2 = c->mlp.W2;
    a.mW3 = c->mlp.W3;
    a.mP = c->mlp.p;
    a.m_in_mu = c->mlp.in_mu;
    a.m_in_isig = c->mlp.in_isig;
    a.m_mu = c->mlp.mu;
    a.m_sig = c->mlp.sig;
    a.m_top = c->mlp.top;
    a.da_margin = c->da_margin;
    a.da_temp = c->da_temp;
    a.da_floor = c->da_floor;
    return a;
}

static int auto_wpc(const ns_ctx *c, int k)
{
    if (c->wpc > 0) return c->wpc;
    // Four waves per chain (two candidate pairs, each wave over half of the
    // rows) measured best from 500 chains (one paper-scale event: 67 M
    // calls/s against 55-60 M at 8 and 40 M at 2) to 16 000 (64 events:
    // 16.5 M calls/s against 13.3 M at 2 and 7.2 M at 1); below 256 chains
    // the GPU is latency-bound and eight waves (more speculation) help.
    long chains = (long)c->n_events * k;
    return chains >= 256 ? 4 : 8;
}

extern "C" {

ns_status ns_init(ns_ctx **out, const ns_config *cfg, const ns_event_desc *events, int32_t n_events)
{
    g_init_error.clear();
    if (!out) return fail(nullptr, NS_EINVAL, "ns_init: out is NULL");
    *out = nullptr;
    if (!cfg || !events) return fail(nullptr, NS_EINVAL, "ns_init: cfg and events are required");
    if (n_events < 1) return fail(nullptr, NS_EINVAL, "ns_init: n_events must be >= 1");
    const ns_config &C = *cfg;
    if (C.n_live < 3 || C.n_live > 4096)
        return fail(nullptr, NS_EINVAL, "ns_init: n_live must be in [3, 4096]");
    if (C.num_delete < 1 || C.num_delete > C.n_live - 2)
        return fail(nullptr, NS_EINVAL, "ns_init: num_delete must be in [1, n_live - 2]");
    if (C.maxmcmc < 1 || C.walk0 < 1 || C.walk0 > C.maxmcmc || C.naccept < 1)
        return fail(nullptr, NS_EINVAL, "ns_init: need naccept >= 1 and 1 <= walk0 <= maxmcmc");
    if (C.term_kind != 0 && C.term_kind != 1)
        return fail(nullptr, NS_EINVAL, "ns_init: term_kind must be 0 or 1");
    if (!(C.term_thr > 0.0)) return fail(nullptr, NS_EINVAL, "ns_init: term_thr must be positive");
    if (C.precision != NS_FP64 && C.precision != NS_MIXED)
        return fail(nullptr, NS_EINVAL, "ns_init: unknown precision");
    int ndim = events[0].ndim;
    for (int i = 0; i < n_events; ++i) {
        std::string msg;
        ns_status s = check_event(events[i], i, msg);
        if (s != NS_OK) return fail(nullptr, s, "ns_init: " + msg);
        if (events[i].ndim != ndim)
            return fail(nullptr, NS_EINVAL, "ns_init: every event must have the same ndim");
    }

    ns_ctx *c = new ns_ctx();
    c->cfg = C;
    c->n_events = n_events;
    c->ndim = ndim;
    c->n_live = C.n_live;
    c->delay = C.delay >= 0.0 ? C.delay : std::max(C.n_live / 10.0 - 1.0, 0.0);
    c->stream = (hipStream_t)C.stream;
    c->timing = (C.flags & NS_FLAG_TIMING) != 0;
    c->use_graph = (C.flags & NS_FLAG_GRAPH) != 0 && !c->timing;
    if (c->use_graph && !C.stream) {
        delete c;
        return fail(nullptr, NS_EINVAL, "ns_init: NS_FLAG_GRAPH needs a stream (the null stream cannot be captured)");
    }
    c->evb.resize(n_events);
    c->hev.resize(n_events);
    c->conv_seen.assign(n_events, 0);
    c->fingerprint = events_fingerprint(events, n_events);
    ns_status s = NS_OK;
    auto bail = [&](ns_status st) {
        g_init_error = c->err;
        ns_free(c);
        return st;
    };
    for (int i = 0; i < n_events; ++i) {
        s = upload_event(c, events[i], c->evb[i], c->hev[i]);
        if (s != NS_OK) return bail(s);
        c->hev[i].n_live = C.n_live;
        c->hev[i].k = C.num_delete;
        if (events[i].likelihood == NS_LIKE_GW || events[i].likelihood == NS_LIKE_GW_RB)
            c->max_det = std::max(c->max_det, events[i].n_det);
    }
    const size_t E = n_events, n = C.n_live, d = ndim;
    hipError_t he = hipSuccess;
#define ALLOC(p, cnt)                                                                          \
    if ((he = dalloc(&(p), (cnt))) != hipSuccess) {                                          \
        c->err = std::string("hipMalloc: ") + hipGetErrorString(he);                          \
        return bail(NS_ENOMEM);                                                                \
    }
    ALLOC(c->d_ev, E);
    ALLOC(c->d_st, E);
    ALLOC(c->live_u[0], E * n * d);
    ALLOC(c->live_u[1], E * n * d);
    ALLOC(c->live_L[0], E * n);
    ALLOC(c->live_L[1], E * n);
    ALLOC(c->snap_u, E * n * d);
    ALLOC(c->snap_L, E * n);
    ALLOC(c->chain_u, E * n * d);
    ALLOC(c->chain_L, E * n);
    ALLOC(c->chain_stats, E * n * 4);
    ALLOC(c->d_order, E);
#undef ALLOC
    {
        // a valid order before the first batch computes one
        std::vector<int32_t> id(E);
        for (size_t i = 0; i < E; ++i) id[i] = (int32_t)i;
        if ((he = hipMemcpy(c->d_order, id.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice)) != hipSuccess) {
            c->err = std::string("hipMemcpy: ") + hipGetErrorString(he);
            return bail(NS_EHIP);
        }
    }
    if ((he = hipMemcpyAsync(c->d_ev, c->hev.data(), sizeof(DevEvent) * E, hipMemcpyHostToDevice,
                             c->stream)) != hipSuccess) {
        c->err = std::string("hipMemcpyAsync: ") + hipGetErrorString(he);
        return bail(NS_EHIP);
    }
    for (int i = 0; i < n_events; ++i) {
        if (events[i].likelihood != NS_LIKE_GW_RB) continue;
        if ((he = launch_prep_rb(c->d_ev + i, c->hev[i], c->evb[i].rb_edges, c->evb[i].rb_theta0,
                                 c->stream)) != hipSuccess) {
            c->err = std::string("relative-binning tables: ") + hipGetErrorString(he);
            return bail(NS_EHIP);
        }
    }
    std::vector<EvState> st(E);
    for (auto &x : st) {
        memset(&x, 0, sizeof x);
        x.logZ = -INFINITY;
        x.logX = 0.0;
        x.sumH = 0.0;
        x.Lstar = -INFINITY;
        x.dlogZ = INFINITY;
        x.log_frac = INFINITY;
        x.W = C.walk0;
        x.walk_this = C.walk0;
        x.active = 1;
    }
    if ((he = hipMemcpyAsync(c->d_st, st.data(), sizeof(EvState) * E, hipMemcpyHostToDevice,
                             c->stream)) != hipSuccess) {
        c->err = std::string("hipMemcpyAsync: ") + hipGetErrorString(he);
        return bail(NS_EHIP);
    }
    if ((s = ensure_dead_capacity(c, 8 * (int64_t)C.num_delete)) != NS_OK) return bail(s);
    if ((he = launch_init_live(c->d_ev, n_events, C.n_live, ndim, C.seed, C.precision == NS_MIXED, c->live_u[0],
                               c->live_L[0], c->max_det, c->stream)) != hipSuccess) {
        c->err = std::string("init_live: ") + hipGetErrorString(he);
        return bail(NS_EHIP);
    }
    if ((he = hipStreamSynchronize(c->stream)) != hipSuccess) {
        c->err = std::string("init: ") + hipGetErrorString(he);
        return bail(NS_EHIP);
    }
    *out = c;
    return NS_OK;
}

void ns_free(ns_ctx *c)
{
    if (!c) return;
    if (c->stream || true) (void)hipStreamSynchronize(c->stream);
    for (auto &b : c->evb) {
        dfree(b.data);
        dfree(b.psd);
        dfree(b.rows64);
        dfree(b.rows32);
        dfree(b.rb_rows);
        dfree(b.rb_edges);
        dfree(b.rb_theta0);
        dfree(b.K);
    }
    dfree(c->d_ev);
    dfree(c->d_st);
    for (int i = 0; i < 2; ++i) {
        dfree(c->live_u[i]);
        dfree(c->live_L[i]);
    }
    dfree(c->snap_u);
    dfree(c->snap_L);
    dfree(c->chain_u);
    dfree(c->chain_L);
    dfree(c->chain_stats);
    dfree(c->d_order);
    dfree(c->dead_u);
    dfree(c->dead_L);
    dfree(c->dead_logw);
    dfree(c->dead_nlive);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (int i = 0; i < 2; ++i) {
        if (c->gexec[i]) (void)hipGraphExecDestroy(c->gexec[i]);
        if (c->graph[i]) (void)hipGraphDestroy(c->graph[i]);
    }
    {
        MlpBuffers &B = c->mlp;
        void *ptrs[] = {B.p, B.g, B.m, B.v, B.W1p, B.W1T, B.W2, B.W3, B.W2T, B.W3T, B.X, B.XT,
                        B.a1, B.a2, B.a3, B.h1, B.h2, B.h3, B.h1T, B.h2T, B.h3T, B.d, B.dT,
                        B.gtmp, B.y, B.dy, B.t, B.stats, B.loss, B.in_mu, B.in_isig, B.ws,
                        B.d2, B.sq};
        for (void *q : ptrs) dfree(q);
    }
    dfree(c->hv_u);
    dfree(c->hv_L);
    dfree(c->hv_count);
    delete c;
}

ns_status ns_surrogate_init(ns_ctx *c, uint64_t seed, int64_t max_rows)
{
    if (!c) return NS_EINVAL;
    if (max_rows < 32 || max_rows > (1 << 20))
        return fail(c, NS_EINVAL, "ns_surrogate_init: max_rows must be in [32, 2^20]");
    if (c->mlp_ready) return fail(c, NS_ESTATE, "ns_surrogate_init: already initialised");
    MlpBuffers &B = c->mlp;
    const int64_t R = (max_rows + 31) / 32 * 32;
    B.max_rows = R;
    const size_t P = MLP_NPARAM, H = MLP_H, K = MLP_KIN;
    HIP_TRY(c, dalloc(&B.p, P));
    HIP_TRY(c, dalloc(&B.g, P));
    HIP_TRY(c, dalloc(&B.m, P));
    HIP_TRY(c, dalloc(&B.v, P));
    HIP_TRY(c, dalloc(&B.W1p, H * K));
    HIP_TRY(c, dalloc(&B.W1T, H * K));
    HIP_TRY(c, dalloc(&B.W2, H * H));
    HIP_TRY(c, dalloc(&B.W3, H * H));
    HIP_TRY(c, dalloc(&B.W2T, H * H));
    HIP_TRY(c, dalloc(&B.W3T, H * H));
    HIP_TRY(c, dalloc(&B.X, R * K));
    HIP_TRY(c, dalloc(&B.XT, R * K));
    HIP_TRY(c, dalloc(&B.a1, R * H));
    HIP_TRY(c, dalloc(&B.a2, R * H));
    HIP_TRY(c, dalloc(&B.a3, R * H));
    HIP_TRY(c, dalloc(&B.h1, R * H));
    HIP_TRY(c, dalloc(&B.h2, R * H));
    HIP_TRY(c, dalloc(&B.h3, R * H));
    HIP_TRY(c, dalloc(&B.h1T, R * H));
    HIP_TRY(c, dalloc(&B.h2T, R * H));
    HIP_TRY(c, dalloc(&B.h3T, R * H));
    HIP_TRY(c, dalloc(&B.d, R * H));
    HIP_TRY(c, dalloc(&B.dT, 3 * R * H));
    HIP_TRY(c, dalloc(&B.d2, R * H));
    HIP_TRY(c, dalloc(&B.gtmp, R * H));
    HIP_TRY(c, dalloc(&B.y, R));
    HIP_TRY(c, dalloc(&B.dy, R));
    HIP_TRY(c, dalloc(&B.t, R));
    HIP_TRY(c, dalloc(&B.stats, 2));
    HIP_TRY(c, dalloc(&B.loss, 1));
    HIP_TRY(c, dalloc(&B.sq, R));
    HIP_TRY(c, dalloc(&B.in_mu, MLP_KIN));
    HIP_TRY(c, dalloc(&B.in_isig, MLP_KIN));
    HIP_TRY(c, dalloc(&B.ws, (size_t)3 * MLP_SPLITK * H * H));
    {
        float z[MLP_KIN], o[MLP_KIN];
        for (int i = 0; i < MLP_KIN; ++i) {
            z[i] = 0.0f;
            o[i] = 1.0f;
        }
        HIP_TRY(c, hipMemcpy(B.in_mu, z, sizeof z, hipMemcpyHostToDevice));
        HIP_TRY(c, hipMemcpy(B.in_isig, o, sizeof o, hipMemcpyHostToDevice));
    }
    HIP_TRY(c, mlp_init_params(B, seed, c->stream));
    c->mlp_ready = true;
    return NS_OK;
}

static ns_status need_mlp(ns_ctx *c, const char *who)
{
    if (!c) return NS_EINVAL;
    if (!c->mlp_ready) return fail(c, NS_ESTATE, std::string(who) + ": call ns_surrogate_init first");
    return NS_OK;
}

ns_status ns_surrogate_set_params(ns_ctx *c, const float *params, int64_t n)
{
    ns_status s = need_mlp(c, "ns_surrogate_set_params");
    if (s != NS_OK) return s;
    invalidate_graphs(c);
    if (!params || n != MLP_NPARAM) return fail(c, NS_EINVAL, "ns_surrogate_set_params: need 134913 floats");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->mlp.p, params, sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice));
    HIP_TRY(c, mlp_refresh_weights(c->mlp, c->stream));
    return NS_OK;
}

ns_status ns_surrogate_get_params(ns_ctx *c, float *params, int64_t n)
{
    ns_status s = need_mlp(c, "ns_surrogate_get_params");
    if (s != NS_OK) return s;
    if (!params || n != MLP_NPARAM) return fail(c, NS_EINVAL, "ns_surrogate_get_params: need 134913 floats");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(params, c->mlp.p, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
    return NS_OK;
}

// A finite top must lie above the clip; +inf selects the linear target.
static bool top_ok(double clip, double top)
{
    return top == HUGE_VAL || (std::isfinite(top) && top > clip);
}

ns_status ns_surrogate_set_norm(ns_ctx *c, double mu, double sigma, double clip, double top)
{
    ns_status s = need_mlp(c, "ns_surrogate_set_norm");
    if (s != NS_OK) return s;
    invalidate_graphs(c);
    if (!std::isfinite(mu) || !(sigma > 0.0) || !std::isfinite(sigma) || std::isnan(clip))
        return fail(c, NS_EINVAL, "ns_surrogate_set_norm: need finite mu, sigma > 0");
    if (!top_ok(clip, top))
        return fail(c, NS_EINVAL, "ns_surrogate_set_norm: top must be +inf or finite and above clip");
    c->mlp.mu = mu;
    c->mlp.sig = sigma;
    c->mlp.clip = clip;
    c->mlp.top = top;
    return NS_OK;
}

ns_status ns_surrogate_get_norm(ns_ctx *c, double *mu, double *sigma, double *clip, double *top)
{
    ns_status s = need_mlp(c, "ns_surrogate_get_norm");
    if (s != NS_OK) return s;
    if (mu) *mu = c->mlp.mu;
    if (sigma) *sigma = c->mlp.sig;
    if (clip) *clip = c->mlp.clip;
    if (top) *top = c->mlp.top;
    return NS_OK;
}

ns_status ns_surrogate_set_input_norm(ns_ctx *c, const double *mean, const double *stdev)
{
    ns_status s = need_mlp(c, "ns_surrogate_set_input_norm");
    if (s != NS_OK) return s;
    invalidate_graphs(c);
    if (!mean || !stdev) return fail(c, NS_EINVAL, "ns_surrogate_set_input_norm: NULL argument");
    float m[MLP_KIN], is[MLP_KIN];
    for (int i = 0; i < MLP_KIN; ++i) {
        m[i] = 0.0f;
        is[i] = 1.0f;
    }
    for (int i = 0; i < c->ndim; ++i) {
        if (!std::isfinite(mean[i]) || !(stdev[i] > 0.0))
            return fail(c, NS_EINVAL, "ns_surrogate_set_input_norm: need finite means and stdev > 0");
        m[i] = (float)mean[i];
        is[i] = (float)(1.0 / stdev[i]);
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->mlp.in_mu, m, sizeof m, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->mlp.in_isig, is, sizeof is, hipMemcpyHostToDevice));
    return NS_OK;
}

ns_status ns_surrogate_get_input_norm(ns_ctx *c, double *mean, double *stdev)
{
    ns_status s = need_mlp(c, "ns_surrogate_get_input_norm");
    if (s != NS_OK) return s;
    float m[MLP_KIN], is[MLP_KIN];
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(m, c->mlp.in_mu, sizeof m, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(is, c->mlp.in_isig, sizeof is, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->ndim; ++i) {
        if (mean) mean[i] = m[i];
        if (stdev) stdev[i] = 1.0 / (double)is[i];
    }
    return NS_OK;
}

ns_status ns_surrogate_predict(ns_ctx *c, const double *u, int64_t n, double *out)
{
    ns_status s = need_mlp(c, "ns_surrogate_predict");
    if (s != NS_OK) return s;
    if (n < 0 || (n > 0 && (!u || !out))) return fail(c, NS_EINVAL, "ns_surrogate_predict: bad arguments");
    if (n == 0) return NS_OK;
    HIP_TRY(c, mlp_forward(c->mlp, u, c->ndim, n, out, c->stream));
    return NS_OK;
}

ns_status ns_surrogate_loss_grad(ns_ctx *c, const double *u, const double *logl, int64_t n,
                                 float *grad, double *loss)
{
    ns_status s = need_mlp(c, "ns_surrogate_loss_grad");
    if (s != NS_OK) return s;
    if (n < 1 || n > c->mlp.max_rows || !u || !logl)
        return fail(c, NS_EINVAL, "ns_surrogate_loss_grad: need 1 <= n <= max_rows and data");
    HIP_TRY(c, mlp_loss_grad(c->mlp, u, c->ndim, logl, n, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (grad) HIP_TRY(c, hipMemcpy(grad, c->mlp.g, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost));
    if (loss) HIP_TRY(c, hipMemcpy(loss, c->mlp.loss, sizeof(double), hipMemcpyDeviceToHost));
    return NS_OK;
}

ns_status ns_surrogate_train(ns_ctx *c, const double *u, const double *logl, int64_t n,
                             int32_t steps, int32_t batch, double lr, double clip, double top,
                             double *loss)
{
    ns_status s = need_mlp(c, "ns_surrogate_train");
    if (s != NS_OK) return s;
    invalidate_graphs(c);
    if (n < 1 || !u || !logl || steps < 0 || batch < 1 || batch > c->mlp.max_rows || !(lr > 0.0) ||
        std::isnan(clip) || !top_ok(clip, top))
        return fail(c, NS_EINVAL, "ns_surrogate_train: bad arguments");
    MlpBuffers &B = c->mlp;
    B.clip = clip;
    B.top = top;
    // every call starts Adam afresh (zero moments, bias correction from step 1)
    HIP_TRY(c, hipMemsetAsync(B.m, 0, sizeof(float) * MLP_NPARAM, c->stream));
    HIP_TRY(c, hipMemsetAsync(B.v, 0, sizeof(float) * MLP_NPARAM, c->stream));
    HIP_TRY(c, mlp_target_stats(B, logl, n, c->stream));
    HIP_TRY(c, mlp_input_stats(B, u, c->ndim, n, c->stream));
    double st[2];
    HIP_TRY(c, hipMemcpyAsync(st, B.stats, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    B.mu = st[0];
    B.sig = st[1];
    // cosine decay of the learning rate from lr to lr / 20
    const double pi = 3.14159265358979323846;
    for (int32_t t = 1; t <= steps; ++t) {
        double frac = steps > 1 ? (double)(t - 1) / (double)(steps - 1) : 0.0;
        double lr_t = lr * (0.05 + 0.95 * 0.5 * (1.0 + std::cos(pi * frac)));
        HIP_TRY(c, mlp_train_step(B, u, logl, c->ndim, n, batch, c->cfg.seed, t, (float)lr_t, c->stream));
    }
    if (loss) {
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        HIP_TRY(c, hipMemcpy(loss, B.loss, sizeof(double), hipMemcpyDeviceToHost));
    }
    return NS_OK;
}

ns_status ns_surrogate_attach(ns_ctx *c, double margin, double temperature, double floor)
{
    ns_status s = need_mlp(c, "ns_surrogate_attach");
    if (s != NS_OK) return s;
    invalidate_graphs(c);
    if (!std::isfinite(margin) || !(temperature > 0.0) || !std::isfinite(temperature))
        return fail(c, NS_EINVAL, "ns_surrogate_attach: need finite margin and temperature > 0");
    if (!(floor >= 0.0 && floor < 1.0))
        return fail(c, NS_EINVAL, "ns_surrogate_attach: floor must lie in [0, 1)");
    if (c->inner != NS_INNER_WALK)
        return fail(c, NS_ESTATE, "ns_surrogate_attach: the screen needs the acceptance walk");
    c->da_on = true;
    c->da_margin = margin;
    c->da_temp = temperature;
    c->da_floor = floor;
    return NS_OK;
}

ns_status ns_surrogate_detach(ns_ctx *c)
{
    if (!c) return NS_EINVAL;
    invalidate_graphs(c);
    c->da_on = false;
    return NS_OK;
}

ns_status ns_harvest(ns_ctx *c, int64_t capacity)
{
    if (!c || capacity < 0) return NS_EINVAL;
    invalidate_graphs(c);
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    dfree(c->hv_u);
    dfree(c->hv_L);
    dfree(c->hv_count);
    c->hv_u = c->hv_L = nullptr;
    c->hv_count = nullptr;
    c->hv_cap = 0;
    if (capacity == 0) return NS_OK;
    HIP_TRY(c, dalloc(&c->hv_u, (size_t)capacity * c->ndim));
    HIP_TRY(c, dalloc(&c->hv_L, (size_t)capacity));
    HIP_TRY(c, dalloc(&c->hv_count, 1));
    HIP_TRY(c, hipMemset(c->hv_count, 0, sizeof(unsigned long long)));
    c->hv_cap = capacity;
    return NS_OK;
}

ns_status ns_harvest_copy(ns_ctx *c, double *u, double *logl, int64_t max_rows, int64_t *n_rows)
{
    if (!c || !n_rows) return NS_EINVAL;
    *n_rows = 0;
    if (!c->hv_count) return NS_OK;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    unsigned long long cnt = 0;
    HIP_TRY(c, hipMemcpy(&cnt, c->hv_count, sizeof cnt, hipMemcpyDeviceToHost));
    int64_t rows = std::min<int64_t>((int64_t)std::min<unsigned long long>(cnt, (unsigned long long)c->hv_cap),
                                     std::max<int64_t>(max_rows, 0));
    if (rows > 0) {
        if (u) HIP_TRY(c, hipMemcpy(u, c->hv_u, sizeof(double) * rows * c->ndim, hipMemcpyDeviceToDevice));
        if (logl) HIP_TRY(c, hipMemcpy(logl, c->hv_L, sizeof(double) * rows, hipMemcpyDeviceToDevice));
    }
    *n_rows = rows;
    return NS_OK;
}

ns_status ns_set_waves_per_chain(ns_ctx *c, int32_t wpc)
{
    if (!c) return NS_EINVAL;
    if (wpc != 0 && wpc != 1 && wpc != 2 && wpc != 4 && wpc != 6 && wpc != 8)
        return fail(c, NS_EINVAL, "ns_set_waves_per_chain: must be 0, 1, 2, 4, 6 or 8");
    c->wpc = wpc;
    return NS_OK;
}

ns_status ns_timing(ns_ctx *c, ns_timing_t *out, int32_t reset)
{
    if (!c || !out) return NS_EINVAL;
    if (!c->timing) return fail(c, NS_ESTATE, "ns_timing: context created without NS_FLAG_TIMING");
    HIP_TRY(c, timing_collect(c));
    *out = c->acc;
    if (reset) c->acc = ns_timing_t{};
    return NS_OK;
}

const char *ns_last_error(const ns_ctx *c)
{
    return c ? c->err.c_str() : g_init_error.c_str();
}

int32_t ns_num_events(const ns_ctx *c) { return c ? c->n_events : 0; }

const char *ns_version(void)
{
    return "nsmi 0.2 gfx950: fp64 speculative walk (1/2/4/8 candidate waves per chain), bitonic select, lane-parallel Philox4x64-10";
}

// The chains' inner kernel: the acceptance walk, or hit-and-run slice sampling.
static hipError_t launch_inner(ns_ctx *c, const StepArgs &a, int wpc)
{
    const int mixed = c->cfg.precision == NS_MIXED;
    if (c->inner == NS_INNER_HRSS) return launch_hrss(a, c->max_det, mixed, c->stream);
    return launch_walk(a, c->max_det, wpc, mixed, c->stream);
}

static hipError_t enqueue_step(ns_ctx *c, const StepArgs &a, int wpc)
{
    hipError_t e;
    if ((e = launch_select(a, c->stream)) != hipSuccess) return e;
    if (a.ev_order && (e = launch_order(a, c->d_order, c->stream)) != hipSuccess) return e;
    if ((e = launch_inner(c, a, wpc)) != hipSuccess) return e;
    return launch_finish(a, c->stream);
}

ns_status ns_step(ns_ctx *c, int32_t k, int32_t walk)
{
    if (!c) return NS_EINVAL;
    if (k <= 0) k = c->cfg.num_delete;
    if (k < 1 || k > c->n_live - 2)
        return fail(c, NS_EINVAL, "ns_step: k must be in [1, n_live - 2]");
    if (walk > c->cfg.maxmcmc) return fail(c, NS_EINVAL, "ns_step: walk exceeds maxmcmc");
    bool all_done = true;
    for (char v : c->conv_seen) all_done = all_done && v;
    if (all_done)
        return fail(c, NS_ESTATE, "ns_step: every event has converged (as last read by ns_evidence)");
    ns_status s = ensure_dead_capacity(c, c->dead_bound + k);
    if (s != NS_OK) return s;
    StepArgs a = make_args(c, k, walk);
    const int wpc = auto_wpc(c, k);
    if (c->use_graph) {
        const int g = c->cur;
        const bool hv = c->hv_count != nullptr;
        if (!c->gexec[g] || c->g_k[g] != k || c->g_walk[g] != walk || c->g_cap[g] != c->dead_cap ||
            c->g_wpc[g] != wpc || c->g_da[g] != c->da_on || c->g_hv[g] != hv) {
            if (c->gexec[g]) HIP_TRY(c, hipGraphExecDestroy(c->gexec[g]));
            if (c->graph[g]) HIP_TRY(c, hipGraphDestroy(c->graph[g]));
            c->gexec[g] = nullptr;
            c->graph[g] = nullptr;
            HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = enqueue_step(c, a, wpc);
            hipGraph_t gr = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
            if (e != hipSuccess) return fail(c, NS_EHIP, std::string("ns_step capture: ") + hipGetErrorString(e));
            if (e2 != hipSuccess) return fail(c, NS_EHIP, std::string("ns_step capture: ") + hipGetErrorString(e2));
            c->graph[g] = gr;
            HIP_TRY(c, hipGraphInstantiate(&c->gexec[g], gr, nullptr, nullptr, 0));
            c->g_k[g] = k;
            c->g_walk[g] = walk;
            c->g_cap[g] = c->dead_cap;
            c->g_wpc[g] = wpc;
            c->g_da[g] = c->da_on;
            c->g_hv[g] = hv;
        }
        HIP_TRY(c, hipGraphLaunch(c->gexec[g], c->stream));
    } else {
        hipEvent_t t[4] = {nullptr, nullptr, nullptr, nullptr};
        if (c->timing) {
            if (c->ev_used + 4 > 4096) HIP_TRY(c, timing_collect(c));
            for (auto &x : t) HIP_TRY(c, timing_event(c, &x));
            HIP_TRY(c, hipEventRecord(t[0], c->stream));
        }
        HIP_TRY(c, launch_select(a, c->stream));
        if (a.ev_order) HIP_TRY(c, launch_order(a, c->d_order, c->stream));
        if (c->timing) HIP_TRY(c, hipEventRecord(t[1], c->stream));
        HIP_TRY(c, launch_inner(c, a, wpc));
        if (c->timing) HIP_TRY(c, hipEventRecord(t[2], c->stream));
        HIP_TRY(c, launch_finish(a, c->stream));
        if (c->timing) HIP_TRY(c, hipEventRecord(t[3], c->stream));
    }
    c->dead_bound += k;
    c->cur = 1 - c->cur;
    return NS_OK;
}

// Shape key of the autotuner cache.
static std::string tune_key(const ns_ctx *c)
{
    std::ostringstream o;
    int maxbins = 0;
    for (const auto &h : c->hev) maxbins = std::max(maxbins, h.n_bins);
    o << "gfx950 events=" << c->n_events << " k=" << c->cfg.num_delete << " n_live=" << c->n_live
      << " ndim=" << c->ndim << " det=" << c->max_det << " bins=" << maxbins
      << " prec=" << c->cfg.precision << " da=" << (c->da_on ? 1 : 0);
    return o.str();
}

ns_status ns_set_inner(ns_ctx *c, int32_t inner)
{
    if (!c) return NS_EINVAL;
    if (inner != NS_INNER_WALK && inner != NS_INNER_HRSS)
        return fail(c, NS_EINVAL, "ns_set_inner: unknown inner kernel");
    if (inner == NS_INNER_HRSS && c->da_on)
        return fail(c, NS_ESTATE, "ns_set_inner: detach the surrogate screen first");
    invalidate_graphs(c);
    c->inner = inner;
    return NS_OK;
}

ns_status ns_autotune(ns_ctx *c, const char *cache_path, int32_t trial_walk, int32_t *chosen)
{
    if (!c) return NS_EINVAL;
    if (c->inner != NS_INNER_WALK)
        return fail(c, NS_ESTATE, "ns_autotune: tunes the acceptance walk's launch shape only");
    if (trial_walk < 1 || trial_walk > c->cfg.maxmcmc)
        return fail(c, NS_EINVAL, "ns_autotune: trial_walk must be in [1, maxmcmc]");
    const std::string key = tune_key(c);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        int found = 0;
        while (std::getline(in, line)) {
            size_t bar = line.rfind(" | ");
            if (bar == std::string::npos || line.substr(0, bar) != key) continue;
            int v = atoi(line.c_str() + bar + 3);
            if (v == 1 || v == 2 || v == 4 || v == 6 || v == 8) found = v;  // last valid entry wins
        }
        if (found) {
            c->wpc = found;
            if (chosen) *chosen = found;
            return NS_OK;
        }
    }
    const int k = c->cfg.num_delete;
    ns_status s = ensure_dead_capacity(c, c->dead_bound + k);
    if (s != NS_OK) return s;
    // save the per-event state; trial batches write only scratch rows
    EvState *saved = nullptr;
    HIP_TRY(c, dalloc(&saved, (size_t)c->n_events));
    HIP_TRY(c, hipMemcpyAsync(saved, c->d_st, sizeof(EvState) * c->n_events, hipMemcpyDeviceToDevice,
                              c->stream));
    hipEvent_t t0, t1;
    HIP_TRY(c, hipEventCreate(&t0));
    HIP_TRY(c, hipEventCreate(&t1));
    StepArgs a = make_args(c, k, trial_walk);
    a.hv_count = nullptr;  // trials are not harvested
    const int cand[5] = {1, 2, 4, 6, 8};
    float best_ms = 0.f;
    int best = 0;
    hipError_t he = hipSuccess;
    for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {  // first pass warms up
        for (int w : cand) {
            if ((he = hipMemcpyAsync(c->d_st, saved, sizeof(EvState) * c->n_events,
                                     hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
                break;
            if ((he = launch_select(a, c->stream)) != hipSuccess) break;
            if (a.ev_order && (he = launch_order(a, c->d_order, c->stream)) != hipSuccess) break;
            if ((he = hipEventRecord(t0, c->stream)) != hipSuccess) break;
            if ((he = launch_walk(a, c->max_det, w, c->cfg.precision == NS_MIXED, c->stream)) != hipSuccess)
                break;
            if ((he = hipEventRecord(t1, c->stream)) != hipSuccess) break;
            if ((he = hipEventSynchronize(t1)) != hipSuccess) break;
            float ms = 0.f;
            if ((he = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) break;
            if (rep == 1 && (best == 0 || ms < best_ms)) {
                best_ms = ms;
                best = w;
            }
        }
    }
    hipError_t hr = hipMemcpyAsync(c->d_st, saved, sizeof(EvState) * c->n_events, hipMemcpyDeviceToDevice,
                                   c->stream);
    hipError_t hs = hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    dfree(saved);
    if (he != hipSuccess) return fail(c, NS_EHIP, std::string("ns_autotune: ") + hipGetErrorString(he));
    if (hr != hipSuccess || hs != hipSuccess)
        return fail(c, NS_EHIP, "ns_autotune: restoring the sampler state failed");
    c->wpc = best;
    if (chosen) *chosen = best;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (out) out << key << " | " << best << "\n";
    }
    return NS_OK;
}

ns_status ns_loglike_batch(ns_ctx *c, int32_t event, const double *theta, int64_t n, double *out,
                           int32_t precision)
{
    if (!c) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_loglike_batch: bad event");
    if (n < 0 || (n > 0 && (!theta || !out)))
        return fail(c, NS_EINVAL, "ns_loglike_batch: bad size or NULL pointer");
    if (precision != NS_FP64 && precision != NS_MIXED)
        return fail(c, NS_EINVAL, "ns_loglike_batch: unknown precision");
    if (c->hev[event].likelihood != NS_LIKE_GW && c->hev[event].likelihood != NS_LIKE_GW_RB)
        return fail(c, NS_EINVAL, "ns_loglike_batch: the event has no strain data");
    HIP_TRY(c, launch_loglike_theta(c->d_ev + event, c->hev[event].n_det, theta, n, out,
                                    precision == NS_MIXED, c->stream));
    return NS_OK;
}

ns_status ns_loglike_batch_u(ns_ctx *c, int32_t event, const double *u, int64_t n, double *out,
                             int32_t precision)
{
    if (!c) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_loglike_batch_u: bad event");
    if (n < 0 || (n > 0 && (!u || !out)))
        return fail(c, NS_EINVAL, "ns_loglike_batch_u: bad size or NULL pointer");
    if (precision != NS_FP64 && precision != NS_MIXED)
        return fail(c, NS_EINVAL, "ns_loglike_batch_u: unknown precision");
    int nd = c->hev[event].likelihood == NS_LIKE_GAUSS ? 1 : c->hev[event].n_det;
    HIP_TRY(c, launch_loglike_u(c->d_ev + event, nd, c->ndim, u, n, out, precision == NS_MIXED,
                                c->stream));
    return NS_OK;
}

ns_status ns_theta_from_u(ns_ctx *c, int32_t event, const double *u, int64_t n, double *theta)
{
    if (!c) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_theta_from_u: bad event");
    if (n < 0 || (n > 0 && (!u || !theta)))
        return fail(c, NS_EINVAL, "ns_theta_from_u: bad size or NULL pointer");
    if (c->hev[event].likelihood == NS_LIKE_GAUSS)
        return fail(c, NS_EINVAL, "ns_theta_from_u: the Gaussian toy has no physical parameters");
    HIP_TRY(c, launch_theta_from_u(c->d_ev + event, u, n, theta, c->stream));
    return NS_OK;
}

ns_status ns_evidence(ns_ctx *c, int32_t event, ns_evidence_t *out)
{
    if (!c || !out) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_evidence: bad event");
    EvState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->d_st + event, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    memset(out, 0, sizeof *out);
    // live-point terms of the current live set
    std::vector<double> L(c->n_live);
    HIP_TRY(c, hipMemcpy(L.data(), c->live_L[c->cur] + (size_t)event * c->n_live,
                         sizeof(double) * c->n_live, hipMemcpyDeviceToHost));
    double mx = -INFINITY;
    for (double v : L) mx = std::max(mx, v);
    double se = 0.0;
    for (double v : L) se += std::exp(v - mx);
    double lme = mx + std::log(se / c->n_live);
    auto lae = [](double a, double b) {
        if (a == -INFINITY) return b;
        if (b == -INFINITY) return a;
        double m = std::max(a, b);
        return m + std::log(std::exp(a - m) + std::exp(b - m));
    };
    out->logZ_dead = st.logZ;
    out->logZ = lae(st.logZ, st.logX + lme);
    out->H = st.sumH - st.logZ;
    // Skilling's error with the batched saw-tooth of live counts (Sec. 3.2.1):
    // about H / mean(1/n_i) deletions cross the posterior bulk, each adding
    // mean(1/n_i^2) to the variance of log Z
    out->logZ_err = st.sum_in > 0.0 ? std::sqrt(std::max(out->H, 0.0) * st.sum_in2 / st.sum_in) : 0.0;
    out->logX = st.logX;
    out->dlogZ = lae(st.logZ, st.logX + mx) - st.logZ;
    out->log_frac = st.logX + lme - st.logZ;
    out->last_Lstar = st.Lstar;
    out->n_dead = st.n_dead;
    out->n_calls = st.n_calls;
    out->n_accept = st.n_acc;
    out->n_oob = st.n_oob;
    out->n_steps = st.n_steps;
    out->n_calls_saved = st.n_saved;
    out->n_spec_discarded = st.n_spec;
    out->batch = st.batch;
    out->W = st.W;
    out->converged = st.converged;
    out->last_accept = st.last_acc;
    out->last_calls = st.last_calls;
    out->walk_capped = st.n_capped;
    c->conv_seen[event] = st.converged ? 1 : 0;
    if (st.err) return fail(c, NS_ESTATE, "ns_step: fewer than two survivors above L* (the live set collapsed)");
    return NS_OK;
}

ns_status ns_get_chain_stats(ns_ctx *c, int32_t event, int64_t *out, int32_t max_chains,
                             int32_t *n_chains)
{
    if (!c || !n_chains || (!out && max_chains > 0) || max_chains < 0) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_get_chain_stats: bad event");
    EvState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->d_st + event, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    // chains of the last batch (none when the event was already inactive)
    const int k = std::max(st.k_this, 0);
    const int nc = std::min(k, max_chains);
    if (nc > 0)
        HIP_TRY(c, hipMemcpy(out, c->chain_stats + (size_t)event * c->n_live * 4,
                             sizeof(int64_t) * 4 * nc, hipMemcpyDeviceToHost));
    *n_chains = nc;
    return NS_OK;
}

ns_status ns_logz_replicates(ns_ctx *c, int32_t event, int32_t R, uint64_t seed, const double *uniforms,
                             double *out)
{
    if (!c || !out || R < 1 || R > (1 << 20)) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_logz_replicates: bad event");
    EvState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->d_st + event, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (st.n_dead < 1) return fail(c, NS_ESTATE, "ns_logz_replicates: no dead points yet");
    const size_t off = (size_t)event * c->dead_cap;
    HIP_TRY(c, launch_replicates(c->dead_L + off, c->dead_nlive + off, st.n_dead,
                                 c->live_L[c->cur] + (size_t)event * c->n_live, c->n_live, uniforms,
                                 seed, R, out, c->stream));
    return NS_OK;
}

ns_status ns_get_live(ns_ctx *c, int32_t event, double *u, double *logl)
{
    if (!c) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_get_live: bad event");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const size_t n = c->n_live, d = c->ndim;
    if (u)
        HIP_TRY(c, hipMemcpy(u, c->live_u[c->cur] + event * n * d, sizeof(double) * n * d,
                             hipMemcpyDeviceToHost));
    if (logl)
        HIP_TRY(c, hipMemcpy(logl, c->live_L[c->cur] + event * n, sizeof(double) * n,
                             hipMemcpyDeviceToHost));
    return NS_OK;
}

ns_status ns_set_live(ns_ctx *c, int32_t event, const double *u, const double *logl)
{
    if (!c || !u || !logl) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_set_live: bad event");
    const size_t n = c->n_live, d = c->ndim;
    for (size_t i = 0; i < n * d; ++i)
        if (!(u[i] >= 0.0 && u[i] <= 1.0)) return fail(c, NS_EINVAL, "ns_set_live: u outside [0, 1]");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipMemcpy(c->live_u[c->cur] + event * n * d, u, sizeof(double) * n * d,
                         hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->live_L[c->cur] + event * n, logl, sizeof(double) * n,
                         hipMemcpyHostToDevice));
    return NS_OK;
}

ns_status ns_get_dead(ns_ctx *c, int32_t event, int64_t max_rows, double *u, double *logl,
                      double *logw, double *nlive, int64_t *n_rows)
{
    if (!c || !n_rows) return NS_EINVAL;
    if (event < 0 || event >= c->n_events) return fail(c, NS_EINVAL, "ns_get_dead: bad event");
    EvState st;
    HIP_TRY(c, hipMemcpyAsync(&st, c->d_st + event, sizeof st, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int64_t rows = std::min<int64_t>(st.n_dead, std::max<int64_t>(max_rows, 0));
    const size_t d = c->ndim, cap = c->dead_cap;
    if (rows > 0) {
        if (u)
            HIP_TRY(c, hipMemcpy(u, c->dead_u + event * cap * d, sizeof(double) * rows * d,
                                 hipMemcpyDeviceToHost));
        if (logl)
            HIP_TRY(c, hipMemcpy(logl, c->dead_L + event * cap, sizeof(double) * rows,
                                 hipMemcpyDeviceToHost));
        if (logw)
            HIP_TRY(c, hipMemcpy(logw, c->dead_logw + event * cap, sizeof(double) * rows,
                                 hipMemcpyDeviceToHost));
        if (nlive)
            HIP_TRY(c, hipMemcpy(nlive, c->dead_nlive + event * cap, sizeof(double) * rows,
                                 hipMemcpyDeviceToHost));
    }
    *n_rows = rows;
    return NS_OK;
}

// ---------------------------------------------------------------------------
// Checkpoint and restore of the sampler state.  Layout (host, native byte
// order): CkptHeader, then per event its EvState, the live set (u, logL) and
// its dead points (u, logL, logw, nlive).  The random numbers are
// counter-based (seed, chain, batch, step), so the batch counter in EvState
// is all a resumed run needs to draw what the uninterrupted run would have.

namespace {
struct CkptHeader {
    char magic[8];
    int32_t version, n_events, n_live, ndim;
    int32_t inner, num_delete, naccept, maxmcmc;
    int32_t precision, term_kind, walk0, pad;
    uint64_t seed;
    double term_thr, delay;
    int64_t state_bytes;
    uint64_t fingerprint;  // of the events (grid, data, PSD)
};
const char CKPT_MAGIC[8] = {'N', 'S', 'M', 'I', 'C', 'K', 'P', '2'};
const int32_t CKPT_VERSION = 2;
}  // namespace

static void fill_header(const ns_ctx *c, CkptHeader &h)
{
    memset(&h, 0, sizeof h);
    memcpy(h.magic, CKPT_MAGIC, 8);
    h.version = CKPT_VERSION;
    h.n_events = c->n_events;
    h.n_live = c->n_live;
    h.ndim = c->ndim;
    h.inner = c->inner;
    h.num_delete = c->cfg.num_delete;
    h.naccept = c->cfg.naccept;
    h.maxmcmc = c->cfg.maxmcmc;
    h.precision = (int32_t)c->cfg.precision;
    h.term_kind = c->cfg.term_kind;
    h.walk0 = c->cfg.walk0;
    h.seed = c->cfg.seed;
    h.term_thr = c->cfg.term_thr;
    h.delay = c->delay;
    h.state_bytes = (int64_t)sizeof(EvState);
    h.fingerprint = c->fingerprint;
}

// Host-side check of a checkpointed per-event state: what ns_step would
// launch with must lie in the ranges the sampler itself produces.
static const char *bad_state(const ns_ctx *c, const EvState &s)
{
    if (s.n_dead < 0 || s.n_dead > (int64_t)1 << 40) return "corrupt dead-point count";
    if (s.W < 1 || s.W > c->cfg.maxmcmc || s.walk_this < 0 || s.walk_this > c->cfg.maxmcmc)
        return "walk length outside [1, maxmcmc]";
    if ((s.converged != 0 && s.converged != 1) || (s.active != 0 && s.active != 1) ||
        (s.err != 0 && s.err != 1))
        return "state flags not 0 or 1";
    if (!(s.logX <= 0.0) || !std::isfinite(s.logX)) return "log X not finite and <= 0";
    if (std::isnan(s.logZ) || s.logZ == INFINITY || std::isnan(s.sumH) || std::isnan(s.Lstar))
        return "evidence accumulators not finite";
    if (s.batch < 0 || s.n_calls < 0 || s.n_acc < 0 || s.n_oob < 0 || s.n_steps < 0 ||
        s.n_capped < 0 || s.m < 0 || s.m > c->n_live || s.k_this < 0 || s.k_this > c->n_live)
        return "negative or out-of-range counters";
    if (!(s.sum_in >= 0.0) || !(s.sum_in2 >= 0.0)) return "corrupt live-count sums";
    return nullptr;
}

static int64_t event_bytes(const ns_ctx *c, int64_t n_dead)
{
    const int64_t n = c->n_live, d = c->ndim;
    return (int64_t)sizeof(EvState) + 8 * (n * d + n) + 8 * n_dead * (d + 3);
}

static ns_status read_states(ns_ctx *c, std::vector<EvState> &st)
{
    st.resize(c->n_events);
    HIP_TRY(c, hipMemcpyAsync(st.data(), c->d_st, sizeof(EvState) * c->n_events,
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return NS_OK;
}

ns_status ns_checkpoint_size(ns_ctx *c, int64_t *bytes)
{
    if (!c || !bytes) return NS_EINVAL;
    std::vector<EvState> st;
    ns_status s = read_states(c, st);
    if (s != NS_OK) return s;
    int64_t total = sizeof(CkptHeader);
    for (const EvState &e : st) total += event_bytes(c, e.n_dead);
    *bytes = total;
    return NS_OK;
}

ns_status ns_checkpoint(ns_ctx *c, void *buf, int64_t bytes, int64_t *written)
{
    if (!c || !buf) return NS_EINVAL;
    std::vector<EvState> st;
    ns_status s = read_states(c, st);
    if (s != NS_OK) return s;
    int64_t total = sizeof(CkptHeader);
    for (const EvState &e : st) total += event_bytes(c, e.n_dead);
    if (bytes < total) return fail(c, NS_EINVAL, "ns_checkpoint: buffer smaller than ns_checkpoint_size");
    char *p = static_cast<char *>(buf);
    CkptHeader h;
    fill_header(c, h);
    memcpy(p, &h, sizeof h);
    p += sizeof h;
    const size_t n = c->n_live, d = c->ndim, cap = c->dead_cap;
    for (int e = 0; e < c->n_events; ++e) {
        memcpy(p, &st[e], sizeof(EvState));
        p += sizeof(EvState);
        const size_t nd = (size_t)st[e].n_dead;
        struct Part { const double *src; size_t count; } parts[] = {
            {c->live_u[c->cur] + e * n * d, n * d}, {c->live_L[c->cur] + e * n, n},
            {c->dead_u + e * cap * d, nd * d},      {c->dead_L + e * cap, nd},
            {c->dead_logw + e * cap, nd},           {c->dead_nlive + e * cap, nd}};
        for (const Part &q : parts) {
            if (q.count)
                HIP_TRY(c, hipMemcpy(p, q.src, sizeof(double) * q.count, hipMemcpyDeviceToHost));
            p += sizeof(double) * q.count;
        }
    }
    if (written) *written = total;
    return NS_OK;
}

ns_status ns_restore(ns_ctx *c, const void *buf, int64_t bytes)
{
    if (!c || !buf) return NS_EINVAL;
    if (bytes < (int64_t)sizeof(CkptHeader)) return fail(c, NS_EINVAL, "ns_restore: buffer too small");
    const char *p = static_cast<const char *>(buf);
    CkptHeader h, mine;
    memcpy(&h, p, sizeof h);
    fill_header(c, mine);
    if (memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != CKPT_VERSION ||
        h.state_bytes != mine.state_bytes)
        return fail(c, NS_EINVAL, "ns_restore: not a checkpoint of this library version");
    if (h.fingerprint != mine.fingerprint)
        return fail(c, NS_EINVAL, "ns_restore: the checkpoint was taken on other event data");
    if (h.n_events != mine.n_events || h.n_live != mine.n_live || h.ndim != mine.ndim)
        return fail(c, NS_EINVAL, "ns_restore: events, live points or dimension differ");
    if (h.inner != mine.inner || h.num_delete != mine.num_delete || h.naccept != mine.naccept ||
        h.maxmcmc != mine.maxmcmc || h.precision != mine.precision || h.term_kind != mine.term_kind ||
        h.walk0 != mine.walk0 || h.seed != mine.seed || h.term_thr != mine.term_thr ||
        h.delay != mine.delay)
        return fail(c, NS_EINVAL, "ns_restore: sampler configuration differs from the checkpoint's");
    // walk the buffer once to validate every event's size before touching the device
    std::vector<EvState> st(c->n_events);
    int64_t off = sizeof h, max_dead = 0;
    const size_t n = c->n_live, d = c->ndim;
    for (int e = 0; e < c->n_events; ++e) {
        if (bytes - off < (int64_t)sizeof(EvState)) return fail(c, NS_EINVAL, "ns_restore: truncated");
        memcpy(&st[e], p + off, sizeof(EvState));
        if (const char *why = bad_state(c, st[e])) return fail(c, NS_EINVAL, std::string("ns_restore: ") + why);
        const int64_t eb = event_bytes(c, st[e].n_dead);
        if (bytes - off < eb) return fail(c, NS_EINVAL, "ns_restore: truncated");
        const double *lu = reinterpret_cast<const double *>(p + off + sizeof(EvState));
        for (size_t i = 0; i < n * d; ++i) {
            double v;
            memcpy(&v, lu + i, sizeof v);
            if (!(v >= 0.0 && v <= 1.0)) return fail(c, NS_EINVAL, "ns_restore: live u outside [0, 1]");
        }
        off += eb;
        max_dead = std::max<int64_t>(max_dead, st[e].n_dead);
    }
    if (off != bytes) return fail(c, NS_EINVAL, "ns_restore: size does not match the checkpoint's contents");
    ns_status s = ensure_dead_capacity(c, max_dead + c->cfg.num_delete);
    if (s != NS_OK) return s;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    off = sizeof h;
    const size_t cap = c->dead_cap;
    for (int e = 0; e < c->n_events; ++e) {
        HIP_TRY(c, hipMemcpy(c->d_st + e, p + off, sizeof(EvState), hipMemcpyHostToDevice));
        off += sizeof(EvState);
        const size_t nd = (size_t)st[e].n_dead;
        struct Part { double *dst; size_t count; } parts[] = {
            {c->live_u[c->cur] + e * n * d, n * d}, {c->live_L[c->cur] + e * n, n},
            {c->dead_u + e * cap * d, nd * d},      {c->dead_L + e * cap, nd},
            {c->dead_logw + e * cap, nd},           {c->dead_nlive + e * cap, nd}};
        for (const Part &q : parts) {
            if (q.count)
                HIP_TRY(c, hipMemcpy(q.dst, p + off, sizeof(double) * q.count, hipMemcpyHostToDevice));
            off += sizeof(double) * q.count;
        }
    }
    c->dead_bound = max_dead;
    for (int e = 0; e < c->n_events; ++e) c->conv_seen[e] = st[e].converged ? 1 : 0;
    invalidate_graphs(c);
    return NS_OK;
}

ns_status ns_signal(const ns_event_desc *desc, const double *theta, double *h)
{
    g_init_error.clear();
    if (!desc || !theta || !h) return fail(nullptr, NS_EINVAL, "ns_signal: NULL argument");
    ns_event_desc e = *desc;
    if (e.n_bins < 1 || e.n_det < 1 || e.n_det > MAXDET || !(e.f_lo > 0) || !(e.df > 0))
        return fail(nullptr, NS_EINVAL, "ns_signal: bad grid or detector count");
    if (!e.fixed_antenna && (!e.det_tensor || !e.det_loc))
        return fail(nullptr, NS_EINVAL, "ns_signal: det_tensor and det_loc are required without fixed_antenna");
    if (!e.prior_lo || !e.prior_hi || !e.fixed_theta)
        return fail(nullptr, NS_EINVAL, "ns_signal: prior_lo, prior_hi and fixed_theta are required");
    e.likelihood = NS_LIKE_GW;
    DevEvent d;
    fill_dev_event(d, e);
    DevEvent *d_ev = nullptr;
    double *d_th = nullptr, *d_h = nullptr;
    size_t nh = 2 * (size_t)e.n_bins * e.n_det;
    hipError_t he;
    ns_status s = NS_OK;
    if ((he = dalloc(&d_ev, 1)) != hipSuccess || (he = dalloc(&d_th, NPAR)) != hipSuccess ||
        (he = dalloc(&d_h, nh)) != hipSuccess) {
        s = fail(nullptr, NS_ENOMEM, std::string("ns_signal: ") + hipGetErrorString(he));
    } else if ((he = hipMemcpy(d_ev, &d, sizeof d, hipMemcpyHostToDevice)) != hipSuccess ||
               (he = hipMemcpy(d_th, theta, sizeof(double) * NPAR, hipMemcpyHostToDevice)) != hipSuccess ||
               (he = launch_signal(d_ev, e.n_bins, e.n_det, d_th, d_h, nullptr)) != hipSuccess ||
               (he = hipMemcpy(h, d_h, sizeof(double) * nh, hipMemcpyDeviceToHost)) != hipSuccess) {
        s = fail(nullptr, NS_EHIP, std::string("ns_signal: ") + hipGetErrorString(he));
    }
    dfree(d_ev);
    dfree(d_th);
    dfree(d_h);
    return s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// ns_signal without allocation: the descriptor, the parameter vector and the
// strain staging live in a file-scope device array (one copy per GPU, held
// until the process ends) instead of buffers allocated per call.
namespace {
constexpr int SIG_MAX_BINS = 65536;
constexpr size_t SIG_OFF_THETA = 4096, SIG_OFF_H = 8192;
constexpr size_t SIG_SCRATCH_BYTES = SIG_OFF_H + sizeof(double) * 2 * (size_t)SIG_MAX_BINS * MAXDET;
static_assert(sizeof(DevEvent) <= SIG_OFF_THETA, "descriptor slot of the signal scratch");
static_assert(sizeof(double) * NPAR <= SIG_OFF_H - SIG_OFF_THETA, "theta slot of the signal scratch");
constexpr int SIG_MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) char scratch[SIG_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static char *g_scratch_ptr[SIG_MAX_DEVICES];  // device address of scratch, per device

// Device address of this GPU's copy of `scratch`, looked up once per device
// (the array's name is a host-side stand-in, never a device address).
static hipError_t scratch_address(char **out)
{
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return he;
    if (dev < 0 || dev >= SIG_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        he = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (he != hipSuccess) return he;
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

extern "C" {

ns_status ns_signal_noalloc(const ns_event_desc *desc, const double *theta, double *h)
{
    g_init_error.clear();
    if (!desc || !theta || !h) return fail(nullptr, NS_EINVAL, "ns_signal_noalloc: NULL argument");
    ns_event_desc e = *desc;
    if (e.n_bins < 1 || e.n_det < 1 || e.n_det > MAXDET || !(e.f_lo > 0) || !(e.df > 0))
        return fail(nullptr, NS_EINVAL, "ns_signal_noalloc: bad grid or detector count");
    if (e.n_bins > SIG_MAX_BINS)
        return fail(nullptr, NS_EINVAL, "ns_signal_noalloc: n_bins exceeds the scratch limit of 65536");
    if (!e.fixed_antenna && (!e.det_tensor || !e.det_loc))
        return fail(nullptr, NS_EINVAL, "ns_signal_noalloc: det_tensor and det_loc are required without fixed_antenna");
    if (!e.prior_lo || !e.prior_hi || !e.fixed_theta)
        return fail(nullptr, NS_EINVAL, "ns_signal_noalloc: prior_lo, prior_hi and fixed_theta are required");
    e.likelihood = NS_LIKE_GW;
    DevEvent d;
    fill_dev_event(d, e);
    char *base = nullptr;
    hipError_t he = scratch_address(&base);
    if (he != hipSuccess)
        return fail(nullptr, NS_EHIP, std::string("ns_signal_noalloc: scratch address: ") + hipGetErrorString(he));
    DevEvent *d_ev = reinterpret_cast<DevEvent *>(base);
    double *d_th = reinterpret_cast<double *>(base + SIG_OFF_THETA);
    double *d_h = reinterpret_cast<double *>(base + SIG_OFF_H);
    const size_t nh = 2 * (size_t)e.n_bins * e.n_det;
    // every output element is written by the kernel: nothing to clear
    if ((he = hipMemcpy(d_ev, &d, sizeof d, hipMemcpyHostToDevice)) != hipSuccess ||
        (he = hipMemcpy(d_th, theta, sizeof(double) * NPAR, hipMemcpyHostToDevice)) != hipSuccess ||
        (he = launch_signal(d_ev, e.n_bins, e.n_det, d_th, d_h, nullptr)) != hipSuccess ||
        (he = hipMemcpy(h, d_h, sizeof(double) * nh, hipMemcpyDeviceToHost)) != hipSuccess)
        return fail(nullptr, NS_EHIP, std::string("ns_signal_noalloc: ") + hipGetErrorString(he));
    return NS_OK;
}

}  // extern "C"
