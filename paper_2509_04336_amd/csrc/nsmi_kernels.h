// Kernel launch interface shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsmi_device.h"

namespace nsmi {

// Per-event sampler state, resident in device memory.
struct EvState {
    double logZ, logX, sumH, Lstar;
    double maxL, lme, dlogZ, log_frac;
    double sum_in, sum_in2;  // over dead points: sum of 1/n_i and of 1/n_i^2 (live counts at deletion)
    int64_t n_dead, n_calls, n_acc, n_oob, n_steps, batch;
    int64_t last_acc, last_calls, n_saved, n_spec;
    int32_t W, walk_this, m, k_this;
    int32_t converged, active, err;
    int32_t n_capped;  // consecutive batches whose tuned walk length is maxmcmc
};

// Sampler arrays shared by the kernels of one batch.
struct StepArgs {
    const DevEvent *ev;   // [n_events]
    EvState *st;          // [n_events]
    const double *live_u; // [e][n_live][ndim]   current live set
    const double *live_L; // [e][n_live]
    double *next_u;       // next live set
    double *next_L;
    double *snap_u;       // [e][n_live][ndim]   survivor snapshot
    double *snap_L;
    double *chain_u;      // [e][n_live][ndim]   chain start points
    double *chain_L;
    int64_t *chain_stats; // [e][n_live][4]      accepts, calls, out-of-bounds, discarded
    double *dead_u;       // [e][dead_cap][ndim]
    double *dead_L, *dead_logw, *dead_nlive;  // [e][dead_cap]
    int64_t dead_cap;
    uint64_t seed;
    int32_t n_live, ndim, k, walk_override;
    int32_t naccept, maxmcmc, term_kind, n_events;
    double delay, term_thr;
    // optional record of every exact evaluation (u, logL)
    double *hv_u, *hv_L;
    unsigned long long *hv_count;
    int64_t hv_cap;
    // delayed acceptance with the surrogate (da_on != 0)
    int32_t da_on, pad1;
    const __bf16 *mW1p, *mW2, *mW3;  // bf16 weights [256][32], [256][256], [256][256]
    const float *mP;                  // fp32 master parameters (biases, W4, b4)
    const float *m_in_mu, *m_in_isig; // input standardisation
    double m_mu, m_sig, m_top, da_margin, da_temp, da_floor;
    // several events: the events by decreasing walk cost of this batch
    // (walk length x bins), from order_kernel; NULL for one event
    const int32_t *ev_order;
};

// Workgroups of a chain launch: events * k workgroups.  With one event,
// workgroup b walks chain b.  With several, the events are taken costliest
// first (walk length x bins of this batch, from order_kernel), so the longest
// chains are dispatched first and the launch does not end on one of them.
__host__ __device__ inline int chain_blocks(const StepArgs &a) { return a.n_events * a.k; }

// Event and chain of workgroup b (false: a workgroup without a chain).
__device__ __forceinline__ bool block_chain(const StepArgs &A, int b, int *e, int *c)
{
    const int k = A.k;
    *e = A.ev_order ? A.ev_order[b / k] : b / k;
    *c = b % k;
    return true;
}

hipError_t launch_prep_event(const DevEvent &host_ev, const double *d_data, const double *d_psd,
                             char *rows64, char *rows32, double *K_out, hipStream_t s);
// Relative-binning tables of one event (d_ev on the device, hev its host copy
// with rb_rows allocated); edges [rb_bins + 1] and theta0 [11] on the device.
hipError_t launch_prep_rb(const DevEvent *d_ev, const DevEvent &hev, const int32_t *d_edges,
                          const double *d_theta0, hipStream_t s);
hipError_t launch_init_live(const DevEvent *d_ev, int n_events, int n_live, int ndim,
                            uint64_t seed, int mixed, double *live_u, double *live_L, int max_det,
                            hipStream_t s);
hipError_t launch_loglike_theta(const DevEvent *d_ev, int n_det, const double *theta, int64_t n,
                                double *out, int mixed, hipStream_t s);
hipError_t launch_theta_from_u(const DevEvent *d_ev, const double *u, int64_t n, double *theta,
                               hipStream_t s);
hipError_t launch_loglike_u(const DevEvent *d_ev, int n_det, int ndim, const double *u,
                            int64_t n, double *out, int mixed, hipStream_t s);
hipError_t launch_select(const StepArgs &a, hipStream_t s);
// Events by decreasing walk cost of this batch into order[n_events] (a
// permutation; ties by event index).  After launch_select.
hipError_t launch_order(const StepArgs &a, int32_t *order, hipStream_t s);
hipError_t launch_walk(const StepArgs &a, int max_det, int waves_per_chain, int mixed,
                       hipStream_t s);
hipError_t launch_finish(const StepArgs &a, hipStream_t s);
// log Z of R replicates of one event's dead points (event e): the expected
// shrinkage of each deletion replaced by log t_i, t_i ~ Beta(n_i, 1) (log t_i
// = log(U_i) / n_i), uniforms U [R][n_dead] from the caller (device) or, when
// U is NULL, 1 - u01 of Philox (seed, i, r, P_REPL); out [R] (device).
hipError_t launch_replicates(const double *dead_L, const double *dead_nlive, int64_t n_dead,
                             const double *live_L, int n_live, const double *U, uint64_t seed,
                             int R, double *out, hipStream_t s);
hipError_t launch_signal(const DevEvent *d_ev, int n_bins, int n_det, const double *theta,
                         double *h, hipStream_t s);

}  // namespace nsmi
