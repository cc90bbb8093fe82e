// C ABI of libpa: argument checks, host-built tables, and dispatch to the kernels.
#include <math.h>
#include <string.h>

#include <new>

#include "pa_common.h"

namespace pa {

static bool geometry_ok(int dim, int L)
{
    if (dim == 1) return L >= 4 && L % 2 == 0 && L <= (1 << 20);
    if (dim == 3) return L >= 2 && L % 2 == 0 && L <= 32;
    return false;
}

static int64_t num_sites(int dim, int L) { return dim == 1 ? (int64_t)L : (int64_t)L * L * L; }
static int64_t num_bonds(int dim, int L) { return dim == 1 ? (int64_t)L : 3 * (int64_t)L * L * L; }

// the runs of a batch take consecutive pa_state blocks, each on a 256-byte boundary
static_assert(sizeof(pa_state) == 256, "pa_state is one 256-byte block");

static int check_run(const pa_run& r)
{
    if (!geometry_ok(r.dim, r.L)) return PA_ERR_ARG;
    if (r.layout != PA_U8 && r.layout != PA_BITS64) return PA_ERR_ARG;
    if (r.couplings != PA_PM1 && r.couplings != PA_GAUSS) return PA_ERR_ARG;
    if (r.couplings == PA_GAUSS && r.layout != PA_U8) return PA_ERR_ARG;
    if (r.capacity <= 0 || r.capacity % 64 != 0 || r.capacity > ((int64_t)1 << 31)) return PA_ERR_ARG;
    if (r.R0 <= 0 || r.R0 > r.capacity || r.n_records <= 0) return PA_ERR_ARG;
    if (!r.J || !r.spins[0] || !r.spins[1] || !r.energy[0] || !r.energy[1] || !r.counts || !r.offsets ||
        !r.work || !r.record || !r.state)
        return PA_ERR_ARG;
    // the kernels move spins and work-buffer arrays in 16-byte pieces from 256-byte aligned bases
    const void* bufs[] = {r.J, r.spins[0], r.spins[1], r.energy[0], r.energy[1], r.counts, r.offsets, r.work,
                          r.record, r.state};
    for (const void* b : bufs)
        if ((uintptr_t)b % 256 != 0) return PA_ERR_ARG;
    // E^3 moments are summed in int64 over the population: |E| <= n_bonds
    const double B = (double)num_bonds(r.dim, r.L);
    if (B * B * B * (double)r.capacity > 9.0e18) return PA_ERR_ARG;
    return PA_OK;
}

// one launch per kernel for all runs: consecutive device states, one stream, one layout, one
// kind of couplings
static bool consecutive_runs(const pa_run* runs, int n)
{
    if (n < 2) return false;
    for (int r = 1; r < n; ++r) {
        if (runs[r].state != runs[0].state + r) return false;
        if (runs[r].stream != runs[0].stream || runs[r].layout != runs[0].layout || runs[r].dim != runs[0].dim ||
            runs[r].couplings != runs[0].couplings)
            return false;
    }
    return true;
}

static bool batchable(const pa_run* runs, int n) { return consecutive_runs(runs, n) && runs[0].couplings == PA_PM1; }

static bool batchable_gauss(const pa_run* runs, int n)
{
    return consecutive_runs(runs, n) && runs[0].couplings == PA_GAUSS;
}

static int check_step(const pa_step* s, bool need_weights)
{
    if (!s) return PA_ERR_ARG;
    if (!isfinite(s->beta_from) || !isfinite(s->beta_to) || s->beta_from < 0.0) return PA_ERR_ARG;
    if (s->n_sweeps < 0 || s->t0 < 0 || s->k <= 0) return PA_ERR_ARG;
    if (need_weights) {
        if (!(s->beta_to >= s->beta_from)) return PA_ERR_ARG;
        if (!s->weights || s->n_weights <= 0) return PA_ERR_ARG;
        if (!(s->R_target <= 0.0) && !isfinite(s->R_target)) return PA_ERR_ARG;
    }
    // sweep counters: 2t + colour must fit 32 bits
    if (s->t0 + s->n_sweeps >= ((int64_t)1 << 31)) return PA_ERR_ARG;
    return PA_OK;
}

int build_thresholds(double beta, int z, uint64_t* T, uint8_t* always)
{
    for (int c = 0; c <= z; ++c) {
        const int dE = 4 * c - 2 * z;
        const double p = exp(-beta * (double)dE);
        if (dE <= 0 || p >= 1.0) {
            T[c] = 0;
            always[c] = 1;
        } else {
            T[c] = (uint64_t)floor(ldexp(p, 64));
            always[c] = 0;
        }
    }
    return PA_OK;
}

// the dynamic part of a run's state, from a checkpoint (pa_resume)
__global__ void k_resume(pa_state* st, pa_info info)
{
    st->R = info.R;
    st->R_new = info.R_new;
    st->cur = info.cur;
    st->status = info.status;
    st->E_lo = info.E_lo;
    st->E_hi = info.E_hi;
    st->k = info.k;
    st->initialised = info.initialised;
    st->acc = info.acc;
    st->ln_omega = info.ln_omega;
    st->beta = info.beta;
}

}  // namespace pa

using namespace pa;

extern "C" {

int pa_buffer_sizes(int dim, int L, int layout, int couplings, int64_t capacity, int n_records, pa_sizes* out)
{
    if (!out || !geometry_ok(dim, L) || (layout != PA_U8 && layout != PA_BITS64)) return PA_ERR_ARG;
    if (couplings != PA_PM1 && couplings != PA_GAUSS) return PA_ERR_ARG;
    if (couplings == PA_GAUSS && layout != PA_U8) return PA_ERR_ARG;
    if (capacity <= 0 || capacity % 64 != 0 || n_records <= 0) return PA_ERR_ARG;
    const int64_t N = num_sites(dim, L);
    const int64_t B = num_bonds(dim, L);
    const int64_t n_bins = B / 2 + 1;
    const int64_t stride = (N + 15) / 16 * 16;
    out->N = N;
    out->n_bonds = B;
    out->n_bins = n_bins;
    out->row_stride = stride;
    out->J_bytes = couplings == PA_GAUSS ? 8 * B : B;
    // bit-packed: one row word of W bits per replica and lattice row
    const int64_t n_rows = dim == 1 ? (N + 31) / 32 : (int64_t)L * L;
    const int64_t W = dim == 1 ? 32 : (L <= 8 ? 8 : (L <= 16 ? 16 : 32));
    out->spins_bytes = layout == PA_U8 ? capacity * stride : capacity * n_rows * (W / 8);
    out->energy_bytes = (couplings == PA_GAUSS ? 8 : 4) * capacity;
    out->counts_bytes = 4 * capacity;
    out->offsets_bytes = 8 * (capacity + 1);
    out->work_bytes = (int64_t)(work_layout(N, n_bins, capacity).total + (couplings == PA_GAUSS ? gauss_table_bytes(N) : 0));
    out->record_bytes = (int64_t)sizeof(pa_record) * n_records;
    out->state_bytes = (int64_t)sizeof(pa_state);
    return PA_OK;
}

int pa_init_couplings(pa_run* runs, int n_runs, const int8_t* const* J_host)
{
    if (!runs || n_runs <= 0) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r) {
        int st = check_run(runs[r]);
        if (st != PA_OK) return st;
    }
    for (int r = 0; r < n_runs; ++r) {
        hipStream_t s = (hipStream_t)runs[r].stream;
        int st = upload_ladder(s);
        if (st != PA_OK) return st;
        st = launch_init(runs[r], J_host ? J_host[r] : nullptr, s);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int pa_sweep(pa_run* runs, int n_runs, const pa_step* step)
{
    if (!runs || n_runs <= 0) return PA_ERR_ARG;
    int st = check_step(step, false);
    if (st != PA_OK) return st;
    for (int r = 0; r < n_runs; ++r) {
        st = check_run(runs[r]);
        if (st != PA_OK) return st;
    }
    if (step->n_sweeps == 0) return PA_OK;
    SweepParams p;
    build_sweep_params(*step, 6, &p);
    bool fast = batchable(runs, n_runs) && runs[0].dim == 3 && n_runs <= 1024 && fast_sweep_thresholds_ok(p);
    for (int r = 0; fast && r < n_runs; ++r) fast = fast_sweep_supported(runs[r].dim, runs[r].L);
    if (fast) {
        st = launch_sweep_batch(runs, n_runs, p, (hipStream_t)runs[0].stream);
        if (st != PA_OK) return st;
        return hip_status(hipGetLastError());
    }
    if (batchable(runs, n_runs) && runs[0].dim == 1 && n_runs <= 65535) {
        bool same = true;
        for (int r = 1; r < n_runs; ++r) same = same && runs[r].L == runs[0].L;
        if (same) return launch_sweep_chain_batch(runs, n_runs, *step, (hipStream_t)runs[0].stream);
    }
    bool all_gauss = true, consecutive = true;
    for (int r = 0; r < n_runs; ++r) {
        all_gauss = all_gauss && runs[r].couplings == PA_GAUSS;
        consecutive = consecutive && runs[r].state == runs[0].state + r && runs[r].stream == runs[0].stream;
    }
    if (all_gauss) return launch_sweep_gauss(runs, n_runs, consecutive, *step, (hipStream_t)runs[0].stream);
    for (int r = 0; r < n_runs; ++r) {
        if (runs[r].couplings == PA_GAUSS) st = launch_sweep_gauss(&runs[r], 1, false, *step, (hipStream_t)runs[r].stream);
        else st = launch_sweep(runs[r], *step, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int pa_resample(pa_run* runs, int n_runs, const pa_step* step)
{
    if (!runs || n_runs <= 0) return PA_ERR_ARG;
    int st = check_step(step, true);
    if (st != PA_OK) return st;
    for (int r = 0; r < n_runs; ++r) {
        st = check_run(runs[r]);
        if (st != PA_OK) return st;
        pa_sizes sz;
        pa_buffer_sizes(runs[r].dim, runs[r].L, runs[r].layout, runs[r].couplings, runs[r].capacity, runs[r].n_records, &sz);
        if (step->n_weights < sz.n_bins || step->k >= runs[r].n_records) return PA_ERR_ARG;
    }
    if (batchable(runs, n_runs)) return launch_resample(runs, n_runs, *step, (hipStream_t)runs[0].stream);
    if (batchable_gauss(runs, n_runs)) return launch_resample_gauss(runs, n_runs, *step, (hipStream_t)runs[0].stream);
    for (int r = 0; r < n_runs; ++r) {
        if (runs[r].couplings == PA_GAUSS) st = launch_resample_gauss(&runs[r], 1, *step, (hipStream_t)runs[r].stream);
        else st = launch_resample(&runs[r], 1, *step, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int pa_measure(pa_run* runs, int n_runs, const int32_t* partner)
{
    if (!runs || n_runs <= 0) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r) {
        int st = check_run(runs[r]);
        if (st != PA_OK) return st;
        if (partner && partner[r] >= 0) {
            if (partner[r] >= n_runs || partner[r] == r) return PA_ERR_ARG;
            const pa_run& p = runs[partner[r]];
            if (p.dim != runs[r].dim || p.L != runs[r].L || p.layout != runs[r].layout) return PA_ERR_ARG;
        }
    }
    if (batchable(runs, n_runs) || batchable_gauss(runs, n_runs)) {
        // partners either absent or the pairs (0,1), (2,3), ...: one launch per kernel
        bool none = partner == nullptr, pairs = partner != nullptr && n_runs % 2 == 0;
        for (int r = 0; partner && r < n_runs; ++r) {
            if (partner[r] >= 0) none = false;
            if (partner[r] != (r ^ 1)) pairs = false;
        }
        const bool g = runs[0].couplings == PA_GAUSS;
        hipStream_t s0 = (hipStream_t)runs[0].stream;
        if (none) return g ? launch_measure_gauss(runs, n_runs, nullptr, 0, s0) : launch_measure(runs, n_runs, nullptr, 0, s0);
        if (pairs) return g ? launch_measure_gauss(runs, n_runs, nullptr, 1, s0) : launch_measure(runs, n_runs, nullptr, 1, s0);
    }
    for (int r = 0; r < n_runs; ++r) {
        const pa_run* p = (partner && partner[r] >= 0) ? &runs[partner[r]] : nullptr;
        int st = runs[r].couplings == PA_GAUSS ? launch_measure_gauss(&runs[r], 1, p, 0, (hipStream_t)runs[r].stream)
                                               : launch_measure(&runs[r], 1, p, 0, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int pa_free_energy(const pa_run* runs, int n_runs, double* minus_betaF_dev)
{
    if (!runs || n_runs <= 0 || !minus_betaF_dev) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r) {
        int st = check_run(runs[r]);
        if (st != PA_OK) return st;
    }
    if (consecutive_runs(runs, n_runs)) return launch_free_energy(runs, n_runs, minus_betaF_dev, (hipStream_t)runs[0].stream);
    for (int r = 0; r < n_runs; ++r) {
        int st = launch_free_energy(&runs[r], 1, minus_betaF_dev + r, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int pa_features(const pa_run* runs, int n_runs, float* x_dev)
{
    if (!runs || n_runs <= 0 || !x_dev) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r) {
        int st = check_run(runs[r]);
        if (st != PA_OK) return st;
    }
    if (batchable(runs, n_runs)) return launch_features(runs, n_runs, x_dev, (hipStream_t)runs[0].stream);
    for (int r = 0; r < n_runs; ++r) {
        int st = launch_features(&runs[r], 1, x_dev + (int64_t)r * 6, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

// shared checks and dispatch of pa_resampled_fraction (mode 0) and pa_rho_steps (mode 1)
static int rho_call(pa_run* runs, int n_runs, const double* args, int n_args, int mode, double cap, int64_t ld,
                    double* out)
{
    if (!runs || n_runs <= 0 || !args || n_args <= 0 || n_args > PA_RHO_MAX || !out) return PA_ERR_ARG;
    for (int j = 0; j < n_args; ++j) {
        if (!isfinite(args[j]) || args[j] < 0.0) return PA_ERR_ARG;
        if (mode == 1 && !(args[j] < 1.0)) return PA_ERR_ARG;
    }
    if (mode == 1 && (!(cap > 0.0) || !isfinite(cap) || ld < n_runs)) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r) {
        int st = check_run(runs[r]);
        if (st != PA_OK) return st;
        if (runs[r].couplings == PA_GAUSS) return PA_ERR_ARG;  // energy histogram needed
    }
    if (batchable(runs, n_runs)) return launch_rho(runs, n_runs, args, n_args, mode, cap, ld, out, (hipStream_t)runs[0].stream);
    for (int r = 0; r < n_runs; ++r) {
        double* o = mode == 0 ? out + (int64_t)r * n_args : out + r;
        int st = launch_rho(&runs[r], 1, args, n_args, mode, cap, ld, o, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int pa_resampled_fraction(pa_run* runs, int n_runs, const double* dbeta, int n_dbeta, double* out_dev)
{
    return rho_call(runs, n_runs, dbeta, n_dbeta, 0, 0.0, 0, out_dev);
}

int pa_rho_steps(pa_run* runs, int n_runs, const double* rho_targets, int n_targets, double cap, int64_t ld,
                 double* out_dev)
{
    return rho_call(runs, n_runs, rho_targets, n_targets, 1, cap, ld, out_dev);
}

int pa_weighted_average(int M, const double* x, const double* R, const double* A, int n_obs, double* A_bar,
                        double* omega, double* minus_betaF_bar, double* var, double* mean)
{
    if (M <= 0 || !x || n_obs < 0 || (n_obs > 0 && (!A || !A_bar)) || !minus_betaF_bar || !var || !mean)
        return PA_ERR_ARG;
    double xmax = -INFINITY;
    for (int r = 0; r < M; ++r) {
        if (!isfinite(x[r]) || (R && !(R[r] > 0.0))) return PA_ERR_ARG;
        const double xr = x[r] + (R ? log(R[r]) : 0.0);
        if (xr > xmax) xmax = xr;
    }
    double Z = 0.0, Rsum = 0.0;
    for (int r = 0; r < M; ++r) {
        Z += exp(x[r] + (R ? log(R[r]) : 0.0) - xmax);
        Rsum += R ? R[r] : 1.0;
    }
    for (int o = 0; o < n_obs; ++o) A_bar[o] = 0.0;
    for (int r = 0; r < M; ++r) {
        const double w = exp(x[r] + (R ? log(R[r]) : 0.0) - xmax) / Z;
        if (omega) omega[r] = w;
        for (int o = 0; o < n_obs; ++o) A_bar[o] += w * A[(size_t)r * n_obs + o];
    }
    *minus_betaF_bar = xmax + log(Z) - log(Rsum);
    double m = 0.0;
    for (int r = 0; r < M; ++r) m += x[r];
    m /= (double)M;
    double v = 0.0;
    for (int r = 0; r < M; ++r) v += (x[r] - m) * (x[r] - m);
    *var = M > 1 ? v / (double)(M - 1) : 0.0;
    *mean = m;
    return PA_OK;
}

int pa_weighted_average_dev(int n_sets, int M, const double* x, const double* R, const double* A, int n_obs,
                            double* out, void* stream)
{
    if (n_sets <= 0 || M <= 0 || !x || n_obs < 0 || (n_obs > 0 && !A) || !out) return PA_ERR_ARG;
    return launch_weighted_average_dev(n_sets, M, x, R, A, n_obs, out, (hipStream_t)stream);
}

int pa_overlap_average_dev(int n_sets, int n_pairs, const double* minus_betaF, const double* R, const double* Q,
                           double* out, void* stream)
{
    if (n_sets <= 0 || n_pairs <= 0 || !minus_betaF || !Q || !out) return PA_ERR_ARG;
    return launch_overlap_average_dev(n_sets, n_pairs, minus_betaF, R, Q, out, (hipStream_t)stream);
}

int pa_bootstrap_dev(int n_sets, int M, const double* x, const double* R, const double* A, int n_obs, int n_boot,
                     const int32_t* idx, double* rep, double* err, void* stream)
{
    if (n_sets <= 0 || M <= 0 || !x || n_obs < 0 || (n_obs > 0 && !A) || n_boot <= 0 || !idx || !rep || !err)
        return PA_ERR_ARG;
    return launch_bootstrap_dev(n_sets, M, x, R, A, n_obs, n_boot, idx, rep, err, (hipStream_t)stream);
}

int pa_status(const pa_run* runs, int n_runs, int32_t* host_flags)
{
    if (!runs || n_runs <= 0) return PA_ERR_ARG;
    int first = PA_OK;
    for (int r = 0; r < n_runs; ++r) {
        pa_info info;
        int st = pa_query(&runs[r], &info);
        if (st != PA_OK) return st;
        if (host_flags) host_flags[r] = info.status;
        if (first == PA_OK && info.status) {
            if (info.status & PA_FLAG_CAPACITY) first = PA_ERR_CAPACITY;
            else if (info.status & PA_FLAG_EXTINCT) first = PA_ERR_EXTINCT;
            else first = PA_ERR_NONFINITE;
        }
    }
    return first;
}

int pa_query(const pa_run* run, pa_info* out)
{
    if (!run || !out || !run->state) return PA_ERR_ARG;
    hipStream_t s = (hipStream_t)run->stream;
    pa_state h;
    if (hipMemcpyAsync(&h, run->state, sizeof(pa_state), hipMemcpyDeviceToHost, s) != hipSuccess) return PA_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PA_ERR_HIP;
    out->R = h.R;
    out->R_new = h.R_new;
    out->cur = h.cur;
    out->status = h.status;
    out->E_lo = h.E_lo;
    out->E_hi = h.E_hi;
    out->k = h.k;
    out->initialised = h.initialised;
    out->acc = h.acc;
    out->ln_omega = h.ln_omega;
    out->beta = h.beta;
    return PA_OK;
}

int pa_resume(const pa_run* runs, int n_runs, const pa_info* infos)
{
    if (!runs || !infos || n_runs <= 0) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r) {
        const pa_info& in = infos[r];
        if (check_run(runs[r]) != PA_OK) return PA_ERR_ARG;
        if (in.cur != 0 && in.cur != 1) return PA_ERR_ARG;
        if (in.R < 0 || in.R > runs[r].capacity || in.R_new < 0 || in.R_new > runs[r].capacity) return PA_ERR_ARG;
        if (in.k < 0 || in.k >= runs[r].n_records || in.initialised != 1) return PA_ERR_ARG;
    }
    for (int r = 0; r < n_runs; ++r)
        hipLaunchKernelGGL(k_resume, dim3(1), dim3(1), 0, (hipStream_t)runs[r].stream, runs[r].state, infos[r]);
    return hip_status(hipGetLastError());
}

const char* pa_strerror(int code)
{
    switch (code) {
        case PA_OK: return "ok";
        case PA_ERR_ARG: return "invalid argument";
        case PA_ERR_CAPACITY: return "resampled population exceeds the buffer capacity";
        case PA_ERR_EXTINCT: return "resampled population is empty";
        case PA_ERR_NONFINITE: return "normalisation sum is not finite and positive";
        case PA_ERR_HIP: return "HIP runtime error";
        case PA_ERR_NOT_INIT: return "run not initialised";
        case PA_ERR_SIZE: return "input larger than the fixed device scratch area holds";
        default: return "unknown status";
    }
}

int pa_graph_begin(void* stream)
{
    if (!stream) return PA_ERR_ARG;  // capture needs a stream of its own, not the null stream
    return hip_status(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
}

int pa_graph_end(void* stream, void** graph_exec)
{
    if (!stream || !graph_exec) return PA_ERR_ARG;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture((hipStream_t)stream, &g) != hipSuccess || !g) return PA_ERR_HIP;
    hipGraphExec_t e = nullptr;
    const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);  // the instantiated graph does not need it
    if (err != hipSuccess) return PA_ERR_HIP;
    *graph_exec = (void*)e;
    return PA_OK;
}

int pa_graph_launch(void* graph_exec, void* stream)
{
    if (!graph_exec) return PA_ERR_ARG;
    return hip_status(hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream));
}

int pa_graph_destroy(void* graph_exec)
{
    if (!graph_exec) return PA_ERR_ARG;
    return hip_status(hipGraphExecDestroy((hipGraphExec_t)graph_exec));
}

int pa_fill_weights(double dbeta, int64_t n, double* w)
{
    if (!w || n <= 0 || !(dbeta >= 0.0) || !isfinite(dbeta)) return PA_ERR_ARG;
    for (int64_t d = 0; d < n; ++d) w[d] = exp(-dbeta * (double)(4 * d));
    return PA_OK;
}

int pa_thresholds(double beta, int z, uint64_t* T, uint8_t* always)
{
    if (!T || !always || (z != 2 && z != 6) || !(beta >= 0.0)) return PA_ERR_ARG;
    return build_thresholds(beta, z, T, always);
}

}  // extern "C"
