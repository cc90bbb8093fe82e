/*
 * pa.h -- C ABI of the MI355X population-annealing library (libpa.so).
 *
 * Population annealing with weighted averages (J. Machta, arXiv:1006.0252) for
 * Ising spin glasses with +-1 couplings: a population of replicas sharing one
 * set of couplings is cooled from beta = 0 through a schedule; each step
 * resamples the population by Boltzmann weights (Sec. II, eqs. Q and wn, Poisson
 * copy numbers), runs theta Metropolis sweeps at the new temperature, measures
 * observables, and accumulates the free-energy estimator (eq. sumQ).  Runs are
 * combined by free-energy weighted averages (Sec. III, eqs. weight, omega, bestf;
 * Sec. IV, eq. omegaprime).
 *
 * Conventions common to every call
 *   - Every function returns an int status (PA_OK = 0) and never aborts; no C++
 *     exception crosses this interface.
 *   - The library allocates no device memory.  All device buffers are owned by the
 *     caller, sized by pa_buffer_sizes(), and described in a pa_run.  Host pointers
 *     are only borrowed for the duration of a call.
 *   - Device work is asynchronous and ordered on run->stream (a hipStream_t, NULL =
 *     the null stream).  Nothing but pa_status() and pa_query() waits for the device.
 *     Population sizes stay on the device, so sweep/resample/measure/free-energy
 *     calls may be captured in a HIP graph.
 *   - Errors found on the host (bad arguments) are returned at once.  Errors found on
 *     the device (capacity overflow, extinction, non-finite weights) set sticky bits in
 *     the run's device state; pa_status() reads them.  A step that raises one leaves
 *     the population unchanged.
 *   - Calls with n_runs > 1 apply the same step to every run (batching).  When the runs'
 *     pa_state blocks are consecutive in device memory (state of run r at runs[0].state + r),
 *     share one stream and one layout, each kernel is launched once for all of them: the
 *     resampling and measurement kernels index runs by grid row, and the cube sweep (even L
 *     from 4 to 16) is one persistent launch whose waves take (run, tile of replicas) items
 *     from a device work list.  Otherwise the runs are processed one after the other.  The
 *     results are the same either way (every draw is keyed by run seed and replica index).
 *
 * Physics conventions
 *   - dim 1: periodic chain of N = L spins; bond b = i joins sites i and i+1 (mod N).
 *     dim 3: periodic simple cubic lattice of N = L^3 spins, site i = x + L (y + L z);
 *     bond b = 3 i + a joins site i and its +a neighbour (a = 0, 1, 2 for x, y, z).
 *     L must be even (checkerboard order needs a bipartite lattice).
 *   - Energy E = + sum_b J_b s_i s_j (the sign printed in Sec. IV), J_b = +-1.
 *   - Spins: 1 means s = -1.  Layout PA_U8: one byte per spin, replica-major rows of
 *     row_stride bytes (N rounded up to 16).  Layout PA_BITS64 (bit-packed, replicas in
 *     groups of 64): the lattice is cut into rows -- (y, z) rows of L sites on the cube,
 *     runs of 32 consecutive sites on the chain -- and each replica stores one W-bit row
 *     word per row (W = 8, 16 or 32, the smallest >= L on the cube; 32 on the chain), bit x
 *     = spin at site x + L row (cube) or 32 row + x (chain); row word (g, row, l) of replica
 *     64 g + l is element (g * n_rows + row) * 64 + l.  An L = 16 replica takes 512 bytes.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the run seed
 *     (couplings: by the disorder seed); counter layouts are documented at each call.
 */
#ifndef PA_H
#define PA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define PA_OK 0
#define PA_ERR_ARG 1        /* invalid argument (odd L, dim not 1/3, beta_to < beta_from, ...) */
#define PA_ERR_CAPACITY 2   /* resampled population larger than the buffers' capacity */
#define PA_ERR_EXTINCT 3    /* resampled population empty */
#define PA_ERR_NONFINITE 4  /* normalisation sum S not finite or not positive */
#define PA_ERR_HIP 5        /* HIP runtime error (launch, copy, synchronisation) */
#define PA_ERR_NOT_INIT 6   /* run not initialised by pa_init_couplings */
#define PA_ERR_SIZE 7       /* input larger than a fixed-size device scratch area holds */

/* sticky device status bits (pa_status) */
#define PA_FLAG_CAPACITY (1 << 0)
#define PA_FLAG_EXTINCT (1 << 1)
#define PA_FLAG_NONFINITE (1 << 2)

/* spin layouts */
#define PA_U8 0
#define PA_BITS64 1 /* bit-packed rows, groups of 64 replicas (see above) */

/* coupling kinds */
#define PA_PM1 0   /* J = +-1 equiprobable (int8 couplings, int32 energies) */
#define PA_GAUSS 1 /* J normal, mean 0, variance 1 (the model of Sec. IV; FP64 couplings and energies) */

/* Per-temperature record, one per schedule index k, written on the device.
 * pa_resample fills beta .. E_lo of record[k]; pa_measure fills the rest. */
typedef struct pa_record {
    double beta;        /* beta_k */
    double lnQ;         /* ln Q(beta_{k-1}, beta_k) (eq. Q); 0 at k = 0 */
    double minus_betaF; /* -beta_k F~(beta_k) = N ln 2 + sum_{l <= k} ln Q_l (eq. sumQ) */
    double S;           /* sum over energies E of h(E) exp(-(beta_k - beta_{k-1})(E - E_lo)) */
    double R;           /* population size after resampling */
    double E_lo;        /* lowest energy in the population before resampling */
    double E_mean;      /* energy mean after the sweeps (no weights inside a run, Sec. II) */
    double E_var;       /* energy variance (population, 1/R) */
    double E_skew;      /* third central moment / var^1.5 */
    double q2;          /* <q^2> over replica pairs with the partner run (Sec. IV) */
    double q4;          /* <q^4> */
    double gamma;       /* Prob(|q| < 0.2) (Sec. IV) */
    double n_pairs;     /* replica pairs behind q2, q4, gamma (0: no partner) */
    double reserved[3];
} pa_record;

/* Device state of one run (caller allocates sizeof(pa_state) bytes of device memory,
 * 256-byte aligned).  Written by pa_init_couplings and the later calls; read on the
 * host only through pa_query. */
typedef struct pa_state {
    /* descriptor, written by pa_init_couplings */
    int32_t dim, L, N, z;
    int32_t n_bonds, layout, n_bins, row_stride;
    int64_t capacity, R0;
    uint64_t seed, disorder_seed;
    int8_t* J;
    void* spins[2];
    int32_t* energy[2];
    int32_t* counts;
    int64_t* offsets;
    uint8_t* work;
    pa_record* record;
    int32_t n_records, E_base;
    /* dynamic state */
    int64_t R;      /* current population size */
    int64_t R_new;  /* size produced by the last resampling scan */
    int32_t cur;    /* which of spins[]/energy[] holds the population */
    int32_t status; /* sticky PA_FLAG_* bits */
    int32_t E_lo, E_hi;
    int32_t k;      /* schedule index of the current temperature */
    int32_t initialised;
    double acc;     /* sum of ln Q so far */
    double ln_omega;/* N ln 2 */
    double beta;    /* current inverse temperature */
    uint32_t work_counter; /* work items taken by a batched sweep (counted in the first run of each group of equal-L runs) */
    uint32_t reserved0;
    int32_t couplings;     /* PA_PM1 or PA_GAUSS */
    uint8_t pad[36];
} pa_state;

/* Host descriptor of one run; every pointer but stream is a device pointer. */
typedef struct pa_run {
    int32_t dim;             /* 1 or 3 */
    int32_t L;               /* linear size (even); N = L or L^3 */
    int32_t layout;          /* PA_U8 or PA_BITS64 */
    int32_t n_records;       /* entries of record[] (schedule length) */
    int32_t couplings;       /* PA_PM1 or PA_GAUSS (PA_GAUSS: layout PA_U8 only) */
    int32_t reserved;        /* 0 */
    int64_t capacity;        /* replicas each population buffer holds; multiple of 64 */
    int64_t R0;              /* initial population size and default target size */
    uint64_t seed;           /* run seed */
    uint64_t disorder_seed;  /* coupling seed */
    int8_t* J;               /* [n_bonds] couplings */
    void* spins[2];          /* two population buffers of spins_bytes */
    int32_t* energy[2];      /* two [capacity] energy buffers */
    int32_t* counts;         /* [capacity] copy numbers of the last resampling */
    int64_t* offsets;        /* [capacity + 1] exclusive scan of counts */
    void* work;              /* work_bytes of scratch (histograms, bin tables, scan) */
    pa_record* record;       /* [n_records] */
    pa_state* state;         /* one pa_state */
    void* stream;            /* hipStream_t */
} pa_run;
/* Every device pointer of a pa_run is 256-byte aligned (as hipMalloc returns it; the runs of a
 * batch take consecutive pa_state blocks, sizeof(pa_state) = 256); calls return PA_ERR_ARG
 * otherwise, before touching the device. */

/* One temperature step beta_from -> beta_to (schedule index k >= 1). */
typedef struct pa_step {
    double beta_from;
    double beta_to;
    double R_target;         /* > 0: target population R_{beta_to} for every run; <= 0: run's R0 */
    int32_t k;               /* schedule index of beta_to */
    int32_t n_sweeps;        /* theta: Metropolis sweeps at beta_to */
    int64_t t0;              /* global index of the first of those sweeps */
    const double* weights;   /* device [n_weights]: w_d = exp(-(beta_to - beta_from) * 4d) */
    int64_t n_weights;       /* >= n_bins of every run (pa_buffer_sizes) */
} pa_step;

/* Buffer sizes (bytes) of one run. */
typedef struct pa_sizes {
    int64_t N, n_bonds, n_bins, row_stride;
    int64_t J_bytes, spins_bytes, energy_bytes, counts_bytes, offsets_bytes;
    int64_t work_bytes, record_bytes, state_bytes;
} pa_sizes;

/* Host-side information read back by pa_query (synchronises run->stream). */
typedef struct pa_info {
    int64_t R, R_new;
    int32_t cur, status, E_lo, E_hi, k, initialised;
    double acc, ln_omega, beta;
} pa_info;

/* Buffer sizes (bytes) of one run.  Returns PA_ERR_ARG for dim not in {1, 3}, odd or
 * too small L (1D: L >= 4; 3D: L >= 2, L <= 32), capacity not a positive multiple of 64, a
 * coupling kind other than PA_PM1 / PA_GAUSS, or Gaussian couplings with a layout other than
 * PA_U8.  Couplings take 1 byte per bond (PA_PM1) or 8 (PA_GAUSS), energies 4 or 8 bytes per
 * replica; with PA_GAUSS the work buffer also holds the sweep's threshold tables (640 N bytes:
 * 16-bit first-look entries and 64-bit thresholds per site and neighbour pattern, rewritten by
 * every pa_sweep), so buffers must be sized with the run's coupling kind. */
int pa_buffer_sizes(int dim, int L, int layout, int couplings, int64_t capacity, int n_records, pa_sizes* out);

/* Initialise runs (Sec. II: R0 replicas at beta = 0, each uniform over the 2^N states):
 *   couplings: J_b = -1 iff bit (b mod 128) of Philox(ctr (b/128, 0, 0, 5), key disorder_seed)
 *              is set, unless J_host[r] (host, [n_bonds] +-1) is given for run r;
 *   spins: spin i of replica r is bit (i mod 128) of Philox(ctr (i/128, r, 0, 1), key seed);
 *   energies computed from the spins; R~ = R0, accumulator 0, ln Omega = N ln 2, k = 0,
 *   record[0] written; status cleared.
 * J_host may be NULL (all runs from their disorder seed) or an array of n_runs host
 * pointers, each NULL or a coupling array.  R0 must not exceed capacity. */
int pa_init_couplings(pa_run* runs, int n_runs, const int8_t* const* J_host);
/* Gaussian couplings (runs with couplings = PA_GAUSS, the model of Sec. IV).  The couplings are
 * drawn on the host and copied to the device before the call returns (J_host must be NULL):
 *   J_b = sqrt(-2 ln u1) cos(2 pi u2), u1 = (m1 + 1) 2^-53, u2 = m2 2^-53, with
 *   m1 = (w0 >> 5) 2^26 + (w1 >> 6), m2 = (w2 >> 5) 2^26 + (w3 >> 6) and (w0..w3) =
 *   Philox(ctr (b, 0, 0, 6), key disorder_seed); libm log, cos and sqrt.
 * Energies are FP64: E = sum over bonds b = 0, 1, ... of J_b s_i s_j added in bond order from 0,
 * recomputed in that order after every pa_sweep.  A flip changes E by dE = -2 s_i h_i with the
 * local field h_i summed in the order +x, +y, +z, -x, -y, -z (chain: +1, -1); a move with
 * dE > 0 is accepted with probability T64 / 2^64, T64 = (uint64)(expd(-(beta dE)) 2^64), by the
 * same draws as for +-1 couplings, where expd is exp evaluated as 2^k e^r, k = floor(x / ln 2 +
 * 1/2), r = (x - k ln2_hi) - k ln2_lo (ln2_hi = 0.6931471803691238, ln2_lo =
 * 1.9082149292705877e-10), e^r by its Taylor series to r^13 in Horner form, and 0 below -745.
 * Resampling: E_lo = min E, w_j = expd(-(dbeta (E_j - E_lo))), S = sum of w_j added in replica
 * order j = 0, 1, ... (eq. Q), ln Q = -dbeta E_lo + ln S - ln R~,
 * copies of j ~ Poisson((R_target w_j) / S) by the ladder of pa_resample.  FP64 products and
 * sums are never fused.  In calls with n_runs > 1, Gaussian runs whose pa_state blocks are
 * consecutive and share a stream take one launch per kernel, others one after the other;
 * pa_resampled_fraction / pa_rho_steps reject them.  pa_sweep tabulates, per call, the top 16
 * bits of T64 for every site and neighbour pattern (cubes of side 4 and 8, chains of 16k <= 1024
 * sites; other shapes compute dE per attempt): the accepted moves are the same. */

/* theta = step->n_sweeps Metropolis sweeps of every replica at beta = step->beta_to
 * (Sec. II, the equilibration loop of the algorithm).  A sweep updates all sites of
 * colour 0 then all of colour 1 (colour (x+y+z) mod 2, or i mod 2 on the chain).
 * Flipping spin i changes the energy by dE = 4c - 2z, c = number of bonds at i with
 * J s_i s_j = -1; the flip is accepted if dE <= 0, else with probability T64 / 2^64,
 * T64 = floor(exp(-beta dE) 2^64), against the uniform U = (u16 << 48) | u48:
 *   u16 = 16-bit field (h mod 8) of Philox(ctr (h/8, r, 2t+colour, 2)), h = i/2
 *         (field f = bits 16 (f mod 2) .. of word f/2);
 *   u48 = word0 | (word1 mod 2^16) << 32 of Philox(ctr (i, r, 2t+colour, 3));
 * t = step->t0 + s is the global sweep index, r the replica's index in the population.
 * Energies are updated with the spins.  Sizes: chains of any length; cubes of even side up
 * to 20, and 24 and 32 (other sides: PA_ERR_ARG, nothing launched); Gaussian couplings: any
 * size the buffers allow (tabled kernels for cube sides 4 and 8 and chains of 16k <= 1024 sites,
 * one thread per replica otherwise). */
int pa_sweep(pa_run* runs, int n_runs, const pa_step* step);

/* Resample beta_from -> beta_to (Sec. II, eqs. Q and wn, Poisson copy numbers):
 *   h(E) = replicas at energy E; E_lo = lowest energy present;
 *   S = sum over E ascending of h(E) * w_{(E - E_lo)/4}   (FP64, in that order);
 *   ln Q = -(beta_to - beta_from) E_lo + ln S - ln R~;  accumulator += ln Q;
 *   copies of replica j ~ Poisson(lambda_j), lambda_j = (R_target * w_{(E_j - E_lo)/4}) / S,
 *   drawn by the power-of-two ladder with thinning (draw d of replica j at step k is word
 *   d mod 4 of Philox(ctr (d/4, j, k, 4), key seed));
 *   offsets = exclusive scan of copies, R~' = total; the new population holds the copies
 *   of replica j at offsets[j] .. offsets[j] + copies - 1 (source order).
 * Writes record[k].beta .. E_lo.  Raises PA_FLAG_CAPACITY (R~' > capacity),
 * PA_FLAG_EXTINCT (R~' = 0) or PA_FLAG_NONFINITE, in which case the population, the
 * accumulator, k and record[k] are left unchanged.  step->weights must hold n_bins entries for
 * dbeta = beta_to - beta_from (pa_fill_weights). */
int pa_resample(pa_run* runs, int n_runs, const pa_step* step);

/* Observables after the sweeps (Sec. II): energy mean, variance and skewness of the
 * population into record[k]; with partner != NULL (host array of n_runs run indices
 * into runs[], -1 for none) also the overlap q = (1/N) sum_i s_i s'_i of replica j
 * with replica j of the partner run for j < min(R~, R~'), giving <q^2>, <q^4> and
 * Gamma = Prob(|q| < 0.2) (Sec. IV). */
int pa_measure(pa_run* runs, int n_runs, const int32_t* partner);

/* -beta_k F~(beta_k) = N ln 2 + sum of ln Q (eq. sumQ) of every run at its current
 * temperature into minus_betaF_dev[r] (device, [n_runs]). */
int pa_free_energy(const pa_run* runs, int n_runs, double* minus_betaF_dev);

/* Weighted average over M runs, host FP64 (Sec. III, eqs. weight, omega, bestf):
 *   x_r = minus_betaF[r] (+ ln R[r] when R != NULL: runs with unequal target sizes);
 *   omega_r = exp(x_r - max x) / sum exp(x - max x);  A_bar[o] = sum_r omega_r A[r][o];
 *   -beta F_bar = max x + ln sum exp(x - max x) - ln sum_r R[r] (R[r] = 1 when NULL);
 *   var = sum (minus_betaF - mean)^2 / (M - 1);  mean = plain mean of minus_betaF.
 * For overlap observables pass minus_betaF[r] = -beta (F~^(1) + F~^(2)) of pair r
 * (eq. omegaprime).  A is [M][n_obs] row-major; omega may be NULL. */
int pa_weighted_average(int M, const double* minus_betaF, const double* R, const double* A, int n_obs,
                        double* A_bar, double* omega, double* minus_betaF_bar, double* var,
                        double* mean);

/* The same on the device for n_sets independent sets of M runs (set s uses
 * minus_betaF[s*M ..], R[s*M ..], A[s*M*n_obs ..]); out is [n_sets][n_obs + 3]:
 * A_bar[0..n_obs-1], -beta F_bar, var, mean.  All pointers are device pointers. */
int pa_weighted_average_dev(int n_sets, int M, const double* minus_betaF, const double* R, const double* A,
                            int n_obs, double* out, void* stream);

/* Overlap observables of pairs of runs on the device (Sec. IV, eqs. pqs and omegaprime), for n_sets
 * independent sets of n_pairs pairs.  Pair p of set s joins runs 2p and 2p + 1 of that set:
 * minus_betaF[s][2 n_pairs] holds -beta F~ of every run and R[s][2 n_pairs] its target size (NULL:
 * equal sizes); Q[s][n_pairs][3] holds the pair's <q^2>, <q^4> and Gamma (record[k].q2, q4, gamma
 * of a pa_measure call with that partner).  The pair weight is
 *   omega'_p = R^(1) R^(2) exp(x^(1) + x^(2)) / sum over pairs of the same,  x = minus_betaF,
 * and out[s][4] receives the weighted [q^2], [q^4], [Gamma] and the Binder ratio
 *   g = (3 - [q^4] / [q^2]^2) / 2.
 * All pointers are device pointers; asynchronous on stream.  PA_ERR_ARG for n_sets or n_pairs
 * not positive or a NULL array other than R. */
int pa_overlap_average_dev(int n_sets, int n_pairs, const double* minus_betaF, const double* R, const double* Q,
                           double* out, void* stream);

/* Bootstrap errors of the device weighted averages (Sec. III: the error is the standard
 * deviation over resampled ensembles, each of M runs).  idx is device int32 [n_boot][M]: run
 * indices in [0, M) drawn by the caller with replacement, one resampled ensemble per row, the
 * same rows for every set.  rep (device [n_sets][n_boot][n_obs + 3]) receives each resampled
 * ensemble's (A_bar, -beta F_bar, var, mean) as pa_weighted_average_dev computes them; err
 * (device [n_sets][n_obs + 3]) their standard deviations over the n_boot rows (1/(n_boot - 1)).
 * A row holding an index outside [0, M) gives NaN for that replicate (and so for err).
 * The other arguments are those of pa_weighted_average_dev. */
int pa_bootstrap_dev(int n_sets, int M, const double* minus_betaF, const double* R, const double* A, int n_obs,
                     int n_boot, const int32_t* idx, double* rep, double* err, void* stream);

/* Synchronise each run's stream and read its sticky status bits into host_flags[r];
 * returns PA_OK, or the PA_ERR_* code of the first raised bit. */
int pa_status(const pa_run* runs, int n_runs, int32_t* host_flags);

/* Synchronise run->stream and copy the dynamic part of its state to the host. */
int pa_query(const pa_run* run, pa_info* out);

/* Resume runs from a checkpoint.  A run's whole state between steps is its couplings, the
 * spins and energies of the current buffer, its records and the dynamic part of its device
 * state (pa_info, as pa_query returns it); resampling and measurement keep nothing else across
 * calls, and every draw is keyed by (seed, replica, sweep or step index), so a resumed run
 * continues bit for bit as the uninterrupted one would.  Protocol: pa_init_couplings on the new
 * buffers (same dim, L, layout, couplings kind, seeds, capacity and n_records as the
 * checkpointed run); then the caller copies the checkpoint's couplings into J, its spins into
 * spins[info.cur], its energies into energy[info.cur] and its records into record; then
 * pa_resume writes infos[r] into run r's device state (stream-ordered on runs[r].stream).
 * PA_ERR_ARG for an invalid run, cur outside {0, 1}, R or R_new outside [0, capacity], k outside
 * [0, n_records) or initialised != 1. */
int pa_resume(const pa_run* runs, int n_runs, const pa_info* infos);

/* Message for a status code. */
const char* pa_strerror(int code);

/* Host tables (FP64, libm exp).  w[d] = exp(-dbeta * 4d), d < n. */
int pa_fill_weights(double dbeta, int64_t n, double* w);
/* T64 thresholds for classes c = 0..z at beta (dE = 4c - 2z): T[c], always[c] = 1
 * when the move is always accepted (dE <= 0 or exp(-beta dE) >= 1). */
int pa_thresholds(double beta, int z, uint64_t* T, uint8_t* always);
/* Inversion table of Poisson(2^m), m in [-20, 6]: C[n] = floor(CDF(n) 2^32), last entry
 * 2^32; returns the length through *len (at most cap entries written). */
int pa_ladder_table(int m, uint64_t* C, int cap, int* len);

/* HIP graph of a whole schedule: every pa_sweep / pa_resample / pa_measure / pa_free_energy
 * call between pa_graph_begin and pa_graph_end on `stream` (a non-null hipStream_t that all
 * the captured runs use) is recorded instead of run; pa_graph_launch replays it on a stream.
 * Population sizes and status live on the device, so a replay is the same computation as the
 * eager calls.  The graph object is host-owned by the library until pa_graph_destroy. */
int pa_graph_begin(void* stream);
int pa_graph_end(void* stream, void** graph_exec);
int pa_graph_launch(void* graph_exec, void* stream);
int pa_graph_destroy(void* graph_exec);

/* Batched sweep schedule, for the autotuner.  The runs of a batch are grouped by lattice size
 * and each group is one launch over the device work list of (run, tile) items:
 *   blocks_per_cu (1..32): resident blocks per compute unit of a persistent launch;
 *   order: 0 groups in order of first appearance, 1 larger tiles first;
 *   launch: 0 by size (persistent loop for L = 0 mod 4, one item per block otherwise),
 *           1 persistent loop for every size, 2 one item per block for every size.
 * (0, 0, 0) restores the defaults (16, 1, 0).  Results do not depend on it. */
int pa_set_batch_config(int blocks_per_cu, int order, int launch);

/* Launch shape of the sweep kernels for later calls in this process: lanes per replica
 * (1, 2 or 4; a replica's rows are split among that many lanes) and waves per block (1..4).
 * (0, 0) restores the built-in choice.  Results do not depend on it (same draws, same
 * order of acceptance tests per site); it exists for the autotuner. */
int pa_set_sweep_config(int lanes_per_replica, int waves_per_block);

/* ------------------------------------------------- learned temperature steps (extension)
 * The paper leaves the temperature schedule to the user: any sequence of temperatures gives
 * an exact method (Sec. II), and Var(beta F~) across runs measures its quality (Sec. III).
 * These calls let a small network propose each step dbeta from statistics of the population
 * itself.  Resampling is unchanged, so any proposed schedule is an exact one; a schedule is
 * produced on a pilot run and then frozen for the production runs, which keeps the
 * estimators of Sec. III valid.
 *
 * Resampled fraction of a step: with the normalised weights tau_j of eq. wn for a step dbeta,
 *   rho(dbeta) = 1 - (1/R~) sum_j min(1, tau_j),
 * the total-variation distance between the population and its reweighting (0 at dbeta = 0,
 * non-decreasing in dbeta, below 1 - fraction at the lowest energy).
 *
 * Network: 6 -> 64 -> 64 -> 64 -> 1, tanh hidden units, BF16 parameters, FP32 arithmetic.
 * Inputs x = (beta, ln N, ln R~, E_mean/N, E_var/N, E_skew) (pa_features), mapped to
 * xh = ((beta - 2.5)/2.5, (ln N - 6)/2, (ln R~ - 10)/2.5, E/N + 1, var/N - 1, skew/2).
 * Output z; the proposed step is dbeta = softplus(z) / sigma_E with sigma_E = sqrt(N var/N),
 * i.e. the network predicts the step in units of the energy spread.  Parameter vector
 * (PA_MLP_PARAMS values, W[out][in] row-major): W1[64][6] @0, b1[64] @384, W2[64][64] @448,
 * b2 @4544, W3[64][64] @4608, b3 @8704, w4[64] @8768, b4 @8832. */
#define PA_MLP_PARAMS 8833
#define PA_RHO_MAX 8

/* Features of every run's population at its current temperature into x_dev[r][6] (device
 * FP32): (beta, ln N, ln R~, E_mean/N, E_var/N, E_skew) from record[k], so call after
 * pa_measure.  Asynchronous on the runs' streams. */
int pa_features(const pa_run* runs, int n_runs, float* x_dev);

/* rho(dbeta[j]) of every run's current population for n_dbeta (1..PA_RHO_MAX) host values
 * dbeta[j] >= 0, into out_dev[r * n_dbeta + j] (device FP64).  NaN for a run with a raised
 * status bit. */
int pa_resampled_fraction(pa_run* runs, int n_runs, const double* dbeta, int n_dbeta, double* out_dev);

/* Step labels: for each host target rho_targets[j] in [0, 1) (n_targets <= PA_RHO_MAX) the
 * dbeta in [0, cap] with rho(dbeta) = rho_targets[j], by 64 halvings of [0, cap]; cap when
 * rho(cap) <= rho_targets[j].  Written to out_dev[j * ld + r] (device FP64, ld >= n_runs).
 * NaN for a run with a raised status bit. */
int pa_rho_steps(pa_run* runs, int n_runs, const double* rho_targets, int n_targets, double cap, int64_t ld,
                 double* out_dev);

/* Proposed steps for B feature rows x[B][6] (device FP32) with BF16 parameters w (device,
 * PA_MLP_PARAMS): dbeta[b] = min(max(softplus(z) / sigma_E, dbeta_min), dbeta_max), and
 * dbeta_max when E_var <= 0 or the result is NaN.  0 <= dbeta_min <= dbeta_max < inf. */
int pa_mlp_forward(const uint16_t* w, const float* x, int64_t B, float dbeta_min, float dbeta_max, float* dbeta,
                   void* stream);

/* Bytes of device work memory pa_mlp_grad needs for a batch of B samples. */
int pa_mlp_work_bytes(int64_t B, int64_t* bytes);

/* Loss and gradient of a batch: loss = (1/B) sum_b (ln softplus(z_b) - ln sigma_E,b -
 * ln target[b])^2, the squared error of ln dbeta (samples with E_var <= 0 or a target that is
 * not a finite positive number contribute 0); grad (device FP32 [PA_MLP_PARAMS]) by
 * backpropagation, loss (device FP32 [1], may be NULL).  target is device FP64 [B] (labels
 * from pa_rho_steps); work is pa_mlp_work_bytes(B) bytes of device memory.  The sums over
 * the batch are taken in a fixed order, so the result is reproducible. */
int pa_mlp_grad(const uint16_t* w, const float* x, const double* target, int64_t B, void* work, float* grad,
                float* loss, void* stream);

/* pa_mlp_grad for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same kernels and the same result, bit for
 * bit, with the work matrix and partial gradients in a fixed device array of the library
 * (PA_MLP_STATIC_MAX_B samples, 6.6 MB, held on each device from the first call until the process
 * ends) instead of caller memory.  Allocates nothing.  B > PA_MLP_STATIC_MAX_B returns PA_ERR_SIZE
 * before any device work.  Every call on a device shares that device's array: calls that overlap
 * on one GPU (different streams, threads or processes' graphs) race and must be serialised by the
 * caller. */
#define PA_MLP_STATIC_MAX_B 4096
int pa_mlp_grad_static(const uint16_t* w, const float* x, const double* target, int64_t B, float* grad, float* loss,
                       void* stream);

/* One Adam step (Kingma and Ba, ICLR 2015), step number t >= 1, on n FP32 master parameters
 * theta with moments m, v (device, zero before the first step): m = beta1 m + (1 - beta1) g,
 * v = beta2 v + (1 - beta2) g^2, theta -= lr (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps);
 * then w = BF16(theta), rounded to nearest, ties to even. */
int pa_mlp_adam(float* theta, float* m, float* v, const float* grad, uint16_t* w, int64_t n, int t, float lr,
                float beta1, float beta2, float eps, void* stream);

/* out[i] = BF16 bits of x[i] (device), round to nearest, ties to even, NaN -> 0x7FC0. */
int pa_bf16_round(const float* x, uint16_t* out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PA_H */
