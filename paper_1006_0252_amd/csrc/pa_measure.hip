// Observables and estimators: energy moments after the sweeps (Sec. II: measured after
// resampling, no weights inside a run), overlap q between replicas of two runs and
// Gamma = Prob(|q| < 0.2) (Sec. IV), free-energy estimator (eq. sumQ), and the device
// version of the weighted average over runs (Sec. III, eqs. weight, omega, bestf).
#include <math.h>

#include <algorithm>

#include "pa_common.h"

#pragma clang fp contract(off)

namespace pa {

constexpr int kMiscEmin = 0, kMiscEmax = 1;

// energy mean (exact integer sum), variance and skewness from the histogram, into record[k]
__global__ void __launch_bounds__(64) k_moments(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
    const int64_t* hist = work_ptr<int64_t>(st, wl.hist);
    const int64_t* misc = work_ptr<int64_t>(st, wl.misc);
    const int E_lo = (int)misc[kMiscEmin], E_hi = (int)misc[kMiscEmax];
    const int Eb = st->E_base;
    const int ilo = (E_lo - Eb) >> 2, ihi = (E_hi - Eb) >> 2;
    const int64_t R = st->R;
    int64_t s1 = 0;
    for (int i = ilo + threadIdx.x; i <= ihi; i += 64) s1 += hist[i] * (int64_t)(Eb + 4 * i);
    for (int off = 32; off > 0; off >>= 1) s1 += __shfl_xor(s1, off, 64);
    const double mean = (double)s1 / (double)R;
    // central moments: strided partial sums over the bins, then a butterfly over the wave
    double m2 = 0.0, m3 = 0.0;
    for (int i = ilo + threadIdx.x; i <= ihi; i += 64) {
        const int64_t h = hist[i];
        if (!h) continue;
        const double d = (double)(Eb + 4 * i) - mean;
        m2 += (double)h * (d * d);
        m3 += (double)h * (d * d * d);
    }
    for (int off = 32; off > 0; off >>= 1) {
        m2 += __shfl_xor(m2, off, 64);
        m3 += __shfl_xor(m3, off, 64);
    }
    if (threadIdx.x != 0) return;
    m2 /= (double)R;
    m3 /= (double)R;
    pa_record* rec = st->record + st->k;
    rec->E_mean = mean;
    rec->E_var = m2;
    rec->E_skew = m2 > 0.0 ? m3 / (m2 * sqrt(m2)) : 0.0;
}

__global__ void k_qhist_clear(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    int64_t* qh = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).qhist);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= st->N; i += gridDim.x * blockDim.x) qh[i] = 0;
}

// Hamming distances, one byte per spin: a wave per replica pair (its lanes over 16-byte pieces of the
// rows, then a wave sum), kOverlapU8Items pairs per wave in turn; the block counts its distances in
// an LDS histogram (cap entries, when N + 1 fits) and adds the non-zero bins to the run's
// histogram (one global atomic per pair serialised on the few bins a population's distances take)
constexpr int kOverlapU8Items = 8;

__global__ void __launch_bounds__(256) k_overlap_u8(pa_state* base, const pa_state* b_given, int pair_xor, int cap)
{
    extern __shared__ uint32_t hloc[];
    if (pair_xor && (blockIdx.y & 1)) return;  // a pair's distances are counted once, by its first run
    pa_state* a = base + blockIdx.y;
    const pa_state* b = pair_xor ? base + (blockIdx.y ^ 1) : b_given;
    if (a->status || b->status) return;
    const int64_t P = min(a->R, b->R);
    const int64_t j0 = (int64_t)blockIdx.x * 4 * kOverlapU8Items;
    if (j0 >= P) return;  // the same for the whole block
    const int stride = a->row_stride, N = a->N;
    const bool local = N + 1 <= cap;
    int64_t* qh = work_ptr<int64_t>(a, work_layout(a->N, a->n_bins, a->capacity).qhist);
    if (local) {
        for (int d = threadIdx.x; d <= N; d += blockDim.x) hloc[d] = 0;
        __syncthreads();
    }
    const int lane = threadIdx.x & 63;
    for (int it = 0; it < kOverlapU8Items; ++it) {
        const int64_t j = j0 + (int64_t)(threadIdx.x >> 6) * kOverlapU8Items + it;
        if (j >= P) break;  // the same for the whole wave
        const uint8_t* x = (const uint8_t*)a->spins[a->cur] + j * stride;
        const uint8_t* y = (const uint8_t*)b->spins[b->cur] + j * stride;
        int d = 0;
        for (int i = lane * 16; i < N; i += 64 * 16) {
            const uint4 u = *(const uint4*)(x + i);
            const uint4 v = *(const uint4*)(y + i);
            // bytes past N are padding: zero in both rows only if never written, so mask them
            uint32_t w[4] = {u.x ^ v.x, u.y ^ v.y, u.z ^ v.z, u.w ^ v.w};
            const int valid = min(16, N - i);
            for (int k = 0; k < 4; ++k) {
                const int vb = valid - 4 * k;
                const uint32_t m = vb >= 4 ? 0xFFFFFFFFu : (vb <= 0 ? 0u : ((1u << (8 * vb)) - 1u));
                d += __popc(w[k] & m & 0x01010101u);
            }
        }
        for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
        if (lane == 0) {
            if (local) atomicAdd(&hloc[d], 1u);
            else atomicAdd((unsigned long long*)&qh[d], 1ull);
        }
    }
    if (local) {
        __syncthreads();
        for (int d = threadIdx.x; d <= N; d += blockDim.x) {
            const uint32_t c = hloc[d];
            if (c) atomicAdd((unsigned long long*)&qh[d], (unsigned long long)c);
        }
    }
}

// Hamming distances of a 64-replica group g of runs A and B, bit-packed layout, one wave: each lane
// loads a 16-byte piece (E replicas' words of one row) of both runs per row it takes, so a row of
// the group is LPR lanes and a pass RPP rows, adds the popcount of each replica's xor word, and the
// RPP lanes of the same piece then add their counts.  (One lane per replica with a load per row
// word issued 16 times as many narrow loads.)  The distances are counted in hloc (LDS) or qh.
template <typename Wt>
__device__ inline void group_distances(const pa_state* a, const pa_state* b, int64_t g, int n_rows, int64_t P,
                                       bool local, uint32_t* hloc, int64_t* qh)
{
    constexpr int E = 16 / (int)sizeof(Wt);  // replicas per piece
    constexpr int LPR = 64 / E;              // lanes per row
    constexpr int RPP = 64 / LPR;            // rows per pass
    constexpr int PER = 4 / (int)sizeof(Wt);  // replicas per 32-bit word of a piece
    const int lane = (int)(threadIdx.x & 63), rr = lane / LPR, c = lane % LPR;
    const uint4* A = reinterpret_cast<const uint4*>((const Wt*)a->spins[a->cur] + g * n_rows * 64);
    const uint4* B = reinterpret_cast<const uint4*>((const Wt*)b->spins[b->cur] + g * n_rows * 64);
    uint32_t cnt[E];
#pragma unroll
    for (int e = 0; e < E; ++e) cnt[e] = 0;
    for (int row = rr; row < n_rows; row += RPP) {
        const uint4 x = A[row * LPR + c], y = B[row * LPR + c];
        const uint32_t w[4] = {x.x ^ y.x, x.y ^ y.y, x.z ^ y.z, x.w ^ y.w};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t v = w[e / PER] >> (8 * (int)sizeof(Wt) * (e % PER));
            cnt[e] += (uint32_t)__popc(sizeof(Wt) == 4 ? v : v & ((1u << (8 * sizeof(Wt))) - 1u));
        }
    }
#pragma unroll
    for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
        for (int e = 0; e < E; ++e) cnt[e] += (uint32_t)__shfl_xor((int)cnt[e], off, 64);
    if (rr == 0) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t j = g * 64 + c * E + e;
            if (j < P) {
                if (local) atomicAdd(&hloc[cnt[e]], 1u);
                else atomicAdd((unsigned long long*)&qh[cnt[e]], 1ull);
            }
        }
    }
}

// Hamming distance of replica j of runs A and B (pair_xor: B is A's partner run in the batch), a
// wave per 64-replica group, four groups per block.  The block counts its distances in an LDS
// histogram (cap entries, when N + 1 fits) and adds its non-zero bins to the run's histogram: the
// distances of a population sit within a few sqrt(N) of a few values, so one global atomic per
// replica would serialise on a handful of addresses.
constexpr int kOverlapGroups = 4;

__global__ void __launch_bounds__(256) k_overlap_bits(pa_state* base, const pa_state* b_given, int pair_xor, int cap)
{
    extern __shared__ uint32_t hloc[];
    if (pair_xor && (blockIdx.y & 1)) return;  // a pair's distances are counted once, by its first run
    pa_state* a = base + blockIdx.y;
    const pa_state* b = pair_xor ? base + (blockIdx.y ^ 1) : b_given;
    if (a->status || b->status) return;  // the same for the whole block
    const int64_t P = min(a->R, b->R);
    const int N = a->N;
    const int n_rows = a->dim == 1 ? (a->N + 31) / 32 : a->L * a->L;
    const int WB = a->dim == 1 ? 4 : (a->L <= 8 ? 1 : (a->L <= 16 ? 2 : 4));
    int64_t* qh = work_ptr<int64_t>(a, work_layout(a->N, a->n_bins, a->capacity).qhist);
    const int64_t g0 = (int64_t)blockIdx.x * kOverlapGroups;
    if (g0 * 64 >= P) return;  // the same for the whole block
    const bool local = N + 1 <= cap;
    if (local) {
        for (int d = threadIdx.x; d <= N; d += blockDim.x) hloc[d] = 0;
        __syncthreads();
    }
    const int64_t g = g0 + (threadIdx.x >> 6);
    if (g * 64 < P) {  // the same for the whole wave
        if (WB == 1) group_distances<uint8_t>(a, b, g, n_rows, P, local, hloc, qh);
        else if (WB == 2) group_distances<uint16_t>(a, b, g, n_rows, P, local, hloc, qh);
        else group_distances<uint32_t>(a, b, g, n_rows, P, local, hloc, qh);
    }
    if (local) {
        __syncthreads();
        for (int d = threadIdx.x; d <= N; d += blockDim.x) {
            const uint32_t c = hloc[d];
            if (c) atomicAdd((unsigned long long*)&qh[d], (unsigned long long)c);
        }
    }
}

// q^2, q^4, Gamma from the overlap histogram (d ascending), into record[k] of run A (with pair_xor,
// both runs of a pair read the histogram of its first run)
// one block per run: strided partial sums over the overlap histogram, then a fixed-order tree
// reduction (P and the Gamma count are integers and exact; q2 and q4 differ from a serial sum only
// in rounding order)
__global__ void __launch_bounds__(256) k_overlap_stats(pa_state* base, const pa_state* b_given, int pair_xor)
{
    pa_state* a = base + blockIdx.y;
    const pa_state* b = pair_xor ? base + (blockIdx.y ^ 1) : b_given;
    if (a->status || b->status) return;
    __shared__ double red[4][256];
    const pa_state* h = pair_xor && (blockIdx.y & 1) ? b : a;
    const int64_t* qh = work_ptr<int64_t>(h, work_layout(h->N, h->n_bins, h->capacity).qhist);
    const int N = a->N;
    double P = 0.0, q2 = 0.0, q4 = 0.0, g = 0.0;
    for (int d = threadIdx.x; d <= N; d += blockDim.x) {
        const double c = (double)qh[d];
        const double q = (double)(N - 2 * d) / (double)N;
        P += c;
        q2 += c * q * q;
        q4 += c * q * q * q * q;
        if (fabs(q) < 0.2) g += c;
    }
    red[0][threadIdx.x] = P;
    red[1][threadIdx.x] = q2;
    red[2][threadIdx.x] = q4;
    red[3][threadIdx.x] = g;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int v = 0; v < 4; ++v) red[v][threadIdx.x] += red[v][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pa_record* rec = a->record + a->k;
        rec->q2 = red[1][0] / red[0][0];
        rec->q4 = red[2][0] / red[0][0];
        rec->gamma = red[3][0] / red[0][0];
        rec->n_pairs = red[0][0];
    }
}

__global__ void k_free_energy(const pa_state* __restrict__ base, int n, double* out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) out[r] = base[r].ln_omega + base[r].acc;
}

// n runs with contiguous states (grid.y = run); partner: NULL, or the partner of a single run
// (n = 1), or pair_xor: run r paired with run r ^ 1 of the same call
int launch_measure(const pa_run* runs, int n, const pa_run* partner, int pair_xor, hipStream_t s)
{
    int rc = launch_hist(runs, n, s);
    if (rc != PA_OK) return rc;
    pa_state* base = runs[0].state;
    hipLaunchKernelGGL(k_moments, dim3(1, n), dim3(64), 0, s, base);
    if (partner || pair_xor) {
        int64_t N = 0, P = 0;
        for (int r = 0; r < n; ++r) {
            N = std::max<int64_t>(N, runs[r].dim == 1 ? runs[r].L : (int64_t)runs[r].L * runs[r].L * runs[r].L);
            P = std::max<int64_t>(P, runs[r].capacity);
        }
        const pa_state* bg = partner ? partner->state : nullptr;
        hipLaunchKernelGGL(k_qhist_clear, dim3((unsigned)((N + 256) / 256), n), dim3(256), 0, s, base);
        // the partner's population must be final before it is read: both runs on the same stream,
        // or the partner's stream joined by the caller
        // LDS histogram of up to 8192 bins (every cube; longer chains count in global memory)
        const int cap = N + 1 <= 8192 ? (int)(N + 1) : 0;
        if (runs[0].layout == PA_U8) {
            const int64_t per_block = 4 * kOverlapU8Items;
            hipLaunchKernelGGL(k_overlap_u8, dim3((unsigned)((P + per_block - 1) / per_block), n), dim3(256),
                               (size_t)cap * 4, s, base, bg, pair_xor, cap);
        } else {
            const int64_t per_block = 64 * kOverlapGroups;
            hipLaunchKernelGGL(k_overlap_bits, dim3((unsigned)((P + per_block - 1) / per_block), n), dim3(256),
                               (size_t)cap * 4, s, base, bg, pair_xor, cap);
        }
        hipLaunchKernelGGL(k_overlap_stats, dim3(1, n), dim3(256), 0, s, base, bg, pair_xor);
    }
    return hip_status(hipGetLastError());
}

// Gaussian couplings: energy moments from the FP64 energies, overlap as for one byte per spin;
// runs as for launch_measure (consecutive states when n > 1)
int launch_measure_gauss(const pa_run* runs, int n, const pa_run* partner, int pair_xor, hipStream_t s)
{
    int rc = launch_moments_gauss(runs, n, s);
    if (rc != PA_OK || !(partner || pair_xor)) return rc;
    int64_t N = 0, P = 0;
    for (int r = 0; r < n; ++r) {
        N = std::max<int64_t>(N, runs[r].dim == 1 ? runs[r].L : (int64_t)runs[r].L * runs[r].L * runs[r].L);
        P = std::max<int64_t>(P, runs[r].capacity);
    }
    pa_state* base = runs[0].state;
    const pa_state* bg = partner ? partner->state : nullptr;
    hipLaunchKernelGGL(k_qhist_clear, dim3((unsigned)((N + 256) / 256), n), dim3(256), 0, s, base);
    const int cap = N + 1 <= 8192 ? (int)(N + 1) : 0;
    const int64_t per_block = 4 * kOverlapU8Items;
    hipLaunchKernelGGL(k_overlap_u8, dim3((unsigned)((P + per_block - 1) / per_block), n), dim3(256),
                       (size_t)cap * 4, s, base, bg, pair_xor, cap);
    hipLaunchKernelGGL(k_overlap_stats, dim3(1, n), dim3(256), 0, s, base, bg, pair_xor);
    return hip_status(hipGetLastError());
}

int launch_free_energy(const pa_run* runs, int n, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_free_energy, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, (const pa_state*)runs[0].state,
                       n, out);
    return hip_status(hipGetLastError());
}

// weighted average of one set of M runs (Sec. III), optionally through a row of resampled run
// indices; same arithmetic order as the host version.  o[0..n_obs-1] = A_bar, o[n_obs] =
// -beta F_bar, o[n_obs+1] = Var, o[n_obs+2] = mean.
__device__ void weighted_one(int M, const double* __restrict__ xs, const double* __restrict__ Rs,
                             const double* __restrict__ As, int n_obs, const int32_t* __restrict__ pick,
                             double* __restrict__ o)
{
    double xmax = -INFINITY;
    for (int i = 0; i < M; ++i) {
        const int r = pick ? pick[i] : i;
        const double xr = xs[r] + (Rs ? log(Rs[r]) : 0.0);
        if (xr > xmax) xmax = xr;
    }
    double Z = 0.0, Rsum = 0.0;
    for (int i = 0; i < M; ++i) {
        const int r = pick ? pick[i] : i;
        Z += exp(xs[r] + (Rs ? log(Rs[r]) : 0.0) - xmax);
        Rsum += Rs ? Rs[r] : 1.0;
    }
    for (int k = 0; k < n_obs; ++k) o[k] = 0.0;
    for (int i = 0; i < M; ++i) {
        const int r = pick ? pick[i] : i;
        const double w = exp(xs[r] + (Rs ? log(Rs[r]) : 0.0) - xmax) / Z;
        for (int k = 0; k < n_obs; ++k) o[k] += w * As[(int64_t)r * n_obs + k];
    }
    o[n_obs] = xmax + log(Z) - log(Rsum);
    double m = 0.0;
    for (int i = 0; i < M; ++i) m += xs[pick ? pick[i] : i];
    m /= (double)M;
    double v = 0.0;
    for (int i = 0; i < M; ++i) {
        const double d = xs[pick ? pick[i] : i] - m;
        v += d * d;
    }
    o[n_obs + 1] = M > 1 ? v / (double)(M - 1) : 0.0;
    o[n_obs + 2] = m;
}

// one thread per set
__global__ void k_weighted_average(int n_sets, int M, const double* __restrict__ x, const double* __restrict__ R,
                                   const double* __restrict__ A, int n_obs, double* __restrict__ out)
{
    const int set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets) return;
    weighted_one(M, x + (int64_t)set * M, R ? R + (int64_t)set * M : nullptr, A + (int64_t)set * M * n_obs, n_obs,
                 nullptr, out + (int64_t)set * (n_obs + 3));
}

int launch_weighted_average_dev(int n_sets, int M, const double* x, const double* R, const double* A, int n_obs,
                                double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_weighted_average, dim3((unsigned)((n_sets + 63) / 64)), dim3(64), 0, s, n_sets, M, x, R, A,
                       n_obs, out);
    return hip_status(hipGetLastError());
}

// Overlap observables over pairs of runs (Sec. IV, eqs. pqs and omegaprime), one thread per set:
// pair p joins runs 2p and 2p + 1 and weighs exp(x^(1) + x^(2)) (times R^(1) R^(2) when R is
// given, Sec. III); Q holds each pair's (<q^2>, <q^4>, Gamma).  The weighted moments give the
// Binder ratio g = (3 - [q^4] / [q^2]^2) / 2.  o = ([q^2], [q^4], [Gamma], g).
__global__ void k_overlap_average(int n_sets, int n_pairs, const double* __restrict__ x, const double* __restrict__ R,
                                  const double* __restrict__ Q, double* __restrict__ out)
{
    const int set = blockIdx.x * blockDim.x + threadIdx.x;
    if (set >= n_sets) return;
    const double* xs = x + (int64_t)set * 2 * n_pairs;
    const double* Rs = R ? R + (int64_t)set * 2 * n_pairs : nullptr;
    const double* Qs = Q + (int64_t)set * n_pairs * 3;
    // exponent of pair p: x^(1) + x^(2) (+ ln(R^(1) R^(2)))
    auto xpair = [&](int p) {
        const double xp = xs[2 * p] + xs[2 * p + 1];
        return xp + (Rs ? log(Rs[2 * p] * Rs[2 * p + 1]) : 0.0);
    };
    double xmax = -INFINITY;
    for (int p = 0; p < n_pairs; ++p) xmax = fmax(xmax, xpair(p));
    double Z = 0.0;
    for (int p = 0; p < n_pairs; ++p) Z += exp(xpair(p) - xmax);
    double o[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < n_pairs; ++p) {
        const double w = exp(xpair(p) - xmax) / Z;
        for (int k = 0; k < 3; ++k) o[k] += w * Qs[3 * p + k];
    }
    double* os = out + (int64_t)set * 4;
    os[0] = o[0];
    os[1] = o[1];
    os[2] = o[2];
    os[3] = 0.5 * (3.0 - o[1] / (o[0] * o[0]));
}

int launch_overlap_average_dev(int n_sets, int n_pairs, const double* x, const double* R, const double* Q,
                               double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_overlap_average, dim3((unsigned)((n_sets + 63) / 64)), dim3(64), 0, s, n_sets, n_pairs, x, R,
                       Q, out);
    return hip_status(hipGetLastError());
}

// bootstrap replicates: thread per (set, replicate b), the weighted average of the runs idx[b][.]
__global__ void k_bootstrap(int n_sets, int M, const double* __restrict__ x, const double* __restrict__ R,
                            const double* __restrict__ A, int n_obs, int n_boot, const int32_t* __restrict__ idx,
                            double* __restrict__ rep)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n_sets * n_boot) return;
    const int set = (int)(t / n_boot), b = (int)(t % n_boot);
    const int32_t* pick = idx + (int64_t)b * M;
    for (int i = 0; i < M; ++i) {
        if ((uint32_t)pick[i] >= (uint32_t)M) {  // an index outside the set: no read, NaN results
            for (int q = 0; q < n_obs + 3; ++q) rep[t * (n_obs + 3) + q] = NAN;
            return;
        }
    }
    weighted_one(M, x + (int64_t)set * M, R ? R + (int64_t)set * M : nullptr, A + (int64_t)set * M * n_obs, n_obs,
                 pick, rep + t * (n_obs + 3));
}

// error of each quantity: standard deviation over the replicates (1 / (n_boot - 1)), in order
__global__ void k_bootstrap_err(int n_sets, int n_obs, int n_boot, const double* __restrict__ rep,
                                double* __restrict__ err)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nq = n_obs + 3;
    if (t >= (int64_t)n_sets * nq) return;
    const int set = (int)(t / nq), q = (int)(t % nq);
    const double* r = rep + (int64_t)set * n_boot * nq + q;
    double m = 0.0;
    for (int b = 0; b < n_boot; ++b) m += r[(int64_t)b * nq];
    m /= (double)n_boot;
    double v = 0.0;
    for (int b = 0; b < n_boot; ++b) {
        const double d = r[(int64_t)b * nq] - m;
        v += d * d;
    }
    err[t] = n_boot > 1 ? sqrt(v / (double)(n_boot - 1)) : 0.0;
}

int launch_bootstrap_dev(int n_sets, int M, const double* x, const double* R, const double* A, int n_obs, int n_boot,
                         const int32_t* idx, double* rep, double* err, hipStream_t s)
{
    const int64_t nr = (int64_t)n_sets * n_boot, ne = (int64_t)n_sets * (n_obs + 3);
    hipLaunchKernelGGL(k_bootstrap, dim3((unsigned)((nr + 63) / 64)), dim3(64), 0, s, n_sets, M, x, R, A, n_obs, n_boot,
                       idx, rep);
    hipLaunchKernelGGL(k_bootstrap_err, dim3((unsigned)((ne + 63) / 64)), dim3(64), 0, s, n_sets, n_obs, n_boot,
                       (const double*)rep, err);
    return hip_status(hipGetLastError());
}

}  // namespace pa
