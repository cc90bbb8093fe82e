// Resampling between temperatures (Sec. II, eqs. Q and wn; Poisson copy numbers with mean
// (R_target / R~) tau_j; the new population of R~' replicas).
//
// Chain of kernels on the run's stream, all sized by capacity and reading the population size
// from the device, with no host synchronisation:
//   hist      energy histogram h (width-4 bins from E_base), E_lo, E_hi      (integer atomics)
//   normalise S = sum_E h(E) w(E - E_lo) in ascending E (FP64, one thread, fixed order),
//             ln Q, and per bin the mean copy number lambda = R_target w / S split into
//             Poisson(64) blocks q, ladder level m and thinning threshold
//   copies    Poisson(lambda) per replica from its Philox stream (integer compares only)
//   scan      exclusive scan of the copy numbers -> offsets, R~', capacity/extinction flags
//   src       source replica of every new replica (binary search of the offsets)
//   gather    copy spins and energies into the other buffer
//   finish    swap buffers, R~ = R~', accumulate ln Q, record
// Every kernel is a no-op once the run's sticky status is set.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "pa_common.h"

#pragma clang fp contract(off)

namespace pa {

// Poisson(2^m) inversion tables, m = kLadderMin .. kLadderMax (host-built, uploaded once)
__device__ uint64_t g_ladder[kLadderLevels][kLadderCap];

// int64 slots of the misc area: E_lo and E_hi of the population being resampled (FP64 bits of E_lo
// with Gaussian couplings), then ln Q and S of the step (FP64 bits), kept there until k_finish
// commits the step to the run's state and record
constexpr int kMiscEmin = 0, kMiscEmax = 1, kMiscLnQ = 2, kMiscS = 3;

// ------------------------------------------------------------------ host tables
// C[n] = floor(CDF_{2^m}(n) 2^32) with pmf recursion p_0 = exp(-Lambda), p_n = p_{n-1} Lambda / n;
// the table ends at the first n >= Lambda with p_n < 2^-40, that entry forced to 2^32.
static int ladder_host(int m, uint64_t* C, int cap)
{
    const double Lam = ldexp(1.0, m);
    double p = exp(-Lam);
    double F = 0.0;
    const double tail = ldexp(1.0, -40);
    int n = 0;
    for (;;) {
        F += p;
        if ((double)n >= Lam && p < tail) {
            C[n] = (uint64_t)1 << 32;
            return n + 1;
        }
        const double c = floor(ldexp(F, 32));
        C[n] = c >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)c;
        ++n;
        p = p * Lam / (double)n;
        if (n >= cap - 1) {
            C[n] = (uint64_t)1 << 32;
            return n + 1;
        }
    }
}

static uint64_t g_ladder_host[kLadderLevels][kLadderCap];
static bool g_ladder_built = false;
static int g_ladder_device_mask = 0;  // devices that hold the table

int upload_ladder(hipStream_t s)
{
    if (!g_ladder_built) {
        for (int m = kLadderMin; m <= kLadderMax; ++m) {
            uint64_t* C = g_ladder_host[m - kLadderMin];
            const int n = ladder_host(m, C, kLadderCap);
            for (int k = n; k < kLadderCap; ++k) C[k] = (uint64_t)1 << 32;
        }
        g_ladder_built = true;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PA_ERR_HIP;
    if (dev < 31 && (g_ladder_device_mask >> dev) & 1) return PA_OK;
    if (hipMemcpyToSymbolAsync(HIP_SYMBOL(g_ladder), g_ladder_host, sizeof(g_ladder_host), 0,
                               hipMemcpyHostToDevice, s) != hipSuccess)
        return PA_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PA_ERR_HIP;
    if (dev < 31) g_ladder_device_mask |= 1 << dev;
    return PA_OK;
}

// ------------------------------------------------------------------ kernels
__global__ void k_hist_clear(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    int64_t* hist = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).hist);
    int64_t* misc = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).misc);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < st->n_bins; i += gridDim.x * blockDim.x) hist[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        misc[kMiscEmin] = INT32_MAX;
        misc[kMiscEmax] = INT32_MIN;
    }
}

constexpr int kHistLoads = 8;

// histogram of the current population's energies, counted in an LDS copy of cap_bins entries
// when the run's bins fit there (the LDS is sized for the call, whose runs may differ in size),
// else directly in global memory
__global__ void __launch_bounds__(256) k_hist(pa_state* base, int cap_bins)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    extern __shared__ uint32_t sh[];
    const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
    int64_t* hist = work_ptr<int64_t>(st, wl.hist);
    int64_t* misc = work_ptr<int64_t>(st, wl.misc);
    const int nb = st->n_bins;
    const bool priv = nb <= cap_bins;
    const int64_t R = st->R;
    // a run takes only the blocks its energies fill (kHistLoads per thread): in a batch, a small
    // run left the rest to clear, scan and merge a histogram each for a few energies
    const int64_t per_block = (int64_t)blockDim.x * kHistLoads;
    const int nblk = (int)min((int64_t)gridDim.x, (R + per_block - 1) / per_block);
    if ((int)blockIdx.x >= nblk) return;  // the same for the whole block
    const int32_t* E = st->energy[st->cur];
    const int Eb = st->E_base;
    if (priv)
        for (int i = threadIdx.x; i < nb; i += blockDim.x) sh[i] = 0;
    __syncthreads();
    int emin = INT32_MAX, emax = INT32_MIN;
    // kHistLoads energies per thread are loaded before any of them is counted, so that many loads
    // are in flight at once (a load and its count in turn wait out the memory latency each time)
    const int64_t stride = (int64_t)nblk * blockDim.x;
    for (int64_t j0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j0 < R; j0 += kHistLoads * stride) {
        int e[kHistLoads];
#pragma unroll
        for (int u = 0; u < kHistLoads; ++u) e[u] = j0 + u * stride < R ? E[j0 + u * stride] : 0;
#pragma unroll
        for (int u = 0; u < kHistLoads; ++u) {
            if (j0 + u * stride >= R) break;
            const int b = (e[u] - Eb) >> 2;
            if (priv) atomicAdd(&sh[b], 1u);
            else atomicAdd((unsigned long long*)&hist[b], 1ull);
            emin = min(emin, e[u]);
            emax = max(emax, e[u]);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        emin = min(emin, __shfl_xor(emin, off, 64));
        emax = max(emax, __shfl_xor(emax, off, 64));
    }
    if ((threadIdx.x & 63) == 0 && emin <= emax) {
        atomicMin((long long*)&misc[kMiscEmin], (long long)emin);
        atomicMax((long long*)&misc[kMiscEmax], (long long)emax);
    }
    __syncthreads();
    if (priv)
        for (int i = threadIdx.x; i < nb; i += blockDim.x)
            if (sh[i]) atomicAdd((unsigned long long*)&hist[i], (unsigned long long)sh[i]);
}

struct ResampleParams {
    double beta_from, beta_to, R_target;
    const double* w;
    int32_t k;
};

// smallest m in [kLadderMin, kLadderMax] with 2^m >= x (0 < x <= 64)
__device__ inline int ladder_level(double x)
{
    int e;
    const double f = frexp(x, &e);
    const int m = (f == 0.5) ? e - 1 : e;
    return m < kLadderMin ? kLadderMin : m;
}

// one block: S in ascending energy order, ln Q, per-bin Poisson parameters (the step's record is
// written by k_finish, once the new population is known to fit)
__global__ void __launch_bounds__(256) k_normalise(pa_state* base, ResampleParams p)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    __shared__ double prod[1024];
    __shared__ double S_sh;
    const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
    const int64_t* hist = work_ptr<int64_t>(st, wl.hist);
    int64_t* misc = work_ptr<int64_t>(st, wl.misc);
    int64_t* bin_q = work_ptr<int64_t>(st, wl.bin_q);
    uint64_t* bin_keep = work_ptr<uint64_t>(st, wl.bin_keep);
    int32_t* bin_m = work_ptr<int32_t>(st, wl.bin_m);
    const int E_lo = (int)misc[kMiscEmin], E_hi = (int)misc[kMiscEmax];
    const int ilo = (E_lo - st->E_base) >> 2, ihi = (E_hi - st->E_base) >> 2;
    const int n = ihi - ilo + 1;
    const double dbeta = p.beta_to - p.beta_from;
    // S = sum_i h_i w_i, i ascending; products in parallel (each rounded once), sum by one thread
    double S = 0.0;
    for (int b0 = 0; b0 < n; b0 += 1024) {
        const int cnt = min(1024, n - b0);
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) prod[t] = (double)hist[ilo + b0 + t] * p.w[b0 + t];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int t = 0; t < cnt; ++t) S = S + prod[t];
        __syncthreads();
    }
    if (threadIdx.x == 0) S_sh = S;
    __syncthreads();
    S = S_sh;
    const double R = (double)st->R;
    const double Rt = p.R_target > 0.0 ? p.R_target : (double)st->R0;
    const bool bad = !isfinite(S) || !(S > 0.0);
    if (threadIdx.x == 0) {
        const double lnQ = -dbeta * (double)E_lo + log(S) - log(R);
        if (bad) {
            st->status |= PA_FLAG_NONFINITE;
        } else {
            *reinterpret_cast<double*>(&misc[kMiscLnQ]) = lnQ;
            *reinterpret_cast<double*>(&misc[kMiscS]) = S;
            st->E_lo = E_lo;
            st->E_hi = E_hi;
        }
    }
    if (bad) return;
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        const double lam = (Rt * p.w[t]) / S;
        const int b = ilo + t;
        if (!(lam > 0.0)) {
            bin_q[b] = 0;
            bin_m[b] = 1000;  // no draws: copy number 0
            bin_keep[b] = 0;
            continue;
        }
        int64_t q = 0;
        double rem = lam;
        if (lam > 64.0) {
            q = (int64_t)ceil(lam / 64.0) - 1;
            rem = lam - 64.0 * (double)q;
        }
        const int m = ladder_level(rem);
        bin_q[b] = q;
        bin_m[b] = m;
        bin_keep[b] = (uint64_t)floor(ldexp(rem, 32 - m));
    }
}

// the smallest n with u < C[n] (C non-decreasing, its last entries 2^32 > u).  Small means walk
// the table from 0 (a few steps); from 2^3 on, a branch-free binary search: n counts the entries
// <= u, eight dependent loads instead of about 2^m (a Poisson(64) block took ~64)
__device__ inline int64_t invert_ladder(int m, uint32_t u)
{
    const uint64_t* C = g_ladder[m - kLadderMin];
    if (m < 3) {
        int64_t n = 0;
        while (!((uint64_t)u < C[n])) ++n;
        return n;
    }
    static_assert(kLadderCap == 256, "binary search over 256 entries");
    int n = 0;
#pragma unroll
    for (int step = 128; step > 0; step >>= 1)
        if (C[n + step - 1] <= (uint64_t)u) n += step;
    return n;
}

// Copy numbers: replica j's Poisson(lambda_j) count at step k is the sum of q Poisson(64) blocks and
// a Poisson(2^m) count K thinned by K draws against keep = rem 2^(32 - m).  Draw d (blocks d = 0 ..
// q - 1, K at d = q, the thinning draws at d = q + 1 ..) is word d mod 4 of Philox(d / 4, j, k, 4).
// Light lanes (no blocks, 2^m < 16) draw in turn; the wave takes each heavy lane's draws
// together, spread over its 64 lanes (the draws are counter-based, so any lane can make any of
// them, and the count is an integer sum), instead of waiting for one lane to make them one by one.
constexpr int kCopiesHeavyM = 4;

struct CopyDraws {
    uint32_t j, k, k0, k1;
    __device__ uint32_t at(uint32_t d) const
    {
        return word_of(philox10(d >> 2, j, k, kTagPoisson, k0, k1), (int)(d & 3));
    }
};

__device__ inline int64_t copies_light(const CopyDraws& cd, int m, uint64_t keep)
{
    uint32_t d = 0;
    uint4v v = {0, 0, 0, 0};
    auto draw = [&]() -> uint32_t {
        if ((d & 3) == 0) v = philox10(d >> 2, cd.j, cd.k, kTagPoisson, cd.k0, cd.k1);
        const uint32_t u = word_of(v, d & 3);
        ++d;
        return u;
    };
    const int64_t K = invert_ladder(m, draw());
    int64_t n = 0;
    for (int64_t e = 0; e < K; ++e)
        if ((uint64_t)draw() < keep) ++n;
    return n;
}

// every lane of the wave calls this (lanes without a replica with heavy = false); returns the
// count of a heavy lane's replica, n unchanged elsewhere
__device__ inline int64_t copies_heavy_by_wave(bool heavy, int64_t n, const CopyDraws& mine, int m, int64_t q,
                                               uint64_t keep)
{
    const int lane = (int)(threadIdx.x & 63);
    uint64_t todo = __ballot(heavy);
    while (todo) {
        const int h = __builtin_ctzll(todo);
        todo &= todo - 1;
        CopyDraws cd = mine;
        cd.j = (uint32_t)__shfl((int)mine.j, h, 64);
        const int mh = __shfl(m, h, 64);
        const int64_t qh = __shfl(q, h, 64);
        const uint64_t keeph = (uint64_t)__shfl((int64_t)keep, h, 64);
        int64_t part = 0;
        for (int64_t blk = lane; blk < qh; blk += 64) part += invert_ladder(kLadderMax, cd.at((uint32_t)blk));
        const int64_t K = invert_ladder(mh, cd.at((uint32_t)qh));
        for (int64_t e = lane; e < K; e += 64)
            if ((uint64_t)cd.at((uint32_t)(qh + 1 + e)) < keeph) ++part;
        for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
        if (lane == h) n = part;
    }
    return n;
}

__global__ void __launch_bounds__(256) k_copies(pa_state* base, int32_t k)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t R = st->R;
    if (j - (int64_t)(threadIdx.x & 63) >= R) return;  // the whole wave past R
    const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
    const int64_t* bin_q = work_ptr<int64_t>(st, wl.bin_q);
    const uint64_t* bin_keep = work_ptr<uint64_t>(st, wl.bin_keep);
    const int32_t* bin_m = work_ptr<int32_t>(st, wl.bin_m);
    const bool live = j < R;
    int m = 1000;  // bins of zero weight carry m = 1000: no copies
    int64_t q = 0;
    uint64_t keep = 0;
    if (live) {
        const int b = (st->energy[st->cur][j] - st->E_base) >> 2;
        m = bin_m[b];
        if (m != 1000) {
            q = bin_q[b];
            keep = bin_keep[b];
        }
    }
    const CopyDraws cd = {(uint32_t)j, (uint32_t)k, (uint32_t)st->seed, (uint32_t)(st->seed >> 32)};
    const bool drawn = live && m != 1000;
    const bool heavy = drawn && (q > 0 || m >= kCopiesHeavyM);
    int64_t n = drawn && !heavy ? copies_light(cd, m, keep) : 0;
    n = copies_heavy_by_wave(heavy, n, cd, m, q, keep);
    if (live) st->counts[j] = (int32_t)min(n, (int64_t)INT32_MAX);
}

// block sums of the copy numbers over tiles of kScanTile replicas
__global__ void __launch_bounds__(256) k_scan_reduce(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    if ((int64_t)blockIdx.x * kScanTile >= st->capacity) return;  // grid sized for the largest run
    __shared__ int64_t part[4];
    const int64_t R = st->R;
    const int64_t tile0 = (int64_t)blockIdx.x * kScanTile;
    int64_t acc = 0;
    for (int t = threadIdx.x; t < kScanTile; t += blockDim.x)
        if (tile0 + t < R) acc += st->counts[tile0 + t];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t* scan = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).scan);
        scan[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
    }
}

// exclusive scan of the block sums (one block), total R~', capacity and extinction checks
__global__ void __launch_bounds__(256) k_scan_top(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    const int n_blocks = (int)((st->capacity + kScanTile - 1) / kScanTile);
    if (st->status) return;
    __shared__ int64_t carry_sh;
    __shared__ int64_t wsum[4];
    int64_t* scan = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).scan);
    if (threadIdx.x == 0) carry_sh = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i0 = 0; i0 < n_blocks; i0 += 256) {
        const int i = i0 + threadIdx.x;
        const int64_t v = i < n_blocks ? scan[i] : 0;
        int64_t x = v;  // inclusive wave scan
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int64_t pre = carry_sh;
        for (int w = 0; w < wv; ++w) pre += wsum[w];
        if (i < n_blocks) scan[i] = pre + x - v;
        __syncthreads();
        if (threadIdx.x == 255) carry_sh = pre + x;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t total = carry_sh;
        st->R_new = total;
        if (total > st->capacity) st->status |= PA_FLAG_CAPACITY;
        else if (total == 0) st->status |= PA_FLAG_EXTINCT;
    }
}

// offsets[j] = scan[tile] + exclusive scan inside the tile; offsets[R] = R~'
__global__ void __launch_bounds__(256) k_scan_down(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    __shared__ int64_t wsum[4];
    __shared__ int64_t carry_sh;
    const int64_t R = st->R;
    const int64_t tile0 = (int64_t)blockIdx.x * kScanTile;
    if (tile0 >= R) return;
    const int64_t* scan = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).scan);
    if (threadIdx.x == 0) carry_sh = scan[blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int t0 = 0; t0 < kScanTile; t0 += 256) {
        const int64_t j = tile0 + t0 + threadIdx.x;
        const int64_t v = j < R ? st->counts[j] : 0;
        int64_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int64_t pre = carry_sh;
        for (int w = 0; w < wv; ++w) pre += wsum[w];
        if (j < R) st->offsets[j] = pre + x - v;
        __syncthreads();
        if (threadIdx.x == 255) carry_sh = pre + x;
        __syncthreads();
    }
    if (tile0 + kScanTile >= R && threadIdx.x == 0) st->offsets[R] = st->R_new;
}

// source replica of each new replica, a block per 256 consecutive sources: their offsets go to LDS,
// and the block's new replicas offsets[j0] .. offsets[j0 + 256] - 1 each find their source there
// (largest j with offsets[j] <= r', 8 LDS steps) and are written in order.  Per new replica over
// the whole array, the same search took ~20 dependent global loads; per source, the writes of
// uneven copy numbers were scattered and slower still.
__global__ void __launch_bounds__(256) k_src(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const int64_t R = st->R;
    const int64_t j0 = (int64_t)blockIdx.x * 256;
    if (j0 >= R) return;
    const int n = (int)(R - j0 < 256 ? R - j0 : 256);
    __shared__ int64_t off[257];
    for (int i = threadIdx.x; i <= n; i += 256) off[i] = st->offsets[j0 + i];  // offsets[R] = R~'
    __syncthreads();
    const int64_t A = off[0], B = off[n];
    int32_t* src = work_ptr<int32_t>(st, work_layout(st->N, st->n_bins, st->capacity).src);
    for (int64_t d = A + threadIdx.x; d < B; d += 256) {
        int lo = 0, hi = n;  // off[lo] <= d < off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (off[mid] <= d) lo = mid;
            else hi = mid;
        }
        src[d] = (int32_t)(j0 + lo);
    }
}

// u8 gather: one thread per 16 bytes of a destination row
__global__ void __launch_bounds__(256) k_gather_u8(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const int per_row = st->row_stride / 16;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rn = t / per_row;
    const int c = (int)(t - rn * per_row);
    if (rn >= st->R_new) return;
    const int32_t* src = work_ptr<int32_t>(st, work_layout(st->N, st->n_bins, st->capacity).src);
    const int64_t j = src[rn];
    const int cur = st->cur;
    const uint4* a = (const uint4*)((const uint8_t*)st->spins[cur] + j * st->row_stride) + c;
    uint4* b = (uint4*)((uint8_t*)st->spins[cur ^ 1] + rn * st->row_stride) + c;
    *b = *a;
    if (c == 0) {
        if (st->couplings == PA_GAUSS)
            reinterpret_cast<double*>(st->energy[cur ^ 1])[rn] = reinterpret_cast<const double*>(st->energy[cur])[j];
        else
            st->energy[cur ^ 1][rn] = st->energy[cur][j];
    }
}

// bit-packed gather of one replica: loop over rows; a row word of replica j sits at
// (j/64 * n_rows + rho) * 64 + j mod 64 (row words of 1, 2 or 4 bytes by lattice size)
// (16 loads in flight per lane: one dependent load-store pair per row leaves the copy latency-
// bound, a few hundred bytes in flight per wave against the microseconds of HBM latency)
template <typename Wt>
__device__ inline void gather_rows(const pa_state* st, int64_t j, int64_t rn, int n_rows)
{
    constexpr int U = 16;
    const int cur = st->cur;
    const Wt* a = (const Wt*)st->spins[cur] + ((j >> 6) * n_rows) * 64 + (j & 63);
    Wt* b = (Wt*)st->spins[cur ^ 1] + ((rn >> 6) * n_rows) * 64 + (rn & 63);
    int rho = 0;
    for (; rho + U <= n_rows; rho += U) {
        Wt v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = a[(int64_t)(rho + u) * 64];
#pragma unroll
        for (int u = 0; u < U; ++u) b[(int64_t)(rho + u) * 64] = v[u];
    }
    for (; rho < n_rows; ++rho) b[(int64_t)rho * 64] = a[(int64_t)rho * 64];
}


// commit an accepted step: swap the buffers, accumulate ln Q (eq. sumQ) and write record[k]; a step
// refused by a sticky flag leaves state and records as they were
__global__ void k_finish(pa_state* base, ResampleParams p)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
    const int64_t* misc = work_ptr<int64_t>(st, wl.misc);
    const double lnQ = *reinterpret_cast<const double*>(&misc[kMiscLnQ]);
    const double E_lo = st->couplings == PA_GAUSS ? *reinterpret_cast<const double*>(&misc[kMiscEmin])
                                                  : (double)misc[kMiscEmin];
    pa_record* rec = st->record + p.k;
    rec->beta = p.beta_to;
    rec->lnQ = lnQ;
    rec->minus_betaF = st->ln_omega + (st->acc + lnQ);
    rec->S = *reinterpret_cast<const double*>(&misc[kMiscS]);
    rec->R = (double)st->R_new;
    rec->E_lo = E_lo;
    st->acc = st->acc + lnQ;
    st->cur ^= 1;
    st->R = st->R_new;
    st->k = p.k;
    st->beta = p.beta_to;
}

// Launch shapes cover the largest run of the call; grid.y indexes the runs, whose states
// are contiguous (state r at runs[0].state + r).  A single run is n = 1.
struct BatchShape {
    int64_t cap_max = 0, bins_max = 0, stride_max = 0;
};

static BatchShape batch_shape(const pa_run* runs, int n)
{
    BatchShape b;
    for (int r = 0; r < n; ++r) {
        pa_sizes sz;
        pa_buffer_sizes(runs[r].dim, runs[r].L, runs[r].layout, runs[r].couplings, runs[r].capacity, runs[r].n_records, &sz);
        b.cap_max = std::max(b.cap_max, runs[r].capacity);
        b.bins_max = std::max(b.bins_max, sz.n_bins);
        b.stride_max = std::max(b.stride_max, sz.row_stride);
    }
    return b;
}

int launch_hist(const pa_run* runs, int n, hipStream_t s)
{
    const BatchShape b = batch_shape(runs, n);
    // an LDS histogram of up to 16384 bins, sized for the largest run of the call that fits (runs
    // with more bins count in global memory)
    int64_t cap_bins = 0;
    for (int r = 0; r < n; ++r) {
        pa_sizes sz;
        pa_buffer_sizes(runs[r].dim, runs[r].L, runs[r].layout, runs[r].couplings, runs[r].capacity, runs[r].n_records, &sz);
        if (sz.n_bins <= 16384) cap_bins = std::max(cap_bins, sz.n_bins);
    }
    const size_t hist_lds = (size_t)cap_bins * 4;
    // few blocks: each block zeroes and scans all bins of its LDS histogram and merges the occupied
    // ones with global atomics that land on the same few bins (L = 16, 1e6 replicas: 1024 blocks
    // 98 us, 256 blocks 29 us, 128 blocks 21 us; with eight loads in flight per thread, 128 blocks
    // 17.5 us, 256 blocks 28 us, and 64, 32, 16 blocks were slower already before)
    const unsigned hist_blocks = (unsigned)std::min<int64_t>(128, (b.cap_max + 255) / 256);
    hipLaunchKernelGGL(k_hist_clear, dim3(32, n), dim3(256), 0, s, runs[0].state);
    hipLaunchKernelGGL(k_hist, dim3(hist_blocks, n), dim3(256), hist_lds, s, runs[0].state, (int)cap_bins);
    return PA_OK;
}

// Bit-packed gather, a block of kStageThreads consecutive destination replicas at a time.  The
// sources of consecutive destinations are non-decreasing, so the block's sources lie in a few
// consecutive source groups; row by row (kStageRows rows per pass) the block stages those groups'
// whole rows in LDS with 16-byte loads and each thread then takes its replica's word from LDS into
// the destination row.  A source row is read from HBM once per block instead of once per
// destination group that needs it (a group's sources straddle two source groups about a third of
// the time).  A block whose sources span more than kStageGroups groups (large copy numbers next to
// long runs of zeros) gathers per replica with gather_rows.
constexpr int kStageThreads = 512;  // destination replicas per block (eight bit-packed groups)
constexpr int kStageGroups = 16;
constexpr int kStageRows = 8;

template <typename Wt>
__device__ __forceinline__ void gather_staged(pa_state* st, uint4* stage)
{
    constexpr int LPL = 64 * (int)sizeof(Wt) / 16;  // 16-byte pieces of a 64-replica row
    const int64_t R_new = st->R_new;
    const int64_t d0 = (int64_t)blockIdx.x * kStageThreads;
    if (d0 >= R_new) return;
    const int64_t d1 = d0 + kStageThreads - 1 < R_new ? d0 + kStageThreads - 1 : R_new - 1;
    const int32_t* src = work_ptr<int32_t>(st, work_layout(st->N, st->n_bins, st->capacity).src);
    const int64_t rn = d0 + threadIdx.x;
    const bool valid = rn < R_new;
    const int64_t j = valid ? src[rn] : 0;
    const int n_rows = st->dim == 1 ? (st->N + 31) / 32 : st->L * st->L;
    const int64_t g_lo = src[d0] >> 6, g_hi = src[d1] >> 6;  // the same for every thread
    const int cur = st->cur;
    if (g_hi - g_lo + 1 > kStageGroups) {
        if (valid) {
            gather_rows<Wt>(st, j, rn, n_rows);
            st->energy[cur ^ 1][rn] = st->energy[cur][j];
        }
        return;
    }
    const int nsrc = (int)(g_hi - g_lo + 1);
    const uint4* A = reinterpret_cast<const uint4*>((const Wt*)st->spins[cur] + g_lo * n_rows * 64);
    Wt* B = (Wt*)st->spins[cur ^ 1] + ((rn >> 6) * n_rows) * 64 + (rn & 63);
    const Wt* S = reinterpret_cast<const Wt*>(stage);
    const int64_t jl = j - g_lo * 64;  // the source's place among the staged groups' replicas
    const int jg = (int)(jl >> 6), jo = (int)(jl & 63);
    for (int r0 = 0; r0 < n_rows; r0 += kStageRows) {
        const int nr = n_rows - r0 < kStageRows ? n_rows - r0 : kStageRows;
        // staged piece e: group e / (nr LPL), row r0 + (e / LPL) mod nr, piece e mod LPL
        for (int e = threadIdx.x; e < nsrc * nr * LPL; e += kStageThreads) {
            const int line = e / LPL, part = e - line * LPL;
            const int gi = line / nr, q = line - gi * nr;
            stage[(gi * kStageRows + q) * LPL + part] = A[((int64_t)gi * n_rows + r0 + q) * LPL + part];
        }
        __syncthreads();
        if (valid) {
            for (int q = 0; q < nr; ++q) B[(int64_t)(r0 + q) * 64] = S[(jg * kStageRows + q) * 64 + jo];
        }
        __syncthreads();
    }
    if (valid) st->energy[cur ^ 1][rn] = st->energy[cur][j];
}

// one block of kStageThreads destinations of run blockIdx.y; the row word's width is the run's (a
// batch may mix lattice sizes), the staging buffer sized for the widest
__global__ void __launch_bounds__(kStageThreads) k_gather_bits_staged(pa_state* base)
{
    __shared__ uint4 stage[kStageGroups * kStageRows * 16];
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const int WB = st->dim == 1 ? 4 : (st->L <= 8 ? 1 : (st->L <= 16 ? 2 : 4));
    if (WB == 1) gather_staged<uint8_t>(st, stage);
    else if (WB == 2) gather_staged<uint16_t>(st, stage);
    else gather_staged<uint32_t>(st, stage);
}

int launch_resample(const pa_run* runs, int n, const pa_step& step, hipStream_t s)
{
    const BatchShape b = batch_shape(runs, n);
    ResampleParams p;
    p.beta_from = step.beta_from;
    p.beta_to = step.beta_to;
    p.R_target = step.R_target;
    p.w = step.weights;
    p.k = step.k;
    pa_state* base = runs[0].state;
    const unsigned cap_blocks = (unsigned)((b.cap_max + 255) / 256);
    const unsigned n_scan = (unsigned)((b.cap_max + kScanTile - 1) / kScanTile);
    launch_hist(runs, n, s);
    hipLaunchKernelGGL(k_normalise, dim3(1, n), dim3(256), 0, s, base, p);
    hipLaunchKernelGGL(k_copies, dim3(cap_blocks, n), dim3(256), 0, s, base, (int32_t)step.k);
    hipLaunchKernelGGL(k_scan_reduce, dim3(n_scan, n), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_scan_top, dim3(1, n), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_scan_down, dim3(n_scan, n), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_src, dim3(cap_blocks, n), dim3(256), 0, s, base);
    if (runs[0].layout == PA_U8) {
        const int64_t threads = b.cap_max * (b.stride_max / 16);
        hipLaunchKernelGGL(k_gather_u8, dim3((unsigned)((threads + 255) / 256), n), dim3(256), 0, s, base);
    } else {
        const unsigned blocks = (unsigned)((b.cap_max + kStageThreads - 1) / kStageThreads);
        hipLaunchKernelGGL(k_gather_bits_staged, dim3(blocks, n), dim3(kStageThreads), 0, s, base);
    }
    hipLaunchKernelGGL(k_finish, dim3(1, n), dim3(1), 0, s, base, p);
    return hip_status(hipGetLastError());
}

// ------------------------------------------------------------------ Gaussian couplings
// Real energies: per-replica weights instead of the energy histogram.  E_lo = min E (exact);
// w_j = expd(-(dbeta (E_j - E_lo))); S = sum of w_j over j = 0, 1, ... in replica order (eq. Q);
// ln Q = -dbeta E_lo + ln S - ln R~; copies of j ~ Poisson((R_target w_j) / S) by the same ladder
// and draws as the histogram path.  The weights are kept in the inactive energy buffer (FP64,
// [capacity]) between their evaluation and the copy numbers; the gather overwrites them.
constexpr int kMiscGaussS = kMiscS;  // misc slot: S (FP64 bits)

__global__ void __launch_bounds__(256) k_gauss_min(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    __shared__ double red[256];
    const double* E = reinterpret_cast<const double*>(st->energy[st->cur]);
    double m = INFINITY;
    for (int64_t j = threadIdx.x; j < st->R; j += blockDim.x) m = fmin(m, E[j]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int64_t* misc = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).misc);
        *reinterpret_cast<double*>(&misc[kMiscEmin]) = red[0];
    }
}

// thread per replica: its weight w_j into the inactive energy buffer
__global__ void __launch_bounds__(256) k_gauss_weights(pa_state* base, double dbeta)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= st->R) return;
    const int64_t* misc = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).misc);
    const double E_lo = *reinterpret_cast<const double*>(&misc[kMiscEmin]);
    const double* E = reinterpret_cast<const double*>(st->energy[st->cur]);
    double* w = reinterpret_cast<double*>(st->energy[st->cur ^ 1]);
    w[j] = expd(-(dbeta * (E[j] - E_lo)));
}

// a block per run: S in replica order, ln Q (the step's record is written by k_finish).  The block
// loads the weights a chunk at a time into LDS with coalesced loads, and one thread adds them in
// order from there: the chain of dependent FP64 additions is then the cost (R = 2000: 22 us; from
// global memory, one thread with eight loads ahead waited out the load latency every eight
// additions: 50 us)
constexpr int kNormChunk = 4096;

__global__ void __launch_bounds__(256) k_gauss_normalise(pa_state* base, ResampleParams p)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    __shared__ double chunk[kNormChunk];
    const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
    int64_t* misc = work_ptr<int64_t>(st, wl.misc);
    const double* w = reinterpret_cast<const double*>(st->energy[st->cur ^ 1]);
    const int64_t R = st->R;
    double S = 0.0;
    for (int64_t j0 = 0; j0 < R; j0 += kNormChunk) {
        const int n = (int)(R - j0 < kNormChunk ? R - j0 : kNormChunk);
        for (int i = threadIdx.x; i < n; i += blockDim.x) chunk[i] = w[j0 + i];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < n; ++i) S = S + chunk[i];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double dbeta = p.beta_to - p.beta_from;
    const double E_lo = *reinterpret_cast<const double*>(&misc[kMiscEmin]);
    if (!isfinite(S) || !(S > 0.0)) {
        st->status |= PA_FLAG_NONFINITE;
        return;
    }
    *reinterpret_cast<double*>(&misc[kMiscLnQ]) = -dbeta * E_lo + log(S) - log((double)R);
    *reinterpret_cast<double*>(&misc[kMiscGaussS]) = S;
}

// copy numbers from the replica weights, drawn as in k_copies
__global__ void __launch_bounds__(256) k_gauss_copies(pa_state* base, ResampleParams p)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t R = st->R;
    if (j - (int64_t)(threadIdx.x & 63) >= R) return;  // the whole wave past R
    const int64_t* misc = work_ptr<int64_t>(st, work_layout(st->N, st->n_bins, st->capacity).misc);
    const double S = *reinterpret_cast<const double*>(&misc[kMiscGaussS]);
    const double* w = reinterpret_cast<const double*>(st->energy[st->cur ^ 1]);
    const double Rt = p.R_target > 0.0 ? p.R_target : (double)st->R0;
    const bool live = j < R;
    const double lam = live ? (Rt * w[j]) / S : 0.0;
    int m = kLadderMin;
    int64_t q = 0;
    uint64_t keep = 0;
    if (lam > 0.0) {
        double rem = lam;
        if (lam > 64.0) {
            q = (int64_t)ceil(lam / 64.0) - 1;
            rem = lam - 64.0 * (double)q;
        }
        m = ladder_level(rem);
        keep = (uint64_t)floor(ldexp(rem, 32 - m));
    }
    const CopyDraws cd = {(uint32_t)j, (uint32_t)p.k, (uint32_t)st->seed, (uint32_t)(st->seed >> 32)};
    const bool drawn = lam > 0.0;
    const bool heavy = drawn && (q > 0 || m >= kCopiesHeavyM);
    int64_t n = drawn && !heavy ? copies_light(cd, m, keep) : 0;
    n = copies_heavy_by_wave(heavy, n, cd, m, q, keep);
    if (live) st->counts[j] = (int32_t)min(n, (int64_t)INT32_MAX);
}

// runs: n runs with consecutive states on one stream (grid.y = run), or a single run
int launch_resample_gauss(const pa_run* runs, int n, const pa_step& step, hipStream_t s)
{
    ResampleParams p;
    p.beta_from = step.beta_from;
    p.beta_to = step.beta_to;
    p.R_target = step.R_target;
    p.w = nullptr;
    p.k = step.k;
    pa_state* base = runs[0].state;
    int64_t cap = 0, stride = 0;
    for (int r = 0; r < n; ++r) {
        const int64_t N = runs[r].dim == 1 ? runs[r].L : (int64_t)runs[r].L * runs[r].L * runs[r].L;
        cap = std::max<int64_t>(cap, runs[r].capacity);
        stride = std::max<int64_t>(stride, (N + 15) / 16 * 16);
    }
    const unsigned cap_blocks = (unsigned)((cap + 255) / 256);
    const unsigned n_scan = (unsigned)((cap + kScanTile - 1) / kScanTile);
    const unsigned ny = (unsigned)n;
    hipLaunchKernelGGL(k_gauss_min, dim3(1, ny), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_gauss_weights, dim3(cap_blocks, ny), dim3(256), 0, s, base, step.beta_to - step.beta_from);
    hipLaunchKernelGGL(k_gauss_normalise, dim3(1, ny), dim3(256), 0, s, base, p);
    hipLaunchKernelGGL(k_gauss_copies, dim3(cap_blocks, ny), dim3(256), 0, s, base, p);
    hipLaunchKernelGGL(k_scan_reduce, dim3(n_scan, ny), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_scan_top, dim3(1, ny), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_scan_down, dim3(n_scan, ny), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_src, dim3(cap_blocks, ny), dim3(256), 0, s, base);
    const int64_t threads = cap * (stride / 16);  // one per 16 bytes of a row
    hipLaunchKernelGGL(k_gather_u8, dim3((unsigned)((threads + 255) / 256), ny), dim3(256), 0, s, base);
    hipLaunchKernelGGL(k_finish, dim3(1, ny), dim3(1), 0, s, base, p);
    return hip_status(hipGetLastError());
}

}  // namespace pa

extern "C" int pa_ladder_table(int m, uint64_t* C, int cap, int* len)
{
    if (!C || !len || cap < 2 || m < pa::kLadderMin || m > pa::kLadderMax) return PA_ERR_ARG;
    *len = pa::ladder_host(m, C, cap);
    return PA_OK;
}
