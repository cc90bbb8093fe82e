// Internal header of libpa: device Philox, work-buffer layout, shared constants.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa.h"

namespace pa {

// stream tags: fourth Philox counter word of each kind of draw
constexpr uint32_t kTagInit = 1;
constexpr uint32_t kTagMet = 2;
constexpr uint32_t kTagTie = 3;
constexpr uint32_t kTagPoisson = 4;
constexpr uint32_t kTagCoupling = 5;

// Poisson ladder: levels 2^m, m in [kLadderMin, kLadderMax]; Poisson(64) blocks above 64
constexpr int kLadderMin = -20;
constexpr int kLadderMax = 6;
constexpr int kLadderLevels = kLadderMax - kLadderMin + 1;
constexpr int kLadderCap = 256;  // entries per level (the largest level, 2^6, needs < 200)

// scan tile: replicas per block of the device-wide exclusive scan
constexpr int kScanTile = 1024;

struct uint4v { uint32_t x, y, z, w; };

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two 32x32->64
// products of counter words 0 and 2, Weyl key schedule between rounds.  The three-way xor
// of each round is one v_bitop3 (truth table 0x96 = a ^ b ^ c) on gfx950.
__device__ inline uint4v philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

__host__ __device__ inline uint32_t word_of(const uint4v& v, int w)
{
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

// byte offsets of the scratch arrays inside pa_run.work
struct WorkLayout {
    size_t hist;      // int64 [n_bins]   replicas per energy bin
    size_t bin_q;     // int64 [n_bins]   Poisson(64) blocks of the bin's mean copy number
    size_t bin_keep;  // uint64 [n_bins]  thinning threshold floor(rem 2^(32-m))
    size_t bin_m;     // int32 [n_bins]   ladder level m
    size_t scan;      // int64 [n_scan + 1] block sums of the copy-number scan
    size_t src;       // int32 [capacity] source replica of each new replica
    size_t qhist;     // int64 [N + 1]    overlap histogram (Hamming distance)
    size_t misc;      // int64 [64]       small reductions (E min/max, pending ln Q)
    size_t batch;     // int64 [1025]     work-list offsets of a batched sweep (first run of a batch)
    size_t total;
};

__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline WorkLayout work_layout(int64_t N, int64_t n_bins, int64_t capacity)
{
    WorkLayout w;
    size_t o = 0;
    w.hist = o;     o = align256(o + 8 * (size_t)n_bins);
    w.bin_q = o;    o = align256(o + 8 * (size_t)n_bins);
    w.bin_keep = o; o = align256(o + 8 * (size_t)n_bins);
    w.bin_m = o;    o = align256(o + 4 * (size_t)n_bins);
    const int64_t n_scan = (capacity + kScanTile - 1) / kScanTile;
    w.scan = o;     o = align256(o + 8 * (size_t)(n_scan + 1));
    w.src = o;      o = align256(o + 4 * (size_t)capacity);
    w.qhist = o;    o = align256(o + 8 * (size_t)(N + 1));
    w.misc = o;     o = align256(o + 8 * 64);
    w.batch = o;    o = align256(o + 8 * 1025);
    w.total = o;    // Gaussian couplings only: the sweep's threshold table starts here
    return w;
}

// bytes of the Gaussian sweep tables after WorkLayout::total: N / 2 sites per colour times 64
// neighbour patterns (cube; 4 for the chain, sized for the cube), a u16 first-look table and then
// a u64 table of the full thresholds
__host__ __device__ inline size_t gauss_table_bytes(int64_t N) { return (2 + 8) * 64 * (size_t)N; }

template <typename T>
__device__ inline T* work_ptr(const pa_state* st, size_t off)
{
    return reinterpret_cast<T*>(st->work + off);
}

// sweep parameters passed by value
struct SweepParams {
    uint32_t thi[8];     // top 16 bits of T64 per class c (0x10000 = always accept)
    uint64_t T64[8];     // full thresholds per class c
    int64_t t0;          // first global sweep index
    int32_t n_sweeps;
    int32_t rpb;         // replicas (u8) or 64-replica groups (bits64) per block
};

// a batched sweep's run order: position p of the work list holds run order.run[p] (at most
// kMaxBatch runs)
constexpr int kMaxBatch = 1024;
struct BatchOrder {
    uint16_t run[kMaxBatch];
};

// lanes per replica of the row-pair batch kernel for each lattice size (L = 2 mod 4 needs one lane
// per replica so that the Philox phase of a plane is uniform over the wave)
__host__ __device__ constexpr int batch_lpr(int L) { return L % 4 != 0 ? 1 : (L >= 12 ? 4 : (L >= 8 ? 2 : 1)); }

// the colour-string kernel: bit-packed cubes of L = 4, 6, 8, 10, one lane per replica
__host__ __device__ inline bool string_sweep_supported(int dim, int L, int layout)
{
    return dim == 3 && layout == PA_BITS64 && (L == 4 || L == 6 || L == 8 || L == 10);
}

// replicas per work item of a batched cube sweep: one 64-replica group for the colour-string
// kernel, 64 / lanes per replica for the row-pair kernel
__host__ __device__ inline int batch_tile_replicas(int L, int layout)
{
    return string_sweep_supported(3, L, layout) ? 64 : 64 / batch_lpr(L);
}

// host launch helpers (defined in the .hip files)
int launch_init(const pa_run& run, const int8_t* J_host, hipStream_t s);
int launch_sweep(const pa_run& run, const pa_step& step, hipStream_t s);
// n > 1 chain runs (dim 1) with consecutive states, one length and layout, one stream
int launch_sweep_chain_batch(const pa_run* runs, int n, const pa_step& step, hipStream_t s);
int launch_sweep_fast(const pa_run& run, const SweepParams& p, int lpr, int wpb, hipStream_t s);
// the colour-packed kernel of the bit-packed L = 16 cube (PA_ERR_ARG for any other run)
int launch_sweep_colour(const pa_run& run, const SweepParams& p, hipStream_t s);
// the colour-string kernel (string_sweep_supported runs): one run, or one group of equal-L runs of a
// batch (waves persistent waves taking items, or one item per wave for waves = the items)
int launch_sweep_strings(const pa_run& run, const SweepParams& p, hipStream_t s);
int launch_sweep_strings_group(int L, pa_state* base, int pos0, int pos1, const BatchOrder& order,
                               const SweepParams& p, bool persistent, int64_t waves, hipStream_t s);
// batched launchers: n runs whose device states are contiguous (runs[r].state == runs[0].state + r)
int launch_resample(const pa_run* runs, int n, const pa_step& step, hipStream_t s);
int launch_hist(const pa_run* runs, int n, hipStream_t s);
int launch_measure(const pa_run* runs, int n, const pa_run* partner, int pair_xor, hipStream_t s);
int launch_free_energy(const pa_run* runs, int n, double* out, hipStream_t s);
int launch_sweep_batch(const pa_run* runs, int n, const SweepParams& p, hipStream_t s);
bool fast_sweep_supported(int dim, int L);
// the fast cube sweep compares first looks against top + 1 in 16 bits: tops up to 0xFFFE (a move
// of dE = 4 accepted with probability below 1 - 2^-16, i.e. beta above about 4e-6)
inline bool fast_sweep_thresholds_ok(const SweepParams& p) { return p.thi[4] <= 0xFFFEu; }
int build_sweep_params(const pa_step& step, int z, SweepParams* p);
int launch_weighted_average_dev(int n_sets, int M, const double* x, const double* R, const double* A, int n_obs,
                                double* out, hipStream_t s);
int launch_overlap_average_dev(int n_sets, int n_pairs, const double* x, const double* R, const double* Q,
                               double* out, hipStream_t s);
int launch_bootstrap_dev(int n_sets, int M, const double* x, const double* R, const double* A, int n_obs, int n_boot,
                         const int32_t* idx, double* rep, double* err, hipStream_t s);
int build_thresholds(double beta, int z, uint64_t* T, uint8_t* always);
int launch_features(const pa_run* runs, int n, float* x, hipStream_t s);
int launch_rho(const pa_run* runs, int n, const double* args, int n_args, int mode, double cap, int64_t ld,
               double* out, hipStream_t s);
int upload_ladder(hipStream_t s);

inline int hip_status(hipError_t e) { return e == hipSuccess ? PA_OK : PA_ERR_HIP; }

// exp written out for the Gaussian-coupling path, so that host and device reach the same bits:
// x = k ln 2 + r, k = floor(x / ln 2 + 1/2), r by a two-part ln 2 (the high part has 32
// significant bits, so k ln2_hi is exact), e^r by its Taylor series to r^13 in Horner form,
// scaled by 2^k; 0 below -745.  Products and sums are rounded one by one.
__device__ inline double expd(double x)
{
#pragma clang fp contract(off)
    if (x < -745.0) return 0.0;
    const double k = floor(x * 1.4426950408889634 + 0.5);
    const double r = (x - k * 0.6931471803691238) - k * 1.9082149292705877e-10;
    double p = 1.6059043836821613e-10;
    p = p * r + 2.08767569878681e-09;
    p = p * r + 2.505210838544172e-08;
    p = p * r + 2.755731922398589e-07;
    p = p * r + 2.7557319223985893e-06;
    p = p * r + 2.48015873015873e-05;
    p = p * r + 0.0001984126984126984;
    p = p * r + 0.001388888888888889;
    p = p * r + 0.008333333333333333;
    p = p * r + 0.041666666666666664;
    p = p * r + 0.16666666666666666;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return ldexp(p, (int)k);
}

// Gaussian-coupling path (separate kernels; n > 1 runs: consecutive states on one stream)
int gauss_couplings_upload(const pa_run& run, hipStream_t s);
int launch_energy_gauss(const pa_run& run, int buf, int64_t n_replicas, hipStream_t s);
// consecutive: the runs' states are consecutive and share runs[0].stream (one launch for all)
int launch_sweep_gauss(const pa_run* runs, int n_runs, bool consecutive, const pa_step& step, hipStream_t s);
int launch_resample_gauss(const pa_run* runs, int n, const pa_step& step, hipStream_t s);
int launch_measure_gauss(const pa_run* runs, int n, const pa_run* partner, int pair_xor, hipStream_t s);
int launch_moments_gauss(const pa_run* runs, int n, hipStream_t s);

}  // namespace pa
