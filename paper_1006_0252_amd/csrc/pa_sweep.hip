// Metropolis sweeps of the whole population (Sec. II: theta MCMC sweeps of every replica
// at the new temperature).
//
// Design: one lane per replica.  A wave owns RPW = 64/LPR replicas; each replica's lattice
// sits in LDS as row bitmasks (one dword per row of the cube, bit x = spin at x, or 32
// consecutive sites of the chain), and LPR lanes share a replica by splitting its rows into
// LPR contiguous blocks.  Per row the six neighbour rows give, bit-parallel over x, the
// bonds with J s s = -1 and their count c (a bit-sliced adder); only the random acceptance
// test of moves with dE = 4c - 2z > 0 is done site by site, against the 16-bit first look
// of the run's Philox stream.  Energies follow from popcounts of the flipped sites.
#include <math.h>
#include <string.h>

#include "pa_common.h"
#include "pa_sweep_util.h"

namespace pa {

constexpr int kLayoutU8 = PA_U8;
constexpr int kLayoutBits = PA_BITS64;

// ---------------------------------------------------------------- geometry
template <int DIM, int L>
struct Geo;

// cube: rows are (y, z), NR = L^2, row bits x = 0..L-1
template <int L>
struct Geo<3, L> {
    static constexpr int NR = L * L;
    static constexpr int H = L / 2;  // sites of one colour per row
    static constexpr uint32_t MASK = (L == 32) ? 0xFFFFFFFFu : ((1u << L) - 1u);
    static constexpr int W = L <= 8 ? 8 : (L <= 16 ? 16 : 32);  // bits of one row word in HBM
};

// chain: rows of 32 consecutive sites; N is a run-time value
template <>
struct Geo<1, 0> {
    static constexpr int W = 32;
};

template <int L>
__device__ __forceinline__ uint32_t rot_up(uint32_t v)  // bit x <- bit (x + 1) mod L
{
    constexpr uint32_t M = Geo<3, L>::MASK;
    return ((v >> 1) | (v << (L - 1))) & M;
}

template <int L>
__device__ __forceinline__ uint32_t rot_down(uint32_t v)  // bit x <- bit (x - 1) mod L
{
    constexpr uint32_t M = Geo<3, L>::MASK;
    return ((v << 1) | (v >> (L - 1))) & M;
}

// LDS addressing: the rows of one wave are [LPR blocks][rows per block][RPW replicas]; the
// blocks are staggered by 16 dwords so that sub-lanes touching equal row offsets in different
// blocks fall in different banks
template <int LPR, int NR>
struct RowAddr {
    static constexpr int RPW = 64 / LPR;
    static constexpr int BS = (NR + LPR - 1) / LPR;          // rows per block
    static constexpr int PITCH = BS * RPW + (LPR > 1 ? 16 : 0);
    static constexpr int WAVE_DWORDS = LPR * PITCH;
    __device__ __forceinline__ static int at(int rho, int q)
    {
        const int b = rho / BS;
        return b * PITCH + (rho - b * BS) * RPW + q;
    }
};

// ---------------------------------------------------------------- 3D kernel
// One block = WPB waves; LDS holds jrow[NR][8] (coupling masks per row, shared by the block)
// and WPB wave areas.  jrow entries: +x, +y, +z, -x, -y, -z bonds with J = -1.
template <int L, int LAYOUT, int LPR, bool ZEROT>
__global__ void __launch_bounds__(256) k_sweep3(const pa_state* __restrict__ st, SweepParams p)
{
    using G = Geo<3, L>;
    using A = RowAddr<LPR, G::NR>;
    constexpr int NR = G::NR, H = G::H, RPW = A::RPW, BS = A::BS;
    if (st->status) return;  // sticky error: the population stays as it is
    extern __shared__ uint32_t lds[];
    uint32_t* jrow = lds;                            // [NR][8]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane % RPW, j = lane / RPW;
    uint32_t* rows = lds + NR * 8 + wave * A::WAVE_DWORDS;
    const int wpb = blockDim.x >> 6;
    const int64_t R = st->R;
    const int cur = st->cur;
    const int64_t rbase = ((int64_t)blockIdx.x * wpb + wave) * RPW;
    const int64_t r = rbase + q;
    const bool valid = r < R;

    // coupling masks per row (block-shared)
    const int8_t* J = st->J;
    for (int rho = threadIdx.x; rho < NR; rho += blockDim.x) {
        const int y = rho % L, z = rho / L;
        const int ym = (y + L - 1) % L, zm = (z + L - 1) % L;
        uint32_t m[6] = {0, 0, 0, 0, 0, 0};
        for (int x = 0; x < L; ++x) {
            const int i = x + L * rho;
            const int xm = (x + L - 1) % L;
            m[0] |= (uint32_t)(J[3 * i + 0] < 0) << x;
            m[1] |= (uint32_t)(J[3 * i + 1] < 0) << x;
            m[2] |= (uint32_t)(J[3 * i + 2] < 0) << x;
            m[3] |= (uint32_t)(J[3 * (xm + L * rho) + 0] < 0) << x;
            m[4] |= (uint32_t)(J[3 * (x + L * (ym + L * z)) + 1] < 0) << x;
            m[5] |= (uint32_t)(J[3 * (x + L * (y + L * zm)) + 2] < 0) << x;
        }
        for (int k = 0; k < 6; ++k) jrow[rho * 8 + k] = m[k];
        jrow[rho * 8 + 6] = 0;
        jrow[rho * 8 + 7] = 0;
    }

    // load this lane's row block
    const int rho0 = j * BS;
    const int rho1 = min(NR, rho0 + BS);
    if (rbase < R) {
        if (LAYOUT == kLayoutBits) {
            constexpr int WB = G::W / 8;
            const int64_t g = r >> 6;
            const int l = (int)(r & 63);
            const uint8_t* base = (const uint8_t*)st->spins[cur] + ((g * NR) * 64 + l) * WB;
            for (int rho = rho0; rho < rho1; ++rho) {
                const uint8_t* a = base + (int64_t)rho * 64 * WB;
                uint32_t v = WB == 1 ? *a : (WB == 2 ? *(const uint16_t*)a : *(const uint32_t*)a);
                rows[A::at(rho, q)] = v;
            }
        } else {
            const uint8_t* base = (const uint8_t*)st->spins[cur] + r * st->row_stride;
            for (int rho = rho0; rho < rho1; ++rho) {
                const uint8_t* a = base + rho * L;
                uint32_t v = 0;
                if (L % 4 == 0) {
#pragma unroll
                    for (int d = 0; d < L / 4; ++d) v |= pack4(((const uint32_t*)a)[d]) << (4 * d);
                } else {
#pragma unroll
                    for (int x = 0; x < L; ++x) v |= (uint32_t)(a[x] & 1) << x;
                }
                rows[A::at(rho, q)] = v;
            }
        }
    }
    __syncthreads();
    if (rbase >= R) return;

    const uint32_t k0 = (uint32_t)st->seed, k1 = (uint32_t)(st->seed >> 32);
    const uint32_t thi4 = p.thi[4], thi5 = p.thi[5], thi6 = p.thi[6];
    const int d5 = (int)thi5 - (int)thi4, d6 = (int)thi6 - (int)thi4;
    uint32_t sum_c = 0, n_flip = 0;
    const uint32_t rr = (uint32_t)r;

    for (int s = 0; s < p.n_sweeps; ++s) {
        const int64_t t = p.t0 + s;
        for (int col = 0; col < 2; ++col) {
            const uint32_t ctr2 = (uint32_t)(2 * t + col);
            uint32_t call = 0xFFFFFFFFu;
            uint4v rnd = {0, 0, 0, 0};
            for (int rho = rho0; rho < rho1; ++rho) {
                const int y = rho % L, z = rho / L;
                const int ryp = (y + 1 == L) ? rho - (L - 1) : rho + 1;
                const int rym = (y == 0) ? rho + (L - 1) : rho - 1;
                const int rzp = (z + 1 == L) ? rho - (NR - L) : rho + L;
                const int rzm = (z == 0) ? rho + (NR - L) : rho - L;
                const uint32_t own = rows[A::at(rho, q)];
                const uint32_t* jr = jrow + rho * 8;
                const uint32_t b0 = own ^ rot_up<L>(own) ^ jr[0];
                const uint32_t b1 = own ^ rows[A::at(ryp, q)] ^ jr[1];
                const uint32_t b2 = own ^ rows[A::at(rzp, q)] ^ jr[2];
                const uint32_t b3 = own ^ rot_down<L>(own) ^ jr[3];
                const uint32_t b4 = own ^ rows[A::at(rym, q)] ^ jr[4];
                const uint32_t b5 = own ^ rows[A::at(rzm, q)] ^ jr[5];
                // bit-sliced count c = b0 + ... + b5 -> (c2 c1 c0)
                const uint32_t s1 = b0 ^ b1 ^ b2, k1c = (b0 & b1) | (b2 & (b0 ^ b1));
                const uint32_t s2 = b3 ^ b4 ^ b5, k2c = (b3 & b4) | (b5 & (b3 ^ b4));
                const uint32_t c0 = s1 ^ s2, k3c = s1 & s2;
                const uint32_t c1 = k1c ^ k2c ^ k3c;
                const uint32_t c2 = (k1c & k2c) | (k3c & (k1c ^ k2c));
                const int par = (col + y + z) & 1;  // x parity of this colour in the row
                const uint32_t colmask = (par ? 0xAAAAAAAAu : 0x55555555u) & G::MASK;
                const uint32_t cand = c2 & colmask;  // dE > 0: random test
                uint32_t acc = 0, tie = 0;
#pragma unroll
                for (int m = 0; m < H; ++m) {
                    const int h = rho * H + m;
                    if (H % 8 == 0) {
                        // a row holds whole 8-site chunks: calls start at fixed m
                        if ((m & 7) == 0) rnd = philox10((uint32_t)(h >> 3), rr, ctr2, kTagMet, k0, k1);
                    } else if ((uint32_t)(h >> 3) != call) {
                        call = (uint32_t)(h >> 3);
                        rnd = philox10(call, rr, ctr2, kTagMet, k0, k1);
                    }
                    const uint32_t u = field16(rnd, h & 7);
                    const int x = 2 * m + par;
                    if (ZEROT) {
                        tie |= (uint32_t)(u == 0u) << x;
                    } else {
                        const int bq0 = (c0 >> x) & 1, bq1 = (c1 >> x) & 1;
                        const uint32_t thi = (uint32_t)((int)thi4 + bq0 * d5 + bq1 * d6);
                        acc |= (uint32_t)(u < thi) << x;
                        tie |= (uint32_t)(u == thi) << x;
                    }
                }
                tie &= cand;
                if (tie) {
                    // exact resolution of first-look ties with the 48 low bits
#pragma unroll 1
                    for (int m = 0; m < H; ++m) {
                        const int x = 2 * m + par;
                        if (!((tie >> x) & 1)) continue;
                        const int h = rho * H + m;
                        const uint4v v = philox10((uint32_t)(h >> 3), rr, ctr2, kTagMet, k0, k1);
                        const uint32_t u = field16(v, h & 7);
                        const int cls = 4 + (int)((c0 >> x) & 1) + 2 * (int)((c1 >> x) & 1);
                        const int i = x + L * rho;
                        if (tie_accept(u, p.T64[cls], (uint32_t)i, rr, ctr2, k0, k1)) acc |= 1u << x;
                        else acc &= ~(1u << x);
                    }
                }
                uint32_t flip = ((~c2) & colmask) | (acc & cand);
                if (!valid) flip = 0;
                rows[A::at(rho, q)] = own ^ flip;
                sum_c += __popc(flip & c0) + 2 * __popc(flip & c1) + 4 * __popc(flip & c2);
                n_flip += __popc(flip);
            }
            // rows of the other colour are read next: every lane's writes of this phase first
            wave_sync();
        }
    }

    // energy change of the replica: sum over flips of (4c - 12)
    int dE = 4 * (int)sum_c - 12 * (int)n_flip;
    for (int off = RPW; off < 64; off <<= 1) dE += __shfl_xor(dE, off, 64);

    // store rows back
    if (LAYOUT == kLayoutBits) {
        constexpr int WB = G::W / 8;
        const int64_t g = r >> 6;
        const int l = (int)(r & 63);
        uint8_t* base = (uint8_t*)st->spins[cur] + ((g * NR) * 64 + l) * WB;
        for (int rho = rho0; rho < rho1; ++rho) {
            uint8_t* a = base + (int64_t)rho * 64 * WB;
            const uint32_t v = rows[A::at(rho, q)];
            if (!valid) continue;
            if (WB == 1) *a = (uint8_t)v;
            else if (WB == 2) *(uint16_t*)a = (uint16_t)v;
            else *(uint32_t*)a = v;
        }
    } else if (valid) {
        uint8_t* base = (uint8_t*)st->spins[cur] + r * st->row_stride;
        for (int rho = rho0; rho < rho1; ++rho) {
            uint8_t* a = base + rho * L;
            const uint32_t v = rows[A::at(rho, q)];
            if (L % 4 == 0) {
#pragma unroll
                for (int d = 0; d < L / 4; ++d) ((uint32_t*)a)[d] = unpack4(v >> (4 * d));
            } else {
#pragma unroll
                for (int x = 0; x < L; ++x) a[x] = (uint8_t)((v >> x) & 1);
            }
        }
    }
    if (valid && j == 0) st->energy[cur][r] += dE;
}

// ---------------------------------------------------------------- 1D kernel (ring)
// rows of 32 sites; row rho holds sites 32 rho .. 32 rho + len - 1; grid.y = run (consecutive
// states of one chain length and layout)
template <int LAYOUT, int LPR, bool ZEROT>
__global__ void __launch_bounds__(256) k_sweep1(const pa_state* __restrict__ base, SweepParams p, int NRr)
{
    constexpr int RPW = 64 / LPR;
    const pa_state* __restrict__ st = base + blockIdx.y;
    if (st->status) return;  // sticky error: the population stays as it is
    extern __shared__ uint32_t lds[];
    const int N = st->N;
    const int NR = NRr;
    const int BS = (NR + LPR - 1) / LPR;
    const int PITCH = BS * RPW + (LPR > 1 ? 16 : 0);
    uint32_t* jrow = lds;  // [NR][2]: bond to +1, bond to -1 with J = -1
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane % RPW, j = lane / RPW;
    uint32_t* rows = lds + NR * 2 + wave * (LPR * PITCH);
    auto at = [&](int rho) { const int b = rho / BS; return b * PITCH + (rho - b * BS) * RPW + q; };
    const int wpb = blockDim.x >> 6;
    const int64_t R = st->R;
    const int cur = st->cur;
    const int64_t rbase = ((int64_t)blockIdx.x * wpb + wave) * RPW;
    const int64_t r = rbase + q;
    const bool valid = r < R;
    const int8_t* J = st->J;
    for (int rho = threadIdx.x; rho < NR; rho += blockDim.x) {
        const int len = min(32, N - 32 * rho);
        uint32_t mp = 0, mm = 0;
        for (int x = 0; x < len; ++x) {
            const int i = 32 * rho + x;
            mp |= (uint32_t)(J[i] < 0) << x;
            mm |= (uint32_t)(J[(i + N - 1) % N] < 0) << x;
        }
        jrow[2 * rho] = mp;
        jrow[2 * rho + 1] = mm;
    }
    const int rho0 = j * BS, rho1 = min(NR, rho0 + BS);
    if (rbase < R) {
        for (int rho = rho0; rho < rho1; ++rho) {
            const int len = min(32, N - 32 * rho);
            uint32_t v = 0;
            if (LAYOUT == kLayoutBits) {
                v = ((const uint32_t*)st->spins[cur])[((r >> 6) * NR + rho) * 64 + (r & 63)];
            } else {
                const uint8_t* a = (const uint8_t*)st->spins[cur] + r * st->row_stride + 32 * rho;
                for (int x = 0; x < len; ++x) v |= (uint32_t)(a[x] & 1) << x;
            }
            rows[at(rho)] = v;
        }
    }
    __syncthreads();
    if (rbase >= R) return;
    const uint32_t k0 = (uint32_t)st->seed, k1 = (uint32_t)(st->seed >> 32);
    const uint32_t thi2 = p.thi[2];
    const uint32_t rr = (uint32_t)r;
    uint32_t sum_c = 0, n_flip = 0;
    for (int s = 0; s < p.n_sweeps; ++s) {
        const int64_t t = p.t0 + s;
        for (int col = 0; col < 2; ++col) {
            const uint32_t ctr2 = (uint32_t)(2 * t + col);
            for (int rho = rho0; rho < rho1; ++rho) {
                const int len = min(32, N - 32 * rho);
                const uint32_t lmask = len == 32 ? 0xFFFFFFFFu : ((1u << len) - 1u);
                const int rn = (rho + 1 == NR) ? 0 : rho + 1;
                const int rp = (rho == 0) ? NR - 1 : rho - 1;
                const int lenp = min(32, N - 32 * rp);
                const uint32_t own = rows[at(rho)];
                const uint32_t nxt = rows[at(rn)], prv = rows[at(rp)];
                const uint32_t up = ((own >> 1) | ((nxt & 1u) << (len - 1))) & lmask;
                const uint32_t dn = ((own << 1) | ((prv >> (lenp - 1)) & 1u)) & lmask;
                const uint32_t b0 = own ^ up ^ jrow[2 * rho];
                const uint32_t b1 = own ^ dn ^ jrow[2 * rho + 1];
                const uint32_t colmask = (col ? 0xAAAAAAAAu : 0x55555555u) & lmask;
                const uint32_t c2 = b0 & b1;         // c = 2: dE = +4
                const uint32_t cand = c2 & colmask;
                uint32_t acc = 0, tie = 0;
                uint4v rnd = {0, 0, 0, 0};
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int x = 2 * m + col;
                    if ((m & 7) == 0) rnd = philox10((uint32_t)(2 * rho + (m >> 3)), rr, ctr2, kTagMet, k0, k1);
                    const uint32_t u = field16(rnd, m & 7);
                    if (ZEROT) {
                        tie |= (uint32_t)(u == 0u) << x;
                    } else {
                        acc |= (uint32_t)(u < thi2) << x;
                        tie |= (uint32_t)(u == thi2) << x;
                    }
                }
                tie &= cand;
                if (tie) {
#pragma unroll 1
                    for (int m = 0; m < 16; ++m) {
                        const int x = 2 * m + col;
                        if (!((tie >> x) & 1)) continue;
                        const uint4v v = philox10((uint32_t)(2 * rho + (m >> 3)), rr, ctr2, kTagMet, k0, k1);
                        const uint32_t u = field16(v, m & 7);
                        if (tie_accept(u, p.T64[2], (uint32_t)(32 * rho + x), rr, ctr2, k0, k1)) acc |= 1u << x;
                        else acc &= ~(1u << x);
                    }
                }
                uint32_t flip = ((~c2) & colmask) | (acc & cand);
                if (!valid) flip = 0;
                rows[at(rho)] = own ^ flip;
                sum_c += __popc(flip & b0) + __popc(flip & b1);
                n_flip += __popc(flip);
            }
            wave_sync();
        }
    }
    int dE = 4 * (int)sum_c - 4 * (int)n_flip;
    for (int off = RPW; off < 64; off <<= 1) dE += __shfl_xor(dE, off, 64);
    if (valid) {
        for (int rho = rho0; rho < rho1; ++rho) {
            const uint32_t v = rows[at(rho)];
            if (LAYOUT == kLayoutBits) {
                ((uint32_t*)st->spins[cur])[((r >> 6) * NR + rho) * 64 + (r & 63)] = v;
            } else {
                const int len = min(32, N - 32 * rho);
                uint8_t* a = (uint8_t*)st->spins[cur] + r * st->row_stride + 32 * rho;
                for (int x = 0; x < len; ++x) a[x] = (uint8_t)((v >> x) & 1);
            }
        }
        if (j == 0) st->energy[cur][r] += dE;
    }
}

// ---------------------------------------------------------------- dispatch
struct SweepConfig {
    int lpr;   // lanes per replica
    int wpb;   // waves per block
};

// LDS bytes one block may use on the current device
static size_t lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64 * 1024;
    return (size_t)v;
}

template <int L, int LAYOUT, int LPR, bool Z>
static int launch3_t(const pa_run& run, const SweepParams& p, int wpb, hipStream_t s)
{
    using A = RowAddr<LPR, L * L>;
    const size_t limit = lds_limit();
    size_t lds = (size_t)(L * L * 8 + wpb * A::WAVE_DWORDS) * 4;
    while (lds > limit && wpb > 1) {
        --wpb;
        lds = (size_t)(L * L * 8 + wpb * A::WAVE_DWORDS) * 4;
    }
    if (lds > limit) return PA_ERR_ARG;
    const int64_t per_block = (int64_t)wpb * A::RPW;
    const int64_t blocks = (run.capacity + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_sweep3<L, LAYOUT, LPR, Z>), dim3((unsigned)blocks), dim3(64 * wpb), lds, s, run.state, p);
    return PA_OK;
}

template <int L, int LAYOUT>
static int launch3_l(const pa_run& run, const SweepParams& p, SweepConfig cfg, bool zero, hipStream_t s)
{
    if (cfg.lpr == 1) return zero ? launch3_t<L, LAYOUT, 1, true>(run, p, cfg.wpb, s)
                                  : launch3_t<L, LAYOUT, 1, false>(run, p, cfg.wpb, s);
    if (cfg.lpr == 2) return zero ? launch3_t<L, LAYOUT, 2, true>(run, p, cfg.wpb, s)
                                  : launch3_t<L, LAYOUT, 2, false>(run, p, cfg.wpb, s);
    return zero ? launch3_t<L, LAYOUT, 4, true>(run, p, cfg.wpb, s)
                : launch3_t<L, LAYOUT, 4, false>(run, p, cfg.wpb, s);
}

template <int L>
static int launch3(const pa_run& run, const SweepParams& p, SweepConfig cfg, bool zero, hipStream_t s)
{
    return run.layout == PA_U8 ? launch3_l<L, kLayoutU8>(run, p, cfg, zero, s)
                               : launch3_l<L, kLayoutBits>(run, p, cfg, zero, s);
}

template <int LAYOUT, int LPR, bool Z>
static int launch1_t(const pa_run& run, const SweepParams& p, int wpb, hipStream_t s, int n_runs, int64_t capacity)
{
    const int N = run.L;
    const int NR = (N + 31) / 32;
    const int RPW = 64 / LPR;
    const int BS = (NR + LPR - 1) / LPR;
    const int PITCH = BS * RPW + (LPR > 1 ? 16 : 0);
    const size_t limit = lds_limit();
    size_t lds = (size_t)(NR * 2 + wpb * LPR * PITCH) * 4;
    while (lds > limit && wpb > 1) {
        --wpb;
        lds = (size_t)(NR * 2 + wpb * LPR * PITCH) * 4;
    }
    if (lds > limit) return PA_ERR_ARG;
    const int64_t per_block = (int64_t)wpb * RPW;
    const int64_t blocks = (capacity + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_sweep1<LAYOUT, LPR, Z>), dim3((unsigned)blocks, (unsigned)n_runs), dim3(64 * wpb), lds, s,
                       run.state, p, NR);
    return PA_OK;
}

static int launch1(const pa_run& run, const SweepParams& p, SweepConfig cfg, bool zero, hipStream_t s, int n_runs = 1,
                   int64_t capacity = 0)
{
    const int64_t cap = capacity > 0 ? capacity : run.capacity;  // the largest of the runs
    if (run.layout == PA_U8) {
        if (cfg.lpr == 2) return zero ? launch1_t<kLayoutU8, 2, true>(run, p, cfg.wpb, s, n_runs, cap)
                                      : launch1_t<kLayoutU8, 2, false>(run, p, cfg.wpb, s, n_runs, cap);
        return zero ? launch1_t<kLayoutU8, 1, true>(run, p, cfg.wpb, s, n_runs, cap)
                    : launch1_t<kLayoutU8, 1, false>(run, p, cfg.wpb, s, n_runs, cap);
    }
    if (cfg.lpr == 2) return zero ? launch1_t<kLayoutBits, 2, true>(run, p, cfg.wpb, s, n_runs, cap)
                                  : launch1_t<kLayoutBits, 2, false>(run, p, cfg.wpb, s, n_runs, cap);
    return zero ? launch1_t<kLayoutBits, 1, true>(run, p, cfg.wpb, s, n_runs, cap)
                : launch1_t<kLayoutBits, 1, false>(run, p, cfg.wpb, s, n_runs, cap);
}

// default launch shape per lattice (lanes per replica, waves per block)
static SweepConfig default_config(int dim, int L)
{
    if (dim == 1) return {1, 4};
    if (L >= 24) return {4, 1};
    if (L >= 16) return {4, 3};
    if (L >= 10) return {2, 4};
    return {1, 4};
}

// launch shape of the fast cube kernel (L = 4, 8, 12, 16)
static SweepConfig fast_config(int L)
{
    if (L >= 12) return {4, 4};
    if (L >= 8) return {2, 4};
    return {1, 4};
}

static SweepConfig g_override = {0, 0};

int build_sweep_params(const pa_step& step, int z, SweepParams* pp)
{
    SweepParams& p = *pp;
    memset(&p, 0, sizeof(p));
    uint64_t T[8];
    uint8_t always[8];
    build_thresholds(step.beta_to, z, T, always);
    for (int c = 0; c <= z; ++c) {
        p.T64[c] = T[c];
        p.thi[c] = always[c] ? 0x10000u : (uint32_t)(T[c] >> 48);
    }
    p.t0 = step.t0;
    p.n_sweeps = step.n_sweeps;
    return PA_OK;
}

int launch_sweep(const pa_run& run, const pa_step& step, hipStream_t s)
{
    SweepParams p;
    const int z = 2 * run.dim;
    build_sweep_params(step, z, &p);
    bool zero = true;
    for (int c = z / 2 + 1; c <= z; ++c)
        if (p.thi[c] != 0) zero = false;
    SweepConfig cfg = default_config(run.dim, run.L);
    if (g_override.lpr) cfg = g_override;
    int st;
    if (fast_sweep_supported(run.dim, run.L) && fast_sweep_thresholds_ok(p)) {
        // bit-packed cubes take the colour-packed kernel (L = 16) or the colour-string kernel (L = 4,
        // 6, 8, 10) unless a launch shape is forced
        if (!g_override.lpr && run.L == 16 && run.layout == PA_BITS64) {
            st = launch_sweep_colour(run, p, s);
        } else if (!g_override.lpr && string_sweep_supported(run.dim, run.L, run.layout)) {
            st = launch_sweep_strings(run, p, s);
        } else {
            SweepConfig fc = g_override.lpr ? g_override : fast_config(run.L);
            st = launch_sweep_fast(run, p, fc.lpr, fc.wpb, s);
        }
        if (st != PA_OK) return st;
        return hip_status(hipGetLastError());
    }
    if (run.dim == 1) {
        const int NR = (run.L + 31) / 32;
        if (cfg.lpr > NR) cfg.lpr = 1;
        if (cfg.lpr > 2) cfg.lpr = 2;
        st = launch1(run, p, cfg, zero, s);
    } else {
        if (cfg.lpr > run.L * run.L) cfg.lpr = 1;
        switch (run.L) {
            case 2: st = launch3<2>(run, p, cfg, zero, s); break;
            case 4: st = launch3<4>(run, p, cfg, zero, s); break;
            case 6: st = launch3<6>(run, p, cfg, zero, s); break;
            case 8: st = launch3<8>(run, p, cfg, zero, s); break;
            case 10: st = launch3<10>(run, p, cfg, zero, s); break;
            case 12: st = launch3<12>(run, p, cfg, zero, s); break;
            case 14: st = launch3<14>(run, p, cfg, zero, s); break;
            case 16: st = launch3<16>(run, p, cfg, zero, s); break;
            case 18: st = launch3<18>(run, p, cfg, zero, s); break;
            case 20: st = launch3<20>(run, p, cfg, zero, s); break;
            case 24: st = launch3<24>(run, p, cfg, zero, s); break;
            case 32: st = launch3<32>(run, p, cfg, zero, s); break;
            default: return PA_ERR_ARG;
        }
    }
    if (st != PA_OK) return st;
    return hip_status(hipGetLastError());
}

// n > 1 chain runs with consecutive states, one length and layout: one launch, grid.y = run
int launch_sweep_chain_batch(const pa_run* runs, int n, const pa_step& step, hipStream_t s)
{
    SweepParams p;
    build_sweep_params(step, 2, &p);
    const bool zero = p.thi[2] == 0;
    SweepConfig cfg = default_config(1, runs[0].L);
    if (g_override.lpr) cfg = g_override;
    const int NR = (runs[0].L + 31) / 32;
    if (cfg.lpr > NR) cfg.lpr = 1;
    if (cfg.lpr > 2) cfg.lpr = 2;
    int64_t cap = 0;
    for (int r = 0; r < n; ++r) cap = runs[r].capacity > cap ? runs[r].capacity : cap;
    const int st = launch1(runs[0], p, cfg, zero, s, n, cap);
    if (st != PA_OK) return st;
    return hip_status(hipGetLastError());
}

}  // namespace pa

// launch-shape override for the autotuner (0, 0 restores the default)
extern "C" int pa_set_sweep_config(int lanes_per_replica, int waves_per_block)
{
    if (lanes_per_replica == 0 && waves_per_block == 0) {
        pa::g_override = {0, 0};
        return PA_OK;
    }
    if ((lanes_per_replica != 1 && lanes_per_replica != 2 && lanes_per_replica != 4) || waves_per_block < 1 ||
        waves_per_block > 4)
        return PA_ERR_ARG;
    pa::g_override = {lanes_per_replica, waves_per_block};
    return PA_OK;
}
