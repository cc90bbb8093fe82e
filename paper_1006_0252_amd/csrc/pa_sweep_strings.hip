// Metropolis sweeps of small cubes (L = 4, 6, 8, 10), bit-packed populations: each replica's
// sites of one colour as one bit string, ordered so that bit b is half-site b.  The same sample as
// the generic kernel (same Philox fields, same acceptance rule, same checkerboard order).
//
// Colour string.  Half-site b = m + (L/2) (y + L z) (m = 0 .. L/2 - 1) holds the sites x = 2 m and
// 2 m + 1 of row (y, z); exactly one of them has colour c, x = 2 m + sigma with sigma = (c + y + z)
// mod 2.  Bit b of the colour-c string is that site, so the string has L^3 / 2 bits, its Metropolis
// field is field b mod 8 of Philox call b / 8, and a 32-bit word is four whole calls.  The
// neighbours of bit b are bits of the other colour's string:
//  - x: bit b itself on one side; bit b + 1 (x + 1, sigma = 1) or b - 1 (x - 1, sigma = 0) on the
//    other, wrapping within the row (b - (L/2 - 1) and b + (L/2 - 1));
//  - y: bits b + L/2 and b - L/2, wrapping within the plane (b -+ (L - 1) L / 2);
//  - z: bits b + L^2/2 and b - L^2/2, wrapping around the string.
// So every neighbour word is a funnel shift of two words of the other string by a constant, and
// the in-row and in-plane wraps are bit selects by per-word masks.  The strings are kept in LDS
// with a few ghost words on both sides holding the string's periodic continuation (refreshed after
// each colour phase), so the z wraps need no selects and no funnel leaves the buffer.
//
// One lane per replica: a wave holds one 64-replica bit-packed group (a block holds four, sharing
// the first-look bound table) and walks the words of a colour in step, so each word's Philox call indices are the same over the wave and the first
// rounds of the generator run on the scalar unit.  The decision step (bond count, packed first
// look, tie paths) is the one of the L = 16 colour-packed kernel.
#include <algorithm>
#include <type_traits>

#include "pa_common.h"
#include "pa_sweep_util.h"
#include "pa_sweep_words.h"

namespace pa {

namespace strings {

using namespace words;

template <int L>
struct Geo {
    static constexpr int H2 = L / 2;              // colour sites per row
    static constexpr int NP = L * L / 2;          // bits per plane
    static constexpr int NH = L * NP;             // bits per string
    static constexpr int NW = (NH + 31) / 32;     // words per string
    static constexpr int G = NP / 32 + 1;         // ghost words on each side: a funnel by up to
                                                  // NP bits reads words k - G .. k + G
    static constexpr int EW = NW + 2 * G;         // words of an extended string
    static constexpr int NR = L * L;              // lattice rows per replica
    static constexpr int WB = L <= 8 ? 1 : 2;     // bytes of a bit-packed row
    static constexpr int TW = 12;                 // table dwords per (colour, word)
    static constexpr uint32_t LAST = NH % 32 ? (1u << (NH % 32)) - 1u : 0xFFFFFFFFu;  // valid bits of the last word
};

// offset of extended-string word e (0 .. EW - 1) inside the string: 32 (e - G) mod NH, taken
// non-negative; a ghost word holds the 32 string bits from there on
template <int L>
__host__ __device__ constexpr int ghost_origin(int e)
{
    using Gm = Geo<L>;
    return ((32 * (e - Gm::G)) % Gm::NH + Gm::NH) % Gm::NH;
}

// every ghost word is a funnel of string words that exist (so the refresh reads no ghost)
template <int L>
constexpr bool ghosts_in_string()
{
    using Gm = Geo<L>;
    for (int e = 0; e < Gm::EW; ++e) {
        if (e >= Gm::G && e < Gm::G + Gm::NW) continue;
        const int o = ghost_origin<L>(e);
        if (o % 32 == 0 ? o / 32 >= Gm::NW : o / 32 + 1 >= Gm::NW) return false;
    }
    return true;
}

// LDS of one wave: the two extended strings (word-major, replica-minor, so the 64 lanes of a word
// load hit 64 banks) and per (colour, word) the coupling masks and geometry masks
template <int L>
struct WaveSmem {
    uint32_t E[2 * Geo<L>::EW * 64];
    uint32_t tab[2 * Geo<L>::NW * Geo<L>::TW];
};

// a block: WPB waves, each sweeping its own 64-replica groups, and the bound table, which depends
// only on the step's thresholds and so serves every wave (whichever run its group belongs to)
constexpr int WPB = 4;
template <int L>
struct Smem {
    WaveSmem<L> w[WPB];
    uint2 tt[256];
};

// the block's bound table, before any wave sweeps (every thread of the block reaches the barrier)
template <int MODE>
__device__ __forceinline__ void block_bounds(uint2* tt, const Thr& th)
{
    if (MODE != 2) build_bounds(tt, th, threadIdx.x, blockDim.x);
    __syncthreads();
}

// word q of the other string relative to word k, shifted by off bits (funnel of two words)
template <int OFF>
__device__ __forceinline__ uint32_t funnel(const uint32_t* Ok)
{
    constexpr int q = OFF >= 0 ? OFF / 32 : -((-OFF + 31) / 32);  // floor(OFF / 32)
    constexpr int r = OFF - 32 * q;
    const uint32_t lo = Ok[q * 64];
    if constexpr (r == 0) {
        return lo;
    } else {
        const uint32_t hi = Ok[(q + 1) * 64];
        return __builtin_amdgcn_alignbit(hi, lo, r);
    }
}

// The per-word tables, built by the wave: lanes 0..31 take bit t of word k of colour 0, lanes 32..63
// the same bit of colour 1, and a ballot of each flag gives the two words at once.  Entries: 0..5
// the coupling masks (bit set where J = -1) of the +x, -x, +y, -y, +z, -z bonds, 6 the sites with
// x even (sigma = 0), 7 and 8 the first and last site of a row (m = 0, m = L/2 - 1), 9 and 10 the
// first and last row of a plane (y = 0, y = L - 1), 11 the bits that are sites (b < L^3 / 2).
template <int L>
__device__ void build_tables(const int8_t* J, uint32_t* tab, int lane)
{
    using Gm = Geo<L>;
    const int c = lane >> 5, t = lane & 31;
    for (int k = 0; k < Gm::NW; ++k) {
        const int b = 32 * k + t;
        bool f[12] = {false, false, false, false, false, false, false, false, false, false, false, false};
        if (b < Gm::NH) {
            const int m = b % Gm::H2, r = b / Gm::H2, y = r % L, z = r / L;
            const int sg = (c + y + z) & 1, x = 2 * m + sg;
            const int xm = (x + L - 1) % L, ym = (y + L - 1) % L, zm = (z + L - 1) % L;
            const int i = x + L * (y + L * z);
            f[0] = J[3 * i + 0] < 0;
            f[1] = J[3 * (xm + L * (y + L * z)) + 0] < 0;
            f[2] = J[3 * i + 1] < 0;
            f[3] = J[3 * (x + L * (ym + L * z)) + 1] < 0;
            f[4] = J[3 * i + 2] < 0;
            f[5] = J[3 * (x + L * (y + L * zm)) + 2] < 0;
            f[6] = sg == 0;
            f[7] = m == 0;
            f[8] = m == Gm::H2 - 1;
            f[9] = y == 0;
            f[10] = y == L - 1;
            f[11] = true;
        }
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const uint64_t v = __ballot(f[e]);
            if (lane == 0) {
                tab[(0 * Gm::NW + k) * Gm::TW + e] = (uint32_t)v;
                tab[(1 * Gm::NW + k) * Gm::TW + e] = (uint32_t)(v >> 32);
            }
        }
    }
}

// the string's periodic continuation into the last word's unused bits and the ghost words (S: the
// string's extended words, this lane's column)
template <int L>
__device__ __forceinline__ void refresh_ghosts(uint32_t* S)
{
    using Gm = Geo<L>;
    static_assert(ghosts_in_string<L>(), "ghost words must come from string words");
    if constexpr (Gm::NH % 32 != 0) {
        constexpr int last = Gm::G + Gm::NW - 1;
        S[last * 64] = select_bits(Gm::LAST, S[last * 64], S[Gm::G * 64] << (Gm::NH % 32));
    }
#pragma unroll
    for (int e = 0; e < Gm::EW; ++e) {
        if (e >= Gm::G && e < Gm::G + Gm::NW) continue;
        const int o = ghost_origin<L>(e), q = Gm::G + o / 32, r = o % 32;
        S[e * 64] = r == 0 ? S[q * 64] : __builtin_amdgcn_alignbit(S[(q + 1) * 64], S[q * 64], r);
    }
}

// the six neighbour words of word k of a colour (Ok: word k of the other string, T: the word's
// table entry)
template <int L>
__device__ __forceinline__ void neighbours(const uint32_t* Ok, const uint32_t* T, uint32_t nb[6])
{
    using Gm = Geo<L>;
    constexpr int H2 = Gm::H2, NP = Gm::NP;
    const uint32_t a0 = Ok[0];
    const uint32_t sig0 = T[6], rf = T[7], rl = T[8], yf = T[9], yl = T[10];
    nb[0] = select_bits(sig0, a0, select_bits(rl, funnel<-(H2 - 1)>(Ok), funnel<1>(Ok)));
    nb[1] = select_bits(sig0, select_bits(rf, funnel<H2 - 1>(Ok), funnel<-1>(Ok)), a0);
    nb[2] = select_bits(yl, funnel<H2 - NP>(Ok), funnel<H2>(Ok));
    nb[3] = select_bits(yf, funnel<NP - H2>(Ok), funnel<-H2>(Ok));
    nb[4] = funnel<NP>(Ok);
    nb[5] = funnel<-NP>(Ok);
}

// rows of the lane's replica (replica g 64 + lane of the run) between HBM and its two strings
template <int L, bool STORE>
__device__ __forceinline__ void replica_io(const pa_state* st, int64_t g, int lane, uint32_t* E0, uint32_t* E1,
                                           bool write)
{
    using Gm = Geo<L>;
    constexpr int H2 = Gm::H2, G = Gm::G;
    constexpr uint32_t HM = (1u << H2) - 1u;
    uint8_t* base = (uint8_t*)st->spins[st->cur] + (g * Gm::NR * 64 + lane) * Gm::WB;
    if (!STORE) {
        uint32_t s0[Gm::NW], s1[Gm::NW];
#pragma unroll
        for (int k = 0; k < Gm::NW; ++k) s0[k] = s1[k] = 0;
#pragma unroll
        for (int r = 0; r < Gm::NR; ++r) {
            const uint8_t* a = base + (int64_t)r * 64 * Gm::WB;
            const uint32_t v = Gm::WB == 1 ? (uint32_t)*a : (uint32_t)*(const uint16_t*)a;
            uint32_t odd;
            const uint32_t even = split_colours(v, &odd) & HM;
            odd &= HM;
            const int y = r % L, z = r / L, b0 = H2 * r, k0 = b0 / 32, sh = b0 % 32;
            // colour 0 takes x = 2 m + (y + z) mod 2
            const uint32_t c0 = ((y + z) & 1) ? odd : even, c1 = ((y + z) & 1) ? even : odd;
            s0[k0] |= c0 << sh;
            s1[k0] |= c1 << sh;
            if (sh + H2 > 32) {
                s0[k0 + 1] |= c0 >> (32 - sh);
                s1[k0 + 1] |= c1 >> (32 - sh);
            }
        }
#pragma unroll
        for (int k = 0; k < Gm::NW; ++k) {
            E0[(G + k) * 64] = s0[k];
            E1[(G + k) * 64] = s1[k];
        }
    } else {
        uint32_t s0[Gm::NW], s1[Gm::NW];
#pragma unroll
        for (int k = 0; k < Gm::NW; ++k) {
            s0[k] = E0[(G + k) * 64];
            s1[k] = E1[(G + k) * 64];
        }
        if (!write) return;
#pragma unroll
        for (int r = 0; r < Gm::NR; ++r) {
            const int y = r % L, z = r / L, b0 = H2 * r, k0 = b0 / 32, sh = b0 % 32;
            uint32_t c0 = s0[k0] >> sh, c1 = s1[k0] >> sh;
            if (sh + H2 > 32) {
                c0 |= s0[k0 + 1] << (32 - sh);
                c1 |= s1[k0 + 1] << (32 - sh);
            }
            c0 &= HM;
            c1 &= HM;
            const uint32_t even = ((y + z) & 1) ? c1 : c0, odd = ((y + z) & 1) ? c0 : c1;
            const uint32_t v = merge_colours(even, odd);
            uint8_t* a = base + (int64_t)r * 64 * Gm::WB;
            if (Gm::WB == 1) *a = (uint8_t)v;
            else *(uint16_t*)a = (uint16_t)v;
        }
    }
}

// N_S sweeps of the 64 replicas of bit-packed group g of one run (one wave; every lane reaches the
// end, those past R only skip their stores)
template <int L, int MODE>
__device__ __forceinline__ void sweep_group(const pa_state* st, int64_t g, WaveSmem<L>& sm, const uint2* tt,
                                            int lane, const SweepParams& p, const Thr& th)
{
    using Gm = Geo<L>;
    constexpr int G = Gm::G, EW = Gm::EW, NW = Gm::NW, TW = Gm::TW;
    build_tables<L>(st->J, sm.tab, lane);
    uint32_t* E0 = sm.E + lane;
    uint32_t* E1 = sm.E + EW * 64 + lane;
    replica_io<L, false>(st, g, lane, E0, E1, false);
    refresh_ghosts<L>(E0);
    refresh_ghosts<L>(E1);
    wave_sync();  // the tables were written by lane 0

    const int64_t R = st->R, r = g * 64 + lane;
    Lane c;
    c.rr = (uint32_t)r;
    c.k0 = (uint32_t)st->seed;
    c.k1 = (uint32_t)(st->seed >> 32);
    for (int s = 0; s < p.n_sweeps; ++s) {
        for (int col = 0; col < 2; ++col) {
            c.ctr2 = (uint32_t)(2 * (p.t0 + s) + col);
            uint32_t* W = col ? E1 : E0;
            const uint32_t* O = col ? E0 : E1;
            auto word = [&](int k, auto nbytes) {
                const uint32_t* T = sm.tab + (col * NW + k) * TW;
                const uint32_t w = W[(G + k) * 64];
                uint32_t nb[6];
                neighbours<L>(O + (G + k) * 64, T, nb);
                uint32_t c0, c1, c2;
                bond_count(xor3(w, nb[0], T[0]), xor3(w, nb[1], T[1]), xor3(w, nb[2], T[2]), xor3(w, nb[3], T[3]),
                           xor3(w, nb[4], T[4]), xor3(w, nb[5], T[5]), c0, c1, c2);
                c2 &= T[11];  // bits past the string are no candidates
                const uint32_t call0 = 4u * (uint32_t)k;
                const uint32_t nw = decide_word<MODE, true, decltype(nbytes)::value>(w, c0, c1, c2, call0, 1u, tt, c, th,
                                                                                     [&]() {
                    // bit b is half-site 32 k + b: site 2 (32 k + b) + sigma
                    return WordSites{call0, 1u, 64u * (uint32_t)k, 16u, ~T[6] & T[11]};
                });
                W[(G + k) * 64] = nw;
            };
            // a partial last word draws only the calls of its bytes with sites
            constexpr int LASTB = (Gm::NH % 32 + 7) / 8;
            constexpr int FULL = LASTB == 0 ? NW : NW - 1;
#pragma unroll 1
            for (int k = 0; k < FULL; ++k) word(k, std::integral_constant<int, 4>{});
            if constexpr (LASTB != 0) word(NW - 1, std::integral_constant<int, LASTB>{});
            refresh_ghosts<L>(W);
        }
    }

    // energy: every bond joins a colour-0 and a colour-1 site, so the six bonds of the colour-0
    // sites count each bond once.  E = n_bonds - 2 (bonds whose word bit is set)
    int neg = 0;
#pragma unroll 1
    for (int k = 0; k < NW; ++k) {
        const uint32_t* T = sm.tab + k * TW;
        const uint32_t w = E0[(G + k) * 64];
        uint32_t nb[6];
        neighbours<L>(E1 + (G + k) * 64, T, nb);
        uint32_t any = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) neg += __popc(xor3(w, nb[d], T[d]) & T[11]);
        (void)any;
    }
    const bool valid = r < R;
    if (valid) st->energy[st->cur][r] = st->n_bonds - 2 * neg;
    replica_io<L, true>(st, g, lane, E0, E1, valid);
    wave_sync();  // the next item of a persistent wave reuses this LDS
}

// ------------------------------------------------------------------ one run: one group per wave
template <int L, int MODE>
__global__ void __launch_bounds__(64 * WPB) k_sweep_cs(const pa_state* __restrict__ st, SweepParams p, Thr th)
{
    __shared__ Smem<L> sm;
    if (st->status) return;  // sticky error: the population stays as it is
    block_bounds<MODE>(sm.tt, th);
    const int wave = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * WPB + wave;
    if (g * 64 >= st->R) return;
    sweep_group<L, MODE>(st, g, sm.w[wave], sm.tt, threadIdx.x & 63, p, th);
}

// ------------------------------------------------------------------ a batch of runs
// Items (run, 64-replica group) laid out by k_batch_tiles; in the persistent form every wave takes
// items from the group's work counter, in the grid form wave w of block b takes item WPB b + w.
__device__ __forceinline__ int find_run(const int64_t* tb, int pos0, int pos1, int64_t item)
{
    int lo = pos0, hi = pos1;  // tb[lo] <= item < tb[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tb[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int L, int MODE>
__global__ void __launch_bounds__(64 * WPB) k_sweep_cs_batch(pa_state* base, int pos0, int pos1, BatchOrder order,
                                                             SweepParams p, Thr th)
{
    __shared__ Smem<L> sm;
    block_bounds<MODE>(sm.tt, th);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t* tb = work_ptr<int64_t>(base, work_layout(base->N, base->n_bins, base->capacity).batch);
    const int64_t first = tb[pos0], total = tb[pos1] - first;
    pa_state* counter = base + order.run[pos0];
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&counter->work_counter, 1u);
        // lane 0's item, as a scalar: the run's state (its seed, hence the Philox keys) and the
        // item's group index then stay wave-uniform, and the generator's uniform rounds run on the
        // scalar unit
        t = __builtin_amdgcn_readfirstlane(t);
        if ((int64_t)t >= total) break;  // every wave leaves once the group's items are taken
        const int64_t item = first + (int64_t)t;
        const int lo = __builtin_amdgcn_readfirstlane(find_run(tb, pos0, pos1, item));
        sweep_group<L, MODE>(base + order.run[lo], item - tb[lo], sm.w[wave], sm.tt, lane, p, th);
    }
}

template <int L, int MODE>
__global__ void __launch_bounds__(64 * WPB) k_sweep_cs_batch_grid(pa_state* base, int pos0, int pos1,
                                                                  BatchOrder order, SweepParams p, Thr th)
{
    __shared__ Smem<L> sm;
    block_bounds<MODE>(sm.tt, th);
    const int wave = threadIdx.x >> 6;
    const int64_t* tb = work_ptr<int64_t>(base, work_layout(base->N, base->n_bins, base->capacity).batch);
    const int64_t item = tb[pos0] + (int64_t)blockIdx.x * WPB + wave;
    if (item >= tb[pos1]) return;
    const int lo = __builtin_amdgcn_readfirstlane(find_run(tb, pos0, pos1, item));
    sweep_group<L, MODE>(base + order.run[lo], item - tb[lo], sm.w[wave], sm.tt, threadIdx.x & 63, p, th);
}

template <int L>
static int launch_solo(const pa_run& run, const SweepParams& p, const Thr& th, hipStream_t s)
{
    const int64_t blocks = (run.capacity / 64 + WPB - 1) / WPB;
    if (blocks <= 0) return PA_OK;
    if (all_tops_zero(th))
        hipLaunchKernelGGL((k_sweep_cs<L, 2>), dim3((unsigned)blocks), dim3(64 * WPB), 0, s, run.state, p, th);
    else
        hipLaunchKernelGGL((k_sweep_cs<L, 0>), dim3((unsigned)blocks), dim3(64 * WPB), 0, s, run.state, p, th);
    return PA_OK;
}

// waves: the persistent form's number of waves, or the grid form's number of items
template <int L>
static void launch_batch(pa_state* base, int pos0, int pos1, const BatchOrder& order, const SweepParams& p,
                         const Thr& th, bool persistent, int64_t waves, hipStream_t s)
{
    const dim3 g((unsigned)std::max<int64_t>(1, (waves + WPB - 1) / WPB)), b(64 * WPB);
    const bool z = all_tops_zero(th);
    if (persistent) {
        if (z) hipLaunchKernelGGL((k_sweep_cs_batch<L, 2>), g, b, 0, s, base, pos0, pos1, order, p, th);
        else hipLaunchKernelGGL((k_sweep_cs_batch<L, 0>), g, b, 0, s, base, pos0, pos1, order, p, th);
    } else {
        if (z) hipLaunchKernelGGL((k_sweep_cs_batch_grid<L, 2>), g, b, 0, s, base, pos0, pos1, order, p, th);
        else hipLaunchKernelGGL((k_sweep_cs_batch_grid<L, 0>), g, b, 0, s, base, pos0, pos1, order, p, th);
    }
}

}  // namespace strings

// one run; PA_ERR_ARG when the run or the thresholds are not ones the kernel handles
int launch_sweep_strings(const pa_run& run, const SweepParams& p, hipStream_t s)
{
    if (!string_sweep_supported(run.dim, run.L, run.layout) || !fast_sweep_thresholds_ok(p)) return PA_ERR_ARG;
    const words::Thr th = words::make_thr(p);
    switch (run.L) {
        case 4: return strings::launch_solo<4>(run, p, th, s);
        case 6: return strings::launch_solo<6>(run, p, th, s);
        case 8: return strings::launch_solo<8>(run, p, th, s);
        default: return strings::launch_solo<10>(run, p, th, s);
    }
}

// one group of equal-L runs of a batch (positions pos0 .. pos1 - 1 of the order): persistent
// (waves taking items) or one item per wave (waves = the group's items)
int launch_sweep_strings_group(int L, pa_state* base, int pos0, int pos1, const BatchOrder& order,
                               const SweepParams& p, bool persistent, int64_t waves, hipStream_t s)
{
    if (!fast_sweep_thresholds_ok(p)) return PA_ERR_ARG;
    const words::Thr th = words::make_thr(p);
    switch (L) {
        case 4: strings::launch_batch<4>(base, pos0, pos1, order, p, th, persistent, waves, s); break;
        case 6: strings::launch_batch<6>(base, pos0, pos1, order, p, th, persistent, waves, s); break;
        case 8: strings::launch_batch<8>(base, pos0, pos1, order, p, th, persistent, waves, s); break;
        case 10: strings::launch_batch<10>(base, pos0, pos1, order, p, th, persistent, waves, s); break;
        default: return PA_ERR_ARG;
    }
    return PA_OK;
}

}  // namespace pa
