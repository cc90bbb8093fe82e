// Gaussian couplings (the model of Sec. IV: J_ij normal with mean 0 and variance 1).
// Energies are real numbers, so the path fixes every floating-point step in order and in the
// operations used: couplings drawn on the host (Box-Muller, libm), energies summed in bond order
// and recomputed after every call of sweeps, local fields summed in incident-bond order, the
// acceptance probability floor(expd(-beta dE) 2^64) / 2^64 with exp written out (expd), and no
// fused multiply-adds.  Population layout: one byte per spin.
#include <math.h>
#include <string.h>

#include <vector>

#include "pa_common.h"
#include "pa_lattice.h"
#include "pa_sweep_words.h"

#pragma clang fp contract(off)

namespace pa {

// ------------------------------------------------------------------ host: couplings
// Philox4x32-10 (Salmon et al., SC'11), host side
static void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// J_b = sqrt(-2 ln u1) cos(2 pi u2) from Philox(ctr (b, 0, 0, 6), key disorder seed): u1 from
// the top 27 + 26 bits of words 0, 1 (plus one, so u1 > 0), u2 from words 2, 3
int gauss_couplings_upload(const pa_run& run, hipStream_t s)
{
    const int64_t B = run.dim == 1 ? run.L : 3 * (int64_t)run.L * run.L * run.L;
    std::vector<double> J((size_t)B);
    const uint32_t k0 = (uint32_t)run.disorder_seed, k1 = (uint32_t)(run.disorder_seed >> 32);
    for (int64_t b = 0; b < B; ++b) {
        uint32_t w[4] = {(uint32_t)b, 0u, 0u, 6u};
        philox_host(w, k0, k1);
        const uint64_t m1 = ((uint64_t)(w[0] >> 5) << 26) | (uint64_t)(w[1] >> 6);
        const uint64_t m2 = ((uint64_t)(w[2] >> 5) << 26) | (uint64_t)(w[3] >> 6);
        const double u1 = ldexp((double)(m1 + 1), -53);
        const double u2 = ldexp((double)m2, -53);
        J[(size_t)b] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
    // synchronous: the host vector is released on return
    if (hipMemcpyAsync(run.J, J.data(), (size_t)B * 8, hipMemcpyHostToDevice, s) != hipSuccess) return PA_ERR_HIP;
    return hip_status(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ device helpers
__device__ inline int gauss_colour(const pa_state* st, int i)
{
    if (st->dim == 1) return i & 1;
    const int L = st->L;
    return ((i % L) + (i / L) % L + i / (L * L)) & 1;
}

// E = sum over bonds b = 0, 1, ... of J_b s_i s_j, in bond order from 0 (s = 1 means sigma = -1)
__device__ double energy_gauss(const pa_state* st, const uint8_t* s)
{
    const double* J = reinterpret_cast<const double*>(st->J);
    const int N = st->N, L = st->L;
    double E = 0.0;
    if (st->dim == 1) {
        for (int i = 0; i < N; ++i) {
            const int j = i + 1 == N ? 0 : i + 1;
            E = E + ((s[i] ^ s[j]) ? -J[i] : J[i]);
        }
    } else {
        for (int i = 0; i < N; ++i) {
            int nb[3];
            plus_neighbours3(i, L, nb);
            for (int a = 0; a < 3; ++a) E = E + ((s[i] ^ s[nb[a]]) ? -J[3 * i + a] : J[3 * i + a]);
        }
    }
    return E;
}

// thread per replica
__global__ void __launch_bounds__(64) k_energy_gauss(const pa_state* __restrict__ st, int buf, int64_t n)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint8_t* s = (const uint8_t*)st->spins[buf] + r * st->row_stride;
    reinterpret_cast<double*>(st->energy[buf])[r] = energy_gauss(st, s);
}

// N_S checkerboard sweeps of one replica per thread; the draws are those of the +-1 path
__global__ void __launch_bounds__(64) k_sweep_gauss(const pa_state* __restrict__ st, double beta, int64_t t0, int ns)
{
    if (st->status) return;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= st->R) return;
    const int N = st->N, L = st->L, dim = st->dim;
    const double* J = reinterpret_cast<const double*>(st->J);
    uint8_t* s = (uint8_t*)st->spins[st->cur] + r * st->row_stride;
    const uint32_t k0 = (uint32_t)st->seed, k1 = (uint32_t)(st->seed >> 32), rr = (uint32_t)r;
    for (int64_t t = t0; t < t0 + ns; ++t) {
        for (int col = 0; col < 2; ++col) {
            const uint32_t ctr2 = (uint32_t)(2 * t + col);
            int cached = -1;
            uint4v v = {0, 0, 0, 0};
            for (int i = 0; i < N; ++i) {
                if (gauss_colour(st, i) != col) continue;
                // local field, incident bonds in the order +x, +y, +z, -x, -y, -z (chain: +1, -1)
                double h = 0.0;
                if (dim == 1) {
                    const int ip = i + 1 == N ? 0 : i + 1, im = i == 0 ? N - 1 : i - 1;
                    h = h + (s[ip] ? -J[i] : J[i]);
                    h = h + (s[im] ? -J[im] : J[im]);
                } else {
                    int nb[3];
                    plus_neighbours3(i, L, nb);
                    const int x = i % L, y = (i / L) % L, z = i / (L * L);
                    const int m[3] = {(x == 0 ? L - 1 : x - 1) + L * (y + L * z), x + L * ((y == 0 ? L - 1 : y - 1) + L * z),
                                      x + L * (y + L * (z == 0 ? L - 1 : z - 1))};
                    for (int a = 0; a < 3; ++a) h = h + (s[nb[a]] ? -J[3 * i + a] : J[3 * i + a]);
                    for (int a = 0; a < 3; ++a) h = h + (s[m[a]] ? -J[3 * m[a] + a] : J[3 * m[a] + a]);
                }
                const double dE = s[i] ? 2.0 * h : -2.0 * h;
                bool accept = dE <= 0.0;
                if (!accept) {
                    const double p = expd(-(beta * dE));
                    if (p >= 1.0) {
                        accept = true;
                    } else {
                        const uint64_t T64 = (uint64_t)ldexp(p, 64);
                        const int hh = i >> 1;
                        if ((hh >> 3) != cached) {
                            cached = hh >> 3;
                            v = philox10((uint32_t)cached, rr, ctr2, kTagMet, k0, k1);
                        }
                        const uint32_t u16 = (word_of(v, (hh & 7) >> 1) >> (16 * (hh & 1))) & 0xFFFFu;
                        const uint32_t thi = (uint32_t)(T64 >> 48);
                        if (u16 != thi) {
                            accept = u16 < thi;
                        } else {
                            const uint4v w = philox10((uint32_t)i, rr, ctr2, kTagTie, k0, k1);
                            const uint64_t U = ((uint64_t)u16 << 48) | (uint64_t)w.x | ((uint64_t)(w.y & 0xFFFFu) << 32);
                            accept = U < T64;
                        }
                    }
                }
                if (accept) s[i] ^= 1;
            }
        }
    }
    if (ns > 0) reinterpret_cast<double*>(st->energy[st->cur])[r] = energy_gauss(st, s);
}

// ------------------------------------------------------------------ tabled sweep
// The same sweeps with lane = replica and a wave of 64 replicas.  Each lane keeps its spins as
// 16-site segments in LDS (bit j of segment m is site 16m + j), so the neighbour bits of a whole
// segment come from a few shifts of at most five segment words.
//
// dE of an attempt depends only on the site and on the pattern b of the bits s_j xor s_i of
// its neighbours in field order: flipping every spin negates each term of h exactly, hence h,
// and leaves dE unchanged.  Per call, k_gauss_table tabulates for every site and pattern
// T64 = floor(p 2^64) with p = expd(-(beta dE)) computed as in k_sweep_gauss (s_i = 0, s_j = bit
// of b), or all ones where the flip is always accepted (dE <= 0 or p >= 1; a p below 1 gives at
// most 2^64 - 2^11), and its top T16 = T64 >> 48.  An attempt compares its 16-bit draw u with T16:
// u < T16 accepts, u > T16 rejects, and u == T16 (rare) compares the 64-bit draw with T64, as
// k_sweep_gauss does (always accepting where T64 is all ones).  The outcome of every attempt is
// therefore the same as there.
//
// Table layout (after the work layout): u16 [colour c][segment m][pattern b][k], k = 0..7 the
// sites of colour c in segment m in ascending order.  Site i of colour c has h = i >> 1 = 8m + k
// (rows have even length, so exactly one of 2h, 2h + 1 has colour c).  The lanes of a wave work on
// the same segment at the same time, so lane b loads the 16-byte row [c][m][b]: one coalesced 1 KB
// load per segment whose address does not depend on the spins, issued a step ahead.  Each
// attempt then takes its entry from lane b = its pattern with ds_bpermute, a lane-to-lane read at
// the latency of LDS, instead of a gather from the cache at the latency of memory.  The u64 table of
// T64 follows in the same order.

constexpr int kGaussWaves = 4;

// h of site i for neighbour pattern b (bit a: neighbour a in field order has s_j != s_i); LC: the
// cube side as a constant (its divisions become shifts), 0 for L at run time
template <int NB, int LC = 0>
__device__ double gauss_field_pattern(const double* __restrict__ J, int i, int b, int L_rt, int N)
{
    const int L = LC ? LC : L_rt;
    double h = 0.0;
    if constexpr (NB == 2) {
        const int im = i == 0 ? N - 1 : i - 1;
        h = h + ((b & 1) ? -J[i] : J[i]);
        h = h + ((b & 2) ? -J[im] : J[im]);
    } else {
        const int x = i % L, y = (i / L) % L, z = i / (L * L);
        const int m[3] = {(x == 0 ? L - 1 : x - 1) + L * (y + L * z), x + L * ((y == 0 ? L - 1 : y - 1) + L * z),
                          x + L * (y + L * (z == 0 ? L - 1 : z - 1))};
        for (int a = 0; a < 3; ++a) h = h + (((b >> a) & 1) ? -J[3 * i + a] : J[3 * i + a]);
        for (int a = 0; a < 3; ++a) h = h + (((b >> (3 + a)) & 1) ? -J[3 * m[a] + a] : J[3 * m[a] + a]);
    }
    return h;
}

// true if the flip is always accepted; otherwise *T64 = floor(p 2^64) with p < 1 (s_i = 0)
__device__ inline bool gauss_threshold(double h, double beta, uint64_t* T64)
{
    const double dE = -2.0 * h;
    if (dE <= 0.0) return true;
    const double p = expd(-(beta * dE));
    if (p >= 1.0) return true;
    *T64 = (uint64_t)ldexp(p, 64);
    return false;
}

__device__ __forceinline__ uint16_t* gauss_table(const pa_state* st)
{
    return reinterpret_cast<uint16_t*>(st->work + work_layout(st->N, st->n_bins, st->capacity).total);
}

// the u64 table of full thresholds, after the NB-pattern u16 table (8-byte aligned)
template <int NB>
__device__ __forceinline__ uint64_t* gauss_table64(const pa_state* st)
{
    return reinterpret_cast<uint64_t*>(gauss_table(st) + ((size_t)st->N << NB));
}

// grid (entries / 256, runs): entry e = (c, m, b, k) of run blockIdx.y; LC as in gauss_field_pattern
template <int NB, int LC>
__global__ void __launch_bounds__(256) k_gauss_table(pa_state* __restrict__ states, double beta)
{
    const pa_state* st = states + blockIdx.y;
    if (st->status) return;
    const int N = st->N, L = LC ? LC : st->L;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (N << NB)) return;
    const int half = (N / 2) << NB;
    const int c = e >= half, rem = e - c * half;
    const int b = (rem >> 3) & ((1 << NB) - 1), hh = 8 * (rem >> (NB + 3)) + (rem & 7);
    const int i0 = 2 * hh;
    const int col0 = NB == 2 ? 0 : ((i0 % L) + (i0 / L) % L + i0 / (L * L)) & 1;
    const int i = i0 + (col0 != c);
    uint64_t T64 = 0;
    const bool always = gauss_threshold(gauss_field_pattern<NB, LC>(reinterpret_cast<const double*>(st->J), i, b, L, N),
                                        beta, &T64);
    if (always) T64 = ~0ull;
    gauss_table(st)[e] = (uint16_t)(T64 >> 48);
    gauss_table64<NB>(st)[e] = T64;
}

__device__ __forceinline__ uint32_t bytes_to_bits4(uint32_t w)  // bytes b0..b3 in {0,1} -> b0 | b1<<1 | ...
{
    return (w * 0x10204080u) >> 28;
}

__device__ __forceinline__ uint32_t bits4_to_bytes(uint32_t n)  // inverse of bytes_to_bits4
{
    return (n * 0x00204081u) & 0x01010101u;
}

// A lane's segments in LDS: segments 2p and 2p + 1 are the low and high halves of the lane's
// 32-bit word of pair p, and the words of a wave's 64 lanes lie side by side ([pair][lane]), so a
// pair is one ds_read_b32 without bank conflicts.  seg points at the lane's word of pair 0.
__device__ __forceinline__ uint16_t& seg_at(uint16_t* seg, int m)
{
    return seg[(m >> 1) * 128 + (m & 1)];
}

__device__ __forceinline__ uint32_t pair_at(const uint16_t* seg, int p)
{
    return *reinterpret_cast<const uint32_t*>(seg + p * 128);
}

__device__ __forceinline__ void pair_store(uint16_t* seg, int p, uint32_t w)
{
    *reinterpret_cast<uint32_t*>(seg + p * 128) = w;
}

// the colour parity of segment m's first site (chain: 0; cube: (q * rows per segment + z) & 1 of
// its segment q in z plane z)
template <int NB, int L>
__device__ __forceinline__ int gauss_segment_parity(int m)
{
    if constexpr (NB == 2) {
        return 0;
    } else {
        constexpr int SP = L * L / 16, NR = 16 / L;
        const int z = m / SP, q = m - z * SP;
        return (q * NR + z) & 1;
    }
}

// the neighbour words of segment m in field order, each xor the segment itself
template <int NB, int L>
__device__ __forceinline__ void gauss_segment_words(uint16_t* __restrict__ seg, int m, int nseg, uint32_t D,
                                                    uint32_t X[NB], int* par)
{
    if constexpr (NB == 2) {
        const uint32_t Sn = seg_at(seg, m + 1 == nseg ? 0 : m + 1);
        const uint32_t Sp = seg_at(seg, m == 0 ? nseg - 1 : m - 1);
        X[0] = (((D >> 1) | (Sn << 15)) & 0xFFFFu) ^ D;
        X[1] = (((D << 1) | (Sp >> 15)) & 0xFFFFu) ^ D;
        *par = 0;
    } else {
        constexpr int SP = L * L / 16;  // segments per z plane
        constexpr int NR = 16 / L;      // rows per segment
        constexpr uint32_t Mhi = L == 4 ? 0x8888u : 0x8080u;  // x = L - 1
        constexpr uint32_t Mlo = L == 4 ? 0x1111u : 0x0101u;  // x = 0
        const int z = m / SP, q = m - z * SP;
        const uint32_t Sn = seg_at(seg, z * SP + (q + 1 == SP ? 0 : q + 1));
        const uint32_t Sp = seg_at(seg, z * SP + (q == 0 ? SP - 1 : q - 1));
        const uint32_t Sz = seg_at(seg, (z + 1 == L ? 0 : z + 1) * SP + q);
        const uint32_t Szm = seg_at(seg, (z == 0 ? L - 1 : z - 1) * SP + q);
        X[0] = (((D >> 1) & ~Mhi) | ((D << (L - 1)) & Mhi)) ^ D;
        X[1] = (((D >> L) | (Sn << (16 - L))) & 0xFFFFu) ^ D;
        X[2] = Sz ^ D;
        X[3] = (((D << 1) & ~Mlo & 0xFFFFu) | ((D >> (L - 1)) & Mlo)) ^ D;
        X[4] = (((D << L) | (Sp >> (16 - L))) & 0xFFFFu) ^ D;
        X[5] = Szm ^ D;
        *par = gauss_segment_parity<NB, L>(m);
    }
}

// Cube side 8: the neighbour words of pair p (four x rows of one z plane, segments 2p and 2p + 1 in
// the low and high halves), each xor the pair itself, formed on whole 32-bit words.  The plane's
// other pair So holds the rows on both y sides.
__device__ __forceinline__ void gauss_pair_words8(const uint16_t* __restrict__ seg, int p, uint32_t D2, uint32_t So,
                                                  uint32_t X[6])
{
    const int z = p >> 1, h = p & 1;  // two pairs per plane
    const uint32_t Sz = pair_at(seg, 2 * (z == 7 ? 0 : z + 1) + h);
    const uint32_t Szm = pair_at(seg, 2 * (z == 0 ? 7 : z - 1) + h);
    constexpr uint32_t Mhi = 0x80808080u, Mlo = 0x01010101u;  // x = 7, x = 0 in each row byte
    X[0] = (((D2 >> 1) & ~Mhi) | ((D2 << 7) & Mhi)) ^ D2;
    X[1] = ((D2 >> 8) | (So << 24)) ^ D2;
    X[2] = Sz ^ D2;
    X[3] = (((D2 << 1) & ~Mlo) | ((D2 >> 7) & Mlo)) ^ D2;
    X[4] = ((D2 << 8) | (So >> 24)) ^ D2;
    X[5] = Szm ^ D2;
}

// Chains of an even number of segments: the neighbour words of pair p (sites 32 p .. 32 p + 31),
// each xor the pair itself, formed on whole 32-bit words (npair pairs, periodic)
__device__ __forceinline__ void gauss_pair_words_chain(const uint16_t* __restrict__ seg, int p, int npair, uint32_t D2,
                                                       uint32_t X[2])
{
    const uint32_t Sn = pair_at(seg, p + 1 == npair ? 0 : p + 1);
    const uint32_t Sp = pair_at(seg, p == 0 ? npair - 1 : p - 1);
    X[0] = ((D2 >> 1) | (Sn << 31)) ^ D2;
    X[1] = ((D2 << 1) | (Sp >> 31)) ^ D2;
}

// the k-th site (k = 0..7, ascending) of colour parity SEL inside a segment (chain: j & 1; cube:
// (x + y) & 1 of the site inside the segment)
template <int NB, int L, int SEL>
__host__ __device__ constexpr int seg_site(int k)
{
    int c = 0;
    for (int j = 0; j < 16; ++j) {
        const int cj = NB == 2 ? (j & 1) : (((j % L) + (j / L)) & 1);
        if (cj == SEL) {
            if (c == k) return j;
            ++c;
        }
    }
    return -1;
}

// ds_bpermute takes the source lane from bits 2..7 of its byte address and ignores the others.
// Shifted by a + 2, bit a of site j's pattern lies at bit j + a + 2, so acc >> j is a valid address
// for site j as long as no other site of acc has a bit in j + 2 .. j + NB + 1.  (For NB = 2, bits
// 4..7 may hold other sites' bits: lanes that agree mod 4 hold the same table row.)  The 8 sites of
// a segment are split greedily into chains of sites at least NB apart, and one and-or chain per
// chain builds its acc.  Evaluated at compile time.
template <int NB, int L, int SEL>
struct SegPlan {
    int site[8], chain[8], n_chains;
    uint32_t mask[8][NB];  // [chain][a]: the bits of the chain's sites taken from X[a] << (a + 2)
    constexpr SegPlan() : site{}, chain{}, n_chains(0), mask{}
    {
        int last[8] = {};
        for (int k = 0; k < 8; ++k) {
            site[k] = seg_site<NB, L, SEL>(k);
            int c = 0;
            while (c < n_chains && site[k] - last[c] < NB) ++c;
            if (c == n_chains) ++n_chains;
            last[c] = site[k];
            chain[k] = c;
            for (int a = 0; a < NB; ++a) mask[c][a] |= 4u << (site[k] + a);
        }
    }
};

// sites 2w and 2w + 1 share one packed compare: they lie in one row, two apart, and 2w below 14
template <int NB, int L, int SEL>
__host__ __device__ constexpr bool seg_pairs_ok()
{
    for (int w = 0; w < 4; ++w)
        if (seg_site<NB, L, SEL>(2 * w + 1) != seg_site<NB, L, SEL>(2 * w) + 2 || seg_site<NB, L, SEL>(2 * w) > 13)
            return false;
    return true;
}

typedef uint32_t gu32x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) gu32x4* grow_ptr;  // table rows, global memory

// v_pk_min_u16, written out: as an expression the optimiser may split it into compares per half
__device__ __forceinline__ uint32_t pk_min_u16(uint32_t a, uint32_t b)
{
    uint32_t r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// (v & m) | (w & ~m) in one v_bfi_b32 with the mask in a scalar register (as an expression, the
// optimiser keeps the unused bits exact, which costs an and and an or per term)
__device__ __forceinline__ uint32_t bfi_sgpr(uint32_t m, uint32_t v, uint32_t w)
{
    uint32_t r;
    asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "s"(m), "v"(v), "v"(w));
    return r;
}

// a - b per 16-bit half, saturated at zero (v_pk_sub_u16 with clamp)
__device__ __forceinline__ uint32_t pk_sub_sat_u16(uint32_t a, uint32_t b)
{
    typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                      __builtin_bit_cast(u16x2, b)));
}

// The table entries of the 8 sites of colour parity SEL in a segment, as lane reads of the rows:
// raw[2w] holds site 2w's entry in its low half, raw[2w + 1] site 2w + 1's in its high half (word w
// of a row holds the entries of sites 2w and 2w + 1 for the row's pattern).  The reads stay in
// flight until gauss_segment_decide uses them.
template <int NB, int L, int SEL, int HALF = 0>
__device__ __forceinline__ void gauss_segment_fetch(const uint32_t X[NB], const gu32x4& row, uint32_t raw[8])
{
    static_assert(seg_pairs_ok<NB, L, SEL>(), "segment sites do not pair");
    // the lane addresses: site j's pattern in bits 2.. of acc >> j (the segment in bits 16 * HALF ..
    // of the neighbour words; shifting right by 14 - a puts bit 16 + j at j + a + 2, and the low
    // half's bits below a + 2, which no chain takes)
    constexpr SegPlan<NB, L, SEL> plan{};
    constexpr int NC = plan.n_chains;
    uint32_t P[NB], acc[NC];
#pragma unroll
    for (int a = 0; a < NB; ++a) P[a] = HALF ? X[a] >> (14 - a) : X[a] << (a + 2);
    // only the chain's fields matter (the lane read ignores the other bits), so each neighbour word
    // is merged in with one bit-field insert of its field bits
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        acc[c] = P[0];
#pragma unroll
        for (int a = 1; a < NB; ++a) acc[c] = bfi_sgpr(plan.mask[c][a], P[a], acc[c]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
        raw[k] = (uint32_t)__builtin_amdgcn_ds_bpermute((int)(acc[plan.chain[k]] >> plan.site[k]), (int)row[k >> 1]);
}

// The attempts of the 8 sites of colour parity SEL in a segment.  Site k's draw is field k of the
// segment's Philox call (half k & 1 of word k >> 1), the same half as its table entry, so one
// packed compare takes sites 2w and 2w + 1.  u < T16 accepts; returns the flips (site bits), and
// *tied is set where some site has u == T16 (those are neither flipped here nor final).
template <int NB, int L, int SEL>
__device__ __forceinline__ uint32_t gauss_segment_decide(const uint32_t raw[8], const uint4v& v, bool* tied)
{
    const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
    uint32_t G = 0, tmin = 0xFFFFFFFFu;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t thi = __builtin_amdgcn_perm(raw[2 * w + 1], raw[2 * w], 0x07060100u);  // low, high half
        tmin = pk_min_u16(tmin, vw[w] ^ thi);  // a zero half: u == T16
        // 1 in each half where u < T16: site 2w's bit at its site, site 2w + 1's 16 above that
        G |= pk_min_u16(pk_sub_sat_u16(thi, vw[w]), 0x00010001u) << seg_site<NB, L, SEL>(2 * w);
    }
    *tied = (tmin & 0xFFFFu) == 0 || (tmin >> 16) == 0;
    // site 2w + 1 lies two above site 2w (and every site 2w below 14): the high bits move down 14
    return (G & 0xFFFFu) | (G >> 14);
}

// the sites of colour parity SEL in a segment with u == T16
template <int NB, int L, int SEL>
__device__ __forceinline__ uint32_t gauss_segment_ties(const uint32_t raw[8], const uint4v& v)
{
    const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
    uint32_t tie = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const uint32_t x = vw[w] ^ __builtin_amdgcn_perm(raw[2 * w + 1], raw[2 * w], 0x07060100u);
        tie |= (uint32_t)((x & 0xFFFFu) == 0) << seg_site<NB, L, SEL>(2 * w);
        tie |= (uint32_t)((x >> 16) == 0) << seg_site<NB, L, SEL>(2 * w + 1);
    }
    return tie;
}

struct GaussWords { uint32_t w[6]; };

// The exact decisions of one lane's tied sites of segment m (site bits ties; X the segment's
// neighbour words, T64m its rows of the u64 table): the 64-bit draw U = (u << 48) | 48 bits of the
// tie stream against T64 (Sec. II).
template <int NB>
__device__ __forceinline__ uint32_t gauss_resolve_ties(const uint64_t* __restrict__ T64m, GaussWords X, uint4v v,
                                                       uint32_t ties, int m, uint32_t rr, uint32_t ctr2, uint32_t k0,
                                                       uint32_t k1)
{
    uint32_t F = 0;
    while (ties) {
        const int j = __builtin_ctz(ties);
        ties &= ties - 1;
        int b = 0;
        for (int a = 0; a < NB; ++a) b |= (int)((X.w[a] >> j) & 1u) << a;
        const int k = j >> 1;  // site j is the k-th of its colour in the segment
        const uint64_t T = T64m[(b << 3) + k];
        const uint32_t u = (word_of(v, k >> 1) >> (16 * (k & 1))) & 0xFFFFu;
        const uint4v w = philox10((uint32_t)(16 * m + j), rr, ctr2, kTagTie, k0, k1);
        const uint64_t U = ((uint64_t)u << 48) | (uint64_t)w.x | ((uint64_t)(w.y & 0xFFFFu) << 32);
        F |= (uint32_t)(T == ~0ull || U < T) << j;
    }
    return F;
}


// The rare first-look ties of segment m, decided exactly before it is written: the neighbour words
// are formed again (segment m's own word has not changed) and the tied lanes compare their 64-bit
// draws with the u64 table.
template <int NB, int L, int SEL>
__device__ __forceinline__ uint32_t gauss_segment_tie_flips(uint16_t* __restrict__ seg, int m, int nseg, uint32_t D,
                                                            const uint32_t raw[8], const uint4v& v,
                                                            const uint64_t* __restrict__ T64c, uint32_t rr,
                                                            uint32_t ctr2, uint32_t k0, uint32_t k1)
{
    const uint32_t ties = gauss_segment_ties<NB, L, SEL>(raw, v);
    if (!ties) return 0;
    uint32_t X[NB];
    int par;
    gauss_segment_words<NB, L>(seg, m, nseg, D, X, &par);
    GaussWords xw = {};
#pragma unroll
    for (int a = 0; a < NB; ++a) xw.w[a] = X[a];
    return gauss_resolve_ties<NB>(T64c + ((size_t)m << (NB + 3)), xw, v, ties, m, rr, ctr2, k0, k1);
}

// The attempts of segments m0 .. m0 + G - 1, all of colour parity SEL (rows: their table rows):
// the lane reads of every segment's entries, then their draws while those are in flight, then the
// decisions.  G is the number of consecutive segments of one colour parity taken per step: cube
// side 8, the four of a z plane (two pairs); chains of an even number of segments, a pair;
// otherwise one (side 4 alternates the parity from segment to segment).
template <int NB, int L, int SEL, int G>
__device__ __forceinline__ void gauss_group_step(uint16_t* __restrict__ seg, int m0, int nseg, const gu32x4 (&rows)[G],
                                                 const uint64_t* __restrict__ T64c, uint32_t rr, uint32_t ctr2,
                                                 uint32_t k0, uint32_t k1)
{
    uint32_t D[G], raw[G][8];
    if constexpr (G == 4) {
        // a z plane: its two pairs, each the other's neighbour in y; the neighbour words once per
        // pair for both halves
        const uint32_t A = pair_at(seg, m0 >> 1), B = pair_at(seg, (m0 >> 1) + 1);
        uint32_t X[6];
        gauss_pair_words8(seg, m0 >> 1, A, B, X);
        gauss_segment_fetch<NB, L, SEL, 0>(X, rows[0], raw[0]);
        gauss_segment_fetch<NB, L, SEL, 1>(X, rows[1], raw[1]);
        gauss_pair_words8(seg, (m0 >> 1) + 1, B, A, X);
        gauss_segment_fetch<NB, L, SEL, 0>(X, rows[2], raw[2]);
        gauss_segment_fetch<NB, L, SEL, 1>(X, rows[3], raw[3]);
        D[0] = A & 0xFFFFu;
        D[1] = A >> 16;
        D[2] = B & 0xFFFFu;
        D[3] = B >> 16;
    } else if constexpr (G == 2) {
        static_assert(NB == 2, "pairs of one parity: chains");
        const uint32_t A = pair_at(seg, m0 >> 1);
        uint32_t X[2];
        gauss_pair_words_chain(seg, m0 >> 1, nseg >> 1, A, X);
        gauss_segment_fetch<NB, L, SEL, 0>(X, rows[0], raw[0]);
        gauss_segment_fetch<NB, L, SEL, 1>(X, rows[1], raw[1]);
        D[0] = A & 0xFFFFu;
        D[1] = A >> 16;
    } else {
        D[0] = seg_at(seg, m0);
        uint32_t X[NB];
        int par;
        gauss_segment_words<NB, L>(seg, m0, nseg, D[0], X, &par);
        gauss_segment_fetch<NB, L, SEL>(X, rows[0], raw[0]);
    }
    uint4v v[G];
#pragma unroll
    for (int g = 0; g < G; ++g) v[g] = words::philox10_lane((uint32_t)(m0 + g), rr, ctr2, kTagMet, k0, k1);
    uint32_t F[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        bool tied;
        F[g] = gauss_segment_decide<NB, L, SEL>(raw[g], v[g], &tied);
        if (__ballot(tied)) F[g] |= gauss_segment_tie_flips<NB, L, SEL>(seg, m0 + g, nseg, D[g], raw[g], v[g], T64c, rr, ctr2, k0, k1);
    }
    if constexpr (G >= 2) pair_store(seg, m0 >> 1, (D[0] | (D[1] << 16)) ^ (F[0] | (F[1] << 16)));
    if constexpr (G == 4) pair_store(seg, (m0 >> 1) + 1, (D[2] | (D[3] << 16)) ^ (F[2] | (F[3] << 16)));
    if constexpr (G == 1) seg_at(seg, m0) = (uint16_t)(D[0] ^ F[0]);
}

// 1-D grid of blocks of kGaussWaves independent waves; block -> (run, group of kGaussWaves tiles):
// with 8 or more runs, the runs are split into 8 contiguous ranges and the blocks of range x are
// those with id = x mod 8 (blocks go round-robin to the 8 XCDs, so a run's table stays in one
// L2); LDS per wave: pairs of segments [N / 32 rounded up][64].  Every lane of a wave takes part in the lane reads of
// the table (lanes past R compute on zero spins and store nothing), so no branch may split a wave
// around them.
template <int NB, int L, int G>
__global__ void __launch_bounds__(kGaussWaves * 64) k_sweep_gauss_tab(pa_state* __restrict__ states, int n_runs,
                                                                      int groups, int64_t t0, int ns)
{
    int run, group;
    if (n_runs >= 8) {
        const int per_xcd = (n_runs + 7) / 8;
        const int k = blockIdx.x >> 3;
        run = (int)(blockIdx.x & 7) * per_xcd + k / groups;
        group = k % groups;
    } else {
        run = blockIdx.x / groups;
        group = blockIdx.x % groups;
    }
    if (run >= n_runs) return;
    const pa_state* st = states + run;
    if (st->status) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tile = (int64_t)group * kGaussWaves + wave;
    const int64_t R = st->R;
    if (tile * 64 >= R) return;
    extern __shared__ uint16_t lds16[];
    const int N = st->N;
    const int nseg = N >> 4;
    const double* __restrict__ J = reinterpret_cast<const double*>(st->J);
    const uint16_t* __restrict__ Tab = gauss_table(st);
    const uint64_t* __restrict__ Tab64 = gauss_table64<NB>(st);
    const int npair = (nseg + 1) >> 1;
    uint16_t* seg = lds16 + wave * npair * 128 + 2 * lane;
    const uint32_t k0 = (uint32_t)st->seed, k1 = (uint32_t)(st->seed >> 32);
    const int64_t r = tile * 64 + lane;
    const bool valid = r < R;
    uint8_t* row = (uint8_t*)st->spins[st->cur] + r * st->row_stride;
#pragma unroll 1
    for (int m = 0; m < nseg; ++m) {
        uint32_t w = 0;
        if (valid) {
            const uint4 q = *reinterpret_cast<const uint4*>(row + 16 * m);
            w = bytes_to_bits4(q.x) | (bytes_to_bits4(q.y) << 4) | (bytes_to_bits4(q.z) << 8) | (bytes_to_bits4(q.w) << 12);
        }
        seg_at(seg, m) = (uint16_t)w;
    }
    const uint32_t rr = (uint32_t)r;
    const int prow = lane & ((1 << NB) - 1);  // the pattern whose table entries this lane holds
    for (int64_t t = t0; t < t0 + ns; ++t) {
        for (int col = 0; col < 2; ++col) {
            const uint32_t ctr2 = (uint32_t)(2 * t + col);
            // this lane's row of segment m is T[m << NB]
            const grow_ptr T = (grow_ptr)(Tab + (col ? ((N / 2) << NB) : 0)) + prow;
            // groups of G segments of one colour parity: their table rows (loaded a group ahead),
            // the lane reads of their entries, their draws while those are in flight, then the
            // decisions
            const uint64_t* __restrict__ T64c = Tab64 + (col ? ((N / 2) << NB) : 0);
            gu32x4 rows[G];
#pragma unroll
            for (int g = 0; g < G; ++g) rows[g] = T[g << NB];
#pragma unroll 1
            for (int m0 = 0; m0 < nseg; m0 += G) {
                const int n0 = m0 + G < nseg ? m0 + G : m0;
                gu32x4 next[G];
#pragma unroll
                for (int g = 0; g < G; ++g) next[g] = T[(n0 + g) << NB];
                if ((gauss_segment_parity<NB, L>(m0) ^ col) == 0)
                    gauss_group_step<NB, L, 0, G>(seg, m0, nseg, rows, T64c, rr, ctr2, k0, k1);
                else
                    gauss_group_step<NB, L, 1, G>(seg, m0, nseg, rows, T64c, rr, ctr2, k0, k1);
#pragma unroll
                for (int g = 0; g < G; ++g) rows[g] = next[g];
            }
        }
    }
    // write back; E in bond order (site i, then axis +x, +y, +z; chain: bond i -- i+1)
    double E = 0.0;
#pragma unroll 1
    for (int m = 0; m < nseg; ++m) {
        const uint32_t D = seg_at(seg, m);
        uint32_t X[NB];
        int par;
        gauss_segment_words<NB, L>(seg, m, nseg, D, X, &par);
        const double* Jm = J + (NB == 2 ? 16 * m : 48 * m);
        // unrolled by 4 only: unrolled fully, the couplings of a whole segment would be held in VGPRs
#pragma unroll 4
        for (int j = 0; j < 16; ++j) {
            if constexpr (NB == 2) {
                E = E + (((X[0] >> j) & 1u) ? -Jm[j] : Jm[j]);
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) E = E + (((X[a] >> j) & 1u) ? -Jm[3 * j + a] : Jm[3 * j + a]);
            }
        }
        if (valid) {
            uint4 q;
            q.x = bits4_to_bytes(D & 15u);
            q.y = bits4_to_bytes((D >> 4) & 15u);
            q.z = bits4_to_bytes((D >> 8) & 15u);
            q.w = bits4_to_bytes((D >> 12) & 15u);
            *reinterpret_cast<uint4*>(row + 16 * m) = q;
        }
    }
    if (valid) reinterpret_cast<double*>(st->energy[st->cur])[r] = E;
}

// the tabled kernels cover cubes of side 4 and 8 and chains of N = 16 k <= 1024 sites
static bool gauss_tab_shape(int dim, int L, int* NB)
{
    if (dim == 3 && (L == 4 || L == 8)) *NB = 6;
    else if (dim == 1 && L % 16 == 0 && L <= 1024) *NB = 2;
    else return false;
    return true;
}

// energy mean, variance, skewness of the population (one block; any summation order: these are
// compared to 1e-12, not bit for bit)
__global__ void __launch_bounds__(256) k_moments_gauss(pa_state* base)
{
    pa_state* st = base + blockIdx.y;
    if (st->status) return;
    __shared__ double red[256];
    const int64_t R = st->R;
    const double* E = reinterpret_cast<const double*>(st->energy[st->cur]);
    auto bsum = [&](double x) {
        red[threadIdx.x] = x;
        __syncthreads();
        for (int o = 128; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        const double v = red[0];
        __syncthreads();
        return v;
    };
    double a = 0.0;
    for (int64_t j = threadIdx.x; j < R; j += blockDim.x) a += E[j];
    const double mean = bsum(a) / (double)R;
    double b2 = 0.0, b3 = 0.0;
    for (int64_t j = threadIdx.x; j < R; j += blockDim.x) {
        const double d = E[j] - mean;
        b2 += d * d;
        b3 += d * d * d;
    }
    const double m2 = bsum(b2) / (double)R;
    const double m3 = bsum(b3) / (double)R;
    if (threadIdx.x == 0) {
        pa_record* rec = st->record + st->k;
        rec->E_mean = mean;
        rec->E_var = m2;
        rec->E_skew = m2 > 0.0 ? m3 / (m2 * sqrt(m2)) : 0.0;
    }
}

// ------------------------------------------------------------------ launchers
int launch_energy_gauss(const pa_run& run, int buf, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_gauss, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, (const pa_state*)run.state,
                       buf, n);
    return hip_status(hipGetLastError());
}

int launch_sweep_gauss(const pa_run* runs, int n_runs, bool consecutive, const pa_step& step, hipStream_t s)
{
    int NB = 0;
    bool tab = gauss_tab_shape(runs[0].dim, runs[0].L, &NB);
    for (int r = 0; r < n_runs; ++r)
        tab = tab && runs[r].dim == runs[0].dim && runs[r].L == runs[0].L && ((uintptr_t)runs[r].spins[0] & 15) == 0 &&
              ((uintptr_t)runs[r].spins[1] & 15) == 0;
    if (!tab) {
        for (int r = 0; r < n_runs; ++r) {
            hipLaunchKernelGGL(k_sweep_gauss, dim3((unsigned)((runs[r].capacity + 63) / 64)), dim3(64), 0,
                               (hipStream_t)runs[r].stream, (const pa_state*)runs[r].state, step.beta_to, step.t0,
                               step.n_sweeps);
            const int st = hip_status(hipGetLastError());
            if (st != PA_OK) return st;
        }
        return PA_OK;
    }
    const int dim = runs[0].dim, L = runs[0].L;
    const int N = dim == 1 ? L : L * L * L;
    const size_t lds = (size_t)kGaussWaves * ((N / 16 + 1) / 2) * 64 * 4;
    auto go = [&](pa_state* base, int n, int64_t capacity, hipStream_t str) {
        const dim3 tgrid((unsigned)(((N << NB) + 255) / 256), (unsigned)n);
        if (NB == 2) hipLaunchKernelGGL((k_gauss_table<2, 0>), tgrid, dim3(256), 0, str, base, step.beta_to);
        else if (L == 4) hipLaunchKernelGGL((k_gauss_table<6, 4>), tgrid, dim3(256), 0, str, base, step.beta_to);
        else hipLaunchKernelGGL((k_gauss_table<6, 8>), tgrid, dim3(256), 0, str, base, step.beta_to);
        int st = hip_status(hipGetLastError());
        if (st != PA_OK) return st;
        const int groups = (int)((capacity / 64 + kGaussWaves - 1) / kGaussWaves);
        const int64_t blocks = n >= 8 ? (int64_t)8 * ((n + 7) / 8) * groups : (int64_t)n * groups;
        if (blocks > INT32_MAX) return PA_ERR_ARG;
        const dim3 grid((unsigned)blocks), block(kGaussWaves * 64);
        if (dim == 1 && (N / 16) % 2 == 0)
            hipLaunchKernelGGL((k_sweep_gauss_tab<2, 0, 2>), grid, block, lds, str, base, n, groups, step.t0, step.n_sweeps);
        else if (dim == 1)
            hipLaunchKernelGGL((k_sweep_gauss_tab<2, 0, 1>), grid, block, lds, str, base, n, groups, step.t0, step.n_sweeps);
        else if (L == 4)
            hipLaunchKernelGGL((k_sweep_gauss_tab<6, 4, 1>), grid, block, lds, str, base, n, groups, step.t0, step.n_sweeps);
        else
            hipLaunchKernelGGL((k_sweep_gauss_tab<6, 8, 4>), grid, block, lds, str, base, n, groups, step.t0, step.n_sweeps);
        return hip_status(hipGetLastError());
    };
    if (consecutive) {
        int64_t cap = 0;
        for (int r = 0; r < n_runs; ++r) cap = runs[r].capacity > cap ? runs[r].capacity : cap;
        return go(runs[0].state, n_runs, cap, s);  // s is the runs' common stream
    }
    for (int r = 0; r < n_runs; ++r) {
        const int st = go(runs[r].state, 1, runs[r].capacity, (hipStream_t)runs[r].stream);
        if (st != PA_OK) return st;
    }
    return PA_OK;
}

int launch_moments_gauss(const pa_run* runs, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments_gauss, dim3(1, (unsigned)n), dim3(256), 0, s, runs[0].state);
    return hip_status(hipGetLastError());
}

}  // namespace pa
