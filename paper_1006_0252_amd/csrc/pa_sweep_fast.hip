// Metropolis sweeps of the cube for even L <= 16: the same sample as the generic kernel
// (same Philox fields, same acceptance rule), laid out for the vector ALU.
//
//  - lane = replica; a replica's rows (bit x = spin) sit in LDS, rows y and y + L/2 of a plane
//    as the low and high half of one 32-bit word; LPR lanes share a replica by taking L/LPR
//    planes each;
//  - the row-pair loop of a plane is unrolled, so every neighbour word is an immediate LDS
//    offset, and the Philox field of every site is a compile-time constant given the plane's
//    phase (the position of its first half-site inside an 8-site Philox chunk: 0 when
//    L = 0 mod 4, 0/2/4/6 by plane when L = 2 mod 4);
//  - per row pair, the six bond words J s s (bit-parallel over x, both rows at once) feed a
//    bit-sliced adder giving c = number of bonds with J s_i s_j = -1 (dE = 4c - 12); c <= 3
//    flips outright;
//  - the 16-bit first look is done on pairs of sites with packed 16-bit ops, specialised by
//    regime:  MODE 2: every threshold of c >= 4 has top 16 bits 0 (beta > ln 2^16 / 4): only
//    u == 0 can accept, and that is a tie;  MODE 1: only c = 4 has a non-zero top;  MODE 0:
//    general, the pair's thresholds from a 16-entry LDS table.  One saturated subtraction
//    (top + 1) - u per site gives all three outcomes at once: 0 rejects, 1 is a tie (u equals
//    the top), 2 or more accepts; clamped to 2, the two-bit outcomes of a row are packed into one
//    word, whose low bits flag ties and whose high bits are the accepted sites.  Ties are
//    resolved exactly with the 48 low bits in a separate (rare) path.  Tops of 0xFFFF and above
//    (beta below 4e-6) do not leave room for the + 1 and take the generic kernel instead;
//  - energies are recomputed once per launch from bond popcounts.
//
// Two launch forms share the per-tile code: one block of waves per group of replicas of one
// run (k_sweep3f, which moves whole 64-replica bit-packed groups block-wide when its waves hold
// one), and a persistent kernel for a batch of runs (k_sweep_batch), one wave per block pulling
// (run, tile) items from a device work counter.
#include <string.h>

#include <algorithm>

#include "pa_common.h"
#include "pa_sweep_util.h"

namespace pa {

struct FastThr {
    uint32_t thi4, thi5, thi6;
    uint64_t T4, T5, T6;
};

// exact random-acceptance mask of the candidate sites (c >= 4) of nh rows held in the 16-bit
// halves of the words c0, c1, cand (nh = 2: the second row's half-sites start hstep and its sites
// istep further on, its colour has x parity parh).  The thresholds come as scalars: a structure
// passed by value to this out-of-line call would go through private (scratch) memory.
static __device__ __noinline__ uint32_t resolve_rows(uint32_t c0, uint32_t c1, uint32_t cand, int par, int parh, int nh, int H,
                                                     int hbase, int hstep, int ibase, int istep, uint32_t rr,
                                                     uint32_t ctr2, uint32_t k0, uint32_t k1, uint32_t thi4,
                                                     uint32_t thi5, uint32_t thi6, uint64_t T4, uint64_t T5, uint64_t T6)
{
    uint32_t racc = 0;
    for (int hh = 0; hh < nh; ++hh) {
        for (int m = 0; m < H; ++m) {
            const int x = 2 * m + (hh ? parh : par), b = 16 * hh + x;
            if (!((cand >> b) & 1u)) continue;
            const int h = hbase + hh * hstep + m;
            const uint4v v = philox10((uint32_t)(h >> 3), rr, ctr2, kTagMet, k0, k1);
            const uint32_t u = field16(v, h & 7);
            const int cls = 4 + (int)((c0 >> b) & 1u) + 2 * (int)((c1 >> b) & 1u);
            const uint32_t thi = cls == 4 ? thi4 : (cls == 5 ? thi5 : thi6);
            const uint64_t T = cls == 4 ? T4 : (cls == 5 ? T5 : T6);
            bool a;
            if (u != thi) a = u < thi;
            else a = tie_accept(u, T, (uint32_t)(ibase + hh * istep + x), rr, ctr2, k0, k1);
            racc |= (uint32_t)a << b;
        }
    }
    return racc;
}

// The same decision for the two rows of a word when each row's eight half-sites of a colour are
// exactly one Philox call (L = 16): the first looks come from the rows' words a, b, already drawn
// on the hot path, and only a first-look tie draws the 48 low bits.
static __device__ __noinline__ uint32_t resolve_pair_words(uint32_t c0, uint32_t c1, uint32_t cand, int par, int ibase,
                                                           int istep, uint32_t a0, uint32_t a1, uint32_t a2,
                                                           uint32_t a3, uint32_t b0, uint32_t b1, uint32_t b2,
                                                           uint32_t b3, uint32_t rr, uint32_t ctr2, uint32_t k0,
                                                           uint32_t k1, uint32_t thi4, uint32_t thi5, uint32_t thi6,
                                                           uint64_t T4, uint64_t T5, uint64_t T6)
{
    const uint32_t w[8] = {a0, a1, a2, a3, b0, b1, b2, b3};
    uint32_t racc = 0;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int x = 2 * m + par, b = 16 * hh + x;
            if (!((cand >> b) & 1u)) continue;
            const uint32_t word = w[4 * hh + (m >> 1)];
            const uint32_t u = (m & 1) ? (word >> 16) : (word & 0xFFFFu);
            const int cls = 4 + (int)((c0 >> b) & 1u) + 2 * (int)((c1 >> b) & 1u);
            const uint32_t thi = cls == 4 ? thi4 : (cls == 5 ? thi5 : thi6);
            const uint64_t T = cls == 4 ? T4 : (cls == 5 ? T5 : T6);
            bool a;
            if (u != thi) a = u < thi;
            else a = tie_accept(u, T, (uint32_t)(ibase + hh * istep + x), rr, ctr2, k0, k1);
            racc |= (uint32_t)a << b;
        }
    }
    return racc;
}

template <int L, int LPR>
struct FastLayout {
    static constexpr int NR = L * L;
    static constexpr int H = L / 2;
    // rows y and y + L/2 of a plane share one 32-bit word (low and high half)
    static constexpr int JROWS = L / 2;                         // coupling-mask entries per plane
    static constexpr int RPW = 64 / LPR;
    static constexpr int PL = L / LPR;                          // planes per lane
    static constexpr int PADW = LPR == 4 ? 8 : 0;               // u16 padding per plane (bank stagger)
    static constexpr int PSTRIDE = L * RPW + PADW;              // u16 per plane
    static constexpr int JPAD = LPR == 4 ? 4 : 0;
    static constexpr int JSTRIDE = JROWS * 8 + JPAD;            // dwords of coupling masks per plane
    static constexpr int JDWORDS = L * JSTRIDE;
    // after the masks: the 16-entry pair-bound table, then (L = 0 mod 4) the 256-entry table of
    // two consecutive pairs of a row (8-byte entries, so 8-byte aligned: JDWORDS is even)
    static constexpr int TDWORDS = L % 4 == 0 ? 16 + 512 : 16;
    static constexpr int TAB_DWORDS = JDWORDS + TDWORDS;        // block-shared tables
    static constexpr int ROW_BYTES = L * PSTRIDE * 2;           // one wave's rows
    static constexpr size_t lds_bytes(int wpb) { return (size_t)TAB_DWORDS * 4 + (size_t)wpb * ROW_BYTES; }
};


// coupling masks of row rho = y + L z, entries +x, +y, +z, -x, -y, -z bonds with J = -1 (bit x)
template <int L>
__device__ void row_masks(const int8_t* J, int rho, uint32_t m[6])
{
    const int y = rho % L, z = rho / L;
    const int ym = (y + L - 1) % L, zm = (z + L - 1) % L;
    for (int k = 0; k < 6; ++k) m[k] = 0;
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
}

// the block-shared tables: coupling masks per row pair (rows y and y + L/2 in one entry);
// then the first-look bounds of a pair of sites by their class bits (two consecutive sites of a
// colour in a row, or site m of both rows of a word when L/2 is odd): entry a + 4 b (a, b = c0 +
// 2 c1 of the first and second site) holds (thi(a) + 1) | (thi(b) + 1) << 16, with class index 0,
// 1, 2 for c = 4, 5, 6 (3 cannot occur at a candidate site).  The launch guarantees thi <= 0xFFFE.
template <int L, int LPR>
__device__ void build_jtab(const pa_state* st, uint32_t* jtab, const FastThr& th, int tid, int nthr)
{
    using F = FastLayout<L, LPR>;
    const uint32_t t[4] = {th.thi4 + 1u, th.thi5 + 1u, th.thi6 + 1u, th.thi6 + 1u};
    for (int e = tid; e < F::TDWORDS; e += nthr) {
        // entry n < 16: the pair of class nibble n; entry 16 + 2n + h (n < 256): the pair of nibble
        // h of byte n (the four class bits of the first pair, then of the second)
        const int n = e < 16 ? e : (((e - 16) >> 1) >> (4 * ((e - 16) & 1))) & 15;
        jtab[F::JDWORDS + e] = t[n & 3] | (t[n >> 2] << 16);
    }
    const int8_t* J = st->J;
    for (int e_i = tid; e_i < L * F::JROWS; e_i += nthr) {
        const int z = e_i / F::JROWS, y = e_i % F::JROWS;
        uint32_t m[6], mh[6];
        row_masks<L>(J, y + L * z, m);
        row_masks<L>(J, y + L / 2 + L * z, mh);
        uint32_t* e = jtab + z * F::JSTRIDE + y * 8;
        for (int k = 0; k < 6; ++k) e[k] = m[k] | (mh[k] << 16);
        e[6] = 0;
        e[7] = 0;
    }
}

struct PlaneCtx {
    uint32_t rr, ctr2, k0, k1;
    bool valid;
};

typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));

// bits of a where m is set, of b elsewhere (one v_bfi_b32)
__device__ __forceinline__ uint32_t select_bits(uint32_t m, uint32_t a, uint32_t b) { return (a & m) | (b & ~m); }

// three-input xor and majority, one v_bitop3_b32 each (truth tables over a = 0xF0, b = 0xCC, c = 0xAA);
// written as builtins so that the optimiser cannot re-split the adder tree into two-input ops
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8); }

// bit-sliced count of the six bond words: c = c0 + 2 c1 + 4 c2 bonds with J s_i s_j = -1 per bit
// (two full adders, a half adder and a final full adder: eight ops)
__device__ __forceinline__ void bond_count(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3, uint32_t b4,
                                           uint32_t b5, uint32_t& c0, uint32_t& c1, uint32_t& c2)
{
    const uint32_t s1 = xor3(b0, b1, b2), k1c = maj3(b0, b1, b2);
    const uint32_t s2 = xor3(b3, b4, b5), k2c = maj3(b3, b4, b5);
    c0 = s1 ^ s2;
    const uint32_t k3c = s1 & s2;
    c1 = xor3(k1c, k2c, k3c);
    c2 = maj3(k1c, k2c, k3c);
}

// raw | (e << k) as one v_lshl_or_b32 (left to itself the compiler pairs shifts into v_or3_b32,
// one and a half ops per field instead of one).  k must be a constant after unrolling: the switch
// then folds to the one asm statement with k as an inline constant.
#define PA_LSHL_OR(K) \
    case K: asm("v_lshl_or_b32 %0, %1, " #K ", %2" : "=v"(r) : "v"(e), "v"(raw)); break;
__device__ __forceinline__ uint32_t lshl_or(uint32_t e, int k, uint32_t raw)
{
    uint32_t r = raw | (e << k);
    switch (k) {
        PA_LSHL_OR(0) PA_LSHL_OR(1) PA_LSHL_OR(2) PA_LSHL_OR(3) PA_LSHL_OR(4) PA_LSHL_OR(5) PA_LSHL_OR(6)
        PA_LSHL_OR(7) PA_LSHL_OR(8) PA_LSHL_OR(9) PA_LSHL_OR(10) PA_LSHL_OR(11) PA_LSHL_OR(12) PA_LSHL_OR(13)
        PA_LSHL_OR(14) PA_LSHL_OR(15) PA_LSHL_OR(16) PA_LSHL_OR(17) PA_LSHL_OR(18) PA_LSHL_OR(19) PA_LSHL_OR(20)
        PA_LSHL_OR(21) PA_LSHL_OR(22) PA_LSHL_OR(23) PA_LSHL_OR(24) PA_LSHL_OR(25) PA_LSHL_OR(26) PA_LSHL_OR(27)
        PA_LSHL_OR(28) PA_LSHL_OR(29) PA_LSHL_OR(30) PA_LSHL_OR(31)
        default: break;
    }
    return r;
}
#undef PA_LSHL_OR

// one colour of one plane z of this lane's replica: rows y and y + L/2 (not neighbours for L >= 6,
// nor for L = 4) sit in the low and high half of one 32-bit word, so one bit-sliced count serves
// both.  The y + 1 word of the last pair and the y - 1 word of the first are the first and last
// pair with halves swapped.  With L/2 odd the high row's colour has the other x parity.  PH: the
// position of the plane's first half-site in its Philox call (0 when L = 0 mod 4).
template <int L, int LPR, int MODE, int PH>
__device__ __forceinline__ void plane_update_pairs(uint32_t* rows32, const uint32_t* jtab, int z, int q, int col,
                                                   const PlaneCtx& c, const FastThr& th)
{
    using F = FastLayout<L, LPR>;
    constexpr int H = F::H, Y = L / 2, RPW = F::RPW, PS = F::PSTRIDE / 2;
    constexpr uint32_t MASK = (1u << L) - 1u;
    constexpr uint32_t XP = (MASK >> 1) | ((MASK >> 1) << 16);  // x <= L - 2 in each half: x + 1 from w >> 1
    constexpr uint32_t XM = XP << 1;                             // x >= 1: x - 1 from w << 1
    const int zp = (z + 1 == L) ? 0 : z + 1;
    const int zm = (z == 0) ? L - 1 : z - 1;
    uint32_t* P0 = rows32 + z * PS + q;
    const uint32_t* Pp = rows32 + zp * PS + q;
    const uint32_t* Pm = rows32 + zm * PS + q;
    const uint32_t* JT = jtab + z * F::JSTRIDE;
    const uint32_t* TT = jtab + F::JDWORDS;               // the pair-threshold table
    const uint32_t cb = (uint32_t)((z * (L * H)) >> 3);  // Philox call of the plane's first half-site
    const int p0 = (col + z) & 1;                        // x parity of colour col at even y
    // colour masks of the word for even and odd yy (halves: rows yy and yy + L/2)
    const uint32_t m0 = (p0 ? 0xAAAAu : 0x5555u) & MASK, m1 = (p0 ? 0x5555u : 0xAAAAu) & MASK;
    const uint32_t cmA = m0 | ((Y % 2 ? m1 : m0) << 16);
    const uint32_t cmB = m1 | ((Y % 2 ? m0 : m1) << 16);
    static_assert(H % 2 == 1 || PH == 0, "paired fields need the plane to start a Philox call");
    const u16x2 t4 = {(uint16_t)(th.thi4 + 1u), (uint16_t)(th.thi4 + 1u)};
    const u16x2 two = {2, 2};
    uint4v rndA = {0, 0, 0, 0}, rndB = {0, 0, 0, 0};
#pragma unroll
    for (int yy = 0; yy < Y; ++yy) {
        const uint32_t own = P0[yy * RPW];
        uint32_t yp = P0[((yy + 1) % Y) * RPW];
        uint32_t ym = P0[((yy + Y - 1) % Y) * RPW];
        if (yy == Y - 1) yp = (yp >> 16) | (yp << 16);
        if (yy == 0) ym = (ym >> 16) | (ym << 16);
        const uint32_t zpv = Pp[yy * RPW];
        const uint32_t zmv = Pm[yy * RPW];
        const uint32_t* jr = JT + yy * 8;
        // x + 1 and x - 1 neighbours, periodic within each half
        const uint32_t rp = select_bits(XP, own >> 1, own << (L - 1));
        const uint32_t rm = select_bits(XM, own << 1, own >> (L - 1));
        uint32_t c0, c1, c2;
        bond_count(xor3(own, rp, jr[0]), xor3(own, yp, jr[1]), xor3(own, zpv, jr[2]), xor3(own, rm, jr[3]),
                   xor3(own, ym, jr[4]), xor3(own, zmv, jr[5]), c0, c1, c2);
        const uint32_t colmask = (yy & 1) ? cmB : cmA;
        const int par = p0 ^ (yy & 1);
        uint32_t flip;
        if constexpr (H % 2 == 0) {
            // sites m and m + 1 (m even) of a row take the two 16-bit fields of one Philox word:
            // both are compared with packed 16-bit ops against their bounds b = top + 1 (thi4 + 1
            // in MODE 1, from the pair table by the sites' class bits in MODE 0): per half
            // e = min(b - u saturated at 0, 2) is 0 (reject), 1 (tie) or 2 (accept).  The two-bit
            // fields gather in one word: row A's at 2m (site m) and 16 + 2m (site m + 1), row B's two
            // bits above those; afterwards the accept bits (the high bit of each field) move to the
            // sites' own bits, site m of row A at 2m + par, site m + 1 at 2m + 2 + par, row B's 16
            // bits higher.
            u16x2 zmin = {0xFFFF, 0xFFFF};
            uint32_t raw = 0;
            // MODE 0: class bits of the colour's sites side by side, c0(x) at bit x and c1(x) at
            // bit x + 1, so the four bits of sites m, m + 1 are one nibble at 2m + par (+ 16), and
            // the two pairs m, m + 2 one byte (one 8-byte entry of the 256-entry table).  With L = 16
            // the c1 bit of the high row's x = 15 would leave the word: that row takes c1(x) at bit x
            // and c0(x) at bit x - 1 instead (the same nibble, one bit lower)
            const uint32_t c01 = (c0 & colmask) | ((c1 << 1) & ~colmask);
            const uint32_t c01h = L == 16 ? ((c1 & colmask) | ((c0 >> 1) & ~colmask)) : c01;
            constexpr int OFFH = L == 16 ? 15 : 16;
            const uint2* TT2 = reinterpret_cast<const uint2*>(TT + 16);
            uint2 bA = {0, 0}, bB = {0, 0};
    #pragma unroll
            for (int m = 0; m < H; m += 2) {
                const int hA = PH + yy * H + m, hB = PH + (yy + Y) * H + m;  // half-site positions from call cb
                if (hA % 8 == 0 || (yy == 0 && m == 0))
                    rndA = philox10(cb + (uint32_t)(hA / 8), c.rr, c.ctr2, kTagMet, c.k0, c.k1);
                if (hB % 8 == 0 || (yy == 0 && m == 0))
                    rndB = philox10(cb + (uint32_t)(hB / 8), c.rr, c.ctr2, kTagMet, c.k0, c.k1);
                const u16x2 wA = __builtin_bit_cast(u16x2, word_of(rndA, (hA & 7) >> 1));
                const u16x2 wB = __builtin_bit_cast(u16x2, word_of(rndB, (hB & 7) >> 1));
                if (MODE == 2) {
                    zmin = __builtin_elementwise_min(zmin, __builtin_elementwise_min(wA, wB));
                } else {
                    if (MODE == 0 && m % 4 == 0) {  // the bounds of pairs m and m + 2 at once
                        if (m + 2 < H) {
                            bA = TT2[(c01 >> (2 * m + par)) & 255u];
                            bB = TT2[(c01h >> (OFFH + 2 * m + par)) & 255u];
                        } else {
                            bA.x = TT[(c01 >> (2 * m + par)) & 15u];
                            bB.x = TT[(c01h >> (OFFH + 2 * m + par)) & 15u];
                        }
                    }
                    const u16x2 tA = MODE == 1 ? t4 : __builtin_bit_cast(u16x2, m % 4 == 0 ? bA.x : bA.y);
                    const u16x2 tB = MODE == 1 ? t4 : __builtin_bit_cast(u16x2, m % 4 == 0 ? bB.x : bB.y);
                    const u16x2 dA = __builtin_elementwise_sub_sat(tA, wA);
                    const u16x2 dB = __builtin_elementwise_sub_sat(tB, wB);
                    // min(d, 2) per half, written out: as an expression the optimiser may expand it
                    // into compares and selects per half
                    uint32_t eA, eB;
                    asm("v_pk_min_u16 %0, %1, %2" : "=v"(eA) : "v"(dA), "v"(two));
                    asm("v_pk_min_u16 %0, %1, %2" : "=v"(eB) : "v"(dB), "v"(two));
                    raw = lshl_or(eA, 2 * m, raw);
                    raw = lshl_or(eB, 2 * m + 2, raw);
                    // MODE 1: classes 5 and 6 have top 0, so u == 0 is a tie there
                    if (MODE == 1) zmin = __builtin_elementwise_min(zmin, __builtin_elementwise_min(wA, wB));
                }
            }
            bool tie = zmin.x == 0 || zmin.y == 0;
            if (MODE == 2) {
                flip = colmask & ~c2;
            } else {
                if (MODE == 0) tie = (raw & 0x55555555u) != 0;  // the low (tie) bit of every field
                else tie = tie || (raw & 0x55555555u) != 0;
                // accept bits to the sites (m = 0, 2, 4, 6): row A's site m from 2m + 1 to 2m + par and
                // row B's site m + 1 from 16 + 2m + 3 to 16 + 2m + 2 + par (right by 1 - par); row A's
                // site m + 1 from 16 + 2m + 1 to 2m + 2 + par (right by 15 - par); row B's site m from
                // 2m + 3 to 16 + 2m + par (left by 13 + par).  Only the colour's sites are kept.
                const uint32_t s1 = (0x44441111u << par), s15 = 0x4444u << par;
                const uint32_t acc = select_bits(s1, raw >> (1 - par), select_bits(s15, raw >> (15 - par), raw << (13 + par)));
                if (MODE == 1) flip = colmask & (~c2 | (acc & ~c1 & ~c0));
                else flip = colmask & (~c2 | acc);
            }
            if (tie) {
                const uint32_t cand = c2 & colmask;
                const int rA = yy + L * z;  // the high row is rA + L/2
                uint32_t racc;
                if constexpr (H == 8)  // each row's half-sites are the whole of calls rndA and rndB
                    racc = resolve_pair_words(c0, c1, cand, par, L * rA, L * Y, rndA.x, rndA.y, rndA.z, rndA.w, rndB.x,
                                              rndB.y, rndB.z, rndB.w, c.rr, c.ctr2, c.k0, c.k1, th.thi4, th.thi5,
                                              th.thi6, th.T4, th.T5, th.T6);
                else
                    racc = resolve_rows(c0, c1, cand, par, par, 2, H, rA * H, Y * H, L * rA, L * Y, c.rr, c.ctr2, c.k0,
                                        c.k1, th.thi4, th.thi5, th.thi6, th.T4, th.T5, th.T6);
                flip = colmask & (~c2 | racc);
            }
        } else {
            // an odd number of half-sites per row, so fields do not pair within a row; but Y H is
            // odd, so site m of the low row and site m of the high row sit in opposite halves of
            // their words: one bit-field insert puts u_A in the low and u_B in the high half, and
            // the pair is compared with the packed ops above.  The high row's accept bits land at
            // 16 + 2m + par and move to its own parity parh at the end.
            const int parh = par ^ (Y & 1);  // x parity of the high row's colour
            u16x2 zmin = {0xFFFF, 0xFFFF};
            uint32_t raw = 0;
            // MODE 0: c0(x) at bit x and c1(x) at bit x + 1 for the colour's sites of both rows
            const uint32_t c01 = (c0 & colmask) | ((c1 << 1) & ~colmask);
#pragma unroll
            for (int m = 0; m < H; ++m) {
                const int hA = PH + yy * H + m, hB = PH + (yy + Y) * H + m;
                if (hA % 8 == 0 || (yy == 0 && m == 0))
                    rndA = philox10(cb + (uint32_t)(hA / 8), c.rr, c.ctr2, kTagMet, c.k0, c.k1);
                if (hB % 8 == 0 || (yy == 0 && m == 0))
                    rndB = philox10(cb + (uint32_t)(hB / 8), c.rr, c.ctr2, kTagMet, c.k0, c.k1);
                const uint32_t wa = word_of(rndA, (hA & 7) >> 1), wb = word_of(rndB, (hB & 7) >> 1);
                static_assert(((Y * H) & 1) == 1, "the two rows' fields of site m sit in opposite halves");
                const uint32_t wv = (hA & 1) ? __builtin_amdgcn_alignbit(wb, wa, 16) : ((wa & 0xFFFFu) | (wb & 0xFFFF0000u));
                const u16x2 w = __builtin_bit_cast(u16x2, wv);
                if (MODE == 2) {
                    zmin = __builtin_elementwise_min(zmin, w);
                } else {
                    const int xA = 2 * m + par, xB = 16 + 2 * m + parh;
                    const u16x2 t = MODE == 1 ? t4
                                              : __builtin_bit_cast(u16x2, TT[((c01 >> xA) & 3u) | (((c01 >> xB) & 3u) << 2)]);
                    const u16x2 d = __builtin_elementwise_sub_sat(t, w);
                    uint32_t e;  // min(d, 2) per half, written out (see above)
                    asm("v_pk_min_u16 %0, %1, %2" : "=v"(e) : "v"(d), "v"(two));
                    raw |= e << (2 * m + par);
                    if (MODE == 1) zmin = __builtin_elementwise_min(zmin, w);
                }
            }
            bool tie = zmin.x == 0 || zmin.y == 0;
            if (MODE == 2) {
                flip = colmask & ~c2;
            } else {
                // fields at 2m + par (row A) and 16 + 2m + par (row B); accept bits one higher
                const uint32_t f1 = 0x55555555u << par;
                if (MODE == 0) tie = (raw & f1) != 0;
                else tie = tie || (raw & f1) != 0;
                // row A's site m to 2m + par, row B's to 16 + 2m + parh (parh = 1 - par)
                const uint32_t acc = ((raw >> 1) & (0x5555u << par)) | ((raw >> (2 * par)) & (0x55550000u << parh));
                if (MODE == 1) flip = colmask & (~c2 | (acc & ~c1 & ~c0));
                else flip = colmask & (~c2 | acc);
            }
            if (tie) {
                const uint32_t cand = c2 & colmask;
                const int rA = yy + L * z;  // the high row is rA + L/2
                const uint32_t racc = resolve_rows(c0, c1, cand, par, parh, 2, H, rA * H, Y * H, L * rA,
                                                   L * Y, c.rr, c.ctr2, c.k0, c.k1, th.thi4, th.thi5, th.thi6, th.T4,
                                                   th.T5, th.T6);
                flip = colmask & (~c2 | racc);
            }
        }
        if (!c.valid) flip = 0;
        P0[yy * RPW] = own ^ flip;
    }
}

// N_S sweeps of the RPW replicas rbase .. rbase + RPW - 1 of one run (one wave)
// u16 slot of row y of a plane, from the lane's plane base: rows y and y + L/2 are the halves of
// word y mod L/2 when paired
template <int L, int LPR>
__device__ __forceinline__ int row_slot(int y)
{
    using F = FastLayout<L, LPR>;
    return 2 * (y % (L / 2)) * F::RPW + y / (L / 2);
}

// The rows of the 64 replicas of bit-packed group g (two bytes per row and replica) between HBM
// and the LDS rows of a block whose waves hold the group's replicas in order (replica r of the
// group: wave r / RPW, slot r % RPW).  Each thread moves 4 replicas of a row as one 8-byte word,
// so a row is one 128-byte line; a wave's own share of a line is only 32 bytes.  Stores skip the
// replicas at or past R.
template <int L, int LPR, bool STORE>
__device__ void group_rows_io(const pa_state* st, int64_t g, uint16_t* rows0, int64_t R, int tid, int nthr)
{
    using F = FastLayout<L, LPR>;
    constexpr int RPW = F::RPW, NR = F::NR;
    static_assert(L > 8, "two bytes per row word");
    uint64_t* G = reinterpret_cast<uint64_t*>((uint8_t*)st->spins[st->cur] + g * (int64_t)NR * 128);
    for (int e = tid; e < NR * 16; e += nthr) {
        const int rho = e >> 4, k = e & 15;  // replicas 4k .. 4k + 3 of row rho
        const int z = rho / L, y = rho % L;
        uint16_t* P = rows0 + z * F::PSTRIDE + row_slot<L, LPR>(y);
        uint16_t* slot[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 4 * k + i, w = r / RPW, qq = r % RPW;
            slot[i] = P + w * (F::ROW_BYTES / 2) + 2 * qq;
        }
        if (!STORE) {
            const uint64_t v = G[e];
#pragma unroll
            for (int i = 0; i < 4; ++i) *slot[i] = (uint16_t)(v >> (16 * i));
        } else {
            const int64_t r0 = g * 64 + 4 * k;
            if (r0 + 3 < R) {
                uint64_t v = 0;
#pragma unroll
                for (int i = 0; i < 4; ++i) v |= (uint64_t)*slot[i] << (16 * i);
                G[e] = v;
            } else {
                uint16_t* G16 = reinterpret_cast<uint16_t*>(G + e);
                for (int i = 0; i < 4; ++i)
                    if (r0 + i < R) G16[i] = *slot[i];
            }
        }
    }
}

// N_S sweeps of the tile; IO: the tile's rows are loaded and stored here (else the block moves
// whole groups with group_rows_io around the call)
template <int L, int LAYOUT, int LPR, int MODE, bool IO = true>
__device__ __forceinline__ void sweep_tile(const pa_state* st, int64_t rbase, const uint32_t* jtab, uint16_t* rows, int lane,
                           const SweepParams& p, const FastThr& th)
{
    using F = FastLayout<L, LPR>;
    constexpr int NR = F::NR, H = F::H, RPW = F::RPW, PL = F::PL, PSTRIDE = F::PSTRIDE;
    constexpr uint32_t MASK = (1u << L) - 1u;
    constexpr int WB = L <= 8 ? 1 : 2;  // bytes of a row word in the bit-packed layout
    static_assert(L % 2 == 0 && L <= 16 && L % LPR == 0, "fast sweep geometry");
    static_assert(L % 4 == 0 || LPR == 1, "L = 2 mod 4 needs one lane per replica");
    const int q = lane % RPW, j = lane / RPW;
    const int64_t R = st->R;
    const int cur = st->cur;
    const int64_t r = rbase + q;
    PlaneCtx c;
    c.valid = r < R;
    c.rr = (uint32_t)r;
    c.k0 = (uint32_t)st->seed;
    c.k1 = (uint32_t)(st->seed >> 32);

    // this lane's planes z = j PL .. j PL + PL - 1 into LDS (plane loops here and in the write-back
    // stay rolled: unrolled, their 64-bit row addresses are shared between the two and held live
    // across the sweeps, which costs two thirds of the waves per SIMD)
#pragma unroll 1
    for (int t = 0; t < (IO ? PL : 0); ++t) {
        const int z = j * PL + t;
        uint16_t* P = rows + z * PSTRIDE + 2 * q;
        for (int y = 0; y < L; ++y) {
            const int rho = y + L * z;
            uint32_t v = 0;
            if (LAYOUT == PA_BITS64) {
                const uint8_t* a = (const uint8_t*)st->spins[cur] + (((r >> 6) * NR + rho) * 64 + (r & 63)) * WB;
                v = WB == 1 ? *a : *(const uint16_t*)a;
            } else if (L % 4 == 0) {
                const uint32_t* a = (const uint32_t*)((const uint8_t*)st->spins[cur] + r * st->row_stride + rho * L);
#pragma unroll
                for (int d = 0; d < L / 4; ++d) v |= pack4(a[d]) << (4 * d);
            } else {
                const uint8_t* a = (const uint8_t*)st->spins[cur] + r * st->row_stride + rho * L;
#pragma unroll
                for (int x = 0; x < L; ++x) v |= (uint32_t)(a[x] & 1) << x;
            }
            P[row_slot<L, LPR>(y)] = (uint16_t)v;
        }
    }
    wave_sync();

    for (int s = 0; s < p.n_sweeps; ++s) {
        const int64_t t_sweep = p.t0 + s;
        for (int col = 0; col < 2; ++col) {
            c.ctr2 = (uint32_t)(2 * t_sweep + col);
            for (int t = 0; t < PL; ++t) {
                const int z = j * PL + t;
                uint32_t* rows32 = reinterpret_cast<uint32_t*>(rows);
                if constexpr (L % 4 == 0) {
                    plane_update_pairs<L, LPR, MODE, 0>(rows32, jtab, z, q, col, c, th);
                } else {
                    switch ((z * (L * H)) & 7) {
                        case 0: plane_update_pairs<L, LPR, MODE, 0>(rows32, jtab, z, q, col, c, th); break;
                        case 2: plane_update_pairs<L, LPR, MODE, 2>(rows32, jtab, z, q, col, c, th); break;
                        case 4: plane_update_pairs<L, LPR, MODE, 4>(rows32, jtab, z, q, col, c, th); break;
                        default: plane_update_pairs<L, LPR, MODE, 6>(rows32, jtab, z, q, col, c, th); break;
                    }
                }
            }
            // the other colour reads these rows next (other lanes of the replica too)
            wave_sync();
        }
    }

    // energy of the final configuration: E = n_bonds - 2 (bonds with J s s = -1)
    int neg = 0;
    for (int t = 0; t < PL; ++t) {
        const int z = j * PL + t;
        const int zp = (z + 1 == L) ? 0 : z + 1;
        const uint32_t* JT = jtab + z * F::JSTRIDE;
        constexpr int Y = L / 2, PS = PSTRIDE / 2;
        constexpr uint32_t MASKP = MASK | (MASK << 16);
        constexpr uint32_t XP = (MASK >> 1) | ((MASK >> 1) << 16);
        const uint32_t* P0 = reinterpret_cast<const uint32_t*>(rows) + z * PS + q;
        const uint32_t* Pp = reinterpret_cast<const uint32_t*>(rows) + zp * PS + q;
#pragma unroll
        for (int yy = 0; yy < Y; ++yy) {
            const uint32_t own = P0[yy * RPW];
            uint32_t yp = P0[((yy + 1) % Y) * RPW];
            if (yy == Y - 1) yp = (yp >> 16) | (yp << 16);
            const uint32_t rp = ((own >> 1) & XP) | ((own << (L - 1)) & ~XP);
            const uint32_t* jr = JT + yy * 8;
            neg += __popc((own ^ rp ^ jr[0]) & MASKP);
            neg += __popc((own ^ yp ^ jr[1]) & MASKP);
            neg += __popc((own ^ Pp[yy * RPW] ^ jr[2]) & MASKP);
        }
    }
    for (int off = RPW; off < 64; off <<= 1) neg += __shfl_xor(neg, off, 64);

    // rows back to HBM; the replica index passes through an empty asm so that the row addresses
    // of the load above are recomputed here rather than kept live across the sweeps
    int64_t rw = r;
    asm volatile("" : "+v"(rw));
    if (c.valid) {
#pragma unroll 1
        for (int t = 0; t < (IO ? PL : 0); ++t) {
            const int z = j * PL + t;
            const uint16_t* P = rows + z * PSTRIDE + 2 * q;
            for (int y = 0; y < L; ++y) {
                const int rho = y + L * z;
                const uint32_t v = P[row_slot<L, LPR>(y)];
                if (LAYOUT == PA_BITS64) {
                    uint8_t* a = (uint8_t*)st->spins[cur] + (((rw >> 6) * NR + rho) * 64 + (rw & 63)) * WB;
                    if (WB == 1) *a = (uint8_t)v;
                    else *(uint16_t*)a = (uint16_t)v;
                } else if (L % 4 == 0) {
                    uint32_t* a = (uint32_t*)((uint8_t*)st->spins[cur] + rw * st->row_stride + rho * L);
#pragma unroll
                    for (int d = 0; d < L / 4; ++d) a[d] = unpack4(v >> (4 * d));
                } else {
                    uint8_t* a = (uint8_t*)st->spins[cur] + rw * st->row_stride + rho * L;
#pragma unroll
                    for (int x = 0; x < L; ++x) a[x] = (uint8_t)((v >> x) & 1u);
                }
            }
        }
        if (j == 0) st->energy[cur][rw] = st->n_bonds - 2 * neg;
    }
    wave_sync();
}

// ------------------------------------------------------------------ one run
template <int L, int LAYOUT, int LPR, int MODE>
__global__ void __launch_bounds__(256) k_sweep3f(const pa_state* __restrict__ st, SweepParams p, FastThr th)
{
    using F = FastLayout<L, LPR>;
    if (st->status) return;  // sticky error: the population stays as it is
    extern __shared__ uint32_t lds[];
    build_jtab<L, LPR>(st, lds, th, threadIdx.x, blockDim.x);
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t* rows0 = reinterpret_cast<uint16_t*>(lds + F::TAB_DWORDS);
    uint16_t* rows = rows0 + wave * (F::ROW_BYTES / 2);
    const int64_t rbase = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * F::RPW;
    if constexpr (LAYOUT == PA_BITS64 && L > 8) {
        // the block's waves hold one whole 64-replica group: it moves between HBM and LDS in
        // whole lines, block-wide (every wave reaches both barriers)
        if ((int)(blockDim.x >> 6) * F::RPW == 64) {
            const int64_t R = st->R;
            if ((int64_t)blockIdx.x * 64 >= R) return;  // the whole block is past the population
            group_rows_io<L, LPR, false>(st, blockIdx.x, rows0, R, threadIdx.x, blockDim.x);
            __syncthreads();
            if (rbase < R) sweep_tile<L, LAYOUT, LPR, MODE, false>(st, rbase, lds, rows, lane, p, th);
            __syncthreads();
            group_rows_io<L, LPR, true>(st, blockIdx.x, rows0, R, threadIdx.x, blockDim.x);
            return;
        }
    }
    if (rbase >= st->R) return;
    sweep_tile<L, LAYOUT, LPR, MODE>(st, rbase, lds, rows, lane, p, th);
}

// ------------------------------------------------------------------ a batch of runs
// The runs' states are contiguous (state r at base + r).  Work items are (run, tile of RPW
// replicas); k_batch_tiles lays them out in the order given by the host (position p holds run
// order[p]) and resets the work counter; k_sweep_batch waves take items in that order.
__global__ void __launch_bounds__(256) k_batch_tiles(pa_state* base, int n_runs, BatchOrder order)
{
    int64_t* tb = work_ptr<int64_t>(base, work_layout(base->N, base->n_bins, base->capacity).batch);
    __shared__ int64_t cnt[kMaxBatch];
    for (int pos = threadIdx.x; pos < n_runs; pos += blockDim.x) {
        pa_state* st = base + order.run[pos];
        const int rpw = batch_tile_replicas(st->L, st->layout);
        cnt[pos] = st->status ? 0 : (st->R + rpw - 1) / rpw;
        st->work_counter = 0;  // a group of equal-L runs counts its items in its first run
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int pos = 0; pos < n_runs; ++pos) {
            tb[pos] = acc;
            acc += cnt[pos];
        }
        tb[n_runs] = acc;
    }
}

// one work item: the coupling table of the item's run is rebuilt for every item (a few
// hundred byte loads per lane against ~10^5 attempts per lane)
template <int L, int LAYOUT, int MODE>
__device__ __forceinline__ void batch_tile(const pa_state* st, int64_t local, uint32_t* lds, int lane,
                                           const SweepParams& p, const FastThr& th)
{
    constexpr int LPR = batch_lpr(L);
    using F = FastLayout<L, LPR>;
    build_jtab<L, LPR>(st, lds, th, lane, 64);
    wave_sync();
    uint16_t* rows = reinterpret_cast<uint16_t*>(lds + F::TAB_DWORDS);
    sweep_tile<L, LAYOUT, LPR, MODE>(st, local * F::RPW, lds, rows, lane, p, th);
}

// Persistent sweep of one group of equal-L runs (positions pos0 .. pos1-1 of the order): each
// wave takes the next item of the group, finds its run by bisection of the tile offsets and
// sweeps that tile.  One specialisation per L keeps the register budget of the one-run kernel
// (two waves per SIMD) instead of the union of all sizes.
template <int L, int LAYOUT, int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_sweep_batch(pa_state* base, int pos0, int pos1, BatchOrder order,
                                                    SweepParams p, FastThr th)
{
    extern __shared__ uint32_t lds[];
    const int lane = threadIdx.x;
    const int64_t* tb = work_ptr<int64_t>(base, work_layout(base->N, base->n_bins, base->capacity).batch);
    const int64_t first = tb[pos0], total = tb[pos1] - first;
    pa_state* counter = base + order.run[pos0];
    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(&counter->work_counter, 1u);
        t = __shfl(t, 0, 64);
        if ((int64_t)t >= total) break;  // every wave leaves once the group's items are taken
        const int64_t item = first + (int64_t)t;
        int lo = pos0, hi = pos1;         // tb[lo] <= item < tb[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tb[mid] <= item) lo = mid;
            else hi = mid;
        }
        const pa_state* st = base + order.run[lo];
        // the lane index passes through an empty asm each item so that the tile's lane-derived
        // addresses are not hoisted out of the item loop (they would stay live across it)
        int lane_i = lane;
        asm volatile("" : "+v"(lane_i));
        batch_tile<L, LAYOUT, MODE>(st, item - tb[lo], lds, lane_i, p, th);
    }
}

// The same items with one item per block (no item loop): for sizes whose tile code does not
// fit the register budget of the persistent loop.  Blocks past the group's items exit.
template <int L, int LAYOUT, int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) k_sweep_batch_grid(
    pa_state* base, int pos0, int pos1, BatchOrder order, SweepParams p, FastThr th)
{
    extern __shared__ uint32_t lds[];
    const int64_t* tb = work_ptr<int64_t>(base, work_layout(base->N, base->n_bins, base->capacity).batch);
    const int64_t item = tb[pos0] + (int64_t)blockIdx.x;
    if (item >= tb[pos1]) return;
    int lo = pos0, hi = pos1;  // tb[lo] <= item < tb[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tb[mid] <= item) lo = mid;
        else hi = mid;
    }
    batch_tile<L, LAYOUT, MODE>(base + order.run[lo], item - tb[lo], lds, threadIdx.x, p, th);
}

// ------------------------------------------------------------------ host side
static size_t fast_lds_limit()
{
    static size_t cached = 0;
    if (cached) return cached;
    int dev = 0, v = 0;
    size_t lim = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        lim = (size_t)v;
    cached = lim;
    return lim;
}

static int cu_count()
{
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
        cached = v;
    else
        cached = 256;
    return cached;
}

static FastThr make_thr(const SweepParams& p, int* mode)
{
    FastThr th;
    th.thi4 = p.thi[4];
    th.thi5 = p.thi[5];
    th.thi6 = p.thi[6];
    th.T4 = p.T64[4];
    th.T5 = p.T64[5];
    th.T6 = p.T64[6];
    *mode = 0;
    if (th.thi4 == 0 && th.thi5 == 0 && th.thi6 == 0) *mode = 2;
    else if (th.thi5 == 0 && th.thi6 == 0) *mode = 1;
    return th;
}

template <int L, int LAYOUT, int LPR, int MODE>
static int fast_t(const pa_run& run, const SweepParams& p, const FastThr& th, int wpb, hipStream_t s)
{
    using F = FastLayout<L, LPR>;
    const size_t limit = fast_lds_limit();
    while (F::lds_bytes(wpb) > limit && wpb > 1) --wpb;
    if (F::lds_bytes(wpb) > limit) return PA_ERR_ARG;
    const int64_t per_block = (int64_t)wpb * F::RPW;
    const int64_t blocks = (run.capacity + per_block - 1) / per_block;
    hipLaunchKernelGGL((k_sweep3f<L, LAYOUT, LPR, MODE>), dim3((unsigned)blocks), dim3(64 * wpb), F::lds_bytes(wpb),
                       s, run.state, p, th);
    return PA_OK;
}

template <int L, int LAYOUT, int LPR>
static int fast_m(const pa_run& run, const SweepParams& p, const FastThr& th, int mode, int wpb, hipStream_t s)
{
    if (mode == 2) return fast_t<L, LAYOUT, LPR, 2>(run, p, th, wpb, s);
    if (mode == 1) return fast_t<L, LAYOUT, LPR, 1>(run, p, th, wpb, s);
    return fast_t<L, LAYOUT, LPR, 0>(run, p, th, wpb, s);
}

template <int L, int LAYOUT>
static int fast_p(const pa_run& run, const SweepParams& p, const FastThr& th, int mode, int lpr, int wpb,
                  hipStream_t s)
{
    if constexpr (L % 4 != 0) {
        return fast_m<L, LAYOUT, 1>(run, p, th, mode, wpb, s);
    } else {
        if (lpr == 4) return fast_m<L, LAYOUT, 4>(run, p, th, mode, wpb, s);
        if (lpr == 2) return fast_m<L, LAYOUT, 2>(run, p, th, mode, wpb, s);
        return fast_m<L, LAYOUT, 1>(run, p, th, mode, wpb, s);
    }
}

template <int L>
static int fast_l(const pa_run& run, const SweepParams& p, const FastThr& th, int mode, int lpr, int wpb,
                  hipStream_t s)
{
    return run.layout == PA_U8 ? fast_p<L, PA_U8>(run, p, th, mode, lpr, wpb, s)
                               : fast_p<L, PA_BITS64>(run, p, th, mode, lpr, wpb, s);
}

bool fast_sweep_supported(int dim, int L) { return dim == 3 && L % 2 == 0 && L >= 4 && L <= 16; }

// returns PA_ERR_ARG when the lattice is not one the fast kernel handles
int launch_sweep_fast(const pa_run& run, const SweepParams& p, int lpr, int wpb, hipStream_t s)
{
    if (!fast_sweep_supported(run.dim, run.L) || !fast_sweep_thresholds_ok(p)) return PA_ERR_ARG;
    int mode;
    const FastThr th = make_thr(p, &mode);
    switch (run.L) {
        case 4: return fast_l<4>(run, p, th, mode, lpr, wpb, s);
        case 6: return fast_l<6>(run, p, th, mode, lpr, wpb, s);
        case 8: return fast_l<8>(run, p, th, mode, lpr, wpb, s);
        case 10: return fast_l<10>(run, p, th, mode, lpr, wpb, s);
        case 12: return fast_l<12>(run, p, th, mode, lpr, wpb, s);
        case 14: return fast_l<14>(run, p, th, mode, lpr, wpb, s);
        case 16: return fast_l<16>(run, p, th, mode, lpr, wpb, s);
        default: return PA_ERR_ARG;
    }
}

static size_t batch_lds_bytes(int L)
{
    switch (L) {
        case 4: return FastLayout<4, batch_lpr(4)>::lds_bytes(1);
        case 6: return FastLayout<6, batch_lpr(6)>::lds_bytes(1);
        case 8: return FastLayout<8, batch_lpr(8)>::lds_bytes(1);
        case 10: return FastLayout<10, batch_lpr(10)>::lds_bytes(1);
        case 12: return FastLayout<12, batch_lpr(12)>::lds_bytes(1);
        case 14: return FastLayout<14, batch_lpr(14)>::lds_bytes(1);
        default: return FastLayout<16, batch_lpr(16)>::lds_bytes(1);
    }
}

static int g_batch_blocks_per_cu = 16;
static int g_batch_order = 1;  // 0: as given, 1: larger lattices first
static int g_batch_launch = 0; // 0: by size, 1: persistent for every size, 2: one item per block for every size

// persistent loop or one item per block: by size, the loop for L = 0 mod 4 (its tile code keeps
// the one-run kernel's register budget inside the loop), one item per block otherwise
static bool group_persistent(int L)
{
    return g_batch_launch == 1 || (g_batch_launch == 0 && L % 4 == 0);
}

template <int L, int LAYOUT>
static void launch_group(pa_state* base, int pos0, int pos1, const BatchOrder& order, const SweepParams& p,
                         const FastThr& th, int mode, int64_t tiles, hipStream_t s)
{
    if (string_sweep_supported(3, L, LAYOUT)) {
        // colour strings: persistent (blocks per CU counted in waves) unless one item per wave is
        // forced
        const bool persistent = g_batch_launch != 2;
        const int64_t waves = persistent ? std::min<int64_t>((int64_t)cu_count() * g_batch_blocks_per_cu, tiles) : tiles;
        launch_sweep_strings_group(L, base, pos0, pos1, order, p, persistent, waves, s);
        return;
    }
    const size_t lds = FastLayout<L, batch_lpr(L)>::lds_bytes(1);
    const dim3 block(64);
    if (group_persistent(L)) {
        const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cu_count() * g_batch_blocks_per_cu, tiles)));
        if (mode == 2) hipLaunchKernelGGL((k_sweep_batch<L, LAYOUT, 2>), grid, block, lds, s, base, pos0, pos1, order, p, th);
        else if (mode == 1) hipLaunchKernelGGL((k_sweep_batch<L, LAYOUT, 1>), grid, block, lds, s, base, pos0, pos1, order, p, th);
        else hipLaunchKernelGGL((k_sweep_batch<L, LAYOUT, 0>), grid, block, lds, s, base, pos0, pos1, order, p, th);
    } else {
        const dim3 grid((unsigned)std::max<int64_t>(1, tiles));
        if (mode == 2) hipLaunchKernelGGL((k_sweep_batch_grid<L, LAYOUT, 2>), grid, block, lds, s, base, pos0, pos1, order, p, th);
        else if (mode == 1) hipLaunchKernelGGL((k_sweep_batch_grid<L, LAYOUT, 1>), grid, block, lds, s, base, pos0, pos1, order, p, th);
        else hipLaunchKernelGGL((k_sweep_batch_grid<L, LAYOUT, 0>), grid, block, lds, s, base, pos0, pos1, order, p, th);
    }
}

template <int LAYOUT>
static void launch_group_L(int L, pa_state* base, int pos0, int pos1, const BatchOrder& order, const SweepParams& p,
                           const FastThr& th, int mode, int64_t tiles, hipStream_t s)
{
    switch (L) {
        case 4: launch_group<4, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
        case 6: launch_group<6, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
        case 8: launch_group<8, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
        case 10: launch_group<10, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
        case 12: launch_group<12, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
        case 14: launch_group<14, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
        default: launch_group<16, LAYOUT>(base, pos0, pos1, order, p, th, mode, tiles, s); break;
    }
}

// Persistent sweep of n_runs contiguous runs (3D, even L in 4..16, one layout): the runs are
// grouped by lattice size (groups ordered by the cost of a tile, larger first, or by first
// appearance), one work list over all groups, one persistent launch per group.
int launch_sweep_batch(const pa_run* runs, int n_runs, const SweepParams& p, hipStream_t s)
{
    if (n_runs > kMaxBatch || !fast_sweep_thresholds_ok(p)) return PA_ERR_ARG;
    for (int r = 0; r < n_runs; ++r)
        if (batch_lds_bytes(runs[r].L) > fast_lds_limit()) return PA_ERR_ARG;
    // distinct sizes in order of first appearance, then (order 1) by tile cost, larger first
    int sizes[kMaxBatch], n_sizes = 0;
    for (int r = 0; r < n_runs; ++r) {
        bool seen = false;
        for (int g = 0; g < n_sizes; ++g) seen = seen || sizes[g] == runs[r].L;
        if (!seen) sizes[n_sizes++] = runs[r].L;
    }
    auto tile_cost = [](int L) { return (double)L * L * L * 64 / batch_lpr(L); };
    if (g_batch_order == 1)
        std::stable_sort(sizes, sizes + n_sizes, [&](int a, int b) { return tile_cost(a) > tile_cost(b); });
    BatchOrder order;
    int group_end[kMaxBatch];
    int64_t group_tiles[kMaxBatch];
    int pos = 0;
    for (int g = 0; g < n_sizes; ++g) {
        group_tiles[g] = 0;
        for (int r = 0; r < n_runs; ++r) {
            if (runs[r].L != sizes[g]) continue;
            order.run[pos++] = (uint16_t)r;
            const int rpw = batch_tile_replicas(runs[r].L, runs[r].layout);
            group_tiles[g] += (runs[r].capacity + rpw - 1) / rpw;
        }
        group_end[g] = pos;
    }
    int mode;
    const FastThr th = make_thr(p, &mode);
    pa_state* base = runs[0].state;
    hipLaunchKernelGGL(k_batch_tiles, dim3(1), dim3(256), 0, s, base, n_runs, order);
    for (int g = 0, pos0 = 0; g < n_sizes; pos0 = group_end[g], ++g) {
        if (runs[0].layout == PA_U8)
            launch_group_L<PA_U8>(sizes[g], base, pos0, group_end[g], order, p, th, mode, group_tiles[g], s);
        else
            launch_group_L<PA_BITS64>(sizes[g], base, pos0, group_end[g], order, p, th, mode, group_tiles[g], s);
    }
    return PA_OK;
}

}  // namespace pa

// batch schedule for the autotuner: blocks per CU of a persistent launch (1..32), order of the
// size groups (0: first appearance, 1: larger tiles first), launch form (0: by size, 1: persistent
// loop, 2: one item per block); (0, 0, 0) restores the defaults
extern "C" int pa_set_batch_config(int blocks_per_cu, int order, int launch)
{
    if (blocks_per_cu == 0 && order == 0 && launch == 0) {
        pa::g_batch_blocks_per_cu = 16;
        pa::g_batch_order = 1;
        pa::g_batch_launch = 0;
        return PA_OK;
    }
    if (blocks_per_cu < 1 || blocks_per_cu > 32 || order < 0 || order > 1 || launch < 0 || launch > 2)
        return PA_ERR_ARG;
    pa::g_batch_blocks_per_cu = blocks_per_cu;
    pa::g_batch_order = order;
    pa::g_batch_launch = launch;
    return PA_OK;
}
