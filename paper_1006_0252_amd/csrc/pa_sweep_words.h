// Device helpers of the sweep kernels whose LDS words hold 32 sites of one colour: the bit-sliced
// bond count, the packed 16-bit first look against a bound table, and the exact tie paths.
//
// The decision step is shared: a word's byte i holds eight sites whose Metropolis fields are the
// eight 16-bit fields of one Philox call (field k for bit k of the byte), so a word takes four
// whole calls.  The kernels differ only in where a word's sites lie on the lattice and hence how its
// neighbour words are formed.
#pragma once

#include "pa_common.h"
#include "pa_sweep_util.h"

namespace pa {
namespace words {

// thresholds by class c = 4, 5, 6 (c bonds of the site with J s_i s_j = -1 in the kernels' bit
// convention: c <= 3 flips outright)
struct Thr {
    uint32_t thi4, thi5, thi6;
    uint64_t T4, T5, T6;
};

inline Thr make_thr(const SweepParams& p)
{
    Thr th;
    th.thi4 = p.thi[4];
    th.thi5 = p.thi[5];
    th.thi6 = p.thi[6];
    th.T4 = p.T64[4];
    th.T5 = p.T64[5];
    th.T6 = p.T64[6];
    return th;
}

// every top of c >= 4 zero: only u = 0 can accept (the second kernel template)
inline bool all_tops_zero(const Thr& th) { return th.thi4 == 0 && th.thi5 == 0 && th.thi6 == 0; }

// Philox4x32-10 with the same rounds as philox10 (the same values), for callers whose counter
// words 0, 2, 3 and key are wave-uniform and whose word 1 (the replica) varies over the wave.  Then
// the first two rounds' products (but one, which does not depend on the call) are wave-uniform,
// and each xor is written so that its uniform inputs combine first: the scalar unit does those, and
// the vector unit one v_xor_b32 (a three-input v_bitop3_b32 with two scalar operands would need a
// copy into a vector register, and a fully uniform one would pull its products onto the vector
// unit).  From the fourth round on every input varies and each xor is one v_bitop3_b32.
__device__ inline uint4v philox10_lane(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    // round 1: both products uniform; the replica word enters n0
    uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
    uint32_t n0 = c1 ^ ((uint32_t)(p1 >> 32) ^ k0);
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
    // round 2: p0 varies (but not with the call), p1 and n0 are uniform
    p0 = (uint64_t)M0 * c0;
    p1 = (uint64_t)M1 * c2;
    n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
    // round 3: p0 uniform, p1 varies
    p0 = (uint64_t)M0 * c0;
    p1 = (uint64_t)M1 * c2;
    n0 = (uint32_t)(p1 >> 32) ^ (c1 ^ k0);
    n2 = ((uint32_t)(p0 >> 32) ^ k1) ^ c3;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
    // round 4: c3 (the low half of round 3's p0) is still uniform
    p0 = (uint64_t)M0 * c0;
    p1 = (uint64_t)M1 * c2;
    n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    n2 = (uint32_t)(p0 >> 32) ^ (c3 ^ k1);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += W0;
    k1 += W1;
#pragma unroll
    for (int round = 4; round < 10; ++round) {
        p0 = (uint64_t)M0 * c0;
        p1 = (uint64_t)M1 * c2;
        n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += W0;
        k1 += W1;
    }
    return {c0, c1, c2, c3};
}

// Philox key and counter words of one lane's replica in one colour phase
struct Lane {
    uint32_t rr, ctr2, k0, k1;
};

// byte B of v, times 8: the offset of entry v.byte[B] of a table of 8-byte entries (one SDWA op)
template <int B>
__device__ __forceinline__ uint32_t byte_x8(uint32_t v)
{
    uint32_t r;
    if constexpr (B == 0)
        asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0" : "=v"(r) : "v"(v));
    else if constexpr (B == 1)
        asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1" : "=v"(r) : "v"(v));
    else if constexpr (B == 2)
        asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2" : "=v"(r) : "v"(v));
    else
        asm("v_lshlrev_b32_sdwa %0, 3, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3" : "=v"(r) : "v"(v));
    return r;
}

// entry idx_bytes.byte[B] of a table of 8-byte entries in LDS (static LDS: the table's offset folds
// into the load's immediate)
template <int B>
__device__ __forceinline__ uint2 tab_entry(const uint2* tt, uint32_t idx_bytes)
{
    return *reinterpret_cast<const uint2*>(reinterpret_cast<const char*>(tt) + byte_x8<B>(idx_bytes));
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96); }
__device__ __forceinline__ uint32_t maj3(uint32_t a, uint32_t b, uint32_t c) { return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8); }
// bits of a where m is set, of b elsewhere: one v_bitop3_b32 (m ? a : b is truth table 0xCA), also
// when m is not a constant (the optimiser would spend a second op on ~m)
__device__ __forceinline__ uint32_t select_bits(uint32_t m, uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_bitop3_b32(m, a, b, 0xCA);
}

// raw | (e << k) as one v_lshl_or_b32; k is a constant after unrolling, and the switch folds to
// the one asm statement with k as an inline constant
#define PA_LSHL_OR(K) \
    case K: asm("v_lshl_or_b32 %0, %1, " #K ", %2" : "=v"(r) : "v"(e), "v"(raw)); break;
__device__ __forceinline__ uint32_t lshl_or(uint32_t e, int k, uint32_t raw)
{
    uint32_t r = raw | (e << k);
    switch (k) {
        PA_LSHL_OR(0) PA_LSHL_OR(2) PA_LSHL_OR(4) PA_LSHL_OR(6) PA_LSHL_OR(8) PA_LSHL_OR(10) PA_LSHL_OR(12)
        PA_LSHL_OR(14)
        default: break;
    }
    return r;
}
#undef PA_LSHL_OR

// min(saturated(b - w), 2) per 16-bit half; the min is written out, since as an expression the
// optimiser may expand it into compares and selects per half
__device__ __forceinline__ uint32_t first_look(uint32_t b, uint32_t w)
{
    typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
    const u16x2 d = __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, b), __builtin_bit_cast(u16x2, w));
    const u16x2 two = {2, 2};
    uint32_t e;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(e) : "v"(d), "v"(two));
    return e;
}

// bit-sliced count of the six bond words: c = c0 + 2 c1 + 4 c2 per bit (two full adders, a half
// adder and a final full adder)
__device__ __forceinline__ void bond_count(uint32_t b0, uint32_t b1, uint32_t b2, uint32_t b3, uint32_t b4,
                                           uint32_t b5, uint32_t& c0, uint32_t& c1, uint32_t& c2)
{
    const uint32_t s1 = xor3(b0, b1, b2), k1 = maj3(b0, b1, b2);
    const uint32_t s2 = xor3(b3, b4, b5), k2 = maj3(b3, b4, b5);
    c0 = s1 ^ s2;
    const uint32_t k3 = s1 & s2;
    c1 = xor3(k1, k2, k3);
    c2 = maj3(k1, k2, k3);
}

// Where a word's sites are: bit b's site index is base + byte_step (b >> 3) + 2 (b & 7) + bit b of
// odd (the site's x parity where it varies within the word); byte i's Philox call is call0 +
// call_step i.
struct WordSites {
    uint32_t call0, call_step, base, byte_step, odd;
};

__device__ __forceinline__ uint32_t site_of(const WordSites& ws, int b)
{
    return ws.base + ws.byte_step * (uint32_t)(b >> 3) + 2u * (uint32_t)(b & 7) + ((ws.odd >> b) & 1u);
}

// Exact decisions of first-look ties (Sec. II: the 16-bit field u is the top of a 64-bit uniform;
// when it equals the top of the threshold, the 48 low bits decide).  A wave takes these paths when
// any of its lanes has a tie, so they touch only the tied sites.
//
// General thresholds: bits = candidate sites whose field equals the top of their class, so u is
// that top and only the low bits need drawing.  Returns the accepted ones.  Arguments come as
// scalars: a structure passed by value to this out-of-line call would go through private memory.
static __device__ __noinline__ uint32_t resolve_ties(uint32_t bits, uint32_t c0, uint32_t c1, uint32_t base,
                                                     uint32_t byte_step, uint32_t odd, uint32_t rr, uint32_t ctr2,
                                                     uint32_t k0, uint32_t k1, uint32_t thi4, uint32_t thi5,
                                                     uint32_t thi6, uint64_t T4, uint64_t T5, uint64_t T6)
{
    const WordSites ws = {0, 0, base, byte_step, odd};
    uint32_t racc = 0;
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        const int cls = (int)((c0 >> b) & 1u) + 2 * (int)((c1 >> b) & 1u);
        const uint32_t u = cls == 0 ? thi4 : (cls == 1 ? thi5 : thi6);
        const uint64_t T = cls == 0 ? T4 : (cls == 1 ? T5 : T6);
        racc |= (uint32_t)tie_accept(u, T, site_of(ws, b), rr, ctr2, k0, k1) << b;
    }
    return racc;
}

// Every top zero: a candidate accepts only if u = 0 and its low bits fall below the threshold.
// bytes: the bytes (bit i) whose fields hold a zero; their Philox calls are drawn again.
static __device__ __noinline__ uint32_t resolve_zero_bytes(uint32_t bytes, uint32_t cand, uint32_t c0, uint32_t c1,
                                                           uint32_t call0, uint32_t call_step, uint32_t base,
                                                           uint32_t byte_step, uint32_t odd, uint32_t rr,
                                                           uint32_t ctr2, uint32_t k0, uint32_t k1, uint64_t T4,
                                                           uint64_t T5, uint64_t T6)
{
    const WordSites ws = {call0, call_step, base, byte_step, odd};
    uint32_t bits = 0;
    while (bytes) {
        const int i = __builtin_ctz(bytes);
        bytes &= bytes - 1u;
        const uint4v v = philox10(call0 + call_step * (uint32_t)i, rr, ctr2, kTagMet, k0, k1);
        for (int k = 0; k < 8; ++k)
            if (field16(v, k) == 0) bits |= 1u << (8 * i + k);
    }
    bits &= cand;
    uint32_t racc = 0;
    while (bits) {
        const int b = __builtin_ctz(bits);
        bits &= bits - 1u;
        const int cls = (int)((c0 >> b) & 1u) + 2 * (int)((c1 >> b) & 1u);
        const uint64_t T = cls == 0 ? T4 : (cls == 1 ? T5 : T6);
        racc |= (uint32_t)tie_accept(0u, T, site_of(ws, b), rr, ctr2, k0, k1) << b;
    }
    return racc;
}

// The Metropolis decision for the 32 sites of word w with bond classes c0, c1, c2 (c2 set: a
// candidate, c >= 4; clear: flips outright); returns the new word.  MODE 0: bounds from the
// 256-entry table tt; MODE 2: every top zero.  UNIFORM_CALLS: call0 is the same over the wave
// (philox10_lane keeps the uniform rounds on the scalar unit).  ws_fn() gives the word's WordSites
// (only the rare tie paths need them).  NBYTES < 4: only bytes 0 .. NBYTES - 1 hold sites (the last
// word of a string); the other bytes' calls are not drawn and their bits come out as non-candidates
// would (flipped), for the caller to ignore.
template <int MODE, bool UNIFORM_CALLS, int NBYTES = 4, class WS>
__device__ __forceinline__ uint32_t decide_word(uint32_t w, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t call0,
                                                uint32_t call_step, const uint2* tt, const Lane& c, const Thr& th,
                                                WS ws_fn)
{
    if constexpr (MODE == 2) {
        // candidates reject unless u = 0 (a tie): the minimum field of each byte, then of the word
        typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
        u16x2 m[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i >= NBYTES) {
                const u16x2 none = {0xFFFF, 0xFFFF};
                m[i] = none;
                continue;
            }
            const uint4v v = UNIFORM_CALLS ? philox10_lane(call0 + call_step * i, c.rr, c.ctr2, kTagMet, c.k0, c.k1)
                                           : philox10(call0 + call_step * i, c.rr, c.ctr2, kTagMet, c.k0, c.k1);
            m[i] = __builtin_elementwise_min(
                __builtin_elementwise_min(__builtin_bit_cast(u16x2, v.x), __builtin_bit_cast(u16x2, v.y)),
                __builtin_elementwise_min(__builtin_bit_cast(u16x2, v.z), __builtin_bit_cast(u16x2, v.w)));
        }
        const u16x2 zmin = __builtin_elementwise_min(__builtin_elementwise_min(m[0], m[1]),
                                                     __builtin_elementwise_min(m[2], m[3]));
        uint32_t nw = w ^ ~c2;
        if (zmin.x == 0 || zmin.y == 0) {
            uint32_t bytes = 0;
#pragma unroll
            for (int i = 0; i < NBYTES; ++i) bytes |= (uint32_t)(m[i].x == 0 || m[i].y == 0) << i;
            const WordSites ws = ws_fn();
            nw = w ^ (~c2 | resolve_zero_bytes(bytes, c2, c0, c1, call0, call_step, ws.base, ws.byte_step, ws.odd,
                                               c.rr, c.ctr2, c.k0, c.k1, th.T4, th.T5, th.T6));
        }
        return nw;
    } else {
        // class bits of sites k = 0..3 (lo) and 4..7 (hi) of byte i as byte i: c0 in the low nibble,
        // c1 in the high one
        const uint32_t cl = select_bits(0x0F0F0F0Fu, c0, c1 << 4);
        const uint32_t ch = select_bits(0x0F0F0F0Fu, c0 >> 4, c1);
        // outcomes: byte i's Philox word j (sites 2 j, 2 j + 1) at 2 j + 8 (i & 1) and 16 higher,
        // bytes 0, 1 in ra and bytes 2, 3 in rb
        uint32_t ra = 0, rb = 0;
#pragma unroll
        for (int i = 0; i < NBYTES; ++i) {
            const uint4v v = UNIFORM_CALLS ? philox10_lane(call0 + call_step * i, c.rr, c.ctr2, kTagMet, c.k0, c.k1)
                                           : philox10(call0 + call_step * i, c.rr, c.ctr2, kTagMet, c.k0, c.k1);
            uint2 bl, bh;
            if (i == 0) { bl = tab_entry<0>(tt, cl); bh = tab_entry<0>(tt, ch); }
            else if (i == 1) { bl = tab_entry<1>(tt, cl); bh = tab_entry<1>(tt, ch); }
            else if (i == 2) { bl = tab_entry<2>(tt, cl); bh = tab_entry<2>(tt, ch); }
            else { bl = tab_entry<3>(tt, cl); bh = tab_entry<3>(tt, ch); }
            const uint32_t e0 = first_look(bl.x, v.x), e1 = first_look(bl.y, v.y);
            const uint32_t e2 = first_look(bh.x, v.z), e3 = first_look(bh.y, v.w);
            const int o = 8 * (i & 1);
            uint32_t r = i < 2 ? ra : rb;
            r = (i & 1) ? lshl_or(e0, o, r) : e0;
            r = lshl_or(e1, o + 2, r);
            r = lshl_or(e2, o + 4, r);
            r = lshl_or(e3, o + 6, r);
            if (i < 2) ra = r;
            else rb = r;
        }
        // accept bits (the high bit of each field) to the sites' bits 8 i + k: bytes 0, 1 even k from
        // ra >> 1, odd k from ra >> 16; bytes 2, 3 even k from rb << 15, odd k in place
        uint32_t acc = select_bits(0x0000FFFFu, select_bits(0x5555u, ra >> 1, ra >> 16),
                                   select_bits(0x55550000u, rb << 15, rb));
        if (((ra | rb) & 0x55555555u) != 0) {
            // tie bits (the low bit of each field) to the sites' bits likewise: ra's even k in place,
            // odd k from ra >> 15; rb's even k from rb << 16, odd k from rb << 1
            const uint32_t ties = select_bits(0x0000FFFFu, select_bits(0x5555u, ra, ra >> 15),
                                              select_bits(0x55550000u, rb << 16, rb << 1)) & c2;
            if (ties) {
                const WordSites ws = ws_fn();
                acc |= resolve_ties(ties, c0, c1, ws.base, ws.byte_step, ws.odd, c.rr, c.ctr2, c.k0, c.k1, th.thi4,
                                    th.thi5, th.thi6, th.T4, th.T5, th.T6);
            }
        }
        return w ^ (~c2 | acc);
    }
}

// first-look bounds of four sites by their class bits: entry n (low nibble: c0 of sites 0..3, high
// nibble: c1 of the same sites) holds (bound(site 0) | bound(site 1) << 16, bound(site 2) |
// bound(site 3) << 16), bound = top + 1 of class c0 + 2 c1 (c = 4, 5, 6; 3 cannot occur at a
// candidate).  The launch guarantees top <= 0xFFFE.
__device__ inline void build_bounds(uint2* tt, const Thr& th, int tid, int nthr)
{
    const uint32_t b[4] = {th.thi4 + 1u, th.thi5 + 1u, th.thi6 + 1u, th.thi6 + 1u};
    for (int n = tid; n < 256; n += nthr) {
        uint32_t a[4];
        for (int t = 0; t < 4; ++t) a[t] = ((n >> t) & 1) | (((n >> (4 + t)) & 1) << 1);
        tt[n] = make_uint2(b[a[0]] | (b[a[1]] << 16), b[a[2]] | (b[a[3]] << 16));
    }
}

// the 16 even-x and the 16 odd-x bits of two 16-bit rows (x = row a | row b << 16) as bytes:
// returns the even bits of row a in byte 0 and of row b in byte 2, odd bits likewise in *odd
__device__ __forceinline__ uint32_t split_colours(uint32_t x, uint32_t* odd)
{
    uint32_t e = x & 0x55555555u, o = (x >> 1) & 0x55555555u;
    e = (e | (e >> 1)) & 0x33333333u;
    o = (o | (o >> 1)) & 0x33333333u;
    e = (e | (e >> 2)) & 0x0F0F0F0Fu;
    o = (o | (o >> 2)) & 0x0F0F0F0Fu;
    e = (e | (e >> 4)) & 0x00FF00FFu;
    o = (o | (o >> 4)) & 0x00FF00FFu;
    *odd = o;
    return e;
}

// inverse: bytes 0 and 2 of e (even x) and of o (odd x) back to two 16-bit rows
__device__ __forceinline__ uint32_t merge_colours(uint32_t e, uint32_t o)
{
    e = (e | (e << 4)) & 0x0F0F0F0Fu;
    o = (o | (o << 4)) & 0x0F0F0F0Fu;
    e = (e | (e << 2)) & 0x33333333u;
    o = (o | (o << 2)) & 0x33333333u;
    e = (e | (e << 1)) & 0x55555555u;
    o = (o | (o << 1)) & 0x55555555u;
    return e | (o << 1);
}

}  // namespace words
}  // namespace pa
