// Metropolis sweeps of the L = 16 cube, bit-packed populations, with every bit of a 32-bit LDS word
// a site of one colour: the same sample as the generic kernel (same Philox fields, same
// acceptance rule, same checkerboard order), with half the bond-count work per attempt of the
// row-pair kernel (whose words carry both colours).
//
// Word layout.  A replica's plane z is eight words W(sigma, rho, h): byte i (0..3) of W holds the
// row y = rho + 2 i + 8 h, bit k (0..7) of that byte the site x = 2 k + sigma.  Every site of a word
// has colour (sigma + rho + z) mod 2, so a colour phase of plane z updates the four words with
// sigma + rho = col + z (mod 2), and every neighbour word is one of the other colour:
//  - x: the word W(1 - sigma, rho, h) holds the x-neighbour on one side bit for bit, the other side
//    is the same word with each byte rotated by one bit (left for sigma = 0, right for sigma = 1);
//  - y: W(sigma, 1 - rho, h) holds one y-neighbour bit for bit, the other is the byte-shifted funnel
//    of W(sigma, 1 - rho, h) and W(sigma, 1 - rho, 1 - h) (one v_alignbit_b32);
//  - z: W(sigma, rho, h) of planes z + 1 and z - 1, bit for bit.
// Row y's eight sites of a colour are the eight 16-bit fields of Philox call 16 z + y (field k for
// site x = 2 k + sigma), so a word takes four whole calls.
//
// First look (Sec. II, the Metropolis rule with exact 64-bit thresholds): per Philox word the two
// fields are compared at once with packed 16-bit ops against bounds top + 1 looked up by the class
// bits of four sites; min(saturated(bound - u), 2) gives 0 (reject), 1 (tie: u equals the top) or 2
// (accept).  The two-bit outcomes of rows 0, 1 and of rows 2, 3 gather in two words, placed so
// that the accept bits reach their sites' bit positions with three shifts and three bit-field
// selects.  Ties are resolved exactly with the 48 low bits in a separate (rare) path.  When every
// top of a class c >= 4 is zero (beta above ln 2^16 / 4) only u = 0 can accept; the table is not
// needed and a running minimum of the fields finds the ties.
//
// Launch: one block of four waves per 64-replica bit-packed group; a wave holds 16 replicas, four
// lanes per replica, lane j taking planes 4 j .. 4 j + 3 (so the plane parity, and with it which
// words a phase updates, is the same over the wave).  All LDS is static, so table offsets fold into
// the instructions' immediate offsets.
#include "pa_common.h"
#include "pa_sweep_util.h"
#include "pa_sweep_words.h"

namespace pa {

namespace colour {

using namespace words;

constexpr int L = 16;
constexpr int NR = L * L;           // rows per replica
constexpr int RPW = 16;             // replicas per wave
constexpr int WPB = 4;              // waves per block: one 64-replica group
constexpr int PS = 8 * RPW + 4;     // dwords per plane of a wave (eight words per replica; padding
                                    // staggers the four lanes of a replica over the banks)
constexpr int ROWW = L * PS;        // dwords of a wave's rows
constexpr int JS = 8 * 6 + 2;       // dwords of coupling masks per plane (six per word)

// The coupling masks (bit set where J = -1) of every word, by role: 0 the aligned x partner, 1 the
// rotated one, 2 the aligned y word, 3 the funnel-shifted one, 4 and 5 the z + 1 and z - 1 words.
// The x partner is the +x bond for sigma = 0 and the -x bond for sigma = 1; the aligned y word is
// the +y bond for rho = 0 and the -y bond for rho = 1.  Thread t (of 256) takes lattice row t
// (y = t mod 16, z = t / 16): the six bond masks of its 16 sites (the -y and -z bonds are the +y
// bonds of row y - 1 and the +z bonds of plane z - 1), split into even-x and odd-x bytes, become
// byte (y >> 1) & 3 of the masks of the words W(sigma, y & 1, y >> 3) of plane z.
__device__ void build_masks(const int8_t* J, uint32_t* jt, int tid)
{
    const int y = tid & (L - 1), z = tid >> 4;
    const int8_t* a = J + 3 * L * (y + L * z);
    const int8_t* b = J + 3 * L * (((y + L - 1) & (L - 1)) + L * z);
    const int8_t* c = J + 3 * L * (y + L * ((z + L - 1) & (L - 1)));
    uint32_t px = 0, py = 0, pz = 0, my = 0, mz = 0;
#pragma unroll
    for (int x = 0; x < L; ++x) {
        px |= (uint32_t)(a[3 * x + 0] < 0) << x;
        py |= (uint32_t)(a[3 * x + 1] < 0) << x;
        pz |= (uint32_t)(a[3 * x + 2] < 0) << x;
        my |= (uint32_t)(b[3 * x + 1] < 0) << x;
        mz |= (uint32_t)(c[3 * x + 2] < 0) << x;
    }
    const uint32_t mx = ((px << 1) | (px >> (L - 1))) & 0xFFFFu;  // the -x bond of x is the +x bond of x - 1
    const int rh = y & 1, i = (y >> 1) & 3, h = y >> 3;
    // roles for sigma = 0: +x, -x, then (rho = 0) +y, -y or (rho = 1) -y, +y, then +z, -z
    uint32_t o_x, o_y, o_z;
    const uint32_t e_x = split_colours(px | (mx << 16), &o_x);
    const uint32_t e_y = split_colours((rh ? my : py) | ((rh ? py : my) << 16), &o_y);
    const uint32_t e_z = split_colours(pz | (mz << 16), &o_z);
    uint8_t* jb = reinterpret_cast<uint8_t*>(jt);
    uint8_t* w0 = jb + 4 * (z * JS + (rh * 2 + h) * 6) + i;  // sigma = 0
    uint8_t* w1 = w0 + 4 * 4 * 6;                             // sigma = 1
    w0[0] = (uint8_t)e_x;          // even x: aligned partner +x, rotated -x
    w0[4] = (uint8_t)(e_x >> 16);
    w1[0] = (uint8_t)(o_x >> 16);  // odd x: aligned partner -x, rotated +x
    w1[4] = (uint8_t)o_x;
    w0[8] = (uint8_t)e_y;
    w0[12] = (uint8_t)(e_y >> 16);
    w1[8] = (uint8_t)o_y;
    w1[12] = (uint8_t)(o_y >> 16);
    w0[16] = (uint8_t)e_z;
    w0[20] = (uint8_t)(e_z >> 16);
    w1[16] = (uint8_t)o_z;
    w1[20] = (uint8_t)(o_z >> 16);
}

// The group's rows between HBM (bit-packed: row rho of replica r of group g is the 16-bit word
// ((g NR + rho) 64 + r) of the spin buffer) and the block's LDS words.  A thread takes four
// replicas (one 8-byte load per row, so a row of the group is one 128-byte line) and one (z, rho,
// h) item: four rows, whose even and odd sites become the words W(0, rho, h) and W(1, rho, h).
// Stores skip the replicas at or past R.
template <bool STORE>
__device__ void group_io(const pa_state* st, int64_t g, uint32_t* rows, int64_t R, int tid)
{
    uint64_t* G = reinterpret_cast<uint64_t*>((uint8_t*)st->spins[st->cur] + g * (int64_t)NR * 128);
    const int rq = tid & 15;  // replicas 4 rq .. 4 rq + 3 of the group
    for (int item = tid >> 4; item < L * 4; item += 16) {
        const int z = item >> 2, rh = (item >> 1) & 1, h = item & 1;
        const int row0 = rh + 8 * h + L * z;  // rows row0 + 2 i, i = 0..3
        uint32_t* W[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int rep = 4 * rq + m;
            W[m] = rows + (rep >> 4) * ROWW + z * PS + (rh * 2 + h) * RPW + (rep & 15);
        }
        if (!STORE) {
            uint64_t v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = G[(row0 + 2 * i) * 16 + rq];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t r0 = (uint32_t)(v[0] >> (16 * m)) & 0xFFFFu, r1 = (uint32_t)(v[1] >> (16 * m)) & 0xFFFFu;
                const uint32_t r2 = (uint32_t)(v[2] >> (16 * m)) & 0xFFFFu, r3 = (uint32_t)(v[3] >> (16 * m)) & 0xFFFFu;
                uint32_t o01, o23;
                const uint32_t e01 = split_colours(r0 | (r1 << 16), &o01);
                const uint32_t e23 = split_colours(r2 | (r3 << 16), &o23);
                // bytes 0 and 2 of the 01 word, then of the 23 word
                W[m][0] = __builtin_amdgcn_perm(e23, e01, 0x06040200u);
                W[m][4 * RPW] = __builtin_amdgcn_perm(o23, o01, 0x06040200u);
            }
        } else {
            uint64_t v[4] = {0, 0, 0, 0};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const uint32_t w0 = W[m][0], w1 = W[m][4 * RPW];
                // bytes 0, 1 of a word to bytes 0, 2 (rows 0, 1), bytes 2, 3 likewise (rows 2, 3)
                const uint32_t r01 = merge_colours(__builtin_amdgcn_perm(0u, w0, 0x0C010C00u),
                                                   __builtin_amdgcn_perm(0u, w1, 0x0C010C00u));
                const uint32_t r23 = merge_colours(__builtin_amdgcn_perm(0u, w0, 0x0C030C02u),
                                                   __builtin_amdgcn_perm(0u, w1, 0x0C030C02u));
                v[0] |= (uint64_t)(r01 & 0xFFFFu) << (16 * m);
                v[1] |= (uint64_t)(r01 >> 16) << (16 * m);
                v[2] |= (uint64_t)(r23 & 0xFFFFu) << (16 * m);
                v[3] |= (uint64_t)(r23 >> 16) << (16 * m);
            }
            const int64_t r0 = g * 64 + 4 * rq;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint64_t* a = G + (row0 + 2 * i) * 16 + rq;
                if (r0 + 3 < R) {
                    *a = v[i];
                } else {
                    uint16_t* a16 = reinterpret_cast<uint16_t*>(a);
                    for (int m = 0; m < 4; ++m)
                        if (r0 + m < R) a16[m] = (uint16_t)(v[i] >> (16 * m));
                }
            }
        }
    }
}

// one colour phase of the two words W(sigma, RHO, h), h = 0, 1, of plane z (rows: the lane's
// replica column of its wave's rows)
template <int MODE, int RHO>
__device__ __forceinline__ void update_words(uint32_t* rows, const uint32_t* jt, const uint2* tt, int z, int sg,
                                             const Lane& c, const Thr& th)
{
    const int zp = (z + 1) & (L - 1), zm = (z + L - 1) & (L - 1);
    uint32_t* own = rows + z * PS + (sg * 4 + RHO * 2) * RPW;
    const uint32_t* part = rows + z * PS + ((sg ^ 1) * 4 + RHO * 2) * RPW;
    const uint32_t* ynb = rows + z * PS + (sg * 4 + (RHO ^ 1) * 2) * RPW;
    const uint32_t* zpw = rows + zp * PS + (sg * 4 + RHO * 2) * RPW;
    const uint32_t* zmw = rows + zm * PS + (sg * 4 + RHO * 2) * RPW;
    const uint32_t* jm = jt + z * JS + (sg * 4 + RHO * 2) * 6;
    // the rotated x partner: each byte left by one bit (sigma = 0: site x - 1) or right by one
    // (sigma = 1: site x + 1)
    const uint32_t mx = sg ? 0x7F7F7F7Fu : 0x01010101u;
    const int ax = sg ? 1 : 7, bx = sg ? 7 : 1;
    const uint32_t y0 = ynb[0], y1 = ynb[RPW];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t w = own[h * RPW];
        const uint32_t p = part[h * RPW];
        const uint32_t ya = h ? y1 : y0, yo = h ? y0 : y1;
        // rho = 0: row y - 1 is byte i - 1 of the same-h word, byte 3 of the other for i = 0;
        // rho = 1: row y + 1 is byte i + 1, byte 0 of the other for i = 3
        const uint32_t ys = RHO == 0 ? __builtin_amdgcn_alignbit(ya, yo, 24) : __builtin_amdgcn_alignbit(yo, ya, 8);
        const uint32_t pr = select_bits(mx, p >> ax, p << bx);
        const uint32_t* J = jm + h * 6;
        uint32_t c0, c1, c2;
        bond_count(xor3(w, p, J[0]), xor3(w, pr, J[1]), xor3(w, ya, J[2]), xor3(w, ys, J[3]), xor3(w, zpw[h * RPW], J[4]),
                   xor3(w, zmw[h * RPW], J[5]), c0, c1, c2);
        const uint32_t call0 = (uint32_t)(L * z + RHO + 8 * h);  // row i: call0 + 2 i
        // site (i, k): x = 2 k + sigma, y = rho + 2 i + 8 h
        const uint32_t site0 = (uint32_t)(sg + L * (RHO + 8 * h) + NR * z);
        const uint32_t nw = decide_word<MODE, false>(w, c0, c1, c2, call0, 2u, tt, c, th,
                                              [&]() { return WordSites{call0, 2u, site0, 2u * L, 0u}; });
        own[h * RPW] = nw;
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_sweep16c(const pa_state* __restrict__ st, SweepParams p, Thr th)
{
    __shared__ uint32_t s_rows[WPB * ROWW];
    __shared__ uint32_t s_jt[L * JS];
    __shared__ uint2 s_tt[256];
    if (st->status) return;  // sticky error: the population stays as it is
    const int64_t R = st->R;
    const int64_t g = blockIdx.x;
    if (g * 64 >= R) return;  // the whole block is past the population
    const int tid = threadIdx.x;
    build_masks(st->J, s_jt, tid);
    if (MODE != 2) build_bounds(s_tt, th, tid, 256);
    group_io<false>(st, g, s_rows, R, tid);
    __syncthreads();

    const int wave = tid >> 6, lane = tid & 63;
    const int q = lane & (RPW - 1), j = lane >> 4;
    uint32_t* rows = s_rows + wave * ROWW + q;
    Lane c;
    c.rr = (uint32_t)(g * 64 + wave * RPW + q);
    c.k0 = (uint32_t)st->seed;
    c.k1 = (uint32_t)(st->seed >> 32);
    for (int s = 0; s < p.n_sweeps; ++s) {
        for (int col = 0; col < 2; ++col) {
            c.ctr2 = (uint32_t)(2 * (p.t0 + s) + col);
            for (int t = 0; t < 4; ++t) {
                const int z = 4 * j + t;
                // words of colour col: sigma + rho = col + z (mod 2), and z = t (mod 2) over the wave
                const int sg0 = (col + t) & 1;
                update_words<MODE, 0>(rows, s_jt, s_tt, z, sg0, c, th);
                update_words<MODE, 1>(rows, s_jt, s_tt, z, sg0 ^ 1, c, th);
            }
            // the other colour reads these words next (other lanes of the replica too)
            wave_sync();
        }
    }

    // energy of the final configuration: E = n_bonds - 2 (bonds whose word bit is set), counting
    // each site's +x, +y and +z bonds
    int neg = 0;
    for (int t = 0; t < 4; ++t) {
        const int z = 4 * j + t, zp = (z + 1) & (L - 1);
#pragma unroll
        for (int wi = 0; wi < 8; ++wi) {
            const int sg = wi >> 2, rh = (wi >> 1) & 1, h = wi & 1;
            const uint32_t w = rows[z * PS + wi * RPW];
            const uint32_t p = rows[z * PS + (wi ^ 4) * RPW];
            const uint32_t ya = rows[z * PS + (wi ^ 2) * RPW];
            const uint32_t yo = rows[z * PS + (wi ^ 3) * RPW];
            const uint32_t* J = s_jt + z * JS + wi * 6;
            // +x: the partner itself (sigma = 0) or its bytes rotated right (sigma = 1)
            const uint32_t px = sg ? (((p >> 1) & 0x7F7F7F7Fu) | ((p << 7) & 0x80808080u)) : p;
            // +y: the aligned word (rho = 0) or the funnel of the pair (rho = 1)
            const uint32_t py = rh ? __builtin_amdgcn_alignbit(yo, ya, 8) : ya;
            (void)h;
            neg += __popc(xor3(w, px, J[sg ? 1 : 0]));
            neg += __popc(xor3(w, py, J[rh ? 3 : 2]));
            neg += __popc(xor3(w, rows[zp * PS + wi * RPW], J[4]));
        }
    }
    for (int off = RPW; off < 64; off <<= 1) neg += __shfl_xor(neg, off, 64);
    const int64_t r = g * 64 + wave * RPW + q;
    if (j == 0 && r < R) st->energy[st->cur][r] = st->n_bonds - 2 * neg;
    __syncthreads();
    group_io<true>(st, g, s_rows, R, tid);
}

}  // namespace colour

// the colour-packed sweep of an L = 16 cube in the bit-packed layout; PA_ERR_ARG when the run or
// the thresholds are not ones it handles (tops above 0xFFFE leave no room for the + 1 of the bound)
int launch_sweep_colour(const pa_run& run, const SweepParams& p, hipStream_t s)
{
    if (run.dim != 3 || run.L != colour::L || run.layout != PA_BITS64 || !fast_sweep_thresholds_ok(p))
        return PA_ERR_ARG;
    const words::Thr th = words::make_thr(p);
    const int64_t blocks = (run.capacity + 63) / 64;
    if (blocks <= 0) return PA_OK;
    if (words::all_tops_zero(th))
        hipLaunchKernelGGL(colour::k_sweep16c<2>, dim3((unsigned)blocks), dim3(256), 0, s, run.state, p, th);
    else
        hipLaunchKernelGGL(colour::k_sweep16c<0>, dim3((unsigned)blocks), dim3(256), 0, s, run.state, p, th);
    return PA_OK;
}

}  // namespace pa
