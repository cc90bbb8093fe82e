// Metropolis sweeps of the cube for L = 4, 8, 12, 16: the same sample as the generic kernel
// (same Philox fields, same acceptance rule), laid out for the vector ALU.
//
//  - lane = replica; a replica's rows (one 16-bit word per (y, z) row, bit x = spin) sit in
//    LDS, planes of L rows per z; LPR lanes share a replica by taking L/LPR planes each;
//  - the y loop of a plane is unrolled, so every neighbour row is an immediate LDS offset;
//  - per row, the six bond words J s s (bit-parallel over x) feed a bit-sliced adder giving
//    c = number of bonds with J s_i s_j = -1 (dE = 4c - 12); c <= 3 flips outright;
//  - the 16-bit first look of each site against its threshold is specialised by regime:
//    MODE 2: every threshold of c >= 4 has top 16 bits 0 (beta > ln 2^16 / 4): only u == 0
//            can accept, and that is a tie;  MODE 1: only c = 4 has a non-zero top;
//    MODE 0: general.  Possible ties are flagged per lane and resolved exactly with the
//    48 low bits in a separate (rare) path;
//  - energies are recomputed once per launch from bond popcounts.
#include <string.h>

#include "pa_common.h"
#include "pa_sweep_util.h"

namespace pa {

struct FastThr {
    uint32_t thi4, thi5, thi6;
    uint64_t T4, T5, T6;
};

// exact random-acceptance mask of the candidate sites (c >= 4) of one row
static __device__ __noinline__ uint32_t resolve_row(uint32_t c0, uint32_t c1, uint32_t cand, int par, int hbase,
                                                    int H, int ibase, uint32_t rr, uint32_t ctr2, uint32_t k0,
                                                    uint32_t k1, FastThr th)
{
    uint32_t racc = 0;
    for (int m = 0; m < H; ++m) {
        const int x = 2 * m + par;
        if (!((cand >> x) & 1u)) continue;
        const int h = hbase + m;
        const uint4v v = philox10((uint32_t)(h >> 3), rr, ctr2, kTagMet, k0, k1);
        const uint32_t u = field16(v, h & 7);
        const int cls = 4 + (int)((c0 >> x) & 1u) + 2 * (int)((c1 >> x) & 1u);
        const uint32_t thi = cls == 4 ? th.thi4 : (cls == 5 ? th.thi5 : th.thi6);
        const uint64_t T = cls == 4 ? th.T4 : (cls == 5 ? th.T5 : th.T6);
        bool a;
        if (u != thi) a = u < thi;
        else a = tie_accept(u, T, (uint32_t)(ibase + x), rr, ctr2, k0, k1);
        racc |= (uint32_t)a << x;
    }
    return racc;
}

template <int L, int LPR>
struct FastLayout {
    static constexpr int NR = L * L;
    static constexpr int RPW = 64 / LPR;
    static constexpr int PL = L / LPR;                          // planes per lane
    static constexpr int PADW = LPR == 4 ? 8 : 0;               // u16 padding per plane (bank stagger)
    static constexpr int PSTRIDE = L * RPW + PADW;              // u16 per plane
    static constexpr int JPAD = LPR == 4 ? 4 : 0;
    static constexpr int JSTRIDE = L * 8 + JPAD;                // dwords of coupling masks per plane
    static constexpr size_t lds_bytes(int wpb) { return (size_t)L * JSTRIDE * 4 + (size_t)wpb * L * PSTRIDE * 2; }
};

template <int L, int LAYOUT, int LPR, int MODE>
__global__ void __launch_bounds__(256) k_sweep3f(const pa_state* __restrict__ st, SweepParams p, FastThr th)
{
    using F = FastLayout<L, LPR>;
    constexpr int NR = F::NR, H = L / 2, RPW = F::RPW, PL = F::PL;
    constexpr int PSTRIDE = F::PSTRIDE, JSTRIDE = F::JSTRIDE;
    constexpr uint32_t MASK = (1u << L) - 1u;
    constexpr int WB = L <= 8 ? 1 : 2;  // bytes of a row word in the bit-packed layout
    static_assert(L % 4 == 0 && L <= 16 && L % LPR == 0, "fast sweep geometry");
    if (st->status) return;  // sticky error: the population stays as it is
    extern __shared__ uint32_t lds[];
    uint32_t* jtab = lds;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int q = lane % RPW, j = lane / RPW;
    uint16_t* rows = reinterpret_cast<uint16_t*>(lds + L * JSTRIDE) + wave * (L * PSTRIDE);
    const int wpb = blockDim.x >> 6;
    const int64_t R = st->R;
    const int cur = st->cur;
    const int64_t rbase = ((int64_t)blockIdx.x * wpb + wave) * RPW;
    const int64_t r = rbase + q;
    const bool valid = r < R;

    // coupling masks per row, entries +x, +y, +z, -x, -y, -z bonds with J = -1
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
        uint32_t* e = jtab + z * JSTRIDE + y * 8;
        for (int k = 0; k < 6; ++k) e[k] = m[k];
        e[6] = 0;
        e[7] = 0;
    }

    // this lane's planes z = j PL .. j PL + PL - 1 into LDS
    if (rbase < R) {
        for (int t = 0; t < PL; ++t) {
            const int z = j * PL + t;
            uint16_t* P = rows + z * PSTRIDE + q;
            for (int y = 0; y < L; ++y) {
                const int rho = y + L * z;
                uint32_t v;
                if (LAYOUT == PA_BITS64) {
                    const uint8_t* a = (const uint8_t*)st->spins[cur] + (((r >> 6) * NR + rho) * 64 + (r & 63)) * WB;
                    v = WB == 1 ? *a : *(const uint16_t*)a;
                } else {
                    const uint32_t* a = (const uint32_t*)((const uint8_t*)st->spins[cur] + r * st->row_stride + rho * L);
                    v = 0;
#pragma unroll
                    for (int d = 0; d < L / 4; ++d) v |= pack4(a[d]) << (4 * d);
                }
                P[y * RPW] = (uint16_t)v;
            }
        }
    }
    __syncthreads();
    if (rbase >= R) return;

    const uint32_t k0 = (uint32_t)st->seed, k1 = (uint32_t)(st->seed >> 32);
    const uint32_t rr = (uint32_t)r;
    const uint32_t thi4 = th.thi4;
    const int d5 = (int)th.thi5 - (int)th.thi4, d6 = (int)th.thi6 - (int)th.thi4;

    for (int s = 0; s < p.n_sweeps; ++s) {
        const int64_t t_sweep = p.t0 + s;
        for (int col = 0; col < 2; ++col) {
            const uint32_t ctr2 = (uint32_t)(2 * t_sweep + col);
            for (int t = 0; t < PL; ++t) {
                const int z = j * PL + t;
                const int zp = (z + 1 == L) ? 0 : z + 1;
                const int zm = (z == 0) ? L - 1 : z - 1;
                uint16_t* P0 = rows + z * PSTRIDE + q;
                const uint16_t* Pp = rows + zp * PSTRIDE + q;
                const uint16_t* Pm = rows + zm * PSTRIDE + q;
                const uint32_t* JT = jtab + z * JSTRIDE;
                const uint32_t cb = (uint32_t)(z * (L * H / 8));  // first Philox call of the plane
                const int p0 = (col + z) & 1;                      // x parity of colour col at y = 0
                const uint32_t cmA = (p0 ? 0xAAAAAAAAu : 0x55555555u) & MASK;
                const uint32_t cmB = (~cmA) & MASK;
                uint4v rnd = {0, 0, 0, 0};
#pragma unroll
                for (int y = 0; y < L; ++y) {
                    const uint32_t own = P0[y * RPW];
                    const uint32_t yp = P0[((y + 1) % L) * RPW];
                    const uint32_t ym = P0[((y + L - 1) % L) * RPW];
                    const uint32_t zpv = Pp[y * RPW];
                    const uint32_t zmv = Pm[y * RPW];
                    const uint32_t* jr = JT + y * 8;
                    const uint32_t dup = own | (own << L);
                    const uint32_t b0 = own ^ (dup >> 1) ^ jr[0];
                    const uint32_t b1 = own ^ yp ^ jr[1];
                    const uint32_t b2 = own ^ zpv ^ jr[2];
                    const uint32_t b3 = own ^ (dup >> (L - 1)) ^ jr[3];
                    const uint32_t b4 = own ^ ym ^ jr[4];
                    const uint32_t b5 = own ^ zmv ^ jr[5];
                    const uint32_t s1 = b0 ^ b1 ^ b2, k1c = (b0 & b1) | (b2 & (b0 ^ b1));
                    const uint32_t s2 = b3 ^ b4 ^ b5, k2c = (b3 & b4) | (b5 & (b3 ^ b4));
                    const uint32_t c0 = s1 ^ s2, k3c = s1 & s2;
                    const uint32_t c1 = k1c ^ k2c ^ k3c;
                    const uint32_t c2 = (k1c & k2c) | (k3c & (k1c ^ k2c));
                    const uint32_t colmask = (y & 1) ? cmB : cmA;
                    const int par = p0 ^ (y & 1);
                    uint32_t acc = 0;
                    bool tie = false;
#pragma unroll
                    for (int m = 0; m < H; ++m) {
                        const int hm = y * H + m;
                        if (hm % 8 == 0) rnd = philox10(cb + (uint32_t)(hm / 8), rr, ctr2, kTagMet, k0, k1);
                        const uint32_t u = field16(rnd, hm & 7);
                        const int xb = 2 * m + par;
                        if (MODE == 2) {
                            tie |= (u == 0u);
                        } else if (MODE == 1) {
                            acc |= (uint32_t)(u < thi4) << xb;
                            tie |= (u == thi4) | (u == 0u);
                        } else {
                            // class bits at x as 0 / -1 masks select the threshold differences
                            const int q0 = __builtin_amdgcn_sbfe((int)c0, xb, 1);
                            const int q1 = __builtin_amdgcn_sbfe((int)c1, xb, 1);
                            const uint32_t thi = (uint32_t)((int)thi4 + (q0 & d5) + (q1 & d6));
                            acc |= (uint32_t)(u < thi) << xb;
                            tie |= (u == thi);
                        }
                    }
                    uint32_t flip;
                    if (MODE == 2) flip = colmask & ~c2;
                    else if (MODE == 1) flip = colmask & (~c2 | (acc & ~c1 & ~c0));
                    else flip = colmask & (~c2 | acc);
                    if (tie) {
                        const uint32_t cand = c2 & colmask;
                        const int rho = y + L * z;
                        const uint32_t racc = resolve_row(c0, c1, cand, par, rho * H, H, L * rho, rr, ctr2, k0, k1, th);
                        flip = colmask & (~c2 | racc);
                    }
                    if (!valid) flip = 0;
                    P0[y * RPW] = (uint16_t)(own ^ flip);
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
        const uint16_t* P0 = rows + z * PSTRIDE + q;
        const uint16_t* Pp = rows + zp * PSTRIDE + q;
        const uint32_t* JT = jtab + z * JSTRIDE;
#pragma unroll
        for (int y = 0; y < L; ++y) {
            const uint32_t own = P0[y * RPW];
            const uint32_t dup = own | (own << L);
            const uint32_t* jr = JT + y * 8;
            neg += __popc((own ^ (dup >> 1) ^ jr[0]) & MASK);
            neg += __popc((own ^ P0[((y + 1) % L) * RPW] ^ jr[1]) & MASK);
            neg += __popc((own ^ Pp[y * RPW] ^ jr[2]) & MASK);
        }
    }
    for (int off = RPW; off < 64; off <<= 1) neg += __shfl_xor(neg, off, 64);

    // rows back to HBM
    if (valid) {
        for (int t = 0; t < PL; ++t) {
            const int z = j * PL + t;
            const uint16_t* P = rows + z * PSTRIDE + q;
            for (int y = 0; y < L; ++y) {
                const int rho = y + L * z;
                const uint32_t v = P[y * RPW];
                if (LAYOUT == PA_BITS64) {
                    uint8_t* a = (uint8_t*)st->spins[cur] + (((r >> 6) * NR + rho) * 64 + (r & 63)) * WB;
                    if (WB == 1) *a = (uint8_t)v;
                    else *(uint16_t*)a = (uint16_t)v;
                } else {
                    uint32_t* a = (uint32_t*)((uint8_t*)st->spins[cur] + r * st->row_stride + rho * L);
#pragma unroll
                    for (int d = 0; d < L / 4; ++d) a[d] = unpack4(v >> (4 * d));
                }
            }
        }
        if (j == 0) st->energy[cur][r] = st->n_bonds - 2 * neg;
    }
}

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
    if (lpr == 4 && L % 4 == 0) return fast_m<L, LAYOUT, (L % 4 == 0 ? 4 : 1)>(run, p, th, mode, wpb, s);
    if (lpr == 2) return fast_m<L, LAYOUT, 2>(run, p, th, mode, wpb, s);
    return fast_m<L, LAYOUT, 1>(run, p, th, mode, wpb, s);
}

template <int L>
static int fast_l(const pa_run& run, const SweepParams& p, const FastThr& th, int mode, int lpr, int wpb,
                  hipStream_t s)
{
    return run.layout == PA_U8 ? fast_p<L, PA_U8>(run, p, th, mode, lpr, wpb, s)
                               : fast_p<L, PA_BITS64>(run, p, th, mode, lpr, wpb, s);
}

// returns PA_ERR_ARG when the lattice is not one the fast kernel handles
int launch_sweep_fast(const pa_run& run, const SweepParams& p, int lpr, int wpb, hipStream_t s)
{
    if (run.dim != 3 || run.L % 4 != 0 || run.L > 16) return PA_ERR_ARG;
    FastThr th;
    th.thi4 = p.thi[4];
    th.thi5 = p.thi[5];
    th.thi6 = p.thi[6];
    th.T4 = p.T64[4];
    th.T5 = p.T64[5];
    th.T6 = p.T64[6];
    int mode = 0;
    if (th.thi4 == 0 && th.thi5 == 0 && th.thi6 == 0) mode = 2;
    else if (th.thi5 == 0 && th.thi6 == 0) mode = 1;
    switch (run.L) {
        case 4: return fast_l<4>(run, p, th, mode, lpr, wpb, s);
        case 8: return fast_l<8>(run, p, th, mode, lpr, wpb, s);
        case 12: return fast_l<12>(run, p, th, mode, lpr, wpb, s);
        case 16: return fast_l<16>(run, p, th, mode, lpr, wpb, s);
        default: return PA_ERR_ARG;
    }
}

}  // namespace pa
