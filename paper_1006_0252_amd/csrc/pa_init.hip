// Run initialisation (Sec. II: R0 replicas at beta = 0, each uniform over the 2^N
// microstates; couplings +-1 from the disorder seed; energies E = + sum J s s).
#include <math.h>
#include <string.h>

#include "pa_common.h"
#include "pa_lattice.h"

namespace pa {

__global__ void k_write_state(pa_state* st, pa_state init) { *st = init; }

// J_b = -1 iff bit (b mod 128) of Philox(ctr (b/128, 0, 0, 5), key disorder seed) is set
__global__ void k_couplings(int8_t* J, int n_bonds, uint32_t k0, uint32_t k1)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bonds) return;
    const uint4v v = philox10((uint32_t)(b >> 7), 0u, 0u, kTagCoupling, k0, k1);
    const uint32_t bit = (word_of(v, (b & 127) >> 5) >> (b & 31)) & 1u;
    J[b] = bit ? (int8_t)-1 : (int8_t)1;
}

// u8: thread per (replica, 16 consecutive sites); spin i of replica r is bit (i mod 128)
// of Philox(ctr (i/128, r, 0, 1), key seed)
__global__ void k_init_u8(const pa_state* __restrict__ st, uint32_t k0, uint32_t k1)
{
    const int N = st->N, stride = st->row_stride;
    const int per_row = stride / 16;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t / per_row;
    const int q = (int)(t - r * per_row);
    if (r >= st->R0) return;
    const int i0 = q * 16;
    const uint4v v = philox10((uint32_t)(i0 >> 7), (uint32_t)r, 0u, kTagInit, k0, k1);
    const uint32_t word = word_of(v, (i0 & 127) >> 5) >> (i0 & 31);  // 16 spins in bits 0..15
    uint8_t b[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) b[j] = (i0 + j < N) ? (uint8_t)((word >> j) & 1u) : (uint8_t)0;
    uint8_t* dst = (uint8_t*)st->spins[0] + r * stride + i0;
    *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<uint4*>(b);
}

// bit-packed rows: thread per replica; row word (g, row, l) of replica 64 g + l at
// (g * n_rows + row) * 64 + l, bit x = site x + L row (cube) or 32 row + x (chain)
__device__ inline int row_len(const pa_state* st, int row) { return st->dim == 1 ? min(32, st->N - 32 * row) : st->L; }
__device__ inline int n_rows_of(const pa_state* st) { return st->dim == 1 ? (st->N + 31) / 32 : st->L * st->L; }
__device__ inline int row_bytes(const pa_state* st) { return st->dim == 1 ? 4 : (st->L <= 8 ? 1 : (st->L <= 16 ? 2 : 4)); }

__device__ inline uint32_t load_row(const pa_state* st, int buf, int64_t r, int row)
{
    const int WB = row_bytes(st);
    const int64_t idx = ((r >> 6) * n_rows_of(st) + row) * 64 + (r & 63);
    const uint8_t* base = (const uint8_t*)st->spins[buf];
    if (WB == 1) return base[idx];
    if (WB == 2) return ((const uint16_t*)base)[idx];
    return ((const uint32_t*)base)[idx];
}

__global__ void __launch_bounds__(256) k_init_bits64(const pa_state* __restrict__ st, uint32_t k0, uint32_t k1)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= st->capacity) return;
    const bool valid = r < st->R0;
    const int NR = n_rows_of(st), WB = row_bytes(st);
    const int rowsites = st->dim == 1 ? 32 : st->L;
    uint8_t* base = (uint8_t*)st->spins[0];
    int blk = -1;
    uint4v v = {0, 0, 0, 0};
    // word q of the replica's stream (spins 32 q .. 32 q + 31), the calls made in increasing order
    auto word_at = [&](int q) -> uint32_t {
        if ((q >> 2) != blk) {
            blk = q >> 2;
            v = philox10((uint32_t)blk, (uint32_t)r, 0u, kTagInit, k0, k1);
        }
        return word_of(v, q & 3);
    };
    for (int row = 0; row < NR; ++row) {
        // the row's spins are the len consecutive stream bits from i0: one word, or the top of one
        // and the bottom of the next
        const int len = row_len(st, row);
        const int i0 = rowsites * row;
        const int q0 = i0 >> 5, q1 = (i0 + len - 1) >> 5;
        const uint32_t lo = word_at(q0);
        const uint32_t hi = q1 != q0 ? word_at(q1) : 0u;
        const uint32_t lm = len == 32 ? 0xFFFFFFFFu : (1u << len) - 1u;
        uint32_t w = (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (i0 & 31)) & lm;
        if (!valid) w = 0;
        const int64_t idx = ((r >> 6) * NR + row) * 64 + (r & 63);
        if (WB == 1) base[idx] = (uint8_t)w;
        else if (WB == 2) ((uint16_t*)base)[idx] = (uint16_t)w;
        else ((uint32_t*)base)[idx] = w;
    }
}

// u8 energies: one wave per replica, lanes over sites, each site owns its + bonds
__global__ void __launch_bounds__(256) k_energy_u8(const pa_state* __restrict__ st, int buf)
{
    const int N = st->N, L = st->L, dim = st->dim, stride = st->row_stride;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= st->R) return;
    const uint8_t* s = (const uint8_t*)st->spins[buf] + r * stride;
    const int8_t* J = st->J;
    int e = 0;
    for (int i = lane; i < N; i += 64) {
        const int si = s[i];
        if (dim == 1) {
            const int j = (i + 1 == N) ? 0 : i + 1;
            e += (int)J[i] * (1 - 2 * (si ^ s[j]));
        } else {
            int nb[3];
            plus_neighbours3(i, L, nb);
#pragma unroll
            for (int a = 0; a < 3; ++a) e += (int)J[3 * i + a] * (1 - 2 * (si ^ s[nb[a]]));
        }
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    if (lane == 0) st->energy[buf][r] = e;
}

// bit-packed energies: thread per replica, E = n_bonds - 2 * (bonds with J s s = -1)
__global__ void __launch_bounds__(256) k_energy_bits64(const pa_state* __restrict__ st, int buf)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int L = st->L;
    const int NR = n_rows_of(st);
    const int8_t* J = st->J;
    int neg = 0;
    if (st->dim == 3) {
        // the block first turns the couplings into sign masks per row and axis (bit x: J < 0 on the
        // bond from site x + L row towards +axis), then each replica counts its unsatisfied bonds a
        // row word at a time
        __shared__ uint32_t jmask[3 * 32 * 32];
        for (int e = threadIdx.x; e < 3 * NR; e += blockDim.x) {
            const int row = e / 3, a = e - 3 * row;
            uint32_t m = 0;
            for (int x = 0; x < L; ++x) m |= (uint32_t)(J[3 * (x + L * row) + a] < 0) << x;
            jmask[e] = m;
        }
        __syncthreads();
        if (r >= st->R) return;
        const uint32_t lm = L == 32 ? 0xFFFFFFFFu : (1u << L) - 1u;
        for (int row = 0; row < NR; ++row) {
            const int y = row % L, z = row / L;
            const uint32_t own = load_row(st, buf, r, row) & lm;
            const uint32_t yp = load_row(st, buf, r, (y + 1) % L + L * z) & lm;
            const uint32_t zp = load_row(st, buf, r, y + L * ((z + 1) % L)) & lm;
            const uint32_t sx = ((own >> 1) | (own << (L - 1))) & lm;  // bit x: site x + 1 (periodic)
            neg += __popc(own ^ sx ^ jmask[3 * row]);
            neg += __popc((own ^ yp ^ jmask[3 * row + 1]) & lm);
            neg += __popc((own ^ zp ^ jmask[3 * row + 2]) & lm);
        }
    } else {
        if (r >= st->R) return;
        for (int row = 0; row < NR; ++row) {
            const int len = row_len(st, row);
            const uint32_t own = load_row(st, buf, r, row);
            const int nrow = row + 1 == NR ? 0 : row + 1;
            const uint32_t nxt = load_row(st, buf, r, nrow);
            for (int x = 0; x < len; ++x) {
                const uint32_t si = (own >> x) & 1u;
                const uint32_t sj = x + 1 < len ? (own >> (x + 1)) & 1u : nxt & 1u;
                neg += (int)(si ^ sj ^ (uint32_t)(J[32 * row + x] < 0));
            }
        }
    }
    st->energy[buf][r] = st->n_bonds - 2 * neg;
}

// record[0] and the energy base E_base = -n_bonds + ((E_0 + n_bonds) mod 4): every energy
// of a +-1 realisation has the residue of E_0 mod 4 (each flip changes E by 4c - 2z)
__global__ void k_init_finish(pa_state* st)
{
    const int B = st->n_bonds;
    if (st->couplings != PA_GAUSS) {
        const int E0 = st->energy[0][0];
        st->E_base = -B + (((E0 + B) % 4) + 4) % 4;
    }
    for (int k = 0; k < st->n_records; ++k) {
        pa_record* rec = st->record + k;
        double* d = reinterpret_cast<double*>(rec);
        for (int j = 0; j < (int)(sizeof(pa_record) / sizeof(double)); ++j) d[j] = 0.0;
    }
    pa_record* r0 = st->record;
    r0->beta = 0.0;
    r0->lnQ = 0.0;
    r0->minus_betaF = st->ln_omega;
    r0->R = (double)st->R;
    st->initialised = 1;
}

int launch_init(const pa_run& run, const int8_t* J_host, hipStream_t s)
{
    pa_sizes sz;
    int rc = pa_buffer_sizes(run.dim, run.L, run.layout, run.couplings, run.capacity, run.n_records, &sz);
    if (rc != PA_OK) return rc;
    pa_state h;
    memset(&h, 0, sizeof(h));
    h.dim = run.dim;
    h.L = run.L;
    h.N = (int32_t)sz.N;
    h.z = 2 * run.dim;
    h.n_bonds = (int32_t)sz.n_bonds;
    h.layout = run.layout;
    h.n_bins = (int32_t)sz.n_bins;
    h.row_stride = (int32_t)sz.row_stride;
    h.capacity = run.capacity;
    h.R0 = run.R0;
    h.seed = run.seed;
    h.disorder_seed = run.disorder_seed;
    h.J = run.J;
    h.spins[0] = run.spins[0];
    h.spins[1] = run.spins[1];
    h.energy[0] = run.energy[0];
    h.energy[1] = run.energy[1];
    h.counts = run.counts;
    h.offsets = run.offsets;
    h.work = (uint8_t*)run.work;
    h.record = run.record;
    h.n_records = run.n_records;
    h.R = run.R0;
    h.R_new = run.R0;
    h.cur = 0;
    h.status = 0;
    h.k = 0;
    h.acc = 0.0;
    h.ln_omega = (double)sz.N * log(2.0);
    h.beta = 0.0;
    h.initialised = 0;
    h.couplings = run.couplings;
    hipLaunchKernelGGL(k_write_state, dim3(1), dim3(1), 0, s, run.state, h);

    const uint32_t s0 = (uint32_t)run.seed, s1 = (uint32_t)(run.seed >> 32);
    if (run.couplings == PA_GAUSS) {
        // couplings from the host (libm), then spins as for +-1 couplings and FP64 energies
        if (J_host) return PA_ERR_ARG;
        rc = gauss_couplings_upload(run, s);
        if (rc != PA_OK) return rc;
        const int64_t threads = run.R0 * (sz.row_stride / 16);
        hipLaunchKernelGGL(k_init_u8, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, run.state, s0, s1);
        rc = launch_energy_gauss(run, 0, run.R0, s);
        if (rc != PA_OK) return rc;
        hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(1), 0, s, run.state);
        return hip_status(hipGetLastError());
    }

    const int B = (int)sz.n_bonds;
    if (J_host) {
        for (int b = 0; b < B; ++b)
            if (J_host[b] != 1 && J_host[b] != -1) return PA_ERR_ARG;
        if (hipMemcpyAsync(run.J, J_host, (size_t)B, hipMemcpyHostToDevice, s) != hipSuccess) return PA_ERR_HIP;
    } else {
        hipLaunchKernelGGL(k_couplings, dim3((B + 255) / 256), dim3(256), 0, s, run.J, B,
                           (uint32_t)run.disorder_seed, (uint32_t)(run.disorder_seed >> 32));
    }
    const uint32_t k0 = (uint32_t)run.seed, k1 = (uint32_t)(run.seed >> 32);
    if (run.layout == PA_U8) {
        const int64_t threads = run.R0 * (sz.row_stride / 16);
        hipLaunchKernelGGL(k_init_u8, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, run.state, k0, k1);
        hipLaunchKernelGGL(k_energy_u8, dim3((unsigned)((run.R0 + 3) / 4)), dim3(256), 0, s, run.state, 0);
    } else {
        const unsigned blocks = (unsigned)((run.capacity + 255) / 256);
        hipLaunchKernelGGL(k_init_bits64, dim3(blocks), dim3(256), 0, s, run.state, k0, k1);
        hipLaunchKernelGGL(k_energy_bits64, dim3(blocks), dim3(256), 0, s, run.state, 0);
    }
    hipLaunchKernelGGL(k_init_finish, dim3(1), dim3(1), 0, s, run.state);
    return hip_status(hipGetLastError());
}

}  // namespace pa
