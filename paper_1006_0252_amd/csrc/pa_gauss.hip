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

// energy mean, variance, skewness of the population (one block; any summation order: these are
// compared to 1e-12, not bit for bit)
__global__ void __launch_bounds__(256) k_moments_gauss(pa_state* st)
{
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

int launch_sweep_gauss(const pa_run& run, const pa_step& step, hipStream_t s)
{
    hipLaunchKernelGGL(k_sweep_gauss, dim3((unsigned)((run.capacity + 63) / 64)), dim3(64), 0, s,
                       (const pa_state*)run.state, step.beta_to, step.t0, step.n_sweeps);
    return hip_status(hipGetLastError());
}

int launch_moments_gauss(const pa_run& run, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments_gauss, dim3(1), dim3(256), 0, s, run.state);
    return hip_status(hipGetLastError());
}

}  // namespace pa
