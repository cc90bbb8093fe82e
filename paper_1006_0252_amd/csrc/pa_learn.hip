// Learned temperature steps: population features, resampled-fraction step labels, and the
// 6-64-64-64-1 network that proposes the next dbeta (forward, loss gradient, Adam).
//
// The paper leaves the schedule to the user (Sec. II: every temperature sequence gives an
// exact method; Sec. III: Var(beta F~) measures how well it worked).  Here a network reads
// (beta, ln N, ln R, E/N, var E/N, skew E) of the population and proposes dbeta; it is
// trained towards the step at which the resampling of Sec. II (normalised weights tau_j,
// eq. wn) replaces a fixed fraction rho* of the population.  Resampling itself is unchanged,
// so every schedule the network produces is an exact schedule.
#include <math.h>

#include <mutex>

#include "pa_common.h"

namespace pa {

// ------------------------------------------------------------------ network geometry
constexpr int kIn = 6, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = 384, kOffW2 = 448, kOffB2 = 4544, kOffW3 = 4608, kOffB3 = 8704, kOffW4 = 8768,
              kOffB4 = 8832, kParams = 8833;
static_assert(kOffB4 + 1 == kParams && kParams == PA_MLP_PARAMS, "parameter layout");

// rows of the training work matrix ([row][ld] floats, ld = B rounded up to 64)
constexpr int kRowXH = 0;     // 6 normalised inputs + a row of ones
constexpr int kRowH1 = 7;     // 64 + ones
constexpr int kRowH2 = 72;    // 64 + ones
constexpr int kRowH3 = 137;   // 64 + ones
constexpr int kRowD1 = 202;   // 64 back-propagated deltas per layer
constexpr int kRowD2 = 266;
constexpr int kRowD3 = 330;
constexpr int kRowGZ = 394;   // dL/dz
constexpr int kRowLS = 395;   // per-sample loss / B
constexpr int kRows = 396;
constexpr int kChunk = 1024;  // samples per partial gradient

__host__ __device__ inline int64_t mlp_ld(int64_t B) { return (B + 63) & ~(int64_t)63; }
__host__ __device__ inline int64_t mlp_chunks(int64_t B) { return (B + kChunk - 1) / kChunk; }

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest, ties to even; NaN -> quiet NaN
__device__ inline uint16_t f32_to_bf16(float x)
{
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return 0x7FC0;
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// fixed affine input map (the same for every trained network)
__device__ inline void normalise(const float* x, float* xh)
{
    xh[0] = (x[0] - 2.5f) / 2.5f;    // beta
    xh[1] = (x[1] - 6.0f) / 2.0f;    // ln N
    xh[2] = (x[2] - 10.0f) / 2.5f;   // ln R
    xh[3] = x[3] + 1.0f;             // E / N
    xh[4] = x[4] - 1.0f;             // var E / N
    xh[5] = x[5] / 2.0f;             // skew E
}

__device__ inline float softplus(float z) { return fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z))); }
__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// one dense tanh layer for the calling lane: out[j][lane] = tanh(b[j] + sum_i W[j][i] in[i]),
// weights in LDS (row-major, n_in inputs), outputs to the lane's column of an LDS buffer and,
// when train, to row `row` of the work matrix at column b
template <int NIN>
__device__ inline void dense_tanh(const float* __restrict__ W, const float* __restrict__ bias, const float (&in)[NIN],
                                  float* __restrict__ buf, int lane, float* __restrict__ work, int64_t ld, int row,
                                  int64_t b, bool train)
{
    for (int j = 0; j < kH; ++j) {
        float acc = bias[j];
#pragma unroll
        for (int i = 0; i < NIN; ++i) acc = fmaf(W[j * NIN + i], in[i], acc);
        const float h = tanhf(acc);
        buf[j * 64 + lane] = h;
        if (train) work[(int64_t)(row + j) * ld + b] = h;
    }
}

// forward (and, with TRAIN, backward) of 64 samples per block, one sample per lane.
// Forward only: out[b] = dbeta = clamp(softplus(z) / sigma_E, dmin, dmax), dmax when var <= 0.
// TRAIN: writes the work matrix (activations, deltas, dL/dz, loss / B); target t[b] = dbeta*.
template <bool TRAIN>
__global__ void __launch_bounds__(64) k_mlp(const uint16_t* __restrict__ w, const float* __restrict__ x, int64_t B,
                                           float dmin, float dmax, float* __restrict__ out,
                                           const double* __restrict__ target, float* __restrict__ work)
{
    __shared__ float Wl[kParams];
    __shared__ float buf[kH * 64];
    const int lane = threadIdx.x;
    for (int p = lane; p < kParams; p += 64) Wl[p] = bf16_to_f32(w[p]);
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * 64 + lane;
    if (b >= B) return;
    const int64_t ld = mlp_ld(B);
    float xr[kIn], xh[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) xr[k] = x[b * kIn + k];
    normalise(xr, xh);
    if (TRAIN) {
#pragma unroll
        for (int k = 0; k < kIn; ++k) work[(int64_t)(kRowXH + k) * ld + b] = xh[k];
        work[(int64_t)(kRowXH + kIn) * ld + b] = 1.0f;
        work[(int64_t)(kRowH1 + kH) * ld + b] = 1.0f;
        work[(int64_t)(kRowH2 + kH) * ld + b] = 1.0f;
        work[(int64_t)(kRowH3 + kH) * ld + b] = 1.0f;
    }
    float h[kH];
    dense_tanh<kIn>(Wl + kOffW1, Wl + kOffB1, xh, buf, lane, work, ld, kRowH1, b, TRAIN);
#pragma unroll
    for (int i = 0; i < kH; ++i) h[i] = buf[i * 64 + lane];
    dense_tanh<kH>(Wl + kOffW2, Wl + kOffB2, h, buf, lane, work, ld, kRowH2, b, TRAIN);
#pragma unroll
    for (int i = 0; i < kH; ++i) h[i] = buf[i * 64 + lane];
    dense_tanh<kH>(Wl + kOffW3, Wl + kOffB3, h, buf, lane, work, ld, kRowH3, b, TRAIN);
#pragma unroll
    for (int i = 0; i < kH; ++i) h[i] = buf[i * 64 + lane];  // h3
    float z = Wl[kOffB4];
#pragma unroll
    for (int i = 0; i < kH; ++i) z = fmaf(Wl[kOffW4 + i], h[i], z);
    const float v = xr[4];
    const bool has_sigma = v > 0.0f;
    const float log_sigma = has_sigma ? 0.5f * (xr[1] + logf(v)) : 0.0f;
    const float sp = softplus(z);
    if (!TRAIN) {
        float d = has_sigma ? sp * expf(-log_sigma) : dmax;
        d = d != d ? dmax : fminf(fmaxf(d, dmin), dmax);
        out[b] = d;
        return;
    }
    const double t = target[b];
    const bool valid = has_sigma && t > 0.0 && t <= 1.0e300;
    float gz = 0.0f, ls = 0.0f;
    if (valid) {
        const float err = logf(sp) - log_sigma - (float)log(t);
        ls = err * err / (float)B;
        gz = (2.0f / (float)B) * err * sigmoid(z) / sp;
    }
    work[(int64_t)kRowGZ * ld + b] = gz;
    work[(int64_t)kRowLS * ld + b] = ls;
    // delta3 = gz w4 (1 - h3^2), kept in h[]
#pragma unroll
    for (int j = 0; j < kH; ++j) {
        h[j] = gz * Wl[kOffW4 + j] * (1.0f - h[j] * h[j]);
        work[(int64_t)(kRowD3 + j) * ld + b] = h[j];
    }
    // delta2[i] = (sum_j W3[j][i] delta3[j]) (1 - h2[i]^2)
    for (int i = 0; i < kH; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < kH; ++j) s = fmaf(Wl[kOffW3 + j * kH + i], h[j], s);
        const float a = work[(int64_t)(kRowH2 + i) * ld + b];
        const float d = s * (1.0f - a * a);
        buf[i * 64 + lane] = d;
        work[(int64_t)(kRowD2 + i) * ld + b] = d;
    }
#pragma unroll
    for (int i = 0; i < kH; ++i) h[i] = buf[i * 64 + lane];
    // delta1[k] = (sum_i W2[i][k] delta2[i]) (1 - h1[k]^2)
    for (int k = 0; k < kH; ++k) {
        float s = 0.0f;
#pragma unroll
        for (int i = 0; i < kH; ++i) s = fmaf(Wl[kOffW2 + i * kH + k], h[i], s);
        const float a = work[(int64_t)(kRowH1 + k) * ld + b];
        work[(int64_t)(kRowD1 + k) * ld + b] = s * (1.0f - a * a);
    }
}

// Partial gradients of one chunk of samples: G[a][c] = sum_b A[a][b] C[c][b] for the four
// products (deltas x layer inputs with their row of ones), tiled through LDS, 256 lanes per
// block, lane (a = t/4, c = t%4 + 4m).  Product 3 carries dL/dz and the per-sample loss.
struct GradProduct { int rowA, nA, rowC, nC; };

__device__ inline GradProduct grad_product(int q)
{
    switch (q) {
    case 0: return {kRowD1, kH, kRowXH, kIn + 1};
    case 1: return {kRowD2, kH, kRowH1, kH + 1};
    case 2: return {kRowD3, kH, kRowH2, kH + 1};
    default: return {kRowGZ, 2, kRowH3, kH + 1};
    }
}

// parameter index of G[a][c] of product q (-1: not a parameter; kParams: the loss sum)
__device__ inline int grad_param(int q, int a, int c)
{
    switch (q) {
    case 0: return c < kIn ? kOffW1 + a * kIn + c : kOffB1 + a;
    case 1: return c < kH ? kOffW2 + a * kH + c : kOffB2 + a;
    case 2: return c < kH ? kOffW3 + a * kH + c : kOffB3 + a;
    default:
        if (a == 0) return c < kH ? kOffW4 + c : kOffB4;
        return c == kH ? kParams : -1;
    }
}

__global__ void __launch_bounds__(256) k_mlp_grad_partial(const float* __restrict__ work, int64_t B,
                                                          float* __restrict__ partial)
{
    __shared__ float As[kH][65];
    __shared__ float Cs[kH + 1][65];
    const int q = blockIdx.x, chunk = blockIdx.y, t = threadIdx.x;
    const GradProduct g = grad_product(q);
    const int64_t ld = mlp_ld(B);
    const int64_t b0 = (int64_t)chunk * kChunk, b1 = min(B, b0 + kChunk);
    const int a = t >> 2;
    float acc[17];
#pragma unroll
    for (int m = 0; m < 17; ++m) acc[m] = 0.0f;
    for (int64_t bt = b0; bt < b1; bt += 64) {
        for (int e = t; e < g.nA * 64; e += 256) {
            const int r = e >> 6, bb = e & 63;
            As[r][bb] = bt + bb < b1 ? work[(int64_t)(g.rowA + r) * ld + bt + bb] : 0.0f;
        }
        for (int e = t; e < g.nC * 64; e += 256) {
            const int r = e >> 6, bb = e & 63;
            Cs[r][bb] = bt + bb < b1 ? work[(int64_t)(g.rowC + r) * ld + bt + bb] : 0.0f;
        }
        __syncthreads();
        if (a < g.nA) {
            for (int bb = 0; bb < 64; ++bb) {
                const float av = As[a][bb];
#pragma unroll
                for (int m = 0; m < 17; ++m) {
                    const int c = (t & 3) + 4 * m;
                    if (c < g.nC) acc[m] = fmaf(av, Cs[c][bb], acc[m]);
                }
            }
        }
        __syncthreads();
    }
    if (a >= g.nA) return;
#pragma unroll
    for (int m = 0; m < 17; ++m) {
        const int c = (t & 3) + 4 * m;
        if (c >= g.nC) continue;
        const int p = grad_param(q, a, c);
        if (p >= 0) partial[(int64_t)chunk * (kParams + 1) + p] = acc[m];
    }
}

// grad[p] = sum over chunks in order; the loss sum goes to loss[0]
__global__ void k_mlp_grad_sum(const float* __restrict__ partial, int n_chunks, float* __restrict__ grad,
                               float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kParams) return;
    float s = 0.0f;
    for (int c = 0; c < n_chunks; ++c) s += partial[(int64_t)c * (kParams + 1) + p];
    if (p < kParams) grad[p] = s;
    else if (loss) loss[0] = s;
}

// Adam (Kingma and Ba, ICLR 2015): FP32 master weights and moments, BF16 copy for the network
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, uint16_t* __restrict__ w, int64_t n, float bc1, float bc2,
                       float lr, float beta1, float beta2, float eps)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float g = grad[p];
    const float mp = beta1 * m[p] + (1.0f - beta1) * g;
    const float vp = beta2 * v[p] + (1.0f - beta2) * (g * g);
    m[p] = mp;
    v[p] = vp;
    const float th = theta[p] - lr * (mp / bc1) / (sqrtf(vp / bc2) + eps);
    theta[p] = th;
    w[p] = f32_to_bf16(th);
}

__global__ void k_bf16_round(const float* __restrict__ x, uint16_t* __restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f32_to_bf16(x[i]);
}

// ------------------------------------------------------------------ population side

// x[r] = (beta, ln N, ln R, E_mean / N, E_var / N, E_skew) of record[k] of run r
__global__ void k_features(const pa_state* base, int n, float* __restrict__ x)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const pa_state* st = base + r;
    const pa_record* rec = st->record + st->k;
    const double N = (double)st->N;
    float* o = x + (int64_t)r * kIn;
    o[0] = (float)st->beta;
    o[1] = (float)log(N);
    o[2] = (float)log((double)st->R);
    o[3] = (float)(rec->E_mean / N);
    o[4] = (float)(rec->E_var / N);
    o[5] = (float)rec->E_skew;
}

constexpr int kMaxRho = 8;
struct RhoArgs { double v[kMaxRho]; };

// block-wide sum in a fixed order (256 lanes)
__device__ inline double block_sum(double x, double* red)
{
    const int t = threadIdx.x;
    red[t] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// rho(dbeta) = 1 - (1/R) sum over energy bins i of h_i min(1, R w_i / S), w_i = exp(-4 dbeta (i - ilo)),
// S = sum_i h_i w_i (the population's normalised weights tau of eq. wn, per energy)
__device__ double rho_of(const int64_t* hist, int ilo, int ihi, double R, double dbeta, double* red)
{
    double s = 0.0;
    for (int i = ilo + threadIdx.x; i <= ihi; i += blockDim.x) {
        const int64_t h = hist[i];
        if (h) s += (double)h * exp(-4.0 * dbeta * (double)(i - ilo));
    }
    const double S = block_sum(s, red);
    double kept = 0.0;
    for (int i = ilo + threadIdx.x; i <= ihi; i += blockDim.x) {
        const int64_t h = hist[i];
        if (h) kept += (double)h * fmin(1.0, R * exp(-4.0 * dbeta * (double)(i - ilo)) / S);
    }
    return 1.0 - block_sum(kept, red) / R;
}

// mode 0: out[r * n + j] = rho(arg_j); mode 1: out[j * ld + r] = dbeta with rho = arg_j in [0, cap]
// (64 halvings; cap when rho(cap) <= arg_j).  NaN for runs with a raised status bit.
__global__ void __launch_bounds__(256) k_rho(pa_state* base, RhoArgs args, int n_args, int mode, double cap,
                                             int64_t ld, double* __restrict__ out)
{
    __shared__ double red[256];
    const pa_state* st = base + blockIdx.y;
    const int j = blockIdx.x;
    double result;
    if (st->status) {
        result = NAN;
    } else {
        const WorkLayout wl = work_layout(st->N, st->n_bins, st->capacity);
        const int64_t* hist = work_ptr<int64_t>(st, wl.hist);
        const int64_t* misc = work_ptr<int64_t>(st, wl.misc);
        const int ilo = (int)((misc[0] - st->E_base) >> 2), ihi = (int)((misc[1] - st->E_base) >> 2);
        const double R = (double)st->R;
        if (mode == 0) {
            result = rho_of(hist, ilo, ihi, R, args.v[j], red);
        } else if (rho_of(hist, ilo, ihi, R, cap, red) <= args.v[j]) {
            result = cap;
        } else {
            double lo = 0.0, hi = cap;
            for (int it = 0; it < 64; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (rho_of(hist, ilo, ihi, R, mid, red) < args.v[j]) lo = mid;
                else hi = mid;
            }
            result = 0.5 * (lo + hi);
        }
    }
    if (threadIdx.x == 0) {
        if (mode == 0) out[(int64_t)blockIdx.y * n_args + j] = result;
        else out[(int64_t)j * ld + blockIdx.y] = result;
    }
}

int launch_features(const pa_run* runs, int n, float* x, hipStream_t s)
{
    hipLaunchKernelGGL(k_features, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, (const pa_state*)runs[0].state,
                       n, x);
    return hip_status(hipGetLastError());
}

int launch_rho(const pa_run* runs, int n, const double* args, int n_args, int mode, double cap, int64_t ld,
               double* out, hipStream_t s)
{
    RhoArgs a;
    for (int j = 0; j < kMaxRho; ++j) a.v[j] = j < n_args ? args[j] : 0.0;
    int rc = launch_hist(runs, n, s);
    if (rc != PA_OK) return rc;
    hipLaunchKernelGGL(k_rho, dim3((unsigned)n_args, (unsigned)n), dim3(256), 0, s, runs[0].state, a, n_args, mode,
                       cap, ld, out);
    return hip_status(hipGetLastError());
}

// The loss gradient of a batch of at most kStaticMaxB samples with its work matrix and partial
// gradients in a fixed device array instead of caller memory, for callers that cannot allocate.
// Every call on a device shares that device's array: calls that overlap on one GPU race.  Nothing
// in it needs clearing between calls (every element a call reads, it has written first).
constexpr int64_t kStaticMaxB = 4096;
constexpr int64_t kStaticFloats = (int64_t)kRows * kStaticMaxB + ((kStaticMaxB + kChunk - 1) / kChunk) * (kParams + 1);
static __device__ __align__(256) float scratch[kStaticFloats];

constexpr int kMaxDevices = 64;
static float* g_scratch_dev[kMaxDevices];  // device address of `scratch` on each device, once looked up
static std::mutex g_scratch_lock;

// the current device's address of `scratch` (the host-side name is not a device address)
static int scratch_address(float** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PA_ERR_HIP;
    std::lock_guard<std::mutex> g(g_scratch_lock);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PA_ERR_HIP;
        g_scratch_dev[dev] = (float*)p;
    }
    *out = g_scratch_dev[dev];
    return PA_OK;
}

// the kernels of pa_mlp_grad on a given work area
static int mlp_grad_launch(const uint16_t* w, const float* x, const double* target, int64_t B, float* wk, float* grad,
                           float* loss, hipStream_t s)
{
    float* partial = wk + (int64_t)kRows * mlp_ld(B);
    const int64_t nc = mlp_chunks(B);
    if (nc > 65535) return PA_ERR_ARG;
    hipLaunchKernelGGL(k_mlp<true>, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, s, w, x, B, 0.0f, 0.0f,
                       (float*)nullptr, target, wk);
    hipLaunchKernelGGL(k_mlp_grad_partial, dim3(4, (unsigned)nc), dim3(256), 0, s, (const float*)wk, B, partial);
    hipLaunchKernelGGL(k_mlp_grad_sum, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, (const float*)partial,
                       (int)nc, grad, loss);
    return hip_status(hipGetLastError());
}

}  // namespace pa

using namespace pa;

extern "C" int pa_mlp_work_bytes(int64_t B, int64_t* bytes)
{
    if (B <= 0 || !bytes) return PA_ERR_ARG;
    *bytes = (int64_t)kRows * mlp_ld(B) * 4 + mlp_chunks(B) * (int64_t)(kParams + 1) * 4;
    return PA_OK;
}

extern "C" int pa_mlp_forward(const uint16_t* w, const float* x, int64_t B, float dbeta_min, float dbeta_max,
                              float* dbeta, void* stream)
{
    if (!w || !x || !dbeta || B <= 0 || B > ((int64_t)1 << 30)) return PA_ERR_ARG;
    if (!(dbeta_min >= 0.0f) || !(dbeta_max >= dbeta_min) || !isfinite(dbeta_max)) return PA_ERR_ARG;
    hipLaunchKernelGGL(k_mlp<false>, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, (hipStream_t)stream, w, x, B,
                       dbeta_min, dbeta_max, dbeta, (const double*)nullptr, (float*)nullptr);
    return hip_status(hipGetLastError());
}

extern "C" int pa_mlp_grad(const uint16_t* w, const float* x, const double* target, int64_t B, void* work,
                           float* grad, float* loss, void* stream)
{
    if (!w || !x || !target || !work || !grad || B <= 0 || B > ((int64_t)1 << 30)) return PA_ERR_ARG;
    return mlp_grad_launch(w, x, target, B, (float*)work, grad, loss, (hipStream_t)stream);
}

extern "C" int pa_mlp_grad_static(const uint16_t* w, const float* x, const double* target, int64_t B, float* grad,
                                  float* loss, void* stream)
{
    if (!w || !x || !target || !grad || B <= 0) return PA_ERR_ARG;
    if (B > kStaticMaxB) return PA_ERR_SIZE;
    float* wk = nullptr;
    const int st = scratch_address(&wk);
    if (st != PA_OK) return st;
    return mlp_grad_launch(w, x, target, B, wk, grad, loss, (hipStream_t)stream);
}

extern "C" int pa_mlp_adam(float* theta, float* m, float* v, const float* grad, uint16_t* w, int64_t n, int t,
                           float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!theta || !m || !v || !grad || !w || n <= 0 || t < 1) return PA_ERR_ARG;
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps >= 0.0f))
        return PA_ERR_ARG;
    // bias corrections 1 - beta^t of the moment estimates
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)t));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, theta, m, v, grad,
                       w, n, bc1, bc2, lr, beta1, beta2, eps);
    return hip_status(hipGetLastError());
}

extern "C" int pa_bf16_round(const float* x, uint16_t* out, int64_t n, void* stream)
{
    if (!x || !out || n <= 0) return PA_ERR_ARG;
    hipLaunchKernelGGL(k_bf16_round, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, x, out, n);
    return hip_status(hipGetLastError());
}
