/*
 * pa_oracle.c -- CPU oracle for population annealing with weighted averages
 * (J. Machta, "Population Annealing with Weighted Averages: A Monte Carlo Method
 * for Rough Free Energy Landscapes", arXiv:1006.0252).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the library never does, and the
 * two share no code (this file has its own Philox, its own tables and its own
 * lattice indexing).
 *
 * Everything here is written for clarity: one Philox call per Metropolis attempt,
 * plain loops in the order the paper states the algorithm, FP64 wherever a real
 * number appears, OpenMP only across independent replicas.
 *
 * Paper passages followed (sections and equation labels of the paper):
 *   Sec. II   -- initial population at beta = 0, Omega = 2^N microstates;
 *                reweighting factor exp[-(beta'-beta) E_j]; normalisation Q (eq. Q);
 *                normalised weights tau_j (eq. wn); Poisson copy numbers with mean
 *                (R_beta'/R~_beta) tau_j; theta MCMC sweeps at the new temperature;
 *                observables measured after resampling and sweeps; ln Q recorded;
 *                free-energy estimator (eq. sumQ); the "Population Annealing" algorithm.
 *   Sec. III  -- weighted average over runs (eqs. weight, omega), unequal target
 *                sizes R^(r), free-energy estimate from averaged exp(-beta F~) (eq. bestf),
 *                Var(beta F~) diagnostic.
 *   Sec. IV   -- Ising spin-glass energy E = sum_(i,j) J_ij s_i s_j (note the + sign),
 *                periodic simple cubic lattice and periodic chain; overlap
 *                q = (1/N) sum_i s_i^(1) s_i^(2) between replicas of two runs;
 *                Gamma = Prob(|q| < 0.2); pair weights (eqs. pqs, omegaprime).
 *
 * Readings where the paper is silent (the paper gives no RNG, no acceptance
 * precision and no Poisson sampler; these make GPU and CPU reach the same sample):
 *   - couplings J_b = +-1 equiprobable from a disorder seed;
 *   - Metropolis in checkerboard order, acceptance exactly T64/2^64 with
 *     T64 = floor(exp(-beta dE) 2^64), compared against a 64-bit uniform made of
 *     16 "first-look" bits plus 48 tie bits;
 *   - Poisson variates by a power-of-two ladder with binomial thinning;
 *   - Philox4x32-10 counters for every random draw (layout in the comments below).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* built with -ffp-contract=off: every product and sum is rounded on its own */

/* status codes (same numeric meaning as the library's, defined independently) */
enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_CAPACITY = 2, ORC_ERR_EXTINCT = 3, ORC_ERR_NONFINITE = 4 };

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from the published definition (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of two    */
/* 32x32->64 multiplies with a Weyl-sequence key schedule.                     */
/* ------------------------------------------------------------------------- */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_seeded(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox(ctr, key, out);
}

/* stream tags (fourth counter word) */
enum { TAG_INIT = 1, TAG_MET = 2, TAG_TIE = 3, TAG_POISSON = 4, TAG_COUPLING = 5 };

/* ------------------------------------------------------------------------- */
/* Lattice (Sec. IV): periodic chain of N = L spins (dim 1) or periodic simple */
/* cubic lattice of N = L^3 spins (dim 3).  Site i = x + L (y + L z).          */
/* Bond b = i (dim 1) joins i and i+1; bond b = 3 i + a (dim 3) joins i and    */
/* its +a neighbour (a = 0, 1, 2 for x, y, z).                                */
/* ------------------------------------------------------------------------- */
int orc_num_sites(int dim, int L) { return dim == 1 ? L : L * L * L; }
int orc_num_bonds(int dim, int L) { return dim == 1 ? L : 3 * L * L * L; }
static int coordination(int dim) { return 2 * dim; }

static int site_shift(int dim, int L, int i, int axis, int dir)
{
    if (dim == 1) return (i + dir + L) % L;
    int x = i % L, y = (i / L) % L, z = i / (L * L);
    if (axis == 0) x = (x + dir + L) % L;
    if (axis == 1) y = (y + dir + L) % L;
    if (axis == 2) z = (z + dir + L) % L;
    return x + L * (y + L * z);
}

/* the k-th bond touching site i: its index and the site at the other end */
static void incident_bond(int dim, int L, int i, int k, int* bond, int* other)
{
    if (dim == 1) {
        if (k == 0) { *bond = i; *other = site_shift(1, L, i, 0, +1); }
        else { int j = site_shift(1, L, i, 0, -1); *bond = j; *other = j; }
        return;
    }
    if (k < 3) { *bond = 3 * i + k; *other = site_shift(3, L, i, k, +1); }
    else { int a = k - 3; int j = site_shift(3, L, i, a, -1); *bond = 3 * j + a; *other = j; }
}

/* the two ends of bond b */
static void bond_ends(int dim, int L, int b, int* i, int* j)
{
    if (dim == 1) { *i = b; *j = site_shift(1, L, b, 0, +1); return; }
    *i = b / 3;
    *j = site_shift(3, L, b / 3, b % 3, +1);
}

int orc_colour(int dim, int L, int i)
{
    if (dim == 1) return i & 1;
    int x = i % L, y = (i / L) % L, z = i / (L * L);
    return (x + y + z) & 1;
}

static int spin_value(uint8_t s) { return s ? -1 : +1; } /* stored 1 means sigma = -1 */

/* ------------------------------------------------------------------------- */
/* Couplings J_b = -1 when bit (b mod 128) of Philox(ctr = (b/128, 0, 0, 5),   */
/* key = disorder seed) is set, +1 otherwise.                                 */
/* ------------------------------------------------------------------------- */
void orc_couplings(int dim, int L, uint64_t disorder_seed, int8_t* J)
{
    int nb = orc_num_bonds(dim, L);
    for (int b = 0; b < nb; ++b) {
        uint32_t out[4];
        philox_seeded((uint32_t)(b >> 7), 0, 0, TAG_COUPLING, disorder_seed, out);
        int bit = (out[(b & 127) >> 5] >> (b & 31)) & 1;
        J[b] = bit ? -1 : +1;
    }
}

/* E = sum over bonds of J_b s_i s_j (Sec. IV, + sign as printed) */
int64_t orc_energy(int dim, int L, const int8_t* J, const uint8_t* s)
{
    int nb = orc_num_bonds(dim, L);
    int64_t E = 0;
    for (int b = 0; b < nb; ++b) {
        int i, j;
        bond_ends(dim, L, b, &i, &j);
        E += (int64_t)J[b] * spin_value(s[i]) * spin_value(s[j]);
    }
    return E;
}

/* energy change when spin i is flipped: -2 s_i sum_(bonds at i) J s_other */
int orc_delta_energy(int dim, int L, const int8_t* J, const uint8_t* s, int i)
{
    int field = 0;
    for (int k = 0; k < coordination(dim); ++k) {
        int b, j;
        incident_bond(dim, L, i, k, &b, &j);
        field += J[b] * spin_value(s[j]);
    }
    return -2 * spin_value(s[i]) * field;
}

/* ------------------------------------------------------------------------- */
/* Initial population (Sec. II): R0 replicas, each uniform over the 2^N        */
/* microstates.  Spin i of replica r is bit (i mod 128) of                    */
/* Philox(ctr = (i/128, r, 0, 1), key = run seed).                            */
/* ------------------------------------------------------------------------- */
void orc_init_range(int dim, int L, const int8_t* J, uint64_t seed, int64_t r_first, int64_t count, uint8_t* s,
                    int32_t* E)
{
    int N = orc_num_sites(dim, L);
    for (int64_t q = 0; q < count; ++q) {
        int64_t r = r_first + q;
        for (int i = 0; i < N; ++i) {
            uint32_t out[4];
            philox_seeded((uint32_t)(i >> 7), (uint32_t)r, 0, TAG_INIT, seed, out);
            s[q * N + i] = (uint8_t)((out[(i & 127) >> 5] >> (i & 31)) & 1);
        }
        E[q] = (int32_t)orc_energy(dim, L, J, s + q * N);
    }
}

void orc_init_population(int dim, int L, const int8_t* J, uint64_t seed, int64_t R, uint8_t* s, int32_t* E)
{
    orc_init_range(dim, L, J, seed, 0, R, s, E);
}

/* ------------------------------------------------------------------------- */
/* Metropolis acceptance.  For dE > 0 the move is accepted with probability    */
/* T64 / 2^64, T64 = floor(exp(-beta dE) 2^64); when exp(-beta dE) >= 1 (only  */
/* at beta = 0) every move is accepted.  The 64-bit uniform is                 */
/* U = (u16 << 48) | u48 with                                                  */
/*   u16 = 16-bit field (h mod 8) of Philox(ctr = (h/8, r, 2t+c, 2))           */
/*         (field f is bits 16 (f mod 2) .. of 32-bit word f/2), h = i/2;      */
/*   u48 = word0 | (word1 mod 2^16) << 32 of Philox(ctr = (i, r, 2t+c, 3)).     */
/* Only when u16 equals the top 16 bits of T64 do the low 48 bits matter.      */
/* ------------------------------------------------------------------------- */
uint64_t orc_threshold(double beta, int dE, int* always)
{
    double p = exp(-beta * (double)dE);
    if (p >= 1.0) { *always = 1; return 0; }
    *always = 0;
    return (uint64_t)floor(ldexp(p, 64));
}

static uint32_t met_u16(uint64_t seed, int64_t r, int64_t t, int colour, int i)
{
    int h = i >> 1;
    uint32_t out[4];
    philox_seeded((uint32_t)(h >> 3), (uint32_t)r, (uint32_t)(2 * t + colour), TAG_MET, seed, out);
    int f = h & 7;
    return (out[f >> 1] >> (16 * (f & 1))) & 0xFFFFu;
}

static uint64_t met_u48(uint64_t seed, int64_t r, int64_t t, int colour, int i)
{
    uint32_t out[4];
    philox_seeded((uint32_t)i, (uint32_t)r, (uint32_t)(2 * t + colour), TAG_TIE, seed, out);
    return (uint64_t)out[0] | ((uint64_t)(out[1] & 0xFFFFu) << 32);
}

int orc_met_accept(uint64_t seed, int64_t r, int64_t t, int colour, int i, uint64_t T64)
{
    uint64_t u_hi = met_u16(seed, r, t, colour, i);
    uint64_t t_hi = T64 >> 48;
    if (u_hi != t_hi) return u_hi < t_hi;
    uint64_t U = (u_hi << 48) | met_u48(seed, r, t, colour, i);
    return U < T64;
}

/* ------------------------------------------------------------------------- */
/* theta = ns Metropolis sweeps of every replica at inverse temperature beta   */
/* (Sec. II; the loop "Equilibrate replica j" of the algorithm).  A sweep is    */
/* all sites of colour 0, then all sites of colour 1 (checkerboard: the sites   */
/* of one colour have no bonds among themselves, so their order is immaterial). */
/* Global sweep index t = t0 + s enters the RNG counters.                       */
/* ------------------------------------------------------------------------- */
/* replicas r_first .. r_first + count - 1 (population indices), stored from spins[0] */
void orc_sweep_range(int dim, int L, const int8_t* J, uint64_t seed, double beta, int64_t r_first,
                     int64_t count, uint8_t* spins, int32_t* E, int64_t t0, int ns)
{
    int N = orc_num_sites(dim, L);
    int z = coordination(dim);
    /* thresholds indexed by dE = -2z .. 2z */
    uint64_t T[25];
    int always[25];
    for (int dE = -2 * z; dE <= 2 * z; ++dE) {
        T[dE + 2 * z] = orc_threshold(beta, dE, &always[dE + 2 * z]);
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; ++q) {
        int64_t r = r_first + q;
        uint8_t* s = spins + q * N;
        for (int64_t t = t0; t < t0 + ns; ++t) {
            for (int colour = 0; colour < 2; ++colour) {
                for (int i = 0; i < N; ++i) {
                    if (orc_colour(dim, L, i) != colour) continue;
                    int dE = orc_delta_energy(dim, L, J, s, i);
                    int accept;
                    if (dE <= 0 || always[dE + 2 * z]) accept = 1;
                    else accept = orc_met_accept(seed, r, t, colour, i, T[dE + 2 * z]);
                    if (accept) {
                        s[i] ^= 1;
                        E[q] += dE;
                    }
                }
            }
        }
    }
}

void orc_sweep(int dim, int L, const int8_t* J, uint64_t seed, double beta,
               int64_t R, uint8_t* spins, int32_t* E, int64_t t0, int ns)
{
    orc_sweep_range(dim, L, J, seed, beta, 0, R, spins, E, t0, ns);
}

/* ------------------------------------------------------------------------- */
/* Poisson variate with mean lambda (the copy number of Sec. II).              */
/* Ladder + thinning: lambda = 64 q + rem with 0 < rem <= 64; q independent    */
/* Poisson(64) draws, then K ~ Poisson(2^m) with 2^m the smallest power of two  */
/* >= rem (m >= -20), each of the K events kept when a 32-bit uniform is below  */
/* floor(rem 2^(32-m)).  Poisson(2^m) is drawn by inversion against the table   */
/* C[n] = floor(F(n) 2^32) (F = CDF), the last entry forced to 2^32.            */
/* Draw d of replica j at step k is word (d mod 4) of                          */
/* Philox(ctr = (d/4, j, k, 4), key = run seed).                               */
/* ------------------------------------------------------------------------- */
#define LADDER_MIN (-20)
#define LADDER_MAX 6
#define LADDER_CAP 512

/* table for Lambda = 2^m: returns its length n_max + 1 */
int orc_ladder_table(int m, uint64_t* C)
{
    double Lam = ldexp(1.0, m);
    double p = exp(-Lam);
    double F = 0.0;
    const double tail = ldexp(1.0, -40);
    int n = 0;
    for (;;) {
        F += p;
        if ((double)n >= Lam && p < tail) { C[n] = (uint64_t)1 << 32; return n + 1; }
        double c = floor(ldexp(F, 32));
        C[n] = c >= 4294967296.0 ? ((uint64_t)1 << 32) : (uint64_t)c;
        ++n;
        p = p * Lam / (double)n;
        if (n >= LADDER_CAP - 1) { C[n] = (uint64_t)1 << 32; return n + 1; }
    }
}

static uint64_t g_ladder[LADDER_MAX - LADDER_MIN + 1][LADDER_CAP];
static int g_ladder_len[LADDER_MAX - LADDER_MIN + 1];
static int g_ladder_ready = 0;

static void ladder_setup(void)
{
    if (g_ladder_ready) return;
#pragma omp critical(orc_ladder)
    {
        if (!g_ladder_ready) {
            for (int m = LADDER_MIN; m <= LADDER_MAX; ++m)
                g_ladder_len[m - LADDER_MIN] = orc_ladder_table(m, g_ladder[m - LADDER_MIN]);
            g_ladder_ready = 1;
        }
    }
}

static uint32_t poisson_u32(uint64_t seed, int64_t j, int64_t k, uint32_t d)
{
    uint32_t out[4];
    philox_seeded(d >> 2, (uint32_t)j, (uint32_t)k, TAG_POISSON, seed, out);
    return out[d & 3];
}

static int64_t invert_ladder(int m, uint32_t u)
{
    const uint64_t* C = g_ladder[m - LADDER_MIN];
    int64_t n = 0;
    while (!((uint64_t)u < C[n])) ++n;
    return n;
}

/* smallest m in [LADDER_MIN, LADDER_MAX] with 2^m >= x (0 < x <= 64) */
static int ladder_level(double x)
{
    int e;
    double f = frexp(x, &e); /* x = f 2^e, 0.5 <= f < 1 */
    int m = (f == 0.5) ? e - 1 : e;
    return m < LADDER_MIN ? LADDER_MIN : m;
}

int64_t orc_poisson(double lambda, uint64_t seed, int64_t j, int64_t k)
{
    ladder_setup();
    if (!(lambda > 0.0)) return 0;
    uint32_t d = 0;
    int64_t n = 0;
    double rem = lambda;
    if (lambda > 64.0) {
        int64_t q = (int64_t)ceil(lambda / 64.0) - 1;
        rem = lambda - 64.0 * (double)q;
        for (int64_t b = 0; b < q; ++b) n += invert_ladder(LADDER_MAX, poisson_u32(seed, j, k, d++));
    }
    int m = ladder_level(rem);
    int64_t K = invert_ladder(m, poisson_u32(seed, j, k, d++));
    uint64_t keep = (uint64_t)floor(ldexp(rem, 32 - m));
    for (int64_t e = 0; e < K; ++e)
        if ((uint64_t)poisson_u32(seed, j, k, d++) < keep) ++n;
    return n;
}

/* ------------------------------------------------------------------------- */
/* One temperature step of resampling, beta_from -> beta_to (Sec. II, eqs. Q,  */
/* wn, and the Poisson copy rule):                                             */
/*   Q = (1/R~) sum_j exp[-(beta'-beta) E_j]                                   */
/*   tau_j = exp[-(beta'-beta) E_j] / Q                                        */
/*   copies_j ~ Poisson((R_target / R~) tau_j)                                 */
/* Evaluated with energies shifted by E_lo = min_j E_j (an exact rescaling of   */
/* numerator and denominator):                                                 */
/*   S = sum over distinct energies in ascending order of                      */
/*       (number of replicas at E) * exp(-(beta'-beta)(E - E_lo))              */
/*   ln Q = -(beta'-beta) E_lo + ln S - ln R~                                  */
/*   mean copies of j = R_target * exp(-(beta'-beta)(E_j - E_lo)) / S          */
/* New population: the copies of replica j, in order of j.                     */
/* out[0] = S, out[1] = ln Q, out[2] = E_lo.                                   */
/* ------------------------------------------------------------------------- */
/* Q and the copy numbers (the first half of the step): counts[j] for j < R, and
 * out[0] = S, out[1] = ln Q, out[2] = E_lo */
int orc_copy_numbers(uint64_t seed, int64_t k, double beta_from, double beta_to, double R_target, int64_t R,
                     const int32_t* E, int32_t* counts, double* out)
{
    double dbeta = beta_to - beta_from;
    if (R <= 0 || !(dbeta >= 0.0) || !(R_target > 0.0)) return ORC_ERR_ARG;

    int32_t E_lo = E[0], E_hi = E[0];
    for (int64_t j = 1; j < R; ++j) {
        if (E[j] < E_lo) E_lo = E[j];
        if (E[j] > E_hi) E_hi = E[j];
    }
    /* every energy of a +-1 realisation is congruent mod 4 (each flip moves E by a multiple of 4) */
    int64_t nlev = (int64_t)(E_hi - E_lo) / 4 + 1;
    int64_t* count = (int64_t*)calloc((size_t)nlev, sizeof(int64_t));
    for (int64_t j = 0; j < R; ++j) {
        if ((E[j] - E_lo) % 4 != 0) { free(count); return ORC_ERR_ARG; }
        count[(E[j] - E_lo) / 4] += 1;
    }
    double S = 0.0;
    for (int64_t d = 0; d < nlev; ++d) {
        double w = exp(-dbeta * (double)(4 * d));
        double term = (double)count[d] * w;
        S = S + term;
    }
    free(count);
    double lnQ = -dbeta * (double)E_lo + log(S) - log((double)R);
    out[0] = S;
    out[1] = lnQ;
    out[2] = (double)E_lo;
    if (!isfinite(S) || !(S > 0.0)) return ORC_ERR_NONFINITE;

#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < R; ++j) {
        double w = exp(-dbeta * (double)(E[j] - E_lo));
        double lam = (R_target * w) / S;
        counts[j] = (int32_t)orc_poisson(lam, seed, j, k);
    }
    return ORC_OK;
}

int orc_resample(int dim, int L, uint64_t seed, int64_t k, double beta_from, double beta_to,
                 double R_target, int64_t R, const uint8_t* spins, const int32_t* E,
                 int64_t capacity, uint8_t* spins_new, int32_t* E_new,
                 int32_t* counts, int64_t* offsets, double* out, int64_t* R_new)
{
    int N = orc_num_sites(dim, L);
    *R_new = 0;
    int st = orc_copy_numbers(seed, k, beta_from, beta_to, R_target, R, E, counts, out);
    if (st != ORC_OK) return st;
    int64_t acc = 0;
    for (int64_t j = 0; j < R; ++j) { offsets[j] = acc; acc += counts[j]; }
    offsets[R] = acc;
    *R_new = acc;
    if (acc > capacity) return ORC_ERR_CAPACITY;
    if (acc == 0) return ORC_ERR_EXTINCT;
    for (int64_t j = 0; j < R; ++j) {
        for (int32_t c = 0; c < counts[j]; ++c) {
            int64_t dst = offsets[j] + c;
            memcpy(spins_new + dst * N, spins + j * N, (size_t)N);
            E_new[dst] = E[j];
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Observables measured after the sweeps (Sec. II): energy mean, variance and  */
/* skewness over the population, no weights inside a run.                      */
/* ------------------------------------------------------------------------- */
void orc_energy_moments(int64_t R, const int32_t* E, double* out)
{
    int64_t sum = 0;
    for (int64_t j = 0; j < R; ++j) sum += E[j];
    double mean = (double)sum / (double)R;
    double m2 = 0.0, m3 = 0.0;
    for (int64_t j = 0; j < R; ++j) {
        double d = (double)E[j] - mean;
        m2 += d * d;
        m3 += d * d * d;
    }
    m2 /= (double)R;
    m3 /= (double)R;
    out[0] = mean;
    out[1] = m2;
    out[2] = m2 > 0.0 ? m3 / (m2 * sqrt(m2)) : 0.0;
}

/* Overlap between two runs (Sec. IV): replica j of run A paired with replica j */
/* of run B for j < min(R_A, R_B); hist[d] counts pairs at Hamming distance d,  */
/* i.e. q = (N - 2d)/N.  Returns the number of pairs.                           */
int64_t orc_overlap_hist(int N, int64_t RA, const uint8_t* sA, int64_t RB, const uint8_t* sB, int64_t* hist)
{
    for (int d = 0; d <= N; ++d) hist[d] = 0;
    int64_t P = RA < RB ? RA : RB;
    for (int64_t j = 0; j < P; ++j) {
        int q_num = 0;
        for (int i = 0; i < N; ++i) q_num += spin_value(sA[j * N + i]) * spin_value(sB[j * N + i]);
        hist[(N - q_num) / 2] += 1;
    }
    return P;
}

/* q^2, q^4 and Gamma = Prob(|q| < 0.2) from the overlap histogram */
void orc_overlap_stats(int N, const int64_t* hist, double* out)
{
    double P = 0.0, q2 = 0.0, q4 = 0.0, g = 0.0;
    for (int d = 0; d <= N; ++d) {
        double c = (double)hist[d];
        double q = (double)(N - 2 * d) / (double)N;
        P += c;
        q2 += c * q * q;
        q4 += c * q * q * q * q;
        if (fabs(q) < 0.2) g += c;
    }
    out[0] = q2 / P;
    out[1] = q4 / P;
    out[2] = g / P;
}

/* ------------------------------------------------------------------------- */
/* Weighted average over M runs (Sec. III, eqs. weight, omega, bestf):         */
/*   omega_r = R^(r) exp(-beta F~_r) / sum_r' R^(r') exp(-beta F~_r')          */
/*   A_bar = sum_r omega_r A_r                                                 */
/*   -beta F_bar = ln[ sum_r R^(r) exp(-beta F~_r) / sum_r R^(r) ]             */
/* (R^(r) = 1 when Rr is NULL).  var = sample variance (1/(M-1)) of -beta F~.   */
/* For overlaps pass x_r = -beta (F~_r^(1) + F~_r^(2)) (eq. omegaprime).        */
/* A is [M][n_obs] row-major.                                                  */
/* ------------------------------------------------------------------------- */
int orc_weighted_average(int M, const double* x, const double* Rr, const double* A, int n_obs,
                         double* A_bar, double* omega, double* mbF_bar, double* var, double* mean_x)
{
    if (M <= 0) return ORC_ERR_ARG;
    double xmax = -INFINITY;
    for (int r = 0; r < M; ++r) {
        double xr = x[r] + (Rr ? log(Rr[r]) : 0.0);
        if (xr > xmax) xmax = xr;
    }
    double Z = 0.0, Rsum = 0.0;
    for (int r = 0; r < M; ++r) {
        double xr = x[r] + (Rr ? log(Rr[r]) : 0.0);
        Z += exp(xr - xmax);
        Rsum += Rr ? Rr[r] : 1.0;
    }
    for (int o = 0; o < n_obs; ++o) A_bar[o] = 0.0;
    for (int r = 0; r < M; ++r) {
        double xr = x[r] + (Rr ? log(Rr[r]) : 0.0);
        double w = exp(xr - xmax) / Z;
        if (omega) omega[r] = w;
        for (int o = 0; o < n_obs; ++o) A_bar[o] += w * A[(int64_t)r * n_obs + o];
    }
    *mbF_bar = xmax + log(Z) - log(Rsum);
    double mean = 0.0;
    for (int r = 0; r < M; ++r) mean += x[r];
    mean /= (double)M;
    double v = 0.0;
    for (int r = 0; r < M; ++r) v += (x[r] - mean) * (x[r] - mean);
    *var = M > 1 ? v / (double)(M - 1) : 0.0;
    *mean_x = mean;
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Overlap observables over pairs of independent runs (Sec. IV, eqs. pqs and    */
/* omegaprime): pair p is runs 2p and 2p+1; its weight is proportional to       */
/* exp(-beta (F~^(1) + F~^(2))), times R^(1) R^(2) for runs with unequal target */
/* sizes (Sec. III).  Q is [n_pairs][3]: the pair's <q^2>, <q^4> and Gamma.     */
/* out = ([q^2], [q^4], [Gamma], g) with the Binder ratio                       */
/*   g = (3 - [q^4] / [q^2]^2) / 2                                              */
/* of the weighted moments (not a paper quantity: the observable the 3D         */
/* configuration asks for).                                                    */
/* ------------------------------------------------------------------------- */
int orc_overlap_average(int n_pairs, const double* x, const double* Rr, const double* Q, double* out)
{
    if (n_pairs <= 0) return ORC_ERR_ARG;
    double* xp = (double*)malloc((size_t)n_pairs * sizeof(double));
    double* Rp = Rr ? (double*)malloc((size_t)n_pairs * sizeof(double)) : NULL;
    double* omega = (double*)malloc((size_t)n_pairs * sizeof(double));
    for (int p = 0; p < n_pairs; ++p) {
        xp[p] = x[2 * p] + x[2 * p + 1];
        if (Rr) Rp[p] = Rr[2 * p] * Rr[2 * p + 1];
    }
    double mbF, var, mean;
    int st = orc_weighted_average(n_pairs, xp, Rp, Q, 3, out, omega, &mbF, &var, &mean);
    free(xp);
    free(Rp);
    free(omega);
    if (st != ORC_OK) return st;
    out[3] = 0.5 * (3.0 - out[1] / (out[0] * out[0]));
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* A whole run, in the order of the paper's algorithm: initialise R0 replicas  */
/* at beta_0 = 0; for each later temperature: resample (Q, tau, Poisson copies) */
/* then theta sweeps, then measure and record -beta F~ = ln Omega + sum ln Q    */
/* (eq. sumQ).  The schedule is indexed upwards here: betas[0] = 0 < betas[1]   */
/* < ... (the paper indexes it downwards).  Sweep index t = (k-1) ns + s.       */
/* rec is [nT][8]: beta, R~, ln Q, -beta F~, E mean, E var, E skew, status.     */
/* Final population left in spins/E (capacity cap).                            */
/* ------------------------------------------------------------------------- */
#define REC_W 8
int orc_run(int dim, int L, const int8_t* J, uint64_t seed, int64_t R0, int nT, const double* betas,
            const double* R_targets, int ns, int64_t cap, double* rec, uint8_t* spins_out, int32_t* E_out,
            int64_t* R_out)
{
    int N = orc_num_sites(dim, L);
    uint8_t* s[2];
    int32_t* E[2];
    s[0] = (uint8_t*)malloc((size_t)cap * N);
    s[1] = (uint8_t*)malloc((size_t)cap * N);
    E[0] = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    E[1] = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int32_t* counts = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int64_t* offsets = (int64_t*)malloc(((size_t)cap + 1) * sizeof(int64_t));
    int status = ORC_OK;
    int cur = 0;
    int64_t R = R0;
    double lnOmega = (double)N * log(2.0);
    double acc = 0.0;
    if (R0 > cap) status = ORC_ERR_CAPACITY;
    else orc_init_population(dim, L, J, seed, R0, s[0], E[0]);
    for (int k = 0; k < nT; ++k) {
        double* rk = rec + (int64_t)k * REC_W;
        if (status == ORC_OK && k > 0) {
            double out[3];
            int64_t R_new;
            double Rt = R_targets ? R_targets[k] : (double)R0;
            status = orc_resample(dim, L, seed, k, betas[k - 1], betas[k], Rt, R, s[cur], E[cur], cap,
                                  s[cur ^ 1], E[cur ^ 1], counts, offsets, out, &R_new);
            if (status == ORC_OK) {
                acc += out[1];
                cur ^= 1;
                R = R_new;
                orc_sweep(dim, L, J, seed, betas[k], R, s[cur], E[cur], (int64_t)(k - 1) * ns, ns);
            }
            rk[2] = out[1];
        } else {
            rk[2] = 0.0;
        }
        double mom[3] = {0, 0, 0};
        if (status == ORC_OK) orc_energy_moments(R, E[cur], mom);
        rk[0] = betas[k];
        rk[1] = (double)R;
        rk[3] = lnOmega + acc;
        rk[4] = mom[0];
        rk[5] = mom[1];
        rk[6] = mom[2];
        rk[7] = (double)status;
    }
    if (spins_out) memcpy(spins_out, s[cur], (size_t)R * N);
    if (E_out) memcpy(E_out, E[cur], (size_t)R * sizeof(int32_t));
    if (R_out) *R_out = R;
    free(s[0]); free(s[1]); free(E[0]); free(E[1]); free(counts); free(offsets);
    return status;
}

/* ========================================================================= */
/* Gaussian couplings (the model of Sec. IV: J_ij independent normal, mean 0,  */
/* variance 1).  Energies are real, so every floating-point step below is      */
/* fixed in order and in the operations used, and the library follows the    */
/* same definitions with its own code:                                         */
/*   J_b: Box-Muller from Philox(ctr = (b, 0, 0, 6), key = disorder seed):     */
/*        m1 = (w0 >> 5) 2^26 + (w1 >> 6), u1 = (m1 + 1) 2^-53 in (0, 1],     */
/*        m2 = (w2 >> 5) 2^26 + (w3 >> 6), u2 = m2 2^-53 in [0, 1),            */
/*        J_b = sqrt(-2 ln u1) cos(2 pi u2)            (libm, host side);      */
/*   E  = sum over bonds b = 0, 1, ... of J_b s_i s_j, added in bond order     */
/*        starting from 0, recomputed after every call of ns sweeps;           */
/*   h_i = sum over the incident bonds in the order +x, +y, +z, -x, -y, -z     */
/*        (chain: +1, -1) of J s_other; dE = -2 s_i h_i;                       */
/*   accept dE <= 0; otherwise p = expd(-(beta dE)); accept if p >= 1, else    */
/*        with T64 = (uint64) (p 2^64) by the lazy 16 + 48-bit compare;        */
/*   resampling: E_lo = min E, w_j = expd(-(dbeta (E_j - E_lo))),              */
/*        S = sum of w_j over j = 0, 1, ... in replica order (eq. Q),         */
/*        ln Q = -dbeta E_lo + ln S - ln R~,                                   */
/*        copies of j ~ Poisson((R_target w_j) / S) as for +-J couplings.      */
/* expd is exp written out: x = k ln 2 + r with k = floor(x / ln 2 + 1/2), r   */
/* by a two-part ln 2 (Cody and Waite), e^r by its Taylor series to r^13 in    */
/* Horner form, then scaled by 2^k; 0 for x < -745.                            */
/* ========================================================================= */
#define TAG_GAUSS 6u

double orc_expd(double x)
{
    static const double c[14] = {1.0, 1.0, 0.5, 0.16666666666666666, 0.041666666666666664, 0.008333333333333333,
                                 0.001388888888888889, 0.0001984126984126984, 2.48015873015873e-05,
                                 2.7557319223985893e-06, 2.755731922398589e-07, 2.505210838544172e-08,
                                 2.08767569878681e-09, 1.6059043836821613e-10};
    const double inv_ln2 = 1.4426950408889634;
    const double ln2_hi = 0.6931471803691238;     /* 32 significant bits: k ln2_hi is exact */
    const double ln2_lo = 1.9082149292705877e-10; /* ln 2 - ln2_hi */
    if (x < -745.0) return 0.0;
    double k = floor(x * inv_ln2 + 0.5);
    double r = (x - k * ln2_hi) - k * ln2_lo;
    double p = c[13];
    for (int n = 12; n >= 0; --n) p = p * r + c[n];
    return ldexp(p, (int)k);
}

void orc_couplings_gauss(int dim, int L, uint64_t disorder_seed, double* J)
{
    int nb = orc_num_bonds(dim, L);
    for (int b = 0; b < nb; ++b) {
        uint32_t w[4];
        philox_seeded((uint32_t)b, 0, 0, TAG_GAUSS, disorder_seed, w);
        uint64_t m1 = ((uint64_t)(w[0] >> 5) << 26) | (uint64_t)(w[1] >> 6);
        uint64_t m2 = ((uint64_t)(w[2] >> 5) << 26) | (uint64_t)(w[3] >> 6);
        double u1 = ldexp((double)(m1 + 1), -53);
        double u2 = ldexp((double)m2, -53);
        J[b] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    }
}

double orc_energy_gauss(int dim, int L, const double* J, const uint8_t* s)
{
    int nb = orc_num_bonds(dim, L);
    double E = 0.0;
    for (int b = 0; b < nb; ++b) {
        int i, j;
        bond_ends(dim, L, b, &i, &j);
        double t = spin_value(s[i]) * spin_value(s[j]) > 0 ? J[b] : -J[b];
        E = E + t;
    }
    return E;
}

double orc_delta_energy_gauss(int dim, int L, const double* J, const uint8_t* s, int i)
{
    double h = 0.0;
    for (int k = 0; k < coordination(dim); ++k) {
        int b, j;
        incident_bond(dim, L, i, k, &b, &j);
        h = h + (spin_value(s[j]) > 0 ? J[b] : -J[b]);
    }
    return spin_value(s[i]) > 0 ? -2.0 * h : 2.0 * h;
}

void orc_init_range_gauss(int dim, int L, const double* J, uint64_t seed, int64_t r_first, int64_t count,
                          uint8_t* s, double* E)
{
    int N = orc_num_sites(dim, L);
    for (int64_t q = 0; q < count; ++q) {
        int64_t r = r_first + q;
        for (int i = 0; i < N; ++i) {
            uint32_t out[4];
            philox_seeded((uint32_t)(i >> 7), (uint32_t)r, 0, TAG_INIT, seed, out);
            s[q * N + i] = (uint8_t)((out[(i & 127) >> 5] >> (i & 31)) & 1);
        }
        E[q] = orc_energy_gauss(dim, L, J, s + q * N);
    }
}

/* acceptance of a move with energy change dE > 0 at beta (the same 64-bit rule as for +-J) */
static int accept_gauss(uint64_t seed, int64_t r, int64_t t, int colour, int i, double beta, double dE)
{
    if (dE <= 0.0) return 1;
    double p = orc_expd(-(beta * dE));
    if (p >= 1.0) return 1;
    uint64_t T64 = (uint64_t)ldexp(p, 64);
    return orc_met_accept(seed, r, t, colour, i, T64);
}

void orc_sweep_range_gauss(int dim, int L, const double* J, uint64_t seed, double beta, int64_t r_first,
                           int64_t count, uint8_t* spins, double* E, int64_t t0, int ns)
{
    int N = orc_num_sites(dim, L);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; ++q) {
        int64_t r = r_first + q;
        uint8_t* s = spins + q * N;
        for (int64_t t = t0; t < t0 + ns; ++t)
            for (int colour = 0; colour < 2; ++colour)
                for (int i = 0; i < N; ++i) {
                    if (orc_colour(dim, L, i) != colour) continue;
                    double dE = orc_delta_energy_gauss(dim, L, J, s, i);
                    if (accept_gauss(seed, r, t, colour, i, beta, dE)) s[i] ^= 1;
                }
        if (ns > 0) E[q] = orc_energy_gauss(dim, L, J, s);
    }
}

/* copy numbers of one resampling step; out[0] = S, out[1] = ln Q, out[2] = E_lo */
int orc_copy_numbers_gauss(uint64_t seed, int64_t k, double beta_from, double beta_to, double R_target, int64_t R,
                           const double* E, int32_t* counts, double* out)
{
    double dbeta = beta_to - beta_from;
    if (R <= 0 || !(dbeta >= 0.0) || !(R_target > 0.0)) return ORC_ERR_ARG;
    double E_lo = E[0];
    for (int64_t j = 1; j < R; ++j)
        if (E[j] < E_lo) E_lo = E[j];
    /* eq. Q with the energies shifted by E_lo, summed over the replicas in their order */
    double S = 0.0;
    for (int64_t j = 0; j < R; ++j) S = S + orc_expd(-(dbeta * (E[j] - E_lo)));
    out[0] = S;
    out[1] = -dbeta * E_lo + log(S) - log((double)R);
    out[2] = E_lo;
    if (!isfinite(S) || !(S > 0.0)) return ORC_ERR_NONFINITE;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < R; ++j) {
        double w = orc_expd(-(dbeta * (E[j] - E_lo)));
        counts[j] = (int32_t)orc_poisson((R_target * w) / S, seed, j, k);
    }
    return ORC_OK;
}

void orc_energy_moments_gauss(int64_t R, const double* E, double* out)
{
    double sum = 0.0;
    for (int64_t j = 0; j < R; ++j) sum += E[j];
    double mean = sum / (double)R;
    double m2 = 0.0, m3 = 0.0;
    for (int64_t j = 0; j < R; ++j) {
        double d = E[j] - mean;
        m2 += d * d;
        m3 += d * d * d;
    }
    m2 /= (double)R;
    m3 /= (double)R;
    out[0] = mean;
    out[1] = m2;
    out[2] = m2 > 0.0 ? m3 / (m2 * sqrt(m2)) : 0.0;
}

/* a whole run with Gaussian couplings; rec as for orc_run */
int orc_run_gauss(int dim, int L, const double* J, uint64_t seed, int64_t R0, int nT, const double* betas,
                  const double* R_targets, int ns, int64_t cap, double* rec, uint8_t* spins_out, double* E_out,
                  int64_t* R_out)
{
    int N = orc_num_sites(dim, L);
    uint8_t* s[2];
    double* E[2];
    s[0] = (uint8_t*)malloc((size_t)cap * N);
    s[1] = (uint8_t*)malloc((size_t)cap * N);
    E[0] = (double*)malloc((size_t)cap * sizeof(double));
    E[1] = (double*)malloc((size_t)cap * sizeof(double));
    int32_t* counts = (int32_t*)malloc((size_t)cap * sizeof(int32_t));
    int status = ORC_OK;
    int cur = 0;
    int64_t R = R0;
    double acc = 0.0, lnOmega = (double)N * log(2.0);
    if (R0 > cap) status = ORC_ERR_CAPACITY;
    else orc_init_range_gauss(dim, L, J, seed, 0, R0, s[0], E[0]);
    for (int k = 0; k < nT; ++k) {
        double* rk = rec + (int64_t)k * REC_W;
        rk[2] = 0.0;
        if (status == ORC_OK && k > 0) {
            double out[3];
            double Rt = R_targets ? R_targets[k] : (double)R0;
            status = orc_copy_numbers_gauss(seed, k, betas[k - 1], betas[k], Rt, R, E[cur], counts, out);
            if (status == ORC_OK) {
                int64_t tot = 0;
                for (int64_t j = 0; j < R; ++j) tot += counts[j];
                if (tot > cap) status = ORC_ERR_CAPACITY;
                else if (tot == 0) status = ORC_ERR_EXTINCT;
            }
            if (status == ORC_OK) {
                int64_t dst = 0;
                for (int64_t j = 0; j < R; ++j)
                    for (int32_t c = 0; c < counts[j]; ++c, ++dst) {
                        memcpy(s[cur ^ 1] + dst * N, s[cur] + j * N, (size_t)N);
                        E[cur ^ 1][dst] = E[cur][j];
                    }
                acc += out[1];
                cur ^= 1;
                R = dst;
                orc_sweep_range_gauss(dim, L, J, seed, betas[k], 0, R, s[cur], E[cur], (int64_t)(k - 1) * ns, ns);
                rk[2] = out[1];
            }
        }
        double mom[3] = {0, 0, 0};
        if (status == ORC_OK) orc_energy_moments_gauss(R, E[cur], mom);
        rk[0] = betas[k];
        rk[1] = (double)R;
        rk[3] = lnOmega + acc;
        rk[4] = mom[0];
        rk[5] = mom[1];
        rk[6] = mom[2];
        rk[7] = (double)status;
    }
    if (spins_out) memcpy(spins_out, s[cur], (size_t)R * N);
    if (E_out) memcpy(E_out, E[cur], (size_t)R * sizeof(double));
    if (R_out) *R_out = R;
    free(s[0]); free(s[1]); free(E[0]); free(E[1]); free(counts);
    return status;
}

/* threads for the oracle's parallel loops from now on (n >= 1) */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* number of OpenMP threads the oracle's parallel loops use */
int orc_num_threads(void)
{
    int n = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
#endif
    return n;
}
