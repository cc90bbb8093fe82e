/* Drives every entry point of the CPU oracle (oracle/pa_oracle.c) on small inputs, including its
 * error paths, so that a build with AddressSanitizer and UndefinedBehaviorSanitizer can check the
 * oracle's memory accesses and arithmetic.  Exits 0 and prints "ok" when every call returned
 * what it should; any sanitizer report aborts the run. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int orc_num_sites(int dim, int L);
int orc_num_bonds(int dim, int L);
int orc_colour(int dim, int L, int i);
void orc_couplings(int dim, int L, uint64_t disorder_seed, int8_t* J);
int64_t orc_energy(int dim, int L, const int8_t* J, const uint8_t* s);
int orc_delta_energy(int dim, int L, const int8_t* J, const uint8_t* s, int i);
void orc_init_population(int dim, int L, const int8_t* J, uint64_t seed, int64_t R, uint8_t* s, int32_t* E);
uint64_t orc_threshold(double beta, int dE, int* always);
void orc_sweep(int dim, int L, const int8_t* J, uint64_t seed, double beta, int64_t R, uint8_t* spins, int32_t* E,
               int64_t t0, int ns);
int orc_ladder_table(int m, uint64_t* C);
int64_t orc_poisson(double lambda, uint64_t seed, int64_t j, int64_t k);
int orc_copy_numbers(uint64_t seed, int64_t k, double beta_from, double beta_to, double R_target, int64_t R,
                     const int32_t* E, int32_t* counts, double* out);
int orc_resample(int dim, int L, uint64_t seed, int64_t k, double beta_from, double beta_to, double R_target,
                 int64_t R, const uint8_t* spins, const int32_t* E, int64_t capacity, uint8_t* spins_new,
                 int32_t* E_new, int32_t* counts, int64_t* offsets, double* out, int64_t* R_new);
void orc_energy_moments(int64_t R, const int32_t* E, double* out);
int64_t orc_overlap_hist(int N, int64_t RA, const uint8_t* sA, int64_t RB, const uint8_t* sB, int64_t* hist);
void orc_overlap_stats(int N, const int64_t* hist, double* out);
int orc_weighted_average(int M, const double* x, const double* Rr, const double* A, int n_obs, double* A_bar,
                         double* omega, double* mbF_bar, double* var, double* mean_x);
int orc_overlap_average(int n_pairs, const double* x, const double* Rr, const double* Q, double* out);
int orc_run(int dim, int L, const int8_t* J, uint64_t seed, int64_t R0, int nT, const double* betas,
            const double* R_targets, int ns, int64_t cap, double* rec, uint8_t* spins_out, int32_t* E_out,
            int64_t* R_out);
double orc_expd(double x);
void orc_couplings_gauss(int dim, int L, uint64_t disorder_seed, double* J);
double orc_energy_gauss(int dim, int L, const double* J, const uint8_t* s);
double orc_delta_energy_gauss(int dim, int L, const double* J, const uint8_t* s, int i);
void orc_init_range_gauss(int dim, int L, const double* J, uint64_t seed, int64_t r_first, int64_t count,
                          uint8_t* s, double* E);
void orc_sweep_range_gauss(int dim, int L, const double* J, uint64_t seed, double beta, int64_t r_first,
                           int64_t count, uint8_t* spins, double* E, int64_t t0, int ns);
int orc_copy_numbers_gauss(uint64_t seed, int64_t k, double beta_from, double beta_to, double R_target, int64_t R,
                           const double* E, int32_t* counts, double* out);
void orc_energy_moments_gauss(int64_t R, const double* E, double* out);
int orc_run_gauss(int dim, int L, const double* J, uint64_t seed, int64_t R0, int nT, const double* betas,
                  const double* R_targets, int ns, int64_t cap, double* rec, uint8_t* spins_out, double* E_out,
                  int64_t* R_out);
void orc_set_num_threads(int n);
int orc_num_threads(void);

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static void pm1_lattice(int dim, int L)
{
    const int N = orc_num_sites(dim, L), B = orc_num_bonds(dim, L);
    const int64_t R = 150, cap = 400;
    int8_t* J = malloc((size_t)B);
    uint8_t* s = malloc((size_t)cap * N);
    uint8_t* s2 = malloc((size_t)cap * N);
    int32_t* E = malloc(sizeof(int32_t) * cap);
    int32_t* E2 = malloc(sizeof(int32_t) * cap);
    int32_t* counts = malloc(sizeof(int32_t) * cap);
    int64_t* offsets = malloc(sizeof(int64_t) * (cap + 1));
    orc_couplings(dim, L, 3, J);
    orc_init_population(dim, L, J, 7, R, s, E);
    for (int64_t j = 0; j < R; ++j) CHECK(E[j] == orc_energy(dim, L, J, s + j * N));
    for (int i = 0; i < N; ++i) (void)orc_delta_energy(dim, L, J, s, i) , (void)orc_colour(dim, L, i);
    orc_sweep(dim, L, J, 7, 0.8, R, s, E, 0, 2);
    for (int64_t j = 0; j < R; ++j) CHECK(E[j] == orc_energy(dim, L, J, s + j * N));
    double out[3];
    int64_t R_new = 0;
    int st = orc_resample(dim, L, 7, 1, 0.8, 1.0, (double)R, R, s, E, cap, s2, E2, counts, offsets, out, &R_new);
    CHECK(st == 0 && R_new > 0 && R_new <= cap && offsets[R] == R_new);
    st = orc_resample(dim, L, 7, 1, 0.8, 1.0, 1e5, R, s, E, cap, s2, E2, counts, offsets, out, &R_new);
    CHECK(st == 2);  /* capacity */
    st = orc_resample(dim, L, 7, 1, 0.8, 1.0, 1e-9, R, s, E, cap, s2, E2, counts, offsets, out, &R_new);
    CHECK(st == 3);  /* extinction */
    st = orc_copy_numbers(7, 1, 1.0, 0.5, (double)R, R, E, counts, out);
    CHECK(st == 1);  /* beta decreasing */
    double mom[3];
    orc_energy_moments(R, E, mom);
    int64_t* hist = calloc((size_t)N + 1, sizeof(int64_t));
    CHECK(orc_overlap_hist(N, R, s, R - 7, s2, hist) == R - 7);
    double q[3];
    orc_overlap_stats(N, hist, q);
    CHECK(q[0] >= 0.0 && q[0] <= 1.0 && q[2] >= 0.0 && q[2] <= 1.0);
    const int nT = 6;
    double betas[6], rec[6 * 8];
    for (int k = 0; k < nT; ++k) betas[k] = 0.3 * k;
    int64_t Rf = 0;
    st = orc_run(dim, L, J, 11, R, nT, betas, NULL, 2, cap, rec, s, E, &Rf);
    CHECK(st == 0 && Rf > 0);
    st = orc_run(dim, L, J, 11, cap + 64, nT, betas, NULL, 2, cap, rec, NULL, NULL, &Rf);
    CHECK(st == 2);
    free(hist); free(J); free(s); free(s2); free(E); free(E2); free(counts); free(offsets);
}

static void gauss_lattice(int dim, int L)
{
    const int N = orc_num_sites(dim, L), B = orc_num_bonds(dim, L);
    const int64_t R = 120, cap = 300;
    double* J = malloc(sizeof(double) * B);
    uint8_t* s = malloc((size_t)cap * N);
    double* E = malloc(sizeof(double) * cap);
    int32_t* counts = malloc(sizeof(int32_t) * cap);
    orc_couplings_gauss(dim, L, 5, J);
    orc_init_range_gauss(dim, L, J, 9, 0, R, s, E);
    for (int i = 0; i < N; ++i) (void)orc_delta_energy_gauss(dim, L, J, s, i);
    orc_sweep_range_gauss(dim, L, J, 9, 1.3, 0, R, s, E, 0, 2);
    CHECK(E[3] == orc_energy_gauss(dim, L, J, s + 3 * N));
    double out[3];
    CHECK(orc_copy_numbers_gauss(9, 1, 1.3, 1.5, (double)R, R, E, counts, out) == 0);
    double mom[3];
    orc_energy_moments_gauss(R, E, mom);
    double betas[5] = {0.0, 0.5, 1.0, 1.5, 2.0}, rec[5 * 8];
    int64_t Rf = 0;
    CHECK(orc_run_gauss(dim, L, J, 13, R, 5, betas, NULL, 2, cap, rec, s, E, &Rf) == 0 && Rf > 0);
    free(J); free(s); free(E); free(counts);
}

int main(void)
{
    uint32_t ctr[4] = {0, 1, 2, 3}, key[2] = {4, 5}, o[4];
    orc_philox(ctr, key, o);
    int always = 0;
    (void)orc_threshold(0.5, 8, &always);
    uint64_t C[512];
    for (int m = -20; m <= 6; ++m) CHECK(orc_ladder_table(m, C) > 1);
    for (int i = 0; i < 200; ++i) (void)orc_poisson(0.01 * i * i, 1, i, 1);
    for (double x = -800.0; x <= 0.0; x += 3.7) (void)orc_expd(x);
    orc_set_num_threads(2);
    CHECK(orc_num_threads() == 2);
    pm1_lattice(1, 64);
    pm1_lattice(3, 2);
    pm1_lattice(3, 6);
    gauss_lattice(1, 40);
    gauss_lattice(3, 4);
    double x[6] = {1.0, 2.0, 3.0, 4.0, 5.0, 6.0}, Rr[6] = {1, 2, 3, 4, 5, 6}, A[12], Ab[2], om[6], mbf, var, mean;
    for (int i = 0; i < 12; ++i) A[i] = 0.1 * i;
    CHECK(orc_weighted_average(6, x, Rr, A, 2, Ab, om, &mbf, &var, &mean) == 0);
    CHECK(orc_weighted_average(0, x, NULL, A, 2, Ab, om, &mbf, &var, &mean) == 1);
    double Q[9] = {0.5, 0.3, 0.1, 0.4, 0.2, 0.2, 0.3, 0.1, 0.3}, ov[4];
    CHECK(orc_overlap_average(3, x, Rr, Q, ov) == 0);
    CHECK(orc_overlap_average(0, x, NULL, Q, ov) == 1);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
