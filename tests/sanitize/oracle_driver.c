/* Exercises every entry point of the C oracle (oracle/wdr_oracle.c) on two
 * small lattices; built with AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_sanitize_cpu.py, which fails on any report.  Test
 * infrastructure only. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_gamma(int mu, double *out);
void oracle_site_maps(const int *L, const int *B, int32_t *block_id, int32_t *colour, int32_t *parity);
void oracle_apply_D(const int *L, const int *bc, double kappa, const double *U, const double *clov, const double *in,
                    double *out);
void oracle_apply_Dblock(const int *L, const int *B, const int *bc, double kappa, const double *U, const double *clov,
                         int colour, const double *in, double *out);
void oracle_apply_Dhop(const int *L, const int *B, const int *bc, double kappa, const double *U, int from_colour,
                       const double *in, double *out);
void oracle_apply_Dee(const int *L, const int *B, const int *bc, double kappa, const double *U, int blocked,
                      const double *in, double *out);
void oracle_mul_g5(long V, const double *in, double *out);
int oracle_cgne(const int *L, const int *B, const int *bc, double kappa, const double *Ud, const double *clov, int op,
                int colour, const double *bd, double *xd, double *yd, double tol, int maxit, double *rel_resid);
void oracle_sap(const int *L, const int *B, const int *bc, double kappa, const double *Ud, const double *clovd,
                int ncy, int nmr, const double *etad, double *xd);
void oracle_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]);
void oracle_noise(const int *L, int kind, uint64_t seed, int32_t step, int32_t k, const uint8_t *mask, double *out);

static double urand(uint64_t *s)
{
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0 - 0.5;
}

static double *fill(long n, uint64_t *s)
{
    double *a = malloc(n * sizeof(double));
    for (long i = 0; i < n; ++i) a[i] = urand(s);
    return a;
}

static int run(const int L[4], const int B[4], const int bc[4])
{
    uint64_t s = 12345;
    long V = (long)L[0] * L[1] * L[2] * L[3], n = 24 * V;
    double *U = fill(V * 72, &s), *clov = fill(V * 288, &s), *in = fill(n, &s);
    /* links near the identity, so that the solves converge */
    for (long x = 0; x < 4 * V; ++x)
        for (int a = 0; a < 3; ++a) U[x * 18 + 2 * (3 * a + a)] += 1.0;
    for (long i = 0; i < V * 288; ++i) clov[i] *= 0.05;
    double *out = calloc(n, sizeof(double)), *x = calloc(n, sizeof(double)), *y = calloc(n, sizeof(double));
    int32_t *bid = malloc(V * 4), *col = malloc(V * 4), *par = malloc(V * 4);
    uint8_t *mask = malloc(V);
    double g[32], res = 0;
    for (int mu = 0; mu < 4; ++mu) oracle_gamma(mu, g);
    oracle_site_maps(L, B, bid, col, par);
    oracle_apply_D(L, bc, 0.12, U, NULL, in, out);
    oracle_apply_D(L, bc, 0.12, U, clov, in, out);
    for (int c = 0; c < 3; ++c) {
        oracle_apply_Dblock(L, B, bc, 0.12, U, NULL, c, in, out);
        oracle_apply_Dblock(L, B, bc, 0.12, U, clov, c, in, out);
    }
    for (int c = 0; c < 2; ++c) oracle_apply_Dhop(L, B, bc, 0.12, U, c, in, out);
    for (int b = 0; b < 2; ++b) oracle_apply_Dee(L, B, bc, 0.12, U, b, in, out);
    oracle_mul_g5(V, in, out);
    int it = oracle_cgne(L, B, bc, 0.1, U, NULL, 0, 2, in, x, y, 1e-10, 5000, &res);
    /* memory safety only: a random (non-hermitian) clover matrix may converge slowly */
    int it2 = oracle_cgne(L, B, bc, 0.1, U, clov, 1, 0, in, x, y, 1e-10, 200, &res);
    int it3 = oracle_cgne(L, B, bc, 0.1, U, NULL, 0, 2, in, x, y, 1e-10, 1, &res); /* iteration cap */
    oracle_sap(L, B, bc, 0.1, U, NULL, 2, 3, in, x);
    oracle_sap(L, B, bc, 0.1, U, clov, 2, 3, in, x);
    uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, o[4];
    oracle_philox4x64_10(ctr, key, o);
    for (long i = 0; i < V; ++i) mask[i] = (uint8_t)(i & 1);
    for (int kind = 0; kind < 2; ++kind) {
        oracle_noise(L, kind, 7, 1, 2, NULL, out);
        oracle_noise(L, kind, 7, 1, 2, mask, out);
    }
    printf("L %d %d %d %d: cgne %d %d %d\n", L[0], L[1], L[2], L[3], it, it2, it3);
    free(U), free(clov), free(in), free(out), free(x), free(y), free(bid), free(col), free(par), free(mask);
    return it > 0 && it2 != 0 && it3 == -1 ? 0 : 1;
}

int main(void)
{
    const int L1[4] = {4, 4, 4, 4}, B1[4] = {2, 2, 2, 2}, bc1[4] = {1, 1, 1, -1};
    const int L2[4] = {4, 2, 2, 6}, B2[4] = {2, 2, 2, 2}, bc2[4] = {1, -1, 0, 1};
    return run(L1, B1, bc1) | run(L2, B2, bc2);
}
