/* Runs the oracle's entry points on small inputs, edge cases and invalid
 * arguments, built with AddressSanitizer and UBSan. Exit status 0 when every
 * call behaves (valid calls return 0, invalid ones -1). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_cost_pred(int n, int m, int k, const int32_t *lits, int pred, int32_t *cost);
int oracle_cost_at_pred(int n, int m, int k, const int32_t *lits, int pred, const uint64_t *xs, int64_t count,
                        int32_t *cost);
int oracle_count_solutions_pred(int n, int m, int k, const int32_t *lits, int pred, uint64_t *count);
int oracle_state(int n, const int32_t *cost, int p, const double *gammas, const double *betas, double *psi);
int oracle_qaoa(int n, const int32_t *cost, int p, const double *gammas, const double *betas, double *psi_out,
                double out[3]);
int oracle_qaoa_grad(int n, const int32_t *cost, int p, const double *gammas, const double *betas, double w_psucc,
                     double w_energy, double *dgammas, double *dbetas, double out[3]);
int oracle_sample(int n, const double *psi, const double *u, int64_t count, uint64_t *out);

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            fprintf(stderr, "FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);   \
            return 1;                                                        \
        }                                                                    \
    } while (0)

int main(void) {
    srand(3);
    for (int trial = 0; trial < 60; trial++) {
        int n = 1 + rand() % 9, k = 1 + rand() % (n < 5 ? n : 5), m = rand() % 20, p = rand() % 4;
        int32_t *lits = malloc(sizeof(int32_t) * (size_t)(m * k + 1));
        for (int i = 0; i < m * k; i++) {
            int v = 1 + rand() % n;
            lits[i] = (rand() & 1) ? -v : v;
        }
        int64_t N = (int64_t)1 << n;
        int32_t *cost = malloc(sizeof(int32_t) * (size_t)N);
        double *psi = malloc(sizeof(double) * 2 * (size_t)N);
        double g[4], b[4], dg[4], db[4], out[3];
        for (int l = 0; l < 4; l++) {
            g[l] = (rand() % 1000) / 300.0;
            b[l] = (rand() % 1000) / 300.0;
        }
        for (int pred = 0; pred < 2; pred++) {
            CHECK(oracle_cost_pred(n, m, k, lits, pred, cost) == 0);
            uint64_t cnt = 0;
            CHECK(oracle_count_solutions_pred(n, m, k, lits, pred, &cnt) == 0);
            uint64_t xs[3] = {0, (uint64_t)(N - 1), (uint64_t)(N / 2)};
            int32_t c3[3];
            CHECK(oracle_cost_at_pred(n, m, k, lits, pred, xs, 3, c3) == 0);
            CHECK(c3[0] == cost[0] && c3[1] == cost[N - 1] && c3[2] == cost[N / 2]);
        }
        CHECK(oracle_cost_pred(n, m, k, lits, 0, cost) == 0);
        CHECK(oracle_qaoa(n, cost, p, g, b, psi, out) == 0);
        CHECK(fabs(out[2] - 1.0) < 1e-12);
        CHECK(oracle_state(n, cost, p, g, b, psi) == 0);
        CHECK(oracle_qaoa_grad(n, cost, p, g, b, 1.0, 0.3, dg, db, out) == 0);
        double u[5] = {0.0, 0.25, 0.5, 0.75, 0.999999};
        uint64_t s[5];
        CHECK(oracle_sample(n, psi, u, 5, s) == 0);
        for (int q = 0; q < 5; q++) CHECK(s[q] < (uint64_t)N);
        free(lits);
        free(cost);
        free(psi);
    }
    /* invalid arguments */
    int32_t bad[2] = {1, 9};
    int32_t c[16];
    CHECK(oracle_cost_pred(3, 1, 2, bad, 0, c) == -1);
    CHECK(oracle_cost_pred(0, 0, 1, NULL, 0, c) == -1);
    CHECK(oracle_cost_pred(3, 0, 1, NULL, 2, c) == -1);
    double psi[4] = {0.6, 0, 0.8, 0}, uu[1] = {1.0};
    uint64_t s1[1];
    CHECK(oracle_sample(1, psi, uu, 1, s1) == -1);
    printf("oracle checks ok\n");
    return 0;
}
