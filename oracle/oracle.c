/*
 * Plain FP64 CPU oracle for depth-p QAOA on random k-NAE-SAT
 * (Elkadi & Bondesan, "Quantum Approximate Optimisation for Not-All-Equal SAT"),
 * with the plain k-SAT clause predicate beside the NAE one.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this library. The GPU
 * library never links, includes or calls it, and it shares no code, header,
 * table or constant with the GPU library.
 *
 * Everything here is the plain definition, written for a reader to check
 * against the paper by eye: no blocking, no fusion, no reordering.
 *
 * Conventions (readings of the paper, listed in the design notes):
 *  - literal l = +(v+1) is x_v, l = -(v+1) is NOT x_v (0 <= v < n);
 *  - basis index x = sum_v x_v 2^v (variable v is bit v);
 *  - |+> is the real uniform state 2^{-n/2};
 *  - layer l (l = 0 .. p-1, applied in array order) applies the phase
 *    U_C(gamma_l) = exp(-i gamma_l H_C) and then the mixer
 *    U_B(beta_l) = exp(-i beta_l sum_j X_j) = prod_j (cos b I - i sin b X_j);
 *  - no renormalisation: p_succ and E[C] are raw expectations on the
 *    evolved state and the norm is reported beside them.
 *
 * All routines return 0 on success and -1 on invalid arguments or when
 * memory cannot be allocated.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Problem encoding                                                    */
/* ------------------------------------------------------------------ */

/* Truth value of one literal at assignment x: a positive literal is true when
 * its variable is 1, a negated one when it is 0 (Section 2.2, CNF literals). */
static int literal_value(uint64_t x, int32_t lit) {
    int v = (lit > 0 ? lit : -lit) - 1;
    int bit = (int)((x >> v) & 1u);
    return lit > 0 ? bit : 1 - bit;
}

/* NAE violation of one clause: the clause is violated exactly when all of its
 * literals are false (the OR-clause is unsatisfied) or all of them are true
 * (Appendix A.2, eq. demorgannae; Section 2.2). Each literal is evaluated on
 * its own, so a variable repeated with both signs never violates. */
static int clause_violated(uint64_t x, const int32_t *clause, int k) {
    int n_true = 0;
    for (int j = 0; j < k; j++) n_true += literal_value(x, clause[j]);
    return n_true == 0 || n_true == k;
}

/* k-SAT (Section 2.2): an OR-clause is satisfied when any of its literals is
 * true, so it is violated exactly when every literal is false. */
static int sat_clause_violated(uint64_t x, const int32_t *clause, int k) {
    for (int j = 0; j < k; j++)
        if (literal_value(x, clause[j])) return 0;
    return 1;
}

/* Clause predicate: 0 = NAE (the paper's problem), 1 = k-SAT. */
static int violated(int pred, uint64_t x, const int32_t *clause, int k) {
    return pred ? sat_clause_violated(x, clause, k) : clause_violated(x, clause, k);
}

static int check_instance(int n, int m, int k, const int32_t *lits) {
    if (n < 1 || n > 40 || m < 0 || k < 1) return -1;
    if (m > 0 && lits == NULL) return -1;
    for (int64_t i = 0; i < (int64_t)m * k; i++) {
        int32_t l = lits[i];
        if (l == 0 || l > n || l < -n) return -1;
    }
    return 0;
}

/* Cost diagonal C(x) = number of violated clauses for every x in [0, 2^n):
 * NAE-violated (pred 0; Section 3.2, eq. knaesatobj) or SAT-violated
 * (pred 1; Section 2.2). */
int oracle_cost_pred(int n, int m, int k, const int32_t *lits, int pred, int32_t *cost) {
    if (check_instance(n, m, k, lits) || cost == NULL || pred < 0 || pred > 1) return -1;
    int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) {
        int32_t c = 0;
        for (int i = 0; i < m; i++) c += violated(pred, (uint64_t)x, lits + (int64_t)i * k, k);
        cost[x] = c;
    }
    return 0;
}

int oracle_cost(int n, int m, int k, const int32_t *lits, int32_t *cost) {
    return oracle_cost_pred(n, m, k, lits, 0, cost);
}

/* C(x) at the given basis states only (same definition as oracle_cost_pred). */
int oracle_cost_at_pred(int n, int m, int k, const int32_t *lits, int pred, const uint64_t *xs,
                        int64_t count, int32_t *cost) {
    if (check_instance(n, m, k, lits) || xs == NULL || cost == NULL || count < 0 || pred < 0 || pred > 1)
        return -1;
    for (int64_t q = 0; q < count; q++)
        if (n < 64 && (xs[q] >> n) != 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; q++) {
        int32_t c = 0;
        for (int i = 0; i < m; i++) c += violated(pred, xs[q], lits + (int64_t)i * k, k);
        cost[q] = c;
    }
    return 0;
}

int oracle_cost_at(int n, int m, int k, const int32_t *lits, const uint64_t *xs, int64_t count,
                   int32_t *cost) {
    return oracle_cost_at_pred(n, m, k, lits, 0, xs, count, cost);
}

/* Number of solutions, #{x : C(x) = 0}, without storing C. Used to keep
 * only satisfiable instances (Section 3.3: evaluation sets are satisfiable). */
int oracle_count_solutions_pred(int n, int m, int k, const int32_t *lits, int pred, uint64_t *count) {
    if (check_instance(n, m, k, lits) || count == NULL || pred < 0 || pred > 1) return -1;
    int64_t N = (int64_t)1 << n;
    uint64_t total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int64_t x = 0; x < N; x++) {
        int sat = 1;
        for (int i = 0; i < m && sat; i++)
            if (violated(pred, (uint64_t)x, lits + (int64_t)i * k, k)) sat = 0;
        total += (uint64_t)sat;
    }
    *count = total;
    return 0;
}

int oracle_count_solutions(int n, int m, int k, const int32_t *lits, uint64_t *count) {
    return oracle_count_solutions_pred(n, m, k, lits, 0, count);
}

/* ------------------------------------------------------------------ */
/* Compensated FP64 sums                                               */
/* ------------------------------------------------------------------ */

/* Neumaier's compensated summation of one term into (s, comp). */
static void neumaier_add(double *s, double *comp, double term) {
    double t = *s + term;
    if (fabs(*s) >= fabs(term)) *comp += (*s - t) + term;
    else *comp += (term - t) + *s;
    *s = t;
}

#define ORACLE_CHUNKS 256

/* Readout on state psi (interleaved re,im): success probability
 * <psi|{H_C = 0}|psi> (Definition of the success probability,
 * eq. psuccnae), expected cost F = <psi|H_C|psi> (Section 2.1) and the norm.
 * The index range is split into a fixed number of chunks, each summed with
 * Neumaier's method, and the chunk sums are combined the same way, so the
 * result does not depend on the thread count. */
static void readout(int n, const int32_t *cost, const double *psi, double out[3]) {
    int64_t N = (int64_t)1 << n;
    double part[ORACLE_CHUNKS][3];
    double comp[ORACLE_CHUNKS][3];
#pragma omp parallel for schedule(static)
    for (int ch = 0; ch < ORACLE_CHUNKS; ch++) {
        int64_t lo = N * ch / ORACLE_CHUNKS, hi = N * (ch + 1) / ORACLE_CHUNKS;
        double s[3] = {0, 0, 0}, c[3] = {0, 0, 0};
        for (int64_t x = lo; x < hi; x++) {
            double pr = psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
            if (cost[x] == 0) neumaier_add(&s[0], &c[0], pr);
            neumaier_add(&s[1], &c[1], (double)cost[x] * pr);
            neumaier_add(&s[2], &c[2], pr);
        }
        for (int q = 0; q < 3; q++) { part[ch][q] = s[q]; comp[ch][q] = c[q]; }
    }
    for (int q = 0; q < 3; q++) {
        double s = 0, c = 0;
        for (int ch = 0; ch < ORACLE_CHUNKS; ch++) {
            neumaier_add(&s, &c, part[ch][q]);
            neumaier_add(&s, &c, comp[ch][q]);
        }
        out[q] = s + c;
    }
}

/* ------------------------------------------------------------------ */
/* QAOA operators                                                      */
/* ------------------------------------------------------------------ */

/* |+>^{tensor n}: every amplitude 2^{-n/2} (Section 2.1). */
static void init_plus(int n, double *psi) {
    int64_t N = (int64_t)1 << n;
    double a = pow(2.0, -0.5 * n);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) { psi[2 * x] = a; psi[2 * x + 1] = 0.0; }
}

static int max_cost(int n, const int32_t *cost) {
    int64_t N = (int64_t)1 << n;
    int32_t cmax = 0;
    for (int64_t x = 0; x < N; x++) if (cost[x] > cmax) cmax = cost[x];
    return cmax;
}

/* Diagonal phase U_C(gamma) = sum_x exp(-i gamma C(x)) |x><x|
 * (Section 3.2; Appendix A.4, the diagonalised unitary). exp(-i g c) is
 * tabulated once per call for c = 0 .. max C with cos/sin, which is the same
 * value as evaluating it per x. */
static void apply_phase(int n, const int32_t *cost, int cmax, double gamma, double *psi) {
    int64_t N = (int64_t)1 << n;
    double *tab = (double *)malloc(sizeof(double) * 2 * (size_t)(cmax + 1));
    for (int c = 0; c <= cmax; c++) { tab[2 * c] = cos(gamma * c); tab[2 * c + 1] = -sin(gamma * c); }
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) {
        double er = tab[2 * cost[x]], ei = tab[2 * cost[x] + 1];
        double pr = psi[2 * x], pi = psi[2 * x + 1];
        psi[2 * x] = er * pr - ei * pi;
        psi[2 * x + 1] = er * pi + ei * pr;
    }
    free(tab);
}

/* Mixer U_B(beta) = prod_j exp(-i beta X_j) = prod_j [cos b I - i sin b X_j]
 * (Section 2.1 for the sign; Appendix A.4 for the product of n single-qubit
 * passes). X_j maps |x> to |x XOR 2^j>, so each pass updates the pairs
 * (x, x | 2^j) with bit j of x clear:
 *   a' = cos b * a - i sin b * b_,   b_' = cos b * b_ - i sin b * a. */
static void apply_mixer(int n, double beta, double *psi) {
    int64_t N = (int64_t)1 << n;
    double c = cos(beta), s = sin(beta);
    for (int j = 0; j < n; j++) {
        int64_t bit = (int64_t)1 << j;
#pragma omp parallel for schedule(static)
        for (int64_t idx = 0; idx < N / 2; idx++) {
            /* idx with a zero inserted at bit position j */
            int64_t x = ((idx >> j) << (j + 1)) | (idx & (bit - 1));
            int64_t y = x | bit;
            double ar = psi[2 * x], ai = psi[2 * x + 1];
            double br = psi[2 * y], bi = psi[2 * y + 1];
            /* -i s (br + i bi) = s bi - i s br */
            psi[2 * x] = c * ar + s * bi;
            psi[2 * x + 1] = c * ai - s * br;
            psi[2 * y] = c * br + s * ai;
            psi[2 * y + 1] = c * bi - s * ar;
        }
    }
}

/* Final QAOA state prod_{l} U_B(beta_l) U_C(gamma_l) |+> (Section 3.3), with
 * layer 0 applied first. psi must hold 2 * 2^n doubles. */
int oracle_state(int n, const int32_t *cost, int p, const double *gammas,
                 const double *betas, double *psi) {
    if (n < 1 || n > 40 || p < 0 || cost == NULL || psi == NULL) return -1;
    if (p > 0 && (gammas == NULL || betas == NULL)) return -1;
    int cmax = max_cost(n, cost);
    init_plus(n, psi);
    for (int l = 0; l < p; l++) {
        apply_phase(n, cost, cmax, gammas[l], psi);
        apply_mixer(n, betas[l], psi);
    }
    return 0;
}

/* p_succ, E[C] and norm of the depth-p QAOA state (out[0], out[1], out[2]).
 * psi_out, when not NULL, receives the final state (2 * 2^n doubles). */
int oracle_qaoa(int n, const int32_t *cost, int p, const double *gammas,
                const double *betas, double *psi_out, double out[3]) {
    if (out == NULL) return -1;
    int64_t N = (int64_t)1 << n;
    double *psi = psi_out ? psi_out : (double *)malloc(sizeof(double) * 2 * (size_t)N);
    if (psi == NULL) return -1;
    int rc = oracle_state(n, cost, p, gammas, betas, psi);
    if (rc == 0) readout(n, cost, psi, out);
    if (psi_out == NULL) free(psi);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Sampling bitstrings from the final state                           */
/* ------------------------------------------------------------------ */

/* Draws count bitstrings from |psi(x)|^2 / sum_y |psi(y)|^2 (the outcome
 * distribution of measuring the final state, Section 4.2, instance running
 * time) by inverting the cumulative distribution in index order: sample q
 * is the smallest x whose cumulative mass exceeds u[q] times the total.
 * The uniforms u[q] in [0, 1) are inputs. psi is interleaved (re, im). */
int oracle_sample(int n, const double *psi, const double *u, int64_t count, uint64_t *out) {
    if (n < 1 || n > 40 || psi == NULL || count < 0 || (count > 0 && (u == NULL || out == NULL))) return -1;
    int64_t N = (int64_t)1 << n;
    double *cum = (double *)malloc(sizeof(double) * (size_t)N);
    if (cum == NULL) return -1;
    double run = 0.0;
    for (int64_t x = 0; x < N; x++) {
        run += psi[2 * x] * psi[2 * x] + psi[2 * x + 1] * psi[2 * x + 1];
        cum[x] = run;
    }
    for (int64_t q = 0; q < count; q++) {
        if (!(u[q] >= 0.0 && u[q] < 1.0)) {
            free(cum);
            return -1;
        }
        double target = u[q] * run;
        int64_t lo = 0, hi = N - 1; /* smallest x with cum[x] > target */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (cum[mid] > target) hi = mid;
            else lo = mid + 1;
        }
        out[q] = (uint64_t)lo;
    }
    free(cum);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gradient by the adjoint method with stored states                  */
/* ------------------------------------------------------------------ */

/* Sum over x of conj(u(x)) v(x), compensated, as (re, im). */
static void inner(int64_t N, const double *u, const double *v, double *re, double *im) {
    double sr = 0, cr = 0, si = 0, ci = 0;
    for (int64_t x = 0; x < N; x++) {
        neumaier_add(&sr, &cr, u[2 * x] * v[2 * x] + u[2 * x + 1] * v[2 * x + 1]);
        neumaier_add(&si, &ci, u[2 * x] * v[2 * x + 1] - u[2 * x + 1] * v[2 * x]);
    }
    *re = sr + cr;
    *im = si + ci;
}

/* Gradient of F = w_psucc * p_succ + w_energy * E[C] with respect to every
 * gamma_l and beta_l. Written from d/dtheta <psi|W|psi> = 2 Re <psi|W d psi>:
 *   with psi_l the state after layer l, phi_l the state after the phase of
 *   layer l, and lambda_l = (U_{l+1} ... U_p)^dagger W psi_p,
 *   dF/dbeta_l  = 2 Im <lambda_l | H_B | psi_l>,          H_B = sum_j X_j,
 *   mu_l        = U_B(beta_l)^dagger lambda_l,
 *   dF/dgamma_l = 2 Im <mu_l | H_C | phi_l>,
 *   lambda_{l-1} = U_C(gamma_l)^dagger mu_l.
 * W = diag(w_psucc [C = 0] + w_energy C). Every forward state is stored
 * (2p states); nothing is uncomputed. out receives the forward readout. */
int oracle_qaoa_grad(int n, const int32_t *cost, int p, const double *gammas,
                     const double *betas, double w_psucc, double w_energy,
                     double *dgammas, double *dbetas, double out[3]) {
    if (n < 1 || n > 34 || p < 0 || cost == NULL || out == NULL) return -1;
    if (p > 0 && (gammas == NULL || betas == NULL || dgammas == NULL || dbetas == NULL)) return -1;
    int64_t N = (int64_t)1 << n;
    size_t bytes = sizeof(double) * 2 * (size_t)N;
    int cmax = max_cost(n, cost);
    /* states[2l] = phi_{l+1} (after the phase), states[2l+1] = psi_{l+1} */
    double **states = (double **)calloc((size_t)(2 * p + 1), sizeof(double *));
    double *lam = (double *)malloc(bytes);
    double *tmp = (double *)malloc(bytes);
    int ok = states && lam && tmp;
    for (int i = 0; ok && i < 2 * p; i++) ok = (states[i] = (double *)malloc(bytes)) != NULL;
    if (!ok) {
        if (states) for (int i = 0; i < 2 * p; i++) free(states[i]);
        free(states); free(lam); free(tmp);
        return -1;
    }
    /* forward, keeping every state */
    init_plus(n, tmp);
    for (int l = 0; l < p; l++) {
        const double *prev = l == 0 ? tmp : states[2 * l - 1];
        memcpy(states[2 * l], prev, bytes);
        apply_phase(n, cost, cmax, gammas[l], states[2 * l]);
        memcpy(states[2 * l + 1], states[2 * l], bytes);
        apply_mixer(n, betas[l], states[2 * l + 1]);
    }
    const double *final_state = p > 0 ? states[2 * p - 1] : tmp;
    readout(n, cost, final_state, out);
    /* lambda_p = W psi_p */
    for (int64_t x = 0; x < N; x++) {
        double w = w_energy * (double)cost[x] + (cost[x] == 0 ? w_psucc : 0.0);
        lam[2 * x] = w * final_state[2 * x];
        lam[2 * x + 1] = w * final_state[2 * x + 1];
    }
    for (int l = p - 1; l >= 0; l--) {
        const double *phi = states[2 * l], *psi = states[2 * l + 1];
        /* <lambda|H_B|psi> = sum_j sum_x conj(lambda(x)) psi(x XOR 2^j) */
        double hr = 0, hc = 0, hi = 0, hic = 0;
        for (int j = 0; j < n; j++) {
            int64_t bit = (int64_t)1 << j;
            for (int64_t x = 0; x < N; x++) {
                int64_t y = x ^ bit;
                tmp[2 * x] = psi[2 * y];
                tmp[2 * x + 1] = psi[2 * y + 1];
            }
            double re, im;
            inner(N, lam, tmp, &re, &im);
            neumaier_add(&hr, &hc, re);
            neumaier_add(&hi, &hic, im);
        }
        dbetas[l] = 2.0 * (hi + hic);
        /* mu = U_B(beta)^dagger lambda = U_B(-beta) lambda */
        apply_mixer(n, -betas[l], lam);
        /* <mu|H_C|phi> */
        for (int64_t x = 0; x < N; x++) {
            tmp[2 * x] = (double)cost[x] * phi[2 * x];
            tmp[2 * x + 1] = (double)cost[x] * phi[2 * x + 1];
        }
        double re, im;
        inner(N, lam, tmp, &re, &im);
        dgammas[l] = 2.0 * im;
        /* lambda_{l-1} = U_C(gamma)^dagger mu = U_C(-gamma) mu */
        apply_phase(n, cost, cmax, -gammas[l], lam);
        (void)hr;
    }
    for (int i = 0; i < 2 * p; i++) free(states[i]);
    free(states); free(lam); free(tmp);
    return 0;
}

/* Number of OpenMP threads the oracle runs with. */
int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing of the oracle itself); returns the
   number now in effect. */
int oracle_set_threads(int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
    return omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}
