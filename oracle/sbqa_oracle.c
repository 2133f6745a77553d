/*
 * FP64 CPU oracle for Simulated Bifurcation Quantum Annealing (SBQA).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, obviously correct
 * statement of what the SBQA time-stepping loop computes. It is used by the
 * tests, by the package's smoke check and by the benchmark's CPU baseline,
 * and never by the library's product path. It shares no code, header, table
 * or helper with the GPU library.
 *
 * Source: arXiv 2604.01050, Sec. II.A (Eqs. 1-8), Sec. II.B (auto-tuning),
 * Supplement S1 (Eq. S12, periodic Trotter ring).
 *
 * Conventions (readings where the paper is silent):
 *  - State X, Y are N x C row-major, C = runs*R, column c = r*R + k holds
 *    replica k of run r.
 *  - Step n (n = 0..S-1) integrates t_n = n*dt -> t_{n+1}; T = S*dt, so the
 *    pump is a_n = a(t_n) = n/S and the threshold Delta_n = 0.7*n/S.
 *  - Integrator: symplectic Euler, momentum kick with the step-n positions
 *    (all replicas at once), then position drift with the new momentum, then
 *    the wall of Eq. 3: |x| > 1 -> x = sign(x), y = 0.
 *  - Where floating point decides a discrete outcome (the threshold of Eq. 8
 *    and the wall), the decision is taken in binary32, the precision of the
 *    GPU state, on the binary32-rounded value.
 *  - Energy: E(s) = -1/2 s^T J s - h^T s (the SBM potential of Eq. 2 at the
 *    hypercube corners), readout s_i = sign(x_i) with sign(0) = +1.
 *  - Three-body terms (the HUBO Hamiltonian of Eq. 11, Sec. III.B, native rather than
 *    reduced to QUBO form): a list of triples (l, m, n) of distinct spins with
 *    weights K, each triple once, adds -K s_l s_m s_n to the energy (the sign
 *    convention of the two-body part: pass -J, -K for the paper's
 *    H = sum J s s + sum K s s s). Its coupling sum is minus the derivative of
 *    that energy with the other two spins replaced by f: spin l receives
 *    K f_m f_n, and likewise m and n.
 *
 * Parity pins: every function here is pinned by tests against closed forms,
 * brute force, Hamilton's equations for Eq. 4 and special cases (Eq. 3).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------------------------------------------------------------------
 * Schedules (Sec. II.A below Eq. 2; Eq. 5; Eq. 8)
 * ------------------------------------------------------------------------- */

/* Pump a(t) = t/T at t = n*dt, T = S*dt. */
double orc_pump(int64_t n, int64_t S) { return (double)n / (double)S; }

/* Threshold Delta(t) = delta_max * t/T of Eq. 8, rounded to binary32.
 * Evaluated as (delta_max * n) / S in float64, then rounded once. */
float orc_delta32(double delta_max, int64_t n, int64_t S) {
    return (float)((delta_max * (double)n) / (double)S);
}

/* Transverse field of Eq. 5: Gamma_x(t) = Gamma_x(0) [ (1 - t/T)^alpha + 1e-5 ]. */
double orc_gamma_x(double gamma0, double alpha, double s) {
    return gamma0 * (pow(1.0 - s, alpha) + 1e-5);
}

/* Inter-replica coupling of Eq. 5 / Eq. S12: J_perp = -(1/(2 beta)) ln tanh(beta Gamma_x / R).
 * Takes Gamma_x/R directly: only that ratio enters. */
double orc_jperp(double beta, double gamma_x_over_R) {
    return -log(tanh(beta * gamma_x_over_R)) / (2.0 * beta);
}

/* J_perp at the start of every step n = 0..S-1 for one run (beta, alpha):
 * s = n/S, Gamma_x(0)/R given. */
void orc_jperp_paper_table(double beta, double alpha, double gamma0_over_R,
                           int64_t S, double *out) {
    for (int64_t n = 0; n < S; ++n)
        out[n] = orc_jperp(beta, orc_gamma_x(gamma0_over_R, alpha, orc_pump(n, S)));
}

/* Linear J_perp reading: J_perp(t) = start + (end - start) t/T. */
void orc_jperp_linear_table(double start, double end, int64_t S, double *out) {
    for (int64_t n = 0; n < S; ++n)
        out[n] = start + (end - start) * orc_pump(n, S);
}

/* ---------------------------------------------------------------------------
 * Energy (Eq. 2 at the hypercube corners; Ising problem statement)
 * ------------------------------------------------------------------------- */

/* E(s) = -1/2 sum_ij J_ij s_i s_j - sum_i h_i s_i for count configurations
 * s (count x N, int8 +-1). J dense row-major N x N. h may be NULL (zero). */
void orc_energy_dense(int32_t N, const double *J, const double *h,
                      const int8_t *s, int32_t count, double *E) {
    #pragma omp parallel for schedule(static)
    for (int32_t m = 0; m < count; ++m) {
        const int8_t *sm = s + (int64_t)m * N;
        double quad = 0.0, lin = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            double phi = 0.0;
            for (int32_t j = 0; j < N; ++j) phi += J[(int64_t)i * N + j] * (double)sm[j];
            quad += (double)sm[i] * phi;
            if (h) lin += h[i] * (double)sm[i];
        }
        E[m] = -0.5 * quad - lin;
    }
}

void orc_energy_csr(int32_t N, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const double *h, const int8_t *s,
                    int32_t count, double *E) {
    #pragma omp parallel for schedule(static)
    for (int32_t m = 0; m < count; ++m) {
        const int8_t *sm = s + (int64_t)m * N;
        double quad = 0.0, lin = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            double phi = 0.0;
            for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) phi += val[p] * (double)sm[col[p]];
            quad += (double)sm[i] * phi;
            if (h) lin += h[i] * (double)sm[i];
        }
        E[m] = -0.5 * quad - lin;
    }
}

/* Three-body part of the energy, -sum_t K_t s_l s_m s_n, for count
 * configurations (count x N, int8 +-1); tri is n3 x 3 (each triple once). */
void orc_energy3(int32_t N, int64_t n3, const int32_t *tri, const double *K,
                 const int8_t *s, int32_t count, double *E) {
    #pragma omp parallel for schedule(static)
    for (int32_t m = 0; m < count; ++m) {
        const int8_t *sm = s + (int64_t)m * N;
        double cub = 0.0;
        for (int64_t t = 0; t < n3; ++t)
            cub += K[t] * (double)sm[tri[3 * t]] * (double)sm[tri[3 * t + 1]] * (double)sm[tri[3 * t + 2]];
        E[m] = -cub;
    }
}

/* Exhaustive minimum of the full energy (two-body dense J, h, three-body
 * triples) for N <= 24 by direct evaluation of every configuration, in
 * binary counting order (bit i of the counter set = spin i is -1; ties keep
 * the first minimum met). */
double orc_bruteforce_hubo(int32_t N, const double *J, const double *h, int64_t n3,
                           const int32_t *tri, const double *K, int8_t *best) {
    if (N < 1 || N > 24) return NAN;
    int8_t *s = (int8_t *)malloc((size_t)N);
    double Emin = INFINITY;
    for (uint64_t g = 0; g < (1ull << N); ++g) {
        for (int32_t i = 0; i < N; ++i) s[i] = ((g >> i) & 1u) ? -1 : 1;
        double E = 0.0;
        for (int32_t i = 0; i < N; ++i) {
            for (int32_t j = 0; j < N; ++j) E += -0.5 * J[(int64_t)i * N + j] * s[i] * s[j];
            if (h) E -= h[i] * s[i];
        }
        for (int64_t t = 0; t < n3; ++t) E -= K[t] * s[tri[3 * t]] * s[tri[3 * t + 1]] * s[tri[3 * t + 2]];
        if (E < Emin) { Emin = E; memcpy(best, s, (size_t)N); }
    }
    free(s);
    return Emin;
}

/* Exhaustive ground state for N <= 30 (Gray-code order; ties keep the first
 * minimum met). Returns the minimum energy and writes one minimiser. */
double orc_bruteforce_dense(int32_t N, const double *J, const double *h, int8_t *best) {
    if (N < 1 || N > 30) return NAN;
    int8_t *s = (int8_t *)malloc((size_t)N);
    double *phi = (double *)malloc(sizeof(double) * (size_t)N);
    for (int32_t i = 0; i < N; ++i) s[i] = -1;
    /* phi_i = sum_j J_ij s_j */
    for (int32_t i = 0; i < N; ++i) {
        phi[i] = 0.0;
        for (int32_t j = 0; j < N; ++j) phi[i] += J[(int64_t)i * N + j] * s[j];
    }
    double E = 0.0;
    for (int32_t i = 0; i < N; ++i) E += -0.5 * s[i] * phi[i] - (h ? h[i] * s[i] : 0.0);
    double Emin = E;
    memcpy(best, s, (size_t)N);
    uint64_t total = 1ull << N;
    for (uint64_t g = 1; g < total; ++g) {
        int32_t i = __builtin_ctzll(g);           /* Gray code: flip bit i */
        /* flipping s_i changes E by 2 s_i (phi_i + h_i) */
        E += 2.0 * s[i] * (phi[i] + (h ? h[i] : 0.0));
        s[i] = (int8_t)-s[i];
        for (int32_t j = 0; j < N; ++j) phi[j] += 2.0 * J[(int64_t)j * N + i] * s[i];
        if (E < Emin) { Emin = E; memcpy(best, s, (size_t)N); }
    }
    free(s);
    free(phi);
    return Emin;
}

/* ---------------------------------------------------------------------------
 * Nonlinearity f (Eq. 8; bSB f(x)=x and dSB f(x)=sign(x) of Sec. II.A)
 * ------------------------------------------------------------------------- */

enum { ORC_F_TERNARY = 0, ORC_F_SIGN = 1, ORC_F_BALLISTIC = 2 };

static double f_of(int32_t fmode, double x, float delta) {
    if (fmode == ORC_F_BALLISTIC) return x;
    float xf = (float)x;                     /* decision in binary32 */
    float d = (fmode == ORC_F_SIGN) ? 0.0f : delta;
    if (fabsf(xf) <= d) return 0.0;          /* sign mode: only x == 0 gives 0 */
    return xf > 0.0f ? 1.0 : -1.0;
}

void orc_apply_f(int32_t fmode, float delta, int64_t count, const double *x, double *g) {
    for (int64_t e = 0; e < count; ++e) g[e] = f_of(fmode, x[e], delta);
}

/* ---------------------------------------------------------------------------
 * Fields Phi = J . G (the coupling sum of Eq. 7), G = f(X), N x C row-major.
 * Summation over j ascending (dense) or in CSR order (sparse).
 * ------------------------------------------------------------------------- */

void orc_fields_dense(int32_t N, int32_t C, const double *J, const double *G, double *Phi) {
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
        double *out = Phi + (int64_t)i * C;
        for (int32_t c = 0; c < C; ++c) out[c] = 0.0;
        for (int32_t j = 0; j < N; ++j) {
            double w = J[(int64_t)i * N + j];
            const double *g = G + (int64_t)j * C;
            for (int32_t c = 0; c < C; ++c) out[c] += w * g[c];
        }
    }
}

void orc_fields_csr(int32_t N, int32_t C, const int32_t *row_ptr, const int32_t *col,
                    const double *val, const double *G, double *Phi) {
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i) {
        double *out = Phi + (int64_t)i * C;
        for (int32_t c = 0; c < C; ++c) out[c] = 0.0;
        for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            double w = val[p];
            const double *g = G + (int64_t)col[p] * C;
            for (int32_t c = 0; c < C; ++c) out[c] += w * g[c];
        }
    }
}

/* ---------------------------------------------------------------------------
 * One SBQA step (Eqs. 6-7 with the wall of Eq. 3), all runs and replicas.
 * ------------------------------------------------------------------------- */

typedef struct {
    int32_t N, R, runs;
    const double *dense;                       /* N*N row-major, or NULL */
    const int32_t *row_ptr, *col;              /* CSR when dense == NULL */
    const double *val;
    const double *h;                           /* N, or NULL */
    double dt, a0, c0;
    int32_t fmode;
    int64_t n3;                                /* three-body triples (may be 0) */
    const int32_t *tri;                        /* n3 x 3 spin indices */
    const double *K;                           /* n3 weights */
} orc_problem;

/* Coupling sum of row i for all C columns: phi[c] = sum_j J_ij G[j][c]. */
static void field_row(const orc_problem *P, int32_t i, const double *G, double *phi) {
    const int32_t N = P->N, C = P->R * P->runs;
    for (int32_t c = 0; c < C; ++c) phi[c] = 0.0;
    if (P->dense) {
        for (int32_t j = 0; j < N; ++j) {
            const double w = P->dense[(int64_t)i * N + j];
            const double *g = G + (int64_t)j * C;
            for (int32_t c = 0; c < C; ++c) phi[c] += w * g[c];
        }
    } else {
        for (int32_t p = P->row_ptr[i]; p < P->row_ptr[i + 1]; ++p) {
            const double w = P->val[p];
            const double *g = G + (int64_t)P->col[p] * C;
            for (int32_t c = 0; c < C; ++c) phi[c] += w * g[c];
        }
    }
}

/* Three-body coupling sums added to Phi (N x C): for every triple t in list
 * order, spin l gains K_t G[m] G[n], spin m gains K_t G[l] G[n] and spin n
 * gains K_t G[l] G[m]. */
void orc_fields3(int32_t N, int32_t C, int64_t n3, const int32_t *tri, const double *K,
                 const double *G, double *Phi) {
    (void)N;
    for (int64_t t = 0; t < n3; ++t) {
        const int32_t v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int e = 0; e < 3; ++e) {
            const double *ga = G + (int64_t)v[(e + 1) % 3] * C, *gb = G + (int64_t)v[(e + 2) % 3] * C;
            double *out = Phi + (int64_t)v[e] * C;
            for (int32_t c = 0; c < C; ++c) out[c] += K[t] * (ga[c] * gb[c]);
        }
    }
}

/* The three-body part of the coupling sum of one row i (list order). */
static void field3_row(const orc_problem *P, int32_t i, const double *G, double *phi) {
    const int32_t C = P->R * P->runs;
    for (int64_t t = 0; t < P->n3; ++t) {
        const int32_t *v = P->tri + 3 * t;
        for (int e = 0; e < 3; ++e) {
            if (v[e] != i) continue;
            const double *ga = G + (int64_t)v[(e + 1) % 3] * C, *gb = G + (int64_t)v[(e + 2) % 3] * C;
            for (int32_t c = 0; c < C; ++c) phi[c] += P->K[t] * (ga[c] * gb[c]);
        }
    }
}

/*
 * Update of row i (all columns) from the step-n positions X0 (Eqs. 6-7 + wall):
 *   ring = X0[i, r*R + (k-1 mod R)] + X0[i, r*R + (k+1 mod R)]   (periodic ring, S1)
 *   y'   = y + dt * ( -((a0 - a_n)/R) x + (c0/R)(phi + h_i) + J_perp[r] ring )
 *   x'   = x + dt * (a0/R) y'
 *   |x'| > 1  ->  x' = sign(x'), y' = 0                         (wall, Sec. II.A)
 */
static void update_row(const orc_problem *P, int32_t i, const double *X0, const double *Yin,
                       const double *phi, double a_n, const double *jperp_r, double *xo, double *yo) {
    const int32_t R = P->R, C = P->R * P->runs;
    const double Rd = (double)R;
    const double hi = P->h ? P->h[i] : 0.0;
    const double *xrow = X0 + (int64_t)i * C;
    for (int32_t c = 0; c < C; ++c) {
        const int32_t r = c / R, k = c % R;
        const double x = xrow[c];
        const double xl = xrow[r * R + (k + R - 1) % R];
        const double xr = xrow[r * R + (k + 1) % R];
        const double force = -((P->a0 - a_n) / Rd) * x
                             + (P->c0 / Rd) * (phi[c] + hi)
                             + jperp_r[r] * (xl + xr);
        double y = Yin[(int64_t)i * C + c] + P->dt * force;
        double xn = x + P->dt * (P->a0 / Rd) * y;
        float xf = (float)xn;                       /* wall decision in binary32 */
        if (fabsf(xf) > 1.0f) {
            xn = xn > 0.0 ? 1.0 : -1.0;
            y = 0.0;
        }
        xo[c] = xn;
        yo[c] = y;
    }
}

/*
 * Advance (X, Y) by one step, all runs and replicas (Jacobi: every term uses
 * the step-n positions): G = f(X) with threshold delta_n (Eq. 8), phi = J G,
 * then update_row for every row.
 * scratch: 3*N*C doubles (G, Phi, old X). Phi_out (optional) receives Phi.
 */
void orc_step(const orc_problem *P, double *X, double *Y, double a_n, float delta_n,
              const double *jperp_r, double *scratch, double *Phi_out) {
    const int32_t N = P->N, C = P->R * P->runs;
    const int64_t NC = (int64_t)N * C;
    double *G = scratch, *Phi = scratch + NC, *X0 = scratch + 2 * NC;
    memcpy(X0, X, sizeof(double) * (size_t)NC);
    orc_apply_f(P->fmode, delta_n, NC, X0, G);
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i) field_row(P, i, G, Phi + (int64_t)i * C);
    if (P->n3) orc_fields3(N, C, P->n3, P->tri, P->K, G, Phi);
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < N; ++i)
        update_row(P, i, X0, Y, Phi + (int64_t)i * C, a_n, jperp_r,
                   X + (int64_t)i * C, Y + (int64_t)i * C);
    if (Phi_out) memcpy(Phi_out, Phi, sizeof(double) * (size_t)NC);
}

/*
 * The same step for a sample of rows only (for checks at sizes where a full
 * step is too slow): X, Y unchanged; rows[nrows]; outputs Xo, Yo, Phio are
 * nrows x C. scratch: N*C doubles (G).
 */
void orc_step_rows(const orc_problem *P, const double *X, const double *Y, double a_n,
                   float delta_n, const double *jperp_r, int32_t nrows, const int32_t *rows,
                   double *scratch, double *Xo, double *Yo, double *Phio) {
    const int32_t N = P->N, C = P->R * P->runs;
    double *G = scratch;
    orc_apply_f(P->fmode, delta_n, (int64_t)N * C, X, G);
    #pragma omp parallel for schedule(static)
    for (int32_t q = 0; q < nrows; ++q) {
        field_row(P, rows[q], G, Phio + (int64_t)q * C);
        if (P->n3) field3_row(P, rows[q], G, Phio + (int64_t)q * C);
        update_row(P, rows[q], X, Y, Phio + (int64_t)q * C, a_n, jperp_r,
                   Xo + (int64_t)q * C, Yo + (int64_t)q * C);
    }
}

/* Readout energies of sign(X) for all C columns (sign(0) = +1). */
static void readout_energies(const orc_problem *P, const double *X, int8_t *S, double *E) {
    const int32_t N = P->N, C = P->R * P->runs;
    for (int32_t c = 0; c < C; ++c)
        for (int32_t i = 0; i < N; ++i)
            S[(int64_t)c * N + i] = X[(int64_t)i * C + c] >= 0.0 ? 1 : -1;
    if (P->dense) orc_energy_dense(N, P->dense, P->h, S, C, E);
    else orc_energy_csr(N, P->row_ptr, P->col, P->val, P->h, S, C, E);
    if (P->n3) {
        double *E3 = (double *)malloc(sizeof(double) * (size_t)C);
        orc_energy3(N, P->n3, P->tri, P->K, S, C, E3);
        for (int32_t c = 0; c < C; ++c) E[c] += E3[c];
        free(E3);
    }
}

/*
 * Full SBQA trajectory of S steps from (X, Y), then the best solution per run
 * (Sec. II.B: evolve every repetition, return the best over its replicas).
 *   jperp:    runs x S table, J_perp of run r at step n.
 *   delta_max: threshold factor of Eq. 8 (0.7 in the paper).
 *   energy_every: 0 = final state only; K > 0 also evaluates after every K-th
 *                 step. Ties: lowest replica k within an evaluation, earliest
 *                 evaluation across evaluations.
 *   best_E [runs], best_s [runs x N] (int8 +-1), best_step [runs] (may be NULL).
 */
int32_t orc_run(const orc_problem *P, double *X, double *Y, int64_t S, const double *jperp,
                double delta_max, int64_t energy_every, double *best_E, int8_t *best_s,
                int64_t *best_step) {
    const int32_t N = P->N, R = P->R, runs = P->runs, C = R * runs;
    const int64_t NC = (int64_t)N * C;
    double *scratch = (double *)malloc(sizeof(double) * 3 * (size_t)NC);
    double *jr = (double *)malloc(sizeof(double) * (size_t)runs);
    int8_t *Sg = (int8_t *)malloc((size_t)NC);
    double *E = (double *)malloc(sizeof(double) * (size_t)C);
    if (!scratch || !jr || !Sg || !E) return -2;
    for (int32_t r = 0; r < runs; ++r) best_E[r] = INFINITY;

    for (int64_t n = 0; n <= S; ++n) {
        int evaluate = (n == S) || (energy_every > 0 && n > 0 && n % energy_every == 0);
        if (evaluate) {
            readout_energies(P, X, Sg, E);
            for (int32_t r = 0; r < runs; ++r)
                for (int32_t k = 0; k < R; ++k) {
                    int32_t c = r * R + k;
                    if (E[c] < best_E[r]) {
                        best_E[r] = E[c];
                        memcpy(best_s + (int64_t)r * N, Sg + (int64_t)c * N, (size_t)N);
                        if (best_step) best_step[r] = n;
                    }
                }
        }
        if (n == S) break;
        for (int32_t r = 0; r < runs; ++r) jr[r] = jperp[(int64_t)r * S + n];
        orc_step(P, X, Y, orc_pump(n, S), orc_delta32(delta_max, n, S), jr, scratch, NULL);
    }
    free(scratch);
    free(jr);
    free(Sg);
    free(E);
    return 0;
}

/*
 * c0 = 0.5 / (sqrt(N) * std(J)) with std(J) read as the root mean square of
 * the N(N-1) off-diagonal entries (zeros included). Returns 0 for J == 0.
 */
double orc_auto_c0_dense(int32_t N, const double *J) {
    double ss = 0.0;
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < N; ++j)
            if (i != j) ss += J[i * N + j] * J[i * N + j];
    if (ss == 0.0 || N < 2) return 0.0;
    return 0.5 / (sqrt((double)N) * sqrt(ss / ((double)N * (double)(N - 1))));
}

double orc_auto_c0_csr(int32_t N, const int32_t *row_ptr, const int32_t *col, const double *val) {
    double ss = 0.0;
    for (int32_t i = 0; i < N; ++i)
        for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            if (col[p] != i) ss += val[p] * val[p];
    if (ss == 0.0 || N < 2) return 0.0;
    return 0.5 / (sqrt((double)N) * sqrt(ss / ((double)N * (double)(N - 1))));
}

/*
 * c0 with three-body terms: 0.5 / sqrt(mean_i Var(Phi_i) * N/(N-1)) where, for
 * independent uniform random spins, Var(Phi_i) = sum_j J_ij^2 + sum_{t ni i}
 * K_t^2; without triples this is the two-body rule above. Two-body part from
 * CSR (diagonal excluded); the triples count once per member spin.
 */
double orc_auto_c0_hubo(int32_t N, const int32_t *row_ptr, const int32_t *col, const double *val,
                        int64_t n3, const double *K) {
    double ss = 0.0;
    for (int32_t i = 0; i < N; ++i)
        for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
            if (col[p] != i) ss += val[p] * val[p];
    for (int64_t t = 0; t < n3; ++t) ss += 3.0 * K[t] * K[t];
    if (ss == 0.0 || N < 2) return 0.0;
    return 0.5 / sqrt(ss / (double)(N - 1));
}
