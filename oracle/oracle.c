/*
 * FP64 CPU oracle for QAOA / approximate-quantum-annealing state-vector evolution.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP path is checked against.  Only tests, the smoke check
 * and the benchmark's CPU-baseline leg may load it; the product never does.
 * It shares no code, header, table or constant with the HIP library.
 *
 * Conventions (paper, Sec. II.A and Sec. III.A):
 *   - An n-qubit state is 2^n complex amplitudes psi[z], stored interleaved
 *     (re, im) as double[2 * 2^n].  Qubit q_0 is the rightmost tensor index,
 *     i.e. bit 0 of the basis index z (Sec. II.A, rank-N tensor notation).
 *   - The paper labels the -1 eigenstate of sigma^z as |0> (Sec. III.A.3, text
 *     after Eq. xtosigma), so the spin of qubit i in basis state z is
 *     s_i(z) = 2*b_i(z) - 1.
 *   - Cost Hamiltonian (Eq. HC): E(z) = sum_i h_i s_i + sum_{i<j} J_ij s_i s_j.
 *   - QAOA state (Eq. QAOA_state): |beta,gamma> = prod_{k=1..p}
 *       exp(-i beta_k H_D) exp(-i gamma_k H_C) |+>^n,  H_D = sum_i sigma^x_i.
 *   - exp(-i beta sigma^x) on one qubit is the 2x2 matrix
 *       [[cos b, -i sin b], [-i sin b, cos b]],
 *     applied to every pair of amplitudes differing in bit i as in
 *     Eq. twocomponentupdates.
 *
 * Every routine is written straight from those definitions: no blocking, no
 * fusion, no reordering of the factors.  Sums over 2^n terms use pairwise
 * (recursive halving) summation in FP64.  OpenMP only splits independent
 * loop iterations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define TWO_PI 6.283185307179586476925286766559

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* spin of qubit i in basis state z: s = 2 b - 1 (|0> is the -1 eigenstate) */
static double spin(uint64_t z, int i) { return ((z >> i) & 1u) ? 1.0 : -1.0; }

/* Eq. HC evaluated on one basis state. */
double orc_energy(int n, const double* h, int m, const int32_t* ei, const int32_t* ej,
                  const double* J, uint64_t z) {
    double e = 0.0;
    for (int i = 0; i < n; i++) e += h[i] * spin(z, i);
    for (int k = 0; k < m; k++) e += J[k] * spin(z, ei[k]) * spin(z, ej[k]);
    return e;
}

/* E(z) for every basis state. */
void orc_energies(int n, const double* h, int m, const int32_t* ei, const int32_t* ej,
                  const double* J, double* E) {
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) E[z] = orc_energy(n, h, m, ei, ej, J, (uint64_t)z);
}

/* Brute-force ground state: minimum energy, number of basis states within tol of
 * it, and the smallest such index (success probability definition, Sec. III.A.3). */
void orc_ground(int n, const double* E, double tol, double* emin, uint64_t* degeneracy,
                uint64_t* argmin) {
    const int64_t N = (int64_t)1 << n;
    double lo = E[0];
    for (int64_t z = 1; z < N; z++)
        if (E[z] < lo) lo = E[z];
    uint64_t cnt = 0, first = UINT64_MAX;
    for (int64_t z = 0; z < N; z++) {
        if (fabs(E[z] - lo) <= tol) {
            cnt++;
            if ((uint64_t)z < first) first = (uint64_t)z;
        }
    }
    *emin = lo;
    *degeneracy = cnt;
    *argmin = first;
}

/* |+>^n: every amplitude 2^{-n/2} (Sec. III.A.1, ground state of H_I). */
void orc_init_plus(int n, double* psi) {
    const int64_t N = (int64_t)1 << n;
    const double a = pow(2.0, -0.5 * n);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) {
        psi[2 * z] = a;
        psi[2 * z + 1] = 0.0;
    }
}

/* psi(z) <- exp(-i gamma E(z)) psi(z): the diagonal factor exp(-i gamma H_C).
 * The angle is reduced to [-pi, pi] with remainder() before cos/sin. */
void orc_cost_phase(int n, const double* E, double gamma, double* psi) {
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) {
        double th = remainder(gamma * E[z], TWO_PI);
        double c = cos(th), s = sin(th);
        double re = psi[2 * z], im = psi[2 * z + 1];
        /* (re + i im)(c - i s) */
        psi[2 * z] = re * c + im * s;
        psi[2 * z + 1] = im * c - re * s;
    }
}

/* exp(-i beta sigma^x_q) on qubit q: Eq. twocomponentupdates with
 * u = [[c, -i s], [-i s, c]]. */
void orc_rx(int n, int q, double beta, double* psi) {
    const int64_t N = (int64_t)1 << n;
    const int64_t bit = (int64_t)1 << q;
    const double c = cos(beta), s = sin(beta);
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) {
        if (z & bit) continue;
        int64_t w = z | bit;
        double ar = psi[2 * z], ai = psi[2 * z + 1];
        double br = psi[2 * w], bi = psi[2 * w + 1];
        /* a' = c a - i s b ;  b' = -i s a + c b */
        psi[2 * z] = c * ar + s * bi;
        psi[2 * z + 1] = c * ai - s * br;
        psi[2 * w] = c * br + s * ai;
        psi[2 * w + 1] = c * bi - s * ar;
    }
}

/* A general 2x2 complex matrix U on qubit q (row-major, interleaved re/im:
 * u00, u01, u10, u11), Eq. twocomponentupdates with an arbitrary u:
 * a' = u00 a + u01 b, b' = u10 a + u11 b for every pair (a, b) = (psi[z], psi[z | 2^q]). */
void orc_gate_1q(int n, int q, const double* U, double* psi) {
    const int64_t N = (int64_t)1 << n;
    const int64_t bit = (int64_t)1 << q;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) {
        if (z & bit) continue;
        int64_t w = z | bit;
        double ar = psi[2 * z], ai = psi[2 * z + 1];
        double br = psi[2 * w], bi = psi[2 * w + 1];
        psi[2 * z] = U[0] * ar - U[1] * ai + U[2] * br - U[3] * bi;
        psi[2 * z + 1] = U[0] * ai + U[1] * ar + U[2] * bi + U[3] * br;
        psi[2 * w] = U[4] * ar - U[5] * ai + U[6] * br - U[7] * bi;
        psi[2 * w + 1] = U[4] * ai + U[5] * ar + U[6] * bi + U[7] * br;
    }
}

/* exp(-i beta H_D) = prod_q exp(-i beta sigma^x_q), qubits 0..n-1 in order. */
void orc_mixer(int n, double beta, double* psi) {
    for (int q = 0; q < n; q++) orc_rx(n, q, beta, psi);
}

/* Eq. QAOA_state: starting from psi as given (pass from_plus=1 to start from |+>^n),
 * for k = 1..p apply exp(-i gamma_k H_C) then exp(-i beta_k H_D). */
void orc_qaoa(int n, const double* E, int p, const double* gamma, const double* beta,
              int from_plus, double* psi) {
    if (from_plus) orc_init_plus(n, psi);
    for (int k = 0; k < p; k++) {
        orc_cost_phase(n, E, gamma[k], psi);
        orc_mixer(n, beta[k], psi);
    }
}

/* pairwise sum of f(z) for z in [lo, hi) */
typedef double (*term_fn)(int64_t z, const void* ctx);

static double pairwise(int64_t lo, int64_t hi, term_fn f, const void* ctx) {
    if (hi - lo <= 64) {
        double s = 0.0;
        for (int64_t z = lo; z < hi; z++) s += f(z, ctx);
        return s;
    }
    int64_t mid = lo + (hi - lo) / 2;
    return pairwise(lo, mid, f, ctx) + pairwise(mid, hi, f, ctx);
}

/* Run the pairwise sum over 2^n terms with the top-level halves spread over threads. */
static double big_sum(int n, term_fn f, const void* ctx) {
    const int64_t N = (int64_t)1 << n;
    if (n <= 12) return pairwise(0, N, f, ctx);
    const int nb = 64; /* 64 equal blocks, each summed pairwise, combined pairwise */
    double part[64];
    const int64_t B = N / nb;
#pragma omp parallel for schedule(static)
    for (int b = 0; b < nb; b++) part[b] = pairwise(b * B, (b + 1) * B, f, ctx);
    /* combine 64 partials pairwise */
    for (int w = 1; w < nb; w *= 2)
        for (int b = 0; b + w < nb; b += 2 * w) part[b] += part[b + w];
    return part[0];
}

typedef struct {
    const double* psi;
    const double* E;
    double emin, tol;
    const double* lam;
} obs_ctx;

static double t_norm(int64_t z, const void* c) {
    const obs_ctx* o = (const obs_ctx*)c;
    return o->psi[2 * z] * o->psi[2 * z] + o->psi[2 * z + 1] * o->psi[2 * z + 1];
}
static double t_energy(int64_t z, const void* c) {
    const obs_ctx* o = (const obs_ctx*)c;
    return o->E[z] * (o->psi[2 * z] * o->psi[2 * z] + o->psi[2 * z + 1] * o->psi[2 * z + 1]);
}
static double t_pgs(int64_t z, const void* c) {
    const obs_ctx* o = (const obs_ctx*)c;
    if (fabs(o->E[z] - o->emin) > o->tol) return 0.0;
    return o->psi[2 * z] * o->psi[2 * z] + o->psi[2 * z + 1] * o->psi[2 * z + 1];
}

/* norm = sum |psi|^2 ; energy = <psi|H_C|psi> = sum E |psi|^2 (Sec. III.B.1);
 * pgs = probability of the ground-state set {z : |E(z) - emin| <= tol}. */
void orc_observables(int n, const double* E, const double* psi, double emin, double tol,
                     double* norm, double* energy, double* pgs) {
    obs_ctx o = {psi, E, emin, tol, NULL};
    *norm = big_sum(n, t_norm, &o);
    *energy = big_sum(n, t_energy, &o);
    *pgs = big_sum(n, t_pgs, &o);
}

/* <sigma^z_i> = sum_z s_i(z) |psi(z)|^2 for every qubit i. */
void orc_spin_z(int n, const double* psi, double* out) {
    const int64_t N = (int64_t)1 << n;
    for (int i = 0; i < n; i++) {
        double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
        for (int64_t z = 0; z < N; z++)
            acc += spin((uint64_t)z, i) * (psi[2 * z] * psi[2 * z] + psi[2 * z + 1] * psi[2 * z + 1]);
        out[i] = acc;
    }
}

/* ------------------------------------------------------------------------------
 * Gradient of f(gamma, beta) = <beta,gamma| H_C |beta,gamma> by forward-mode
 * tangents: alongside psi carry T_j = d psi / d theta_j for all 2p parameters.
 *   d/dgamma_k exp(-i gamma_k H_C) = -i H_C exp(-i gamma_k H_C)
 *   d/dbeta_k  exp(-i beta_k  H_D) = -i H_D exp(-i beta_k  H_D)
 * Every factor is applied to psi and to every tangent; right after factor k is
 * applied, its own tangent is set to (-i G) psi.  Then
 *   df/dtheta_j = 2 Re <psi| H_C |T_j>.
 * Memory: (2p+1) state vectors.  Returns f in *energy.
 * ---------------------------------------------------------------------------- */
static void apply_minus_i_HD(int n, const double* in, double* out) {
    /* out = -i sum_q sigma^x_q in */
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) {
        double sr = 0.0, si = 0.0;
        for (int q = 0; q < n; q++) {
            int64_t w = z ^ ((int64_t)1 << q);
            sr += in[2 * w];
            si += in[2 * w + 1];
        }
        /* -i (sr + i si) = si - i sr */
        out[2 * z] = si;
        out[2 * z + 1] = -sr;
    }
}

static void apply_minus_i_HC(int n, const double* E, const double* in, double* out) {
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < N; z++) {
        out[2 * z] = E[z] * in[2 * z + 1];
        out[2 * z + 1] = -E[z] * in[2 * z];
    }
}

typedef struct {
    const double* psi;
    const double* T;
    const double* E;
} grad_ctx;

static double t_grad(int64_t z, const void* c) {
    const grad_ctx* g = (const grad_ctx*)c;
    /* Re( conj(psi) * E * T ) */
    return g->E[z] * (g->psi[2 * z] * g->T[2 * z] + g->psi[2 * z + 1] * g->T[2 * z + 1]);
}

int orc_grad_tangent(int n, const double* E, int p, const double* gamma, const double* beta,
                     double* energy, double* dgamma, double* dbeta) {
    const int64_t N = (int64_t)1 << n;
    const int nt = 2 * p; /* tangent j: j = 2k -> gamma_k, j = 2k+1 -> beta_k */
    double* psi = (double*)malloc(sizeof(double) * 2 * N);
    double* T = (double*)calloc((size_t)nt * 2 * N, sizeof(double));
    if (!psi || !T) {
        free(psi);
        free(T);
        return 1;
    }
    orc_init_plus(n, psi);
    for (int k = 0; k < p; k++) {
        orc_cost_phase(n, E, gamma[k], psi);
        for (int j = 0; j < 2 * k; j++) orc_cost_phase(n, E, gamma[k], T + (size_t)j * 2 * N);
        apply_minus_i_HC(n, E, psi, T + (size_t)(2 * k) * 2 * N);
        orc_mixer(n, beta[k], psi);
        for (int j = 0; j < 2 * k + 1; j++) orc_mixer(n, beta[k], T + (size_t)j * 2 * N);
        apply_minus_i_HD(n, psi, T + (size_t)(2 * k + 1) * 2 * N);
    }
    obs_ctx o = {psi, E, 0.0, 0.0, NULL};
    *energy = big_sum(n, t_energy, &o);
    for (int k = 0; k < p; k++) {
        grad_ctx g0 = {psi, T + (size_t)(2 * k) * 2 * N, E};
        grad_ctx g1 = {psi, T + (size_t)(2 * k + 1) * 2 * N, E};
        dgamma[k] = 2.0 * big_sum(n, t_grad, &g0);
        dbeta[k] = 2.0 * big_sum(n, t_grad, &g1);
    }
    free(psi);
    free(T);
    return 0;
}
