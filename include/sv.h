/*
 * sv.h -- C ABI of libsv.so: full state-vector evolution of n-qubit Ising
 * problems under QAOA layers and approximate-quantum-annealing (AQA) steps on
 * one AMD MI355X (gfx950).
 *
 * Method (Willsch et al., "GPU-accelerated simulations of quantum annealing and
 * the quantum approximate optimization algorithm", arXiv:2104.03293):
 *   - state: 2^n complex amplitudes psi[z], qubit q_0 = bit 0 of z (Sec. II.A);
 *   - spin of qubit i in basis state z: s_i = 2 b_i(z) - 1, because the paper
 *     names the -1 eigenstate of sigma^z |0> (Sec. III.A.3);
 *   - cost Hamiltonian H_C = sum_i h_i s_i + sum_{i<j} J_ij s_i s_j (Eq. HC);
 *   - mixer H_D = sum_i sigma^x_i (Sec. III.A.2);
 *   - QAOA state prod_{k=1..p} exp(-i beta_k H_D) exp(-i gamma_k H_C) |+>^n
 *     (Eq. QAOA_state); exp(-i beta sigma^x) acts on amplitude pairs as in
 *     Eq. twocomponentupdates; exp(-i gamma H_C) is diagonal.
 *
 * Conventions of this ABI
 *   - Amplitudes are interleaved (re, im): SV_C128 = 2 x double (16 B),
 *     SV_C64 = 2 x float (8 B).  Phase angles, energies and every reduction
 *     are computed in FP64 for both storage types.
 *   - Device pointers are HIP device pointers on the current device; streams
 *     are hipStream_t passed as void* (NULL = the null stream).
 *   - Every call returns an int status (sv_status).  On failure
 *     sv_last_error() returns a thread-local message.  Argument errors leave
 *     every object unchanged.  After a HIP error a state is marked failed and
 *     later calls on it return SV_ERR_HIP.
 *   - Calls that return host scalars (sv_expect, sv_grad, sv_ground,
 *     sv_aqa_run with outputs, sv_batch_p1_scan) synchronise the state's
 *     stream before returning; all other calls only enqueue work.
 *   - Objects are not thread-safe: calls that use one state or instance from
 *     several host threads at once must be serialised by the caller.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { SV_C64 = 1, SV_C128 = 2 } sv_dtype;

typedef enum {
    SV_OK = 0,
    SV_ERR_ARG = 1,         /* bad argument (nothing was changed)              */
    SV_ERR_OOM = 2,         /* device or host allocation failed                 */
    SV_ERR_HIP = 3,         /* HIP runtime error (state marked failed)          */
    SV_ERR_UNSUPPORTED = 4, /* valid request the library does not handle        */
    SV_ERR_NUMERIC = 5      /* non-finite angle or coefficient                  */
} sv_status;

typedef struct sv_state_s* sv_state;
typedef struct sv_ising_s* sv_ising;

/* Thread-local message describing the last failure ("" if none). */
const char* sv_last_error(void);

/* Library version string and the GPU architecture the kernels were built for. */
const char* sv_version(void);

/* ---------------------------------------------------------------- states --
 * A state holds 2^n amplitudes in one device buffer.
 * n: 1 <= n <= 33 for SV_C128, 1 <= n <= 34 for SV_C64.
 */

/* Allocate 2^n amplitudes on the current device (contents undefined).  The
 * library owns the memory; sv_free releases it.  Fails with SV_ERR_OOM,
 * without allocating, if hipMemGetInfo reports too little free memory. */
int sv_alloc(int n, sv_dtype dtype, void* hip_stream, sv_state* out);

/* Borrow caller-owned device memory (e.g. a torch tensor's data_ptr()).
 * bytes must be at least 2^n * element size and dev_ptr 16-byte aligned.
 * The caller keeps ownership and must keep the buffer alive until sv_free. */
int sv_wrap(int n, sv_dtype dtype, void* dev_ptr, size_t bytes, void* hip_stream, sv_state* out);

/* Release the handle (and the memory if the library allocated it). */
int sv_free(sv_state s);

/* Change the stream later work on this state is enqueued on. */
int sv_set_stream(sv_state s, void* hip_stream);

/* psi(z) = 2^{-n/2} for all z: |+>^n, the ground state of H_I = -H_D
 * (Sec. III.A.1, Eq. HI) and the QAOA initial state (Eq. QAOA_state). */
int sv_init_plus(sv_state s);

/* Copy the whole state to / from host memory (interleaved, bytes = 2^n * elem).
 * Synchronous.  Meant for tests and small states. */
int sv_copy_to_host(sv_state s, void* host, size_t bytes);
int sv_copy_from_host(sv_state s, const void* host, size_t bytes);

/* ------------------------------------------------------------- instances --
 * Ising instance of Eq. HC.  Host arrays are copied and not retained.
 *   n: number of spins (1..34); h: n fields; m couplings (i, j, J) with
 *   0 <= i, j < n, i != j, no pair listed twice (in either order).
 *   All values finite (else SV_ERR_NUMERIC).  The instance tables are placed
 *   on the current device.
 */
int sv_ising_create(int n, const double* h, int m, const int32_t* ei, const int32_t* ej,
                    const double* J, sv_ising* out);
int sv_ising_free(sv_ising H);

/* Exact cover instance (Sec. III.A.3): the Boolean problem matrix a
 * (nrows x ncols, row-major, entries 0/1) of sum_f (sum_i a_if x_i - 1)^2
 * becomes, with x_i = (1 + s_i)/2 (Eq. xtosigma), the Ising instance of
 * Eqs. HChi and HCJij (h_i = sum_j (a a^T)_ij / 2 - (a b)_i, J_ij =
 * (a a^T)_ij / 2 for every pair with a nonzero overlap) plus the constant C
 * of Eq. HCC, returned in *constant (may be NULL): E(z) + C is the objective.
 * nrows = qubits (1..34), ncols >= 1; entries other than 0/1 are an error
 * (SV_ERR_ARG).  The half-integer coefficients use the phase tables. */
int sv_ising_exact_cover(int nrows, int ncols, const uint8_t* a, double* constant, sv_ising* out);

/* r of Eq. rescale for an instance: max of max(h)/2, min(h)/(-2), max(J)/1,
 * min(J)/(-1) and 0.  Dividing h, J and C by r does not change the solutions;
 * callers apply it as gamma / r and <H_C> * r (the state depends only on gamma E). */
int sv_rescale_factor(sv_ising H, double* r);

/* Brute-force ground state over all 2^n basis states (the full-enumeration
 * search of Sec. III.C.2, Table III): minimum energy, number of basis states
 * at that energy and the smallest such index.  Energies of instances whose
 * h and J are all integers compare exactly; otherwise states within
 * 1e-9 * max(1, sum|h| + sum|J|) of the minimum count.  The result is cached
 * in the instance.  Runs on the null stream; synchronous. */
int sv_ground(sv_ising H, double* e_min, uint64_t* degeneracy, uint64_t* argmin);

/* ------------------------------------------------------------ primitives --
 * Both are asynchronous on the state's stream.  n of state and instance must match.
 */

/* psi(z) <- exp(-i gamma E(z)) psi(z): the diagonal factor exp(-i gamma H_C)
 * of Eq. QAOA_state, E(z) from Eq. HC evaluated from the bits of z. */
int sv_cost_phase(sv_state s, sv_ising H, double gamma);

/* psi <- exp(-i beta H_D) psi = prod_i exp(-i beta sigma^x_i) psi: one
 * 2-component update per qubit (Eq. twocomponentupdates) with
 * u = [[cos b, -i sin b], [-i sin b, cos b]]. */
int sv_mixer(sv_state s, double beta);

/* --------------------------------------------------------------- drivers --
 * QAOA circuit of Eq. QAOA_state with p >= 1 layers: for k = 1..p apply
 * exp(-i gamma_k H_C) then exp(-i beta_k H_D).  from_plus != 0 starts from
 * |+>^n (the state's previous contents are ignored), otherwise from the
 * state's current contents.  Asynchronous. */
int sv_qaoa_forward(sv_state s, sv_ising H, int p, const double* gamma, const double* beta,
                    int from_plus);

/* One energy evaluation of the QAOA objective (Sec. III.B.1: each optimiser
 * call returns <H_C> of the p-layer state): sv_qaoa_forward followed by the
 * observables of sv_expect, with the reductions fused into the circuit's
 * last tile pass instead of a separate read of the state.  The final state
 * is stored as by sv_qaoa_forward.  Any output pointer may be NULL.
 * Synchronises the stream.  Errors as sv_qaoa_forward. */
int sv_qaoa_energy(sv_state s, sv_ising H, int p, const double* gamma, const double* beta, int from_plus,
                   double* energy, double* p_gs, double* norm);

/* sv_qaoa_energy for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same program, kernels and results as sv_qaoa_energy, but:
 *   - d_out: caller-owned DEVICE array of 3 doubles, written on the state's
 *     stream as (norm, energy, p_gs); the call returns after enqueueing and
 *     does not synchronise (read d_out after the stream has completed);
 *   - the reduction partials and phase tables live in a fixed ~32 MiB device
 *     array of the library (one per GPU, held until the process ends); the
 *     call makes no hipMalloc / hipFree / pinned-host allocation;
 *   - limits: partials of at most 2^20 tiles (every n up to 33 complex128 and
 *     34 complex64) and phase tables of at most 2^19 entries (about
 *     p * (33 + 2L) with L the integer-energy table half width: p = 4 at
 *     L = 341 uses 3 k); beyond them SV_ERR_UNSUPPORTED, nothing enqueued;
 *   - the instance must already hold its device tables for this n and dtype
 *     and its ground-state cache: run sv_qaoa_energy once with a state of the
 *     same n and dtype (or sv_ground and such a call) before; otherwise
 *     SV_ERR_UNSUPPORTED, nothing enqueued;
 *   - the state's device must be the current device (else SV_ERR_ARG).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams or host threads) race and must be serialised by the
 * caller.  d_out NULL or not 8-byte aligned: SV_ERR_ARG. */
int sv_qaoa_energy_noalloc(sv_state s, sv_ising H, int p, const double* gamma, const double* beta, int from_plus,
                           double* d_out);

/* Approximate quantum annealing (Sec. III.B.2): the same circuit, from |+>^n,
 * with `steps` (gamma_k, beta_k) pairs built by one of the schedule helpers
 * below.  If pgs_per_step / energy_per_step are non-NULL they receive, after
 * every step k, the ground-state probability and <H_C> (length `steps`);
 * then the call synchronises. */
int sv_aqa_run(sv_state s, sv_ising H, int steps, const double* gamma, const double* beta,
               double* pgs_per_step, double* energy_per_step);

/* sv_aqa_run plus the spin expectations <sigma^z_i> after every step (the
 * annealing observables of Sec. III.B.2): spinz_per_step receives steps * n
 * values, row k = step k, column i = qubit i (sigma^z eigenvalue -1 for bit 0,
 * Sec. III.A.3).  The n sums ride in the tile pass that ends each step.  Any
 * output may be NULL; with a non-NULL output the call synchronises. */
int sv_aqa_run_observe(sv_state s, sv_ising H, int steps, const double* gamma, const double* beta,
                       double* pgs_per_step, double* energy_per_step, double* spinz_per_step);

/* Observables of the current state (Sec. III.B.1): energy = <psi|H_C|psi>,
 * p_gs = sum of |psi(z)|^2 over the ground-state set of sv_ground (computed
 * first if needed), norm = <psi|psi>.  Any output pointer may be NULL.
 * FP64 accumulation, deterministic order.  Synchronises the stream. */
int sv_expect(sv_state s, sv_ising H, double* energy, double* p_gs, double* norm);

/* <psi|sigma^z_i|psi> for every qubit i of the current state (out: n values;
 * sigma^z eigenvalue -1 for bit 0, Sec. III.A.3).  One read-only tile pass,
 * FP64 sums in a fixed order.  Synchronises the stream. */
int sv_spin_z(sv_state s, double* out);

/* --------------------------------------------------- general single-qubit layers --
 * Apply nlayers layers of single-qubit gates: layer k applies the 2x2 complex
 * matrix U_{k,q} to every qubit q (the gate set of the Hadamard benchmark,
 * Sec. II.B, and the single-spin factors of Eq. AQA4).
 *   U: host, [nlayers][n][8] doubles, row-major (u00 re, u00 im, u01 re, u01 im,
 *      u10 re, u10 im, u11 re, u11 im); u00 maps the amplitude with bit q = 0
 *      to itself.  Any complex matrix is accepted (unitarity is not checked).
 *   nlayers == 0 is a no-op.  Since gates on different qubits commute, each
 *   tile group takes up to four consecutive layers per pass over the state.
 * SV_ERR_NUMERIC for a non-finite entry.  Asynchronous on the state's stream
 * (U is copied before the call returns). */
int sv_gate_layers(sv_state s, int nlayers, const double* U);

/* Time stepping of Eq. AQA4 (the paper's TDSE solver for annealing): for
 * l = 0..steps-1, with A_l = A[l], B_l = B[l] (the annealing functions sampled
 * at the step's time, e.g. s = l/steps for t_anneal = steps * tau),
 *   |psi> <- M_l exp(i tau sum_{i<j} Jt_ij Z_i Z_j) M_l |psi>,
 *   M_l = prod_i exp(i tau/2 (A_l X_i + ht_i Z_i)),  ht_i = -B_l h_i,  Jt_ij = -B_l J_ij
 * (Eqs. AQA0-AQA3: x fields A, z fields -B h, zz couplings -B J; Z has
 * eigenvalue -1 on bit 0, Sec. III.A.3).  from_plus != 0 starts from |+>^n
 * (the paper's initial state), else from the current state.
 * Per-step outputs (host, may each be NULL): energy_per_step[steps] = <H_C>,
 * pgs_per_step[steps] = ground-state probability, spinz_per_step[steps][n] =
 * <sigma^z_i>, all after the step.  With every output NULL the outer half
 * steps of consecutive steps are merged into one single-qubit layer (one pass
 * per tile group and step); with outputs each step costs two layers.
 * SV_ERR_NUMERIC for non-finite tau, A or B.  Synchronises when an output is
 * requested. */
int sv_qsds_run(sv_state s, sv_ising H, int steps, double tau, const double* A, const double* B,
                int from_plus, double* energy_per_step, double* pgs_per_step, double* spinz_per_step);

/* ---------------------------------------------------------------- adjoint --
 * Gradient of f(gamma, beta) = <beta,gamma| H_C |beta,gamma> with respect to
 * all 2p parameters in one reverse sweep that uncomputes the state instead of
 * storing it (the paper's optimiser only evaluates f, Sec. III.B.1; this is
 * the reverse-mode derivative of that same circuit).
 *   psi, lam: two states with equal n and dtype (lam is scratch).
 *   psi_is_forward != 0: psi already holds the QAOA state for (gamma, beta);
 *   otherwise the forward circuit is run from |+>^n first.
 *   Outputs: energy and p_gs (the ground-state probability of the same state,
 *   Sec. III.B.1; either may be NULL), dgamma[p], dbeta[p] (host).
 * On return psi and lam hold unspecified values.  Synchronises. */
int sv_grad(sv_state psi, sv_state lam, sv_ising H, int p, const double* gamma,
            const double* beta, int psi_is_forward, double* energy, double* p_gs,
            double* dgamma, double* dbeta);

/* ------------------------------------------------------------- schedules --
 * Host-only helpers that fill gamma[], beta[] (no GPU work).
 *
 * First-order coarse annealing with the linear stand-in schedule A(s) = 1 - s,
 * B(s) = s (the DW_2000Q_6 data of Fig. 4 is not available): step k = 1..steps,
 * s_k = k/steps, applies exp(-i tau B(s_k) H_C) then exp(-i tau A(s_k) H_I),
 * H_I = -H_D (Eqs. HI, Hofs), i.e. gamma_k = tau s_k and
 * beta_k = -tau (1 - s_k).  paper_sign == 0 gives beta_k = +tau (1 - s_k). */
int sv_schedule_linear(int steps, double tau, int paper_sign, double* gamma, double* beta);

/* Second-order Suzuki-Trotter parameters (Eqs. beta_k-gamma_k, Appendix A) on
 * the grid s_k = (k-1)/(p-1), k = 1..p (p >= 2; for AQA with n steps use
 * p = n + 1).  A, B: values of the annealing functions on that grid (length
 * p), or NULL for the linear stand-in A = 1 - s, B = s. */
int sv_schedule_second_order(int p, double tau, const double* A, const double* B,
                             double* gamma, double* beta);

/* ----------------------------------------------------------------- batch --
 * p = 1 landscape scan (Sec. III.C.1, Fig. 5) over many small instances in
 * persistent launches: for every instance i and grid point (gamma_a, beta_b)
 * evaluate |psi> = exp(-i beta_b H_D) exp(-i gamma_a H_C_i) |+>^{n_i} and write
 *   energy_out[(i * n_gamma + a) * n_beta + b] = <H_C_i>
 *   pgs_out   [(i * n_gamma + a) * n_beta + b] = ground-state probability.
 * Instances may differ in n (1..19 for SV_C64, 1..18 for SV_C128; larger n
 * returns SV_ERR_UNSUPPORTED).  dtype selects the amplitude storage.
 * Outputs are host arrays.  Runs on the given stream; synchronises. */
int sv_batch_p1_scan(int n_inst, const sv_ising* insts, int n_gamma, const double* gammas,
                     int n_beta, const double* betas, sv_dtype dtype, void* hip_stream,
                     double* energy_out, double* pgs_out);

/* -------------------------------------------------------------- tuning --
 * Tile and launch choices.  sv_tune_set overrides a named knob for later
 * calls in this process (names and ranges in sv_tune_describe); sv_tune_get
 * reads it back; sv_tune_describe writes a JSON description of all knobs and
 * of the plan chosen for (n, dtype) into buf (truncated to len bytes,
 * NUL-terminated) and returns SV_OK.  Host-only. */
int sv_tune_set(const char* name, int value);
int sv_tune_get(const char* name, int* value);
int sv_tune_describe(int n, sv_dtype dtype, char* buf, size_t len);

/* Per-(dtype, n) knob overrides chosen by the autotuner: a text file of lines
 * "<c64|c128> <n> <knob> <value>".  Read from $SV_TUNE_CACHE at the first
 * plan, or (replacing what was loaded) by sv_tune_load(path); path NULL
 * clears them.  Overrides take precedence over sv_tune_set values. */
int sv_tune_load(const char* path);

/* ------------------------------------------------------------- profiling --
 * sv_profile_enable(1) clears the record and starts timing every tile-pass
 * launch with a pair of HIP events on the launch stream; (0) stops it.
 * sv_profile_report synchronises on the recorded events and writes JSON
 *   {"<kernel kind>": {"launches": N, "ms": total, "bytes": total}, ...}
 * where bytes counts the algorithmic traffic of each launch (state vectors
 * read plus state vectors written, 2^n * element size each); then clears. */
int sv_profile_enable(int on);
int sv_profile_report(char* buf, size_t len);

/* Streaming ceiling of the tile passes' access pattern (no paper passage:
 * the reference rate the pass bandwidth is compared with).  One in-place
 * read + write of the whole state, tile by tile, with the passes' tile size
 * (2^13 amplitudes for SV_C128, 2^14 for SV_C64), lane order, nontemporal
 * accesses and tile order, and no arithmetic: the state is unchanged.  A tile
 * holds the c lowest index bits (runs of 2^c amplitudes) and the T - c bits
 * starting at lo; c = T is the contiguous tile (lo ignored).  *ms receives the
 * kernel time from HIP events on the state's stream.  Requires n >= T,
 * 0 <= c <= T and c <= lo, lo + T - c <= n (else SV_ERR_ARG).  Synchronises. */
int sv_stream_ceiling(sv_state s, int c, int lo, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* SV_H */
