/*
 * sbqa.h - C ABI of the MI355X (gfx950) SBQA time-stepping library.
 *
 * Simulated Bifurcation Quantum Annealing (arXiv 2604.01050). An Ising problem
 * (couplings J, fields h; Sec. II.A, the energy of Eq. 2 at the hypercube
 * corners) is solved by R replicas per run coupled in a periodic Trotter ring
 * (Supplement S1) and evolved with the equations of motion of Eqs. 6-7, the
 * wall condition of Eq. 3 and the nonlinearity f of Eq. 8. Many independent
 * runs ("repetitions" of Sec. II.B), each with its own (beta, alpha), evolve
 * side by side and the best solution over replicas is returned.
 *
 * Conventions used throughout
 *   - N spins, R replicas per run, `runs` runs; C = runs * R columns.
 *   - State matrices are N x C row-major float32; column c = r*R + k holds
 *     replica k of run r. x is the position q of Eq. 6, y the momentum p.
 *   - Step n (0 <= n < steps) integrates t_n = n*dt -> t_{n+1} with
 *     T = steps*dt: pump a_n = n/steps (Sec. II.A), threshold
 *     Delta_n = delta_max*n/steps (Eq. 8), coupling J_perp[r][n] (Eq. 5).
 *     Symplectic Euler: y += dt*F(x_n); x += dt*(a0/R)*y; |x| > 1 ->
 *     x = sign(x), y = 0.
 *   - Energy E(s) = -1/2 s^T J s - h^T s; spins are int8 +-1 with the
 *     readout s_i = sign(x_i), sign(0) = +1 (Sec. II.A, where the position is q_i).
 *   - Every pointer argument is a HOST pointer unless stated otherwise.
 *     Inputs are copied before the call returns (the caller keeps ownership
 *     and may free them). Outputs are caller-allocated.
 *   - Every call returns an sbqa_status; on failure a thread-local message is
 *     available from sbqa_last_error(). The library never aborts the process.
 *   - A context is not thread-safe: use one context per thread, or serialise.
 *   - All device work of a context is issued on its stream (default: the
 *     library's non-blocking stream of the device, shared by every context
 *     created without a stream of the caller's, so their work is ordered;
 *     see sbqa_set_stream). Calls that return data to the host synchronise
 *     that stream.
 */
#ifndef SBQA_H
#define SBQA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBQA_ABI_VERSION 1

typedef struct sbqa_ctx sbqa_ctx;
typedef struct sbqa_server sbqa_server;

typedef enum {
    SBQA_OK = 0,
    SBQA_EINVAL = -1,   /* invalid argument or instance (message says which)   */
    SBQA_ENOMEM = -2,   /* host or device allocation failed                    */
    SBQA_EDEVICE = -3,  /* HIP runtime error, or no gfx950 device              */
    SBQA_ESTATE = -4,   /* call not valid in this state (e.g. past the end)    */
    SBQA_EBUDGET = -5,  /* instance can never fit the server's memory budget   */
    SBQA_EAGAIN = -6    /* result not ready yet (serving)                      */
} sbqa_status;

/* Nonlinearity f of the coupling sum: Eq. 8 (ternary, the paper's choice),
 * dSB f(x) = sign(x) and bSB f(x) = x (Sec. II.A). In sign mode sign(0) = 0. */
typedef enum { SBQA_F_TERNARY = 0, SBQA_F_SIGN = 1, SBQA_F_BALLISTIC = 2 } sbqa_fmode;

/* Arithmetic of the dense coupling sum J.f(X) (the CSR form is always fp32):
 *   FP32   fp32 J, fp32 operand, fp32 accumulation (MFMA f32).
 *   FP8    J and f(X) in e4m3, fp32 accumulation. Exact when J is in
 *          {-1,0,+1} and f is ternary or sign; rejected otherwise.
 *   INT8   J and f(X) in int8, int32 accumulation, each field rounded once to
 *          fp32. Exact integer sums for integer J with |J| <= 127 (e.g. the
 *          Sidon28 couplings of the QAC benchmarks, Sec. III, scaled by 28 to
 *          {8, 13, 19, 28}: 19 has no e4m3 encoding) and f ternary or sign;
 *          rejected otherwise.
 *   FP4    J and f(X) in e2m1 fp4 (4 bits, the CDNA4 matrix cores' fastest
 *          format), fp32 accumulation. +-1 and 0 are exact in e2m1, so it is
 *          exact where FP8 is (J in {-1,0,+1}, f ternary or sign) and gives
 *          the same bits; rejected otherwise.
 *   BF16X3 J and f(X) split into bf16 hi + lo; J_hi f_hi + J_hi f_lo + J_lo f_hi
 *          accumulated in fp32 (ballistic / real-valued contraction).
 *   AUTO   with f ternary or sign: FP4 for J in {-1,0,+1} (the fastest exact
 *          form), else INT8 for integer J with |J| <= 127, else FP32; with f
 *          ballistic: FP32. */
typedef enum {
    SBQA_PREC_AUTO = 0, SBQA_PREC_FP32 = 1, SBQA_PREC_FP8 = 2, SBQA_PREC_BF16X3 = 3, SBQA_PREC_INT8 = 4,
    SBQA_PREC_FP4 = 5
} sbqa_prec;

/* Inter-replica coupling schedule J_perp[r][n]:
 *   LINEAR  jp_start + (jp_end - jp_start) * n/steps, the same for every run.
 *   PAPER   Eq. 5: -(1/(2 beta_r)) ln tanh(beta_r Gamma_x(t)/R) with
 *           Gamma_x(t)/R = gamma0_over_R * ((1 - n/steps)^alpha_r + 1e-5),
 *           beta_r, alpha_r per run (Sec. II.B auto-tuning).
 *   TABLE   caller-supplied float32 table jp_table[runs*steps]. */
typedef enum { SBQA_JP_LINEAR = 0, SBQA_JP_PAPER = 1, SBQA_JP_TABLE = 2 } sbqa_jpkind;

/* Step-loop kernel.
 *   AUTO      RESIDENT when the instance fits a resident loop, else STREAM.
 *   STREAM    one fused launch per step, state streamed through HBM.
 *   RESIDENT  many steps per launch with the state on chip:
 *             - sparse (CSR): the register-resident loop (ternary or sign f,
 *               R a multiple of 8, N <= 4096, small degree, all column blocks
 *               co-resident on the GPU); it computes the same bits as STREAM;
 *             - dense: the small-instance loop (N <= 128, R*N <= 4096, any
 *               precision but BF16X3: it computes in float32), one workgroup
 *               per run with the rows of J in registers and the run's
 *               positions in LDS; fields are summed in a fixed order over j,
 *               or counted over bit masks of J and f(x) when J is in
 *               {-1,0,+1} and f is ternary or sign (the same bits as STREAM
 *               when J and the operand are integral).
 *             sbqa_create fails with EINVAL when the instance does not fit. */
typedef enum { SBQA_LOOP_AUTO = 0, SBQA_LOOP_STREAM = 1, SBQA_LOOP_RESIDENT = 2 } sbqa_loop_kernel;

/* Storage of J for the dense FP8 and FP4 contractions:
 *   AUTO   one bit per coupling when every off-diagonal J_ij is +-1 (SK-type
 *          instances: 8x (FP8) or 4x (FP4) fewer J bytes to stream per
 *          step); expanded to e4m3 / e2m1 in registers, so the fields are the
 *          same exact integers.
 *   BYTES  one e4m3 byte (FP8) or e2m1 nibble (FP4) per coupling. */
typedef enum { SBQA_JPACK_AUTO = 0, SBQA_JPACK_BYTES = 1 } sbqa_j_packing;

/* Spin order inside the library for CSR couplings (the contraction gathers
 * the operand rows of a spin's neighbours and triple partners, which stay in
 * cache only when their indices are close):
 *   AUTO  relabel the spins by reverse Cuthill-McKee (breadth-first over the
 *         pair and triple adjacency) when N >= 16384, the given numbering
 *         puts neighbours far apart (mean |i - j| over the adjacency above
 *         N/64) and the new order cuts that mean at least 4x; else keep it;
 *   OFF   keep the given order;
 *   ON    relabel whenever the instance has couplings.
 * Relabelling is internal: every spin-indexed input and output (state, best
 * spins, the spins of sbqa_energy, fields) stays in the caller's order, the
 * initial state is drawn by the caller's spin index, and each spin's
 * couplings are summed in the given order, so trajectories are the same bit
 * for bit (real-valued energies up to the order of their FP64 sums). Dense
 * couplings ignore it. */
typedef enum { SBQA_REORDER_AUTO = 0, SBQA_REORDER_OFF = 1, SBQA_REORDER_ON = 2 } sbqa_reorder;

/* Couplings: exactly one of `dense` or the CSR triple is non-NULL.
 * J must be symmetric with a zero diagonal and finite entries.
 *   dense    N*N float64, row-major.
 *   row_ptr  N+1 int32, col nnz int32 (0 <= col < N), val nnz float64;
 *            both (i,j) and (j,i) stored; duplicate entries are rejected;
 *            col and val may be NULL when nnz is 0.
 * Optional native three-body terms (the cubic part of the HUBO Hamiltonian,
 * Eq. 11; CSR couplings only, nnz may be 0):
 *   n3       number of triples (0: none)
 *   tri      n3*3 int32 spin indices, three distinct per triple, each triple
 *            listed once
 *   K        n3 float64 finite weights
 * Energy E(s) = -1/2 s^T J s - h^T s - sum_t K_t s_l s_m s_n, so the paper's
 * H = sum J s s + sum K s s s is J -> -J (both entries of each pair) and
 * K -> -K. In the equations of motion spin l receives K f(x_m) f(x_n) in its
 * coupling sum (likewise m and n). Three-body instances run on the streaming
 * CSR kernel (no resident loop). */
typedef struct {
    const double *dense;
    const int32_t *row_ptr;
    const int32_t *col;
    const double *val;
    int64_t nnz;
    int64_t n3;
    const int32_t *tri;
    const double *K;
} sbqa_coupling;

/* Hyper-parameters of one solve. Start from sbqa_schedule_default(). */
typedef struct {
    uint32_t steps;          /* S >= 1 (total evolution T = steps*dt)              */
    double dt;               /* > 0                                                */
    double a0;               /* > 0, Eq. 3 / Eq. 6                                 */
    double c0;               /* > 0; <= 0 selects 0.5/(sqrt(N) rms(J_offdiag)); with
                                three-body terms 0.5/sqrt(v/(N-1)), v = sum of
                                J_ij^2 over i != j plus 3 sum K_t^2            */
    int32_t fmode;           /* sbqa_fmode                                         */
    double delta_max;        /* Eq. 8 threshold factor (paper: 0.7)                */
    int32_t jp_kind;         /* sbqa_jpkind                                        */
    double jp_start, jp_end; /* LINEAR                                             */
    double gamma0_over_R;    /* PAPER: Gamma_x(0)/R (> 0)                          */
    double beta_lo, beta_hi; /* PAPER: beta_r ~ U[lo,hi] when `beta` is NULL       */
    double alpha_lo, alpha_hi; /* PAPER: alpha_r ~ U[lo,hi] when `alpha` is NULL   */
    const double *beta;      /* optional [runs] explicit beta_r (copied)           */
    const double *alpha;     /* optional [runs] explicit alpha_r (copied)          */
    const float *jp_table;   /* TABLE: [runs*steps], run-major (copied)            */
    uint64_t seed;           /* initial state and beta/alpha draws                 */
    double init_amp;         /* x, y ~ U[-init_amp, init_amp] (counter-based RNG)  */
    int32_t precision;       /* sbqa_prec                                          */
    uint32_t energy_every;   /* 0: best over the final state only; K > 0: also
                                track the best after every K-th step              */
    int32_t loop_kernel;     /* sbqa_loop_kernel                                   */
    int32_t dense_tile;      /* dense path: replica columns per workgroup tile,
                                64, 128 or 256; 0 = autotuned (each candidate's
                                step timed on scratch buffers of the instance's
                                shape once per device and shape; every tile
                                gives the same bits). Choices persist across
                                processes in a text file: the path in the
                                environment variable SBQA_TUNE_CACHE ("off":
                                none), else $XDG_CACHE_HOME/sbqa/dense_tiles.txt,
                                else $HOME/.cache/sbqa/dense_tiles.txt; a file
                                that cannot be read or written is ignored     */
    int32_t j_packing;       /* sbqa_j_packing (dense FP8 / FP4 only)              */
    int32_t reorder;         /* sbqa_reorder (CSR couplings only)                  */
} sbqa_schedule;

/* Defaults: steps 1000, dt 0.5, a0 1, c0 auto, ternary f, delta_max 0.7,
 * PAPER schedule with gamma0_over_R 1, beta in [0.5,1.5], alpha in [0.5,1.0]
 * (Sec. II.B), seed 0, init_amp 0.1, precision AUTO, energy_every 0,
 * loop_kernel AUTO, dense_tile 0 (autotuned), j_packing AUTO, reorder AUTO. */
sbqa_schedule sbqa_schedule_default(void);

/* Context information (sbqa_info). */
typedef struct {
    int32_t N, R, runs;
    uint32_t steps;          /* S                                                  */
    uint32_t step;           /* steps already taken                                */
    int32_t path;            /* 0 dense fp32, 1 dense fp8, 2 dense bf16x3, 3 csr,
                                4 dense int8, 5 dense fp8 with bit-packed J,
                                6 dense fp4, 7 dense fp4 with bit-packed J      */
    int32_t fmode;
    double c0;               /* c0 actually used                                   */
    int32_t j_integral;      /* 1 when every J_ij and h_i is an integer            */
    size_t device_bytes;     /* device memory held by the context                  */
    int32_t resident;        /* 1 when steps run in a resident loop
                                (sbqa_loop_kernel), 0 otherwise                   */
    int32_t tile_cols;       /* dense path: replica columns per workgroup tile   */
    int32_t reordered;       /* 1 when CSR spins are relabelled internally
                                (sbqa_reorder), 0 otherwise                       */
} sbqa_info_t;

/*
 * Create a solver for one Ising instance (Sec. II.A problem statement):
 * validates J and h, draws (beta_r, alpha_r) per run (Sec. II.B), builds the
 * schedule tables (Eq. 5, Eq. 8), uploads J in the contraction precision and
 * initialises x, y ~ U[-init_amp, init_amp] on the device.
 *   J     couplings (see sbqa_coupling), copied.
 *   h     N float64 fields, or NULL for h = 0, copied.
 *   out   receives the context; owned by the caller until sbqa_destroy.
 * Errors: EINVAL (N, R, runs, steps < 1; dt, a0 <= 0; J not symmetric, non-zero
 * diagonal, non-finite, malformed CSR; FP8 with ballistic f or J outside
 * {-1,0,+1}; BF16X3 with CSR; LOOP_RESIDENT for an instance that does not
 * fit a resident loop), ENOMEM, EDEVICE.
 */
sbqa_status sbqa_create(const sbqa_coupling *J, const double *h, int32_t N, int32_t R,
                        int32_t runs, const sbqa_schedule *s, sbqa_ctx **out);

/*
 * Advance every run and replica by n steps of Eqs. 6-7 (contraction J.f(X),
 * fused pump/ring/kick/drift/wall update). Asynchronous on the context stream.
 * Errors: ESTATE if step + n > steps (nothing is done), EDEVICE (also reported
 * by the next synchronising call when a resident launch could not complete a
 * step: the state is then invalid).
 */
sbqa_status sbqa_step(sbqa_ctx *ctx, uint32_t n);

/*
 * Best solution per run (Sec. II.B: the output of a solve): the minimum
 * energy over the run's R replicas of the current state (and over the tracked
 * evaluations when energy_every > 0). Ties: lowest replica, earliest step.
 *   energies  [runs] float64 out (may be NULL)
 *   spins     [runs*N] int8 +-1 out, run-major (may be NULL)
 * Energies are exact for integer J and h; float64 otherwise. Synchronises.
 */
sbqa_status sbqa_best(sbqa_ctx *ctx, double *energies, int8_t *spins);

/* Step index (0..steps) at which each run's best was found ([runs] int64). */
sbqa_status sbqa_best_step(sbqa_ctx *ctx, int64_t *step_of_best);

/*
 * Energies of caller-given spin configurations on the device (the Ising
 * energy, Eq. 2 at the corners): spins [count*N] int8 +-1, out [count]
 * float64. Exact for integer J and h. Synchronises.
 */
sbqa_status sbqa_energy(sbqa_ctx *ctx, const int8_t *spins, int32_t count, double *out);

/*
 * sbqa_energy for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc. It
 * calls no allocating routine and does not synchronise.
 *   spins  DEVICE pointer, count*N int8 (+-1, not validated: other values are
 *          used as given), the caller's spin order.
 *   out    DEVICE pointer, count float64, written by the context's stream.
 * The result equals sbqa_energy's bit for bit (same kernels, same order).
 * Scratch: a library-owned device array of SBQA_NOALLOC_SCRATCH_BYTES per GPU,
 * created when the library's code is loaded on that GPU and held until the
 * process ends. Dense couplings need 8*cp*Np*(1 + es) bytes of it (cp = count
 * rounded up to 128, Np the padded N, es in {1,2,4,8} the K splits of the
 * float64 GEMM), relabelled CSR couplings count*N bytes, other CSR couplings
 * none; a call that needs more returns SBQA_EINVAL before any device work.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams or threads) race. spins and out must be device memory
 * (SBQA_EINVAL otherwise).
 */
#define SBQA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
sbqa_status sbqa_energy_noalloc(sbqa_ctx *ctx, const int8_t *spins, int32_t count, double *out);

/*
 * Coupling sum of Eq. 7 for the current state: phi[N*C] float32 (row-major
 * like the state) = J . f(X) with the threshold of the current step, in the
 * context's contraction precision. Test hook; synchronises.
 */
sbqa_status sbqa_fields(sbqa_ctx *ctx, float *phi);

/* Read / overwrite the state (x, y: N*C float32 row-major each). set_state
 * also rebuilds the contraction operand f(X). Synchronise. */
sbqa_status sbqa_get_state(sbqa_ctx *ctx, float *x, float *y);
sbqa_status sbqa_set_state(sbqa_ctx *ctx, const float *x, const float *y);

/* Per-run parameters of the inter-replica coupling schedule in use (Sec. II.B:
 * each run draws its own beta_r and alpha_r from the stated ranges; Eq. 5
 * takes them): [runs] float64 each, caller-allocated; NULL skips that
 * output. Host-only (no device work). EINVAL for a NULL context. */
sbqa_status sbqa_run_params(sbqa_ctx *ctx, double *beta, double *alpha);

/* The inter-replica coupling J_perp(t_n) of Eq. 5 (or the linear or caller
 * table the schedule names) as the kernels read it: jp[runs*steps] float32,
 * run-major (jp[r*steps + n] for run r at step n), caller-allocated. Read
 * from the host copy the device table was uploaded from (no device work).
 * EINVAL for NULL arguments. */
sbqa_status sbqa_jperp_table(sbqa_ctx *ctx, float *jp);

/* Issue the context's device work on `hip_stream` (a hipStream_t, e.g.
 * torch.cuda.current_stream().cuda_stream); NULL restores the library's
 * stream of the device. The context's work issued so far completes first.
 * The caller keeps the stream alive while the context uses it. */
sbqa_status sbqa_set_stream(sbqa_ctx *ctx, void *hip_stream);

sbqa_status sbqa_info(sbqa_ctx *ctx, sbqa_info_t *info);

/* Block until the context's device work has finished. EDEVICE when a
 * resident sparse launch could not complete a step (a ring-neighbour wait
 * timed out); the state is then invalid. */
sbqa_status sbqa_sync(sbqa_ctx *ctx);

/* Failure-path test hook of the resident sparse loop: sets the context's
 * device error word as a ring-neighbour wait timeout would (a neighbouring
 * workgroup that never published its step), so that the next resident launch
 * skips its waits and the next call that synchronises (sbqa_best, sbqa_sync)
 * reports SBQA_EDEVICE; every kernel still runs to its end. The state is
 * invalid afterwards. EINVAL on a context without the resident sparse loop.
 * Asynchronous on the context stream. */
sbqa_status sbqa_inject_wait_timeout(sbqa_ctx *ctx);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *sbqa_last_error(void);

/* Release the context and its device memory. NULL is a no-op. */
void sbqa_destroy(sbqa_ctx *ctx);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of many instances on one GPU.               */
/* ------------------------------------------------------------------------ */

/*
 * Create a server with a device-memory budget (bytes) and at most max_slots
 * instances resident at once. A scheduler thread admits queued requests in
 * arrival order while their device footprint fits the budget and a slot is
 * free, steps all resident instances together in batched launches, retires
 * finished ones and admits the next. out receives the handle.
 * Errors: EINVAL (budget 0, max_slots < 1), ENOMEM, EDEVICE.
 */
sbqa_status sbqa_server_create(size_t hbm_budget_bytes, int32_t max_slots, sbqa_server **out);

/*
 * Queue one instance (same arguments and validation as sbqa_create). Inputs
 * are copied. ticket receives an id for sbqa_poll.
 * Errors: EINVAL, EBUDGET (the instance alone exceeds the budget), ESTATE
 * (server shutting down).
 */
sbqa_status sbqa_submit(sbqa_server *srv, const sbqa_coupling *J, const double *h, int32_t N,
                        int32_t R, int32_t runs, const sbqa_schedule *s, uint64_t *ticket);

/*
 * Result of a ticket: energies [runs], spins [runs*N] (either may be NULL),
 * latency_s = completion - submission (wall clock, seconds; may be NULL).
 * Returns EAGAIN while pending, OK once (the ticket is then released),
 * EINVAL for unknown tickets.
 */
sbqa_status sbqa_poll(sbqa_server *srv, uint64_t ticket, double *energies, int8_t *spins,
                      double *latency_s);

/* Counters: completed instances, replica-spin updates done, busy seconds. */
sbqa_status sbqa_server_stats(sbqa_server *srv, uint64_t *completed, double *updates,
                              double *busy_s);

/* Finish resident work, drop the queue, join the scheduler, free memory. */
void sbqa_server_destroy(sbqa_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SBQA_H */
