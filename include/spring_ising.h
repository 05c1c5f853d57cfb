/*
 * spring_ising.h -- C ABI of the MI355X (gfx950) Spring-Ising hot path.
 *
 * The library iterates the Spring-Ising Algorithm of Jiang et al.,
 * "Point convolutional neural network algorithm for Ising model ground state
 * research based on spring vibration" (arXiv 2305.07187):
 *
 *   Ising energy, Eq. (1):   H = - sum_{i<j} J_ij s_i s_j - sum_i h_i s_i
 *   iteration, Eq. (8) (Eq. (5) with the mass m kept):
 *     q_i(n+1) = q_i(n) + (Delta_n/m) p_i(n)
 *     p_i(n+1) = p_i(n) - Delta_n k q_i(n) + zeta_n Delta_n sum_j J_ij q_j(n) [+ zeta_n Delta_n h_i]
 *   walls: q clamped to [-qmax, qmax] (Eq. 6, qmax = sqrt 2) and p to
 *     [-pmax, pmax] (Methods, constraints of Eq. 8, pmax = 2);
 *   zeta_n: piecewise-constant, linear in the iteration count
 *     (Methods; Fig. 4 and Fig. 5 captions);
 *   readout: s = sign(q) after the last step (Methods, hardware mapping).
 *
 * Many independent replicas run side by side; they are the pixels of the
 * paper's point-convolution feature map (Fig. 3).  One step is a dense
 * N x N by N x R product (the 1x1 convolution) fused with the update.
 *
 * Conventions for every entry point
 *   - Every call returns si_status and never throws.  On failure a message
 *     is available from spring_ising_last_error() (thread-local, valid until
 *     the next call on the same thread).
 *   - Array arguments are DEVICE pointers (e.g. a torch tensor's data_ptr())
 *     unless marked "host".  Host memory passed where device memory is
 *     required is rejected with SI_ERR_INVALID.
 *   - All device work is ordered on the stream given to the init call; no
 *     call synchronises the host except init (one validation round trip).
 *     Outputs written to caller buffers are complete once that stream has
 *     passed the call.
 *   - Layouts are row-major, replica-major: x[r*N + i] is spin i of
 *     replica r (channels-last feature map), J[i*N + j].
 *   - A context is single-stream and not thread-safe; distinct contexts are
 *     independent.  A HIP failure poisons the context: later calls other
 *     than destroy return SI_ERR_STATE.
 */
#ifndef SPRING_ISING_H
#define SPRING_ISING_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct si_ctx si_ctx; /* opaque; owns every device buffer it allocates */

typedef enum {
  SI_OK = 0,
  SI_ERR_INVALID = -1,     /* bad argument or input (asymmetric J, host pointer, ...) */
  SI_ERR_OOM = -2,         /* device allocation failed */
  SI_ERR_HIP = -3,         /* a HIP call failed; the context is poisoned */
  SI_ERR_STATE = -4,       /* context poisoned or not usable for this call */
  SI_ERR_UNSUPPORTED = -5, /* valid request this build or input cannot serve */
  SI_ERR_RANGE = -6        /* step index past the schedule length */
} si_status;

/* Update order.  PAPER: Eq. (8) as printed, both right-hand sides read the
 * step-n state.  SYMPLECTIC: p first, then q moves with the new (clamped) p. */
typedef enum { SI_ORDER_PAPER = 0, SI_ORDER_SYMPLECTIC = 1 } si_order;

/* Wall model.  CLAMP: q and p clamped independently (Eq. 6 and the momentum
 * box of Methods).  INELASTIC: additionally p = 0 wherever q ran past its
 * wall (the perfectly inelastic wall that Methods refers to). */
typedef enum { SI_WALL_CLAMP = 0, SI_WALL_INELASTIC = 1 } si_wall;

/* Arithmetic of the coupling product J.Q (accumulation is always FP32).
 *   FP32        : FP32 J and FP32 positions (plain method).
 *   BF16X_FP8J  : J stored as FP8 e4m3 (must be exact, e.g. +-1), positions
 *                 as a BF16 copy of the FP32 master state.
 *   BF16X_BF16J : J stored as BF16 (must be exact), positions BF16.
 *   BF16X_HILOJ : any real J split as hi = bf16(J), lo = bf16(J - hi),
 *                 two BF16 products into one FP32 accumulator; positions BF16.
 *   BF16X3_EXACTJ: J exact in BF16 (e.g. +-1); the FP32 positions split into
 *                 three BF16 pieces whose sum is the FP32 value exactly, so
 *                 every product is exact and only the FP32 accumulation
 *                 rounds (FP32-equivalent, on the BF16 matrix cores).
 *   BF16X_MIXEDJ: per instance, BF16X_FP8J when J is exact in FP8 e4m3 and
 *                 BF16X_HILOJ otherwise; spring_ising_info reports the form
 *                 chosen for a single instance.
 * The master positions and momenta are FP32 in every mode. */
typedef enum {
  SI_PREC_FP32 = 0,
  SI_PREC_BF16X_FP8J = 1,
  SI_PREC_BF16X_BF16J = 2,
  SI_PREC_BF16X_HILOJ = 3,
  SI_PREC_BF16X3_EXACTJ = 4,
  SI_PREC_BF16X_MIXEDJ = 5
} si_precision;

/* Scalar parameters.  spring_ising_default_params() fills the paper's values:
 * k = 0.5, m = 1, dt = 0.2, zeta from 0.8*zeta0 = 0.04 to 10*zeta0 = 0.5
 * (zeta0 = 0.05), stair_len = 1 (exactly linear), qmax = sqrt 2, pmax = 2
 * (Fig. 4 and Fig. 5 captions, Eq. 6, Methods). */
typedef struct {
  float k;            /* spring constant (finite) */
  float m;            /* mass, > 0 */
  float dt;           /* time step Delta for the generated schedule, > 0 */
  float zeta_start;   /* zeta at the first step */
  float zeta_end;     /* zeta at the last stair */
  int32_t total_steps;/* S, length of the schedules, >= 1 */
  int32_t stair_len;  /* L >= 1: zeta constant over runs of L steps; 1 = linear */
  float qmax;         /* position wall, > 0 */
  float pmax;         /* momentum wall, > 0 */
  int32_t order;      /* si_order */
  int32_t wall;       /* si_wall */
  int32_t precision;  /* si_precision */
  int32_t tile;       /* 0 = automatic kernel choice (the process's tile
                         cache when it holds this context's key, else the
                         built-in preference order); otherwise a tile id
                         reported by spring_ising_info (tuning override).
                         A batch takes 0, 1 (128 x 64 work items) or 2
                         (64 x 64). */
  int32_t energy_every; /* E >= 0.  E > 0: in-run energy checks.  After every
                         step that brings the step index t to a multiple of E,
                         the Eq. (1) energies of all replicas' spins are
                         written on the device to row t/E - 1 of the
                         context's energy trace (total_steps / E rows) and
                         update the best-state record (see update_best); the
                         check is part of the step sequence, so it also runs
                         inside captured HIP graphs.  The paper follows the
                         energy over the iterations (Fig. 4).  0 = off. */
} si_params;

/* Where the step kernel's tile of a context came from (si_info.tile_source). */
typedef enum {
  SI_TILE_FROM_TABLE = 0,   /* built-in preference order (from tile sweeps) */
  SI_TILE_FROM_CACHE = 1,   /* the process's tile cache (see tile_cache_load) */
  SI_TILE_FROM_CALLER = 2,  /* si_params.tile */
  SI_TILE_FROM_AUTOTUNE = 3 /* an autotune call on this context */
} si_tile_source;

/* Read-only facts about a context (host struct). */
typedef struct {
  int32_t n, r;             /* problem size */
  int32_t n_pad, r_pad;     /* padded device layout */
  int32_t t;                /* steps taken so far */
  int32_t total_steps;      /* schedule length S */
  int32_t j_integer;        /* 1 if every J_ij is an integer with |J_ij| <= 127 */
  int32_t j_fp8_exact;      /* 1 if every J_ij is exact in FP8 e4m3 */
  int32_t j_bf16_exact;     /* 1 if every J_ij is exact in BF16 */
  int32_t tile;             /* tile id of the step kernel in use */
  int32_t precision;        /* si_precision in use */
  int32_t graph_steps;      /* steps per captured HIP graph (0: not captured) */
  int64_t device_bytes;     /* device memory owned by the context */
  char kernel_name[64];     /* name of the step kernel in use */
  int32_t resident_steps;   /* run() calls of at least this many steps use the
                               resident launch (0: off or not available) */
  int32_t resident_groups;  /* workgroups of that launch (0: not available) */
  int32_t tile_source;      /* si_tile_source of `tile` */
  int32_t n_inst;           /* instances of a batch (0: single instance) */
} si_info;

/* Fill *prm (host) with the paper's parameter values and total_steps = S:
 * k = 0.5, m = 1, Delta = 0.2 and zeta from 0.8 zeta0 to 10 zeta0 with
 * zeta0 = 0.05 (Fig. 4 caption, Methods), the position wall sqrt 2
 * (Eq. (6)) and the momentum wall 2 (Methods). */
si_status spring_ising_default_params(si_params *prm, int32_t total_steps);

/* Create a context for n spins and r replicas.
 *   J  : device, n*n floats, row-major; must be symmetric with a zero
 *        diagonal and finite (Eq. 1 sums over pairs i<j; the diagonal has no
 *        meaning).  Violations -> SI_ERR_INVALID.  Precision modes that need
 *        an exact J format reject other J with SI_ERR_UNSUPPORTED.
 *   x0 : device, r*n floats, replica-major initial positions.
 *   p0 : device, r*n floats, or NULL for zero initial momenta.
 *   prm: host; copied.  Schedules Delta_n = prm->dt and zeta_n (linear in
 *        stairs of prm->stair_len) are generated for prm->total_steps steps.
 *   hip_stream: hipStream_t for all work of this context (NULL = null stream).
 * The inputs are copied into library-owned, padded buffers; the caller may
 * release them once the stream has passed this call.  Synchronises once. */
si_status spring_ising_init(si_ctx **out, int32_t n, int32_t r, const float *J,
                            const float *x0, const float *p0, const si_params *prm,
                            void *hip_stream);

/* Batched form: n_inst independent instances of uneven size stepped together
 * (one grouped launch per step covers every instance), sharing r, the
 * parameters and the schedules.  The paper runs many independent tests at
 * once as the pixels of one feature map (Fig. 3; Methods, hardware
 * implementation); here the independent problems may also differ in N.
 *   n : host, n_inst sizes (1 .. 65536).
 *   J : host array of n_inst device pointers, instance i an n[i]*n[i]
 *       symmetric zero-diagonal matrix.
 *   x0: host array of n_inst device pointers, instance i r*n[i] floats.
 *   p0: host array of n_inst device pointers (instance i r*n[i] floats, or
 *       NULL for zero momenta of that instance), or NULL: all momenta 0.
 * Precisions: FP32, or the BF16 forms BF16X_FP8J (every J exact in FP8),
 * BF16X_HILOJ and BF16X_MIXEDJ (FP8 J where exact, hi + lo BF16 J
 * otherwise), with instances padded to 128; BF16X_BF16J and BF16X3_EXACTJ:
 * SI_ERR_UNSUPPORTED.  Work items of 128 x 64 (batch tile 1) or 64 x 64
 * (batch tile 2): prm->tile, else the tile cache's entry for this batch's
 * key, else tile 1; autotune times both.  Each instance's trajectory equals
 * the single-instance run of the same form on the 64x64 tile of that slab
 * depth (FP32: tile 14; FP8 J: BF16 tile 9; hi + lo: BF16 tile 7) bit for
 * bit, with either batch tile.  In every later call the
 * instances are concatenated: state/spin arrays hold instance i's r*n[i]
 * values (replica-major) at offset r * (n[0] + ... + n[i-1]); energies hold
 * instance i's r values at offset r*i.  set_field and
 * relaxed_energy_grad are not available for a batch.  Synchronises once. */
si_status spring_ising_init_batch(si_ctx **out, int32_t n_inst, const int32_t *n, int32_t r,
                                  const float *const *J, const float *const *x0,
                                  const float *const *p0, const si_params *prm,
                                  void *hip_stream);

/* Replace the per-step schedules (device, total_steps floats each): the time
 * step Delta_n and the dynamic-equilibrium weight zeta_n of Eq. (8).  The
 * paper varies zeta with the iteration count (Methods: zeta(t_step), a
 * piecewise-constant function) and compares fixed and staircase strategies
 * in Fig. 5; any such schedule is given here as explicit per-step values.
 * Delta_n must be > 0; values are not checked on the host.  The arrays are
 * copied on the context's stream. */
si_status spring_ising_set_schedule(si_ctx *ctx, const float *dt, const float *zeta);

/* Copy the per-step schedules Delta_n, zeta_n of Eq. (8) out (device,
 * total_steps floats each; either may be NULL). */
si_status spring_ising_get_schedule(si_ctx *ctx, float *dt, float *zeta);

/* Set an external field h (device, n floats; Eq. 1).  It adds zeta_n h_i to
 * the force of Eq. (4) and -sum_i h_i s_i to the energy.  NULL clears it. */
si_status spring_ising_set_field(si_ctx *ctx, const float *h);

/* One iteration of Eq. (8) with the walls at step index t; t += 1.
 * SI_ERR_RANGE if t == total_steps. */
si_status spring_ising_step(si_ctx *ctx);

/* n_steps iterations (n_steps >= 0).  SI_ERR_RANGE, with nothing run, if
 * t + n_steps > total_steps.  Asynchronous: no host round trip per step. */
si_status spring_ising_run(si_ctx *ctx, int32_t n_steps);

/* Execute run() calls of at least min_steps steps as HIP graphs: the launch
 * sequence of such a call is captured once (keyed by its start step, length
 * and buffer parity; up to four are kept) and replayed as one graph launch.
 * Results are bit-identical to direct launches.  0 turns graphs off. */
si_status spring_ising_set_graph(si_ctx *ctx, int32_t min_steps);

/* Split the contraction of the coupling product over k: ksplit ranges are
 * multiplied in parallel into a device workspace (ksplit x the state's size)
 * and a second launch adds them in a fixed order and applies Eq. (8).  This
 * gives problems with fewer output tiles than CUs (few replicas, e.g. the
 * adjoint's R = 64) enough workgroups.  0 (the default) chooses
 * automatically: a split only when the tile is chosen automatically and its
 * tiles number fewer than the CUs, enough ranges (at most 8, each at least
 * 128 deep) to give every CU two workgroups; the adjoint's backward product
 * follows the same rule for its 32 x 32 tiles.  1 turns the split off; 2..16
 * force it.  Results are deterministic, but the split changes the order of
 * the FP32 sums (so trajectories differ from unsplit ones by rounding).
 * SI_ERR_INVALID outside 0..16; SI_ERR_UNSUPPORTED for 2..16 on a batch, a
 * BF16 form or a tile without a split form. */
si_status spring_ising_set_ksplit(si_ctx *ctx, int32_t ksplit);

/* Execute run() calls of at least min_steps steps as one resident launch
 * (FP32 single instance; the per-step loop of Eq. (8) moved onto the device):
 * every workgroup owns one output tile for the whole call and keeps that
 * tile's q and p in registers, only q (which every other tile's coupling
 * product reads) passes through memory, and a grid-wide barrier separates
 * consecutive steps.  Used only when all workgroups of the step kernel in
 * use fit on the device at once (cooperative launch); otherwise run()
 * launches per step.  Results are bit-identical to per-step launches.  A
 * resident run() returns after the launch has completed, having checked the
 * barrier's time-out flag: a barrier that does not open within about 2 s
 * ends the launch and poisons the context (SI_ERR_HIP).  The barrier costs
 * about as much as a kernel launch, so the resident form pays off only for
 * small, launch-bound problems (a few dozen workgroups).  0 (the default)
 * turns it off.  SI_ERR_INVALID if min_steps < 0. */
si_status spring_ising_set_resident(si_ctx *ctx, int32_t min_steps);

/* Autotuner: time `steps` steps of every step kernel that can serve this
 * context (its precision and padded shape; on a batch, both batch tiles),
 * starting from the current state, in two rounds over all candidates (each
 * candidate keeps its faster round), restore the state after each run, and
 * keep the fastest for later steps.  The choice is also stored in the
 * process's tile cache under this context's key, so that later contexts of
 * that key created with tile 0 start on it.  *best_tile and *best_us (host,
 * nullable) receive the choice and its time per step.  Kernels with a
 * different MFMA shape add the contraction in a different order, so later
 * trajectories may differ in the last bits (the two batch tiles never do).
 * Synchronises once per candidate.  The paper streams the replicas of
 * independent tests through one feature map (Methods, hardware
 * implementation); the tile that maps them best is measured here. */
si_status spring_ising_autotune(si_ctx *ctx, int32_t steps, int32_t *best_tile, float *best_us);

/* Timeline of the batched step (tracing of the grouped launch that runs the
 * paper's independent tests side by side, Fig. 3): runs n_steps steps (1..16)
 * of a batch exactly as run() does, and records for every work item of every
 * step when its workgroup started and ended on the device's real-time clock
 * and which CU ran it.  The results are bit-identical to run(n_steps).
 *   out      : host, at least n_steps * (work items) records of 4 uint64:
 *              {start, end, CU, step << 32 | item}, step-major; CU is
 *              XCC_ID << 16 | bits 15:8 of the wave's HW_ID register.
 *   cap      : records out holds; *n_records (host, nullable) receives the
 *              count needed, also when cap is too small (SI_ERR_INVALID).
 *   clock_mhz: host, nullable: the clock's rate.
 * SI_ERR_UNSUPPORTED on a single-instance context, SI_ERR_RANGE past the
 * schedule.  Synchronises once. */
si_status spring_ising_batch_timeline(si_ctx *ctx, int32_t n_steps, uint64_t *out, int64_t cap,
                                      int64_t *n_records, double *clock_mhz);

/* Tile cache of the process (shared by every context and thread; library
 * bookkeeping with no counterpart in the paper).  Key:
 *   single instance: (precision, N-bucket, R rounded up to 64, CU count);
 *   batch: (precision, bucket of the sum of the padded N_i, bucket of the
 *          largest padded N_i, R rounded up to 64, CU count);
 * the N-bucket of x is b with 2^(b-1) < x <= 2^b.  Value: tile id and its
 * time per step.  autotune writes it; init and init_batch with tile 0 read
 * it.  The file form is text:
 *   line 1: "# spring_ising tile cache 1"
 *   line 2: "build <build id>"
 *   then one line per entry: "<kind> <precision> <nb> <mb> <r64> <cus>
 *   <tile> <us>" (kind 0: single instance, mb 0; kind 1: batch).
 * save writes every entry (SI_ERR_INVALID if the file cannot be written).
 * load merges a file's entries into the cache and sets *n_loaded (host,
 * nullable): SI_ERR_INVALID, with nothing loaded, for a file that does not
 * parse or names a tile that cannot serve its key; SI_ERR_STATE, with
 * nothing loaded, for a file written by another build (tile ids may differ).
 * clear empties the cache. */
si_status spring_ising_tile_cache_save(const char *path);
si_status spring_ising_tile_cache_load(const char *path, int32_t *n_loaded);
si_status spring_ising_tile_cache_clear(void);

/* Readout: the spins are the signs of the final positions (Methods: the
 * oscillators' positions are sampled as the Ising spins):
 * s[r*n + i] = +1 if q_i >= 0 (also -0.0), else -1 (device int8). */
si_status spring_ising_spins(si_ctx *ctx, int8_t *s);

/* Eq. (1) energy of the current spins s = sign(q), per replica.
 *   e_int : device, r int32, or NULL.  Exact; needs integer J (|J_ij| <= 127)
 *           and an integer field, else SI_ERR_UNSUPPORTED.
 *   e_real: device, r doubles, or NULL.  For integer J it equals e_int; for
 *           real J it is an FP32 product with a compensated FP32 sum.
 * On a batch every instance is computed in two grouped launches (integer
 * instances, then real ones), with the values of its single-instance call. */
si_status spring_ising_energy(si_ctx *ctx, int32_t *e_int, double *e_real);

/* Allocation-free variant of spring_ising_energy, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops): the exact int32 energy of Eq. (1), per replica, of s = sign(x)
 * (+1 for x >= 0, also -0.0) for caller-owned couplings and positions, with
 * no context.
 *   n, r : 1 <= n <= 65536 and 1 <= r <= 65536; SI_ERR_INVALID beyond.
 *   J    : device, n*n floats, row-major, symmetric with a zero diagonal
 *          (not checked) and integer entries |J_ij| <= 127; any other entry
 *          makes every e_int entry INT32_MIN.
 *   x    : device, r*n floats, replica-major positions (x[r*n + i]).
 *   e_int: device, r int32; INT32_MIN where the energy does not fit in int32.
 * Its scratch memory (per-replica sums, 512 KiB) is one static device array
 * per GPU, held until the process ends; every call clears the part it uses
 * before using it.  Calls that overlap on one GPU (on different streams)
 * share that array and race.  Nothing is allocated or freed and no
 * allocating library routine is called.  Asynchronous on hip_stream (NULL =
 * null stream). */
si_status spring_ising_energy_noalloc(int32_t n, int32_t r, const float *J, const float *x,
                                      int32_t *e_int, void *hip_stream);

/* Best state seen along the trajectory (the paper samples the spins of the
 * final state, Methods; tracking the lowest energy met on the way, Fig. 4,
 * keeps the best of them): evaluate the Eq. (1) energy of the current spins
 * (exactly for integer J, else as the real energy) and keep, per replica,
 * the lowest value seen since init or the last set_state together with its
 * spins.  Also done by every in-run energy check (si_params.energy_every).
 * On a batch, per instance and replica. */
si_status spring_ising_update_best(si_ctx *ctx);

/* Copy the recorded best energies (device, r doubles; a batch: n_inst*r,
 * instance i's replicas at offset r*i) and spins (device, r*n int8,
 * replica-major; a batch: concatenated as at init_batch); either may be
 * NULL.  SI_ERR_STATE if no best-state update was issued since init or the
 * last set_state. */
si_status spring_ising_get_best(si_ctx *ctx, double *best_e, int8_t *best_s);

/* Energy trace of the in-run checks (si_params.energy_every = E > 0; the
 * Eq. (1) energy followed over the iterations, as in Fig. 4): copy
 * the rows recorded for the checks at steps E, 2E, ... <= t into e (device,
 * doubles, row k holding the energies of check k: r values, or n_inst*r on
 * a batch in the order of spring_ising_energy), and the number of rows to
 * *n_checks (host, may be NULL).  e may be NULL to query the count.  The
 * values are exact integers for integer J (and field).  SI_ERR_STATE if the
 * context was created with E = 0. */
si_status spring_ising_get_energy_trace(si_ctx *ctx, double *e, int32_t *n_checks);

/* Hamiltonian of the spring system, Eq. (7), per replica (device, r
 * doubles): sum_i p_i^2/(2m) + k q_i^2/2 + zeta_t H_Ising(q) with the
 * continuous Ising energy H_Ising(q) = -1/2 q^T J q - h.q and zeta_t the
 * schedule value of the current step (the last one once the run is over).
 * FP32 products, compensated FP32 sums. */
si_status spring_ising_hamiltonian(si_ctx *ctx, double *H);

/* Copy the state out: the positions q (x) and momenta p of Eq. (8) after
 * t steps, device r*n floats each (replica-major; either may be NULL), and
 * *t (host, may be NULL) the step index.  On a batch the instances are
 * concatenated as described at init_batch. */
si_status spring_ising_get_state(si_ctx *ctx, float *x, float *p, int32_t *t);

/* Overwrite the state (q, p) of Eq. (8) and the step index: x, p device
 * r*n floats (p may be NULL for zeros), 0 <= t <= total_steps, so that the
 * next step uses Delta_t, zeta_t.  Resuming from a state saved with
 * get_state is bit-identical to an uninterrupted run.  Resets the best-state
 * record of update_best. */
si_status spring_ising_set_state(si_ctx *ctx, const float *x, const float *p, int32_t t);

/* Gradient of the relaxed end-energy with respect to the step schedules
 * (adjoint; the paper gives the forward iteration only, Eq. (8), and its
 * walls, Eq. (6) and Methods).  From the current state at step t0 the
 * context runs the remaining total_steps - t0 steps (ending there, as run()
 * would) and evaluates
 *   loss = (1/R) sum_r -1/2 q_r^T J q_r   (final positions, field excluded)
 * and dloss/ddt[n], dloss/dzeta[n] for every step n >= t0 (entries n < t0
 * are set to 0).  Reverse mode with checkpoints every ckpt_every steps and
 * a recomputed forward per segment; the clamp derivative is 1 on the closed
 * interval.  The per-step inner products are accumulated in FP64.
 *   loss  : device, 1 double.
 *   dL_ddt, dL_dzeta: device, total_steps doubles each.
 * Supported for the paper order, clamping walls, FP32 precision and no
 * field; otherwise SI_ERR_UNSUPPORTED.  Allocates its workspace on first use
 * (about (C + 1 + 2 (S - t0)/C) state copies, C = min(ckpt_every, S - t0)). */
si_status spring_ising_relaxed_energy_grad(si_ctx *ctx, int32_t ckpt_every, double *loss,
                                           double *dL_ddt, double *dL_dzeta);

/* The same gradient in two halves, for callers that evaluate the loss first
 * and ask for its gradient later (an autograd function's forward and
 * backward).  relaxed_energy_forward runs the remaining steps with
 * checkpoints every ckpt_every steps, writes loss (device, 1 double) and
 * records a tape in the context: the checkpoints, the seed of the reverse
 * sweep, the start step t0 and the context's state epoch.  Every call that
 * changes the trajectory (set_schedule, set_field, set_state, step, run,
 * set_ksplit, autotune) advances the epoch.
 * relaxed_energy_backward runs the reverse sweep over that tape and writes
 * dL_ddt, dL_dzeta (device, total_steps doubles each, entries n < t0 set to
 * 0).  It consumes the tape: without a forward half since the last change of
 * the trajectory, or a second time after one, it returns SI_ERR_STATE and
 * writes nothing.  Conditions and workspace as for relaxed_energy_grad,
 * whose results equal forward followed by backward bit for bit. */
si_status spring_ising_relaxed_energy_forward(si_ctx *ctx, int32_t ckpt_every, double *loss);
si_status spring_ising_relaxed_energy_backward(si_ctx *ctx, double *dL_ddt, double *dL_dzeta);

/* Fill *info (host). */
si_status spring_ising_info(si_ctx *ctx, si_info *info);

/* Release every device buffer of the context (waits for its stream). */
si_status spring_ising_destroy(si_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). */
const char *spring_ising_last_error(void);

/* Build id of this library: 16 hex digits of a hash over the sources and
 * compiler flags it was built from (static string). */
const char *spring_ising_build_id(void);

/* Test hook for callers' error handling: the n-th HIP call that the context
 * checks after this call (n >= 1) reports a failure although the call itself
 * succeeded, which poisons the context exactly as a real HIP failure does
 * (that call returns SI_ERR_HIP, every later call other than destroy
 * SI_ERR_STATE).  No device operation is altered.  n = 0 cancels a pending
 * injection; SI_ERR_INVALID if n < 0. */
si_status spring_ising_debug_inject_hip_error(si_ctx *ctx, int32_t n);

#ifdef __cplusplus
}
#endif
#endif /* SPRING_ISING_H */
