/*
 * mdeos.h -- C ABI of libmdeos, an MI355X (gfx950) engine for the in-line
 * molecular-dynamics equation of state of arXiv 2508.06012.
 *
 * The paper closes the Euler equations with p = f(rho, e) (Sec. II.A,
 * Eq. EOS) evaluated by an independent MD run at every quadrature point and
 * every time step (Sec. III). One such evaluation here is a "cell": the
 * lifting operator maps (rho, e) to a periodic FCC box of N = 4 n_c^3 atoms
 * with velocities that carry the energy e above the cold lattice (Sec. III,
 * Eqs. numdens, numAtoms, Tcontribution); the box is advanced with velocity
 * Verlet or the GJF Langevin integrator (Sec. II.B), for a truncated-shifted
 * Lennard-Jones fluid or a many-body material of the embedded-atom form
 * (Eq. Etot) in reduced units; the restricting operator returns the time
 * average of one third of the trace of the kinetic + virial stress (Sec. III,
 * Eq. stress), the full stress tensor and the temperature, with block
 * standard errors.
 *
 * Conventions for every call:
 *   - Host arrays passed in are read during the call only; host arrays passed
 *     out are written before the call returns. Per-atom host arrays are
 *     row-major [N][3] doubles. The library owns all device memory.
 *   - `stream` is a hipStream_t (NULL = the context's own stream). Calls that
 *     return host results synchronise that stream.
 *   - Call-level errors are negative mdeos_status values. Per-cell failures
 *     are MDEOS_CELL_* bits in mdeos_result.status; a batch call returns
 *     MDEOS_OK even when some cells failed.
 *   - A context is used by one thread at a time, except the serving calls,
 *     which are thread-safe.
 *
 * Diagnostic environment switches, read when a context is created:
 *   MDEOS_FORCE_VARIANT="block,apt,ext,list_lds,wpe,mi[,nvt,eam]" runs every
 *     bucket the shape fits with that launch shape (no tuning);
 *   MDEOS_TUNE_LOG=1 prints the autotuner's timings to stderr;
 *   MDEOS_SHRINK_CAPS=1 plans every cell with a tiny neighbour capacity, so
 *     the batch paths' capacity retry runs.
 */
#ifndef MDEOS_H
#define MDEOS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int mdeos_status;

/* call-level status */
#define MDEOS_OK 0
#define MDEOS_INVALID_ARG (-1)
#define MDEOS_OUT_OF_MEMORY (-2)
#define MDEOS_DEVICE_ERROR (-3)
#define MDEOS_NOT_READY (-4)
#define MDEOS_ADMISSION_FULL (-5)
#define MDEOS_NO_DEVICE (-6)

/* per-cell status bits (mdeos_result.status) */
#define MDEOS_CELL_NONFINITE 1          /* K, W or E_pot became NaN/Inf; the cell stopped */
#define MDEOS_CELL_ENERGY_BELOW_COLD 2  /* a re-pin found N e <= E_pot - E_cold; no rescale */
#define MDEOS_CELL_DRIFT 4              /* |E(n) - E(n - n_avg)| / N > drift_tol */
#define MDEOS_CELL_OVERFLOW 8           /* neighbour or ghost capacity exceeded; the cell stopped */
#define MDEOS_CELL_COLD_RELIFT 16       /* warm start fell back to a cold lift */

#define MDEOS_MAX_RESCALE 8
#define MDEOS_MAX_BLOCKS 16
#define MDEOS_MAX_NC 10                 /* N <= 4000 atoms per box */

/* One EOS query (lifting-operator input, Sec. III). */
typedef struct {
    double rho;               /* reduced number density rho* > 0 (n = rho in reduced units) */
    double e;                 /* specific internal energy per atom above the cold lattice, > 0 */
    int n_c;                  /* FCC cells per edge, 1..MDEOS_MAX_NC; N = 4 n_c^3 */
    float rc;                 /* cutoff of the context's potential, 0 < rc < L */
    double dt;                /* MD time step, > 0 */
    unsigned long long seed;  /* Philox4x64-10 key word 0 */
    long long cell_id;        /* Philox4x64-10 key word 1 (and the caller's cell label) */
} mdeos_cell_spec;

/* Run schedule of one query. */
typedef struct {
    int n_steps;                          /* MD steps after the lift, >= 1 */
    int n_avg;                            /* samples averaged: steps n_steps-n_avg+1 .. n_steps */
    int n_blocks;                         /* blocks for the standard error, 2..MDEOS_MAX_BLOCKS, divides n_avg */
    int n_rescale;                        /* 0..MDEOS_MAX_RESCALE energy re-pins (Eq. Tcontribution) */
    int rescale_steps[MDEOS_MAX_RESCALE]; /* each in [0, n_steps - n_avg]; 0 = right after the lift */
    int energy_every;                     /* E_pot is computed on steps divisible by this (>= 1) */
    double drift_tol;                     /* per-atom production drift that sets MDEOS_CELL_DRIFT */
    int ensemble;                         /* MDEOS_NVE_REPIN (default) or MDEOS_NVT_LANGEVIN */
    double gamma;                         /* Langevin friction for MDEOS_NVT_LANGEVIN (>= 0) */
} mdeos_schedule;

/* Integration and equilibration (Sec. II.B, Sec. III).
 * MDEOS_NVE_REPIN: velocity Verlet; at each rescale step the kinetic energy
 *   is set to N e - (E_pot - E_cold) (Eq. Tcontribution with the
 *   instantaneous E_pot); production is energy-conserving.
 * MDEOS_NVT_LANGEVIN: the GJF Langevin integrator (friction gamma, unit
 *   mass) thermostats at T_th, first 2 N e / N_DOF (all energy kinetic). At
 *   each rescale step, Eq. Tcontribution with E_pot averaged over the second
 *   half of the segment since the previous one (steps divisible by
 *   energy_every, and the rescale step itself) gives the new temperature; the
 *   velocities are scaled to it and it becomes T_th. Production is canonical
 *   at the last T_th; the drift status does not apply. Noise: Philox4x64-10
 *   keyed (seed, cell_id) at counter (atom, step, 1, 0), Box-Muller giving
 *   three normal numbers per atom and step. */
enum { MDEOS_NVE_REPIN = 0, MDEOS_NVT_LANGEVIN = 1 };

/* Restricted result of one query (restricting operator, Sec. III). */
typedef struct {
    double P;          /* <P> = <(2K + W) / (3V)> over the averaging window */
    double P_se;       /* block standard error of <P> */
    double P_rms;      /* RMS deviation of the instantaneous P from <P> */
    double T;          /* <T> = <2K / (3N - 3)> */
    double T_se;       /* block standard error of <T> */
    double Epot_mean;  /* <E_pot> / N over energy steps in the window */
    double Ecold;      /* E_cold / N of the static lattice at rho */
    double drift;      /* (E(n) - E(n - n_avg)) / N; NaN before step n */
    double pairs;      /* ordered pairs within rc per step, averaged over energy steps */
    int n_samples;     /* samples averaged */
    int status;        /* MDEOS_CELL_* bits */
    int n_builds;      /* neighbour-list builds */
    int max_list;      /* largest neighbour count seen (capacity diagnostics) */
    int max_ext;       /* largest real + ghost atom count seen */
    int reserved;
    double stress[6];  /* <sigma> of Eq. stress, (xx, yy, zz, xy, xz, yz): (sum m v_a v_b + sum over pairs
                          d_a f_b) / V, pressure convention (trace / 3 = P), averaged over the window
                          steps where E_pot is sampled */
} mdeos_result;

typedef struct {
    int device;                /* HIP device ordinal */
    size_t hbm_budget;         /* bytes of resident cell state the context may hold; 0 = 64 GiB */
    float skin;                /* Verlet skin; <= 0 selects, per cell, the measured best: LJTS 0.3 up
                                  to 150 atoms, 0.4 up to 600 atoms or for rc > 3.5, 0.6 above (0.4
                                  if the extended box does not fit at 0.6); MDEOS_POT_EAM 0.5 up to
                                  1000 atoms and 0.3 above */
    int autotune;              /* 1 = time candidate launch shapes on first use of a bucket */
    const char* tune_cache;    /* JSON file of tuned launch shapes (read and written); NULL = none */
    int precision;             /* how each atom sums its pair energies and virials (forces are FP32):
                                  MDEOS_PREC_FP64 (default) or MDEOS_PREC_KAHAN */
    int potential;             /* the material of every cell of the context: MDEOS_POT_LJTS (default)
                                  or MDEOS_POT_EAM */
    double eam_c;              /* embedding strength c of MDEOS_POT_EAM; <= 0 selects 39.432 */
    float prune_skin;          /* MDEOS_POT_EAM: inner-list skin s_in. Between list builds, every time
                                  an atom has moved s_in / 2, the force walks switch to the list entries
                                  within rc + s_in. Results are bit-identical with and without (dropped
                                  entries add exact zeros). 0 selects 0.12; < 0 turns it off. No effect
                                  when s_in >= skin, for lists held in LDS, with MDEOS_PREC_KAHAN, or for
                                  MDEOS_POT_LJTS (whose shapes are built without inner lists).
                                  NaN or infinity: MDEOS_INVALID_ARG. */
} mdeos_config;

/* Per-atom accumulation of pair energy and virial terms. The box sums that
 * follow are FP64 in both modes. */
enum { MDEOS_PREC_FP64 = 0, MDEOS_PREC_KAHAN = 1 };

/* Interatomic potential, in reduced units with unit atomic mass.
 * MDEOS_POT_LJTS: Lennard-Jones truncated and shifted at the cell's rc
 *   (energy eps = 1, length sigma = 1).
 * MDEOS_POT_EAM: the embedded-atom form of Eq. Etot (appendix),
 *   E_pot = 1/2 sum_{i != j} V(r_ij) + sum_i F(rhobar_i), rhobar_i = sum_{j != i} f(r_ij),
 *   with the analytic Sutton-Chen functions V = r^-9, f = r^-6 and
 *   F = -c sqrt(rhobar) (energy eps = 1, length = the lattice parameter a of
 *   the fitted crystal; c = 39.432 is the published copper value) standing
 *   in for the paper's tabulated copper potential. V and f are truncated at
 *   the cell's rc in shifted-force form, g(r) - g(rc) - (r - rc) g'(rc), so
 *   forces are continuous there. Densities are atoms per a^3 (4 at the
 *   fitted lattice). For copper (a = 3.6153 A, eps = 0.012382 eV, 63.546 u)
 *   the time unit is 2.64 ps, the pressure unit 0.0420 GPa and the
 *   temperature unit 143.7 K. */
enum { MDEOS_POT_LJTS = 0, MDEOS_POT_EAM = 1 };

typedef struct mdeos_ctx mdeos_ctx;
typedef long long mdeos_handle;

/* Shape of the device work for one cell, as planned on the host. */
typedef struct {
    int N;            /* atoms */
    float L;          /* box edge */
    float rl;         /* neighbour-list radius rc + skin */
    int ext_cap;      /* real + ghost atom capacity */
    int list_cap;     /* neighbour capacity per atom (multiple of 8) */
    int ncell;        /* binning cells over the extended box */
    int lds_bytes;    /* LDS bytes the cell needs */
    int list_in_lds;  /* 1 if the neighbour list lives in LDS, 0 if in device memory */
    int multi_image;  /* 1 if rc > L/2 (several periodic images of one atom are in range) */
} mdeos_plan_info;

/* ---- host-only calls (no device needed) ---------------------------------- */

const char* mdeos_strerror(mdeos_status s);
/* Message of the last failed call on this thread ("" if none). */
const char* mdeos_last_error(void);
const char* mdeos_version(void);
/* Validates a query and its schedule; MDEOS_OK or MDEOS_INVALID_ARG. */
mdeos_status mdeos_validate(const mdeos_cell_spec* spec, const mdeos_schedule* sched);
/* Plans the device work of one query (capacities, LDS bytes, variant) at
   Verlet skin `skin`; skin <= 0 selects the LJTS default of mdeos_config. */
mdeos_status mdeos_plan(const mdeos_cell_spec* spec, float skin, mdeos_plan_info* out);
/* Device bytes one resident cell of n_c holds (used for HBM admission). */
size_t mdeos_cell_bytes(int n_c);
/* Number of visible HIP devices (0 when none or on a host without ROCm devices). */
int mdeos_device_count(void);

/* ---- context ------------------------------------------------------------ */

mdeos_status mdeos_create(const mdeos_config* cfg, mdeos_ctx** out);
mdeos_status mdeos_destroy(mdeos_ctx* ctx);

/* ---- lift / advance / restrict (Sec. III) --------------------------------- */

/* Lifting operator: for each spec, builds the FCC lattice (Eq. numdens), its
 * cold energy, Gaussian velocities at T0 = 2 N e / (3N - 3) with zero net
 * momentum, scaled so K = N e exactly, and the initial forces. Handles of the
 * new resident cells are written to out[n]. Cells follow `sched`. */
mdeos_status mdeos_lift(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched,
                        mdeos_handle* out, void* stream);

/* Lifts one cell from a given state instead of the lattice draw: xyz and v
 * ([N][3] doubles; positions are wrapped into [0, L)).
 * E_cold is always computed from the lattice at spec->rho. */
mdeos_status mdeos_lift_from_state(mdeos_ctx* ctx, const mdeos_cell_spec* spec, const mdeos_schedule* sched,
                                   const double* xyz, const double* v, mdeos_handle* out, void* stream);

/* Re-targets resident cells to a new (rho, e) with a warm start: positions
 * are dilated by L'/L (Eq. numdens at the new density), E_cold is recomputed
 * at rho', forces are recomputed and the energy is re-pinned to e' at step 0
 * of `sched` (which must list step 0). If the re-pin finds no kinetic energy
 * left the cell is lifted cold instead (MDEOS_CELL_COLD_RELIFT). */
mdeos_status mdeos_warm_start(mdeos_ctx* ctx, int n, const mdeos_handle* h, const double* rho, const double* e,
                              const mdeos_schedule* sched, void* stream);

/* Microscopic model (Sec. II.B): advances each cell by up to n_steps MD steps
 * (velocity Verlet, or the GJF Langevin integrator the paper cites, as its
 * schedule's ensemble says; never past the schedule's end), with the
 * temperature updates of Eq. Tcontribution (Sec. III) at the schedule's
 * steps, in one persistent launch per size bucket. h[n] are handles of
 * resident cells (MDEOS_INVALID_ARG for a stale or unknown handle).
 * n_steps = 0 runs only a pending lift or warm-start phase; n_steps < 0 is
 * MDEOS_INVALID_ARG. Asynchronous on the stream. */
mdeos_status mdeos_advance(mdeos_ctx* ctx, int n, const mdeos_handle* h, int n_steps, void* stream);

/* Restricting operator (Sec. III, Eq. stress): writes one result per handle
 * into out[n] (host memory; blocks on the stream). Cells that have not
 * reached the end of their schedule make the call return MDEOS_NOT_READY;
 * their results hold the averages of the window samples recorded so far
 * (n_samples of them), block errors over the completed blocks only (NaN with
 * fewer than two) and a NaN drift. */
mdeos_status mdeos_restrict(mdeos_ctx* ctx, int n, const mdeos_handle* h, mdeos_result* out, void* stream);

/* One equation-of-state evaluation per spec, the equation-free coupling of
 * Sec. III (lifting, microscopic model of Sec. II.B, restriction): lift +
 * full schedule + restrict for n cells, with one persistent launch per size
 * bucket, replayed from a cached HIP graph for repeated batch shapes.
 * specs[n] and out[n] are host arrays read / written during the call; the
 * call blocks until out is written. Per-cell failures are status bits of
 * out[i]; invalid specs or schedules fail the whole call with
 * MDEOS_INVALID_ARG before any device work. The cells are released
 * afterwards. */
mdeos_status mdeos_eval_batch(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched,
                              mdeos_result* out, void* stream);

/* The plain path: the same kernels, one cell per launch, cells one after
 * another on one stream. */
mdeos_status mdeos_eval_plain(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs, const mdeos_schedule* sched,
                              mdeos_result* out, void* stream);

/* For callers that cannot allocate memory: code under HIP graph capture of
 * their own work around it, tight serving loops, harnesses that forbid
 * allocation. The same evaluation as mdeos_eval_batch (lift + full schedule +
 * restrict; the same results, bit for bit), without allocating anything: no
 * hipMalloc / hipHostMalloc / hipFree, no HIP graphs, no C++ heap. Every
 * device buffer the kernels use beyond specs and out lives in a static
 * workspace of MDEOS_NOALLOC_SCRATCH_MIB MiB per GPU (held by each GPU the
 * library runs on until the process ends); host staging is static too.
 * Limits (MDEOS_INVALID_ARG beyond them, with mdeos_last_error saying which):
 * n <= MDEOS_NOALLOC_MAX_CELLS; at most 16 groups of (atom count, image
 * method); cell records, the atom state (72 B per atom), work lists and
 * device-memory neighbour lists of at least one workgroup per group must fit
 * the workspace (fewer workgroups are launched when the lists of more would
 * not). No autotuning (the static launch-shape model) and no capacity retry:
 * a cell that outgrows its planned capacities reports MDEOS_CELL_OVERFLOW.
 * Uses ctx's device, stream, potential, precision and skins. specs[n] and
 * out[n] are host arrays; blocks until out is written. Calls on one GPU share
 * its workspace, which keeps the last call's contents: calls that overlap on
 * one GPU would race, so this library serializes the calls of a process and
 * returns only after their device work has ended. */
#define MDEOS_NOALLOC_SCRATCH_MIB 64
#define MDEOS_NOALLOC_MAX_CELLS 4096
mdeos_status mdeos_eval_batch_noalloc(mdeos_ctx* ctx, int n, const mdeos_cell_spec* specs,
                                      const mdeos_schedule* sched, mdeos_result* out, void* stream);

mdeos_status mdeos_release(mdeos_ctx* ctx, int n, const mdeos_handle* h);

/* Device time (ms, from HIP events on the launch stream) of the last
 * persistent advance launch set of this context (all size buckets of one
 * eval_batch / advance call), and the number of bucket launches in it. */
mdeos_status mdeos_last_advance_time(mdeos_ctx* ctx, double* ms, int* n_launches);

/* Copies a resident cell's state to the host: positions wrapped into [0, L),
 * velocities, and the number of steps completed. Any pointer may be NULL. */
mdeos_status mdeos_state_export(mdeos_ctx* ctx, mdeos_handle h, double* xyz, double* v, int* step);

/* ---- parity hooks --------------------------------------------------------- */

/* Forces, potential energy and pair virial sum W = sum_pairs r.f for the
 * given positions ([N][3], rounded to float, wrapped) of a box described by
 * spec (N = 4 n_c^3, L from rho), through the same neighbour build and force
 * kernel as the MD path. F ([N][3]) may be NULL. */
mdeos_status mdeos_debug_forces(mdeos_ctx* ctx, const mdeos_cell_spec* spec, const double* xyz, double* F,
                                double* U, double* W);

/* Advances a resident cell by n_steps, one launch per step, with E_pot
 * computed every step, and records forces (F: (n_steps+1) x N x 3, may be
 * NULL) and K, U, W (n_steps+1 each, may be NULL) for the starting state and
 * after each step. A pending lift or warm start runs first, so the starting
 * state of a warm-started cell is the re-targeted one (after its step-0
 * re-pin). */
mdeos_status mdeos_debug_trajectory(mdeos_ctx* ctx, mdeos_handle h, int n_steps, double* F, double* K, double* U,
                                    double* W);

/* ---- serving (continuous batching) --------------------------------------- */

typedef struct {
    mdeos_schedule cold;  /* schedule of a cell's first query (cold lift) */
    mdeos_schedule warm;  /* schedule of later queries (warm start; must list step 0) */
    float rc;             /* cutoff of every served cell */
    double dt;            /* time step of every served cell */
    unsigned long long seed;
    int chunk_steps;      /* MD steps per scheduling round, >= 1 */
    int max_slots;        /* cap on cells advancing at once (0 = as many as HBM allows) */
} mdeos_serve_config;

typedef struct {
    long long submitted, completed, cold, warm, relifts, evictions;
    long long chunks;          /* scheduling rounds launched */
    long long queued;          /* queries waiting now */
    long long active;          /* cells advancing now */
    long long resident;        /* cells with resident state now */
    size_t resident_bytes;     /* device bytes of resident state */
    double atom_steps;         /* MD atom-steps executed */
} mdeos_serve_stats;

/* Starts the scheduler thread. Cells left resident by an earlier session
 * (a stop keeps them) are released first: every session starts cold. */
mdeos_status mdeos_serve_start(mdeos_ctx* ctx, const mdeos_serve_config* cfg);
/* Queues one EOS query for cell `cell_id` at time t_arrival (seconds on the
 * caller's clock, see mdeos_serve_now). Queries of one cell run in order,
 * each warm-started from the previous one's final state. */
mdeos_status mdeos_serve_submit(mdeos_ctx* ctx, long long cell_id, double rho, double e, int n_c, double t_arrival,
                                long long* ticket);
/* Returns up to max finished queries: tickets, results and completion times. */
mdeos_status mdeos_serve_poll(mdeos_ctx* ctx, int max, long long* tickets, mdeos_result* out, double* t_done,
                              int* n_out);
/* Seconds on the serving clock (monotonic, zero at mdeos_serve_start). */
double mdeos_serve_now(mdeos_ctx* ctx);
mdeos_status mdeos_serve_stats_get(mdeos_ctx* ctx, mdeos_serve_stats* out);
/* Finishes queued work (drain = 1) or drops it (drain = 0) and joins the thread. */
mdeos_status mdeos_serve_stop(mdeos_ctx* ctx, int drain);

#ifdef __cplusplus
}
#endif

#endif /* MDEOS_H */
