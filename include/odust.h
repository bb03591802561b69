/*
 * odust.h -- C-ABI of the MI355X dust-in-ion-flow library (libodust.so).
 *
 * The library advances the self-consistent model of Kolotinskii & Timofeev,
 * "OpenDust: A fast GPU-accelerated code for calculation forces, acting on
 * microparticles in a plasma flow" (arXiv 2205.06557): ion superparticles in
 * a cylinder (Section 2), electron-screened (Yukawa) ion-ion forces and bare
 * Coulomb ion-dust forces, a staggered leapfrog push, constant-frequency
 * charge exchange with neutrals, absorption of ions by fixed dust grains with
 * the grain charge update, and flux-conserving reinjection of lost ions on
 * the boundary (Appendix B).  The per-grain observables are the charge and
 * the four force parts of Eqs. (1)-(4).
 *
 * Conventions
 *  - Inputs follow the paper's parameter objects (Section 3): SI units.
 *  - Pointers named *host* are host memory owned by the caller; the library
 *    copies what it needs during the call.  All device memory belongs to the
 *    library (hipMalloc, or the caller's allocator, see od_allocator).
 *  - Every call returns od_status.  On failure od_last_error() returns a
 *    thread-local message.  Kernels report numerical trouble (a NaN in a
 *    charge or force, a failed initial placement, fixed-point overflow)
 *    through a device status word; it is read, and returned as OD_ENUMERIC /
 *    OD_ESTATE, by the next call that synchronises (od_sync, od_get_*).
 *  - od_step is asynchronous on the system's HIP stream.
 *  - A system is used by one host thread at a time; distinct systems are
 *    independent.
 */
#ifndef ODUST_H
#define ODUST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OD_OK = 0,
    OD_EINVAL = -1,     /* invalid argument or parameter combination      */
    OD_EDEVICE = -2,    /* a HIP call failed                              */
    OD_ENUMERIC = -3,   /* NaN/Inf or overflow detected on the device     */
    OD_ESTATE = -4,     /* invalid state (e.g. an ion could not be placed) */
    OD_ENOMEM = -5      /* allocation failed                              */
} od_status;

/* Charging models of Section 2 ("given", "oml", "consistent"); one model for
 * all grains (Section 3). */
typedef enum {
    OD_CHARGE_GIVEN = 0,
    OD_CHARGE_OML = 1,
    OD_CHARGE_CONSISTENT = 2
} od_charge_mode;

/* od_sim.flags */
#define OD_FLAG_LITERAL_SIDE 1u  /* side injection with radial + axial velocity only
                                    (Eqs. B.10-B.11 as printed); default adds the
                                    tangential thermal component Eq. (B.1) implies */
#define OD_FLAG_NO_ION_ION 2u    /* test-particle mode: ion-ion force switched off */
#define OD_FLAG_CONFINEMENT 4u   /* confinement field of the plasma outside the domain
                                    (Appendix A): computed once, from the ions placed by
                                    initialisation, and added to every ion's acceleration
                                    and, as Q_d E_out, to the force of Eq. (1) */
#define OD_FLAG_FIELD_DRIVEN 8u  /* field-driven collisional flow: initial and injected v_z
                                    follow the flow's stationary distribution, a Gaussian of
                                    width sigma convolved with an exponential of mean a/nu
                                    (a = eE/m_i), the phi(v_z) of Eq. (B.1) for this flow;
                                    without it v_z is N(M c_s, sigma^2).  Needs nu_in > 0 and
                                    a/nu > sigma/30, else OD_EINVAL */

/* od_sim.precision */
#define OD_PREC_FP32 0           /* FP32 state and pair tiles, FP64 charge/force sums */
#define OD_PREC_FP64 1           /* FP64 state and pair forces throughout              */

#define OD_MAX_DUST 32

/* Plasma parameters (Section 3, plasma parameter classes), SI. */
typedef struct {
    double T_e;      /* electron temperature, K                                    */
    double T_i;      /* ion (and neutral) temperature, K                           */
    double n_inf;    /* ion density of the quasi-neutral plasma, m^-3               */
    double m_i;      /* ion mass, kg                                               */
    double mach;     /* flow speed along +z in units of sqrt(kB T_e / m_i)          */
    double nu_in;    /* ion-neutral charge-exchange frequency, s^-1 (0: collisionless) */
    double E_ext;    /* driving field along +z, V/m; NaN: m_i nu_in u / e           */
} od_plasma;

/* Simulation parameters (Section 3, simulation parameter class), SI. */
typedef struct {
    double R;            /* cylinder radius, m                              */
    double H;            /* cylinder height, m (axis from -H/2 to +H/2)      */
    double dt;           /* time step, s                                    */
    int64_t n_ions;      /* number of ion superparticles N, 2 .. 2^29        */
    int64_t n_discard;   /* steps excluded from the time averages           */
    uint64_t seed;       /* random stream key, word 0                       */
    uint64_t system_id;  /* random stream key, word 1                       */
    int32_t charge_mode; /* od_charge_mode                                  */
    int32_t precision;   /* OD_PREC_FP32 or OD_PREC_FP64                    */
    uint32_t flags;      /* OD_FLAG_*                                       */
    uint32_t reserved;   /* must be 0                                       */
} od_sim;

/* One dust grain (Section 3, dust particle class): fixed position, radius,
 * initial charge. */
typedef struct {
    double x, y, z;      /* m                                               */
    double radius;       /* m                                               */
    double q0;           /* initial charge, C                               */
} od_dust;

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` bytes, 256-byte aligned, or
 * NULL; release gives it back.  Both are called only from od_init_system and
 * od_destroy. */
typedef struct {
    void* (*alloc)(void* ctx, size_t bytes);
    void (*release)(void* ctx, void* ptr);
    void* ctx;
} od_allocator;

typedef struct od_system od_system;

/* Creates a system and draws its initial state on the device: positions
 * uniform in the cylinder outside every grain, velocities from the shifted
 * Maxwellian N((0,0,u), kB T_i/m_i), charges q0 (Section 2).
 *   dust:      n_dust grains, host, 0 <= n_dust <= OD_MAX_DUST;
 *   hip_stream: hipStream_t to run on (NULL: the default stream);
 *   allocator: NULL for hipMalloc/hipFree.
 * Errors: OD_EINVAL (N outside [2, 2^29], non-positive sizes or temperatures,
 * a grain that crosses the wall or overlaps another, bad mode/precision/flags),
 * OD_ENOMEM, OD_EDEVICE (no HIP device visible, or a HIP call failed),
 * OD_ESTATE (an ion could not be placed). */
od_status od_init_system(const od_plasma* plasma, const od_sim* sim, const od_dust* dust,
                         int32_t n_dust, void* hip_stream, const od_allocator* allocator,
                         od_system** out);

/* Advances n_steps >= 0 time steps (Section 2 and Appendix B): forces at the
 * current positions and charges, kick, charge exchange, drift, absorption,
 * exit, charge update, collection force (Eq. 3), reinjection, recording.
 * Asynchronous; returns after the launches are queued. */
od_status od_step(od_system* sys, int64_t n_steps);

/* Waits for the system's stream and returns the device status. */
od_status od_sync(od_system* sys);

/* Dust charges, C: q_now[n_dust] after the last step; q_avg[n_dust] (may be
 * NULL) the mean of the recorded charges over steps >= n_discard. */
od_status od_get_dust_charges(od_system* sys, double* q_now_host, double* q_avg_host);

/* Dust forces, N, f_host[n_dust][4][3]: parts orbit (Eq. 1), dust-dust
 * (Eq. 2), collection (Eq. 3), external field (Eq. 4).
 *   which = 0: the forces recorded at the last step;
 *   which = 1: their means over steps >= n_discard. */
od_status od_get_dust_forces(od_system* sys, int32_t which, double* f_host);

/* Frees the system's device memory. NULL is ignored. */
void od_destroy(od_system* sys);

/* Thread-local text of the last error. */
const char* od_last_error(void);

/* ---- inspection and test surface ---------------------------------------
 * The calls of this section expose the state, the events of a step and the
 * library's own choices (pair kernel, source splits, timing) for tests,
 * measurement and checkpointing.  The paper's interface is the parameter
 * objects and per-grain observables above; a call below cites a passage only
 * where one defines what it returns (the cutoff of Section 4, the
 * confinement field of Appendix A, the absorbed ions and the history of
 * Sections 2 and 3); the others have none. */

/* Units of the dimensionless state: units_host[4] = {length r_De (m),
 * time 1/omega_pi (s), velocity c_s = r_De omega_pi (m/s),
 * acceleration r_De omega_pi^2 (m/s^2)}. */
od_status od_get_units(od_system* sys, double* units_host);

/* Ion-ion cutoff with a switching function (Section 4: the option for long
 * domains, a switching function that is zero beyond a fixed cutoff
 * distance).  The screened Coulomb energy of an ion pair is multiplied by
 * S(r) = 1 for r <= r_switch, 1 - 6x^5 + 15x^4 - 10x^3 with
 * x = (r - r_switch)/(r_cut - r_switch) up to r_cut, and 0 beyond; the ion
 * force is minus the gradient of that energy.  Grain terms and the sum of
 * Eq. (1) stay complete.  Distances in m; r_cut <= 0 returns to the
 * all-pairs sum.  FP32 systems only (OD_EINVAL otherwise); needs
 * 0 <= r_switch < r_cut.  Each step then sorts the ions into slabs along z
 * (width about r_cut / 16, or r_cut / 8 where that would pass 1024 slabs;
 * at most 1024) and evaluates each pair of
 * blocks of 256 sorted ions within reach once (both reactions, int64 fixed
 * point as the symmetric all-pairs kernel).
 * Allocates the sort buffers (about 44 bytes per ion plus 4 bytes per slab
 * and block of 256 ions) with the system's allocator; synchronises the
 * system's stream. */
od_status od_set_cutoff(od_system* sys, double r_switch, double r_cut);

/* Cutoff bookkeeping of the last step: *nslab slabs and *pairs_evaluated,
 * the ordered ion pairs the cutoff kernel covered (each pair of 256-ion
 * blocks counted both ways, padding included).  OD_ESTATE without a cutoff.
 * Synchronises. */
od_status od_get_cutoff_info(od_system* sys, int32_t* nslab, int64_t* pairs_evaluated);

/* Confinement field of a system created with OD_FLAG_CONFINEMENT (Appendix A).
 * At creation the potential of Eq. (A.1) -- the screened potential
 * k_B T_e / e of an infinite homogeneous ion background minus the screened
 * Coulomb potential of the initial ions -- is computed on the grid of
 * Eq. (A.2), nodes (k R / nr, 0, p (H/2) / nz) for k = 0..nr, p = 0..nz
 * (nr = nz = 32), and fitted by least squares, every node weighted alike,
 * with the fifteen terms of Eq. (A.3) written in r/R and z/(H/2):
 * coef_host[m] (volts) multiplies (r/R)^(2 a_m) (z/(H/2))^(2 b_m), (a_m, b_m)
 * = (0,0) (1,0) (0,1) (1,1) (2,0) (0,2) (2,1) (1,2) (3,0) (0,3) (2,2) (3,1)
 * (1,3) (4,0) (0,4).  The field E_out = -grad P (Eq. (A.4)) stays fixed for
 * the life of the system (od_set_state does not refit it).
 * grid_host[(nz + 1) k + p] receives the grid potentials in volts
 * ((nr + 1)(nz + 1) doubles); coef_host, grid_host, nr, nz may be NULL.
 * OD_ESTATE if the system was created without the flag. */
od_status od_get_confinement(od_system* sys, double* coef_host, double* grid_host, int32_t* nr,
                             int32_t* nz);

/* Sizes: out_host[4] = {N, n_dust, precision, padded N}. */
od_status od_get_sizes(od_system* sys, int64_t* out_host);

/* State in dimensionless units, structure of arrays: x_host[3][N] and
 * v_host[3][N] (v is the half-step velocity), float for OD_PREC_FP32 and
 * double for OD_PREC_FP64; q_host[n_dust] in C; *step the step counter.
 * Any pointer may be NULL. */
od_status od_get_state(od_system* sys, void* x_host, void* v_host, double* q_host, int64_t* step);

/* Replaces the state (same layouts; NULL leaves a part unchanged). Ions
 * inside a grain give OD_ESTATE, non-finite values OD_ENUMERIC. */
od_status od_set_state(od_system* sys, const void* x_host, const void* v_host, const double* q_host,
                       int64_t step);

/* Accelerations of the last step's force evaluation, dimensionless, [3][N]
 * (float or double as the state). */
od_status od_get_accelerations(od_system* sys, void* a_host);

/* All-pairs ion-ion kernel (FP32 systems).
 * OD_PAIR_ONE_SIDED evaluates every ordered pair (one target per lane, all
 * sources); OD_PAIR_SYMMETRIC evaluates each unordered pair once and applies
 * the reaction to the source (Newton's third law of the screened Coulomb
 * force), accumulating both sides in int64 fixed point (a power of two set
 * from the ion density n per r_De^3, 2^(27 - (2/3) log2 n), so that the
 * resolution is about 1e-8 of a typical sum), so the result does not depend
 * on scheduling and is bitwise reproducible; it rounds differently from the
 * one-sided kernel.  A pair closer than about 4e-6 of the mean ion spacing
 * overflows the range and is reported as OD_ENUMERIC.
 * OD_PAIR_AUTO (the default) takes the symmetric kernel, which is the faster
 * one at every size (1.5x at 2^20, 1.8x at 2^18 and 2.4x at 2^12 ions on
 * MI355X).
 * The symmetric kernel needs 24 bytes per ion of accumulators.  FP64 systems
 * always use the one-sided kernel; a cutoff (od_set_cutoff) takes precedence
 * over either.  In test-particle mode (OD_FLAG_NO_ION_ION) the symmetric
 * setting runs no pair kernel at all: the step's tail adds the grain, drive
 * and confinement terms (the one-sided setting adds them in a pair kernel
 * without ion-ion terms, in FP64).  od_get_pair_kernel reports the kernel in
 * use. */
#define OD_PAIR_AUTO 0
#define OD_PAIR_ONE_SIDED 1
#define OD_PAIR_SYMMETRIC 2
od_status od_set_pair_kernel(od_system* sys, int32_t kind);
od_status od_get_pair_kernel(od_system* sys, int32_t* kind);

/* Source splits of the one-sided pair sum (FP32 mode): the sources are cut
 * into nsplit (1..4) ranges evaluated by separate blocks whose partial
 * accelerations the push adds in order, so that small systems fill the GPU.
 * Chosen at creation for about four blocks per compute unit; changing it
 * changes rounding only.  With the symmetric kernel or a cutoff the sum is
 * not split: od_get_pair_split reports 1 and od_set_pair_split accepts only 1
 * (OD_ESTATE otherwise). */
od_status od_set_pair_split(od_system* sys, int32_t nsplit);
od_status od_get_pair_split(od_system* sys, int32_t* nsplit);

/* Events of the last step: ev_host[N] bytes (0 none, 1 exited, 2 + d
 * absorbed by grain d; bit 7 set if a charge-exchange collision happened),
 * n_abs_host[n_dust] absorbed counts, *n_exit, *n_coll.  Any may be NULL.
 * Test surface (the per-ion view of the events of Section 2). */
od_status od_get_step_events(od_system* sys, uint8_t* ev_host, int64_t* n_abs_host,
                             int64_t* n_exit, int64_t* n_coll);

/* Ions absorbed in the last step (Section 2: an ion whose drift segment
 * meets a grain's surface is absorbed by that grain and delivers its charge
 * and momentum, Eq. (3)): absorbed_host[k] the ion index and by_dust_host[k]
 * the grain, for k < min(*n_absorbed, cap), in increasing ion order;
 * *n_absorbed the total, which may exceed cap; *n_exited the ions that left
 * through the cylinder's surface.  Any pointer may be NULL.  Synchronises. */
od_status od_get_absorbed(od_system* sys, int64_t* absorbed_host, int32_t* by_dust_host, int64_t cap,
                          int64_t* n_absorbed, int64_t* n_exited);

/* Per-step history of the observables of Section 3 (the charge q(n) and the
 * four force parts of Eqs. (1)-(4) of every step), kept on the device.
 * od_set_history(sys, capacity) records the next `capacity` steps, from the
 * current step counter on (0 turns recording off and frees the buffer;
 * capacity * n_dust * 14 doubles of device memory); it drops a captured graph
 * and synchronises.  od_get_history copies the records out:
 * rec_host[k][n_dust][14] for the k-th recorded step = {Q^n (C), the twelve
 * force components of od_get_dust_forces (N), absorbed count}, and sets
 * *n_recorded (at most capacity).  rec_host may be NULL. */
od_status od_set_history(od_system* sys, int64_t capacity);
od_status od_get_history(od_system* sys, double* rec_host, int64_t* n_recorded);

/* One Philox4x64-10 block computed on the device: out_host[4] for counter
 * ctr_host[4] and key (seed, system).  Test surface: no passage of the paper
 * defines it (the paper specifies no random generator); it lets a test check
 * the device generator against a reference implementation. */
od_status od_rng_block(uint64_t seed, uint64_t system, const uint64_t* ctr_host, uint64_t* out_host);

/* Kernel timing with HIP events on the system's stream (measurement
 * surface, no paper passage).  While enabled, od_step brackets every launch;
 * od_get_kernel_times synchronises and returns, per kernel class {0 pair
 * forces (with a cutoff: the slab sort and its epilogue too), 1 the step's
 * tail (acceleration of the symmetric sum, push, absorption, exit, and the
 * charge and force bookkeeping of the step in its last block), 2 reinjection
 * (systems above 16,384 ions; smaller ones reinject inside the tail), 3 not
 * used}, the summed milliseconds ms_host[4] and launch counts
 * launches_host[4] since enabling, then resets them. */
od_status od_set_timing(od_system* sys, int32_t enable);
od_status od_get_kernel_times(od_system* sys, double* ms_host, int64_t* launches_host);

/* Capture steps_per_graph (0..1000; 0: no graph) whole steps as one HIP graph
 * that od_step replays (n_steps / steps_per_graph replays, the remainder
 * launched one kernel at a time), for systems whose steps are short enough
 * for launch costs to matter.  The graph is captured on the system's stream,
 * which must not be the null stream (pass one to od_init_system; else
 * OD_ESTATE).  Results equal those of the same steps launched one at a time,
 * bit for bit.  od_set_state, od_set_cutoff, od_set_pair_kernel and
 * od_set_pair_split drop the graph and the next od_step captures it again;
 * while timing is on (od_set_timing) steps are launched one at a time so
 * that the per-kernel times stay meaningful.  Synchronizes the stream. */
od_status od_set_graph(od_system* sys, int32_t steps_per_graph);

/* ---- batches of independent systems ------------------------------------ */

/* Many independent dust systems (each one the model above, with its own
 * parameters, grains and N) advanced together on one stream: one launch per
 * step phase for all systems, the pair forces as a cost-ordered work list
 * pulled by a persistent grid, optionally captured as a HIP graph of several
 * steps.  Results of a system equal those of the same system run alone
 * with the same pair kernel, bit for bit (for the one-sided kernel, when its
 * pair sum is not split; see od_batch_set_config).
 * FP32 only (sim[s].precision must be OD_PREC_FP32); all-pairs ion-ion sums
 * only (the cutoff of od_set_cutoff is an option of single systems, whose
 * long domains fill the chip alone).
 *   plasma_host[n_systems], sim_host[n_systems]: per-system parameters;
 *   dust_host: all grains, system after system; n_dust_host[n_systems];
 *   hip_stream: NULL creates a private non-blocking stream (graph capture
 *   cannot use the null stream).
 * Errors as od_init_system, prefixed with the system index. */
typedef struct od_batch od_batch;
od_status od_init_batch(const od_plasma* plasma_host, const od_sim* sim_host, const od_dust* dust_host,
                        const int32_t* n_dust_host, int32_t n_systems, void* hip_stream,
                        const od_allocator* allocator, od_batch** out);
void od_destroy_batch(od_batch* b);

/* Work decomposition of the pair forces.  persistent: a grid of
 * (CUs x resident blocks) pulls work items from an atomic queue (else one
 * block per item).  Systems with N <= split_max_n have their source range cut
 * into jsplit (1..4) parts whose partial accelerations are added, in order,
 * by the push (changes rounding, not the method).  Drops a captured graph. */
od_status od_batch_set_config(od_batch* b, int32_t persistent, int32_t jsplit, int64_t split_max_n);
od_status od_batch_get_config(od_batch* b, int32_t* persistent, int32_t* jsplit, int64_t* split_max_n,
                              int32_t* n_items);

/* Pair kernel of the batch: OD_PAIR_SYMMETRIC (the default; OD_PAIR_AUTO
 * selects it too), each unordered pair once with int64 fixed-point totals
 * (see od_set_pair_kernel), or OD_PAIR_ONE_SIDED.  The persistent, jsplit and
 * split_max_n settings apply to the one-sided kernel only.  Drops a captured
 * graph. */
od_status od_batch_set_pair_kernel(od_batch* b, int32_t kind);
od_status od_batch_get_pair_kernel(od_batch* b, int32_t* kind);

/* Decomposition of the symmetric pair sums of the batch.  persistent: a grid
 * of (CUs x resident blocks) pulls the work items, ordered most work first,
 * from an atomic queue (else, the default, one block per item, which the
 * hardware dispatches in the same order).  one_row: one target tile row per
 * item for every system (else, the default, each system split as it is when
 * run alone: three rows per item from 2^16 ions on).  items_target: the
 * number of work items each system's split aims at (0: the default, 65536;
 * at most 2^24).  Scheduling does not change the results (integer totals);
 * one_row and items_target change the FP32 partial sums that each item
 * flushes, so a system then differs from its run alone by rounding.  Drops a
 * captured graph.  The getter reports the target in effect and *n_items, the
 * length of the work list (any pointer may be NULL). */
od_status od_batch_set_sym_config(od_batch* b, int32_t persistent, int32_t one_row, int64_t items_target);
od_status od_batch_get_sym_config(od_batch* b, int32_t* persistent, int32_t* one_row, int64_t* items_target,
                                  int32_t* n_items);

/* Times the pair phase for each candidate configuration (one-sided:
 * persistent or not, jsplit 1, 2, 4, split_max_n 2^15, 2^16; symmetric:
 * persistent or not, one target row per item or the size rule), keeps the
 * fastest, and returns its time in *best_ms.  With cache_path (a text file of one JSON object per
 * line, keyed by GPU architecture, CU count and the histogram of log2 N of
 * the systems) a cached choice is reused and a new one appended.  The
 * systems' state is unchanged. */
od_status od_batch_autotune(od_batch* b, const char* cache_path, double* best_ms);

/* Capture steps_per_graph (0..1000; 0: no graph) steps as one HIP graph that
 * od_step_batch replays; the remainder of a step count runs eagerly. */
od_status od_batch_set_graph(od_batch* b, int32_t steps_per_graph);
od_status od_step_batch(od_batch* b, int64_t n_steps);
od_status od_batch_sync(od_batch* b);

/* Per-system access, as the single-system calls (x/v/a float [3][N]):
 * sizes out_host[4] = {N, n_dust, pair splits, padded N}. */
od_status od_batch_get_sizes(od_batch* b, int32_t system, int64_t* out_host);
od_status od_batch_get_dust_charges(od_batch* b, int32_t system, double* q_now_host, double* q_avg_host);
od_status od_batch_get_dust_forces(od_batch* b, int32_t system, int32_t which, double* f_host);
od_status od_batch_get_state(od_batch* b, int32_t system, float* x_host, float* v_host, double* q_host,
                             int64_t* step);
od_status od_batch_set_state(od_batch* b, int32_t system, const float* x_host, const float* v_host,
                             const double* q_host, int64_t step);
od_status od_batch_get_accelerations(od_batch* b, int32_t system, float* a_host);
/* As od_get_confinement, for one member of the batch. */
od_status od_batch_get_confinement(od_batch* b, int32_t system, double* coef_host, double* grid_host,
                                   int32_t* nr, int32_t* nz);
od_status od_batch_get_step_events(od_batch* b, int32_t system, uint8_t* ev_host, int64_t* n_abs_host,
                                   int64_t* n_exit, int64_t* n_coll);

/* Timing as od_set_timing; classes {0 pair, 1 push, 2 reinjection,
 * 3 finalize, 4 graph replay}: ms_host[5], launches_host[5]. */
od_status od_batch_set_timing(od_batch* b, int32_t enable);
od_status od_batch_get_kernel_times(od_batch* b, double* ms_host, int64_t* launches_host);

/* ---- charge warm start --------------------------------------------------- */

/* Floating charge (C) of an isolated grain of the given radius (m) in the
 * plasma: the root of I_i + I_e = 0 with the OML currents of the "oml"
 * charging model (Section 2; ion current of the drifting Maxwellian).
 * Host computation; used to start charges near equilibrium. */
od_status od_oml_floating_charge(const od_plasma* plasma, double radius, double* q_host);

/* ---- surrogate network --------------------------------------------------- */

/* A fully connected network 5 -> 128 -> 128 -> 128 -> 16 (tanh on hidden
 * layers, FP32) trained and evaluated by the library's kernels (matrix
 * products on the matrix cores).  It learns a map from five inputs to
 * sixteen outputs; the caller chooses their meaning (here: Mach number,
 * grain radius, grain spacing, collision frequency, T_e/T_i -> charge and
 * axial force of each grain of an 8-grain chain).  Parameters are one flat
 * float vector of 35,856 values: for layers l = 1..4, W_l [in][out] then
 * b_l [out].  Inputs are mapped from the box [in_lo, in_hi] to [-1, 1];
 * outputs are produced as out_mean + out_std * (network output). */
typedef struct od_mlp od_mlp;
typedef struct {
    int32_t epochs;     /* passes over the training set                     */
    int32_t batch;      /* rows per step, 1..4096, <= n                      */
    double lr;          /* Adam learning rate at the first step              */
    double lr_final;    /* at the last step (exponential decay in between)  */
    uint64_t seed;      /* shuffling stream                                  */
} od_train_cfg;

/* Glorot-uniform weights drawn from Philox(seed), zero biases, identity
 * normalisation. */
od_status od_mlp_create(uint64_t seed, void* hip_stream, od_mlp** out);
void od_mlp_destroy(od_mlp* q);
od_status od_mlp_get_params(od_mlp* q, float* params_host);
od_status od_mlp_set_params(od_mlp* q, const float* params_host);
od_status od_mlp_set_normalization(od_mlp* q, const float* in_lo_host, const float* in_hi_host,
                                   const float* out_mean_host, const float* out_std_host);
/* Y_host[n][16] for X_host[n][5] (raw units); inside_host[n] (may be NULL) is
 * 1 where every input lies inside the normalisation box, else 0 (callers fall
 * back to the full method there). */
od_status od_mlp_predict(od_mlp* q, const float* X_host, int64_t n, float* Y_host, int32_t* inside_host);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * prediction of od_mlp_predict with X_dev [n][5] (raw units), Y_dev [n][16]
 * and inside_dev [n] (may be NULL) in device memory, asynchronous on the
 * network's stream.  It calls no allocating routine: the normalised inputs
 * and hidden activations go to a fixed device buffer of the library
 * (OD_MLP_NOALLOC_MAX_ROWS rows, 1.6 MB, one copy per GPU, held until the
 * process ends; its address is looked up when the first network on that GPU
 * is created).  Results equal od_mlp_predict's bit for bit.  n must be in
 * [0, OD_MLP_NOALLOC_MAX_ROWS] (OD_EINVAL otherwise).  Every call on one GPU
 * uses that GPU's one buffer: calls that overlap in time on one GPU (on
 * different streams, or from several threads) race and must be ordered by
 * the caller; calls in one stream are ordered by the stream. */
#define OD_MLP_NOALLOC_MAX_ROWS 1024
od_status od_mlp_predict_noalloc(od_mlp* q, const float* X_dev, int64_t n, float* Y_dev, int32_t* inside_dev);
/* The surrogate of the batched-solver study as two calls: od_surrogate_train
 * creates a network (weights from Philox(seed)), maps inputs from the box
 * [in_lo_host, in_hi_host] (5 floats each) to [-1, 1], standardises the 16
 * outputs by the training set's mean and standard deviation, and trains it
 * with Adam (cfg) on X_host[n][5], Y_host[n][16]; od_surrogate_predict is
 * od_mlp_predict.  The network is released with od_mlp_destroy. */
od_status od_surrogate_train(const float* X_host, const float* Y_host, int64_t n, const float* in_lo_host,
                             const float* in_hi_host, const od_train_cfg* cfg, uint64_t seed, void* hip_stream,
                             od_mlp** out);
od_status od_surrogate_predict(od_mlp* q, const float* X_host, int64_t n, float* Y_host, int32_t* inside_host);
/* Mean-squared error and its gradient (grad_host[35856]) on n <= 4096 rows of
 * already normalised inputs Xn_host[n][5] and standardised targets
 * Tn_host[n][16]. */
od_status od_mlp_loss_grad(od_mlp* q, const float* Xn_host, const float* Tn_host, int64_t n,
                           float* grad_host, double* loss);
/* Adam training on raw X_host[n][5], T_host[n][16] (normalised on the device
 * with the current normalisation); loss_per_epoch_host[epochs] (may be NULL)
 * receives the mean standardised squared error of each epoch. */
od_status od_mlp_train(od_mlp* q, const float* X_host, const float* T_host, int64_t n,
                       const od_train_cfg* cfg, double* loss_per_epoch_host);

#ifdef __cplusplus
}
#endif
#endif /* ODUST_H */
