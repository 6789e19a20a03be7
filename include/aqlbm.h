/*
 * aqlbm: MI355X (gfx950) library for the coupled lattice Boltzmann model of
 * aqueous-humour dynamics of Qin, Meng, Yang, Zhang & Wen (arXiv:2102.12663).
 *
 * One time step is one fused pull-stream / collide kernel over the active nodes of a 2D
 * lattice:
 *   - flow: incompressible D2Q9 BGK (section 2.3, eq. 6-10) with the buoyancy force of
 *     eq. 15-17 and a Darcy drag (eq. 4) in POROUS nodes;
 *   - heat: a D2Q5 convection-diffusion BGK (eq. 11-14; rest weight w0 = 0 is the
 *     paper's D2Q4);
 *   - link-wise boundaries: bounce-back walls (cornea, iris/lens floor, outer box), a
 *     moving-wall secretion inlet, an anti-bounce-back pressure outlet, and
 *     anti-bounce-back Dirichlet temperatures;
 *   - every `check_interval` steps the same kernel also reduces the IOP (mean pressure of
 *     the chamber, sections 2.2.4 and 3.1), the outflow rate (Fig. 2), the cornea and iris
 *     wall shear stress (section 3.6) and the convergence residuals.
 *
 * Conventions
 *   - Lattice units, delta_x = delta_t = c = 1.  Node (x, y) is element y*nx + x of every
 *     host array (row-major, x fastest).
 *   - Status codes: AQ_OK (0) or a negative AQ_E* value.  Out-parameters are written only
 *     on AQ_OK.  aq_last_error() returns a message for the calling thread's last failure.
 *   - Ownership: the caller owns every host array and keeps it only for the duration of
 *     the call (the library copies what it needs).  The library owns the solver and, for
 *     aq_create, its device memory.  With aq_create_ext the caller owns the device arena
 *     and the HIP stream; both must outlive the solver.
 *   - Threading: a solver handle may be used by one thread at a time.  Calls on distinct
 *     handles are independent.
 *   - Asynchrony: aq_step only enqueues work on the solver's stream.  aq_observe,
 *     aq_read_field, aq_run_to_steady, aq_save and aq_write_populations synchronise it.
 */
#ifndef AQLBM_H
#define AQLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    AQ_OK = 0,
    AQ_EINVAL = -1,        /* invalid argument, parameter or mask */
    AQ_ENOMEM = -2,        /* device or host allocation failed, or arena too small */
    AQ_EDEVICE = -3,       /* HIP runtime error */
    AQ_EDIVERGED = -4,     /* a non-finite moment was seen at a check step (latched) */
    AQ_ENOTCONVERGED = -5, /* aq_run_to_steady reached max_steps */
    AQ_EBUSY = -6,         /* no free slot or memory (serving admission) */
    AQ_ESTATE = -7         /* call not valid in the solver's current state */
};

/* Storage precision of the populations.  F64: stored and computed in double.  F32:
 * stored and computed in float.  F16S: stored as binary16 of (deviation * 2^s) with a
 * per-solver power-of-two scale, computed in float; the intermediate step of a two-step
 * launch stays in float on chip, so the state is rounded to binary16 where it is stored
 * (every other step in the plain steps of an interval).  F32X: stored in float, computed in
 * double (the float arithmetic's rounding, not the storage, sets F32's error against
 * FP64 at buoyant steady states).  Reductions are always double. */
enum { AQ_F64 = 0, AQ_F32 = 1, AQ_F16S = 2, AQ_F32X = 3 };

/* Fields for aq_read_field. */
enum {
    AQ_FIELD_P = 0,        /* absolute pressure p (eq. 9) */
    AQ_FIELD_UX = 1,       /* velocity x (eq. 9) */
    AQ_FIELD_UY = 2,       /* velocity y */
    AQ_FIELD_T = 3,        /* temperature (eq. 13) */
    AQ_FIELD_POP_FLOW = 4, /* pre-collision flow population q = 1..8, deviation form */
    AQ_FIELD_POP_HEAT = 5  /* pre-collision thermal population q = 0..4, deviation form */
};

/* Mask byte (input): bits 0-2 node class, bits 3-4 wall id of a SOLID node; for an OUTLET
 * node under AQ_OUTLET_LUMPED, bits 3-4 are the outward seepage direction (AQ_DIR_*). */
enum { AQ_SOLID = 0, AQ_FLUID = 1, AQ_POROUS = 2, AQ_INLET = 3, AQ_OUTLET = 4 };
enum { AQ_WALL_BOX = 0, AQ_WALL_CORNEA = 1, AQ_WALL_IRIS = 2 };
enum { AQ_DIR_PX = 0, AQ_DIR_PY = 1, AQ_DIR_MX = 2, AQ_DIR_MY = 3 };

/* Outlet models: a pressure outlet at p_out, or the lumped trabecular meshwork of
 * section 2.2.4 (Darcy seepage driven by the IOP, applied as a velocity condition). */
enum { AQ_OUTLET_PRESSURE = 0, AQ_OUTLET_LUMPED = 1 };

/* Boundary schemes: link-wise (half-way bounce-back walls) or the paper's (section 2.3:
 * the interpolated bounce-back of Bouzidi et al. on CORNEA and IRIS walls). */
enum { AQ_BC_LINKWISE = 0, AQ_BC_PAPER = 1 };

/*
 * Solver parameters (lattice units).  struct_size must be sizeof(aq_params).
 *
 *   tau_f, tau_t      flow / thermal relaxation times, > 1/2 (eq. 6, eq. 11);
 *                     viscosity (2 tau_f - 1)/6 (eq. 10), diffusivity
 *                     (1 - w0)(2 tau_t - 1)/4 (eq. 14 at w0 = 0)
 *   w0                thermal rest weight in [0, 1); the axis weights are (1 - w0)/4
 *   u_in_x, u_in_y    velocity of the secretion inlet (moving-wall bounce-back)
 *   p_ref             pressure about which flow populations are stored:
 *                     h_i = f_i - lambda_i p_ref (lambda_{1-4} = 1/3, lambda_{5-8} = 1/12,
 *                     the reading sigma = 5/12 of the constraints under eq. 7)
 *   p_out             absolute pressure at OUTLET nodes (anti-bounce-back), and the
 *                     reference of iop_gauge
 *   p_init, T_init    initial equilibrium state, at rest
 *   T_ref             temperature about which thermal populations are stored:
 *                     g_i = T_i - w^T_i T_ref
 *   T0                Boussinesq reference temperature (eq. 5)
 *   T_cornea, T_iris  wall temperatures of CORNEA and IRIS solids; T_inlet of INLET cells
 *   gbeta             g*beta; buoyant force g*beta*(T - T0)*(sin phi, cos phi) (eq. 16-17)
 *   gravity_angle     phi in radians; 0 means gravity along -y
 *   K                 Darcy permeability of POROUS nodes (eq. 4), > 0
 *   storage           AQ_F64, AQ_F32, AQ_F16S or AQ_F32X
 *   check_interval    steps between reductions; even, >= 2
 *   fp16_exp_flow, fp16_exp_thermal
 *                     F16S scale exponents s (values stored as deviation * 2^s);
 *                     -1 picks them from the parameters
 *   outlet_mode       AQ_OUTLET_PRESSURE, or AQ_OUTLET_LUMPED: the meshwork is not
 *                     resolved; its pressure falls linearly over the thickness h_tm from
 *                     the IOP (mean pressure over FLUID nodes) to p_sc, so Darcy's law
 *                     (eq. 4, viscosity nu at unit density) gives the seepage speed
 *                     u_s = K_tm (IOP - p_sc) / (nu h_tm).  u_s is re-evaluated at every
 *                     check step and holds for the next check_interval steps (the first
 *                     interval uses p_init); every OUTLET node is a wall moving at u_s
 *                     along its outward direction (moving-wall bounce-back).
 *   K_tm, h_tm, p_sc  lumped meshwork permeability and thickness (> 0) and Schlemm's-
 *                     canal pressure (absolute)
 *   bc_scheme         AQ_BC_LINKWISE, or AQ_BC_PAPER: the flow populations of a wall-list
 *                     node's links into CORNEA / IRIS solids take the linear interpolated
 *                     bounce-back of Bouzidi et al. with the link fractions q of the wall
 *                     list (q < 1/2: 2q h*_o(x) + (1 - 2q) h*_o(x - e_o); q >= 1/2:
 *                     h*_o(x)/(2q) + (2q - 1)/(2q) h*_i(x), o the link toward the wall,
 *                     i its opposite, h* post-collision; half-way bounce-back when q < 1/2
 *                     and x - e_o is not active).  Not mass-conserving on curved walls.
 *   reserved1         0
 */
typedef struct aq_params {
    uint32_t struct_size;
    int32_t nx, ny;
    int32_t storage;
    int32_t check_interval;
    int32_t fp16_exp_flow, fp16_exp_thermal;
    int32_t outlet_mode;
    int32_t bc_scheme, reserved1;
    double tau_f, tau_t, w0;
    double u_in_x, u_in_y;
    double p_ref, p_out, p_init;
    double T_ref, T_init, T0;
    double T_cornea, T_iris, T_inlet;
    double gbeta, gravity_angle, K;
    double K_tm, h_tm, p_sc;
} aq_params;

/* Wall node: an active FLUID node next to a CORNEA or IRIS solid, with the unit normal
 * (n_x, n_y) pointing into the fluid (wall shear stress) and, for each link i = 1..8, the
 * fraction q[i-1] in (0, 1] of the link along e_i at which it meets the wall when the
 * neighbour along e_i is a CORNEA or IRIS solid, else -1 (AQ_BC_PAPER).  Lists must be
 * sorted by node. */
typedef struct aq_wall_node {
    int32_t node;   /* y*nx + x */
    int32_t wall;   /* AQ_WALL_CORNEA or AQ_WALL_IRIS */
    double n_x, n_y;
    double q[8];
} aq_wall_node;

/*
 * Observables of one check step, all in lattice units and computed from that step's
 * pre-collision moments:
 *   iop_gauge       mean pressure over FLUID nodes minus p_out (IOP; sections 2.2.4, 3.1)
 *   p_mean_fluid    mean absolute pressure over FLUID nodes
 *   q_in, q_out     flow mass entering through INLET links / leaving through OUTLET links
 *                   during the step (outflow rate of Fig. 2)
 *   wss_*           mean and maximum wall shear stress over the CORNEA and IRIS wall
 *                   nodes, |t - (t.n) n| with t = sigma n and
 *                   sigma = -(1 - 1/(2 tau_f)) sum_i e_i e_i (h_i - h_i^eq) (section 3.6)
 *   resid_u         ||u - u_prev|| / (check_interval ||u||) over active nodes (or the
 *                   absolute form when ||u|| = 0); resid_T the same with T - T_ref
 *   u_max           max |u|; mass_flow = sum h, mass_thermal = sum g over active nodes
 *   n_nonfinite     number of active nodes with a non-finite moment
 *   u_seep          AQ_OUTLET_LUMPED: the seepage speed evaluated at this check step
 *                   (in effect for the next check_interval steps); 0 otherwise
 */
typedef struct aq_observables {
    int64_t step;
    double iop_gauge, p_mean_fluid, q_in, q_out;
    double wss_cornea_mean, wss_cornea_max, wss_iris_mean, wss_iris_max;
    double resid_u, resid_T, u_max, mass_flow, mass_thermal;
    int64_t n_nonfinite;
    double u_seep;
} aq_observables;

/* Read-only facts about a solver. */
typedef struct aq_info {
    int64_t active_nodes, fluid_nodes, lattice_nodes;
    int32_t nx, ny, pitch, storage;
    int32_t tile_x, tile_y, n_tiles, check_interval;
    int32_t fp16_exp_flow, fp16_exp_thermal;
    int32_t fusion;                 /* 1: the plain steps run two per launch */
    int32_t graph_launches;         /* launches replayed from a graph per check interval */
    int32_t nt_store;               /* 1: population stores bypass the caches (non-temporal) */
    int32_t fused_tile_rows;        /* rows of a two-step tile (64 wide): 8, or 4 (F32, F16S) */
    int64_t step;
    size_t device_bytes;
    double bytes_per_node_update;   /* algorithmic HBM bytes per active-node update */
} aq_info;

typedef struct aq_solver aq_solver;

const char* aq_version(void);
const char* aq_last_error(void);

/* Device bytes aq_create_ext needs for these parameters and mask (admission check). */
int aq_required_bytes(const aq_params* params, const uint8_t* mask, size_t* bytes);

/* Create a solver.  mask: ny*nx bytes; walls: n_walls entries (may be NULL if 0).  The
 * state starts as the equilibrium of (p_init, u = 0, T_init).  Errors: AQ_EINVAL for
 * tau <= 1/2, nx or ny < 4, more than 2^30 nodes or, in F32 storage, a population plane
 * beyond 4 GiB (ny x nx rounded up to 64 columns, times 4 bytes), an active node on the
 * outer frame, unknown storage, an odd or < 2 check_interval, K <= 0, or an invalid wall
 * list; AQ_ENOMEM; AQ_EDEVICE. */
int aq_create(const aq_params* params, const uint8_t* mask, const aq_wall_node* walls,
              int32_t n_walls, aq_solver** out);

/* As aq_create, with device memory carved from the caller's arena (256-byte aligned,
 * arena_bytes >= aq_required_bytes) and work enqueued on the caller's HIP stream
 * (hipStream_t, may be NULL for the default stream). */
int aq_create_ext(const aq_params* params, const uint8_t* mask, const aq_wall_node* walls,
                  int32_t n_walls, void* device_arena, size_t arena_bytes, void* hip_stream,
                  aq_solver** out);

int aq_destroy(aq_solver* s);

/* Enqueue nsteps time steps (eq. 6 and eq. 11 with their boundaries).  Steps whose global
 * index is a multiple of check_interval also run the reductions.  Whole check intervals
 * replay a captured HIP graph. */
int aq_step(aq_solver* s, int64_t nsteps);

/* Step until max(resid_u, resid_T) < tol at a check step, or max_steps.  Writes the last
 * check step's observables.  Returns AQ_ENOTCONVERGED at the step cap and AQ_EDIVERGED on
 * a non-finite state. */
int aq_run_to_steady(aq_solver* s, double tol, int64_t max_steps, aq_observables* out);

/* Observables of the most recent check step (step = 0 and zeros before the first). */
int aq_observe(aq_solver* s, aq_observables* out);

/* Copy a field of the current state to host (count must be nx*ny): p, u_x, u_y, T in
 * absolute lattice units, or pre-collision population q in deviation form.  NaN at
 * non-active nodes. */
int aq_read_field(aq_solver* s, int32_t field, int32_t q, double* host, size_t count);

/* Replace the pre-collision state by flow[8][ny][nx] (q = 1..8) and heat[5][ny][nx]
 * (q = 0..4), deviation form; values at non-active nodes are ignored.  Also resets the
 * residual reference to this state's moments.  count must be nx*ny. */
int aq_write_populations(aq_solver* s, const double* flow, const double* heat, size_t count);

/* Checkpoint: the stored populations (in storage precision), the residual reference and
 * the step counter.  aq_load requires a solver created with the same parameters and mask;
 * a resumed run is bitwise identical to an uninterrupted one. */
int aq_save(aq_solver* s, const char* path);
int aq_load(aq_solver* s, const char* path);

int aq_get_info(aq_solver* s, aq_info* out);

/* Choose the tile shape (tile_x a multiple of 64 up to 256, tile_y with
 * tile_x * tile_y in [64, 1024]).  Rebuilds the tile list and graphs. */
int aq_set_tile(aq_solver* s, int32_t tile_x, int32_t tile_y);

/* Time n_launch back-to-back launches of the plain (non-reducing) step kernel with HIP
 * events on the solver's stream; *ms_per_launch receives the average.  The state
 * advances by n_launch steps (n_launch must be even). */
int aq_time_step_kernel(aq_solver* s, int32_t n_launch, double* ms_per_launch);

/* Two-steps-per-launch (temporal blocking) on the plain steps of each check interval: on
 * (enable != 0) or off.  The default is on for F64, F32X and F16S, and for F32 from 2^18
 * active nodes or when a step's working set exceeds the last-level cache.  F64, F32 and F32X give bitwise the same
 * results either way.  F16S does not: a two-step launch keeps its intermediate step in
 * float, single steps round every step to binary16.  Batched instances always run two
 * steps per launch, so an instance reduces bitwise the same alone (with the default) and
 * in a batch. */
int aq_set_fusion(aq_solver* s, int32_t enable);

/* Rows of the two-step tiles (64 wide): 8, or 4 in F32 and F16S (twice the blocks, for
 * lattices too small to fill the chip with 64 x 8 tiles).  The default is 4 for F32 and
 * F16S lattices below 2^20 active nodes, else 8 (aq_info.fused_tile_rows).  Results are
 * bitwise the same either way.  Synchronises the solver's stream; AQ_EINVAL for other
 * values. */
int aq_set_fused_tile_rows(aq_solver* s, int32_t rows);

/*
 * Vortex diagnostics of the current state (section 3.5, Table 3, Figs. 6-7), computed on
 * the device from the velocity (eq. 9):
 *   vortex_intensity  I = 2 sum over FLUID nodes of |omega_z| (unit cell area), with
 *                     omega_z = (d u_y/dx - d u_x/dy)/2 (eq. 18); a derivative is the central
 *                     difference where both neighbours along the axis are active, the
 *                     one-sided difference toward the active one where only one is, else 0.
 *                     The magnitude is summed: the signed integral of eq. 18 is the
 *                     circulation around the no-slip boundary, which vanishes.
 *   u_max_fluid       max |u| over FLUID nodes
 *   psi_max, psi_min  extrema over FLUID nodes of the stream function
 *                     psi(x, y) = sum over y' <= y of u_x(x, y') (active nodes of column x),
 *                     i.e. u_x = d psi/dy; their nodes (x, y) are the centres of the
 *                     counter-rotating and co-rotating vortices (smallest y*nx + x on ties;
 *                     -1 when the lattice has no FLUID node)
 */
typedef struct aq_diagnostics {
    int64_t step;
    double vortex_intensity, u_max_fluid, psi_max, psi_min;
    int32_t psi_max_x, psi_max_y, psi_min_x, psi_min_y;
} aq_diagnostics;

/* Device workspace aq_diagnose needs for these parameters (about 16 bytes per node). */
int aq_diagnostics_bytes(const aq_params* params, size_t* bytes);

/* Compute the diagnostics above.  workspace: device memory of at least
 * aq_diagnostics_bytes (caller-owned, 8-byte aligned, contents overwritten).  Synchronises
 * the solver's stream.  AQ_EINVAL for a null or too small workspace. */
int aq_diagnose(aq_solver* s, void* workspace, size_t workspace_bytes, aq_diagnostics* out);

/* aq_diagnose without a caller workspace and without any device allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a fixed 64 MiB array in device
 * memory, one per GPU, held from the first call on that GPU until the process ends; the
 * lattice must need at most that much (aq_diagnostics_bytes <= 64 MiB, about 4 M nodes),
 * else AQ_EINVAL and nothing is launched.  Results are identical to aq_diagnose's.  All
 * calls on one GPU share its array and leave their contents in it (nothing in it needs
 * to start cleared): calls that overlap on one GPU, from different threads or on
 * different streams without ordering, race.  Synchronises the solver's stream. */
int aq_diagnose_noalloc(aq_solver* s, aq_diagnostics* out);

/* Lumped meshwork outlet (AQ_OUTLET_LUMPED only): replace K_tm, h_tm and p_sc of a live
 * solve (the calibration loop of section 3.1 adjusts the meshwork thickness until the
 * steady IOP is the healthy one).  The seepage speed in effect becomes that of the new
 * values at the last check step's IOP (p_init before the first check); later check steps
 * re-evaluate it as usual.  Synchronises the solver's stream.  AQ_EINVAL for another
 * outlet, invalid values or a coupling the check interval cannot hold (as aq_create). */
int aq_set_outlet(aq_solver* s, double K_tm, double h_tm, double p_sc);

/* Time n_launch back-to-back two-step launches (HIP events on the solver's stream);
 * *ms_per_launch receives the average per launch (two time steps).  One single step
 * follows, untimed.  The state advances by 2 * n_launch + 1 steps without reductions. */
int aq_time_fused_kernel(aq_solver* s, int32_t n_launch, double* ms_per_launch);

/* Whole-interval graph replays with HIP events around the graph part of each interval:
 * runs n_intervals * check_interval steps (the current step must be a multiple of
 * check_interval) and returns the total elapsed milliseconds and the milliseconds spent
 * in the graph part of every interval, i.e. aq_info.graph_launches launches per interval:
 * (check_interval - 2) / 2 two-step launches when fusion is on (F16S: that number
 * rounded down to even, as in a batch), else check_interval - 1 single steps.  The
 * remaining single steps and the reducing step are outside the graph part. */
int aq_run_intervals_timed(aq_solver* s, int32_t n_intervals, double* total_ms,
                           double* plain_ms);

/* Bandwidth of a plain device copy on the current device (context for the step kernels'
 * HBM rates): allocates two buffers of `bytes` bytes (a multiple of 16, at least 1 MiB),
 * copies the first into the second `reps` times with a grid-stride kernel of 16-byte
 * words with non-temporal stores on 256 CUs x 8 blocks, and frees them.  *gbs receives the best rep's
 * (read + written bytes) / time in GB/s, timed with HIP events.  AQ_EINVAL for invalid
 * sizes, AQ_ENOMEM if the buffers do not fit, AQ_EDEVICE on a HIP error. */
int aq_copy_bandwidth(size_t bytes, int32_t reps, double* gbs);

/* ------------------------------------------------------------------------------------
 * Batched serving form: many independent solves (parameter sweeps of uneven lattice
 * sizes) resident in one device arena and stepped together, one multi-instance kernel
 * launch per storage mode and time step, replayed from a captured HIP graph per check
 * interval.  Requests are admitted while others run (continuous batching); each one runs
 * to its own steady-state residual.  An admitted instance computes exactly what the
 * single-lattice solver computes for the same parameters, mask and tile shape (fields and
 * observables bitwise equal).
 * ------------------------------------------------------------------------------------ */
typedef struct aq_batch aq_batch;

/* Result status of an F16S solve accepted at binary16's rounding floor (not an error
 * code; only aq_result.status takes it): its residual stopped above tol, and its IOP
 * (iop_gauge) moved by at most drift_tol, relative, against the IOP at least 1000 steps
 * earlier (the IOP drift check). */
enum { AQ_RESULT_FLOOR = 1 };

/* A finished request.  status: AQ_OK (residual below tol), AQ_RESULT_FLOOR (F16S, above),
 * AQ_ENOTCONVERGED (max_steps), AQ_EDIVERGED (non-finite moments), or AQ_EDEVICE if the
 * F16S -> F32 hand-off failed on the device.  storage: the storage the final state is held
 * in; fallback: 1 when an F16S solve failed the IOP drift check and was continued in F32
 * storage. */
typedef struct aq_result {
    int64_t request_id;
    int32_t slot, status, storage, fallback;
    int64_t steps;
    aq_observables obs;
} aq_result;

typedef struct aq_batch_info {
    int32_t max_slots, running, finished;
    int32_t n_work[4];              /* tiles per storage mode (AQ_F64 .. AQ_F32X) in the work lists */
    int64_t active_nodes;           /* over running instances */
    size_t budget_bytes, used_bytes, largest_free_bytes;
    int64_t step;                   /* time steps run by the batch */
    int32_t fused_tile_rows[4];     /* rows of the two-step tiles (64 x rows) per storage mode */
} aq_batch_info;

/* Create a batch: budget_bytes of device memory for instances (allocated once), at most
 * max_slots instances, at most max_active_nodes active nodes running at once (0 = no cap),
 * work lists of max_tiles tiles per storage mode, and a common check_interval (even).
 * hip_stream may be NULL (the batch creates its own). */
int aq_batch_create(size_t budget_bytes, int32_t max_slots, int64_t max_active_nodes, int32_t max_tiles,
                    int32_t check_interval, void* hip_stream, aq_batch** out);

/* Admit one solve.  Parameters, mask and walls as for aq_create; tile_x * tile_y must be
 * 256.  tol: residual at which the solve is done (an F16S solve first runs to
 * max(tol, 2e-5), or until its residual stops falling by 10% over 50 check intervals:
 * binary16 rounding noise sets a floor; if that floor is above tol, the IOP drift check
 * decides: an IOP within drift_tol, relative, of the IOP at least 1000 steps earlier
 * finishes it with AQ_RESULT_FLOOR, otherwise it continues in F32 storage to tol);
 * max_steps: step cap; request_id: returned with the result; keep != 0 keeps the finished
 * state readable (aq_batch_read_field) until aq_batch_release.  An F16S instance takes
 * arena space for its F32 continuation as well (the F32 layout and a 104-byte-per-node
 * conversion image), so the hand-off needs nothing beyond its admission.  *slot receives
 * the slot.  AQ_EBUSY when no slot, arena space, active-node or work-list capacity is free. */
int aq_batch_admit(aq_batch* b, const aq_params* params, const uint8_t* mask, const aq_wall_node* walls,
                   int32_t n_walls, int32_t tile_x, int32_t tile_y, double tol, double drift_tol,
                   int64_t max_steps, int64_t request_id, int32_t keep, int32_t* slot);

/* Run n_intervals check intervals of every running instance, then retire the instances
 * that converged, diverged or reached max_steps (synchronises the stream).  An interval is
 * two HIP graphs (the two-step launches of every kernel class, then the rest) with one
 * block per work item; admissions and retirements that change the work lists make the
 * next run capture them again. */
int aq_batch_run(aq_batch* b, int32_t n_intervals);

/* As aq_batch_run, with HIP events on the batch stream: *total_ms receives the elapsed
 * time of the n_intervals intervals, *fused_ms the time spent in their two-step launches
 * (two time steps of every running instance per launch, all kernel classes), and
 * *fused_launches the number of those launches.  AQ_ESTATE if nothing is running. */
int aq_batch_run_timed(aq_batch* b, int32_t n_intervals, double* total_ms, double* fused_ms,
                       int32_t* fused_launches);

/* Collect up to cap finished results not yet collected; their slots and memory are freed
 * unless they were admitted with keep. */
int aq_batch_poll(aq_batch* b, aq_result* done, int32_t cap, int32_t* n_done);

/* aq_read_field / aq_observe on the instance in a slot (running, or finished and kept). */
int aq_batch_read_field(aq_batch* b, int32_t slot, int32_t field, int32_t q, double* host, size_t count);
int aq_batch_observe(aq_batch* b, int32_t slot, aq_observables* out);

/* Free a slot (running or finished). */
int aq_batch_release(aq_batch* b, int32_t slot);

/* aq_set_outlet on the instance in a slot (running or finished and kept). */
int aq_batch_set_outlet(aq_batch* b, int32_t slot, double K_tm, double h_tm, double p_sc);

/* Put a finished instance admitted with keep back into the batch from its current state
 * (a warm start, e.g. after aq_batch_set_outlet), to run until its residual falls below
 * tol or for at most max_steps more steps; its result is reported again by aq_batch_poll.
 * AQ_ESTATE if the slot is running, was not kept, or failed (diverged); AQ_EBUSY if the
 * active-node cap or the work list has no room. */
int aq_batch_resume(aq_batch* b, int32_t slot, double tol, int64_t max_steps);

/* aq_diagnose on the instance in a slot (running, or finished and kept). */
int aq_batch_diagnose(aq_batch* b, int32_t slot, void* workspace, size_t workspace_bytes, aq_diagnostics* out);

int aq_batch_get_info(aq_batch* b, aq_batch_info* out);

/* Rows of the two-step tiles (64 x rows) of the batch's F32 and F16S instances: 0 chooses
 * by size (64 x 4, six blocks per CU, while a kernel class's running instances hold fewer
 * than 2^20 active nodes, so a small batch still spreads over the chip; 64 x 8 otherwise),
 * 4 or 8 fixes it.  FP64 and F32X always use 64 x 8, and a class whose 64 x 4 list would
 * exceed the work-list capacity takes 64 x 8.  Results are bitwise the same with either
 * height.  Applies from the next interval; synchronises the batch's stream.  AQ_EINVAL for
 * any other value. */
int aq_batch_set_fused_tile_rows(aq_batch* b, int32_t rows);

/* Autotune the tile shape of a solver: time n_launch plain launches for each candidate
 * shape (64x4, 128x2, 256x1, and 64x1, 64x2, 128x1 unless only_256 is set) and keep the
 * fastest; *tile_x, *tile_y and *ms_per_launch receive it.  When two steps run per launch
 * in an F32 or F16S solver, the two-step tiles 64x8 and 64x4 are timed too (n_launch / 2
 * launches each) and the faster kept (aq_info.fused_tile_rows).  The state advances by
 * the launched steps (n_launch even; reductions are skipped, as in aq_time_step_kernel). */
int aq_autotune_tile(aq_solver* s, int32_t n_launch, int32_t only_256, int32_t* tile_x, int32_t* tile_y,
                     double* ms_per_launch);

int aq_batch_destroy(aq_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* AQLBM_H */
