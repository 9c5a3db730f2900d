/*
 * dclbm.h -- C ABI of the MI355X (gfx950) library for the lattice Boltzmann
 * step on nested-box refined meshes with the cell-vertex direct grid coupling
 * of Astoul, Wissocq, Boussuge, Sengissen & Sagaut, "Lattice Boltzmann method
 * for computational aeroacoustics on non-uniform meshes: a direct grid
 * coupling approach" (arXiv:2004.14887).
 *
 * Conventions
 *  - Every call returns dclbm_status: 0 on success, a negative code on error;
 *    no C++ exception crosses this boundary.  dclbm_last_error() gives a
 *    message for the calling thread's last failure.
 *  - The caller owns ALL device memory and the HIP stream.  The library
 *    never allocates device memory for a simulation: it carves the caller's
 *    workspace (size from dclbm_workspace_bytes).  It owns only host handles.
 *  - Pointers named d_* are device pointers, h_* host pointers; they are
 *    borrowed for the duration of the call.  Device work is enqueued on the
 *    simulation's stream; calls that return host values synchronise it.
 *  - Node coordinates are integers; level l+1 refines level l by 2 in space
 *    and time (Sec. 3.1, acoustic scaling).  Dense level arrays are ordered
 *    x fastest, then y, then z: index = (z*ny + y)*nx + x.
 */
#ifndef DCLBM_H
#define DCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DCLBM_ABI_VERSION 5
#define DCLBM_MAX_LEVELS 4

typedef enum {
    DCLBM_OK = 0,
    DCLBM_ERR_INVALID = -1,  /* bad argument or geometry */
    DCLBM_ERR_NOMEM = -2,    /* workspace too small */
    DCLBM_ERR_HIP = -3,      /* a HIP runtime call failed; message in dclbm_last_error() */
    DCLBM_ERR_NEWTON = -4,   /* Newton solve at a co-located node did not converge */
    DCLBM_ERR_UNSTABLE = -5, /* a non-finite density was found */
    DCLBM_ERR_BUSY = -6
} dclbm_status;

typedef enum { DCLBM_D2Q9 = 0, DCLBM_D3Q19 = 1 } dclbm_lattice;

/* Arithmetic and storage of the populations.
 *  FP64:         FP64 everywhere.
 *  FP32:         FP32 collision and interface arithmetic, populations stored
 *                as FP32 deviations f_i - w_i from the rest state.
 *  FP32_FP16:    FP32 arithmetic, populations stored as FP16 values of
 *                256 (f_i - w_i) (round to nearest even).
 * In both reduced forms w_i generalises to E_i = f0_i(1, u_ref), the
 * equilibrium of a uniform reference flow (dclbm_config.u_ref; the rest
 * state when zero), and velocities are carried relative to u_ref, so that a
 * mean flow does not eat the precision of the deviations.
 * Probes and balances always accumulate in FP64. */
typedef enum { DCLBM_FP64 = 0, DCLBM_FP32 = 1, DCLBM_FP32_FP16 = 2 } dclbm_precision;

/* Choice of (Gamma_i, gamma_i) couples at co-located nodes, Sec. 3.4 Table
 * "choice_Gamma_fine": DC1 takes P from the fine grid, DC2 from the coarse. */
typedef enum { DCLBM_DC1 = 1, DCLBM_DC2 = 2 } dclbm_coupling;

/* Collision model.
 *  BGK:  f* = f0 + (1 - 1/tau)(f - f0) (Eq.(LBMscheme_reg) with f1 = f - f0,
 *        psi = 0); every mesh.
 *  HRR:  the hybrid recursive regularised collision of Sec. 2: a_1^(2) of
 *        Eq.(a12_HRR) mixing the projection of Eq.(a1Proj) (weight sigma)
 *        and the centred finite differences of Eq.(a1FD_scheme), a_1^(3) of
 *        Eq.(a13RR), the cubic Mach correction psi_i of App. A (optional).
 *        Every mesh.  On refined meshes the steps follow Sec. 3.5: a level
 *        streams and completes its interface nodes, runs its child's two
 *        substeps, then collides all its nodes; the gradients at co-located
 *        and hanging nodes are those of Sec. 3.3 (coarse stencil, rescaled
 *        by Eq.(PijResc) and Eq.(PSIResc)).  Refined H-RR steps are launched
 *        eagerly (no graph). */
typedef enum { DCLBM_BGK = 0, DCLBM_HRR = 1 } dclbm_collision;

typedef struct {
    int32_t abi_version;      /* DCLBM_ABI_VERSION */
    int32_t lattice;          /* dclbm_lattice: D2Q9 (Fig. 1 numbering) or D3Q19 (Eq.(xi_i)) */
    int32_t precision;        /* dclbm_precision */
    int32_t coupling;         /* dclbm_coupling */
    int32_t eq_order;         /* 2: second-order equilibrium; 3: adds the H3 terms of Eq.(fEq_herm) */
    int32_t n0[3];            /* periodic coarse domain, nodes per axis (n0[2] ignored in 2-D) */
    int32_t n_levels;         /* 1..DCLBM_MAX_LEVELS */
    /* box of level l+1 (index l), as [lo, hi) in level-l node coordinates.
     * Constraints: side >= 3 parent cells, margin >= 2 parent cells to the
     * parent's own boundary (to the domain edge for level 1). */
    int32_t box_lo[DCLBM_MAX_LEVELS - 1][3];
    int32_t box_hi[DCLBM_MAX_LEVELS - 1][3];
    double tau0;              /* level-0 relaxation time (> 1/2); tau_{l+1} = 2 tau_l - 1/2, Eq.(rescTau) */
    int32_t n_probes;         /* pressure probes, 0..64, p' = (rho - 1)/3 after each coarse step */
    const int32_t* h_probe_xyz; /* [n_probes][3] level-0 node coordinates (host) */
    int64_t probe_capacity;   /* coarse steps of probe history kept on the device */
    int32_t newton_max_iter;  /* 0 -> 20 */
    double newton_tol;        /* 0 -> 1e-12 (FP64) or 2e-6 (FP32 forms); Sec. 3.2 stop rule |dX| < tol */
    double u_ref[3];          /* reference velocity of the reduced-precision storage (ignored by FP64);
                               * |u_ref| below the sound speed; zero: deviations from w_i */
    int32_t collision;        /* dclbm_collision */
    double hrr_sigma;         /* HRR: weight of the projected part, 0..1 (0.98 in the paper's runs) */
    int32_t hrr_psi;          /* HRR: cubic Mach correction of App. A on (1) or off (0) */
    /* Absorbing layer on level 0 (Sec. 4.2.1 uses one; its form is a reading):
     * after each coarse step's collision, nodes within sponge_cells cells of
     * the periodic seam take f_i - s(x) (f0_i(rho, u) - f0_i(1, u_ref)), with
     * s(x) = sponge_sigma ((W - e) / W)^2, e the node's distance in cells to
     * the domain's outermost nodes.  0 cells: none.  The level-1 box must lie
     * outside the layer.  Steps with a layer are launched eagerly. */
    int32_t sponge_cells;
    double sponge_sigma;      /* 0..1 */
    /* Refined region of level 1 made of level-0 cells (Sec. 3.4 closing
     * paragraph, App. B: the interface may have any stair-stepped shape; the
     * node sets follow from which neighbours exist).  NULL: the whole box.
     * Otherwise a host mask over the cells of level 1's box, x fastest,
     * (hi - lo) per axis, 1 = refined, read during dclbm_workspace_bytes and
     * dclbm_create only.  A level-0 node is a hole when its four cells are
     * refined and co-located when some are; a level-1 node exists when any of
     * its parent cells is refined and is on the interface when not all are.
     * Hanging nodes interpolate along their boundary run: centred 4-point,
     * else one-sided 4-point, else linear on a one-cell run.  With H-RR, a
     * point of a co-located node's coarse stencil missing from the region is
     * the parent node there.  D2Q9 and two levels only (DCLBM_ERR_INVALID
     * otherwise, or when a co-located node admits no valid couples). */
    const uint8_t* h_region;
} dclbm_config;

typedef struct dclbm_sim dclbm_sim;

/* Bytes of device workspace a simulation with this configuration needs.
 * Validates the configuration (DCLBM_ERR_INVALID with a message). */
dclbm_status dclbm_workspace_bytes(const dclbm_config* cfg, size_t* bytes);

/* Create a simulation in the caller's workspace (256-byte aligned, at least
 * dclbm_workspace_bytes bytes) on the given HIP stream (hipStream_t passed as
 * void*; NULL means the default stream, where no graphs are used).  All
 * populations start as NaN until dclbm_init_equilibrium fills each level. */
dclbm_status dclbm_create(const dclbm_config* cfg, void* d_workspace, size_t bytes, void* stream,
                          dclbm_sim** out);
dclbm_status dclbm_destroy(dclbm_sim* sim);

/* Node counts of a level (dense box, holes included) and its active nodes. */
dclbm_status dclbm_level_shape(const dclbm_sim* sim, int32_t level, int32_t dims[3], int64_t* n_active);

/* Node-update count of one coarse step: sum over levels of 2^l * active nodes. */
dclbm_status dclbm_updates_per_step(const dclbm_sim* sim, int64_t* updates);

/* Set every active node of a level to the equilibrium of (rho, u) (Sec. 4.1:
 * populations initialised at equilibrium).  d_rho: [n] FP64, d_u: [D][n]
 * FP64, dense over the level.  Initialise every level before stepping. */
dclbm_status dclbm_init_equilibrium(dclbm_sim* sim, int32_t level, const double* d_rho, const double* d_u);

/* Advance n coarse steps (Sec. 3.5: each coarse step is one asynchronous and
 * one synchronous fine iteration per refinement level, recursively).  Work
 * is enqueued on the stream; after the first step each coarse step is one
 * hipGraph launch.  Newton failures latch a device flag read by dclbm_check. */
dclbm_status dclbm_step(dclbm_sim* sim, int32_t n_coarse_steps);

/* Synchronise and report latched device errors (DCLBM_ERR_NEWTON, DCLBM_ERR_UNSTABLE). */
dclbm_status dclbm_check(dclbm_sim* sim);

/* Post-collision populations of a level as FP64 f_i, [Q][n] dense, NaN on holes. */
dclbm_status dclbm_read_populations(const dclbm_sim* sim, int32_t level, double* d_out);

/* Density [n] and velocity [D][n] of a level from the post-collision populations, NaN on holes. */
dclbm_status dclbm_read_macros(const dclbm_sim* sim, int32_t level, double* d_rho, double* d_u);

/* Velocity divergence of a level (Sec. 4.1.1, 4.1.2: the field in which the
 * reflection of an acoustic pulse at a refinement interface is shown):
 * centred differences (u_a(x + e_a) - u_a(x - e_a)) / 2 summed over the D
 * axes, in the level's lattice units.  d_u is the level's velocity [D][n]
 * as dclbm_read_macros writes it (device memory, caller-owned); d_div [n]
 * receives the divergence, NaN where a stencil point is a hole or lies
 * beyond a refined level's extent (level 0 wraps periodically).  Enqueued
 * on the simulation's stream; DCLBM_ERR_INVALID for a null pointer or a bad
 * level. */
dclbm_status dclbm_velocity_divergence(const dclbm_sim* sim, int32_t level, const double* d_u, double* d_div);

/* Shared macroscopic state X = (rho, u) found by Newton at the co-located
 * nodes of a refined level (Sec. 3.2), [4][n] dense, NaN elsewhere. */
dclbm_status dclbm_read_shared(const dclbm_sim* sim, int32_t level, double* d_out);

/* Pressure probes, the "microphones" of Sec. 4.2 (36 pressure probes on a
 * circle around the source, whose series give the OASPL of the spurious
 * acoustics).  Reading of the paper: the probe records p' = c_s^2 (rho - 1)
 * = (rho - 1)/3 from the post-collision populations after each coarse step,
 * at a level-0 node coordinate, on the finest level whose closed box holds
 * the point.  Series [steps][n_probes] FP64 into d_out (may be NULL to
 * query); *n_steps receives the number of coarse steps recorded (at most
 * probe_capacity).  Synchronises. */
dclbm_status dclbm_read_probes(const dclbm_sim* sim, double* d_out, int64_t* n_steps);

/* Running sums of the probes over a window of coarse steps, from which the
 * OASPL of Sec. 4.2 follows without keeping the series: every coarse step s
 * with start <= s < stop (numbered as the rows of the series, from 0) that
 * the probes sample adds to FP64 sums on the device, whatever
 * probe_capacity is.  The sums are kept about K, each probe's first sample
 * in the window, so that a mean far above the fluctuations does not cancel
 * them: sum (p' - K) and sum (p' - K)^2 (each product rounded on its own).
 * dclbm_set_probe_window sets the window and clears the sums; it is
 * enqueued on the simulation's stream, so it applies to the steps enqueued
 * after it (a simulation starts with the empty window [0, 0)).  Errors:
 * DCLBM_ERR_INVALID unless 0 <= start <= stop.  The sums are part of a
 * checkpoint. */
dclbm_status dclbm_set_probe_window(dclbm_sim* sim, int64_t start, int64_t stop);

/* The running sums [3][n_probes] FP64 into d_out (device memory, may be
 * NULL to query): sum (p' - K), sum (p' - K)^2, then K (NaN before the first
 * sample); *n_summed receives the number of coarse steps summed.  Samples
 * the last step's probes if they are pending.  Synchronises. */
dclbm_status dclbm_read_probe_sums(const dclbm_sim* sim, double* d_out, int64_t* n_summed);

/* FP64 balances of the moments of Eq.(moment_rho) and Eq.(moment_rhoU):
 * mass sum rho, momentum sum rho u and kinetic energy sum rho |u|^2 / 2
 * over the nodes each level owns (the finest level containing a point owns
 * it; the coarse co-located nodes of Sec. 3.2 belong to the finer level),
 * each node weighted by its cell volume 2^(-D l) (Sec. 3.1: level l has
 * spacing 2^-l).  The paper reports no balances; they are the conservation
 * diagnostics of the method (mass is exact on one level and drifts at the
 * interfaces, whose interpolations do not conserve it).  Synchronises; also
 * latches DCLBM_ERR_UNSTABLE on a non-finite density. */
dclbm_status dclbm_balance(dclbm_sim* sim, double h_out[5]);

/* For callers that cannot allocate or synchronise, such as code under HIP
 * graph capture or a serving loop that must not block: the balances of
 * dclbm_balance, enqueued on the simulation's stream and written to the
 * caller's device buffer d_out (5 FP64: mass, momentum[3], kinetic energy),
 * bit-identical to dclbm_balance's.  It allocates nothing, copies nothing to
 * the host and does not synchronise; a non-finite density latches
 * DCLBM_ERR_UNSTABLE for the next dclbm_check.  Its block partial sums live
 * in a static device array of the library (each GPU's copy holds 4 levels x
 * 1024 blocks x 5 doubles plus 4 x 5 totals, about 160 KB, until the process
 * ends); a simulation needing more is rejected (DCLBM_ERR_INVALID).  Calls
 * on one GPU share that array: calls that overlap on one GPU (two streams)
 * race, so serialise them.  The simulation's device must be current. */
dclbm_status dclbm_balance_static(dclbm_sim* sim, double* d_out);

/* Checkpoint and resume.  The state that the sub-cycling of Sec. 3.5
 * carries from one coarse step to the next:
 *   - the current populations of every level;
 *   - the coarse history rings that feed Eq.(TempInt);
 *   - the shared states X;
 *   - the probe series and the latched error flags;
 *   - on the host: the A/B parity, the capture count of every level, and
 *     the number of coarse steps done.
 * The interface tables and the other A/B buffer are not part of it: create
 * rebuilds the tables from the configuration, and the next step writes the
 * other buffer.
 *
 * dclbm_checkpoint_bytes: size of the checkpoint of this simulation.
 *
 * dclbm_save: writes the checkpoint into the caller's device buffer d_blob
 * (256-byte aligned, at least dclbm_checkpoint_bytes long).  It first
 * samples the probes of the last step if they are pending.  Copies run on
 * the simulation's stream; the call synchronises before it returns.
 *
 * dclbm_load: restores a checkpoint into a simulation of the same
 * configuration: same lattice, precision, mesh, tau0, coupling, equilibrium
 * order, probes, probe capacity, Newton settings and u_ref.  The target may
 * be the simulation that wrote it, or another one created from the same
 * configuration.  Stepping on from the restored state gives results
 * identical, bit for bit, to stepping on from the saved one.  Synchronises.
 *
 * Errors (DCLBM_ERR_INVALID, nothing changed): a null or misaligned
 * buffer, bytes below the checkpoint size, a blob that is not a checkpoint,
 * or a checkpoint written for another configuration. */
dclbm_status dclbm_checkpoint_bytes(const dclbm_sim* sim, size_t* bytes);
dclbm_status dclbm_save(dclbm_sim* sim, void* d_blob, size_t bytes);
dclbm_status dclbm_load(dclbm_sim* sim, const void* d_blob, size_t bytes);

/* Instrumentation: when on, steps run without graphs and every level-substep
 * launch carries start/stop events in its dispatch (a split 3-D FP16 substep,
 * two kernels side by side, is timed from the fork to the join by events on
 * the stream); dclbm_bulk_time returns
 * the summed milliseconds, the launch count and the nodes one launch of that
 * level updates (active nodes minus the coarse co-located nodes, which the
 * child's synchronous substep updates). */
dclbm_status dclbm_set_timing(dclbm_sim* sim, int32_t on);

/* Launch layout (no effect on results, which are bit-identical either way):
 * with FP16 storage in 3-D a refined level's substep runs either as one
 * launch, its interface segments interleaved over the front of the grid, or
 * split into two kernels side by side on a second stream (the bulk alone at
 * a higher occupancy; the probe, capture and segment workgroups beside it).
 * mode -1 (the default) splits where the bulk outweighs the segments by
 * enough to pay for it, 0 never splits, 1 splits every substep with
 * segments; other forms ignore it.  Synchronises and drops the cached
 * coarse-step graphs, which the next step rebuilds.  Errors:
 * DCLBM_ERR_INVALID for another mode. */
dclbm_status dclbm_set_split(dclbm_sim* sim, int32_t mode);
dclbm_status dclbm_bulk_time(dclbm_sim* sim, int32_t level, double* ms, int64_t* launches,
                             int64_t* nodes_per_launch);

/* Instrumentation: the algorithmic interface bytes of one launch of a level
 * substep (averaged over its two substeps), beyond the 2 Q values read and
 * written per updated node that dclbm_bulk_time's node count covers.  They
 * are the O(surface) traffic of the coupling of Sec. 3.5: the coarse history
 * ring shift at coarse co-located nodes (the input of Eq.(TempInt)), the
 * ring reads of the Gamma = R directions and the X writes at fine
 * co-located nodes, and the restriction of Eq.(rescfc) into the parent at
 * the synchronous substep.  Interface tables are not counted. */
dclbm_status dclbm_interface_bytes(const dclbm_sim* sim, int32_t level, double* bytes_per_launch);

/* Bandwidth reference: copies `bytes` (multiple of 16, 16-byte aligned
 * device buffers) from d_src to d_dst `repeats` times on the stream with a
 * plain 16-byte-per-lane copy kernel and returns the mean milliseconds per
 * copy (read + write of `bytes` each).  Used to state the achievable HBM
 * bandwidth and to scale the HBM byte counters. */
dclbm_status dclbm_copy_calibration(void* d_dst, const void* d_src, size_t bytes, void* stream, int32_t repeats,
                                    double* ms_per_copy);

/* ------------------------------------------------------------------ serving
 * Continuous batching of many simulations of one class (lattice, precision,
 * eq_order) on one GPU and one stream.  The caller owns the server's device
 * workspace: fixed tables plus an arena from which every admitted request
 * takes exactly dclbm_workspace_bytes of its configuration (first fit);
 * admission waits for a free slot and a fitting block.  A tick retires
 * finished requests, admits queued ones (arrival order; later requests may
 * pass one that does not fit yet, a bounded number of times) and enqueues
 * steps_per_tick coarse steps of every resident simulation as one hipGraph
 * launch: one persistent launch per level substep of a max_levels mesh plus
 * one for probes.  Each simulation advances exactly as dclbm_step would
 * advance it alone (Sec. 3.5 sub-cycling; its own arguments, tables and
 * state), so its result does not depend on the mix.  A request finishes
 * after its own step count; its probe series then comes back to the host.
 * submit may be called from another thread while a thread ticks. */
typedef struct dclbm_server dclbm_server;

typedef enum { DCLBM_REQ_QUEUED = 0, DCLBM_REQ_RUNNING = 1, DCLBM_REQ_DONE = 2, DCLBM_REQ_FAILED = 3 } dclbm_request_state;

typedef struct {
    int32_t abi_version;      /* DCLBM_ABI_VERSION */
    int32_t lattice;          /* class of every request: lattice, precision, eq_order */
    int32_t precision;
    int32_t eq_order;
    int32_t max_levels;       /* deepest mesh admitted, 1..DCLBM_MAX_LEVELS (sets the phases per step: 2^L - 1) */
    int32_t max_slots;        /* simulations resident at once, 1..1024 */
    int32_t steps_per_tick;   /* coarse steps per tick, 1..64 */
    int32_t max_probes;       /* probes per request, 0..32 */
    int64_t max_probe_steps;  /* largest step count of a request (its probe series is kept whole) */
    int64_t max_level_nodes;  /* dense nodes of the largest level of any request (staging of initial fields) */
    int32_t grid;             /* workgroups of every phase launch (multiple of 8); 0: per tick, the smallest
                               * power of two from 2048 to 262144 covering the largest phase */
    int32_t max_inflight;     /* ticks enqueued ahead of the GPU before a tick waits (at most 6); 0: 2 */
} dclbm_server_config;

typedef struct {
    double t_submit, t_admit, t_done; /* seconds since the server was created (host clock) */
    int64_t steps;            /* coarse steps requested */
    int64_t updates;          /* node updates: steps * sum_l 2^l active_l */
    int64_t workspace_bytes;  /* footprint taken from the arena while resident */
    int32_t slot;             /* slot it ran in (-1 before admission) */
    int32_t state;            /* dclbm_request_state */
    int32_t status;           /* DCLBM_OK, or the latched error (DCLBM_ERR_NEWTON, DCLBM_ERR_UNSTABLE) */
    int32_t n_probes;
} dclbm_request_info;

typedef struct {
    int64_t ticks;            /* graph launches so far */
    int32_t running, queued;  /* resident (including finishing) and waiting requests */
    int64_t arena_bytes, arena_free, arena_largest_free;
    int32_t grid;             /* workgroups of the phase launches of the last tick */
    int32_t n_phases;         /* persistent launches per coarse step, before the probe launch */
} dclbm_server_info;

/* Device bytes of a server whose arena holds arena_bytes. */
dclbm_status dclbm_server_workspace_bytes(const dclbm_server_config* cfg, size_t arena_bytes, size_t* total);
/* Create a server in the caller's workspace (256-byte aligned) on a
 * non-default stream (hipStream_t as void*); captures its tick graph. */
dclbm_status dclbm_server_create(const dclbm_server_config* cfg, void* d_workspace, size_t bytes, void* stream,
                                 dclbm_server** out);
dclbm_status dclbm_server_destroy(dclbm_server* server);
/* Queue a request: a configuration of the server's class (its probe_capacity
 * is replaced by steps), `steps` coarse steps, and initial fields per level
 * (h_rho[l]: [n_l] FP64, h_u[l]: [D][n_l] FP64, dense as for
 * dclbm_init_equilibrium, host memory, copied before return).  The geometry
 * is validated here (DCLBM_ERR_INVALID; DCLBM_ERR_NOMEM if it can never fit). */
dclbm_status dclbm_server_submit(dclbm_server* server, const dclbm_config* cfg, int64_t steps,
                                 const double* const* h_rho, const double* const* h_u, uint64_t* id);
/* One scheduling round (see above).  Blocks only to keep at most
 * max_inflight ticks queued on the stream. */
dclbm_status dclbm_server_tick(dclbm_server* server, int32_t* n_running, int32_t* n_queued);
dclbm_status dclbm_server_poll(dclbm_server* server, uint64_t id, int32_t* state);
/* Probe series [steps][n_probes] FP64 of a finished request (h_probes may
 * be NULL) and its record; DCLBM_ERR_BUSY while it has not finished, the
 * latched error if it failed. */
dclbm_status dclbm_server_result(dclbm_server* server, uint64_t id, double* h_probes, int64_t* n_steps,
                                 dclbm_request_info* info);
/* Forget a finished request. */
dclbm_status dclbm_server_release(dclbm_server* server, uint64_t id);
dclbm_status dclbm_server_stats(dclbm_server* server, dclbm_server_info* out);

/* Lattice table: Q, velocities [Q][3] and weights [Q] of a lattice. */
dclbm_status dclbm_lattice_table(int32_t lattice, int32_t* q, int32_t* h_xi, double* h_w);

const char* dclbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
