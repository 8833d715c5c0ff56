/*
 * tissue.h -- C-ABI of libtissue.so, the MI355X (gfx950) implementation of the
 * operator-split multicellular stochastic simulation of Coulier & Hellander,
 * "Orchestral: a lightweight framework for parallel simulations of cell-cell
 * communication".
 *
 * The problem statement follows the paper's orchestration section: a tissue
 * is a network of cells with neighbours and per-cell parameters, among them
 * a seed (Fig. 2, the network file); it is advanced n_steps times by a
 * splitting interval dt (Fig. 3, the configuration file's n_steps; each
 * module run with an end time); then its state is read back.  One splitting
 * step is the internal-dynamics operator chi on every cell independently,
 * followed by the pairwise signalling operator S (Algorithm section,
 * splitting assumption; Fig. 1: chi first, then S).
 *
 *   chi : per cell, a Gillespie direct-method SSA over the cell's voxels
 *         (RDME: reactions inside a voxel, diffusion jumps between adjacent
 *         voxels) on [0, dt)  (Introduction: SSA and RDME as single-cell
 *         modules; "Internal cell dynamics module").
 *   S   : per lattice edge, an SSA on [0, dt) of the trans reaction
 *         N_i + D_j -> I_i between the voxels of the two cells' facing
 *         membrane groups ("Cell signaling module"; Results, Model: Delta
 *         near the shared face turns into the neighbour's NICD, each molecule
 *         handled by a single face's signalling model).
 *
 * Numerical contract (identical bits to the CPU FP64 oracle): Philox4x32-10
 * counter (draw j, global step n, cell or edge id, sim_id << 2 | tag) keyed
 * by the seed; U1 = (m1 + 1) 2^-53, U2 = m2 2^-53 from the two 53-bit halves;
 * tau = -plog(U1) / a0; per-voxel propensity = left fold over the channels
 * (reactions, then one aggregated diffusion channel per diffusing species);
 * a0 = binary sum tree over the next power of two >= V leaves; the selection
 * and tie rules are written out in the design notes.
 *
 * Conventions for every entry point:
 *   - all functions return TISSUE_OK (0) or a negative TISSUE_E* code; a
 *     thread-local detail string is available from tissue_last_error();
 *   - host arrays passed in are copied; the caller keeps ownership;
 *   - device memory comes from the caller (dev_buf) and must outlive the
 *     handle; the library allocates no device memory of its own for a
 *     tissue (graphs and the launch plan live in host memory);
 *   - work is enqueued on the tissue's HIP stream; reads synchronise it;
 *   - handles are not thread-safe; distinct handles are independent;
 *   - results depend only on the descriptor and the sequence of
 *     (dt, n_steps) calls -- never on batching, streams or launch shapes.
 */
#ifndef TISSUE_H
#define TISSUE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TISSUE_ABI_VERSION 2u

enum {
    TISSUE_OK = 0,
    TISSUE_EINVAL = -1,    /* invalid descriptor or argument; nothing enqueued */
    TISSUE_ENOMEM = -2,    /* dev_bytes smaller than tissue_required_bytes()   */
    TISSUE_EOVERFLOW = -3, /* a count left [0, 2^26); state unspecified        */
    TISSUE_EDEVICE = -4,   /* a HIP call failed (detail in tissue_last_error)  */
    TISSUE_EBUSY = -5,     /* resource exhausted; retry later                  */
    TISSUE_ESTATE = -6,    /* call not valid in the handle's state             */
    TISSUE_ELIMIT = -7     /* a unit-step reached event_cap and was stopped     */
};

enum { TISSUE_LATTICE_SQUARE = 0, TISSUE_LATTICE_HEX = 1 };

/* descriptor flags */
#define TISSUE_FLAG_TRACE 1u  /* keep per-(unit, step) event counts and clocks */
#define TISSUE_FLAG_NO_JIT 2u /* use the ahead-of-time generic chi kernels only  */
/* Strang's symmetric splitting (G. Strang 1968) instead of the paper's
 * sequential (Lie) splitting: each step is chi over dt/2 (counter tag 0),
 * S over dt (tag 1), chi over dt/2 (tag 2).  The per-(cell, step) chi trace
 * then sums both halves' events and holds the second half's clock.  Members
 * of one batch must agree on this flag. */
#define TISSUE_FLAG_STRANG 4u
/* First-order signalling (the paper's model, Results, Setup, Model): S
 * turns each trans_d molecule in a face voxel of a cell into a trans_i
 * molecule of the neighbour at trans_rate per molecule.  The receiving voxel
 * is the facing one: face groups are slices of the cells' membrane rings,
 * traversed the same way round, so the k-th voxel of a group of m faces the
 * (m' - 1 - floor(k m' / m))-th of the neighbour's group of m'.  Channels in
 * order: k_i * D_i(a) for a in A, then k_j * D_j(b) for b in B, where k_c is
 * trans_rate, or the signal_rate of cell c's network under per-cell models. */
#define TISSUE_FLAG_SIGNAL_FIRST_ORDER 8u

#define TISSUE_MAX_SPECIES 8
#define TISSUE_MAX_REACTIONS 16
#define TISSUE_MAX_MESH 8
#define TISSUE_COUNT_LIMIT (1 << 26)
#define TISSUE_DEFAULT_EVENT_CAP (1u << 20)

typedef struct tissue tissue_t;
typedef struct tissue_batch tissue_batch_t;

/*
 * One more intracellular network over the tissue's species, for per-cell
 * models (the paper's Discussion: detailed modules where cells signal,
 * coarser ones where little happens; in the network file each cell names
 * its own model, Fig. 2).  The tables follow the descriptor's own reaction
 * tables below, with the same rules and limits; the channel order of a cell
 * is its own network's (reactions, then its diffusing species in species
 * order).  S, the seed and the counters are the tissue's, whatever the
 * cells' networks.
 */
typedef struct {
    uint32_t n_reactions;     /* 0..TISSUE_MAX_REACTIONS                        */
    const int32_t *reactants; /* [n_reactions][2]                               */
    const int32_t *stoich;    /* [n_reactions][n_species]                       */
    const double *rates;      /* [n_reactions]                                  */
    const double *diffusion;  /* [n_species]                                    */
    double signal_rate;       /* under TISSUE_FLAG_SIGNAL_FIRST_ORDER: the rate per
                                 trans_d molecule of this network's cells (a
                                 sender's own network sets it; trans_rate plays
                                 this part for network 0), in [0, 1e12]; with
                                 the second-order reaction it must equal
                                 trans_rate                                     */
} tissue_model_t;

#define TISSUE_MAX_MODELS 7   /* extra networks per tissue (8 with its own)     */

/*
 * Tissue descriptor.  Cells: i = y*nx + x (hex: axial q = x, r = y, rhombus).
 * Square directions 0 +x, 1 +y, 2 -x, 3 -y; hex 0 E(+1,0), 1 SE(0,+1),
 * 2 SW(-1,+1), 3 W(-1,0), 4 NW(0,-1), 5 NE(+1,-1); open boundaries.
 * Cell c has a w x h voxel mesh, voxel v = y*w + x.
 */
typedef struct {
    uint32_t abi_version;     /* = TISSUE_ABI_VERSION                          */
    uint32_t lattice;         /* TISSUE_LATTICE_SQUARE or TISSUE_LATTICE_HEX   */
    uint32_t nx, ny;          /* lattice extent, nx*ny >= 1                     */
    const uint8_t *mesh_w;    /* [nx*ny] per-cell mesh width 1..8, or NULL     */
    const uint8_t *mesh_h;    /* [nx*ny] per-cell mesh height 1..8, or NULL    */
    uint32_t mesh_w0, mesh_h0;/* uniform mesh when mesh_w/mesh_h are NULL      */
    uint32_t n_species;       /* 1..TISSUE_MAX_SPECIES                          */
    uint32_t n_reactions;     /* 0..TISSUE_MAX_REACTIONS (intracellular)        */
    const int32_t *reactants; /* [n_reactions][2] species index or -1 (order 0..2) */
    const int32_t *stoich;    /* [n_reactions][n_species] net change; a species
                                 may only lose as many as it supplies as reactant */
    const double *rates;      /* [n_reactions] in [0, 1e12]: propensity constants */
    const double *diffusion;  /* [n_species] in [0, 1e12]: jump rate per direction */
    int32_t trans_n, trans_d, trans_i; /* S reaction N_i + D_j -> I_i; trans_n < 0
                                          disables S; otherwise three distinct species.
                                          With TISSUE_FLAG_SIGNAL_FIRST_ORDER:
                                          D_i -> I_j, trans_n unused, trans_d < 0
                                          disables S; trans_d, trans_i distinct */
    uint32_t flags;           /* TISSUE_FLAG_*                                  */
    double trans_rate;        /* in [0, 1e12]                                   */
    const int32_t *init_counts; /* [sum_c V_c][n_species], each in [0, 2^26)   */
    uint64_t seed;            /* Philox key                                     */
    uint32_t sim_id;          /* < 2^30, part of every counter                  */
    uint32_t start_step;      /* global index of the next step (resume)         */
    uint32_t event_cap;       /* events per unit-step; 0 = TISSUE_DEFAULT_EVENT_CAP */
    uint32_t trace_steps;     /* steps of trace kept when TISSUE_FLAG_TRACE     */
    uint32_t n_models;        /* 0..TISSUE_MAX_MODELS extra networks; 0: every
                                 cell runs the network above                    */
    const tissue_model_t *models; /* [n_models]: network m is models[m - 1]     */
    const uint8_t *cell_model;    /* [nx*ny] each cell's network, 0..n_models
                                     (0: the network above); NULL: all 0        */
} tissue_desc_t;

typedef struct {
    uint64_t chi_events;      /* accepted chi events since create/restart       */
    uint64_t s_events;        /* accepted S events                              */
    uint64_t draws;           /* Philox blocks drawn (events + overshoots)      */
    uint32_t steps_done;      /* global index of the next step                  */
    uint32_t overflow;        /* nonzero: a count left [0, 2^26)                */
    uint32_t capped;          /* nonzero: a unit-step hit event_cap             */
    uint32_t n_cells, n_edges, n_voxels; /* n_edges: edges of the S operator (0 without S) */
    uint32_t jit;             /* nonzero: chi runs kernels compiled for the tissue's
                                 networks (every one of them)                   */
} tissue_stats_t;

/* Validate d and compile the chi kernels for its networks' structures
 * without loading them (needs no device).  TISSUE_EDEVICE with the compiler
 * log in tissue_last_error() if the compilation fails. */
int tissue_network_check(const tissue_desc_t *d);

/* Device bytes a tissue needs in dev_buf (admission by free memory).
 * Returns 0 for an invalid descriptor. */
size_t tissue_required_bytes(const tissue_desc_t *d);

/* Create a tissue: the cell network of the paper's network file (Fig. 2:
 * each cell with its neighbours and its parameters, among them a seed).
 * Validate d, build the lattice, edges, colour classes, meshes and face
 * groups on the host, lay the state out in dev_buf (>= required bytes,
 * 256-byte aligned) and upload it on hip_stream (NULL: the null stream).
 * Errors: TISSUE_EINVAL (descriptor; nothing allocated or enqueued),
 * TISSUE_ENOMEM (dev_bytes too small), TISSUE_EDEVICE (a HIP call failed).
 * Unless TISSUE_FLAG_NO_JIT is set, the chi kernels are compiled for the
 * network's structure (hipRTC, cached per process by structure, not rates);
 * if that compilation fails the generic kernels are used (same bits). */
int tissue_create(const tissue_desc_t *d, void *dev_buf, size_t dev_bytes,
                  void *hip_stream, tissue_t **out);

/* Enqueue n_steps splitting steps of length dt (finite, > 0); n_steps >= 0.
 * One step is chi on every cell over dt, then S over every edge (Algorithm
 * section, the splitting assumption; Fig. 1); n_steps is the configuration
 * file's number of steps and dt each module's end time (Fig. 3).  Step
 * indices continue from steps_done.  Asynchronous.  TISSUE_EINVAL (nothing
 * enqueued) for a bad dt or n_steps, or when steps_done + n_steps would pass
 * 2^32 (the step index is part of every random counter). */
int tissue_step(tissue_t *t, double dt, int32_t n_steps);

/* Synchronise and copy the counts out, layout as init_counts (the state the
 * paper's modules write to their output files after each run, Fig. 3).
 * host_out is caller-owned, n_out must be sum_c V_c * n_species.  Returns
 * TISSUE_EOVERFLOW / TISSUE_ELIMIT if that condition was flagged (the counts
 * are still copied). */
int tissue_read_counts(tissue_t *t, int32_t *host_out, size_t n_out);

/* Synchronise and report the running totals. */
int tissue_read_stats(tissue_t *t, tissue_stats_t *out);

/* The same totals without blocking, for loops that must not wait on the
 * device (serving): tissue_stats_enqueue puts a copy of the tissue's
 * statistics block (TISSUE_STATS_BLOCK_BYTES bytes) into host memory `dst`
 * on the tissue's stream (use pinned host memory for the copy to be
 * asynchronous; `dst` must stay valid until the stream has passed it).
 * After that point tissue_stats_decode turns the block into the totals;
 * steps_done is the count of steps enqueued when decoding. */
#define TISSUE_STATS_BLOCK_BYTES 64
int tissue_stats_enqueue(tissue_t *t, void *dst);
int tissue_stats_decode(tissue_t *t, const void *block, tissue_stats_t *out);

/* Trace of the last trace_steps steps (tissues created with
 * TISSUE_FLAG_TRACE): for global steps [first_step, first_step + n_steps),
 * chi_events/chi_t_bits are [n_steps][n_cells] and s_events/s_t_bits
 * [n_steps][n_edges] (clock after the last accepted event, as bits).  Any
 * output pointer may be NULL. */
int tissue_read_trace(tissue_t *t, uint32_t first_step, uint32_t n_steps,
                      uint32_t *chi_events, uint64_t *chi_t_bits,
                      uint32_t *s_events, uint64_t *s_t_bits);

/* Restore the counts given at create (kept on the device), zero the
 * statistics and flags, and continue as simulation sim_id from step
 * start_step.  Enqueued on the tissue's stream. */
int tissue_restart(tissue_t *t, uint32_t sim_id, uint32_t start_step);

/* Overwrite the counts from host memory (same layout as init_counts). */
int tissue_write_counts(tissue_t *t, const int32_t *host_in, size_t n_in);

/* Launch shape of the chi operator: 0 = one workgroup per work item,
 * 1 = persistent workgroups pulling items from a device queue (the
 * default), with workgroups_per_cu resident workgroups per CU (0 = auto).
 * Results are bit-identical for every choice. */
int tissue_set_launch(tissue_t *t, int32_t persistent, int32_t workgroups_per_cu);

/* Kernel of the chi operator.  0 = one lane per cell with the full sum tree
 * and 32-bit counts in LDS (every cell); 1 = one row of max(16, P) lanes per
 * cell of P leaves, one lane per voxel (16, 32 or 64 lanes); 4 = rows of
 * max(32, P) lanes (the same kernel with at most two cells per wavefront:
 * twice the wavefronts of mode 1 for cells of at most 16 voxels);
 * 3 = the compact layout: one lane per 16 voxels of a cell (1, 2 or 4
 * lanes per cell of P = 16, 32 or 64 leaves), each holding its voxels' 16
 * FP64 leaves and 16-bit counts, the tree levels above them rebuilt in
 * registers and combined across the cell's lanes; cells that reach 2^16
 * molecules of a species are handed to a full-width lane launch that redoes
 * their step; 2 = automatic (the default): cells of at most 8 voxels take
 * mode 0; a class of cells of 9 to 64 voxels takes the compact layout when
 * it holds at least 16 lanes of it per SIMD of the device (cells x P / 16),
 * else rows; in a single tissue whose 33-64-voxel class is compact and
 * regrouped by load, that class's heaviest min(SIMDs, cells / 4) cells run
 * in rows of 64 lanes.  Results are bit-identical for every choice.  Other
 * values: TISSUE_EINVAL. */
int tissue_set_chi_mode(tissue_t *t, int32_t mode);

/* Steps captured per HIP graph launch (0 disables graphs). */
int tissue_set_graph_chunk(tissue_t *t, int32_t steps_per_graph);

/* Small tissues in one launch per call (Algorithm section and Results >
 * Scaling: at small splitting intervals the scheduling of the per-step tasks
 * outweighs the tasks themselves).  enable = 1 (the default): when the
 * tissue's chi operator is one work item of the one-lane-per-cell layout
 * (at most 64 cells of one leaf class of at most 8 voxels) with a compiled
 * network, it has at most 8 S passes of at most 2 work items (128 edges)
 * each, and its state fits 48 KiB, tissue_step runs all its steps in one
 * workgroup of one kernel (up to 100 steps per launch) with the state
 * copied into LDS for the call: the chi item, then the S passes in order,
 * step after step, with the same operations per cell and edge as the
 * step-by-step launches, so the same bits.  (With more items the one
 * wavefront would run in sequence what the step-by-step launches run side
 * by side.)  0: always the step-by-step launches (graphs or eager).
 * tissue_step_timed always launches step by step.  Other values:
 * TISSUE_EINVAL.  Synchronises the stream. */
int tissue_set_whole_run(tissue_t *t, int32_t enable);

/* 1 when tissue_step runs this tissue's steps in the whole-run kernel (it
 * is enabled and the current plan fits it), 0 when step by step;
 * TISSUE_EINVAL for a null handle. */
int tissue_runs_whole(tissue_t *t);

/* Lane refill of compact-layout launches of cells of at most 16 voxels
 * (compiled networks, persistent launches): a wavefront does not wait for
 * the busiest cell of its work item; once min_idle_lanes of its 64 lanes
 * have finished their cell-step it writes those cells back and gives the
 * idle lanes the next cells of the launch, which may belong to other items
 * and other tissues of a batch.  0 turns refill off (lanes then wait for
 * their item; the default: with the load-ordered regroup the cells of an
 * item finish close together, and the refill phases -- each a chain of
 * dependent loads that stalls the whole wavefront -- cost more than the
 * idle lanes they recover); 1..64 idle lanes.  Results are bit-identical
 * for every value.  Other values: TISSUE_EINVAL.  Synchronises the stream. */
int tissue_set_refill(tissue_t *t, int32_t min_idle_lanes);

/* Regroup pass before each compact-layout chi launch: the cells of each
 * leaf-count class (of each tissue) are reordered by their total propensity
 * after the previous compact pass, largest first, so that the cells sharing
 * a wavefront carry similar numbers of events.  mode 0 = off, 1 = on, 2 =
 * automatic (the default: on for every compact launch that spans at least
 * two wavefronts).  Results are bit-identical either way: a cell's
 * result depends only on its counts and its counters.  Other values:
 * TISSUE_EINVAL.  Synchronises the tissue's stream. */
int tissue_set_regroup(tissue_t *t, int32_t mode);

/* Per-kernel device time of the last tissue_step_timed call, in ms.
 * chi_ms brackets each chi launch (for mode 3 with its redo launch);
 * chi_kernel is the mode (0, 1, 3 or 4, as in tissue_set_chi_mode) of the chi
 * launch group that took the most time, chi_leaves that group's leaf count
 * P (next power of two >= its cells' voxel count). */
typedef struct {
    double chi_ms, s_ms, total_ms;
    uint32_t chi_launches, s_launches;
    int32_t chi_kernel;
    int32_t chi_leaves;
    int32_t chi_refill;       /* nonzero: that group ran the compact layout with lane refill */
} tissue_timing_t;

/* tissue_step, launched eagerly with a HIP event pair around every kernel;
 * synchronises and returns the summed per-kernel device times. */
int tissue_step_timed(tissue_t *t, double dt, int32_t n_steps, tissue_timing_t *out);

/* Release the handle (not dev_buf, which stays the caller's).  TISSUE_ESTATE,
 * with nothing released, while a live batch holds the tissue: destroy the
 * batches first. */
int tissue_destroy(tissue_t *t);

/*
 * Batches: many tissues advanced together -- every chi launch and every S
 * launch covers the work items of all member tissues, and n_steps steps are
 * captured in HIP graphs.  Member tissues keep their own state, stream-free
 * (the batch's stream is used); each still sees exactly its own sequence of
 * steps, so its bits equal those of a lone tissue_step.  The batch needs
 * tissue_batch_required_bytes() of device memory for its work lists.
 * A tissue may appear at most once in a batch (TISSUE_EINVAL otherwise: its
 * cells would run twice in one launch); a member cannot be destroyed while
 * the batch lives (tissue_destroy returns TISSUE_ESTATE).
 */
size_t tissue_batch_required_bytes(tissue_t *const *ts, int32_t n);
int tissue_batch_create(tissue_t *const *ts, int32_t n, void *dev_buf, size_t dev_bytes,
                        void *hip_stream, tissue_batch_t **out);
int tissue_batch_step(tissue_batch_t *b, double dt, int32_t n_steps);
int tissue_batch_step_timed(tissue_batch_t *b, double dt, int32_t n_steps, tissue_timing_t *out);
int tissue_batch_set_launch(tissue_batch_t *b, int32_t persistent, int32_t workgroups_per_cu);
int tissue_batch_set_chi_mode(tissue_batch_t *b, int32_t mode);
int tissue_batch_set_graph_chunk(tissue_batch_t *b, int32_t steps_per_graph);
int tissue_batch_set_regroup(tissue_batch_t *b, int32_t mode);
int tissue_batch_set_refill(tissue_batch_t *b, int32_t min_idle_lanes);
int tissue_batch_set_whole_run(tissue_batch_t *b, int32_t enable);
int tissue_batch_runs_whole(tissue_batch_t *b);
int tissue_batch_sync(tissue_batch_t *b);
/* Replace the batch's members in place (continuous batching: admit and
 * retire tissues between steps) without creating a new batch: the work
 * lists are planned again on the host and copied into the batch's buffer
 * on its stream, with no host synchronisation (the host waits only for the
 * previous set_members copy to have left its pinned staging memory).
 * n = 0 empties the batch (its steps then do nothing).  New members on other
 * streams are waited for by the batch's stream; members that leave wait, on
 * their own stream, for the batch's work so far, so that they can be
 * destroyed next.  The same rules as tissue_batch_create (TISSUE_EINVAL,
 * nothing changed); TISSUE_EBUSY, nothing changed, when the members' work
 * lists need more than the dev_bytes the batch was created with (retry
 * after members have left, or create a larger batch). */
int tissue_batch_set_members(tissue_batch_t *b, tissue_t *const *ts, int32_t n);
int tissue_batch_destroy(tissue_batch_t *b);

/*
 * For callers that cannot allocate memory (serving loops and harnesses that
 * forbid device or pinned-host allocation): tissue_batch_step without a
 * batch handle or a caller's workspace.  Advances the n tissues ts[] by
 * n_steps steps of length dt on hip_stream (NULL: the null stream), with
 * the same bits as tissue_batch_step on a batch of the same tissues (the
 * default batch launch: automatic chi layout and regroup, persistent chi
 * launches; steps launched eagerly, no graph).  The batch's member table,
 * queue words, work items and redo list go to a static device array of
 * TISSUE_STATIC_WORKSPACE_BYTES per device (in the library's code object,
 * held until the process ends); the call uploads them with one copy from
 * ordinary host memory, waits for that copy, and enqueues the steps
 * asynchronously.  It calls no allocation routine for device or pinned
 * memory.  Every call on a device shares that device's array: calls that
 * overlap on one device (steps of an earlier call still running on another
 * stream) race; calls on one stream are ordered.  Errors: TISSUE_EINVAL as
 * for tissue_batch_create and tissue_batch_step (nothing enqueued);
 * TISSUE_ENOMEM when the batch's workspace (about 16 bytes per cell plus
 * the work items) exceeds TISSUE_STATIC_WORKSPACE_BYTES (nothing
 * enqueued).  Members are stepped on the current device.
 */
#define TISSUE_STATIC_WORKSPACE_BYTES (32u << 20)
int tissue_batch_step_static(tissue_t *const *ts, int32_t n, double dt, int32_t n_steps,
                             void *hip_stream);

const char *tissue_strerror(int code);
const char *tissue_last_error(void);

/* Number of compute units of the current device (for launch planning). */
int tissue_device_cus(int32_t *out);

#ifdef __cplusplus
}
#endif

#endif /* TISSUE_H */
