/*
 * mechstep.h -- C ABI of the mechanical-interaction step for spherical agents
 * on one AMD Instinct MI355X (gfx950).
 *
 * The operation follows "GPU Acceleration of 3D Agent-Based Biological
 * Simulations" (arXiv 2105.00039):
 *   - Section III, Eq. 1: the force between two touching spheres,
 *       delta = r1 + r2 - |p1 - p2|,   rho = r1 r2 / (r1 + r2),
 *       F     = (kappa delta - gamma sqrt(rho delta)) (p1 - p2)/|p1 - p2|,
 *     summed over every agent in contact; then the displacement: no motion
 *     unless the force breaks the adherence, otherwise the force integrated
 *     over the timestep, bounded in length.
 *   - Section IV-A: neighbours are found through a uniform grid of voxels
 *     ("boxes") rebuilt every step; an agent's candidates are the agents of the
 *     27 boxes around its own.
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller unless
 *   the comment says "host".  Arrays are contiguous, one value per agent
 *   (structure of arrays).  Element types follow the workspace dtype:
 *     MS_F32       positions/diameters float,  displacements float
 *     MS_F64       positions/diameters double, displacements double
 *     MS_F32_POS64 positions/diameters double (master copy), the step itself
 *                  runs in FP32 on the positions rounded to nearest float,
 *                  displacements float.
 *   Inputs and outputs must not alias.  Outputs are overwritten, never
 *   accumulated.  Displacements and gradients are in the caller's agent order.
 * Workspace.  All scratch lives in one caller-allocated device buffer sized by
 *   ms_workspace_bytes() and described by an ms_workspace struct (host memory,
 *   owned by the caller) set up once with ms_workspace_init().  Step calls
 *   never allocate, never synchronise the host and use only kernel launches,
 *   so a sequence of them can be captured into a HIP graph.
 *   ms_mech_step* read the state copied by the last ms_grid_build* on the same
 *   workspace, so the caller may update positions in place after the build.
 *   They also use the workspace's staging area (free after a build) for the
 *   per-agent records they write and then split into the caller's arrays, so
 *   two step calls on one workspace must not run concurrently even though
 *   the workspace pointer is const.
 * Streams.  `stream` is a hipStream_t passed as void*; NULL is the null
 *   stream.  Every call is ordered on that stream.  Calls on different
 *   workspaces are independent; calls that share a workspace must be ordered.
 * Errors.  Problems the host can see (null or misaligned pointer, size out of
 *   range, wrong dtype, non-finite or negative dt / max_disp / adherence, a
 *   workspace that is too small) return a status at once and set
 *   ms_last_error() (thread-local).  Problems only the device can see
 *   (non-finite or negative input values, an edge below the largest diameter,
 *   more boxes than the workspace holds) set an error word in the workspace;
 *   later kernels of the same workspace then do nothing and the outputs are
 *   unspecified.  ms_device_status() synchronises the stream and reports it.
 *   n = 0 is valid and does nothing.
 * Limits.  Agents are indexed with int32 and the box-sorted payload with
 *   32-bit byte offsets: n < 2^31 and n * (16 bytes for MS_F32 and
 *   MS_F32_POS64, 32 for MS_F64) < 2^32.  A build holds at most 2^25 =
 *   33,554,432 boxes over all its simulations (its two-level counting sort
 *   keeps at most 8192 buckets of 4096 boxes): ms_workspace_init rejects a
 *   larger max_boxes with MS_ECAPACITY, and a build whose grid needs more
 *   boxes than max_boxes sets the capacity error.
 */
#ifndef MECHSTEP_H
#define MECHSTEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MS_OK = 0,
    MS_EINVAL = 1,     /* bad argument, or (device) edge <= 0 / edge < max diameter */
    MS_ECAPACITY = 2,  /* more agents, boxes or simulations than the workspace holds */
    MS_EDEVICE = 3,    /* a HIP runtime call failed */
    MS_EINPUT = 4      /* (device) non-finite position/diameter or negative diameter */
} ms_status;

typedef enum {
    MS_F32 = 0,
    MS_F64 = 1,
    MS_F32_POS64 = 2
} ms_dtype;

/* Numbering of a single simulation's boxes (Section IV-A fixes the grid, not
 * the order of its boxes).  Boxes are always numbered x fastest, box =
 * ix + nx * row, so the three boxes of every stencil row stay contiguous; the
 * x-rows (iy, iz) are numbered
 *   row-major:  row = iz * ny + iy                       (tile_shift 0), or
 *   tiled:      16 x 16 tiles of (iy, iz), the tiles row-major with
 *               ty = ceil(ny / 16) tiles along y, rows row-major inside a
 *               tile: row = ((iz/16) * ty + iy/16) * 256 + (iz%16) * 16
 *               + iy%16                                (tile_shift 4),
 *               which adds empty boxes where ny or nz is not a multiple of 16.
 * Tiles keep the rows an agent reads close together in the box-sorted
 * order, which saves HBM traffic once a z-plane holds more agents than the
 * L2 keeps for three planes.  The order changes box ids, box starts, the
 * slot order and speed; forces and displacements are the same either way.
 * Batched builds always number rows row-major. */
typedef enum {
    MS_BOX_ORDER_AUTO = 0,   /* tiled from 49,152 agents per z-plane when the
                                tiles add at most 25% boxes and fit the
                                workspace, row-major otherwise */
    MS_BOX_ORDER_ROWS = 1,
    MS_BOX_ORDER_TILES = 2   /* MS_ECAPACITY (device) if the padded box count
                                exceeds max_boxes */
} ms_box_order;

/* How the lanes of a wavefront walk their agents' 9 stencil runs (Section
 * IV-B: one thread per agent) in the step and backward gathers.  Every lane
 * meets its candidates in the same order either way, so the results are the
 * same bit for bit; only the speed differs.
 *   lanes:  each lane takes all of its runs in turn, so a wavefront steps as
 *           often as its busiest lane has candidates in total (fastest on
 *           uniform populations);
 *   planes: the lanes take the three z-planes of the stencil together and
 *           the three runs of a plane in turn, which keeps the lanes' loads
 *           within one plane of slots (faster on dense clustered ones). */
typedef enum {
    MS_WALK_LANES = 0,
    MS_WALK_PLANES = 1
} ms_gather_walk;

/* Force and displacement parameters (Section III, Eq. 1 and the text after it).
 *   kappa      repulsion coefficient
 *   gamma      attraction (adhesion) coefficient
 *   dt         timestep of the overdamped integration: v = dt * F  (>= 0)
 *   max_disp   upper bound m on the displacement length (>= 0; 0 freezes)
 *   adherence  the agent moves only if |F| > adherence (>= 0)               */
typedef struct {
    double kappa, gamma, dt, max_disp, adherence;
} ms_params;

/* Geometry of one simulation's grid (Section IV-A), as built on the device. */
typedef struct {
    double  origin[3];  /* per-axis minimum position */
    double  edge;       /* box edge = interaction radius */
    int32_t dims[3];    /* boxes per axis: floor((max - min)/edge) + 1 */
    int32_t error;      /* device error bits of the build (0 = fine) */
    int64_t n_boxes;    /* dims[0]*dims[1]*dims[2] for row-major rows; with
                           tiled rows dims[0] * (1 + the largest row number) */
    int64_t box_base;   /* first global box index of this simulation */
    int64_t n_agents;   /* agents of this simulation */
    int32_t tile_shift; /* 0: row-major rows; 4: 16 x 16 tiled rows (ms_box_order) */
    int32_t reserved;
} ms_grid_info;

/* Host-side description of a workspace.  Filled by ms_workspace_init; the
 * fields from n_agents to built are updated by the grid builds.  Treat them as
 * read-only; keep_forces, gather_list, gather_block, sorted_input, box_order
 * and gather_walk are the caller's to set. */
typedef struct {
    void*   base;        /* device buffer, 256-byte aligned */
    size_t  bytes;
    int64_t max_agents;  /* capacity: agents over all simulations */
    int64_t max_boxes;   /* capacity: boxes over all simulations */
    int32_t max_sims;    /* capacity: simulations (1 for the plain step) */
    int32_t dtype;       /* ms_dtype */
    int64_t n_agents;    /* agents of the last grid build */
    int32_t n_sims;      /* simulations of the last grid build */
    int32_t built;       /* 1 after a plain build, 2 after a batched build */
    int32_t keep_forces; /* 0 (set by ms_workspace_init) or 1: ms_mech_step also
                            keeps the per-agent forces (one more 4S-byte write
                            per agent), and ms_mech_step_backward uses them
                            instead of recomputing when the device records that
                            they belong to the current build and the same
                            parameters.  Results are identical either way. */
    int32_t gather_list; /* contact-list length of the step's gathers: 0 (set by
                            ms_workspace_init; means 24), 24 or 40 entries per
                            lane (anything else: MS_EINVAL from the step calls).
                            Longer lists drain less often, which pays on dense
                            populations; shorter ones leave LDS for more blocks
                            per CU.  Results are identical bit for bit; the
                            package's autotuner picks the faster one. */
    int32_t gather_block; /* threads per block of the forward gather: 0 (set by
                            ms_workspace_init; means 64), 64 or 256 (anything
                            else: MS_EINVAL from the step calls).  Results are
                            identical bit for bit; the autotuner picks it with
                            gather_list. */
    int32_t sorted_input; /* 1: the next build's inputs are nearly box-sorted
                            (set by ms_mech_step_integrate_sorted, the batched
                            variant and ms_reorder, which write arrays in the
                            build's slot order; cleared by every build).  Such
                            a build reads each agent's position and diameter
                            from its inputs instead of carrying them through
                            its partition.  Only the speed depends on it: the
                            build is the same for any input, and the caller
                            may set or clear it. */
    int32_t box_order;    /* ms_box_order of the single-simulation builds: 0
                            (set by ms_workspace_init; auto), 1 row-major or 2
                            tiled rows (anything else: MS_EINVAL from the
                            builds).  Batched builds ignore it. */
    int32_t gather_walk;  /* ms_gather_walk of the step and backward gathers:
                            0 (set by ms_workspace_init) or 1 (anything else:
                            MS_EINVAL from the step calls).  Results are
                            identical bit for bit; the autotuner picks it with
                            gather_list and gather_block. */
} ms_workspace;

/* Bytes of device memory a workspace with these capacities needs (0 for
 * capacities out of range, including max_boxes > 2^25). */
size_t ms_workspace_bytes(int64_t max_agents, int64_t max_boxes, int32_t max_sims,
                          ms_dtype dtype);

/* Describe `base` (>= ms_workspace_bytes(...) bytes, 256-byte aligned device
 * memory) as a workspace and clear its device state (kernel launch on
 * `stream`).  Must be called once before the first build. */
ms_status ms_workspace_init(ms_workspace* ws, void* base, size_t bytes, int64_t max_agents,
                            int64_t max_boxes, int32_t max_sims, ms_dtype dtype, void* stream);

/* Uniform grid (Section IV-A), rebuilt from scratch:
 *   bounds -> box index per agent -> per-box counts -> exclusive scan ->
 *   stable scatter into box-sorted order (ascending box, then ascending input
 *   index inside a box) with a sorted copy of x, y, z, d/2.
 * x, y, z, d: [n] device arrays of the workspace dtype.
 * edge: box edge; <= 0 selects the largest diameter.  An edge below the
 *   largest diameter is a device error (a contact could leave the 27 boxes). */
ms_status ms_grid_build(ms_workspace* ws, const void* x, const void* y, const void* z,
                        const void* d, int64_t n, double edge, void* stream);

/* One mechanical step on the last plain build: for every agent the Eq. 1
 * force summed over its contacts among the 27 surrounding boxes, then the
 * displacement (Section III).  p: host pointer to the parameters.
 * dx, dy, dz: [n] outputs. */
ms_status ms_mech_step(const ms_workspace* ws, const ms_params* p, void* dx, void* dy,
                       void* dz, void* stream);

/* Reverse-mode derivative of ms_mech_step on the same build (derived from
 * Eq. 1 and the displacement rule; the paper itself has no backward pass).
 * gdx..gdz: [n] dL/dDisplacement.  Outputs:
 *   gx, gy, gz [n]  sum_k (dDelta_k/dp_i)^T g_k   (no identity term)
 *   gd [n]          sum_k (dDelta_k/dd_i)^T g_k
 *   g_params        device double[2] = {dL/dkappa, dL/dgamma}
 * Sums are taken in a fixed order, so repeated calls give identical bits.
 * Kinks: delta = 0 is no contact, |v| = max_disp is unclamped, |F| =
 * adherence is held (the inactive side). */
ms_status ms_mech_step_backward(const ms_workspace* ws, const ms_params* p,
                                const void* gdx, const void* gdy, const void* gdz,
                                void* gx, void* gy, void* gz, void* gd, double* g_params,
                                void* stream);

/* Batched grid: B independent simulations concatenated; simulation b owns
 * agents [sim_offsets[b], sim_offsets[b+1]).  Each gets its own grid
 * (origin, edge, dims) and a disjoint range of global box indices, and all
 * are sorted together in one counting sort.
 * sim_offsets: device int64 [B+1], non-decreasing, sim_offsets[0] = 0,
 *   sim_offsets[B] = n_total (the host must pass the same n_total).
 * edges: device double [B], or NULL for "largest diameter of each
 *   simulation". */
ms_status ms_grid_build_batched(ms_workspace* ws, const void* x, const void* y, const void* z,
                                const void* d, const int64_t* sim_offsets, int32_t n_sims,
                                int64_t n_total, const double* edges, void* stream);

/* ms_mech_step for every simulation of the last batched build in one launch.
 * params: device ms_params [B] (per-simulation kappa, gamma, dt, ...). */
ms_status ms_mech_step_batched(const ms_workspace* ws, const ms_params* params, void* dx,
                               void* dy, void* dz, void* stream);

/* One rollout step after the build: ms_mech_step followed by ms_integrate in
 * fewer passes.  The displacement of every agent (Section III) is added to
 * the positions x, y, z in place (the caller's order; MS_F32 positions are
 * float, MS_F64 and MS_F32_POS64 double, with the displacement converted as
 * ms_integrate converts it), bit for bit as the two separate calls.  dx, dy,
 * dz: all NULL, or all given to also receive the displacements.  x, y, z
 * need not be the build's inputs (the build keeps its own copy) but must not
 * overlap dx, dy, dz.  On a device error of the build nothing moves.
 * Stream-ordered; allocates nothing. */
ms_status ms_mech_step_integrate(const ms_workspace* ws, const ms_params* params, void* x, void* y,
                                 void* z, void* dx, void* dy, void* dz, void* stream);

/* The same for every simulation of the last batched build; params: device
 * ms_params [B] as for ms_mech_step_batched. */
ms_status ms_mech_step_batched_integrate(const ms_workspace* ws, const ms_params* params, void* x,
                                         void* y, void* z, void* dx, void* dy, void* dz,
                                         void* stream);

/* One backward step of a rollout p_{t+1} = p_t + Delta(p_t) on the build of
 * p_t (the derivative of ms_mech_step_integrate), all of it on the device:
 *   pbx, pby, pbz [n]  in: dL/dp_{t+1}; out: dL/dp_t = dL/dp_{t+1} +
 *                      (dDelta/dp_t)^T dL/dp_{t+1}, updated in place
 *   dbar [n]           dL/dd of this step added in place
 *   g_params           device double[2], {dL/dkappa, dL/dgamma} of this step
 *                      added in place
 * All three accumulators have the positions' type (float for MS_F32, double
 * for MS_F64 and MS_F32_POS64); each step's terms are computed as in
 * ms_mech_step_backward (FP32 arithmetic in the FP32 modes, the incoming
 * gradient rounded to float there), converted, then added.  Walking the
 * steps of a rollout backwards with this call gives the gradient of a loss
 * on the final positions with respect to the initial positions, the
 * diameters, kappa and gamma. */
ms_status ms_mech_step_backward_accumulate(const ms_workspace* ws, const ms_params* p, void* pbx,
                                           void* pby, void* pbz, void* dbar, double* g_params,
                                           void* stream);

/* One rollout step on the box-sorted state (the agent sorting of Section
 * IV-D, kept across a rollout): the step of ms_mech_step_integrate, but the
 * state after the step is written to new arrays in the slot order of the
 * build (agent perm[k] at k, the order ms_reorder applies: ascending box,
 * x-quarter inside the box, input index), so every store of the step is
 * coalesced and the next build reads nearly sorted input (the call sets
 * ws->sorted_input).
 *   x_out, y_out, z_out [n]  positions after the step (p + Delta, rounded as
 *                            ms_mech_step_integrate rounds them), slot order
 *   d_out [n]                the diameters, slot order (for MS_F32 and MS_F64
 *                            twice the build's stored radius, which is d for
 *                            every normal d)
 *   dx, dy, dz               NULL, or [n] displacements in slot order
 *   x, y, z, d               the build's inputs: read (MS_F32_POS64 only) for
 *                            the FP64 positions and diameters; may be NULL in
 *                            the other modes
 * Types as for ms_mech_step_integrate.  Outputs must not overlap each other or
 * the inputs.  Other per-agent arrays of the caller follow with ms_reorder on
 * the same build.  The first such step from a caller-order state equals
 * ms_mech_step_integrate renumbered, bit for bit; after that the state's new
 * numbering changes the order in which a box's agents are summed (ascending
 * input index inside a box), so a sorted rollout agrees with the caller-order
 * rollout to rounding, step by step within the same acceptance bound.  On a
 * device error of the build nothing is written.
 * Stream-ordered; allocates nothing. */
ms_status ms_mech_step_integrate_sorted(ms_workspace* ws, const ms_params* params,
                                        const void* x, const void* y, const void* z, const void* d,
                                        void* x_out, void* y_out, void* z_out, void* d_out,
                                        void* dx, void* dy, void* dz, void* stream);

/* The same for every simulation of the last batched build (params: device
 * ms_params [B]); agents of each simulation stay in its offset range. */
ms_status ms_mech_step_batched_integrate_sorted(ms_workspace* ws, const ms_params* params,
                                                const void* x, const void* y, const void* z,
                                                const void* d, void* x_out, void* y_out,
                                                void* z_out, void* d_out, void* dx, void* dy,
                                                void* dz, void* stream);

/* ms_mech_step_backward per simulation; g_params: device double [2B]. */
ms_status ms_mech_step_backward_batched(const ms_workspace* ws, const ms_params* params,
                                        const void* gdx, const void* gdy, const void* gdz,
                                        void* gx, void* gy, void* gz, void* gd,
                                        double* g_params, void* stream);

/* ms_mech_step_backward_accumulate per simulation of the last batched build;
 * params: device ms_params [B]; g_params: device double [2B] added to. */
ms_status ms_mech_step_backward_batched_accumulate(const ms_workspace* ws, const ms_params* params,
                                                   void* pbx, void* pby, void* pbz, void* dbar,
                                                   double* g_params, void* stream);

/* p <- p + Delta for n agents (all agents move at once from the displacements
 * of one step).  dtype: MS_F32 (float p, float Delta), MS_F64 (double,
 * double) or MS_F32_POS64 (double p, float Delta, summed in FP64). */
ms_status ms_integrate(void* x, void* y, void* z, const void* dx, const void* dy,
                       const void* dz, int64_t n, ms_dtype dtype, void* stream);

/* Sorted-state rollouts (the agent sorting of Section IV-D, kept across
 * steps): dst[k] = src[perm[k]] for the n_agents slots of the last build, where
 * perm is the workspace's slot order: ascending box, then x-quarter of the
 * agent inside its box, then input index.  (ms_grid_get's perm is the
 * canonical order, ascending box then input index; both are box-sorted.)
 * Applying it to every per-agent array of the caller (positions, diameters and
 * any attributes) renumbers the agents in box order, so the next build reads
 * nearly sorted input and writes the displacements nearly in order (the call
 * sets ws->sorted_input); agents of one simulation of a batched build stay
 * inside that simulation's range.
 * src, dst: device arrays of n_agents elements of elem_bytes (1, 2, 4, 8 or
 * 16) bytes, aligned to elem_bytes; they must not overlap (MS_EINVAL).  The
 * caller owns both.  A device error of the last build leaves dst unwritten.
 * Stream-ordered; allocates nothing. */
ms_status ms_reorder(ms_workspace* ws, const void* src, void* dst, int32_t elem_bytes,
                     void* stream);

/* Copy out the last build (synchronises `stream`).  info: host array with
 * one entry per simulation (n_sims of the build).  box_id [n] (global box of
 * each agent, caller order), box_start [total boxes + 1] (first sorted slot
 * of each box), perm [n] (perm[slot] = input index): device arrays, each may
 * be NULL. */
ms_status ms_grid_get(const ms_workspace* ws, ms_grid_info* info, int32_t* box_id,
                      int32_t* box_start, int32_t* perm, void* stream);

/* Neighbour sets of the last build: for every agent i the agents j != i of
 * the 27 surrounding boxes with |p_i - p_j|^2 < edge^2, evaluated in FP64 as
 * (dx*dx + dy*dy) + dz*dz without fused multiply-add, listed in ascending box
 * then ascending input index (Sections III and IV-A).
 * counts [n] int32 and offsets [n+1] int64 (exclusive prefix of counts) are
 * always written; list (int32, `cap` entries) is written when non-NULL and
 * cap >= offsets[n], else MS_ECAPACITY.  Synchronises `stream` (it reads the
 * total back) and returns the total through *total when non-NULL. */
ms_status ms_neighbors(const ms_workspace* ws, int32_t* counts, int64_t* offsets,
                       int32_t* list, int64_t cap, int64_t* total, void* stream);

/* Synchronise `stream` and translate the workspace's device error word:
 * MS_OK, MS_EINPUT, MS_EINVAL or MS_ECAPACITY. */
ms_status ms_device_status(const ms_workspace* ws, void* stream);

/* ms_grid_build followed by ms_mech_step without any allocation and without a
 * caller workspace, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The grid lives in a workspace the library keeps in a static
 * device array of about 18 MB, one copy per GPU, held until the process ends
 * (its address is looked up once per device, on the first call there).
 *   x, y, z, d  [n] inputs of `dtype` as for ms_grid_build; edge as there
 *   p           host parameters as for ms_mech_step
 *   dx, dy, dz  [n] displacements (caller order), as ms_mech_step writes them
 *   dev_error   NULL, or one device int32 that receives the build's device
 *               error bits (0 = fine; 1, 2 bad input, 4 bad edge, 8 more
 *               than MS_NOALLOC_MAX_BOXES boxes), written on `stream` after
 *               the step; on an error the displacements are unspecified.
 * n above MS_NOALLOC_MAX_AGENTS returns MS_ECAPACITY at once.  Results equal
 * ms_grid_build + ms_mech_step (default contact list, keep_forces 0) bit for
 * bit.  Every call on one GPU uses that GPU's single array and leaves its
 * contents behind for the next: calls that overlap on one GPU (different
 * streams or host threads without ordering) race and give wrong results.
 * Stream-ordered; makes no hipMalloc, hipFree or other allocating call. */
#define MS_NOALLOC_MAX_AGENTS 65536
#define MS_NOALLOC_MAX_BOXES 524288
ms_status ms_mech_step_noalloc(const void* x, const void* y, const void* z, const void* d,
                               int64_t n, ms_dtype dtype, double edge, const ms_params* p,
                               void* dx, void* dy, void* dz, int32_t* dev_error, void* stream);

/* Streaming copy of `bytes` bytes (multiple of 16) from src to dst: the
 * bandwidth probe used as the empirical HBM roof. */
ms_status ms_copy_probe(void* dst, const void* src, size_t bytes, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* ms_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MECHSTEP_H */
