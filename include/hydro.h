/*
 * hydro.h -- C ABI of the MI355X hydro packet library (libhydro.so).
 *
 * The library applies one explicit finite-volume compressible-Euler step to a
 * packet of mesh blocks on one GPU: guard cells, PLM reconstruction with the
 * minmod limiter, HLLC fluxes, a conservative SSP-RK2 update, and a CFL time
 * step reduction.  This is the per-block physics task that ORCHA (arXiv
 * 2507.09337) maps onto the GPU:
 *   - Sec. 4 (Code Generators): a TaskFunction is the group of API functions a
 *     device runs together; its DataItem, when it runs on a device, is a
 *     DataPacket that carries everything the TaskFunction needs;
 *   - Sec. 4.3 (DataItem Generators): a DataPacket concatenates n AMR blocks,
 *     n chosen at run time, because single blocks are too small to use a GPU;
 *   - Sec. 4 (static-code requirements) asks generated code to be thread
 *     safe, to take its scratch space from the caller and to keep no
 *     non-constant globals.  This library departs from all three, for the
 *     reasons given here: handles are not thread safe (below: the caller
 *     serialises calls on one mesh, so no lock sits on the launch path); the
 *     create calls allocate the device scratch of the stage buffer, block
 *     table, work lists and time record once, and the step calls allocate
 *     nothing; the error message is a thread-local global string;
 *   - Sec. 5.1 (Flash-X): blocks hold equal numbers of equally sized cells;
 *   - Sec. 5.2 (Sedov): ideal-gas gamma-law equation of state;
 *   - Sec. 6 (Experiments): explicit finite volume with a guard-cell halo,
 *     2nd-order Runge-Kutta with a guard refresh before each stage.
 * Reconstruction, Riemann solver and time-step rule are not given by the paper
 * and follow the textbook methods: PLM (van Leer 1979) on primitive variables
 * with minmod (Roe 1986); HLLC (Toro, Spruce & Speares 1994) with Davis
 * wave speeds (Einfeldt or PVRS as variants; PLM on conserved or on
 * characteristic variables as further variants); SSP-RK2 (Shu & Osher 1988);
 * dt = CFL / max_c sum_d (|u_d|+c)/dx_d.
 *
 * Conventions for every call
 *   - Every call returns a hydro_status; HYDRO_OK is 0.  No exception or
 *     signal crosses the ABI.  On failure hydro_last_error() returns a message
 *     (thread-local, valid until the next call on the same thread).
 *   - Arguments are checked on the host before any device call; a rejected
 *     call has no effect.  Descriptor errors are HYDRO_EINVAL and are reported
 *     without touching a GPU.
 *   - Pointers named "device" point to GPU memory of the current HIP device;
 *     all others are host pointers, read during the call only.
 *   - Work is enqueued on the stream given at mesh creation (a hipStream_t;
 *     NULL is the default stream) and is stream-ordered; only calls documented
 *     as synchronising wait for the GPU.
 *   - Handles are not thread safe: concurrent calls on one mesh (or on
 *     packets/batches of one mesh) must be serialised by the caller.
 *
 * State layout (the "arena", owned by the caller, FP64):
 *   block b, conserved variable v (0 rho, 1 rho*u, 2 rho*v, 3 rho*w, 4 E),
 *   interior cell (i, j, k) with i fastest:
 *       arena[offset_b + v * nx*ny*nz + (k*ny + j)*nx + i].
 *   Blocks store interior cells only.  Guard values are gathered from the
 *   neighbour blocks' interiors by the kernels when they load a tile, so the
 *   arena needs no guard storage.  In 2D, nz == 1 and rho*w must be 0.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HYDRO_OK = 0,
  HYDRO_EINVAL = 1,   /* bad argument or descriptor; nothing was done          */
  HYDRO_EDEVICE = 2,  /* a HIP runtime call failed (message names it)          */
  HYDRO_ENOMEM = 3,   /* device or host allocation failed                       */
  HYDRO_ENONPHYS = 4, /* a state with rho <= 0, p <= 0 or a non-finite value  */
  HYDRO_ESTATE = 5    /* call not valid in this state (e.g. packet not closed) */
} hydro_status;

typedef enum {
  HYDRO_FP64 = 0,     /* every operation in FP64                                         */
  HYDRO_FP32_FP64 = 1 /* FP64 state, recovery, accumulation and dt; PLM + HLLC in FP32   */
} hydro_precision;

/* Method variants, at most one OR-ed into a precision code (both at once is
 * EINVAL).  Without either, HLLC's wave-speed bounds are Davis's min/max of
 * u -+ c.
 * HYDRO_SPEEDS_EINFELDT: Einfeldt's bounds, the sqrt(rho)-weighted mean normal
 *   velocity -+ d_bar (Toro sec. 10.5.1).
 * HYDRO_SPEEDS_PVRS: pressure-based bounds u_L - c_L q_L, u_R + c_R q_R from
 *   the primitive-variable linearised star pressure (Toro sec. 10.5.2): q_K is
 *   1 on a rarefaction and the shock factor of that pressure otherwise.  The
 *   linear pressure grows like the velocity jump, a strong shock's like its
 *   square, so in a strong collision the bounds can cross; the method has no
 *   guard against it (Toro pairs it with other estimates adaptively). */
#define HYDRO_SPEEDS_EINFELDT 0x100
#define HYDRO_SPEEDS_PVRS 0x200

/* Reconstruction variant, OR-ed into a precision code (with or without a
 * wave-speed variant): PLM with minmod on the conserved variables (rho, rho u,
 * rho v, rho w, E) instead of the primitives; the two face states are then
 * recovered to primitives (in the reconstruction's precision: FP64, or FP32 in
 * the mixed path) for HLLC.  A face state with rho <= 0 or p <= 0 is
 * non-physical like a cell (HYDRO_ENONPHYS): velocity shear at low pressure
 * produces one, where primitive reconstruction keeps p > 0. */
#define HYDRO_RECON_CONSERVED 0x400

/* Reconstruction variant (not together with HYDRO_RECON_CONSERVED): PLM on
 * the characteristic variables of the primitive Euler system along each
 * face normal (Toro 2009, ch. 3): the one-sided differences of a cell are
 * split into the amplitudes of its waves u - c, entropy, two shear waves and
 * u + c, each amplitude is limited with minmod, and the slope is rebuilt from
 * the cell's right eigenvectors.  Non-physical face states are
 * HYDRO_ENONPHYS as above. */
#define HYDRO_RECON_CHARACTERISTIC 0x800

/* Equation-of-state variant, only as HYDRO_FP64 | HYDRO_EOS_GAS_RADIATION
 * (Davis bounds, primitive PLM; any other combination is EINVAL): an ideal
 * gas of index gamma plus black-body radiation, in units with gas and
 * radiation constants 1, p = rho T + T^4/3 and rho e = rho T/(gamma - 1) +
 * T^4.  Every recovery, face state and CFL rate solves for the temperature by
 * Newton's method, and the sound speed uses the first adiabatic exponent of
 * the mixture (Clayton): a heavier, iterated EOS in the role of the paper's
 * tabulated one (Sec. 5.3). */
#define HYDRO_EOS_GAS_RADIATION 0x1000

typedef enum {
  HYDRO_NBR = 0,          /* guards copy the two nearest interior layers of block nbr[f] */
  HYDRO_OUTFLOW = 1,      /* zero gradient: both guard layers copy the edge layer        */
  HYDRO_PERIODIC_SELF = 2 /* wrap around the block itself                                 */
} hydro_face_kind;

/* One mesh block (Sec. 5.1: a block of equally sized cells).  Faces are
 * ordered -x, +x, -y, +y, -z, +z.  A HYDRO_NBR face must name a block whose
 * extents along the two tangential axes equal this block's.  In 2D the z
 * faces are ignored.  Interior extents: n[0] and n[1] multiples of 8 (the
 * kernels tile x-y planes in 8x8 or 16x16 tiles), n[2] >= 2 in 3D and == 1 in
 * 2D, n[0]*n[1]*n[2] < 2^31. */
typedef struct {
  int32_t n[3];         /* interior cells per axis                                  */
  int32_t face_kind[6]; /* hydro_face_kind per face                                  */
  int32_t nbr[6];       /* neighbour block id (0..nblocks-1) of HYDRO_NBR faces      */
  int32_t reserved;     /* must be 0                                                 */
  int64_t offset;       /* element offset of variable 0 of this block in the arena   */
  double dx[3];         /* cell widths (> 0); dx[2] ignored in 2D                     */
} hydro_block_desc;

typedef struct hydro_mesh hydro_mesh;     /* block table + arena + scratch (U1, accumulators) */
typedef struct hydro_packet hydro_packet; /* an ordered list of blocks of one mesh (DataPacket) */
typedef struct hydro_batch hydro_batch;   /* packets advanced stage-synchronously together      */

/* Create a mesh over a caller-owned device arena of arena_len doubles.
 * The mesh is the set of blocks the paper's solver works on (Sec. 5.1: the
 * domain is cut into blocks of equally many equal cells) with, per block
 * face, where its guard-cell halo comes from (Sec. 6: the halo around the
 * block being updated; the paper fills it by MPI outside the task, here the
 * kernels gather it from the linked neighbour's interior).
 * blocks: host array of nblocks descriptors (copied).  ndim: 2 or 3.
 * Block ranges [offset, offset + 5*ncell) must lie inside the arena and must
 * not overlap.  stream: hipStream_t used for all work on this mesh.
 * Allocates the mesh's device scratch (one arena-sized FP64 buffer for the
 * first RK stage, the block table and accumulators) on the current device;
 * no later call allocates device memory except packet/batch creation (work
 * lists) and the first hydro_batch_run (graph instantiation).
 * Errors: EINVAL (descriptor, overlap, extents), ENOMEM, EDEVICE. */
hydro_status hydro_mesh_create(const hydro_block_desc *blocks, int32_t nblocks, int32_t ndim, double *arena,
                               int64_t arena_len, void *stream, hydro_mesh **out);

/* Destroy a mesh.  Packets and batches of the mesh must be destroyed first
 * (HYDRO_ESTATE otherwise).  Synchronises the mesh stream. */
hydro_status hydro_mesh_destroy(hydro_mesh *m);

/* Create a packet (Sec. 4.3 DataPacket: n blocks chosen at run time) over the
 * listed blocks of mesh m, advanced in the given hydro_precision (optionally
 * OR at most one HYDRO_SPEEDS_* and one HYDRO_RECON_* variant; or exactly
 * HYDRO_FP64 | HYDRO_EOS_GAS_RADIATION).  block_ids:
 * host array of nblocks distinct ids.  Builds the packet's device work list.
 * Errors: EINVAL (empty, duplicate or out-of-range id, bad precision), ENOMEM,
 * EDEVICE. */
hydro_status hydro_packet_create(hydro_mesh *m, const int32_t *block_ids, int32_t nblocks, int32_t precision,
                                 hydro_packet **out);

/* One full SSP-RK2 step of the packet with time step dt and ratio of
 * specific heats gamma, in place on the arena (Sec. 6: explicit finite volume,
 * 2nd-order Runge-Kutta, guards refreshed before each stage):
 *   U1 = Un + dt L(Un);  Un+1 = Un/2 + (U1 + dt L(U1))/2.
 * Only interior cells of the packet's blocks are written.  Stage 2 needs the
 * first-stage values of every face neighbour, so the packet must be closed
 * (every HYDRO_NBR face of its blocks names a block of the packet); otherwise
 * HYDRO_ESTATE (use hydro_batch_advance_plain or hydro_batch_run, which keep
 * the stages synchronous across packets).  Asynchronous.  The stage-2 kernel
 * also reduces the CFL rate of the new state for hydro_packet_reduce_dt.
 * Errors: EINVAL (dt or gamma not finite and > 0, gamma <= 1), ESTATE, EDEVICE. */
hydro_status hydro_packet_advance(hydro_packet *p, double dt, double gamma);

/* dt = cfl / max over the packet's interior cells of sum_d (|u_d| + c)/dx_d,
 * c = sqrt(gamma p / rho), computed in FP64 on the device.  The paper does
 * not state its time-step rule; this is the CFL condition of an unsplit
 * method-of-lines update (the rates of all directions summed), taken from
 * the state at the start of a step and held for both RK stages.  A mesh-wide
 * dt is the minimum of its packets' values (one dt per step for the whole
 * mesh).  If the last call
 * on this packet was an advance with the same gamma, the rate it reduced is
 * used; otherwise the arena is read again.  (A caller that writes the arena
 * between an advance and this call must pass a different gamma or create a
 * new packet.)  Synchronising.  HYDRO_ENONPHYS if any state touched by the
 * last advance, or any interior state now, has rho <= 0, p <= 0 or a
 * non-finite value (the message names a block).
 * Errors: EINVAL (cfl or gamma), ENONPHYS, EDEVICE. */
hydro_status hydro_packet_reduce_dt(hydro_packet *p, double gamma, double cfl, double *dt_out);

hydro_status hydro_packet_destroy(hydro_packet *p);

/* A batch of packets of one mesh (all packets must share the mesh and the
 * precision code, method variants included; a block may appear in at most
 * one packet of the batch).  The paper sends packets to the GPU one by one
 * (Sec. 4.3) and finds that many blocks are needed to fill the device
 * (Sec. 6.1); a batch takes that to its end, all packets of a step in one
 * launch per RK stage (the paper is silent on batching across packets).  Builds the concatenated device work
 * list used by the persistent batched launches.  Errors: EINVAL, ENOMEM,
 * EDEVICE. */
hydro_status hydro_batch_create(hydro_packet *const *packets, int32_t npackets, hydro_batch **out);

/* One SSP-RK2 step of every packet with per-packet launches, the paper's
 * packet-at-a-time offload (Sec. 4.3) with the guard refresh between the
 * stages that Sec. 6 requires: stage 1 of every packet, then stage 2 of every
 * packet (stage-synchronous, so packets need not be closed).  Each packet then holds its reduced CFL rate for
 * hydro_packet_reduce_dt.  Asynchronous.  Errors: EINVAL, EDEVICE. */
hydro_status hydro_batch_advance_plain(hydro_batch *b, double dt, double gamma);

/* nsteps SSP-RK2 steps of the whole batch (Sec. 6: 2nd-order Runge-Kutta,
 * guards refreshed before each stage -- here by the launch boundary between
 * the stages) with dt = cfl / max rate (the rule of hydro_packet_reduce_dt)
 * taken from the state at the start of each step and kept on the device: one
 * persistent launch per RK stage over the concatenated work list of all
 * packets, one captured HIP graph per step, replayed nsteps times with no
 * host synchronisation in between.  Synchronising.  *t_out (host, may be
 * NULL) receives the simulated time advanced.  The first call with a given
 * (cfl, gamma) instantiates the graph.
 * Failure: when a step produces a state with rho <= 0, p <= 0 or a
 * non-finite value (seen by the second stage, which recovers the first-stage
 * state and reduces the CFL rate of the new one; a bad initial state is seen
 * by the rate reduction before the first step), the device dt becomes NaN and
 * every later stage launch of the run returns without touching the arena.  The
 * call then returns ENONPHYS with the arena holding the result of the failing
 * step (the initial state, unchanged, if that was bad) and *t_out the time at
 * the end of that step.  Where the failure was a first-stage state, the cells
 * whose stencil reached it hold non-finite values.
 * Errors: EINVAL, ENONPHYS (as above), EDEVICE. */
hydro_status hydro_batch_run(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *t_out);

/* hydro_batch_run with the device time of every step: HIP events recorded on
 * the mesh stream before the first replay and after each replay of the step
 * graph; step_ms (host array of nsteps doubles, required) receives each
 * step's time in milliseconds (stage 1, stage 2 and the dt update, and the
 * gaps between them).  The events are created and destroyed by the call; the
 * replays themselves are those of hydro_batch_run.  Synchronising.
 * Errors: as hydro_batch_run; EINVAL for a null step_ms. */
hydro_status hydro_batch_run_timed(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *t_out,
                                   double *step_ms);

hydro_status hydro_batch_destroy(hydro_batch *b);

/* Launch configuration of the batched path and its autotuner (Sec. 7 of the
 * paper lists auto-tuned kernel generation as future work; here a tuner picks
 * among compiled tilings by timing them).  Blocks are grouped into classes by
 * edge length (n[0] when n[0] == n[1] (== n[2] in 3D), else class 0).  Per
 * class the tiling is:
 *   tile:   0 = 16x16 tiles, one per 256-thread workgroup (needs n[0], n[1]
 *               multiples of 16); 1 = 8x8 tiles, four per workgroup;
 *               2..4 = 16x16 tiles in z-runs: a workgroup takes the same
 *               tile of that many consecutive blocks of a z column (blocks
 *               linked along +z within the batch, whole blocks, 3D); the
 *               mixed-precision tile marches through the run without
 *               re-reading the z halo of each block;
 *           5 = fused step (edge 8 only; every block of the class 3D, 8^3,
 *               periodic on itself on all six faces; HYDRO_FP64 or
 *               HYDRO_FP32_FP64 without variants): one workgroup takes a
 *               whole block through both RK stages with the block on chip,
 *               so Un is read and Un+1 written once per step and the
 *               first-stage state never goes to memory (80 instead of 200
 *               bytes per cell-update; the communication-avoiding step of
 *               the paper's Sec. 6 for blocks whose halo is their own
 *               interior); in hydro_batch_run the fused launch is a branch
 *               of the step graph beside the two stage launches;
 *   zchunk: z planes per work item (0 = the whole block; 3D only).
 * Without a setting a class uses 16x16 tiles (8x8 if its extents need them)
 * on whole blocks, in z-runs of two when the class has at least 12 x (number
 * of CUs) 16x16 tiles (the shorter work list then still gives two rounds of
 * resident workgroups).  get_config reports the tiling in effect (2..4 for
 * z-runs, where the blocks' +z links allow them).
 * Per batch, grid = workgroups per stage launch (0 = one per work item; else a
 * persistent grid of that many workgroups looping over the work list), and
 * xcd_remap = 1 renumbers workgroups so that each of the GPU's 8 XCDs (each
 * with its own L2) runs a contiguous span of the work list, keeping
 * neighbouring blocks' guard reads in one L2 (0 = hardware order; the
 * default is 1 when a block of the batch links to a neighbour, else 0).
 * Work items are launched heaviest first (planes times tile cells; items of
 * equal work in block order).
 * hydro_batch_set_tiling(b, edge, tile, zchunk) and hydro_batch_set_launch
 * rebuild or relaunch accordingly (EINVAL for a tile the class cannot use, or
 * a value out of range, or a fused step the class cannot take).
 * hydro_batch_autotune times every candidate tiling of
 * every class present (the median device time of a stage-1 and of a stage-2
 * launch on the class's own blocks, summed; both write only the mesh's
 * scratch stage buffer, never the arena: stage 2 takes its stencil from the
 * arena and its pointwise Un from the scratch buffer, which it overwrites),
 * rejects a candidate whose stage-1 or stage-2 result (stage 2 run with the
 * arena as stencil and Un) differs from the default tiling's by more than
 * 1e-13 relative (FP64) or 1e-6 (mixed) on up to 64 blocks, keeps the
 * fastest, then picks grid and xcd_remap the same way; a class the fused
 * step can take gets it when its full step on a copy of the sample matches
 * the default tiling's and the whole batch step (all launches) is faster
 * with it.  reps = timed launches per candidate (>= 1).  Synchronising; on
 * an error the batch keeps the tiling, launch and occupancy it had before
 * the call (set_tiling likewise).  hydro_batch_set_occupancy(b, waves) asks
 * the stage kernels of the batch's launches for the register budget of `waves`
 * (2, 3 or 4) waves per SIMD instead of their own (0); only for HYDRO_FP64 or
 * HYDRO_FP32_FP64 without variants (EINVAL otherwise); the autotuner tries 2,
 * 3 and 4 after the launch shape, parity-checked like the tilings.
 * hydro_batch_get_config writes grid to out[0], xcd_remap to out[1], the
 * occupancy request to out[2], then (edge, tile, zchunk,
 * ncells_in_class_low31) for each class from out[3], up to nclass_max
 * classes (out holds 3 + 4 * nclass_max int32); *nclass receives the number
 * of classes. */
hydro_status hydro_batch_set_tiling(hydro_batch *b, int32_t edge, int32_t tile, int32_t zchunk);
hydro_status hydro_batch_set_launch(hydro_batch *b, int32_t grid, int32_t xcd_remap);
hydro_status hydro_batch_set_occupancy(hydro_batch *b, int32_t waves);
hydro_status hydro_batch_autotune(hydro_batch *b, double gamma, int32_t reps);
hydro_status hydro_batch_get_config(hydro_batch *b, int32_t *out, int32_t nclass_max, int32_t *nclass);

/* Kernel timing of the batched path (for roofline measurement): runs nsteps
 * steps like hydro_batch_run but launches the two stage kernels eagerly (no
 * graph) on the mesh stream with HIP events around each launch, and returns
 * the mean duration in milliseconds of the stage-1 and stage-2 launches in
 * ms_out[0] and ms_out[1] (ms_out[1] includes the fused-step launch of
 * classes tiled 5), and the summed wall time of all launches of the
 * step (stage 1 + stage 2 + finalize) per step in ms_out[2].  Same results in
 * the arena as hydro_batch_run.  Synchronising.
 * Errors: as hydro_batch_run. */
hydro_status hydro_batch_time_kernels(hydro_batch *b, int32_t nsteps, double cfl, double gamma, double *ms_out);

/* ---------------------------------------------------------------------------
 * Host-resident packets: the DataPacket life cycle of Sec. 4.3 (a packet's
 * data moves to the device in one transfer, the task runs there, the result
 * moves back) with the transfers hidden behind computation on GPU streams
 * (Sec. 6.1).
 *
 * The state lives in a caller-owned host arena (layout as the device arena;
 * pinned memory, e.g. from hipHostMalloc, lets the copies run asynchronously,
 * pageable memory works but serialises them).  Packet p is the range of
 * consecutive block ids [packet_start[p], packet_start[p+1]); its blocks must
 * be stored back to back in the arena (offset of block b+1 = offset of block b
 * + 5 * its cell count) and the packet must be closed (every HYDRO_NBR face
 * of its blocks names a block of the same packet), so that it takes a full
 * SSP-RK2 step on its own.  nslots (1..16) device staging slots, each with
 * its own stream (default priority) and buffers sized for the largest
 * transfer unit (one packet by default, see hydro_stream_set_unit_bytes),
 * take the units in order, each going to the slot with the fewest bytes so
 * far: a unit is copied in, advanced (one launch per RK stage) and copied
 * back on its slot's stream, so one unit's copies overlap other units'
 * copies and kernels.  dt = cfl / max rate over all packets, from the
 * state at the start of each step, stays on the device: the control stream
 * waits for every slot's last stage-2 launch of a step, updates dt, and each
 * slot waits for that update only after it has issued the copy-in of its
 * first unit of the next step.  All device memory is allocated by create
 * (and, when a larger transfer unit is asked for, by
 * hydro_stream_set_unit_bytes).  Errors (create): EINVAL (descriptors as for hydro_mesh_create, packet
 * ranges, non-contiguous packet, open packet, nslots, precision), ENOMEM,
 * EDEVICE. */
typedef struct hydro_stream hydro_stream;
hydro_status hydro_stream_create(const hydro_block_desc *blocks, int32_t nblocks, int32_t ndim, double *host_arena,
                                 int64_t arena_len, const int32_t *packet_start, int32_t npackets,
                                 int32_t precision, int32_t nslots, hydro_stream **out);

/* nsteps steps of every packet, in place in the host arena.  Synchronising;
 * *t_out (may be NULL) receives the simulated time advanced.  A non-physical
 * state is handled as in hydro_batch_run: the steps after the failing one
 * copy every packet in and back unchanged, so the host arena holds the
 * result of the failing step and *t_out its end time.  Errors: EINVAL,
 * ENONPHYS, EDEVICE. */
hydro_status hydro_stream_run(hydro_stream *s, int32_t nsteps, double cfl, double gamma, double *t_out);

/* CPU/GPU split of a stream's packets (Sec. 6.1 and its Sedov table: a
 * number of blocks per cycle goes to the host cores, the rest to the GPU,
 * both at once).  The last cpu_packets packets (0..npackets; 0, the default,
 * is GPU only) are advanced by nthreads host threads (0 = one per hardware
 * thread) with a host kernel: FP64, Davis bounds, primitive PLM, gamma law,
 * the FP64 GPU path's operations in its order (the same results bit for bit),
 * in place in the host arena, while the GPU's slots stream the other packets.
 * Each step the host reads the device dt (one synchronisation per step), runs
 * both stages of its packets and folds their CFL rate and non-physical flag
 * into the device accumulator before the dt update; failures follow
 * hydro_stream_run's contract.  A stream whose precision code carries a
 * method variant takes no host share (EINVAL); on a mixed-precision stream
 * the host packets still compute in FP64.  On an error the stream keeps
 * its previous split.  Errors: EINVAL, ENOMEM, EDEVICE. */
hydro_status hydro_stream_set_cpu_share(hydro_stream *s, int32_t cpu_packets, int32_t nthreads);

/* Transfer granularity of a stream (the paper's packet size knob, Sec. 6.1:
 * packets amortise the cost of each transfer and each launch).  Consecutive
 * GPU packets that are adjacent in the host arena are copied in, advanced
 * (one launch per RK stage over all of them) and copied back together, in
 * units of at least min_bytes each (the last unit may be smaller; a single
 * packet larger than min_bytes is a unit of its own); min_bytes = 0, the
 * default, keeps one packet per unit.  The staging slots grow to the
 * largest unit.  Results are the same bit for bit at any setting.  On an
 * error the stream keeps its previous units and buffers.  Errors: EINVAL,
 * ENOMEM, EDEVICE. */
hydro_status hydro_stream_set_unit_bytes(hydro_stream *s, int64_t min_bytes);

hydro_status hydro_stream_destroy(hydro_stream *s);

/* ---------------------------------------------------------------------------
 * Allocation-free step, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  One full SSP-RK2 step of all nblocks blocks with time step dt,
 * in place on the caller's device arena -- what hydro_packet_advance does for
 * a packet of every block of a mesh made from the same descriptors -- but
 * with no mesh, packet or other allocation: the first-stage state, the device
 * block table, the work list and the time record live in one fixed array of
 * the library, 64 MiB per GPU, held from the first call on that GPU until the
 * process ends.
 *   Limits: nblocks <= 4096, and 8 * arena_len + 176 * nblocks + 40 * (work
 *   items) plus alignment must fit in 64 MiB (arena_len up to about 8.3e6
 *   doubles, i.e. 1.6e6 cells); a larger mesh is EINVAL, checked before any
 *   device work.
 *   Tiling: 16x16 tiles where a block's x and y extents allow, else 8x8 tiles
 *   packed four to a work item within the block; no z-runs, no tuning.
 *   blocks: host array, read during the call (each block's resolved table
 *   entry is passed to a setup kernel by value, so nothing refers to it
 *   afterwards).  precision: as for hydro_packet_create.  stream: hipStream_t
 *   of all the call's work (NULL = default stream); stream-ordered,
 *   asynchronous.  The array keeps the last call's contents; every call
 *   rewrites what it reads.  All calls on one GPU share the array, so calls
 *   that overlap on one GPU (other streams, other threads) race: the caller
 *   serialises them.
 * Errors: EINVAL (descriptors as for hydro_mesh_create, precision, dt or gamma
 * as for hydro_packet_advance, size beyond the limits), EDEVICE. */
hydro_status hydro_step_static(const hydro_block_desc *blocks, int32_t nblocks, int32_t ndim, double *arena,
                               int64_t arena_len, int32_t precision, double dt, double gamma, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *hydro_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HYDRO_H */
