/*
 * lbm.h -- C ABI of the MI355X plane-strain lattice Boltzmann library.
 *
 * The library advances the method of Schlueter, Yan, Faust, Mueller and
 * Mueller, "A Lattice Boltzmann Method for Elastic Solids Under Plane Strain
 * Deformation" (arXiv 2301.00228): per time step, two D2Q5 wave-equation
 * LBMs (dilatation phi = div u with speed c_d, rotation psi = (curl u).e_z
 * with speed c_s; Sec. 2, eq. wave-eqs; Sec. 3), the Dirichlet and Neumann
 * boundary rules of Sec. 3.1, the periodic synchronization of Sec. 3.2, and
 * the recovery of the displacement u by the explicit Newmark update of
 * eq. integration.  Many independent plates advance together.
 *
 * Conventions for every entry point:
 *  - every call returns lbm_status: LBM_OK (0) or a negative error code;
 *    nothing throws, aborts or prints; lbm_last_error() describes the last
 *    failure of a context;
 *  - arrays are row-major with x fastest: node (i, j) of an nx-by-ny plate
 *    is element j*nx + i; vector fields are planar [2][ny][nx] (x component
 *    first);
 *  - unless an entry point says "device", pointers are host pointers; the
 *    library copies inputs before returning and the caller keeps ownership
 *    of everything it passes;
 *  - units are the caller's; dh is the lattice spacing, dt the time step;
 *  - a context must not be used from two threads at once.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_E_INVAL = -1,        /* invalid argument (sizes, mask, node lists, ...)          */
  LBM_E_UNSTABLE_DT = -2,  /* dt gives a_{0,phi} < 0 (Sec. 3, eq. feq_req)              */
  LBM_E_NOMEM = -3,        /* host or device allocation failed                          */
  LBM_E_DEVICE = -4,       /* no usable GPU, or a HIP call failed                       */
  LBM_E_NONFINITE = -5,    /* a non-finite or blown-up displacement was detected       */
  LBM_E_STATE = -6         /* call not allowed in the current state                     */
} lbm_status;

/* Storage of the populations (Sec. 3, eq. LBE) in device memory.
 *  F64     : 5+5 populations in FP64, FP64 arithmetic, u and du/dt in FP64.
 *  F32     : 5+5 populations in FP32, FP32 arithmetic, u and du/dt in FP32.
 *  F32DEV  : per field, the zeroth moment rho and flux J in FP32 and the two
 *            remaining moments of the deviation f - f_eq(rho, J = 0) from the
 *            local rest equilibrium (N = f1 + f3 - f2 - f4 and
 *            Q - 4 a rho with Q = f1 + f2 + f3 + f4) in FP32;
 *  F16DEV  : as F32DEV with the two deviation moments in IEEE FP16 (scaled
 *            by a per-plate, per-field power of two);
 *  BF16DEV : as F16DEV with bfloat16.
 * The DEV variants collide in FP32 and keep u, du/dt and all boundary
 * arithmetic in FP64.  The update itself is the same for every storage. */
typedef enum {
  LBM_STORE_F64 = 0,
  LBM_STORE_F32 = 1,
  LBM_STORE_F32DEV = 2,
  LBM_STORE_F16DEV = 3,
  LBM_STORE_BF16DEV = 4
} lbm_storage;

/* Boundary condition kinds for lbm_set_bc (Sec. 2: u = u* on the Dirichlet
 * part, sigma n = t* on the Neumann part). */
enum { LBM_BC_NEUMANN = 0, LBM_BC_DIRICHLET = 1 };

/* One plate: the body B of Sec. 2 on a regular lattice (Sec. 3, Fig. 2). */
typedef struct {
  int32_t nx, ny;            /* lattice size, each >= 3                                  */
  const uint8_t *mask;       /* nx*ny bytes, nonzero = node belongs to the body; NULL =
                                the full rectangle.  Every body node needs a body
                                neighbour on at least one side along each axis.          */
  uint8_t periodic_x;        /* nonzero: the x axis wraps around                          */
  uint8_t periodic_y;        /* nonzero: the y axis wraps around                          */
  double lambda, mu, rho_m;  /* Lame parameters and mass density (Sec. 2, eq. hooke)
                                c_d = sqrt((lambda + 2 mu)/rho_m), c_s = sqrt(mu/rho_m)   */
  double dh, dt;             /* lattice spacing and time step; the equilibrium weights
                                follow from a = (c dt/dh)^2 / 2 for each field
                                (Sec. 3, eqs. parameters_to_wavespeed_relation,
                                conditions-parameters); dt must keep a_{0,phi} =
                                1 - 4 a_phi >= 0, i.e. dt <= dh / (sqrt(2) c_d)           */
  int32_t sync_every;        /* l of Sec. 3.2: synchronize after every l-th step; 0 = off.
                                All plates of one context must use the same value.        */
  const double *u0, *v0;     /* initial displacement and velocity, planar [2][ny][nx];
                                NULL = 0                                                   */
  const double *e0, *w0;     /* optional initial dilatation / rotation (nx*ny); NULL =
                                finite differences of u0 (Sec. 3, Fig. 4)                 */
  int32_t integrator;        /* displacement update. 0: eq. integration as printed (u +=
                                dt v + dt^2/2 a, v += dt a with a at t; first order in
                                dt). 1: central difference (Newmark gamma = 1/2, second
                                order): v is kept, and reported by lbm_fields, at t - dt/2
                                (v0 is the velocity at t = 0); u is the same after the
                                first step.  Other values: LBM_E_INVAL.                    */
  int32_t readings;          /* readings of two points Sec. 3.1 leaves open, bits (other
                                bits: LBM_E_INVAL).  0 (default) = R1 and M1.
                                LBM_READ_FLUX_STREAMED (R2): the flux J(x_k, t) of eq.
                                correction-f is that of the post-collision populations
                                streaming into the boundary node from its body neighbours
                                (a missing one adds 0), not that of its own populations.
                                LBM_READ_EQ_OLD (M2): the equilibrium of eq. LBE_mod is that
                                of the boundary node's populations at t, not that of the
                                time-averaged populations.  With either bit on any plate
                                the context runs each step's boundary work in a launch of
                                its own after the interior launch (no two-step pairs;
                                slower, the same update) and lbm_autotune returns
                                LBM_E_STATE.                                              */
} lbm_plate;

enum { LBM_READ_FLUX_STREAMED = 1, LBM_READ_EQ_OLD = 2 };

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns device memory of at least `bytes` bytes or NULL; free releases it.
 * Both are called only from lbm_create / lbm_destroy. */
typedef struct {
  void *(*alloc)(size_t bytes, void *user);
  void (*free)(void *ptr, void *user);
  void *user;
} lbm_alloc;

/* Create a context for n_plates plates with the given population storage.
 * hip_stream: the hipStream_t every device operation is ordered on (NULL =
 * the null stream).  alloc: NULL = hipMalloc/hipFree.  Classifies every
 * node (interior, boundary, second row; Sec. 3.1, Fig. 5), builds the
 * boundary cells with the mask rule (the cell spans half a spacing towards
 * each body neighbour and ends at the node towards a missing one), uploads
 * the initial state and sets the populations to f_eq(field, J = 0).  All
 * boundary nodes start traction-free Neumann.
 * Errors: LBM_E_INVAL (sizes, mask with a node lacking both neighbours along
 * an axis, mixed sync_every), LBM_E_UNSTABLE_DT, LBM_E_NOMEM, LBM_E_DEVICE
 * (no GPU or HIP failure).  On error *out is NULL. */
lbm_status lbm_create(const lbm_plate *plates, int32_t n_plates, lbm_storage storage,
                      void *hip_stream, const lbm_alloc *alloc, lbm_ctx **out);

/* Boundary data of n boundary nodes of one plate (Sec. 3.1).
 * xy   : 2n node coordinates (i, j); each must be a boundary node (a body node
 *        with at least one missing D2Q5 neighbour), else LBM_E_INVAL.
 * kind : n bytes, LBM_BC_NEUMANN or LBM_BC_DIRICHLET.  Where a Dirichlet and a
 *        Neumann edge meet, list the corner as Dirichlet.
 * val  : 2n values.  Dirichlet: the prescribed displacement u* (eq.
 *        acc_dirichlet, applied so that u(t+dt) = u*(t+dt)).  Neumann: the
 *        external force integral of t* over the cell's external boundary
 *        (eq. acc_neumann), per unit thickness.
 * cell : NULL, or 5n values (V_C, l_E, l_N, l_W, l_S) replacing the mask-rule
 *        cell volume and the lengths of the internal sides towards the E, N,
 *        W, S neighbours (for boundaries that do not follow the lattice, e.g.
 *        from lbm_exact_cells).  Lengths towards neighbours outside the body
 *        are not used (eq. acc_neumann sums over the neighbours).
 * knots: n_knots (t, g) pairs of a piecewise linear amplitude g(t) (clamped
 *        outside the knot range, times strictly increasing) multiplying val;
 *        NULL (n_knots = 0) means g = 1.  Neumann loads are taken at t = n dt,
 *        Dirichlet values at t = (n+1) dt during step n.
 * Later calls override earlier ones node by node.  At most 16 amplitude
 * tables of at most 64 knots per plate.  Only allowed before the first
 * lbm_step (else LBM_E_STATE). */
lbm_status lbm_set_bc(lbm_ctx *ctx, int32_t plate, int32_t n, const int32_t *xy,
                      const uint8_t *kind, const double *val, const double *cell,
                      int32_t n_knots, const double *knots);

/* Shapes bounding a body for lbm_exact_cells: an ellipse with centre (cx,
 * cy), semi-axes a and b and the angle (radians) of its a axis to the x axis,
 * in lattice units (node (i, j) sits at (i, j)).  LBM_SHAPE_HOLE removes its
 * open interior from the body, LBM_SHAPE_BOUND its open exterior. */
enum { LBM_SHAPE_HOLE = 0, LBM_SHAPE_BOUND = 1 };
typedef struct {
  double cx, cy, a, b, angle;
  int32_t kind;
  int32_t pad;
} lbm_shape;

/* Exact-geometry boundary cells (Sec. 3.1: the preprocessing computes cell
 * volumes and surface measures at boundary lattice points by cutting the
 * square cell of side dh around each point to the body's boundary; used by
 * eq. acc_neumann).  Host computation only; needs no context or GPU.
 * The body is the lattice rectangle [0, nx-1] x [0, ny-1] (an axis with
 * periodic_* nonzero is not bounded) minus the shapes' removed sets, which
 * must be pairwise disjoint; shapes are not wrapped across periodic axes.
 * A node belongs to the body iff its position does (points on an ellipse
 * belong to the body): build the plate's mask the same way.
 * For each of the n nodes xy[2m], xy[2m+1] (any node of the lattice):
 *   cell[5m..5m+4]  = V_C, l_E, l_N, l_W, l_S: area of the node's square
 *                     inside the body (dh^2 units) and, for each of its four
 *                     sides towards a neighbour in the body, the side's
 *                     length inside the body (dh units); the layout of
 *                     lbm_set_bc's cell table.  A side towards a neighbour
 *                     outside the body has length 0 even where the boundary
 *                     passes beyond it: the sliver of body between that side
 *                     and the boundary belongs to no cell and, massless,
 *                     passes the boundary's traction on to the cell.
 *   ext_normal[2m..2m+1] (ext_normal may be NULL) = the integral of the
 *                     outward unit normal over the body boundary of the cell
 *                     and of those slivers, -(l_E - l_W, l_N - l_S) by
 *                     closure; times -p it is the external force of a
 *                     uniform pressure p (the Neumann value of lbm_set_bc).
 * Outputs are caller-owned host arrays.  A node whose square lies outside
 * the body gets V_C = 0.  Errors: LBM_E_INVAL for sizes, a node outside the
 * lattice, a non-positive or non-finite semi-axis, an unknown kind. */
lbm_status lbm_exact_cells(int32_t nx, int32_t ny, uint8_t periodic_x, uint8_t periodic_y,
                           double dh, int32_t n_shapes, const lbm_shape *shapes, int32_t n,
                           const int32_t *xy, double *cell, double *ext_normal);

/* Advance every plate by n_steps time steps (Fig. 4: accelerations,
 * Newmark update, boundary reset, LBE with the second-row rule, and the
 * synchronization after every l-th step).  Stream-ordered and asynchronous:
 * returns once the work is enqueued.  With two-step tilings part of the work
 * runs on a second stream of the library's that forks from and joins back
 * into the context's stream with events within the call (see
 * lbm_use_overlap), so to the caller the work is ordered on the context's
 * stream.  A blow-up detected by earlier work is reported as
 * LBM_E_NONFINITE by this or the next synchronizing call. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n_steps);

/* Copy one plate's state to host buffers (any may be NULL): e = sum of the
 * dilatation populations, omega = sum of the rotation populations (eq.
 * interpretation), each nx*ny; u, v = displacement and velocity, planar
 * 2*nx*ny.  Nodes outside the body read 0.  Synchronizes the stream.
 * Returns LBM_E_NONFINITE if a blow-up was detected. */
lbm_status lbm_fields(lbm_ctx *ctx, int32_t plate, double *e, double *omega, double *u,
                      double *v);

/* As lbm_fields, but the outputs are device pointers (FP64, same layout),
 * written in stream order without synchronizing. */
lbm_status lbm_fields_device(lbm_ctx *ctx, int32_t plate, double *e, double *omega, double *u,
                             double *v);

/* As lbm_fields, for callers that cannot allocate device memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it).
 * The fields are staged in a fixed 48 MiB area of device memory that the
 * library holds on each GPU it runs on until the process ends (looked up at
 * lbm_create); the call allocates nothing.  The requested outputs of the
 * plate must fit that area: (n_e + n_omega + 2 n_u + 2 n_v) * nx * ny * 8
 * bytes <= 48 MiB, where n_x is 1 if that output is requested (all four:
 * nx * ny <= 1,048,576); otherwise LBM_E_INVAL with the sizes in the error
 * text.  Every context on one GPU shares the area, so calls that overlap in
 * time on one GPU (from several threads) race; serialize them.  Each call
 * writes every element it copies back, so nothing from an earlier call is
 * read.  Synchronizes the stream.  Other errors as lbm_fields; LBM_E_DEVICE
 * if the area could not be located at lbm_create. */
lbm_status lbm_fields_noalloc(lbm_ctx *ctx, int32_t plate, double *e, double *omega, double *u,
                              double *v);

/* Consistency error of Sec. 4 (tension example, the error measure e(x, t)):
 * for each body node of one plate the 2-norm of (omega - (curl u).e_z,
 * e - div u), where omega and e are the sums of the rotation and dilatation
 * populations and the derivatives of u are the finite differences the method
 * uses at that node (the ones of the synchronization, Sec. 3.2); 0 outside
 * the body.  err: caller-owned host array of nx*ny doubles, x fastest.
 * Synchronizes the stream.  Errors: LBM_E_INVAL (bad plate, NULL err),
 * LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_NONFINITE as for lbm_fields. */
lbm_status lbm_consistency_error(lbm_ctx *ctx, int32_t plate, double *err);

/* Summary of a context.  Filled by lbm_info. */
typedef struct {
  int64_t nodes_in_body;      /* body nodes over all plates (lattice updates per step)       */
  int64_t nodes_allocated;    /* nodes stored, including row padding                        */
  int64_t boundary_nodes;     /* nodes with a missing neighbour                             */
  int64_t second_row_nodes;   /* interior nodes with a boundary neighbour                   */
  int64_t nodes_two_step;     /* body nodes in two-step tiles (tiling steps = 2)            */
  int64_t steps_done;
  int64_t device_bytes;       /* device memory held                                         */
  double bytes_per_update;    /* algorithmic HBM bytes per body node and step (read+write) */
  int32_t n_plates;
  int32_t storage;
  int32_t tile_lanes, tile_rows; /* interior-kernel tile: lanes per workgroup, rows        */
  int32_t tile_order;         /* interior-tile packing order (see lbm_set_tiling)           */
  int32_t tile_edge_rows;     /* rows of the tiles that carry boundary work                 */
  int32_t tile_align;         /* column-strip alignment in nodes (0: equal-width strips)    */
  int32_t tile_steps;         /* time steps per pass over the tiles away from boundaries    */
  int32_t n_tiles;
  int32_t tile_edge_cols;     /* width of the first and last column strip (0: no such strip) */
  int64_t nodes_deep;         /* body nodes in deep two-step tiles (see lbm_use_overlap)    */
  int32_t overlap;            /* 1: pairs of steps overlapped on two streams                */
  int32_t graphs_cached;      /* captured step graphs held (see lbm_step)                   */
  int64_t steps_in_graphs;    /* steps run so far by replaying captured graphs              */
  int64_t syncs_done;         /* synchronization steps (Sec. 3.2) enqueued so far           */
  int32_t tile_stream_stores; /* two-step passes store with nontemporal stores (lbm_tiling) */
  int32_t pad;
} lbm_info_t;
lbm_status lbm_info(const lbm_ctx *ctx, lbm_info_t *info);

/* Interior-kernel tiling.  A tile is a strip of columns times a band of
 * rows; one workgroup marches up (or down) its rows.
 *  lanes      workgroup size, 64, 128 or 256; a tile owns at most lanes-2
 *             columns (the two others read the halo columns);
 *  rows       rows per tile (>= 1);
 *  order      packing order of the tile list (0: plate by plate, row band by
 *             row band; 1: plate by plate, column strip by column strip; 2:
 *             as 0 with the largest plates first; 3: plate by plate in
 *             groups of 4 row bands, strip by strip within a group with the
 *             group's bands of a strip consecutive, so that tiles sharing
 *             halo rows or columns run at about the same time on one XCD);
 *  edge_rows  rows of the tiles whose area or one-node halo ring holds
 *             boundary or second-row nodes (those tiles finish the previous
 *             step's boundary work before their march; 0 or >= rows: no
 *             shorter tiles);
 *  align      0: column strips of equal width; > 0: strips of the largest
 *             multiple of align nodes that fits (strip starts aligned to
 *             align nodes, so that every row segment a tile writes covers
 *             whole cache lines);
 *  steps      1 (or 0): one time step per launch; 2: tiles with no boundary
 *             or second-row node within two nodes of their area take two
 *             time steps per pass over HBM (the other tiles take the two
 *             steps in two launches); a tile then owns at most lanes-4
 *             columns;
 *  edge_cols  0: the column strips of a plate are as `align` says; > 0: on
 *             plates whose x axis is not periodic and that are wider than
 *             2 edge_cols + 2, the first and the last strip are edge_cols
 *             columns wide (the others as `align` says, between them), so
 *             that with steps = 2 the strips next to a boundary column are
 *             narrow and the rest of the plate takes two steps per pass;
 *  stream_stores  0 or 1: with steps = 2, the two-step tiles write the
 *             state at the end of their pass with nontemporal stores (it is
 *             not read again in that launch; the caches stay free for the
 *             halo rows the neighbouring tiles read).  Faster where the
 *             state streams through HBM with a large halo share (the
 *             256-plate batch), slower where it stays in the Infinity Cache
 *             (a 1024^2 FP64 plate); the autotuner decides.
 * Any tiling gives bitwise the same results.  May be changed between steps;
 * invalidates captured step graphs.  LBM_E_INVAL on values out of range
 * (order: 0..3, align: 0..4096, edge_cols: 0..lanes-4, stream_stores: 0..1). */
typedef struct {
  int32_t lanes, rows, order, edge_rows, align, steps;
  int32_t edge_cols;
  int32_t stream_stores;
} lbm_tiling;
lbm_status lbm_set_tiling(lbm_ctx *ctx, const lbm_tiling *tiling);

/* Autotuner: time one step's interior launches (with the boundary work they
 * carry) on this context's plates for the tilings of a two-stage search
 * (steps x lanes x rows, then edge rows, edge columns, alignment, rows, the
 * band-group order 3, -- with several plates -- orders 1 and 2, nontemporal
 * stores, and rows with edge rows once more, one at a time around the best,
 * about 35 tilings), `steps` launches and at least 10 ms each, eager, on one
 * stream.  Repeating those launches leaves the state unchanged, except at
 * step 0, at a synchronization step and right after a two-step pair, where
 * the autotuner first takes one real step (steps_done grows by one; the
 * trajectory is the same as without the autotuner).  The three fastest are
 * then timed again captured in HIP graphs as lbm_step runs them, on one
 * stream and -- with overlapped pairs allowed (lbm_use_overlap on, the
 * default) -- overlapped (frame tiles of their own edge rows, 2 and 4 rows);
 * the fastest one-stream tiling is kept unless an overlapped one is at least
 * 3 % faster (then overlap is turned on, else off).  Nontemporal stores are
 * not tried when the state fits in the 256 MB Infinity Cache.  The result
 * applies to this context only (every context starts from the same default
 * tiling, whatever ran before in the process).  best_ms (nullable) receives
 * the fastest interior time per step (for two-step tilings half the time of
 * a pair's launches). */
lbm_status lbm_autotune(lbm_ctx *ctx, int32_t steps, double *best_ms);

/* Run n_steps steps eagerly (no graph) with HIP events recorded before and
 * after every kernel launch on the stream it runs on, and return the summed
 * time between the two events per kernel kind in ms (a launch's device time
 * plus the gap after the previous launch on its stream, or after what it
 * waited for): ms[0] single-step interior launches (stream+collide of one
 * step), ms[1] boundary/second-row, ms[2] synchronization, ms[3] two-step
 * interior launches (the first launch of a pair: two steps of the two-step
 * tiles -- of the frame tiles only when the pair is overlapped -- and one of
 * the others), ms[4] the deep-tile launches of overlapped pairs (see
 * lbm_use_overlap); and the number of launches of each kind in
 * launches[0..4] (nullable).  Overlapped launches run at the same time, so
 * the sum over kinds can exceed the wall time.  Synchronizes the stream. */
lbm_status lbm_profile(lbm_ctx *ctx, int64_t n_steps, double *ms, int64_t *launches);

/* Capture, without running them, the HIP graphs that lbm_step(ctx,
 * n_steps) would replay from the current state, so that the lbm_step call
 * that follows launches only cached graphs (e.g. before a timed or
 * latency-critical call).  Starts the context like the first lbm_step (the
 * boundary accelerations of step 0 are enqueued) but takes no step.  No-op
 * with graphs off.  Errors as lbm_step. */
lbm_status lbm_prepare_steps(lbm_ctx *ctx, int64_t n_steps);

/* Use (nonzero) or bypass (0) captured HIP graphs in lbm_step.  Default on.
 * With graphs on, lbm_step runs whole synchronization periods (from a step
 * that is a multiple of the period) as one cached graph each and any other
 * run of steps as a graph captured for that run's length and starting
 * phase; up to 8 graphs are kept (least recently used dropped).  Changing
 * the tiling or the overlap setting drops them. */
lbm_status lbm_use_graphs(lbm_ctx *ctx, int32_t enable);

/* Overlapped pairs (nonzero, the default) or one stream (0), for two-step
 * tilings.  The two-step tiles split into frame tiles (a node of a
 * single-step tile within two nodes of their area) and deep tiles (the
 * others).  In an overlapped pair -- every pair but one starting at step 0
 * -- the deep tiles take their two steps in a launch of their own on a
 * second stream (default priority), ordered by events after the previous
 * pair's first launch and before the next pair's first launch, so that it
 * runs beside this pair's single-step launches; the frame tiles take theirs
 * in the first launch of the pair, with the single-step tiles' first step.
 * The launches beside each other read and write disjoint nodes: the results
 * are bitwise the same either way.  Synchronizes the stream; rebuilds the
 * tiles (frame tiles are cut to edge_rows rows with overlap); invalidates
 * captured step graphs.  Errors: LBM_E_INVAL (NULL ctx), LBM_E_NOMEM,
 * LBM_E_DEVICE. */
lbm_status lbm_use_overlap(lbm_ctx *ctx, int32_t enable);

void lbm_destroy(lbm_ctx *ctx);

/* Text of the last error of ctx (or of the last failed lbm_create when ctx is
 * NULL).  The pointer stays valid until the next call on ctx. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Measurement aid: the rate (GB/s, bytes read + written per second) of a
 * plain device-to-device copy of `bytes` bytes on the current device (a
 * grid-stride copy of 16-byte vectors, nontemporal, 1024-lane workgroups),
 * averaged over reps launches after three untimed ones -- the HBM rate a
 * pure stream reaches, to set the kernels' measured rates against.
 * Allocates and frees two device buffers of `bytes` bytes; synchronizes
 * the device.  Errors (text via lbm_last_error(NULL)): LBM_E_INVAL (bytes <
 * 16, reps < 1, NULL gbs), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_copy_rate(size_t bytes, int32_t reps, double *gbs);

/* Measurement aid: the rate (GB/s, bytes read + written per second) of a
 * plain copy with the array structure of `storage`'s state (LBM_STORE_*):
 * each of its arrays over `nodes` nodes (rounded up to a multiple of
 * 8192 x 16) -- the two fields' population slots and the four arrays of u
 * and du/dt, at their storage widths -- copied to an array of its own by
 * 256-lane workgroups marching 256 x 16 blocks of 8192-node rows, as the
 * interior tiles march, without their arithmetic or halo.  Many arrays
 * streamed at once reach less than lbm_copy_rate's single stream; this is
 * the ceiling the layout sets for one pass over the state.  Averaged over
 * reps launches after two untimed ones; allocates and frees 2 x (number of
 * arrays) device arrays; synchronizes the device.  Errors (text via
 * lbm_last_error(NULL)): LBM_E_INVAL (unknown storage, nodes outside
 * 1 .. 2^32, reps < 1, NULL gbs), LBM_E_NOMEM, LBM_E_DEVICE. */
lbm_status lbm_layout_copy_rate(int32_t storage, int64_t nodes, int32_t reps, double *gbs);

/* Library version string. */
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif
#endif
