// lbm_kernels.h -- launchers of the gfx950 kernels (defined in lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_types.h"

namespace lbm {

// Interior stream+collide, u and du/dt update of every interior node
// (reads buffer cur, writes cur ^ 1).  lanes: 64, 128 or 256.
hipError_t launch_interior(int storage, const DevState &s, const Tile *tiles, int ntiles,
                           int lanes, int cur, hipStream_t stream);
// Boundary kernel over nchunks chunks (see k_boundary): u(t+dt) from buffer
// gb (boundary nodes) or recomputed from buffer cur (interior nodes, if
// recompute); resets and second-row pulls (if do_reset) into buffer cur ^ 1;
// boundary accelerations of step counter[cslot] + step_off from buffer gb
// written into buffer ub.
hipError_t launch_boundary(int storage, const DevState &s, const Chunk *chunks, int nchunks,
                           const UNode *un, const GradNode *gn, const BTask *bt, const STask *stk,
                           int cur, int gb, int ub, int do_reset, int recompute, int cslot,
                           int step_off, hipStream_t stream);
// Synchronization of the state held in buffer b.
hipError_t launch_sync(int storage, const DevState &s, const Tile *tiles, int ntiles, int lanes,
                       int b, hipStream_t stream);
// Initial state of one plate from dense device arrays (any may be null).
hipError_t launch_init(int storage, const DevState &s, int plate, int64_t nodes, const double *u0,
                       const double *v0, const double *e0, const double *w0, hipStream_t stream);
// Dense FP64 fields of one plate from buffer b (any output may be null).
hipError_t launch_fields(int storage, const DevState &s, int plate, int64_t nodes, int b,
                         double *e, double *w, double *u, double *v, hipStream_t stream);

}  // namespace lbm
