// lbm_kernels.h -- launchers of the gfx950 kernels (defined in lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_types.h"

namespace lbm {

// Interior stream+collide, u and du/dt update of every interior node
// (reads buffer cur, writes cur ^ 1).  lanes: 64, 128 or 256.
hipError_t launch_interior(int storage, const DevState &s, const Tile *tiles, int ntiles,
                           int lanes, int cur, hipStream_t stream);
// Boundary reset, second-row pull and (if do_bacc) next-step boundary
// accelerations; nb boundary records then ns second-row records.
hipError_t launch_post(int storage, const DevState &s, int nb, int ns, int cur, int do_bacc,
                       hipStream_t stream);
// Boundary accelerations of the first step (buffer 0 -> buffer 1).
hipError_t launch_bacc0(int storage, const DevState &s, int nb, hipStream_t stream);
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
