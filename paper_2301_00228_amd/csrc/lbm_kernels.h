// lbm_kernels.h -- launchers of the gfx950 kernels (defined in lbm_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_types.h"

namespace lbm {

// Interior stream+collide, u and du/dt update of every interior node at
// step n (buffers b, see StepBufs); tiles with a prologue list first finish
// the previous step's boundary work if pro.enabled.  lanes: 64, 128 or 256.
hipError_t launch_interior(int storage, const DevState &s, const Tile *tiles, int ntiles,
                           int lanes, const StepBufs &b, const Prologue &pro, hipStream_t stream);
// The two steps n, n + 1 of deep two-step tiles (no boundary, second-row or
// single-step tile within two nodes; b.out2 >= 0): the launch may run beside
// the other launches of the step, whose tiles it neither reads nor writes,
// and is never the run's first step.
hipError_t launch_deep(int storage, const DevState &s, const Tile *tiles, int ntiles, int lanes,
                       const StepBufs &b, hipStream_t stream);
// Boundary kernel over nchunks chunks (see k_boundary): the boundary work of
// step n - 1 on the state of t_n in buffer bc (resets and second-row pulls
// only if do_reset).
hipError_t launch_boundary(int storage, const DevState &s, const Chunk *chunks, int nchunks,
                           const UNode *un, const GradNode *gn, const BTask *bt, const STask *stk,
                           int bc, int bp, int ub, int ub2, int sr, int do_reset,
                           hipStream_t stream);
// Synchronization of the state in buffers b.
hipError_t launch_sync(int storage, const DevState &s, const Tile *tiles, int ntiles, int lanes,
                       int b, hipStream_t stream);
// Initial state of one plate from dense device arrays (any may be null).
hipError_t launch_init(int storage, const DevState &s, int plate, int64_t nodes, const double *u0,
                       const double *v0, const double *e0, const double *w0, hipStream_t stream);
// Dense FP64 fields of one plate from buffers b (any output may be null).
hipError_t launch_fields(int storage, const DevState &s, int plate, int64_t nodes, int b,
                         double *e, double *w, double *u, double *v, hipStream_t stream);
hipError_t launch_cons_err(int storage, const DevState &s, int plate, int64_t nodes, int b,
                           double *err, hipStream_t stream);

// Rate in GB/s (read + write) of a plain device copy of `bytes` bytes,
// averaged over reps launches after 3 untimed ones; allocates and frees
// its two buffers.
hipError_t copy_rate(size_t bytes, int reps, double *gbs);
// Rate in GB/s (read + write) of a copy with the array structure of
// `storage`'s state over `nodes` nodes (rounded up to 8192 x 16), marched
// like the interior tiles; averaged over reps launches after 2 untimed
// ones; allocates and frees its arrays.
hipError_t layout_copy_rate(int storage, int64_t nodes, int reps, double *gbs);

// Size of the fixed device staging area of lbm_fields_noalloc (per GPU).
constexpr size_t kNoAllocBytes = (size_t)48 << 20;
// Device address of that area on `device`, which must be the current
// device; looked up on the first call per device and kept (thread-safe).
hipError_t noalloc_staging(int device, void **ptr);

}  // namespace lbm
