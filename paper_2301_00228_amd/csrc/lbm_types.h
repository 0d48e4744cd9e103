// lbm_types.h -- device-visible records shared by the host runtime and the
// HIP kernels of the plane-strain LBM library.
#pragma once

#include <stdint.h>

namespace lbm {

// Per-node class byte.  Bits 0..3: the D2Q5 neighbour in that direction
// belongs to the body (periodic axes wrap).  CL_IN: the node belongs to the
// body.  CL_B: boundary node (a body node with a missing neighbour, Sec. 3.1).
// CL_S: "second row" node (interior node with a boundary neighbour, Fig. 5g).
enum : uint8_t {
  NB_E = 1,
  NB_N = 2,
  NB_W = 4,
  NB_S = 8,
  NB_ALL = 15,
  CL_IN = 16,
  CL_B = 32,
  CL_S = 64
};

enum { FLD_PHI = 0, FLD_PSI = 1 };

constexpr int kMaxLoadsPerPlate = 16;
constexpr int kMaxKnots = 64;

// Per-plate constants.  off is the packed index of node (0, 0); node (i, j)
// lives at off + j * pitch + i.
struct PlateDev {
  int64_t off;
  int32_t nx, ny, pitch;
  int32_t periodic;  // bit 0: x wraps, bit 1: y wraps
  double dt, dh, cd2, cs2, rho_m, lam, mu;
  double a[2], a0[2];    // equilibrium weights per field (phi, psi)
  float af[2], a0f[2];   // the same in FP32
  float scale[2];        // 16-bit storage scale of the deviation moments
  float iscale[2];
};

// Interior-kernel tile: owned columns [x0, x1) and rows [y0, y1) of a plate.
struct Tile {
  int32_t plate, x0, x1, y0, y1;
  int32_t pad[3];
};

// Boundary node record (one per node with a missing neighbour).
struct BndNode {
  int64_t node;
  int32_t plate, i, j;
  int32_t kind;    // 0 Neumann, 1 Dirichlet
  int32_t load;    // index into the load table, -1 = amplitude 1
  int32_t pad;
  double val[2];   // u* (Dirichlet) or integrated external force (Neumann)
  double cell[5];  // V, l_E, l_N, l_W, l_S
};

// Second-row node record.
struct SecNode {
  int64_t node;
  int32_t plate, i, j;
};

// Piecewise linear amplitude g(t).
struct LoadTable {
  int32_t n;
  int32_t pad;
  double t[kMaxKnots];
  double g[kMaxKnots];
};

// Device pointers of the state.  Slot meaning depends on the storage: for
// the population storages slot s is population alpha = s; for the deviation
// storages slots are (rho, J_x, J_y, N, Q - 4 a rho), where the 16-bit
// variants pack N and Q - 4 a rho into slot 3 and leave slot 4 unused.
struct DevState {
  void *pop[2][2][5];  // [buffer][field][slot]
  void *u[2][2];       // [buffer][component]
  void *v[2][2];
  const uint8_t *cls;
  const PlateDev *plates;
  const LoadTable *loads;
  const BndNode *bnd;
  const SecNode *sec;
  unsigned long long *counter;  // completed steps (device side)
  int *flag;                    // nonzero once a non-finite / blown-up u is seen
};

}  // namespace lbm
