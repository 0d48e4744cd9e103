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
  double inv_h, inv_2h;  // 1/dh and 1/(2 dh)
  double a[2], a0[2];    // equilibrium weights per field (phi, psi)
  float af[2], a0f[2];   // the same in FP32
  float scale[2];        // 16-bit storage scale of the deviation moments
  float iscale[2];
  int32_t integ;         // 0: v += dt a(t) (the paper's update); 1: central difference
  int32_t readings;      // RD_* bits: readings of eqs. correction-f and LBE_mod
};

// Readings of two points Sec. 3.1 leaves open.  RD_FLUX_STREAMED (R2): the
// flux J(x_k, t) of eq. correction-f is that of the post-collision
// populations streaming into the boundary node from its body neighbours (a
// missing one adds 0) instead of that of its own populations (R1).
// RD_EQ_OLD (M2): the equilibrium of eq. LBE_mod is that of the boundary
// node's populations at t instead of that of the averaged populations (M1).
enum { RD_FLUX_STREAMED = 1, RD_EQ_OLD = 2 };

// Interior-kernel tile: owned columns [x0, x1) and rows [y0, y1) of a plate;
// chunk: index of its prologue work list (-1 = none).  A single-step tile
// may own a second column segment [bx0, bx1) of the same rows (bx1 > bx0):
// the last strip of a plate paired with its first one, so that the narrow
// edge strips of both sides share one workgroup (lanes 0 .. x1-x0+1 march
// the first segment with its two halo columns, the next bx1-bx0+2 lanes the
// second).
struct Tile {
  int32_t plate, x0, x1, y0, y1;
  int32_t chunk;  // prologue work list (-1: none)
  int32_t dir;    // 1: the march visits the rows downwards
  // bits 0-3: export the t_{n+1} populations of the first/last owned column
  // and row (W, E, S, N) of a two-step tile; bit 4: two-step tile; bit 5:
  // frame tile (a two-step tile with a node of a single-step tile in its
  // two-node ring); bit 6: a tile whose area a paired tile owns as its
  // second segment (kept for the host's lookups, never launched)
  int32_t flags;
  int32_t bx0, bx1;  // second column segment (single-step tiles; bx1 <= bx0: none)
};
enum {
  TF_EXP_W = 1, TF_EXP_E = 2, TF_EXP_S = 4, TF_EXP_N = 8, TF_TWO = 16, TF_FRAME = 32,
  TF_MERGED = 64
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

// Finite-difference stencil along one axis at a node (the per-axis rule of
// the boundary finite differences): central, one-sided 3-point second order
// forwards / backwards, 2-point first order forwards / backwards, none.
enum { FD_NONE = 0, FD_CENTRAL = 1, FD_FWD3 = 2, FD_BWD3 = 3, FD_FWD2 = 4, FD_BWD2 = 5 };

constexpr int kChunkNodes = 64;    // boundary nodes per boundary-kernel block (at most)
constexpr int kBoundaryThreads = 256;  // threads per boundary-kernel block
constexpr int kMaxGrad = 1024;     // gradient nodes per boundary-kernel block
constexpr int kMaxU = 1024;        // displacement nodes per boundary-kernel block

// A node whose u(t+dt) a boundary-kernel block needs.  bnd: it is a
// boundary node (its u(t+dt) is in the state); otherwise it is an interior
// node and the block recomputes u(t+dt) from the state at t exactly as the
// interior kernel does.
struct UNode {
  int64_t node;
  int32_t i, j;
  int32_t bnd;
  int32_t pad;
};

// A body node where a boundary-kernel block needs the finite-difference
// gradient of u.  code: x stencil in bits 0..2, y stencil in bits 3..5;
// u: block-local UNode indices of the node itself, of the two further nodes
// of its x stencil and of the two further nodes of its y stencil (the node
// itself where a stencil uses fewer).
struct GradNode {
  int32_t code;
  int32_t u[5];
};

// Work of one boundary-kernel block (all of one plate): displacement nodes
// [u0, u1), gradient nodes [g0, g1), boundary tasks [b0, b1), second-row
// tasks [s0, s1).  Thread t < b1 - b0 runs boundary task b0 + t; the next
// 2 (s1 - s0) threads run the second-row tasks, one field each.
struct Chunk {
  int32_t u0, u1, g0, g1, b0, b1, s0, s1;
  int32_t plate;
  int32_t pad[3];
};

// Boundary task: the boundary record of the node and the block-local
// gradient indices of the node itself and of its E, N, W, S neighbours
// (-1 where the neighbour is not in the body).  accel: the task also
// computes the node's next boundary acceleration (else only its reset).
struct BTask {
  BndNode b;
  int32_t g[5];
  int32_t accel;
  int32_t pad[2];
};

// Work list of an interior tile's prologue: gradient nodes [g0, g1) (their
// gradients go to the scratch rows g0..g1-1), boundary tasks [b0, b1),
// second-row tasks [s0, s1), all of one plate.
struct TileChunk {
  int32_t g0, g1, b0, b1, s0, s1;
  int32_t plate;
  int32_t pad;
};

// Gradient node of a tile prologue (stencil read straight from u).
struct TGradNode {
  int64_t node;
  int32_t i, j, code;
  int32_t pad;
};

// Second-row task: the node and, per lattice direction alpha, the
// block-local gradient index of the upwind node x - c^alpha if that node is
// a boundary node (-1 otherwise).
struct STask {
  int64_t node;
  int32_t i, j;
  int32_t g[5];
  int32_t si;  // second-row index
  int32_t pad[2];
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
  // [buffer][field][slot]: buffers 0 and 1 hold the state between launches
  // (the current one alternates), buffer 2 the intermediate time level of
  // a two-step launch near boundaries
  void *pop[3][2][5];
  void *u[3][2];       // [buffer][component]
  void *v[3][2];
  // Pulled populations of the second-row nodes from their non-boundary
  // upwind nodes, written by the march of step n into side[(n + 1) & 1] (the
  // collision type, [field][alpha][second-row index]); sidx: second-row
  // index of a node (-1 elsewhere).
  void *side[2];
  const int32_t *sidx;
  int64_t nsec;
  const uint8_t *cls;
  const PlateDev *plates;
  const LoadTable *loads;
  const BndNode *bnd;
  const SecNode *sec;
  // counter[b]: index of the time step whose state buffer b holds; a
  // launch writing buffer b sets it.
  unsigned long long *counter;
  int *flag;                    // nonzero once a non-finite / blown-up u is seen
};

// Buffers of one single-step launch (step n): the state of t_n in buffer
// `in`, t_{n+1} written to `out`; the boundary nodes' populations of t_{n-1}
// in `prev` (read by the prologue); sp = n & 1 (the prologue reads side[sp],
// the march writes side[sp ^ 1]).  A two-step tile (kind 1) writes t_{n+2}
// to out2 (with nontemporal stores if nt) and the t_{n+1} populations of its
// export bands to `out`.
struct StepBufs {
  int in, out, prev, sp, out2;
  int nt;  // two-step tiles write t_{n+2} with nontemporal stores
};

// Prologue work lists of the interior kernel (see k_interior); grad:
// per-tile gradient scratch (4 values of the displacement type per gradient
// node).
struct Prologue {
  const TileChunk *chunks;
  const TGradNode *gn;
  const BTask *bt;
  const STask *st;
  void *grad;
  int enabled;
};

}  // namespace lbm
