// lbm_host.cpp -- host runtime and C ABI of the plane-strain LBM library.
//
// Preprocessing (Fig. 4 "Preprocessing"): node classification from the body
// mask, boundary cells by the mask rule, second-row lists, interior tiles.
// Runtime: device buffers, initial state, the time-step launch sequence,
// captured HIP graphs of whole synchronization periods, tile autotuning,
// per-kernel profiling with HIP events, blow-up detection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_kernels.h"
#include "lbm_types.h"

using namespace lbm;

namespace {

thread_local std::string g_create_error;

struct PlateHost {
  int nx = 0, ny = 0, pitch = 0;
  int64_t off = 0;
  bool px = false, py = false;
  std::vector<uint8_t> cls;  // dense nx*ny copy of the class bytes
  int64_t b0 = 0, b1 = 0;    // range in the boundary list
  int nloads = 0;
  int64_t body = 0;
  double field_mag[2] = {0, 0};  // magnitude of the initial fields (16-bit storage scale)
  int ns = 0;          // interior tiles: column strips
  std::vector<int> sx;  // first column of each strip, then nx (ns + 1 entries)
  // per strip: (first row, tile index) of its tiles, by increasing row
  std::vector<std::vector<std::pair<int, int>>> strips;
};

struct Buffer {
  void *p = nullptr;
  size_t bytes = 0;
};

const char *storage_name(int st) {
  switch (st) {
    case LBM_STORE_F64: return "f64";
    case LBM_STORE_F32: return "f32";
    case LBM_STORE_F32DEV: return "f32dev";
    case LBM_STORE_F16DEV: return "f16dev";
    case LBM_STORE_BF16DEV: return "bf16dev";
  }
  return "?";
}

// Algorithmic HBM bytes per body node and step: populations read + written,
// u and du/dt read + written.
double bytes_per_update(int st) {
  switch (st) {
    case LBM_STORE_F64: return 2 * 10 * 8 + 2 * 4 * 8;   // 224
    case LBM_STORE_F32: return 2 * 10 * 4 + 2 * 4 * 4;   // 112
    case LBM_STORE_F32DEV: return 2 * 10 * 4 + 2 * 4 * 8; // 144
    default: return 2 * 2 * (3 * 4 + 4) + 2 * 4 * 8;      // 128
  }
}

int slot_count(int st) { return (st == LBM_STORE_F16DEV || st == LBM_STORE_BF16DEV) ? 4 : 5; }
size_t slot_bytes(int st) {
  return st == LBM_STORE_F64 ? 8 : 4;
}
size_t uv_bytes(int st) { return st == LBM_STORE_F32 ? 4 : 8; }


}  // namespace

struct lbm_ctx {
  int storage = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // graph capture
  bool have_alloc = false;
  lbm_alloc alloc{};
  int device = 0;
  std::string err;

  std::vector<PlateHost> ph;
  std::vector<PlateDev> pd;
  int64_t n_alloc = 0;
  int64_t n_two = 0;  // body nodes in two-step tiles
  int64_t n_body = 0;
  int sync_every = 0;
  // some plate uses readings other than R1 + M1: every step's boundary work
  // runs in the boundary kernel (the interior kernel's prologues carry only
  // the default readings), so every step is a segment of its own
  bool variant_readings = false;

  std::vector<BndNode> bnd;
  std::vector<SecNode> sec;
  std::vector<Chunk> chunks;
  std::vector<UNode> unodes;
  std::vector<GradNode> gnodes;
  std::vector<BTask> btasks;
  std::vector<int64_t> btask_bnd;  // boundary record of each boundary task
  std::vector<STask> stasks;
  Chunk *d_chunks = nullptr;
  UNode *d_unodes = nullptr;
  // prologue work lists of the interior tiles
  std::vector<TileChunk> tchunks;
  std::vector<TGradNode> tgn;
  std::vector<BTask> tbt;
  std::vector<int64_t> tbt_bnd;
  std::vector<STask> tst;
  TileChunk *d_tchunks = nullptr;
  TGradNode *d_tgn = nullptr;
  BTask *d_tbt = nullptr;
  STask *d_tst = nullptr;
  void *d_tgrad = nullptr;
  size_t cap_tchunks = 0, cap_tgn = 0, cap_tbt = 0, cap_tst = 0, cap_tgrad = 0;
  GradNode *d_gnodes = nullptr;
  BTask *d_btasks = nullptr;
  STask *d_stasks = nullptr;
  std::vector<LoadTable> loads;
  std::vector<Tile> tiles;    // every tile (host lookups), with merged-away ones
  std::vector<int> partner;   // per tile: the tile paired in as its second segment (-1: none)
  std::vector<Tile> ltiles;   // the tiles launched: all but the merged-away ones
  std::vector<Tile> etiles;  // the single-step tiles (second launch of a two-step pair)
  std::vector<Tile> ftiles;  // single-step and frame tiles (first launch of an overlapped pair)
  std::vector<Tile> dtiles;  // deep two-step tiles (the side stream's launch)
  int lanes = 128, rows = 32, order = 0, edge_rows = 0, align = 0, two = 0, edge_cols = 0;
  int nt = 0;  // two-step passes store their final state with nontemporal stores

  std::vector<Buffer> bufs;
  DevState ds{};
  PlateDev *d_plates = nullptr;
  Tile *d_tiles = nullptr;
  Tile *d_etiles = nullptr;
  size_t etiles_cap = 0;
  Tile *d_ftiles = nullptr, *d_dtiles = nullptr;
  size_t ftiles_cap = 0, dtiles_cap = 0;
  int64_t n_deep = 0;  // body nodes in deep tiles
  // Overlapped pairs: the deep tiles of a pair run on a side stream beside
  // the single-step launch of the previous pair.  ev_f[i]: after the first
  // launch of a pair on the main stream; ev_d[i]: after a deep launch
  // (alternating by pair, so that a wait never binds to a later record).
  bool overlap = true;
  hipStream_t side = nullptr;
  hipEvent_t ev_f[2] = {nullptr, nullptr}, ev_d[2] = {nullptr, nullptr};
  BndNode *d_bnd = nullptr;
  SecNode *d_sec = nullptr;
  LoadTable *d_loads = nullptr;
  unsigned long long *d_counter = nullptr;
  int *d_flag = nullptr;
  uint8_t *d_cls = nullptr;
  double *d_scratch = nullptr;
  size_t scratch_bytes = 0;
  // fixed staging area of lbm_fields_noalloc on this context's device
  double *na_stage = nullptr;
  hipError_t na_err = hipSuccess;
  size_t tiles_cap = 0;

  int64_t step = 0;
  int cur = 0;   // buffer holding the state of t_step
  int prev = 1;  // buffer holding the boundary populations of t_{step-1}
  bool started = false;
  bool bnd_dirty = true;

  bool use_graphs = true;
  // Captured step graphs, keyed by what the launch sequence of k steps from
  // step s depends on: k, s modulo lcm(l, 2) (synchronization points, step
  // parity), s == 0 (the first step of a run differs) and the buffers (cur,
  // prev) at s.  Least recently used ones are dropped beyond kMaxGraphs.
  struct GraphEntry {
    int64_t k = 0, phase = 0;
    bool first = false;
    int cur = 0, prev = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  int64_t steps_in_graphs = 0;  // steps run by graph replays so far
  int64_t syncs_done = 0;       // synchronization steps enqueued so far

  int *h_flag = nullptr;
  hipEvent_t flag_ev = nullptr;
  bool flag_pending = false;
  bool nonfinite = false;

  int64_t device_bytes = 0;
};

namespace {

lbm_status fail(lbm_ctx *c, lbm_status st, const std::string &msg) {
  if (c)
    c->err = msg;
  else
    g_create_error = msg;
  return st;
}

lbm_status hip_fail(lbm_ctx *c, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(c, LBM_E_NOMEM, m);
  return fail(c, LBM_E_DEVICE, m);
}

#define HIP_TRY(c, expr, what)                        \
  do {                                                \
    hipError_t _e = (expr);                           \
    if (_e != hipSuccess) return hip_fail(c, _e, what); \
  } while (0)

void *dev_alloc(lbm_ctx *c, size_t bytes) {
  if (bytes == 0) bytes = 256;
  void *p = nullptr;
  if (c->have_alloc) {
    p = c->alloc.alloc(bytes, c->alloc.user);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    c->bufs.push_back({p, bytes});
    c->device_bytes += (int64_t)bytes;
  }
  return p;
}

void dev_free(lbm_ctx *c, void *p) {
  if (!p) return;
  for (size_t k = 0; k < c->bufs.size(); k++)
    if (c->bufs[k].p == p) {
      if (c->have_alloc)
        c->alloc.free(p, c->alloc.user);
      else
        (void)hipFree(p);
      c->device_bytes -= (int64_t)c->bufs[k].bytes;
      c->bufs.erase(c->bufs.begin() + (long)k);
      return;
    }
}

// Grow a device array to hold n elements of T (contents not kept).
template <class T>
bool dev_reserve(lbm_ctx *c, T *&ptr, size_t &cap, size_t n) {
  if (n <= cap && ptr) return true;
  dev_free(c, ptr);
  const size_t want = std::max<size_t>(1, n + n / 4);
  ptr = (T *)dev_alloc(c, want * sizeof(T));
  cap = ptr ? want : 0;
  return ptr != nullptr;
}

void dev_free_all(lbm_ctx *c) {
  for (auto &b : c->bufs) {
    if (c->have_alloc)
      c->alloc.free(b.p, c->alloc.user);
    else
      (void)hipFree(b.p);
  }
  c->bufs.clear();
}

void drop_graph(lbm_ctx *c) {
  for (auto &g : c->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  c->graphs.clear();
}

// Equilibrium weights and wave speeds (Sec. 2; Sec. 3, eqs. feq_req,
// parameters_to_wavespeed_relation, conditions-parameters).
lbm_status plate_params(const lbm_plate &p, PlateDev &d) {
  if (!(p.dh > 0) || !(p.dt > 0) || !(p.rho_m > 0) || !(p.mu > 0) || !(p.lambda + 2.0 * p.mu > 0))
    return LBM_E_INVAL;
  const double cd = std::sqrt((p.lambda + 2.0 * p.mu) / p.rho_m);
  const double cs = std::sqrt(p.mu / p.rho_m);
  const double rd = cd * p.dt / p.dh, rs = cs * p.dt / p.dh;
  d.a[0] = 0.5 * rd * rd;
  d.a[1] = 0.5 * rs * rs;
  d.a0[0] = 1.0 - 4.0 * d.a[0];
  d.a0[1] = 1.0 - 4.0 * d.a[1];
  if (d.a0[0] < -1e-12) return LBM_E_UNSTABLE_DT;
  for (int f = 0; f < 2; f++) {
    d.af[f] = (float)d.a[f];
    d.a0f[f] = (float)d.a0[f];
  }
  d.cd2 = cd * cd;
  d.cs2 = cs * cs;
  d.dt = p.dt;
  d.dh = p.dh;
  d.inv_h = 1.0 / p.dh;
  d.inv_2h = 1.0 / (2.0 * p.dh);
  d.rho_m = p.rho_m;
  d.lam = p.lambda;
  d.mu = p.mu;
  if (p.integrator != 0 && p.integrator != 1) return LBM_E_INVAL;
  d.integ = p.integrator;
  if (p.readings < 0 || p.readings > (RD_FLUX_STREAMED | RD_EQ_OLD)) return LBM_E_INVAL;
  d.readings = p.readings;
  return LBM_OK;
}

// Classification of one plate; fills the dense class bytes.  Returns false
// for a body node without a body neighbour on either side along an axis.
bool classify(const lbm_plate &p, PlateHost &h, std::string &why) {
  const int nx = p.nx, ny = p.ny;
  std::vector<uint8_t> in((size_t)nx * ny);
  for (size_t k = 0; k < in.size(); k++) in[k] = p.mask ? (p.mask[k] != 0) : 1;
  auto inb = [&](int i, int j) -> bool {
    if (i < 0 || i >= nx) {
      if (!p.periodic_x) return false;
      i = (i + nx) % nx;
    }
    if (j < 0 || j >= ny) {
      if (!p.periodic_y) return false;
      j = (j + ny) % ny;
    }
    return in[(size_t)j * nx + i] != 0;
  };
  h.cls.assign((size_t)nx * ny, 0);
  h.body = 0;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      const size_t k = (size_t)j * nx + i;
      if (!in[k]) continue;
      const bool E = inb(i + 1, j), N = inb(i, j + 1), W = inb(i - 1, j), S = inb(i, j - 1);
      if ((!E && !W) || (!N && !S)) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "node (%d, %d) has no body neighbour on either side along an axis", i, j);
        why = buf;
        return false;
      }
      uint8_t c = CL_IN | (E ? NB_E : 0) | (N ? NB_N : 0) | (W ? NB_W : 0) | (S ? NB_S : 0);
      if ((c & NB_ALL) != NB_ALL) c |= CL_B;
      h.cls[k] = c;
      h.body++;
    }
  // second row: interior node with a boundary neighbour
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      const size_t k = (size_t)j * nx + i;
      const uint8_t c = h.cls[k];
      if (!(c & CL_IN) || (c & CL_B)) continue;
      const int di[4] = {1, 0, -1, 0}, dj[4] = {0, 1, 0, -1};
      for (int d = 0; d < 4; d++) {
        const int ii = (i + di[d] + nx) % nx, jj = (j + dj[d] + ny) % ny;
        if (h.cls[(size_t)jj * nx + ii] & CL_B) {
          h.cls[k] |= CL_S;
          break;
        }
      }
    }
  return true;
}

// Stencil code of the finite difference along axis ax at body node (i, j).
int fd_code_host(const PlateHost &h, int i, int j, int ax) {
  const uint8_t c0 = h.cls[(size_t)j * h.nx + i];
  const uint8_t bp = ax == 0 ? NB_E : NB_N, bm = ax == 0 ? NB_W : NB_S;
  const int di = ax == 0 ? 1 : 0, dj = ax == 0 ? 0 : 1;
  if ((c0 & bp) && (c0 & bm)) return FD_CENTRAL;
  if (c0 & bp) {
    const int ii = (i + di) % h.nx, jj = (j + dj) % h.ny;
    return (h.cls[(size_t)jj * h.nx + ii] & bp) ? FD_FWD3 : FD_FWD2;
  }
  if (c0 & bm) {
    const int ii = (i - di + h.nx) % h.nx, jj = (j - dj + h.ny) % h.ny;
    return (h.cls[(size_t)jj * h.nx + ii] & bm) ? FD_BWD3 : FD_BWD2;
  }
  return FD_NONE;
}

// Work lists of the boundary kernel.  Boundary nodes are cut in row-major
// chunks (at most kChunkNodes, fewer where a chunk's closure would not fit
// the block's LDS); each second-row node joins the chunk of its first
// boundary neighbour.  Per chunk: the gradient nodes its tasks read (its
// boundary nodes, their body neighbours, the boundary neighbours of its
// second-row nodes) and the displacement nodes those gradients' stencils
// touch.
bool build_boundary_tables(lbm_ctx *c, std::string &why) {
  static const int DI[5] = {0, 1, 0, -1, 0}, DJ[5] = {0, 0, 1, 0, -1};
  // neighbour order of BTask.g[1..4]: E, N, W, S
  static const int NI[4] = {1, 0, -1, 0}, NJ[4] = {0, 1, 0, -1};
  static const uint8_t NB[4] = {NB_E, NB_N, NB_W, NB_S};
  c->chunks.clear();
  c->unodes.clear();
  c->gnodes.clear();
  c->btasks.clear();
  c->btask_bnd.clear();
  c->stasks.clear();
  auto find_b = [&](const PlateHost &h, int64_t node) -> int64_t {
    auto first = c->bnd.begin() + h.b0, last = c->bnd.begin() + h.b1;
    auto it = std::lower_bound(first, last, node,
                               [](const BndNode &b, int64_t v) { return b.node < v; });
    return (it != last && it->node == node) ? (int64_t)(it - c->bnd.begin()) : -1;
  };
  // second-row nodes by their first boundary neighbour
  std::vector<std::vector<int>> sec_of_b(c->bnd.size());
  for (size_t si = 0; si < c->sec.size(); si++) {
    const SecNode &S = c->sec[si];
    const PlateHost &h = c->ph[S.plate];
    for (int al = 1; al < 5; al++) {
      const int ii = (S.i - DI[al] + h.nx) % h.nx, jj = (S.j - DJ[al] + h.ny) % h.ny;
      if (h.cls[(size_t)jj * h.nx + ii] & CL_B) {
        const int64_t b = find_b(h, h.off + (int64_t)jj * h.pitch + ii);
        if (b < 0) {
          why = "second-row node without its boundary record";
          return false;
        }
        sec_of_b[(size_t)b].push_back((int)si);
        break;
      }
    }
  }
  typedef std::pair<int64_t, std::pair<int, int>> Key;  // node, (i, j)
  // Closure of boundary records [b0, b1) of plate p; false if too large.
  auto closure = [&](int p, int64_t b0, int64_t b1, std::vector<Key> &g, std::vector<Key> &u) {
    const PlateHost &h = c->ph[p];
    g.clear();
    u.clear();
    auto key = [&](int i, int j) { return Key{h.off + (int64_t)j * h.pitch + i, {i, j}}; };
    for (int64_t b = b0; b < b1; b++) {
      const BndNode &B = c->bnd[b];
      g.push_back(key(B.i, B.j));
      const uint8_t cl = h.cls[(size_t)B.j * h.nx + B.i];
      for (int d = 0; d < 4; d++)
        if (cl & NB[d]) g.push_back(key((B.i + NI[d] + h.nx) % h.nx, (B.j + NJ[d] + h.ny) % h.ny));
      for (int si : sec_of_b[(size_t)b]) {
        const SecNode &S = c->sec[si];
        for (int al = 1; al < 5; al++) {
          const int ii = (S.i - DI[al] + h.nx) % h.nx, jj = (S.j - DJ[al] + h.ny) % h.ny;
          if (h.cls[(size_t)jj * h.nx + ii] & CL_B) g.push_back(key(ii, jj));
        }
      }
    }
    std::sort(g.begin(), g.end());
    g.erase(std::unique(g.begin(), g.end()), g.end());
    for (const Key &e : g) {
      const int i = e.second.first, j = e.second.second;
      u.push_back(key(i, j));
      for (int ax = 0; ax < 2; ax++) {
        const int di = ax == 0 ? 1 : 0, dj = ax == 0 ? 0 : 1;
        const int code = fd_code_host(h, i, j, ax);
        auto at = [&](int m) { return key((i + m * di + 2 * h.nx) % h.nx, (j + m * dj + 2 * h.ny) % h.ny); };
        if (code == FD_CENTRAL) { u.push_back(at(1)); u.push_back(at(-1)); }
        if (code == FD_FWD3) { u.push_back(at(1)); u.push_back(at(2)); }
        if (code == FD_BWD3) { u.push_back(at(-1)); u.push_back(at(-2)); }
        if (code == FD_FWD2) u.push_back(at(1));
        if (code == FD_BWD2) u.push_back(at(-1));
      }
    }
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    int ns = 0;
    for (int64_t b = b0; b < b1; b++) ns += (int)sec_of_b[(size_t)b].size();
    return (int)g.size() <= kMaxGrad && (int)u.size() <= kMaxU &&
           (b1 - b0) + 2 * ns <= kBoundaryThreads;
  };
  std::vector<Key> g, u;
  for (size_t p = 0; p < c->ph.size(); p++) {
    const PlateHost &h = c->ph[p];
    int64_t b = h.b0;
    while (b < h.b1) {
      int64_t n = std::min<int64_t>(kChunkNodes, h.b1 - b);
      while (!closure((int)p, b, b + n, g, u)) {
        if (n == 1) {
          why = "boundary chunk closure does not fit a block";
          return false;
        }
        n /= 2;
      }
      auto local = [](const std::vector<Key> &v, int64_t node) -> int {
        auto it = std::lower_bound(v.begin(), v.end(), Key{node, {INT32_MIN, INT32_MIN}});
        return (it != v.end() && it->first == node) ? (int)(it - v.begin()) : -1;
      };
      auto nodeat = [&](int i, int j) { return h.off + (int64_t)j * h.pitch + i; };
      Chunk ch{};
      ch.plate = (int)p;
      ch.u0 = (int)c->unodes.size();
      ch.g0 = (int)c->gnodes.size();
      ch.b0 = (int)c->btasks.size();
      ch.s0 = (int)c->stasks.size();
      for (const Key &e : u) {
        UNode U{};
        U.node = e.first;
        U.i = e.second.first;
        U.j = e.second.second;
        U.bnd = (h.cls[(size_t)U.j * h.nx + U.i] & CL_B) ? 1 : 0;
        c->unodes.push_back(U);
      }
      for (const Key &e : g) {
        const int i = e.second.first, j = e.second.second;
        GradNode G{};
        const int cx = fd_code_host(h, i, j, 0), cy = fd_code_host(h, i, j, 1);
        G.code = cx | (cy << 3);
        const int self = local(u, e.first);
        for (int q = 0; q < 5; q++) G.u[q] = self;
        for (int ax = 0; ax < 2; ax++) {
          const int di = ax == 0 ? 1 : 0, dj = ax == 0 ? 0 : 1;
          const int code = ax == 0 ? cx : cy;
          auto at = [&](int m) {
            return local(u, nodeat((i + m * di + 2 * h.nx) % h.nx, (j + m * dj + 2 * h.ny) % h.ny));
          };
          int a = self, bb = self;
          if (code == FD_CENTRAL) { a = at(1); bb = at(-1); }
          if (code == FD_FWD3) { a = at(1); bb = at(2); }
          if (code == FD_BWD3) { a = at(-1); bb = at(-2); }
          if (code == FD_FWD2) a = at(1);
          if (code == FD_BWD2) a = at(-1);
          G.u[1 + 2 * ax] = a;
          G.u[2 + 2 * ax] = bb;
        }
        c->gnodes.push_back(G);
      }
      for (int64_t bi = b; bi < b + n; bi++) {
        const BndNode &B = c->bnd[bi];
        const uint8_t cl = h.cls[(size_t)B.j * h.nx + B.i];
        BTask T{};
        T.b = B;
        T.g[0] = local(g, B.node);
        for (int d = 0; d < 4; d++)
          T.g[1 + d] = (cl & NB[d]) ? local(g, nodeat((B.i + NI[d] + h.nx) % h.nx,
                                                      (B.j + NJ[d] + h.ny) % h.ny))
                                    : -1;
        c->btasks.push_back(T);
        c->btask_bnd.push_back(bi);
        for (int si : sec_of_b[(size_t)bi]) {
          const SecNode &S = c->sec[si];
          STask Q{};
          Q.node = S.node;
          Q.i = S.i;
          Q.j = S.j;
          Q.g[0] = -1;
          Q.si = si;
          for (int al = 1; al < 5; al++) {
            const int ii = (S.i - DI[al] + h.nx) % h.nx, jj = (S.j - DJ[al] + h.ny) % h.ny;
            Q.g[al] = (h.cls[(size_t)jj * h.nx + ii] & CL_B) ? local(g, nodeat(ii, jj)) : -1;
          }
          c->stasks.push_back(Q);
        }
      }
      ch.u1 = (int)c->unodes.size();
      ch.g1 = (int)c->gnodes.size();
      ch.b1 = (int)c->btasks.size();
      ch.s1 = (int)c->stasks.size();
      c->chunks.push_back(ch);
      b += n;
    }
  }
  return true;
}

// Row bands of height `rows` on a plate of ny rows; the band holding row j.
int band_of(int j, int rows, int nb) { return std::min(j / rows, nb - 1); }

// The column strip of plate h holding column x (0 <= x < nx).
int strip_of(const PlateHost &h, int x) {
  const int s = (int)(std::upper_bound(h.sx.begin(), h.sx.end(), x) - h.sx.begin()) - 1;
  return std::min(std::max(s, 0), h.ns - 1);
}

// v within [lo - r, hi - 1 + r] (an owned range of a tile plus a ring of r
// nodes), with wrap-around on a periodic axis of length n.
bool in_ring_r(int v, int lo, int hi, int n, bool per, int r) {
  if (!per) return v >= lo - r && v <= hi - 1 + r;
  const int d = ((v - (lo - r)) % n + n) % n;
  return d <= hi - lo - 1 + 2 * r;
}

// Calls fn(tile index, owned) for every tile of plate p whose owned area or
// ring of r nodes holds node (i, j) (plate strips built).
template <class F>
void tiles_near(const lbm_ctx *c, int p, int i, int j, int r, F &&fn) {
  const PlateHost &h = c->ph[(size_t)p];
  int strips[8], ns = 0;
  for (int dx = -r; dx <= r; dx++) {
    int x = i + dx;
    if (x < 0 || x >= h.nx) {
      if (!h.px) continue;
      x = ((x % h.nx) + h.nx) % h.nx;
    }
    const int st = strip_of(h, x);
    bool dup = false;
    for (int q = 0; q < ns; q++) dup = dup || strips[q] == st;
    if (!dup && ns < 8) strips[ns++] = st;
  }
  int cand[64], nc = 0;
  for (int q = 0; q < ns; q++) {
    const auto &col = h.strips[(size_t)strips[q]];
    for (int dy = -r; dy <= r; dy++) {
      int y = j + dy;
      if (y < 0 || y >= h.ny) {
        if (!h.py) continue;
        y = ((y % h.ny) + h.ny) % h.ny;
      }
      auto it = std::upper_bound(col.begin(), col.end(), std::make_pair(y, INT32_MAX));
      const int ti = std::prev(it)->second;
      bool dup = false;
      for (int k = 0; k < nc; k++) dup = dup || cand[k] == ti;
      if (!dup && nc < 64) cand[nc++] = ti;
    }
  }
  for (int q = 0; q < nc; q++) {
    const Tile &t = c->tiles[(size_t)cand[q]];
    if (!in_ring_r(i, t.x0, t.x1, h.nx, h.px, r) || !in_ring_r(j, t.y0, t.y1, h.ny, h.py, r))
      continue;
    fn(cand[q], i >= t.x0 && i < t.x1 && j >= t.y0 && j < t.y1);
  }
}

// The tile of plate p that owns node (i, j).
int tile_at(const lbm_ctx *c, int p, int i, int j) {
  const PlateHost &h = c->ph[(size_t)p];
  const auto &col = h.strips[(size_t)strip_of(h, i)];
  auto it = std::upper_bound(col.begin(), col.end(), std::make_pair(j, INT32_MAX));
  return std::prev(it)->second;
}

// Two-step tiles (steps = 2): tiles with no boundary or second-row node in
// their area or two-node ring and some body node, so that two time steps of
// the plain scheme cover their area; the others take single steps.  A
// two-step tile exports the t_{n+1} populations of its owned nodes that lie
// in the one-node ring of a single-step tile.
void classify_two_step(lbm_ctx *c) {
  c->n_two = 0;
  for (Tile &t : c->tiles) t.flags = 0;
  if (c->two == 0) return;
  std::vector<uint8_t> near(c->tiles.size(), 0);
  auto mark = [&](int p, int i, int j) {
    tiles_near(c, p, i, j, 2, [&](int ti, bool) { near[(size_t)ti] = 1; });
  };
  for (const BndNode &B : c->bnd) mark(B.plate, B.i, B.j);
  for (const SecNode &S : c->sec) mark(S.plate, S.i, S.j);
  for (size_t ti = 0; ti < c->tiles.size(); ti++) {
    Tile &t = c->tiles[ti];
    const PlateHost &h = c->ph[(size_t)t.plate];
    // (the two-node ring must not wrap more than once around a periodic plate)
    if (!near[ti] && h.nx >= 4 && h.ny >= 4 && (h.cls[(size_t)t.y0 * h.nx + t.x0] & CL_IN))
      t.flags |= TF_TWO;
  }
  for (const Tile &t : c->tiles)
    if (t.flags & TF_TWO) c->n_two += (int64_t)(t.x1 - t.x0) * (t.y1 - t.y0);
  // Frame tiles: two-step tiles owning a node of the two-node ring of a
  // single-step tile (the relation is symmetric), so that the other
  // two-step tiles (deep tiles) neither read nor write what single-step
  // tiles own.
  for (const Tile &e : c->tiles) {
    if (e.flags & TF_TWO) continue;
    const PlateHost &h = c->ph[(size_t)e.plate];
    auto frame = [&](int i, int j) {
      if (i < 0 || i >= h.nx) {
        if (!h.px) return;
        i = ((i % h.nx) + h.nx) % h.nx;
      }
      if (j < 0 || j >= h.ny) {
        if (!h.py) return;
        j = ((j % h.ny) + h.ny) % h.ny;
      }
      Tile &o = c->tiles[(size_t)tile_at(c, e.plate, i, j)];
      if (o.flags & TF_TWO) o.flags |= TF_FRAME;
    };
    for (int j = e.y0 - 2; j < e.y1 + 2; j++) {
      if (j < e.y0 || j >= e.y1) {
        for (int i = e.x0 - 2; i < e.x1 + 2; i++) frame(i, j);
      } else {
        frame(e.x0 - 2, j);
        frame(e.x0 - 1, j);
        frame(e.x1, j);
        frame(e.x1 + 1, j);
      }
    }
  }
  c->n_deep = 0;
  for (const Tile &t : c->tiles)
    if ((t.flags & TF_TWO) && !(t.flags & TF_FRAME))
      c->n_deep += (int64_t)(t.x1 - t.x0) * (t.y1 - t.y0);
  for (const Tile &e : c->tiles) {
    if (e.flags & TF_TWO) continue;
    const PlateHost &h = c->ph[(size_t)e.plate];
    auto exp = [&](int i, int j, int bit) {
      if (i < 0 || i >= h.nx) {
        if (!h.px) return;
        i = (i + h.nx) % h.nx;
      }
      if (j < 0 || j >= h.ny) {
        if (!h.py) return;
        j = (j + h.ny) % h.ny;
      }
      Tile &o = c->tiles[(size_t)tile_at(c, e.plate, i, j)];
      if (o.flags & TF_TWO) o.flags |= bit;
    };
    for (int j = e.y0; j < e.y1; j++) {
      exp(e.x0 - 1, j, TF_EXP_E);  // west ring column: the east column of its owner
      exp(e.x1, j, TF_EXP_W);
    }
    for (int i = e.x0; i < e.x1; i++) {
      exp(i, e.y0 - 1, TF_EXP_N);
      exp(i, e.y1, TF_EXP_S);
    }
  }
}

// Paired edge strips: on a plate with narrow first and last column strips
// (edge_cols), each single-step tile of the last strip becomes the second
// column segment of the single-step tile of the first strip with the same
// rows and march direction, when both segments and their halo columns fit
// the workgroup, so that the edge strips run with about twice the live
// lanes and half the tiles.  The last-strip tile stays in the list
// (TF_MERGED) for the host's lookups; the first-strip tile carries both
// prologue work lists (build_tile_tables).  Any workgroup size: since the
// prologue issues its reads together, the joint prologue of a pair costs
// little more than one, and on the 8192^2 plate pairs take 15-35 us off
// the second launch of 128- and 256-lane tilings at no cost to the first.
void pair_edge_tiles(lbm_ctx *c) {
  c->partner.assign(c->tiles.size(), -1);
  if (c->edge_cols <= 0) return;
  for (size_t p = 0; p < c->ph.size(); p++) {
    const PlateHost &h = c->ph[p];
    const int ec = c->edge_cols;
    if (h.px || h.ns < 3 || h.sx[1] != ec || h.sx[(size_t)h.ns - 1] != h.nx - ec) continue;
    const auto &L = h.strips[0];
    const auto &R = h.strips[(size_t)h.ns - 1];
    size_t ir = 0;
    for (const auto &l : L) {
      while (ir < R.size() && R[ir].first < l.first) ir++;
      if (ir >= R.size()) break;
      if (R[ir].first != l.first) continue;
      Tile &A = c->tiles[(size_t)l.second];
      Tile &B = c->tiles[(size_t)R[ir].second];
      if (A.y1 != B.y1 || A.dir != B.dir || (A.flags & TF_TWO) || (B.flags & TF_TWO)) continue;
      if ((A.x1 - A.x0) + (B.x1 - B.x0) + 4 > c->lanes) continue;
      A.bx0 = B.x0;
      A.bx1 = B.x1;
      B.flags |= TF_MERGED;
      c->partner[(size_t)l.second] = R[ir].second;
    }
  }
}

// Interior tiles: per plate, column strips of at most lanes-2 columns (of
// equal width, or of a multiple of align columns but the last; with
// edge_cols the first and last strip of a plate whose x axis is not periodic
// are edge_cols wide and the others fill the columns between) times row
// bands of `rows` rows; a band piece whose area or
// halo ring holds boundary or second-row nodes (a tile with a prologue) is
// cut into pieces of edge_rows rows, so that its boundary work plus its
// shorter march ends with the other tiles' marches.  Vertically adjacent
// tiles march in opposite directions (dir).  order 0: plate by
// plate, band by band (strips of a band adjacent); 1: plate by plate, strip
// by strip (bands of a strip adjacent); 2: as 0 with the plates by decreasing
// size; 3: plate by plate in groups of kBandGroup row bands, within a group
// strip by strip with the group's bands of one strip consecutive.
// Consecutive tiles land on the same XCD (see k_interior) and start at about
// the same time, so the order decides which halo rows / columns share an L2:
// with order 0 a tile's x-neighbours are its list neighbours but its
// y-neighbours a whole band of strips away (on an 8192^2 plate long gone from
// the L2 when they read the shared halo rows); order 3 keeps both close, the
// bands of a group marching in alternating directions so that each shared
// pair of halo rows is read by its two tiles at the same end of their
// marches.  With overlapped
// two-step pairs the band pieces around those with boundary work are cut to
// edge_rows as well (they hold the frame tiles, see classify_two_step).
constexpr int kBandGroup = 4;
// MI355X's Infinity Cache (the memory-side cache in front of HBM).
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;

void build_tiles(lbm_ctx *c) {
  c->tiles.clear();
  const int own = c->lanes - (c->two ? 4 : 2);
  const int rows = c->rows;
  const int er = (c->edge_rows > 0 && c->edge_rows < rows) ? c->edge_rows : rows;
  std::vector<int> plates(c->ph.size());
  for (size_t p = 0; p < plates.size(); p++) plates[p] = (int)p;
  if (c->order == 2)
    std::stable_sort(plates.begin(), plates.end(), [&](int a, int b) {
      return (int64_t)c->ph[a].nx * c->ph[a].ny > (int64_t)c->ph[b].nx * c->ph[b].ny;
    });
  // band pieces with boundary work, per plate (strip-major)
  std::vector<std::vector<uint8_t>> work(c->ph.size());
  for (size_t p = 0; p < c->ph.size(); p++) {
    PlateHost &h = c->ph[p];
    // strips over [a, b): aligned or equal widths of at most `own` columns
    auto span = [&](int a, int b) {
      const int n = b - a;
      if (c->align > 0 && own >= c->align) {
        const int w = own / c->align * c->align;
        for (int x = a; x < b; x += w) h.sx.push_back(x);
      } else {
        const int k = (n + own - 1) / own, w = (n + k - 1) / k;
        for (int x = a; x < b; x += w) h.sx.push_back(x);
      }
    };
    h.sx.clear();
    const int ec = c->edge_cols;
    if (ec > 0 && !h.px && h.nx > 2 * ec + 2) {
      h.sx.push_back(0);
      span(ec, h.nx - ec);
      h.sx.push_back(h.nx - ec);
    } else {
      span(0, h.nx);
    }
    h.ns = (int)h.sx.size();
    h.sx.push_back(h.nx);
    const int nb = (h.ny + rows - 1) / rows;
    if (er < rows) work[p].assign((size_t)h.ns * nb, 0);
  }
  if (er < rows) {
    auto mark = [&](int p, int i, int j) {
      const PlateHost &h = c->ph[(size_t)p];
      const int nb = (h.ny + rows - 1) / rows;
      const int s0 = strip_of(h, i), b0 = band_of(j, rows, nb);
      for (int ds = -1; ds <= 1; ds++)
        for (int db = -1; db <= 1; db++) {
          int s = s0 + ds, b = b0 + db;
          if (s < 0 || s >= h.ns) {
            if (!h.px) continue;
            s = (s + h.ns) % h.ns;
          }
          if (b < 0 || b >= nb) {
            if (!h.py) continue;
            b = (b + nb) % nb;
          }
          const int x0 = h.sx[(size_t)s], x1 = h.sx[(size_t)s + 1];
          const int y0 = b * rows, y1 = std::min(h.ny, (b + 1) * rows);
          if (in_ring_r(i, x0, x1, h.nx, h.px, 1) && in_ring_r(j, y0, y1, h.ny, h.py, 1))
            work[(size_t)p][(size_t)s * nb + b] = 1;
        }
    };
    for (const BndNode &B : c->bnd) mark(B.plate, B.i, B.j);
    for (const SecNode &S : c->sec) mark(S.plate, S.i, S.j);
    // With overlapped two-step pairs, the band pieces next to those are cut
    // too: they hold the frame tiles, whose two steps a single-step launch
    // waits for.
    if (c->two && c->overlap) {
      for (size_t p = 0; p < c->ph.size(); p++) {
        const PlateHost &h = c->ph[p];
        const int nb = (h.ny + rows - 1) / rows;
        const std::vector<uint8_t> w0 = work[p];
        for (int s = 0; s < h.ns; s++)
          for (int b = 0; b < nb; b++) {
            if (!w0[(size_t)s * nb + b]) continue;
            for (int ds = -1; ds <= 1; ds++)
              for (int db = -1; db <= 1; db++) {
                int s2 = s + ds, b2 = b + db;
                if (s2 < 0 || s2 >= h.ns) {
                  if (!h.px) continue;
                  s2 = (s2 + h.ns) % h.ns;
                }
                if (b2 < 0 || b2 >= nb) {
                  if (!h.py) continue;
                  b2 = (b2 + nb) % nb;
                }
                work[p][(size_t)s2 * nb + b2] = 1;
              }
          }
      }
    }
  }
  for (int p : plates) {
    PlateHost &h = c->ph[p];
    const int ns = h.ns;
    const int nb = (h.ny + rows - 1) / rows;
    h.strips.assign((size_t)ns, {});
    auto add = [&](int s, int b) {
      const int x0 = h.sx[(size_t)s], x1 = h.sx[(size_t)s + 1];
      const int y0 = b * rows, y1 = std::min(h.ny, (b + 1) * rows);
      const int hgt = (er < rows && work[(size_t)p][(size_t)s * nb + b]) ? er : rows;
      for (int y = y0, piece = 0; y < y1; y += hgt, piece++) {
        Tile t{};
        t.plate = p;
        t.chunk = -1;
        t.dir = (b + piece) & 1;
        t.x0 = x0;
        t.x1 = x1;
        t.y0 = y;
        t.y1 = std::min(y1, y + hgt);
        h.strips[(size_t)s].push_back({y, (int)c->tiles.size()});
        c->tiles.push_back(t);
      }
    };
    if (c->order == 1) {
      for (int s = 0; s < ns; s++)
        for (int b = 0; b < nb; b++) add(s, b);
    } else if (c->order == 3) {
      // groups of kBandGroup bands; in a group, strip by strip, the group's
      // bands of a strip one after the other
      for (int g = 0; g < nb; g += kBandGroup)
        for (int s = 0; s < ns; s++)
          for (int b = g; b < std::min(nb, g + kBandGroup); b++) add(s, b);
    } else {
      for (int b = 0; b < nb; b++)
        for (int s = 0; s < ns; s++) add(s, b);
    }
  }
  classify_two_step(c);
  pair_edge_tiles(c);
}

// Prologue work lists.  A boundary or second-row node belongs to every tile
// whose owned area or one-node halo ring contains it (the march reads the
// populations of the ring).  Per tile: the boundary tasks (all reset, owned
// ones also accelerate), the second-row tasks, and the gradient nodes they
// read (their boundary nodes, the body neighbours of owned boundary nodes,
// the boundary neighbours of the second-row nodes).
void build_tile_tables(lbm_ctx *c) {
  static const int DI[5] = {0, 1, 0, -1, 0}, DJ[5] = {0, 0, 1, 0, -1};
  static const int NI[4] = {1, 0, -1, 0}, NJ[4] = {0, 1, 0, -1};
  static const uint8_t NB[4] = {NB_E, NB_N, NB_W, NB_S};
  c->tchunks.clear();
  c->tgn.clear();
  c->tbt.clear();
  c->tbt_bnd.clear();
  c->tst.clear();
  for (Tile &t : c->tiles) t.chunk = -1;
  std::vector<std::vector<std::pair<int64_t, int>>> tb(c->tiles.size());  // (bnd index, owned)
  std::vector<std::vector<int>> ts(c->tiles.size());                       // sec index
  // the tiles whose owned area or halo ring holds node (i, j)
  auto visit = [&](int p, int i, int j, auto &&fn) { tiles_near(c, p, i, j, 1, fn); };
  for (size_t b = 0; b < c->bnd.size(); b++) {
    const BndNode &B = c->bnd[b];
    visit(B.plate, B.i, B.j, [&](int ti, bool owned) { tb[ti].push_back({(int64_t)b, owned ? 1 : 0}); });
  }
  for (size_t si = 0; si < c->sec.size(); si++) {
    const SecNode &S = c->sec[si];
    visit(S.plate, S.i, S.j, [&](int ti, bool) { ts[ti].push_back((int)si); });
  }
  // a paired tile carries its second segment's lists too (a node in the
  // rings of both segments is listed once, owned if either segment owns it)
  for (size_t ti = 0; ti < c->tiles.size(); ti++) {
    const int pb = ti < c->partner.size() ? c->partner[ti] : -1;
    if (pb < 0) continue;
    for (auto &e : tb[(size_t)pb]) tb[ti].push_back(e);
    for (int si : ts[(size_t)pb]) ts[ti].push_back(si);
    std::sort(tb[ti].begin(), tb[ti].end(), [](const std::pair<int64_t, int> &a,
                                               const std::pair<int64_t, int> &b) {
      return a.first != b.first ? a.first < b.first : a.second > b.second;
    });
    tb[ti].erase(std::unique(tb[ti].begin(), tb[ti].end(),
                             [](const std::pair<int64_t, int> &a, const std::pair<int64_t, int> &b) {
                               return a.first == b.first;
                             }),
                 tb[ti].end());
    std::sort(ts[ti].begin(), ts[ti].end());
    ts[ti].erase(std::unique(ts[ti].begin(), ts[ti].end()), ts[ti].end());
  }
  typedef std::pair<int64_t, std::pair<int, int>> Key;
  std::vector<Key> g;
  for (size_t ti = 0; ti < c->tiles.size(); ti++) {
    if (c->tiles[ti].flags & TF_MERGED) continue;
    if (tb[ti].empty() && ts[ti].empty()) continue;
    Tile &t = c->tiles[ti];
    const PlateHost &h = c->ph[t.plate];
    auto key = [&](int i, int j) { return Key{h.off + (int64_t)j * h.pitch + i, {i, j}}; };
    auto nodeat = [&](int i, int j) { return h.off + (int64_t)j * h.pitch + i; };
    g.clear();
    for (auto &e : tb[ti]) {
      const BndNode &B = c->bnd[(size_t)e.first];
      g.push_back(key(B.i, B.j));
      if (!e.second) continue;
      const uint8_t cl = h.cls[(size_t)B.j * h.nx + B.i];
      for (int d = 0; d < 4; d++)
        if (cl & NB[d]) g.push_back(key((B.i + NI[d] + h.nx) % h.nx, (B.j + NJ[d] + h.ny) % h.ny));
    }
    for (int si : ts[ti]) {
      const SecNode &S = c->sec[si];
      for (int al = 1; al < 5; al++) {
        const int ii = (S.i - DI[al] + h.nx) % h.nx, jj = (S.j - DJ[al] + h.ny) % h.ny;
        if (h.cls[(size_t)jj * h.nx + ii] & CL_B) g.push_back(key(ii, jj));
      }
    }
    std::sort(g.begin(), g.end());
    g.erase(std::unique(g.begin(), g.end()), g.end());
    auto local = [&](int64_t node) -> int {
      auto it = std::lower_bound(g.begin(), g.end(), Key{node, {INT32_MIN, INT32_MIN}});
      return (it != g.end() && it->first == node) ? (int)(it - g.begin()) : -1;
    };
    TileChunk ch{};
    ch.plate = t.plate;
    ch.g0 = (int)c->tgn.size();
    ch.b0 = (int)c->tbt.size();
    ch.s0 = (int)c->tst.size();
    for (const Key &e : g) {
      TGradNode G{};
      G.node = e.first;
      G.i = e.second.first;
      G.j = e.second.second;
      G.code = fd_code_host(h, G.i, G.j, 0) | (fd_code_host(h, G.i, G.j, 1) << 3);
      c->tgn.push_back(G);
    }
    for (auto &e : tb[ti]) {
      const BndNode &B = c->bnd[(size_t)e.first];
      const uint8_t cl = h.cls[(size_t)B.j * h.nx + B.i];
      BTask T{};
      T.b = B;
      T.accel = e.second;
      T.g[0] = local(B.node);
      for (int d = 0; d < 4; d++)
        T.g[1 + d] = (e.second && (cl & NB[d]))
                         ? local(nodeat((B.i + NI[d] + h.nx) % h.nx, (B.j + NJ[d] + h.ny) % h.ny))
                         : -1;
      c->tbt.push_back(T);
      c->tbt_bnd.push_back(e.first);
    }
    for (int si : ts[ti]) {
      const SecNode &S = c->sec[si];
      STask Q{};
      Q.node = S.node;
      Q.i = S.i;
      Q.j = S.j;
      Q.g[0] = -1;
      Q.si = si;
      for (int al = 1; al < 5; al++) {
        const int ii = (S.i - DI[al] + h.nx) % h.nx, jj = (S.j - DJ[al] + h.ny) % h.ny;
        Q.g[al] = (h.cls[(size_t)jj * h.nx + ii] & CL_B) ? local(nodeat(ii, jj)) : -1;
      }
      c->tst.push_back(Q);
    }
    ch.g1 = (int)c->tgn.size();
    ch.b1 = (int)c->tbt.size();
    ch.s1 = (int)c->tst.size();
    t.chunk = (int)c->tchunks.size();
    c->tchunks.push_back(ch);
  }
}

lbm_status upload_tile_tables(lbm_ctx *c) {
  for (size_t k = 0; k < c->tbt.size(); k++) c->tbt[k].b = c->bnd[(size_t)c->tbt_bnd[k]];
  const size_t gsz = c->storage == LBM_STORE_F32 ? 4 : 8;
  if (!dev_reserve(c, c->d_tchunks, c->cap_tchunks, c->tchunks.size()) ||
      !dev_reserve(c, c->d_tgn, c->cap_tgn, c->tgn.size()) ||
      !dev_reserve(c, c->d_tbt, c->cap_tbt, c->tbt.size()) ||
      !dev_reserve(c, c->d_tst, c->cap_tst, c->tst.size()))
    return fail(c, LBM_E_NOMEM, "prologue table allocation failed");
  if (c->tgn.size() * 4 * gsz > c->cap_tgrad || !c->d_tgrad) {
    dev_free(c, c->d_tgrad);
    c->cap_tgrad = std::max<size_t>(256, c->tgn.size() * 4 * gsz);
    c->d_tgrad = dev_alloc(c, c->cap_tgrad);
    if (!c->d_tgrad) return fail(c, LBM_E_NOMEM, "prologue scratch allocation failed");
  }
  if (!c->tchunks.empty())
    HIP_TRY(c, hipMemcpy(c->d_tchunks, c->tchunks.data(), c->tchunks.size() * sizeof(TileChunk),
                         hipMemcpyHostToDevice), "prologue table upload");
  if (!c->tgn.empty())
    HIP_TRY(c, hipMemcpy(c->d_tgn, c->tgn.data(), c->tgn.size() * sizeof(TGradNode),
                         hipMemcpyHostToDevice), "prologue table upload");
  if (!c->tbt.empty())
    HIP_TRY(c, hipMemcpy(c->d_tbt, c->tbt.data(), c->tbt.size() * sizeof(BTask),
                         hipMemcpyHostToDevice), "prologue table upload");
  if (!c->tst.empty())
    HIP_TRY(c, hipMemcpy(c->d_tst, c->tst.data(), c->tst.size() * sizeof(STask),
                         hipMemcpyHostToDevice), "prologue table upload");
  return LBM_OK;
}

lbm_status upload_tile_list(lbm_ctx *c, const std::vector<Tile> &v, Tile *&d, size_t &cap) {
  if (v.size() > cap || !d) {
    const size_t nc = std::max<size_t>(16, v.size() * 2);
    Tile *p = (Tile *)dev_alloc(c, nc * sizeof(Tile));
    if (!p) return fail(c, LBM_E_NOMEM, "tile list allocation failed");
    dev_free(c, d);
    d = p;
    cap = nc;
  }
  if (!v.empty())
    HIP_TRY(c, hipMemcpy(d, v.data(), v.size() * sizeof(Tile), hipMemcpyHostToDevice),
            "tile upload");
  return LBM_OK;
}

lbm_status upload_tiles(lbm_ctx *c) {
  c->etiles.clear();
  c->ftiles.clear();
  c->dtiles.clear();
  c->ltiles.clear();
  for (const Tile &t : c->tiles) {
    if (t.flags & TF_MERGED) continue;
    c->ltiles.push_back(t);
    if (!(t.flags & TF_TWO)) c->etiles.push_back(t);
    if ((t.flags & TF_TWO) && !(t.flags & TF_FRAME))
      c->dtiles.push_back(t);
    else
      c->ftiles.push_back(t);
  }
  lbm_status st = upload_tile_list(c, c->ltiles, c->d_tiles, c->tiles_cap);
  if (st) return st;
  st = upload_tile_list(c, c->ftiles, c->d_ftiles, c->ftiles_cap);
  if (st) return st;
  st = upload_tile_list(c, c->dtiles, c->d_dtiles, c->dtiles_cap);
  if (st) return st;
  return upload_tile_list(c, c->etiles, c->d_etiles, c->etiles_cap);
}

lbm_status upload_boundary(lbm_ctx *c) {
  if (!c->bnd.empty())
    HIP_TRY(c, hipMemcpy(c->d_bnd, c->bnd.data(), c->bnd.size() * sizeof(BndNode),
                         hipMemcpyHostToDevice),
            "boundary upload");
  for (size_t t = 0; t < c->btasks.size(); t++) c->btasks[t].b = c->bnd[(size_t)c->btask_bnd[t]];
  {
    lbm_status st = upload_tile_tables(c);
    if (st) return st;
  }
  if (!c->btasks.empty())
    HIP_TRY(c, hipMemcpy(c->d_btasks, c->btasks.data(), c->btasks.size() * sizeof(BTask),
                         hipMemcpyHostToDevice),
            "boundary task upload");
  if (!c->loads.empty())
    HIP_TRY(c, hipMemcpy(c->d_loads, c->loads.data(), c->loads.size() * sizeof(LoadTable),
                         hipMemcpyHostToDevice),
            "load table upload");
  c->bnd_dirty = false;
  return LBM_OK;
}

bool have_third(const lbm_ctx *c) { return c->ds.u[2][0] != nullptr; }

// Buffer 2 (the intermediate level of two-step pairs), allocated when a
// two-step tiling is first used.  Its u, du/dt start as a copy of buffer
// cur ^ 1, which holds the boundary nodes' u(t_{step+1}) that the first
// step of a pair reads there too.
lbm_status ensure_third(lbm_ctx *c) {
  if (have_third(c)) return LBM_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  const int64_t N = c->n_alloc;
  const int nsl = slot_count(c->storage);
  for (int fl = 0; fl < 2; fl++)
    for (int sl = 0; sl < nsl; sl++) {
      void *p = dev_alloc(c, (size_t)N * slot_bytes(c->storage));
      if (!p) return fail(c, LBM_E_NOMEM, "population allocation failed");
      HIP_TRY(c, hipMemset(p, 0, (size_t)N * slot_bytes(c->storage)), "memset");
      c->ds.pop[2][fl][sl] = p;
    }
  void *uv[4];
  for (int q = 0; q < 4; q++) {
    uv[q] = dev_alloc(c, (size_t)N * uv_bytes(c->storage));
    if (!uv[q]) return fail(c, LBM_E_NOMEM, "u/v allocation failed");
  }
  const int src = c->cur ^ 1;
  for (int comp = 0; comp < 2; comp++) {
    HIP_TRY(c, hipMemcpy(uv[comp], c->ds.u[src][comp], (size_t)N * uv_bytes(c->storage),
                         hipMemcpyDeviceToDevice), "u copy");
    HIP_TRY(c, hipMemcpy(uv[2 + comp], c->ds.v[src][comp], (size_t)N * uv_bytes(c->storage),
                         hipMemcpyDeviceToDevice), "v copy");
    c->ds.u[2][comp] = uv[comp];
    c->ds.v[2][comp] = uv[2 + comp];
  }
  drop_graph(c);
  return LBM_OK;
}

void release_third(lbm_ctx *c) {
  if (!have_third(c)) return;
  (void)hipStreamSynchronize(c->stream);
  for (int fl = 0; fl < 2; fl++)
    for (int sl = 0; sl < 5; sl++) {
      dev_free(c, c->ds.pop[2][fl][sl]);
      c->ds.pop[2][fl][sl] = nullptr;
    }
  for (int comp = 0; comp < 2; comp++) {
    dev_free(c, c->ds.u[2][comp]);
    dev_free(c, c->ds.v[2][comp]);
    c->ds.u[2][comp] = c->ds.v[2][comp] = nullptr;
  }
  drop_graph(c);
}

Prologue make_prologue(const lbm_ctx *c, bool enabled) {
  Prologue p{};
  p.chunks = c->d_tchunks;
  p.gn = c->d_tgn;
  p.bt = c->d_tbt;
  p.st = c->d_tst;
  p.grad = c->d_tgrad;
  p.enabled = enabled && !c->tchunks.empty();
  return p;
}

// Steps [s, s + k) from a complete state at t_s (populations of t_s at every
// body node, u and du/dt of t_s in buffer cur, the boundary nodes' u and
// du/dt of t_{s+1} in the output buffers of the next step): one interior
// launch per step -- or, with two-step tiles, per pair of steps a launch
// that takes those tiles two steps and the others one, and a launch that
// takes the others the second step -- every launch but the first finishing
// the previous step's boundary work in its prologues; then one boundary
// launch finishing step s + k - 1, which leaves the state complete at
// t_{s+k}; then the synchronization if s + k is a multiple of l.  cur and
// prev (buffers of t_s and of the boundary populations of t_{s-1}) are
// advanced.
//
// Overlapped pairs (c->overlap, pairs after the run's first step): the deep
// tiles' two steps go to a launch of their own on the side stream, which
// waits for the first launch of the previous pair (the frame tiles' part of
// its ring) and which the first launch of the next pair waits for; so it
// runs beside this pair's first launch (single-step and frame tiles) and
// its second launch, whose tiles and buffers it does not touch: it reads
// buffer cur at deep and frame nodes only, writes buffer cur ^ 1 at deep
// nodes only, and the other launches write cur ^ 1 and buffer 2 at other
// nodes only and read cur ^ 1 at boundary nodes only.
//
// rec (profiling): events before and after every launch on its stream,
// with the launch's kind (0 single-step interior, 1 boundary, 2
// synchronization, 3 two-step interior, 4 deep tiles).
struct LaunchRecorder {
  struct Rec {
    hipEvent_t a, b;
    int kind;
  };
  std::vector<Rec> recs;
};

bool overlapped_pair(const lbm_ctx *c, int64_t n) {
  return c->two && c->overlap && n > 0 && !c->dtiles.empty() && c->side != nullptr;
}

hipError_t enqueue_segment(lbm_ctx *c, int64_t s, int64_t k, int &cur, int &prev, hipStream_t st,
                           LaunchRecorder *rec) {
  auto timed = [&](int kind, hipStream_t on, auto &&fn) -> hipError_t {
    if (!rec) return fn();
    LaunchRecorder::Rec r{nullptr, nullptr, kind};
    hipError_t e = hipEventCreate(&r.a);
    if (e == hipSuccess) e = hipEventCreate(&r.b);
    if (e == hipSuccess) e = hipEventRecord(r.a, on);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(r.b, on);
    if (r.a || r.b) rec->recs.push_back(r);
    return e;
  };
  const int T = 2;  // intermediate buffer of a two-step pair
  hipError_t e = hipSuccess;
  bool pend_d = false;  // a deep launch that st has not waited for: ev_d[par ^ 1]
  bool have_f = false;  // ev_f[par ^ 1] marks what the next deep launch waits for
  int par = 0;          // parity of the pair (events alternate)
  auto join = [&]() -> hipError_t {
    if (!pend_d) return hipSuccess;
    pend_d = false;
    return hipStreamWaitEvent(st, c->ev_d[par ^ 1], 0);
  };
  for (int64_t n = s; n < s + k && e == hipSuccess;) {
    if (c->two && s + k - n >= 2) {
      const StepBufs b1{cur, T, prev, (int)(n & 1), cur ^ 1, c->nt};
      const Prologue p1 = make_prologue(c, n > s);
      const StepBufs b2{T, cur ^ 1, cur, (int)((n + 1) & 1), -1};
      const Prologue p2 = make_prologue(c, true);
      if (overlapped_pair(c, n)) {
        e = join();
        if (e == hipSuccess && !have_f) e = hipEventRecord(c->ev_f[par ^ 1], st);
        if (e == hipSuccess)
          e = timed(3, st, [&] {
            return launch_interior(c->storage, c->ds, c->d_ftiles, (int)c->ftiles.size(),
                                   c->lanes, b1, p1, st);
          });
        if (e == hipSuccess) e = hipEventRecord(c->ev_f[par], st);
        if (e == hipSuccess)
          e = timed(0, st, [&] {
            return launch_interior(c->storage, c->ds, c->d_etiles, (int)c->etiles.size(),
                                   c->lanes, b2, p2, st);
          });
        if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_f[par ^ 1], 0);
        if (e == hipSuccess)
          e = timed(4, c->side, [&] {
            return launch_deep(c->storage, c->ds, c->d_dtiles, (int)c->dtiles.size(), c->lanes,
                               b1, c->side);
          });
        if (e == hipSuccess) e = hipEventRecord(c->ev_d[par], c->side);
        if (e != hipSuccess) break;
        pend_d = true;
        have_f = true;
        par ^= 1;
      } else {
        e = join();
        if (e == hipSuccess)
          e = timed(3, st, [&] {
            return launch_interior(c->storage, c->ds, c->d_tiles, (int)c->ltiles.size(), c->lanes,
                                   b1, p1, st);
          });
        if (e == hipSuccess)
          e = timed(0, st, [&] {
            return launch_interior(c->storage, c->ds, c->d_etiles, (int)c->etiles.size(),
                                   c->lanes, b2, p2, st);
          });
        have_f = false;
      }
      prev = T;
      cur ^= 1;
      n += 2;
    } else {
      const StepBufs b1{cur, cur ^ 1, prev, (int)(n & 1), -1};
      const Prologue p1 = make_prologue(c, n > s);
      e = join();
      if (e == hipSuccess)
        e = timed(0, st, [&] {
          return launch_interior(c->storage, c->ds, c->d_tiles, (int)c->ltiles.size(), c->lanes,
                                 b1, p1, st);
        });
      have_f = false;
      prev = cur;
      cur ^= 1;
      n += 1;
    }
  }
  if (e == hipSuccess) e = join();
  if (e != hipSuccess) return e;
  // The boundary work of step s + k - 1; the boundary nodes' u(t_{s+k+1})
  // goes to both buffers the next step may write.
  const int c_now = cur, p_now = prev;
  e = timed(1, st, [&] {
    return launch_boundary(c->storage, c->ds, c->d_chunks, (int)c->chunks.size(), c->d_unodes,
                           c->d_gnodes, c->d_btasks, c->d_stasks, c_now, p_now, c_now ^ 1,
                           have_third(c) ? T : -1,
                           (int)((s + k) & 1), 1, st);
  });
  if (e != hipSuccess) return e;
  if (c->sync_every > 0 && (s + k) % c->sync_every == 0) {
    e = timed(2, st, [&] {
      return launch_sync(c->storage, c->ds, c->d_tiles, (int)c->ltiles.size(), c->lanes, c_now,
                         st);
    });
  }
  return e;
}

// Length of the segment starting at step s (ends at the next synchronization;
// one step with readings other than R1 + M1).
int64_t segment_limit(const lbm_ctx *c, int64_t s, int64_t n) {
  if (c->variant_readings) return std::min<int64_t>(n, 1);
  if (c->sync_every <= 0) return n;
  return std::min<int64_t>(n, c->sync_every - s % c->sync_every);
}

// Buffers after the steps [s, s + n) from buffers (cur, prev), as
// enqueue_segment leaves them.
void advance_buffers(const lbm_ctx *c, int64_t s, int64_t n, int &cur, int &prev) {
  while (n > 0) {
    const int64_t k = segment_limit(c, s, n);
    for (int64_t m = s; m < s + k;) {
      if (c->two && s + k - m >= 2) {
        prev = 2;
        m += 2;
      } else {
        prev = cur;
        m += 1;
      }
      cur ^= 1;
    }
    s += k;
    n -= k;
  }
}

// Steps per captured graph of whole periods: a multiple of l that starts
// and ends on the same buffers.
int64_t graph_period(const lbm_ctx *c) {
  int64_t g = c->sync_every > 0 ? c->sync_every : 64;
  while (g < 32) g *= 2;
  for (int r = 0; r < 4; r++, g *= 2) {
    int cur = c->cur, prev = c->prev;
    advance_buffers(c, 0, g, cur, prev);
    if (cur == c->cur && prev == c->prev) return g;
  }
  return 0;  // no period found: graphs of at most kMaxGraphSteps steps
}

constexpr size_t kMaxGraphs = 8;
constexpr int64_t kMaxGraphSteps = 256;

// Period of the launch sequence's dependence on the starting step.
int64_t phase_period(const lbm_ctx *c) {
  if (c->sync_every <= 0) return 2;
  return c->sync_every % 2 == 0 ? c->sync_every : 2 * (int64_t)c->sync_every;
}

// Steps of the next graph of a run of n steps from step s.
int64_t graph_chunk(const lbm_ctx *c, int64_t s, int64_t n) {
  const int64_t G = graph_period(c);
  if (G <= 0) return std::min(n, kMaxGraphSteps);
  if (s % G == 0 && n >= G) return G;
  return std::min(n, G - s % G);
}

// The captured graph of steps [s, s + k) from buffers (cur, prev), from the
// cache or captured now.
lbm_status graph_for(lbm_ctx *c, int64_t s, int64_t k, int cur, int prev, hipGraphExec_t *out) {
  const int64_t phase = s % phase_period(c);
  const bool first = s == 0;
  const int cur0 = cur, prev0 = prev;
  for (auto &g : c->graphs)
    if (g.k == k && g.phase == phase && g.first == first && g.cur == cur && g.prev == prev) {
      g.used = ++c->graph_clock;
      *out = g.exec;
      return LBM_OK;
    }
  if (!c->cap_stream)
    HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal),
          "begin capture");
  hipError_t e = hipSuccess;
  for (int64_t m = s; m < s + k && e == hipSuccess;) {
    const int64_t q = segment_limit(c, m, s + k - m);
    e = enqueue_segment(c, m, q, cur, prev, c->cap_stream, nullptr);
    m += q;
  }
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(c, e, "capture launch");
  }
  if (e2 != hipSuccess) return hip_fail(c, e2, "end capture");
  hipGraphExec_t ge = nullptr;
  e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(c, e, "graph instantiate");
  }
  if (c->graphs.size() >= kMaxGraphs) {
    auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                [](const lbm_ctx::GraphEntry &a, const lbm_ctx::GraphEntry &b) {
                                  return a.used < b.used;
                                });
    (void)hipGraphExecDestroy(lru->exec);
    (void)hipGraphDestroy(lru->graph);
    c->graphs.erase(lru);
  }
  lbm_ctx::GraphEntry ent;
  ent.k = k;
  ent.phase = phase;
  ent.first = first;
  ent.cur = cur0;
  ent.prev = prev0;
  ent.graph = g;
  ent.exec = ge;
  ent.used = ++c->graph_clock;
  c->graphs.push_back(ent);
  *out = ge;
  return LBM_OK;
}

// Synchronization steps among [s, s + n).
int64_t syncs_in(const lbm_ctx *c, int64_t s, int64_t n) {
  if (c->sync_every <= 0 || n <= 0) return 0;
  const int64_t l = c->sync_every;
  return (s + n) / l - s / l;
}

lbm_status check_flag(lbm_ctx *c, bool wait) {
  if (c->nonfinite) return fail(c, LBM_E_NONFINITE, "non-finite or blown-up displacement");
  if (c->flag_pending) {
    hipError_t q = wait ? hipEventSynchronize(c->flag_ev) : hipEventQuery(c->flag_ev);
    if (q == hipSuccess) {
      c->flag_pending = false;
      if (*c->h_flag) c->nonfinite = true;
    } else if (q != hipErrorNotReady) {
      return hip_fail(c, q, "flag event");
    }
  }
  if (c->nonfinite) return fail(c, LBM_E_NONFINITE, "non-finite or blown-up displacement");
  return LBM_OK;
}

// 16-bit storage scale of one field for fields of magnitude about m: a
// power of two that puts m near 2^12 (the deviation moments are a small
// fraction of the fields, far from the FP16 limit of 65504; BF16 has FP32's
// exponent range), 2^14 when m is 0.
void set_scale(PlateDev &d, int fl, double m) {
  const int e = m > 0 ? 12 - (int)std::ceil(std::log2(m)) : 14;
  const int ec = std::max(-100, std::min(100, e));
  d.scale[fl] = std::ldexp(1.0f, ec);
  d.iscale[fl] = std::ldexp(1.0f, -ec);
}

// Rough magnitude of the strains the boundary data of plate p impose: a
// Neumann force F on a cell of side dh is a traction of about |F|/dh, a
// strain of about |F|/((lambda + 2 mu) dh); a prescribed displacement u*
// next to nodes at rest is a gradient of about |u*|/dh (each times the
// largest amplitude of its load table).
double load_magnitude(const lbm_ctx *c, int p) {
  const PlateHost &h = c->ph[(size_t)p];
  const PlateDev &d = c->pd[(size_t)p];
  double m = 0;
  for (int64_t b = h.b0; b < h.b1; b++) {
    const BndNode &B = c->bnd[(size_t)b];
    double g = 1.0;
    if (B.load >= 0) {
      const LoadTable &L = c->loads[(size_t)B.load];
      g = 0;
      for (int k = 0; k < L.n; k++) g = std::max(g, std::fabs(L.g[k]));
    }
    const double v = g * std::max(std::fabs(B.val[0]), std::fabs(B.val[1]));
    m = std::max(m, B.kind == LBM_BC_DIRICHLET ? v / d.dh : v / ((d.lam + 2.0 * d.mu) * d.dh));
  }
  return m;
}

lbm_status start(lbm_ctx *c) {
  if (c->started) return LBM_OK;
  // side stream and events of overlapped pairs (default priority)
  if (!c->side) {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "side stream");
    for (int i = 0; i < 2; i++) {
      HIP_TRY(c, hipEventCreateWithFlags(&c->ev_f[i], hipEventDisableTiming), "pair event");
      HIP_TRY(c, hipEventCreateWithFlags(&c->ev_d[i], hipEventDisableTiming), "pair event");
    }
  }
  if (c->bnd_dirty) {
    lbm_status st = upload_boundary(c);
    if (st) return st;
  }
  if (c->storage == LBM_STORE_F16DEV || c->storage == LBM_STORE_BF16DEV) {
    // 16-bit scale from the initial fields and the boundary data: a plate
    // that starts at rest is driven to strains its loads set.  The stored
    // deviation moments are all 0 before the first step (f = f_eq), so the
    // scale can change here without re-encoding.
    bool changed = false;
    for (size_t p = 0; p < c->pd.size(); p++) {
      const double ml = load_magnitude(c, (int)p);
      for (int fl = 0; fl < 2; fl++) {
        const float before = c->pd[p].scale[fl];
        set_scale(c->pd[p], fl, std::max(c->ph[p].field_mag[fl], ml));
        changed |= c->pd[p].scale[fl] != before;
      }
    }
    if (changed)
      HIP_TRY(c, hipMemcpy(c->d_plates, c->pd.data(), c->pd.size() * sizeof(PlateDev),
                           hipMemcpyHostToDevice),
              "plate upload");
  }
  // boundary accelerations of step 0: u(t_1) of the boundary nodes, into
  // both buffers the first step may write
  HIP_TRY(c, launch_boundary(c->storage, c->ds, c->d_chunks, (int)c->chunks.size(), c->d_unodes,
                             c->d_gnodes, c->d_btasks, c->d_stasks, c->cur, c->prev, c->cur ^ 1,
                             have_third(c) ? 2 : -1, 0, 0, c->stream),
          "first boundary step");
  c->started = true;
  return LBM_OK;
}

// Rough magnitude of the initial fields for the 16-bit scale.
double field_magnitude(const lbm_plate &p, const PlateHost &h, int fl) {
  const double *given = fl == 0 ? p.e0 : p.w0;
  const int nx = p.nx, ny = p.ny;
  double m = 0;
  if (given) {
    for (size_t k = 0; k < (size_t)nx * ny; k++)
      if (h.cls[k] & CL_IN) m = std::max(m, std::fabs(given[k]));
    return m;
  }
  if (!p.u0) return 0.0;
  const size_t N = (size_t)nx * ny;
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      const size_t k = (size_t)j * nx + i;
      if (!(h.cls[k] & CL_IN)) continue;
      double g = 0;
      for (int comp = 0; comp < 2; comp++) {
        const double *u = p.u0 + comp * N;
        if (i + 1 < nx && (h.cls[k + 1] & CL_IN)) g += std::fabs(u[k + 1] - u[k]);
        if (j + 1 < ny && (h.cls[k + nx] & CL_IN)) g += std::fabs(u[k + nx] - u[k]);
      }
      m = std::max(m, 2 * g / p.dh);
    }
  return m;
}

}  // namespace

extern "C" {

lbm_status lbm_copy_rate(size_t bytes, int32_t reps, double *gbs) {
  if (!gbs || bytes < 16 || reps < 1) return fail(nullptr, LBM_E_INVAL, "bad copy-rate arguments");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, LBM_E_DEVICE, "no HIP device available");
  const hipError_t e = copy_rate(bytes, reps, gbs);
  if (e != hipSuccess) return hip_fail(nullptr, e, "copy probe");
  return LBM_OK;
}

lbm_status lbm_layout_copy_rate(int32_t storage, int64_t nodes, int32_t reps, double *gbs) {
  if (!gbs || storage < LBM_STORE_F64 || storage > LBM_STORE_BF16DEV || nodes < 1 ||
      nodes > ((int64_t)1 << 32) || reps < 1)
    return fail(nullptr, LBM_E_INVAL, "bad layout-copy arguments");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return fail(nullptr, LBM_E_DEVICE, "no HIP device available");
  const hipError_t e = layout_copy_rate(storage, nodes, reps, gbs);
  if (e != hipSuccess) return hip_fail(nullptr, e, "layout copy probe");
  return LBM_OK;
}

const char *lbm_version(void) { return "paper_2301_00228_amd lbm 0.1 (gfx950)"; }

const char *lbm_last_error(const lbm_ctx *c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  for (int i = 0; i < 2; i++) {
    if (c->ev_f[i]) (void)hipEventDestroy(c->ev_f[i]);
    if (c->ev_d[i]) (void)hipEventDestroy(c->ev_d[i]);
  }

  if (c->flag_ev) (void)hipEventDestroy(c->flag_ev);
  if (c->h_flag) (void)hipHostFree(c->h_flag);
  dev_free_all(c);
  delete c;
}

lbm_status lbm_create(const lbm_plate *plates, int32_t n_plates, lbm_storage storage,
                      void *hip_stream, const lbm_alloc *alloc, lbm_ctx **out) {
  if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
  *out = nullptr;
  if (!plates || n_plates <= 0) return fail(nullptr, LBM_E_INVAL, "no plates");
  if ((int)storage < LBM_STORE_F64 || (int)storage > LBM_STORE_BF16DEV)
    return fail(nullptr, LBM_E_INVAL, "unknown storage");
  if (alloc && (!alloc->alloc || !alloc->free))
    return fail(nullptr, LBM_E_INVAL, "allocator needs alloc and free");

  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(nullptr, LBM_E_NOMEM, "context allocation failed");
  c->storage = (int)storage;
  c->stream = (hipStream_t)hip_stream;
  if (alloc) {
    c->have_alloc = true;
    c->alloc = *alloc;
  }
  c->ph.resize(n_plates);
  c->pd.resize(n_plates);
  c->sync_every = plates[0].sync_every;
  int64_t off = 0;
  // ---- host-side validation and preprocessing (no HIP call yet)
  for (int p = 0; p < n_plates; p++) {
    const lbm_plate &pl = plates[p];
    if (pl.nx < 3 || pl.ny < 3 || pl.nx > (1 << 20) || pl.ny > (1 << 20) || pl.sync_every < 0) {
      delete c;
      return fail(nullptr, LBM_E_INVAL, "plate " + std::to_string(p) + ": bad size or sync_every");
    }
    if (pl.sync_every != c->sync_every) {
      delete c;
      return fail(nullptr, LBM_E_INVAL, "all plates must share sync_every");
    }
    lbm_status st = plate_params(pl, c->pd[p]);
    if (st != LBM_OK) {
      delete c;
      return fail(nullptr, st,
                  st == LBM_E_UNSTABLE_DT
                      ? "plate " + std::to_string(p) + ": dt gives a0_phi < 0 (dt > dh/(sqrt(2) c_d))"
                      : "plate " + std::to_string(p) + ": bad material or lattice parameters");
    }
    if (pl.readings != 0) c->variant_readings = true;
    PlateHost &h = c->ph[p];
    h.nx = pl.nx;
    h.ny = pl.ny;
    h.px = pl.periodic_x != 0;
    h.py = pl.periodic_y != 0;
    h.pitch = (pl.nx + 63) / 64 * 64;
    h.off = off;
    std::string why;
    if (!classify(pl, h, why)) {
      delete c;
      return fail(nullptr, LBM_E_INVAL, "plate " + std::to_string(p) + ": " + why);
    }
    off += (int64_t)h.pitch * pl.ny;
    off = (off + 255) / 256 * 256;
    c->n_body += h.body;
    PlateDev &d = c->pd[p];
    d.off = h.off;
    d.nx = h.nx;
    d.ny = h.ny;
    d.pitch = h.pitch;
    d.periodic = (h.px ? 1 : 0) | (h.py ? 2 : 0);
    for (int fl = 0; fl < 2; fl++) {
      h.field_mag[fl] = field_magnitude(pl, h, fl);
      set_scale(d, fl, h.field_mag[fl]);
    }
    // boundary and second-row lists (row-major order)
    h.b0 = (int64_t)c->bnd.size();
    for (int j = 0; j < h.ny; j++)
      for (int i = 0; i < h.nx; i++) {
        const uint8_t cl = h.cls[(size_t)j * h.nx + i];
        const int64_t node = h.off + (int64_t)j * h.pitch + i;
        if (cl & CL_B) {
          BndNode b{};
          b.node = node;
          b.plate = p;
          b.i = i;
          b.j = j;
          b.kind = LBM_BC_NEUMANN;
          b.load = -1;
          const int E = (cl & NB_E) ? 1 : 0, N = (cl & NB_N) ? 1 : 0, W = (cl & NB_W) ? 1 : 0,
                    S = (cl & NB_S) ? 1 : 0;
          const double wx = 0.5 * pl.dh * (W + E);
          const double wy = 0.5 * pl.dh * (S + N);
          b.cell[0] = wx * wy;
          b.cell[1] = E ? wy : 0.0;
          b.cell[2] = N ? wx : 0.0;
          b.cell[3] = W ? wy : 0.0;
          b.cell[4] = S ? wx : 0.0;
          c->bnd.push_back(b);
        } else if (cl & CL_S) {
          SecNode s{};
          s.node = node;
          s.plate = p;
          s.i = i;
          s.j = j;
          c->sec.push_back(s);
        }
      }
    h.b1 = (int64_t)c->bnd.size();
  }
  c->n_alloc = off;
  if (c->bnd.size() + c->sec.size() > (size_t)0x3fffffff) {
    delete c;
    return fail(nullptr, LBM_E_INVAL, "too many boundary nodes");
  }
  {
    std::string why;
    if (!build_boundary_tables(c, why)) {
      delete c;
      return fail(nullptr, LBM_E_INVAL, why);
    }
  }

  // ---- device
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    delete c;
    return fail(nullptr, LBM_E_DEVICE, "no HIP device available");
  }
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, LBM_E_DEVICE, "hipGetDevice failed");
  }
  {
    // the staging area of lbm_fields_noalloc, looked up once per device
    // with the device current; a failure only disables that entry point
    void *p = nullptr;
    c->na_err = noalloc_staging(c->device, &p);
    c->na_stage = static_cast<double *>(p);
  }
  auto bail = [&](lbm_status st, const std::string &m) {
    g_create_error = m;
    lbm_destroy(c);
    return st;
  };
  const int64_t N = c->n_alloc;
  const int nsl = slot_count(c->storage);
  // buffers 0 and 1; buffer 2 (two-step pairs) is allocated on first use
  for (int b = 0; b < 2; b++)
    for (int fl = 0; fl < 2; fl++)
      for (int sl = 0; sl < 5; sl++) {
        if (sl >= nsl) {
          c->ds.pop[b][fl][sl] = nullptr;
          continue;
        }
        void *p = dev_alloc(c, (size_t)N * slot_bytes(c->storage));
        if (!p) return bail(LBM_E_NOMEM, "population allocation failed");
        if (hipMemset(p, 0, (size_t)N * slot_bytes(c->storage)) != hipSuccess)
          return bail(LBM_E_DEVICE, "memset");
        c->ds.pop[b][fl][sl] = p;
      }
  {
    // second-row side buffers and the node -> second-row index map
    const int64_t ns = (int64_t)c->sec.size();
    const size_t cb = c->storage == LBM_STORE_F64 ? sizeof(double) : sizeof(float);
    c->ds.nsec = ns;
    for (int b = 0; b < 2; b++) {
      c->ds.side[b] = dev_alloc(c, (size_t)std::max<int64_t>(1, ns) * 10 * cb);
      if (!c->ds.side[b]) return bail(LBM_E_NOMEM, "side buffer allocation failed");
    }
    std::vector<int32_t> sidx((size_t)N, -1);
    for (int64_t q = 0; q < ns; q++) sidx[(size_t)c->sec[(size_t)q].node] = (int32_t)q;
    int32_t *d = (int32_t *)dev_alloc(c, (size_t)N * sizeof(int32_t));
    if (!d) return bail(LBM_E_NOMEM, "second-row index allocation failed");
    if (hipMemcpy(d, sidx.data(), (size_t)N * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
      return bail(LBM_E_DEVICE, "second-row index upload");
    c->ds.sidx = d;
  }
  for (int b = 0; b < 2; b++)
    for (int comp = 0; comp < 2; comp++) {
      c->ds.u[b][comp] = dev_alloc(c, (size_t)N * uv_bytes(c->storage));
      c->ds.v[b][comp] = dev_alloc(c, (size_t)N * uv_bytes(c->storage));
      if (!c->ds.u[b][comp] || !c->ds.v[b][comp]) return bail(LBM_E_NOMEM, "u/v allocation failed");
    }
  c->d_cls = (uint8_t *)dev_alloc(c, (size_t)N);
  c->d_plates = (PlateDev *)dev_alloc(c, c->pd.size() * sizeof(PlateDev));
  c->d_bnd = (BndNode *)dev_alloc(c, std::max<size_t>(1, c->bnd.size()) * sizeof(BndNode));
  c->d_sec = (SecNode *)dev_alloc(c, std::max<size_t>(1, c->sec.size()) * sizeof(SecNode));
  c->d_loads = (LoadTable *)dev_alloc(c, (size_t)n_plates * kMaxLoadsPerPlate * sizeof(LoadTable));
  c->d_counter = (unsigned long long *)dev_alloc(c, 256);
  c->d_flag = (int *)(((char *)c->d_counter) + 64);
  if (!c->d_cls || !c->d_plates || !c->d_bnd || !c->d_sec || !c->d_loads || !c->d_counter)
    return bail(LBM_E_NOMEM, "metadata allocation failed");
  c->ds.cls = c->d_cls;
  c->ds.plates = c->d_plates;
  c->ds.loads = c->d_loads;
  c->ds.bnd = c->d_bnd;
  c->ds.sec = c->d_sec;
  c->ds.counter = c->d_counter;
  c->ds.flag = c->d_flag;

  hipError_t e;
  if ((e = hipMemset(c->d_counter, 0, 256)) != hipSuccess) return bail(LBM_E_DEVICE, "memset");
  if ((e = hipMemset(c->d_cls, 0, (size_t)N)) != hipSuccess) return bail(LBM_E_DEVICE, "memset");
  for (int b = 0; b < 2; b++)
    for (int comp = 0; comp < 2; comp++) {
      if (hipMemset(c->ds.u[b][comp], 0, (size_t)N * uv_bytes(c->storage)) != hipSuccess ||
          hipMemset(c->ds.v[b][comp], 0, (size_t)N * uv_bytes(c->storage)) != hipSuccess)
        return bail(LBM_E_DEVICE, "memset");
    }
  for (int p = 0; p < n_plates; p++) {
    const PlateHost &h = c->ph[p];
    if (hipMemcpy2D(c->d_cls + h.off, (size_t)h.pitch, h.cls.data(), (size_t)h.nx, (size_t)h.nx,
                    (size_t)h.ny, hipMemcpyHostToDevice) != hipSuccess)
      return bail(LBM_E_DEVICE, "class upload");
  }
  if (hipMemcpy(c->d_plates, c->pd.data(), c->pd.size() * sizeof(PlateDev),
                hipMemcpyHostToDevice) != hipSuccess)
    return bail(LBM_E_DEVICE, "plate upload");
  if (!c->sec.empty() && hipMemcpy(c->d_sec, c->sec.data(), c->sec.size() * sizeof(SecNode),
                                   hipMemcpyHostToDevice) != hipSuccess)
    return bail(LBM_E_DEVICE, "second-row upload");
  c->d_chunks = (Chunk *)dev_alloc(c, std::max<size_t>(1, c->chunks.size()) * sizeof(Chunk));
  c->d_unodes = (UNode *)dev_alloc(c, std::max<size_t>(1, c->unodes.size()) * sizeof(UNode));
  c->d_gnodes = (GradNode *)dev_alloc(c, std::max<size_t>(1, c->gnodes.size()) * sizeof(GradNode));
  c->d_btasks = (BTask *)dev_alloc(c, std::max<size_t>(1, c->btasks.size()) * sizeof(BTask));
  c->d_stasks = (STask *)dev_alloc(c, std::max<size_t>(1, c->stasks.size()) * sizeof(STask));
  if (!c->d_chunks || !c->d_unodes || !c->d_gnodes || !c->d_btasks || !c->d_stasks)
    return bail(LBM_E_NOMEM, "boundary table allocation failed");
  {
    hipError_t e1 = hipSuccess;
    if (!c->chunks.empty())
      e1 = hipMemcpy(c->d_chunks, c->chunks.data(), c->chunks.size() * sizeof(Chunk),
                     hipMemcpyHostToDevice);
    if (e1 == hipSuccess && !c->unodes.empty())
      e1 = hipMemcpy(c->d_unodes, c->unodes.data(), c->unodes.size() * sizeof(UNode),
                     hipMemcpyHostToDevice);
    if (e1 == hipSuccess && !c->gnodes.empty())
      e1 = hipMemcpy(c->d_gnodes, c->gnodes.data(), c->gnodes.size() * sizeof(GradNode),
                     hipMemcpyHostToDevice);
    if (e1 == hipSuccess && !c->btasks.empty())
      e1 = hipMemcpy(c->d_btasks, c->btasks.data(), c->btasks.size() * sizeof(BTask),
                     hipMemcpyHostToDevice);
    if (e1 == hipSuccess && !c->stasks.empty())
      e1 = hipMemcpy(c->d_stasks, c->stasks.data(), c->stasks.size() * sizeof(STask),
                     hipMemcpyHostToDevice);
    if (e1 != hipSuccess) return bail(LBM_E_DEVICE, "boundary table upload");
  }

  // initial state, plate by plate, through a temporary dense staging buffer
  size_t maxn = 0;
  for (auto &h : c->ph) maxn = std::max(maxn, (size_t)h.nx * h.ny);
  double *stage = nullptr;
  if (hipMalloc(&stage, maxn * 6 * sizeof(double)) != hipSuccess)
    return bail(LBM_E_NOMEM, "staging allocation failed");
  for (int p = 0; p < n_plates && e == hipSuccess; p++) {
    const lbm_plate &pl = plates[p];
    const size_t n = (size_t)pl.nx * pl.ny;
    double *du = stage, *dv = stage + 2 * n, *de = stage + 4 * n, *dw = stage + 5 * n;
    if (pl.u0) e = hipMemcpy(du, pl.u0, 2 * n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && pl.v0) e = hipMemcpy(dv, pl.v0, 2 * n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && pl.e0) e = hipMemcpy(de, pl.e0, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && pl.w0) e = hipMemcpy(dw, pl.w0, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = launch_init(c->storage, c->ds, p, (int64_t)n, pl.u0 ? du : nullptr, pl.v0 ? dv : nullptr,
                      pl.e0 ? de : nullptr, pl.w0 ? dw : nullptr, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  (void)hipFree(stage);
  if (e != hipSuccess) return bail(LBM_E_DEVICE, std::string("initial state: ") + hipGetErrorString(e));

  // default tiling (what the autotuner picks on 1024^2 plates unaligned and
  // on 4096^2 plates aligned); every context starts from it, whatever ran
  // before in the process, so that timings do not depend on history
  c->lanes = 128;
  c->rows = 8;
  c->edge_rows = 2;
  c->align = c->n_body < ((int64_t)4 << 20) ? 0 : 16;
  build_tiles(c);
  build_tile_tables(c);
  if (upload_tiles(c) != LBM_OK || upload_tile_tables(c) != LBM_OK)
    return bail(LBM_E_NOMEM, c->err);
  if (hipHostMalloc((void **)&c->h_flag, sizeof(int), hipHostMallocDefault) != hipSuccess)
    return bail(LBM_E_NOMEM, "pinned flag allocation failed");
  *c->h_flag = 0;
  if (hipEventCreateWithFlags(&c->flag_ev, hipEventDisableTiming) != hipSuccess)
    return bail(LBM_E_DEVICE, "event creation failed");
  if (hipDeviceSynchronize() != hipSuccess) return bail(LBM_E_DEVICE, "synchronize");
  *out = c;
  return LBM_OK;
}

lbm_status lbm_set_bc(lbm_ctx *c, int32_t plate, int32_t n, const int32_t *xy, const uint8_t *kind,
                      const double *val, const double *cell, int32_t n_knots,
                      const double *knots) {
  if (!c) return LBM_E_INVAL;
  if (c->started) return fail(c, LBM_E_STATE, "lbm_set_bc after the first step");
  if (plate < 0 || plate >= (int)c->ph.size()) return fail(c, LBM_E_INVAL, "bad plate index");
  if (n < 0 || (n > 0 && (!xy || !kind || !val))) return fail(c, LBM_E_INVAL, "bad node arrays");
  if (n_knots < 0 || n_knots > kMaxKnots || (n_knots > 0 && !knots))
    return fail(c, LBM_E_INVAL, "bad knot table");
  for (int m = 1; m < n_knots; m++)
    if (!(knots[2 * m] > knots[2 * m - 2])) return fail(c, LBM_E_INVAL, "knot times must increase");
  PlateHost &h = c->ph[plate];
  std::vector<int64_t> idx((size_t)n);
  for (int m = 0; m < n; m++) {
    const int i = xy[2 * m], j = xy[2 * m + 1];
    if (i < 0 || i >= h.nx || j < 0 || j >= h.ny)
      return fail(c, LBM_E_INVAL, "node outside the plate");
    if (!(h.cls[(size_t)j * h.nx + i] & CL_B))
      return fail(c, LBM_E_INVAL, "node (" + std::to_string(i) + ", " + std::to_string(j) +
                                      ") is not a boundary node");
    if (kind[m] > 1) return fail(c, LBM_E_INVAL, "bad boundary kind");
    if (!std::isfinite(val[2 * m]) || !std::isfinite(val[2 * m + 1]))
      return fail(c, LBM_E_INVAL, "non-finite boundary value");
    if (cell && !(cell[5 * m] > 0 && std::isfinite(cell[5 * m])))
      return fail(c, LBM_E_INVAL, "cell volume must be positive");
    if (cell)
      for (int q = 1; q < 5; q++)
        if (!(cell[5 * m + q] >= 0 && std::isfinite(cell[5 * m + q])))
          return fail(c, LBM_E_INVAL, "cell side lengths must be finite and >= 0");
    const int64_t node = h.off + (int64_t)j * h.pitch + i;
    auto first = c->bnd.begin() + h.b0, last = c->bnd.begin() + h.b1;
    auto it = std::lower_bound(first, last, node,
                               [](const BndNode &b, int64_t v) { return b.node < v; });
    idx[m] = it - c->bnd.begin();
  }
  int load = -1;
  if (n_knots > 0) {
    if (h.nloads >= kMaxLoadsPerPlate) return fail(c, LBM_E_INVAL, "too many load tables");
    LoadTable L{};
    L.n = n_knots;
    for (int m = 0; m < n_knots; m++) {
      L.t[m] = knots[2 * m];
      L.g[m] = knots[2 * m + 1];
    }
    load = (int)c->loads.size();
    c->loads.push_back(L);
    h.nloads++;
  }
  for (int m = 0; m < n; m++) {
    BndNode &b = c->bnd[(size_t)idx[m]];
    b.kind = kind[m];
    b.val[0] = val[2 * m];
    b.val[1] = val[2 * m + 1];
    b.load = load;
    if (cell)
      for (int q = 0; q < 5; q++) b.cell[q] = cell[5 * m + q];
  }
  c->bnd_dirty = true;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t n) {
  if (!c || n < 0) return LBM_E_INVAL;
  lbm_status st = check_flag(c, false);
  if (st) return st;
  st = start(c);
  if (st) return st;
  while (n > 0) {
    if (c->use_graphs) {
      const int64_t k = graph_chunk(c, c->step, n);
      hipGraphExec_t ge = nullptr;
      st = graph_for(c, c->step, k, c->cur, c->prev, &ge);
      if (st) return st;
      HIP_TRY(c, hipGraphLaunch(ge, c->stream), "graph launch");
      advance_buffers(c, c->step, k, c->cur, c->prev);
      c->syncs_done += syncs_in(c, c->step, k);
      c->steps_in_graphs += k;
      c->step += k;
      n -= k;
      continue;
    }
    const int64_t k = segment_limit(c, c->step, n);
    HIP_TRY(c, enqueue_segment(c, c->step, k, c->cur, c->prev, c->stream, nullptr),
            "step launch");
    c->syncs_done += syncs_in(c, c->step, k);
    c->step += k;
    n -= k;
  }
  HIP_TRY(c, hipMemcpyAsync(c->h_flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream),
          "flag copy");
  HIP_TRY(c, hipEventRecord(c->flag_ev, c->stream), "flag event");
  c->flag_pending = true;
  return LBM_OK;
}

lbm_status lbm_prepare_steps(lbm_ctx *c, int64_t n) {
  if (!c || n < 0) return LBM_E_INVAL;
  lbm_status st = check_flag(c, false);
  if (st) return st;
  if (!c->use_graphs) return LBM_OK;
  st = start(c);
  if (st) return st;
  int64_t s = c->step;
  int cur = c->cur, prev = c->prev;
  while (n > 0) {
    const int64_t k = graph_chunk(c, s, n);
    hipGraphExec_t ge = nullptr;
    st = graph_for(c, s, k, cur, prev, &ge);
    if (st) return st;
    advance_buffers(c, s, k, cur, prev);
    s += k;
    n -= k;
  }
  return LBM_OK;
}

lbm_status lbm_fields_device(lbm_ctx *c, int32_t plate, double *e, double *w, double *u,
                             double *v) {
  if (!c) return LBM_E_INVAL;
  if (plate < 0 || plate >= (int)c->ph.size()) return fail(c, LBM_E_INVAL, "bad plate index");
  const PlateHost &h = c->ph[plate];
  HIP_TRY(c, launch_fields(c->storage, c->ds, plate, (int64_t)h.nx * h.ny, c->cur, e,
                           w, u, v, c->stream),
          "field kernel");
  return LBM_OK;
}

lbm_status lbm_fields(lbm_ctx *c, int32_t plate, double *e, double *w, double *u, double *v) {
  if (!c) return LBM_E_INVAL;
  if (plate < 0 || plate >= (int)c->ph.size()) return fail(c, LBM_E_INVAL, "bad plate index");
  const PlateHost &h = c->ph[plate];
  const size_t n = (size_t)h.nx * h.ny;
  const size_t need = 6 * n * sizeof(double);
  if (need > c->scratch_bytes) {
    double *p = (double *)dev_alloc(c, need);
    if (!p) return fail(c, LBM_E_NOMEM, "field scratch allocation failed");
    // (every earlier use of the old scratch ended with a stream synchronize)
    if (c->d_scratch) dev_free(c, c->d_scratch);
    c->d_scratch = p;
    c->scratch_bytes = need;
  }
  double *de = c->d_scratch, *dw = de + n, *du = dw + n, *dv = du + 2 * n;
  lbm_status st = lbm_fields_device(c, plate, e ? de : nullptr, w ? dw : nullptr,
                                    u ? du : nullptr, v ? dv : nullptr);
  if (st) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  if (e) HIP_TRY(c, hipMemcpy(e, de, n * sizeof(double), hipMemcpyDeviceToHost), "copy e");
  if (w) HIP_TRY(c, hipMemcpy(w, dw, n * sizeof(double), hipMemcpyDeviceToHost), "copy omega");
  if (u) HIP_TRY(c, hipMemcpy(u, du, 2 * n * sizeof(double), hipMemcpyDeviceToHost), "copy u");
  if (v) HIP_TRY(c, hipMemcpy(v, dv, 2 * n * sizeof(double), hipMemcpyDeviceToHost), "copy v");
  int flag = 0;
  HIP_TRY(c, hipMemcpy(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost), "copy flag");
  if (flag) c->nonfinite = true;
  return check_flag(c, true);
}

lbm_status lbm_fields_noalloc(lbm_ctx *c, int32_t plate, double *e, double *w, double *u,
                              double *v) {
  if (!c) return LBM_E_INVAL;
  if (plate < 0 || plate >= (int)c->ph.size()) return fail(c, LBM_E_INVAL, "bad plate index");
  if (!c->na_stage)
    return fail(c, LBM_E_DEVICE, std::string("fixed staging area unavailable: ") +
                                     hipGetErrorString(c->na_err));
  const PlateHost &h = c->ph[plate];
  const size_t n = (size_t)h.nx * h.ny;
  const size_t need = ((e ? n : 0) + (w ? n : 0) + (u ? 2 * n : 0) + (v ? 2 * n : 0)) * sizeof(double);
  if (need > kNoAllocBytes)
    return fail(c, LBM_E_INVAL,
                "lbm_fields_noalloc: the requested fields of plate " + std::to_string(plate) +
                    " need " + std::to_string(need) + " bytes of staging; the fixed area holds " +
                    std::to_string(kNoAllocBytes));
  double *q = c->na_stage;
  double *de = e ? q : nullptr;
  q += e ? n : 0;
  double *dw = w ? q : nullptr;
  q += w ? n : 0;
  double *du = u ? q : nullptr;
  q += u ? 2 * n : 0;
  double *dv = v ? q : nullptr;
  // every element of the requested outputs is written by the field kernel
  // (0 outside the body), so nothing left by an earlier call is read
  lbm_status st = lbm_fields_device(c, plate, de, dw, du, dv);
  if (st) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  if (e) HIP_TRY(c, hipMemcpy(e, de, n * sizeof(double), hipMemcpyDeviceToHost), "copy e");
  if (w) HIP_TRY(c, hipMemcpy(w, dw, n * sizeof(double), hipMemcpyDeviceToHost), "copy omega");
  if (u) HIP_TRY(c, hipMemcpy(u, du, 2 * n * sizeof(double), hipMemcpyDeviceToHost), "copy u");
  if (v) HIP_TRY(c, hipMemcpy(v, dv, 2 * n * sizeof(double), hipMemcpyDeviceToHost), "copy v");
  int flag = 0;
  HIP_TRY(c, hipMemcpy(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost), "copy flag");
  if (flag) c->nonfinite = true;
  return check_flag(c, true);
}

lbm_status lbm_consistency_error(lbm_ctx *c, int32_t plate, double *err) {
  if (!c || !err) return LBM_E_INVAL;
  if (plate < 0 || plate >= (int)c->ph.size()) return fail(c, LBM_E_INVAL, "bad plate index");
  const PlateHost &h = c->ph[plate];
  const size_t n = (size_t)h.nx * h.ny;
  const size_t need = n * sizeof(double);
  if (need > c->scratch_bytes) {
    double *p = (double *)dev_alloc(c, need);
    if (!p) return fail(c, LBM_E_NOMEM, "field scratch allocation failed");
    // (every earlier use of the old scratch ended with a stream synchronize)
    if (c->d_scratch) dev_free(c, c->d_scratch);
    c->d_scratch = p;
    c->scratch_bytes = need;
  }
  HIP_TRY(c, launch_cons_err(c->storage, c->ds, plate, (int64_t)n, c->cur, c->d_scratch, c->stream),
          "consistency error kernel");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  HIP_TRY(c, hipMemcpy(err, c->d_scratch, need, hipMemcpyDeviceToHost), "copy error");
  return check_flag(c, true);
}

lbm_status lbm_info(const lbm_ctx *c, lbm_info_t *info) {
  if (!c || !info) return LBM_E_INVAL;
  std::memset(info, 0, sizeof *info);
  info->nodes_in_body = c->n_body;
  info->nodes_allocated = c->n_alloc;
  info->boundary_nodes = (int64_t)c->bnd.size();
  info->second_row_nodes = (int64_t)c->sec.size();
  info->nodes_two_step = c->n_two;
  info->steps_done = c->step;
  info->device_bytes = c->device_bytes;
  info->bytes_per_update = bytes_per_update(c->storage);
  info->n_plates = (int32_t)c->ph.size();
  info->storage = c->storage;
  info->tile_lanes = c->lanes;
  info->tile_rows = c->rows;
  info->tile_order = c->order;
  info->tile_stream_stores = c->nt;
  info->tile_edge_rows = (c->edge_rows > 0 && c->edge_rows < c->rows) ? c->edge_rows : c->rows;
  info->tile_align = c->align;
  info->tile_steps = c->two ? 2 : 1;
  info->n_tiles = (int32_t)c->ltiles.size();
  info->tile_edge_cols = c->edge_cols;
  info->nodes_deep = c->two ? c->n_deep : 0;
  info->overlap = (c->two && c->overlap) ? 1 : 0;
  info->steps_in_graphs = c->steps_in_graphs;
  info->syncs_done = c->syncs_done;
  info->graphs_cached = (int32_t)c->graphs.size();
  return LBM_OK;
}

lbm_status lbm_set_tiling(lbm_ctx *c, const lbm_tiling *t) {
  if (!c || !t) return LBM_E_INVAL;
  const int32_t lanes = t->lanes, rows = t->rows, order = t->order, edge_rows = t->edge_rows,
                align = t->align, steps = t->steps, edge_cols = t->edge_cols,
                stream = t->stream_stores;
  if ((lanes != 64 && lanes != 128 && lanes != 256) || rows < 1 || rows > 65536 || order < 0 ||
      order > 3 || edge_rows < 0 || align < 0 || align > 4096 || steps < 0 || steps > 2 ||
      edge_cols < 0 || edge_cols > lanes - 4 || stream < 0 || stream > 1)
    return fail(c, LBM_E_INVAL,
                "lanes must be 64, 128 or 256, rows >= 1, order 0..3, edge_rows >= 0, "
                "align 0..4096, steps 0..2, edge_cols 0..lanes-4, stream_stores 0..1");
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  c->lanes = lanes;
  c->rows = rows;
  c->order = order;
  c->edge_rows = edge_rows;
  c->edge_cols = edge_cols;
  c->align = align;
  c->nt = stream;
  c->two = steps == 2 ? 1 : 0;
  if (c->two) {
    lbm_status st3 = ensure_third(c);
    if (st3) {
      c->two = 0;
      return st3;
    }
  }
  build_tiles(c);
  build_tile_tables(c);
  lbm_status st = upload_tiles(c);
  if (st) return st;
  st = upload_tile_tables(c);
  if (st) return st;
  drop_graph(c);
  return LBM_OK;
}

lbm_status lbm_use_graphs(lbm_ctx *c, int32_t enable) {
  if (!c) return LBM_E_INVAL;
  c->use_graphs = enable != 0;
  return LBM_OK;
}

lbm_status lbm_use_overlap(lbm_ctx *c, int32_t enable) {
  if (!c) return LBM_E_INVAL;
  if (c->overlap == (enable != 0)) return LBM_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  c->overlap = enable != 0;
  // (the frame tiles are cut shorter with overlapped pairs)
  build_tiles(c);
  build_tile_tables(c);
  lbm_status st = upload_tiles(c);
  if (st) return st;
  st = upload_tile_tables(c);
  if (st) return st;
  drop_graph(c);
  return LBM_OK;
}

lbm_status lbm_profile(lbm_ctx *c, int64_t n, double *ms, int64_t *launches) {
  if (!c || n < 0 || !ms) return LBM_E_INVAL;
  lbm_status st = check_flag(c, false);
  if (st) return st;
  st = start(c);
  if (st) return st;
  // Launches on one stream go back to back; the time between the events
  // around a launch is its device time plus the gap to the previous
  // launch's end (on the side stream: to the end of what it waited for).
  LaunchRecorder rec;
  double acc[5] = {0, 0, 0, 0, 0};
  int64_t cnt[5] = {0, 0, 0, 0, 0};
  hipError_t e = hipSuccess;
  while (n > 0 && e == hipSuccess) {
    const int64_t k = segment_limit(c, c->step, n);
    e = enqueue_segment(c, c->step, k, c->cur, c->prev, c->stream, &rec);
    if (e == hipSuccess) {
      c->syncs_done += syncs_in(c, c->step, k);
      c->step += k;
      n -= k;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  for (size_t i = 0; e == hipSuccess && i < rec.recs.size(); i++) {
    float t = 0;
    (void)hipEventElapsedTime(&t, rec.recs[i].a, rec.recs[i].b);
    acc[rec.recs[i].kind] += t;
    cnt[rec.recs[i].kind] += 1;
  }
  for (auto &r : rec.recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  if (e != hipSuccess) return hip_fail(c, e, "profiled step");
  for (int k = 0; k < 5; k++) {
    ms[k] = acc[k];
    if (launches) launches[k] = cnt[k];
  }
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx *c, int32_t steps, double *best_ms) {
  if (!c || steps < 1) return LBM_E_INVAL;
  if (c->variant_readings)
    return fail(c, LBM_E_STATE,
                "lbm_autotune times the interior launches with their boundary prologues, which "
                "carry only the default readings (R1, M1)");
  lbm_status st = check_flag(c, false);
  if (st) return st;
  st = start(c);
  if (st) return st;
  // The timed launches are those of step n with their prologues (the
  // boundary work of step n - 1).  From a complete state at t_n the
  // single-step launch rewrites the boundary values of t_n and t_{n+1} with
  // the values they already hold and the t_{n+1} buffers from the t_n ones,
  // so repeating it leaves the state unchanged; so do the two launches of a
  // two-step pair, repeated, except that the second one writes the side
  // buffer the first one's prologue reads: the timed second launches write
  // a scratch buffer in its place.  That needs the boundary populations of t_{n-1} in a
  // buffer neither launch writes and a state of t_n that does not come from
  // a synchronization (nor n = 0): otherwise one real step is taken first.
  const bool syncs_now = c->sync_every > 0 && c->step % c->sync_every == 0;
  if (c->step == 0 || (syncs_now && c->sync_every > 1) || c->prev == 2) {
    HIP_TRY(c, enqueue_segment(c, c->step, 1, c->cur, c->prev, c->stream, nullptr),
            "step launch");
    c->syncs_done += syncs_in(c, c->step, 1);
    c->step += 1;
  }
  const bool with_prologue = !(c->sync_every > 0 && c->step % c->sync_every == 0);
  HIP_TRY(c, hipStreamSynchronize(c->stream), "synchronize");
  const int64_t n = c->step;
  const size_t side_bytes = (size_t)std::max<int64_t>(1, c->ds.nsec) * 10 *
                            (c->storage == LBM_STORE_F64 ? sizeof(double) : sizeof(float));
  void *side_scratch = dev_alloc(c, side_bytes);
  if (!side_scratch) return fail(c, LBM_E_NOMEM, "autotuner scratch allocation failed");
  // two-step candidates only if the third state buffer fits in memory
  const bool had_third = have_third(c);
  const int max_steps = ensure_third(c) == LBM_OK ? 2 : 1;
  // state of the timed second launches: all buffers as allocated by now,
  // side buffer n & 1 replaced by the scratch buffer
  DevState ds_b = c->ds;
  ds_b.side[n & 1] = side_scratch;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0), "event");
  HIP_TRY(c, hipEventCreate(&e1), "event");
  int reps = steps;  // timed repetitions per candidate
  // Time body(st, k), which enqueues k repetitions of the timed launches on
  // stream st: eagerly (`reps` repetitions to warm up, then `reps` timed on the
  // library stream) or captured in a graph of `reps` repetitions (launched
  // once to warm up and once timed), as lbm_step runs its steps.
  auto time_body = [&](auto &&body, bool graph) -> double {
    hipError_t e = hipSuccess;
    if (!graph) {
      // as many untimed repetitions first: each candidate's tile lists are
      // built on the host while the GPU idles, and its clocks ramp up again
      e = body(c->stream, reps);
      if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) e = body(c->stream, reps);
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
    } else {
      if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return 1e300;
      const hipError_t eb = body(c->cap_stream, reps);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(c->cap_stream, &g);
      if (eb != hipSuccess) e = eb;
      hipGraphExec_t ge = nullptr;
      if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (e == hipSuccess) e = hipGraphLaunch(ge, c->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) e = hipGraphLaunch(ge, c->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (ge) (void)hipGraphExecDestroy(ge);
      if (g) (void)hipGraphDestroy(g);
    }
    if (e != hipSuccess) return 1e300;
    float t = 0;
    (void)hipEventElapsedTime(&t, e0, e1);
    return t / reps;
  };
  const int cur = c->cur, prev = c->prev;
  // interior time per step of one tiling (1e300 if it cannot run), with
  // overlapped pairs if ov, timed eagerly or in a graph
  auto eval = [&](const lbm_tiling &T, bool ov, bool graph) -> double {
    c->lanes = T.lanes;
    c->rows = T.rows;
    c->order = T.order;
    c->edge_rows = T.edge_rows;
    c->edge_cols = T.edge_cols;
    c->align = T.align;
    c->nt = T.stream_stores;
    c->two = T.steps == 2 ? 1 : 0;
    c->overlap = ov;
    build_tiles(c);
    build_tile_tables(c);
    if (upload_tiles(c) != LBM_OK || upload_tile_tables(c) != LBM_OK) return 1e300;
    const Prologue pro = make_prologue(c, with_prologue);
    if (T.steps == 1) {
      const StepBufs sb{cur, cur ^ 1, prev, (int)(n & 1), -1};
      return time_body([&](hipStream_t st, int k) {
        hipError_t e = hipSuccess;
        for (int i = 0; i < k && e == hipSuccess; i++)
          e = launch_interior(c->storage, c->ds, c->d_tiles, (int)c->ltiles.size(), T.lanes, sb,
                              pro, st);
        return e;
      }, graph);
    }
    // (two-step launches use buffer 2, in both state copies)
    if (!have_third(c) || !ds_b.pop[2][0][0] || !ds_b.u[2][0]) return 1e300;
    const StepBufs b1{cur, 2, prev, (int)(n & 1), cur ^ 1, c->nt};
    const StepBufs b2{2, cur ^ 1, cur, (int)((n + 1) & 1), -1};
    const Prologue pro2 = make_prologue(c, true);
    if (ov && !c->dtiles.empty() && c->side) {
      // overlapped pairs as enqueue_segment runs them: the deep launch of a
      // pair waits for the previous pair's first launch and the next pair's
      // first launch for it
      return 0.5 * time_body([&](hipStream_t st, int k) {
        hipError_t e = hipEventRecord(c->ev_f[1], st);
        int par = 0;
        for (int i = 0; i < k && e == hipSuccess; i++) {
          if (i > 0) e = hipStreamWaitEvent(st, c->ev_d[par ^ 1], 0);
          if (e == hipSuccess)
            e = launch_interior(c->storage, c->ds, c->d_ftiles, (int)c->ftiles.size(), c->lanes,
                                b1, pro, st);
          if (e == hipSuccess) e = hipEventRecord(c->ev_f[par], st);
          if (e == hipSuccess)
            e = launch_interior(c->storage, ds_b, c->d_etiles, (int)c->etiles.size(), c->lanes,
                                b2, pro2, st);
          if (e == hipSuccess) e = hipStreamWaitEvent(c->side, c->ev_f[par ^ 1], 0);
          if (e == hipSuccess)
            e = launch_deep(c->storage, c->ds, c->d_dtiles, (int)c->dtiles.size(), c->lanes, b1,
                            c->side);
          if (e == hipSuccess) e = hipEventRecord(c->ev_d[par], c->side);
          par ^= 1;
        }
        if (e == hipSuccess) e = hipStreamWaitEvent(st, c->ev_d[par ^ 1], 0);
        return e;
      }, graph);
    }
    // one stream: the pair's two launches in turn, as enqueue_segment runs them
    return 0.5 * time_body([&](hipStream_t st, int k) {
      hipError_t e = hipSuccess;
      for (int i = 0; i < k && e == hipSuccess; i++) {
        e = launch_interior(c->storage, c->ds, c->d_tiles, (int)c->ltiles.size(), T.lanes, b1, pro,
                            st);
        if (e == hipSuccess)
          e = launch_interior(c->storage, ds_b, c->d_etiles, (int)c->etiles.size(), T.lanes, b2,
                              pro2, st);
      }
      return e;
    }, graph);
  };
  double best = 1e300;
  lbm_tiling bt{c->lanes, c->rows, c->order, c->edge_rows, c->align, c->two ? 2 : 1, c->edge_cols,
                c->nt};
  const bool ov_user = c->overlap;  // the search runs on one stream; the end may turn it on
  bool best_ov = false;
  std::vector<std::pair<double, lbm_tiling>> tried;  // every candidate and its time
  auto consider = [&](lbm_tiling T) {
    if (T.edge_rows >= T.rows) T.edge_rows = 0;
    const double per = eval(T, false, false);
    if (per < 1e299) tried.push_back({per, T});
    if (per < best) {
      best = per;
      bt = T;
    }
  };
  // Warm-up with the current tiling for at least 20 ms (the clocks ramp up
  // from idle; on small plates the whole search takes well under a second),
  // then at least 10 ms of launches per candidate (shorter timings differ by
  // a few per cent from run to run, which decided close calls).
  {
    lbm_tiling T0 = bt;
    if (T0.steps == 2 && max_steps < 2) T0.steps = 1;
    const double t0 = eval(T0, false, false);
    if (t0 < 1e299) {
      reps = std::max(steps, std::min(2000, (int)std::ceil(20.0 / (2.0 * t0))));
      (void)eval(T0, false, false);
      reps = std::max(steps, std::min(400, (int)std::ceil(10.0 / (2.0 * t0))));
    }
  }
  // Stage 1: steps per pass x lanes x rows, short tiles near boundaries,
  // strips aligned on large plates.
  const int a0 = c->n_body >= ((int64_t)4 << 20) ? 16 : 0;
  for (int S = max_steps; S >= 1; S--)
    for (int L : {64, 128, 256})
      for (int R : {8, 16, 32}) consider(lbm_tiling{L, R, 0, std::min(4, R / 2), a0, S, 0, 0});
  // Stage 2: one dimension at a time around the best.
  {
    const lbm_tiling b0 = bt;
    for (int E : {0, 2, 4, 8})
      if (E != b0.edge_rows) {
        lbm_tiling T = b0;
        T.edge_rows = E;
        consider(T);
      }
  }
  if (bt.steps == 2) {
    const lbm_tiling b0 = bt;
    for (int W : {0, 4, 8, 16})
      if (W != b0.edge_cols) {
        lbm_tiling T = b0;
        T.edge_cols = W;
        consider(T);
      }
  }
  {
    lbm_tiling T = bt;
    T.align = bt.align ? 0 : 16;
    consider(T);
  }
  {
    const lbm_tiling b0 = bt;
    for (int R : {b0.rows / 2, b0.rows * 2})
      if (R >= 4 && R <= 64) {
        lbm_tiling T = b0;
        T.rows = R;
        consider(T);
      }
  }
  {
    // band groups (order 3): tiles sharing halo rows run together
    lbm_tiling T = bt;
    T.order = 3;
    if (T.order != bt.order) consider(T);
  }
  if (c->ph.size() > 1) {
    const lbm_tiling b0 = bt;
    for (int O : {1, 2}) {
      lbm_tiling T = b0;
      T.order = O;
      consider(T);
    }
  }
  // Bytes of the two state buffers the steps alternate between (read and
  // written once per step): populations and u, du/dt per body node.
  const double state_bytes =
      (double)c->n_body * (c->storage == LBM_STORE_F64   ? 224.0
                           : c->storage == LBM_STORE_F32 ? 112.0
                           : c->storage == LBM_STORE_F32DEV ? 144.0
                                                            : 128.0);
  if (bt.steps == 2 && state_bytes > kInfinityCacheBytes) {
    // nontemporal stores of the two-step passes' final state: they leave the
    // L2 to the halo rows where the state streams through HBM (8-row tiles
    // of small plates), and lose where the state stays in the Infinity Cache.
    // Not tried there: the timed pairs restart from the same state, which
    // then stays in that cache whatever the stores do, while real steps read
    // back what the previous pair wrote (on the 1024^2 FP64 plate a tiling
    // with them timed 7 % faster here and ran 25 % slower).
    lbm_tiling T = bt;
    T.stream_stores = bt.stream_stores ? 0 : 1;
    consider(T);
  }
  {
    // rows and edge rows once more, with the packing order and stores now
    // chosen: on the 256-plate batch 16-row tiles with 8-row edge tiles win
    // only with band groups and nontemporal stores (+3 % over 8 / 4)
    const lbm_tiling b0 = bt;
    for (int R : {b0.rows / 2, b0.rows, b0.rows * 2})
      for (int E : {b0.edge_rows, R / 2})
        if (R >= 4 && R <= 64 && !(R == b0.rows && E == b0.edge_rows)) {
          lbm_tiling T = b0;
          T.rows = R;
          T.edge_rows = E;
          consider(T);
        }
  }
  // Final choice.  The search compared one eager timing per candidate; the
  // three fastest are timed again in captured graphs of at least 5 ms of
  // steps, as lbm_step runs them, on one stream and -- two-step tilings with
  // overlapped pairs allowed -- overlapped, with frame tiles of their own edge
  // rows, 2 and 4 rows.  The fastest one-stream timing wins unless an
  // overlapped one is at least 3 % faster than it (the timed pairs lack the
  // filling and draining of the overlap at each synchronization; eager
  // launches of overlapped pairs pay for more API calls).
  {
    auto same = [](const lbm_tiling &a, const lbm_tiling &b) {
      return a.lanes == b.lanes && a.rows == b.rows && a.order == b.order &&
             a.edge_rows == b.edge_rows && a.align == b.align && a.steps == b.steps &&
             a.edge_cols == b.edge_cols && a.stream_stores == b.stream_stores;
    };
    std::stable_sort(tried.begin(), tried.end(),
                     [](const std::pair<double, lbm_tiling> &a,
                        const std::pair<double, lbm_tiling> &b) { return a.first < b.first; });
    std::vector<lbm_tiling> fin;
    for (const auto &e : tried) {
      if (fin.size() == 3) break;
      bool dup = false;
      for (const lbm_tiling &f : fin) dup = dup || same(f, e.second);
      if (!dup) fin.push_back(e.second);
    }
    if (!fin.empty() && best < 1e299) {
      reps = std::max(steps, std::min(400, (int)std::ceil(5.0 / best)));
      double one_best = 1e300, ov_best = 1e300;
      lbm_tiling one_t = bt, ov_t = bt;
      for (const lbm_tiling &T0 : fin) {
        const int r = reps;
        if (T0.steps == 2) reps = std::max(steps, (r + 1) / 2);  // pairs
        const double per = eval(T0, false, true);
        if (per < one_best) {
          one_best = per;
          one_t = T0;
        }
        if (ov_user && T0.steps == 2) {
          std::vector<int> rows_tried;
          for (int E : {T0.edge_rows, 2, 4}) {
            lbm_tiling T = T0;
            T.edge_rows = E >= T.rows ? 0 : E;
            if (std::find(rows_tried.begin(), rows_tried.end(), T.edge_rows) != rows_tried.end())
              continue;
            rows_tried.push_back(T.edge_rows);
            const double pov = eval(T, true, true);
            if (pov < ov_best) {
              ov_best = pov;
              ov_t = T;
            }
          }
        }
        reps = r;
      }
      if (one_best < 1e299) {
        best = one_best;
        bt = one_t;
      }
      if (ov_best < 0.97 * one_best) {
        best = ov_best;
        bt = ov_t;
        best_ov = true;
      }
    }
  }
  // The second launch of a pair wrote the boundary nodes' u(t_{n+2}) where
  // the next step expects u(t_{n+1}): recompute that from u(t_n).
  HIP_TRY(c, launch_boundary(c->storage, c->ds, c->d_chunks, (int)c->chunks.size(), c->d_unodes,
                             c->d_gnodes, c->d_btasks, c->d_stasks, cur, prev, cur ^ 1,
                             have_third(c) ? 2 : -1,
                             (int)(n & 1), 0, c->stream),
          "boundary accelerations");
  (void)hipStreamSynchronize(c->stream);
  dev_free(c, side_scratch);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->lanes = bt.lanes;
  c->rows = bt.rows;
  c->order = bt.order;
  c->edge_rows = bt.edge_rows;
  c->edge_cols = bt.edge_cols;
  c->align = bt.align;
  c->nt = bt.stream_stores;
  c->two = bt.steps == 2 ? 1 : 0;
  c->overlap = best_ov;
  if (!c->two && !had_third) release_third(c);
  build_tiles(c);
  build_tile_tables(c);
  st = upload_tiles(c);
  if (st) return st;
  st = upload_tile_tables(c);
  if (st) return st;
  drop_graph(c);
  if (best_ms) *best_ms = best;
  return LBM_OK;
}

}  // extern "C"
