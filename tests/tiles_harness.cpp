// Host-only check of the interior tiling (no GPU): builds the tiles of the
// library's host code for plates read from stdin and checks the invariants
// that the two-step and overlapped launches rely on.  Built by
// tests/test_tiles_cpu.py together with the library's host source; the
// kernel launchers are stubs that are never called.
//
// stdin: n_plates lanes rows order edge_rows align steps edge_cols overlap
//        then per plate: nx ny periodic_x periodic_y, ny rows of nx 0/1
// stdout: "tiles T single S frame F deep D" and one line per violation.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <iostream>
#include <string>
#include <vector>

#include "../paper_2301_00228_amd/csrc/lbm_host.cpp"

namespace lbm {
hipError_t launch_interior(int, const DevState &, const Tile *, int, int, const StepBufs &,
                           const Prologue &, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_deep(int, const DevState &, const Tile *, int, int, const StepBufs &,
                       hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_boundary(int, const DevState &, const Chunk *, int, const UNode *,
                           const GradNode *, const BTask *, const STask *, int, int, int, int, int,
                           int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_sync(int, const DevState &, const Tile *, int, int, int, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_init(int, const DevState &, int, int64_t, const double *, const double *,
                       const double *, const double *, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_fields(int, const DevState &, int, int64_t, int, double *, double *, double *,
                         double *, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_cons_err(int, const DevState &, int, int64_t, int, double *, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t copy_rate(size_t, int, double *gbs) {
  *gbs = 0;
  return hipErrorInvalidValue;
}
hipError_t layout_copy_rate(int, int64_t, int, double *gbs) {
  *gbs = 0;
  return hipErrorInvalidValue;
}
hipError_t noalloc_staging(int, void **ptr) {
  *ptr = nullptr;
  return hipErrorInvalidValue;
}
}  // namespace lbm

int main() {
  int np, lanes, rows, order, er, align, steps, ec, ov;
  if (!(std::cin >> np >> lanes >> rows >> order >> er >> align >> steps >> ec >> ov)) return 2;
  lbm_ctx *c = new lbm_ctx();
  c->ph.resize(np);
  std::vector<std::vector<uint8_t>> masks(np);
  int64_t off = 0;
  for (int p = 0; p < np; p++) {
    lbm_plate pl{};
    int px, py;
    std::cin >> pl.nx >> pl.ny >> px >> py;
    masks[p].resize((size_t)pl.nx * pl.ny);
    for (auto &m : masks[p]) {
      int v;
      std::cin >> v;
      m = (uint8_t)v;
    }
    pl.mask = masks[p].data();
    pl.periodic_x = (uint8_t)px;
    pl.periodic_y = (uint8_t)py;
    PlateHost &h = c->ph[p];
    h.nx = pl.nx;
    h.ny = pl.ny;
    h.px = px != 0;
    h.py = py != 0;
    h.pitch = (pl.nx + 63) / 64 * 64;
    h.off = off;
    off += (int64_t)h.pitch * pl.ny;
    std::string why;
    if (!classify(pl, h, why)) {
      printf("classify: %s\n", why.c_str());
      return 3;
    }
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
  }
  c->lanes = lanes;
  c->rows = rows;
  c->order = order;
  c->edge_rows = er;
  c->align = align;
  c->two = steps == 2 ? 1 : 0;
  c->edge_cols = ec;
  c->overlap = ov != 0;
  build_tiles(c);

  int bad = 0;
  auto report = [&](const char *what, int p, int i, int j, int t) {
    if (bad++ < 20) printf("violation: %s plate %d node (%d, %d) tile %d\n", what, p, i, j, t);
  };
  // owner of every node, by brute force over the tiles
  std::vector<std::vector<int>> owner(np);
  for (int p = 0; p < np; p++) owner[p].assign((size_t)c->ph[p].nx * c->ph[p].ny, -1);
  for (size_t t = 0; t < c->tiles.size(); t++) {
    const Tile &T = c->tiles[t];
    const int own = lanes - (c->two ? 4 : 2);
    if (T.x1 - T.x0 > own || T.x1 <= T.x0 || T.y1 <= T.y0) report("tile shape", T.plate, T.x0, T.y0, (int)t);
    for (int j = T.y0; j < T.y1; j++)
      for (int i = T.x0; i < T.x1; i++) {
        int &o = owner[T.plate][(size_t)j * c->ph[T.plate].nx + i];
        if (o >= 0) report("owned twice", T.plate, i, j, (int)t);
        o = (int)t;
      }
  }
  for (int p = 0; p < np; p++)
    for (size_t k = 0; k < owner[p].size(); k++)
      if (owner[p][k] < 0) report("not owned", p, (int)(k % c->ph[p].nx), (int)(k / c->ph[p].nx), -1);
  // the same owner through the library's own lookup
  for (int p = 0; p < np; p++)
    for (int j = 0; j < c->ph[p].ny; j++)
      for (int i = 0; i < c->ph[p].nx; i++)
        if (tile_at(c, p, i, j) != owner[p][(size_t)j * c->ph[p].nx + i]) report("tile_at", p, i, j, -1);
  int ns = 0, nf = 0, nd = 0;
  for (size_t t = 0; t < c->tiles.size(); t++) {
    const Tile &T = c->tiles[t];
    const PlateHost &h = c->ph[T.plate];
    const bool two = (T.flags & TF_TWO) != 0, frame = (T.flags & TF_FRAME) != 0;
    if (!two) ns++;
    else if (frame) nf++;
    else nd++;
    if (frame && !two) report("frame tile not two-step", T.plate, T.x0, T.y0, (int)t);
    if (!two) continue;
    // the two-node ring (and area) of a two-step tile: no boundary or
    // second-row node; of a deep tile: only nodes of two-step tiles, and no
    // ring node of a single-step tile's one-node ring
    for (int j = T.y0 - 2; j < T.y1 + 2; j++)
      for (int i = T.x0 - 2; i < T.x1 + 2; i++) {
        int ii = i, jj = j;
        if (ii < 0 || ii >= h.nx) {
          if (!h.px) {
            report("two-step ring leaves the plate", T.plate, i, j, (int)t);
            continue;
          }
          ii = ((ii % h.nx) + h.nx) % h.nx;
        }
        if (jj < 0 || jj >= h.ny) {
          if (!h.py) {
            report("two-step ring leaves the plate", T.plate, i, j, (int)t);
            continue;
          }
          jj = ((jj % h.ny) + h.ny) % h.ny;
        }
        const uint8_t cl = h.cls[(size_t)jj * h.nx + ii];
        if (cl & (CL_B | CL_S)) report("boundary or second row near a two-step tile", T.plate, ii, jj, (int)t);
        const int o = owner[T.plate][(size_t)jj * h.nx + ii];
        if (!frame && o >= 0 && !(c->tiles[(size_t)o].flags & TF_TWO))
          report("single-step node in a deep tile's ring", T.plate, ii, jj, (int)t);
      }
    if (!frame && (T.flags & (TF_EXP_W | TF_EXP_E | TF_EXP_S | TF_EXP_N)))
      report("deep tile exports", T.plate, T.x0, T.y0, (int)t);
  }
  // The launched tiles (all but the merged-away ones, a paired tile owning
  // its second segment too) partition every plate; a paired tile is
  // single-step, its partner is merged away with the same rows, direction
  // and columns, and both segments with their halo columns fit the lanes.
  int npaired = 0;
  std::vector<std::vector<int>> lowner(np);
  for (int p = 0; p < np; p++) lowner[p].assign((size_t)c->ph[p].nx * c->ph[p].ny, -1);
  for (size_t t = 0; t < c->tiles.size(); t++) {
    const Tile &T = c->tiles[t];
    const int pb = c->partner[t];
    if (T.flags & TF_MERGED) {
      bool found = false;
      for (size_t a = 0; a < c->tiles.size(); a++) found = found || c->partner[a] == (int)t;
      if (!found) report("merged tile without partner", T.plate, T.x0, T.y0, (int)t);
      continue;
    }
    const bool paired = T.bx1 > T.bx0;
    if (paired != (pb >= 0)) report("pairing bookkeeping", T.plate, T.x0, T.y0, (int)t);
    if (paired) {
      npaired++;
      const Tile &B = c->tiles[(size_t)pb];
      if ((T.flags & TF_TWO) || (B.flags & TF_TWO)) report("paired two-step tile", T.plate, T.x0, T.y0, (int)t);
      if (!(B.flags & TF_MERGED) || B.x0 != T.bx0 || B.x1 != T.bx1 || B.y0 != T.y0 || B.y1 != T.y1 ||
          B.dir != T.dir || B.plate != T.plate)
        report("partner mismatch", T.plate, T.x0, T.y0, (int)t);
      if ((T.x1 - T.x0) + (T.bx1 - T.bx0) + 4 > lanes) report("paired tile too wide", T.plate, T.x0, T.y0, (int)t);
    }
    for (int seg = 0; seg < (paired ? 2 : 1); seg++) {
      const int x0 = seg ? T.bx0 : T.x0, x1 = seg ? T.bx1 : T.x1;
      for (int j = T.y0; j < T.y1; j++)
        for (int i = x0; i < x1; i++) {
          int &o = lowner[T.plate][(size_t)j * c->ph[T.plate].nx + i];
          if (o >= 0) report("launched twice", T.plate, i, j, (int)t);
          o = (int)t;
        }
    }
  }
  for (int p = 0; p < np; p++)
    for (size_t k = 0; k < lowner[p].size(); k++)
      if (lowner[p][k] < 0) report("not launched", p, (int)(k % c->ph[p].nx), (int)(k / c->ph[p].nx), -1);
  // Prologue lists: a launched tile lists every boundary node (and
  // accelerates exactly those it owns) and every second-row node of its
  // segments' areas and one-node rings.
  build_tile_tables(c);
  for (size_t t = 0; t < c->tiles.size(); t++) {
    const Tile &T = c->tiles[t];
    if (T.flags & TF_MERGED) continue;
    const PlateHost &h = c->ph[T.plate];
    std::vector<int> want_b, want_s;  // node index in plate, owned flag in want_b as +/-
    for (int seg = 0; seg < (T.bx1 > T.bx0 ? 2 : 1); seg++) {
      const int x0 = seg ? T.bx0 : T.x0, x1 = seg ? T.bx1 : T.x1;
      for (int j = T.y0 - 1; j <= T.y1; j++)
        for (int i = x0 - 1; i <= x1; i++) {
          int ii = i, jj = j;
          if (ii < 0 || ii >= h.nx) {
            if (!h.px) continue;
            ii = (ii + h.nx) % h.nx;
          }
          if (jj < 0 || jj >= h.ny) {
            if (!h.py) continue;
            jj = (jj + h.ny) % h.ny;
          }
          const uint8_t cl = h.cls[(size_t)jj * h.nx + ii];
          const bool own = lowner[T.plate][(size_t)jj * h.nx + ii] == (int)t;
          const int k = jj * h.nx + ii;
          if (cl & CL_B) want_b.push_back(own ? k + 1 : -(k + 1));
          else if (cl & CL_S) want_s.push_back(k);
        }
    }
    std::sort(want_s.begin(), want_s.end());
    want_s.erase(std::unique(want_s.begin(), want_s.end()), want_s.end());
    std::vector<int> have_b, have_s;
    if (T.chunk >= 0) {
      const TileChunk &ch = c->tchunks[(size_t)T.chunk];
      if (ch.plate != T.plate) report("chunk plate", T.plate, T.x0, T.y0, (int)t);
      for (int q = ch.b0; q < ch.b1; q++) {
        const BTask &B = c->tbt[(size_t)q];
        const int k = B.b.j * h.nx + B.b.i;
        have_b.push_back(B.accel ? k + 1 : -(k + 1));
      }
      for (int q = ch.s0; q < ch.s1; q++) have_s.push_back(c->tst[(size_t)q].j * h.nx + c->tst[(size_t)q].i);
    }
    // a node seen twice (rings of both segments) is listed once, owned if owned anywhere
    std::sort(want_b.begin(), want_b.end(), [](int a, int b) {
      return std::abs(a) != std::abs(b) ? std::abs(a) < std::abs(b) : a > b;
    });
    want_b.erase(std::unique(want_b.begin(), want_b.end(), [](int a, int b) { return std::abs(a) == std::abs(b); }),
                 want_b.end());
    std::sort(have_b.begin(), have_b.end(), [](int a, int b) {
      return std::abs(a) != std::abs(b) ? std::abs(a) < std::abs(b) : a > b;
    });
    std::sort(have_s.begin(), have_s.end());
    if (want_b != have_b) report("prologue boundary list", T.plate, T.x0, T.y0, (int)t);
    if (want_s != have_s) report("prologue second-row list", T.plate, T.x0, T.y0, (int)t);
  }
  printf("tiles %zu single %d frame %d deep %d paired %d n_two %lld n_deep %lld violations %d\n",
         c->tiles.size(), ns, nf, nd, npaired, (long long)c->n_two, (long long)c->n_deep, bad);
  return bad ? 1 : 0;
}
