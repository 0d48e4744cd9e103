// Exact-geometry boundary cells for bodies bounded by ellipses (Sec. 3.1:
// the preprocessing computes cell volumes and surface measures at boundary
// lattice points, starting from the square cell of side dh around the point
// and cutting it to the body's boundary).  Host code only.
//
// The body is the lattice rectangle R = [0, nx-1] x [0, ny-1] (lattice units,
// node (i, j) at (i, j); a periodic axis is not bounded) minus the open
// interiors of the holes and the open exteriors of the bounding ellipses.
// The cell of node (i, j) is its unit square S = [i-1/2, i+1/2] x
// [j-1/2, j+1/2] intersected with the body; its volume is the area of that
// set and the length of each side towards a neighbour in the body is the
// part of the square's side that lies in the body.  A side towards a
// neighbour outside the body gets length 0 even where the boundary passes
// beyond it: the thin part of the body between that side and the boundary
// belongs to no cell, and taken as massless it passes the boundary's
// traction on to the cell, so that side counts as part of the cell's
// external boundary.  Areas are computed in the coordinates in which an ellipse is
// the unit circle: there the clipped square is a parallelogram, and the area
// of a convex polygon inside the unit disc is a sum over its edges of the
// disc's share of the triangle spanned by the origin and the edge (a
// triangle part where the edge runs inside the circle, a circular sector
// where it runs outside).
#include <cmath>
#include <cstdint>
#include <vector>

#include "lbm.h"

namespace {

struct V2 {
  double x, y;
};
inline V2 sub(V2 a, V2 b) { return {a.x - b.x, a.y - b.y}; }
inline double dot(V2 a, V2 b) { return a.x * b.x + a.y * b.y; }
inline double cross(V2 a, V2 b) { return a.x * b.y - a.y * b.x; }

// Parameters t0 <= t1 where the line a + t d meets the unit circle; false if
// it misses (or only touches) it.
bool circle_hits(V2 a, V2 d, double &t0, double &t1) {
  const double A = dot(d, d), B = dot(a, d), C = dot(a, a) - 1.0;
  if (A == 0.0) return false;
  const double disc = B * B - A * C;
  if (!(disc > 0.0)) return false;
  const double r = std::sqrt(disc);
  // roots of A t^2 + 2 B t + C without cancellation
  const double q = B >= 0.0 ? -(B + r) : -(B - r);
  double u0 = q / A, u1 = q != 0.0 ? C / q : -u0;
  if (u0 > u1) std::swap(u0, u1);
  t0 = u0;
  t1 = u1;
  return true;
}

// Signed area of (triangle 0, a, b) intersected with the unit disc.
double tri_disc_area(V2 a, V2 b) {
  const V2 d = sub(b, a);
  V2 pts[4];
  int np = 0;
  pts[np++] = a;
  double t0, t1;
  if (circle_hits(a, d, t0, t1)) {
    if (t0 > 0.0 && t0 < 1.0) pts[np++] = {a.x + t0 * d.x, a.y + t0 * d.y};
    if (t1 > 0.0 && t1 < 1.0) pts[np++] = {a.x + t1 * d.x, a.y + t1 * d.y};
  }
  pts[np++] = b;
  double s = 0.0;
  for (int k = 0; k + 1 < np; k++) {
    const V2 p = pts[k], q = pts[k + 1];
    const V2 m = {0.5 * (p.x + q.x), 0.5 * (p.y + q.y)};
    if (dot(m, m) <= 1.0)
      s += 0.5 * cross(p, q);  // piece inside the circle: the triangle
    else
      s += 0.5 * std::atan2(cross(p, q), dot(p, q));  // outside: the sector
  }
  return s;
}

struct Ellipse {
  double cx, cy, a, b, c, s;  // centre, semi-axes, cos / sin of the angle
  int kind;
  // to the coordinates in which the ellipse is the unit circle
  V2 map(V2 p) const {
    const double dx = p.x - cx, dy = p.y - cy;
    return {(c * dx + s * dy) / a, (-s * dx + c * dy) / b};
  }
};

// Area of the rectangle [x0, x1] x [y0, y1] inside ellipse e.
double rect_in_ellipse(double x0, double x1, double y0, double y1, const Ellipse &e) {
  const V2 q[4] = {e.map({x0, y0}), e.map({x1, y0}), e.map({x1, y1}), e.map({x0, y1})};
  double s = 0.0;
  for (int k = 0; k < 4; k++) s += tri_disc_area(q[k], q[(k + 1) % 4]);
  return std::fabs(s) * e.a * e.b;
}

// Length of the segment p -> r inside ellipse e.
double seg_in_ellipse(V2 p, V2 r, const Ellipse &e) {
  const double len = std::sqrt(dot(sub(r, p), sub(r, p)));
  if (len == 0.0) return 0.0;
  const V2 a = e.map(p), d = sub(e.map(r), a);
  double t0, t1;
  if (!circle_hits(a, d, t0, t1)) return 0.0;
  t0 = std::fmax(t0, 0.0);
  t1 = std::fmin(t1, 1.0);
  return t1 > t0 ? (t1 - t0) * len : 0.0;
}

// Whether node (i, j) lies in the body (points on an ellipse do).
bool node_in_body(int i, int j, int nx, int ny, bool px, bool py, const std::vector<Ellipse> &E) {
  if (!px && (i < 0 || i > nx - 1)) return false;
  if (!py && (j < 0 || j > ny - 1)) return false;
  for (const Ellipse &e : E) {
    const V2 q = e.map({(double)i, (double)j});
    const double r2 = dot(q, q);
    if ((e.kind == LBM_SHAPE_HOLE && r2 < 1.0) || (e.kind == LBM_SHAPE_BOUND && r2 > 1.0))
      return false;
  }
  return true;
}

// The part of a body-bounding set inside [lo, hi]: [lo, hi] itself on a
// periodic axis, else clipped to [0, n - 1].
bool clip(double lo, double hi, int n, bool periodic, double &a, double &b) {
  a = periodic ? lo : std::fmax(lo, 0.0);
  b = periodic ? hi : std::fmin(hi, (double)(n - 1));
  return b > a;
}

}  // namespace

extern "C" lbm_status lbm_exact_cells(int32_t nx, int32_t ny, uint8_t periodic_x,
                                      uint8_t periodic_y, double dh, int32_t n_shapes,
                                      const lbm_shape *shapes, int32_t n, const int32_t *xy,
                                      double *cell, double *ext_normal) {
  if (nx < 3 || ny < 3 || !(dh > 0.0) || n_shapes < 0 || n < 0) return LBM_E_INVAL;
  if ((n_shapes > 0 && !shapes) || (n > 0 && (!xy || !cell))) return LBM_E_INVAL;
  std::vector<Ellipse> E;
  for (int q = 0; q < n_shapes; q++) {
    const lbm_shape &sh = shapes[q];
    if (!(sh.a > 0.0) || !(sh.b > 0.0) || !std::isfinite(sh.cx) || !std::isfinite(sh.cy) ||
        !std::isfinite(sh.a) || !std::isfinite(sh.b) || !std::isfinite(sh.angle))
      return LBM_E_INVAL;
    if (sh.kind != LBM_SHAPE_HOLE && sh.kind != LBM_SHAPE_BOUND) return LBM_E_INVAL;
    E.push_back({sh.cx, sh.cy, sh.a, sh.b, std::cos(sh.angle), std::sin(sh.angle), sh.kind});
  }
  for (int m = 0; m < n; m++) {
    const int i = xy[2 * m], j = xy[2 * m + 1];
    if (i < 0 || i >= nx || j < 0 || j >= ny) return LBM_E_INVAL;
    double x0, x1, y0, y1;
    const bool okx = clip(i - 0.5, i + 0.5, nx, periodic_x != 0, x0, x1);
    const bool oky = clip(j - 0.5, j + 0.5, ny, periodic_y != 0, y0, y1);
    double V = 0.0, l[4] = {0.0, 0.0, 0.0, 0.0};  // E, N, W, S
    if (okx && oky) {
      V = (x1 - x0) * (y1 - y0);
      // sides of the square inside R (on a non-periodic axis the square of
      // an edge node is cut at the node: that cut lies on the body's
      // boundary and is not a side towards a neighbour)
      const bool hasE = periodic_x || i + 0.5 <= nx - 1;
      const bool hasW = periodic_x || i - 0.5 >= 0;
      const bool hasN = periodic_y || j + 0.5 <= ny - 1;
      const bool hasS = periodic_y || j - 0.5 >= 0;
      const V2 pE0 = {i + 0.5, y0}, pE1 = {i + 0.5, y1};
      const V2 pW0 = {i - 0.5, y0}, pW1 = {i - 0.5, y1};
      const V2 pN0 = {x0, j + 0.5}, pN1 = {x1, j + 0.5};
      const V2 pS0 = {x0, j - 0.5}, pS1 = {x1, j - 0.5};
      const bool px = periodic_x != 0, py = periodic_y != 0;
      if (hasE && node_in_body(i + 1, j, nx, ny, px, py, E)) l[0] = y1 - y0;
      if (hasN && node_in_body(i, j + 1, nx, ny, px, py, E)) l[1] = x1 - x0;
      if (hasW && node_in_body(i - 1, j, nx, ny, px, py, E)) l[2] = y1 - y0;
      if (hasS && node_in_body(i, j - 1, nx, ny, px, py, E)) l[3] = x1 - x0;
      // The removed regions (hole interiors, bounding-ellipse exteriors) are
      // disjoint inside the square: subtract each one's share.
      const double area = V, full[4] = {l[0], l[1], l[2], l[3]};
      const V2 side[4][2] = {{pE0, pE1}, {pN0, pN1}, {pW0, pW1}, {pS0, pS1}};
      for (const Ellipse &e : E) {
        const bool hole = e.kind == LBM_SHAPE_HOLE;
        const double in = rect_in_ellipse(x0, x1, y0, y1, e);
        V -= hole ? in : area - in;
        for (int k = 0; k < 4; k++) {
          if (full[k] == 0.0) continue;
          const double li = seg_in_ellipse(side[k][0], side[k][1], e);
          l[k] -= hole ? li : full[k] - li;
        }
      }
    }
    V = std::fmax(V, 0.0);
    for (int k = 0; k < 4; k++) l[k] = std::fmax(l[k], 0.0);
    cell[5 * m + 0] = V * dh * dh;
    cell[5 * m + 1] = l[0] * dh;
    cell[5 * m + 2] = l[1] * dh;
    cell[5 * m + 3] = l[2] * dh;
    cell[5 * m + 4] = l[3] * dh;
    if (ext_normal) {
      // closure: the outward normal integrated over the boundary of the cell
      // and the massless parts beyond it vanishes, so the external part is
      // minus that of the sides towards neighbours
      ext_normal[2 * m + 0] = -(l[0] - l[2]) * dh;
      ext_normal[2 * m + 1] = -(l[1] - l[3]) * dh;
    }
  }
  return LBM_OK;
}
