// lbm_kernels.hip -- gfx950 kernels of the plane-strain LBM
// (Schlueter et al., arXiv 2301.00228).
//
// One time step is two launches (plus the synchronization every l steps):
//
//  k_interior  every body node of every plate, tiled.  A workgroup owns a
//              strip of columns and marches up a band of rows.  Each lane
//              loads its node's populations once, collides them (eq. LBE,
//              dt/tau = 2) and hands the post-collision populations and the
//              zeroth moments to its x-neighbours through LDS and to its
//              y-neighbours through registers.  Interior nodes then take the
//              acceleration of eq. navier from the neighbours' phi and psi,
//              advance u and du/dt by eq. integration, and (unless a
//              neighbour is a boundary node) store the streamed populations.
//  k_post      boundary and second-row nodes: the boundary reset of
//              eqs. psi_phi_at_bound and correction-f from finite
//              differences of u(t+dt); the second-row pull of eq. LBE_mod
//              with the time-averaged boundary populations; and the boundary
//              accelerations of eqs. acc_neumann / acc_dirichlet of the next
//              step with their Newmark update, written into the other u
//              buffer.
//
// Buffers ping-pong: step n reads populations, u and du/dt from buffer
// cur = n & 1 and writes buffer cur ^ 1.  Boundary nodes' u(t_{n+1}) is
// written one step ahead by k_post (or k_bacc0 before the first step).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "lbm_kernels.h"
#include "lbm_types.h"

namespace lbm {

// ------------------------------------------------------------------ codecs
//
// A codec maps the stored representation of one field's five populations
// to populations in the collision precision C and back.  eq_pops gives the
// populations of f_eq(rho, J) (eq. feq, lattice units c = 1, b = 1) exactly
// as load() returns them after store_eq().

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
  return __half_as_ushort(__float2half_rn(x));
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }

template <class T>
__device__ __forceinline__ T ldg(const void *p, int64_t k) {
  return static_cast<const T *>(p)[k];
}
template <class T>
__device__ __forceinline__ void stg(void *p, int64_t k, T v) {
  static_cast<T *>(p)[k] = v;
}

template <class C>
__device__ __forceinline__ void eq_populations(C a0, C a, C rho, C jx, C jy, C f[5]) {
  const C ar = a * rho;
  f[0] = a0 * rho;
  f[1] = ar + C(0.5) * jx;
  f[2] = ar + C(0.5) * jy;
  f[3] = ar - C(0.5) * jx;
  f[4] = ar - C(0.5) * jy;
}

// Plain populations, FP64 or FP32.
template <class T>
struct PopCodec {
  using C = T;
  using U = T;
  __device__ static C aw(const PlateDev &P, int fl) { return (C)P.a[fl]; }
  __device__ static C a0w(const PlateDev &P, int fl) { return (C)P.a0[fl]; }
  __device__ static void load(const DevState &s, int b, int fl, int64_t k, const PlateDev &,
                              C f[5]) {
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = ldg<T>(s.pop[b][fl][q], k);
  }
  __device__ static void store(const DevState &s, int b, int fl, int64_t k, const PlateDev &,
                               const C f[5]) {
#pragma unroll
    for (int q = 0; q < 5; q++) stg<T>(s.pop[b][fl][q], k, f[q]);
  }
  __device__ static void flux(const DevState &s, int b, int fl, int64_t k, const PlateDev &,
                              C &jx, C &jy) {
    jx = ldg<T>(s.pop[b][fl][1], k) - ldg<T>(s.pop[b][fl][3], k);
    jy = ldg<T>(s.pop[b][fl][2], k) - ldg<T>(s.pop[b][fl][4], k);
  }
  __device__ static void eq_pops(const PlateDev &P, int fl, C rho, C jx, C jy, C f[5]) {
    eq_populations<C>(a0w(P, fl), aw(P, fl), rho, jx, jy, f);
  }
  __device__ static void store_eq(const DevState &s, int b, int fl, int64_t k, const PlateDev &P,
                                  C rho, C jx, C jy) {
    C f[5];
    eq_pops(P, fl, rho, jx, jy, f);
    store(s, b, fl, k, P, f);
  }
  __device__ static double field(const DevState &s, int b, int fl, int64_t k, const PlateDev &P) {
    C f[5];
    load(s, b, fl, k, P, f);
    return (double)(f[0] + ((f[1] + f[3]) + (f[2] + f[4])));
  }
};

// Deviation from the local rest equilibrium in a moment basis:
// rho, J_x = f1 - f3, J_y = f2 - f4 in FP32; N = (f1 + f3) - (f2 + f4) and
// D = (f1 + f2 + f3 + f4) - 4 a rho in FP32 (H = 0) or in a 16-bit type
// (H = 1 FP16, H = 2 BF16) scaled by a power of two and packed in one word.
template <int H>
struct DevCodec {
  using C = float;
  using U = double;
  __device__ static C aw(const PlateDev &P, int fl) { return P.af[fl]; }
  __device__ static C a0w(const PlateDev &P, int fl) { return P.a0f[fl]; }
  __device__ static void unpack(uint32_t w, const PlateDev &P, int fl, float &n, float &d) {
    const uint16_t lo = (uint16_t)(w & 0xffffu), hi = (uint16_t)(w >> 16);
    if (H == 1) {
      n = f16_to_f32(lo) * P.iscale[fl];
      d = f16_to_f32(hi) * P.iscale[fl];
    } else {
      n = bf16_to_f32(lo) * P.iscale[fl];
      d = bf16_to_f32(hi) * P.iscale[fl];
    }
  }
  __device__ static uint32_t pack(float n, float d, const PlateDev &P, int fl) {
    const float sn = n * P.scale[fl], sd = d * P.scale[fl];
    uint16_t lo, hi;
    if (H == 1) {
      lo = f32_to_f16_rne(sn);
      hi = f32_to_f16_rne(sd);
    } else {
      lo = f32_to_bf16_rne(sn);
      hi = f32_to_bf16_rne(sd);
    }
    return (uint32_t)lo | ((uint32_t)hi << 16);
  }
  __device__ static void load_moments(const DevState &s, int b, int fl, int64_t k,
                                      const PlateDev &P, float m[5]) {
    m[0] = ldg<float>(s.pop[b][fl][0], k);
    m[1] = ldg<float>(s.pop[b][fl][1], k);
    m[2] = ldg<float>(s.pop[b][fl][2], k);
    if (H == 0) {
      m[3] = ldg<float>(s.pop[b][fl][3], k);
      m[4] = ldg<float>(s.pop[b][fl][4], k);
    } else {
      unpack(ldg<uint32_t>(s.pop[b][fl][3], k), P, fl, m[3], m[4]);
    }
  }
  __device__ static void moments_to_pops(const PlateDev &P, int fl, const float m[5], C f[5]) {
    const float q = m[4] + 4.0f * aw(P, fl) * m[0];
    const float s13 = 0.5f * (q + m[3]);
    const float s24 = 0.5f * (q - m[3]);
    f[0] = m[0] - q;
    f[1] = 0.5f * (s13 + m[1]);
    f[3] = 0.5f * (s13 - m[1]);
    f[2] = 0.5f * (s24 + m[2]);
    f[4] = 0.5f * (s24 - m[2]);
  }
  __device__ static void load(const DevState &s, int b, int fl, int64_t k, const PlateDev &P,
                              C f[5]) {
    float m[5];
    load_moments(s, b, fl, k, P, m);
    moments_to_pops(P, fl, m, f);
  }
  __device__ static void store_moments(const DevState &s, int b, int fl, int64_t k,
                                       const PlateDev &P, const float m[5]) {
    stg<float>(s.pop[b][fl][0], k, m[0]);
    stg<float>(s.pop[b][fl][1], k, m[1]);
    stg<float>(s.pop[b][fl][2], k, m[2]);
    if (H == 0) {
      stg<float>(s.pop[b][fl][3], k, m[3]);
      stg<float>(s.pop[b][fl][4], k, m[4]);
    } else {
      stg<uint32_t>(s.pop[b][fl][3], k, pack(m[3], m[4], P, fl));
    }
  }
  __device__ static void store(const DevState &s, int b, int fl, int64_t k, const PlateDev &P,
                               const C f[5]) {
    const float s13 = f[1] + f[3], s24 = f[2] + f[4];
    const float q = s13 + s24;
    float m[5];
    m[0] = f[0] + q;
    m[1] = f[1] - f[3];
    m[2] = f[2] - f[4];
    m[3] = s13 - s24;
    m[4] = q - 4.0f * aw(P, fl) * m[0];
    store_moments(s, b, fl, k, P, m);
  }
  __device__ static void flux(const DevState &s, int b, int fl, int64_t k, const PlateDev &,
                              C &jx, C &jy) {
    jx = ldg<float>(s.pop[b][fl][1], k);
    jy = ldg<float>(s.pop[b][fl][2], k);
  }
  __device__ static void eq_pops(const PlateDev &P, int fl, C rho, C jx, C jy, C f[5]) {
    const float m[5] = {rho, jx, jy, 0.0f, 0.0f};
    moments_to_pops(P, fl, m, f);
  }
  __device__ static void store_eq(const DevState &s, int b, int fl, int64_t k, const PlateDev &P,
                                  C rho, C jx, C jy) {
    const float m[5] = {rho, jx, jy, 0.0f, 0.0f};
    store_moments(s, b, fl, k, P, m);
  }
  __device__ static double field(const DevState &s, int b, int fl, int64_t k, const PlateDev &) {
    return (double)ldg<float>(s.pop[b][fl][0], k);
  }
};

template <int ST>
struct CodecOf;
template <>
struct CodecOf<LBM_STORE_F64> {
  using type = PopCodec<double>;
};
template <>
struct CodecOf<LBM_STORE_F32> {
  using type = PopCodec<float>;
};
template <>
struct CodecOf<LBM_STORE_F32DEV> {
  using type = DevCodec<0>;
};
template <>
struct CodecOf<LBM_STORE_F16DEV> {
  using type = DevCodec<1>;
};
template <>
struct CodecOf<LBM_STORE_BF16DEV> {
  using type = DevCodec<2>;
};

// --------------------------------------------------------- node geometry

__device__ __forceinline__ int64_t node_of(const PlateDev &P, int i, int j) {
  return P.off + (int64_t)j * P.pitch + i;
}
__device__ __forceinline__ int wrapc(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Finite-difference derivative of q along axis ax at body node (i, j), per
// axis: central if both neighbours are in the body, else the one-sided
// 3-point second-order formula, else 2-point first order, else 0.  The
// neighbour bits of the class byte already account for periodic wrapping.
template <class U>
__device__ U fd_axis(const DevState &s, const U *q, const PlateDev &P, int i, int j, int ax) {
  const int64_t k0 = node_of(P, i, j);
  const uint8_t c0 = s.cls[k0];
  const uint8_t bp = ax == 0 ? NB_E : NB_N, bm = ax == 0 ? NB_W : NB_S;
  const int di = ax == 0 ? 1 : 0, dj = ax == 0 ? 0 : 1;
  const U h = (U)P.dh;
  const bool hp = (c0 & bp) != 0, hm = (c0 & bm) != 0;
  if (hp && hm) {
    const int64_t kp = node_of(P, wrapc(i + di, P.nx), wrapc(j + dj, P.ny));
    const int64_t km = node_of(P, wrapc(i - di, P.nx), wrapc(j - dj, P.ny));
    return (q[kp] - q[km]) / (U(2.0) * h);
  }
  if (hp) {
    const int ip = wrapc(i + di, P.nx), jp = wrapc(j + dj, P.ny);
    const int64_t kp = node_of(P, ip, jp);
    if (s.cls[kp] & bp) {
      const int64_t kpp = node_of(P, wrapc(ip + di, P.nx), wrapc(jp + dj, P.ny));
      return ((U(-3.0) * q[k0] + U(4.0) * q[kp]) - q[kpp]) / (U(2.0) * h);
    }
    return (q[kp] - q[k0]) / h;
  }
  if (hm) {
    const int im = wrapc(i - di, P.nx), jm = wrapc(j - dj, P.ny);
    const int64_t km = node_of(P, im, jm);
    if (s.cls[km] & bm) {
      const int64_t kmm = node_of(P, wrapc(im - di, P.nx), wrapc(jm - dj, P.ny));
      return ((U(3.0) * q[k0] - U(4.0) * q[km]) + q[kmm]) / (U(2.0) * h);
    }
    return (q[k0] - q[km]) / h;
  }
  return U(0.0);
}

// div u and (curl u).e_z (Sec. 2, eq. phi-psi) by finite differences.
template <class U>
__device__ void div_curl(const DevState &s, int b, const PlateDev &P, int i, int j, U &dv, U &cu) {
  const U *ux = static_cast<const U *>(s.u[b][0]);
  const U *uy = static_cast<const U *>(s.u[b][1]);
  const U dxux = fd_axis<U>(s, ux, P, i, j, 0), dyuy = fd_axis<U>(s, uy, P, i, j, 1);
  const U dxuy = fd_axis<U>(s, uy, P, i, j, 0), dyux = fd_axis<U>(s, ux, P, i, j, 1);
  dv = dxux + dyuy;
  cu = dxuy - dyux;
}

// Hooke's law (Sec. 2, eq. hooke) with the strain from finite differences.
template <class U>
__device__ void stress(const DevState &s, int b, const PlateDev &P, int i, int j, U &sxx, U &syy,
                       U &sxy) {
  const U *ux = static_cast<const U *>(s.u[b][0]);
  const U *uy = static_cast<const U *>(s.u[b][1]);
  const U exx = fd_axis<U>(s, ux, P, i, j, 0);
  const U eyy = fd_axis<U>(s, uy, P, i, j, 1);
  const U exy = U(0.5) * (fd_axis<U>(s, ux, P, i, j, 1) + fd_axis<U>(s, uy, P, i, j, 0));
  const U tr = exx + eyy;
  const U lam = (U)P.lam, mu = (U)P.mu;
  sxx = lam * tr + U(2.0) * mu * exx;
  syy = lam * tr + U(2.0) * mu * eyy;
  sxy = U(2.0) * mu * exy;
}

__device__ double load_amp(const DevState &s, int li, double t) {
  if (li < 0) return 1.0;
  const LoadTable &L = s.loads[li];
  const int n = L.n;
  if (n <= 0) return 1.0;
  if (t <= L.t[0]) return L.g[0];
  if (t >= L.t[n - 1]) return L.g[n - 1];
  for (int m = 0; m + 1 < n; m++) {
    if (t <= L.t[m + 1]) {
      const double w = (t - L.t[m]) / (L.t[m + 1] - L.t[m]);
      return L.g[m] + w * (L.g[m + 1] - L.g[m]);
    }
  }
  return L.g[n - 1];
}

// Boundary acceleration of step n (eq. acc_dirichlet or eq. acc_neumann)
// from u, du/dt in buffer sb, followed by the Newmark update of eq.
// integration into buffer db.
template <class U>
__device__ void boundary_accel_update(const DevState &s, int sb, int db, const BndNode &B,
                                      const PlateDev &P, unsigned long long n) {
  const int64_t k = B.node;
  const U ux = ldg<U>(s.u[sb][0], k), uy = ldg<U>(s.u[sb][1], k);
  const U vx = ldg<U>(s.v[sb][0], k), vy = ldg<U>(s.v[sb][1], k);
  const U dt = (U)P.dt;
  U ax, ay;
  if (B.kind == LBM_BC_DIRICHLET) {
    const double g = load_amp(s, B.load, (double)(n + 1) * P.dt);
    const U usx = (U)(g * B.val[0]), usy = (U)(g * B.val[1]);
    ax = U(2.0) / (dt * dt) * (usx - ux) - U(2.0) / dt * vx;
    ay = U(2.0) / (dt * dt) * (usy - uy) - U(2.0) / dt * vy;
  } else {
    const double g = load_amp(s, B.load, (double)n * P.dt);
    const uint8_t c0 = s.cls[k];
    const int i = B.i, j = B.j;
    const U V = (U)B.cell[0], lE = (U)B.cell[1], lN = (U)B.cell[2], lW = (U)B.cell[3],
            lS = (U)B.cell[4];
    U sxx, syy, sxy, rxx, ryy, rxy;
    stress<U>(s, sb, P, i, j, sxx, syy, sxy);
    U tEx = 0, tEy = 0, tWx = 0, tWy = 0, tNx = 0, tNy = 0, tSx = 0, tSy = 0;
    if (c0 & NB_E) {
      stress<U>(s, sb, P, wrapc(i + 1, P.nx), j, rxx, ryy, rxy);
      tEx = U(0.5) * (sxx + rxx) * lE;
      tEy = U(0.5) * (sxy + rxy) * lE;
    }
    if (c0 & NB_W) {
      stress<U>(s, sb, P, wrapc(i - 1, P.nx), j, rxx, ryy, rxy);
      tWx = -(U(0.5) * (sxx + rxx)) * lW;
      tWy = -(U(0.5) * (sxy + rxy)) * lW;
    }
    if (c0 & NB_N) {
      stress<U>(s, sb, P, i, wrapc(j + 1, P.ny), rxx, ryy, rxy);
      tNx = U(0.5) * (sxy + rxy) * lN;
      tNy = U(0.5) * (syy + ryy) * lN;
    }
    if (c0 & NB_S) {
      stress<U>(s, sb, P, i, wrapc(j - 1, P.ny), rxx, ryy, rxy);
      tSx = -(U(0.5) * (sxy + rxy)) * lS;
      tSy = -(U(0.5) * (syy + ryy)) * lS;
    }
    const U Fx = (U)(g * B.val[0]), Fy = (U)(g * B.val[1]);
    const U m = (U)P.rho_m * V;
    ax = (((tEx + tWx) + (tNx + tSx)) + Fx) / m;
    ay = (((tEy + tWy) + (tNy + tSy)) + Fy) / m;
  }
  const U nux = ux + dt * vx + dt * dt / U(2.0) * ax;
  const U nuy = uy + dt * vy + dt * dt / U(2.0) * ay;
  stg<U>(s.u[db][0], k, nux);
  stg<U>(s.u[db][1], k, nuy);
  stg<U>(s.v[db][0], k, vx + dt * ax);
  stg<U>(s.v[db][1], k, vy + dt * ay);
  if (!(fabs((double)nux) < 1e30) || !(fabs((double)nuy) < 1e30)) s.flag[0] = 1;
}

// Post-collision populations f* = f - 2 (f - f_eq(f)) and zeroth moment of
// one field at node k from buffer b (eq. LBE with dt/tau = 2).
template <class CD>
__device__ __forceinline__ void collide(const DevState &s, int b, int fl, int64_t k,
                                        const PlateDev &P, typename CD::C &rho,
                                        typename CD::C fs[5]) {
  using C = typename CD::C;
  C f[5];
  CD::load(s, b, fl, k, P, f);
  const C r = f[0] + ((f[1] + f[3]) + (f[2] + f[4]));
  const C jx = f[1] - f[3], jy = f[2] - f[4];
  C e[5];
  eq_populations<C>(CD::a0w(P, fl), CD::aw(P, fl), r, jx, jy, e);
#pragma unroll
  for (int q = 0; q < 5; q++) fs[q] = f[q] - C(2.0) * (f[q] - e[q]);
  rho = r;
}

// -------------------------------------------------------- interior kernel

// Exchange slots in LDS per lane and row.
enum { X_RHO0 = 0, X_RHO1, X_F1_0, X_F1_1, X_F3_0, X_F3_1, X_N };

__device__ __forceinline__ int tile_index(int b, int q) { return (b & 7) * q + (b >> 3); }

template <int ST, int TWL>
__global__ void __launch_bounds__(TWL)
    k_interior(DevState s, const Tile *__restrict__ tiles, int ntiles, int q, int cur) {
  using CD = typename CodecOf<ST>::type;
  using C = typename CD::C;
  using U = typename CD::U;
  __shared__ C ex[3][X_N][TWL];

  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(s.counter, 1ull);
  const int tix = tile_index(blockIdx.x, q);
  if (tix >= ntiles) return;
  const Tile t = tiles[tix];
  const PlateDev P = s.plates[t.plate];
  const int nxt = cur ^ 1;
  const int lane = threadIdx.x;
  const int w = t.x1 - t.x0;
  int x = t.x0 - 1 + lane;
  bool xok = lane <= w + 1;
  if (x < 0 || x >= P.nx) {
    if (P.periodic & 1)
      x = wrapc(x, P.nx);
    else
      xok = false;
  }
  const bool owned = xok && lane >= 1 && lane <= w;
  const bool py = (P.periodic & 2) != 0;

  // Source values of row y for this lane's column.
  auto source = [&](int y, uint8_t &cl, C rho[2], C fs[2][5]) {
    bool ok = xok;
    if (y < 0 || y >= P.ny) {
      if (py)
        y = wrapc(y, P.ny);
      else
        ok = false;
    }
    cl = 0;
    if (ok) cl = s.cls[node_of(P, x, y)];
    if (cl & CL_IN) {
      const int64_t k = node_of(P, x, y);
      collide<CD>(s, cur, 0, k, P, rho[0], fs[0]);
      collide<CD>(s, cur, 1, k, P, rho[1], fs[1]);
    } else {
#pragma unroll
      for (int fl = 0; fl < 2; fl++) {
        rho[fl] = C(0);
#pragma unroll
        for (int qq = 0; qq < 5; qq++) fs[fl][qq] = C(0);
      }
    }
  };
  auto publish = [&](int slot, const C rho[2], const C fs[2][5]) {
    ex[slot][X_RHO0][lane] = rho[0];
    ex[slot][X_RHO1][lane] = rho[1];
    ex[slot][X_F1_0][lane] = fs[0][1];
    ex[slot][X_F1_1][lane] = fs[1][1];
    ex[slot][X_F3_0][lane] = fs[0][3];
    ex[slot][X_F3_1][lane] = fs[1][3];
  };

  C pr_rho[2], pr_f2[2];  // row r-1: zeroth moments and f*_2 (moving +y)
  C cu_f0[2], cu_rho[2], cu_f2[2];
  uint8_t cu_cl;
  {
    uint8_t cl;
    C rho[2], fs[2][5];
    source(t.y0 - 1, cl, rho, fs);
    pr_rho[0] = rho[0];
    pr_rho[1] = rho[1];
    pr_f2[0] = fs[0][2];
    pr_f2[1] = fs[1][2];
    source(t.y0, cu_cl, rho, fs);
    publish(0, rho, fs);
    cu_rho[0] = rho[0];
    cu_rho[1] = rho[1];
    cu_f0[0] = fs[0][0];
    cu_f0[1] = fs[1][0];
    cu_f2[0] = fs[0][2];
    cu_f2[1] = fs[1][2];
  }
  int slot = 0;
  const U dt = (U)P.dt;
  const U h2 = U(2.0) * (U)P.dh;
  const U cd2 = (U)P.cd2, cs2 = (U)P.cs2;
  for (int r = t.y0; r < t.y1; r++) {
    const int nslot = slot == 2 ? 0 : slot + 1;
    const bool fin = owned && (cu_cl & (CL_IN | CL_B)) == CL_IN;
    const int64_t k = node_of(P, x, r);
    U ux = 0, uy = 0, vx = 0, vy = 0;
    if (fin) {
      ux = ldg<U>(s.u[cur][0], k);
      uy = ldg<U>(s.u[cur][1], k);
      vx = ldg<U>(s.v[cur][0], k);
      vy = ldg<U>(s.v[cur][1], k);
    }
    uint8_t nx_cl;
    C nx_rho[2], nx_fs[2][5];
    source(r + 1, nx_cl, nx_rho, nx_fs);
    publish(nslot, nx_rho, nx_fs);
    __syncthreads();
    if (fin) {
      const C wr0 = ex[slot][X_RHO0][lane - 1], er0 = ex[slot][X_RHO0][lane + 1];
      const C wr1 = ex[slot][X_RHO1][lane - 1], er1 = ex[slot][X_RHO1][lane + 1];
      // Acceleration of eq. navier: c_d^2 grad phi - c_s^2 curl(psi e_z),
      // with curl(psi e_z) = (d_y psi, -d_x psi).
      const U dphix = ((U)er0 - (U)wr0) / h2;
      const U dphiy = ((U)nx_rho[0] - (U)pr_rho[0]) / h2;
      const U dpsix = ((U)er1 - (U)wr1) / h2;
      const U dpsiy = ((U)nx_rho[1] - (U)pr_rho[1]) / h2;
      const U ax = cd2 * dphix - cs2 * dpsiy;
      const U ay = cd2 * dphiy - cs2 * (-dpsix);
      stg<U>(s.u[nxt][0], k, ux + dt * vx + dt * dt / U(2.0) * ax);
      stg<U>(s.u[nxt][1], k, uy + dt * vy + dt * dt / U(2.0) * ay);
      stg<U>(s.v[nxt][0], k, vx + dt * ax);
      stg<U>(s.v[nxt][1], k, vy + dt * ay);
      if (!(cu_cl & CL_S)) {
        // Pull: f_alpha(x, t+dt) = f*_alpha(x - c^alpha dt).
#pragma unroll
        for (int fl = 0; fl < 2; fl++) {
          C f[5];
          f[0] = cu_f0[fl];
          f[1] = ex[slot][fl == 0 ? X_F1_0 : X_F1_1][lane - 1];
          f[2] = pr_f2[fl];
          f[3] = ex[slot][fl == 0 ? X_F3_0 : X_F3_1][lane + 1];
          f[4] = nx_fs[fl][4];
          CD::store(s, nxt, fl, k, P, f);
        }
      }
    }
    pr_rho[0] = cu_rho[0];
    pr_rho[1] = cu_rho[1];
    pr_f2[0] = cu_f2[0];
    pr_f2[1] = cu_f2[1];
    cu_rho[0] = nx_rho[0];
    cu_rho[1] = nx_rho[1];
    cu_f0[0] = nx_fs[0][0];
    cu_f0[1] = nx_fs[1][0];
    cu_f2[0] = nx_fs[0][2];
    cu_f2[1] = nx_fs[1][2];
    cu_cl = nx_cl;
    slot = nslot;
  }
}

// ------------------------------------------- boundary / second-row kernel

// Boundary reset value of field fl at boundary node (i, j): the field from
// finite differences of u(t+dt) in buffer nb, the flux of the populations
// stored at time t in buffer cb (eqs. psi_phi_at_bound, correction-f).
template <class CD>
__device__ void reset_state(const DevState &s, int cb, int nb, const PlateDev &P, int i, int j,
                            typename CD::C rho[2], typename CD::C jx[2], typename CD::C jy[2]) {
  using U = typename CD::U;
  using C = typename CD::C;
  U dv, cu;
  div_curl<U>(s, nb, P, i, j, dv, cu);
  const int64_t k = node_of(P, i, j);
  rho[0] = (C)dv;
  rho[1] = (C)cu;
  CD::flux(s, cb, 0, k, P, jx[0], jy[0]);
  CD::flux(s, cb, 1, k, P, jx[1], jy[1]);
}

template <int ST>
__global__ void __launch_bounds__(256)
    k_post(DevState s, int nb, int ns, int cur, int do_bacc) {
  using CD = typename CodecOf<ST>::type;
  using C = typename CD::C;
  using U = typename CD::U;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nxt = cur ^ 1;
  if (tid < nb) {
    const BndNode B = s.bnd[tid];
    const PlateDev P = s.plates[B.plate];
    C rho[2], jx[2], jy[2];
    reset_state<CD>(s, cur, nxt, P, B.i, B.j, rho, jx, jy);
    CD::store_eq(s, nxt, 0, B.node, P, rho[0], jx[0], jy[0]);
    CD::store_eq(s, nxt, 1, B.node, P, rho[1], jx[1], jy[1]);
    if (do_bacc) {
      const unsigned long long n = *s.counter;  // steps completed = index of the next step
      boundary_accel_update<U>(s, nxt, cur, B, P, n);
    }
  } else if (tid < nb + ns) {
    const SecNode S = s.sec[tid - nb];
    const PlateDev P = s.plates[S.plate];
    const int di[5] = {0, 1, 0, -1, 0};
    const int dj[5] = {0, 0, 1, 0, -1};
    C fo[2][5];
#pragma unroll
    for (int al = 0; al < 5; al++) {
      // upwind node x - c^alpha dt (always in the body: x is interior)
      const int yi = wrapc(S.i - di[al], P.nx), yj = wrapc(S.j - dj[al], P.ny);
      const int64_t ky = node_of(P, yi, yj);
      if (s.cls[ky] & CL_B) {
        // eq. LBE_mod: time-averaged boundary populations, collided with the
        // equilibrium of their own moments.
        C rho[2], jx[2], jy[2];
        reset_state<CD>(s, cur, nxt, P, yi, yj, rho, jx, jy);
#pragma unroll
        for (int fl = 0; fl < 2; fl++) {
          C fnew[5], fold[5], fh[5];
          CD::eq_pops(P, fl, rho[fl], jx[fl], jy[fl], fnew);
          CD::load(s, cur, fl, ky, P, fold);
#pragma unroll
          for (int qq = 0; qq < 5; qq++) fh[qq] = C(0.5) * (fnew[qq] + fold[qq]);
          const C r = fh[0] + ((fh[1] + fh[3]) + (fh[2] + fh[4]));
          C e[5];
          eq_populations<C>(CD::a0w(P, fl), CD::aw(P, fl), r, fh[1] - fh[3], fh[2] - fh[4], e);
          fo[fl][al] = fh[al] - C(2.0) * (fh[al] - e[al]);
        }
      } else {
#pragma unroll
        for (int fl = 0; fl < 2; fl++) {
          C r, fs[5];
          collide<CD>(s, cur, fl, ky, P, r, fs);
          fo[fl][al] = fs[al];
        }
      }
    }
    CD::store(s, nxt, 0, S.node, P, fo[0]);
    CD::store(s, nxt, 1, S.node, P, fo[1]);
  }
}

// Boundary accelerations of the first step (before any k_post has run).
template <int ST>
__global__ void __launch_bounds__(256) k_bacc0(DevState s, int nb) {
  using U = typename CodecOf<ST>::type::U;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= nb) return;
  const BndNode B = s.bnd[tid];
  const PlateDev P = s.plates[B.plate];
  boundary_accel_update<U>(s, 0, 1, B, P, *s.counter);
}

// Periodic synchronization (Sec. 3.2): at every body node the fields become
// the finite differences of u, the populations f_eq(field, current J).
template <int ST, int TWL>
__global__ void __launch_bounds__(TWL)
    k_sync(DevState s, const Tile *__restrict__ tiles, int ntiles, int q, int b) {
  using CD = typename CodecOf<ST>::type;
  using C = typename CD::C;
  using U = typename CD::U;
  const int tix = tile_index(blockIdx.x, q);
  if (tix >= ntiles) return;
  const Tile t = tiles[tix];
  const PlateDev P = s.plates[t.plate];
  const int x = t.x0 + (int)threadIdx.x;
  if (x >= t.x1) return;
  for (int y = t.y0; y < t.y1; y++) {
    const int64_t k = node_of(P, x, y);
    if (!(s.cls[k] & CL_IN)) continue;
    U dv, cu;
    div_curl<U>(s, b, P, x, y, dv, cu);
    C jx, jy;
    CD::flux(s, b, 0, k, P, jx, jy);
    CD::store_eq(s, b, 0, k, P, (C)dv, jx, jy);
    CD::flux(s, b, 1, k, P, jx, jy);
    CD::store_eq(s, b, 1, k, P, (C)cu, jx, jy);
    const double ux = (double)ldg<U>(s.u[b][0], k), uy = (double)ldg<U>(s.u[b][1], k);
    if (!(fabs(ux) < 1e30) || !(fabs(uy) < 1e30)) s.flag[0] = 1;
  }
}

// Initial state of one plate (Fig. 4): u, du/dt from the dense host arrays;
// populations f_eq(field, J = 0) with the field from finite differences of
// u0 unless given directly.
template <int ST>
__global__ void k_init_uv(DevState s, int plate, const double *__restrict__ u0,
                          const double *__restrict__ v0) {
  using U = typename CodecOf<ST>::type::U;
  const PlateDev P = s.plates[plate];
  const int64_t n = (int64_t)P.nx * P.ny;
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(d % P.nx), j = (int)(d / P.nx);
    const int64_t k = node_of(P, i, j);
    const bool in = (s.cls[k] & CL_IN) != 0;
    const U ux = in && u0 ? (U)u0[d] : U(0), uy = in && u0 ? (U)u0[n + d] : U(0);
    const U vx = in && v0 ? (U)v0[d] : U(0), vy = in && v0 ? (U)v0[n + d] : U(0);
    for (int b = 0; b < 2; b++) {
      stg<U>(s.u[b][0], k, ux);
      stg<U>(s.u[b][1], k, uy);
      stg<U>(s.v[b][0], k, vx);
      stg<U>(s.v[b][1], k, vy);
    }
  }
}

template <int ST>
__global__ void k_init_pops(DevState s, int plate, const double *__restrict__ e0,
                            const double *__restrict__ w0) {
  using CD = typename CodecOf<ST>::type;
  using C = typename CD::C;
  using U = typename CD::U;
  const PlateDev P = s.plates[plate];
  const int64_t n = (int64_t)P.nx * P.ny;
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(d % P.nx), j = (int)(d / P.nx);
    const int64_t k = node_of(P, i, j);
    if (!(s.cls[k] & CL_IN)) continue;
    U dv, cu;
    div_curl<U>(s, 0, P, i, j, dv, cu);
    const C phi = e0 ? (C)e0[d] : (C)dv;
    const C psi = w0 ? (C)w0[d] : (C)cu;
    for (int b = 0; b < 2; b++) {
      CD::store_eq(s, b, 0, k, P, phi, C(0), C(0));
      CD::store_eq(s, b, 1, k, P, psi, C(0), C(0));
    }
  }
}

// Fields of one plate into dense FP64 device arrays (zero outside the body).
template <int ST>
__global__ void k_fields(DevState s, int plate, int b, double *e, double *w, double *u,
                         double *v) {
  using CD = typename CodecOf<ST>::type;
  using U = typename CD::U;
  const PlateDev P = s.plates[plate];
  const int64_t n = (int64_t)P.nx * P.ny;
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(d % P.nx), j = (int)(d / P.nx);
    const int64_t k = node_of(P, i, j);
    const bool in = (s.cls[k] & CL_IN) != 0;
    if (e) e[d] = in ? CD::field(s, b, 0, k, P) : 0.0;
    if (w) w[d] = in ? CD::field(s, b, 1, k, P) : 0.0;
    if (u) {
      u[d] = in ? (double)ldg<U>(s.u[b][0], k) : 0.0;
      u[n + d] = in ? (double)ldg<U>(s.u[b][1], k) : 0.0;
    }
    if (v) {
      v[d] = in ? (double)ldg<U>(s.v[b][0], k) : 0.0;
      v[n + d] = in ? (double)ldg<U>(s.v[b][1], k) : 0.0;
    }
  }
}

// --------------------------------------------------------------- launchers

template <int ST>
static hipError_t launch_interior_t(const DevState &s, const Tile *tiles, int ntiles, int lanes,
                                    int cur, hipStream_t st) {
  const int q = (ntiles + 7) / 8;
  const dim3 grid(8 * q);
  switch (lanes) {
    case 64:
      hipLaunchKernelGGL((k_interior<ST, 64>), grid, dim3(64), 0, st, s, tiles, ntiles, q, cur);
      break;
    case 128:
      hipLaunchKernelGGL((k_interior<ST, 128>), grid, dim3(128), 0, st, s, tiles, ntiles, q, cur);
      break;
    case 256:
      hipLaunchKernelGGL((k_interior<ST, 256>), grid, dim3(256), 0, st, s, tiles, ntiles, q, cur);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ST>
static hipError_t launch_sync_t(const DevState &s, const Tile *tiles, int ntiles, int lanes, int b,
                                hipStream_t st) {
  const int q = (ntiles + 7) / 8;
  const dim3 grid(8 * q);
  switch (lanes) {
    case 64:
      hipLaunchKernelGGL((k_sync<ST, 64>), grid, dim3(64), 0, st, s, tiles, ntiles, q, b);
      break;
    case 128:
      hipLaunchKernelGGL((k_sync<ST, 128>), grid, dim3(128), 0, st, s, tiles, ntiles, q, b);
      break;
    case 256:
      hipLaunchKernelGGL((k_sync<ST, 256>), grid, dim3(256), 0, st, s, tiles, ntiles, q, b);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define LBM_DISPATCH(st, CALL)                                   \
  switch (st) {                                                  \
    case LBM_STORE_F64: { constexpr int ST = LBM_STORE_F64; CALL; } break;       \
    case LBM_STORE_F32: { constexpr int ST = LBM_STORE_F32; CALL; } break;       \
    case LBM_STORE_F32DEV: { constexpr int ST = LBM_STORE_F32DEV; CALL; } break; \
    case LBM_STORE_F16DEV: { constexpr int ST = LBM_STORE_F16DEV; CALL; } break; \
    case LBM_STORE_BF16DEV: { constexpr int ST = LBM_STORE_BF16DEV; CALL; } break; \
    default: return hipErrorInvalidValue;                        \
  }

hipError_t launch_interior(int st, const DevState &s, const Tile *tiles, int ntiles, int lanes,
                           int cur, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  LBM_DISPATCH(st, return launch_interior_t<ST>(s, tiles, ntiles, lanes, cur, stream));
  return hipSuccess;
}

hipError_t launch_post(int st, const DevState &s, int nb, int ns, int cur, int do_bacc,
                       hipStream_t stream) {
  const int n = nb + ns;
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + 255) / 256);
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_post<ST>), grid, dim3(256), 0, stream, s, nb, ns, cur,
                                      do_bacc));
  return hipGetLastError();
}

hipError_t launch_bacc0(int st, const DevState &s, int nb, hipStream_t stream) {
  if (nb <= 0) return hipSuccess;
  const dim3 grid((nb + 255) / 256);
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_bacc0<ST>), grid, dim3(256), 0, stream, s, nb));
  return hipGetLastError();
}

hipError_t launch_sync(int st, const DevState &s, const Tile *tiles, int ntiles, int lanes, int b,
                       hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  LBM_DISPATCH(st, return launch_sync_t<ST>(s, tiles, ntiles, lanes, b, stream));
  return hipSuccess;
}

hipError_t launch_init(int st, const DevState &s, int plate, int64_t nodes, const double *u0,
                       const double *v0, const double *e0, const double *w0, hipStream_t stream) {
  int64_t blocks = (nodes + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_init_uv<ST>), dim3((unsigned)blocks), dim3(256), 0,
                                      stream, s, plate, u0, v0));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_init_pops<ST>), dim3((unsigned)blocks), dim3(256), 0,
                                      stream, s, plate, e0, w0));
  return hipGetLastError();
}

hipError_t launch_fields(int st, const DevState &s, int plate, int64_t nodes, int b, double *e,
                         double *w, double *u, double *v, hipStream_t stream) {
  int64_t blocks = (nodes + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_fields<ST>), dim3((unsigned)blocks), dim3(256), 0,
                                      stream, s, plate, b, e, w, u, v));
  return hipGetLastError();
}

}  // namespace lbm
