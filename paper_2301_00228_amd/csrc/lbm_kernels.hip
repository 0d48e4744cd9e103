// lbm_kernels.hip -- gfx950 kernels of the plane-strain LBM
// (Schlueter et al., arXiv 2301.00228).
//
// One time step is one launch of k_interior:
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
//              Workgroups whose tile or halo ring holds boundary or
//              second-row nodes first finish the previous step there (the
//              prologue): the boundary reset of eqs. psi_phi_at_bound and
//              correction-f, the second-row pull of eq. LBE_mod with the
//              time-averaged boundary populations, and the boundary
//              accelerations of eqs. acc_neumann / acc_dirichlet with their
//              Newmark update.  The latency of that work hides behind the
//              other workgroups' streaming.
//  k_boundary  the same boundary work for every boundary node, one block
//              per chunk of boundary nodes; it closes each run of steps (and
//              precedes every synchronization) so the state is complete.
//  k_sync      the synchronization of Sec. 3.2 every l steps.
//
// Populations, u and du/dt ping-pong through two buffers (a third holds the
// intermediate time level of two-step launches).  The march never writes
// boundary or second-row nodes: boundary nodes keep their populations of
// t_{n-1} in the previous buffer, which the prologue reads, and second-row
// nodes' pulls go to a small side buffer (two of them, by step parity) that
// the next step's boundary work completes.  Boundary nodes' u(t_{n+1}) is
// written one step ahead.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <mutex>

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

// 16-bit conversions for the stored non-equilibrium moments.
//
// x to BF16 by truncation after adding r (0 <= r < 2^16) below its last
// significand bit: with r uniform, x rounds away from zero with probability
// equal to its distance from the truncated value in ulps (the magnitude
// bits are linear in the value within a binade; a carry moves to the next
// binade as it should).  NaN stays NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_sr(float x, uint32_t r) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0x007fffffu) ? 0x40 : 0));
  return (uint16_t)((u + r) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ uint16_t f32_to_f16_rne(float x) {
  return __half_as_ushort(__float2half_rn(x));
}
__device__ __forceinline__ float f16_to_f32(uint16_t h) { return __half2float(__ushort_as_half(h)); }
// x to FP16 by adding r (0 <= r < 2^13) below the last significand bit of
// an FP16 normal number and clearing the FP32 bits below it: in the FP16
// normal range the result converts exactly, so x rounds away from zero
// with probability equal to its fraction of an ulp.  Below that range
// (|x| < 2^-14) the conversion rounds to nearest once more; infinity and
// NaN convert as they are.
__device__ __forceinline__ uint16_t f32_to_f16_sr(float x, uint32_t r) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return f32_to_f16_rne(x);
  return f32_to_f16_rne(__uint_as_float((u + r) & 0xffffe000u));
}

// 32 well-mixed bits from three words and a small tag: each word enters
// through a multiply by an odd constant, then the lowbias32 finalizer
// (C. Wellons, "Prospecting for hash functions", 2018).
__device__ __forceinline__ uint32_t rand_bits(uint32_t a, uint32_t b, uint32_t c, uint32_t tag) {
  uint32_t h = a * 0x9e3779b1u + b * 0x85ebca77u + c * 0xc2b2ae3du + tag * 0x27d4eb2fu;
  h ^= h >> 16;
  h *= 0x7feb352du;
  h ^= h >> 15;
  h *= 0x846ca68bu;
  h ^= h >> 16;
  return h;
}

template <class T>
__device__ __forceinline__ T ldg(const void *p, int64_t k) {
  return static_cast<const T *>(p)[k];
}
// Store; NT: a nontemporal store (data written once and not read again in
// the launch: the final state of a two-step pass).
template <class T, bool NT = false>
__device__ __forceinline__ void stg(void *p, int64_t k, T v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, static_cast<T *>(p) + k);
  else
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

// Post-collision populations f* = f - 2 (f - f_eq(f)) and zeroth moment of
// one field (eq. LBE with dt/tau = 2).
template <class C>
__device__ __forceinline__ void collide_populations(C a0, C a, const C f[5], C &rho, C fs[5]) {
  const C r = f[0] + ((f[1] + f[3]) + (f[2] + f[4]));
  const C jx = f[1] - f[3], jy = f[2] - f[4];
  C e[5];
  eq_populations<C>(a0, a, r, jx, jy, e);
#pragma unroll
  for (int q = 0; q < 5; q++) fs[q] = f[q] - C(2.0) * (f[q] - e[q]);
  rho = r;
}

// Plain populations, FP64 or FP32.
template <class T>
struct PopCodec {
  using C = T;
  using U = T;
  using Slot = T;  // raw stored word of one slot
  __device__ static void load_raw(const DevState &s, int b, int fl, int64_t k, Slot r[5]) {
#pragma unroll
    for (int q = 0; q < 5; q++) r[q] = ldg<T>(s.pop[b][fl][q], k);
  }
  __device__ static void raw_to_pops(const PlateDev &, int, const Slot r[5], C f[5]) {
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = r[q];
  }
  __device__ static void raw_flux(const Slot r[5], C &jx, C &jy) {
    jx = r[1] - r[3];
    jy = r[2] - r[4];
  }
  __device__ static C raw_rho(const Slot r[5]) { return r[0] + ((r[1] + r[3]) + (r[2] + r[4])); }
  // (a select of the two fields' values, not an index: fl may differ between
  // lanes, and an indexed plate record would have to live in scratch memory)
  __device__ static C aw(const PlateDev &P, int fl) { return (C)(fl ? P.a[1] : P.a[0]); }
  __device__ static C a0w(const PlateDev &P, int fl) { return (C)(fl ? P.a0[1] : P.a0[0]); }
  __device__ static void load(const DevState &s, int b, int fl, int64_t k, const PlateDev &,
                              C f[5]) {
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = ldg<T>(s.pop[b][fl][q], k);
  }
  template <bool NT = false>
  __device__ static void store(const DevState &s, int b, int fl, int64_t k, const PlateDev &,
                               const C f[5]) {
#pragma unroll
    for (int q = 0; q < 5; q++) stg<T, NT>(s.pop[b][fl][q], k, f[q]);
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
  // rho and f* of the stored populations r (eq. LBE)
  __device__ static void collide_raw(const PlateDev &P, int fl, const Slot r[5], C &rho,
                                     C fs[5]) {
    collide_populations<C>(a0w(P, fl), aw(P, fl), r, rho, fs);
  }
  // rho and f* of populations f as a store and a load would return them
  // (plain storage keeps them exactly)
  __device__ static void collide_stored(const PlateDev &P, int fl, const C f[5], C &rho,
                                        C fs[5]) {
    collide_populations<C>(a0w(P, fl), aw(P, fl), f, rho, fs);
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
  using Slot = uint32_t;  // raw stored word of one slot
  __device__ static C aw(const PlateDev &P, int fl) { return fl ? P.af[1] : P.af[0]; }
  __device__ static C a0w(const PlateDev &P, int fl) { return fl ? P.a0f[1] : P.a0f[0]; }
  __device__ static float scale(const PlateDev &P, int fl) { return fl ? P.scale[1] : P.scale[0]; }
  __device__ static float iscale(const PlateDev &P, int fl) {
    return fl ? P.iscale[1] : P.iscale[0];
  }
  __device__ static void unpack(uint32_t w, const PlateDev &P, int fl, float &n, float &d) {
    const uint16_t lo = (uint16_t)(w & 0xffffu), hi = (uint16_t)(w >> 16);
    if (H == 1) {
      n = f16_to_f32(lo) * iscale(P, fl);
      d = f16_to_f32(hi) * iscale(P, fl);
    } else {
      n = bf16_to_f32(lo) * iscale(P, fl);
      d = bf16_to_f32(hi) * iscale(P, fl);
    }
  }
  // N = m[3] and D = m[4] in the 16-bit type, rounded stochastically:
  // each value rounds away from zero with probability equal to its fraction
  // of an ulp, so the rounding errors are unbiased and uncorrelated from
  // step to step (round-to-nearest leaves nearly the same error on a slowly
  // varying moment step after step, and those errors add up).  The random
  // bits are a hash of the node's stored rho and J, whose low bits change
  // from step to step, so the stored state stays a function of the state
  // it comes from (every tiling and launch shape gives the same bits).
  __device__ static uint32_t pack(const float m[5], const PlateDev &P, int fl) {
    const float sn = m[3] * scale(P, fl), sd = m[4] * scale(P, fl);
    uint16_t lo, hi;
    const uint32_t r = rand_bits(__float_as_uint(m[0]), __float_as_uint(m[1]),
                                 __float_as_uint(m[2]), (uint32_t)fl);
    if (H == 1) {
      lo = f32_to_f16_sr(sn, r & 0x1fffu);
      hi = f32_to_f16_sr(sd, (r >> 16) & 0x1fffu);
    } else {
      lo = f32_to_bf16_sr(sn, r & 0xffffu);
      hi = f32_to_bf16_sr(sd, r >> 16);
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
  __device__ static void load_raw(const DevState &s, int b, int fl, int64_t k, Slot r[5]) {
    r[0] = ldg<uint32_t>(s.pop[b][fl][0], k);
    r[1] = ldg<uint32_t>(s.pop[b][fl][1], k);
    r[2] = ldg<uint32_t>(s.pop[b][fl][2], k);
    r[3] = ldg<uint32_t>(s.pop[b][fl][3], k);
    r[4] = H == 0 ? ldg<uint32_t>(s.pop[b][fl][4], k) : 0u;
  }
  __device__ static void raw_flux(const Slot r[5], C &jx, C &jy) {
    jx = __uint_as_float(r[1]);
    jy = __uint_as_float(r[2]);
  }
  __device__ static C raw_rho(const Slot r[5]) { return __uint_as_float(r[0]); }
  __device__ static void raw_to_pops(const PlateDev &P, int fl, const Slot r[5], C f[5]) {
    float m[5];
    m[0] = __uint_as_float(r[0]);
    m[1] = __uint_as_float(r[1]);
    m[2] = __uint_as_float(r[2]);
    if (H == 0) {
      m[3] = __uint_as_float(r[3]);
      m[4] = __uint_as_float(r[4]);
    } else {
      unpack(r[3], P, fl, m[3], m[4]);
    }
    moments_to_pops(P, fl, m, f);
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
  template <bool NT = false>
  __device__ static void store_moments(const DevState &s, int b, int fl, int64_t k,
                                       const PlateDev &P, const float m[5]) {
    stg<float, NT>(s.pop[b][fl][0], k, m[0]);
    stg<float, NT>(s.pop[b][fl][1], k, m[1]);
    stg<float, NT>(s.pop[b][fl][2], k, m[2]);
    if (H == 0) {
      stg<float, NT>(s.pop[b][fl][3], k, m[3]);
      stg<float, NT>(s.pop[b][fl][4], k, m[4]);
    } else {
      stg<uint32_t, NT>(s.pop[b][fl][3], k, pack(m, P, fl));
    }
  }
  template <bool NT = false>
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
    store_moments<NT>(s, b, fl, k, P, m);
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
  // The collision in the moment basis: rho and J are kept and the two
  // non-equilibrium moments N and D change sign (f* = 2 f_eq - f with
  // f_eq of rho and J, eq. LBE with dt/tau = 2), so rho is conserved
  // exactly whatever the rounding of the weights.
  __device__ static void post_collision(const PlateDev &P, int fl, const float m[5], C &rho,
                                        C fs[5]) {
    const float mc[5] = {m[0], m[1], m[2], -m[3], -m[4]};
    moments_to_pops(P, fl, mc, fs);
    rho = m[0];
  }
  // rho and f* of the stored moments r
  __device__ static void collide_raw(const PlateDev &P, int fl, const Slot r[5], C &rho,
                                     C fs[5]) {
    float m[5];
    m[0] = __uint_as_float(r[0]);
    m[1] = __uint_as_float(r[1]);
    m[2] = __uint_as_float(r[2]);
    if (H == 0) {
      m[3] = __uint_as_float(r[3]);
      m[4] = __uint_as_float(r[4]);
    } else {
      unpack(r[3], P, fl, m[3], m[4]);
    }
    post_collision(P, fl, m, rho, fs);
  }
  // rho and f* of populations f as store() followed by a load returns them:
  // the same moments and rounding, without the memory
  __device__ static void collide_stored(const PlateDev &P, int fl, const C f[5], C &rho,
                                        C fs[5]) {
    const float s13 = f[1] + f[3], s24 = f[2] + f[4];
    const float q = s13 + s24;
    float m[5];
    m[0] = f[0] + q;
    m[1] = f[1] - f[3];
    m[2] = f[2] - f[4];
    m[3] = s13 - s24;
    m[4] = q - 4.0f * aw(P, fl) * m[0];
    if (H != 0) unpack(pack(m, P, fl), P, fl, m[3], m[4]);
    post_collision(P, fl, m, rho, fs);
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

// Collision of populations that are not a stored state (the averaged
// populations of the second-row rule).
template <class CD>
__device__ __forceinline__ void collide_pops(const PlateDev &P, int fl, const typename CD::C f[5],
                                             typename CD::C &rho, typename CD::C fs[5]) {
  collide_populations<typename CD::C>(CD::a0w(P, fl), CD::aw(P, fl), f, rho, fs);
}

// ------------------------------------------- boundary / second-row work

// Finite difference with a precomputed stencil code from the node's value
// q0 and the values qa, qb of the further stencil nodes, branch-free:
// ((c0 q0 + ca qa) + cb qb) * scale with the coefficients of the code
// (central: qa - qb, one-sided 3-point: (-3 q0 + 4 qa) - qb and its mirror,
// 2-point: qa - q0 and q0 - qa; these sums round exactly as the written-out
// formulas); scale is 1/(2 dh) or 1/dh.
template <class U>
__device__ __forceinline__ U fd_vals(int code, U q0, U qa, U qb, const PlateDev &P) {
  const bool cen = code == FD_CENTRAL, f3 = code == FD_FWD3, b3 = code == FD_BWD3;
  const bool f2 = code == FD_FWD2, b2 = code == FD_BWD2;
  const U c0 = f3 ? U(-3.0) : b3 ? U(3.0) : f2 ? U(-1.0) : b2 ? U(1.0) : U(0.0);
  const U ca = (cen || f2) ? U(1.0) : f3 ? U(4.0) : b3 ? U(-4.0) : b2 ? U(-1.0) : U(0.0);
  const U cb = (cen || f3) ? U(-1.0) : b3 ? U(1.0) : U(0.0);
  const U sc = (f2 || b2) ? (U)P.inv_h : (cen || f3 || b3) ? (U)P.inv_2h : U(0.0);
  return ((c0 * q0 + ca * qa) + cb * qb) * sc;
}

// Further stencil nodes a and b of a finite difference with code `code`
// along axis ax at node (i, j) (the node k0 itself where the stencil has no
// such node).  Every index touched lies in the body (the code was built from
// the mask).
__device__ __forceinline__ void fd_nodes(const PlateDev &P, int i, int j, int ax, int code,
                                         int64_t k0, int64_t &ka, int64_t &kb) {
  const int di = ax == 0 ? 1 : 0, dj = ax == 0 ? 0 : 1;
  ka = k0;
  kb = k0;
  if (code == FD_CENTRAL || code == FD_FWD3 || code == FD_FWD2) {
    const int ip = wrapc(i + di, P.nx), jp = wrapc(j + dj, P.ny);
    ka = node_of(P, ip, jp);
    if (code == FD_CENTRAL) kb = node_of(P, wrapc(i - di, P.nx), wrapc(j - dj, P.ny));
    if (code == FD_FWD3) kb = node_of(P, wrapc(ip + di, P.nx), wrapc(jp + dj, P.ny));
  } else if (code == FD_BWD3 || code == FD_BWD2) {
    const int im = wrapc(i - di, P.nx), jm = wrapc(j - dj, P.ny);
    ka = node_of(P, im, jm);
    if (code == FD_BWD3) kb = node_of(P, wrapc(im - di, P.nx), wrapc(jm - dj, P.ny));
  }
}

// The values of q that the finite differences along x (code cx) and y
// (code cy) at node (i, j) combine, read straight from q: v[0] at the node,
// v[1], v[2] the x stencil's nodes a, b, v[3], v[4] the y stencil's (fd_vals
// of (v[0], v[1], v[2]) is d/dx, of (v[0], v[3], v[4]) d/dy).
template <class U>
__device__ __forceinline__ void fd_stencil_values(const U *q, const PlateDev &P, int i, int j,
                                                  int cx, int cy, U v[5]) {
  const int64_t k0 = node_of(P, i, j);
  int64_t xa, xb, ya, yb;
  fd_nodes(P, i, j, 0, cx, k0, xa, xb);
  fd_nodes(P, i, j, 1, cy, k0, ya, yb);
  v[0] = q[k0];
  v[1] = q[xa];
  v[2] = q[xb];
  v[3] = q[ya];
  v[4] = q[yb];
}

// Hooke's law (Sec. 2, eq. hooke) from a displacement gradient
// g = (d_x u_x, d_y u_x, d_x u_y, d_y u_y).
template <class U>
__device__ __forceinline__ void hooke(const PlateDev &P, const U *g, U &sxx, U &syy, U &sxy) {
  const U exx = g[0], eyy = g[3];
  const U exy = U(0.5) * (g[1] + g[2]);
  const U tr = exx + eyy;
  const U lam = (U)P.lam, mu = (U)P.mu;
  sxx = lam * tr + U(2.0) * mu * exx;
  syy = lam * tr + U(2.0) * mu * eyy;
  sxy = U(2.0) * mu * exy;
}

// Flux of eq. correction-f under reading R2 at boundary node (i, j) with
// class byte cl, field fl: the first moment (lattice units) of the
// post-collision populations (eq. LBE, dt/tau = 2) that the LBE would
// stream into the node at t from its body neighbours x - c^alpha, their
// populations at t - dt being in buffer po (those neighbours are boundary
// or second-row nodes, whose populations the march never overwrites); a
// missing neighbour contributes 0.
template <class CD>
__device__ void streamed_in_flux(const DevState &s, const PlateDev &P, int i, int j, uint8_t cl,
                                 int fl, int po, typename CD::C &jx, typename CD::C &jy) {
  using C = typename CD::C;
  using Slot = typename CD::Slot;
  // population alpha arrives from x - c^alpha: 1 from W, 2 from S, 3 from E,
  // 4 from N (one neighbour at a time)
  C sx = C(0), sy = C(0);
#pragma unroll 1
  for (int al = 1; al < 5; al++) {
    const int di = (al == 1) - (al == 3), dj = (al == 2) - (al == 4);
    const uint8_t from = al == 1 ? NB_W : al == 2 ? NB_S : al == 3 ? NB_E : NB_N;
    if (!(cl & from)) continue;
    const int64_t ky = node_of(P, wrapc(i - di, P.nx), wrapc(j - dj, P.ny));
    Slot r[5];
    CD::load_raw(s, po, fl, ky, r);
    C rho, fs[5];
    CD::collide_raw(P, fl, r, rho, fs);
    // fs[al] (a select, not a dynamic index into a local array)
    const C g = al == 1 ? fs[1] : al == 2 ? fs[2] : al == 3 ? fs[3] : fs[4];
    if (di != 0) sx += C(di) * g;
    if (dj != 0) sy += C(dj) * g;
  }
  jx = sx;
  jy = sy;
}

// Inputs of one boundary task read from memory: the flux of eq.
// correction-f of both fields and u, du/dt at t.
template <class CD>
struct BoundaryIn {
  typename CD::C jx[2], jy[2];
  typename CD::U ux, uy, vx, vy;
};

// The reads of one boundary task (see boundary_task): the flux from the
// populations at t - dt in buffer po (reading R1, or R2 for variant
// contexts) if reset, u and du/dt from buffer ua if accel.  Kept apart from
// the arithmetic so that a caller can issue them early.
template <class CD, bool VAR>
__device__ __forceinline__ void boundary_load(const DevState &s, const PlateDev &P, const BTask &T,
                                              int po, bool reset, bool accel, int ua,
                                              BoundaryIn<CD> &in) {
  using U = typename CD::U;
  const BndNode &B = T.b;
  const int64_t k = B.node;
  if (reset) {
    if (VAR && (P.readings & RD_FLUX_STREAMED)) {
      const uint8_t cl = s.cls[k];
      streamed_in_flux<CD>(s, P, B.i, B.j, cl, 0, po, in.jx[0], in.jy[0]);
      streamed_in_flux<CD>(s, P, B.i, B.j, cl, 1, po, in.jx[1], in.jy[1]);
    } else {
      CD::flux(s, po, 0, k, P, in.jx[0], in.jy[0]);
      CD::flux(s, po, 1, k, P, in.jx[1], in.jy[1]);
    }
  }
  if (accel) {
    in.ux = ldg<U>(s.u[ua][0], k);
    in.uy = ldg<U>(s.u[ua][1], k);
    in.vx = ldg<U>(s.v[ua][0], k);
    in.vy = ldg<U>(s.v[ua][1], k);
  }
}

// One boundary node.  grad: rows of 4 gradient values (d_x u_x, d_y u_x,
// d_x u_y, d_y u_y) of u at time t, indexed by the task's g[].
//  reset (eqs. psi_phi_at_bound, correction-f): populations at t from the
//    field div u / (curl u).e_z and the flux in `in`, written to buffer pn;
//  accel (eq. acc_dirichlet or eq. acc_neumann, step n with loads at n dt /
//    (n+1) dt): from u, du/dt at t in `in`, Newmark update (eq.
//    integration) into buffer ub (and ub2 if >= 0).
template <class CD>
__device__ __forceinline__ void boundary_finish(const DevState &s, const PlateDev &P, const BTask &T,
                                const typename CD::U *grad, const BoundaryIn<CD> &in, int pn,
                                bool reset, bool accel, int ub, int ub2, unsigned long long n) {
  using C = typename CD::C;
  using U = typename CD::U;
  const BndNode &B = T.b;
  const int64_t k = B.node;
  const U *gs = grad + 4 * T.g[0];
  if (reset) {
    const U dv = gs[0] + gs[3];
    const U cu = gs[2] - gs[1];
    CD::store_eq(s, pn, 0, k, P, (C)dv, in.jx[0], in.jy[0]);
    CD::store_eq(s, pn, 1, k, P, (C)cu, in.jx[1], in.jy[1]);
  }
  if (!accel) return;
  const U ux0 = in.ux, uy0 = in.uy, vx0 = in.vx, vy0 = in.vy;
  const U dt = (U)P.dt;
  U ax, ay;
  if (B.kind == LBM_BC_DIRICHLET) {
    const double g = load_amp(s, B.load, (double)(n + 1) * P.dt);
    const U usx = (U)(g * B.val[0]), usy = (U)(g * B.val[1]);
    // the acceleration that makes u(t + dt) = u* under the update in use
    if (P.integ && n != 0) {
      ax = (usx - ux0) / (dt * dt) - vx0 / dt;
      ay = (usy - uy0) / (dt * dt) - vy0 / dt;
    } else {
      ax = U(2.0) / (dt * dt) * (usx - ux0) - U(2.0) / dt * vx0;
      ay = U(2.0) / (dt * dt) * (usy - uy0) - U(2.0) / dt * vy0;
    }
  } else {
    const double g = load_amp(s, B.load, (double)n * P.dt);
    const U V = (U)B.cell[0], lE = (U)B.cell[1], lN = (U)B.cell[2], lW = (U)B.cell[3],
            lS = (U)B.cell[4];
    U sxx, syy, sxy, rxx, ryy, rxy;
    hooke<U>(P, gs, sxx, syy, sxy);
    U tEx = 0, tEy = 0, tWx = 0, tWy = 0, tNx = 0, tNy = 0, tSx = 0, tSy = 0;
    // sigma_kr n_kr l_kr with sigma_kr the mean of the nodal stresses
    if (T.g[1] >= 0) {
      hooke<U>(P, grad + 4 * T.g[1], rxx, ryy, rxy);
      tEx = U(0.5) * (sxx + rxx) * lE;
      tEy = U(0.5) * (sxy + rxy) * lE;
    }
    if (T.g[3] >= 0) {
      hooke<U>(P, grad + 4 * T.g[3], rxx, ryy, rxy);
      tWx = -(U(0.5) * (sxx + rxx)) * lW;
      tWy = -(U(0.5) * (sxy + rxy)) * lW;
    }
    if (T.g[2] >= 0) {
      hooke<U>(P, grad + 4 * T.g[2], rxx, ryy, rxy);
      tNx = U(0.5) * (sxy + rxy) * lN;
      tNy = U(0.5) * (syy + ryy) * lN;
    }
    if (T.g[4] >= 0) {
      hooke<U>(P, grad + 4 * T.g[4], rxx, ryy, rxy);
      tSx = -(U(0.5) * (sxy + rxy)) * lS;
      tSy = -(U(0.5) * (syy + ryy)) * lS;
    }
    const U Fx = (U)(g * B.val[0]), Fy = (U)(g * B.val[1]);
    const U m = (U)P.rho_m * V;
    ax = (((tEx + tWx) + (tNx + tSx)) + Fx) / m;
    ay = (((tEy + tWy) + (tNy + tSy)) + Fy) / m;
  }
  U nux, nuy, nvx, nvy;
  newmark<U>(P, kick_of<U>(P, n == 0), ax, ay, ux0, uy0, vx0, vy0, nux, nuy, nvx, nvy);
  stg<U>(s.u[ub][0], k, nux);
  stg<U>(s.u[ub][1], k, nuy);
  stg<U>(s.v[ub][0], k, nvx);
  stg<U>(s.v[ub][1], k, nvy);
  if (ub2 >= 0) {
    stg<U>(s.u[ub2][0], k, nux);
    stg<U>(s.u[ub2][1], k, nuy);
    stg<U>(s.v[ub2][0], k, nvx);
    stg<U>(s.v[ub2][1], k, nvy);
  }
  if (!(fabs((double)nux) < 1e30) || !(fabs((double)nuy) < 1e30)) s.flag[0] = 1;
}

// One boundary node's reset and acceleration (reads from buffers po and ua,
// writes to pn, ub, ub2; see boundary_load and boundary_finish).
template <class CD, bool VAR>
__device__ void boundary_task(const DevState &s, const PlateDev &P, const BTask &T,
                              const typename CD::U *grad, int po, int pn, bool reset, bool accel,
                              int ua, int ub, int ub2, unsigned long long n) {
  BoundaryIn<CD> in;
  boundary_load<CD, VAR>(s, P, T, po, reset, accel, ua, in);
  boundary_finish<CD>(s, P, T, grad, in, pn, reset, accel, ub, ub2, n);
}

// Population AL that second-row node Q pulls from its upwind boundary node
// y = x - c^AL by eq. LBE_mod under the plate's readings (used when they are
// not R1 + M1): the average of y's populations at t - dt (buffer po) and of
// their reset values at t (field from grad, flux of eq. correction-f by
// reading R1 or R2), collided towards the equilibrium of its own moments (M1)
// or of y's populations at t - dt (M2).
template <class CD, int AL>
__device__ typename CD::C pull_from_boundary(const DevState &s, const PlateDev &P, const STask &Q,
                                             int fl, const typename CD::U *grad, int po) {
  using C = typename CD::C;
  using U = typename CD::U;
  using Slot = typename CD::Slot;
  constexpr int di = (AL == 1) - (AL == 3), dj = (AL == 2) - (AL == 4);
  const int yi = wrapc(Q.i - di, P.nx), yj = wrapc(Q.j - dj, P.ny);
  const int64_t ky = node_of(P, yi, yj);
  Slot raw[5];
  CD::load_raw(s, po, fl, ky, raw);
  const U *gy = grad + 4 * Q.g[AL];
  const C fld = fl == 0 ? (C)(gy[0] + gy[3]) : (C)(gy[2] - gy[1]);
  C jx, jy, f[5], fnew[5];
  if (P.readings & RD_FLUX_STREAMED)
    streamed_in_flux<CD>(s, P, yi, yj, s.cls[ky], fl, po, jx, jy);
  else
    CD::raw_flux(raw, jx, jy);
  CD::eq_pops(P, fl, fld, jx, jy, fnew);
  CD::raw_to_pops(P, fl, raw, f);
#pragma unroll
  for (int q = 0; q < 5; q++) f[q] = C(0.5) * (fnew[q] + f[q]);
  if (P.readings & RD_EQ_OLD) {
    // f~ - 2 (f~ - f_eq(rho, J of the populations at t - dt))
    C jox, joy, e[5];
    CD::raw_flux(raw, jox, joy);
    CD::eq_pops(P, fl, CD::raw_rho(raw), jox, joy, e);
    return f[AL] - C(2.0) * (f[AL] - e[AL]);
  }
  C r, fs[5];
  collide_pops<CD>(P, fl, f, r, fs);
  return fs[AL];
}

// Inputs of one field of one second-row task read from memory (readings
// R1 and M1): the side buffer's pulls and the stored state at t - dt of its
// first upwind boundary node (direction a1, 0 if none).
template <class CD>
struct SecondRowIn {
  typename CD::C fo[5];
  typename CD::Slot raw[5];
  int a1;
};

template <class CD>
__device__ __forceinline__ void second_row_load(const DevState &s, const PlateDev &P,
                                                const STask &Q, int fl, int po, int sr,
                                                SecondRowIn<CD> &in) {
  using C = typename CD::C;
  const C *side = static_cast<const C *>(s.side[sr]);
#pragma unroll
  for (int al = 0; al < 5; al++) in.fo[al] = side[(int64_t)(fl * 5 + al) * s.nsec + Q.si];
  in.a1 = Q.g[1] >= 0 ? 1 : Q.g[2] >= 0 ? 2 : Q.g[3] >= 0 ? 3 : Q.g[4] >= 0 ? 4 : 0;
  if (in.a1 != 0) {
    const int di = (in.a1 == 1) - (in.a1 == 3), dj = (in.a1 == 2) - (in.a1 == 4);
    const int64_t ky = node_of(P, wrapc(Q.i - di, P.nx), wrapc(Q.j - dj, P.ny));
    CD::load_raw(s, po, fl, ky, in.raw);
  }
}

// One field of one second-row node: its populations at t, pulled from the
// upwind nodes at t - dt.  Those pulled from non-boundary upwind nodes were
// left in the side buffer by the march of the previous step (in.fo); one
// leaving a boundary node follows eq. LBE_mod: the average of the boundary
// node's populations at t - dt (buffer po; in.raw for the first such node)
// and of their reset values at t (field from grad, flux of eq. correction-f
// by reading R1: that of the populations at t - dt), collided with the
// equilibrium of their own moments (reading M1).  Written to buffer pn.
template <class CD>
__device__ __forceinline__ void second_row_finish(const DevState &s, const PlateDev &P, const STask &Q, int fl,
                                  const typename CD::U *grad, int po, int pn,
                                  const SecondRowIn<CD> &in) {
  using C = typename CD::C;
  using U = typename CD::U;
  using Slot = typename CD::Slot;
  C fo[5];
#pragma unroll
  for (int al = 0; al < 5; al++) fo[al] = in.fo[al];
#pragma unroll
  for (int al = 1; al < 5; al++) {
    if (Q.g[al] < 0) continue;
    Slot raw[5];
    if (al == in.a1) {
#pragma unroll
      for (int q = 0; q < 5; q++) raw[q] = in.raw[q];
    } else {
      // a further upwind boundary node (a corner)
      const int di = (al == 1) - (al == 3), dj = (al == 2) - (al == 4);
      const int64_t ky = node_of(P, wrapc(Q.i - di, P.nx), wrapc(Q.j - dj, P.ny));
      CD::load_raw(s, po, fl, ky, raw);
    }
    C f[5], r, fs[5];
    CD::raw_to_pops(P, fl, raw, f);
    const U *gy = grad + 4 * Q.g[al];
    const C fld = fl == 0 ? (C)(gy[0] + gy[3]) : (C)(gy[2] - gy[1]);
    C fnew[5], jx, jy;
    CD::raw_flux(raw, jx, jy);
    CD::eq_pops(P, fl, fld, jx, jy, fnew);
#pragma unroll
    for (int qq = 0; qq < 5; qq++) f[qq] = C(0.5) * (fnew[qq] + f[qq]);
    collide_pops<CD>(P, fl, f, r, fs);
    fo[al] = fs[al];
  }
  CD::store(s, pn, fl, Q.node, P, fo);
}

// One field of one second-row node under the plate's readings (buffers po,
// pn, side buffer sr): R1 and M1 by second_row_load and second_row_finish;
// the variant readings (VAR contexts only) through pull_from_boundary.
template <class CD, bool VAR>
__device__ void second_row_task(const DevState &s, const PlateDev &P, const STask &Q, int fl,
                                const typename CD::U *grad, int po, int pn, int sr) {
  using C = typename CD::C;
  if (VAR && P.readings != 0) {
    const C *side = static_cast<const C *>(s.side[sr]);
    C fo[5];
#pragma unroll
    for (int al = 0; al < 5; al++) fo[al] = side[(int64_t)(fl * 5 + al) * s.nsec + Q.si];
    if (Q.g[1] >= 0) fo[1] = pull_from_boundary<CD, 1>(s, P, Q, fl, grad, po);
    if (Q.g[2] >= 0) fo[2] = pull_from_boundary<CD, 2>(s, P, Q, fl, grad, po);
    if (Q.g[3] >= 0) fo[3] = pull_from_boundary<CD, 3>(s, P, Q, fl, grad, po);
    if (Q.g[4] >= 0) fo[4] = pull_from_boundary<CD, 4>(s, P, Q, fl, grad, po);
    CD::store(s, pn, fl, Q.node, P, fo);
    return;
  }
  SecondRowIn<CD> in;
  second_row_load<CD>(s, P, Q, fl, po, sr, in);
  second_row_finish<CD>(s, P, Q, fl, grad, po, pn, in);
}

// Prologue of an interior tile at step n (buffers sb): the boundary work
// (readings R1 and M1 only: contexts with other readings run every step's
// boundary work in k_boundary) of step n - 1 for the boundary and
// second-row nodes of the tile and its
// halo ring (resets and pulls into buffer sb.in, which the march then reads,
// from the populations of t_{n-1} in buffer sb.prev and the side buffer
// sb.sp) and the next boundary accelerations of the tile's own boundary
// nodes (u buffer sb.in to sb.out).  Gradients of u(t_n) go to LDS (lds,
// lds_bytes: the march's exchange buffer, unused until the march starts) if
// they fit, else to a per-tile scratch area in global memory.  `plate` is
// the tile's plate (the chunk's).
//
// The prologue is a chain of dependent memory reads on a tile's critical
// path.  Each lane's first gradient node, boundary task and second-row task
// therefore read their records first and then all their inputs (stencil
// values of u, the flux and u, du/dt of the boundary node, the side-buffer
// pulls and the first upwind boundary node's state) before any of them is
// used, so that the chain is records -> inputs -> barrier -> arithmetic and
// stores; further items (lists longer than the workgroup) follow one by one.
template <class CD>
__device__ void prologue(const DevState &s, const Prologue &pro, int chunk, int plate,
                         const StepBufs &sb, int tid, int nthreads, void *lds, int lds_bytes) {
  using U = typename CD::U;
  const TileChunk ch = pro.chunks[chunk];
  const PlateDev P = s.plates[plate];
  const bool in_lds = (int64_t)(ch.g1 - ch.g0) * 4 * (int64_t)sizeof(U) <= (int64_t)lds_bytes;
  U *grad = in_lds ? static_cast<U *>(lds) : static_cast<U *>(pro.grad) + (int64_t)4 * ch.g0;
  const U *ux = static_cast<const U *>(s.u[sb.in][0]);
  const U *uy = static_cast<const U *>(s.u[sb.in][1]);
  const unsigned long long n = s.counter[sb.in];
  const int nst = 2 * (ch.s1 - ch.s0);
  const int g = ch.g0 + tid, b = ch.b0 + tid;
  const bool hg = g < ch.g1, hb = b < ch.b1, hs = tid < nst;
  TGradNode G{};
  BTask T{};
  STask Q{};
  if (hg) G = pro.gn[g];
  if (hb) T = pro.bt[b];
  if (hs) Q = pro.st[ch.s0 + (tid >> 1)];
  U gu[2][5];
  if (hg) {
    const int cx = G.code & 7, cy = (G.code >> 3) & 7;
    fd_stencil_values<U>(ux, P, G.i, G.j, cx, cy, gu[0]);
    fd_stencil_values<U>(uy, P, G.i, G.j, cx, cy, gu[1]);
  }
  BoundaryIn<CD> bin;
  if (hb) boundary_load<CD, false>(s, P, T, sb.prev, true, T.accel != 0, sb.in, bin);
  SecondRowIn<CD> sin;
  if (hs) second_row_load<CD>(s, P, Q, tid & 1, sb.prev, sb.sp, sin);
  for (int g2 = g; g2 < ch.g1; g2 += nthreads) {
    if (g2 != g) {
      G = pro.gn[g2];
      const int cx = G.code & 7, cy = (G.code >> 3) & 7;
      fd_stencil_values<U>(ux, P, G.i, G.j, cx, cy, gu[0]);
      fd_stencil_values<U>(uy, P, G.i, G.j, cx, cy, gu[1]);
    }
    const int cx = G.code & 7, cy = (G.code >> 3) & 7;
    U *d = grad + 4 * (g2 - ch.g0);
    d[0] = fd_vals<U>(cx, gu[0][0], gu[0][1], gu[0][2], P);
    d[1] = fd_vals<U>(cy, gu[0][0], gu[0][3], gu[0][4], P);
    d[2] = fd_vals<U>(cx, gu[1][0], gu[1][1], gu[1][2], P);
    d[3] = fd_vals<U>(cy, gu[1][0], gu[1][3], gu[1][4], P);
  }
  __syncthreads();
  for (int b2 = b; b2 < ch.b1; b2 += nthreads) {
    if (b2 != b) {
      T = pro.bt[b2];
      boundary_load<CD, false>(s, P, T, sb.prev, true, T.accel != 0, sb.in, bin);
    }
    boundary_finish<CD>(s, P, T, grad, bin, sb.in, true, T.accel != 0, sb.out, -1, n);
  }
  for (int t = tid; t < nst; t += nthreads) {
    if (t != tid) {
      Q = pro.st[ch.s0 + (t >> 1)];
      second_row_load<CD>(s, P, Q, t & 1, sb.prev, sb.sp, sin);
    }
    second_row_finish<CD>(s, P, Q, t & 1, grad, sb.prev, sb.in, sin);
  }
  __syncthreads();
}

// Boundary work of step n - 1 for every boundary node, one block per chunk
// of boundary nodes (all of one plate): the same work as the prologues of
// step n.  The state of t_n is in buffer bc, the boundary populations of
// t_{n-1} in bp, the second-row pulls in side[sr].  Phase 1 puts u(t_n) of
// every node the chunk's stencils touch into LDS, phase 2 the
// finite-difference gradients; phase 3 runs the boundary tasks (reset into
// buffer bc if do_reset; acceleration into u buffer ub, and ub2 if >= 0) and,
// if do_reset, the second-row tasks (one field per thread).
template <int ST>
__global__ void __launch_bounds__(kBoundaryThreads)
    k_boundary(DevState s, const Chunk *__restrict__ chunks, const UNode *__restrict__ un,
               const GradNode *__restrict__ gn, const BTask *__restrict__ btask,
               const STask *__restrict__ stask, int bc, int bp, int ub, int ub2, int sr,
               int do_reset) {
  using CD = typename CodecOf<ST>::type;
  using U = typename CD::U;
  __shared__ U uu[kMaxU][2];
  __shared__ U grad[kMaxGrad][4];
  const Chunk ch = chunks[blockIdx.x];
  const PlateDev P = s.plates[ch.plate];
  const int tid = threadIdx.x;
  for (int g = ch.u0 + tid; g < ch.u1; g += kBoundaryThreads) {
    const int64_t k = un[g].node;
    uu[g - ch.u0][0] = ldg<U>(s.u[bc][0], k);
    uu[g - ch.u0][1] = ldg<U>(s.u[bc][1], k);
  }
  __syncthreads();
  for (int g = ch.g0 + tid; g < ch.g1; g += kBoundaryThreads) {
    const GradNode G = gn[g];
    const int cx = G.code & 7, cy = (G.code >> 3) & 7;
    U *d = grad[g - ch.g0];
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const U q0 = uu[G.u[0]][c];
      d[2 * c + 0] = fd_vals<U>(cx, q0, uu[G.u[1]][c], uu[G.u[2]][c], P);
      d[2 * c + 1] = fd_vals<U>(cy, q0, uu[G.u[3]][c], uu[G.u[4]][c], P);
    }
  }
  __syncthreads();
  const unsigned long long n = s.counter[bc];
  const int nb = ch.b1 - ch.b0;
  if (tid < nb) {
    const BTask T = btask[ch.b0 + tid];
    boundary_task<CD, true>(s, P, T, &grad[0][0], bp, bc, do_reset != 0, true, bc, ub, ub2, n);
  } else if (do_reset) {
    const int t = tid - nb;
    if (ch.s0 + (t >> 1) < ch.s1)
      second_row_task<CD, true>(s, P, stask[ch.s0 + (t >> 1)], t & 1, &grad[0][0], bp, bc, sr);
  }
}

// Displacement update of step n from u, v and the acceleration a at t_n,
// as u += dt v + m a, v += k a with step coefficients (k, m):
// integ 0, eq. integration as printed: k = dt, m = dt^2/2.
// integ 1, central difference (Newmark gamma = 1/2, beta = 0) in
// half-step form (v kept at t - dt/2: v += dt a, then u += dt v): k = dt,
// m = dt^2; the first step (n = 0, v given at t = 0) takes half the velocity
// increment, k = dt/2, m = dt^2/2, which gives the same u(t_1) as the
// printed update.  The coefficients are uniform over a launch.
template <class U>
struct Kick {
  U k, m;
};
template <class U>
__device__ __forceinline__ Kick<U> kick_of(const PlateDev &P, bool first) {
  const U dt = (U)P.dt;
  if (P.integ) {
    const U k = first ? U(0.5) * dt : dt;
    return {k, dt * k};
  }
  return {dt, dt * dt / U(2.0)};
}
template <class U>
__device__ __forceinline__ void newmark(const PlateDev &P, const Kick<U> &K, U ax, U ay, U ux,
                                        U uy, U vx, U vy, U &nux, U &nuy, U &nvx, U &nvy) {
  const U dt = (U)P.dt;
  nux = ux + dt * vx + K.m * ax;
  nuy = uy + dt * vy + K.m * ay;
  nvx = vx + K.k * ax;
  nvy = vy + K.k * ay;
}

// Interior acceleration of eq. navier, c_d^2 grad phi - c_s^2 curl(psi e_z)
// with curl(psi e_z) = (d_y psi, -d_x psi) and central differences of the
// neighbours' zeroth moments (E, W, N, S; field 0 = phi, 1 = psi), followed
// by the displacement update with coefficients K.  Shared by the interior kernel
// and the boundary kernel's recomputation so both give identical values.
// Differences are scaled by the precomputed 1/(2 dh) (exact for dh = 1).
template <class U>
__device__ __forceinline__ void interior_update(const PlateDev &P, const Kick<U> &K, U e0, U w0,
                                                U n0, U s0, U e1, U w1, U n1, U s1, U ux, U uy,
                                                U vx, U vy, U &nux, U &nuy, U &nvx, U &nvy) {
  const U i2h = (U)P.inv_2h;
  const U cd2 = (U)P.cd2, cs2 = (U)P.cs2;
  const U dphix = (e0 - w0) * i2h;
  const U dphiy = (n0 - s0) * i2h;
  const U dpsix = (e1 - w1) * i2h;
  const U dpsiy = (n1 - s1) * i2h;
  const U ax = cd2 * dphix - cs2 * dpsiy;
  const U ay = cd2 * dphiy - cs2 * (-dpsix);
  newmark<U>(P, K, ax, ay, ux, uy, vx, vy, nux, nuy, nvx, nvy);
}

// -------------------------------------------------------- interior kernel

// Exchange slots in LDS per lane and row.
enum { X_RHO0 = 0, X_RHO1, X_F1_0, X_F1_1, X_F3_0, X_F3_1, X_N };

// LDS rows of the x-exchange per march stage.  Each row is published one
// iteration before it is read, with one barrier per iteration.  Several
// waves need three rows (a wave one barrier ahead may publish the next row
// while another still reads the previous one); a single wave executes its
// LDS accesses in order, so two rows suffice, which leaves LDS room for
// more waves per CU.
__host__ __device__ constexpr int ex_rows(int lanes) { return lanes == 64 ? 2 : 3; }

__device__ __forceinline__ int tile_index(int b, int q) { return (b & 7) * q + (b >> 3); }

// Two steps of a tile whose area and two-node halo ring hold only interior
// nodes (no boundary or second-row node): step n on the area plus its
// one-node ring (from t_n on the two-node ring, buffer sb.in), step n + 1 on
// the area (buffer sb.out2); the t_{n+1} populations of the export bands
// (owned columns / rows next to single-step tiles) go to buffer sb.out.  Lane
// l holds column x0 - 2 + l.  Rows are indexed i = 0..h-1 in the march
// direction (i = -2, -1, h, h+1: halo rows).  The front row a of t_n is
// collided while row a - 1 takes step n and row a - 2 step n + 1; each
// stage hands its post-collision values to the x-neighbours through its own
// triple-buffered LDS slots (exA: t_n, exB: t_{n+1}).  deep: a launch of
// deep tiles, never the run's first step (it does not read the step
// counters, which the launches beside it may be writing).
template <class CD, int TWL, bool NT>
__device__ void march2(const DevState &s, const Tile &t, const StepBufs &sb,
                       typename CD::C (*exA)[X_N][TWL], typename CD::C (*exB)[X_N][TWL],
                       bool deep) {
  using C = typename CD::C;
  using U = typename CD::U;
  using Slot = typename CD::Slot;
  const PlateDev P = s.plates[t.plate];
  const int lane = threadIdx.x;
  const int w = t.x1 - t.x0;
  const bool live = lane <= w + 3;
  const int x = wrapc(t.x0 - 2 + lane, P.nx);
  const bool stepA = lane >= 1 && lane <= w + 2;  // step n on columns x0-1 .. x1
  const bool stepB = lane >= 2 && lane <= w + 1;  // step n+1 on the owned columns
  const int d = t.dir ? -1 : 1;
  const int h = t.y1 - t.y0;
  auto row_y = [&](int i) { return wrapc(d > 0 ? t.y0 + i : t.y1 - 1 - i, P.ny); };
  // Every lane loads (lanes past the tile from column x0, their values are
  // not used): a load under a branch, or a default written over the
  // registers of a load in flight, makes the compiler wait for all
  // outstanding memory operations right there.
  const int xl = live ? x : t.x0;
  auto load_raw = [&](int i, Slot raw[2][5]) {
    const int64_t k = node_of(P, xl, row_y(i));
    CD::load_raw(s, sb.in, 0, k, raw[0]);
    CD::load_raw(s, sb.in, 1, k, raw[1]);
  };
  auto load_uv = [&](int i, U uv[4]) {
    const int64_t k = node_of(P, xl, row_y(i));
    uv[0] = ldg<U>(s.u[sb.in][0], k);
    uv[1] = ldg<U>(s.u[sb.in][1], k);
    uv[2] = ldg<U>(s.v[sb.in][0], k);
    uv[3] = ldg<U>(s.v[sb.in][1], k);
  };
  auto collide_raw = [&](const Slot raw[2][5], C rho[2], C fs[2][5]) {
#pragma unroll
    for (int fl = 0; fl < 2; fl++) CD::collide_raw(P, fl, raw[fl], rho[fl], fs[fl]);
  };
  // t_n values of lanes past the tile (their loads read column x0)
  auto clear_dead = [&](C rho[2], C fs[2][5]) {
    if (!live) {
#pragma unroll
      for (int fl = 0; fl < 2; fl++) {
        rho[fl] = C(0);
#pragma unroll
        for (int qq = 0; qq < 5; qq++) fs[fl][qq] = C(0);
      }
    }
  };
  auto publish = [&](C(*ex)[X_N][TWL], int slot, const C rho[2], const C fs[2][5]) {
    ex[slot][X_RHO0][lane] = rho[0];
    ex[slot][X_RHO1][lane] = rho[1];
    ex[slot][X_F1_0][lane] = fs[0][1];
    ex[slot][X_F1_1][lane] = fs[1][1];
    ex[slot][X_F3_0][lane] = fs[0][3];
    ex[slot][X_F3_1][lane] = fs[1][3];
  };
  // population a row streams into the row after it (behind) / before it
  auto behind_pop = [&](const C fs[5]) { return d > 0 ? fs[2] : fs[4]; };
  auto ahead_pop = [&](const C fs[5]) { return d > 0 ? fs[4] : fs[2]; };
  constexpr int NS = ex_rows(TWL);
  auto slot_of = [](int i) { return (i + 3 * NS) % NS; };  // i >= -3
  // Pull into row i of one stage: f0 of the row, f1 / f3 from the x
  // neighbours (slot of row i), the behind row's and the ahead row's pops;
  // then the u, du/dt update from the neighbours' rho.
  auto finalize = [&](C(*ex)[X_N][TWL], int i, const C f0[2], const C fbe[2], const C fah[2],
                      const C rbe[2], const C rah[2], const U uv[4], C f[2][5], U nu[4],
                      const Kick<U> &K) {
    const int sl = slot_of(i);
    // (the end lanes read a clamped neighbour; their results are not used)
    const int lw = lane > 0 ? lane - 1 : 0, le = lane < TWL - 1 ? lane + 1 : TWL - 1;
#pragma unroll
    for (int fl = 0; fl < 2; fl++) {
      f[fl][0] = f0[fl];
      f[fl][1] = ex[sl][fl == 0 ? X_F1_0 : X_F1_1][lw];
      f[fl][3] = ex[sl][fl == 0 ? X_F3_0 : X_F3_1][le];
      f[fl][2] = d > 0 ? fbe[fl] : fah[fl];
      f[fl][4] = d > 0 ? fah[fl] : fbe[fl];
    }
    const C wr0 = ex[sl][X_RHO0][lw], er0 = ex[sl][X_RHO0][le];
    const C wr1 = ex[sl][X_RHO1][lw], er1 = ex[sl][X_RHO1][le];
    const C n0 = d > 0 ? rah[0] : rbe[0], s0 = d > 0 ? rbe[0] : rah[0];
    const C n1 = d > 0 ? rah[1] : rbe[1], s1 = d > 0 ? rbe[1] : rah[1];
    interior_update<U>(P, K, (U)er0, (U)wr0, (U)n0, (U)s0, (U)er1, (U)wr1, (U)n1, (U)s1, uv[0],
                       uv[1], uv[2], uv[3], nu[0], nu[1], nu[2], nu[3]);
  };
  // displacement-update coefficients of steps n (the run's first if n = 0)
  // and n + 1
  const Kick<U> kickA = kick_of<U>(P, !deep && s.counter[sb.in] == 0ull),
                kickB = kick_of<U>(P, false);

  // t_n stage registers: row a-2 (rho, behind pop), row a-1 (rho, f0, behind pop)
  C a2_rho[2], a2_fb[2], a1_rho[2], a1_f0[2], a1_fb[2];
  // t_{n+1} stage registers: row a-3 (rho, behind pop), row a-2 (rho, f0, behind pop)
  C b3_rho[2], b3_fb[2], b2_rho[2], b2_f0[2], b2_fb[2];
  U uvA[4];   // u, du/dt of t_n, row a-1 (row a once step n of row a-1 is done)
  U uvB[4];   // u, du/dt of t_{n+1}, row a-2
  Slot rawn[2][5];  // t_n populations of row a
  {
    Slot raw[2][5];
    C rho[2], fs[2][5];
    load_raw(-2, raw);
    load_raw(-1, rawn);
    collide_raw(raw, rho, fs);
    clear_dead(rho, fs);
    a2_rho[0] = rho[0];
    a2_rho[1] = rho[1];
    a2_fb[0] = behind_pop(fs[0]);
    a2_fb[1] = behind_pop(fs[1]);
#pragma unroll
    for (int fl = 0; fl < 2; fl++)
#pragma unroll
      for (int qq = 0; qq < 5; qq++) raw[fl][qq] = rawn[fl][qq];
    load_raw(0, rawn);
    load_uv(-1, uvA);
    collide_raw(raw, rho, fs);
    clear_dead(rho, fs);
    publish(exA, slot_of(-1), rho, fs);
    a1_rho[0] = rho[0];
    a1_rho[1] = rho[1];
    a1_f0[0] = fs[0][0];
    a1_f0[1] = fs[1][0];
    a1_fb[0] = behind_pop(fs[0]);
    a1_fb[1] = behind_pop(fs[1]);
#pragma unroll
    for (int q = 0; q < 4; q++) uvB[q] = U(0);
#pragma unroll
    for (int fl = 0; fl < 2; fl++)
      b3_rho[fl] = b3_fb[fl] = b2_rho[fl] = b2_f0[fl] = b2_fb[fl] = C(0);
  }
  for (int a = 0; a <= h + 1; a++) {
    // collide t_n row a and prefetch row a+1 into the registers it used
    // (the last iteration reloads row h+1)
    Slot raw[2][5];
    C rho[2], fs[2][5];
#pragma unroll
    for (int fl = 0; fl < 2; fl++)
#pragma unroll
      for (int qq = 0; qq < 5; qq++) raw[fl][qq] = rawn[fl][qq];
    load_raw(a + 1 <= h + 1 ? a + 1 : h + 1, rawn);
    collide_raw(raw, rho, fs);
    clear_dead(rho, fs);
    publish(exA, slot_of(a), rho, fs);
    __syncthreads();
    // step n at row a-1 (columns x0-1 .. x1)
    const C fa[2] = {ahead_pop(fs[0]), ahead_pop(fs[1])};
    C g[2][5];
    U nu[4];
    finalize(exA, a - 1, a1_f0, a2_fb, fa, a2_rho, rho, uvA, g, nu, kickA);
    // u of row a (for the next row's step n) into the registers just used
    load_uv(a <= h ? a : h, uvA);
    const int ya = row_y(a - 1);
    if (stepA && a - 1 >= 0 && a - 1 < h) {
      const bool exp = ((t.flags & TF_EXP_W) && lane == 2) ||
                       ((t.flags & TF_EXP_E) && lane == w + 1) ||
                       ((t.flags & TF_EXP_S) && ya == t.y0) ||
                       ((t.flags & TF_EXP_N) && ya == t.y1 - 1);
      if (exp && stepB) {
        const int64_t k = node_of(P, x, ya);
        CD::store(s, sb.out, 0, k, P, g[0]);
        CD::store(s, sb.out, 1, k, P, g[1]);
      }
    }
    // collide t_{n+1} row a-1 (as a store and a load between two launches
    // would leave it) and hand it to the x-neighbours
    C rho1[2], fs1[2][5];
    CD::collide_stored(P, 0, g[0], rho1[0], fs1[0]);
    CD::collide_stored(P, 1, g[1], rho1[1], fs1[1]);
    if (!stepA) {
#pragma unroll
      for (int fl = 0; fl < 2; fl++) {
        rho1[fl] = C(0);
#pragma unroll
        for (int qq = 0; qq < 5; qq++) fs1[fl][qq] = C(0);
      }
    }
    publish(exB, slot_of(a - 1), rho1, fs1);
    // step n+1 at row a-2 (owned columns); its x-neighbours' values were
    // published in the previous iteration
    if (a - 2 >= 0 && a - 2 < h) {
      const C fa1[2] = {ahead_pop(fs1[0]), ahead_pop(fs1[1])};
      C g2[2][5];
      U nu2[4];
      finalize(exB, a - 2, b2_f0, b3_fb, fa1, b3_rho, rho1, uvB, g2, nu2, kickB);
      if (stepB) {
        // NT: the pass's final state is not read again in this launch;
        // nontemporal stores leave the caches to the halo rows
        const int64_t k = node_of(P, x, row_y(a - 2));
        stg<U, NT>(s.u[sb.out2][0], k, nu2[0]);
        stg<U, NT>(s.u[sb.out2][1], k, nu2[1]);
        stg<U, NT>(s.v[sb.out2][0], k, nu2[2]);
        stg<U, NT>(s.v[sb.out2][1], k, nu2[3]);
        CD::template store<NT>(s, sb.out2, 0, k, P, g2[0]);
        CD::template store<NT>(s, sb.out2, 1, k, P, g2[1]);
      }
    }
    // shift the stages by one row
#pragma unroll
    for (int fl = 0; fl < 2; fl++) {
      a2_rho[fl] = a1_rho[fl];
      a2_fb[fl] = a1_fb[fl];
      a1_rho[fl] = rho[fl];
      a1_f0[fl] = fs[fl][0];
      a1_fb[fl] = behind_pop(fs[fl]);
      b3_rho[fl] = b2_rho[fl];
      b3_fb[fl] = b2_fb[fl];
      b2_rho[fl] = rho1[fl];
      b2_f0[fl] = fs1[fl][0];
      b2_fb[fl] = behind_pop(fs1[fl]);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) uvB[q] = nu[q];
  }
}

// (FP64 with two-step tiles of one wave: at most 168 VGPRs, so that three
// waves fit per SIMD; with more lanes per tile LDS allows only two.)
// DEEP: a launch of deep two-step tiles (no boundary or single-step tile
// within two nodes), which runs beside the launches that own the step
// counters and so leaves them alone.
template <int ST, int TWL, bool TWO, bool DEEP, bool NT>
__global__ void __launch_bounds__(TWL)
    __attribute__((amdgpu_waves_per_eu((TWO && ST == LBM_STORE_F64 && TWL == 64) ? 3 : 1)))
    k_interior(DevState s, const Tile *__restrict__ tiles, int ntiles, int q, StepBufs sb,
               Prologue pro) {
  using CD = typename CodecOf<ST>::type;
  using C = typename CD::C;
  using U = typename CD::U;
  using Slot = typename CD::Slot;
  constexpr int NS = ex_rows(TWL);
  __shared__ __align__(16) C exs[TWO ? 2 * NS : NS][X_N][TWL];
  C(*ex)[X_N][TWL] = exs;

  // populations and u, du/dt of t_n in buffers sb.in, of t_{n+1} in sb.out
  const int pc = sb.in, pn = sb.out, uc = sb.in, un = sb.out;
  // With overlapped pairs this launch's chain (single-step and frame tiles)
  // paces the step while the deep launch runs beside it: its waves get the
  // higher instruction-issue priority on a SIMD (-1 % per step on the
  // 1024^2 plate; no effect on one stream).
  if constexpr (!DEEP) __builtin_amdgcn_s_setprio(1);
  if (!DEEP && blockIdx.x == 0 && threadIdx.x == 0) s.counter[un] = s.counter[uc] + 1ull;
  const int tix = tile_index(blockIdx.x, q);
  if (tix >= ntiles) return;
  const Tile t = tiles[tix];
  if constexpr (DEEP) {
    march2<CD, TWL, NT>(s, t, sb, exs, exs + NS, true);
    return;
  }
  if (TWO && sb.out2 >= 0 && (t.flags & TF_TWO)) {
    march2<CD, TWL, NT>(s, t, sb, exs, exs + NS, false);
    return;
  }
  if (pro.enabled && t.chunk >= 0)
    prologue<CD>(s, pro, t.chunk, t.plate, sb, (int)threadIdx.x, TWL, exs, (int)sizeof(exs));
  const PlateDev P = s.plates[t.plate];
  const Kick<U> kick = kick_of<U>(P, s.counter[sb.in] == 0ull);
  const int lane = threadIdx.x;
  // this lane's column segment: lanes 0 .. w+1 the first (a halo column on
  // each side), the next wb+2 lanes the second of a paired tile; a lane
  // reads its x-neighbours' values from lanes lane -+ 1, which for an owned
  // column are its own segment's
  const int wa = t.x1 - t.x0, wb = t.bx1 > t.bx0 ? t.bx1 - t.bx0 : 0;
  const bool segb = wb > 0 && lane >= wa + 2;
  const int sl = segb ? lane - (wa + 2) : lane;  // lane within the segment
  const int w = segb ? wb : wa;
  int x = (segb ? t.bx0 : t.x0) - 1 + sl;
  bool xok = sl <= w + 1;
  if (x < 0 || x >= P.nx) {
    if (P.periodic & 1)
      x = wrapc(x, P.nx);
    else
      xok = false;
  }
  const bool owned = xok && sl >= 1 && sl <= w;
  const bool py = (P.periodic & 2) != 0;

  // Node of row y in this lane's column; false if there is none.
  auto row_node = [&](int y, int64_t &k) -> bool {
    bool ok = xok;
    if (y < 0 || y >= P.ny) {
      if (py)
        y = wrapc(y, P.ny);
      else
        ok = false;
    }
    k = node_of(P, x, y);
    return ok;
  };
  auto load_cls = [&](int y) -> uint8_t {
    int64_t k;
    return row_node(y, k) ? s.cls[k] : (uint8_t)0;
  };
  // Raw populations of row y (only for body nodes: cl from load_cls).
  auto load_raw = [&](int y, uint8_t cl, Slot raw[2][5]) {
    int64_t k;
    const bool ok = row_node(y, k) && (cl & CL_IN);
#pragma unroll
    for (int fl = 0; fl < 2; fl++)
#pragma unroll
      for (int qq = 0; qq < 5; qq++) raw[fl][qq] = Slot(0);
    if (ok) {
      CD::load_raw(s, pc, 0, k, raw[0]);
      CD::load_raw(s, pc, 1, k, raw[1]);
    }
  };
  auto load_uv = [&](int y, uint8_t cl, U uv[4]) {
    uv[0] = uv[1] = uv[2] = uv[3] = U(0);
    if (owned && (cl & (CL_IN | CL_B)) == CL_IN) {
      const int64_t k = node_of(P, x, y);
      uv[0] = ldg<U>(s.u[uc][0], k);
      uv[1] = ldg<U>(s.u[uc][1], k);
      uv[2] = ldg<U>(s.v[uc][0], k);
      uv[3] = ldg<U>(s.v[uc][1], k);
    }
  };
  auto collide_row = [&](uint8_t cl, const Slot raw[2][5], C rho[2], C fs[2][5]) {
#pragma unroll
    for (int fl = 0; fl < 2; fl++) {
      CD::collide_raw(P, fl, raw[fl], rho[fl], fs[fl]);
      if (!(cl & CL_IN)) {
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

  // The march visits the rows upwards (d = +1) or downwards (d = -1, tiles
  // with dir set): vertically adjacent tiles march in opposite directions,
  // so the halo rows they share are read by both at about the same time and
  // the second read hits in L2.  "Behind" is row r - d, "ahead" row r + d.
  // Software pipeline over rows: while row r is finalized, the populations
  // of row r + 2d, u and du/dt of row r + d and the class bytes of row r + 3d
  // are in flight.
  const int d = t.dir ? -1 : 1;
  const int h = t.y1 - t.y0;
  const int r0 = t.dir ? t.y1 - 1 : t.y0;
  // rows of the tile plus its halo rows: y0 - 1 .. y1
  auto in_reach = [&](int k) { return k <= h; };  // row r0 + k d, k >= -1
  C be_rho[2], be_f[2];                  // row r - d: rho, population streaming into r
  C cu_rho[2], cu_f0[2], cu_fb[2];       // row r (cu_fb: streams into r + d)
  uint8_t cu_cl, cl1, cl2, cl3;          // classes of rows r, r + d, r + 2d, r + 3d
  Slot raw1[2][5];                       // populations of row r + d
  U uv0[4];                              // u, du/dt of row r
  // the behind row streams population 2 (d = +1, from the south) or 4 into
  // row r, the ahead row the other one
  auto behind_pop = [&](const C fs[5]) { return d > 0 ? fs[2] : fs[4]; };
  {
    const uint8_t clm = load_cls(r0 - d);
    cu_cl = load_cls(r0);
    cl1 = load_cls(r0 + d);
    cl2 = load_cls(r0 + 2 * d);
    Slot raw[2][5];
    C rho[2], fs[2][5];
    load_raw(r0 - d, clm, raw);
    collide_row(clm, raw, rho, fs);
    be_rho[0] = rho[0];
    be_rho[1] = rho[1];
    be_f[0] = behind_pop(fs[0]);
    be_f[1] = behind_pop(fs[1]);
    load_raw(r0, cu_cl, raw);
    load_raw(r0 + d, cl1, raw1);
    load_uv(r0, cu_cl, uv0);
    collide_row(cu_cl, raw, rho, fs);
    publish(0, rho, fs);
    cu_rho[0] = rho[0];
    cu_rho[1] = rho[1];
    cu_f0[0] = fs[0][0];
    cu_f0[1] = fs[1][0];
    cu_fb[0] = behind_pop(fs[0]);
    cu_fb[1] = behind_pop(fs[1]);
  }
  int slot = 0;
  for (int k = 0; k < h; k++) {
    const int r = r0 + k * d;
    const int nslot = slot + 1 == NS ? 0 : slot + 1;
    // prefetch
    cl3 = in_reach(k + 3) ? load_cls(r + 3 * d) : (uint8_t)0;
    Slot raw2[2][5];
    if (in_reach(k + 2)) {
      load_raw(r + 2 * d, cl2, raw2);
    } else {
#pragma unroll
      for (int fl = 0; fl < 2; fl++)
#pragma unroll
        for (int qq = 0; qq < 5; qq++) raw2[fl][qq] = Slot(0);
    }
    U uv1[4];
    load_uv(r + d, (k + 1 < h) ? cl1 : (uint8_t)0, uv1);
    // collide row r + d and hand its values to the x-neighbours
    C nx_rho[2], nx_fs[2][5];
    collide_row(cl1, raw1, nx_rho, nx_fs);
    publish(nslot, nx_rho, nx_fs);
    __syncthreads();
    const bool fin = owned && (cu_cl & (CL_IN | CL_B)) == CL_IN;
    if (fin) {
      const int64_t kn = node_of(P, x, r);
      const C wr0 = ex[slot][X_RHO0][lane - 1], er0 = ex[slot][X_RHO0][lane + 1];
      const C wr1 = ex[slot][X_RHO1][lane - 1], er1 = ex[slot][X_RHO1][lane + 1];
      // rho of the north / south neighbours
      const C n0 = d > 0 ? nx_rho[0] : be_rho[0], s0 = d > 0 ? be_rho[0] : nx_rho[0];
      const C n1 = d > 0 ? nx_rho[1] : be_rho[1], s1 = d > 0 ? be_rho[1] : nx_rho[1];
      U nux, nuy, nvx, nvy;
      interior_update<U>(P, kick, (U)er0, (U)wr0, (U)n0, (U)s0, (U)er1, (U)wr1, (U)n1, (U)s1,
                         uv0[0], uv0[1], uv0[2], uv0[3], nux, nuy, nvx, nvy);
      stg<U>(s.u[un][0], kn, nux);
      stg<U>(s.u[un][1], kn, nuy);
      stg<U>(s.v[un][0], kn, nvx);
      stg<U>(s.v[un][1], kn, nvy);
      // Pull: f_alpha(x, t+dt) = f*_alpha(x - c^alpha dt).  A second-row
      // node keeps it in the side buffer; the next step's boundary work
      // replaces the populations that leave boundary nodes and stores it.
      const bool sec = (cu_cl & CL_S) != 0;
      const int64_t si = sec ? (int64_t)s.sidx[kn] : 0;
      C *side = static_cast<C *>(s.side[sb.sp ^ 1]);
#pragma unroll
      for (int fl = 0; fl < 2; fl++) {
        C f[5];
        f[0] = cu_f0[fl];
        f[1] = ex[slot][fl == 0 ? X_F1_0 : X_F1_1][lane - 1];
        f[3] = ex[slot][fl == 0 ? X_F3_0 : X_F3_1][lane + 1];
        f[2] = d > 0 ? be_f[fl] : nx_fs[fl][2];
        f[4] = d > 0 ? nx_fs[fl][4] : be_f[fl];
        if (!sec) {
          CD::store(s, pn, fl, kn, P, f);
        } else {
#pragma unroll
          for (int qq = 0; qq < 5; qq++) side[(int64_t)(fl * 5 + qq) * s.nsec + si] = f[qq];
        }
      }
    }
    be_rho[0] = cu_rho[0];
    be_rho[1] = cu_rho[1];
    be_f[0] = cu_fb[0];
    be_f[1] = cu_fb[1];
    cu_rho[0] = nx_rho[0];
    cu_rho[1] = nx_rho[1];
    cu_f0[0] = nx_fs[0][0];
    cu_f0[1] = nx_fs[1][0];
    cu_fb[0] = behind_pop(nx_fs[0]);
    cu_fb[1] = behind_pop(nx_fs[1]);
    cu_cl = cl1;
    cl1 = cl2;
    cl2 = cl3;
#pragma unroll
    for (int fl = 0; fl < 2; fl++)
#pragma unroll
      for (int qq = 0; qq < 5; qq++) raw1[fl][qq] = raw2[fl][qq];
#pragma unroll
    for (int qq = 0; qq < 4; qq++) uv0[qq] = uv1[qq];
    slot = nslot;
  }
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
  // owned columns of the tile's first segment, then of its second
  const int wa = t.x1 - t.x0, lane = (int)threadIdx.x;
  const int x = lane < wa ? t.x0 + lane : t.bx0 + (lane - wa);
  if (lane >= wa && x >= t.bx1) return;
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
    CD::store_eq(s, 0, 0, k, P, phi, C(0), C(0));
    CD::store_eq(s, 0, 1, k, P, psi, C(0), C(0));
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

// Consistency error of Sec. 4 (tension example): per body node the 2-norm
// of (omega - (curl u).e_z, e - div u), the fields being the sums of the
// populations and the derivatives of u the finite differences the method
// uses at that node; 0 outside the body.
template <int ST>
__global__ void k_cons_err(DevState s, int plate, int b, double *err) {
  using CD = typename CodecOf<ST>::type;
  using U = typename CD::U;
  const PlateDev P = s.plates[plate];
  const int64_t n = (int64_t)P.nx * P.ny;
  for (int64_t d = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(d % P.nx), j = (int)(d / P.nx);
    const int64_t k = node_of(P, i, j);
    if (!(s.cls[k] & CL_IN)) {
      err[d] = 0.0;
      continue;
    }
    U dv, cu;
    div_curl<U>(s, b, P, i, j, dv, cu);
    const double d1 = CD::field(s, b, 1, k, P) - (double)cu;
    const double d0 = CD::field(s, b, 0, k, P) - (double)dv;
    err[d] = sqrt(d1 * d1 + d0 * d0);
  }
}

// --------------------------------------------------------------- launchers

template <int ST, bool TWO, bool DEEP, bool NT>
static hipError_t launch_interior_t(const DevState &s, const Tile *tiles, int ntiles, int lanes,
                                    const StepBufs &b, const Prologue &pro, hipStream_t st) {
  // at least one block: block 0 advances the step counter
  const int q = ntiles > 0 ? (ntiles + 7) / 8 : 1;
  const dim3 grid(8 * q);
  switch (lanes) {
    case 64:
      hipLaunchKernelGGL((k_interior<ST, 64, TWO, DEEP, NT>), grid, dim3(64), 0, st, s, tiles, ntiles,
                         q, b, pro);
      break;
    case 128:
      hipLaunchKernelGGL((k_interior<ST, 128, TWO, DEEP, NT>), grid, dim3(128), 0, st, s, tiles,
                         ntiles, q, b, pro);
      break;
    case 256:
      hipLaunchKernelGGL((k_interior<ST, 256, TWO, DEEP, NT>), grid, dim3(256), 0, st, s, tiles,
                         ntiles, q, b, pro);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int ST>
static hipError_t launch_sync_t(const DevState &s, const Tile *tiles, int ntiles, int lanes,
                                int b, hipStream_t st) {
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
                           const StepBufs &b, const Prologue &pro, hipStream_t stream) {
  if (b.out2 >= 0 && b.nt) {
    LBM_DISPATCH(st, return (launch_interior_t<ST, true, false, true>(s, tiles, ntiles, lanes, b,
                                                                      pro, stream)));
  } else if (b.out2 >= 0) {
    LBM_DISPATCH(st, return (launch_interior_t<ST, true, false, false>(s, tiles, ntiles, lanes, b,
                                                                       pro, stream)));
  } else {
    LBM_DISPATCH(st, return (launch_interior_t<ST, false, false, false>(s, tiles, ntiles, lanes, b,
                                                                        pro, stream)));
  }
  return hipSuccess;
}

hipError_t launch_deep(int st, const DevState &s, const Tile *tiles, int ntiles, int lanes,
                       const StepBufs &b, hipStream_t stream) {
  if (ntiles <= 0) return hipSuccess;
  if (b.out2 < 0) return hipErrorInvalidValue;
  const Prologue none{};
  if (b.nt) {
    LBM_DISPATCH(st, return (launch_interior_t<ST, true, true, true>(s, tiles, ntiles, lanes, b,
                                                                     none, stream)));
  } else {
    LBM_DISPATCH(st, return (launch_interior_t<ST, true, true, false>(s, tiles, ntiles, lanes, b,
                                                                      none, stream)));
  }
  return hipSuccess;
}

hipError_t launch_boundary(int st, const DevState &s, const Chunk *chunks, int nchunks,
                           const UNode *un, const GradNode *gn, const BTask *bt, const STask *stk,
                           int bc, int bp, int ub, int ub2, int sr, int do_reset,
                           hipStream_t stream) {
  if (nchunks <= 0) return hipSuccess;
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_boundary<ST>), dim3(nchunks), dim3(kBoundaryThreads), 0,
                                      stream, s, chunks, un, gn, bt, stk, bc, bp, ub, ub2, sr,
                                      do_reset));
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

hipError_t launch_cons_err(int st, const DevState &s, int plate, int64_t nodes, int b, double *err,
                           hipStream_t stream) {
  int64_t blocks = (nodes + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  LBM_DISPATCH(st, hipLaunchKernelGGL((k_cons_err<ST>), dim3((unsigned)blocks), dim3(256), 0,
                                      stream, s, plate, b, err));
  return hipGetLastError();
}

// ------------------------------------------- fixed staging of lbm_fields_noalloc
//
// Device memory of the library's own, for callers that cannot allocate: a
// file-scope array that every context on a GPU shares (each GPU holds its
// own copy, at its own address, until the process ends).  Host code never
// passes the array's name to a kernel or a copy (on the host it only stands
// for the symbol); it uses the device address hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) double scratch[kNoAllocBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_staging(int device, void **ptr) {
  *ptr = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    g_scratch_done[device] = true;
  }
  *ptr = g_scratch_ptr[device];
  return g_scratch_err[device];
}

}  // namespace lbm
