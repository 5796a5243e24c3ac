// Solid sites anywhere on a lattice periodic in x and y: a byte mask [ny][nx]
// (nonzero = solid), e.g. the staircase circular no-slip wall of the
// curved-interface transient (Sec. IV, dynamics of curved interfaces; App. D).
//
// Links that would enter a solid site are bounced back half-way (the rule the
// walls use), and a stencil tap that falls on a solid site reads the field's
// value at the stencil's own centre (zero-gradient continuation: a uniform
// field has zero derivative beside any obstacle).  The step runs as four
// passes over per-site field planes, since the tap substitution depends on
// the centre site and a solid site may sit anywhere in a strip:
//   1. gather (with bounce-back), colour densities, momentum, rho^N, Phi';
//   2. grad rho^N and the director m;
//   3. curvature K = div n (n = -m), force G and velocity u (or the fields);
//   4. grad Phi', div u, collision and recolour of the re-gathered site, store.
// The per-site arithmetic and the order of every stencil sum are those of the
// fused step kernel, so a mask without solid sites reproduces it.  For the
// stencil profiles it is instantiated for, the fused step kernel also runs
// with a mask (its MASK variant: per-site bounce bits in the gather, NaN
// markers for the taps); these passes are the reference it is tested against
// and serve the other profiles.
#pragma once

#include "chromo_kernels.hpp"

namespace chromo {
namespace solid {

// field planes of the workspace, each [ny][nx] of the arithmetic type
enum { P_RR, P_RB, P_JX, P_JY, P_RN, P_PHI, P_MX, P_MY, P_GNX, P_GNY, P_UX, P_UY, P_GX, P_GY, P_N };
// The workspace holds the P_N planes, then (at the next 256-byte boundary) the
// [ny][nx] bounce bits of the fused kernel.
inline size_t bits_offset(size_t plane, size_t elem) { return (P_N * plane * elem + 255) / 256 * 256; }

// periodic index for offsets of at most the lattice size (the host requires
// nx, ny >= 4 and offsets are at most 3)
__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ size_t at(const Geom& g, int x, int y) { return (size_t)y * g.nx + x; }

// App. B gradient of field s at fluid site (x, y); a solid tap reads s(x, y).
// Same differences and accumulation order as ring_grad.
template <int R, typename T>
__device__ __forceinline__ void mask_grad(const T* __restrict__ s, const unsigned char* __restrict__ solid,
                                          const Geom& g, int x, int y, T& gx, T& gy) {
  const T c0 = s[at(g, x, y)];
  auto v = [&](int xx, int yy) {
    const size_t k = at(g, xx, yy);
    return solid[k] ? c0 : s[k];
  };
  gx = T(0);
  gy = T(0);
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T bd = stencil_bd<R, T>(n), ba = stencil_ba<R, T>(n);
    const int xp = wrap(x + n, g.nx), xm = wrap(x - n, g.nx), yp = wrap(y + n, g.ny), ym = wrap(y - n, g.ny);
    const T d1 = v(xp, yp) - v(xm, ym);
    const T d3 = v(xm, yp) - v(xp, ym);
    const T d8 = v(xp, y) - v(xm, y);
    const T d2 = v(x, yp) - v(x, ym);
    gx += ba * d8;
    gx += bd * (d1 - d3);
    gy += ba * d2;
    gy += bd * (d1 + d3);
  }
}

// div of the vector field (sx, sy); same order as ring_div.
template <int R, typename T>
__device__ __forceinline__ T mask_div(const T* __restrict__ sx, const T* __restrict__ sy,
                                      const unsigned char* __restrict__ solid, const Geom& g, int x, int y) {
  const size_t c = at(g, x, y);
  const T cx = sx[c], cy = sy[c];
  auto vx = [&](int xx, int yy) {
    const size_t k = at(g, xx, yy);
    return solid[k] ? cx : sx[k];
  };
  auto vy = [&](int xx, int yy) {
    const size_t k = at(g, xx, yy);
    return solid[k] ? cy : sy[k];
  };
  T acc = T(0);
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T bd = stencil_bd<R, T>(n), ba = stencil_ba<R, T>(n);
    const int xp = wrap(x + n, g.nx), xm = wrap(x - n, g.nx), yp = wrap(y + n, g.ny), ym = wrap(y - n, g.ny);
    const T d1 = vx(xp, yp) - vx(xm, ym);
    const T d3 = vx(xm, yp) - vx(xp, ym);
    const T d8 = vx(xp, y) - vx(xm, y);
    const T e1 = vy(xp, yp) - vy(xm, ym);
    const T e3 = vy(xm, yp) - vy(xp, ym);
    const T e2 = vy(x, yp) - vy(x, ym);
    acc += ba * (d8 + e2);
    acc += bd * ((d1 - d3) + (e1 + e3));
  }
  return acc;
}

// Pull gather of the storage words of fluid site (x, y): word q (link i)
// comes from r - c_i, or, when r - c_i is solid, from the reversed link's word
// at r itself.  Layout [y][word][x].
template <typename S>
__device__ __forceinline__ void gather(const typename S::W* __restrict__ src, const unsigned char* __restrict__ solid,
                                       const Geom& g, int x, int y, typename S::W w[S::NW]) {
#pragma unroll
  for (int q = 0; q < S::NW; ++q) {
    const int i = word_link<S>(q);
    const int xs = wrap(x - link_cx(i), g.nx), ys = wrap(y - link_cy(i), g.ny);
    w[q] = solid[at(g, xs, ys)] ? src[((size_t)y * S::NW + word_bounce<S>(q)) * g.nx + x]
                                : src[((size_t)ys * S::NW + q) * g.nx + xs];
  }
}

// Re-encode a population buffer for a new mask, in place: the word a fluid
// site's link now bounces into takes the value the link pulled before (so the
// pre-collision populations of every fluid site are kept).  Reads words of
// solid sites only and writes words of fluid sites only.
template <typename S>
__global__ void __launch_bounds__(256) rebounce_kernel(void* popsv, const unsigned char* __restrict__ solid, Geom g) {
  using W = typename S::W;
  W* pops = static_cast<W*>(popsv);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx || solid[at(g, x, y)]) return;
#pragma unroll
  for (int q = 0; q < S::NW; ++q) {
    const int i = word_link<S>(q);
    const int xd = wrap(x + link_cx(i), g.nx), yd = wrap(y + link_cy(i), g.ny);
    if (solid[at(g, xd, yd)])
      pops[((size_t)y * S::NW + q) * g.nx + x] = pops[((size_t)yd * S::NW + word_bounce<S>(q)) * g.nx + xd];
  }
}

// Bounce bits of every site for the fused step kernel: bit i - 1 set when the
// source r - c_i of link i is solid; all bits at a solid site (its gather then
// reads its own zero words).  (A template only so that every format's
// translation unit has its own copy.)
template <typename S>
__global__ void __launch_bounds__(256) bounce_bits_kernel(const unsigned char* __restrict__ solid, Geom g,
                                                          unsigned char* __restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const size_t site = at(g, x, y);
  unsigned b = 0xffu;
  if (!solid[site]) {
    b = 0u;
#pragma unroll
    for (int i = 1; i < 9; ++i)
      if (solid[at(g, wrap(x - link_cx(i), g.nx), wrap(y - link_cy(i), g.ny))]) b |= 1u << (i - 1);
  }
  out[site] = (unsigned char)b;
}

// The words of zero populations (all-zero bits for the float formats, the
// offset encoding of zero for the 16-bit ones).
template <typename S>
__device__ __forceinline__ void zero_words(const Coef<typename S::math>& c, typename S::W w[S::NW]) {
  using T = typename S::math;
  T R[9], B[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) R[i] = B[i] = T(0);
  encode<S>(R, B, c, w);
}

// Clear the words of solid sites (they carry no state and no mass).
template <typename S>
__global__ void __launch_bounds__(256) clear_solid_kernel(void* popsv, const unsigned char* __restrict__ solid,
                                                          Geom g, Coef<typename S::math> c) {
  using W = typename S::W;
  W* pops = static_cast<W*>(popsv);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx || !solid[at(g, x, y)]) return;
  W w[S::NW];
  zero_words<S>(c, w);
#pragma unroll
  for (int q = 0; q < S::NW; ++q) pops[((size_t)y * S::NW + q) * g.nx + x] = w[q];
}

// pass 1: colour densities, raw momentum, colour index, Phi'
template <typename S>
__global__ void __launch_bounds__(256) sites_kernel(const void* __restrict__ srcv,
                                                    const unsigned char* __restrict__ solid, Geom g,
                                                    Coef<typename S::math> c, typename S::math* __restrict__ ws) {
  using T = typename S::math;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const size_t site = at(g, x, y), P = g.plane;
  T* o = ws + site;
  if (solid[site]) {
    o[P_RR * P] = o[P_RB * P] = o[P_JX * P] = o[P_JY * P] = o[P_RN * P] = o[P_PHI * P] = T(0);
    return;
  }
  typename S::W w[S::NW];
  gather<S>(static_cast<const typename S::W*>(srcv), solid, g, x, y, w);
  T pr[9], pb[9], f[9];
  decode<S>(w, c, pr, pb, f);
  const T rR = ((pr[0] + pr[2]) + (pr[4] + pr[6])) + ((pr[1] + pr[3]) + (pr[5] + pr[7])) + pr[8];
  const T rB = ((pb[0] + pb[2]) + (pb[4] + pb[6])) + ((pb[1] + pb[3]) + (pb[5] + pb[7])) + pb[8];
  T jx, jy;
  momenta(f, jx, jy);
  o[P_RR * P] = rR;
  o[P_RB * P] = rB;
  o[P_JX * P] = jx;
  o[P_JY * P] = jy;
  o[P_RN * P] = colour_index(rR * c.inv_rho0R, rB * c.inv_rho0B);
  o[P_PHI * P] = c.c06R * rR + c.phiB * rB - (rR + rB) * T(1.0 / 3.0);
}

// pass 2: grad rho^N and the director m = grad rho^N / sqrt(|grad rho^N|^2 + eps^2)
template <typename T, int RG>
__global__ void __launch_bounds__(256) director_kernel(const unsigned char* __restrict__ solid, Geom g, Coef<T> c,
                                                       T* __restrict__ ws) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const size_t site = at(g, x, y), P = g.plane;
  T* o = ws + site;
  if (solid[site]) {
    o[P_MX * P] = o[P_MY * P] = o[P_GNX * P] = o[P_GNY * P] = T(0);
    return;
  }
  T gx, gy;
  mask_grad<RG>(ws + P_RN * P, solid, g, x, y, gx, gy);
  const T is = rsqrt_pos(gx * gx + gy * gy + c.eps2);
  o[P_MX * P] = gx * is;
  o[P_MY * P] = gy * is;
  o[P_GNX * P] = gx;
  o[P_GNY * P] = gy;
}

// pass 3: K = div n = -div m, G = sigma K grad rho^N / 2 + g + G_ext, u = (j + G/2)/rho.
// FIELDS: write rho, u, rho^N to the caller's arrays (NaN at solid sites).
template <typename T, int RK, bool FIELDS>
__global__ void __launch_bounds__(256) force_kernel(const unsigned char* __restrict__ solid, Geom g, Coef<T> c,
                                                    const T* __restrict__ force, T* __restrict__ ws, T* out_rho,
                                                    T* out_ux, T* out_uy, T* out_rhoN) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const size_t site = at(g, x, y), P = g.plane;
  T* o = ws + site;
  if (solid[site]) {
    if (FIELDS) {
      const T nan = __builtin_nan("");
      if (out_rho) out_rho[site] = nan;
      if (out_ux) out_ux[site] = nan;
      if (out_uy) out_uy[site] = nan;
      if (out_rhoN) out_rhoN[site] = nan;
    } else {
      o[P_UX * P] = o[P_UY * P] = o[P_GX * P] = o[P_GY * P] = T(0);
    }
    return;
  }
  const T K = c.fixed_K ? c.K_fixed : -mask_div<RK>(ws + P_MX * P, ws + P_MY * P, solid, g, x, y);
  T Gx = c.half_sigma * K * o[P_GNX * P] + c.gx;
  T Gy = c.half_sigma * K * o[P_GNY * P] + c.gy;
  if (force) {
    Gx += force[site];
    Gy += force[P + site];
  }
  const T rho = o[P_RR * P] + o[P_RB * P];
  const T ir = recip(rho);
  const T ux = (o[P_JX * P] + T(0.5) * Gx) * ir;
  const T uy = (o[P_JY * P] + T(0.5) * Gy) * ir;
  if (FIELDS) {
    if (out_rho) out_rho[site] = rho;
    if (out_ux) out_ux[site] = ux;
    if (out_uy) out_uy[site] = uy;
    if (out_rhoN) out_rhoN[site] = o[P_RN * P];
  } else {
    o[P_UX * P] = ux;
    o[P_UY * P] = uy;
    o[P_GX * P] = Gx;
    o[P_GY * P] = Gy;
  }
}

// pass 4: grad Phi', div u, collision and recolour (collide_store), store at own site
template <typename S, int RP, int RU>
__global__ void __launch_bounds__(256) collide_kernel(StepArgs<typename S::math> a,
                                                      const unsigned char* __restrict__ solid,
                                                      const typename S::math* __restrict__ ws) {
  using T = typename S::math;
  using W = typename S::W;
  const Geom& g = a.g;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const size_t site = at(g, x, y), P = g.plane;
  if (solid[site]) {
    W* dst = static_cast<W*>(a.dst);
    W w[S::NW];
    zero_words<S>(a.c, w);
#pragma unroll
    for (int q = 0; q < S::NW; ++q) dst[((size_t)y * S::NW + q) * g.nx + x] = w[q];
    return;
  }
  T dPx, dPy;
  mask_grad<RP>(ws + P_PHI * P, solid, g, x, y, dPx, dPy);
  const T theta = mask_div<RU>(ws + P_UX * P, ws + P_UY * P, solid, g, x, y);
  W w[S::NW];
  gather<S>(static_cast<const W*>(a.src), solid, g, x, y, w);
  T pr[9], pb[9], f[9];
  decode<S>(w, a.c, pr, pb, f);
  const T* o = ws + site;
  const T rR = o[P_RR * P], rB = o[P_RB * P];
  Thread t;
  t.tx = threadIdx.x;
  t.ty = 0;
  t.xg = x;
  t.ya = t.yb = t.nit = 0;
  t.own = true;
  t.cols.o = x * (int)sizeof(W);
  t.cols.m = t.cols.p = t.cols.o;
  collide_store<S, T, MODE_STEP>(a, a.dst, f, rR, rB, o[P_UX * P], o[P_UY * P], o[P_GX * P], o[P_GY * P],
                                 recip(rR + rB), dPx, dPy, theta, o[P_RN * P], o[P_MX * P], o[P_MY * P], y, t);
}

}  // namespace solid
}  // namespace chromo
