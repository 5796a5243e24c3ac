// Adjoint of one time step (reverse-mode derivative of the step of
// chromo_kernels.hpp) on periodic lattices, walled lattices and lattices with
// a mask of solid sites.
//
// The step maps the stored populations buf_t (post-recolour, pull layout) to
// buf_{t+1}.  Given lambda_{t+1} = dL/dbuf_{t+1} (same layout, arithmetic
// type), the passes below compute lambda_t = (d buf_{t+1} / d buf_t)^T
// lambda_{t+1}, and add dL/dsigma (FP64) and dL/dG_ext (per-site force) to
// their outputs.  The chain is walked backwards:
//   pass 1 (local)  : the step kernel in MODE_ADJ recomputes the forward
//                     quantities of each site and, instead of storing the new
//                     populations, runs local_backward: recolour,
//                     reconstruction, relaxation, correction tensor (App. A)
//                     -> adjoints of f_i, rho_R, rho_B, u, G, grad Phi', div u,
//                     rho^N, director m; it also saves rho_C, u, K, grad rho^N;
//   pass 2 (stencil): div u and grad Phi' transposed, then u = (j + G/2)/rho,
//                     Phi' and G = sigma K grad(rho^N)/2 + G_ext (Sec. II);
//   pass 3 (stencil): K = -div m transposed, then m = g/sqrt(|g|^2 + eps^2);
//   pass 4 (stencil): g = grad rho^N transposed, then the colour index;
//   pass 5 (gather) : pre-collision populations from rho_C, f_i, j, and the
//                     pull-streaming gather transposed (a push).
// Every App. B stencil D is a sum of antisymmetric pair differences, so on a
// periodic lattice its transpose is -D.  With a mask, a tap on a solid site
// reads the centre value; for an adjoint field lambda that is zero at solid
// sites the transpose is then -D lambda plus lambda at the centre times the
// summed weights of the centre's solid taps.
#pragma once

#include "chromo_kernels.hpp"

namespace chromo {
namespace adj {

// Planes of the adjoint workspace, in groups: SV (forward values pass 1
// saves, SV_*), A (pass 1's local adjoints), B (pass 2's outputs), C (pass 3),
// D (pass 4).  A workspace row holds the row of every plane, group after
// group ([y][WS_PLANES][x]).
enum {
  A_F = 0,  // 9 planes: adjoint of f_i through the collision
  A_RR = 9, A_RB, A_UX, A_UY, A_GX, A_GY, A_DPX, A_DPY, A_TH, A_RN, A_MX, A_MY,
  A_END
};
static_assert(A_END == A_N, "local adjoint count");
enum { B_RR, B_RB, B_JX, B_JY, B_K, B_GX, B_GY, B_N };
enum { C_GX, C_GY, C_N };
enum { D_RR, D_RB, D_N };
static_assert(WS_PLANES == SV_N + A_N + B_N + C_N + D_N, "workspace planes");
// first plane of each group within a workspace row
constexpr int G_SV = 0, G_A = SV_N, G_B = G_A + A_N, G_C = G_B + B_N, G_D = G_C + C_N;
// FP64 partial sums of dL/dsigma, one per 256-site block of a row; the
// workspace keeps RED2 more doubles of slack
__host__ __device__ inline int red_blocks(int nx, int ny) { return ((nx + 255) / 256) * ny; }
constexpr int RED2 = 256;

// v mod n for the index of a stencil tap: v lies within 3 of [0, n) (or, for
// the mirrored rows of a walled lattice, within [-n, 2n)), so on lattices of
// 4 or more rows and columns one correction either way suffices; smaller ones
// take the division (n is the same in every lane: a scalar branch).
__device__ __forceinline__ int wrapi(int v, int n) {
  if (n >= 4) {
    v = v < 0 ? v + n : v;
    return v >= n ? v - n : v;
  }
  v %= n;
  return v < 0 ? v + n : v;
}

// App. B first-derivative stencil of radius R applied to a periodic field at
// (x, y): (d/dx, d/dy), the same sums as the forward ring stencils.  f points
// at the field's element (0, 0); rows lie rs elements apart (a workspace
// plane: rs = WS_PLANES nx).
template <int R, typename T>
__device__ __forceinline__ void grad_at(const T* f, size_t rs, int nx, int ny, int x, int y, T& gx, T& gy) {
  const T wd = T(1.0 / 36.0), wa = T(1.0 / 9.0);
  const T* r0 = f + (size_t)y * rs;
  gx = T(0);
  gy = T(0);
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T b = stencil_b<R, T>(n);
    const int xp = wrapi(x + n, nx), xm = wrapi(x - n, nx);
    const T* rp = f + (size_t)wrapi(y + n, ny) * rs;
    const T* rm = f + (size_t)wrapi(y - n, ny) * rs;
    const T d1 = rp[xp] - rm[xm];
    const T d3 = rp[xm] - rm[xp];
    const T d8 = r0[xp] - r0[xm];
    const T d2 = rp[x] - rm[x];
    gx += b * (wd * (d1 - d3) + wa * d8);
    gy += b * (wd * (d1 + d3) + wa * d2);
  }
}

template <int R, typename T>
__device__ __forceinline__ T div_at(const T* fx, const T* fy, size_t rs, int nx, int ny, int x, int y) {
  T ax, ay, bx, by;
  grad_at<R>(fx, rs, nx, ny, x, y, ax, ay);
  grad_at<R>(fy, rs, nx, ny, x, y, bx, by);
  return ax + by;
}

template <typename T>
__device__ __forceinline__ void grad_r(int r, const T* f, size_t rs, int nx, int ny, int x, int y, T& gx, T& gy) {
  if (r == 3) {
    grad_at<3>(f, rs, nx, ny, x, y, gx, gy);
  } else {
    grad_at<1>(f, rs, nx, ny, x, y, gx, gy);
  }
}

template <typename T>
__device__ __forceinline__ T div_r(int r, const T* fx, const T* fy, size_t rs, int nx, int ny, int x, int y) {
  return r == 3 ? div_at<3>(fx, fy, rs, nx, ny, x, y) : div_at<1>(fx, fy, rs, nx, ny, x, y);
}

// Transposes of the App. B stencils on a walled lattice (solid rows 0 and
// ny - 1).  The forward stencil at fluid row y' reads, for link i and
// distance n, the fluid row fold(y' + n c_iy) of the mirror-extended strip
// (negated for a y-component): so fluid row `row` receives from y' =
// row - n c_iy directly and from y' = 2F - 1 - row - n c_iy through the mirror
// (both mod 2F, kept when inside the strip).  Returns (D_x^T l, D_y^T l) at
// the fluid site (x, y) for a field l given on the lattice's rows (rs
// elements apart).
template <int R, typename T>
__device__ __forceinline__ void gradT_walls_at(const T* l, size_t rs, int nx, int ny, int x, int y, bool odd, T& tx,
                                               T& ty) {
  const int F = ny - 2, row = y - 1, F2 = 2 * F;
  const T wd = T(1.0 / 36.0), wa = T(1.0 / 9.0);
  const T sg = odd ? T(-1) : T(1);
  tx = T(0);
  ty = T(0);
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T b = stencil_b<R, T>(n);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int cx = link_cx(i), cy = link_cy(i);
      const T bw = b * ((i & 1) ? wd : wa);
      const int xs = wrapi(x - n * cx, nx);
      const int y1 = wrapi(row - n * cy, F2), y2 = wrapi(F2 - 1 - row - n * cy, F2);
      T v = T(0);
      if (y1 < F) v += l[(size_t)(y1 + 1) * rs + xs];
      if (y2 < F) v += sg * l[(size_t)(y2 + 1) * rs + xs];
      tx += bw * T(cx) * v;
      ty += bw * T(cy) * v;
    }
  }
}

template <typename T>
__device__ __forceinline__ void gradT_walls(int r, const T* l, size_t rs, int nx, int ny, int x, int y, bool odd,
                                            T& tx, T& ty) {
  if (r == 3) {
    gradT_walls_at<3>(l, rs, nx, ny, x, y, odd, tx, ty);
  } else {
    gradT_walls_at<1>(l, rs, nx, ny, x, y, odd, tx, ty);
  }
}

__device__ __forceinline__ bool solid_row(const Geom& g, int y) { return g.walls && (y == 0 || y == g.ny - 1); }

// the same, with the lattice kind fixed at compile time (periodic: never)
template <bool W>
__device__ __forceinline__ bool solid_row_w(const Geom& g, int y) {
  return W && (y == 0 || y == g.ny - 1);
}

// solid site: a wall row (W) or a site of the mask (M)
template <bool W, bool M>
__device__ __forceinline__ bool solid_at(const Geom& g, const unsigned char* solid, int x, int y) {
  if constexpr (M) return solid[(size_t)y * g.nx + x] != 0;
  return solid_row_w<W>(g, y);
}

// Summed weights b_n w_i c_i of the taps of the radius-R stencil at (x, y)
// that fall on solid sites of the mask (the weight the centre value takes).
template <int R, typename T>
__device__ __forceinline__ void solid_tap_weights(const unsigned char* solid, int nx, int ny, int x, int y, T& wx,
                                                  T& wy) {
  const T wd = T(1.0 / 36.0), wa = T(1.0 / 9.0);
  wx = T(0);
  wy = T(0);
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T b = stencil_b<R, T>(n);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int cx = link_cx(i), cy = link_cy(i);
      const int xs = wrapi(x + n * cx, nx), ys = wrapi(y + n * cy, ny);
      if (solid[(size_t)ys * nx + xs]) {
        const T bw = b * ((i & 1) ? wd : wa);
        wx += bw * T(cx);
        wy += bw * T(cy);
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void solid_tap_weights_r(int r, const unsigned char* solid, int nx, int ny, int x, int y,
                                                    T& wx, T& wy) {
  if (r == 3) {
    solid_tap_weights<3>(solid, nx, ny, x, y, wx, wy);
  } else {
    solid_tap_weights<1>(solid, nx, ny, x, y, wx, wy);
  }
}

struct Radii {
  int g, k, p, u;
};

// ---------------------------------------------------------------------------
// pass 1: local adjoint of correction tensor, relaxation, reconstruction and
// recolour at one site.  Inputs: pre-collision totals f_i, colour densities,
// the site's u, G, grad Phi', div u, rho^N, director m, and lR, lB = dL/d of
// the site's post-recolour populations.  out[A_*] receives the adjoints.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void local_backward(const Coef<T>& c, const T* f, T rR, T rB, T ux, T uy, T Gx, T Gy, T dPx, T dPy,
                               T theta, T rhoN, T mx, T my, const T* lR, const T* lB, T* out) {
  // ---- forward, as in the step (App. A, Sec. II) --------------------------
  const T rho = rR + rB;
  const T d15 = f[1] - f[5], d37 = f[3] - f[7], d84 = f[8] - f[4], d26 = f[2] - f[6];
  const T s15 = f[1] + f[5], s37 = f[3] + f[7], sd = s15 + s37;
  const T pxx = sd + (f[4] + f[8]);
  const T pyy = sd + (f[2] + f[6]);
  const T pxy = s15 - s37;
  const T N = f[0] - T(2) * ((f[2] + f[6]) + (f[4] + f[8])) + T(4) * sd;
  const T Jx = T(4) * (d15 - d37) - T(2) * d84;
  const T Jy = T(4) * (d15 + d37) - T(2) * d26;
  const T nu = c.hnuR * (T(1) + rhoN) + c.hnuB * (T(1) - rhoN);
  const T l3 = T(2) / (T(6) * nu + T(1));
  const T k = T(1) - T(0.5) * l3;
  const T iso = ux * dPx + uy * dPy - rho * theta * T(1.0 / 3.0);
  const T ex = Gx - dPx, ey = Gy - dPy;
  const T Cxx = k * (T(2) * ux * ex - iso);
  const T Cyy = k * (T(2) * uy * ey - iso);
  const T Cxy = k * (ux * ey + uy * ex);
  const T P0 = c.c06R * rR + c.c06B * rB;
  const T qxx = (pxx - P0) - rho * ux * ux;
  const T qyy = (pyy - P0) - rho * uy * uy;
  const T qxy = pxy - rho * ux * uy;
  const T dxx = Cxx - l3 * qxx;
  const T dyy = Cyy - l3 * qyy;
  const T dxy = Cxy - l3 * qxy;
  const T N0 = c.ghost_eq ? T(0) : T(1.8) * (c.alphaR * rR + c.alphaB * rB) - T(0.8) * rho;
  const T dN = -c.lambda6 * (N - N0);
  const T dJx = -c.lambda7 * Jx;
  const T dJy = -c.lambda7 * Jy;
  const T tr = dxx + dyy;
  T fp[9];
  fp[0] = f[0] + T(4.0 / 9.0) * (T(0.25) * dN - T(1.5) * tr);
  const T axc = -T(1.5) * tr - T(0.5) * dN;
  const T sx = T(1.0 / 9.0) * (axc + T(4.5) * dxx);
  const T sy = T(1.0 / 9.0) * (axc + T(4.5) * dyy);
  const T ax = T(1.0 / 9.0) * (T(3) * Gx - T(0.75) * dJx);
  const T ay = T(1.0 / 9.0) * (T(3) * Gy - T(0.75) * dJy);
  fp[8] = f[8] + (sx + ax);
  fp[4] = f[4] + (sx - ax);
  fp[2] = f[2] + (sy + ay);
  fp[6] = f[6] + (sy - ay);
  const T dgc = T(3) * tr + dN;
  const T dsp = T(1.0 / 36.0) * (dgc + T(9) * dxy);
  const T dsm = T(1.0 / 36.0) * (dgc - T(9) * dxy);
  const T a15 = T(1.0 / 36.0) * (T(3) * (Gx + Gy) + T(1.5) * (dJx + dJy));
  const T a73 = T(1.0 / 36.0) * (T(3) * (Gx - Gy) + T(1.5) * (dJx - dJy));
  fp[1] = f[1] + (dsp + a15);
  fp[5] = f[5] + (dsp - a15);
  fp[7] = f[7] + (dsm + a73);
  fp[3] = f[3] + (dsm - a73);
  const T irho = T(1) / rho;
  const T aR = rR * irho, aB = rB * irho;
  const T moving = (c.c1R * rR + c.c1B * rB) * irho;
  const T X = rR * rB * irho;
  const T q = c.recolor ? c.beta18 * X * moving : T(0);
  const T qa = q * T(1.0 / 9.0);
  const T qd = q * T(1.0 / 36.0) * T(0.70710678118654752440);

  // ---- backward ------------------------------------------------------------
  // recolour: R_i = aR fp_i + t_i, B_i = aB fp_i - t_i (t_0 = 0)
  T lfp[9];
  T laR = T(0), laB = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    lfp[i] = aR * lR[i] + aB * lB[i];
    laR += fp[i] * lR[i];
    laB += fp[i] * lB[i];
  }
  const T lt1 = (lR[1] - lB[1]) - (lR[5] - lB[5]);
  const T lt3 = (lR[3] - lB[3]) - (lR[7] - lB[7]);
  const T lt2 = (lR[2] - lB[2]) - (lR[6] - lB[6]);
  const T lt8 = (lR[8] - lB[8]) - (lR[4] - lB[4]);
  T lmx = T(0), lmy = T(0), lq = T(0);
  if (c.recolor) {
    // t8 = qa mx, t2 = qa my, t1 = qd (mx + my), t3 = qd (my - mx)
    lmx = qa * lt8 + qd * (lt1 - lt3);
    lmy = qa * lt2 + qd * (lt1 + lt3);
    lq = (lt8 * mx + lt2 * my) * T(1.0 / 9.0) +
         (lt1 * (mx + my) + lt3 * (my - mx)) * (T(1.0 / 36.0) * T(0.70710678118654752440));
  }
  // q = beta18 X moving, X = rR rB / rho, moving = (c1R rR + c1B rB) / rho
  T lrR = T(0), lrB = T(0), lrho = T(0);
  {
    const T lX = lq * c.beta18 * moving;
    const T lmv = lq * c.beta18 * X;
    lrR += lX * rB * irho + lmv * c.c1R * irho;
    lrB += lX * rR * irho + lmv * c.c1B * irho;
    lrho -= (lX * X + lmv * moving) * irho;
    lrR += laR * irho;
    lrB += laB * irho;
    lrho -= (laR * aR + laB * aB) * irho;
  }
  // reconstruction f+ = f + M^{-1}(m+ - m)
  T lf[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) lf[i] = lfp[i];
  T ltr = T(0), ldxx = T(0), ldyy = T(0), ldxy = T(0), ldN = T(0), ldJx = T(0), ldJy = T(0);
  T lGx = T(0), lGy = T(0);
  ldN += lfp[0] * T(1.0 / 9.0);
  ltr -= lfp[0] * T(2.0 / 3.0);
  const T lsx = lfp[8] + lfp[4], lsy = lfp[2] + lfp[6];
  const T lax = lfp[8] - lfp[4], lay = lfp[2] - lfp[6];
  const T laxc = (lsx + lsy) * T(1.0 / 9.0);
  ldxx += lsx * T(0.5);
  ldyy += lsy * T(0.5);
  ltr -= T(1.5) * laxc;
  ldN -= T(0.5) * laxc;
  lGx += lax * T(1.0 / 3.0);
  ldJx -= lax * T(1.0 / 12.0);
  lGy += lay * T(1.0 / 3.0);
  ldJy -= lay * T(1.0 / 12.0);
  const T ldsp = lfp[1] + lfp[5], ldsm = lfp[7] + lfp[3];
  const T la15 = lfp[1] - lfp[5], la73 = lfp[7] - lfp[3];
  const T ldgc = (ldsp + ldsm) * T(1.0 / 36.0);
  ldxy += (ldsp - ldsm) * T(0.25);
  lGx += (la15 + la73) * T(1.0 / 12.0);
  lGy += (la15 - la73) * T(1.0 / 12.0);
  ldJx += (la15 + la73) * T(1.0 / 24.0);
  ldJy += (la15 - la73) * T(1.0 / 24.0);
  ltr += T(3) * ldgc;
  ldN += ldgc;
  ldxx += ltr;
  ldyy += ltr;
  // relaxation
  const T lJx = -c.lambda7 * ldJx, lJy = -c.lambda7 * ldJy;
  const T lN = -c.lambda6 * ldN;
  if (!c.ghost_eq) {
    const T lN0 = c.lambda6 * ldN;
    lrR += T(1.8) * c.alphaR * lN0;
    lrB += T(1.8) * c.alphaB * lN0;
    lrho -= T(0.8) * lN0;
  }
  // d = C - l3 q
  T lCxx = ldxx, lCyy = ldyy, lCxy = ldxy;
  T ll3 = -(ldxx * qxx + ldyy * qyy + ldxy * qxy);
  const T lpxx = -l3 * ldxx, lpyy = -l3 * ldyy, lpxy = -l3 * ldxy;
  const T lP = l3 * (ldxx + ldyy);
  lrho += l3 * (ldxx * ux * ux + ldyy * uy * uy + ldxy * ux * uy);
  T lux = l3 * rho * (T(2) * ux * ldxx + uy * ldxy);
  T luy = l3 * rho * (T(2) * uy * ldyy + ux * ldxy);
  lrR += c.c06R * lP;
  lrB += c.c06B * lP;
  // correction tensor
  T lk = lCxx * (T(2) * ux * ex - iso) + lCyy * (T(2) * uy * ey - iso) + lCxy * (ux * ey + uy * ex);
  lux += k * (T(2) * ex * lCxx + ey * lCxy);
  luy += k * (T(2) * ey * lCyy + ex * lCxy);
  const T lex = k * (T(2) * ux * lCxx + uy * lCxy);
  const T ley = k * (T(2) * uy * lCyy + ux * lCxy);
  lGx += lex;
  lGy += ley;
  T ldPx = -lex, ldPy = -ley;
  const T liso = -k * (lCxx + lCyy);
  lux += dPx * liso;
  luy += dPy * liso;
  ldPx += ux * liso;
  ldPy += uy * liso;
  lrho -= theta * liso * T(1.0 / 3.0);
  const T lth = -rho * liso * T(1.0 / 3.0);
  ll3 -= T(0.5) * lk;
  // l3 = 2 / (6 nu + 1), nu linear in rho^N
  const T lnu = -T(3) * l3 * l3 * ll3;
  const T lrN = (c.hnuR - c.hnuB) * lnu;
  // modes of f
  lf[0] += lN;
  {
    const T e = lpxx + lpyy + T(4) * lN;  // common to the diagonal links
    lf[1] += e + lpxy + T(4) * (lJx + lJy);
    lf[5] += e + lpxy - T(4) * (lJx + lJy);
    lf[3] += e - lpxy + T(4) * (lJy - lJx);
    lf[7] += e - lpxy - T(4) * (lJy - lJx);
    lf[8] += lpxx - T(2) * lN - T(2) * lJx;
    lf[4] += lpxx - T(2) * lN + T(2) * lJx;
    lf[2] += lpyy - T(2) * lN - T(2) * lJy;
    lf[6] += lpyy - T(2) * lN + T(2) * lJy;
  }
  lrR += lrho;
  lrB += lrho;

#pragma unroll
  for (int i = 0; i < 9; ++i) out[A_F + i] = lf[i];
  out[A_RR] = lrR;
  out[A_RB] = lrB;
  out[A_UX] = lux;
  out[A_UY] = luy;
  out[A_GX] = lGx;
  out[A_GY] = lGy;
  out[A_DPX] = ldPx;
  out[A_DPY] = ldPy;
  out[A_TH] = lth;
  out[A_RN] = lrN;
  out[A_MX] = lmx;
  out[A_MY] = lmy;
}

static __device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __shared__ double red[4];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// Passes 2-5.  The workspace is [y][WS_PLANES][x] (rows interleaved, as the
// populations): sv, A, B, C, D point at the first plane of their group in row
// 0, plane k of a group at row y starts (y WS_PLANES + k) nx elements after
// it.  dforce is [2][ny][nx].
// ---------------------------------------------------------------------------
__device__ __forceinline__ size_t ws_rs(const Geom& g) { return (size_t)WS_PLANES * (size_t)g.nx; }

// Local part of pass 2 at one site: from the adjoints of u (with the
// transposed div u already added: lux, luy) and of Phi' (lphi), the site's
// saved forward values s and local adjoints a (pointers at the site, planes nx
// apart) give the B values, dL/dG_ext and the site's dL/dsigma term.
template <typename T>
struct Pass2 {
  T b[B_N];
  T lGx, lGy;
  double dsig;
};

template <typename T>
__device__ __forceinline__ Pass2<T> pass2_site(const Coef<T>& c, T sigma, const T* a, const T* s, int nx, T lux,
                                               T luy, T lphi) {
  Pass2<T> q;
  const T rR = s[SV_RR * nx], rB = s[SV_RB * nx];
  const T rho = rR + rB;
  const T ux = s[SV_UX * nx], uy = s[SV_UY * nx];
  const T K = s[SV_K * nx];
  const T gx = s[SV_GNX * nx], gy = s[SV_GNY * nx];
  // Phi' = c06R rR + phiB rB - rho / 3
  T lrR = a[A_RR * nx] + (c.c06R - T(1.0 / 3.0)) * lphi;
  T lrB = a[A_RB * nx] + (c.phiB - T(1.0 / 3.0)) * lphi;
  // u = (j + G/2) / rho
  const T irho = T(1) / rho;
  const T ljx = lux * irho, ljy = luy * irho;
  const T lrho = -(lux * ux + luy * uy) * irho;
  lrR += lrho;
  lrB += lrho;
  q.lGx = a[A_GX * nx] + T(0.5) * ljx;
  q.lGy = a[A_GY * nx] + T(0.5) * ljy;
  // G = sigma K g / 2 + G_ext
  const T lGg = q.lGx * gx + q.lGy * gy;
  q.dsig = 0.5 * (double)K * (double)lGg;
  q.b[B_RR] = lrR;
  q.b[B_RB] = lrB;
  q.b[B_JX] = ljx;
  q.b[B_JY] = ljy;
  q.b[B_K] = c.fixed_K ? T(0) : T(0.5) * sigma * lGg;
  q.b[B_GX] = T(0.5) * sigma * K * q.lGx;
  q.b[B_GY] = T(0.5) * sigma * K * q.lGy;
  return q;
}

// pass 2: div u and grad Phi' transposed; u, Phi', G local
template <typename T, bool W, bool M = false>
__global__ void __launch_bounds__(256) force_kernel(Geom g, Coef<T> c, T sigma, Radii r, const T* __restrict__ sv,
                                                    const T* __restrict__ A, T* __restrict__ B,
                                                    T* __restrict__ dforce, double* __restrict__ part,
                                                    const unsigned char* __restrict__ solid) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  const int nx = g.nx, P = g.plane, site = y * nx + x;
  const size_t RS = ws_rs(g), row = (size_t)y * RS + x;
  const T* a = A + row;
  const T* s = sv + row;
  T* b = B + row;
  double acc = 0.0;
  if (M && x < nx && solid_at<W, M>(g, solid, x, y)) {
#pragma unroll
    for (int k = 0; k < B_N; ++k) b[k * nx] = T(0);   // read by the next passes' stencils
  }
  if (x < nx && !solid_at<W, M>(g, solid, x, y)) {
    T lux, luy, lphi;
    if constexpr (M) {
      T tx, ty, wx, wy;
      grad_r(r.u, A + A_TH * nx, RS, nx, g.ny, x, y, tx, ty);
      solid_tap_weights_r(r.u, solid, nx, g.ny, x, y, wx, wy);
      const T lth = a[A_TH * nx];
      lux = a[A_UX * nx] - tx + lth * wx;
      luy = a[A_UY * nx] - ty + lth * wy;
      solid_tap_weights_r(r.p, solid, nx, g.ny, x, y, wx, wy);
      lphi = -div_r(r.p, A + A_DPX * nx, A + A_DPY * nx, RS, nx, g.ny, x, y) + a[A_DPX * nx] * wx +
             a[A_DPY * nx] * wy;
    } else if constexpr (W) {
      T ax, ay, bx, by;
      gradT_walls(r.u, A + A_TH * nx, RS, nx, g.ny, x, y, false, ax, ay);  // theta = D_x u_x + D_y u_y (u_y odd)
      gradT_walls(r.u, A + A_TH * nx, RS, nx, g.ny, x, y, true, bx, by);
      lux = a[A_UX * nx] + ax;
      luy = a[A_UY * nx] + by;
      gradT_walls(r.p, A + A_DPX * nx, RS, nx, g.ny, x, y, false, ax, ay);  // grad Phi' (even)
      gradT_walls(r.p, A + A_DPY * nx, RS, nx, g.ny, x, y, false, bx, by);
      lphi = ax + by;
    } else {
      T tx, ty;
      grad_r(r.u, A + A_TH * nx, RS, nx, g.ny, x, y, tx, ty);
      lux = a[A_UX * nx] - tx;  // theta = div u: transpose -grad
      luy = a[A_UY * nx] - ty;
      lphi = -div_r(r.p, A + A_DPX * nx, A + A_DPY * nx, RS, nx, g.ny, x, y);
    }
    const Pass2<T> q = pass2_site(c, sigma, a, s, nx, lux, luy, lphi);
    if (dforce) {
      dforce[site] += q.lGx;
      dforce[P + site] += q.lGy;
    }
    acc = q.dsig;
#pragma unroll
    for (int k = 0; k < B_N; ++k) b[k * nx] = q.b[k];
  }
  const double tot = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// ---------------------------------------------------------------------------
// pass 3: K = -div m transposed; m = g / sqrt(|g|^2 + eps^2)
// ---------------------------------------------------------------------------
// Local part of pass 3 at one site: (kx, ky) = the transposed K = -div m
// applied to lambda_K; bgx, bgy: the site's B_GX, B_GY.
template <typename T>
__device__ __forceinline__ void pass3_site(const Coef<T>& c, const T* a, const T* s, int nx, T bgx, T bgy, T kx, T ky,
                                           T& cgx, T& cgy) {
  const T lmx = a[A_MX * nx] + kx;  // -(-D)^T = D
  const T lmy = a[A_MY * nx] + ky;
  const T gx = s[SV_GNX * nx], gy = s[SV_GNY * nx];
  const T s2 = gx * gx + gy * gy + c.eps2;
  const T is = T(1) / sqrt(s2);
  const T dot = (lmx * gx + lmy * gy) * is * is * is;
  cgx = bgx + lmx * is - gx * dot;
  cgy = bgy + lmy * is - gy * dot;
}


// One extra row of workgroups, dispatched first (blockIdx.y == 0; lattice row y
// is blockIdx.y - 1): its first workgroup adds the sum of pass 2's
// per-workgroup dL/dsigma partials to *dsigma while the other workgroups run
// the pass.  Each thread sums a fixed strided subset in 8 interleaved
// accumulators, combined in a fixed order (deterministic).
template <typename T, bool W, bool M = false>
__global__ void __launch_bounds__(256) director_kernel(Geom g, Coef<T> c, Radii r, const T* __restrict__ sv,
                                                       const T* __restrict__ A, const T* __restrict__ B,
                                                       T* __restrict__ C, const double* __restrict__ part,
                                                       int npart, double* dsigma,
                                                       const unsigned char* __restrict__ solid) {
  if (blockIdx.y == 0) {
    if (blockIdx.x == 0 && dsigma) {
      constexpr int U = 8, BS = 256;
      double v[U] = {};
      int i = threadIdx.x;
      for (; i + (U - 1) * BS < npart; i += U * BS) {
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] += part[i + k * BS];
      }
#pragma unroll
      for (int k = 0; k < U - 1; ++k)
        if (i + k * BS < npart) v[k] += part[i + k * BS];
      const double tot = block_sum(((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])));
      if (threadIdx.x == 0) *dsigma += tot;
    }
    return;
  }
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y - 1;
  if (x >= g.nx) return;
  const int nx = g.nx;
  const size_t RS = ws_rs(g), row = (size_t)y * RS + x;
  T* o = C + row;
  if (solid_at<W, M>(g, solid, x, y)) {
    if (M) o[C_GX * nx] = o[C_GY * nx] = T(0);
    return;
  }
  const T* a = A + row;
  const T* b = B + row;
  const T* s = sv + row;
  T kx, ky;
  if constexpr (M) {  // lambda_m = -D^T lambda_K = D lambda_K - lambda_K(s) (solid tap weights)
    T wx, wy;
    grad_r(r.k, B + B_K * nx, RS, nx, g.ny, x, y, kx, ky);
    solid_tap_weights_r(r.k, solid, nx, g.ny, x, y, wx, wy);
    const T lk = b[B_K * nx];
    kx -= lk * wx;
    ky -= lk * wy;
  } else if constexpr (W) {  // K = -(D_x m_x + D_y m_y), m_y odd: lambda_m = -D^T lambda_K
    T ax, ay, bx, by;
    gradT_walls(r.k, B + B_K * nx, RS, nx, g.ny, x, y, false, ax, ay);
    gradT_walls(r.k, B + B_K * nx, RS, nx, g.ny, x, y, true, bx, by);
    kx = -ax;
    ky = -by;
  } else {
    grad_r(r.k, B + B_K * nx, RS, nx, g.ny, x, y, kx, ky);
  }
  pass3_site(c, a, s, nx, b[B_GX * nx], b[B_GY * nx], kx, ky, o[C_GX * nx], o[C_GY * nx]);
}

// ---------------------------------------------------------------------------
// pass 4: grad rho^N transposed; colour index
// ---------------------------------------------------------------------------
// Local part of pass 4 at one site: dv = div lambda_g (the transposed
// grad rho^N with its sign); brr, brb: the site's B_RR, B_RB.
template <typename T>
__device__ __forceinline__ void pass4_site(const Coef<T>& c, const T* a, const T* s, int nx, T brr, T brb, T dv,
                                           T& drr, T& drb) {
  const T lrN = a[A_RN * nx] - dv;
  const T ra = s[SV_RR * nx] * c.inv_rho0R, rb = s[SV_RB * nx] * c.inv_rho0B;
  const T is = T(1) / (ra + rb);
  const T w = T(2) * lrN * is * is;
  drr = brr + w * rb * c.inv_rho0R;
  drb = brb - w * ra * c.inv_rho0B;
}


template <typename T, bool W, bool M = false>
__global__ void __launch_bounds__(256) colour_kernel(Geom g, Coef<T> c, Radii r, const T* __restrict__ sv,
                                                     const T* __restrict__ A, const T* __restrict__ B,
                                                     const T* __restrict__ C, T* __restrict__ D,
                                                     const unsigned char* __restrict__ solid) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const int nx = g.nx;
  const size_t RS = ws_rs(g), row = (size_t)y * RS + x;
  T* o = D + row;
  if (solid_at<W, M>(g, solid, x, y)) {
    if (M) o[D_RR * nx] = o[D_RB * nx] = T(0);
    return;
  }
  const T* cc = C + row;
  T dv;
  if constexpr (M) {  // lambda_rhoN += D^T lambda_g = -div lambda_g + lambda_g(s) . (solid tap weights)
    T wx, wy;
    solid_tap_weights_r(r.g, solid, nx, g.ny, x, y, wx, wy);
    dv = div_r(r.g, C + C_GX * nx, C + C_GY * nx, RS, nx, g.ny, x, y) - cc[C_GX * nx] * wx - cc[C_GY * nx] * wy;
  } else if constexpr (W) {  // g = grad rho^N (even): lambda_rhoN += D_x^T lambda_gx + D_y^T lambda_gy
    T ax, ay, bx, by;
    gradT_walls(r.g, C + C_GX * nx, RS, nx, g.ny, x, y, false, ax, ay);
    gradT_walls(r.g, C + C_GY * nx, RS, nx, g.ny, x, y, false, bx, by);
    dv = -(ax + by);
  } else {
    dv = div_r(r.g, C + C_GX * nx, C + C_GY * nx, RS, nx, g.ny, x, y);
  }
  const T* b = B + row;
  pass4_site(c, A + row, sv + row, nx, b[B_RR * nx], b[B_RB * nx], dv, o[D_RR * nx], o[D_RB * nx]);
}

// ---------------------------------------------------------------------------
// pass 5: pre-collision adjoints and the transposed pull gather:
// lambda_t[C][i](s) = dL/dC_i(s + c_i), dL/dC_i = lambda_f_i + lambda_rho_C + lambda_j . c_i
// ---------------------------------------------------------------------------
template <typename T, bool W, bool M = false>
__global__ void __launch_bounds__(256) push_kernel(Geom g, const T* __restrict__ A, const T* __restrict__ B,
                                                   const T* __restrict__ D, T* __restrict__ out,
                                                   const unsigned char* __restrict__ solid) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const int nx = g.nx;
  const size_t RS = ws_rs(g);
  if (solid_at<W, M>(g, solid, x, y)) {  // no fluid site reads a solid site's words
#pragma unroll
    for (int q = 0; q < 18; ++q) out[((size_t)y * 18 + q) * nx + x] = T(0);
    return;
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = link_cx(i), cy = link_cy(i);
    int xs = x + cx, ys = y + cy;
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
    // the word is pulled by link i of site s + c_i, or, when that site is
    // solid, bounced back into link opp(i) of s itself
    const bool bounce = solid_at<W, M>(g, solid, xs, ys);
    const int k = bounce ? link_opp(i) : i;
    const size_t r = bounce ? (size_t)y * RS + x : (size_t)ys * RS + xs;
    const T common = A[r + (A_F + k) * nx] + T(link_cx(k)) * B[r + B_JX * nx] + T(link_cy(k)) * B[r + B_JY * nx];
    out[((size_t)y * 18 + i) * nx + x] = common + D[r + D_RR * nx];
    out[((size_t)y * 18 + 9 + i) * nx + x] = common + D[r + D_RB * nx];
  }
}

// ---------------------------------------------------------------------------
// adjoint of the colour-index field of the pre-collision state:
// lambda[C][i](s) = dL/drho^N(s + c_i) * drho^N/drho_C(s + c_i)
// ---------------------------------------------------------------------------
// M: a mask of solid sites (bnc: the bounce bits of the masked gather)
template <typename S, bool M = false>
__global__ void __launch_bounds__(256) rhoN_adjoint_kernel(const void* popsv, Geom g, Coef<typename S::math> c,
                                                           const typename S::math* __restrict__ lrN,
                                                           typename S::math* __restrict__ out,
                                                           const unsigned char* __restrict__ solid,
                                                           const unsigned char* __restrict__ bnc) {
  using T = typename S::math;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  auto is_solid = [&](int xx, int yy) { return M ? solid[(size_t)yy * g.nx + xx] != 0 : solid_row(g, yy); };
  if (is_solid(x, y)) {
#pragma unroll
    for (int q = 0; q < 18; ++q) out[((size_t)y * 18 + q) * g.nx + x] = typename S::math(0);
    return;
  }
  const int E = (int)sizeof(typename S::W);
  // word i of site s is pulled by site r = s + c_i, or, when that site is
  // solid, bounced back into s itself: every site needs rho_R, rho_B of r
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int xs = x + link_cx(i), ys = y + link_cy(i);
    xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
    ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
    if (is_solid(xs, ys)) {
      xs = x;
      ys = y;
    }
    Cols cols;
    cols.o = xs * E;
    cols.m = (xs == 0 ? g.nx - 1 : xs - 1) * E;
    cols.p = (xs == g.nx - 1 ? 0 : xs + 1) * E;
    typename S::W w[S::NW];
    if constexpr (M) {
      gather_words<S, false, true>(popsv, g, ys, cols, w, bounce_bits_at(bnc, g, ys, xs));
    } else {
      gather_words_any<S>(popsv, g, ys, cols, w);
    }
    T R[9], B[9];
    decode<S>(w, c, R, B);
    T rR = T(0), rB = T(0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      rR += R[k];
      rB += B[k];
    }
    const T a = rR * c.inv_rho0R, b = rB * c.inv_rho0B;
    const T is = T(1) / (a + b);
    const T wgt = T(2) * lrN[ys * g.nx + xs] * is * is;
    out[((size_t)y * 18 + i) * g.nx + x] = wgt * b * c.inv_rho0R;
    out[((size_t)y * 18 + 9 + i) * g.nx + x] = -wgt * a * c.inv_rho0B;
  }
}

// ---------------------------------------------------------------------------
// adjoint of the initial state (rest state of rho^N_0, written un-streamed):
// dL/drho^N_0(r) = sum_{C,i} lambda_0[C][i](r - c_i) d(rho_C phi_i)(r)/drho^N_0
// ---------------------------------------------------------------------------
//
// M: with a mask, a fluid site's word i holds the rest population of link
// opp(i) at the site itself when s + c_i is solid (lbm_set_solid re-encodes
// the rest state so), and solid sites hold nothing.
template <typename T, bool M = false>
__global__ void __launch_bounds__(256) init_adjoint_kernel(const T* __restrict__ rhoN0, const T* __restrict__ lam0,
                                                           Geom g, Coef<T> c, T rho0R, T rho0B,
                                                           T* __restrict__ out, const unsigned char* __restrict__ solid) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  auto is_solid = [&](int xx, int yy) { return M ? solid[(size_t)yy * g.nx + xx] != 0 : solid_row(g, yy); };
  if (x >= g.nx || is_solid(x, y)) return;
  const int site = y * g.nx + x;
  const T rn = rhoN0[site];
  const T rR = rho0R * (T(1) + rn) * T(0.5), rB = rho0B * (T(1) - rn) * T(0.5);
  const T dR = rho0R * T(0.5), dB = -rho0B * T(0.5);
  const T rho = rR + rB, drho = dR + dB;
  const T irho = T(1) / rho;
  const T a0 = c.alphaR * rR + c.alphaB * rB, da0 = c.alphaR * dR + c.alphaB * dB;
  const T mv = c.c1R * rR + c.c1B * rB, dmv = c.c1R * dR + c.c1B * dB;
  T acc = T(0);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    int xs = x - link_cx(i), ys = y - link_cy(i);
    xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
    ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
    T phi, dphi;
    if (i == 0) {
      phi = a0 * irho;
      dphi = (da0 - phi * drho) * irho;
    } else {
      const T wt = (i & 1) ? T(1.8 / 36.0) : T(1.8 / 9.0);
      phi = wt * mv * irho;
      dphi = wt * (dmv - mv * irho * drho) * irho;
    }
    // word i at s - c_i holds the rest population of link i at s when s - c_i
    // is fluid; with walls, word i at s itself holds that of link opp(i) (the
    // same rest fraction) when s + c_i is solid
    if (!is_solid(xs, ys)) {
      const T* l = lam0 + (size_t)ys * 18 * g.nx + xs;  // [y][C i][x], as the populations
      acc += l[i * g.nx] * (dR * phi + rR * dphi) + l[(9 + i) * g.nx] * (dB * phi + rB * dphi);
    }
    if (M ? is_solid(wrapi(x + link_cx(i), g.nx), wrapi(y + link_cy(i), g.ny)) : solid_row(g, y + link_cy(i))) {
      const T* l = lam0 + (size_t)y * 18 * g.nx + x;
      acc += l[i * g.nx] * (dR * phi + rR * dphi) + l[(9 + i) * g.nx] * (dB * phi + rB * dphi);
    }
  }
  out[site] += acc;
}

}  // namespace adj
}  // namespace chromo
