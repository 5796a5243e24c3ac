// Device code of the chromodynamic MRT lattice Boltzmann step for gfx950.
//
// One fused kernel performs a whole time step (Sec. II, Sec. III and App. A of
// Spendlove et al., arXiv 2005.04642): pull-streaming gather, colour densities
// and moments, colour index, App. B gradient and director, curvature and
// Lishchuk force with Guo's velocity, density-difference correction tensor,
// modal relaxation and reconstruction, d'Ortona recolour, store.
//
// Work decomposition ("march"): a workgroup owns a strip of TX lattice columns
// and a chunk of rows and walks up the chunk three rows at a time.  The chain of
// stencils (rho^N -> n -> K, G, u -> div u; Phi' -> grad Phi') needs rho^N up to
// 9 rows ahead of the row being written, so each iteration works on four rows
// bands at once:
//     M  row v+9 : gather 18 populations, moments, rho^N        -> LDS ring
//     N  row v+6 : grad rho^N, director m = grad/|grad|         -> LDS ring
//     U  row v+3 : K = -div m, G, u, Phi'                       -> LDS ring
//     O  row v   : grad Phi', div u, C, collide, recolour, store
// Populations are read once per strip from HBM; per-row fields live in 12-row
// LDS rings (the halo in x is recomputed by the strip's edge threads); the
// moments a thread needs nine rows later stay in its registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chromo {

constexpr int NR = 3;     // rows per march iteration, one per thread row
constexpr int RING = 12;  // LDS ring depth in rows (4 iterations x NR)

template <typename T>
struct Coef {
  T inv_rho0R, inv_rho0B;  // 1/rho_0C
  T alphaR, alphaB;        // alpha_C
  T c1R, c1B;              // 1 - alpha_C
  T c06R, c06B;            // 3/5 (1 - alpha_C): isotropic pressure P = c06R rho_R + c06B rho_B
  T phiB;                  // 3/5 (1 - alpha_R) Lambda: Phi' = c06R rho_R + phiB rho_B - rho/3
  T hnuR, hnuB;            // nu_C / 2
  T half_sigma;            // sigma / 2
  T beta18;                // 9/5 beta
  T lambda6, keepJ;        // lambda_6, 1 - lambda_7
  T gx, gy, K_fixed, eps2;
  int ghost_eq, fixed_K, recolor;
};

struct Geom {
  int nx, ny, walls, F;    // F = fluid rows: ny, or ny - 2 with walls
  int TX, nstrips, TY, nchunks;
  int plane;               // nx * ny
};

template <typename T>
struct StepArgs {
  const T* __restrict__ src;
  T* __restrict__ dst;
  const T* __restrict__ force;  // [2][ny][nx] or null
  T* out_rho;                   // fields mode outputs ([ny][nx] or null)
  T* out_ux;
  T* out_uy;
  T* out_rhoN;
  Geom g;
  Coef<T> c;
};

// Virtual row v of the march (fluid-row index, any integer) -> physical row of
// the lattice and whether it is a mirror image.  y periodic: plain wrap.
// Walls: the fluid strip is reflected about the two wall planes, which is the
// picture every stencil near a wall sees.
__device__ __forceinline__ void virt_row(int v, const Geom& g, int& phys, bool& refl) {
  if (!g.walls) {
    int r = v % g.ny;
    if (r < 0) r += g.ny;
    phys = r;
    refl = false;
  } else {
    const int P = 2 * g.F;
    int t = v % P;
    if (t < 0) t += P;
    if (t < g.F) {
      phys = 1 + t;
      refl = false;
    } else {
      phys = 1 + (P - 1 - t);
      refl = true;
    }
  }
}

// Pull-streaming gather of the 18 pre-collision populations of site (x, p):
// f_i(r) = buf_i(r - c_i), or buf_opp(i)(r) when r - c_i is a solid row
// (half-way bounce-back).  Link order c0..c8 as in the public header.
template <typename T>
__device__ __forceinline__ void gather(const T* __restrict__ src, const Geom& g, int p,
                                       int xm, int x, int xp, T R[9], T B[9]) {
  const int nx = g.nx;
  const int plane = g.plane;
  int rm = p - 1, rp = p + 1;
  bool bm = false, bp = false;
  if (g.walls) {
    bm = (rm == 0);
    bp = (rp == g.ny - 1);
  } else {
    if (rm < 0) rm += g.ny;
    if (rp >= g.ny) rp -= g.ny;
  }
  const int o_p = p * nx, o_m = rm * nx, o_pp = rp * nx;
  // source element offsets within a plane
  const int s0 = o_p + x;
  const int s1 = bm ? o_p + x : o_m + xm;
  const int s2 = bm ? o_p + x : o_m + x;
  const int s3 = bm ? o_p + x : o_m + xp;
  const int s4 = o_p + xp;
  const int s5 = bp ? o_p + x : o_pp + xp;
  const int s6 = bp ? o_p + x : o_pp + x;
  const int s7 = bp ? o_p + x : o_pp + xm;
  const int s8 = o_p + xm;
  // planes read (bounce-back reads the opposite link at the own site)
  const int q1 = bm ? 5 : 1, q2 = bm ? 6 : 2, q3 = bm ? 7 : 3;
  const int q5 = bp ? 1 : 5, q6 = bp ? 2 : 6, q7 = bp ? 3 : 7;
#pragma unroll
  for (int col = 0; col < 2; ++col) {
    const T* b = src + col * 9 * plane;
    T* out = col ? B : R;
    out[0] = b[s0];
    out[1] = b[q1 * plane + s1];
    out[2] = b[q2 * plane + s2];
    out[3] = b[q3 * plane + s3];
    out[4] = b[4 * plane + s4];
    out[5] = b[q5 * plane + s5];
    out[6] = b[q6 * plane + s6];
    out[7] = b[q7 * plane + s7];
    out[8] = b[8 * plane + s8];
  }
}

// Moments of one site: colour densities and the nine modes m = M f of f = R + B
// (App. A / Table A1 projectors 1, c_x, c_y, c_x^2, c_y^2, c_x c_y, g, g c_x, g c_y),
// summed with antisymmetric pair differences.  mom[] layout:
//   0 rho_R  1 rho_B  2 j_x  3 j_y  4 Pi_xx  5 Pi_yy  6 Pi_xy  7 N  8 J_x  9 J_y
template <typename T>
__device__ __forceinline__ void site_moments(const T R[9], const T B[9], bool refl, T mom[10]) {
  T rR = ((R[0] + R[2]) + (R[4] + R[6])) + ((R[1] + R[3]) + (R[5] + R[7])) + R[8];
  T rB = ((B[0] + B[2]) + (B[4] + B[6])) + ((B[1] + B[3]) + (B[5] + B[7])) + B[8];
  T f[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) f[i] = R[i] + B[i];
  const T d15 = f[1] - f[5], d37 = f[3] - f[7], d84 = f[8] - f[4], d26 = f[2] - f[6];
  const T sd = (f[1] + f[5]) + (f[3] + f[7]);
  T jx = (d15 - d37) + d84;
  T jy = (d15 + d37) + d26;
  const T pxx = sd + (f[4] + f[8]);
  const T pyy = sd + (f[2] + f[6]);
  T pxy = (f[1] + f[5]) - (f[3] + f[7]);
  const T N = f[0] - T(2) * ((f[2] + f[6]) + (f[4] + f[8])) + T(4) * sd;
  const T Jx = T(4) * (d15 - d37) - T(2) * d84;
  T Jy = T(4) * (d15 + d37) - T(2) * d26;
  if (refl) {  // mirror image about a wall plane: y-odd modes change sign
    jy = -jy;
    pxy = -pxy;
    Jy = -Jy;
  }
  mom[0] = rR; mom[1] = rB; mom[2] = jx; mom[3] = jy; mom[4] = pxx;
  mom[5] = pyy; mom[6] = pxy; mom[7] = N; mom[8] = Jx; mom[9] = Jy;
}

__device__ __forceinline__ int ring_row(int r) {
  r %= RING;
  return r < 0 ? r + RING : r;
}

// App. B first-derivative stencil coefficients b_N (radius 1: 3; radius 3:
// 9/2, -9/10, 1/10), applied to sum_i w_i c_i f(r + N c_i).
template <int R, typename T>
__device__ __forceinline__ T stencil_b(int n) {
  if (R == 1) return T(3);
  return n == 1 ? T(4.5) : (n == 2 ? T(-0.9) : T(0.1));
}

// (d/dx, d/dy) of a ring field at (ring row `row`, column tx).
template <int R, int NTX, typename T>
__device__ __forceinline__ void ring_grad(const T (*s)[NTX], int row, int tx, T& gx, T& gy) {
  const T wd = T(1.0 / 36.0), wa = T(1.0 / 9.0);
  gx = T(0);
  gy = T(0);
  const T* md = &s[ring_row(row)][tx];
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T b = stencil_b<R, T>(n);
    const T* up = &s[ring_row(row + n)][tx];
    const T* dn = &s[ring_row(row - n)][tx];
    const T d1 = up[n] - dn[-n];
    const T d3 = up[-n] - dn[n];
    const T d8 = md[n] - md[-n];
    const T d2 = up[0] - dn[0];
    gx += b * (wd * (d1 - d3) + wa * d8);
    gy += b * (wd * (d1 + d3) + wa * d2);
  }
}

// d vx/dx + d vy/dy of a ring vector field.
template <int R, int NTX, typename T>
__device__ __forceinline__ T ring_div(const T (*sx)[NTX], const T (*sy)[NTX], int row, int tx) {
  const T wd = T(1.0 / 36.0), wa = T(1.0 / 9.0);
  T acc = T(0);
  const T* mdx = &sx[ring_row(row)][tx];
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T b = stencil_b<R, T>(n);
    const T* upx = &sx[ring_row(row + n)][tx];
    const T* dnx = &sx[ring_row(row - n)][tx];
    const T* upy = &sy[ring_row(row + n)][tx];
    const T* dny = &sy[ring_row(row - n)][tx];
    const T d1 = upx[n] - dnx[-n];
    const T d3 = upx[-n] - dnx[n];
    const T d8 = mdx[n] - mdx[-n];
    const T e1 = upy[n] - dny[-n];
    const T e3 = upy[-n] - dny[n];
    const T e2 = upy[0] - dny[0];
    acc += b * (wd * ((d1 - d3) + (e1 + e3)) + wa * (d8 + e2));
  }
  return acc;
}

template <typename T, int NTX>
struct Smem {
  T rhoN[RING][NTX];
  T mx[RING][NTX];
  T my[RING][NTX];
  T ux[RING][NTX];
  T uy[RING][NTX];
  T phi[RING][NTX];
};

template <typename T>
struct March {
  T mom[4][10];  // moments of rows v+9 .. v (one slot per iteration)
  T gn[2][2];    // grad rho^N, from band N to band U
  T gr[2][2];    // G, from band U to band O
  T pr[9], pb[9];  // populations prefetched for the next band-M row
};

struct Thread {
  int tx, ty, xg, xm, xp, ya, yb, nit;
  bool own;
};

// Collision, recolour and store for one site (band O).
template <typename T, bool FIELDS>
__device__ __forceinline__ void collide_store(const StepArgs<T>& a, const T m[10], T ux, T uy,
                                              T Gx, T Gy, T dPx, T dPy, T theta, T rhoN,
                                              T mx, T my, int p, int x) {
  const Coef<T>& c = a.c;
  const T rR = m[0], rB = m[1];
  const T rho = rR + rB;
  const int site = p * a.g.nx + x;
  if (FIELDS) {
    if (a.out_rho) a.out_rho[site] = rho;
    if (a.out_ux) a.out_ux[site] = ux;
    if (a.out_uy) a.out_uy[site] = uy;
    if (a.out_rhoN) a.out_rhoN[site] = rhoN;
    return;
  }
  // lambda_3 from nu(rho^N) = (2/lambda_3 - 1)/6 (Sec. II), nu linear in rho^N
  const T nu = c.hnuR * (T(1) + rhoN) + c.hnuB * (T(1) - rhoN);
  const T l3 = T(2) / (T(6) * nu + T(1));
  // correction tensor C_ab (App. A, eq. Correction)
  const T k = T(1) - T(0.5) * l3;
  const T iso = ux * dPx + uy * dPy - rho * theta * T(1.0 / 3.0);
  const T Cxx = k * (T(2) * ux * (Gx - dPx) - iso);
  const T Cyy = k * (T(2) * uy * (Gy - dPy) - iso);
  const T Cxy = k * (ux * (Gy - dPy) + uy * (Gx - dPx));
  // modal relaxation (App. A, modal evolution eqs.)
  const T P = c.c06R * rR + c.c06B * rB;
  const T pxx = m[4] - l3 * (m[4] - (P + rho * ux * ux)) + Cxx;
  const T pyy = m[5] - l3 * (m[5] - (P + rho * uy * uy)) + Cyy;
  const T pxy = m[6] - l3 * (m[6] - rho * ux * uy) + Cxy;
  const T N0 = c.ghost_eq ? T(0) : T(1.8) * (c.alphaR * rR + c.alphaB * rB) - T(0.8) * rho;
  const T Np = m[7] - c.lambda6 * (m[7] - N0);
  const T Jxp = c.keepJ * m[8];
  const T Jyp = c.keepJ * m[9];
  const T jxp = m[2] + Gx;
  const T jyp = m[3] + Gy;
  // reconstruction f+ = M^{-1} m+ (closed form of Sec. III / App. A)
  const T tr = pxx + pyy;
  T f[9];
  f[0] = T(4.0 / 9.0) * (T(2) * rho - T(1.5) * tr + T(0.25) * Np);
  const T axc = T(0.5) * rho - T(1.5) * tr - T(0.5) * Np;
  const T sx = T(1.0 / 9.0) * (axc + T(4.5) * pxx);
  const T sy = T(1.0 / 9.0) * (axc + T(4.5) * pyy);
  const T ax = T(1.0 / 9.0) * (T(3) * jxp - T(0.75) * Jxp);
  const T ay = T(1.0 / 9.0) * (T(3) * jyp - T(0.75) * Jyp);
  f[8] = sx + ax;
  f[4] = sx - ax;
  f[2] = sy + ay;
  f[6] = sy - ay;
  const T dgc = -rho + T(3) * tr + Np;
  const T dsp = T(1.0 / 36.0) * (dgc + T(9) * pxy);
  const T dsm = T(1.0 / 36.0) * (dgc - T(9) * pxy);
  const T a15 = T(1.0 / 36.0) * (T(3) * (jxp + jyp) + T(1.5) * (Jxp + Jyp));
  const T a73 = T(1.0 / 36.0) * (T(3) * (jxp - jyp) + T(1.5) * (Jxp - Jyp));
  f[1] = dsp + a15;
  f[5] = dsp - a15;
  f[7] = dsm + a73;
  f[3] = dsm - a73;
  // d'Ortona recolour (Sec. II): t_i = beta phi_i rho_R rho_B / rho (m . c_hat_i)
  const T aR = rR / rho, aB = rB / rho;
  T t1 = T(0), t3 = T(0), t2 = T(0), t8 = T(0);
  if (c.recolor) {
    const T moving = (c.c1R * rR + c.c1B * rB) / rho;
    const T q = c.beta18 * (rR * rB / rho) * moving;
    const T qa = q * T(1.0 / 9.0);
    const T qd = q * T(1.0 / 36.0) * T(0.70710678118654752440);
    t8 = qa * mx;
    t2 = qa * my;
    t1 = qd * (mx + my);
    t3 = qd * (my - mx);
  }
  T R[9], B[9];
  R[0] = aR * f[0];
  B[0] = aB * f[0];
  R[1] = aR * f[1] + t1; B[1] = aB * f[1] - t1;
  R[5] = aR * f[5] - t1; B[5] = aB * f[5] + t1;
  R[3] = aR * f[3] + t3; B[3] = aB * f[3] - t3;
  R[7] = aR * f[7] - t3; B[7] = aB * f[7] + t3;
  R[2] = aR * f[2] + t2; B[2] = aB * f[2] - t2;
  R[6] = aR * f[6] - t2; B[6] = aB * f[6] + t2;
  R[8] = aR * f[8] + t8; B[8] = aB * f[8] - t8;
  R[4] = aR * f[4] - t8; B[4] = aB * f[4] + t8;
  const int plane = a.g.plane;
  T* d = a.dst + site;
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i * plane] = R[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[(9 + i) * plane] = B[i];
}

// One march iteration; S = it mod 4 selects the register-ring slots.
template <int S, typename T, int NTX, int RG, int RK, int RP, int RU, bool FIELDS>
__device__ __forceinline__ void march_iter(int it, const StepArgs<T>& a, Smem<T, NTX>& sm,
                                           March<T>& st, const Thread& t) {
  const Geom& g = a.g;
  const Coef<T>& c = a.c;
  const int tx = t.tx, ty = t.ty;
  const int base = t.ya - 18 + 3 * it + ty;  // band-O virtual row of this thread
  constexpr int sM = S, sU = (S + 2) & 3, sO = (S + 1) & 3;
  // ring rows of the four bands (row index = virtual row - (ya - 18))
  const int rowM = 3 * S + ty + 9, rowN = 3 * S + ty + 6, rowU = 3 * S + ty + 3, rowO = 3 * S + ty;

  // ---- band M: moments and colour index of row base + 9 -------------------
  {
    int p;
    bool refl;
    virt_row(base + 9, g, p, refl);
    T* m = st.mom[sM];
    site_moments(st.pr, st.pb, refl, m);
    const T a0 = m[0] * c.inv_rho0R, b0 = m[1] * c.inv_rho0B;
    sm.rhoN[ring_row(rowM)][tx] = (a0 - b0) / (a0 + b0);
    if (it + 1 < t.nit) {  // prefetch the next band-M row
      int pn;
      bool rn;
      virt_row(base + 12, g, pn, rn);
      gather(a.src, g, pn, t.xm, t.xg, t.xp, st.pr, st.pb);
    }
  }
  __syncthreads();

  // ---- band N: grad rho^N and director of row base + 6 -----------------------
  if (it >= 2 && tx >= RG && tx < NTX - RG) {
    T gx, gy;
    ring_grad<RG, NTX>(sm.rhoN, rowN, tx, gx, gy);
    const T s = sqrt(gx * gx + gy * gy + c.eps2);
    sm.mx[ring_row(rowN)][tx] = gx / s;
    sm.my[ring_row(rowN)][tx] = gy / s;
    st.gn[S & 1][0] = gx;
    st.gn[S & 1][1] = gy;
  }
  __syncthreads();

  // ---- band U: Phi', curvature, force and velocity of row base + 3 ---------
  if (it >= 4) {
    const T* m = st.mom[sU];
    const T rho = m[0] + m[1];
    sm.phi[ring_row(rowU)][tx] = c.c06R * m[0] + c.phiB * m[1] - rho * T(1.0 / 3.0);
    if (tx >= RG + RK && tx < NTX - RG - RK) {
      int p;
      bool refl;
      virt_row(base + 3, g, p, refl);
      T K;
      if (c.fixed_K) {
        K = c.K_fixed;
      } else {
        K = -ring_div<RK, NTX>(sm.mx, sm.my, rowU, tx);  // K = div n, n = -m
      }
      const T gnx = st.gn[(S + 1) & 1][0], gny = st.gn[(S + 1) & 1][1];
      T Gx = c.half_sigma * K * gnx + c.gx;
      T Gy = c.half_sigma * K * gny + (refl ? -c.gy : c.gy);
      if (a.force) {
        const int site = p * g.nx + t.xg;
        Gx += a.force[site];
        Gy += refl ? -a.force[g.plane + site] : a.force[g.plane + site];
      }
      const T inv = T(1) / rho;
      sm.ux[ring_row(rowU)][tx] = (m[2] + T(0.5) * Gx) * inv;
      sm.uy[ring_row(rowU)][tx] = (m[3] + T(0.5) * Gy) * inv;
      st.gr[S & 1][0] = Gx;
      st.gr[S & 1][1] = Gy;
    }
  }
  __syncthreads();

  // ---- band O: correction, collision, recolour, store of row base ----------
  if (it >= 6 && t.own && base < t.yb) {
    const T* m = st.mom[sO];
    T dPx, dPy;
    ring_grad<RP, NTX>(sm.phi, rowO, tx, dPx, dPy);
    const T theta = ring_div<RU, NTX>(sm.ux, sm.uy, rowO, tx);
    const int ro = ring_row(rowO);
    const T ux = sm.ux[ro][tx], uy = sm.uy[ro][tx];
    const T rhoN = sm.rhoN[ro][tx];
    const T mx = sm.mx[ro][tx], my = sm.my[ro][tx];
    const int p = g.walls ? base + 1 : base;
    collide_store<T, FIELDS>(a, m, ux, uy, st.gr[(S + 1) & 1][0], st.gr[(S + 1) & 1][1], dPx, dPy,
                             theta, rhoN, mx, my, p, t.xg);
  }
}

template <typename T, int NTX, int RG, int RK, int RP, int RU, bool FIELDS>
__global__ void __launch_bounds__(NTX * NR, 1) chromo_step_kernel(StepArgs<T> a) {
  constexpr int H = RG + RK + RU;
  static_assert(NTX > 2 * H, "strip must be wider than its halo");
  __shared__ Smem<T, NTX> sm;
  const Geom& g = a.g;
  Thread t;
  t.tx = threadIdx.x % NTX;
  t.ty = threadIdx.x / NTX;
  const int strip = blockIdx.x % g.nstrips;
  const int chunk = blockIdx.x / g.nstrips;
  const int x0 = strip * g.TX;
  const int txe = min(g.TX, g.nx - x0);
  const int col = t.tx - H;
  int xg = (x0 + col) % g.nx;
  if (xg < 0) xg += g.nx;
  t.xg = xg;
  t.xm = xg == 0 ? g.nx - 1 : xg - 1;
  t.xp = xg == g.nx - 1 ? 0 : xg + 1;
  t.own = col >= 0 && col < txe;
  t.ya = chunk * g.TY;
  t.yb = min(g.F, t.ya + g.TY);
  t.nit = 6 + (t.yb - t.ya + 2) / 3;

  March<T> st;
  {
    int p;
    bool refl;
    virt_row(t.ya - 9 + t.ty, g, p, refl);
    gather(a.src, g, p, t.xm, t.xg, t.xp, st.pr, st.pb);
  }
  for (int it = 0; it < t.nit; it += 4) {
    march_iter<0, T, NTX, RG, RK, RP, RU, FIELDS>(it, a, sm, st, t);
    if (it + 1 < t.nit) march_iter<1, T, NTX, RG, RK, RP, RU, FIELDS>(it + 1, a, sm, st, t);
    if (it + 2 < t.nit) march_iter<2, T, NTX, RG, RK, RP, RU, FIELDS>(it + 2, a, sm, st, t);
    if (it + 3 < t.nit) march_iter<3, T, NTX, RG, RK, RP, RU, FIELDS>(it + 3, a, sm, st, t);
  }
}

// ---------------------------------------------------------------------------
// streaming only (test mode): buf'_i(r) = f_i(r)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) stream_only_kernel(const T* __restrict__ src, T* __restrict__ dst, Geom g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;  // fluid row index
  if (x >= g.nx) return;
  const int p = g.walls ? k + 1 : k;
  const int xm = x == 0 ? g.nx - 1 : x - 1;
  const int xp = x == g.nx - 1 ? 0 : x + 1;
  T R[9], B[9];
  gather(src, g, p, xm, x, xp, R, B);
  T* d = dst + p * g.nx + x;
#pragma unroll
  for (int i = 0; i < 9; ++i) d[i * g.plane] = R[i];
#pragma unroll
  for (int i = 0; i < 9; ++i) d[(9 + i) * g.plane] = B[i];
}

// ---------------------------------------------------------------------------
// initial state: pre-collision populations C_i = rho_C phi_i at rest
// (Sec. II equilibrium with u = 0), written "un-streamed" so that the first
// gather of lbm_step reproduces them exactly.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void rest_state(const T* __restrict__ rhoN0, const Coef<T>& c, T rho0R, T rho0B,
                                           int site, int i, T& r, T& b) {
  const T rn = rhoN0[site];
  const T rR = rho0R * (T(1) + rn) * T(0.5);
  const T rB = rho0B * (T(1) - rn) * T(0.5);
  const T rho = rR + rB;
  T phi;
  if (i == 0) {
    phi = (c.alphaR * rR + c.alphaB * rB) / rho;
  } else {
    const T w = (i & 1) ? T(1.0 / 36.0) : T(1.0 / 9.0);
    phi = T(1.8) * w * ((c.c1R * rR + c.c1B * rB) / rho);
  }
  r = rR * phi;
  b = rB * phi;
}

template <typename T>
__global__ void __launch_bounds__(256) init_kernel(const T* __restrict__ rhoN0, T* __restrict__ dst, Geom g,
                                                   Coef<T> c, T rho0R, T rho0B) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  constexpr int CX[9] = {0, 1, 0, -1, -1, -1, 0, 1, 1};
  constexpr int CY[9] = {0, 1, 1, 1, 0, -1, -1, -1, 0};
  constexpr int OPP[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
  const bool solid = g.walls && (y == 0 || y == g.ny - 1);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    T r = T(0), b = T(0);
    if (!solid) {
      int yd = y + CY[i];
      int xd = x + CX[i];
      xd = xd < 0 ? xd + g.nx : (xd >= g.nx ? xd - g.nx : xd);
      if (g.walls && (yd == 0 || yd == g.ny - 1)) {
        rest_state(rhoN0, c, rho0R, rho0B, y * g.nx + x, OPP[i], r, b);  // returns on link opp(i)
      } else {
        yd = yd < 0 ? yd + g.ny : (yd >= g.ny ? yd - g.ny : yd);
        rest_state(rhoN0, c, rho0R, rho0B, yd * g.nx + xd, i, r, b);
      }
    }
    dst[i * g.plane + y * g.nx + x] = r;
    dst[(9 + i) * g.plane + y * g.nx + x] = b;
  }
}

// ---------------------------------------------------------------------------
// per-colour masses in FP64: block partials, then one ordered pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__global__ void __launch_bounds__(256) mass_partial_kernel(const T* __restrict__ pops, Geom g, double* partial) {
  const int row0 = g.walls ? 1 : 0;
  const long long nsite = (long long)g.F * g.nx;
  double sr = 0.0, sb = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < nsite;
       s += (long long)gridDim.x * blockDim.x) {
    const int off = (int)(row0 * g.nx + s);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      sr += (double)pops[i * g.plane + off];
      sb += (double)pops[(9 + i) * g.plane + off];
    }
  }
  sr = wave_sum(sr);
  sb = wave_sum(sb);
  __shared__ double red[2][4];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) {
    red[0][w] = sr;
    red[1][w] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    partial[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

__global__ void __launch_bounds__(256) mass_final_kernel(const double* partial, int nblocks, double* out) {
  double sr = 0.0, sb = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    sr += partial[2 * b];
    sb += partial[2 * b + 1];
  }
  sr = wave_sum(sr);
  sb = wave_sum(sb);
  __shared__ double red[2][4];
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  if (l == 0) {
    red[0][w] = sr;
    red[1][w] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    out[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) fill_rows_kernel(T* a, T* b, T* c, T* d, int nx, int row0, int row1) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= nx) return;
  const T nan = T(__builtin_nan(""));
  const int rows[2] = {row0, row1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int s = rows[k] * nx + x;
    if (a) a[s] = nan;
    if (b) b[s] = nan;
    if (c) c[s] = nan;
    if (d) d[s] = nan;
  }
}

}  // namespace chromo
