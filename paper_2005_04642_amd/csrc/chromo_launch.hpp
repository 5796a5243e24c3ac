// Launchers of the step, field, streaming, initial-state and mass kernels for
// one storage format S.  Included once per format by chromo_<format>.hip, so
// the formats compile as separate translation units.
#pragma once

#include <cstring>

#include "chromo_adjoint.hpp"
#include "chromo_host.hpp"
#include "chromo_solid.hpp"

namespace chromo {
namespace launch {

template <typename S, int MODE = MODE_STEP>
struct Shape {
  static constexpr bool f64 = sizeof(typename S::math) == 8;
  static constexpr int ntx = f64 ? NTX_F64 : (MODE == MODE_ADJ ? NTX_ADJ_F32 : NTX_F32);
  static constexpr int nr = f64 ? NR_F64 : NR_F32;
};

// Per-site constants of the scheme (Sec. II, App. A) in the arithmetic type.
template <typename S>
Coef<typename S::math> make_coef(const lbm_params& p) {
  using T = typename S::math;
  Coef<T> c;
  const double Lam = p.rho0_R / p.rho0_B;
  c.inv_rho0R = (T)(1.0 / p.rho0_R);
  c.inv_rho0B = (T)(1.0 / p.rho0_B);
  c.alphaR = (T)p.alpha_R;
  c.alphaB = (T)p.alpha_B;
  c.c1R = (T)(1.0 - p.alpha_R);
  c.c1B = (T)(1.0 - p.alpha_B);
  c.c06R = (T)(0.6 * (1.0 - p.alpha_R));
  c.c06B = (T)(0.6 * (1.0 - p.alpha_B));
  c.phiB = (T)(0.6 * (1.0 - p.alpha_R) * Lam);
  c.hnuR = (T)(0.5 * p.nu_R);
  c.hnuB = (T)(0.5 * p.nu_B);
  c.half_sigma = (T)(0.5 * p.sigma);
  c.beta18 = (T)(1.8 * p.beta);
  c.lambda6 = (T)p.lambda6;
  c.lambda7 = (T)p.lambda7;
  c.gx = (T)p.gx;
  c.gy = (T)p.gy;
  c.K_fixed = (T)p.K_fixed;
  c.eps2 = (T)(p.eps_n * p.eps_n);
  // rest value of f_i on axis and diagonal links: (9/5) w_i rho_0R (1 - alpha_R)
  const double moving = p.rho0_R * (1.0 - p.alpha_R);
  const double fr[3] = {1.0, 0.2 * moving, 0.05 * moving};
  for (int k = 0; k < 3; ++k) {
    const double f = (double)(T)fr[k];
    c.fref[k] = (T)f;
    c.fq[k] = (T)(f / 1024.0);
    c.inv_fq[k] = (T)(1024.0 / f);
    c.sq[k] = (T)(4.0 * f);
    c.inv_sq[k] = (T)(0.25 / f);
  }
  c.ghost_eq = p.ghost_eq;
  c.fixed_K = (p.flags & LBM_FLAG_FIXED_K) ? 1 : 0;
  c.recolor = (p.flags & LBM_FLAG_NO_RECOLOR) ? 0 : 1;
  return c;
}


// Per-format geometry: byte strides of the storage words ([y][word][x]: the
// NW words of one lattice row are NW consecutive runs of nx words) and the row
// period of the march.
template <typename S>
Geom geom_for(const Geom& g0) {
  Geom g = g0;
  g.pb = (unsigned)g.nx * (unsigned)sizeof(typename S::W);
  g.rb = (unsigned)S::NW * g.pb;
  g.period = g.walls ? 2 * g.F : g.ny;
  g.nr_mod = Shape<S>::nr % g.period;
  return g;
}

template <typename S, int RG, int RK, int RP, int RU, int MODE>
hipError_t march(const StepArgs<typename S::math>& a, hipStream_t s) {
  constexpr int NTX = Shape<S, MODE>::ntx, NR = Shape<S, MODE>::nr;
  const int ntiles = a.g.nstrips * a.g.nchunks;
  const int nblocks = 8 * ((ntiles + 7) / 8);  // whole rounds over the 8 XCDs (see the kernel)
  if (a.g.walls) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, RG, RK, RP, RU, true, MODE>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
  } else {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, RG, RK, RP, RU, false, MODE>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
  }
  return hipGetLastError();
}

template <typename S, int MODE>
hipError_t dispatch_radii(const StepArgs<typename S::math>& a, const int* r, hipStream_t s) {
  const int code = (r[0] == 3) * 8 + (r[1] == 3) * 4 + (r[2] == 3) * 2 + (r[3] == 3);
#define CHROMO_CASE(C, A, B, P, U) \
  case C:                          \
    return march<S, A, B, P, U, MODE>(a, s);
  switch (code) {
    CHROMO_CASE(0, 1, 1, 1, 1)
    CHROMO_CASE(1, 1, 1, 1, 3)
    CHROMO_CASE(2, 1, 1, 3, 1)
    CHROMO_CASE(3, 1, 1, 3, 3)
    CHROMO_CASE(4, 1, 3, 1, 1)
    CHROMO_CASE(5, 1, 3, 1, 3)
    CHROMO_CASE(6, 1, 3, 3, 1)
    CHROMO_CASE(7, 1, 3, 3, 3)
    CHROMO_CASE(8, 3, 1, 1, 1)
    CHROMO_CASE(9, 3, 1, 1, 3)
    CHROMO_CASE(10, 3, 1, 3, 1)
    CHROMO_CASE(11, 3, 1, 3, 3)
    CHROMO_CASE(12, 3, 3, 1, 1)
    CHROMO_CASE(13, 3, 3, 1, 3)
    CHROMO_CASE(14, 3, 3, 3, 1)
    CHROMO_CASE(15, 3, 3, 3, 3)
  }
#undef CHROMO_CASE
  return hipErrorInvalidValue;
}

template <typename S>
StepArgs<typename S::math> args(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force) {
  using T = typename S::math;
  StepArgs<T> a;
  a.src = src;
  a.dst = dst;
  a.force = static_cast<const T*>(force);
  a.out_rho = a.out_ux = a.out_uy = a.out_rhoN = a.out_save = a.out_adj = nullptr;
  a.lam_next = nullptr;
  a.bnc = nullptr;
  a.g = geom_for<S>(g);
  a.c = make_coef<S>(p);
  return a;
}

template <typename S>
hipError_t step(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force, hipStream_t s) {
  return dispatch_radii<S, MODE_STEP>(args<S>(p, g, src, dst, force), p.stencil, s);
}

template <typename S>
hipError_t fields(const lbm_params& p, const Geom& g, const void* src, const void* force, void* rho, void* ux,
                  void* uy, void* rhoN, hipStream_t s) {
  using T = typename S::math;
  StepArgs<T> a = args<S>(p, g, src, nullptr, force);
  a.out_rho = static_cast<T*>(rho);
  a.out_ux = static_cast<T*>(ux);
  a.out_uy = static_cast<T*>(uy);
  a.out_rhoN = static_cast<T*>(rhoN);
  hipError_t e = dispatch_radii<S, MODE_FIELDS>(a, p.stencil, s);
  if (e != hipSuccess || !g.walls) return e;
  hipLaunchKernelGGL(fill_rows_kernel<T>, dim3((g.nx + 255) / 256), dim3(256), 0, s, a.out_rho, a.out_ux, a.out_uy,
                     a.out_rhoN, g.nx, 0, g.ny - 1);
  return hipGetLastError();
}

template <typename S>
hipError_t stream_only(const Geom& g, const void* src, void* dst, hipStream_t s) {
  dim3 grid((g.nx + 255) / 256, g.F);
  hipLaunchKernelGGL(stream_only_kernel<S>, grid, dim3(256), 0, s, src, dst, geom_for<S>(g));
  return hipGetLastError();
}

template <typename S>
hipError_t init(const lbm_params& p, const Geom& g, const void* rhoN0, void* dst, hipStream_t s) {
  using T = typename S::math;
  dim3 grid((g.nx + 255) / 256, g.ny);
  hipLaunchKernelGGL(init_kernel<S>, grid, dim3(256), 0, s, static_cast<const T*>(rhoN0), dst, geom_for<S>(g),
                     make_coef<S>(p),
                     (T)p.rho0_R, (T)p.rho0_B);
  return hipGetLastError();
}

template <typename S>
hipError_t mass(const lbm_params& p, const Geom& g, const void* pops, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(mass_partial_kernel<S>, dim3(MASS_BLOCKS), dim3(256), 0, s, pops, geom_for<S>(g),
                     make_coef<S>(p), partial);
  hipLaunchKernelGGL(mass_final_kernel, dim3(1), dim3(256), 0, s, partial, MASS_BLOCKS, out);
  return hipGetLastError();
}

// passes 2-5 of the adjoint, with the lattice kind (periodic, walled, or with
// a mask of solid sites: M) fixed at compile time
template <typename T, bool W, bool M>
void adjoint_tail(const StepArgs<T>& a, const Geom& g, const adj::Radii& r, T sigma, const T* sv, const T* A, T* B,
                  T* C, T* D, double* part, double* dsigma, T* dforce, T* lam_out, const unsigned char* solid,
                  hipStream_t s) {
  const dim3 grid((g.nx + 255) / 256, g.ny);
  hipLaunchKernelGGL((adj::force_kernel<T, W, M>), grid, dim3(256), 0, s, g, a.c, sigma, r, sv, A, B, dforce, part,
                     solid);
  // pass 3, plus the sum of pass 2's dL/dsigma partials in one extra row of workgroups
  hipLaunchKernelGGL((adj::director_kernel<T, W, M>), dim3(grid.x, g.ny + 1), dim3(256), 0, s, g, a.c, r, sv, A,
                     (const T*)B, C, (const double*)part, adj::red_blocks(g.nx, g.ny), dsigma, solid);
  hipLaunchKernelGGL((adj::colour_kernel<T, W, M>), grid, dim3(256), 0, s, g, a.c, r, sv, A, (const T*)B,
                     (const T*)C, D, solid);
  hipLaunchKernelGGL((adj::push_kernel<T, W, M>), grid, dim3(256), 0, s, g, A, (const T*)B, (const T*)D, lam_out,
                     solid);
}

// pass 1 with a mask: the step kernel's mask variant in MODE_ADJ, built for the
// stencil profiles (3,3,3,3), (3,1,3,1) and (1,1,1,1)
template <typename S>
hipError_t march_adj_masked(const StepArgs<typename S::math>& a, const int* r, hipStream_t s) {
  constexpr int NTX = Shape<S, MODE_ADJ>::ntx, NR = Shape<S, MODE_ADJ>::nr;
  const int ntiles = a.g.nstrips * a.g.nchunks;
  const int nblocks = 8 * ((ntiles + 7) / 8);
  if (r[0] == 3 && r[1] == 3 && r[2] == 3 && r[3] == 3) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, 3, 3, 3, 3, false, MODE_ADJ, true>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
  } else if (r[0] == 3 && r[1] == 1 && r[2] == 3 && r[3] == 1) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, 3, 1, 3, 1, false, MODE_ADJ, true>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
} else if (r[0] == 1 && r[1] == 1 && r[2] == 1 && r[3] == 1) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, 1, 1, 1, 1, false, MODE_ADJ, true>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
  } else {
    return hipErrorNotSupported;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint: save pass of the step kernel, then the five passes of
// chromo_adjoint.hpp.  ws holds adj::WS_PLANES planes of the arithmetic type,
// interleaved by rows ([y][WS_PLANES][x]), followed, at the next multiple of 256 bytes, by adj::red_blocks() + adj::RED2
// doubles.
// ---------------------------------------------------------------------------
template <typename S>
hipError_t adjoint(const lbm_params& p, const Geom& g0, const void* pops, const void* force, const void* lam_next,
                   void* lam_out, void* ws, double* dsigma, void* dforce, const unsigned char* solid,
                   const unsigned char* bnc, hipStream_t s) {
  using T = typename S::math;
  StepArgs<T> a = args<S>(p, g0, pops, nullptr, force);
  const Geom& g = a.g;
  // groups of planes within a row of the row-interleaved workspace
  T* sv = static_cast<T*>(ws) + (size_t)adj::G_SV * g.nx;
  T* A = static_cast<T*>(ws) + (size_t)adj::G_A * g.nx;
  T* B = static_cast<T*>(ws) + (size_t)adj::G_B * g.nx;
  T* C = static_cast<T*>(ws) + (size_t)adj::G_C * g.nx;
  T* D = static_cast<T*>(ws) + (size_t)adj::G_D * g.nx;
  const size_t plane_bytes = ((size_t)adj::WS_PLANES * g.plane * sizeof(T) + 255) / 256 * 256;
  double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + plane_bytes);
  a.out_save = sv;
  a.out_adj = A;
  a.lam_next = static_cast<const T*>(lam_next);
  a.bnc = bnc;
  hipError_t e = solid ? march_adj_masked<S>(a, p.stencil, s) : dispatch_radii<S, MODE_ADJ>(a, p.stencil, s);
  if (e != hipSuccess) return e;
  const adj::Radii r = {p.stencil[0], p.stencil[1], p.stencil[2], p.stencil[3]};
  T* dfo = static_cast<T*>(dforce);
  T* lo = static_cast<T*>(lam_out);
  if (solid) {
    adjoint_tail<T, false, true>(a, g, r, (T)p.sigma, sv, A, B, C, D, part, dsigma, dfo, lo, solid, s);
  } else if (g.walls) {
    adjoint_tail<T, true, false>(a, g, r, (T)p.sigma, sv, A, B, C, D, part, dsigma, dfo, lo, nullptr, s);
  } else {
    adjoint_tail<T, false, false>(a, g, r, (T)p.sigma, sv, A, B, C, D, part, dsigma, dfo, lo, nullptr, s);
  }
  return hipGetLastError();
}

template <typename S>
hipError_t rhoN_adjoint(const lbm_params& p, const Geom& g0, const void* pops, const void* lrN, void* out,
                        const unsigned char* solid, const unsigned char* bnc, hipStream_t s) {
  using T = typename S::math;
  const Geom g = geom_for<S>(g0);
  const dim3 grid((g.nx + 255) / 256, g.ny);
  if (solid) {
    hipLaunchKernelGGL((adj::rhoN_adjoint_kernel<S, true>), grid, dim3(256), 0, s, pops, g, make_coef<S>(p),
                       static_cast<const T*>(lrN), static_cast<T*>(out), solid, bnc);
  } else {
    hipLaunchKernelGGL((adj::rhoN_adjoint_kernel<S, false>), grid, dim3(256), 0, s, pops, g, make_coef<S>(p),
                       static_cast<const T*>(lrN), static_cast<T*>(out), nullptr, nullptr);
  }
  return hipGetLastError();
}

template <typename S>
hipError_t init_adjoint(const lbm_params& p, const Geom& g0, const void* rhoN0, const void* lam0, void* out,
                        const unsigned char* solid, hipStream_t s) {
  using T = typename S::math;
  const Geom g = geom_for<S>(g0);
  const dim3 grid((g.nx + 255) / 256, g.ny);
  if (solid) {
    hipLaunchKernelGGL((adj::init_adjoint_kernel<T, true>), grid, dim3(256), 0, s, static_cast<const T*>(rhoN0),
                       static_cast<const T*>(lam0), g, make_coef<S>(p), (T)p.rho0_R, (T)p.rho0_B,
                       static_cast<T*>(out), solid);
  } else {
    hipLaunchKernelGGL((adj::init_adjoint_kernel<T, false>), grid, dim3(256), 0, s, static_cast<const T*>(rhoN0),
                       static_cast<const T*>(lam0), g, make_coef<S>(p), (T)p.rho0_R, (T)p.rho0_B,
                       static_cast<T*>(out), nullptr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// batched periodic step (chromo_batch_kernel)
// ---------------------------------------------------------------------------
template <typename S, int NTX, int RG, int RK, int RP, int RU, bool WALLS = false, bool MASK = false>
hipError_t batch_launch(const BatchArgs<typename S::math>& b, int nbins, hipStream_t s) {
  hipLaunchKernelGGL((chromo_batch_kernel<S, NTX, Shape<S>::nr, RG, RK, RP, RU, WALLS, MASK>), dim3(nbins),
                     dim3(NTX * Shape<S>::nr), 0, s, b);
  return hipGetLastError();
}

// batches of walled lattices, or with solid-site masks on some lattices
// (MASK): built for the stencil profiles (3,3,3,3), (3,1,3,1) and (1,1,1,1)
template <typename S, int NTX, bool WALLS, bool MASK>
hipError_t batch_special(const BatchArgs<typename S::math>& b, const int* r, int nbins, hipStream_t s) {
  if (r[0] == 3 && r[1] == 3 && r[2] == 3 && r[3] == 3)
    return batch_launch<S, NTX, 3, 3, 3, 3, WALLS, MASK>(b, nbins, s);
  if (r[0] == 3 && r[1] == 1 && r[2] == 3 && r[3] == 1)
    return batch_launch<S, NTX, 3, 1, 3, 1, WALLS, MASK>(b, nbins, s);
  if (r[0] == 1 && r[1] == 1 && r[2] == 1 && r[3] == 1)
    return batch_launch<S, NTX, 1, 1, 1, 1, WALLS, MASK>(b, nbins, s);
  return hipErrorNotSupported;
}

template <typename S, int NTX>
hipError_t batch_radii(const BatchArgs<typename S::math>& b, const int* r, int nbins, hipStream_t s) {
  const int code = (r[0] == 3) * 8 + (r[1] == 3) * 4 + (r[2] == 3) * 2 + (r[3] == 3);
#define CHROMO_CASE(C, A, B, P, U) \
  case C:                          \
    return batch_launch<S, NTX, A, B, P, U>(b, nbins, s);
  switch (code) {
    CHROMO_CASE(0, 1, 1, 1, 1)
    CHROMO_CASE(1, 1, 1, 1, 3)
    CHROMO_CASE(2, 1, 1, 3, 1)
    CHROMO_CASE(3, 1, 1, 3, 3)
    CHROMO_CASE(4, 1, 3, 1, 1)
    CHROMO_CASE(5, 1, 3, 1, 3)
    CHROMO_CASE(6, 1, 3, 3, 1)
    CHROMO_CASE(7, 1, 3, 3, 3)
    CHROMO_CASE(8, 3, 1, 1, 1)
    CHROMO_CASE(9, 3, 1, 1, 3)
    CHROMO_CASE(10, 3, 1, 3, 1)
    CHROMO_CASE(11, 3, 1, 3, 3)
    CHROMO_CASE(12, 3, 3, 1, 1)
    CHROMO_CASE(13, 3, 3, 1, 3)
    CHROMO_CASE(14, 3, 3, 3, 1)
    CHROMO_CASE(15, 3, 3, 3, 3)
  }
#undef CHROMO_CASE
  return hipErrorInvalidValue;
}

template <typename S, int NTX>
hipError_t batch_kind(const BatchArgs<typename S::math>& b, const int* r, int walls, int masked, int nbins,
                      hipStream_t s) {
  if (walls) return batch_special<S, NTX, true, false>(b, r, nbins, s);
  if (masked) return batch_special<S, NTX, false, true>(b, r, nbins, s);
  return batch_radii<S, NTX>(b, r, nbins, s);
}

template <typename S>
hipError_t batch(int ntx, const int* radii, int walls, int masked, const void* src, void* dst, const void* sims,
                 const int* bin_start, const int* items, int nbins, hipStream_t s) {
  using T = typename S::math;
  BatchArgs<T> b;
  b.src = static_cast<const char*>(src);
  b.dst = static_cast<char*>(dst);
  b.sims = static_cast<const SimDesc<T>*>(sims);
  b.bin_start = bin_start;
  b.items = items;
  if constexpr (Shape<S>::f64) {
    if (ntx == NTX_F64) return batch_kind<S, NTX_F64>(b, radii, walls, masked, nbins, s);
  } else {
    if (ntx == 128) return batch_kind<S, 128>(b, radii, walls, masked, nbins, s);
    if (ntx == 192) return batch_kind<S, 192>(b, radii, walls, masked, nbins, s);
  }
  return hipErrorInvalidValue;
}

template <typename S>
void sim_desc(const lbm_params& p, const Geom& g, unsigned long long off, const void* force,
              const unsigned char* bnc, void* out) {
  SimDesc<typename S::math> d;
  d.g = geom_for<S>(g);
  d.c = make_coef<S>(p);
  d.off = off;
  d.force = static_cast<const typename S::math*>(force);
  d.bnc = bnc;
  memcpy(out, &d, sizeof(d));
}

// ---------------------------------------------------------------------------
// solid sites anywhere (chromo_solid.hpp): four passes per step over the
// field planes of ws
// ---------------------------------------------------------------------------
template <typename S>
hipError_t solid_prepare(const lbm_params& p, const Geom& g0, void* pops, const unsigned char* mask, void* ws,
                         hipStream_t s) {
  const Geom g = geom_for<S>(g0);
  const dim3 grid((g.nx + 255) / 256, g.ny);
  hipLaunchKernelGGL(solid::rebounce_kernel<S>, grid, dim3(256), 0, s, pops, mask, g);
  hipLaunchKernelGGL(solid::clear_solid_kernel<S>, grid, dim3(256), 0, s, pops, mask, g, make_coef<S>(p));
  unsigned char* bits = static_cast<unsigned char*>(ws) + solid::bits_offset(g.plane, sizeof(typename S::math));
  hipLaunchKernelGGL(solid::bounce_bits_kernel<S>, grid, dim3(256), 0, s, mask, g, bits);
  return hipGetLastError();
}

// The fused step kernel with a mask, for the stencil profiles (3,3,3,3),
// (3,1,3,1) and (1,1,1,1); hipErrorNotSupported for the others (the caller
// then runs the four passes).
template <typename S>
hipError_t solid_fused(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force, void* ws,
                       hipStream_t s) {
  constexpr int NTX = Shape<S>::ntx, NR = Shape<S>::nr;
  StepArgs<typename S::math> a = args<S>(p, g, src, dst, force);
  a.bnc = static_cast<const unsigned char*>(ws) + solid::bits_offset(g.plane, sizeof(typename S::math));
  const int ntiles = a.g.nstrips * a.g.nchunks;
  const int nblocks = 8 * ((ntiles + 7) / 8);
  const int* r = p.stencil;
  if (r[0] == 3 && r[1] == 3 && r[2] == 3 && r[3] == 3) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, 3, 3, 3, 3, false, MODE_STEP, true>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
  } else if (r[0] == 3 && r[1] == 1 && r[2] == 3 && r[3] == 1) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, 3, 1, 3, 1, false, MODE_STEP, true>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
} else if (r[0] == 1 && r[1] == 1 && r[2] == 1 && r[3] == 1) {
    hipLaunchKernelGGL((chromo_step_kernel<S, NTX, NR, 1, 1, 1, 1, false, MODE_STEP, true>), dim3(nblocks),
                       dim3(NTX * NR), 0, s, a);
  } else {
    return hipErrorNotSupported;
  }
  return hipGetLastError();
}

// passes 1-3; FIELDS: pass 3 writes the caller's field arrays
template <typename S, bool FIELDS>
void solid_front(const StepArgs<typename S::math>& a, const int* r, const unsigned char* mask,
                 typename S::math* ws, hipStream_t s) {
  using T = typename S::math;
  const Geom& g = a.g;
  const dim3 grid((g.nx + 255) / 256, g.ny);
  hipLaunchKernelGGL(solid::sites_kernel<S>, grid, dim3(256), 0, s, a.src, mask, g, a.c, ws);
  if (r[0] == 3) {
    hipLaunchKernelGGL((solid::director_kernel<T, 3>), grid, dim3(256), 0, s, mask, g, a.c, ws);
  } else {
    hipLaunchKernelGGL((solid::director_kernel<T, 1>), grid, dim3(256), 0, s, mask, g, a.c, ws);
  }
  if (r[1] == 3) {
    hipLaunchKernelGGL((solid::force_kernel<T, 3, FIELDS>), grid, dim3(256), 0, s, mask, g, a.c, a.force, ws,
                       a.out_rho, a.out_ux, a.out_uy, a.out_rhoN);
  } else {
    hipLaunchKernelGGL((solid::force_kernel<T, 1, FIELDS>), grid, dim3(256), 0, s, mask, g, a.c, a.force, ws,
                       a.out_rho, a.out_ux, a.out_uy, a.out_rhoN);
  }
}

template <typename S>
hipError_t solid_step(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force,
                      const unsigned char* mask, void* wsv, hipStream_t s) {
  using T = typename S::math;
  const StepArgs<T> a = args<S>(p, g, src, dst, force);
  T* ws = static_cast<T*>(wsv);
  solid_front<S, false>(a, p.stencil, mask, ws, s);
  const dim3 grid((g.nx + 255) / 256, g.ny);
  const int code = (p.stencil[2] == 3) * 2 + (p.stencil[3] == 3);
  switch (code) {
    case 0:
      hipLaunchKernelGGL((solid::collide_kernel<S, 1, 1>), grid, dim3(256), 0, s, a, mask, (const T*)ws);
      break;
    case 1:
      hipLaunchKernelGGL((solid::collide_kernel<S, 1, 3>), grid, dim3(256), 0, s, a, mask, (const T*)ws);
      break;
    case 2:
      hipLaunchKernelGGL((solid::collide_kernel<S, 3, 1>), grid, dim3(256), 0, s, a, mask, (const T*)ws);
      break;
    default:
      hipLaunchKernelGGL((solid::collide_kernel<S, 3, 3>), grid, dim3(256), 0, s, a, mask, (const T*)ws);
  }
  return hipGetLastError();
}

template <typename S>
hipError_t solid_fields(const lbm_params& p, const Geom& g, const void* src, const void* force,
                        const unsigned char* mask, void* wsv, void* rho, void* ux, void* uy, void* rhoN,
                        hipStream_t s) {
  using T = typename S::math;
  StepArgs<T> a = args<S>(p, g, src, nullptr, force);
  a.out_rho = static_cast<T*>(rho);
  a.out_ux = static_cast<T*>(ux);
  a.out_uy = static_cast<T*>(uy);
  a.out_rhoN = static_cast<T*>(rhoN);
  solid_front<S, true>(a, p.stencil, mask, static_cast<T*>(wsv), s);
  return hipGetLastError();
}

template <typename S>
Ops make_ops() {
  Ops o;
  o.step = step<S>;
  o.fields = fields<S>;
  o.stream_only = stream_only<S>;
  o.init = init<S>;
  o.mass = mass<S>;
  if constexpr (is_ofs16<S>::value) {
    o.adjoint = nullptr;
    o.rhoN_adjoint = nullptr;
    o.init_adjoint = nullptr;
  } else {
    o.adjoint = adjoint<S>;
    o.rhoN_adjoint = rhoN_adjoint<S>;
    o.init_adjoint = init_adjoint<S>;
  }
  o.solid_prepare = solid_prepare<S>;
  o.solid_fused = solid_fused<S>;
  o.solid_step = solid_step<S>;
  o.solid_fields = solid_fields<S>;
  o.batch_ntx[0] = o.batch_ntx[1] = o.batch_ntx[2] = 0;
  o.batch = batch<S>;
  o.sim_desc = sim_desc<S>;
  o.sim_desc_bytes = (int)sizeof(SimDesc<typename S::math>);
  if constexpr (Shape<S>::f64) {
    o.batch_ntx[0] = NTX_F64;
    o.batch_ntx[1] = 0;
  } else {
    o.batch_ntx[0] = 128;
    o.batch_ntx[1] = 192;
    o.batch_ntx[2] = 0;
  }
  o.words = S::NW;
  o.word_bytes = (int)sizeof(typename S::W);
  o.math_bytes = (int)sizeof(typename S::math);
  return o;
}

}  // namespace launch
}  // namespace chromo
