// C ABI of the chromodynamic MRT lattice Boltzmann step (see include/chromo_lbm.h).
// Host side: parameter validation, launch planning, kernel dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "chromo_lbm.h"
#include "chromo_adjoint.hpp"
#include "chromo_host.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

bool radius_ok(int r) { return r == 1 || r == 3; }

int halo(const lbm_params& p) { return p.stencil[0] + p.stencil[1] + p.stencil[3]; }

using chromo::MASS_BLOCKS;

const chromo::Ops* ops_of(int storage) {
  switch (storage) {
    case LBM_STORAGE_F64:
      return &chromo::ops_f64();
    case LBM_STORAGE_F32:
      return &chromo::ops_f32();
    case LBM_STORAGE_F16_OFS:
      return &chromo::ops_f16o();
    case LBM_STORAGE_BF16_OFS:
      return &chromo::ops_bf16o();
  }
  return nullptr;
}

// words per site and bytes per word of each storage format
int words_of(int storage) { return (storage == LBM_STORAGE_F16_OFS || storage == LBM_STORAGE_BF16_OFS) ? 10 : 18; }
int word_bytes_of(int storage) { return storage == LBM_STORAGE_F64 ? 8 : 4; }

int validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1) return fail(LBM_EINVAL, "lattice %dx%d is empty", p->nx, p->ny);
  if (p->walls_y != 0 && p->walls_y != 1) return fail(LBM_EINVAL, "walls_y must be 0 or 1");
  if (p->walls_y && p->ny < 3) return fail(LBM_EINVAL, "walls need ny >= 3 (one fluid row)");
  if (p->storage < LBM_STORAGE_F64 || p->storage > LBM_STORAGE_BF16_OFS)
    return fail(LBM_EINVAL, "storage %d not provided by this build", p->storage);
  const double bytes = (double)words_of(p->storage) * word_bytes_of(p->storage) * (double)p->nx * (double)p->ny;
  if (bytes >= 4294967296.0)
    return fail(LBM_EINVAL, "lattice too large: one population buffer must stay below 4 GiB");
  for (int k = 0; k < 4; ++k)
    if (!radius_ok(p->stencil[k])) return fail(LBM_EINVAL, "stencil radius %d not in {1,3}", p->stencil[k]);
  if (!(p->rho0_R > 0.0) || !(p->rho0_B > 0.0)) return fail(LBM_EINVAL, "densities must be positive");
  if (!(p->alpha_R >= 0.0 && p->alpha_R < 1.0) || !(p->alpha_B >= 0.0 && p->alpha_B < 1.0))
    return fail(LBM_EINVAL, "alpha must lie in [0,1)");
  const double Lam = p->rho0_R / p->rho0_B;
  if (std::fabs((1.0 - p->alpha_B) - Lam * (1.0 - p->alpha_R)) > 1e-9 * (1.0 - p->alpha_B))
    return fail(LBM_EINVAL, "density ratio relation violated: (1-alpha_B)=%.12g but Lambda(1-alpha_R)=%.12g",
                1.0 - p->alpha_B, Lam * (1.0 - p->alpha_R));
  if (!(p->nu_R > 0.0) || !(p->nu_B > 0.0)) return fail(LBM_EINVAL, "viscosities must be positive");
  if (!(p->lambda6 > 0.0 && p->lambda6 < 2.0) || !(p->lambda7 > 0.0 && p->lambda7 < 2.0))
    return fail(LBM_EINVAL, "ghost rates must lie in (0,2)");
  if (!(p->eps_n > 0.0)) return fail(LBM_EINVAL, "eps_n must be positive");
  if (!std::isfinite(p->sigma) || !std::isfinite(p->beta) || !std::isfinite(p->gx) || !std::isfinite(p->gy) ||
      !std::isfinite(p->K_fixed))
    return fail(LBM_EINVAL, "non-finite parameter");
  if (p->ghost_eq != 0 && p->ghost_eq != 1) return fail(LBM_EINVAL, "ghost_eq must be 0 or 1");
  if (p->flags & ~(LBM_FLAG_STREAM_ONLY | LBM_FLAG_FIXED_K | LBM_FLAG_NO_RECOLOR))
    return fail(LBM_EINVAL, "unknown flag bits 0x%x", p->flags);
  return LBM_OK;
}

// Strips of at most NTX-2H columns; chunks of rows such that all tiles run in
// a single wave of workgroups (one workgroup fills a CU: its 8 wavefronts use
// the whole register file), i.e. nstrips * nchunks <= number of CUs, with
// chunks no shorter than 24 rows.
chromo::Geom plan(const lbm_params& p, int ncu, int ntx) {
  chromo::Geom g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.walls = p.walls_y;
  g.F = p.walls_y ? p.ny - 2 : p.ny;
  g.plane = p.nx * p.ny;
  const int txmax = ntx - 2 * halo(p);
  g.nstrips = (p.nx + txmax - 1) / txmax;
  g.TX = (p.nx + g.nstrips - 1) / g.nstrips;
  int nch = ncu / g.nstrips;
  if (nch < 1) nch = 1;
  int maxchunks = g.F / 24;
  if (maxchunks < 1) maxchunks = 1;
  if (nch > maxchunks) nch = maxchunks;
  g.TY = (g.F + nch - 1) / nch;
  g.nchunks = (g.F + g.TY - 1) / g.TY;
  return g;
}

}  // namespace

struct lbm_handle {
  lbm_params p;
  void* pops[2];
  int live;
  void* ws;
  size_t ws_bytes;
  const void* force;
  int64_t steps;
  chromo::Geom g;      // forward step kernel
  chromo::Geom g_adj;  // adjoint pass 1 (workgroup shape ntx_for(storage, true))
  const chromo::Ops* ops;
};

namespace {

int mass_into(lbm_handle* h, double* out, hipStream_t s) {
  HIP_TRY(h->ops->mass(h->p, h->g, h->pops[h->live], static_cast<double*>(h->ws), out, s));
  return LBM_OK;
}

int step_impl(lbm_handle* h, int nsteps, hipStream_t s) {
  for (int k = 0; k < nsteps; ++k) {
    const void* src = h->pops[h->live];
    void* dst = h->pops[1 - h->live];
    hipError_t e = (h->p.flags & LBM_FLAG_STREAM_ONLY) ? h->ops->stream_only(h->g, src, dst, s)
                                                       : h->ops->step(h->p, h->g, src, dst, h->force, s);
    if (e != hipSuccess) return fail(LBM_EHIP, "step launch: %s", hipGetErrorString(e));
    h->live = 1 - h->live;
    h->steps += 1;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_validate_params(const lbm_params* p) {
  g_last_error.clear();
  return validate(p);
}

size_t lbm_pops_elems(const lbm_params* p) {
  if (!p || p->nx < 1 || p->ny < 1 || p->storage < LBM_STORAGE_F64 || p->storage > LBM_STORAGE_BF16_OFS) return 0;
  return (size_t)words_of(p->storage) * (size_t)p->nx * (size_t)p->ny;
}

size_t lbm_pops_bytes(const lbm_params* p) { return lbm_pops_elems(p) * (p ? word_bytes_of(p->storage) : 0); }

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  return (size_t)(MASS_BLOCKS + 1) * 2 * sizeof(double);  // partials + the lbm_masses_host target
}

int lbm_init(const lbm_params* p, const void* rhoN0, const void* force, void* pops_a, void* pops_b,
             void* workspace, size_t ws_bytes, hipStream_t stream, lbm_handle** out) {
  g_last_error.clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int st = validate(p);
  if (st != LBM_OK) return st;
  if (!rhoN0 || !pops_a || !pops_b || !workspace)
    return fail(LBM_EINVAL, "rhoN0, pops_a, pops_b and workspace must be non-NULL");
  if (pops_a == pops_b) return fail(LBM_EINVAL, "pops_a and pops_b must differ");
  const size_t elem = (size_t)word_bytes_of(p->storage);
  const size_t bytes = lbm_pops_bytes(p);
  const char* a = static_cast<const char*>(pops_a);
  const char* b = static_cast<const char*>(pops_b);
  if (a < b + bytes && b < a + bytes) return fail(LBM_EINVAL, "pops_a and pops_b overlap");
  if (ws_bytes < lbm_workspace_bytes(p)) return fail(LBM_EINVAL, "workspace too small: %zu < %zu", ws_bytes,
                                                     lbm_workspace_bytes(p));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  if (reinterpret_cast<uintptr_t>(pops_a) % elem || reinterpret_cast<uintptr_t>(pops_b) % elem)
    return fail(LBM_EINVAL, "population buffers misaligned");

  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));

  lbm_handle* h = new (std::nothrow) lbm_handle;
  if (!h) return fail(LBM_EINVAL, "out of host memory");
  h->p = *p;
  h->pops[0] = pops_a;
  h->pops[1] = pops_b;
  h->live = 0;
  h->ws = workspace;
  h->ws_bytes = ws_bytes;
  h->force = force;
  h->steps = 0;
  h->g = plan(*p, ncu > 0 ? ncu : 1, chromo::ntx_for(p->storage));
  h->g_adj = plan(*p, ncu > 0 ? ncu : 1, chromo::ntx_for(p->storage, true));
  h->ops = ops_of(p->storage);

  hipError_t e = h->ops->init(*p, h->g, rhoN0, pops_a, stream);
  if (e != hipSuccess) {
    delete h;
    return fail(LBM_EHIP, "init launch: %s", hipGetErrorString(e));
  }
  *out = h;
  return LBM_OK;
}

int lbm_step(lbm_handle* h, int32_t nsteps, double* mass_RB_dev, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  int st = step_impl(h, nsteps, stream);
  if (st != LBM_OK || !mass_RB_dev) return st;
  return mass_into(h, mass_RB_dev, stream);
}

int lbm_fields(lbm_handle* h, void* rho, void* ux, void* uy, void* rhoN, double* mass_RB_dev,
               hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = LBM_OK;
  if (rho || ux || uy || rhoN) {
    hipError_t e = h->ops->fields(h->p, h->g, h->pops[h->live], h->force, rho, ux, uy, rhoN, stream);
    if (e != hipSuccess) st = fail(LBM_EHIP, "fields launch: %s", hipGetErrorString(e));
  }
  if (st != LBM_OK || !mass_RB_dev) return st;
  return mass_into(h, mass_RB_dev, stream);
}

int lbm_masses_host(lbm_handle* h, double out[2], hipStream_t stream) {
  g_last_error.clear();
  if (!h || !out) return fail(LBM_EINVAL, "handle or out is NULL");
  double* tgt = static_cast<double*>(h->ws) + 2 * MASS_BLOCKS;  // pair after the block partials
  int st = mass_into(h, tgt, stream);
  if (st != LBM_OK) return st;
  HIP_TRY(hipMemcpyAsync(out, tgt, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
    return fail(LBM_ENONFINITE, "per-colour mass not finite: %g %g", out[0], out[1]);
  return LBM_OK;
}

size_t lbm_adjoint_workspace_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  if (p->walls_y || !ops_of(p->storage)->adjoint) return 0;
  const size_t elem = p->storage == LBM_STORAGE_F64 ? 8 : 4;
  size_t bytes = (size_t)chromo::adj::WS_PLANES * (size_t)p->nx * (size_t)p->ny * elem;
  bytes = (bytes + 255) / 256 * 256;
  return bytes + (size_t)chromo::adj::red_blocks(p->nx, p->ny) * sizeof(double);
}

static int adjoint_supported(const lbm_handle* h) {
  if (!h->ops->adjoint) return fail(LBM_ENOTIMPL, "the adjoint is provided for F64 and F32 storage only");
  if (h->p.walls_y) return fail(LBM_ENOTIMPL, "the adjoint is provided for periodic lattices only");
  if (h->p.flags & LBM_FLAG_STREAM_ONLY) return fail(LBM_ENOTIMPL, "no adjoint of the streaming-only test mode");
  return LBM_OK;
}

int lbm_adjoint_step(lbm_handle* h, const void* pops_t, const void* adj_next, void* adj_out, void* workspace,
                     size_t ws_bytes, double* dL_dsigma_dev, void* dL_dforce_dev, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = adjoint_supported(h);
  if (st != LBM_OK) return st;
  if (!pops_t || !adj_next || !adj_out || !workspace)
    return fail(LBM_EINVAL, "pops_t, adj_next, adj_out and workspace must be non-NULL");
  if (adj_next == adj_out) return fail(LBM_EINVAL, "adj_next and adj_out must differ");
  if (ws_bytes < lbm_adjoint_workspace_bytes(&h->p))
    return fail(LBM_EINVAL, "adjoint workspace too small: %zu < %zu", ws_bytes, lbm_adjoint_workspace_bytes(&h->p));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  hipError_t e = h->ops->adjoint(h->p, h->g_adj, pops_t, h->force, adj_next, adj_out, workspace, dL_dsigma_dev,
                                 dL_dforce_dev, stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "adjoint launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_rhoN_adjoint(lbm_handle* h, const void* pops, const void* dL_drhoN, void* adj_out, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = adjoint_supported(h);
  if (st != LBM_OK) return st;
  if (!pops || !dL_drhoN || !adj_out) return fail(LBM_EINVAL, "pops, dL_drhoN and adj_out must be non-NULL");
  hipError_t e = h->ops->rhoN_adjoint(h->p, h->g, pops, dL_drhoN, adj_out, stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "rhoN adjoint launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_init_adjoint(lbm_handle* h, const void* rhoN0, const void* adj_pops0, void* dL_drhoN0, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = adjoint_supported(h);
  if (st != LBM_OK) return st;
  if (!rhoN0 || !adj_pops0 || !dL_drhoN0) return fail(LBM_EINVAL, "rhoN0, adj_pops0 and dL_drhoN0 must be non-NULL");
  hipError_t e = h->ops->init_adjoint(h->p, h->g, rhoN0, adj_pops0, dL_drhoN0, stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "init adjoint launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_current_pops(const lbm_handle* h) { return h ? h->live : -1; }

int64_t lbm_step_count(const lbm_handle* h) { return h ? h->steps : -1; }

void lbm_destroy(lbm_handle* h) { delete h; }

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
