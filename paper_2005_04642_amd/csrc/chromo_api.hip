// C ABI of the chromodynamic MRT lattice Boltzmann step (see include/chromo_lbm.h).
// Host side: parameter validation, launch planning, kernel dispatch.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <vector>

#include "chromo_lbm.h"
#include "chromo_adjoint.hpp"
#include "chromo_host.hpp"
#include "chromo_solid.hpp"

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

constexpr long long MAX_SITES = 1LL << 30;  // nx ny: 32-bit indices of two field planes
constexpr int MAX_ROWS = 65535;             // grid dimension y of the per-row kernels
// CU masks of streams: the runtime numbers the CUs round-robin over the 8
// XCDs (bits 0-31 select 4 CUs on each), so ranges in multiples of 8 give
// every XCD the same share
constexpr int PARTITION_GRAIN = 8;
// whole population buffers addressed through one buffer resource (the mask
// variant of the gather and the four-pass masked step) stay below 2^32 bytes
constexpr double WHOLE_BUFFER_LIMIT = 4294967296.0;

int halo(const lbm_params& p) { return p.stencil[0] + p.stencil[1] + p.stencil[3]; }

// Stencil profiles with instantiations of the step kernel's mask variant, the
// walled batch kernel and the masked adjoint: (3,3,3,3), the "fast" (3,1,3,1)
// and the "compact" (1,1,1,1).
bool special_profile(const int* r) {
  return (r[0] == 3 && r[1] == 3 && r[2] == 3 && r[3] == 3) || (r[0] == 3 && r[1] == 1 && r[2] == 3 && r[3] == 1) ||
         (r[0] == 1 && r[1] == 1 && r[2] == 1 && r[3] == 1);
}

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
    return fail(LBM_EINVAL, "storage %d not provided by this library", p->storage);
  // the step kernels address each lattice row through a buffer resource of its
  // own (byte offsets below 2^32 within a row); field planes are indexed with
  // 32-bit integers (two planes for a force field); rows index grid dimension y
  const double row_bytes = (double)words_of(p->storage) * word_bytes_of(p->storage) * (double)p->nx;
  if (row_bytes >= 4294967296.0)
    return fail(LBM_EINVAL, "lattice too wide: one row of a population buffer must stay below 4 GiB");
  if ((double)p->nx * (double)p->ny > (double)MAX_SITES)
    return fail(LBM_EINVAL, "lattice too large: at most %lld sites", (long long)MAX_SITES);
  if (p->ny > MAX_ROWS) return fail(LBM_EINVAL, "lattice too tall: at most %d rows", MAX_ROWS);
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
  if (p->flags & ~(LBM_FLAG_STREAM_ONLY | LBM_FLAG_FIXED_K | LBM_FLAG_NO_RECOLOR | LBM_FLAG_MASK_PASSES))
    return fail(LBM_EINVAL, "unknown flag bits 0x%x", p->flags);
  return LBM_OK;
}

// Strips of at most NTX-2H columns; chunks of rows such that all tiles run in
// a single wave of workgroups (one workgroup fills a CU: its LDS rings take
// nearly all of the CU's LDS), i.e. nstrips * nchunks <= number of CUs, with
// chunks no shorter than one march iteration (4 rows).  A chunk's march
// starts with a fixed pipeline fill, so on small lattices the time per step is
// the fill plus a few iterations whatever the chunk height: there, more and
// shorter chunks (down to 4 rows) run faster (512^2 FP32: 40 -> 24 us per step
// against a 24-row minimum), while large lattices are bound by the CU count.
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
  int maxchunks = g.F / 4;
  if (maxchunks < 1) maxchunks = 1;
  if (nch > maxchunks) nch = maxchunks;
  g.TY = (g.F + nch - 1) / nch;
  g.nchunks = (g.F + g.TY - 1) / g.TY;
  return g;
}

// ---------------------------------------------------------------------------
// Device scratch of lbm_step_static: the FP64 per-block partial sums of the
// mass reduction (MASS_BLOCKS pairs, 8 KiB), one copy on every GPU the library
// runs on, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is only a stand-in for the symbol): it
// uses the device address hipGetSymbolAddress returns for each device.
// ---------------------------------------------------------------------------
constexpr int SCRATCH_PAIRS = MASS_BLOCKS;
static __device__ __align__(256) double scratch[2 * SCRATCH_PAIRS];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // indexed by device ordinal

// Address of the current device's scratch, looked up once per device (the
// device must be current).  LBM_OK or LBM_EHIP.
int scratch_of_device(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (dev < 0) return fail(LBM_EHIP, "invalid device %d", dev);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
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
  double* scratch = nullptr;             // this device's static scratch (lbm_step_static)
  const unsigned char* solid = nullptr;  // device mask of solid sites (lbm_set_solid), or null
  void* solid_ws = nullptr;              // its field planes
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
    hipError_t e;
    if (h->solid) {
      e = hipErrorNotSupported;
      if (!(h->p.flags & LBM_FLAG_MASK_PASSES))
        e = h->ops->solid_fused(h->p, h->g, src, dst, h->force, h->solid_ws, s);
      if (e == hipErrorNotSupported)
        e = h->ops->solid_step(h->p, h->g, src, dst, h->force, h->solid, h->solid_ws, s);
    } else {
      e = (h->p.flags & LBM_FLAG_STREAM_ONLY) ? h->ops->stream_only(h->g, src, dst, s)
                                              : h->ops->step(h->p, h->g, src, dst, h->force, s);
    }
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
  double* scr = nullptr;
  st = scratch_of_device(dev, &scr);
  if (st != LBM_OK) return st;

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
  h->scratch = scr;

  hipError_t e = h->ops->init(*p, h->g, rhoN0, pops_a, stream);
  if (e != hipSuccess) {
    delete h;
    return fail(LBM_EHIP, "init launch: %s", hipGetErrorString(e));
  }
  *out = h;
  return LBM_OK;
}

int lbm_set_cu_budget(lbm_handle* h, int32_t ncu_step, int32_t ncu_adjoint) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (ncu_step < 0 || ncu_adjoint < 0) return fail(LBM_EINVAL, "CU budgets must be >= 0");
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (ncu < 1) ncu = 1;
  const int bs = ncu_step > 0 ? std::min(ncu_step, ncu) : ncu;
  const int ba = ncu_adjoint > 0 ? std::min(ncu_adjoint, ncu) : ncu;
  h->g = plan(h->p, bs, chromo::ntx_for(h->p.storage));
  h->g_adj = plan(h->p, ba, chromo::ntx_for(h->p.storage, true));
  return LBM_OK;
}

int lbm_partition_stream(int32_t cu_first, int32_t cu_count, hipStream_t* out) {
  g_last_error.clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (cu_first < 0 || cu_count < 1 || cu_first % PARTITION_GRAIN || cu_count % PARTITION_GRAIN)
    return fail(LBM_EINVAL, "CU range [%d, %d + %d) must start and extend in multiples of %d", cu_first, cu_first,
                cu_count, PARTITION_GRAIN);
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (cu_first + cu_count > ncu)
    return fail(LBM_EINVAL, "CU range [%d, %d) beyond the device's %d CUs", cu_first, cu_first + cu_count, ncu);
  std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
  for (int b = cu_first; b < cu_first + cu_count; ++b) mask[b / 32] |= 1u << (b % 32);
  hipStream_t s = nullptr;
  HIP_TRY(hipExtStreamCreateWithCUMask(&s, (uint32_t)mask.size(), mask.data()));
  *out = s;
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

int lbm_step_static(lbm_handle* h, int32_t nsteps, double* mass_RB_dev, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (!h->scratch) return fail(LBM_EHIP, "no device scratch for this handle");
  static_assert(MASS_BLOCKS <= SCRATCH_PAIRS, "the mass reduction's partials must fit the scratch");
  int st = step_impl(h, nsteps, stream);
  if (st != LBM_OK || !mass_RB_dev) return st;
  HIP_TRY(h->ops->mass(h->p, h->g, h->pops[h->live], h->scratch, mass_RB_dev, stream));
  return LBM_OK;
}

int lbm_step_into(lbm_handle* h, const void* from, int32_t nsteps, void* const* states, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (nsteps == 0) return LBM_OK;
  if (!from || !states) return fail(LBM_EINVAL, "from and states must be non-NULL");
  for (int j = 0; j < nsteps; ++j) {
    const void* prev = j ? states[j - 1] : from;
    if (!states[j] || states[j] == prev) return fail(LBM_EINVAL, "states[%d] is NULL or equal to its source", j);
  }
  for (int j = 0; j < nsteps; ++j) {
    h->pops[h->live] = const_cast<void*>(j ? states[j - 1] : from);
    h->pops[1 - h->live] = states[j];
    const int st = step_impl(h, 1, stream);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

int lbm_fields(lbm_handle* h, void* rho, void* ux, void* uy, void* rhoN, double* mass_RB_dev,
               hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = LBM_OK;
  if (rho || ux || uy || rhoN) {
    hipError_t e = h->solid ? h->ops->solid_fields(h->p, h->g, h->pops[h->live], h->force, h->solid, h->solid_ws,
                                                   rho, ux, uy, rhoN, stream)
                            : h->ops->fields(h->p, h->g, h->pops[h->live], h->force, rho, ux, uy, rhoN, stream);
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
  if (!ops_of(p->storage)->adjoint) return 0;
  const size_t elem = p->storage == LBM_STORAGE_F64 ? 8 : 4;
  size_t bytes = (size_t)chromo::adj::WS_PLANES * (size_t)p->nx * (size_t)p->ny * elem;
  bytes = (bytes + 255) / 256 * 256;
  return bytes + (size_t)(chromo::adj::red_blocks(p->nx, p->ny) + chromo::adj::RED2) * sizeof(double);
}

static int adjoint_supported(const lbm_handle* h) {
  if (!h->ops->adjoint) return fail(LBM_ENOTIMPL, "the adjoint is provided for F64 and F32 storage only");
  if (h->p.flags & LBM_FLAG_STREAM_ONLY) return fail(LBM_ENOTIMPL, "no adjoint of the streaming-only test mode");
  if (h->solid && !special_profile(h->p.stencil))
    return fail(LBM_ENOTIMPL, "the adjoint with a solid-site mask is built for stencil profiles 3333, 3131 and 1111");
  return LBM_OK;
}

// bounce bits of the handle's mask (inside its solid workspace), or null
static const unsigned char* bounce_bits(const lbm_handle* h) {
  if (!h->solid) return nullptr;
  const size_t elem = h->p.storage == LBM_STORAGE_F64 ? 8 : 4;
  return static_cast<const unsigned char*>(h->solid_ws) + chromo::solid::bits_offset((size_t)h->g.plane, elem);
}

// argument checks shared by lbm_adjoint_step and lbm_adjoint_steps
static int adjoint_args(lbm_handle* h, const void* adj_a, const void* adj_b, const void* workspace,
                        size_t ws_bytes) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = adjoint_supported(h);
  if (st != LBM_OK) return st;
  if (!adj_a || !adj_b || !workspace) return fail(LBM_EINVAL, "adjoint buffers and workspace must be non-NULL");
  if (adj_a == adj_b) return fail(LBM_EINVAL, "the two adjoint buffers must differ");
  if (ws_bytes < lbm_adjoint_workspace_bytes(&h->p))
    return fail(LBM_EINVAL, "adjoint workspace too small: %zu < %zu", ws_bytes, lbm_adjoint_workspace_bytes(&h->p));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  return LBM_OK;
}

int lbm_adjoint_step(lbm_handle* h, const void* pops_t, const void* adj_next, void* adj_out, void* workspace,
                     size_t ws_bytes, double* dL_dsigma_dev, void* dL_dforce_dev, hipStream_t stream) {
  g_last_error.clear();
  int st = adjoint_args(h, adj_next, adj_out, workspace, ws_bytes);
  if (st != LBM_OK) return st;
  if (!pops_t) return fail(LBM_EINVAL, "pops_t must be non-NULL");
  hipError_t e = h->ops->adjoint(h->p, h->g_adj, pops_t, h->force, adj_next, adj_out, workspace, dL_dsigma_dev,
                                 dL_dforce_dev, h->solid, bounce_bits(h), stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "adjoint launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_adjoint_steps(lbm_handle* h, int32_t nsteps, const void* const* states, void* adj_a, void* adj_b,
                      void* workspace, size_t ws_bytes, double* dL_dsigma_dev, void* dL_dforce_dev,
                      hipStream_t stream) {
  g_last_error.clear();
  int st = adjoint_args(h, adj_a, adj_b, workspace, ws_bytes);
  if (st != LBM_OK) return st;
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (nsteps > 0 && !states) return fail(LBM_EINVAL, "states must be non-NULL");
  for (int j = 0; j < nsteps; ++j)
    if (!states[j]) return fail(LBM_EINVAL, "states[%d] is NULL", j);
  for (int k = 0; k < nsteps; ++k) {
    const void* in = (k & 1) ? adj_b : adj_a;
    void* out = (k & 1) ? adj_a : adj_b;
    hipError_t e = h->ops->adjoint(h->p, h->g_adj, states[nsteps - 1 - k], h->force, in, out, workspace,
                                   dL_dsigma_dev, dL_dforce_dev, h->solid, bounce_bits(h), stream);
    if (e != hipSuccess) return fail(LBM_EHIP, "adjoint launch: %s", hipGetErrorString(e));
  }
  return LBM_OK;
}

int lbm_rhoN_adjoint(lbm_handle* h, const void* pops, const void* dL_drhoN, void* adj_out, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = adjoint_supported(h);
  if (st != LBM_OK) return st;
  if (!pops || !dL_drhoN || !adj_out) return fail(LBM_EINVAL, "pops, dL_drhoN and adj_out must be non-NULL");
  hipError_t e = h->ops->rhoN_adjoint(h->p, h->g, pops, dL_drhoN, adj_out, h->solid, bounce_bits(h), stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "rhoN adjoint launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

int lbm_init_adjoint(lbm_handle* h, const void* rhoN0, const void* adj_pops0, void* dL_drhoN0, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int st = adjoint_supported(h);
  if (st != LBM_OK) return st;
  if (!rhoN0 || !adj_pops0 || !dL_drhoN0) return fail(LBM_EINVAL, "rhoN0, adj_pops0 and dL_drhoN0 must be non-NULL");
  hipError_t e = h->ops->init_adjoint(h->p, h->g, rhoN0, adj_pops0, dL_drhoN0, h->solid, stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "init adjoint launch: %s", hipGetErrorString(e));
  return LBM_OK;
}

size_t lbm_solid_workspace_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  if (!ops_of(p->storage)->solid_step || p->walls_y || (p->flags & LBM_FLAG_STREAM_ONLY)) return 0;
  if ((double)lbm_pops_bytes(p) >= WHOLE_BUFFER_LIMIT) return 0;
  const size_t elem = p->storage == LBM_STORAGE_F64 ? 8 : 4;
  const size_t plane = (size_t)p->nx * (size_t)p->ny;
  return (chromo::solid::bits_offset(plane, elem) + plane + 255) / 256 * 256;
}

int lbm_set_solid(lbm_handle* h, const uint8_t* solid_dev, void* workspace, size_t ws_bytes, hipStream_t stream) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!solid_dev || !workspace) return fail(LBM_EINVAL, "solid mask and workspace must be non-NULL");
  if (h->solid) return fail(LBM_EINVAL, "the handle already has a solid-site mask");
  if (h->p.walls_y) return fail(LBM_EINVAL, "with a solid-site mask walls_y must be 0 (put the wall rows in the mask)");
  if (h->p.flags & LBM_FLAG_STREAM_ONLY) return fail(LBM_ENOTIMPL, "no solid-site mask in the streaming-only test mode");
  if (h->p.nx < 4 || h->p.ny < 4) return fail(LBM_EINVAL, "a solid-site mask needs nx, ny >= 4");
  if ((double)lbm_pops_bytes(&h->p) >= WHOLE_BUFFER_LIMIT)
    return fail(LBM_EINVAL, "with a solid-site mask one population buffer must stay below 4 GiB");
  const size_t need = lbm_solid_workspace_bytes(&h->p);
  if (ws_bytes < need) return fail(LBM_EINVAL, "solid workspace too small: %zu < %zu", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  hipError_t e = h->ops->solid_prepare(h->p, h->g, h->pops[h->live], solid_dev, workspace, stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "solid mask launch: %s", hipGetErrorString(e));
  h->solid = solid_dev;
  h->solid_ws = workspace;
  return LBM_OK;
}

int lbm_current_pops(const lbm_handle* h) { return h ? h->live : -1; }

int lbm_set_pops(lbm_handle* h, void* live, void* next) {
  g_last_error.clear();
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!live || !next) return fail(LBM_EINVAL, "population buffer is NULL");
  if (live == next) return fail(LBM_EINVAL, "the two population buffers must differ");
  h->pops[h->live] = live;
  h->pops[1 - h->live] = next;
  return LBM_OK;
}

int64_t lbm_step_count(const lbm_handle* h) { return h ? h->steps : -1; }

void lbm_destroy(lbm_handle* h) { delete h; }

const char* lbm_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// ===========================================================================
// Batches of independent lattices (all periodic or all walled) stepped by one launch
// ===========================================================================
namespace {

constexpr int BATCH_MAX_BINS = 1024;
const int BATCH_TYCAPS[] = {32, 64, 128, 256, 1 << 30};

size_t round256(size_t n) { return (n + 255) / 256 * 256; }

// Byte offset of every lattice's population buffer inside the packed buffers.
size_t batch_offsets(const lbm_params* p, int nsim, std::vector<size_t>* off) {
  size_t total = 0;
  if (off) off->resize(nsim);
  for (int k = 0; k < nsim; ++k) {
    if (off) (*off)[k] = total;
    total += round256(lbm_pops_bytes(&p[k]));
  }
  return total;
}

int batch_validate(const lbm_params* p, int nsim) {
  if (!p || nsim < 1) return fail(LBM_EINVAL, "empty batch");
  for (int k = 0; k < nsim; ++k) {
    const int st = validate(&p[k]);
    if (st != LBM_OK) return fail(st, "lattice %d: %s", k, g_last_error.c_str());
    if (p[k].walls_y != p[0].walls_y)
      return fail(LBM_EINVAL, "lattice %d: walls differ from lattice 0 (a batch is all periodic or all walled)", k);
    if (p[k].flags & LBM_FLAG_STREAM_ONLY) return fail(LBM_EINVAL, "lattice %d: no stream-only mode in batches", k);
    if (p[k].storage != p[0].storage) return fail(LBM_EINVAL, "lattice %d: storage differs from lattice 0", k);
    for (int r = 0; r < 4; ++r)
      if (p[k].stencil[r] != p[0].stencil[r]) return fail(LBM_EINVAL, "lattice %d: stencil radii differ", k);
  }
  if (p[0].walls_y && !special_profile(p[0].stencil))
    return fail(LBM_ENOTIMPL, "batches of walled lattices are built for stencils 3333, 3131 and 1111");
  return LBM_OK;
}

// Tile plan of one lattice for workgroup width ntx and chunk height cap.
chromo::Geom batch_geom(const lbm_params& p, int ntx, int tycap) {
  chromo::Geom g;
  g.nx = p.nx;
  g.ny = p.ny;
  g.walls = p.walls_y;
  g.F = p.walls_y ? p.ny - 2 : p.ny;
  g.plane = p.nx * p.ny;
  const int txmax = ntx - 2 * halo(p);
  g.nstrips = (p.nx + txmax - 1) / txmax;
  g.TX = (p.nx + g.nstrips - 1) / g.nstrips;
  int nch = (g.F + tycap - 1) / tycap;
  if (nch < 1) nch = 1;
  g.TY = (g.F + nch - 1) / nch;
  g.nchunks = (g.F + g.TY - 1) / g.TY;
  return g;
}

size_t batch_tiles(const lbm_params* p, int nsim, int ntx, int tycap) {
  size_t n = 0;
  for (int k = 0; k < nsim; ++k) {
    const chromo::Geom g = batch_geom(p[k], ntx, tycap);
    n += (size_t)g.nstrips * g.nchunks;
  }
  return n;
}

size_t batch_items_cap(const lbm_params* p, int nsim) {
  size_t cap = 0;
  const chromo::Ops* ops = ops_of(p[0].storage);
  for (int i = 0; i < 3 && ops->batch_ntx[i]; ++i)
    for (int tc : BATCH_TYCAPS) cap = std::max(cap, batch_tiles(p, nsim, ops->batch_ntx[i], tc));
  return cap;
}

struct BatchPlan {
  int ntx = 0, tycap = 0, nbins = 0;
  std::vector<unsigned char> sims;
  std::vector<int> bin_start, items;
  double max_cost = 0.0;  // largest bin, in march iterations
};

// Longest-processing-time-first assignment of the tiles of every lattice to
// nbins bins (one workgroup each), costs counted in march iterations.
BatchPlan batch_plan(const lbm_params* p, int nsim, const std::vector<size_t>& off, int nbins, int ntx, int tycap,
                     const chromo::Ops& ops, int nr, int it0, const std::vector<const void*>& force,
                     const std::vector<const unsigned char*>& bnc) {
  BatchPlan b;
  b.ntx = ntx;
  b.tycap = tycap;
  b.nbins = nbins;
  b.sims.resize((size_t)nsim * ops.sim_desc_bytes);
  struct Tile {
    int sim, tile;
    int cost;
  };
  std::vector<Tile> tiles;
  for (int k = 0; k < nsim; ++k) {
    const chromo::Geom g = batch_geom(p[k], ntx, tycap);
    ops.sim_desc(p[k], g, (unsigned long long)off[k], force[k], bnc[k], &b.sims[(size_t)k * ops.sim_desc_bytes]);
    for (int t = 0; t < g.nstrips * g.nchunks; ++t) {
      const int chunk = t / g.nstrips;
      const int rows = std::min(g.TY, g.F - chunk * g.TY);
      tiles.push_back({k, t, it0 + (rows + nr - 1) / nr});
    }
  }
  std::stable_sort(tiles.begin(), tiles.end(), [](const Tile& a, const Tile& c) { return a.cost > c.cost; });
  typedef std::pair<long long, int> Load;  // (cost, bin)
  std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
  for (int i = 0; i < nbins; ++i) heap.push(Load(0, i));
  std::vector<std::vector<int>> bins(nbins);
  for (size_t i = 0; i < tiles.size(); ++i) {
    Load l = heap.top();
    heap.pop();
    bins[l.second].push_back((int)i);
    l.first += tiles[i].cost;
    b.max_cost = std::max(b.max_cost, (double)l.first);
    heap.push(l);
  }
  b.bin_start.assign(nbins + 1, 0);
  for (int i = 0; i < nbins; ++i) {
    b.bin_start[i + 1] = b.bin_start[i] + (int)bins[i].size();
    for (int j : bins[i]) {
      b.items.push_back(tiles[j].sim);
      b.items.push_back(tiles[j].tile);
    }
  }
  return b;
}

}  // namespace

struct lbm_batch {
  int nsim;
  std::vector<lbm_params> p;
  std::vector<size_t> off;
  std::vector<const void*> force;  // per-lattice force fields (lbm_batch_set_force), or null
  std::vector<const unsigned char*> bnc;  // per-lattice mask bounce bits (lbm_batch_set_solid), or null
  int masked;                      // some lattice has a mask: step with the mask variant
  char* pops[2];
  int live;
  int64_t steps;
  int ncu;
  const chromo::Ops* ops;
  void* d_sims;
  int* d_bin_start;
  int* d_items;
  double* d_mass;
  size_t items_cap;
  BatchPlan plan;
  std::vector<lbm_handle> view;  // one single-lattice handle per lattice (fields, masses)
};

namespace {

// Strip widths the batch kernels of this batch may use.  With FP32 arithmetic
// the 192-wide strips (768 threads, at most 168 VGPRs) spill registers in the
// walled and masked variants (hipcc: 5 VGPRs for walls at stencil 3333, 13 and
// 57 for masks at 3131 and 3333), so walled and masked batches use 128-wide
// strips only (no spills).  Returns the count written to out.
int batch_widths(const lbm_batch* b, int* out) {
  int n = 0;
  for (int i = 0; i < 3 && b->ops->batch_ntx[i]; ++i) {
    const int w = b->ops->batch_ntx[i];
    if (b->ops->math_bytes == 4 && w > 128 && (b->p[0].walls_y || b->masked)) continue;
    out[n++] = w;
  }
  return n;
}

int batch_upload(lbm_batch* b, BatchPlan&& pl, hipStream_t s) {
  if (pl.items.size() / 2 > b->items_cap || pl.nbins > BATCH_MAX_BINS)
    return fail(LBM_EINVAL, "batch plan exceeds the workspace tables");
  b->plan = std::move(pl);
  HIP_TRY(hipMemcpyAsync(b->d_sims, b->plan.sims.data(), b->plan.sims.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->d_bin_start, b->plan.bin_start.data(), b->plan.bin_start.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
  if (!b->plan.items.empty())
    HIP_TRY(hipMemcpyAsync(b->d_items, b->plan.items.data(), b->plan.items.size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
  // the host vectors must outlive the copies
  HIP_TRY(hipStreamSynchronize(s));
  return LBM_OK;
}

int batch_step_impl(lbm_batch* b, int nsteps, hipStream_t s) {
  for (int k = 0; k < nsteps; ++k) {
    hipError_t e = b->ops->batch(b->plan.ntx, b->p[0].stencil, b->p[0].walls_y, b->masked, b->pops[b->live],
                                 b->pops[1 - b->live], b->d_sims,
                                 b->d_bin_start, b->d_items, b->plan.nbins, s);
    if (e != hipSuccess) return fail(LBM_EHIP, "batch step launch: %s", hipGetErrorString(e));
    b->live = 1 - b->live;
    b->steps += 1;
  }
  return LBM_OK;
}

lbm_handle* batch_view(lbm_batch* b, int k) {
  lbm_handle* h = &b->view[k];
  h->live = b->live;
  h->steps = b->steps;
  return h;
}

}  // namespace

extern "C" {

size_t lbm_batch_pops_bytes(const lbm_params* p, int nsim) {
  if (batch_validate(p, nsim) != LBM_OK) return 0;
  return batch_offsets(p, nsim, nullptr);
}

int lbm_batch_offsets(const lbm_params* p, int nsim, size_t* offsets) {
  g_last_error.clear();
  int st = batch_validate(p, nsim);
  if (st != LBM_OK) return st;
  if (!offsets) return fail(LBM_EINVAL, "offsets is NULL");
  std::vector<size_t> off;
  batch_offsets(p, nsim, &off);
  for (int k = 0; k < nsim; ++k) offsets[k] = off[k];
  return LBM_OK;
}

size_t lbm_batch_workspace_bytes(const lbm_params* p, int nsim) {
  if (batch_validate(p, nsim) != LBM_OK) return 0;
  const chromo::Ops* ops = ops_of(p[0].storage);
  return round256((size_t)nsim * ops->sim_desc_bytes) + round256((BATCH_MAX_BINS + 1) * sizeof(int)) +
         round256(batch_items_cap(p, nsim) * 2 * sizeof(int)) + (size_t)(MASS_BLOCKS + 1) * 2 * sizeof(double);
}

int lbm_batch_init(const lbm_params* p, int nsim, const void* const* rhoN0, void* pops_a, void* pops_b,
                   void* workspace, size_t ws_bytes, hipStream_t stream, lbm_batch** out) {
  g_last_error.clear();
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int st = batch_validate(p, nsim);
  if (st != LBM_OK) return st;
  if (!rhoN0 || !pops_a || !pops_b || !workspace)
    return fail(LBM_EINVAL, "rhoN0, pops_a, pops_b and workspace must be non-NULL");
  for (int k = 0; k < nsim; ++k)
    if (!rhoN0[k]) return fail(LBM_EINVAL, "rhoN0[%d] is NULL", k);
  const size_t total = batch_offsets(p, nsim, nullptr);
  const char* a = static_cast<const char*>(pops_a);
  const char* bb = static_cast<const char*>(pops_b);
  if (a < bb + total && bb < a + total) return fail(LBM_EINVAL, "pops_a and pops_b overlap");
  if (reinterpret_cast<uintptr_t>(pops_a) % 256 || reinterpret_cast<uintptr_t>(pops_b) % 256)
    return fail(LBM_EINVAL, "packed population buffers must be 256-byte aligned");
  if (ws_bytes < lbm_batch_workspace_bytes(p, nsim))
    return fail(LBM_EINVAL, "workspace too small: %zu < %zu", ws_bytes, lbm_batch_workspace_bytes(p, nsim));
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  int dev = 0, ncu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  if (ncu < 1) ncu = 1;
  if (ncu > BATCH_MAX_BINS) ncu = BATCH_MAX_BINS;

  lbm_batch* b = new (std::nothrow) lbm_batch;
  if (!b) return fail(LBM_EINVAL, "out of host memory");
  b->nsim = nsim;
  b->p.assign(p, p + nsim);
  b->force.assign(nsim, nullptr);
  b->bnc.assign(nsim, nullptr);
  b->masked = 0;
  batch_offsets(p, nsim, &b->off);
  b->pops[0] = static_cast<char*>(pops_a);
  b->pops[1] = static_cast<char*>(pops_b);
  b->live = 0;
  b->steps = 0;
  b->ncu = ncu;
  b->ops = ops_of(p[0].storage);
  char* w = static_cast<char*>(workspace);
  b->d_sims = w;
  w += round256((size_t)nsim * b->ops->sim_desc_bytes);
  b->d_bin_start = reinterpret_cast<int*>(w);
  w += round256((BATCH_MAX_BINS + 1) * sizeof(int));
  b->items_cap = batch_items_cap(p, nsim);
  b->d_items = reinterpret_cast<int*>(w);
  w += round256(b->items_cap * 2 * sizeof(int));
  b->d_mass = reinterpret_cast<double*>(w);
  b->view.resize(nsim);
  for (int k = 0; k < nsim; ++k) {
    lbm_handle& h = b->view[k];
    h.p = p[k];
    h.pops[0] = b->pops[0] + b->off[k];
    h.pops[1] = b->pops[1] + b->off[k];
    h.live = 0;
    h.ws = b->d_mass;
    h.ws_bytes = (size_t)(MASS_BLOCKS + 1) * 2 * sizeof(double);
    h.force = nullptr;
    h.steps = 0;
    h.g = plan(p[k], ncu, chromo::ntx_for(p[k].storage));
    h.g_adj = plan(p[k], ncu, chromo::ntx_for(p[k].storage, true));
    h.ops = b->ops;
    hipError_t e = b->ops->init(p[k], h.g, rhoN0[k], h.pops[0], stream);
    if (e != hipSuccess) {
      delete b;
      return fail(LBM_EHIP, "init launch: %s", hipGetErrorString(e));
    }
  }
  const int nr = b->ops->math_bytes == 8 ? chromo::NR_F64 : chromo::NR_F32;
  const int it0 = 3 * ((nr * ((3 + nr - 1) / nr) + 3 + nr - 1) / nr);
  int widths[3];
  const int nw = batch_widths(b, widths);
  int ntx0 = widths[0];
  for (int i = 1; i < nw; ++i) ntx0 = std::max(ntx0, widths[i]);
  st = batch_upload(b, batch_plan(p, nsim, b->off, ncu, ntx0, 128, *b->ops, nr, it0, b->force, b->bnc), stream);
  if (st != LBM_OK) {
    delete b;
    return st;
  }
  *out = b;
  return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int32_t nsteps, hipStream_t stream) {
  g_last_error.clear();
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  return batch_step_impl(b, nsteps, stream);
}

int lbm_batch_autotune(lbm_batch* b, void* scratch, size_t scratch_bytes, int32_t steps_per_trial,
                       hipStream_t stream, int32_t* chosen) {
  g_last_error.clear();
  if (!b || !scratch) return fail(LBM_EINVAL, "batch and scratch must be non-NULL");
  const size_t total = b->off.back() + round256(lbm_pops_bytes(&b->p.back()));
  if (scratch_bytes < total) return fail(LBM_EINVAL, "scratch too small: %zu < %zu", scratch_bytes, total);
  if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial < 1");
  const int live0 = b->live;
  const int64_t steps0 = b->steps;
  HIP_TRY(hipMemcpyAsync(scratch, b->pops[live0], total, hipMemcpyDeviceToDevice, stream));
  const int nr = b->ops->math_bytes == 8 ? chromo::NR_F64 : chromo::NR_F32;
  const int it0 = 3 * ((nr * ((3 + nr - 1) / nr) + 3 + nr - 1) / nr);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  float best = -1.0f;
  int best_ntx = b->plan.ntx, best_tycap = b->plan.tycap;
  int st = LBM_OK;
  int widths[3];
  const int nw = batch_widths(b, widths);
  for (int i = 0; i < nw && st == LBM_OK; ++i) {
    for (int tc : BATCH_TYCAPS) {
      st = batch_upload(b, batch_plan(b->p.data(), b->nsim, b->off, b->ncu, widths[i], tc, *b->ops, nr,
                                      it0, b->force, b->bnc),
                        stream);
      if (st != LBM_OK) break;
      if (hipMemcpyAsync(b->pops[live0], scratch, total, hipMemcpyDeviceToDevice, stream) != hipSuccess) {
        st = fail(LBM_EHIP, "autotune: restoring the state failed");
        break;
      }
      b->live = live0;
      if ((st = batch_step_impl(b, 1, stream)) != LBM_OK) break;  // warm-up
      if (hipEventRecord(e0, stream) != hipSuccess) {
        st = fail(LBM_EHIP, "autotune: event record failed");
        break;
      }
      if ((st = batch_step_impl(b, steps_per_trial, stream)) != LBM_OK) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = fail(LBM_EHIP, "autotune: timing a candidate failed");
        break;
      }
      if (best < 0.0f || ms < best) {
        best = ms;
        best_ntx = widths[i];
        best_tycap = tc;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the state and install the winner
  HIP_TRY(hipMemcpyAsync(b->pops[live0], scratch, total, hipMemcpyDeviceToDevice, stream));
  b->live = live0;
  b->steps = steps0;
  if (st != LBM_OK) return st;
  st = batch_upload(b, batch_plan(b->p.data(), b->nsim, b->off, b->ncu, best_ntx, best_tycap, *b->ops, nr, it0,
                                  b->force, b->bnc),
                    stream);
  if (st != LBM_OK) return st;
  if (chosen) {
    chosen[0] = best_ntx;
    chosen[1] = best_tycap;
  }
  return LBM_OK;
}

int lbm_batch_set_force(lbm_batch* b, int32_t k, const void* force, hipStream_t stream) {
  g_last_error.clear();
  if (!b || k < 0 || k >= b->nsim) return fail(LBM_EINVAL, "bad batch or lattice index");
  b->force[k] = force;
  b->view[k].force = force;
  const chromo::Geom g = batch_geom(b->p[k], b->plan.ntx, b->plan.tycap);
  unsigned char* desc = &b->plan.sims[(size_t)k * b->ops->sim_desc_bytes];
  b->ops->sim_desc(b->p[k], g, (unsigned long long)b->off[k], force, b->bnc[k], desc);
  HIP_TRY(hipMemcpyAsync(static_cast<char*>(b->d_sims) + (size_t)k * b->ops->sim_desc_bytes, desc,
                         b->ops->sim_desc_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));  // the host copy may change with the next plan
  return LBM_OK;
}

int lbm_batch_set_solid(lbm_batch* b, int32_t k, const uint8_t* solid_dev, void* workspace, size_t ws_bytes,
                        hipStream_t stream) {
  g_last_error.clear();
  if (!b || k < 0 || k >= b->nsim) return fail(LBM_EINVAL, "bad batch or lattice index");
  if (!solid_dev || !workspace) return fail(LBM_EINVAL, "solid mask and workspace must be non-NULL");
  if (b->bnc[k]) return fail(LBM_EINVAL, "lattice %d already has a solid-site mask", k);
  const lbm_params& p = b->p[k];
  if (p.walls_y) return fail(LBM_EINVAL, "masks go in batches of periodic lattices (put wall rows in the mask)");
  if (!special_profile(p.stencil))
    return fail(LBM_ENOTIMPL, "masks in batches are built for stencil profiles 3333, 3131 and 1111");
  if (p.nx < 4 || p.ny < 4) return fail(LBM_EINVAL, "a solid-site mask needs nx, ny >= 4");
  if ((double)lbm_pops_bytes(&p) >= WHOLE_BUFFER_LIMIT)
    return fail(LBM_EINVAL, "with a solid-site mask one population buffer must stay below 4 GiB");
  const size_t need = lbm_solid_workspace_bytes(&p);
  if (ws_bytes < need) return fail(LBM_EINVAL, "solid workspace too small: %zu < %zu", ws_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
  lbm_handle* h = batch_view(b, k);
  hipError_t e = b->ops->solid_prepare(p, h->g, h->pops[h->live], solid_dev, workspace, stream);
  if (e != hipSuccess) return fail(LBM_EHIP, "solid mask launch: %s", hipGetErrorString(e));
  h->solid = solid_dev;
  h->solid_ws = workspace;
  b->bnc[k] = static_cast<const unsigned char*>(workspace) +
              chromo::solid::bits_offset((size_t)p.nx * (size_t)p.ny, (size_t)b->ops->math_bytes);
  b->masked = 1;
  int widths[3];
  const int nw = batch_widths(b, widths);
  bool allowed = false;
  for (int i = 0; i < nw; ++i) allowed = allowed || widths[i] == b->plan.ntx;
  if (!allowed) {  // the batch steps with the mask variant from now on: re-plan at a width it is built for
    const int nr = b->ops->math_bytes == 8 ? chromo::NR_F64 : chromo::NR_F32;
    const int it0 = 3 * ((nr * ((3 + nr - 1) / nr) + 3 + nr - 1) / nr);
    int st = batch_upload(b, batch_plan(b->p.data(), b->nsim, b->off, b->ncu, widths[0], b->plan.tycap, *b->ops, nr,
                                        it0, b->force, b->bnc),
                          stream);
    return st;
  }
  const chromo::Geom g = batch_geom(p, b->plan.ntx, b->plan.tycap);
  unsigned char* desc = &b->plan.sims[(size_t)k * b->ops->sim_desc_bytes];
  b->ops->sim_desc(p, g, (unsigned long long)b->off[k], b->force[k], b->bnc[k], desc);
  HIP_TRY(hipMemcpyAsync(static_cast<char*>(b->d_sims) + (size_t)k * b->ops->sim_desc_bytes, desc,
                         b->ops->sim_desc_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return LBM_OK;
}

int lbm_batch_plan_info(const lbm_batch* b, int32_t* info) {
  if (!b || !info) return fail(LBM_EINVAL, "batch and info must be non-NULL");
  info[0] = b->plan.ntx;
  info[1] = b->plan.tycap;
  info[2] = b->plan.nbins;
  info[3] = (int32_t)(b->plan.items.size() / 2);
  info[4] = (int32_t)b->plan.max_cost;
  return LBM_OK;
}

int lbm_batch_fields(lbm_batch* b, int32_t k, void* rho, void* ux, void* uy, void* rhoN, hipStream_t stream) {
  g_last_error.clear();
  if (!b || k < 0 || k >= b->nsim) return fail(LBM_EINVAL, "bad batch or lattice index");
  return lbm_fields(batch_view(b, k), rho, ux, uy, rhoN, nullptr, stream);
}

int lbm_batch_masses_host(lbm_batch* b, int32_t k, double out[2], hipStream_t stream) {
  g_last_error.clear();
  if (!b || k < 0 || k >= b->nsim) return fail(LBM_EINVAL, "bad batch or lattice index");
  return lbm_masses_host(batch_view(b, k), out, stream);
}

int lbm_batch_current_pops(const lbm_batch* b) { return b ? b->live : -1; }

int64_t lbm_batch_step_count(const lbm_batch* b) { return b ? b->steps : -1; }

void lbm_batch_destroy(lbm_batch* b) { delete b; }

}  // extern "C"
