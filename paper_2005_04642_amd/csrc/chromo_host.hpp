// Host-side pieces shared by the C ABI (chromo_api.hip) and the per-format
// kernel instantiations (chromo_<format>.hip): the launch plan and the table
// of launchers each format provides.
#pragma once

#include <hip/hip_runtime.h>

#include "chromo_lbm.h"
#include "chromo_kernels.hpp"

namespace chromo {

constexpr int MASS_BLOCKS = 512;

// Workgroup shape of the step kernel: NTX lattice columns x NR rows, one
// thread each, one workgroup per CU.  FP32 arithmetic: 768 threads (12
// waves, 3 per SIMD) within 168 VGPRs and the whole 160 KB of LDS; wider
// strips re-read fewer halo columns.
constexpr int NTX_F32 = 192;  // every format with FP32 arithmetic
constexpr int NR_F32 = 4;
constexpr int NTX_F64 = 64;   // double (validation format)
constexpr int NR_F64 = 4;
// The adjoint's first pass (the step kernel in MODE_ADJ) holds the forward
// and backward values of a site at once: 512 threads leave 256 VGPRs.
constexpr int NTX_ADJ_F32 = 128;

inline int ntx_for(int storage, bool adjoint = false) {
  return storage == LBM_STORAGE_F64 ? NTX_F64 : (adjoint ? NTX_ADJ_F32 : NTX_F32);
}

// Launchers of one storage format.  Pointers are device pointers in that
// format (populations) or in its arithmetic type (fields, rho^N, force).
struct Ops {
  hipError_t (*step)(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force,
                     hipStream_t s);
  hipError_t (*fields)(const lbm_params& p, const Geom& g, const void* src, const void* force, void* rho,
                       void* ux, void* uy, void* rhoN, hipStream_t s);
  hipError_t (*stream_only)(const Geom& g, const void* src, void* dst, hipStream_t s);
  hipError_t (*init)(const lbm_params& p, const Geom& g, const void* rhoN0, void* dst, hipStream_t s);
  hipError_t (*mass)(const lbm_params& p, const Geom& g, const void* pops, double* partial, double* out,
                     hipStream_t s);
  // adjoint (F64/F32, periodic or walled; null for formats without it)
  // g: geometry planned for the adjoint workgroup shape (ntx_for(storage, true))
  hipError_t (*adjoint)(const lbm_params& p, const Geom& g, const void* pops, const void* force,
                        const void* lam_next, void* lam_out, void* ws, double* dsigma, void* dforce,
                        const unsigned char* solid, const unsigned char* bnc, hipStream_t s);
  hipError_t (*rhoN_adjoint)(const lbm_params& p, const Geom& g, const void* pops, const void* lrN, void* out,
                             const unsigned char* solid, const unsigned char* bnc, hipStream_t s);
  hipError_t (*init_adjoint)(const lbm_params& p, const Geom& g, const void* rhoN0, const void* lam0, void* out,
                             const unsigned char* solid, hipStream_t s);
  // solid sites anywhere (every format).  mask: device [ny][nx] bytes, nonzero
  // = solid; ws: solid::P_N planes of the arithmetic type, then the bounce bits
  hipError_t (*solid_prepare)(const lbm_params& p, const Geom& g, void* pops, const unsigned char* mask, void* ws,
                              hipStream_t s);
  // the fused step kernel with the mask (hipErrorNotSupported for stencil
  // profiles it is not built for)
  hipError_t (*solid_fused)(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force,
                            void* ws, hipStream_t s);
  hipError_t (*solid_step)(const lbm_params& p, const Geom& g, const void* src, void* dst, const void* force,
                           const unsigned char* mask, void* ws, hipStream_t s);
  hipError_t (*solid_fields)(const lbm_params& p, const Geom& g, const void* src, const void* force,
                             const unsigned char* mask, void* ws, void* rho, void* ux, void* uy, void* rhoN,
                             hipStream_t s);
  // batched periodic step: ntx in batch_ntx (0-terminated); tables in device memory
  hipError_t (*batch)(int ntx, const int* radii, int walls, int masked, const void* src, void* dst,
                      const void* sims, const int* bin_start, const int* items, int nbins, hipStream_t s);
  // one SimDesc<math> of lattice p with tile plan g, byte offset off, force
  // field (device [2][ny][nx] or null) and mask bounce bits (or null), written to out
  void (*sim_desc)(const lbm_params& p, const Geom& g, unsigned long long off, const void* force,
                   const unsigned char* bnc, void* out);
  int sim_desc_bytes;
  int batch_ntx[3];
  int words;        // words per site
  int word_bytes;   // bytes per word
  int math_bytes;   // bytes of the arithmetic type (fields, rho^N, force)
};

const Ops& ops_f64();
const Ops& ops_f32();
const Ops& ops_f16o();
const Ops& ops_bf16o();

}  // namespace chromo
