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

inline int ntx_for(int storage) { return storage == LBM_STORAGE_F64 ? NTX_F64 : NTX_F32; }

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
  int words;        // words per site
  int word_bytes;   // bytes per word
  int math_bytes;   // bytes of the arithmetic type (fields, rho^N, force)
};

const Ops& ops_f64();
const Ops& ops_f32();
const Ops& ops_f16o();
const Ops& ops_bf16o();

}  // namespace chromo
