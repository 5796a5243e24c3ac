// Device code of the chromodynamic MRT lattice Boltzmann step for gfx950.
//
// One fused kernel performs a whole time step (Sec. II, Sec. III and App. A of
// Spendlove et al., arXiv 2005.04642): pull-streaming gather, colour densities
// and moments, colour index, App. B gradient and director, curvature and
// Lishchuk force with Guo's velocity, density-difference correction tensor,
// modal relaxation and reconstruction, d'Ortona recolour, store.
//
// Work decomposition ("march"): a workgroup owns a strip of TX lattice columns
// and a chunk of rows and walks up the chunk NR rows at a time (one row per
// thread row).  The chain of stencils (rho^N -> n -> K, G, u -> div u;
// Phi' -> grad Phi') needs rho^N up to 9 rows ahead of the row being written, so
// each iteration works on four bands of rows at once (LU = 3 for NR = 3, 4 for
// NR = 4):
//     M  row v+3LU : gather 18 populations, colour densities, rho^N  -> LDS ring
//     N  row v+2LU : grad rho^N, director m = grad/|grad|            -> LDS ring
//     U  row v+LU  : K = -div m, G, u, Phi'                          -> LDS ring
//     O  row v     : grad Phi', div u, C, collide, recolour, store
// Populations are read once per strip from HBM; per-row fields live in LDS
// rings of 4 NR rows (the halo in x is recomputed by the strip's edge
// threads); the populations a thread needs 3 iterations later stay in its
// registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chromo {

// Rows handled per march iteration (one per thread row) is the template
// parameter NR; the four bands are LU, 2 LU and 3 LU rows ahead of the output
// row, with LU the smallest multiple of NR not below the largest stencil
// radius (3), so every lagged quantity stays with the thread that made it.
template <int NR>
struct Pipe {
  static constexpr int LU = NR * ((3 + NR - 1) / NR);
  static constexpr int LN = 2 * LU;
  static constexpr int LM = 3 * LU;
  static constexpr int RING = 4 * NR;                   // LDS ring depth in rows
  // Iterations from the start of one band to the start of the next: a band
  // at row v needs its producer's rows up to v + 3, and the producer runs LU
  // rows ahead.  Band N starts at ITN, band U at ITU, band O at IT0.
  static constexpr int GAP = (LU + 3 + NR - 1) / NR;
  static constexpr int ITN = GAP;
  static constexpr int ITU = 2 * GAP;
  static constexpr int IT0 = 3 * GAP;
  static_assert(LN == NR + LU && LU == NR * (LU / NR), "band hand-over must stay within one thread");
  static_assert(LU >= 3 && RING >= LM + NR, "ring must hold every row a band still reads");
};

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
  T lambda6, lambda7;      // ghost-mode rates
  T gx, gy, K_fixed, eps2;
  // 16-bit offset formats, per link class (rest, axis, diagonal; class 0
  // unused): rest value fref of f_i, the offset unit fref / 2^10 and its
  // reciprocal, the colour unit 4 fref and its reciprocal
  T fref[3], fq[3], inv_fq[3], sq[3], inv_sq[3];
  int ghost_eq, fixed_K, recolor;
};

struct Geom {
  int nx, ny, walls, F;    // F = fluid rows: ny, or ny - 2 with walls
  int TX, nstrips, TY, nchunks;
  int plane;               // nx * ny
  // set per storage format and workgroup shape at launch:
  unsigned pb, rb;         // byte strides of the storage words: word q of row y at q pb + y rb
  int period;              // period of the virtual row index: ny, or 2 F with walls
  int nr_mod;              // rows per march iteration, modulo period
};

template <typename T>
struct StepArgs {
  const void* src;              // population buffers (storage format)
  void* dst;
  const T* __restrict__ force;  // [2][ny][nx] or null
  T* out_rho;                   // fields mode outputs ([ny][nx] or null)
  T* out_ux;
  T* out_uy;
  T* out_rhoN;
  // adjoint mode: dL/d(next state) at the own site ([ny][18][nx], as the
  // populations), and the outputs: forward intermediates (planes SV_*) and
  // local adjoints (planes adj::A_*), each a group of planes of the adjoint
  // workspace (row-interleaved; the pointers address the group's first plane
  // in row 0)
  const T* lam_next;
  T* out_save;
  T* out_adj;
  // solid sites anywhere: per site, bit i - 1 set when the source r - c_i of
  // link i is solid (all set at a solid site); [ny][nx] bytes, or null
  const unsigned char* bnc;
  Geom g;
  Coef<T> c;
};

// Launch modes of the step kernel: advance one step, write the macroscopic
// fields, or run the first (local) pass of the adjoint.
enum { MODE_STEP = 0, MODE_FIELDS = 1, MODE_ADJ = 3 };

// Forward intermediates the later adjoint passes read.
enum { SV_RR, SV_RB, SV_UX, SV_UY, SV_K, SV_GNX, SV_GNY, SV_N };

namespace adj {
constexpr int A_N = 21;  // local adjoints per site (see chromo_adjoint.hpp)
// planes of the adjoint workspace: the SV_N saved forward values, the A_N
// local adjoints and 11 planes of the later passes, interleaved by rows
// ([y][WS_PLANES][x], as the populations): plane k of row y starts at
// (y WS_PLANES + k) nx
constexpr int WS_PLANES = 39;
template <typename T>
__device__ __forceinline__ T* ws_row(T* group, int nx, int y) {
  return group + (size_t)y * WS_PLANES * (size_t)nx;
}
template <typename T>
__device__ void local_backward(const Coef<T>& c, const T* f, T rR, T rB, T ux, T uy, T Gx, T Gy, T dPx, T dPy,
                               T theta, T rhoN, T mx, T my, const T* lR, const T* lB, T* out);
}  // namespace adj

// ---------------------------------------------------------------------------
// Lattice links (same order as the public header): c0 = (0,0), c1 = (1,1),
// c2 = (0,1), c3 = (-1,1), c4 = (-1,0), c5 = (-1,-1), c6 = (0,-1),
// c7 = (1,-1), c8 = (1,0); opp(i) = i +- 4.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int link_cx(int i) { return (i == 1 || i == 7 || i == 8) ? 1 : ((i >= 3 && i <= 5) ? -1 : 0); }
__host__ __device__ constexpr int link_cy(int i) { return (i >= 1 && i <= 3) ? 1 : ((i >= 5 && i <= 7) ? -1 : 0); }
__host__ __device__ constexpr int link_opp(int i) { return i == 0 ? 0 : (i <= 4 ? i + 4 : i - 4); }
// link class: 0 rest, 1 axis (even i), 2 diagonal (odd i)
__host__ __device__ constexpr int link_class(int i) { return i == 0 ? 0 : ((i & 1) ? 2 : 1); }

// ---------------------------------------------------------------------------
// Population storage formats.  A format keeps the 18 populations of a site as
// NW words; a buffer is laid out [ny][NW][nx] (x fastest), word q of site
// (x, y) at (y NW + q) nx + x.
//   F64, F32 : NW = 18, word q = population (colour q / 9, link q % 9).
//   F16O, BF16O (16-bit offset formats, FP32 arithmetic): NW = 10 words of
//     4 bytes.  Words 0 and 1 are R_0 and B_0 as float.  Word 1 + i, i = 1..8,
//     packs the moving link i of both colours:
//       bits 0-15 : 2^10 (f_i - fref_i) / fref_i in FP16 (F16O) or BF16
//                   (BF16O), where f_i = R_i + B_i and
//                   fref_i = (9/5) w_i rho_0C (1 - alpha_C) is the rest value
//                   of f_i, the same in both pure phases by the density-ratio
//                   relation (Sec. II); the factor 2^10 keeps relative
//                   departures down to 6e-8 out of FP16's subnormal range;
//       bits 16-31: s_i / (4 fref_i) in FP16, clamped to magnitude below 2,
//                   with bit 14 (clear in every such FP16 value) telling which
//                   colour s_i is: 0 red, 1 blue.  s_i is the colour of
//                   smaller magnitude (with its sign), the other colour is
//                   f_i - s_i; the clamp is reached only when both colours
//                   exceed 8 fref_i in magnitude.
//     The minority colour thus keeps FP16's relative precision down to its
//     smallest tails, and f_i keeps it relative to its departure from rest.
// Memory access goes through buffer resources: word and row offsets are
// wave-uniform (SGPR soffset), only the column offset lives in a VGPR.
// ---------------------------------------------------------------------------
struct F64 {
  using W = double;
  using math = double;
  static constexpr int NW = 18;
};
struct F32 {
  using W = float;
  using math = float;
  static constexpr int NW = 18;
};
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Low-half formats of the 16-bit offset words.  pack(d, z) returns the word
// with d in the low half and FP16(z) in the high half (round to nearest even).
struct Half16 {
  static __device__ __forceinline__ unsigned pack(float d, float z) {
    const f32x2 v = {d, z};
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v, f16x2));
  }
  static __device__ __forceinline__ float low(unsigned w) {
    return (float)__builtin_bit_cast(f16x2, w)[0];
  }
};
struct BHalf16 {
  static __device__ __forceinline__ unsigned pack(float d, float z) {
    const unsigned lo = __builtin_bit_cast(unsigned short, (__bf16)d);
    const unsigned hi = __builtin_bit_cast(unsigned short, (_Float16)z);
    return lo | (hi << 16);
  }
  static __device__ __forceinline__ float low(unsigned w) { return __builtin_bit_cast(float, w << 16); }
};
template <typename H>
struct Ofs16 {
  using W = unsigned;
  using math = float;
  using Low = H;
  static constexpr int NW = 10;
};
using F16O = Ofs16<Half16>;
using BF16O = Ofs16<BHalf16>;

template <typename S>
struct is_ofs16 {
  static constexpr bool value = S::NW == 10;
};

// link carried by word q, and the word holding the reversed link of the
// same colour(s) at the same site (half-way bounce-back)
template <typename S>
__host__ __device__ constexpr int word_link(int q) {
  return S::NW == 18 ? q % 9 : (q < 2 ? 0 : q - 1);
}
template <typename S>
__host__ __device__ constexpr int word_bounce(int q) {
  return S::NW == 18 ? (q / 9) * 9 + link_opp(q % 9) : (q < 2 ? q : 1 + link_opp(q - 1));
}

template <typename W>
__device__ __forceinline__ W load_word(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(W) == 8) {
    return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  }
}
template <typename W>
__device__ __forceinline__ void store_word(W v, __amdgpu_buffer_rsrc_t r, int voff, int soff) {
  if constexpr (sizeof(W) == 8) {
    using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, voff, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
  }
}

// words -> populations (R_0..R_8, B_0..B_8) and, when F is given, the totals
// f_i = R_i + B_i (the 16-bit formats carry f_i itself for the moving links)
template <typename S, typename T>
__device__ __forceinline__ void decode(const typename S::W* w, const Coef<T>& c, T* R, T* B, T* F = nullptr) {
  if constexpr (!is_ofs16<S>::value) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      R[i] = w[i];
      B[i] = w[9 + i];
      if (F) F[i] = R[i] + B[i];
    }
  } else {
    R[0] = __builtin_bit_cast(float, w[0]);
    B[0] = __builtin_bit_cast(float, w[1]);
    if (F) F[0] = R[0] + B[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int k = link_class(i);
      const unsigned v = w[1 + i];
      const float f = __builtin_fmaf(S::Low::low(v), c.fq[k], c.fref[k]);
      // (a multiply-add of the high half, one mixed-precision instruction in
      // place of a convert and a multiply: FP16 4096^2 0.413 -> 0.406 ms; it
      // differs from the product only in the sign of a zero)
      const float s = __builtin_fmaf((float)__builtin_bit_cast(f16x2, v & 0xbfffffffu)[1], c.sq[k], 0.0f);
      const float o = f - s;
      const bool blue = (v & 0x40000000u) != 0u;
      R[i] = blue ? o : s;
      B[i] = blue ? s : o;
      if (F) F[i] = f;
    }
  }
}

// populations -> words
template <typename S, typename T>
__device__ __forceinline__ void encode(const T* R, const T* B, const Coef<T>& c, typename S::W* w) {
  if constexpr (!is_ofs16<S>::value) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      w[i] = R[i];
      w[9 + i] = B[i];
    }
  } else {
    w[0] = __builtin_bit_cast(unsigned, R[0]);
    w[1] = __builtin_bit_cast(unsigned, B[0]);
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int k = link_class(i);
      const float f = R[i] + B[i];
      const bool blue = __builtin_fabsf(B[i]) < __builtin_fabsf(R[i]);
      const float s = blue ? B[i] : R[i];
      const float z = __builtin_amdgcn_fmed3f(s * c.inv_sq[k], -1.9990234375f, 1.9990234375f);
      w[1 + i] = S::Low::pack((f - c.fref[k]) * c.inv_fq[k], z) | (blue ? 0x40000000u : 0u);
    }
  }
}

// Buffer resource over a whole population buffer below 2^32 bytes (the host
// keeps masked lattices' buffers so: the mask variant of the gather lets a
// lane choose between rows).
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, int plane) {
  const unsigned bytes = (unsigned)S::NW * (unsigned)plane * (unsigned)sizeof(typename S::W);
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)bytes, 0x00020000);
}

// Buffer resource over one lattice row of a population buffer: a 64-bit base
// at the row's first word and the row's NW nx words as its extent, so word q of
// the site in column x sits at byte offset q pb + x sizeof(W).  Offsets then
// stay within one row (below 2^32 bytes for every lattice the host accepts)
// whatever the size of the whole buffer.  The row is wave-uniform, so the
// base is formed in scalar registers.  Used only for buffers of 2^32 bytes or
// more: a buffer below that goes through one resource with the row in the
// scalar offset, which is faster for the stores (4096^2 FP32 step: 0.540 ms
// against 0.595 ms with row-based resources, the same addresses).
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* buf, const Geom& g, int row) {
  const char* base = static_cast<const char*>(buf) + (size_t)(unsigned)row * (size_t)g.rb;
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)g.rb, 0x00020000);
}

// Address a buffer of format S through one resource (the row in the scalar
// offset) rather than row by row?  For the plain float formats when the whole
// buffer is below 2^32 bytes; the 16-bit offset formats always go row by row
// (their VALU-bound step runs 0.415 ms on 4096^2 that way, 0.447 ms with both
// paths in the kernel).
template <typename S>
__device__ __forceinline__ bool one_resource(const Geom& g) {
  if constexpr (S::NW == 10) {
    return false;
  } else {
    return (unsigned long long)g.rb * (unsigned long long)g.ny < (1ull << 32);
  }
}

// Column byte offsets of one thread: x - 1, x, x + 1 (periodic).
struct Cols {
  int m, o, p;
};

// Pull-streaming gather of the words of site (x, p): the word of link i comes
// from the source site r - c_i, or, when r - c_i is a solid row, from the
// reversed link's word at r itself (half-way bounce-back).  p is wave-uniform,
// so the three rows' resources and every word offset are scalar.  WALLS: rows
// 0 and ny - 1 are solid (else y is periodic).
//
// MASK (solid sites anywhere, y periodic): the link's bounce bit of the site
// (bits: the site's byte of bounce bits) chooses, per lane, between the source
// word and the reversed link's word at the site itself; the whole byte offset,
// row included, then goes in the per-lane offset of one resource over the
// whole buffer.
template <typename S, bool WALLS, bool MASK = false, int Q0 = 0, int Q1 = S::NW>
__device__ __forceinline__ void gather_words(const void* buf, const Geom& g, int p, const Cols& x,
                                             typename S::W out[S::NW], unsigned bits = 0) {
  int rm = p - 1, rp = p + 1;
  bool bm = false, bp = false;
  if (WALLS) {
    bm = (rm == 0);
    bp = (rp == g.ny - 1);
  } else {
    if (rm < 0) rm += g.ny;
    if (rp >= g.ny) rp -= g.ny;
  }
  if constexpr (MASK) {
    const __amdgpu_buffer_rsrc_t src = make_rsrc<S>(buf, g.plane);
    const unsigned ro = (unsigned)p * g.rb, rom = (unsigned)rm * g.rb, rop = (unsigned)rp * g.rb;
#pragma unroll
    for (int q = Q0; q < Q1; ++q) {
      const int i = word_link<S>(q);
      const int dy = link_cy(i), dx = link_cx(i);
      const unsigned soff = (unsigned)q * g.pb + (dy == 1 ? rom : (dy == -1 ? rop : ro));
      const int voff = dx == 1 ? x.m : (dx == -1 ? x.p : x.o);
      if (i != 0) {
        const unsigned own = (unsigned)x.o + (unsigned)word_bounce<S>(q) * g.pb + ro;
        const unsigned off = ((bits >> (i - 1)) & 1u) ? own : (unsigned)voff + soff;
        out[q] = load_word<typename S::W>(src, (int)off, 0);
      } else {
        out[q] = load_word<typename S::W>(src, voff, (int)soff);
      }
    }
  } else if (one_resource<S>(g)) {
    const __amdgpu_buffer_rsrc_t src = make_rsrc<S>(buf, g.plane);
    const unsigned ro = (unsigned)p * g.rb, rom = (unsigned)rm * g.rb, rop = (unsigned)rp * g.rb;
#pragma unroll
    for (int q = Q0; q < Q1; ++q) {
      const int i = word_link<S>(q);
      const int dy = link_cy(i), dx = link_cx(i);
      const bool bounce = WALLS && ((dy == 1 && bm) || (dy == -1 && bp));
      const unsigned soff = bounce ? (unsigned)word_bounce<S>(q) * g.pb + ro
                                   : (unsigned)q * g.pb + (dy == 1 ? rom : (dy == -1 ? rop : ro));
      const int voff = bounce ? x.o : (dx == 1 ? x.m : (dx == -1 ? x.p : x.o));
      out[q] = load_word<typename S::W>(src, voff, (int)soff);
    }
  } else {
    const __amdgpu_buffer_rsrc_t r0 = row_rsrc<S>(buf, g, p);
    const __amdgpu_buffer_rsrc_t rM = row_rsrc<S>(buf, g, rm);
    const __amdgpu_buffer_rsrc_t rP = row_rsrc<S>(buf, g, rp);
#pragma unroll
    for (int q = Q0; q < Q1; ++q) {
      const int i = word_link<S>(q);
      const int dy = link_cy(i), dx = link_cx(i);
      const bool bounce = WALLS && ((dy == 1 && bm) || (dy == -1 && bp));
      const unsigned soff = (unsigned)(bounce ? word_bounce<S>(q) : q) * g.pb;
      const int voff = bounce ? x.o : (dx == 1 ? x.m : (dx == -1 ? x.p : x.o));
      const __amdgpu_buffer_rsrc_t r = bounce ? r0 : (dy == 1 ? rM : (dy == -1 ? rP : r0));
      out[q] = load_word<typename S::W>(r, voff, (int)soff);
    }
  }
}

// Byte of bounce bits of site (p, xg).
__device__ __forceinline__ unsigned bounce_bits_at(const unsigned char* bnc, const Geom& g, int p, int xg) {
  return bnc[(size_t)p * g.nx + xg];
}

// The same through a buffer resource over the plane of bytes: the row offset
// stays scalar and the lane's column is the only per-lane offset (no 64-bit
// address per lane).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bounce_rsrc(const unsigned char* bnc, int plane) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)bnc, (short)0, plane, 0x00020000);
}
__device__ __forceinline__ unsigned bounce_bits_at(__amdgpu_buffer_rsrc_t r, const Geom& g, int p, int xg) {
  return (unsigned)__builtin_amdgcn_raw_buffer_load_b8(r, xg, p * g.nx, 0);
}

template <typename S>
__device__ __forceinline__ void gather_words_any(const void* src, const Geom& g, int p, const Cols& x,
                                                 typename S::W out[S::NW]) {
  if (g.walls) {
    gather_words<S, true>(src, g, p, x, out);
  } else {
    gather_words<S, false>(src, g, p, x, out);
  }
}

// Wave-uniform virtual row of the march, kept modulo its period (ny, or the
// 2 F rows of the fluid strip and its mirror image with walls) and advanced
// by one march iteration at a time.
template <bool WALLS>
struct RowTrack {
  int t;
  __device__ __forceinline__ void init(int v, const Geom& g) {
    t = v % g.period;
    if (t < 0) t += g.period;
  }
  __device__ __forceinline__ void advance(const Geom& g) {
    t += g.nr_mod;
    if (t >= g.period) t -= g.period;
  }
  // physical row; with walls the strip is reflected about the two wall planes
  __device__ __forceinline__ int phys(const Geom& g) const { return WALLS ? (t >= g.F ? 2 * g.F - t : 1 + t) : t; }
  __device__ __forceinline__ bool refl(const Geom& g) const { return WALLS && t >= g.F; }
};

template <int RING>
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
// b_N w_i for the diagonal (w = 1/36) and axis (w = 1/9) links, each product
// formed in double and rounded once to T
template <int R, typename T>
__device__ __forceinline__ T stencil_bd(int n) {
  return T(stencil_b<R, double>(n) * (1.0 / 36.0));
}
template <int R, typename T>
__device__ __forceinline__ T stencil_ba(int n) {
  return T(stencil_b<R, double>(n) * (1.0 / 9.0));
}

// (d/dx, d/dy) of a ring field at (ring row `row`, column tx); s points at the
// field's first element, successive ring rows are STRIDE elements apart and
// successive columns CS.  Row pointers start R columns left of tx so that
// every column offset is non-negative (LDS instruction offsets are unsigned).
//
// MASK: solid sites hold NaN in every stencil operand, and a NaN tap reads the
// value at the stencil's centre instead (the zero-gradient continuation into
// the solid).  A fluid site's own value is never NaN unless the run has
// already failed, which the masses then report.
template <typename T>
__device__ __forceinline__ T tap_or(T v, T c0) {
  return v == v ? v : c0;
}

template <int R, int RING, int STRIDE, int CS, typename T, bool MASK = false>
__device__ __forceinline__ void ring_grad(const T* s, int row, int tx, T& gx, T& gy) {
  gx = T(0);
  gy = T(0);
  const T* md = s + ring_row<RING>(row) * STRIDE + (tx - R) * CS;
  const T c0 = MASK ? md[R * CS] : T(0);
  auto v = [&](T x) { return MASK ? tap_or(x, c0) : x; };
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T bd = stencil_bd<R, T>(n), ba = stencil_ba<R, T>(n);
    const T* up = s + ring_row<RING>(row + n) * STRIDE + (tx - R) * CS;
    const T* dn = s + ring_row<RING>(row - n) * STRIDE + (tx - R) * CS;
    const T d1 = v(up[(R + n) * CS]) - v(dn[(R - n) * CS]);
    const T d3 = v(up[(R - n) * CS]) - v(dn[(R + n) * CS]);
    const T d8 = v(md[(R + n) * CS]) - v(md[(R - n) * CS]);
    const T d2 = v(up[R * CS]) - v(dn[R * CS]);
    gx += ba * d8;
    gx += bd * (d1 - d3);
    gy += ba * d2;
    gy += bd * (d1 + d3);
  }
}

// d vx/dx + d vy/dy of a ring vector field.
template <int R, int RING, int STRIDE, int CS, typename T, bool MASK = false>
__device__ __forceinline__ T ring_div(const T* sx, const T* sy, int row, int tx) {
  T acc = T(0);
  const T* mdx = sx + ring_row<RING>(row) * STRIDE + (tx - R) * CS;
  const T cx = MASK ? mdx[R * CS] : T(0);
  const T cy = MASK ? sy[ring_row<RING>(row) * STRIDE + tx * CS] : T(0);
  auto vx = [&](T x) { return MASK ? tap_or(x, cx) : x; };
  auto vy = [&](T x) { return MASK ? tap_or(x, cy) : x; };
#pragma unroll
  for (int n = 1; n <= R; ++n) {
    const T bd = stencil_bd<R, T>(n), ba = stencil_ba<R, T>(n);
    const T* upx = sx + ring_row<RING>(row + n) * STRIDE + (tx - R) * CS;
    const T* dnx = sx + ring_row<RING>(row - n) * STRIDE + (tx - R) * CS;
    const T* upy = sy + ring_row<RING>(row + n) * STRIDE + (tx - R) * CS;
    const T* dny = sy + ring_row<RING>(row - n) * STRIDE + (tx - R) * CS;
    const T d1 = vx(upx[(R + n) * CS]) - vx(dnx[(R - n) * CS]);
    const T d3 = vx(upx[(R - n) * CS]) - vx(dnx[(R + n) * CS]);
    const T d8 = vx(mdx[(R + n) * CS]) - vx(mdx[(R - n) * CS]);
    const T e1 = vy(upy[(R + n) * CS]) - vy(dny[(R - n) * CS]);
    const T e3 = vy(upy[(R - n) * CS]) - vy(dny[(R + n) * CS]);
    const T e2 = vy(upy[R * CS]) - vy(dny[R * CS]);
    acc += ba * (d8 + e2);
    acc += bd * ((d1 - d3) + (e1 + e3));
  }
  return acc;
}

// LDS rings, laid out [ring row][column][field]: the fields of one site and
// its stencil neighbours in the same row are within the immediate offset range
// of paired LDS reads from one address (fewer address computations; the
// 13-element column stride is odd, so lanes of a wave hit distinct banks).
enum {
  // stencil operands
  F_RHON, F_MX, F_MY, F_UX, F_UY, F_PHI,
  // values handed from one band to a later one at the same site
  F_RR, F_RB,    // colour densities, band M -> bands U, O
  F_GNX, F_GNY,  // grad rho^N, band N -> band U
  F_GX, F_GY,    // force G, band U -> band O
  F_IRHO,        // 1/rho, band U -> band O
  NFIELD
};

template <typename T, int NTX, int RING>
struct Smem {
  static constexpr int STRIDE = NFIELD * NTX;  // elements per ring row
  static constexpr int CS = NFIELD;            // elements between neighbouring columns
  static constexpr int PAD = 3 * NFIELD;       // keeps (tx - 3) CS inside the array
  T pad[PAD];
  T d[RING * STRIDE];
  __device__ __forceinline__ T& at(int field, int row, int tx) { return d[row * STRIDE + tx * CS + field]; }
  __device__ __forceinline__ const T* field(int f) const { return d + f; }
};

// Register state of one thread: the nine total populations of the rows it
// gathered (one slot per iteration, read again 2 and 3 iterations later) and
// the storage words prefetched for the next band-M row (decoded only when
// used, so the loads stay in flight for a whole iteration).
template <typename S>
struct March {
  using T = typename S::math;
  T rf[4][9];
  typename S::W pw[S::NW];
  T fx[2], fy[2];  // body force of the band-U rows, loaded one iteration ahead
  unsigned bn;     // mask variant: bounce bits of the next band-M row, loaded one iteration ahead
  int prow;        // the next band-M row (wave-uniform), whose words are gathered in two parts
  unsigned bng;    // mask variant: that row's bounce bits (bn moves on to the following row)
};

// The words of the next band-M row are gathered in two parts: the first two
// thirds in band M, the rest just before band U.  Measured on the 4096^2 step
// (one MI355X, back to back, same results): FP32 0.540 -> 0.493 ms, FP16
// 0.408 -> 0.404 ms, with a mask (21.6 % solid) FP32 0.667 -> 0.563 ms; one
// third or one half first ran slower than two thirds, and five sixths or more
// first slower than a single part.  The adjoint's march (pass 1) runs 0.5 %
// slower split and keeps one part.
template <typename S>
constexpr int gather_split() {
  return S::NW * 2 / 3;
}
template <int MODE, bool MASK>
constexpr bool split_gather() {
  return MODE != MODE_ADJ;
}

struct Thread {
  int tx, ty, xg, ya, yb, nit;
  Cols cols;
  bool own;
};

template <typename T>
__device__ __forceinline__ void momenta(const T* f, T& jx, T& jy) {
  const T d15 = f[1] - f[5], d37 = f[3] - f[7];
  jx = (d15 - d37) + (f[8] - f[4]);
  jy = (d15 + d37) + (f[2] - f[6]);
}

// Colour index (Sec. II); exactly +-1 in the pure phases (IEEE division).
template <typename T>
__device__ __forceinline__ T colour_index(T a0, T b0) {
  return (a0 - b0) / (a0 + b0);
}

// 1/x and 1/sqrt(x) where no exact value is needed: in float the hardware
// estimate refined by one Newton step (within about one unit in the last
// place), in double the IEEE operations.
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(r, __builtin_fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_pos(float x) {
  const float r = __builtin_amdgcn_rsqf(x);
  return r * __builtin_fmaf(-0.5f * x * r, r, 1.5f);
}
__device__ __forceinline__ double rsqrt_pos(double x) { return 1.0 / sqrt(x); }

// Collision, recolour and store of one site (band O).
// MASK: a site without mass (a solid site, whose words encode zero populations)
// stores zero populations.
template <typename S, typename T, int MODE, bool MASK = false>
__device__ __forceinline__ void collide_store(const StepArgs<T>& a, void* dst, const T* f, T rR,
                                              T rB, T ux, T uy, T Gx, T Gy, T inv_rho, T dPx, T dPy, T theta,
                                              T rhoN, T mx, T my, int p, const Thread& t,
                                              const T* lam = nullptr) {
  const Coef<T>& c = a.c;
  const T rho = rR + rB;
  if (MODE == MODE_FIELDS) {
    const int site = p * a.g.nx + t.xg;
    if (a.out_rho) a.out_rho[site] = rho;
    if (a.out_ux) a.out_ux[site] = ux;
    if (a.out_uy) a.out_uy[site] = uy;
    if (a.out_rhoN) a.out_rhoN[site] = rhoN;
    return;
  }
  if (MODE == MODE_ADJ) {
    const int nx = a.g.nx;
    T lR[9], lB[9], out[adj::A_N];  // lam: dL/d(next state) at this site, [C i]
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      lR[i] = lam[i];
      lB[i] = lam[9 + i];
    }
    adj::local_backward(c, f, rR, rB, ux, uy, Gx, Gy, dPx, dPy, theta, rhoN, mx, my, lR, lB, out);
    if constexpr (MASK) {
      // a solid site has no adjoints (the transposed stencils read them as 0)
      if (rho == T(0)) {
#pragma unroll
        for (int q = 0; q < adj::A_N; ++q) out[q] = T(0);
      }
    }
    T* oa = adj::ws_row(a.out_adj, nx, p) + t.xg;
#pragma unroll
    for (int q = 0; q < adj::A_N; ++q) oa[q * nx] = out[q];
    T* sv = adj::ws_row(a.out_save, nx, p) + t.xg;
    sv[SV_RR * nx] = rR;
    sv[SV_RB * nx] = rB;
    sv[SV_UX * nx] = ux;
    sv[SV_UY * nx] = uy;
    return;
  }
  // modes of f (App. A projectors), summed with antisymmetric pair differences
  const T d15 = f[1] - f[5], d37 = f[3] - f[7], d84 = f[8] - f[4], d26 = f[2] - f[6];
  const T s15 = f[1] + f[5], s37 = f[3] + f[7], sd = s15 + s37;
  const T pxx = sd + (f[4] + f[8]);
  const T pyy = sd + (f[2] + f[6]);
  const T pxy = s15 - s37;
  const T N = f[0] - T(2) * ((f[2] + f[6]) + (f[4] + f[8])) + T(4) * sd;
  const T Jx = T(4) * (d15 - d37) - T(2) * d84;
  const T Jy = T(4) * (d15 + d37) - T(2) * d26;
  // lambda_3 from nu(rho^N) = (2/lambda_3 - 1)/6 (Sec. II), nu linear in rho^N
  const T nu = c.hnuR * (T(1) + rhoN) + c.hnuB * (T(1) - rhoN);
  const T l3 = T(2) * recip(T(6) * nu + T(1));
  // correction tensor C_ab (App. A, eq. Correction)
  const T k = T(1) - T(0.5) * l3;
  const T iso = ux * dPx + uy * dPy - rho * theta * T(1.0 / 3.0);
  const T Cxx = k * (T(2) * ux * (Gx - dPx) - iso);
  const T Cyy = k * (T(2) * uy * (Gy - dPy) - iso);
  const T Cxy = k * (ux * (Gy - dPy) + uy * (Gx - dPx));
  // modal increments m+ - m (App. A, modal evolution eqs.): rho fixed, j += G,
  // Pi relaxes to P delta + rho u u with source C, ghosts relax at lambda_6, lambda_7
  const T P = c.c06R * rR + c.c06B * rB;
  const T dxx = Cxx - l3 * ((pxx - P) - rho * ux * ux);
  const T dyy = Cyy - l3 * ((pyy - P) - rho * uy * uy);
  const T dxy = Cxy - l3 * (pxy - rho * ux * uy);
  const T N0 = c.ghost_eq ? T(0) : T(1.8) * (c.alphaR * rR + c.alphaB * rB) - T(0.8) * rho;
  const T dN = -c.lambda6 * (N - N0);
  const T dJx = -c.lambda7 * Jx;
  const T dJy = -c.lambda7 * Jy;
  // f+ = f + M^{-1} (m+ - m): closed-form columns k^(p) of App. A
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
  // d'Ortona recolour (Sec. II): t_i = beta phi_i rho_R rho_B / rho (m . c_hat_i),
  // R_i = (rho_R/rho) f_i+ + t_i, B_i = (rho_B/rho) f_i+ - t_i.  The colour in
  // the minority takes its share amin f_i+ -+ t_i (amin = its density times
  // 1/rho, exactly 0 in a pure phase) and the majority colour the rest,
  // f_i+ minus that.  So R_i + B_i = f_i+ up to one rounding of the majority,
  // and no rounded split factor (1 - amin) multiplies every population: on a
  // steady interface such a factor's rounding repeats with the same sign every
  // step and shifts the colour masses (FP32, density ratio 100: 4e-5 of the
  // local density after 1000 steps, against 8e-6 this way).
  const bool red_major = rB <= rR;
  const T amin = (red_major ? rB : rR) * inv_rho;
  T t1 = T(0), t3 = T(0), t2 = T(0), t8 = T(0);
  if (c.recolor) {
    const T moving = (c.c1R * rR + c.c1B * rB) * inv_rho;
    const T q = c.beta18 * (amin * (red_major ? rR : rB)) * moving;
    const T qa = q * T(1.0 / 9.0);
    const T qd = q * T(1.0 / 36.0) * T(0.70710678118654752440);
    // the minority colour carries -t_i when it is blue
    const T sg = red_major ? T(-1) : T(1);
    t8 = sg * (qa * mx);
    t2 = sg * (qa * my);
    t1 = sg * (qd * (mx + my));
    t3 = sg * (qd * (my - mx));
  }
  T mn[9];  // minority colour's populations
  mn[0] = amin * fp[0];
  mn[1] = amin * fp[1] + t1;
  mn[5] = amin * fp[5] - t1;
  mn[3] = amin * fp[3] + t3;
  mn[7] = amin * fp[7] - t3;
  mn[2] = amin * fp[2] + t2;
  mn[6] = amin * fp[6] - t2;
  mn[8] = amin * fp[8] + t8;
  mn[4] = amin * fp[4] - t8;
  T R[9], B[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const T mj = fp[i] - mn[i];
    R[i] = red_major ? mj : mn[i];
    B[i] = red_major ? mn[i] : mj;
  }
  if constexpr (MASK) {
    if (rho == T(0)) {  // a solid site keeps the encoding of zero populations
#pragma unroll
      for (int i = 0; i < 9; ++i) R[i] = B[i] = T(0);
    }
  }
  typename S::W w[S::NW];
  encode<S>(R, B, c, w);
  if (one_resource<S>(a.g)) {
    const __amdgpu_buffer_rsrc_t dr = make_rsrc<S>(dst, a.g.plane);
    const unsigned ro = (unsigned)p * a.g.rb;
#pragma unroll
    for (int q = 0; q < S::NW; ++q) store_word<typename S::W>(w[q], dr, t.cols.o, (int)(q * a.g.pb + ro));
  } else {
    const __amdgpu_buffer_rsrc_t dr = row_rsrc<S>(dst, a.g, p);
#pragma unroll
    for (int q = 0; q < S::NW; ++q) store_word<typename S::W>(w[q], dr, t.cols.o, (int)(q * a.g.pb));
  }
}

// One march iteration; S = it mod 4 selects the register-ring slots.  tM and
// tU track the virtual rows of the next band-M gather and of band U.
template <int S, typename ST, typename T, int NTX, int NR, int RG, int RK, int RP, int RU, bool WALLS, int MODE,
          bool MASK = false>
__device__ __forceinline__ void march_iter(int it, const StepArgs<T>& a, const void* src, void* dst,
                                           Smem<T, NTX, Pipe<NR>::RING>& sm,
                                           March<ST>& st, const Thread& t, RowTrack<WALLS>& tM,
                                           RowTrack<WALLS>& tU) {
  using PP = Pipe<NR>;
  constexpr int RING = PP::RING;
  using SM = Smem<T, NTX, RING>;
  const Geom& g = a.g;
  const Coef<T>& c = a.c;
  // ty passes through an opaque scalar move each iteration, so the ring-row
  // addresses derived from it are formed when used rather than hoisted out of
  // the loop for all four unrolled copies (which exhausts the VGPR budget)
  const int tx = t.tx;
  int ty;
  asm volatile("s_mov_b32 %0, %1" : "=s"(ty) : "s"(t.ty));
  // band-O virtual row of this thread (wave-uniform)
  const int base = t.ya - NR * PP::IT0 + NR * it + ty;
  constexpr int sM = S, sU = (S + 2) & 3, sO = (S + 1) & 3;
  // ring rows of the four bands (row index = virtual row - (ya - NR IT0))
  const int rowO = NR * S + ty;
  const int rowU = rowO + PP::LU, rowN = rowO + PP::LN, rowM = rowO + PP::LM;

  // ---- band M: colour densities, total populations, colour index ----------
  {
    T* rf = st.rf[sM];
    T pr[9], pb[9];
    decode<ST>(st.pw, c, pr, pb, rf);
    T rR = ((pr[0] + pr[2]) + (pr[4] + pr[6])) + ((pr[1] + pr[3]) + (pr[5] + pr[7])) + pr[8];
    T rB = ((pb[0] + pb[2]) + (pb[4] + pb[6])) + ((pb[1] + pb[3]) + (pb[5] + pb[7])) + pb[8];
    const int rm = ring_row<RING>(rowM);
    sm.at(F_RR, rm, tx) = rR;
    sm.at(F_RB, rm, tx) = rB;
    sm.at(F_RHON, rm, tx) = colour_index(rR * c.inv_rho0R, rB * c.inv_rho0B);
    // prefetch the next band-M row (after the last iteration: a row never used).
    // The loads of the plain float formats go out at a raised wave priority, so
    // they issue ahead of other waves' arithmetic (FP32 4096^2: 3.6 % faster);
    // the VALU-bound 16-bit formats run slower with it and keep the default.
    // The mask variant loads a row's bounce bits one iteration before its
    // gather (just after the previous gather), so the gather need not wait for
    // a load of its own before it forms its addresses (4096^2: 3.4 % faster;
    // through a buffer resource, which spills no registers, 2 % more).
    st.prow = tM.phys(g);
    if constexpr (!is_ofs16<ST>::value) __builtin_amdgcn_s_setprio(1);
    if constexpr (!split_gather<MODE, MASK>()) {
      gather_words<ST, WALLS, MASK>(src, g, st.prow, t.cols, st.pw, st.bn);
    } else {
      if constexpr (MASK) st.bng = st.bn;
      gather_words<ST, WALLS, MASK, 0, gather_split<ST>()>(src, g, st.prow, t.cols, st.pw, MASK ? st.bng : 0u);
    }
    if constexpr (!is_ofs16<ST>::value) __builtin_amdgcn_s_setprio(0);
    tM.advance(g);
    if constexpr (MASK) st.bn = bounce_bits_at(bounce_rsrc(a.bnc, g.plane), g, tM.phys(g), t.xg);
  }
  __syncthreads();

  // ---- band N: grad rho^N and director m -------------------------------------
  if (a.force) {
    // the next iteration's band-U row: its force is waited for with this
    // iteration's stores, before band M, instead of right where it is used
    RowTrack<WALLS> nu = tU;
    nu.advance(g);
    const int site = nu.phys(g) * g.nx + t.xg;
    st.fx[(S + 1) & 1] = a.force[site];
    st.fy[(S + 1) & 1] = a.force[g.plane + site];
  }
  if (it >= PP::ITN && tx >= RG && tx < NTX - RG) {
    T gx, gy;
    ring_grad<RG, RING, SM::STRIDE, SM::CS, T, MASK>(sm.field(F_RHON), rowN, tx, gx, gy);
    const T is = rsqrt_pos(gx * gx + gy * gy + c.eps2);
    const int rn = ring_row<RING>(rowN);
    T mx = gx * is, my = gy * is;
    if (MASK) {
      // a solid site (rho^N = 0/0) marks m as well: its stencil sums mix
      // fluid taps and are finite when the site has fluid all round
      const T r0 = sm.at(F_RHON, rn, tx);
      if (!(r0 == r0)) mx = my = __builtin_nan("");
    }
    sm.at(F_MX, rn, tx) = mx;
    sm.at(F_MY, rn, tx) = my;
    sm.at(F_GNX, rn, tx) = gx;
    sm.at(F_GNY, rn, tx) = gy;
  }
  __syncthreads();

  // the rest of the next band-M row's words (see gather_split)
  if constexpr (split_gather<MODE, MASK>()) {
    if constexpr (!is_ofs16<ST>::value) __builtin_amdgcn_s_setprio(1);
    gather_words<ST, WALLS, MASK, gather_split<ST>(), ST::NW>(src, g, st.prow, t.cols, st.pw,
                                                              MASK ? st.bng : 0u);
    if constexpr (!is_ofs16<ST>::value) __builtin_amdgcn_s_setprio(0);
  }

  // ---- band U: Phi', curvature, force and velocity -------------------------
  if (it >= PP::ITU) {
    const T* rf = st.rf[sU];
    const int ru = ring_row<RING>(rowU);
    const T rR = sm.at(F_RR, ru, tx), rB = sm.at(F_RB, ru, tx);
    const T rho = rR + rB;
    T phi = c.c06R * rR + c.phiB * rB - rho * T(1.0 / 3.0);
    if (MASK && rho == T(0)) phi = __builtin_nan("");  // solid site: the stencils' marker
    sm.at(F_PHI, ru, tx) = phi;
    if (tx >= RG + RK && tx < NTX - RG - RK) {
      const int p = tU.phys(g);
      const bool refl = tU.refl(g);
      T K;
      if (c.fixed_K) {
        K = c.K_fixed;
      } else {
        K = -ring_div<RK, RING, SM::STRIDE, SM::CS, T, MASK>(sm.field(F_MX), sm.field(F_MY), rowU,
                                                            tx);  // K = div n, n = -m
      }
      if (MODE == MODE_ADJ) {
        const int v = base + PP::LU;  // virtual row of band U
        if (t.own && v >= t.ya && v < t.yb) adj::ws_row(a.out_save, g.nx, p)[SV_K * g.nx + t.xg] = K;
      }
      const T gnx = sm.at(F_GNX, ru, tx), gny = sm.at(F_GNY, ru, tx);
      T Gx = c.half_sigma * K * gnx + c.gx;
      T Gy = c.half_sigma * K * gny + (refl ? -c.gy : c.gy);
      if (a.force) {
        Gx += st.fx[S & 1];
        Gy += refl ? -st.fy[S & 1] : st.fy[S & 1];
      }
      T jx, jy;
      momenta(rf, jx, jy);
      if (refl) jy = -jy;   // mirror image: the y-momentum changes sign
      const T ir = recip(rho);
      T ux = (jx + T(0.5) * Gx) * ir, uy = (jy + T(0.5) * Gy) * ir;
      if (MASK && rho == T(0)) ux = uy = __builtin_nan("");  // solid site (1/0 need not give NaN)
      sm.at(F_UX, ru, tx) = ux;
      sm.at(F_UY, ru, tx) = uy;
      sm.at(F_GX, ru, tx) = Gx;
      sm.at(F_GY, ru, tx) = Gy;
      sm.at(F_IRHO, ru, tx) = ir;
    }
  }
  tU.advance(g);
  __syncthreads();

  // ---- band O: correction, collision, recolour, store ----------------------
  if (it >= PP::IT0 && t.own && base < t.yb) {
    // the adjoint's dL/d(next state) at this row, loaded before the stencils
    // rather than in the local backward: 4096^2 pass 1 1.5 % faster (a band
    // earlier, or with the two-part gather, slower); same results
    T lam[18];
    if constexpr (MODE == MODE_ADJ) {
      const T* ln = a.lam_next + (size_t)(WALLS ? base + 1 : base) * 18 * g.nx + t.xg;  // [y][C i][x]
#pragma unroll
      for (int q = 0; q < 18; ++q) lam[q] = ln[q * g.nx];
    }
    T dPx, dPy;
    ring_grad<RP, RING, SM::STRIDE, SM::CS, T, MASK>(sm.field(F_PHI), rowO, tx, dPx, dPy);
    __builtin_amdgcn_sched_barrier(0);  // bound register pressure: finish one stencil before the next
    const T theta = ring_div<RU, RING, SM::STRIDE, SM::CS, T, MASK>(sm.field(F_UX), sm.field(F_UY), rowO, tx);
    __builtin_amdgcn_sched_barrier(0);
    const int ro = ring_row<RING>(rowO);
    const int p = WALLS ? base + 1 : base;
    if (MODE == MODE_ADJ) {
      T* sv = adj::ws_row(a.out_save, g.nx, p) + t.xg;
      sv[SV_GNX * g.nx] = sm.at(F_GNX, ro, tx);
      sv[SV_GNY * g.nx] = sm.at(F_GNY, ro, tx);
    }
    collide_store<ST, T, MODE, MASK>(a, dst, st.rf[sO], sm.at(F_RR, ro, tx), sm.at(F_RB, ro, tx), sm.at(F_UX, ro, tx), sm.at(F_UY, ro, tx),
                                 sm.at(F_GX, ro, tx), sm.at(F_GY, ro, tx), sm.at(F_IRHO, ro, tx), dPx, dPy, theta,
                                 sm.at(F_RHON, ro, tx), sm.at(F_MX, ro, tx), sm.at(F_MY, ro, tx), p, t, lam);
  }
}

// One tile (strip x chunk of rows) of one lattice: the whole march.
template <typename ST, int NTX, int NR, int RG, int RK, int RP, int RU, bool WALLS, int MODE, bool MASK = false>
__device__ __forceinline__ void march_tile(const StepArgs<typename ST::math>& a, int tile,
                                           Smem<typename ST::math, NTX, Pipe<NR>::RING>& sm) {
  using T = typename ST::math;
  using PP = Pipe<NR>;
  constexpr int H = RG + RK + RU;
  const Geom& g = a.g;
  const void* src = a.src;
  void* dst = MODE != MODE_STEP ? const_cast<void*>(a.src) : a.dst;  // no store outside MODE_STEP
  Thread t;
  t.tx = threadIdx.x % NTX;
  t.ty = __builtin_amdgcn_readfirstlane(threadIdx.x / NTX);
  const int strip = tile % g.nstrips;
  const int chunk = tile / g.nstrips;
  const int x0 = strip * g.TX;
  const int txe = min(g.TX, g.nx - x0);
  const int col = t.tx - H;
  int xg = (x0 + col) % g.nx;
  if (xg < 0) xg += g.nx;
  t.xg = xg;
  const int E = (int)sizeof(typename ST::W);
  t.cols.o = xg * E;
  t.cols.m = (xg == 0 ? g.nx - 1 : xg - 1) * E;
  t.cols.p = (xg == g.nx - 1 ? 0 : xg + 1) * E;
  t.own = col >= 0 && col < txe;
  t.ya = chunk * g.TY;
  t.yb = min(g.F, t.ya + g.TY);
  t.nit = PP::IT0 + (t.yb - t.ya + NR - 1) / NR;

  March<ST> st;
  const int v0 = t.ya - NR * PP::IT0 + t.ty;  // band-O virtual row of iteration 0
  RowTrack<WALLS> tM, tU;
  tM.init(v0 + PP::LM, g);
  st.bn = 0;
  if constexpr (MASK) st.bn = bounce_bits_at(bounce_rsrc(a.bnc, g.plane), g, tM.phys(g), t.xg);
  gather_words<ST, WALLS, MASK>(src, g, tM.phys(g), t.cols, st.pw, st.bn);
  tM.advance(g);
  if constexpr (MASK) st.bn = bounce_bits_at(bounce_rsrc(a.bnc, g.plane), g, tM.phys(g), t.xg);
  tU.init(v0 + PP::LU, g);
  if (a.force) {
    const int site = tU.phys(g) * g.nx + t.xg;
    st.fx[0] = a.force[site];
    st.fy[0] = a.force[g.plane + site];
  }
  for (int it = 0; it < t.nit; it += 4) {
    march_iter<0, ST, T, NTX, NR, RG, RK, RP, RU, WALLS, MODE, MASK>(it, a, src, dst, sm, st, t, tM, tU);
    if (it + 1 < t.nit)
      march_iter<1, ST, T, NTX, NR, RG, RK, RP, RU, WALLS, MODE, MASK>(it + 1, a, src, dst, sm, st, t, tM, tU);
    if (it + 2 < t.nit)
      march_iter<2, ST, T, NTX, NR, RG, RK, RP, RU, WALLS, MODE, MASK>(it + 2, a, src, dst, sm, st, t, tM, tU);
    if (it + 3 < t.nit)
      march_iter<3, ST, T, NTX, NR, RG, RK, RP, RU, WALLS, MODE, MASK>(it + 3, a, src, dst, sm, st, t, tM, tU);
  }
}

template <typename ST, int NTX, int NR, int RG, int RK, int RP, int RU, bool WALLS, int MODE, bool MASK = false>
__global__ void __launch_bounds__(NTX * NR, 1) chromo_step_kernel(StepArgs<typename ST::math> a) {
  using T = typename ST::math;
  using PP = Pipe<NR>;
  static_assert(NTX > 2 * (RG + RK + RU), "strip must be wider than its halo");
  static_assert(NTX % 64 == 0, "a wavefront must cover a single lattice row");
  __shared__ Smem<T, NTX, PP::RING> sm;
  const Geom& g = a.g;
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each
  // XCD gets a contiguous run of tiles (neighbouring strips of the same rows),
  // whose shared halo columns and boundary cache lines then meet in one L2.
  const int ntiles = g.nstrips * g.nchunks;
  const int per_xcd = (ntiles + 7) / 8;
  const int tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (tile >= ntiles) return;
  march_tile<ST, NTX, NR, RG, RK, RP, RU, WALLS, MODE, MASK>(a, tile, sm);
}

// ---------------------------------------------------------------------------
// Batched step: many independent lattices in one launch.  Each
// workgroup owns a bin of work items (lattice, tile), planned on the host so
// that the bins' costs are balanced, and runs them one after the other.
// ---------------------------------------------------------------------------
template <typename T>
struct SimDesc {
  Geom g;                 // per-lattice geometry and tile plan
  Coef<T> c;              // per-lattice constants
  unsigned long long off; // byte offset of the lattice's populations in both packed buffers
  const T* force;         // per-site force density [2][ny][nx] of the lattice, or null
  const unsigned char* bnc;  // bounce bits of the lattice's solid-site mask, or null
};

template <typename T>
struct BatchArgs {
  const char* src;              // packed population buffers
  char* dst;
  const SimDesc<T>* sims;
  const int* bin_start;         // [nbins + 1] offsets into items
  const int* items;             // pairs (lattice, tile)
};

template <typename ST, int NTX, int NR, int RG, int RK, int RP, int RU, bool WALLS = false, bool MASK = false>
__global__ void __launch_bounds__(NTX * NR, 1) chromo_batch_kernel(BatchArgs<typename ST::math> b) {
  using T = typename ST::math;
  using PP = Pipe<NR>;
  static_assert(NTX > 2 * (RG + RK + RU), "strip must be wider than its halo");
  __shared__ Smem<T, NTX, PP::RING> sm;
  const int k0 = b.bin_start[blockIdx.x], k1 = b.bin_start[blockIdx.x + 1];
  for (int k = k0; k < k1; ++k) {
    const int sim = b.items[2 * k], tile = b.items[2 * k + 1];
    StepArgs<T> a;
    a.src = b.src + b.sims[sim].off;
    a.dst = b.dst + b.sims[sim].off;
    a.force = b.sims[sim].force;
    a.out_rho = a.out_ux = a.out_uy = a.out_rhoN = a.out_save = a.out_adj = nullptr;
    a.lam_next = nullptr;
    a.bnc = b.sims[sim].bnc;
    a.g = b.sims[sim].g;
    a.c = b.sims[sim].c;
    // in a batch with masks, lattices without one take the plain march
    if constexpr (MASK) {
      if (a.bnc) {
        march_tile<ST, NTX, NR, RG, RK, RP, RU, WALLS, MODE_STEP, true>(a, tile, sm);
      } else {
        march_tile<ST, NTX, NR, RG, RK, RP, RU, WALLS, MODE_STEP, false>(a, tile, sm);
      }
    } else {
      march_tile<ST, NTX, NR, RG, RK, RP, RU, WALLS, MODE_STEP, false>(a, tile, sm);
    }
    __syncthreads();  // the next tile reuses the LDS rings
  }
}

// ---------------------------------------------------------------------------
// streaming only (test mode): buf'_i(r) = f_i(r)
// ---------------------------------------------------------------------------
template <typename S>
__global__ void __launch_bounds__(256) stream_only_kernel(const void* src, void* dst, Geom g) {
  using W = typename S::W;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;  // fluid row index
  if (x >= g.nx) return;
  const int p = g.walls ? k + 1 : k;
  const int E = (int)sizeof(W);
  Cols cols;
  cols.o = x * E;
  cols.m = (x == 0 ? g.nx - 1 : x - 1) * E;
  cols.p = (x == g.nx - 1 ? 0 : x + 1) * E;
  W v[S::NW];
  gather_words_any<S>(src, g, p, cols, v);
  W* d = static_cast<W*>(dst) + (size_t)p * S::NW * g.nx + x;
#pragma unroll
  for (int q = 0; q < S::NW; ++q) d[q * g.nx] = v[q];
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

template <typename S>
__global__ void __launch_bounds__(256) init_kernel(const typename S::math* __restrict__ rhoN0, void* dstv, Geom g,
                                                   Coef<typename S::math> c, typename S::math rho0R,
                                                   typename S::math rho0B) {
  using T = typename S::math;
  using W = typename S::W;
  W* dst = static_cast<W*>(dstv);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= g.nx) return;
  const bool solid = g.walls && (y == 0 || y == g.ny - 1);
  W w[S::NW];
  if (solid) {
#pragma unroll
    for (int q = 0; q < S::NW; ++q) w[q] = W(0);
  } else {
    // value stored for link i at r: the rest population of link i at r + c_i
    // (pull layout), or of link opp(i) at r itself when r + c_i is solid
    T R[9], B[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      int yd = y + link_cy(i);
      int xd = x + link_cx(i);
      xd = xd < 0 ? xd + g.nx : (xd >= g.nx ? xd - g.nx : xd);
      if (g.walls && (yd == 0 || yd == g.ny - 1)) {
        rest_state(rhoN0, c, rho0R, rho0B, y * g.nx + x, link_opp(i), R[i], B[i]);
      } else {
        yd = yd < 0 ? yd + g.ny : (yd >= g.ny ? yd - g.ny : yd);
        rest_state(rhoN0, c, rho0R, rho0B, yd * g.nx + xd, i, R[i], B[i]);
      }
    }
    encode<S>(R, B, c, w);
  }
#pragma unroll
  for (int q = 0; q < S::NW; ++q) dst[((size_t)y * S::NW + q) * g.nx + x] = w[q];
}

// ---------------------------------------------------------------------------
// per-colour masses in FP64: block partials, then one ordered pass
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename S>
__global__ void __launch_bounds__(256) mass_partial_kernel(const void* popsv, Geom g, Coef<typename S::math> c,
                                                           double* partial) {
  using T = typename S::math;
  const typename S::W* pops = static_cast<const typename S::W*>(popsv);
  const int row0 = g.walls ? 1 : 0;
  const long long nsite = (long long)g.F * g.nx;
  double sr = 0.0, sb = 0.0;
  for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < nsite;
       s += (long long)gridDim.x * blockDim.x) {
    const int y = row0 + (int)(s / g.nx), x = (int)(s % g.nx);
    const typename S::W* r = pops + (size_t)y * S::NW * g.nx + x;
    typename S::W w[S::NW];
#pragma unroll
    for (int q = 0; q < S::NW; ++q) w[q] = r[q * g.nx];
    T R[9], B[9];
    decode<S>(w, c, R, B);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      sr += (double)R[i];
      sb += (double)B[i];
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

static __global__ void __launch_bounds__(256) mass_final_kernel(const double* partial, int nblocks, double* out) {
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
