/*
 * chromo_lbm.h -- C ABI of the MI355X (gfx950) chromodynamic MRT lattice
 * Boltzmann step.
 *
 * The method is the two-colour, density-contrast, Dellar-type MRT scheme of
 * Spendlove, Xu, Halliday, Schenkel and Halliday, "Chromodynamic multi-relaxation
 * time lattice Boltzmann scheme for fluids with density difference"
 * (arXiv 2005.04642):
 *   - red/blue populations R_i, B_i on a D2Q9 lattice (Sec. II);
 *   - colour index rho^N and its App. B gradient; Brackbill curvature
 *     K = div n and Lishchuk force G = sigma K grad(rho^N) / 2 with Guo's
 *     velocity u = (sum f c + G/2)/rho (Sec. II);
 *   - modal relaxation with density-difference sources and explicit
 *     reconstruction f+ = M^{-1} m+ (Sec. III, App. A);
 *   - d'Ortona recolour (Sec. II) and streaming with periodic x, and either
 *     periodic y or half-way bounce-back walls at rows 0 and ny-1, or solid
 *     sites anywhere given by a mask (lbm_set_solid).
 *
 * Memory: every device buffer belongs to the caller.  The library keeps only a
 * small host-side handle (pointers, parameters, step counter, which of the two
 * population buffers is live).  Nothing here allocates device memory.
 *
 * Populations: two buffers of lbm_pops_bytes() bytes each, holding NW words
 * per site, laid out [ny][NW][nx] (x fastest): each lattice row is NW
 * consecutive runs of nx words, word q of site (x, y) at index
 * (y NW + q) nx + x.  The live buffer holds, for
 * every site r and link i, the post-recolour populations of the previous step
 * at their source site (a "pull" layout): the pre-collision population of the
 * current step is C_i(r) = buf_i(r - c_i), or buf_opp(i)(r) when r - c_i is a
 * solid row.  Link order: c0=(0,0) c1=(1,1) c2=(0,1) c3=(-1,1) c4=(-1,0)
 * c5=(-1,-1) c6=(0,-1) c7=(1,-1) c8=(1,0) (odd links are the diagonal ones,
 * opp(i) = i +- 4).  Storage formats:
 *   LBM_STORAGE_F64 / _F32: NW = 18 words of double / float, word 9 c + i =
 *     population of colour c (0 red, 1 blue) on link i.
 *   LBM_STORAGE_F16_OFS / _BF16_OFS (16-bit offsets, FP32 arithmetic): NW = 10
 *     words of 4 bytes.  Word 0 = R_0, word 1 = B_0 (float).  Word 1 + i
 *     (i = 1..8) packs link i of both colours: bits 0-15 =
 *     1024 (f_i - fref_i) / fref_i in FP16 (F16_OFS) or BF16 (BF16_OFS),
 *     f_i = R_i + B_i, fref_i = (9/5) w_i rho0_R (1 - alpha_R) (the rest value
 *     of f_i, equal in both pure phases by the density-ratio relation of
 *     Sec. II); bits 16-31 = the one of R_i, B_i of smaller magnitude,
 *     divided by 4 fref_i, as FP16 clamped to |.| < 2, with bit 14 (always
 *     clear in such an FP16 value) set when that colour is blue; the other
 *     colour is f_i minus it.  Values are rounded to nearest even.  40 bytes
 *     per site instead of 72 (F32).
 * rhoN0, force and the field outputs use the arithmetic type: double for
 * LBM_STORAGE_F64, float for every other format.
 *
 * Streams: every call only enqueues work on the given stream, except those
 * whose comments say they wait for it: lbm_masses_host, and the batch calls
 * that copy host tables to the device (lbm_batch_init, lbm_batch_autotune,
 * lbm_batch_set_force, lbm_batch_set_solid) or read results back
 * (lbm_batch_masses_host).
 *
 * Errors: every entry point returns an lbm_status value; on failure
 * lbm_last_error() gives a message (thread-local).  Handles are not thread-safe.
 */
#ifndef CHROMO_LBM_H
#define CHROMO_LBM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* bad sizes, NULL pointers or inconsistent parameters */
  LBM_EHIP = -2,        /* a HIP runtime call or kernel launch failed */
  LBM_ENOTIMPL = -3,    /* entry point or option not provided by this library */
  LBM_ENONFINITE = -4   /* a per-colour mass is not finite */
} lbm_status;

enum {
  LBM_STORAGE_F64 = 0,      /* populations and arithmetic in double */
  LBM_STORAGE_F32 = 1,      /* populations and arithmetic in float */
  LBM_STORAGE_F16_OFS = 2,  /* 16-bit FP16 offset words (see above), arithmetic in float */
  LBM_STORAGE_BF16_OFS = 3  /* as F16_OFS with the f_i offset in BF16 */
};

enum {
  LBM_FLAG_STREAM_ONLY = 1, /* lbm_step only streams: buf'_i(r) = f_i(r) (no collision) */
  LBM_FLAG_FIXED_K = 2,     /* curvature K := K_fixed instead of div n (Sec. IV, fixed K) */
  LBM_FLAG_NO_RECOLOR = 4,  /* skip the segregation term of the recolour (proportional split) */
  LBM_FLAG_MASK_PASSES = 8  /* with a solid-site mask: always step with the four-pass kernels */
};

/* Parameters of one lattice (Sec. II, App. A).  Units are lattice units
 * (delta_t = 1, |c_i| = 1 or sqrt 2). */
typedef struct lbm_params {
  int32_t nx, ny;       /* lattice size; x is always periodic */
  int32_t walls_y;      /* 0: y periodic; 1: rows 0 and ny-1 are solid (half-way bounce-back) */
  int32_t storage;      /* LBM_STORAGE_* */
  int32_t stencil[4];   /* App. B stencil radius (1 or 3) for grad rho^N, div n, grad Phi', div u */
  int32_t ghost_eq;     /* 0: N^(0) = h^(6).f^(0) (projected); 1: N^(0) = 0 (App. A, modal eqs.) */
  int32_t flags;        /* LBM_FLAG_* */
  double rho0_R, rho0_B;   /* bulk densities; Lambda = rho0_R / rho0_B (Sec. II) */
  double alpha_R, alpha_B; /* rest fractions; must satisfy (1-alpha_B) = Lambda (1-alpha_R) */
  double nu_R, nu_B;       /* kinematic viscosity of each bulk phase; nu(rho^N) linear in between */
  double sigma;            /* interfacial tension */
  double beta;             /* segregation parameter of the recolour */
  double lambda6, lambda7; /* ghost-mode relaxation rates (App. A), each in (0, 2) */
  double gx, gy;           /* uniform body-force density added to G */
  double K_fixed;          /* curvature used with LBM_FLAG_FIXED_K */
  double eps_n;            /* |grad rho^N| regularisation: n = grad/sqrt(|grad|^2 + eps_n^2) */
} lbm_params;

typedef struct lbm_handle lbm_handle;

/* Host-only check of a parameter set (no GPU call).  LBM_OK or LBM_EINVAL.
 * Rejects: nx, ny < 1; walls with fewer than 1 fluid row; unknown storage;
 * one lattice row of a population buffer of 4 GiB or more (the whole buffer may
 * be larger: the kernels address it row by row); more than 2^30 sites; more
 * than 65535 rows; a stencil radius not in {1, 3}; non-positive densities;
 * |(1-alpha_B) - Lambda (1-alpha_R)| > 1e-9 (1-alpha_B) (Sec. II density-ratio
 * relation); alpha outside [0, 1); nu <= 0 (lambda_3 = 2/(6 nu + 1) must lie in
 * (0, 2)); lambda6, lambda7 outside (0, 2); eps_n <= 0. */
int lbm_validate_params(const lbm_params* p);

/* Words of one population buffer: NW * nx * ny (NW = 18 for F64/F32, 10 for
 * the 16-bit offset formats); 0 for an empty lattice or unknown storage. */
size_t lbm_pops_elems(const lbm_params* p);

/* Bytes of one population buffer: lbm_pops_elems() times the word size (8 for
 * F64, 4 otherwise). */
size_t lbm_pops_bytes(const lbm_params* p);

/* Bytes of device workspace lbm_init needs (per-block FP64 partial sums of the
 * mass reduction).  0 on invalid parameters. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a handle and write the initial populations into pops_a (Sec. II
 * equilibrium at rest): rho_R = rho0_R (1 + rho^N)/2, rho_B = rho0_B (1 - rho^N)/2,
 * C_i = rho_C phi_i.  rhoN0: device [ny][nx] array of the arithmetic type,
 * values in [-1, 1] (solid rows ignored).  force: NULL or device [2][ny][nx]
 * per-site body force density (x then y component, arithmetic type) added to G
 * every step; it must stay valid and unchanged while the handle is used.
 * pops_a, pops_b: device buffers of lbm_pops_bytes() bytes, aligned to the word
 * size, not overlapping.  workspace: device memory of at
 * least lbm_workspace_bytes() bytes, 256-byte aligned.  The handle is written
 * to *out; free it with lbm_destroy.  Enqueued on `stream`. */
int lbm_init(const lbm_params* p, const void* rhoN0, const void* force,
             void* pops_a, void* pops_b, void* workspace, size_t ws_bytes,
             hipStream_t stream, lbm_handle** out);

/* Advance nsteps >= 0 time steps (the whole path: fields, stencils, force,
 * collision, recolour, streaming), swapping the two buffers each step.  If
 * mass_RB_dev is not NULL, the FP64 per-colour masses (sum of all red and all
 * blue populations over fluid sites, exact invariants of the scheme) after the
 * last step are written there (2 doubles, device).  Enqueued on `stream`. */
int lbm_step(lbm_handle* h, int32_t nsteps, double* mass_RB_dev, hipStream_t stream);

/* lbm_step for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same steps, and the same FP64 masses bit for bit, but the mass reduction's
 * per-block partial sums go to a static device array of the library (512
 * pairs of doubles, 8 KiB, one copy per GPU, resolved by lbm_init for its
 * device) instead of the handle's workspace.  The call allocates nothing and
 * calls no allocating routine.  The array is shared by every call on the same
 * GPU and keeps the last call's contents; nothing in it needs to start at
 * zero (each partial is written before it is read), but calls that overlap in
 * time on one GPU (different streams or threads) race on it.  Every lattice
 * lbm_validate_params accepts fits: the reduction uses 512 partial pairs at
 * any size.  Errors as lbm_step (LBM_EINVAL for a NULL handle or nsteps < 0). */
int lbm_step_static(lbm_handle* h, int32_t nsteps, double* mass_RB_dev, hipStream_t stream);

/* Advance nsteps >= 0 steps from the state in `from` (a population buffer of
 * the handle's format), writing the state after step j into states[j] (host
 * array of nsteps device buffers of lbm_pops_bytes(), each distinct from its
 * source): a trajectory kept whole, as the checkpointed adjoint recomputes
 * it, in one call.  The handle then steps on from states[nsteps-1] (as after
 * lbm_set_pops), with states[nsteps-2] (`from` when nsteps is 1) as its other
 * buffer: the next lbm_step writes there, so re-point the handle with
 * lbm_set_pops first to keep the trajectory whole.  LBM_EINVAL for NULL arrays
 * or entries, or a state equal to its source.  Enqueued on `stream`. */
int lbm_step_into(lbm_handle* h, const void* from, int32_t nsteps, void* const* states, hipStream_t stream);

/* Macroscopic fields of the current state (Sec. II, force-adjusted
 * observables): rho, u = (sum f c + G/2)/rho, rho^N.  Each output is NULL
 * (skipped) or a device [ny][nx] array of the arithmetic type; solid rows are
 * written as NaN.  mass_RB_dev as in lbm_step.  Enqueued on `stream`. */
int lbm_fields(lbm_handle* h, void* rho, void* ux, void* uy, void* rhoN,
               double* mass_RB_dev, hipStream_t stream);

/* Synchronising helper: enqueue the mass reduction, wait for `stream`, copy the
 * two masses to host out[2].  Returns LBM_ENONFINITE if either is not finite. */
int lbm_masses_host(lbm_handle* h, double out[2], hipStream_t stream);

/* ---- adjoint (reverse-mode derivative of lbm_step) ------------------------
 * Provided for LBM_STORAGE_F64 and LBM_STORAGE_F32, periodic, walled
 * (walls_y = 1: the transposes of the wall-mirrored stencils and of the
 * bounce-back) or with a mask of solid sites (lbm_set_solid; stencil profiles
 * (3,3,3,3), (3,1,3,1) and (1,1,1,1), others LBM_ENOTIMPL); the 16-bit formats return
 * LBM_ENOTIMPL.  The words of solid rows and sites carry no state: their
 * adjoints are written as 0.  Adjoint buffers have the
 * layout of an F64/F32 population buffer ([ny][colour 2][link 9][nx], the
 * arithmetic type), aligned with the pull layout: adj[C][i](s) is dL/d of the
 * stored word buf[C][i](s).  The step that is differentiated is the one
 * lbm_step performs with the handle's parameters and force field. */

/* Bytes of device workspace lbm_adjoint_step needs (256-byte aligned): the
 * saved intermediates and adjoint fields (39 planes of nx*ny values of the
 * arithmetic type, interleaved by rows: [ny][39][nx]) and the FP64 partial
 * sums of dL/dsigma.  0 if the adjoint is not provided for these parameters
 * (every lattice lbm_validate_params accepts, up to 2^30 sites: 167 GB of
 * workspace in FP32 at that size). */
size_t lbm_adjoint_workspace_bytes(const lbm_params* p);

/* One step backwards.  pops_t: the state the step starts from (a population
 * buffer in the handle's storage format).  adj_next: dL/d(state after the
 * step).  adj_out: receives dL/d(pops_t) (overwritten; must differ from
 * adj_next).  dL_dsigma_dev: NULL or one device double to which dL/dsigma of
 * this step is added (FP64 reduction).  dL_dforce_dev: NULL or a device
 * [2][ny][nx] array (arithmetic type) to which dL/dG_ext of this step is added,
 * G_ext being the per-site force density of lbm_init (the derivative exists
 * whether or not a force field was given).  Enqueued on `stream`. */
int lbm_adjoint_step(lbm_handle* h, const void* pops_t, const void* adj_next, void* adj_out, void* workspace,
                     size_t ws_bytes, double* dL_dsigma_dev, void* dL_dforce_dev, hipStream_t stream);

/* nsteps >= 0 steps backwards through a trajectory in one call: the adjoint
 * of the step from states[nsteps-1], then from states[nsteps-2], ... down to
 * states[0] (states: host array of nsteps device population buffers).  adj_a
 * holds dL/d(state after the step from states[nsteps-1]) on entry; the steps
 * alternate between adj_a and adj_b (a -> b -> a ...), so dL/d(states[0])
 * ends in adj_a if nsteps is even and in adj_b if it is odd.  dL/dsigma and
 * dL/dG_ext of every step are added as in lbm_adjoint_step.  The same kernels
 * in the same order as nsteps lbm_adjoint_step calls, without a host call per
 * step (on small lattices the host's per-step calls otherwise cost about as
 * much as the GPU's work).  Enqueued on `stream`. */
int lbm_adjoint_steps(lbm_handle* h, int32_t nsteps, const void* const* states, void* adj_a, void* adj_b,
                      void* workspace, size_t ws_bytes, double* dL_dsigma_dev, void* dL_dforce_dev,
                      hipStream_t stream);

/* Adjoint of the colour index that lbm_fields reports for the state pops:
 * adj_out (overwritten) = dL/dpops given dL_drhoN, a device [ny][nx] array
 * (arithmetic type).  Starts the backward pass of a loss on rho^N. */
int lbm_rhoN_adjoint(lbm_handle* h, const void* pops, const void* dL_drhoN, void* adj_out, hipStream_t stream);

/* Adjoint of lbm_init's rest state: adds to dL_drhoN0 (device [ny][nx],
 * arithmetic type) the derivative of the loss with respect to the initial
 * colour index rhoN0, given adj_pops0 = dL/d(initial populations). */
int lbm_init_adjoint(lbm_handle* h, const void* rhoN0, const void* adj_pops0, void* dL_drhoN0, hipStream_t stream);

/* ---- batches: many independent lattices, one launch per step ---------------
 * All lattices of a batch share the storage format and the stencil radii; each
 * has its own size and physical parameters (lbm_params) and, optionally, its
 * own per-site force field (lbm_batch_set_force).  A batch is all periodic or
 * all walled (walls_y; walled batches are built for the stencil profiles
 * (3,3,3,3), (3,1,3,1) and (1,1,1,1), LBM_ENOTIMPL for the others); lattices of a
 * periodic batch may have solid-site masks (lbm_batch_set_solid; same three
 * profiles).  Their population buffers are packed one after the other (each
 * at a 256-byte aligned offset, lbm_batch_offsets) in two caller-owned buffers
 * of lbm_batch_pops_bytes() bytes.  Every lbm_batch_step is one launch of a
 * persistent-style kernel: each workgroup owns a bin of (lattice, tile) work
 * items, planned on the host so that the bins' costs (march iterations) are
 * balanced (longest processing time first).  The tile shape (workgroup width
 * and chunk height) comes from a table of candidates; lbm_batch_autotune times
 * them on the batch itself and keeps the fastest.  Each lattice evolves exactly
 * as it would alone under lbm_step. */
typedef struct lbm_batch lbm_batch;

/* Bytes of each packed population buffer of the batch p[0..nsim-1]; 0 on
 * invalid input. */
size_t lbm_batch_pops_bytes(const lbm_params* p, int nsim);

/* Byte offset of every lattice's buffer inside a packed buffer (offsets[nsim]). */
int lbm_batch_offsets(const lbm_params* p, int nsim, size_t* offsets);

/* Bytes of device workspace of a batch (work-list tables, mass partials). */
size_t lbm_batch_workspace_bytes(const lbm_params* p, int nsim);

/* Create a batch and write every lattice's rest state (as lbm_init) into
 * pops_a.  rhoN0[k]: device [ny_k][nx_k] colour index of lattice k (arithmetic
 * type).  pops_a, pops_b: device, 256-byte aligned, lbm_batch_pops_bytes()
 * each.  Copies the initial work list to the workspace and waits for that
 * copy. */
int lbm_batch_init(const lbm_params* p, int nsim, const void* const* rhoN0, void* pops_a, void* pops_b,
                   void* workspace, size_t ws_bytes, hipStream_t stream, lbm_batch** out);

/* Advance every lattice by nsteps steps (one launch per step). */
int lbm_batch_step(lbm_batch* b, int32_t nsteps, hipStream_t stream);

/* Time every candidate tile shape for steps_per_trial steps on the batch's
 * current state, keep the fastest, and restore the state (the step count is
 * unchanged).  scratch: device memory of lbm_batch_pops_bytes() bytes.
 * chosen (NULL or int32[2]) receives the workgroup width and chunk-height cap.
 * Synchronises the stream. */
int lbm_batch_autotune(lbm_batch* b, void* scratch, size_t scratch_bytes, int32_t steps_per_trial,
                       hipStream_t stream, int32_t* chosen);

/* Give lattice k a per-site force density G_ext (device [2][ny_k][nx_k],
 * arithmetic type, as in lbm_init; caller-owned, kept valid while the batch
 * steps), or remove it (NULL).  Updates the lattice's entry of the batch's
 * device table and waits for that copy on `stream`.  LBM_EINVAL for a bad
 * batch or index. */
int lbm_batch_set_force(lbm_batch* b, int32_t k, const void* force, hipStream_t stream);

/* Give lattice k of a periodic batch a mask of solid sites, as lbm_set_solid
 * does for a single lattice (same mask and workspace contract, workspace of
 * lbm_solid_workspace_bytes(&p[k]) bytes); from then on the batch steps with
 * the kernel's mask variant (lattices without a mask are unaffected) and
 * lbm_batch_fields reads NaN at lattice k's solid sites.  Waits for the
 * update of the batch table on `stream`.  LBM_EINVAL for a bad index, NULL
 * pointers, a small workspace, a walled batch or a lattice that has a mask;
 * LBM_ENOTIMPL for stencil profiles other than 3333, 3131 and 1111. */
int lbm_batch_set_solid(lbm_batch* b, int32_t k, const uint8_t* solid_dev, void* workspace, size_t ws_bytes,
                        hipStream_t stream);

/* info[5]: workgroup width, chunk-height cap, number of bins, number of work
 * items, largest bin cost in march iterations. */
int lbm_batch_plan_info(const lbm_batch* b, int32_t* info);

/* Fields (as lbm_fields) and per-colour masses (as lbm_masses_host) of lattice k. */
int lbm_batch_fields(lbm_batch* b, int32_t k, void* rho, void* ux, void* uy, void* rhoN, hipStream_t stream);
int lbm_batch_masses_host(lbm_batch* b, int32_t k, double out[2], hipStream_t stream);

/* 0 if pops_a holds the live states, 1 if pops_b does; steps taken. */
int lbm_batch_current_pops(const lbm_batch* b);
int64_t lbm_batch_step_count(const lbm_batch* b);

/* Free the host object (device buffers stay with the caller). */
void lbm_batch_destroy(lbm_batch* b);

/* ---- solid sites anywhere (a mask) -----------------------------------------
 * For obstacles that are not whole rows, such as the staircase circular
 * no-slip wall of the curved-interface transient (Sec. IV, dynamics of curved
 * interfaces; App. D).  Provided for every storage format on a handle with
 * walls_y = 0 (put wall rows in the mask instead); both x and y
 * are periodic around the mask.  A link whose target is solid is bounced back
 * half-way (as at the walls); an App. B stencil tap that falls on a solid site
 * reads the field's value at the stencil's centre (a zero-gradient
 * continuation of every field into the solid; the paper gives no rule for
 * stencils at a curved wall).  Solid sites hold zero populations (all-zero
 * words in F64/F32, the offset encoding of zero in the 16-bit formats), carry
 * no mass, and read as NaN from lbm_fields.  For the stencil profiles
 * (3,3,3,3), (3,1,3,1) and (1,1,1,1) the step is one launch of the fused step kernel in
 * its mask variant (per-site bounce bits, NaN markers for stencil taps); for
 * the other profiles, or with LBM_FLAG_MASK_PASSES, four launches over
 * per-site field planes.  Both give the same results bit for bit. */

/* Bytes of device workspace lbm_set_solid needs: 14 planes of nx*ny values of
 * the arithmetic type and nx*ny bytes of bounce bits (256-byte multiple); 0
 * where masks are not provided, which includes population buffers of 4 GiB or
 * more (the masked gather addresses the whole buffer through one 32-bit
 * offset; lbm_set_solid and lbm_batch_set_solid return LBM_EINVAL there). */
size_t lbm_solid_workspace_bytes(const lbm_params* p);

/* Give the handle a mask of solid sites.  solid_dev: device [ny][nx] bytes,
 * nonzero = solid; workspace: device, 256-byte aligned, at least
 * lbm_solid_workspace_bytes() bytes.  Both stay owned by the caller and must
 * stay valid and unchanged for as long as the handle steps.  Re-encodes the
 * live population buffer in place so that every fluid site keeps the
 * pre-collision populations it had (the words its links now bounce into take
 * the values those links pulled before), and zeroes the words of solid sites;
 * call it on the state to start from (usually right after lbm_init).  From
 * then on lbm_step and lbm_fields use the mask.  Every state the handle
 * steps from (lbm_set_pops buffers, lbm_adjoint_step's pops_t) must hold zero
 * populations at solid sites, as the re-encoded buffer and every step's output do:
 * the fused kernel recognises solid sites by their zero mass.  A handle takes one mask:
 * LBM_EINVAL if it has one already, for NULL pointers, a small workspace,
 * walls_y = 1 or nx, ny < 4; LBM_ENOTIMPL for the streaming-only mode.  The adjoint entry points work on such a handle for
 * the stencil profiles (3,3,3,3), (3,1,3,1) and (1,1,1,1) (LBM_ENOTIMPL for the others);
 * lbm_init_adjoint then differentiates the rest state as lbm_set_solid
 * re-encoded it. */
int lbm_set_solid(lbm_handle* h, const uint8_t* solid_dev, void* workspace, size_t ws_bytes, hipStream_t stream);

/* 0 if pops_a holds the live state, 1 if pops_b does. */
int lbm_current_pops(const lbm_handle* h);

/* Re-point the handle at two other caller-owned population buffers (host-side
 * only, nothing is copied or enqueued): `live` must hold a state in the
 * handle's storage format and layout (it becomes the live buffer, in the slot
 * lbm_current_pops reports), `next` receives the next lbm_step (each step still
 * alternates between the two).  Lets a caller run a trajectory straight into
 * its own array of states, as the checkpointed adjoint's recompute does.  Both
 * must be lbm_pops_bytes() long and distinct; LBM_EINVAL for NULL or equal
 * pointers.  Work already enqueued keeps the buffers it was given. */
int lbm_set_pops(lbm_handle* h, void* live, void* next);

/* Steps taken since lbm_init. */
int64_t lbm_step_count(const lbm_handle* h);

/* ---- sharing the GPU between two streams of work --------------------------
 * For callers that run independent work side by side on one GPU (the
 * checkpointed adjoint recomputes the next segment's states while it runs the
 * current segment's adjoint steps).  On small lattices a step keeps few CUs
 * busy for long (each tile's march starts with a fixed pipeline fill), so two
 * streams confined to disjoint sets of CUs overlap where two unconfined ones
 * would queue one kernel behind the other. */

/* Plan the tiles of the forward step (lbm_step, lbm_fields) for ncu_step CUs
 * and those of the adjoint's first pass for ncu_adjoint CUs instead of the
 * whole device (0: the whole device; larger values are clamped to it).
 * Results do not depend on the plan (every site takes the same arithmetic).
 * Host-side only; applies to launches made after the call.  LBM_EINVAL for a
 * NULL handle or a negative count. */
int lbm_set_cu_budget(lbm_handle* h, int32_t ncu_step, int32_t ncu_adjoint);

/* Create a HIP stream whose kernels run only on CUs [cu_first, cu_first +
 * cu_count) of the current device, in the runtime's CU numbering (round-robin
 * over the 8 XCDs: both bounds must be multiples of 8, so every XCD gets
 * cu_count / 8 CUs; multiples of 32 also keep the CUs of each XCD evenly
 * spread, and run markedly faster than other splits).  Default priority.
 * The caller owns the stream
 * (hipStreamDestroy).  LBM_EINVAL for a bad range or NULL out, LBM_EHIP if the
 * runtime refuses the mask. */
int lbm_partition_stream(int32_t cu_first, int32_t cu_count, hipStream_t* out);

/* Free the host handle (device buffers stay with the caller). */
void lbm_destroy(lbm_handle* h);

/* Message of the last failure on this thread ("" if none). */
const char* lbm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHROMO_LBM_H */
