/*
 * lt.h - C ABI of the MI355X (gfx950) constant-memory differentiable light
 * tracer.  Plain C types only: pointers are host or device as stated, sizes
 * are element or byte counts as stated.
 *
 * Paper: "Constant-Memory Differentiable Light Tracing" (Beresna, Fiume).
 * The forward pass is the light-tracing estimator of Sec. 3.1 (Eq. 1-2):
 * light paths start on the emitter, and at every non-specular vertex
 * x_i (i >= 1) a sensor connection L_i = W_e f_i G V is splatted through a
 * reconstruction filter at film position u_i (Eq. 20).  Three reverse modes
 * compute the gradient of a loss whose image adjoint dL/dI the caller
 * supplies (Sec. 3.2, Sec. 4.3.1 "Pass 1"):
 *   - naive reverse-mode AD over a per-vertex tape (memory linear in depth);
 *   - ResLRB: seed replay to the reservoir-selected connection
 *     (Sec. 4.2, Eq. 8-13);
 *   - LRB-3-pass: accumulate then consume downstream adjoints in two replays
 *     (Sec. 4.3, Eq. 14-19).
 * Attached variants also differentiate vertex positions and splat
 * positions through per-segment ray Jacobians (Sec. 3.3, Eq. 4-7; Sec. 4.4,
 * Eq. 21).
 *
 * Conventions shared by every call:
 *   - The caller owns every buffer passed in (images, adjoints, parameters,
 *     gradients, side state).  The library owns only its copy of the scene,
 *     the BVH and a small workspace.  No pointer is retained after the call
 *     returns.
 *   - Calls are ordered on the context's HIP stream and asynchronous:
 *     LT_OK means the work is enqueued.  A device fault surfaces as
 *     LT_ERR_HIP from a later call that synchronizes.
 *   - Arguments are validated before anything is enqueued; a rejected call
 *     writes nothing and lt_last_error() says why.
 *   - Randomness is counter-based (Philox-4x32-10 keyed by the seed,
 *     counter = (path, vertex, block)), so the same (seed, n_paths,
 *     max_depth, flags, params) gives the same paths and decisions on every
 *     call; only the order of floating-point atomic sums may differ.
 *   - A context (and a batch runner) is used by one host thread at a time:
 *     calls on the same handle must not overlap.  Distinct contexts may be
 *     driven concurrently; each has its own stream, workspace and scene.
 *   - No exception crosses this boundary.
 */
#ifndef LT_H
#define LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LT_OK = 0,
  LT_ERR_ARG = 1,         /* invalid argument; nothing enqueued */
  LT_ERR_OOM = 2,         /* allocation failed or the memory cap was exceeded */
  LT_ERR_HIP = 3,         /* a HIP runtime call failed */
  LT_ERR_STATE = 4,       /* call out of order (e.g. no scene uploaded) */
  LT_ERR_UNSUPPORTED = 5  /* flag combination not implemented */
} lt_status;

/* material types (lt_scene_desc.mat_type) */
enum { LT_MAT_ABSORBER = 0, LT_MAT_LAMBERT = 1, LT_MAT_DIELECTRIC = 2, LT_MAT_CONDUCTOR = 3 };
/* emitter types (lt_scene_desc.em_type): an area quad with cosine-weighted
 * emission, an isotropic point, or a directional quad (a collimated beam
 * leaving the quad along its normal, as the directional emitter of the
 * paper's Tumbler scene, Sec. 6.1) */
enum { LT_EMIT_QUAD = 0, LT_EMIT_POINT = 1, LT_EMIT_DIRECTIONAL = 2 };

/* lt_trace_args.flags */
enum {
  LT_ATTACHED = 1u,         /* differentiate geometry (heightfield heights), Sec. 3.3: a
                               dielectric or rough-conductor heightfield (a Lambertian
                               heightfield is rejected, LT_ERR_UNSUPPORTED) */
  LT_SPLAT_SELECTED = 2u,   /* primal image splats only (Omega_k/w_R) L_R (Eq. 9) */
  LT_RECORD_TAPE = 4u,      /* lt_trace writes the naive-AD tape */
  LT_RECORD_RESERVOIR = 8u, /* lt_trace writes the per-path ResLRB record */
  LT_CONTRIB_ADJOINT = 16u, /* attached backward: path_contrib gets |delta_total| (below) */
  LT_RECORD_SPLATS = 32u,   /* lt_trace writes the buffered two-pass splat records (detached) */
  LT_GUIDE_DIFFUSE = 64u,   /* with params->guide_w: Lambertian vertices scatter from the
                               learned guide too (diffuse guide table, see the guide section) */
  LT_CAMERA_ALL = 128u      /* camera side (lt_camera_trace, lt_camera_backward_prb): every
                               camera sample, not only those whose first vertex is specular */
};

typedef struct lt_ctx lt_ctx;

/* Scene description: HOST arrays, copied by lt_scene_upload.
 *  tri_v  [n_tris][3][3]  static triangle vertices (world space)
 *  tri_uv [n_tris][3][2]  per-vertex texture coordinates in [0,1]
 *  tri_mat[n_tris]        material index in [0, n_mats)
 *  mat_type/mat_tex/mat_ior [n_mats]: type, texture index (Lambertian: its
 *                         albedo; rough conductor: its reflectance F0), and
 *                         refractive index (dielectric) or GGX roughness in
 *                         [1e-3, 1] (conductor).  The rough conductor (the
 *                         roughened mirror of the attached validation, Sec. 6.1):
 *                         f = F0 D(h) G1(wi) G1(wo) / (4 (wi.n)(wo.n)) with GGX D,
 *                         Smith's separable G1 and n the shading normal (on the
 *                         heightfield the blended slopes, as for glass); its
 *                         vertices connect to the sensor, and scatter by
 *                         reflecting about a microfacet normal drawn with density
 *                         D(m)(m.n) from the vertex's first two uniforms, weight
 *                         F0 G1(wi) G1(wo) (wi.m) / ((wi.n)(m.n)).  Attached
 *                         passes hold the microfacet normal in the local frame of
 *                         the shading normal; the weight and the connection then
 *                         carry derivatives w.r.t. the heights (attached batches
 *                         reject conductor scenes).
 *  n_tex, tex_res         albedo parameters are [n_tex][tex_res][tex_res][3]
 *  emitter: quad (o, e1, e2; one-sided, normal normalize(e1 x e2)), point (o) or
 *          directional quad (o, e1, e2; the beam leaves along the normal, radiance
 *          = irradiance across the quad, beta_1 = L_e * area); em_tex_res > 0 (quad
 *          and directional): L_e is an em_tex_res^2 RGB texture over the quad, the
 *          emission point's texel (floor(u0 R), floor(u1 R)) of its quad coordinates
 *          u0 along e1, u1 along e2; 0: one RGB radiance
 *  camera: pinhole at cam_pos looking at cam_target, vertical FOV, film
 *          width x height pixels; image row 0 is the top row
 *  heightfield (hf_G >= 2, else none): vertex (i, j) at
 *          (hf_x0 + i dx, hf_base + h[j*G + i], hf_z0 + j dx), material hf_mat;
 *          cell (i, j) is split into triangles (A, C, B) and (A, D, C) with
 *          A=(i,j) B=(i+1,j) C=(i+1,j+1) D=(i,j+1). */
typedef struct {
  int32_t n_tris;
  const double* tri_v;
  const double* tri_uv;
  const int32_t* tri_mat;
  int32_t n_mats;
  const int32_t* mat_type;
  const int32_t* mat_tex;
  const double* mat_ior;
  int32_t n_tex, tex_res;
  int32_t em_type;
  double em_o[3], em_e1[3], em_e2[3];
  double cam_pos[3], cam_target[3], cam_up[3], cam_fov_deg;
  int32_t width, height;
  int32_t hf_G;
  double hf_x0, hf_z0, hf_dx, hf_base;
  int32_t hf_mat;
  int32_t em_tex_res;   /* 0 or the emitter texture's side (see emitter above) */
} lt_scene_desc;

/* Per-call trace arguments. */
typedef struct {
  uint64_t seed;            /* Philox key */
  int64_t n_paths;          /* N light paths, 1 <= N < 2^31; also the 1/N of the estimator */
  int32_t max_depth;        /* D: at most D scattering vertices x_1..x_D, 1 <= D <= 64 */
  uint32_t flags;           /* LT_* flags above */
  const uint8_t* path_mask; /* DEVICE [n_paths] or NULL: paths whose byte is 0
                               contribute nothing (forward and backward) */
  uint32_t* path_sig;       /* DEVICE [n_paths] or NULL: lt_trace writes each path's
                               decision signature (FNV-1a of hit primitive, texel,
                               connection validity, lobe and R) */
  uint32_t* path_info;      /* DEVICE [n_paths] or NULL: the attached passes write
                               per-path flags - bit 0: the determinant guard zeroed a
                               projected adjoint on this path (it then zeroes every later
                               one: the later accumulated Jacobians are singular too);
                               bit 1: the path has an
                               ill-conditioned vertex (grazing hit, |cos| < 0.02;
                               refraction with cos_t < 0.1; or a segment shorter than
                               0.02 scene units) whose FP32 derivatives carry rounding
                               amplified by 1/cos^2 or 1/length, or a connection
                               within 1e-3 px of a kink of the tent filter (Eq. 20),
                               where the splat-position derivative is one-sided */
  float* path_contrib;      /* DEVICE [n_paths] or NULL: a per-path training signal S
                               for the emission guide.  lt_trace writes the path's
                               image contribution sum_i lum(C_i) over its connections
                               (Rec. 709 luminance, the reservoir weight of Eq. 8);
                               lt_backward_lrb3 and lt_backward_naive write the
                               path's adjoint-weighted contribution
                               sum_c |delta_total,c| (Eq. 14) - detached, or attached
                               with LT_CONTRIB_ADJOINT - else, attached, the L1 norm
                               of its heights-gradient contributions */
} lt_trace_args;

/* Parameters: DEVICE float arrays owned by the caller. */
typedef struct {
  const float* albedo;    /* [n_tex][tex_res][tex_res][3] */
  const float* emitter_L; /* [3] radiance (quad, directional) or intensity (point), or
                             [em_tex_res][em_tex_res][3] for a textured emitter (detached
                             passes only: LT_ATTACHED rejects a textured emitter) */
  const float* heights;   /* [G][G] heightfield offsets, or NULL when hf_G < 2 */
  const float* guide_w;   /* [LT_GUIDE_NPARAMS] emission-guide weights, or NULL for
                             cosine-weighted emission (see the guide section) */
  const float* normal_map; /* [G][G][2] or NULL: a normal map on the heightfield (the
                             normal-mapped dielectric panel of Sec. 6.1): the shading
                             slopes (Sx, Sz) at each grid vertex, blended
                             barycentrically, shading normal normalize(-Sx, 1, -Sz);
                             NULL: the slopes are central differences of the heights.
                             The geometry always comes from the heights. */
} lt_params;

/* Gradients: DEVICE float arrays, same shapes as lt_params, ACCUMULATED
 * into (the caller zeroes them).  A NULL member is not written.
 * heights and normal_map are written by LT_ATTACHED backward passes. */
typedef struct {
  float* albedo;
  float* emitter_L;
  float* heights;
  float* normal_map;
} lt_grads;

/* Launch shape and strategy knobs (see lt_set_tuning). */
typedef struct {
  int32_t block;           /* threads per workgroup: 64..1024, multiple of 64 */
  int32_t blocks_per_cu;   /* persistent workgroups per compute unit, 1..64 */
  int32_t lds_grad;        /* 1 (default): each workgroup pre-reduces albedo gradients in LDS
                              when the texture set takes at most 48 KB and the copy costs
                              the kernel no resident workgroups; the detached replay
                              backwards then run the same threads per CU in workgroups of
                              block, 2 block, 4 block ... threads (at most 1024, dividing
                              blocks_per_cu), the first at which the copy fits.  The
                              detached backwards (single-instance calls) also pre-reduce a
                              textured emitter's gradients in LDS when that texture takes
                              at most 16 KB and costs no resident workgroups.  0: never
                              (waves then write-combine albedo gradients into the gradient
                              array; every path adds its emitter-texel gradient there) */
  int32_t lrb3_split;      /* how lt_backward_lrb3 runs its two replays.  Split: pass 2 and
                              pass 3 as two kernels, each connected path's state (delta_total,
                              validity bits, last connection depth; attached also A) handed
                              over in library workspace, 40 or 64 bytes per path, flat in
                              depth.  Fused: one kernel runs both passes per path, state in
                              registers.  0: fused always; 1: split always; 2 (default):
                              split for LT_ATTACHED calls, fused for detached ones */
} lt_tuning;

/* Counters from the last call that produced them. */
typedef struct {
  uint64_t guard_triggers;  /* attached: projections through singular accumulated
                               Jacobians zeroed (Sec. 5), counting the later vertices of a
                               path once the guard has fired on it */
  uint64_t nonfinite;       /* non-finite values (splats, gradient contributions) dropped
                               before they reach the image or a gradient */
} lt_stats;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  *out receives the handle.
 * Errors: LT_ERR_ARG (bad device / out == NULL), LT_ERR_HIP, LT_ERR_OOM. */
lt_status lt_create(int device, void* hip_stream, lt_ctx** out);
/* Release the context and everything the library owns. NULL is ignored. */
void lt_destroy(lt_ctx* ctx);
/* Message of the last non-OK status on this context ("" if none). */
const char* lt_last_error(const lt_ctx* ctx);
/* Switch the stream later calls enqueue on. */
lt_status lt_set_stream(lt_ctx* ctx, void* hip_stream);
/* Launch shape: NULL restores the defaults {128, 10, 1, 2} (the attached kernels
 * choose their own workgroup size, 256 or 768 threads, and take blocks_per_cu
 * only). Errors: LT_ERR_ARG. */
lt_status lt_set_tuning(lt_ctx* ctx, const lt_tuning* tuning);
lt_status lt_get_tuning(const lt_ctx* ctx, lt_tuning* out);
/* Cap, in bytes, on side state plus library workspace a call may use
 * (0 = no cap).  Calls above it fail with LT_ERR_OOM before any launch,
 * which is how the linear memory of the naive tape is shown against the
 * flat memory of the replay methods (Sec. 6.2). */
lt_status lt_set_memory_cap(lt_ctx* ctx, uint64_t bytes);
lt_status lt_get_stats(const lt_ctx* ctx, lt_stats* out);
/* Diagnostic event counts (a library built with -DLT_COUNTERS only; others
 * return LT_ERR_UNSUPPORTED).  Synchronizes the stream, copies 16 uint64
 * totals to HOST out16 - [0] closest-hit rays, [1] shadow rays, [2] BVH
 * node fetches, [3] triangle tests, [4] film splats, [5] adjoint gathers,
 * [6] gradient values scattered, [7] paths emitted, [8] tape records
 * written, [9] tape records read - and zeroes them when reset != 0.
 * They feed the algorithmic byte model of the roofline. */
lt_status lt_read_counters(lt_ctx* ctx, uint64_t* out16, int reset);

/* Upload a scene (Sec. 3.1 setting): copies the host arrays, builds a
 * binned-SAH BVH over the static triangles on the host and uploads it; rays
 * find the heightfield by walking its grid cells (each cell's two
 * triangles tested as a BVH leaf's, the same tie rule), so a call that
 * brings new heights rewrites only the heightfield's triangles and height
 * range.  Synchronizes the context's stream.  Replaces any previous scene.
 * Errors: LT_ERR_ARG (inconsistent sizes/indices), LT_ERR_OOM, LT_ERR_HIP. */
lt_status lt_scene_upload(lt_ctx* ctx, const lt_scene_desc* scene);

/* Bytes of caller-provided side state lt_trace writes for these args:
 * LT_RECORD_TAPE: the naive-AD tape, N*D records (32 bytes, 128 attached;
 * linear in depth) plus one path length per path, and with a diffuse guide
 * or rough conductors in the scene (detached) a 4-byte scatter weight per
 * record; LT_RECORD_RESERVOIR: one ResLRB record per path (Sec. 4.2.1:
 * selected depth R, weight Omega_k/w_R, u_R, reweighted splat; 32 bytes, 160
 * attached);
 * LT_RECORD_SPLATS: the buffered two-pass buffer, a 16-byte header per path
 * (last connection depth, one validity bit per vertex) and a 20-byte record
 * (u_i, C_i) for every vertex up to max_depth, preallocated (linear in
 * depth).  The flags' buffers are laid out one after the other.  0 for none. */
size_t lt_side_state_bytes(const lt_ctx* ctx, const lt_trace_args* args);
/* Library workspace bytes a call with these args may use (flat in depth):
 * the scene copy and BVH, the guide's packed weights and 16 bytes per path
 * (guided passes only), and the LRB-3 backward's per-path hand-off between
 * its two kernels when they are split (lt_tuning.lrb3_split): 40 bytes per
 * path, 64 with LT_ATTACHED. */
size_t lt_workspace_bytes(const lt_ctx* ctx, const lt_trace_args* args);

/* Light tracing forward (Eq. 1-2, Eq. 20; Sec. 4.3.1 Pass 1).
 * image: DEVICE float [height][width][3], overwritten with the estimate
 *   I[p] = sum over paths and connections of F(u_i, p) L_i, where L_i
 *   carries the per-sample normalization s = width*height/(A_film N).
 * With LT_SPLAT_SELECTED only the reservoir-selected (Omega_k/w_R) L_R is
 * splatted (Listing "ResLRB primal" of Sec. 5).
 * side/side_bytes: DEVICE buffer of at least lt_side_state_bytes(args)
 * when a RECORD flag is set (else may be NULL/0).
 * Errors: LT_ERR_ARG, LT_ERR_STATE, LT_ERR_OOM (memory cap), LT_ERR_HIP. */
lt_status lt_trace(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                   float* image, void* side, size_t side_bytes);

/* Mean-squared-error loss and image adjoint (Sec. 6.1: L2 loss):
 *   loss = sum_k (I_k - T_k)^2 / n,  d_image_k = 2 (I_k - T_k) / n.
 * image, target, d_image: DEVICE float [n]; loss: DEVICE float [1].
 * Errors: LT_ERR_ARG, LT_ERR_HIP. */
lt_status lt_loss_l2(lt_ctx* ctx, const float* image, const float* target, int64_t n,
                     float* d_image, float* loss);

/* Naive reverse-mode AD (Sec. 3.2): sweeps the tape written by lt_trace
 * with LT_RECORD_TAPE (same args and params) from the last vertex to the
 * first, applying the exact chain rule with image adjoint d_image
 * (DEVICE float [height][width][3]).  Gradients are accumulated into grads.
 * Errors: LT_ERR_ARG (tape too small / flags), LT_ERR_STATE, LT_ERR_HIP. */
lt_status lt_backward_naive(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                            const float* d_image, const void* tape, size_t tape_bytes,
                            lt_grads* grads);

/* ResLRB adjoint pass (Sec. 4.2, Eq. 11; attached Eq. 12-13): replays each
 * path from its seed up to the selected depth R read from `records`
 * (written by lt_trace with LT_RECORD_RESERVOIR, same args and params) and
 * applies the log-derivative identity weighted by dI(u_R) * S_hat.
 * Errors: as lt_backward_naive. */
lt_status lt_backward_reslrb(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                             const float* d_image, const void* records, size_t records_bytes,
                             lt_grads* grads);

/* Buffered two-pass backward (the lrb_2pass variant of Sec. 6; Sec. 4.1
 * explains why its memory stays linear in depth): delta_total = sum_i
 * dI(u_i) C_i (Eq. 14) is read back from the splat records lt_trace wrote
 * with LT_RECORD_SPLATS (same args and params), then one replay per path
 * consumes it as LRB-3's Pass 3 does (Eq. 15-17), taking u_i and C_i from the
 * records (no shadow rays, no connection geometry).  The gradient equals
 * naive AD's per path.  Detached only.
 * Errors: LT_ERR_ARG (records too small / flags), LT_ERR_UNSUPPORTED
 * (LT_ATTACHED), LT_ERR_STATE, LT_ERR_HIP. */
lt_status lt_backward_lrb2(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                           const float* d_image, const void* records, size_t records_bytes,
                           lt_grads* grads);

/* LRB-3-pass backward (Sec. 4.3): Pass 2 replays each path and accumulates
 * delta_total = sum_i dI(u_i) * L_i (Eq. 14; attached also A_pos, Eq. 18);
 * Pass 3 replays again, backpropagating the splat (Eq. 15), subtracting
 * (Eq. 16) and applying the log-derivative with delta_rem (Eq. 17;
 * attached Eq. 19).  Needs no side state.  Errors: LT_ERR_ARG,
 * LT_ERR_STATE, LT_ERR_HIP. */
lt_status lt_backward_lrb3(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                           const float* d_image, lt_grads* grads);

/* lt_backward_lrb3 for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with every piece of working
 * memory (work counters, statistics, the FP64 emitter-gradient accumulators,
 * the pass-2 -> pass-3 hand-off) in a static device array of 32 MiB that the
 * library holds on each GPU it runs on until the process ends.  The call
 * allocates nothing; the caller still passes inputs and outputs.
 * Limits: with the two-kernel form (lt_tuning.lrb3_split) n_paths is at most
 * 524,216 attached (64-byte hand-off entries) or 838,752 detached (40-byte
 * entries); the fused form has no limit.  No emission guide (its per-path
 * records are allocated).  lt_get_stats does not report its counters.
 * Every call on a GPU shares that GPU's array (all contexts on it included)
 * and clears what must start at zero, so calls that overlap on one GPU race
 * and must be ordered by the caller.
 * Errors: as lt_backward_lrb3, plus LT_ERR_ARG (n_paths above the limit),
 * LT_ERR_UNSUPPORTED (guide weights set, or no scratch address on this
 * device). */
lt_status lt_backward_lrb3_noalloc(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                                   const float* d_image, lt_grads* grads);

/* ------------------------------------------------------------------------
 * Camera side of the bidirectional combination.  Sec. 7 names a
 * bidirectional formulation with path replay (Sec. 3.2) on the camera side
 * and LRB-3 on the light side as the next step.  Every path of the
 * measurement (Eq. 1) leaves the camera through a specular (dielectric) or
 * a non-specular vertex; light-path sensor connections reach only the
 * second kind, so light tracing plus camera samples restricted to the first
 * kind estimate the whole image, each path by exactly one of the two:
 *   image = lt_trace(...) then lt_camera_trace(...) (which adds),
 *   grads = lt_backward_lrb3(...) + lt_camera_backward_prb(...) (both add).
 * Camera sample s (args->n_paths samples N, a multiple of width*height)
 * renders pixel s mod (width*height) through a film offset drawn from the
 * tent filter of Eq. 20 around the pixel centre, and weighs
 * width*height / N.  It is traced by a path tracer: next-event estimation at
 * Lambertian and rough-conductor vertices (a point on the quad emitter, or
 * the point emitter; shadow ray against the scene), emission counted when a
 * ray leaving a specular vertex meets the quad emitter's front face before
 * any scene hit (the emitter occludes nothing, the ray goes on), cosine
 * (Lambertian) or microfacet (conductor) continuation, the Fresnel lobe at
 * dielectrics, at most max_depth vertices; without LT_CAMERA_ALL a sample
 * whose first vertex is not specular contributes nothing.
 * Random numbers: Philox counter (s, 0, 2) for the film offset (u0, u1),
 * (s, j, 2) at vertex j (u0, u1 direction, u2 Fresnel lobe), (s, j, 3) for
 * the next-event point (u0 along e1, u1 along e2).
 * Detached only (albedo and emitter radiance); args->flags may hold
 * LT_CAMERA_ALL only (LT_ERR_UNSUPPORTED otherwise); a directional emitter
 * is rejected (LT_ERR_UNSUPPORTED: a camera path cannot reach it); the
 * emission guide does not apply to camera samples (params->guide_w is
 * ignored).  path_mask / path_sig index camera samples.
 * ------------------------------------------------------------------------ */
/* Adds the camera samples' estimate to image (DEVICE float
 * [height][width][3], not cleared).  path_sig: each sample's decision
 * signature (FNV-1a of hit primitives, texels, next-event visibility, lobes,
 * emission hits).  Errors: LT_ERR_ARG (n_paths not a multiple of the pixel
 * count, ...), LT_ERR_UNSUPPORTED, LT_ERR_STATE, LT_ERR_HIP. */
lt_status lt_camera_trace(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params, float* image);
/* Path-replay backward of the camera samples (Sec. 3.2): each sample's
 * pixel adjoint d_image[p] is known before the replay; a primal pass
 * recomputes the sample's radiance L (and adds the emitter gradient of each
 * term), a replay then adds d_image[p] (L - sum of the terms before vertex
 * i) / rho_i to the gradient of vertex i's albedo texel, per channel (a
 * texel with rho = 0 gets nothing from the later terms).  Needs no side
 * state.  Gradients accumulate into grads (albedo required).
 * Errors: as lt_camera_trace. */
lt_status lt_camera_backward_prb(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                                 const float* d_image, lt_grads* grads);

/* ------------------------------------------------------------------------
 * Learned emission guide.  An extension of the method, not in the paper:
 * the paper samples emitted directions cosine-weighted (Sec. 3.1).  With
 * params->guide_w set, every pass draws the emitted direction of an area
 * emitter from a density q learned by a small network and weights the path
 * by A cos / q (so beta_1 = L_e A cos / q); q is held fixed in every reverse
 * mode (a detached density), which keeps the gradients unbiased.
 *
 * Network: features (position normalised to the scene box, unit normal) ->
 * 64 -> 64 -> 64 (ReLU) -> 41 outputs; products in bfloat16 on the matrix
 * cores with FP32 accumulation.  Outputs: 8 von Mises-Fisher lobes
 * {mean direction (3, normalised), log-concentration (1, clamped to
 * [-3, 8]), logit (1, softmax)} and a mixing logit (alpha = 0.9 sigmoid).
 *   q(w) = alpha sum_k pi_k [v_k(w) + v_k(mirror(w))] + (1 - alpha) max(w.n, 0) / pi
 * where mirror reflects about the emitter plane (lobes folded onto the
 * emitting hemisphere).  Parameter layout (FP32, row-major out x in):
 *   W1[64][6] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[41][64] b4[41].
 * Uniforms: Philox counter (path, 0, 1): g0 picks the component (cosine when
 * g0 >= alpha, else the lobe whose cumulative weight first exceeds
 * g0/alpha), (g1, g2) the direction.
 * A guided pass uses 16 extra bytes of library workspace per path (the
 * direction and density of each path, recomputed by every pass).
 * Errors: LT_ERR_UNSUPPORTED for a point emitter with a guide.
 * ------------------------------------------------------------------------ */
/* Diffuse vertices (LT_GUIDE_DIFFUSE).  The same network also guides the
 * scattered direction at Lambertian vertices, queried per albedo texel: once
 * per pass the library evaluates it at every texel centre - the chart centre
 * ((tx + 1/2)/R, (ty + 1/2)/R) placed on the lowest-index static Lambertian
 * triangle of the texel's texture whose chart triangle holds it - with the
 * triangle's unit normal +n (side 0) and -n (side 1), and keeps the folded
 * mixtures in a table (2 x 16 float4 per texel, L2-resident).  A vertex
 * reached against its triangle's geometric normal uses side 0, else side 1;
 * it draws from the mixture folded about its arrival-side normal, the
 * component by the third uniform of its vertex counter (path, j, 0), the
 * direction by the first two, and weights the path by rho cos / (pi q) in
 * place of rho, q held fixed in every reverse mode.  Attached passes keep
 * the drawn direction fixed in the vertex's local frame, as for a cosine
 * sample.  A texel that no triangle holds samples the cosine density.
 * Workspace: + 512 bytes per texel; a detached naive tape: + 4 bytes per
 * vertex record (the scatter weight).
 * ------------------------------------------------------------------------ */
#define LT_GUIDE_NPARAMS 11433
#define LT_GUIDE_NOUT 41

/* One training sample, 48 bytes: vertex position and normal, the sampled
 * direction, its sampling density q, its contribution S, the component
 * that drew it (0 cosine, k + 1 lobe k; informational). */
typedef struct {
  float x[3], n[3], w[3];
  float pdf, S, comp;
} lt_guide_sample;

/* Raw network outputs. x, n: DEVICE [count][3] positions and unit normals;
 * out: DEVICE [count][41].  Needs an uploaded scene (its box normalises x).
 * Errors: LT_ERR_ARG, LT_ERR_STATE (no scene), LT_ERR_HIP. */
lt_status lt_guide_eval(lt_ctx* ctx, const float* guide_w, const float* x, const float* n, int64_t count,
                        float* out);

/* The guided emission of paths [0, args->n_paths) exactly as the passes
 * draw it, written as training samples out: DEVICE [n_paths]; S is taken
 * from path_contrib (DEVICE [n_paths], e.g. lt_trace's output) or 0 when
 * NULL.  Uses args->seed and params->guide_w only.
 * Errors: LT_ERR_ARG, LT_ERR_STATE, LT_ERR_UNSUPPORTED (point emitter). */
lt_status lt_guide_emit(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                        const float* path_contrib, lt_guide_sample* out);

/* Training samples of the diffuse guide, one per path of
 * [0, args->n_paths): the path's first guided Lambertian scatter (position,
 * arrival-side normal, direction, density q, component) with S = the sum
 * of lum(C_i) over the path's later connections (Rec. 709 luminance), as
 * the guided pass with args draws it; an all-zero sample (S = 0) for a path
 * with none.  out: DEVICE [n_paths].  args->flags: 0 or LT_GUIDE_DIFFUSE
 * (the pass is guided at diffuse vertices either way); params->guide_w set.
 * Writes no image.
 * Errors: as lt_trace, LT_ERR_ARG (other flags, null out or guide_w). */
lt_status lt_guide_vertex_samples(lt_ctx* ctx, const lt_trace_args* args, const lt_params* params,
                                  lt_guide_sample* out);

/* Training loss L = -sum_b (S_b / q_b) log q_theta(w_b | x_b, n_b) / Z with
 * Z = sum_b S_b / q_b (a self-normalised Monte Carlo estimate of the KL
 * divergence from the S-proportional density to q_theta, up to a constant;
 * invariant to the scale of S, which falls as 1/n_paths) and its gradient.
 * samples: DEVICE [count]; grad: DEVICE [LT_GUIDE_NPARAMS], overwritten;
 * loss: DEVICE [1] or NULL.  Samples with q <= 0 or S == 0 contribute
 * nothing; with no contributing sample the loss and gradient are zero.
 * Deterministic (fixed reduction order).
 * Errors: LT_ERR_ARG, LT_ERR_STATE, LT_ERR_OOM (cap), LT_ERR_HIP. */
lt_status lt_guide_grad(lt_ctx* ctx, const float* guide_w, const lt_guide_sample* samples, int64_t count,
                        float* grad, float* loss);

/* One Adam step (Kingma & Ba 2015, bias-corrected) on the guide weights,
 * in place.  w, m, v: DEVICE [LT_GUIDE_NPARAMS] (m, v zero before step 1);
 * grad: DEVICE [LT_GUIDE_NPARAMS]; step: 1-based.
 * Errors: LT_ERR_ARG (step < 1, lr <= 0, betas outside [0, 1)). */
lt_status lt_guide_adam(lt_ctx* ctx, float* w, const float* grad, float* m, float* v, int32_t step, float lr,
                        float beta1, float beta2, float eps);

/* One online training step of the guide, after a pass made with `args` and
 * guide_w: the guided emission of paths [0, min(args->n_paths, n_samples))
 * paired with path_contrib (as lt_guide_emit, into samples: DEVICE
 * [n_samples]), the loss gradient over those samples (as lt_guide_grad,
 * into grad: DEVICE [LT_GUIDE_NPARAMS]; loss: DEVICE [1] or NULL) and an
 * Adam step on guide_w in place (as lt_guide_adam; m, v: DEVICE
 * [LT_GUIDE_NPARAMS], zero before step 1).  All arguments are checked
 * before anything is enqueued.
 * Errors: as those three calls. */
lt_status lt_guide_train_step(lt_ctx* ctx, const lt_trace_args* args, float* guide_w, const float* path_contrib,
                              lt_guide_sample* samples, int64_t n_samples, float* grad, float* m, float* v,
                              float* loss, int32_t step, float lr, float beta1, float beta2, float eps);

/* ------------------------------------------------------------------------
 * Batches.  An extension for training many inverse-rendering problems at
 * once (not in the paper).  Instances of uneven scene size, film, path count
 * and depth each take one optimisation step - the forward of lt_trace, the
 * L2 loss and image adjoint of lt_loss_l2, the LRB-3-pass backward of
 * lt_backward_lrb3 (Sec. 4.3) - as one persistent launch per pass over an
 * instance table: every wave takes work tickets (path indices) from one
 * instance at a time and moves to the next when it has drained it.
 * Instances of 2^20 paths or more take a backward launch each, and those
 * of 2^22 or more a forward launch each, through kernels with the
 * single-instance calls' register budgets and launch shapes (the
 * multi-instance kernels hold fewer waves or spill more).  With
 * use_graph the step is captured once into a hipGraph and replayed; between
 * replays only the seeds may change (they are read from device memory).
 * Results equal the per-instance calls up to the order of floating-point
 * atomic sums.
 * ------------------------------------------------------------------------ */
typedef struct lt_batch lt_batch;

typedef struct {
  lt_ctx* ctx;            /* context holding this instance's uploaded scene; every
                             instance's context uses the batch's device */
  lt_trace_args args;     /* seed, n_paths, max_depth, flags: 0 or LT_ATTACHED; path_mask
                             as for lt_trace (DEVICE [n_paths] or NULL); signatures,
                             info and contributions must be NULL */
  lt_params params;       /* as for lt_backward_lrb3 (guide_w allowed) */
  const float* target;    /* DEVICE [height][width][3] loss target */
  float* image;           /* DEVICE [height][width][3], overwritten with the estimate */
  float* d_image;         /* DEVICE [height][width][3], overwritten with dL/dI */
  float* loss;            /* DEVICE [1], overwritten with the mean squared error */
  lt_grads grads;         /* accumulated into, as by lt_backward_lrb3 */
} lt_instance;

/* A batch runner on HIP device `device`, enqueuing on `hip_stream`.
 * Errors: LT_ERR_ARG, LT_ERR_HIP, LT_ERR_OOM. */
lt_status lt_batch_create(int device, void* hip_stream, lt_batch** out);
/* Release the runner (its graph and tables). NULL is ignored. */
void lt_batch_destroy(lt_batch* b);
const char* lt_batch_last_error(const lt_batch* b);
/* One step for instances inst[0..n-1] (1 <= n <= 4096), on the batch's
 * stream; the instance contexts' streams are set to it.  use_graph: 0 eager
 * launches; 1 replay the captured hipGraph, capturing it first when the
 * instance set differs from the captured one in anything but the seeds.
 * Errors: LT_ERR_ARG (bad instance), LT_ERR_STATE (scene missing),
 * LT_ERR_UNSUPPORTED (flags or outputs outside the list above), LT_ERR_OOM,
 * LT_ERR_HIP. */
lt_status lt_batch_step(lt_batch* b, const lt_instance* inst, int32_t n, int32_t use_graph);
/* Launch shape of the batched passes: block and blocks_per_cu as in
 * lt_set_tuning (the attached backward chooses its own workgroup size;
 * lrb3_split is ignored: batches run both LRB-3 passes in one kernel, and
 * the attached instances that run on their own the two-kernel pair).  The
 * instances that run on their own take their contexts' tuning, as the
 * single-instance calls do.
 * Default {256, 4, 1, 0}.  The backward passes keep per-workgroup LDS copies of
 * the gradient arrays (heights always, albedo with lds_grad = 1) for the
 * instances whose arrays fit one budget per pass: the largest requested size
 * that costs the pass no resident workgroups per compute unit.  The other
 * instances accumulate into their gradient arrays directly. */
lt_status lt_batch_set_tuning(lt_batch* b, const lt_tuning* t);
lt_status lt_batch_get_tuning(const lt_batch* b, lt_tuning* out);
/* Pick block size and workgroups per compute unit for these instances by
 * timing trial steps (each instance at 1/16 of its paths, at least 65536)
 * over a fixed candidate set, keep the fastest, and remember it in
 * cache_path (a JSON object keyed by device and workload; NULL: no cache).
 * A cached entry is reused without trials.  Trial steps overwrite the
 * instances' images, adjoints and losses and accumulate into their
 * gradients: clear those afterwards.  *out (may be NULL) receives the choice.
 * Errors: as lt_batch_step. */
lt_status lt_batch_autotune(lt_batch* b, const lt_instance* inst, int32_t n, const char* cache_path,
                            lt_tuning* out);

#ifdef __cplusplus
}
#endif

#endif /* LT_H */
