/*
 * mpg.h -- C ABI of the MI355X batched manifold-walk library (libmpg.so).
 *
 * The library implements the data-parallel hot path of manifold path guiding
 * (Fan et al., "Manifold Path Guiding for Importance Sampling Specular
 * Chains", ACM TOG 42(6), 2023): seed chains are drawn from a guided
 * distribution (Sec. 5.4-5.5), driven to admissible specular chains by
 * manifold walks (Newton's method plus reprojection, Sec. 3), scored with the
 * sub-path throughput terms kappa and G (Eq. ThroughputEval), and their
 * reciprocal sampling probability is estimated by repeated independent
 * trials (Sec. 5.8).  Guide fitting (weighted EM per spatial cell) and an
 * implicit-function-theorem adjoint of the converged chain complete it.
 *
 * Conventions shared by every entry point:
 *  - Arguments named d_* are device pointers owned by the caller; host
 *    descriptors are read during the call only.  The library never frees
 *    caller memory.
 *  - Per-chain arrays are structure-of-arrays: points [3][N] (component
 *    major), chain vertices [K][N] and [3][K][N] with K = MPG_KMAX = 8.
 *  - Every compute call is asynchronous on the given HIP stream (NULL = the
 *    null stream); it performs no device synchronization and no allocation
 *    except where stated (scene / guide / workspace creation).
 *  - Argument errors (NULL where required, N < 0, sizes out of range) are
 *    detected on the host before any launch and return MPG_ERR_INVALID_ARG;
 *    HIP launch failures return MPG_ERR_HIP.  mpg_last_error() gives a
 *    thread-local message for the last non-OK status.
 *  - Per-chain failures are data, not errors: they are reported in the
 *    per-chain status array (MPG_CONVERGED ... MPG_BAD_INPUT).
 *  - The persistent form (MPG_FORM_PERSISTENT) keeps its bucket order, queue
 *    heads and counters in an mpg_workspace: a workspace serves one call at a
 *    time (calls on one stream are ordered; calls on different streams need
 *    different workspaces).  Its per-length kernels run on hip_stream and
 *    three internal streams per device, forked from and joined back to
 *    hip_stream with events, which graph capture records as dependencies;
 *    such calls must not be issued from several host threads on one device
 *    at the same time.
 */
#ifndef MPG_H
#define MPG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mpg_status;
#define MPG_OK 0
#define MPG_ERR_INVALID_ARG (-1)
#define MPG_ERR_HIP (-2)
#define MPG_ERR_OOM (-3)
#define MPG_ERR_UNSUPPORTED (-4)

/* per-chain status codes */
#define MPG_CONVERGED 0     /* admissible chain found, sides valid, visible from x_L */
#define MPG_MAX_ITER 1      /* iteration budget spent without convergence */
#define MPG_SINGULAR 2      /* a pivot of the block-tridiagonal solve vanished */
#define MPG_SIDE_INVALID 3  /* converged, but a vertex violates its R / T side condition */
#define MPG_OCCLUDED 4      /* converged, but x_n cannot see x_L */
#define MPG_SEED_INVALID 5  /* the seed could not be drawn or deduced */
#define MPG_FP64_REJECT 6   /* near-singular chain failed the FP64 residual check */
#define MPG_BAD_INPUT 7     /* non-finite endpoint or chain length outside 1..8 */
#define MPG_NEEDS_FP64 8    /* converged in FP32, awaiting manifold_walk_fp64 (defer_fp64 only) */

#define MPG_MAT_MIRROR 0
#define MPG_MAT_DIELECTRIC 1

#define MPG_KMAX 8
#define MPG_PRIM_NONE ((int32_t)0x80000000)
#define MPG_P0_ANY_OBJECT (-1)
#define MPG_P0_DIRECTION (-2)

const char* mpg_last_error(void);
/* version string of the library build */
const char* mpg_version(void);

/* ------------------------------------------------------------------------ */
/* Scene                                                                      */
/* ------------------------------------------------------------------------ */

/* Sine-sum height field z = z0 + sum_k amp_k sin(freq_k (cos psi_k x + sin psi_k y) + phase_k)
 * on a res x res vertex grid over [x0,x1] x [y0,y1]; its vertices are
 * first_vert + j res + i and its triangles first_tri + 2 (j (res-1) + i) + {0,1}.
 * The amplitudes and phases are the differentiable surface parameters of
 * manifold_walk_adjoint (two per sine, in declaration order). */
typedef struct {
  int32_t obj, res, first_vert, first_tri, n_sines;
  float x0, x1, y0, y1, z0;
  float amp[8], freq[8], psi[8], phase[8];
} mpg_heightfield;

/* Host description of the specular surfaces M_S (Sec. 5.3, operator r).
 * Triangles carry per-vertex shading normals; analytic spheres use their
 * exact normal.  Primitive ids: triangles 0..n_tris-1 in this order,
 * spheres -1 - s.  Each object has a material (MPG_MAT_*) and, for
 * dielectrics, the index of refraction inside (outside is 1); triangle
 * windings are counter-clockwise about the outward normal. */
typedef struct {
  int32_t n_verts;
  const float* verts;    /* host [n_verts][3] */
  const float* normals;  /* host [n_verts][3] */
  int32_t n_tris;
  const int32_t* tris;     /* host [n_tris][3] */
  const int32_t* tri_obj;  /* host [n_tris] */
  int32_t n_objects;
  const int32_t* obj_material;  /* host [n_objects] */
  const float* obj_ior;         /* host [n_objects] */
  int32_t n_spheres;
  const float* spheres;       /* host [n_spheres][4]: centre, radius */
  const int32_t* sphere_obj;  /* host [n_spheres] */
  float scale;                /* scene scale L (longest side of the specular bounding box) */
  int32_t n_heightfields;
  const mpg_heightfield* heightfields;
} mpg_scene_desc;

typedef struct mpg_scene mpg_scene;

/* Builds the device scene on the current device: uploads geometry, builds a
 * binned-SAH BVH (collapsed into 4-wide 128-byte nodes) and per-object
 * area tables.
 * Allocates device memory; synchronous. */
mpg_status mpg_scene_create(const mpg_scene_desc* desc, mpg_scene** out);
void mpg_scene_destroy(mpg_scene* scene);
/* BVH statistics: node count, maximum depth (the traversal stack needs depth+1 entries). */
mpg_status mpg_scene_stats(const mpg_scene* scene, int32_t* n_nodes, int32_t* max_depth, int32_t* n_tris);

/* Replaces the height-field parameters theta -- the differentiable surface
 * parameters of manifold_walk_adjoint (Sec. 5.2): d_theta is device float
 * [n_params], n_params = 2 * sum of n_sines over the scene's height fields,
 * amplitude then phase per sine in height-field order.  Height-field
 * vertices and normals are recomputed (FP32 evaluation of the sine sum), the
 * BVH keeps its topology and every box is refitted to the triangles under
 * it, and the per-object area tables used by p_0 and the scene top used by
 * guided seeds are recomputed on the device.  Stream ordered with no host
 * synchronization and no allocation, so it may be captured into a HIP graph
 * together with the walks that follow; work on this scene queued on other
 * streams must not overlap it.  Host-detected errors: n_params differs from
 * the scene's count, NULL theta.  A non-finite theta is detected on the
 * device: the scene is left unchanged and the scene's error word (read with
 * mpg_scene_params_error) becomes MPG_ERR_INVALID_ARG; a valid update resets
 * it to MPG_OK. */
mpg_status mpg_scene_set_params(mpg_scene* scene, const float* d_theta, int32_t n_params, void* hip_stream);
/* Copies the scene's error word of the last mpg_scene_set_params (MPG_OK
 * initially) into d_out[0] (device int32), in stream order on hip_stream
 * (a device-to-device copy; no host synchronization).  Errors: NULL scene or
 * d_out. */
mpg_status mpg_scene_params_error(const mpg_scene* scene, int32_t* d_out, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Batches                                                                    */
/* ------------------------------------------------------------------------ */

/* Configurations (x_D, x_L) with their chain length n and type tau (Sec. 3,
 * Table 1; Eq. eq_div1): bit i of type is 1 for a transmission at vertex
 * i+1.  obj1 selects the p_0 draw of the first vertex: an object id,
 * MPG_P0_ANY_OBJECT or MPG_P0_DIRECTION. */
typedef struct {
  int32_t N;
  const float* d_xD;    /* [3][N] shading points */
  const float* d_nD;    /* [3][N] unit normals at x_D */
  const float* d_xL;    /* [3][N] point-light positions */
  const uint8_t* d_len;   /* [N] 1..8 */
  const uint8_t* d_type;  /* [N] */
  const int32_t* d_obj1;  /* [N] */
  const float* d_offset;  /* [2][K][N] offset normals (o_s, o_t) of glossy chains (Sec. 5.7), or NULL for
                             specular chains: vertex i of chain c is specular about m = o_s s + o_t t +
                             sqrt(1 - |o|^2) n_s, with s the world x axis projected on the tangent plane
                             and t = n_s x s (see sample_offsets) */
} mpg_endpoints;

/* Chains: primitive id and position of each specular vertex. */
typedef struct {
  int32_t* d_prim; /* [K][N] */
  float* d_pos;    /* [3][K][N] */
} mpg_chains;

/* Walk outputs; any pointer may be NULL to skip it. */
typedef struct {
  int8_t* d_status;        /* [N] MPG_CONVERGED ... */
  uint8_t* d_iters;        /* [N] Newton trials used */
  uint64_t* d_solution_id; /* [N] hash of (n, type, primitive ids); 0 unless converged */
  float* d_G;              /* [N] generalized geometric term */
  float* d_kappa;          /* [N] product of Fresnel / mirror coefficients */
  float* d_residual;       /* [N] max-norm of the constraint at the returned chain */
} mpg_walk_out;

#define MPG_FORM_PLAIN 0
#define MPG_FORM_PERSISTENT 1

typedef struct {
  int32_t max_iter;          /* Newton trials per walk (default 20) */
  float tol_vertex;          /* converged when a full step moves every vertex <= tol_vertex * scale (1e-4) */
  float tol_residual;        /* ... and leaves max|C| <= tol_residual (1e-5) */
  float scale;               /* scene scale L */
  float tmin_rel;            /* ray offset, relative to L (1e-5) */
  float match_rel;           /* trial-to-target match distance, relative to L (1e-3) */
  float fp64_cond_threshold; /* FP64 residual check when the condition estimate exceeds this (1e4) */
  float fp64_graze_cos;      /* ... or when a vertex scatters with |cos| below this (0.02) */
  float cone_cos;            /* MPG_P0_DIRECTION: cosine of the cone half-angle about n_D */
  int32_t form;              /* MPG_FORM_PLAIN or MPG_FORM_PERSISTENT */
  int32_t bucketing;         /* persistent form: group chains by length (1), by length and then by the
                                spatial cell of x_D on a 32^3 Morton-ordered grid (2), as 2 with each
                                bucket split into 8 spatial ranges, one per XCD, for the lane-refill
                                walk (3), or not at all (0) */
  int32_t waves_per_group;   /* wavefronts per workgroup (1, 2, 4) */
  int32_t stack_depth;       /* LDS traversal stack entries per lane (>= BVH depth + 1; 0 = automatic) */
  int32_t refill;            /* persistent form with bucketing: each lane takes a new chain as soon as its own
                                finishes (1) instead of whole 64-chain batches (0, default) */
  int32_t max_len;           /* longest chain in the batch (1..8, default 8); longer chains get MPG_BAD_INPUT */
  int32_t defer_fp64;        /* 1: leave MPG_NEEDS_FP64 chains for a later manifold_walk_fp64 call (0) */
  uint32_t length_order;     /* persistent form with bucketing: the order in which the per-length walk
                                and seed kernels are dealt round robin to the four workers (the caller's stream and
                                three internal streams), as eight 4-bit lengths, the first in the lowest
                                nibble; every length 1..8 exactly once (lengths above max_len are skipped).
                                0 = longest first (0x12345678).  Results do not depend on it. */
} mpg_walk_params;

/* Fills defaults for a scene of scale L. */
mpg_status mpg_walk_params_default(float scale, mpg_walk_params* out);

/* Device scratch for the persistent form, estimate_inv_prob's queue and
 * fit_guide's binning, sized for up to max_chains chains / samples.
 * Allocates device memory; synchronous. */
typedef struct mpg_workspace mpg_workspace;
mpg_status mpg_workspace_create(int32_t max_chains, mpg_workspace** out);
void mpg_workspace_destroy(mpg_workspace* ws);

/* ------------------------------------------------------------------------ */
/* Guide: 8-component 2-D Gaussian mixtures over (x, y) of x_1 on a res^3     */
/* grid of cells over the x_D bounding box.                                   */
/* ------------------------------------------------------------------------ */

typedef struct mpg_guide mpg_guide;

typedef struct {
  float lo[3], hi[3]; /* x_D bounding box of the grid */
  int32_t res;        /* cells per axis (32) */
  int32_t comps;      /* mixture components (8) */
  int32_t em_iters;   /* EM iterations (30) */
  int32_t min_samples;/* cells with fewer samples stay invalid (p_0 only) (16) */
  float reg;          /* covariance regularizer added to the diagonal (1e-6 L^2) */
  int32_t target_obj; /* object the guided (x, y) is lifted onto */
} mpg_guide_desc;

/* Allocates an empty guide (every cell invalid).  Synchronous. */
mpg_status mpg_guide_create(const mpg_guide_desc* desc, mpg_guide** out);
void mpg_guide_destroy(mpg_guide* g);
/* Host upload / download of the per-cell mixtures.  Layouts: valid [cells],
 * pi [cells][comps], mu [cells][comps][2], cov [cells][comps][3] (xx, xy, yy),
 * count [cells] (download only; may be NULL).  Synchronous. */
mpg_status mpg_guide_upload(mpg_guide* g, const int32_t* valid, const float* pi, const float* mu, const float* cov);
mpg_status mpg_guide_download(const mpg_guide* g, int32_t* valid, float* pi, float* mu, float* cov,
                              int32_t* count);

/* ------------------------------------------------------------------------ */
/* Hot path                                                                   */
/* ------------------------------------------------------------------------ */

/* Draws one seed chain per configuration (Sec. 5.4-5.5): with probability
 * alpha (or always when guide is NULL or the cell is invalid) from p_0,
 * otherwise from the cell's Gaussian mixture over (x, y) lifted onto the
 * guide's target object; then w_D = normalize(p - x_D), x_1 = r(x_D, w_D)
 * and x_2..x_n by Eq. (deduction).  Random numbers: Philox4x64-10 with key
 * (philox_seed, 0) and counter (chain, trial, attempt, 0).  Writes prim/pos
 * for vertices 0..n-1 and d_status (0 or MPG_SEED_INVALID / MPG_BAD_INPUT).
 * With params->form == MPG_FORM_PERSISTENT and bucketing on, the chains are
 * grouped by length (and spatial cell) in the workspace ws (capacity >= N)
 * and drawn by one persistent kernel per length; the seeds are identical to
 * the plain launch's (ws may be NULL for the plain form). */
mpg_status sample_seeds(const mpg_scene* scene, const mpg_guide* guide, const mpg_walk_params* params,
                        const mpg_endpoints* ep, uint64_t philox_seed, uint32_t trial, float alpha,
                        mpg_chains* out, int8_t* d_status, mpg_workspace* ws, void* hip_stream);

/* Offset normals of glossy chains (Sec. 5.7), sampled before the walk: per
 * chain and vertex, (o_s, o_t) = sin theta_m (cos phi, sin phi) of a
 * microfacet normal drawn from the GGX distribution D(m) cos theta_m with
 * the given roughness (tan^2 theta_m = roughness^2 u / (1 - u), phi = 2 pi
 * v; Philox block (chain, trial, 16 + i / 4), uniforms 2 (i mod 4) and
 * 2 (i mod 4) + 1 for vertex i).  d_offset is [2][K][N]; pass it as
 * mpg_endpoints.d_offset to seed, walk and estimate glossy chains.  Errors:
 * N < 0, NULL output, roughness outside [0, 1]. */
mpg_status sample_offsets(int32_t N, uint64_t philox_seed, uint32_t trial, float roughness, float* d_offset,
                          void* hip_stream);

/* Manifold walks (Sec. 3): Newton's method on the generalized half-vector
 * constraints with a block-tridiagonal Jacobian, reprojection by ray casting,
 * step halving; then side / visibility checks, an FP64 residual check for
 * near-singular chains, and G and kappa (Eq. ThroughputEval).  seeds and out
 * may alias.  d_seed_status (nullable) marks seeds to skip.  The persistent
 * form needs a workspace of at least N chains. */
mpg_status manifold_walk_batch(const mpg_scene* scene, const mpg_walk_params* params, const mpg_endpoints* ep,
                               const mpg_chains* seeds, const int8_t* d_seed_status, mpg_chains* out,
                               const mpg_walk_out* wout, mpg_workspace* ws, void* hip_stream);

/* Allocation-free manifold_walk_batch, for callers that cannot allocate
 * device memory or create streams: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, results
 * and kernels as manifold_walk_batch, without a workspace: the persistent
 * form keeps its bucket order, queue heads and per-chain class bytes in a
 * static device array of about 5.3 MB per device (held until the process
 * ends), and every per-length kernel runs on hip_stream.  Limits: N <=
 * MPG_NOALLOC_MAX_CHAINS (else MPG_ERR_INVALID_ARG); bucketing 0 or 1 in the
 * persistent form (2 and 3 need a workspace: MPG_ERR_UNSUPPORTED).  Every
 * call on one device shares that array, which keeps the last call's
 * contents (each call resets what it reads first): calls that overlap on one
 * device, on different streams or host threads, race and must not be
 * issued. */
#define MPG_NOALLOC_MAX_CHAINS (1 << 20)
mpg_status manifold_walk_batch_noalloc(const mpg_scene* scene, const mpg_walk_params* params,
                                       const mpg_endpoints* ep, const mpg_chains* seeds, const int8_t* d_seed_status,
                                       mpg_chains* out, const mpg_walk_out* wout, void* hip_stream);

/* FP64 pass of the walk (normally run by manifold_walk_batch itself): chains
 * whose status is MPG_NEEDS_FP64 (converged in FP32 but near-singular, stalled
 * at the FP32 residual floor, or scattering within fp64_graze_cos of grazing)
 * get an FP64 residual check with up to two FP64 Newton steps inside their
 * primitives, then their side / visibility tests, G and kappa in FP64.  The
 * chain arrays are read and updated in place.  Other chains are untouched. */
mpg_status manifold_walk_fp64(const mpg_scene* scene, const mpg_walk_params* params, const mpg_endpoints* ep,
                              mpg_chains* chains, const mpg_walk_out* wout, void* hip_stream);

/* Profiling variant of the plain walk (FP64 pass included): same outputs as
 * manifold_walk_batch, plus work tallies reduced into d_counts[8] (device,
 * uint64): BVH box tests, triangle tests, sphere tests, rays, residual-only
 * vertex evaluations, Jacobian vertex evaluations, FP64 Jacobian vertex
 * evaluations, chains.  The counters cost time: do not time this call. */
mpg_status mpg_walk_count(const mpg_scene* scene, const mpg_walk_params* params, const mpg_endpoints* ep,
                          const mpg_chains* seeds, const int8_t* d_seed_status, mpg_chains* out,
                          const mpg_walk_out* wout, uint64_t* d_counts, void* hip_stream);

/* Reciprocal probability by repeated independent trials (Sec. 5.8): for each
 * target with status MPG_CONVERGED, seeds are redrawn from the same
 * distribution (trial counters 1 + r max_trials + k - 1) and walked until one
 * reaches the target again (same objects, every vertex within match_rel L);
 * K = that trial count, or max_trials when none matched (d_truncated = 1).
 * d_inv_prob = mean_r K_r / P(n) with P(n) = 1 (n is given), d_trials =
 * sum_r K_r.  Other targets, and targets longer than params->max_len (which
 * bounds the per-length kernels launched), get 0.  d_truncated may be NULL.  With
 * params->form == MPG_FORM_PERSISTENT and bucketing on, the targets are
 * grouped by length in ws (capacity >= N) and every lane of one persistent
 * kernel per length takes the next target as soon as its trials end; the
 * results equal the plain launch's (ws may be NULL for the plain form). */
mpg_status estimate_inv_prob(const mpg_scene* scene, const mpg_guide* guide, const mpg_walk_params* params,
                             const mpg_endpoints* ep, const mpg_chains* target, const int8_t* d_target_status,
                             int32_t max_trials, int32_t repeats, uint64_t philox_seed, float alpha,
                             int32_t* d_trials, float* d_inv_prob, uint8_t* d_truncated,
                             mpg_workspace* ws, void* hip_stream);

/* Weighted EM per cell (weights w = T <1/P>, Eq. eq_weight) on 32-byte sample
 * records {x_D.x, x_D.y, x_D.z, u, v, w, 0, 0} (u, v = x, y of x_1); samples
 * with w <= 0 are ignored.  Initialization per cell: the weighted mean and
 * covariance (+ reg I), component j centred on the cell's sample of rank
 * floor((j + 1/2) m / comps) in input order, equal weights; then exactly
 * em_iters iterations.  Needs a workspace of at least n_samples. */
mpg_status fit_guide(const mpg_scene* scene, const float* d_samples, int32_t n_samples, mpg_guide* guide,
                     mpg_workspace* ws, void* hip_stream);

/* Packs walked chains into fit_guide's 32-byte sample records: {x_D, x and y
 * of x_1, w, 0, 0} with the sample weight w = T <1/P> (Eq. eq_weight),
 * T = kappa G (L_o = 1) and <1/P> = d_inv_prob; w = 0 unless d_status is
 * MPG_CONVERGED.  d_samples is [N][8] float. */
mpg_status make_guide_samples(const mpg_endpoints* ep, const mpg_chains* chains, const int8_t* d_status,
                              const float* d_G, const float* d_kappa, const float* d_inv_prob, float* d_samples,
                              void* hip_stream);

/* Adjoint of converged chains by the implicit function theorem (Sec. 5.2):
 * given cotangents of the vertex positions (d_grad_pos [3][K][N], nullable)
 * and of G (d_grad_G [N], nullable) for the loss
 *   l = sum_chains (sum_i grad_pos_i . x_i + grad_G G),
 * writes the per-chain gradients with respect to x_D (d_grad_xD [3][N]) and
 * x_L (d_grad_xL [3][N]), and ADDS the gradient with respect to the
 * height-field parameters (d_grad_theta [P], P = 2 * sum of n_sines, in
 * scene order: amplitude, phase per sine; the caller zeroes it first; atomic
 * float additions, so the summation order is not deterministic; may be NULL
 * when P = 0).  The surface parameters move triangle vertices and vertex
 * normals; a chain vertex rides on its triangle at fixed barycentric
 * coordinates.  Chains whose status is not MPG_CONVERGED (or whose primitive
 * ids are out of range) get zero gradients and add nothing.  The chains must
 * be the converged output of manifold_walk_batch on the same scene and
 * endpoints; params->max_len bounds the lengths handled.  All buffers are
 * device memory owned by the caller; the call is asynchronous on hip_stream.
 * With params->form == MPG_FORM_PERSISTENT and bucketing on, chains are
 * grouped by length in ws (capacity >= N) and each length runs in its own
 * persistent kernel (ws may be NULL for the plain form). */
mpg_status manifold_walk_adjoint(const mpg_scene* scene, const mpg_walk_params* params, const mpg_endpoints* ep,
                                 const mpg_chains* converged, const int8_t* d_status, const float* d_grad_pos,
                                 const float* d_grad_G, float* d_grad_xD, float* d_grad_xL, float* d_grad_theta,
                                 mpg_workspace* ws, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* The paper's guide (Sec. 5.5, 5.6): a binary tree over the 6-D              */
/* configuration (x_D, x_L); per leaf the weighted distributions of the chain */
/* length n and type tau (Eq. eq_div2) and a mixture of von Mises-Fisher      */
/* lobes over w_D (Eq. vMF), one per sub-path sample.                         */
/* ------------------------------------------------------------------------ */

typedef struct mpg_stree mpg_stree;

typedef struct {
  float lo[6], hi[6];   /* root box over (x_D, x_L); samples outside it are not used */
  float eps;            /* child overlap: a child keeps its parent's samples inside its box widened by eps times
                           its extent along the split axis (0.1) */
  float thr_scale;      /* a node with more than thr_scale sqrt(|S|) samples is split (1) */
  int32_t max_depth;    /* depth limit of the tree (20) */
  float sigma_min;      /* lower bound of a lobe's footprint angle, radians (1e-3) */
  float sigma_lone;     /* footprint of a lobe alone in its (n, tau) group, radians (0.1) */
  float p0n[8];         /* P_0(n), n = 1..8 (normalised by the library) */
  float alpha;          /* probability of the initial distributions in the defensive mixtures (0.5) */
  float p_transmit;     /* p_0's probability of transmission at a dielectric vertex (0.5) */
} mpg_stree_desc;

/* Fills the defaults noted above (root box [0, 1]^6, P_0 uniform). */
mpg_status mpg_stree_desc_default(mpg_stree_desc* desc);
/* Creates an empty guide (one leaf without samples: p_0 only).  Allocates
 * device memory; synchronous. */
mpg_status mpg_stree_create(const mpg_stree_desc* desc, mpg_stree** out);
void mpg_stree_destroy(mpg_stree* tree);
/* Replaces P_0(n), alpha and p_transmit (host values; takes effect for the
 * calls issued afterwards). */
mpg_status mpg_stree_set_prior(mpg_stree* tree, const float* p0n, float alpha, float p_transmit);

/* Fits the guide to sub-path sample records d_records [n][16] float: x_D
 * (3), x_L (3), w_D (3, unit), w, n, tau, 0 x 4 (as written by
 * make_guide_records).  Records with w <= 0, non-finite values, n outside
 * 1..8 or x outside the root box are ignored.  The tree is built breadth
 * first: a node with more than thr_scale sqrt(|S|) samples is halved across
 * its longest side; each child keeps its parent's samples inside its box
 * widened by eps of its extent along the split axis (Sec. 5.6).  Per leaf:
 * W, W_n; lobes grouped by (n, tau) with kappa = sigma^-2, sigma the angle to
 * the nearest other direction of the group.  The whole build runs on the
 * GPU, level by level; the split and leaf decisions and the per-leaf and
 * per-group weight sums are taken in FP64 in record order, so the tree does
 * not depend on the launch shape.  Synchronous on hip_stream (each level's
 * size steers the next level's launches); allocates the new tree and frees
 * the old one only on success (on an error the guide is unchanged). */
mpg_status fit_guide_stree(mpg_stree* tree, const float* d_records, int32_t n_records, void* hip_stream);

/* Node, leaf, group and lobe counts of the fitted guide. */
mpg_status mpg_stree_stats(const mpg_stree* tree, int32_t* n_nodes, int32_t* n_leaves, int32_t* n_groups,
                           int32_t* n_lobes);
/* Host copies of the guide (any pointer may be NULL): per node axis (-1 =
 * leaf), mid, child, W, W_n [8], own samples, leaf groups (first, count);
 * per group key (n | tau << 8), weight, lobes (first, count); per lobe
 * (direction, kappa) [4] and the inclusive prefix of lobe weights in its
 * group.  Synchronous. */
mpg_status mpg_stree_download(const mpg_stree* tree, int32_t* axis, float* mid, int32_t* child, float* W, float* Wn,
                              int32_t* own, int32_t* leaf_groups, int32_t* grp_key, float* grp_w, int32_t* grp_lobes,
                              float* lobe, float* lobe_cdf);

/* Seeds from the guide (Sec. 5.3-5.5): per configuration the leaf of (x_D,
 * x_L); n = ep->d_len[c] when it is 1..8, else (0) drawn from alpha P_0(n) +
 * (1 - alpha) P_e(n); then (w_D, tau) from alpha p_0 + (1 - alpha) p_e: p_0
 * takes x_1 by ep->d_obj1 and decides tau at each vertex as the ray reaches
 * it (a mirror reflects, a dielectric transmits with p_transmit); p_e draws
 * tau from P_e(tau | n), a lobe by weight and w_D from the lobe; x_2..x_n
 * follow by Eq. (deduction).  ep->d_type is not read.  Outputs: n
 * (d_len_out), tau (d_type_out), P(n) of the mixture (d_pn), the seed chain
 * and d_status (0, MPG_SEED_INVALID or MPG_BAD_INPUT).  Random numbers:
 * Philox4x64-10, key (philox_seed, 0), counters (chain, trial, 0..2, 0).
 * params->form = MPG_FORM_PERSISTENT with bucketing != 0 draws the lengths
 * first and samples each length's seeds in a kernel of its own over the
 * configurations bucketed in ws (capacity >= N, else MPG_ERR_INVALID_ARG);
 * otherwise one thread per configuration and ws may be NULL.  Both forms
 * give identical seeds. */
mpg_status sample_seeds_stree(const mpg_scene* scene, const mpg_stree* tree, const mpg_walk_params* params,
                              const mpg_endpoints* ep, uint64_t philox_seed, uint32_t trial, uint8_t* d_len_out,
                              uint8_t* d_type_out, float* d_pn, mpg_chains* out, int8_t* d_status,
                              mpg_workspace* ws, void* hip_stream);

/* Reciprocal probability with the guide (Sec. 5.8): for each target with
 * status MPG_CONVERGED, n = ep->d_len is kept and each trial draws (w_D,
 * tau) from the same mixture as sample_seeds_stree (trial counters 1 + r
 * max_trials + k - 1) and walks it; a trial matches when its tau equals
 * ep->d_type and its chain the target (same objects, vertices within
 * match_rel L).  d_trials = sum_r K_r, d_pn = P(n), d_inv_prob = mean_r K_r /
 * P(n) (P(n) factored out of the estimate).  Other targets, and targets
 * longer than params->max_len, get 0; glossy offsets are not read.
 * params->form = MPG_FORM_PERSISTENT with bucketing != 0 runs one lane-refill
 * kernel per length over the targets bucketed in ws (capacity >= N, else
 * MPG_ERR_INVALID_ARG); otherwise one thread per configuration and ws may be
 * NULL.  Both forms give identical results. */
mpg_status estimate_inv_prob_stree(const mpg_scene* scene, const mpg_stree* tree, const mpg_walk_params* params,
                                   const mpg_endpoints* ep, const mpg_chains* target, const int8_t* d_target_status,
                                   int32_t max_trials, int32_t repeats, uint64_t philox_seed, int32_t* d_trials,
                                   float* d_inv_prob, uint8_t* d_truncated, float* d_pn, mpg_workspace* ws,
                                   void* hip_stream);

/* Sample records for fit_guide_stree from walked chains: {x_D, x_L, w_D =
 * normalize(x_1 - x_D), w, n, tau, 0 x 4} with w = T <1/P> (Eq. eq_weight),
 * T = kappa G, <1/P> = d_inv_prob; w = 0 unless d_status is MPG_CONVERGED. */
mpg_status make_guide_records(const mpg_endpoints* ep, const mpg_chains* chains, const int8_t* d_status,
                              const float* d_G, const float* d_kappa, const float* d_inv_prob, float* d_records,
                              void* hip_stream);

/* Selective activation (Sec. 5.8): d_active[c] = 1 when the leaf of
 * configuration c holds own samples of the last fit (samples kept only for
 * the child overlap do not count), else 0 (the caller falls back to path
 * tracing there). */
mpg_status mpg_stree_active(const mpg_stree* tree, const mpg_endpoints* ep, uint8_t* d_active, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Progressive training (Sec. 5.8): iterations with doubling sample counts,   */
/* training stopped at a share of the budget, the guide fitted from the last  */
/* iteration's samples only.  Host-side state machine; the caller owns the    */
/* clock and the sample batches.                                              */
/* ------------------------------------------------------------------------ */

#define MPG_TRAIN 0
#define MPG_RENDER 1

typedef struct {
  double budget;          /* total budget (any unit of time) */
  double train_fraction;  /* share of the budget for training (0.3) */
  int64_t base_samples;   /* samples of iteration 0; iteration k takes base 2^k */
} mpg_train_plan;

typedef struct {
  int32_t phase;      /* MPG_TRAIN or MPG_RENDER */
  int32_t iteration;  /* current training iteration */
  int64_t target;     /* its sample count (base 2^iteration) */
  int64_t done;       /* samples gathered in it so far */
  int32_t refit;      /* set by mpg_train_step: fit the guide now from the samples of the iteration that
                         just ended (then gather the next iteration's samples afresh) */
} mpg_train_state;

/* Starts training (MPG_RENDER at once when train_fraction is 0). */
mpg_status mpg_train_init(const mpg_train_plan* plan, mpg_train_state* state);
/* Records `batch` more samples of the current iteration at time `elapsed`
 * (since the start of the budget) and advances the schedule: once elapsed
 * reaches train_fraction budget, training ends (phase MPG_RENDER, refit for
 * the last iteration); when the iteration has its target count and less than
 * half of the training budget is used, refit and start the next iteration
 * with twice the samples; otherwise the current iteration goes on
 * (gathering past its target once half of the training budget is used). */
mpg_status mpg_train_step(const mpg_train_plan* plan, mpg_train_state* state, int64_t batch, double elapsed);

#ifdef __cplusplus
}
#endif
#endif /* MPG_H */
