/*
 * gavis.h -- C ABI of the MI355X (gfx950) visibility-field path of GAVIS
 * ("Uncertainty-driven 3D Gaussian Splatting Active Mapping via Anisotropic
 * Visibility Field").
 *
 * Three calls follow the paper's statement of the problem:
 *   vf_build         builds the per-Gaussian SH coefficients gamma of the
 *                    anisotropic visibility field from the training views
 *                    (Alg. 2 per view, accumulated as in Alg. 3, eq. vis_gamma);
 *   vf_query_views   queries gamma in each candidate view's direction with the
 *                    AM-GM bound (Alg. 1 / Alg. 4, eq. vis_bound) and
 *                    rasterises the per-pixel entropy bound (Alg. 6, eq.
 *                    alpha_comp, eq. huber) into one score per view (eq. id,
 *                    with the spatial-correlation correction taken as zero);
 *   select_next_view picks the candidate with the largest score (eq. i_gain).
 *
 * Conventions shared by every call
 *   - All data pointers named "device" point to GPU memory owned by the
 *     caller.  The library never frees them and keeps no reference to them
 *     after the call returns (a captured graph, see gv_uq_params.use_graph,
 *     keeps the pointers it was captured with until they change).
 *   - Camera: pinhole, x_cam = R x_world + t (R row major), image x right,
 *     y down, z forward; pixel (i, j) is sampled at (i + 0.5, j + 0.5).
 *   - Gaussians: SoA, means [n][3], scales [n][3] (linear, not log),
 *     quats [n][4] as (w, x, y, z) (normalised inside), opacity [n] in [0, 1].
 *   - gamma is planar: coefficient k of Gaussian g at gamma[k * n + g],
 *     k = l^2 + l + m for the real SH basis Y_lm (world frame, theta from +z),
 *     K = (L + 1)^2 coefficients, L = sh_degree <= GV_MAX_SH_DEGREE.
 *   - vf_build and vf_query_views only enqueue work on `hip_stream`
 *     (a hipStream_t, NULL for the default stream); outputs are valid once
 *     the stream reaches that point.  The *_workspace_size calls and
 *     select_next_view synchronise the stream.
 *   - Errors: calls return a negative gv_status and never throw;
 *     gv_last_error() describes the last failure on the calling thread.
 *   - Threading: one context per host thread, or serialise calls on it.
 *     Calls on different streams need different workspaces.
 */
#ifndef GAVIS_H
#define GAVIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GV_MAX_SH_DEGREE 3
#define GV_MAX_IMAGE_SIDE 16384

typedef enum {
    GV_OK = 0,
    GV_ERR_INVALID_ARG = -1,    /* bad pointer, size or parameter */
    GV_ERR_OUT_OF_MEMORY = -2,  /* a small context-owned buffer could not be allocated */
    GV_ERR_HIP = -3,            /* a HIP runtime call failed */
    GV_ERR_CAPACITY = -4,       /* the workspace is smaller than the work needs */
    GV_ERR_UNSUPPORTED = -5     /* valid but not supported (e.g. sh_degree > 3) */
} gv_status;

typedef enum { GV_F32 = 0, GV_F16 = 1, GV_BF16 = 2 } gv_dtype;

typedef struct gv_context gv_context;

/* One pinhole camera (host memory). */
typedef struct {
    float R[9];                 /* world -> camera rotation, row major */
    float t[3];                 /* world -> camera translation */
    float fx, fy, cx, cy;       /* focal lengths and principal point, pixels */
    int32_t width, height;      /* 1 .. GV_MAX_IMAGE_SIDE */
} gv_camera;

/* A resident 3DGS scene (device memory).  For GV_F16 / GV_BF16 storage the
 * means are half offsets from per-block FP32 anchors: mean of Gaussian g =
 * anchors[g / anchor_block] + means[g]; scales, quats and opacity are plain
 * half values.  The last n_virtual Gaussians are virtual particles of the
 * visibility-field density control: their queried visibility is 0. */
typedef struct {
    int64_t n;
    int64_t n_virtual;
    gv_dtype dtype;
    const void *means;
    const void *scales;
    const void *quats;
    const void *opacity;
    const float *anchors;       /* [ceil(n / anchor_block)][3], NULL for GV_F32 */
    int32_t anchor_block;
} gv_gaussians;

/* Parameters of the visibility-field construction (Alg. 2 / Alg. 3). */
typedef struct {
    int32_t sh_degree;          /* L, 0..3; the paper uses 2 */
    float kappa;                /* vMF concentration; the paper uses 1 */
    float eps_T;                /* transmittance cutoff, 1e-4 */
    float znear;                /* Gaussians with camera z <= znear are not in view */
    float lowpass;              /* dilation added to the 2D covariance diagonal, px^2 */
    float cut;                  /* overlap predicate: Mahalanobis^2 <= cut (9) */
    int32_t views_per_pass;     /* training views rasterised per pass, 0 = all */
    int32_t accumulate;         /* 0: gamma = result, 1: gamma += result */
} gv_vf_params;

/* Parameters of the uncertainty rasterisation (Alg. 6). */
typedef struct {
    float beta;                 /* opacity reliability, 0.5 */
    float o0;                   /* prior opacity of invisible particles, 0.15 */
    float half_logdet_Q0;       /* 1/2 log|Q0|, 0 for Q0 = I */
    float half_logdet_Qc;       /* 1/2 log|Q_c| of the constant colour covariance */
    float eps_T;                /* transmittance cutoff, 1e-4 */
    float znear;
    float lowpass;
    float cut;
    int32_t write_maps;         /* 1: also write the per-pixel entropy maps */
    int32_t use_graph;          /* 1: capture the launch sequence in a hipGraph and
                                   replay it while shapes and pointers repeat */
    int32_t count_pairs;        /* 1: count composited (pixel, Gaussian) pairs, read
                                   back by gv_workspace_check (costs one add per pair) */
    int32_t write_depth;        /* 1 (with write_maps): maps also receives each pixel's
                                   expected depth under the same compositing weights,
                                   sum w* z / sum w* (0 where nothing contributes), the
                                   per-pixel depth of the spatial-correlation correction
                                   of eq. id; it follows the entropy maps in the same
                                   packing, so maps then holds 2 x total pixels floats */
} gv_uq_params;

/* Workspace plan, filled by the *_workspace_size calls.  The caller
 * allocates `bytes` of device memory and passes both to the compute call.
 * max_records / max_instances may be raised to leave slack for other
 * camera sets; `bytes` must then be recomputed with gv_workspace_bytes. */
typedef struct {
    size_t bytes;
    int64_t max_records;        /* (Gaussian, view) pairs kept after culling */
    int64_t max_instances;      /* (tile, record) pairs after binning */
    int64_t n;                  /* Gaussians the plan was made for */
    int32_t n_views;            /* views per pass the plan was made for */
    int32_t total_tiles;        /* largest per-pass tile count */
    int64_t total_pixels;       /* largest per-pass pixel count */
    int32_t kind;               /* 0 build, 1 query, 2 density control */
    int32_t sh_degree;
    int32_t emit_mode;          /* how instances find their output offsets: 1 a scan of
                                   the records' tile counts, carried into depth order by
                                   the depth sort; 2 a single-pass scan with decoupled
                                   look-back inside the emission (one read of each
                                   record's binning line); 0 chosen from the sizes (2 when
                                   the binning lines exceed the last-level cache and
                                   records average at most 4 tiles).  The sizing calls
                                   fill in the choice; results do not depend on it. */
    int32_t reserved;
} gv_workspace;

/* Context: small host state, a few bytes of device counters, cached graphs.
 * `device` is the HIP device ordinal the context works on. */
gv_status gv_create(int device, gv_context **out);
void gv_destroy(gv_context *ctx);

/* Message for the last failure on this thread ("" if none).  The pointer is
 * valid until the next call on the same thread. */
const char *gv_last_error(void);

/* Paper defaults (see the field comments). */
void gv_default_vf_params(gv_vf_params *p);
void gv_default_uq_params(gv_uq_params *p);

/* Workspace for vf_build over `n_train` training views (host array).  Runs
 * the culling and binning counts on the GPU (synchronises hip_stream) and
 * fills `plan` with exact capacities for these inputs. */
gv_status vf_build_workspace_size(gv_context *ctx, const gv_gaussians *g, const gv_camera *train,
                                  int32_t n_train, const gv_vf_params *params, gv_workspace *plan,
                                  void *hip_stream);

/* Alg. 3 over the training views: gamma (device, planar [K][n], dtype
 * gamma_dtype) = sum over views of v_p[g] a_l Y_k(d_p^g), with v_p from Alg. 2
 * computed by rasterising each view (no per-view host synchronisation).  With
 * params->accumulate = 1 the result is added to gamma (gamma is linear in the
 * view set, so a field can be extended with new views).  Returns
 * GV_ERR_CAPACITY (after synchronising) when the workspace was too small for
 * these inputs; gamma is then unspecified. */
gv_status vf_build(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                   const gv_vf_params *params, void *gamma, gv_dtype gamma_dtype,
                   const gv_workspace *plan, void *workspace, void *hip_stream);

/* Multi-view visibility of the visibility-field density control (Alg. 5):
 * visibility[g] = 1 - prod over the training views of (1 - v_p[g]), with
 * v_p[g] the single-view particle visibility of Alg. 2 (device, float [n]).
 * Virtual particles are passed as ordinary Gaussians with opacity 0: they are
 * measured but never occlude.  Uses the workspace plan of vf_build (same
 * scene, views and params).  Enqueue only, except between passes when
 * views_per_pass splits the views (then it synchronises to check capacity).
 * The caller keeps the virtual particles with visibility <= eps_v (0.95). */
gv_status vf_multiview_visibility(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                                  const gv_vf_params *params, float *visibility, const gv_workspace *plan,
                                  void *workspace, void *hip_stream);

/* Visibility-field density control (Alg. 5): virtual particles fill the
 * scene's box at density rho; those the training views see at most eps_v
 * (multi-view visibility 1 - prod_p (1 - v_p), as vf_multiview_visibility)
 * are kept as invisible space.  N_virt = floor(rho * volume of [lo, hi]);
 * particle i sits at lo + u_i (hi - lo), formed in FP64 and stored in FP32,
 * with isotropic scale s, (4/3) pi s^3 rho = 1 + eta, identity rotation and
 * opacity 0 (measured, never occluding).  The paper uses rho = 100, eta = 0.5,
 * eps_v = 0.95. */
typedef struct {
    float lo[3], hi[3];         /* box corners (world units) */
    float rho;                  /* particles per unit volume */
    float eta;                  /* overlap of the particles' 1-sigma balls */
    float eps_v;                /* keep particles with visibility <= eps_v */
} gv_density_params;

/* Alg. 5's particle count and scale for these parameters (host arithmetic
 * only): *n_virt = N_virt, *scale = s rounded to FP32 (either may be NULL).
 * GV_ERR_INVALID_ARG for an empty box or parameters out of range. */
gv_status vf_virtual_particle_count(const gv_density_params *dp, int64_t *n_virt, float *scale);

/* Workspace for vf_density_control.  g (device, FP32, n_virtual = 0) holds
 * the real Gaussians in rows 0 .. n_real - 1 and room for the particles after
 * them: g->n must be n_real + N_virt.  u: device float [n_draw][3] uniform
 * draws in [0, 1), n_draw >= N_virt (the random numbers Alg. 5 consumes).
 * Writes the particles into rows n_real .. of g's arrays (the arrays must be
 * writable), runs the counting pass on the GPU over everything (synchronises
 * hip_stream) and fills plan; *n_virt (host, optional) receives N_virt.
 * GV_ERR_INVALID_ARG when the counts, the box or the draws do not fit,
 * GV_ERR_UNSUPPORTED for half-precision attributes. */
gv_status vf_density_control_workspace_size(gv_context *ctx, const gv_gaussians *g, int64_t n_real,
                                            const float *u, int64_t n_draw, const gv_density_params *dp,
                                            const gv_camera *train, int32_t n_train, const gv_vf_params *params,
                                            gv_workspace *plan, int64_t *n_virt, void *hip_stream);

/* Alg. 5 on the GPU: (re)writes the particles into rows n_real .. of g as the
 * sizing call does, measures the multi-view visibility of all g->n rows
 * (visibility: device float [g->n]), and keeps the particles with visibility
 * <= eps_v: kept (device int32 [N_virt]) receives their indices (0-based
 * among the particles, ascending) and *n_kept (host) their number; their
 * attributes are packed into rows n_real .. n_real + *n_kept - 1 of g, so the
 * first n_real + *n_kept rows, with n_virtual = *n_kept, are the scene the
 * query takes (its last n_virtual Gaussians have V = 0).  Synchronises
 * hip_stream.  Errors as the sizing call, GV_ERR_CAPACITY when the workspace
 * was too small for these inputs. */
gv_status vf_density_control(gv_context *ctx, const gv_gaussians *g, int64_t n_real, const float *u, int64_t n_draw,
                             const gv_density_params *dp, const gv_camera *train, int32_t n_train,
                             const gv_vf_params *params, float *visibility, int32_t *kept, int64_t *n_kept,
                             const gv_workspace *plan, void *workspace, void *hip_stream);

/* Per-view single-view visibility, the input of the exact validation mode:
 * view_vis[p * n + g] = v_p[g] (device, float [n_train][n]), the visibility of
 * Alg. 2 that vf_build weights each view's vMF lobe with (eq. vis_p without
 * its directional factor); 0 where view p culls g or reaches none of its
 * pixels.  train_centres (device, float [n_train][3], optional: NULL skips it)
 * receives the camera centres C_p = -R_p^T t_p.  Uses the workspace plan of
 * vf_build (same scene, views and params).  Enqueue only, except between
 * passes when views_per_pass splits the views (then it synchronises to check
 * capacity). */
gv_status vf_view_visibility(gv_context *ctx, const gv_gaussians *g, const gv_camera *train, int32_t n_train,
                             const gv_vf_params *params, float *view_vis, float *train_centres,
                             const gv_workspace *plan, void *workspace, void *hip_stream);

/* Workspace for vf_query_views over `n_cand` candidate views. */
gv_status vf_query_workspace_size(gv_context *ctx, const gv_gaussians *g, const gv_camera *cand,
                                  int32_t n_cand, const gv_uq_params *params, int32_t sh_degree,
                                  gv_workspace *plan, void *hip_stream);

/* Alg. 4 + Alg. 6 for every candidate view, all views in one launch
 * sequence.  gamma: device, planar [K][n] of gamma_dtype, K = (sh_degree+1)^2;
 * n_train = |P| of the AM-GM bound (0 gives V = 0 everywhere).
 * scores: device [n_cand] float, sum over the view's pixels of the entropy
 * bound.  maps: device float, optional (NULL, or params->write_maps = 0):
 * the per-pixel maps packed view after view, row major, view v starting at
 * the sum of width*height of views < v (followed by the expected-depth maps
 * when params->write_depth is set).  Enqueue only; a capacity overflow
 * is reported by gv_workspace_check (the scores of an overflowed call are
 * NaN). */
gv_status vf_query_views(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                         int32_t sh_degree, int64_t n_train, const gv_camera *cand, int32_t n_cand,
                         const gv_uq_params *params, float *scores, float *maps,
                         const gv_workspace *plan, void *workspace, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture setup, tight serving loops, harnesses that forbid hipMalloc):
 * vf_query_views without a caller workspace.  The workspace is a static
 * device array of GV_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, part of the
 * library's code object and held until the process ends; the call allocates
 * nothing (no hipMalloc, no graph; the host view table was reserved by
 * gv_create).  It runs the sizing pass of vf_query_workspace_size into that
 * array and synchronises hip_stream once to read it, then enqueues the query
 * as vf_query_views does.  Arguments, outputs and results as vf_query_views;
 * params->use_graph must be 0 (GV_ERR_INVALID_ARG otherwise).  Errors:
 * GV_ERR_CAPACITY when the views' workspace exceeds GV_NOALLOC_SCRATCH_BYTES
 * or n_cand exceeds GV_NOALLOC_MAX_VIEWS (nothing is enqueued then);
 * GV_ERR_HIP if the array's device address could not be taken at gv_create.
 * Every call on a GPU shares that GPU's array and leaves its contents
 * behind (each call clears what it needs cleared): calls that overlap on
 * one GPU -- from two threads, or on two streams before the first has
 * finished -- race and give undefined results; order them on one stream or
 * synchronise between them. */
#define GV_NOALLOC_SCRATCH_BYTES (64u << 20)
#define GV_NOALLOC_MAX_VIEWS 4096
gv_status vf_query_views_noalloc(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                                 int32_t sh_degree, int64_t n_train, const gv_camera *cand, int32_t n_cand,
                                 const gv_uq_params *params, float *scores, float *maps, void *hip_stream);

/* vf_query_views with a per-Gaussian colour covariance in place of the
 * constant Q_c (Appendix, integration with FisherRF; the hook through which
 * a radiance-field uncertainty method refines the colour term of eq. huber).
 * The colour is linear in its SH coefficients, so with independent
 * coefficients channel k of Gaussian g seen in direction d has variance
 * Q_k(d) = sum_j Y_j(d)^2 var_gjk, and the record's colour constant becomes
 * 1/2 sum_k log max(Q_k(d), 1e-30) + 3/2 log(2 pi e).
 * color_var: device float, planar [3][Kc][n]: the variance of colour SH
 * coefficient j (index l^2 + l + m, real basis as for gamma) in channel k of
 * Gaussian g at color_var[(k * Kc + j) * n + g], Kc = (color_sh_degree+1)^2,
 * color_sh_degree 0..3.  params->half_logdet_Qc is not used.  Other
 * arguments, outputs and errors as vf_query_views. */
gv_status vf_query_views_color(gv_context *ctx, const gv_gaussians *g, const void *gamma, gv_dtype gamma_dtype,
                               int32_t sh_degree, int64_t n_train, const float *color_var, int32_t color_sh_degree,
                               const gv_camera *cand, int32_t n_cand, const gv_uq_params *params, float *scores,
                               float *maps, const gv_workspace *plan, void *workspace, void *hip_stream);

/* Validation mode of vf_query_views: the same Alg. 6 rasterisation and
 * scores, with each Gaussian's visibility in direction d = camera -> Gaussian
 * taken exactly from the per-view visibilities instead of from the field and
 * its AM-GM bound: V = 1 - prod_p (1 - v_p exp(kappa (d . d_p - 1))) (eq.
 * vis_all with eq. vis_p), d_p the unit direction from training camera p.
 * The gap to vf_query_views measures the AM-GM and SH truncation error.
 * view_vis: device float [n_train][n] and train_centres: device float
 * [n_train][3], both as written by vf_view_visibility; kappa as in the
 * field.  Costs O(n_train) per (Gaussian, candidate view) record.  Any query
 * plan for these Gaussians and candidate views serves (its sh_degree is not
 * used).  Virtual particles get V = 0; a training camera at a Gaussian's
 * centre contributes nothing.  Enqueue only, as vf_query_views. */
gv_status vf_query_views_exact(gv_context *ctx, const gv_gaussians *g, const float *view_vis,
                               const float *train_centres, int32_t n_train, float kappa, const gv_camera *cand,
                               int32_t n_cand, const gv_uq_params *params, float *scores, float *maps,
                               const gv_workspace *plan, void *workspace, void *hip_stream);

/* Synchronises hip_stream and reads the workspace's status words of the last
 * call (the last pass of a multi-pass build): out[0] records, out[1]
 * instances, out[2] overflow flags (nonzero if a capacity was exceeded),
 * out[3] composited (pixel, Gaussian) pairs -- always counted by vf_build,
 * counted by vf_query_views when params->count_pairs is set.  Returns
 * GV_ERR_CAPACITY on overflow. */
gv_status gv_workspace_check(gv_context *ctx, const gv_workspace *plan, const void *workspace,
                             int64_t out[4], void *hip_stream);

/* Launch schedule of the blend kernels, chosen per workload class by the
 * autotuner, for the VF CONST (vis_) and VF QUERY (uq_) blends:
 *   *_batch  depth-ordered records a tile stages into LDS per batch (64, 128
 *            or 256): larger batches need fewer barriers, smaller ones use
 *            less LDS (more resident workgroups);
 *   *_order  which tile each workgroup blends (0: workgroup b takes tile b;
 *            1: the eight XCDs, which take the workgroups in turn, each take
 *            a contiguous run of tiles, so that neighbouring tiles, which
 *            share most of their records, share an L2 cache; 2: the tiles of
 *            all views by decreasing list length, sorted on the device before
 *            the blend, so that the longest tiles start first; 3 and 4:
 *            persistent workgroups, about one per resident slot, take tiles
 *            from a queue through an atomic counter until it is empty, in
 *            tile order (3) or by decreasing list length (4)).
 * Results do not depend on the choice (VF CONST's float atomics may add in
 * another order).  Defaults: VF CONST 64 records, order 2; VF QUERY 256
 * records, order 0. */
typedef struct {
    int32_t vis_batch;
    int32_t uq_batch;
    int32_t vis_order;
    int32_t uq_order;
} gv_tuning;
gv_status gv_set_tuning(gv_context *ctx, const gv_tuning *t);
gv_status gv_get_tuning(const gv_context *ctx, gv_tuning *t);

/* Stage timing for measurement.  While enabled, the context records a pair
 * of HIP events around each stage of every call on the call's stream.
 * gv_profile_read synchronises `hip_stream`, adds the elapsed times of all
 * completed stages into ms[stage] and their launch counts into calls[stage]
 * (arrays of GV_PROFILE_STAGES entries, caller-owned host memory) and clears
 * the accumulators.  gv_profile_stage_name gives the stage names. */
#define GV_PROFILE_STAGES 9
gv_status gv_profile_enable(gv_context *ctx, int32_t on);
gv_status gv_profile_read(gv_context *ctx, double *ms, int64_t *calls, void *hip_stream);
const char *gv_profile_stage_name(int32_t stage);

/* Bytes needed for a plan whose capacities the caller edited. */
size_t gv_workspace_bytes(const gv_workspace *plan);

/* Next-best view (eq. i_gain): index of the largest of the n device scores,
 * lowest index on exact ties, NaN never wins (-1 if all are NaN).  Runs a
 * device argmax that writes the index into pinned host memory of the
 * context, synchronises the stream and stores it in `*best` (host). */
gv_status select_next_view(gv_context *ctx, const float *scores, int32_t n, int32_t *best, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* GAVIS_H */
