/*
 * shvis.h - C ABI of the MI355X (gfx950) SH soft-shadow library.
 *
 * Method: "Efficient and Differentiable Shadow Computation for Inverse
 * Problems" (Lyu et al., ICCV 2021).  Occluders are spheres (c_i, r_i); for a
 * receiver x with normal n(x) and albedo a(x), under lighting SH vector L:
 *
 *   visibility  V(x) = exp*( sum_i f_i(x) )                    Sec. 3.3.2
 *       f_i = log-visibility of sphere i: -eps on the cone of half-angle
 *             asin(r_i / |c_i - x|) around (c_i - x)/|c_i - x|, 0 elsewhere
 *             (Eq. 13, eps = 3), projected about z analytically and rotated
 *             to that direction; exp* is the SH exponential by DC isolation,
 *             scaling by 2^-k, optimal linear approximation and k truncated
 *             squarings with the triple product of Eqs. 6-7;
 *   radiance    B(x) = a(x) * ( L . (V(x) * H(x)) )            Eq. 8
 *       H(x) = rotated clamped cosine max(n . w, 0) (Eqs. 10-11).
 *
 * Conventions shared by every entry point
 *   - SH vectors have N = n_bands^2 coefficients, index i = l*l + l + m
 *     (Sec. 3.2), real orthonormal basis without Condon-Shortley phase
 *     (y_lm ~ cos(m phi) for m > 0, sin(|m| phi) for m < 0).
 *   - Every array pointer is a DEVICE pointer owned by the caller; FP32.
 *     Per-receiver arrays are structure-of-arrays: points / normals are
 *     [3][P] (all x, then all y, then all z), SH arrays are [N][P]
 *     (coefficient-major), albedo and radiance are [P].  Spheres are [S][4]
 *     (cx, cy, cz, r), 16-byte aligned.  Lighting is [N].
 *   - Outputs are overwritten, never accumulated.  An optional output may
 *     be NULL; it is then not computed.
 *   - Work is enqueued on `stream` (0 = the null stream); no entry point
 *     allocates device memory, frees it, or synchronises the host.  Scratch
 *     memory comes from the caller's workspace `ws` of `ws_bytes` bytes
 *     (256-byte aligned), sized by shv_workspace_bytes().
 *   - P = 0 is a valid no-op; S = 0 means "no occluders" (V = sqrt(4 pi) e_0).
 *   - Errors: validation failures return before any launch; a failed launch
 *     returns SHV_ERR_HIP.  shv_last_error() gives the thread's last message.
 *     No C++ exception crosses this boundary.
 *   - Results are deterministic: reductions run in a fixed order, so two
 *     identical calls give bit-identical outputs.
 */
#ifndef SHVIS_H
#define SHVIS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t shv_status;
#define SHV_OK 0
#define SHV_ERR_INVALID_ARG (-1)     /* NULL required pointer, negative size, misalignment */
#define SHV_ERR_UNSUPPORTED (-2)     /* n_bands outside [1, 8], n_squarings outside [0, 12] */
#define SHV_ERR_WORKSPACE (-3)       /* ws_bytes smaller than shv_workspace_bytes() */
#define SHV_ERR_NOT_INITIALIZED (-4) /* shv_init() not called for the current device */
#define SHV_ERR_HIP (-5)             /* a HIP runtime call or kernel launch failed */

#define SHV_MAX_BANDS_API 8
#define SHV_MAX_SQUARINGS 12
#define SHV_MAX_TAYLOR_ORDER 8   /* K of SHV_FLAG_EXP_TAYLOR */
#define SHV_RANGE_ALIGN 256   /* receiver-range granularity of batched calls */
#define SHV_MAX_CHANNELS 4    /* colour channels of one multi-channel shading call */
#define SHV_MAX_ENVMAP_ROWS 65536     /* environment-map rows (polar samples) */
#define SHV_MAX_ENVMAP_COLS 1048576   /* environment-map columns (azimuth samples) */

/* Method parameters.  n_bands: number of SH bands n (l < n), the paper uses
 * n = 8 (Sec. 3.2).  n_squarings: k, the number of squarings of the SH
 * exponential (fixed per call; 4 by default).  eps: depth of the log-blocker,
 * log V' = -eps inside a sphere's cone (Eq. 13; the paper uses 3).  flags:
 * 0 or one of the SHV_FLAG_* values below.  The first two select a kernel
 * variant, never the result (both variants are bitwise identical); the
 * quadrature and product flags select a different way of forming V. */
#define SHV_FLAG_EXP_ONE_WAVE 1u   /* exponential: one receiver per lane, one wave per 64 receivers */
#define SHV_FLAG_EXP_FOUR_WAVES 2u /* exponential: each receiver's squarings spread over 4 waves
                                      (without a layout flag the library picks by band count and
                                      size; both layouts give identical bits) */
#define SHV_FLAG_EXP_QUADRATURE 4u /* a different exponential (this flag changes the result): the
                                      projection of the pointwise exponential, V = exp(c) sum_q w_q
                                      exp(Fhat~(w_q)) y(w_q), over the product rule of degree 8n - 1
                                      (4n Gauss-Legendre nodes in z times 8n azimuths), on MFMA.
                                      n_squarings is unused.  Only sh_visibility_forward /
                                      sh_visibility_backward accept it; saved then holds F [N][P]. */
#define SHV_FLAG_EXP_PRODUCT 8u    /* V without logarithms (this flag changes the result): the chain of
                                      truncated SH products of Eq. 12, V = V'_1 * V'_2 * ... * V'_S,
                                      left to right in sphere order, of the projected floored
                                      blockers of Eq. 13 (e^-eps on each sphere's cone, 1 elsewhere;
                                      a large eps gives Eq. 12's binary blockers).  Costs one Gaunt
                                      product per pair forward and three in the adjoint (which runs
                                      the chain again to record its states in the workspace,
                                      S * N * P floats).  n_squarings is unused; no other flag may
                                      be set.  Only sh_visibility_forward / sh_visibility_backward
                                      accept it; nothing is saved and saved may be NULL. */
#define SHV_FLAG_EXP_TAYLOR 16u    /* a different exponential (this flag changes the result): the
                                      scaling-and-squaring scheme with the linear approximation
                                      replaced by the Taylor series of exp truncated after the
                                      term of degree K, E_0 = sum_{j <= K} G^{*j} / j! with
                                      truncated products, then the k squarings.  K (1 ..
                                      SHV_MAX_TAYLOR_ORDER) goes into the flags with
                                      SHV_FLAG_EXP_TAYLOR_ORDER(K); no other flag may be set.  Only
                                      sh_visibility_forward / sh_visibility_backward accept it;
                                      saved then holds (1 + (k + K) N) * P values. */
#define SHV_FLAG_EXP_TAYLOR_ORDER(K) (((uint32_t)(K) & 15u) << 8)
typedef struct shv_params {
  int32_t n_bands;
  int32_t n_squarings;
  float eps;
  uint32_t flags;
} shv_params;

/* Makes `device` current and prepares the library for it.  Idempotent and
 * thread-safe.  Returns SHV_ERR_HIP if the device is unusable. */
shv_status shv_init(int device);

/* Human-readable text of a status code (static storage). */
const char* shv_status_string(shv_status s);

/* The calling thread's last error message ("" if none; thread-local storage). */
const char* shv_last_error(void);

/* Number of FP32 values the forward saves for the backward, per call:
 * (1 + k * N) * P  (the DC value c and E_0 .. E_{k-1} of the exponential);
 * with SHV_FLAG_EXP_QUADRATURE the larger of that and N * P (F itself); with
 * SHV_FLAG_EXP_PRODUCT 0; with SHV_FLAG_EXP_TAYLOR (1 + (k + K) N) * P. */
int64_t shv_saved_floats(int64_t P, const shv_params* prm);

/* Workspace bytes that every entry point below needs for P receivers and S
 * spheres (the maximum over all of them, so one buffer serves a whole
 * forward + backward).  Returns 0 for invalid parameters. */
size_t shv_workspace_bytes(int64_t P, int64_t S, const shv_params* prm);

/* Visibility in SH space (Sec. 3.3.2: per-sphere log-cap projected about z
 * and rotated to the sphere direction, summed, exponentiated).
 *   points  [3][P]  receiver positions x
 *   spheres [S][4]  occluders (cx, cy, cz, r), r >= 0
 *   vis     [N][P]  out: V(x)
 *   saved   out: state for sh_visibility_backward, shv_saved_floats(P, prm)
 *           FP32 values ((1 + k N) P for the default exponential); may be
 *           NULL when no backward will follow (saved_bytes is then ignored)
 *   saved_bytes  size of the saved buffer in bytes; a non-NULL saved smaller
 *           than 4 shv_saved_floats(P, prm) bytes is refused with
 *           SHV_ERR_WORKSPACE before anything is launched
 * A receiver inside a sphere (r >= |c - x|) sees a hemisphere cap; a sphere
 * centred exactly on the receiver contributes nothing. */
shv_status sh_visibility_forward(const float* points, int64_t P, const float* spheres, int64_t S,
                                 const shv_params* prm, float* vis, float* saved, size_t saved_bytes,
                                 void* ws, size_t ws_bytes, hipStream_t stream);

/* Diffuse SH shading B = a (L . (V * H)) (Eq. 8), H the clamped cosine
 * rotated to n / |n| (Eqs. 10-11).
 *   vis [N][P], normals [3][P] (need not be unit), albedo [P], light [N]
 *   radiance [P] out. */
shv_status sh_shade(const float* vis, const float* normals, const float* albedo, const float* light,
                    int64_t P, const shv_params* prm, float* radiance, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* Adjoint of sh_shade for the cotangent grad_radiance [P] (the gradients of
 * Sec. 3.5's objective with respect to L and a, and through H to n):
 *   grad_vis [N][P], grad_normals [3][P], grad_albedo [P], grad_light [N]
 * (any may be NULL).  grad_light is summed over all receivers. */
shv_status sh_shade_backward(const float* grad_radiance, const float* vis, const float* normals,
                             const float* albedo, const float* light, int64_t P,
                             const shv_params* prm, float* grad_vis, float* grad_normals,
                             float* grad_albedo, float* grad_light, void* ws, size_t ws_bytes,
                             hipStream_t stream);

/* Several colour channels lit through one visibility (Eq. 8 once per channel:
 * B_c = a_c (L_c . (V * H)), the usual RGB setting of the paper's renders).
 *   channels  C in [1, SHV_MAX_CHANNELS]
 *   vis [N][P], normals [3][P] as for sh_shade
 *   albedo [C][P], light [C][N], radiance [C][P] out
 * Channel c's radiance is bitwise what sh_shade gives for albedo[c] and
 * light[c].  ws must hold shv_channels_workspace_bytes(P, C, prm) bytes (0 is
 * returned for invalid arguments). */
size_t shv_channels_workspace_bytes(int64_t P, int channels, const shv_params* prm);
shv_status sh_shade_channels(const float* vis, const float* normals, const float* albedo, const float* light,
                             int channels, int64_t P, const shv_params* prm, float* radiance, void* ws,
                             size_t ws_bytes, hipStream_t stream);

/* Adjoint of sh_shade_channels for the cotangent grad_radiance [C][P]:
 *   grad_albedo [C][P], grad_light [C][N] (summed over receivers): channel c
 *   bitwise as sh_shade_backward for that channel alone;
 *   grad_vis [N][P], grad_normals [3][P]: summed over the channels, since V
 *   and n are shared (channel-order sum of the per-channel cotangents).
 * Any output may be NULL.  Same workspace as sh_shade_channels. */
shv_status sh_shade_channels_backward(const float* grad_radiance, const float* vis, const float* normals,
                                      const float* albedo, const float* light, int channels, int64_t P,
                                      const shv_params* prm, float* grad_vis, float* grad_normals,
                                      float* grad_albedo, float* grad_light, void* ws, size_t ws_bytes,
                                      hipStream_t stream);

/* Distant lighting from an environment map (Eq. 9: L_i is the integral of the
 * map times y_i over the sphere), by summation over the pixels of an
 * equirectangular map.
 *   image [C][H][W]: row r covers polar angles [r, r + 1] pi / H measured
 *     from +z, column x azimuths [x, x + 1] 2 pi / W from +x towards +y;
 *     each pixel is sampled at its centre and weighted by its exact solid
 *     angle (cos th_r - cos th_{r+1}) 2 pi / W (the weights sum to 4 pi)
 *   light [C][N] out (N = n_bands^2; eps, n_squarings and flags are unused)
 *   1 <= C <= SHV_MAX_CHANNELS, 0 <= H <= SHV_MAX_ENVMAP_ROWS,
 *   0 <= W <= SHV_MAX_ENVMAP_COLS; an empty map gives L = 0.
 * Rows are summed in row order (deterministic).  ws must hold
 * shv_envmap_workspace_bytes(C, H, W, prm) bytes (0 for invalid arguments). */
size_t shv_envmap_workspace_bytes(int channels, int64_t H, int64_t W, const shv_params* prm);
shv_status sh_envmap_project(const float* image, int channels, int64_t H, int64_t W, const shv_params* prm,
                             float* light, void* ws, size_t ws_bytes, hipStream_t stream);

/* ---- Scene parameterisation upstream of the spheres (Sec. 3.3.1, Sec. 3.5) ----
 * The sphere centres g_k are the nodes of an embedded deformation graph:
 * sphere k is attached to its K nearest template vertices and carries an
 * axis-angle rotation a_k (rotation by |a_k| about a_k / |a_k|, Rodrigues'
 * formula) and a translation t_k; a global rigid pose (a_0, t_0) follows:
 *   y_j = sum_k w_jk (R_k (v_j - g_k) + g_k + t_k) + (1 - sum_k w_jk) v_j
 *   points  x_j = R_0 y_j + t_0
 *   normals n_j = R_0 (sum_k w_jk R_k m_j + (1 - sum_k w_jk) m_j)  (not renormalised)
 *   spheres c_k = R_0 (g_k + t_k) + t_0, radius unchanged.
 * params [S + 1][6]: row k < S is (a_k, t_k), row S is (a_0, t_0).
 * Weights: u_jk = (1 - |v_j - g_k| / d_k)^2, d_k the distance from g_k to its
 * (K+1)-th nearest vertex (K-th when K = P), normalised over the spheres
 * attached to vertex j (0 when that sum is 0). */
typedef struct shv_deform_graph {
  const float* vertices;   /* [3][P] template vertex positions v_j (device) */
  const float* normals;    /* [3][P] template normals m_j (device) */
  const float* spheres;    /* [S][4] template spheres (g_k, r_k) (device) */
  const int32_t* vert_ptr; /* [P + 1] per-vertex ranges of the two arrays below (device) */
  const int32_t* vert_sph; /* [S K] spheres attached to each vertex, ascending (device) */
  const float* vert_w;     /* [S K] their normalised weights w_jk (device) */
  const int32_t* sph_vert; /* [S][K] the vertices attached to each sphere, nearest first (device) */
  const float* sph_w;      /* [S][K] their normalised weights (device) */
  int64_t P;
  int64_t S;
  int32_t K;
} shv_deform_graph;

/* Builds the attachment on the host (a one-time preprocessing of the
 * template): vertices [3][P] and spheres [S][4] are host arrays; the outputs
 * are host arrays of the sizes above (vert_ptr P + 1, vert_sph / vert_w /
 * sph_vert / sph_w S K).  Distances are compared as squared FP64 distances of
 * the FP32 inputs, ties to the lower vertex index.  1 <= K <= P, S >= 1,
 * S K < 2^31. */
shv_status shv_deform_graph_build(const float* vertices, int64_t P, const float* spheres, int64_t S, int32_t K,
                                  int32_t* vert_ptr, int32_t* vert_sph, float* vert_w, int32_t* sph_vert,
                                  float* sph_w);

/* ------------------------------------------------------------------ rasteriser
 * Rendering the shaded mesh into an image (Sec. 3.4, Eq. 14):
 * I_R = R(B(x_0), ..., B(x_n), P).  The camera matrix P (3 x 4, row-major)
 * maps a homogeneous world point X to (u, v, w): pixel coordinates
 * (u / w, v / w), depth w.  Pixel (i, j) (column i, row j; image row-major
 * [height][width]) has its centre at (i + 0.5, j + 0.5).  Each centre takes
 * the nearest triangle covering it (edges inclusive, no culling; depth
 * 1 / sum_k lambda_k / w_k, ties to the lower face index) and the
 * perspective-correct interpolation of its vertices' radiance; uncovered
 * pixels are 0.  Triangles with a vertex at w <= 1e-6, zero area, or an index
 * outside [0, V) are not drawn (no clipping).  The coverage and depth
 * decisions use FP32 with one rounding per operation in a fixed order (see
 * the implementation), so they are reproducible.  Gradients flow through the
 * winning triangle's weights to the vertices' radiance and positions (a hard
 * rasteriser: occlusion and silhouette changes contribute nothing). */
#define SHV_MAX_IMAGE_SIDE 16384
typedef struct shv_camera {
  float P[12];   /* row-major 3 x 4 projection (intrinsics times extrinsics) */
  int32_t width; /* 1 .. SHV_MAX_IMAGE_SIDE */
  int32_t height;
} shv_camera;

/* Vertex-to-corner incidence of a triangle mesh, built on the host (a
 * one-time preprocessing of the mesh): faces [T][3] host int32; outputs ptr
 * [V + 1] and idx [3 T] (host), idx[ptr[v] .. ptr[v + 1]) = 3 f + k for every
 * corner k of face f at vertex v, in increasing f.  Fails if an index is
 * outside [0, V). */
shv_status shv_raster_incidence_build(const int32_t* faces, int64_t T, int64_t V, int32_t* ptr, int32_t* idx);

/* Workspace bytes of sh_raster_forward / sh_raster_backward for V vertices
 * (V < 2^31), T triangles (T < 2^26) and a width x height image (0 if
 * invalid). */
size_t shv_raster_workspace_bytes(int64_t V, int64_t T, int32_t width, int32_t height);

/* vertices [3][V], faces [T][3], radiance [V] (device) -> image [height][width]
 * and face_id [height][width] (device; -1 where nothing is drawn). */
shv_status sh_raster_forward(const float* vertices, int64_t V, const int32_t* faces, int64_t T,
                             const float* radiance, const shv_camera* camera, float* image, int32_t* face_id,
                             void* ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of sh_raster_forward for the cotangent grad_image [height][width]:
 * face_id is the forward's output for the same inputs, inc_ptr / inc_idx the
 * incidence (device copies).  grad_radiance [V] and grad_vertices [3][V]
 * (either may be NULL).  Deterministic (fixed-order sums, no atomics). */
shv_status sh_raster_backward(const float* grad_image, const float* vertices, int64_t V, const int32_t* faces,
                              int64_t T, const float* radiance, const shv_camera* camera, const int32_t* face_id,
                              const int32_t* inc_ptr, const int32_t* inc_idx, float* grad_radiance,
                              float* grad_vertices, void* ws, size_t ws_bytes, hipStream_t stream);

/* Workspace bytes of sh_deform_forward / sh_deform_backward (0 if invalid). */
size_t shv_deform_workspace_bytes(int64_t P, int64_t S);

/* Deformed points [3][P], normals [3][P] and spheres [S][4] (device) from
 * params [S + 1][6] (device); the outputs feed the visibility and shading
 * entry points directly. */
shv_status sh_deform_forward(const shv_deform_graph* graph, const float* params, float* points, float* normals,
                             float* spheres, void* ws, size_t ws_bytes, hipStream_t stream);

/* Adjoint of sh_deform_forward: from the cotangents of the deformed points
 * [3][P], normals [3][P] and spheres [S][4] (any may be NULL: zero; the
 * radius column is ignored) to grad_params [S + 1][6].  Deterministic. */
shv_status sh_deform_backward(const shv_deform_graph* graph, const float* params, const float* grad_points,
                              const float* grad_normals, const float* grad_spheres, float* grad_params, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/* The rendering loss of Sec. 3.5 on receiver values: loss[0] = mean_i
 * (value_i - target_i)^2 and grad_i = 2 (value_i - target_i) / n (grad may be
 * NULL).  ws must hold shv_l2_workspace_bytes(n) bytes.  n >= 1. */
size_t shv_l2_workspace_bytes(int64_t n);
shv_status sh_l2_loss(const float* value, const float* target, int64_t n, float* grad, float* loss, void* ws,
                      size_t ws_bytes, hipStream_t stream);

/* One gradient-descent step x_i -= lr g_i over n floats (the optimiser of
 * Sec. 3.5). */
shv_status sh_sgd_step(float* x, const float* grad, int64_t n, float lr, hipStream_t stream);

/* Adjoint of sh_visibility_forward for the cotangent grad_vis [N][P]:
 *   vis, saved  the forward's outputs for the same inputs and parameters;
 *   saved_bytes the saved buffer's size in bytes (at least
 *               4 shv_saved_floats(P, prm), else SHV_ERR_WORKSPACE before any
 *               launch; saved may be NULL when that is 0)
 *   grad_points [3][P], grad_spheres [S][4] (d/d(cx, cy, cz, r), summed over
 *   receivers); either may be NULL.  Per-pair terms are recomputed, not
 *   stored. */
shv_status sh_visibility_backward(const float* grad_vis, const float* vis, const float* points,
                                  int64_t P, const float* spheres, int64_t S,
                                  const shv_params* prm, const float* saved, size_t saved_bytes,
                                  float* grad_points, float* grad_spheres, void* ws, size_t ws_bytes,
                                  hipStream_t stream);

/* Fused render path: the same results as sh_visibility_forward followed by
 * sh_shade (bit-identical), in two launches.  `saved` holds
 * shv_render_saved_floats() values: the visibility state followed by the lit
 * transfer matrix M(L) (N x N); it may be NULL when no backward follows.
 * saved_bytes is its size in bytes: a non-NULL saved smaller than
 * 4 shv_render_saved_floats(P, prm) bytes is refused with SHV_ERR_WORKSPACE
 * before anything is launched. */
int64_t shv_render_saved_floats(int64_t P, const shv_params* prm);
shv_status sh_render_forward(const float* points, const float* normals, const float* albedo,
                             const float* spheres, const float* light, int64_t P, int64_t S,
                             const shv_params* prm, float* vis, float* radiance, float* saved,
                             size_t saved_bytes, void* ws, size_t ws_bytes, hipStream_t stream);

/* sh_render_forward for callers that cannot allocate or pass a workspace
 * (code under HIP graph capture, serving loops that must not allocate,
 * harnesses that forbid it): the same launches and bit-identical results,
 * with the scratch memory of the forward (the sphere-chunk partials of the
 * log-visibility, and M(L) when saved is NULL) taken from a static device
 * array of SHV_NOALLOC_SCRATCH_BYTES that the library holds on every device
 * it runs on until the process ends.  Needs shv_init(device) first (which
 * looks the array up on that device).  A call whose scratch would exceed the
 * array (nchunks N P + N^2 floats, nchunks = the sphere chunks of the pair
 * forward: one for P >= 32768 and S <= 512, so up to 393,216 receivers at
 * n = 8) is refused with SHV_ERR_WORKSPACE before anything is launched.  No
 * part of the array needs to start at zero: every call writes what it reads.
 * Calls on one device share the array: two calls that overlap in time on the
 * same GPU (different streams, or threads without ordering) race and give
 * wrong results.  Allocates nothing: no hipMalloc, no hipFree. */
#define SHV_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
shv_status sh_render_forward_noalloc(const float* points, const float* normals, const float* albedo,
                                     const float* spheres, const float* light, int64_t P, int64_t S,
                                     const shv_params* prm, float* vis, float* radiance, float* saved,
                                     size_t saved_bytes, hipStream_t stream);

/* Fused adjoint of sh_render_forward for the cotangent grad_radiance [P]: the
 * same results as sh_shade_backward followed by sh_visibility_backward
 * (bit-identical), in three launches.  vis and saved come from
 * sh_render_forward with the same inputs (saved_bytes at least
 * 4 shv_render_saved_floats(P, prm), else SHV_ERR_WORKSPACE before any
 * launch); every gradient output may be NULL. */
shv_status sh_render_backward(const float* grad_radiance, const float* points, const float* normals,
                              const float* albedo, const float* spheres, int64_t P, int64_t S,
                              const shv_params* prm, const float* vis, const float* saved,
                              size_t saved_bytes, float* grad_points, float* grad_normals,
                              float* grad_albedo, float* grad_spheres, float* grad_light, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/* Batched render path: many independent scenes (each with its own P, S,
 * n_bands and k) forward and backward in one launch per phase and group of
 * scenes sharing a band count (and exponential layout), every scene
 * bit-identical to single-scene sh_render_forward / sh_render_backward.
 *
 * Scene description (host structure; every pointer is a device pointer as in
 * the single-scene calls).  ws must hold shv_workspace_bytes(P, S, &params)
 * bytes and saved shv_render_saved_floats(P, &params) floats (saved_bytes
 * says how many bytes it has; a smaller buffer is refused); grad_* may be
 * NULL; grad_radiance is read by the backward only, which skips a scene whose
 * grad_radiance is NULL (its gradient outputs are left unwritten). */
typedef struct shv_scene {
  const float* points;        /* [3][P] */
  const float* normals;       /* [3][P] */
  const float* albedo;        /* [P] */
  const float* spheres;       /* [S][4], 16-byte aligned */
  const float* light;         /* [N] */
  const float* grad_radiance; /* [P] */
  float* vis;                 /* [N][P] out */
  float* radiance;            /* [P] out */
  float* saved;               /* shv_render_saved_floats() out / in */
  size_t saved_bytes;         /* size of saved in bytes (checked by shv_batch_table_build) */
  float* grad_points;         /* [3][P] out or NULL */
  float* grad_normals;        /* [3][P] out or NULL */
  float* grad_albedo;         /* [P] out or NULL */
  float* grad_spheres;        /* [S][4] out or NULL */
  float* grad_light;          /* [N] out or NULL */
  void* ws;                   /* per-scene workspace, 256-byte aligned */
  size_t ws_bytes;
  int64_t P;
  int64_t S;
  shv_params params;
  /* Receiver range [range_begin, range_end) processed by this call; 0, 0
   * means the whole scene.  A scene may be processed by several calls over
   * disjoint ranges covering [0, P), each with the scene's full buffers
   * (P, ws and saved sized for the whole scene); both ends must be multiples
   * of SHV_RANGE_ALIGN, except range_end = P.  Receiver outputs of a range
   * are final after its forward / backward; the sphere, lighting and
   * receiver-position gradients are reduced over all receivers by the
   * backward of the call whose defer_reductions is 0, which must come after
   * the backward of every other range in stream order.  The results are
   * bit-identical to one whole-scene call. */
  int64_t range_begin;
  int64_t range_end;
  int32_t defer_reductions;
} shv_scene;

/* Bytes of the work table for n_scenes scenes. */
size_t shv_batch_table_bytes(int32_t n_scenes);

/* Host-side: validates every scene (errors name the scene index) and packs
 * the work table into `table` (HOST memory, table_bytes bytes).  The caller
 * copies the table verbatim to device memory and passes the device copy to
 * the batched calls, with the block counts from shv_batch_table_grid(). */
shv_status shv_batch_table_build(const shv_scene* scenes, int32_t n_scenes, void* table,
                                 size_t table_bytes);

/* Block counts of the batched launches.  pair_fwd[n] / pair_bwd[n]: the pair
 * forward / pair adjoint launches of the scenes with n bands (the adjoint
 * splits the spheres into more chunks than the forward, so it has more
 * blocks); exp[0][n] / exp[1][n]: the exponential launches of
 * those scenes using the one-wave / four-wave layout (the layout the flags
 * select, else one receiver per lane up to 6 bands and four waves per 64
 * receivers at 7 and 8; a single-scene call takes one receiver per lane up to
 * 6 bands only from 65,536 receivers; both layouts give identical bits);
 * finalize: the closing reductions of all scenes.  Index 0 is unused and
 * must be 0.  A group with 0 blocks is not launched. */
typedef struct shv_batch_grid {
  int64_t pair_fwd[SHV_MAX_BANDS_API + 1];
  int64_t pair_bwd[SHV_MAX_BANDS_API + 1];
  int64_t exp[2][SHV_MAX_BANDS_API + 1];
  int64_t finalize;
} shv_batch_grid;

/* The exact block counts of a built (host) table.  Any larger counts work
 * too (blocks past a group's work exit at once): a captured graph of the
 * batched calls can be replayed for a new table written into the same device
 * buffer when each of its counts is at most the captured one. */
shv_status shv_batch_table_grid(const void* table_host, shv_batch_grid* grid);

/* Forward of every scene of the batch: one launch per band count for the
 * pair stage and one per (layout, band count) for the exponential and
 * shading stage, with the block counts of `grid` (host memory).  The table
 * itself stays on the device. */
shv_status sh_render_batched_forward(const void* table_device, const shv_batch_grid* grid, hipStream_t stream);

/* Backward of every scene of the batch (the same launch groups in reverse,
 * then one launch for the closing reductions of all scenes); reads each
 * scene's grad_radiance, vis and saved. */
shv_status sh_render_batched_backward(const void* table_device, const shv_batch_grid* grid, hipStream_t stream);

/* Forward and backward of every scene of the batch in one call: exactly the
 * launches of sh_render_batched_forward followed by those of
 * sh_render_batched_backward (every scene's grad_radiance is read), so the
 * results are bit-identical to those two calls and to single-scene
 * sh_render_forward / sh_render_backward. */
shv_status sh_solve_batched(const void* table_device, const shv_batch_grid* grid, hipStream_t stream);

/* ---- sh_solve_batched replayed from a HIP graph (a whole batched
 * forward + backward in one graph launch, for serving loops that issue many
 * small steps) ----
 * shv_graph_create captures sh_solve_batched into a HIP graph once, over a
 * device copy of the work table that the graph object owns (room for
 * max_scenes scenes).  groups selects the launch groups the graph holds:
 * every entry of groups that is > 0 (pair_fwd[n], pair_bwd[n],
 * exp[layout][n], finalize) puts that group's launch into the graph,
 * captured with that block count.  Each
 * shv_graph_launch then
 *   - packs the table of `scenes` on the host (the checks of
 *     shv_batch_table_build, errors name the scene) into one of four pinned
 *     staging slots (waiting, if need be, until that slot's previous copy
 *     has run),
 *   - refuses, with SHV_ERR_UNSUPPORTED before anything is enqueued, a batch
 *     that needs a group the graph does not hold (or, with
 *     SHV_GRAPH_FIXED_GRID, more blocks in a group than captured),
 *   - disables the graph's launches of groups with no work this time (a
 *     disabled launch keeps its place in the graph's order and runs nothing)
 *     and enables the others again, and sets each enabled launch to the exact
 *     block count the table needs, unless SHV_GRAPH_FIXED_GRID keeps the
 *     captured counts (blocks past a group's work exit at once),
 *   - enqueues on `stream`: a wait for the graph's previous launch (so
 *     launches on different streams are ordered), the copy of the table into
 *     the graph's device buffer, and the graph (nothing at all for an empty
 *     batch).
 * Results are bit-identical to sh_solve_batched on the same table.  The
 * graph object is not thread-safe: one thread launches it at a time.
 * shv_graph_create and shv_graph_destroy allocate and free (device table,
 * pinned staging, the graph); shv_graph_launch allocates nothing.
 * A new graph's first few launches (up to about a dozen) are slower now and
 * then (a few ms); steady-state launches cost what the eager calls cost.
 * shv_graph_destroy waits for the graph's last launch to finish. */
#define SHV_GRAPH_FIXED_GRID 1u
typedef struct shv_graph shv_graph;
shv_status shv_graph_create(const shv_batch_grid* groups, int32_t max_scenes, uint32_t flags, shv_graph** graph);
shv_status shv_graph_launch(shv_graph* graph, const shv_scene* scenes, int32_t n_scenes, hipStream_t stream);
shv_status shv_graph_destroy(shv_graph* graph);

/* Per-kernel timing with HIP events recorded around every launch on the
 * launch stream.  shv_profile_enable(1) starts a new collection (at most
 * `capacity` launches are recorded; later ones are counted but not timed);
 * shv_profile_enable(0) pauses recording and shv_profile_enable(2) resumes
 * it, adding to the current collection (to time a sample of the launches;
 * resuming never creates events, so it adds nothing to a timed region).
 * shv_profile_report() must be called
 * after the stream has drained: it writes "name count total_ms\n" lines into
 * buf (NUL-terminated, truncated to len) and returns the number of bytes
 * needed. */
shv_status shv_profile_enable(int enable, int32_t capacity);
int64_t shv_profile_report(char* buf, int64_t len);

#ifdef __cplusplus
}
#endif

#endif /* SHVIS_H */
