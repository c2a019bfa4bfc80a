// Internal launcher declarations (host side).  Every launcher enqueues one
// kernel on `st` and returns the launch status; none allocates or syncs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shv_config.h"

namespace shv {

// Split of the sphere set into chunks for the pair kernels ("split-S"): the
// log-visibility is a sum over spheres (Sec. 3.3.2), so partial sums from
// sphere chunks add up, and so do the receiver gradients of the adjoint.
// Pure functions of (P, S): the same scene is always reduced in the same
// order.  The forward's chunk partials are N floats per receiver that go
// through HBM, the adjoint's 3, so the forward takes fewer, longer chunks.
struct Split {
  int nchunks;
  int chunk;
};
Split fwd_split(int64_t P, int64_t S);  // pair forward: partials of F'
Split bwd_split(int64_t P, int64_t S);  // pair adjoint: receiver-gradient partials

int64_t point_blocks(int64_t P);  // ceil(P / 256)
int64_t pair_blocks(int64_t P);   // ceil(P / 64): pair-kernel blocks (rows of the sphere partials)

// light / M: when M is non-NULL the first block also writes M(L) (fused render path).
hipError_t launch_pair_fwd(int nb, const float* pts, int64_t P, const float* sph, int S, Split sp,
                           float* Fpart, const float* light, float* M, hipStream_t st);
hipError_t launch_exp_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k,
                          float* vis, float* saved, uint32_t flags, hipStream_t st);
// M(L) for `channels` lights light + c N into M + c N^2.
hipError_t launch_build_M(int nb, const float* light, float* M, hipStream_t st, int channels = 1);
// out[y][c] = sum over r of part[y][r][c] (rows in order; y < batch).
hipError_t launch_reduce_rows(const float* part, int rows, int cols, float* out, hipStream_t st, int batch = 1);
// Several colour channels sharing V (channel c's data at M + c N^2, alb / rad / gB / gA + c P,
// Lpart + c ceil(P / 64) N); 1 <= channels <= SHV_MAX_CHANNELS.
hipError_t launch_shade_ch_fwd(int nb, const float* vis, const float* nrm, const float* alb, const float* M,
                               int channels, int64_t P, float* rad, hipStream_t st);
hipError_t launch_shade_ch_bwd(int nb, const float* gB, const float* vis, const float* nrm, const float* alb,
                               const float* M, int channels, int64_t P, float* gV, float* gN, float* gA,
                               float* Lpart, hipStream_t st);
// Partial sums of Eq. 9 over an equirectangular map [channels][H][W], one per block of
// envmap_row_blocks(H, W) row blocks -> part [channels][row blocks][N].
hipError_t launch_envmap_rows(int nb, const float* img, int channels, int64_t H, int64_t W, float* part,
                              hipStream_t st);
int64_t envmap_row_blocks(int64_t H, int64_t W);
// Rows per block of that projection: about 4096 pixels per block.
inline int envmap_rows_per_block(int64_t W) {
  const int64_t r = (4096 + W - 1) / W;
  return (int)(r < 1 ? 1 : (r > SHV_ENV_MAX_ROWS ? SHV_ENV_MAX_ROWS : r));
}
hipError_t launch_exp_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P,
                          float eps, int k, float* W, uint32_t flags, hipStream_t st);
// The exponential by quadrature projection (SHV_FLAG_EXP_QUADRATURE); saved holds F [N][P];
// table is scratch of quad_table_floats(nb) floats (the rule's basis and weights), part of
// quad_part_floats(nb, P) (partial sums over two interleaved halves of the nodes).
inline int64_t quad_table_floats(int nb) { return (int64_t)((32 * nb * nb + 63) / 64 * 64) * 65; }
inline int64_t quad_part_floats(int nb, int64_t P) { return 2 * (int64_t)nb * nb * P; }
hipError_t launch_exp_quad_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, float* vis,
                               float* saved, float* table, float* part, hipStream_t st);
hipError_t launch_exp_quad_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P, float eps,
                               float* W, float* table, float* part, hipStream_t st);
// The exponential with a Taylor series of order K in place of the linear approximation
// (SHV_FLAG_EXP_TAYLOR); saved holds (1 + (k + K) N) rows of P.
hipError_t launch_exp_taylor_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k, int K,
                                 float* vis, float* saved, hipStream_t st);
hipError_t launch_exp_taylor_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P, float eps,
                                 int k, int K, float* W, hipStream_t st);
// The direct product chain (SHV_FLAG_EXP_PRODUCT).  states, when not NULL, receives each step's
// input [S][N][P] (the adjoint's input); vis may be NULL.  gs_part is [4 pair_blocks(P)][S] float4.
hipError_t launch_prod_fwd(int nb, const float* pts, int64_t P, const float* sph, int S, float eps, float* vis,
                           float* states, hipStream_t st);
hipError_t launch_prod_bwd(int nb, const float* gvis, const float* states, const float* pts, int64_t P,
                           const float* sph, int S, float eps, float* gpts, float* gs_part, hipStream_t st);
hipError_t launch_pair_bwd(int nb, const float* W, const float* pts, int64_t P, const float* sph, int S,
                           Split sp, float* gp_part, float* gs_part, hipStream_t st);
// Zero n floats with a plain kernel (safe inside captured graphs).
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st);
hipError_t launch_sum_chunks(const float* part, int nchunks, int64_t len, float* out, hipStream_t st);
// Receiver-chunk sums, sphere-gradient and lighting-gradient column reductions in one launch
// (each output may be NULL to skip it).
hipError_t launch_finalize(const float* gp_part, int nchunks, int64_t P, float* grad_points, const float* gs_part,
                           int rows_s, int64_t S, float* grad_spheres, const float* l_part, int rows_l, int N,
                           float* grad_light, hipStream_t st);
// Exponential with the shading step (forward) or the shading adjoint (backward) fused in.
hipError_t launch_render_exp_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k, float* vis,
                                 float* saved, const float* nrm, const float* alb, const float* M, float* rad,
                                 uint32_t flags, hipStream_t st);
hipError_t launch_render_exp_bwd(int nb, const float* gB, const float* vis, const float* saved, int64_t P, float eps,
                                 int k, float* W, const float* nrm, const float* alb, const float* M, float* gN,
                                 float* gA, float* Lpart, uint32_t flags, hipStream_t st);

// Batched phases; `table` is the device copy of a batch table.  phase: 0 pair
// forward, 1 exponential + shading forward, 2 their adjoint, 3 pair adjoint;
// one launch of `blocks` blocks covers every scene with nb bands (and, for
// the exponential phases, with the given layout).
hipError_t launch_batch_nb(int nb, int phase, bool four, const void* table, int64_t blocks, hipStream_t st);
hipError_t launch_batch_finalize(const void* table, int64_t blocks, hipStream_t st);

// Per-band-count launchers (defined in the per-band-count translation units).
template <int NB>
hipError_t pair_fwd_nb(const float* pts, int64_t P, const float* sph, int S, Split sp, float* Fpart,
                       const float* light, float* M, hipStream_t st);
template <int NB>
hipError_t pair_bwd_nb(const float* W, const float* pts, int64_t P, const float* sph, int S, Split sp, float* gp_part,
                       float* gs_part, hipStream_t st);
template <int NB, bool SHADE>
hipError_t exp_fwd_nb(const float* Fpart, int nchunks, int64_t P, float eps, int k, float* vis, float* saved,
                      const float* nrm, const float* alb, const float* M, float* rad, uint32_t flags, hipStream_t st);
template <int NB, bool SHADE>
hipError_t exp_bwd_nb(const float* gIn, const float* vis, const float* saved, int64_t P, float eps, int k, float* W,
                      const float* nrm, const float* alb, const float* M, float* gN, float* gA, float* Lpart,
                      uint32_t flags, hipStream_t st);
template <int NB>
hipError_t build_M_nb(const float* light, float* M, int channels, hipStream_t st);
template <int NB>
hipError_t shade_ch_fwd_nb(const float* vis, const float* nrm, const float* alb, const float* M, int channels,
                           int64_t P, float* rad, hipStream_t st);
template <int NB>
hipError_t shade_ch_bwd_nb(const float* gB, const float* vis, const float* nrm, const float* alb, const float* M,
                           int channels, int64_t P, float* gV, float* gN, float* gA, float* Lpart, hipStream_t st);
template <int NB>
hipError_t envmap_rows_nb(const float* img, int channels, int64_t H, int64_t W, float* part, hipStream_t st);
template <int NB>
hipError_t exp_quad_fwd_nb(const float* Fpart, int nchunks, int64_t P, float eps, float* vis, float* saved,
                           float* table, float* part, hipStream_t st);
template <int NB>
hipError_t exp_quad_bwd_nb(const float* gV, const float* vis, const float* saved, int64_t P, float eps, float* W,
                           float* table, float* part, hipStream_t st);
template <int NB>
hipError_t exp_taylor_fwd_nb(const float* Fpart, int nchunks, int64_t P, float eps, int k, int K, float* vis,
                             float* saved, hipStream_t st);
template <int NB>
hipError_t exp_taylor_bwd_nb(const float* gIn, const float* vis, const float* saved, int64_t P, float eps, int k,
                             int K, float* W, hipStream_t st);
template <int NB>
hipError_t prod_fwd_nb(const float* pts, int64_t P, const float* sph, int S, float eps, float* vis, float* states,
                       hipStream_t st);
template <int NB>
hipError_t prod_bwd_nb(const float* gvis, const float* states, const float* pts, int64_t P, const float* sph, int S,
                       float eps, float* gpts, float* gs_part, hipStream_t st);
template <int NB>
hipError_t batch_pair_fwd_nb(const void* table, int64_t blocks, hipStream_t st);
template <int NB>
hipError_t batch_pair_bwd_nb(const void* table, int64_t blocks, hipStream_t st);
template <int NB>
hipError_t batch_exp_fwd_nb(const void* table, bool four, int64_t blocks, hipStream_t st);
template <int NB>
hipError_t batch_exp_bwd_nb(const void* table, bool four, int64_t blocks, hipStream_t st);

// Exponential layout of a launch (true: four waves per 64 receivers; false:
// one receiver per lane): the flags' choice, else by band count and size.
bool exp_four_waves(int nb, int64_t P, uint32_t flags, bool batched);

// Rasteriser (the camera as in shv_camera).  rec is scratch of raster_record_bytes(T); bins of
// raster_bin_bytes (forward); part of 12 T floats (per-face corner cotangents, backward).
struct RasterCam {
  float P[12];
  int width, height;
};
size_t raster_record_bytes(int64_t T);
size_t raster_bin_bytes(int64_t T, int width, int height);  // forward scratch after the records
int64_t raster_tiles(int width, int height);
hipError_t launch_raster_forward(const float* verts, int64_t V, const int32_t* faces, int64_t T, const float* radiance,
                                 const RasterCam& cam, float* image, int32_t* face_id, void* rec, void* bins,
                                 hipStream_t st);
hipError_t launch_raster_backward(const float* grad_image, const float* verts, int64_t V, const int32_t* faces,
                                  int64_t T, const float* radiance, const RasterCam& cam, const int32_t* face_id,
                                  const int32_t* inc_ptr, const int32_t* inc, float* grad_radiance,
                                  float* grad_verts, void* rec, float* part, hipStream_t st);

// Scene parameterisation upstream of the spheres (embedded deformation graph
// and global pose).  Device pointers as in shv_deform_graph.
struct DeformGraphDev {
  const float* vertices;
  const float* normals;
  const float* spheres;
  const int32_t* vert_ptr;
  const int32_t* vert_sph;
  const float* vert_w;
  const int32_t* sph_vert;
  const float* sph_w;
  int64_t P, S;
  int K;
};
int deform_graph_build(const float* vertices, int64_t P, const float* spheres, int64_t S, int K, int32_t* vert_ptr,
                       int32_t* vert_sph, float* vert_w, int32_t* sph_vert, float* sph_w);
int64_t deform_vert_blocks(int64_t P);
// Rm [(S + 1) * 9] scratch; pts / nrm [3][P], sph [S][4] out.
hipError_t launch_deform_forward(const DeformGraphDev& g, const float* params, float* Rm, float* pts, float* nrm,
                                 float* sph, hipStream_t st);
// Rm as above, Yb [6][P], Gpart [(deform_vert_blocks(P) + S) * 12], G [12] scratch; gp [S + 1][6] out.
hipError_t launch_deform_backward(const DeformGraphDev& g, const float* params, const float* gx, const float* gn,
                                  const float* gs, float* Rm, float* Yb, float* Gpart, float* G, float* gp,
                                  hipStream_t st);
// part [ceil(n / 256)] scratch; loss [1] and grad [n] out.
hipError_t launch_l2(const float* v, const float* t, int64_t n, float* grad, float* part, float* loss,
                     hipStream_t st);
hipError_t launch_sgd(float* x, const float* g, int64_t n, float lr, hipStream_t st);

}  // namespace shv
