// Host-side dispatch on the band count, kernel-variant choices, and the
// kernels that do not depend on the band count (fills and the deterministic
// reductions that close a backward pass, single-scene and batched).

#include <hip/hip_runtime.h>

#include "shv_batch.h"
#include "shv_config.h"
#include "shv_launch.h"
#include "shvis.h"

namespace shv {

// About target_waves waves over the chunks, at least 8 spheres per wave, at
// most SHV_MAX_CHUNK spheres per chunk.
static Split split_for(int64_t P, int64_t S, int64_t target_waves) {
  Split sp{1, (int)(S > 0 ? S : 1)};
  if (S <= 0) return sp;
  const int64_t waves = 4 * pair_blocks(P);  // 4 waves per 64-receiver tile
  int64_t n = waves > 0 ? (target_waves + waves - 1) / waves : 1;
  const int64_t max_by_size = (S + 31) / 32;  // keep >= 8 spheres per wave
  if (n > max_by_size) n = max_by_size;
  const int64_t min_by_lds = (S + SHV_MAX_CHUNK - 1) / SHV_MAX_CHUNK;
  if (n < min_by_lds) n = min_by_lds;
  if (n < 1) n = 1;
  const int64_t chunk = (S + n - 1) / n;
  sp.chunk = (int)chunk;
  sp.nchunks = (int)((S + chunk - 1) / chunk);
  return sp;
}

// Forward: two waves per SIMD on 256 CUs x 4 SIMDs.  Each chunk writes N
// floats per receiver that the exponential forward reads back; against the
// adjoint's target this halves the chunks of scenes under 32,768 receivers
// (2% off the 64-scene batched step; a 20,000-receiver scene's pair forward
// loses about what its exponential forward gains).
Split fwd_split(int64_t P, int64_t S) { return split_for(P, S, 2048); }
// Adjoint: four waves per SIMD (its receiver partials are 3 floats).
Split bwd_split(int64_t P, int64_t S) { return split_for(P, S, 4096); }

int64_t point_blocks(int64_t P) { return (P + SHV_BLOCK - 1) / SHV_BLOCK; }
int64_t pair_blocks(int64_t P) { return (P + 63) / 64; }


__global__ __launch_bounds__(SHV_BLOCK) void k_fill_zero(float* __restrict__ p, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (j < n) p[j] = 0.0f;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_fill_zero<<<(unsigned)((n + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(p, n);
  return hipGetLastError();
}

// out[j] = sum_c part[c * len + j], c in order.
__device__ __forceinline__ void sum_chunks_at(const float* __restrict__ part, int nchunks, int64_t len, int64_t j,
                                              float* __restrict__ out) {
  if (j >= len) return;
  // chunks added in increasing order; their loads issued eight at a time
  float a = part[j];
  for (int c0 = 1; c0 < nchunks; c0 += 8) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = c0 + u < nchunks ? part[(int64_t)(c0 + u) * len + j] : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c0 + u < nchunks) a += v[u];
  }
  out[j] = a;
}

__global__ __launch_bounds__(SHV_BLOCK) void k_sum_chunks(const float* __restrict__ part, int nchunks, int64_t len,
                                                          float* __restrict__ out) {
  sum_chunks_at(part, nchunks, len, (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x, out);
}

hipError_t launch_sum_chunks(const float* part, int nchunks, int64_t len, float* out, hipStream_t st) {
  if (len <= 0) return hipSuccess;
  k_sum_chunks<<<(unsigned)((len + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(part, nchunks, len, out);
  return hipGetLastError();
}

// out[c] = sum_r part[r * cols + c] for the 16 columns c = 16 cb .. 16 cb + 15.
// Thread t owns column 16 cb + (t % 16) and row group g = t / 16 (16 groups);
// it sums rows g, g + 16, g + 32, ... in increasing order (loads issued 16 rows
// at a time, the last batch predicated; each wave reads four contiguous
// 64-byte row segments), then the
// 16 group partials of a column are added in group order.  The canonical
// order of every column reduction (receiver tiles -> sphere and lighting
// gradients).
constexpr int kColsPerBlock = 16;
constexpr int kRowGroups = SHV_BLOCK / kColsPerBlock;

__device__ __forceinline__ void reduce_columns(const float* __restrict__ part, int rows, int cols, int cb,
                                               float* __restrict__ out, float* buf) {
  const int l = threadIdx.x % kColsPerBlock, g = threadIdx.x / kColsPerBlock;
  const int c = cb * kColsPerBlock + l;
  float a = 0.0f;
  if (c < cols) {
    for (int r = g; r < rows; r += 16 * kRowGroups) {
      float v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        v[u] = r + u * kRowGroups < rows ? part[(int64_t)(r + u * kRowGroups) * cols + c] : 0.0f;
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (r + u * kRowGroups < rows) a += v[u];
    }
  }
  buf[threadIdx.x] = a;
  __syncthreads();
  if (g == 0 && c < cols) {
    float t = buf[l];
#pragma unroll
    for (int q = 1; q < kRowGroups; ++q) t += buf[q * kColsPerBlock + l];
    out[c] = t;
  }
}

// Blocks of kColsPerBlock columns.
__host__ __device__ __forceinline__ int column_blocks(int cols) { return (cols + kColsPerBlock - 1) / kColsPerBlock; }

// Batch y = blockIdx.y reduces part + y rows cols into out + y cols.
__global__ __launch_bounds__(SHV_BLOCK) void k_reduce_rows(const float* __restrict__ part, int rows, int cols,
                                                           float* __restrict__ out) {
  __shared__ float buf[SHV_BLOCK];
  const int64_t y = blockIdx.y;
  reduce_columns(part + y * rows * cols, rows, cols, blockIdx.x, out + y * cols, buf);
}

// All reductions that close a backward pass, in one launch: blocks
// [0, nb_pts) sum the receiver-gradient chunks, the next blocks reduce the
// 4S sphere-gradient columns (16 per block), the last ones the N
// lighting-gradient columns.
__device__ __forceinline__ void finalize_item(const float* __restrict__ gp_part, int nchunks, int64_t P,
                                              float* __restrict__ grad_points, int nb_pts,
                                              const float* __restrict__ gs_part, int rows_s, int cols_s,
                                              float* __restrict__ grad_spheres, const float* __restrict__ l_part,
                                              int rows_l, int cols_l, float* __restrict__ grad_light, int b,
                                              float* buf) {
  const int nb_s = column_blocks(cols_s);
  if (b < nb_pts) {
    sum_chunks_at(gp_part, nchunks, 3 * P, (int64_t)b * SHV_BLOCK + threadIdx.x, grad_points);
  } else if (b < nb_pts + nb_s) {
    reduce_columns(gs_part, rows_s, cols_s, b - nb_pts, grad_spheres, buf);
  } else {
    reduce_columns(l_part, rows_l, cols_l, b - nb_pts - nb_s, grad_light, buf);
  }
}

__global__ __launch_bounds__(SHV_BLOCK) void k_finalize(const float* __restrict__ gp_part, int nchunks, int64_t P,
                                                        float* __restrict__ grad_points, int nb_pts,
                                                        const float* __restrict__ gs_part, int rows_s, int cols_s,
                                                        float* __restrict__ grad_spheres,
                                                        const float* __restrict__ l_part, int rows_l, int cols_l,
                                                        float* __restrict__ grad_light) {
  __shared__ float buf[SHV_BLOCK];
  finalize_item(gp_part, nchunks, P, grad_points, nb_pts, gs_part, rows_s, cols_s, grad_spheres, l_part, rows_l,
                cols_l, grad_light, blockIdx.x, buf);
}

hipError_t launch_finalize(const float* gp_part, int nchunks, int64_t P, float* grad_points, const float* gs_part,
                           int rows_s, int64_t S, float* grad_spheres, const float* l_part, int rows_l, int N,
                           float* grad_light, hipStream_t st) {
  const int nb_pts = grad_points ? (int)((3 * P + SHV_BLOCK - 1) / SHV_BLOCK) : 0;
  const int cols_s = grad_spheres ? (int)(4 * S) : 0;
  const int cols_l = grad_light ? N : 0;
  const int grid = nb_pts + column_blocks(cols_s) + column_blocks(cols_l);
  if (grid == 0) return hipSuccess;
  k_finalize<<<(unsigned)grid, SHV_BLOCK, 0, st>>>(gp_part, nchunks, P, grad_points, nb_pts, gs_part, rows_s, cols_s,
                                                    grad_spheres, l_part, rows_l, cols_l, grad_light);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const float* part, int rows, int cols, float* out, hipStream_t st, int batch) {
  if (cols <= 0 || batch <= 0) return hipSuccess;
  k_reduce_rows<<<dim3((unsigned)column_blocks(cols), (unsigned)batch), SHV_BLOCK, 0, st>>>(part, rows, cols, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched closing reductions (all scenes of a batch in one launch).

__global__ __launch_bounds__(SHV_BLOCK) void k_batch_finalize(const char* __restrict__ table) {
  __shared__ float buf[SHV_BLOCK];
  const BatchView v(table);
  const int64_t item = blockIdx.x;
  if (item >= v.h->total_fin) return;
  const BatchScene S = in_global(v.scene_of_fin(item));
  if (!S.grad_radiance) return;  // uniform: scene packed without a cotangent
  const int b = (int)(item - S.off_fin);
  finalize_item(S.gp, S.nchunks_b, S.P, S.fin_pts ? S.grad_points : nullptr, S.fin_pts, S.gs, (int)S.pair_tiles,
                S.fin_cols_s, S.grad_spheres, S.lp, (int)S.pair_tiles, S.fin_cols_l, S.grad_light, b, buf);
}

hipError_t launch_batch_finalize(const void* table, int64_t blocks, hipStream_t st) {
  k_batch_finalize<<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  return hipGetLastError();
}

bool exp_four_waves(int nb, int64_t P, uint32_t flags, bool batched) {
  if (flags & SHV_FLAG_EXP_ONE_WAVE) return false;
  if (flags & SHV_FLAG_EXP_FOUR_WAVES) return true;
  // Up to 6 bands a receiver's whole squaring fits one lane's registers, and
  // one receiver per lane (no LDS exchange, no barriers) is faster than four
  // waves per 64 receivers; a launch then has 4x fewer blocks, so a single
  // scene takes it only from 256 blocks (65,536 receivers) up.  At 7 and 8
  // bands the four-wave layout is faster for the adjoint (both layouts give
  // identical bits).
  return !(nb <= 6 && (batched || P >= 65536));
}

// ---------------------------------------------------------------------------
// Dispatch on the band count to the per-band-count launchers.

#define SHV_NB_SWITCH(nb, CALL)          \
  switch (nb) {                          \
    case 1: return CALL(1);              \
    case 2: return CALL(2);              \
    case 3: return CALL(3);              \
    case 4: return CALL(4);              \
    case 5: return CALL(5);              \
    case 6: return CALL(6);              \
    case 7: return CALL(7);              \
    case 8: return CALL(8);              \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_pair_fwd(int nb, const float* pts, int64_t P, const float* sph, int S, Split sp, float* Fpart,
                           const float* light, float* M, hipStream_t st) {
#define C(N) pair_fwd_nb<N>(pts, P, sph, S, sp, Fpart, light, M, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_pair_bwd(int nb, const float* W, const float* pts, int64_t P, const float* sph, int S, Split sp,
                           float* gp_part, float* gs_part, hipStream_t st) {
#define C(N) pair_bwd_nb<N>(W, pts, P, sph, S, sp, gp_part, gs_part, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_exp_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k, float* vis,
                          float* saved, uint32_t flags, hipStream_t st) {
#define C(N) exp_fwd_nb<N, false>(Fpart, nchunks, P, eps, k, vis, saved, nullptr, nullptr, nullptr, nullptr, flags, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_render_exp_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k, float* vis,
                                 float* saved, const float* nrm, const float* alb, const float* M, float* rad,
                                 uint32_t flags, hipStream_t st) {
#define C(N) exp_fwd_nb<N, true>(Fpart, nchunks, P, eps, k, vis, saved, nrm, alb, M, rad, flags, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_exp_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P, float eps,
                          int k, float* W, uint32_t flags, hipStream_t st) {
#define C(N) \
  exp_bwd_nb<N, false>(gV, vis, saved, P, eps, k, W, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, flags, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_render_exp_bwd(int nb, const float* gB, const float* vis, const float* saved, int64_t P, float eps,
                                 int k, float* W, const float* nrm, const float* alb, const float* M, float* gN,
                                 float* gA, float* Lpart, uint32_t flags, hipStream_t st) {
#define C(N) exp_bwd_nb<N, true>(gB, vis, saved, P, eps, k, W, nrm, alb, M, gN, gA, Lpart, flags, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_build_M(int nb, const float* light, float* M, hipStream_t st, int channels) {
#define C(N) build_M_nb<N>(light, M, channels, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_exp_quad_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, float* vis,
                               float* saved, float* table, float* part, hipStream_t st) {
#define C(N) exp_quad_fwd_nb<N>(Fpart, nchunks, P, eps, vis, saved, table, part, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_exp_quad_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P, float eps,
                               float* W, float* table, float* part, hipStream_t st) {
#define C(N) exp_quad_bwd_nb<N>(gV, vis, saved, P, eps, W, table, part, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_exp_taylor_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k, int K,
                                 float* vis, float* saved, hipStream_t st) {
#define C(N) exp_taylor_fwd_nb<N>(Fpart, nchunks, P, eps, k, K, vis, saved, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_exp_taylor_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P, float eps,
                                 int k, int K, float* W, hipStream_t st) {
#define C(N) exp_taylor_bwd_nb<N>(gV, vis, saved, P, eps, k, K, W, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_prod_fwd(int nb, const float* pts, int64_t P, const float* sph, int S, float eps, float* vis,
                           float* states, hipStream_t st) {
#define C(N) prod_fwd_nb<N>(pts, P, sph, S, eps, vis, states, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_prod_bwd(int nb, const float* gvis, const float* states, const float* pts, int64_t P,
                           const float* sph, int S, float eps, float* gpts, float* gs_part, hipStream_t st) {
#define C(N) prod_bwd_nb<N>(gvis, states, pts, P, sph, S, eps, gpts, gs_part, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_shade_ch_fwd(int nb, const float* vis, const float* nrm, const float* alb, const float* M,
                               int channels, int64_t P, float* rad, hipStream_t st) {
#define C(N) shade_ch_fwd_nb<N>(vis, nrm, alb, M, channels, P, rad, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_shade_ch_bwd(int nb, const float* gB, const float* vis, const float* nrm, const float* alb,
                               const float* M, int channels, int64_t P, float* gV, float* gN, float* gA,
                               float* Lpart, hipStream_t st) {
#define C(N) shade_ch_bwd_nb<N>(gB, vis, nrm, alb, M, channels, P, gV, gN, gA, Lpart, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

int64_t envmap_row_blocks(int64_t H, int64_t W) {
  const int64_t R = envmap_rows_per_block(W);
  return (H + R - 1) / R;
}

hipError_t launch_envmap_rows(int nb, const float* img, int channels, int64_t H, int64_t W, float* part,
                              hipStream_t st) {
#define C(N) envmap_rows_nb<N>(img, channels, H, W, part, st)
  SHV_NB_SWITCH(nb, C)
#undef C
}

hipError_t launch_batch_nb(int nb, int phase, bool four, const void* table, int64_t blocks, hipStream_t st) {
  switch (phase) {
#define C(N) batch_pair_fwd_nb<N>(table, blocks, st)
    case 0: SHV_NB_SWITCH(nb, C)
#undef C
#define C(N) batch_exp_fwd_nb<N>(table, four, blocks, st)
    case 1: SHV_NB_SWITCH(nb, C)
#undef C
#define C(N) batch_exp_bwd_nb<N>(table, four, blocks, st)
    case 2: SHV_NB_SWITCH(nb, C)
#undef C
#define C(N) batch_pair_bwd_nb<N>(table, blocks, st)
    case 3: SHV_NB_SWITCH(nb, C)
#undef C
    default: return hipErrorInvalidValue;
  }
}

}  // namespace shv
