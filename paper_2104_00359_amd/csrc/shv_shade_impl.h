// Diffuse SH shading B = a (L . (V * H)) (Eq. 8) and its adjoint, as
// separate entry points (sh_shade, sh_shade_backward).
//
// With the lit transfer matrix M(L)_jk = sum_i L_i C_ijk (symmetric, built once
// per call from L), B = a V^T M H.  The clamped-cosine transfer is
// H_lm = A_l y_lm(n / |n|) (Eqs. 10-11): its odd bands above 1 vanish, so only
// the columns of M on H's support are ever read (31 of 64 at n = 8).
// M is read with wave-uniform addresses, so it is served by scalar loads.
//
// Adjoint for the cotangent Bbar, w = Bbar a:
//   abar = Bbar (V^T M H),  Vbar = w M H,  Hbar = w M V  -> nbar through the
//   gradient of the SH polynomial (tangential part / |n|);
//   Lbar_i = sum_x w(x) (V(x) * H(x))_i = sum_jk C_ijk Q_jk with the small
//   GEMM Q_jk = sum_x V_j(x) (w H_k)(x) over the transfer support, formed per
//   tile of 64 receivers in LDS and contracted with C; the tile partials are
//   summed afterwards in tile order.

#pragma once

#include "shv_launch.h"
#include "shv_shade_common.h"

namespace shv {


template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_build_M(const float* __restrict__ L, float* __restrict__ M) {
  build_M_range<NB>(L, M, blockIdx.x * SHV_BLOCK + threadIdx.x, gridDim.x * SHV_BLOCK);
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_shade_fwd(const float* __restrict__ vis, const float* __restrict__ nrm,
                                                         const float* __restrict__ alb, const float* __restrict__ M,
                                                         int64_t P, float* __restrict__ rad) {
  constexpr int N = NB * NB;
  __shared__ float Ms[MSupp<NB>::SIZE];
  stage_M<NB>(M, Ms, threadIdx.x, SHV_BLOCK);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (p >= P) return;
  float V[N], H[N], Hb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) V[i] = vis[(int64_t)i * P + p];
  float ux, uy, uz;
  transfer<NB>(nrm[p], nrm[P + p], nrm[2 * P + p], H, ux, uy, uz);
  rad[p] = alb[p] * shade_value<NB, false>(V, H, Ms, 0.0f, Hb);
}

// One receiver per lane, 256 receivers per block (4 tiles of 64).
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_shade_bwd(const float* __restrict__ gB, const float* __restrict__ vis,
                                                         const float* __restrict__ nrm, const float* __restrict__ alb,
                                                         const float* __restrict__ M, int64_t P,
                                                         float* __restrict__ gV, float* __restrict__ gN,
                                                         float* __restrict__ gA, float* __restrict__ Lpart) {
  constexpr int N = NB * NB;
  __shared__ LightTile T;
  __shared__ float Ms[MSupp<NB>::SIZE];
  stage_M<NB>(M, Ms, threadIdx.x, SHV_BLOCK);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const bool ok = p < P;
  float V[N], H[N], Hb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) V[i] = ok ? vis[(int64_t)i * P + p] : 0.0f;
  float ux, uy, uz;
  const float inv = transfer<NB>(ok ? nrm[p] : 0.0f, ok ? nrm[P + p] : 0.0f, ok ? nrm[2 * P + p] : 1.0f, H, ux, uy, uz);
  const float bb = ok ? gB[p] : 0.0f;
  const float w = bb * (ok ? alb[p] : 0.0f);
  const float s = shade_value<NB, true>(V, H, Ms, w, Hb);
  if (ok) {
    if (gA) gA[p] = bb * s;
    if (gV) {
#pragma unroll
      for (int j = 0; j < N; ++j) gV[(int64_t)j * P + p] = vbar_entry<NB>(j, H, Ms, w);
    }
    if (gN) {
      float gx, gy, gz;
      normal_grad<NB>(Hb, ux, uy, uz, inv, gx, gy, gz);
      gN[p] = gx;
      gN[P + p] = gy;
      gN[2 * P + p] = gz;
    }
  }
  if (!Lpart) return;  // uniform
  for (int r = 0; r < SHV_WAVES_PER_BLOCK; ++r) {
    const int64_t tile = (int64_t)blockIdx.x * SHV_WAVES_PER_BLOCK + r;
    if (tile * 64 >= P) break;  // uniform
    if (wave == r) {
      tile_put_v<NB>(T, lane, V);
      tile_put_wh<NB>(T, lane, H, w);
    }
    __syncthreads();
    tile_light_partial<NB>(T, Lpart + tile * N);
  }
}

// ---------------------------------------------------------------------------
// Launchers for one band count (instantiated per band count in shv_nb.hip).

template <int NB>
hipError_t build_M_nb(const float* light, float* M, hipStream_t st) {
  constexpr int NN = NB * NB * NB * NB;
  k_build_M<NB><<<(unsigned)((NN + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(light, M);
  return hipGetLastError();
}

template <int NB>
hipError_t shade_fwd_nb(const float* vis, const float* nrm, const float* alb, const float* M, int64_t P, float* rad,
                        hipStream_t st) {
  k_shade_fwd<NB><<<(unsigned)point_blocks(P), SHV_BLOCK, 0, st>>>(vis, nrm, alb, M, P, rad);
  return hipGetLastError();
}

template <int NB>
hipError_t shade_bwd_nb(const float* gB, const float* vis, const float* nrm, const float* alb, const float* M,
                        int64_t P, float* gV, float* gN, float* gA, float* Lpart, hipStream_t st) {
  k_shade_bwd<NB><<<(unsigned)point_blocks(P), SHV_BLOCK, 0, st>>>(gB, vis, nrm, alb, M, P, gV, gN, gA, Lpart);
  return hipGetLastError();
}

}  // namespace shv
