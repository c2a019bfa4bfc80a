// Diffuse SH shading B = a (L . (V * H)) (Eq. 8) and its adjoint, as
// separate entry points (sh_shade, sh_shade_backward).
//
// With the lit transfer matrix M(L)_jk = sum_i L_i C_ijk (symmetric, built once
// per call from L), B = a V^T M H.  The clamped-cosine transfer is
// H_lm = A_l y_lm(n / |n|) (Eqs. 10-11): its odd bands above 1 vanish, so only
// the columns of M on H's support are ever read (31 of 64 at n = 8).
// Each block first copies those columns of M into LDS (stage_M).
//
// Several colour channels (one light L_c and albedo a_c per channel, one
// shared visibility, Eq. 8 per channel) are shaded by one launch that stages
// every channel's M and reads V and H once; channel c's radiance, albedo
// gradient and lighting gradient are bitwise those of a one-channel call, and
// the V and normal cotangents are summed over the channels in channel order.
//
// Environment-map projection (Eq. 9): L_i = integral of L(w) y_i(w) dw over
// an equirectangular map, as the sum over pixels of value * y_i(pixel centre)
// * pixel solid angle; one block per (row, channel) forms the row's sum, the
// rows are then added in row order.
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

// Several channels (CH of them, 1 .. SHV_MAX_CHANNELS): channel c's light
// matrix at M + c N^2, albedo and radiance at alb + c P, rad + c P.
template <int NB, int CH>
__global__ __launch_bounds__(SHV_BLOCK) void k_shade_ch_fwd(const float* __restrict__ vis,
                                                            const float* __restrict__ nrm,
                                                            const float* __restrict__ alb,
                                                            const float* __restrict__ M, int64_t P,
                                                            float* __restrict__ rad) {
  constexpr int N = NB * NB;
  constexpr int SZ = MSupp<NB>::SIZE;
  __shared__ float Ms[CH * SZ];
#pragma unroll
  for (int c = 0; c < CH; ++c) stage_M<NB>(M + c * N * N, Ms + c * SZ, threadIdx.x, SHV_BLOCK);
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (p >= P) return;
  float V[N], H[N], Hb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) V[i] = vis[(int64_t)i * P + p];
  float ux, uy, uz;
  transfer<NB>(nrm[p], nrm[P + p], nrm[2 * P + p], H, ux, uy, uz);
#pragma unroll
  for (int c = 0; c < CH; ++c)
    rad[c * P + p] = alb[c * P + p] * shade_value<NB, false>(V, H, Ms + c * SZ, 0.0f, Hb);
}

// Adjoint of k_shade_ch_fwd.  gB, gA [CH][P]; gV [N][P] and gN [3][P] summed
// over the channels; Lpart [CH][ceil(P / 64)][N] tile partials.
template <int NB, int CH>
__global__ __launch_bounds__(SHV_BLOCK) void k_shade_ch_bwd(const float* __restrict__ gB,
                                                            const float* __restrict__ vis,
                                                            const float* __restrict__ nrm,
                                                            const float* __restrict__ alb,
                                                            const float* __restrict__ M, int64_t P,
                                                            float* __restrict__ gV, float* __restrict__ gN,
                                                            float* __restrict__ gA, float* __restrict__ Lpart) {
  constexpr int N = NB * NB;
  constexpr int SZ = MSupp<NB>::SIZE;
  __shared__ LightTile T;
  __shared__ float Ms[CH * SZ];
#pragma unroll
  for (int c = 0; c < CH; ++c) stage_M<NB>(M + c * N * N, Ms + c * SZ, threadIdx.x, SHV_BLOCK);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const bool ok = p < P;
  float V[N], H[N], Hb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) V[i] = ok ? vis[(int64_t)i * P + p] : 0.0f;
  float ux, uy, uz;
  const float inv = transfer<NB>(ok ? nrm[p] : 0.0f, ok ? nrm[P + p] : 0.0f, ok ? nrm[2 * P + p] : 1.0f, H, ux, uy, uz);
#pragma unroll
  for (int i = 0; i < N; ++i) Hb[i] = 0.0f;
  float w[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const float bb = ok ? gB[c * P + p] : 0.0f;
    w[c] = bb * (ok ? alb[c * P + p] : 0.0f);
    const float s = shade_value_acc<NB>(V, H, Ms + c * SZ, w[c], Hb);
    if (ok && gA) gA[c * P + p] = bb * s;
  }
  if (ok) {
    if (gV) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        float acc = vbar_entry<NB>(j, H, Ms, w[0]);
#pragma unroll
        for (int c = 1; c < CH; ++c) acc += vbar_entry<NB>(j, H, Ms + c * SZ, w[c]);
        gV[(int64_t)j * P + p] = acc;
      }
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
  const int64_t tiles = (P + 63) / 64;
  for (int r = 0; r < SHV_WAVES_PER_BLOCK; ++r) {
    const int64_t tile = (int64_t)blockIdx.x * SHV_WAVES_PER_BLOCK + r;
    if (tile * 64 >= P) break;  // uniform
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      if (wave == r) {  // the V rows too: tile_light_partial reuses them for Q
        tile_put_v<NB>(T, lane, V);
        tile_put_wh<NB>(T, lane, H, w[c]);
      }
      __syncthreads();
      tile_light_partial<NB>(T, Lpart + (c * tiles + tile) * N);
    }
  }
}

// Eq. 9 on an equirectangular map img [channels][H][W]: row r spans polar
// angles [r, r + 1] pi / H from +z, column x azimuths [x, x + 1] 2 pi / W;
// a pixel's solid angle is (cos th_r - cos th_{r+1}) 2 pi / W, evaluated as
// 2 sin(th_centre) sin(pi / 2H) 2 pi / W (no cancellation near the poles).
// Block (r, c) writes part[(c H + r) N + i] = sum over the row's pixels of
// value * y_i(centre direction) * solid angle.  Lanes stride over the row,
// the 64 lanes of a wave are summed by a fixed butterfly and the four waves
// in order.
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_envmap_rows(const float* __restrict__ img, int64_t H, int64_t W,
                                                           float* __restrict__ part) {
  constexpr int N = NB * NB;
  __shared__ float red[SHV_WAVES_PER_BLOCK][N];
  const int64_t r = blockIdx.x;
  const int c = blockIdx.y;
  const double th = (double)M_PI * ((double)r + 0.5) / (double)H;
  const float st = (float)sin(th), ct = (float)cos(th);
  const float wrow = (float)(2.0 * sin(th) * sin(M_PI / (2.0 * (double)H)) * (2.0 * M_PI / (double)W));
  const float dphi = (float)(2.0 * M_PI / (double)W);
  const float* row = img + ((int64_t)c * H + r) * W;
  float acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0.0f;
  for (int64_t x = threadIdx.x; x < W; x += SHV_BLOCK) {
    float sp, cp;
    sincosf(((float)x + 0.5f) * dphi, &sp, &cp);
    float Y[N];
    sh_eval<NB>(st * cp, st * sp, ct, Y);
    const float v = row[x];
#pragma unroll
    for (int i = 0; i < N; ++i) acc[i] = fmaf(v, Y[i], acc[i]);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float t = wave_sum(acc[i]);
    if (lane == 0) red[wave][i] = t;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int i = threadIdx.x;
    float s = red[0][i];
#pragma unroll
    for (int g = 1; g < SHV_WAVES_PER_BLOCK; ++g) s += red[g][i];
    part[((int64_t)c * H + r) * N + i] = s * wrow;
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

template <int NB>
hipError_t shade_ch_fwd_nb(const float* vis, const float* nrm, const float* alb, const float* M, int channels,
                           int64_t P, float* rad, hipStream_t st) {
  const unsigned g = (unsigned)point_blocks(P);
  switch (channels) {
    case 1: k_shade_ch_fwd<NB, 1><<<g, SHV_BLOCK, 0, st>>>(vis, nrm, alb, M, P, rad); break;
    case 2: k_shade_ch_fwd<NB, 2><<<g, SHV_BLOCK, 0, st>>>(vis, nrm, alb, M, P, rad); break;
    case 3: k_shade_ch_fwd<NB, 3><<<g, SHV_BLOCK, 0, st>>>(vis, nrm, alb, M, P, rad); break;
    case 4: k_shade_ch_fwd<NB, 4><<<g, SHV_BLOCK, 0, st>>>(vis, nrm, alb, M, P, rad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NB>
hipError_t shade_ch_bwd_nb(const float* gB, const float* vis, const float* nrm, const float* alb, const float* M,
                           int channels, int64_t P, float* gV, float* gN, float* gA, float* Lpart, hipStream_t st) {
  const unsigned g = (unsigned)point_blocks(P);
  switch (channels) {
#define SHV_CH_BWD(c) \
  case c: k_shade_ch_bwd<NB, c><<<g, SHV_BLOCK, 0, st>>>(gB, vis, nrm, alb, M, P, gV, gN, gA, Lpart); break;
    SHV_CH_BWD(1)
    SHV_CH_BWD(2)
    SHV_CH_BWD(3)
    SHV_CH_BWD(4)
#undef SHV_CH_BWD
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int NB>
hipError_t envmap_rows_nb(const float* img, int channels, int64_t H, int64_t W, float* part, hipStream_t st) {
  k_envmap_rows<NB><<<dim3((unsigned)H, (unsigned)channels), SHV_BLOCK, 0, st>>>(img, H, W, part);
  return hipGetLastError();
}

}  // namespace shv
