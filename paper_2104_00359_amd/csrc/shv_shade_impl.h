// Diffuse SH shading B = a (L . (V * H)) (Eq. 8) and its adjoint, as
// separate entry points (sh_shade, sh_shade_backward).
//
// With the lit transfer matrix M(L)_jk = sum_i L_i C_ijk (symmetric, built once
// per call from L), B = a V^T M H.  The clamped-cosine transfer is
// H_lm = A_l y_lm(n / |n|) (Eqs. 10-11): its odd bands above 1 vanish, so only
// the columns of M on H's support are ever read (31 of 64 at n = 8).
// Each block first copies those columns of M into LDS (stage_M).
//
// One to four colour channels (one light L_c and albedo a_c per channel, one
// shared visibility, Eq. 8 per channel) are shaded by one launch that stages
// every channel's M and reads V and H once; sh_shade is the one-channel case.
// Channel c's radiance, albedo gradient and lighting gradient are bitwise
// those of a one-channel call, and the V and normal cotangents are summed
// over the channels in channel order.
//
// Environment-map projection (Eq. 9): L_i = integral of L(w) y_i(w) dw over
// an equirectangular map, as the sum over pixels of value * y_i(pixel centre)
// * pixel solid angle; a block covers several rows of one channel, and the
// block partials are then added in row order.
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

// Channel y = blockIdx.y: M + y N^2 from L + y N.
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_build_M(const float* __restrict__ L, float* __restrict__ M) {
  constexpr int N = NB * NB;
  const int y = blockIdx.y;
  build_M_range<NB>(L + y * N, M + y * N * N, blockIdx.x * SHV_BLOCK + threadIdx.x, gridDim.x * SHV_BLOCK);
}

// Rows i = G, G + 4, ... of a row-major [N][P] array at receiver p into LDS
// dst[i * row_pitch + lane * lane_pitch] (0 when !ok).  The row index is
// formed at run time from the wave number, so every load is issued before
// the first wait (no per-row branch).
template <int N>
__device__ __forceinline__ void load_rows_by_wave(const float* __restrict__ src, int64_t P, int64_t p, bool ok, int G,
                                                  float* dst, int row_pitch, int lane_pitch, int lane) {
  constexpr int T = (N + 3) / 4;
  float v[T];
  const int64_t pp = ok ? p : 0;
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int i = 4 * t + G;
    const int ii = i < N ? i : N - 1;  // in bounds; the value is dropped below
    v[t] = src[(int64_t)ii * P + pp];
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int i = 4 * t + G;
    if (i < N) dst[i * row_pitch + lane * lane_pitch] = ok ? v[t] : 0.0f;
  }
}

template <int NB, int CH>
struct ShadeCh4Shared {
  float X[NB * NB][64];        // V exchange (row i, receiver lane)
  float Ms[CH * MSupp<NB>::SIZE];
  float Bx[CH][4][64];         // shading partials per channel and column group
};

// Wave G's column group of every channel's shading value: shade_partial's
// sums (each column over j in index order, then the group's columns in
// order), for all channels in one pass over the rows, with V_j read from the
// LDS exchange (X[j][lane]) as it is consumed rather than held in registers.
template <int NB, int G, int CH>
__device__ __forceinline__ void shade_ch_fwd_group(ShadeCh4Shared<NB, CH>& sh, const float (&H)[NB * NB], int lane) {
  constexpr int N = NB * NB;
  float t[CH][MSupp<NB>::CPG], Hb[N];
  col_sums<NB, G, CH>([&](int j) { return sh.X[j][lane]; }, sh.Ms, t);
#pragma unroll
  for (int c = 0; c < CH; ++c) sh.Bx[c][G][lane] = shade_from_cols<NB, G, false>(t[c], H, 0.0f, Hb);
}

template <int NB, int CH>
__global__ __launch_bounds__(SHV_BLOCK, 2) void k_shade_ch_fwd(const float* __restrict__ vis,
                                                            const float* __restrict__ nrm,
                                                            const float* __restrict__ alb,
                                                            const float* __restrict__ M, int64_t P,
                                                            float* __restrict__ rad) {
  constexpr int N = NB * NB;
  constexpr int SZ = MSupp<NB>::SIZE;
  __shared__ ShadeCh4Shared<NB, CH> sh;
  const int G = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = p < P;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  load_rows_by_wave<N>(vis, P, p, ok, G, &sh.X[0][0], 64, 1, lane);
#pragma unroll
  for (int c = 0; c < CH; ++c) stage_M<NB>(M + c * N * N, sh.Ms + c * SZ, threadIdx.x);
  float H[N], ux, uy, uz;
  transfer<NB>(sel0(ok, nrm[q]), sel0(ok, nrm[P + q]), sel0(ok, nrm[2 * P + q], 1.0f), H, ux, uy, uz);
  __syncthreads();
  switch (G) {
    case 0: shade_ch_fwd_group<NB, 0, CH>(sh, H, lane); break;
    case 1: shade_ch_fwd_group<NB, 1, CH>(sh, H, lane); break;
    case 2: shade_ch_fwd_group<NB, 2, CH>(sh, H, lane); break;
    default: shade_ch_fwd_group<NB, 3, CH>(sh, H, lane); break;
  }
  __syncthreads();
  if (!ok) return;
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if ((c & 3) == G)
      rad[c * P + p] = alb[c * P + p] * (((sh.Bx[c][0][lane] + sh.Bx[c][1][lane]) + sh.Bx[c][2][lane]) +
                                         sh.Bx[c][3][lane]);
}

template <int NB, int CH>
struct ShadeCh4BwdShared {
  LightTile LT;                // its V rows hold the block's V (tile layout) throughout
  float Ms[CH * MSupp<NB>::SIZE];
  float Sx[CH][4][64];         // shading partials per channel and column group
  union {
    float HbX[32][64];         // shading blocks: y_k cotangents (summed over channels) on the transfer support
    float Q[NB * NB * 32];     // lighting blocks: the tile GEMM's Q (the V rows survive)
  };
  float W[CH][64];             // w = Bbar a per channel and receiver
};

// Wave G's part of the adjoint: its column group of the shading value and of
// the y_k cotangents (summed over channels; all channels' column sums in one
// pass, so their matrix chains interleave), and the V cotangent rows
// j = G (mod 4), each summed over the channels in channel order.
template <int NB, int G, int CH>
__device__ __forceinline__ void shade_ch_bwd_group(ShadeCh4BwdShared<NB, CH>& sh, int lane, int64_t p, bool ok,
                                                   int64_t P, const float* __restrict__ nrm,
                                                   float* __restrict__ gV) {
  constexpr int N = NB * NB;
  constexpr int SZ = MSupp<NB>::SIZE;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  float H[N], Hb[N], ux, uy, uz;
  transfer<NB>(sel0(ok, nrm[q]), sel0(ok, nrm[P + q]), sel0(ok, nrm[2 * P + q], 1.0f), H, ux, uy, uz);
#pragma unroll
  for (int i = 0; i < N; ++i) Hb[i] = 0.0f;
  {
    float t[CH][MSupp<NB>::CPG];
    col_sums<NB, G, CH>([&](int j) { return sh.LT.Vt[lane * kTileVS + j]; }, sh.Ms, t);  // V_j read as consumed
#pragma unroll
    for (int c = 0; c < CH; ++c) sh.Sx[c][G][lane] = shade_from_cols<NB, G, true, true>(t[c], H, sh.W[c][lane], Hb);
  }
  int kk = 0;
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (!h_support(l)) continue;
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      if ((kk & 3) == G) sh.HbX[kk][lane] = Hb[idx(l, m)];
      ++kk;
    }
  }
  constexpr int R = (N - G + 3) / 4;  // rows j = G, G + 4, ... (none for some waves at 1 band)
  if constexpr (R > 0) {
    if (!gV) return;  // uniform: the matrix steps need every lane
    float acc[R], vb[R];
    vbar_rows<NB, R>([](int r) { return G + 4 * r; }, H, sh.Ms, sh.W[0][lane], acc);
#pragma nounroll
    for (int c = 1; c < CH; ++c) {
      vbar_rows<NB, R>([](int r) { return G + 4 * r; }, H, sh.Ms + c * SZ, sh.W[c][lane], vb);
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] += vb[r];
    }
    if (ok) {
#pragma unroll
      for (int r = 0; r < R; ++r) gV[(int64_t)(G + 4 * r) * P + p] = acc[r];
    }
  }
}

// Adjoint of k_shade_ch_fwd.  gB, gA [CH][P]; gV [N][P] and gN [3][P] summed
// over the channels; Lpart [CH][ceil(P / 64)][N]: one lighting-gradient
// partial per tile of 64 receivers and channel.  A tile's work is split over
// blocks (grid.y = 1 + CH when Lpart is wanted): y = 0 the shading adjoint
// (abar, Vbar, nbar), y = 1 + c channel c's lighting-gradient GEMM, so more
// and shorter blocks share the chip at sizes that do not fill it.
template <int NB, int CH>
__global__ __launch_bounds__(SHV_BLOCK, 2) void k_shade_ch_bwd(const float* __restrict__ gB,
                                                               const float* __restrict__ vis,
                                                               const float* __restrict__ nrm,
                                                               const float* __restrict__ alb,
                                                               const float* __restrict__ M, int64_t P,
                                                               float* __restrict__ gV, float* __restrict__ gN,
                                                               float* __restrict__ gA, float* __restrict__ Lpart) {
  constexpr int N = NB * NB;
  constexpr int SZ = MSupp<NB>::SIZE;
  __shared__ ShadeCh4BwdShared<NB, CH> sh;
  const int G = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t tile = blockIdx.x;
  const int64_t p = tile * 64 + lane;
  const bool ok = p < P;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const bool light = blockIdx.y > 0;  // uniform
  load_rows_by_wave<N>(vis, P, p, ok, G, sh.LT.Vt, 1, kTileVS, lane);
  if (!light) {
#pragma unroll
    for (int c = 0; c < CH; ++c) stage_M<NB>(M + c * N * N, sh.Ms + c * SZ, threadIdx.x);
  }
  if (G == 0) {
#pragma unroll
    for (int c = 0; c < CH; ++c) sh.W[c][lane] = sel0(ok, gB[c * P + q] * alb[c * P + q]);
  }
  if (light) {
    float H[N], ux, uy, uz;
    transfer<NB>(sel0(ok, nrm[q]), sel0(ok, nrm[P + q]), sel0(ok, nrm[2 * P + q], 1.0f), H, ux, uy, uz);
    __syncthreads();  // W and the V rows in place
    const int c = (int)blockIdx.y - 1;
    // w H rows of channel c, wave G writing the support columns kk = G (mod 4)
    const float w = sh.W[c][lane];
    int kk = 0;
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      if (!h_support(l)) continue;
#pragma unroll
      for (int m = -l; m <= l; ++m) {
        if ((kk & 3) == G) sh.LT.Ht[lane * kTileHS + kk] = w * H[idx(l, m)];
        ++kk;
      }
    }
    __syncthreads();
    tile_light_partial<NB>(sh.LT, Lpart + (c * ((P + 63) / 64) + tile) * N, sh.Q);
    return;
  }
  __syncthreads();
  switch (G) {
    case 0: shade_ch_bwd_group<NB, 0, CH>(sh, lane, p, ok, P, nrm, gV); break;
    case 1: shade_ch_bwd_group<NB, 1, CH>(sh, lane, p, ok, P, nrm, gV); break;
    case 2: shade_ch_bwd_group<NB, 2, CH>(sh, lane, p, ok, P, nrm, gV); break;
    default: shade_ch_bwd_group<NB, 3, CH>(sh, lane, p, ok, P, nrm, gV); break;
  }
  __syncthreads();  // Sx, HbX, HsX complete
  if (G == 0 && ok && gA) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
      gA[c * P + p] = gB[c * P + p] *
                      (((sh.Sx[c][0][lane] + sh.Sx[c][1][lane]) + sh.Sx[c][2][lane]) + sh.Sx[c][3][lane]);
  }
  if (G == 1 && ok && gN) {
    float Hb[N], ux, uy, uz;
    const float inv = unit_normal(nrm[p], nrm[P + p], nrm[2 * P + p], ux, uy, uz);
#pragma unroll
    for (int i = 0; i < N; ++i) Hb[i] = 0.0f;
    int kk = 0;
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      if (!h_support(l)) continue;
#pragma unroll
      for (int m = -l; m <= l; ++m) Hb[idx(l, m)] = sh.HbX[kk++][lane];
    }
    float gx, gy, gz;
    normal_grad<NB>(Hb, ux, uy, uz, inv, gx, gy, gz);
    gN[p] = gx;
    gN[P + p] = gy;
    gN[2 * P + p] = gz;
  }
}

// Eq. 9 on an equirectangular map img [channels][H][W]: row r spans polar
// angles [r, r + 1] pi / H from +z, column x azimuths [x, x + 1] 2 pi / W;
// a pixel's solid angle is (cos th_r - cos th_{r+1}) 2 pi / W, evaluated as
// 2 sin(th_centre) sin(pi / 2H) 2 pi / W (no cancellation near the poles).
// Block (b, c) covers rows [b R, b R + R) of channel c: each lane takes the
// columns x = lane, lane + 256, ... (the azimuth's sine and cosine once per
// column) over those rows and accumulates value * solid angle * y_i; the
// block's 256 x N sums are then added through LDS in a fixed order (64-lane
// quarters, then the four quarters in order) into
// part[(c * gridDim.x + b) * N + i].
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_envmap_rows(const float* __restrict__ img, int64_t H, int64_t W,
                                                           int R, float* __restrict__ part) {
  constexpr int N = NB * NB;
  __shared__ float red[SHV_BLOCK * (N + 1)];
  __shared__ float rs[SHV_ENV_MAX_ROWS], rc[SHV_ENV_MAX_ROWS], rw[SHV_ENV_MAX_ROWS];
  const int c = blockIdx.y;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int nr = (int)((H - r0) < R ? (H - r0) : R);
  const int tid = threadIdx.x;
  if (tid < nr) {
    const double th = (double)M_PI * ((double)(r0 + tid) + 0.5) / (double)H;
    rs[tid] = (float)sin(th);
    rc[tid] = (float)cos(th);
    rw[tid] = (float)(2.0 * sin(th) * sin(M_PI / (2.0 * (double)H)) * (2.0 * M_PI / (double)W));
  }
  __syncthreads();
  const float dphi = (float)(2.0 * M_PI / (double)W);
  const float* base = img + ((int64_t)c * H + r0) * W;
  float acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0.0f;
  for (int64_t x = tid; x < W; x += SHV_BLOCK) {
    float sp, cp;
    sincosf(((float)x + 0.5f) * dphi, &sp, &cp);
    for (int r = 0; r < nr; ++r) {
      const float st = rs[r];
      float Y[N];
      sh_eval<NB>(st * cp, st * sp, rc[r], Y);
      const float v = base[(int64_t)r * W + x] * rw[r];
#pragma unroll
      for (int i = 0; i < N; ++i) acc[i] = fmaf(v, Y[i], acc[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i) red[tid * (N + 1) + i] = acc[i];
  __syncthreads();
  const int i = tid & 63, q = tid >> 6;
  float s = 0.0f;
  if (i < N) {
    for (int x = 0; x < 64; ++x) s += red[(q * 64 + x) * (N + 1) + i];
  }
  __syncthreads();
  if (i < N) red[q * 64 + i] = s;
  __syncthreads();
  if (tid < N)
    part[((int64_t)c * gridDim.x + blockIdx.x) * N + tid] = ((red[tid] + red[64 + tid]) + red[128 + tid]) + red[192 + tid];
}

// ---------------------------------------------------------------------------
// Launchers for one band count (instantiated per band count in shv_nb.hip).

template <int NB>
hipError_t build_M_nb(const float* light, float* M, int channels, hipStream_t st) {
  constexpr int NN = NB * NB * NB * NB;
  k_build_M<NB><<<dim3((unsigned)((NN + SHV_BLOCK - 1) / SHV_BLOCK), (unsigned)channels), SHV_BLOCK, 0, st>>>(light,
                                                                                                              M);
  return hipGetLastError();
}

template <int NB>
hipError_t shade_ch_fwd_nb(const float* vis, const float* nrm, const float* alb, const float* M, int channels,
                           int64_t P, float* rad, hipStream_t st) {
  const unsigned g = (unsigned)pair_blocks(P);
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
  const dim3 g((unsigned)pair_blocks(P), Lpart ? 1u + (unsigned)channels : 1u);
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
  const int R = envmap_rows_per_block(W);
  const unsigned nblk = (unsigned)((H + R - 1) / R);
  k_envmap_rows<NB><<<dim3(nblk, (unsigned)channels), SHV_BLOCK, 0, st>>>(img, H, W, R, part);
  return hipGetLastError();
}

}  // namespace shv
