// SH exponential V = exp*(F) and its adjoint.
//
// The paper replaces the product of blocker vectors (Eq. 12) by the
// exponential of the summed log-blockers and adopts Ren et al.'s scaling,
// squaring and optimal linear approximation.  With N = n^2 coefficients:
//   c   = F_0 / sqrt(4 pi)                 (the constant value of the DC part)
//   G   = (F with F_0 := 0) * 2^-k
//   E_0 = a (sqrt(4 pi) e_0 + G),  a = exp(|G|^2 / (8 pi))
//         (least-squares line a + b g through exp(g) when g's values over the
//          sphere are Gaussian with variance |G|^2 / (4 pi); it gives a = b)
//   E_{j+1} = E_j * E_j  (k truncated triple-product squarings, Eqs. 6-7)
//   V   = exp(c) E_k
// The squaring is straight-line generated code (coefficients are literals).
// Saved for the adjoint, coefficient-major: row 0 = c, rows 1 + j*N + i = E_j[i].
//
// The forward kernels also sum the sphere-chunk partials of F' in a fixed
// order and apply F_lm = eps * LAMBDA[l][|m|] * F'_lm.  The adjoint writes
// W = eps * LAMBDA * dLoss/dF, the weights the pair adjoint consumes.
//
// Two layouts, bitwise identical in their results: one receiver per lane
// (large receiver counts), or each receiver's squarings spread over the 4
// waves of a block, one output group per wave, exchanged through LDS (small
// receiver counts, where one wave per 64 receivers would leave most SIMDs
// idle).  With SHADE the kernels also run the shading step (forward) or its
// adjoint (backward) in the same launch, for the fused render entry points.

#pragma once

#include "shv_batch.h"
#include "shv_launch.h"
#include "shv_shade_common.h"
#include "shvis.h"

namespace shv {


template <int NB>
__device__ __forceinline__ void square(const float* e, float* o);
template <int NB>
__device__ __forceinline__ void square_adj(const float* ob, const float* e, float* eb);

#define SHV_SQ(n)                                                                                    \
  template <>                                                                                        \
  __device__ __forceinline__ void square<n>(const float* e, float* o) { shv_square_##n(e, o); }      \
  template <>                                                                                        \
  __device__ __forceinline__ void square_adj<n>(const float* ob, const float* e, float* eb) {        \
    shv_square_adj_##n(ob, e, eb);                                                                   \
  }
SHV_SQ(1)
SHV_SQ(2)
SHV_SQ(3)
SHV_SQ(4)
SHV_SQ(5)
SHV_SQ(6)
SHV_SQ(7)
SHV_SQ(8)
#undef SHV_SQ

// Group g of the output coefficients of one squaring (see the generator).
template <int NB, int G>
struct SqGroup;
#define SHV_SQG(n, g)                                                                                        \
  template <>                                                                                                \
  struct SqGroup<n, g> {                                                                                     \
    static __device__ __forceinline__ void square(const float* e, float* o) { shv_square_##n##_g##g(e, o); } \
    static __device__ __forceinline__ void adj(const float* ob, const float* e, float* eb) {                 \
      shv_square_adj_##n##_g##g(ob, e, eb);                                                                  \
    }                                                                                                        \
  };
#define SHV_SQG4(n) SHV_SQG(n, 0) SHV_SQG(n, 1) SHV_SQG(n, 2) SHV_SQG(n, 3)
SHV_SQG4(1)
SHV_SQG4(2)
SHV_SQG4(3)
SHV_SQG4(4)
SHV_SQG4(5)
SHV_SQG4(6)
SHV_SQG4(7)
SHV_SQG4(8)
#undef SHV_SQG4
#undef SHV_SQG

// Output group of coefficient i: in the adjoint squaring (and the canonical
// grouping of the backward's sums), and in the forward squaring.
template <int NB>
__device__ __forceinline__ constexpr int group_of(int i);
template <int NB>
__device__ __forceinline__ constexpr int fgroup_of(int i);
#define SHV_GOF(n)                                                                          \
  template <>                                                                               \
  __device__ __forceinline__ constexpr int group_of<n>(int i) { return SHV_GRP_##n[i]; }    \
  template <>                                                                               \
  __device__ __forceinline__ constexpr int fgroup_of<n>(int i) { return SHV_FGRP_##n[i]; }
SHV_GOF(1)
SHV_GOF(2)
SHV_GOF(3)
SHV_GOF(4)
SHV_GOF(5)
SHV_GOF(6)
SHV_GOF(7)
SHV_GOF(8)
#undef SHV_GOF

// The output-group table as a host-and-device constant expression.
template <int NB>
__host__ __device__ constexpr int group_entry(int i);
#define SHV_GENT(n) \
  template <>       \
  __host__ __device__ constexpr int group_entry<n>(int i) { return SHV_GRP_##n[i]; }
SHV_GENT(1)
SHV_GENT(2)
SHV_GENT(3)
SHV_GENT(4)
SHV_GENT(5)
SHV_GENT(6)
SHV_GENT(7)
SHV_GENT(8)
#undef SHV_GENT

// The coefficients of output group G in index order: v[0 .. n - 1].
template <int NB, int G>
struct GroupRows {
  int v[NB * NB];
  int n;
  constexpr GroupRows() : v{}, n(0) {
    for (int j = 0; j < NB * NB; ++j)
      if (group_entry<NB>(j) == G) v[n++] = j;
  }
};

// LAMBDA[l][|m|] of coefficient i (constant-folded after unrolling).
__device__ __forceinline__ float coef_lambda(int i) {
  int l = 0;
  while ((l + 1) * (l + 1) <= i) ++l;
  const int m = i - l * l - l;
  return SHV_LAMBDA[l][m < 0 ? -m : m];
}

// d loss / d c = V . Vbar, summed as four partial sums over the output groups
// (index order within a group), then over groups 0..3: the same order in the
// one-wave and four-wave kernels.
template <int NB>
__device__ __forceinline__ float cbar_canonical(const float* vb, const float* v) {
  constexpr int N = NB * NB;
  float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int i = 0; i < N; ++i) part[group_of<NB>(i)] = fmaf(vb[i], v[i], part[group_of<NB>(i)]);
  return ((part[0] + part[1]) + part[2]) + part[3];
}

// E_0 from the summed F' of one receiver (in place): returns c.
template <int NB>
__device__ __forceinline__ float exp_prologue(float (&E)[NB * NB], float eps, int k) {
  constexpr int N = NB * NB;
#pragma unroll
  for (int i = 0; i < N; ++i) E[i] *= eps * coef_lambda(i);
  const float c = E[0] * SHV_INV_SQRT_4PI;
  const float scale = __builtin_ldexpf(1.0f, -k);
  float sig = 0.0f;
#pragma unroll
  for (int i = 1; i < N; ++i) {
    E[i] *= scale;
    sig = fmaf(E[i], E[i], sig);
  }
  const float a = expf(sig * SHV_INV_8PI);
  E[0] = a * SHV_SQRT_4PI;
#pragma unroll
  for (int i = 1; i < N; ++i) E[i] *= a;
  return c;
}

// Adjoint of the linear approximation and of the scaling; E holds E_0 and Eb
// its cotangent.  Writes W_i = eps LAMBDA_i Fbar_i for coefficients i with
// keep(i).
template <int NB, class Keep>
__device__ __forceinline__ void exp_epilogue(float (&E)[NB * NB], const float (&Eb)[NB * NB], float cbar, float eps,
                                             int k, int64_t P, int64_t p, float* __restrict__ Wout, Keep keep) {
  constexpr int N = NB * NB;
  const float a = E[0] * SHV_INV_SQRT_4PI;
  const float inva = 1.0f / a;
  float dot = SHV_SQRT_4PI * Eb[0];
#pragma unroll
  for (int i = 1; i < N; ++i) {
    E[i] *= inva;  // G_i
    dot = fmaf(Eb[i], E[i], dot);
  }
  // Gbar_i = a (Ebar_i + G_i / (4 pi) (sqrt(4 pi) Ebar_0 + sum_j Ebar_j G_j))
  const float scale = __builtin_ldexpf(1.0f, -k);
  const float kdot = dot * SHV_INV_4PI;
  if (keep(0)) Wout[p] = eps * SHV_LAMBDA[0][0] * cbar * SHV_INV_SQRT_4PI;
#pragma unroll
  for (int l = 1; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const int i = idx(l, m);
      if (!keep(i)) continue;
      const float gb = a * fmaf(E[i], kdot, Eb[i]);
      Wout[(int64_t)i * P + p] = eps * SHV_LAMBDA[l][m < 0 ? -m : m] * scale * gb;
    }
  }
}

struct ShadeArgs {
  const float* nrm;  // [3][P]
  const float* alb;  // [P]
  const float* M;    // [N][N]
  float* rad;        // forward: radiance [P]
  float* gN;         // backward: normal cotangent [3][P] (may be NULL)
  float* gA;         // backward: albedo cotangent [P] (may be NULL)
  float* Lpart;      // backward: per-tile lighting-gradient partials [tiles][N] (may be NULL)
};

__device__ __forceinline__ void load_normal(const float* nrm, int64_t P, int64_t p, bool ok, float& x, float& y,
                                            float& z) {
  const int64_t q = ok ? p : 0;
  x = sel0(ok, nrm[q]);
  y = sel0(ok, nrm[P + q]);
  z = sel0(ok, nrm[2 * P + q], 1.0f);
}

// ===========================================================================
// One receiver per lane.

// With SHADE, Ms is block-local LDS of MSupp<NB>::SIZE floats for the staged M.
template <int NB, bool SHADE>
__device__ __forceinline__ void exp_fwd1_item(const float* __restrict__ Fpart, int nchunks, int64_t P, float eps,
                                              int k, float* __restrict__ vis, float* __restrict__ saved,
                                              const ShadeArgs& sa, int64_t bx, float* Ms) {
  constexpr int N = NB * NB;
  if constexpr (SHADE) {
    stage_M<NB>(sa.M, Ms, threadIdx.x);
    __syncthreads();
  }
  const int64_t p = bx * SHV_BLOCK + threadIdx.x;
  // Without shading a lane past the end leaves at once.  The shading's matrix
  // steps need every lane of the wave: there only waves wholly past the end
  // leave (no barrier follows), and tail lanes run receiver 0 and store
  // nothing.
  if (SHADE ? bx * SHV_BLOCK + (threadIdx.x & ~63) >= P : p >= P) return;
  const bool ok = p < P;
  const int64_t q = ok ? p : 0;
  float E[N], O[N];
#pragma unroll
  for (int i = 0; i < N; ++i) E[i] = Fpart[(int64_t)i * P + q];
  for (int c = 1; c < nchunks; ++c) {
    const float* src = Fpart + (int64_t)c * N * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] += src[(int64_t)i * P];
  }
  const float c = exp_prologue<NB>(E, eps, k);
  if (saved && ok) saved[p] = c;
  for (int j = 0; j < k; ++j) {
    if (saved && ok) {
      float* dst = saved + (int64_t)(1 + j * N) * P + p;
#pragma unroll
      for (int i = 0; i < N; ++i) dst[(int64_t)i * P] = E[i];
    }
    square<NB>(E, O);
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = O[i];
  }
  const float ec = expf(c);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    E[i] = ec * E[i];
    if (ok) vis[(int64_t)i * P + p] = E[i];
  }
  if constexpr (SHADE) {
    float H[N], Hb[N], nx, ny, nz, ux, uy, uz;
    load_normal(sa.nrm, P, p, ok, nx, ny, nz);
    transfer<NB>(nx, ny, nz, H, ux, uy, uz);
    const float s = shade_value<NB, false>(E, H, Ms, 0.0f, Hb);
    if (ok) sa.rad[p] = sa.alb[p] * s;
  }
}

template <int NB, bool SHADE>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_fwd(const float* __restrict__ Fpart, int nchunks, int64_t P,
                                                       float eps, int k, float* __restrict__ vis,
                                                       float* __restrict__ saved, ShadeArgs sa) {
  if constexpr (SHADE) {
    __shared__ float Ms[MSupp<NB>::SIZE];
    exp_fwd1_item<NB, SHADE>(Fpart, nchunks, P, eps, k, vis, saved, sa, blockIdx.x, Ms);
  } else {
    exp_fwd1_item<NB, SHADE>(Fpart, nchunks, P, eps, k, vis, saved, sa, blockIdx.x, nullptr);
  }
}

template <int NB, bool SHADE>
__device__ __forceinline__ void exp_bwd1_item(const float* __restrict__ gIn, const float* __restrict__ vis,
                                              const float* __restrict__ saved, int64_t P, float eps, int k,
                                              float* __restrict__ Wout, const ShadeArgs& sa, int64_t bx,
                                              LightTile* LTp, float* Ms) {
  constexpr int N = NB * NB;
  const int64_t p = bx * SHV_BLOCK + threadIdx.x;
  const bool ok = p < P;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  if (!SHADE && !ok) return;  // no barriers in the unfused kernel
  if constexpr (SHADE) {
    stage_M<NB>(sa.M, Ms, threadIdx.x);
    __syncthreads();
  }
  float Eb[N], E[N], T[N];
#pragma unroll
  for (int i = 0; i < N; ++i) E[i] = sel0(ok, vis[(int64_t)i * P + q]);  // V
  if constexpr (SHADE) {
    // gIn is the radiance cotangent: shading adjoint first (Vbar into Eb).
    LightTile& LT = *LTp;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float H[N], Hb[N], nx, ny, nz, ux, uy, uz;
#pragma unroll
    for (int i = 0; i < N; ++i) Hb[i] = 0.0f;
    load_normal(sa.nrm, P, p, ok, nx, ny, nz);
    const float inv = transfer<NB>(nx, ny, nz, H, ux, uy, uz);
    const float bb = sel0(ok, gIn[q]);
    const float w = bb * sel0(ok, sa.alb[q]);
    const float s = shade_value<NB, true>(E, H, Ms, w, Hb);
    if (ok && sa.gA) sa.gA[p] = bb * s;
    if (ok && sa.gN) {
      float gx, gy, gz;
      normal_grad<NB>(Hb, ux, uy, uz, inv, gx, gy, gz);
      sa.gN[p] = gx;
      sa.gN[P + p] = gy;
      sa.gN[2 * P + p] = gz;
    }
    if (sa.Lpart) {
      for (int r = 0; r < SHV_WAVES_PER_BLOCK; ++r) {
        const int64_t tile = bx * SHV_WAVES_PER_BLOCK + r;
        if (tile * 64 >= P) break;  // uniform
        if (wave == r) {
          tile_put_v<NB>(LT, lane, E);
          tile_put_wh<NB>(LT, lane, H, w);
        }
        __syncthreads();
        tile_light_partial<NB>(LT, sa.Lpart + tile * N);
      }
    }
    vbar_rows<NB, N>([](int r) { return r; }, H, Ms, w, Eb);
    if (!ok) return;  // no barriers or matrix steps below
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) Eb[i] = gIn[(int64_t)i * P + p];
  }
  const float c = saved[p];
  const float ec = expf(c);
  const float cbar = cbar_canonical<NB>(Eb, E);  // d/dc of exp(c) E_k . Vbar = V . Vbar
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (k == 0) E[i] = E[i] / ec;  // E_0 itself when there is no squaring
    Eb[i] = ec * Eb[i];
  }
  for (int j = k - 1; j >= 0; --j) {
    const float* src = saved + (int64_t)(1 + j * N) * P + p;
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = src[(int64_t)i * P];
    square_adj<NB>(Eb, E, T);  // Ebar_j = 2 (Ebar_{j+1} * E_j)
#pragma unroll
    for (int i = 0; i < N; ++i) Eb[i] = T[i];
  }
  exp_epilogue<NB>(E, Eb, cbar, eps, k, P, p, Wout, [](int) { return true; });
}

template <int NB, bool SHADE>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_bwd(const float* __restrict__ gIn, const float* __restrict__ vis,
                                                       const float* __restrict__ saved, int64_t P, float eps, int k,
                                                       float* __restrict__ Wout, ShadeArgs sa) {
  if constexpr (SHADE) {
    __shared__ LightTile LT;
    __shared__ float Ms[MSupp<NB>::SIZE];
    exp_bwd1_item<NB, SHADE>(gIn, vis, saved, P, eps, k, Wout, sa, blockIdx.x, &LT, Ms);
  } else {
    exp_bwd1_item<NB, SHADE>(gIn, vis, saved, P, eps, k, Wout, sa, blockIdx.x, nullptr, nullptr);
  }
}

// ===========================================================================
// Four waves per 64 receivers; wave G owns output group G.

template <int NB, int G, bool SHADE>
__device__ __forceinline__ void exp_fwd_group(float (*X)[NB * NB][64], float (*Bx)[64], int lane, int64_t p, bool ok,
                                              const float* __restrict__ Fpart, int nchunks, int64_t P, float eps,
                                              int k, float* __restrict__ vis, float* __restrict__ saved,
                                              const ShadeArgs& sa) {
  constexpr int N = NB * NB;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  // Sphere-chunk partials of this wave's group, summed in chunk order; the
  // loads of one chunk are issued together.
  float F[N];
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (fgroup_of<NB>(i) == G) F[i] = sel0(ok, Fpart[(int64_t)i * P + q]);
  for (int c = 1; c < nchunks; ++c) {
    const float* src = Fpart + (int64_t)c * N * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (fgroup_of<NB>(i) == G) F[i] += sel0(ok, src[(int64_t)i * P]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (fgroup_of<NB>(i) == G) X[0][i][lane] = F[i];
  __syncthreads();
  float E[N], O[N];
#pragma unroll
  for (int i = 0; i < N; ++i) E[i] = X[0][i][lane];
  const float c = exp_prologue<NB>(E, eps, k);
  if (G == 0 && saved && ok) saved[p] = c;
  for (int j = 0; j < k; ++j) {
    if (saved && ok) {
      float* dst = saved + (int64_t)(1 + j * N) * P + p;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (fgroup_of<NB>(i) == G) dst[(int64_t)i * P] = E[i];
    }
    SqGroup<NB, G>::square(E, O);
    const int b = (j + 1) & 1;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (fgroup_of<NB>(i) == G) X[b][i][lane] = O[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = X[b][i][lane];
  }
  const float ec = expf(c);
#pragma unroll
  for (int i = 0; i < N; ++i) E[i] = ec * E[i];  // V, complete in every wave
  if (ok) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (fgroup_of<NB>(i) == G) vis[(int64_t)i * P + p] = E[i];
  }
  if constexpr (SHADE) {
    // After the last barrier above every wave has read its final squares:
    // the other exchange buffer is free for the staged M.
    float* Ms = &X[(k + 1) & 1][0][0];
    stage_M<NB>(sa.M, Ms, G * 64 + lane);
    float H[N], Hb[N], nx, ny, nz, ux, uy, uz;
    load_normal(sa.nrm, P, p, ok, nx, ny, nz);
    transfer<NB>(nx, ny, nz, H, ux, uy, uz);
    __syncthreads();
    Bx[G][lane] = shade_partial<NB, G, false>(E, H, Ms, 0.0f, Hb);
    __syncthreads();
    if (G == 0 && ok) sa.rad[p] = sa.alb[p] * (((Bx[0][lane] + Bx[1][lane]) + Bx[2][lane]) + Bx[3][lane]);
  }
}

template <int NB>
struct Exp4FwdShared {
  float X[2][NB * NB][64];
  float Bx[4][64];
};

template <int NB, bool SHADE>
__device__ __forceinline__ void exp_fwd4_item(const float* __restrict__ Fpart, int nchunks, int64_t P, float eps,
                                              int k, float* __restrict__ vis, float* __restrict__ saved,
                                              const ShadeArgs& sa, int64_t bx, Exp4FwdShared<NB>& sh) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = bx * 64 + lane;
  const bool ok = p < P;
  switch (wave) {
    case 0: exp_fwd_group<NB, 0, SHADE>(sh.X, sh.Bx, lane, p, ok, Fpart, nchunks, P, eps, k, vis, saved, sa); break;
    case 1: exp_fwd_group<NB, 1, SHADE>(sh.X, sh.Bx, lane, p, ok, Fpart, nchunks, P, eps, k, vis, saved, sa); break;
    case 2: exp_fwd_group<NB, 2, SHADE>(sh.X, sh.Bx, lane, p, ok, Fpart, nchunks, P, eps, k, vis, saved, sa); break;
    default: exp_fwd_group<NB, 3, SHADE>(sh.X, sh.Bx, lane, p, ok, Fpart, nchunks, P, eps, k, vis, saved, sa); break;
  }
}

template <int NB, bool SHADE>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_fwd4(const float* __restrict__ Fpart, int nchunks, int64_t P,
                                                        float eps, int k, float* __restrict__ vis,
                                                        float* __restrict__ saved, ShadeArgs sa) {
  __shared__ Exp4FwdShared<NB> sh;
  exp_fwd4_item<NB, SHADE>(Fpart, nchunks, P, eps, k, vis, saved, sa, blockIdx.x, sh);
}

struct Bwd4Shared {
  float Cb[4][64];   // cbar partial per output group
  float Sx[4][64];   // shading partial per support-column group
  float HbX[32][64]; // y_k cotangents on the transfer support
};

// LDS of the four-wave adjoint.  The shading adjoint and the set-up of the
// squarings use X (V and Vbar), the partial sums, the lighting tile and the
// staged M; the squarings' adjoint then reuses all of it for two
// double-buffered exchanges (E_j by the parity of j, and each step's group
// outputs), so a step needs one barrier and the block no more LDS.
template <int NB>
struct Bwd4Loop {
  float E[2][NB * NB][64];
  float T[2][NB * NB][64];
};

template <int NB, int G, bool SHADE>
__device__ __forceinline__ void exp_bwd_group(float (*X)[NB * NB][64], Bwd4Shared& sh, LightTile& LT, float* Ms,
                                              Bwd4Loop<NB>& LB, int64_t bx,
                                              int lane, int64_t p, bool ok, const float* __restrict__ gIn,
                                              const float* __restrict__ vis, const float* __restrict__ saved,
                                              int64_t P, float eps, int k, float* __restrict__ Wout,
                                              const ShadeArgs& sa) {
  constexpr int N = NB * NB;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const float c = sel0(ok, saved[q]);
  const float ec = expf(c);
  float Eb[N], E[N], T[N];
  if constexpr (!SHADE) {
    // exchange Vbar (X[1]) and V (X[0]); group part of cbar in index order
    float part = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (group_of<NB>(i) != G) continue;
      const float vb = sel0(ok, gIn[(int64_t)i * P + q]);
      const float v = sel0(ok, vis[(int64_t)i * P + q]);
      part = fmaf(vb, v, part);
      X[1][i][lane] = vb;
      X[0][i][lane] = v;
    }
    sh.Cb[G][lane] = part;
    __syncthreads();
  } else {
    // V from the group loads, M staged; then the shading adjoint split over
    // the waves
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) X[0][i][lane] = sel0(ok, vis[(int64_t)i * P + q]);
    stage_M<NB>(sa.M, Ms, G * 64 + lane);
    __syncthreads();
    float V[N], H[N], Hb[N], nx, ny, nz, ux, uy, uz;
#pragma unroll
    for (int i = 0; i < N; ++i) V[i] = X[0][i][lane];
    load_normal(sa.nrm, P, p, ok, nx, ny, nz);
    const float inv = transfer<NB>(nx, ny, nz, H, ux, uy, uz);
    const float bb = sel0(ok, gIn[q]);
    const float w = bb * sel0(ok, sa.alb[q]);
    sh.Sx[G][lane] = shade_partial<NB, G, true>(V, H, Ms, w, Hb);
    {
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
    }
    constexpr GroupRows<NB, G> GR{};
    float vb[GR.n > 0 ? GR.n : 1];  // a group may be empty at 1 or 2 bands
    if constexpr (GR.n > 0) vbar_rows<NB, GR.n>([GR](int r) { return GR.v[r]; }, H, Ms, w, vb);
    float part = 0.0f;
#pragma unroll
    for (int r = 0; r < GR.n; ++r) {
      part = fmaf(vb[r], V[GR.v[r]], part);
      X[1][GR.v[r]][lane] = vb[r];
    }
    sh.Cb[G][lane] = part;
    if (G == 2) tile_put_v<NB>(LT, lane, V);
    if (G == 3) tile_put_wh<NB>(LT, lane, H, w);
    __syncthreads();
    if (G == 0 && ok && sa.gA)
      sa.gA[p] = bb * (((sh.Sx[0][lane] + sh.Sx[1][lane]) + sh.Sx[2][lane]) + sh.Sx[3][lane]);
    if (G == 1 && ok && sa.gN) {
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
      sa.gN[p] = gx;
      sa.gN[P + p] = gy;
      sa.gN[2 * P + p] = gz;
    }
    if (sa.Lpart) tile_light_partial<NB>(LT, sa.Lpart + bx * N);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) Eb[i] = ec * X[1][i][lane];
  if (k == 0) {  // E_0 = V / exp(c) when there is no squaring; the loop below loads E_j otherwise
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = X[0][i][lane] / ec;
  }
  const float cbar = ((sh.Cb[0][lane] + sh.Cb[1][lane]) + sh.Cb[2][lane]) + sh.Cb[3][lane];
  // This wave's group of E_j is loaded one step ahead, so the loads are in
  // flight during the previous step's product (barriers wait on LDS only).
  float pre[N];
  if (k > 0) {
    const float* src = saved + (int64_t)(1 + (k - 1) * N) * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) pre[i] = sel0(ok, src[(int64_t)i * P]);
  }
  __syncthreads();  // every wave has read X and the partials: the loop buffers overlay them from here
  if (k > 0) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) LB.E[(k - 1) & 1][i][lane] = pre[i];
    if (k > 1) {
      const float* src = saved + (int64_t)(1 + (k - 2) * N) * P + q;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) pre[i] = sel0(ok, src[(int64_t)i * P]);
    }
    __syncthreads();
  }
  // Step j reads E_j from LB.E[j & 1] (complete since the previous barrier),
  // stores its group of E_{j-1} into the other buffer (last read at step
  // j + 1, before that barrier), and exchanges its outputs through
  // LB.T[j & 1] (last read at step j + 2): one barrier per step.
  for (int j = k - 1; j >= 0; --j) {
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = LB.E[j & 1][i][lane];
    if (j > 0) {
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) LB.E[(j - 1) & 1][i][lane] = pre[i];
      if (j > 1) {
        const float* src = saved + (int64_t)(1 + (j - 2) * N) * P + q;
#pragma unroll
        for (int i = 0; i < N; ++i)
          if (group_of<NB>(i) == G) pre[i] = sel0(ok, src[(int64_t)i * P]);
      }
    }
    SqGroup<NB, G>::adj(Eb, E, T);
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) LB.T[j & 1][i][lane] = T[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) Eb[i] = LB.T[j & 1][i][lane];
  }
  if (!ok) return;
  exp_epilogue<NB>(E, Eb, cbar, eps, k, P, p, Wout, [](int i) { return group_of<NB>(i) == G; });
}

template <int NB>
struct Exp4BwdSetup {
  float X[2][NB * NB][64];
  Bwd4Shared sh;
  LightTile LT;
  float Ms[MSupp<NB>::SIZE];  // staged M (fused shading adjoint)
};

template <int NB>
union Exp4BwdShared {
  Exp4BwdSetup<NB> s;  // the shading adjoint and the set-up of the squarings
  Bwd4Loop<NB> loop;   // the adjoint squarings (overlays s: a barrier separates them)
};

template <int NB, bool SHADE>
__device__ __forceinline__ void exp_bwd4_item(const float* __restrict__ gIn, const float* __restrict__ vis,
                                              const float* __restrict__ saved, int64_t P, float eps, int k,
                                              float* __restrict__ Wout, const ShadeArgs& sa, int64_t bx,
                                              Exp4BwdShared<NB>& S) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = bx * 64 + lane;
  const bool ok = p < P;
  switch (wave) {
    case 0: exp_bwd_group<NB, 0, SHADE>(S.s.X, S.s.sh, S.s.LT, S.s.Ms, S.loop, bx, lane, p, ok, gIn, vis, saved, P, eps, k, Wout, sa); break;
    case 1: exp_bwd_group<NB, 1, SHADE>(S.s.X, S.s.sh, S.s.LT, S.s.Ms, S.loop, bx, lane, p, ok, gIn, vis, saved, P, eps, k, Wout, sa); break;
    case 2: exp_bwd_group<NB, 2, SHADE>(S.s.X, S.s.sh, S.s.LT, S.s.Ms, S.loop, bx, lane, p, ok, gIn, vis, saved, P, eps, k, Wout, sa); break;
    default:
      exp_bwd_group<NB, 3, SHADE>(S.s.X, S.s.sh, S.s.LT, S.s.Ms, S.loop, bx, lane, p, ok, gIn, vis, saved, P, eps, k, Wout, sa);
      break;
  }
}

template <int NB, bool SHADE>
__global__ __launch_bounds__(SHV_BLOCK, 2) void k_exp_bwd4(const float* __restrict__ gIn, const float* __restrict__ vis,
                                                        const float* __restrict__ saved, int64_t P, float eps, int k,
                                                        float* __restrict__ Wout, ShadeArgs sa) {
  __shared__ Exp4BwdShared<NB> S;
  exp_bwd4_item<NB, SHADE>(gIn, vis, saved, P, eps, k, Wout, sa, blockIdx.x, S);
}

// ---------------------------------------------------------------------------
// Launchers for one band count (instantiated per band count in shv_nb.hip).

template <int NB, bool SHADE>
hipError_t exp_fwd_nb(const float* Fpart, int nchunks, int64_t P, float eps, int k, float* vis, float* saved,
                      const float* nrm, const float* alb, const float* M, float* rad, uint32_t flags, hipStream_t st) {
  const ShadeArgs sa{nrm, alb, M, rad, nullptr, nullptr, nullptr};
  if (exp_four_waves(NB, P, flags, false)) {
    k_exp_fwd4<NB, SHADE><<<(unsigned)((P + 63) / 64), SHV_BLOCK, 0, st>>>(Fpart, nchunks, P, eps, k, vis, saved, sa);
  } else {
    k_exp_fwd<NB, SHADE><<<(unsigned)point_blocks(P), SHV_BLOCK, 0, st>>>(Fpart, nchunks, P, eps, k, vis, saved, sa);
  }
  return hipGetLastError();
}

template <int NB, bool SHADE>
hipError_t exp_bwd_nb(const float* gIn, const float* vis, const float* saved, int64_t P, float eps, int k, float* W,
                      const float* nrm, const float* alb, const float* M, float* gN, float* gA, float* Lpart,
                      uint32_t flags, hipStream_t st) {
  const ShadeArgs sa{nrm, alb, M, nullptr, gN, gA, Lpart};
  if (exp_four_waves(NB, P, flags, false)) {
    k_exp_bwd4<NB, SHADE><<<(unsigned)((P + 63) / 64), SHV_BLOCK, 0, st>>>(gIn, vis, saved, P, eps, k, W, sa);
  } else {
    k_exp_bwd<NB, SHADE><<<(unsigned)point_blocks(P), SHV_BLOCK, 0, st>>>(gIn, vis, saved, P, eps, k, W, sa);
  }
  return hipGetLastError();
}

// Batched phases of the fused render path: scenes with NB bands whose
// exponential uses the four-wave layout (FOUR) or the one-wave layout; one
// block per item of the group's item space (blocks beyond it exit).
template <int NB, bool FOUR>
__global__ __launch_bounds__(SHV_BLOCK) void k_batch_exp_fwd(const char* __restrict__ table) {
  __shared__ Exp4FwdShared<NB> sh;
  const BatchView v(table);
  const int64_t item = blockIdx.x;
  if (item >= v.h->total_exp[FOUR][NB]) return;
  const BatchScene S = in_global(v.scene_of_exp(FOUR, NB, item));
  const int64_t bx = S.exp_block0 + (item - S.off_exp);
  const ShadeArgs sa{S.normals, S.albedo, S.M, S.radiance, nullptr, nullptr, nullptr};
  if constexpr (FOUR) exp_fwd4_item<NB, true>(S.Fpart, S.nchunks_f, S.P, S.eps, S.k, S.vis, S.saved, sa, bx, sh);
  else exp_fwd1_item<NB, true>(S.Fpart, S.nchunks_f, S.P, S.eps, S.k, S.vis, S.saved, sa, bx, &sh.X[0][0][0]);
}

template <int NB, bool FOUR>
__global__ __launch_bounds__(SHV_BLOCK, FOUR ? 2 : 1) void k_batch_exp_bwd(const char* __restrict__ table) {
  __shared__ Exp4BwdShared<NB> sh;
  const BatchView v(table);
  const int64_t item = blockIdx.x;
  if (item >= v.h->total_exp[FOUR][NB]) return;
  const BatchScene S = in_global(v.scene_of_exp(FOUR, NB, item));
  if (!S.grad_radiance) return;  // uniform: scene packed without a cotangent
  const int64_t bx = S.exp_block0 + (item - S.off_exp);
  const ShadeArgs sa{S.normals, S.albedo, S.M, nullptr, S.grad_normals, S.grad_albedo, S.grad_light ? S.lp : nullptr};
  if constexpr (FOUR) exp_bwd4_item<NB, true>(S.grad_radiance, S.vis, S.saved, S.P, S.eps, S.k, S.W, sa, bx, sh);
  else exp_bwd1_item<NB, true>(S.grad_radiance, S.vis, S.saved, S.P, S.eps, S.k, S.W, sa, bx, &sh.s.LT, sh.s.Ms);
}

template <int NB>
hipError_t batch_exp_fwd_nb(const void* table, bool four, int64_t blocks, hipStream_t st) {
  if (four) k_batch_exp_fwd<NB, true><<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  else k_batch_exp_fwd<NB, false><<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  return hipGetLastError();
}

template <int NB>
hipError_t batch_exp_bwd_nb(const void* table, bool four, int64_t blocks, hipStream_t st) {
  if (four) k_batch_exp_bwd<NB, true><<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  else k_batch_exp_bwd<NB, false><<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  return hipGetLastError();
}

}  // namespace shv
