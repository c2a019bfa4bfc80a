// The scaling-and-squaring exponential with a truncated Taylor series in
// place of the linear approximation, and its adjoint.
//
// With c = F_0 / sqrt(4 pi) and G = (F with F_0 := 0) 2^-k as in the main
// exponential:
//   E_0 = sum_{j <= K} G^{*j} / j!   (truncated products, G^{*0} = 1)
//   E_{j+1} = E_j * E_j,  V = exp(c) E_k.
// E_0 is formed by Horner's rule, R_K = 1, R_{j-1} = 1 + (R_j * G) / j,
// E_0 = R_0 (the same sum: truncated products are linear in each factor).
// Adjoint of one Horner step, with Rb the cotangent of R_{j-1}:
//   Gbar += (Rb * R_j) / j,   Rbar_j = (Rb * G) / j
// (the triple-product tensor is symmetric).  The generated adjoint of the
// squaring computes 2 (a * b) for any a and b, output group by output group.
//
// Saved for the adjoint, coefficient-major [rows][P]: row 0 = c, rows
// 1 + j N + i = E_j[i] (j < k), rows 1 + k N + i = G[i], rows
// 1 + (k + 1 + j - 1) N + i = R_j[i] (1 <= j < K).
//
// Layout: four waves per 64 receivers, wave G owning one output group of each
// product, the full vectors exchanged through double-buffered LDS (as the
// four-wave squaring kernels).

#pragma once

#include "shv_exp_impl.h"

namespace shv {

template <int NB>
struct TaylorShared {
  float X[2][NB * NB][64];
  float Gx[NB * NB][64];  // G, read in full by every wave in the adjoint
  float Cb[4][64];        // cbar partial per output group
};

template <int NB, int G>
__device__ __forceinline__ void taylor_fwd_group(TaylorShared<NB>& sh, int lane, int64_t p, bool ok,
                                                 const float* __restrict__ Fpart, int nchunks, int64_t P, float eps,
                                                 int k, int K, float* __restrict__ vis, float* __restrict__ saved) {
  constexpr int N = NB * NB;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  // Sphere-chunk partials of this wave's group, summed in chunk order.
  float F[N];
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (group_of<NB>(i) == G) F[i] = sel0(ok, Fpart[(int64_t)i * P + q]);
  for (int c = 1; c < nchunks; ++c) {
    const float* src = Fpart + (int64_t)c * N * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) F[i] += sel0(ok, src[(int64_t)i * P]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (group_of<NB>(i) == G) sh.X[0][i][lane] = F[i];
  __syncthreads();
  int b = 1;  // next exchange buffer
  float Gv[N], R[N], T[N];
#pragma unroll
  for (int i = 0; i < N; ++i) Gv[i] = sh.X[0][i][lane] * (eps * coef_lambda(i));
  const float c = Gv[0] * SHV_INV_SQRT_4PI;
  const float scale = __builtin_ldexpf(1.0f, -k);
  Gv[0] = 0.0f;
#pragma unroll
  for (int i = 1; i < N; ++i) Gv[i] *= scale;
  float* const grow = saved ? saved + (int64_t)(1 + k * N) * P + p : nullptr;
  if (saved && ok) {
    if (G == 0) saved[p] = c;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) grow[(int64_t)i * P] = Gv[i];
  }
  // Horner: R_K = 1, R_{j-1} = 1 + (R_j * G) / j.
#pragma unroll
  for (int i = 0; i < N; ++i) R[i] = i == 0 ? SHV_SQRT_4PI : 0.0f;
  for (int j = K; j >= 1; --j) {
    if (j < K && saved && ok) {
      float* dst = grow + (int64_t)j * N * P;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) dst[(int64_t)i * P] = R[i];
    }
    SqGroup<NB, G>::adj(R, Gv, T);  // group G of 2 (R_j * G)
    const float h = 0.5f / (float)j;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) sh.X[b][i][lane] = i == 0 ? fmaf(h, T[i], SHV_SQRT_4PI) : h * T[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) R[i] = sh.X[b][i][lane];
    b ^= 1;
  }
  // k truncated squarings of E_0 = R_0.
  for (int j = 0; j < k; ++j) {
    if (saved && ok) {
      float* dst = saved + (int64_t)(1 + j * N) * P + p;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (fgroup_of<NB>(i) == G) dst[(int64_t)i * P] = R[i];
    }
    SqGroup<NB, G>::square(R, T);
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (fgroup_of<NB>(i) == G) sh.X[b][i][lane] = T[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) R[i] = sh.X[b][i][lane];
    b ^= 1;
  }
  if (ok) {
    const float ec = expf(c);
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) vis[(int64_t)i * P + p] = ec * R[i];
  }
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_taylor_fwd(const float* __restrict__ Fpart, int nchunks, int64_t P,
                                                              float eps, int k, int K, float* __restrict__ vis,
                                                              float* __restrict__ saved) {
  __shared__ TaylorShared<NB> sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = p < P;
  switch (wave) {
    case 0: taylor_fwd_group<NB, 0>(sh, lane, p, ok, Fpart, nchunks, P, eps, k, K, vis, saved); break;
    case 1: taylor_fwd_group<NB, 1>(sh, lane, p, ok, Fpart, nchunks, P, eps, k, K, vis, saved); break;
    case 2: taylor_fwd_group<NB, 2>(sh, lane, p, ok, Fpart, nchunks, P, eps, k, K, vis, saved); break;
    default: taylor_fwd_group<NB, 3>(sh, lane, p, ok, Fpart, nchunks, P, eps, k, K, vis, saved); break;
  }
}

// Writes W_i = eps LAMBDA_i dLoss/dF_i, the weights of the pair adjoint.
template <int NB, int G>
__device__ __forceinline__ void taylor_bwd_group(TaylorShared<NB>& sh, int lane, int64_t p, bool ok,
                                                 const float* __restrict__ gIn, const float* __restrict__ vis,
                                                 const float* __restrict__ saved, int64_t P, float eps, int k, int K,
                                                 float* __restrict__ Wout) {
  constexpr int N = NB * NB;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const float c = sel0(ok, saved[q]);
  const float ec = expf(c);
  const float* const grow = saved + (int64_t)(1 + k * N) * P + q;
  {
    // Vbar (X[1]), G (Gx); group part of cbar = Vbar . V in index order
    float part = 0.0f;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (group_of<NB>(i) != G) continue;
      const float vb = sel0(ok, gIn[(int64_t)i * P + q]);
      const float v = sel0(ok, vis[(int64_t)i * P + q]);
      part = fmaf(vb, v, part);
      sh.X[1][i][lane] = vb;
      sh.Gx[i][lane] = grow[(int64_t)i * P];
    }
    sh.Cb[G][lane] = part;
  }
  __syncthreads();
  float Eb[N], A[N], T[N];
#pragma unroll
  for (int i = 0; i < N; ++i) Eb[i] = ec * sh.X[1][i][lane];
  const float cbar = ((sh.Cb[0][lane] + sh.Cb[1][lane]) + sh.Cb[2][lane]) + sh.Cb[3][lane];
  // Reverse squarings: Ebar_j = 2 (Ebar_{j+1} * E_j).
  for (int j = k - 1; j >= 0; --j) {
    __syncthreads();  // everyone has read X[0] / X[1] of the previous step
    const float* src = saved + (int64_t)(1 + j * N) * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) sh.X[0][i][lane] = src[(int64_t)i * P];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) A[i] = sh.X[0][i][lane];
    SqGroup<NB, G>::adj(Eb, A, T);
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) sh.X[1][i][lane] = T[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) Eb[i] = sh.X[1][i][lane];
  }
  // Horner adjoint, j = 1 .. K; Eb holds the cotangent of R_{j-1}.
  float Gb[N];
#pragma unroll
  for (int i = 0; i < N; ++i) Gb[i] = 0.0f;
  for (int j = 1; j <= K; ++j) {
    __syncthreads();  // everyone has read X[0] / X[1] of the previous step
    if (j < K) {
      const float* src = grow + (int64_t)j * N * P;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) sh.X[0][i][lane] = src[(int64_t)i * P];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < N; ++i) A[i] = sh.X[0][i][lane];
    } else {
#pragma unroll
      for (int i = 0; i < N; ++i) A[i] = i == 0 ? SHV_SQRT_4PI : 0.0f;
    }
    const float h = 0.5f / (float)j;
    SqGroup<NB, G>::adj(Eb, A, T);  // group G of 2 (Rb * R_j)
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) Gb[i] = fmaf(h, T[i], Gb[i]);
    if (j < K) {
#pragma unroll
      for (int i = 0; i < N; ++i) A[i] = sh.Gx[i][lane];
      SqGroup<NB, G>::adj(Eb, A, T);  // group G of 2 (Rb * G)
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) sh.X[1][i][lane] = h * T[i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < N; ++i) Eb[i] = sh.X[1][i][lane];
    }
  }
  if (!ok) return;
  const float scale = __builtin_ldexpf(1.0f, -k);
#pragma unroll
  for (int l = 0; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const int i = idx(l, m);
      if (group_of<NB>(i) != G) continue;
      const float lam = eps * SHV_LAMBDA[l][m < 0 ? -m : m];
      Wout[(int64_t)i * P + p] = i == 0 ? lam * (cbar * SHV_INV_SQRT_4PI) : lam * (scale * Gb[i]);
    }
  }
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_taylor_bwd(const float* __restrict__ gIn,
                                                              const float* __restrict__ vis,
                                                              const float* __restrict__ saved, int64_t P, float eps,
                                                              int k, int K, float* __restrict__ Wout) {
  __shared__ TaylorShared<NB> sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = p < P;
  switch (wave) {
    case 0: taylor_bwd_group<NB, 0>(sh, lane, p, ok, gIn, vis, saved, P, eps, k, K, Wout); break;
    case 1: taylor_bwd_group<NB, 1>(sh, lane, p, ok, gIn, vis, saved, P, eps, k, K, Wout); break;
    case 2: taylor_bwd_group<NB, 2>(sh, lane, p, ok, gIn, vis, saved, P, eps, k, K, Wout); break;
    default: taylor_bwd_group<NB, 3>(sh, lane, p, ok, gIn, vis, saved, P, eps, k, K, Wout); break;
  }
}

// ---------------------------------------------------------------------------
// Launchers for one band count (instantiated per band count in shv_nb.hip).

template <int NB>
hipError_t exp_taylor_fwd_nb(const float* Fpart, int nchunks, int64_t P, float eps, int k, int K, float* vis,
                             float* saved, hipStream_t st) {
  k_exp_taylor_fwd<NB><<<(unsigned)pair_blocks(P), SHV_BLOCK, 0, st>>>(Fpart, nchunks, P, eps, k, K, vis, saved);
  return hipGetLastError();
}

template <int NB>
hipError_t exp_taylor_bwd_nb(const float* gIn, const float* vis, const float* saved, int64_t P, float eps, int k,
                             int K, float* W, hipStream_t st) {
  k_exp_taylor_bwd<NB><<<(unsigned)pair_blocks(P), SHV_BLOCK, 0, st>>>(gIn, vis, saved, P, eps, k, K, W);
  return hipGetLastError();
}

}  // namespace shv
