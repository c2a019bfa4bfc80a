// Scene parameterisation upstream of the spheres (Sec. 3.3.1, Sec. 3.5): the
// sphere centres are the nodes of an embedded deformation graph, each sphere
// attached to its K nearest template vertices and carrying a rotation
// (axis-angle a_k) and a translation t_k; a global rigid pose (a_0, t_0)
// follows.
//
//   y_j = sum_k w_jk (R_k (v_j - g_k) + g_k + t_k) + (1 - sum_k w_jk) v_j
//   z_j = sum_k w_jk R_k m_j + (1 - sum_k w_jk) m_j
//   x_j = R_0 y_j + t_0,   n_j = R_0 z_j,   c_k = R_0 (g_k + t_k) + t_0
//
// Rotation matrices by Rodrigues' formula R = I + A K + B K^2 with K = [a]x,
// A = sin t / t, B = (1 - cos t) / t^2, t = |a|; its derivative
// dR/da_i = A E_i + B (E_i K + K E_i) + a_i (C K + D K^2) with E_i = [e_i]x,
// C = A'(t) / t and D = B'(t) / t.  Below t = 0.5 the four coefficients are
// evaluated by their Taylor series (no cancellation).
//
// Adjoint, for cotangents xbar, nbar (per vertex) and cbar (per sphere):
//   ybar_j = R_0^T xbar_j,  zbar_j = R_0^T nbar_j
//   tbar_k = sum_{j attached to k} w_jk ybar_j + R_0^T cbar_k
//   Rbar_k = sum_{j attached to k} w_jk (ybar_j (v_j - g_k)^T + zbar_j m_j^T)
//   Rbar_0 = sum_j (xbar_j y_j^T + nbar_j z_j^T) + sum_k cbar_k (g_k + t_k)^T
//   tbar_0 = sum_j xbar_j + sum_k cbar_k
//   abar_i = <Rbar, dR/da_i>
// Every sum runs in a fixed order (per-vertex entries in sphere order, per
// sphere its K vertices in block-strided order reduced by a fixed tree, the
// global partials by the column reduction), so results are deterministic.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "shv_config.h"
#include "shv_device.h"
#include "shv_launch.h"

namespace shv {

// ---------------------------------------------------------------------------
// Attachment (host; a one-time preprocessing of the template).

int deform_graph_build(const float* vertices, int64_t P, const float* spheres, int64_t S, int K, int32_t* vert_ptr,
                       int32_t* vert_sph, float* vert_w, int32_t* sph_vert, float* sph_w) {
  std::vector<double> d2(P), u((size_t)S * K), tot(P, 0.0);
  std::vector<int64_t> order(P);
  std::vector<int32_t> count(P, 0);
  for (int64_t k = 0; k < S; ++k) {
    const double gx = spheres[4 * k], gy = spheres[4 * k + 1], gz = spheres[4 * k + 2];
    for (int64_t j = 0; j < P; ++j) {
      const double dx = (double)vertices[j] - gx, dy = (double)vertices[P + j] - gy,
                   dz = (double)vertices[2 * P + j] - gz;
      d2[j] = dx * dx + dy * dy + dz * dz;
    }
    std::iota(order.begin(), order.end(), 0);
    const int64_t take = std::min<int64_t>(P, (int64_t)K + 1);
    std::partial_sort(order.begin(), order.begin() + take, order.end(), [&](int64_t a, int64_t b) {
      return d2[a] < d2[b] || (d2[a] == d2[b] && a < b);
    });
    const double dmax = std::sqrt(K < P ? d2[order[K]] : d2[order[K - 1]]);
    for (int q = 0; q < K; ++q) {
      const int64_t j = order[q];
      double w = 0.0;
      if (dmax > 0.0) {
        const double r = 1.0 - std::sqrt(d2[j]) / dmax;
        w = r * r;
      }
      sph_vert[k * K + q] = (int32_t)j;
      u[k * K + q] = w;
      tot[j] += w;
      ++count[j];
    }
  }
  vert_ptr[0] = 0;
  for (int64_t j = 0; j < P; ++j) vert_ptr[j + 1] = vert_ptr[j] + count[j];
  std::vector<int32_t> fill(vert_ptr, vert_ptr + P);
  for (int64_t k = 0; k < S; ++k) {
    for (int q = 0; q < K; ++q) {
      const int64_t j = sph_vert[k * K + q];
      const double den = tot[j];
      const float w = den > 0.0 ? (float)(u[k * K + q] / den) : 0.0f;
      sph_w[k * K + q] = w;
      vert_sph[fill[j]] = (int32_t)k;
      vert_w[fill[j]] = w;
      ++fill[j];
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Rotation helpers (row-major 3 x 3).

__device__ __forceinline__ void rot_coeffs(float t2, float& A, float& B, float& C, float& D) {
  if (t2 < 0.25f) {
    A = 1.0f + t2 * (-1.0f / 6 + t2 * (1.0f / 120 + t2 * (-1.0f / 5040 + t2 * (1.0f / 362880))));
    B = 0.5f + t2 * (-1.0f / 24 + t2 * (1.0f / 720 + t2 * (-1.0f / 40320 + t2 * (1.0f / 3628800))));
    C = -1.0f / 3 + t2 * (1.0f / 30 + t2 * (-1.0f / 840 + t2 * (1.0f / 45360 + t2 * (-1.0f / 3991680))));
    D = -1.0f / 12 + t2 * (1.0f / 180 + t2 * (-1.0f / 6720 + t2 * (1.0f / 453600 + t2 * (-1.0f / 47900160))));
  } else {
    const float t = sqrtf(t2);
    float s, c;
    sincosf(t, &s, &c);
    A = s / t;
    B = (1.0f - c) / t2;
    C = (t * c - s) / (t2 * t);
    D = (t * s - 2.0f * (1.0f - c)) / (t2 * t2);
  }
}

__device__ __forceinline__ void skew3(const float* a, float (&K)[9]) {
  K[0] = 0.0f;  K[1] = -a[2]; K[2] = a[1];
  K[3] = a[2];  K[4] = 0.0f;  K[5] = -a[0];
  K[6] = -a[1]; K[7] = a[0];  K[8] = 0.0f;
}

__device__ __forceinline__ void mul3(const float (&X)[9], const float (&Y)[9], float (&Z)[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) Z[3 * r + c] = fmaf(X[3 * r], Y[c], fmaf(X[3 * r + 1], Y[3 + c], X[3 * r + 2] * Y[6 + c]));
}

__device__ __forceinline__ void rodrigues3(const float* a, float (&R)[9]) {
  float A, B, C, D, K[9], K2[9];
  rot_coeffs(a[0] * a[0] + a[1] * a[1] + a[2] * a[2], A, B, C, D);
  skew3(a, K);
  mul3(K, K, K2);
#pragma unroll
  for (int e = 0; e < 9; ++e) R[e] = (e % 4 == 0 ? 1.0f : 0.0f) + A * K[e] + B * K2[e];
}

// abar_i = <Rbar, dR/da_i>.
__device__ __forceinline__ void rodrigues3_adjoint(const float* a, const float (&Rb)[9], float* abar) {
  float A, B, C, D, K[9], K2[9];
  rot_coeffs(a[0] * a[0] + a[1] * a[1] + a[2] * a[2], A, B, C, D);
  skew3(a, K);
  mul3(K, K, K2);
  float rk = 0.0f, rk2 = 0.0f;
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    rk = fmaf(Rb[e], K[e], rk);
    rk2 = fmaf(Rb[e], K2[e], rk2);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float ei[3] = {0.0f, 0.0f, 0.0f}, E[9], EK[9], KE[9];
    ei[i] = 1.0f;
    skew3(ei, E);
    mul3(E, K, EK);
    mul3(K, E, KE);
    float re = 0.0f, rs = 0.0f;
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      re = fmaf(Rb[e], E[e], re);
      rs = fmaf(Rb[e], EK[e] + KE[e], rs);
    }
    abar[i] = A * re + B * rs + a[i] * (C * rk + D * rk2);
  }
}

// ---------------------------------------------------------------------------
// Kernels.

// R of every row of params [S + 1][6] into Rm [S + 1][9].
__global__ __launch_bounds__(SHV_BLOCK) void k_deform_rot(const float* __restrict__ params, int64_t rows,
                                                          float* __restrict__ Rm) {
  const int64_t r = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (r >= rows) return;
  float R[9];
  rodrigues3(params + 6 * r, R);
#pragma unroll
  for (int e = 0; e < 9; ++e) Rm[9 * r + e] = R[e];
}

// y_j and z_j of vertex j (the local stage).
__device__ __forceinline__ void deform_local(const DeformGraphDev& g, const float* __restrict__ params,
                                             const float* __restrict__ Rm, int64_t j, float (&y)[3],
                                             float (&z)[3]) {
  const int64_t P = g.P;
  const float v[3] = {g.vertices[j], g.vertices[P + j], g.vertices[2 * P + j]};
  const float m[3] = {g.normals[j], g.normals[P + j], g.normals[2 * P + j]};
  float sy[3] = {0.0f, 0.0f, 0.0f}, sz[3] = {0.0f, 0.0f, 0.0f}, wsum = 0.0f;
  const int32_t e0 = g.vert_ptr[j], e1 = g.vert_ptr[j + 1];
  for (int32_t e = e0; e < e1; ++e) {
    const int k = g.vert_sph[e];
    const float w = g.vert_w[e];
    const float* R = Rm + 9 * k;
    const float* gk = g.spheres + 4 * k;
    const float* tk = params + 6 * k + 3;
    const float d[3] = {v[0] - gk[0], v[1] - gk[1], v[2] - gk[2]};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const float rd = fmaf(R[3 * r], d[0], fmaf(R[3 * r + 1], d[1], R[3 * r + 2] * d[2]));
      const float rm = fmaf(R[3 * r], m[0], fmaf(R[3 * r + 1], m[1], R[3 * r + 2] * m[2]));
      sy[r] = fmaf(w, rd + gk[r] + tk[r], sy[r]);
      sz[r] = fmaf(w, rm, sz[r]);
    }
    wsum += w;
  }
  const float keep = wsum > 0.0f ? 0.0f : 1.0f;  // attached vertices: the weights sum to one
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    y[r] = fmaf(keep, v[r], sy[r]);
    z[r] = fmaf(keep, m[r], sz[r]);
  }
}

// Threads [0, P) deform vertex j; threads [P, P + S) move sphere k.
__global__ __launch_bounds__(SHV_BLOCK) void k_deform_fwd(DeformGraphDev g, const float* __restrict__ params,
                                                          const float* __restrict__ Rm, float* __restrict__ pts,
                                                          float* __restrict__ nrm, float* __restrict__ sph) {
  const int64_t i = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const int64_t P = g.P, S = g.S;
  const float* R0 = Rm + 9 * S;
  const float* t0 = params + 6 * S + 3;
  if (i < P) {
    float y[3], z[3];
    deform_local(g, params, Rm, i, y, z);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      pts[r * P + i] = fmaf(R0[3 * r], y[0], fmaf(R0[3 * r + 1], y[1], fmaf(R0[3 * r + 2], y[2], t0[r])));
      nrm[r * P + i] = fmaf(R0[3 * r], z[0], fmaf(R0[3 * r + 1], z[1], R0[3 * r + 2] * z[2]));
    }
  } else if (i < P + S) {
    const int64_t k = i - P;
    const float* gk = g.spheres + 4 * k;
    const float* tk = params + 6 * k + 3;
    const float c[3] = {gk[0] + tk[0], gk[1] + tk[1], gk[2] + tk[2]};
#pragma unroll
    for (int r = 0; r < 3; ++r)
      sph[4 * k + r] = fmaf(R0[3 * r], c[0], fmaf(R0[3 * r + 1], c[1], fmaf(R0[3 * r + 2], c[2], t0[r])));
    sph[4 * k + 3] = gk[3];
  }
}

// Sum of a value over the block's 256 threads in a fixed order (wave
// butterflies, then the four waves in order); every thread gets the total.
__device__ __forceinline__ float block_sum(float v, float* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// The same for 12 values at once (one pair of barriers); thread e < 12 of the
// block receives the total of value e in tot.
__device__ __forceinline__ void block_sum12(const float (&v)[12], float (*red)[12], float& tot) {
  const int wave = threadIdx.x >> 6;
  float w[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) w[e] = wave_sum(v[e]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int e = 0; e < 12; ++e) red[wave][e] = w[e];
  }
  __syncthreads();
  const int e = threadIdx.x < 12 ? threadIdx.x : 0;
  tot = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
}

// Per vertex: ybar, zbar into Yb [6][P]; the vertex terms of the global
// gradient (Rbar_0 row-major, then tbar_0) summed per block into
// Gpart[block][12].
__global__ __launch_bounds__(SHV_BLOCK) void k_deform_bwd_vert(DeformGraphDev g, const float* __restrict__ params,
                                                               const float* __restrict__ Rm,
                                                               const float* __restrict__ gx,
                                                               const float* __restrict__ gn, float* __restrict__ Yb,
                                                               float* __restrict__ Gpart) {
  __shared__ float red[SHV_WAVES_PER_BLOCK][12];
  const int64_t j = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const int64_t P = g.P, S = g.S;
  const float* R0 = Rm + 9 * S;
  float xb[3] = {0.0f, 0.0f, 0.0f}, nb[3] = {0.0f, 0.0f, 0.0f}, y[3] = {0.0f, 0.0f, 0.0f}, z[3] = {0.0f, 0.0f, 0.0f};
  if (j < P) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      xb[r] = gx ? gx[r * P + j] : 0.0f;
      nb[r] = gn ? gn[r * P + j] : 0.0f;
    }
    deform_local(g, params, Rm, j, y, z);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Yb[c * P + j] = fmaf(R0[c], xb[0], fmaf(R0[3 + c], xb[1], R0[6 + c] * xb[2]));
      Yb[(3 + c) * P + j] = fmaf(R0[c], nb[0], fmaf(R0[3 + c], nb[1], R0[6 + c] * nb[2]));
    }
  }
  float v[12], tot;
#pragma unroll
  for (int e = 0; e < 12; ++e) v[e] = e < 9 ? fmaf(xb[e / 3], y[e % 3], nb[e / 3] * z[e % 3]) : xb[e - 9];
  block_sum12(v, red, tot);
  if (threadIdx.x < 12) Gpart[(int64_t)blockIdx.x * 12 + threadIdx.x] = tot;
}

// Block k: sphere k's gradient (abar_k, tbar_k) into gp[6 k ..] and its
// terms of the global gradient into Gpart[row0 + k][12].
__global__ __launch_bounds__(SHV_BLOCK) void k_deform_bwd_sphere(DeformGraphDev g, const float* __restrict__ params,
                                                                 const float* __restrict__ Rm,
                                                                 const float* __restrict__ gs,
                                                                 const float* __restrict__ Yb, int64_t row0,
                                                                 float* __restrict__ Gpart, float* __restrict__ gp) {
  __shared__ float red[SHV_WAVES_PER_BLOCK][12];
  __shared__ float tot_s[12];
  const int64_t k = blockIdx.x;
  const int64_t P = g.P, S = g.S;
  const int K = g.K;
  const float* gk = g.spheres + 4 * k;
  float acc[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) acc[e] = 0.0f;
  for (int q = threadIdx.x; q < K; q += SHV_BLOCK) {
    const int64_t j = g.sph_vert[k * K + q];
    const float w = g.sph_w[k * K + q];
    const float yb[3] = {w * Yb[j], w * Yb[P + j], w * Yb[2 * P + j]};
    const float zb[3] = {w * Yb[3 * P + j], w * Yb[4 * P + j], w * Yb[5 * P + j]};
    const float d[3] = {g.vertices[j] - gk[0], g.vertices[P + j] - gk[1], g.vertices[2 * P + j] - gk[2]};
    const float m[3] = {g.normals[j], g.normals[P + j], g.normals[2 * P + j]};
#pragma unroll
    for (int e = 0; e < 9; ++e) acc[e] = fmaf(yb[e / 3], d[e % 3], fmaf(zb[e / 3], m[e % 3], acc[e]));
#pragma unroll
    for (int r = 0; r < 3; ++r) acc[9 + r] += yb[r];
  }
  float te;
  block_sum12(acc, red, te);
  if (threadIdx.x < 12) tot_s[threadIdx.x] = te;
  __syncthreads();
  if (threadIdx.x != 0) return;
  float tot[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) tot[e] = tot_s[e];
  const float* R0 = Rm + 9 * S;
  const float* tk = params + 6 * k + 3;
  const float cb[3] = {gs ? gs[4 * k] : 0.0f, gs ? gs[4 * k + 1] : 0.0f, gs ? gs[4 * k + 2] : 0.0f};
  float Rb[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) Rb[e] = tot[e];
  rodrigues3_adjoint(params + 6 * k, Rb, gp + 6 * k);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    gp[6 * k + 3 + c] = tot[9 + c] + fmaf(R0[c], cb[0], fmaf(R0[3 + c], cb[1], R0[6 + c] * cb[2]));
  const float q[3] = {gk[0] + tk[0], gk[1] + tk[1], gk[2] + tk[2]};
  float* out = Gpart + (row0 + k) * 12;
#pragma unroll
  for (int e = 0; e < 9; ++e) out[e] = cb[e / 3] * q[e % 3];
#pragma unroll
  for (int r = 0; r < 3; ++r) out[9 + r] = cb[r];
}

// The global row of the gradient from the reduced Rbar_0 | tbar_0 (G[12]).
__global__ void k_deform_global(const float* __restrict__ params, int64_t S, const float* __restrict__ G,
                                float* __restrict__ gp) {
  if (threadIdx.x != 0) return;
  float Rb[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) Rb[e] = G[e];
  rodrigues3_adjoint(params + 6 * S, Rb, gp + 6 * S);
#pragma unroll
  for (int r = 0; r < 3; ++r) gp[6 * S + 3 + r] = G[9 + r];
}

// loss partials: per block sum of (v - t)^2 / n; grad = 2 (v - t) / n.
__global__ __launch_bounds__(SHV_BLOCK) void k_l2(const float* __restrict__ v, const float* __restrict__ t, int64_t n,
                                                  float* __restrict__ grad, float* __restrict__ part) {
  __shared__ float red[SHV_WAVES_PER_BLOCK];
  const int64_t i = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const float inv = 1.0f / (float)n;
  float r = 0.0f;
  if (i < n) {
    r = v[i] - t[i];
    if (grad) grad[i] = 2.0f * r * inv;
  }
  const float s = block_sum(r * r * inv, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(SHV_BLOCK) void k_sgd(float* __restrict__ x, const float* __restrict__ g, int64_t n,
                                                   float lr) {
  const int64_t i = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (i < n) x[i] = fmaf(-lr, g[i], x[i]);
}

// ---------------------------------------------------------------------------
// Launchers.

int64_t deform_vert_blocks(int64_t P) { return (P + SHV_BLOCK - 1) / SHV_BLOCK; }

hipError_t launch_deform_forward(const DeformGraphDev& g, const float* params, float* Rm, float* pts, float* nrm,
                                 float* sph, hipStream_t st) {
  const int64_t rows = g.S + 1;
  k_deform_rot<<<(unsigned)((rows + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(params, rows, Rm);
  const int64_t n = g.P + g.S;
  k_deform_fwd<<<(unsigned)((n + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(g, params, Rm, pts, nrm, sph);
  return hipGetLastError();
}

hipError_t launch_deform_backward(const DeformGraphDev& g, const float* params, const float* gx, const float* gn,
                                  const float* gs, float* Rm, float* Yb, float* Gpart, float* G, float* gp,
                                  hipStream_t st) {
  const int64_t rows = g.S + 1;
  k_deform_rot<<<(unsigned)((rows + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(params, rows, Rm);
  const int64_t vb = deform_vert_blocks(g.P);
  if (vb > 0) k_deform_bwd_vert<<<(unsigned)vb, SHV_BLOCK, 0, st>>>(g, params, Rm, gx, gn, Yb, Gpart);
  k_deform_bwd_sphere<<<(unsigned)g.S, SHV_BLOCK, 0, st>>>(g, params, Rm, gs, Yb, vb, Gpart, gp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_reduce_rows(Gpart, (int)(vb + g.S), 12, G, st);
  if (e != hipSuccess) return e;
  k_deform_global<<<1, 64, 0, st>>>(params, g.S, G, gp);
  return hipGetLastError();
}

hipError_t launch_l2(const float* v, const float* t, int64_t n, float* grad, float* part, float* loss,
                     hipStream_t st) {
  const int64_t nb = (n + SHV_BLOCK - 1) / SHV_BLOCK;
  k_l2<<<(unsigned)nb, SHV_BLOCK, 0, st>>>(v, t, n, grad, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_rows(part, (int)nb, 1, loss, st);
}

hipError_t launch_sgd(float* x, const float* g, int64_t n, float lr, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_sgd<<<(unsigned)((n + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(x, g, n, lr);
  return hipGetLastError();
}

}  // namespace shv
