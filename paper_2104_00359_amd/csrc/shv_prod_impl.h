// Visibility as the direct product chain of Eq. 12, and its adjoint.
//
// V = V'_1 * V'_2 * ... * V'_S: truncated SH products (Eqs. 6-7) of the
// projected floored blockers V'_i (Eq. 13), taken left to right in sphere
// order (truncated products are not associative, so the order is part of the
// result).  With h_i = LAMBDA (.) F'_i, the pair's log-cap vector without the
// factor eps (F'_i exactly as the pair kernels form it), V'_i has the
// coefficients sqrt(4 pi) e_0 + beta h_i with beta = 1 - e^-eps.  A product
// with the constant 1 is exact under truncation, so each step is
//   V <- V + beta (V * h_i),        starting from V = sqrt(4 pi) e_0.
// The adjoint of one step, with Vb the cotangent of its output:
//   hbar_i = beta (Vb * V_in),      Vb_in = Vb + beta (Vb * h_i)
// (the triple-product tensor is symmetric in its three indices).  hbar_i
// becomes the pair weights W_lm = LAMBDA_lm hbar_lm of the pair adjoint.
//
// The generated adjoint of the squaring computes 2 (a * b) for any a and b,
// output group by output group; one step costs one such product forward and
// two in the adjoint.  The chain is sequential in the spheres, so the
// parallelism is over receivers only.
//
// Layout: four waves per 64 receivers, wave G owning output group G of each
// product; the full vectors are exchanged through LDS once per sphere, in
// double buffers, one barrier per sphere.  Every wave forms the blocker
// vector h_i itself (a few hundred flops against a quarter of a product).
// The forward can record each step's input V_in, [S][N][P]; the adjoint reads
// them back in reverse, one sphere ahead.  The pair adjoint is linear in its
// weights, so each wave runs it on its own output group's share of hbar and
// writes its own sphere-gradient partial (rows (block, wave), reduced in
// order afterwards); only the two vectors cross LDS, which keeps a block's
// LDS small enough for two blocks per CU.

#pragma once

#include <cmath>

#include "shv_exp_impl.h"
#include "shv_pair_impl.h"

namespace shv {

// h = LAMBDA (.) F' of one pair: the same recurrence and products as the pair
// forward kernel, each coefficient scaled by its LAMBDA[l][|m|].
template <int NB>
__device__ __forceinline__ void blocker_vec(const PairGeom& G, float (&h)[NB * NB]) {
  float R[NB + 1], g[NB], C[NB], Sn[NB];
  legendre_resid<NB>(G.t, G.u, R);
  cap_zonal<NB>(G.u, R, g);
  cs_powers<NB>(G.x, G.y, C, Sn);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    float r2 = 0.0f, r1 = 1.0f;
#pragma unroll
    for (int l = m; l < NB; ++l) {
      float u;
      if (l == m) {
        u = g[l];
      } else {
        const float r = (l == m + 1) ? G.z : fmaf(G.z, r1, SHV_GAMMA[l][m] * r2);
        r2 = r1;
        r1 = r;
        u = g[l] * r;
      }
      if (m == 0) {
        h[idx(l, 0)] = SHV_LAMBDA[l][0] * u;
      } else {
        h[idx(l, m)] = SHV_LAMBDA[l][m] * (u * C[m]);
        h[idx(l, -m)] = SHV_LAMBDA[l][m] * (u * Sn[m]);
      }
    }
  }
}

template <int NB>
struct ProdFwdShared {
  float X[2][NB * NB][64];
};

template <int NB, int G>
__device__ __forceinline__ void prod_fwd_group(float (*X)[NB * NB][64], int lane, int64_t p, bool ok,
                                               const float* __restrict__ pts, int64_t P,
                                               const float4* __restrict__ sph, int S, float hbeta,
                                               float* __restrict__ vis, float* __restrict__ states) {
  constexpr int N = NB * NB;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const float px = sel0(ok, pts[q]);
  const float py = sel0(ok, pts[P + q]);
  const float pz = sel0(ok, pts[2 * P + q]);
  float V[N];
#pragma unroll
  for (int i = 0; i < N; ++i) V[i] = i == 0 ? SHV_SQRT_4PI : 0.0f;
  for (int s = 0; s < S; ++s) {
    if (states && ok) {
      float* dst = states + (int64_t)s * N * P + p;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) dst[(int64_t)i * P] = V[i];
    }
    float h[N], T[N];
    blocker_vec<NB>(pair_geom(px, py, pz, sph[s]), h);
    SqGroup<NB, G>::adj(V, h, T);  // group G of 2 (V * h)
    const int b = s & 1;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) X[b][i][lane] = fmaf(hbeta, T[i], V[i]);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) V[i] = X[b][i][lane];
  }
  if (vis && ok) {
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) vis[(int64_t)i * P + p] = V[i];
  }
}

// hbeta = beta / 2 (the generated product returns twice the product).
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_prod_fwd(const float* __restrict__ pts, int64_t P,
                                                        const float4* __restrict__ sph, int S, float hbeta,
                                                        float* __restrict__ vis, float* __restrict__ states) {
  __shared__ ProdFwdShared<NB> sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = p < P;
  switch (wave) {
    case 0: prod_fwd_group<NB, 0>(sh.X, lane, p, ok, pts, P, sph, S, hbeta, vis, states); break;
    case 1: prod_fwd_group<NB, 1>(sh.X, lane, p, ok, pts, P, sph, S, hbeta, vis, states); break;
    case 2: prod_fwd_group<NB, 2>(sh.X, lane, p, ok, pts, P, sph, S, hbeta, vis, states); break;
    default: prod_fwd_group<NB, 3>(sh.X, lane, p, ok, pts, P, sph, S, hbeta, vis, states); break;
  }
}

template <int NB>
struct ProdBwdShared {
  float Vb[2][NB * NB][64];  // cotangent of the chain state
  float Vi[2][NB * NB][64];  // the current step's input V_in
  float gp[3][3][64];        // receiver-gradient partials of waves 1..3
};

template <int NB, int G>
__device__ __forceinline__ void prod_bwd_group(ProdBwdShared<NB>& sh, int lane, int64_t bx, int64_t p, bool ok,
                                               const float* __restrict__ gvis, const float* __restrict__ states,
                                               const float* __restrict__ pts, int64_t P,
                                               const float4* __restrict__ sph, int S, float hbeta,
                                               float* __restrict__ gpts, float4* __restrict__ gs_part) {
  constexpr int N = NB * NB;
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const float px = sel0(ok, pts[q]);
  const float py = sel0(ok, pts[P + q]);
  const float pz = sel0(ok, pts[2 * P + q]);
  float gpx = 0.0f, gpy = 0.0f, gpz = 0.0f;
  float4* gs_row = gs_part + (bx * 4 + G) * S;
  // Cotangent of the chain's output (zero on tail lanes, so they add nothing
  // to the sphere sums), the input of the last step, and the next one ahead.
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (group_of<NB>(i) == G) sh.Vb[S & 1][i][lane] = sel0(ok, gvis[(int64_t)i * P + q]);
  float pre[N];
  if (S > 0) {
    const float* src = states + (int64_t)(S - 1) * N * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) sh.Vi[(S - 1) & 1][i][lane] = src[(int64_t)i * P];
  }
  if (S > 1) {
    const float* src = states + (int64_t)(S - 2) * N * P + q;
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) pre[i] = src[(int64_t)i * P];
  }
  __syncthreads();
  for (int s = S - 1; s >= 0; --s) {
    const int b = s & 1;
    float Vb[N], A[N], T[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Vb[i] = sh.Vb[b ^ 1][i][lane];
      A[i] = sh.Vi[b][i][lane];
    }
    SqGroup<NB, G>::adj(Vb, A, T);  // group G of 2 (Vb * V_in)
    const PairGeom geo = pair_geom(px, py, pz, sph[s]);
    {
      // This wave's share of the pair weights: W_lm = LAMBDA_lm hbar_lm on
      // its output group, 0 elsewhere (the pair adjoint is linear in W).
      float W[N], Wz[N];
#pragma unroll
      for (int l = 0; l < NB; ++l) {
#pragma unroll
        for (int m = -l; m <= l; ++m) {
          const int i = idx(l, m);
          const float w = group_of<NB>(i) == G ? SHV_LAMBDA[l][m < 0 ? -m : m] * (hbeta * T[i]) : 0.0f;
          W[i] = w;
          Wz[i] = w * SHV_RHO[l][m < 0 ? -m : m];
        }
      }
      float gvx, gvy, gvz, gr;
      pair_adjoint<NB>(geo, W, Wz, gvx, gvy, gvz, gr);
      gpx -= gvx;
      gpy -= gvy;
      gpz -= gvz;
      const float4 tot = make_float4(wave_sum_last(gvx), wave_sum_last(gvy), wave_sum_last(gvz), wave_sum_last(gr));
      if (lane == 63) gs_row[s] = tot;
    }
    blocker_vec<NB>(geo, A);
    SqGroup<NB, G>::adj(Vb, A, T);  // group G of 2 (Vb * h)
#pragma unroll
    for (int i = 0; i < N; ++i)
      if (group_of<NB>(i) == G) sh.Vb[b][i][lane] = fmaf(hbeta, T[i], Vb[i]);
    if (s > 0) {
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) sh.Vi[b ^ 1][i][lane] = pre[i];
    }
    if (s > 1) {
      const float* src = states + (int64_t)(s - 2) * N * P + q;
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (group_of<NB>(i) == G) pre[i] = src[(int64_t)i * P];
    }
    __syncthreads();
  }
  if (G > 0) {
    sh.gp[G - 1][0][lane] = gpx;
    sh.gp[G - 1][1][lane] = gpy;
    sh.gp[G - 1][2][lane] = gpz;
  }
  __syncthreads();
  if (G == 0 && ok && gpts) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      gpx += sh.gp[w][0][lane];
      gpy += sh.gp[w][1][lane];
      gpz += sh.gp[w][2][lane];
    }
    gpts[p] = gpx;
    gpts[P + p] = gpy;
    gpts[2 * P + p] = gpz;
  }
}

// gs_part: [4 * pair_blocks(P)][S], one row per (block, wave).
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK, 2) void k_prod_bwd(const float* __restrict__ gvis,
                                                           const float* __restrict__ states,
                                                           const float* __restrict__ pts, int64_t P,
                                                           const float4* __restrict__ sph, int S, float hbeta,
                                                           float* __restrict__ gpts, float4* __restrict__ gs_part) {
  __shared__ ProdBwdShared<NB> sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t bx = blockIdx.x;
  const int64_t p = bx * 64 + lane;
  const bool ok = p < P;
  switch (wave) {
    case 0: prod_bwd_group<NB, 0>(sh, lane, bx, p, ok, gvis, states, pts, P, sph, S, hbeta, gpts, gs_part); break;
    case 1: prod_bwd_group<NB, 1>(sh, lane, bx, p, ok, gvis, states, pts, P, sph, S, hbeta, gpts, gs_part); break;
    case 2: prod_bwd_group<NB, 2>(sh, lane, bx, p, ok, gvis, states, pts, P, sph, S, hbeta, gpts, gs_part); break;
    default: prod_bwd_group<NB, 3>(sh, lane, bx, p, ok, gvis, states, pts, P, sph, S, hbeta, gpts, gs_part); break;
  }
}

// ---------------------------------------------------------------------------
// Launchers for one band count (instantiated per band count in shv_nb.hip).
// beta = 1 - e^-eps is formed in double precision and rounded once.

inline float prod_half_beta(float eps) { return (float)(-0.5 * std::expm1(-(double)eps)); }

template <int NB>
hipError_t prod_fwd_nb(const float* pts, int64_t P, const float* sph, int S, float eps, float* vis, float* states,
                       hipStream_t st) {
  k_prod_fwd<NB><<<(unsigned)pair_blocks(P), SHV_BLOCK, 0, st>>>(pts, P, (const float4*)sph, S,
                                                                 prod_half_beta(eps), vis, states);
  return hipGetLastError();
}

template <int NB>
hipError_t prod_bwd_nb(const float* gvis, const float* states, const float* pts, int64_t P, const float* sph, int S,
                       float eps, float* gpts, float* gs_part, hipStream_t st) {
  k_prod_bwd<NB><<<(unsigned)pair_blocks(P), SHV_BLOCK, 0, st>>>(gvis, states, pts, P, (const float4*)sph, S,
                                                                 prod_half_beta(eps), gpts, (float4*)gs_part);
  return hipGetLastError();
}

}  // namespace shv
