// Device building blocks for the SH soft-shadow kernels (gfx950, wave64).
//
// Real SH in a polynomial form: for a unit vector (x, y, z),
//   y_lm = LAMBDA[l][|m|] * r_l^|m|(z) * T_m(x, y),
//   T_m = Re (x + i y)^m for m >= 0, Im (x + i y)^|m| for m < 0,
//   r_m^m = 1, r_{m+1}^m = z, r_l^m = z r_{l-1}^m + GAMMA[l][m] r_{l-2}^m,
//   d r_l^m / dz = RHO[l][m] r_l^{m+1}.
// r_l^m is d^m P_l / dz^m up to a constant, so no square roots or
// trigonometric functions are needed and every derivative stays polynomial.
//
// Coefficient index i = l*l + l + m (Sec. 3.2 of the paper).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "generated/shv_constants.h"
#include "generated/shv_gaunt.h"

#include "shv_config.h"

namespace shv {

__device__ __forceinline__ constexpr int idx(int l, int m) { return l * l + l + m; }

__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Re / Im of (x + i y)^m, m < NB.
template <int NB>
__device__ __forceinline__ void cs_powers(float x, float y, float (&C)[NB], float (&S)[NB]) {
  C[0] = 1.0f;
  S[0] = 0.0f;
  if constexpr (NB > 1) {
    C[1] = x;
    S[1] = y;
  }
#pragma unroll
  for (int m = 1; m + 1 < NB; ++m) {
    C[m + 1] = fmaf(x, C[m], -y * S[m]);
    S[m + 1] = fmaf(x, S[m], y * C[m]);
  }
}

// Residual Legendre values R_l = 1 - P_l(t), l = 0 .. NB, from u = 1 - t.
// Bonnet's recurrence rewritten for R: R_0 = 0, R_1 = u,
//   R_{l+1} = (2l+1)/(l+1) (u + t R_l) - l/(l+1) R_{l-1}.
// For small caps (t near 1) every g_l is a difference of Legendre values
// that all tend to 1; recurring on R keeps the leading digits.
template <int NB>
__device__ __forceinline__ void legendre_resid(float t, float u, float (&R)[NB + 1]) {
  R[0] = 0.0f;
  R[1] = u;
#pragma unroll
  for (int l = 1; l < NB; ++l) R[l + 1] = fmaf(SHV_BONNET_A[l], fmaf(t, R[l], u), -SHV_BONNET_B[l] * R[l - 1]);
}

// eps-free log-cap zonal coefficients g_l(t) = -2 pi/(2l+1) (P_{l-1} - P_{l+1})
// with P_{-1} = 1, i.e. g_0 = -2 pi u and g_l = -2 pi/(2l+1) (R_{l+1} - R_{l-1}):
// the projection of "-1 on the cap {w . s >= t}" rotated to s, divided by
// y_lm(s).  d g_l / dt = 2 pi P_l(t) = 2 pi (1 - R_l).
template <int NB>
__device__ __forceinline__ void cap_zonal(float u, const float (&R)[NB + 1], float (&g)[NB]) {
  g[0] = SHV_CAPK[0] * u;
#pragma unroll
  for (int l = 1; l < NB; ++l) g[l] = SHV_CAPK[l] * (R[l + 1] - R[l - 1]);
}

// y_i(x, y, z) for all i < NB^2 (unit vector).
template <int NB>
__device__ __forceinline__ void sh_eval(float x, float y, float z, float (&Y)[NB * NB]) {
  float C[NB], S[NB];
  cs_powers<NB>(x, y, C, S);
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    float r2 = 0.0f, r1 = 1.0f;
#pragma unroll
    for (int l = m; l < NB; ++l) {
      float r;
      if (l == m) r = 1.0f;
      else if (l == m + 1) r = z;
      else r = fmaf(z, r1, SHV_GAMMA[l][m] * r2);
      if (l > m) { r2 = r1; r1 = r; }
      const float q = SHV_LAMBDA[l][m] * r;
      if (m == 0) {
        Y[idx(l, 0)] = q;
      } else {
        Y[idx(l, m)] = q * C[m];
        Y[idx(l, -m)] = q * S[m];
      }
    }
  }
}

// Gradient of the polynomial extension of sum_i c_i y_i at (x, y, z).
// The tangential part of the result is the surface gradient on the sphere.
template <int NB>
__device__ __forceinline__ void sh_grad(float x, float y, float z, const float (&c)[NB * NB], float& gx,
                                        float& gy, float& gz) {
  float C[NB], S[NB];
  cs_powers<NB>(x, y, C, S);
  gx = 0.0f;
  gy = 0.0f;
  gz = 0.0f;
  // Pass m evaluates r_l^m; it closes the x/y sums of order m and the z sums
  // of order m - 1 (because d r_l^{m-1}/dz = RHO[l][m-1] r_l^m).
#pragma unroll
  for (int m = 1; m < NB; ++m) {
    float Xc = 0.0f, Xs = 0.0f, Zc = 0.0f, Zs = 0.0f;
    float r2 = 0.0f, r1 = 1.0f;
#pragma unroll
    for (int l = m; l < NB; ++l) {
      float r;
      if (l == m) r = 1.0f;
      else if (l == m + 1) r = z;
      else r = fmaf(z, r1, SHV_GAMMA[l][m] * r2);
      if (l > m) { r2 = r1; r1 = r; }
      Xc = fmaf(c[idx(l, m)] * SHV_LAMBDA[l][m], r, Xc);
      Xs = fmaf(c[idx(l, -m)] * SHV_LAMBDA[l][m], r, Xs);
      const float kz = SHV_LAMBDA[l][m - 1] * SHV_RHO[l][m - 1];
      Zc = fmaf(c[idx(l, m - 1)] * kz, r, Zc);
      if (m - 1 >= 1) Zs = fmaf(c[idx(l, -(m - 1))] * kz, r, Zs);
    }
    gz = fmaf(Zc, C[m - 1], fmaf(Zs, S[m - 1], gz));
    const float fm = (float)m;
    gx = fmaf(fm, fmaf(Xc, C[m - 1], Xs * S[m - 1]), gx);
    gy = fmaf(fm, fmaf(Xs, C[m - 1], -Xc * S[m - 1]), gy);
  }
}

// v on an in-range lane, `other` on a tail lane.  The load that produces v
// reads a clamped, always valid address (receiver 0 instead of a receiver
// past the end), so the compiler places no branch around it and a group of
// such loads is in flight together.
__device__ __forceinline__ float sel0(bool ok, float v, float other = 0.0f) { return ok ? v : other; }

// Sum over the 64 lanes of a wave; every lane receives the total.  Fixed
// butterfly order, so the result is deterministic.
// v + (v moved by the DPP control CTRL) in the rows of ROWS (a lane whose
// source lies outside its row adds 0; lanes of other rows add 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_add(float v) {
  const int m = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, true);
  return v + __int_as_float(m);
}

// Sum of v over the wave's 64 lanes, complete in lane 63 (the other lanes
// hold partial sums), with DPP moves only, no LDS: row_shr 1, 2, 4, 8 leave
// each 16-lane row's sum in its lane 15; row_bcast 15 adds row 0's sum to
// row 1 and row 2's to row 3, and row_bcast 31 adds lane 31 (rows 0 + 1) to
// row 3.  A fixed order of additions, so the result is deterministic.
__device__ __forceinline__ float wave_sum_last(float v) {
  v = dpp_add<0x111, 0xF>(v);  // row_shr:1
  v = dpp_add<0x112, 0xF>(v);  // row_shr:2
  v = dpp_add<0x114, 0xF>(v);  // row_shr:4
  v = dpp_add<0x118, 0xF>(v);  // row_shr:8
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

// The value of v in the lane that DPP control CTRL selects (0 where that lane
// lies outside the row).
template <int CTRL>
__device__ __forceinline__ float dpp_from(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// v[l] + v[l ^ 16] and v[l] + v[l ^ 32] in every lane l, by gfx950's
// permlane swaps of v with itself (the two results hold v[l] and its partner
// in some order; the sum is the same bits either way).
__device__ __forceinline__ float xor16_add(float v) {
  const int i = __float_as_int(v);
  const auto r = __builtin_amdgcn_permlane16_swap(i, i, false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ float xor32_add(float v) {
  const int i = __float_as_int(v);
  const auto r = __builtin_amdgcn_permlane32_swap(i, i, false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// Totals over the wave of four per-lane values, transposed: lane l returns
// the total of value (l & 3) (a, b, c, d in that order), complete in lanes
// 12..15 of every row (so in lanes 60..63).  Lanes l and l ^ 1 first split the
// four values between them (even lanes keep a and c), lanes l and l ^ 2 then
// split the two sums, so each lane carries one value from there on: quads of a
// row by row_shr 4 and 8, rows by the xor-16 and xor-32 swaps.  A fixed order
// of additions, about 17 instructions for the four sums.
__device__ __forceinline__ float wave_sum4(float a, float b, float c, float d) {
  const int lane = threadIdx.x & 63;
  const bool odd = (lane & 1) != 0, hi = (lane & 2) != 0;
  const float u = (odd ? b : a) + dpp_from<0xB1>(odd ? a : b);  // quad_perm [1,0,3,2]: lane l ^ 1
  const float v = (odd ? d : c) + dpp_from<0xB1>(odd ? c : d);
  float w = (hi ? v : u) + dpp_from<0x4E>(hi ? u : v);           // quad_perm [2,3,0,1]: lane l ^ 2
  w += dpp_from<0x114>(w);                                        // row_shr:4
  w += dpp_from<0x118>(w);                                        // row_shr:8
  w = xor16_add(w);
  return xor32_add(w);
}

__device__ __forceinline__ float wave_sum(float v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

}  // namespace shv

// Template dispatch on the number of bands (1 .. 8) for kernel launches.
#define SHV_DISPATCH(nb, KERNEL, ...)            \
  switch (nb) {                                  \
    case 1: KERNEL<1><<<__VA_ARGS__; break;      \
    case 2: KERNEL<2><<<__VA_ARGS__; break;      \
    case 3: KERNEL<3><<<__VA_ARGS__; break;      \
    case 4: KERNEL<4><<<__VA_ARGS__; break;      \
    case 5: KERNEL<5><<<__VA_ARGS__; break;      \
    case 6: KERNEL<6><<<__VA_ARGS__; break;      \
    case 7: KERNEL<7><<<__VA_ARGS__; break;      \
    case 8: KERNEL<8><<<__VA_ARGS__; break;      \
    default: return hipErrorInvalidValue;        \
  }

// Same, for kernels with a second (bool) template parameter.
#define SHV_DISPATCH2(nb, KERNEL, B, ...)           \
  switch (nb) {                                     \
    case 1: KERNEL<1, B><<<__VA_ARGS__; break;      \
    case 2: KERNEL<2, B><<<__VA_ARGS__; break;      \
    case 3: KERNEL<3, B><<<__VA_ARGS__; break;      \
    case 4: KERNEL<4, B><<<__VA_ARGS__; break;      \
    case 5: KERNEL<5, B><<<__VA_ARGS__; break;      \
    case 6: KERNEL<6, B><<<__VA_ARGS__; break;      \
    case 7: KERNEL<7, B><<<__VA_ARGS__; break;      \
    case 8: KERNEL<8, B><<<__VA_ARGS__; break;      \
    default: return hipErrorInvalidValue;           \
  }
