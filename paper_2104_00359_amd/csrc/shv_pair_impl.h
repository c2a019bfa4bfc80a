// Pair kernels: the O(P * S) part of the method (Sec. 3.3.2).
//
// Forward, per (receiver x, sphere i): direction s = (c - x)/|c - x|, cap
// half-angle alpha = asin(r/|c - x|), t = cos(alpha); the log-blocker
// -eps * 1[w . s >= t] (Eq. 13) has zonal coefficients g_l(t) about s, and
// rotating them to s multiplies by y_lm(s).  The kernel accumulates
//   F'_lm(x) = sum_i g_l(t_i) r_l^|m|(s_z) T_m(s_x, s_y)
// in registers; the constant factor eps * LAMBDA[l][|m|] that turns F' into
// the log-visibility F is applied once per receiver by the exponential
// kernel.
//
// Backward: per pair the terms are recomputed (nothing per pair is stored).
// With W_lm = dLoss/dF'_lm:
//   dLoss/dt  = 2 pi sum_lm W_lm P_l(t) r_l^|m| T_m         (g_l' = 2 pi P_l)
//   dLoss/ds  = grad of sum_lm W_lm g_l r_l^|m| T_m, projected on the tangent
//   plane, then chained through s = v/|v|, t = sqrt(1 - r^2/|v|^2), v = c - x.
// Receiver gradients stay in registers; a sphere's four gradient values are
// summed over the wave together (a transposed reduction: DPP moves and
// gfx950's permlane swaps, no LDS), written per sphere to LDS by the wave
// that owns the sphere, and stored as per-block partials reduced by a second
// deterministic pass.
//
// Layout: one receiver per lane.  A block holds 64 receivers and 4 waves;
// grid.y splits the sphere set into chunks and the block's chunk is split
// again over its 4 waves (sphere w, w + 4, ...), so small receiver sets still
// fill 256 CUs.  The waves' partial sums are combined through LDS in wave
// order.  The block's chunk of sphere records is staged in LDS once and read
// back as wave-uniform broadcasts (measured faster than scalar loads of each
// record: pair adjoint 748 -> 703 us at 8 bands on the 64-scene batch).

#pragma once

#include "shv_batch.h"
#include "shv_launch.h"
#include "shv_shade_common.h"

namespace shv {

struct PairGeom {
  float x, y, z;  // unit direction receiver -> centre
  float inv;      // 1 / |c - x| (0 for a sphere centred on the receiver)
  float rs;       // r / |c - x|
  float t;        // cos(alpha), 0 when the receiver is inside the sphere
  float u;        // 1 - t, formed as s^2 / (1 + t) so small caps keep their digits
};

__device__ __forceinline__ PairGeom pair_geom(float px, float py, float pz, float4 q) {
  PairGeom g;
  const float vx = q.x - px, vy = q.y - py, vz = q.z - pz;
  const float d2 = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
  g.inv = d2 > 0.0f ? fast_rsqrt(d2) : 0.0f;
  g.x = vx * g.inv;
  g.y = vy * g.inv;
  g.z = vz * g.inv;
  g.rs = q.w * g.inv;
  g.t = fast_sqrt(fmaxf(fmaf(-g.rs, g.rs, 1.0f), 0.0f));
  g.u = fminf(g.rs * g.rs * fast_rcp(1.0f + g.t), 1.0f);  // = 1 when inside (t = 0)
  return g;
}

// The sphere chunk is needed during the sphere loop, X only after it: they
// share the storage (a barrier separates them), so staging the spheres costs
// the forward no LDS at 4 or more bands.  The waves' partial sums are
// exchanged half of the coefficients at a time, which halves X and lets more
// blocks share a CU.
template <int NB>
struct PairFwdHalf {
  static constexpr int N = NB * NB;
  static constexpr int H = (N + 1) / 2;  // coefficients per exchange
};
template <int NB>
union PairFwdShared {
  float X[SHV_WAVES_PER_BLOCK - 1][PairFwdHalf<NB>::H][64];
  float4 sph[SHV_MAX_CHUNK];
};

// One block of the pair forward: receivers [64 bx, 64 bx + 64), sphere chunk
// by.  Blocks of chunk 0 also build M(L), block m_idx of m_count taking every
// m_count-th entry.
template <int NB>
__device__ __forceinline__ void pair_fwd_item(const float* __restrict__ pts, int64_t P, const float4* __restrict__ sph,
                                              int S, int chunk, float* __restrict__ Fpart,
                                              const float* __restrict__ L, float* __restrict__ M, int64_t bx, int by,
                                              int64_t m_idx, int64_t m_count, PairFwdShared<NB>& sh) {
  constexpr int N = NB * NB;
  auto& X = sh.X;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = bx * 64 + lane;
  const bool ok = p < P;
  const int s0 = by * chunk;
  const int s1 = min(S, s0 + chunk);
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const float px = sel0(ok, pts[q]);
  const float py = sel0(ok, pts[P + q]);
  const float pz = sel0(ok, pts[2 * P + q]);

  float acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0.0f;
  // The DC coefficient sets V's overall scale through exp(F_0 / sqrt(4 pi)),
  // so its sum over spheres is compensated (Kahan).
  float dc_comp = 0.0f;

  for (int j = threadIdx.x; j < s1 - s0; j += SHV_BLOCK) sh.sph[j] = sph[s0 + j];
  __syncthreads();
  for (int s = s0 + wave; s < s1; s += SHV_WAVES_PER_BLOCK) {
    const PairGeom G = pair_geom(px, py, pz, sh.sph[s - s0]);
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
        if (m == 0 && l == 0) {
          const float y = u - dc_comp;
          const float t = acc[0] + y;
          dc_comp = (t - acc[0]) - y;
          acc[0] = t;
        } else if (m == 0) {
          acc[idx(l, 0)] += u;
        } else {
          acc[idx(l, m)] = fmaf(u, C[m], acc[idx(l, m)]);
          acc[idx(l, -m)] = fmaf(u, Sn[m], acc[idx(l, -m)]);
        }
      }
    }
  }
  // Coefficient i of the block is ((acc_0 + acc_1) + acc_2) + acc_3 over the
  // waves, formed by wave 0 in two exchanges of half the coefficients.
  constexpr int H = PairFwdHalf<NB>::H;
  float* out = Fpart + (int64_t)by * N * P + p;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    __syncthreads();  // the spheres (h = 0) or the previous half (h = 1) are no longer read
    if (wave > 0) {
#pragma unroll
      for (int i = h * H; i < N && i < (h + 1) * H; ++i) X[wave - 1][i - h * H][lane] = acc[i];
    }
    __syncthreads();
    if (wave == 0 && ok) {
#pragma unroll
      for (int i = h * H; i < N && i < (h + 1) * H; ++i) {
        float v = acc[i];
#pragma unroll
        for (int w = 0; w < SHV_WAVES_PER_BLOCK - 1; ++w) v += X[w][i - h * H][lane];
        out[(int64_t)i * P] = v;
      }
    }
  }
  // Side job for the fused render path, spread over the first chunk's blocks:
  // the lit transfer matrix M(L), needed by the shading that follows in
  // stream order.
  if (M && by == 0) build_M_range<NB>(L, M, (int)(m_idx * SHV_BLOCK) + threadIdx.x, (int)(m_count * SHV_BLOCK));
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_pair_fwd(const float* __restrict__ pts, int64_t P,
                                                        const float4* __restrict__ sph, int S, int chunk,
                                                        float* __restrict__ Fpart, const float* __restrict__ L,
                                                        float* __restrict__ M) {
  __shared__ PairFwdShared<NB> sh;
  pair_fwd_item<NB>(pts, P, sph, S, chunk, Fpart, L, M, blockIdx.x, blockIdx.y, blockIdx.x, gridDim.x, sh);
}

struct PairBwdShared {
  float4 sph[SHV_MAX_CHUNK];
  float4 red[SHV_MAX_CHUNK];
  float gpx_w[SHV_WAVES_PER_BLOCK - 1][3][64];
};

// Adjoint of one pair's term for the weights W_lm = dLoss/dF'_lm (and
// Wz_lm = RHO[l][|m|] W_lm): the cotangent of v = c - x (gvx, gvy, gvz) and
// of the radius (gr).
template <int NB>
__device__ __forceinline__ void pair_adjoint(const PairGeom& G, const float (&W)[NB * NB], const float (&Wz)[NB * NB],
                                             float& gvx, float& gvy, float& gvz, float& gr) {
  float R[NB + 1], g[NB], C[NB], Sn[NB];
  legendre_resid<NB>(G.t, G.u, R);
  cap_zonal<NB>(G.u, R, g);
  cs_powers<NB>(G.x, G.y, C, Sn);
  float Gx = 0.0f, Gy = 0.0f, Gz = 0.0f, Gt = 0.0f;
#pragma unroll
  for (int m = 0; m < NB; ++m) {
    float Xc = 0.0f, Xs = 0.0f, Tc = 0.0f, Ts = 0.0f, Zc = 0.0f, Zs = 0.0f;
    float r2 = 0.0f, r1 = 1.0f;
#pragma unroll
    for (int l = m; l < NB; ++l) {
      float r;
      if (l == m) r = 1.0f;
      else if (l == m + 1) r = G.z;
      else r = fmaf(G.z, r1, SHV_GAMMA[l][m] * r2);
      if (l > m) { r2 = r1; r1 = r; }
      const float v = g[l] * r;   // value weight of r_l^m
      const float w = fmaf(-R[l], r, r);  // P_l(t) r: t-derivative weight (times 1 / 2 pi)
      if (m == 0) {
        Tc = fmaf(W[idx(l, 0)], w, Tc);
      } else {
        Xc = fmaf(W[idx(l, m)], v, Xc);
        Xs = fmaf(W[idx(l, -m)], v, Xs);
        Tc = fmaf(W[idx(l, m)], w, Tc);
        Ts = fmaf(W[idx(l, -m)], w, Ts);
        Zc = fmaf(Wz[idx(l, m - 1)], v, Zc);
        if (m - 1 >= 1) Zs = fmaf(Wz[idx(l, -(m - 1))], v, Zs);
      }
    }
    Gt = fmaf(Tc, C[m], fmaf(Ts, Sn[m], Gt));
    if (m >= 1) {
      const float fm = (float)m;
      Gz = fmaf(Zc, C[m - 1], fmaf(Zs, Sn[m - 1], Gz));
      Gx = fmaf(fm, fmaf(Xc, C[m - 1], Xs * Sn[m - 1]), Gx);
      Gy = fmaf(fm, fmaf(Xs, C[m - 1], -Xc * Sn[m - 1]), Gy);
    }
  }
  Gt *= SHV_TWO_PI;
  // chain rule: s = v/|v| (tangential part / |v|), t(|v|, r)
  const float sd = fmaf(Gx, G.x, fmaf(Gy, G.y, Gz * G.z));
  gvx = (Gx - sd * G.x) * G.inv;
  gvy = (Gy - sd * G.y) * G.inv;
  gvz = (Gz - sd * G.z) * G.inv;
  gr = 0.0f;
  if (G.t > 0.0f) {
    const float k = Gt * G.rs * fast_rcp(G.t) * G.inv;  // dLoss/dt * (-dt/dr); t > 0 here
    const float kd = k * G.rs;                // dLoss/dt * dt/d|v|
    gvx = fmaf(kd, G.x, gvx);
    gvy = fmaf(kd, G.y, gvy);
    gvz = fmaf(kd, G.z, gvz);
    gr = -k;
  }
}

template <int NB>
__device__ __forceinline__ void pair_bwd_item(const float* __restrict__ Wg, const float* __restrict__ pts, int64_t P,
                                              const float4* __restrict__ sph, int S, int chunk,
                                              float* __restrict__ gp_part, float4* __restrict__ gs_part, int64_t bx,
                                              int by, PairBwdShared& sh) {
  constexpr int N = NB * NB;
  auto& red = sh.red;
  auto& gpx_w = sh.gpx_w;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p = bx * 64 + lane;
  const bool ok = p < P;
  const int s0 = by * chunk;
  const int s1 = min(S, s0 + chunk);
  const int64_t q = ok ? p : 0;  // valid receiver for the loads of tail lanes
  const float px = sel0(ok, pts[q]);
  const float py = sel0(ok, pts[P + q]);
  const float pz = sel0(ok, pts[2 * P + q]);

  // W_lm and its z-derivative weights RHO[l][|m|] W_lm (zero on tail lanes,
  // so they contribute nothing to the sphere sums).
  float W[N], Wz[N];
#pragma unroll
  for (int l = 0; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const float w = sel0(ok, Wg[(int64_t)idx(l, m) * P + q]);
      W[idx(l, m)] = w;
      Wz[idx(l, m)] = w * SHV_RHO[l][m < 0 ? -m : m];
    }
  }

  float gpx = 0.0f, gpy = 0.0f, gpz = 0.0f;
  for (int j = threadIdx.x; j < s1 - s0; j += SHV_BLOCK) sh.sph[j] = sph[s0 + j];
  __syncthreads();
  for (int s = s0 + wave; s < s1; s += SHV_WAVES_PER_BLOCK) {
    const PairGeom G = pair_geom(px, py, pz, sh.sph[s - s0]);
    float gvx, gvy, gvz, gr;
    pair_adjoint<NB>(G, W, Wz, gvx, gvy, gvz, gr);
    gpx -= gvx;
    gpy -= gvy;
    gpz -= gvz;
    const float tot = wave_sum4(gvx, gvy, gvz, gr);  // total of (gvx, gvy, gvz, gr)[lane & 3]
    if (lane >= 60) reinterpret_cast<float*>(red)[(s - s0) * 4 + (lane & 3)] = tot;  // one wave per sphere
  }
  if (wave > 0) {
    gpx_w[wave - 1][0][lane] = gpx;
    gpx_w[wave - 1][1][lane] = gpy;
    gpx_w[wave - 1][2][lane] = gpz;
  }
  __syncthreads();
  if (wave == 0 && ok) {
#pragma unroll
    for (int w = 0; w < SHV_WAVES_PER_BLOCK - 1; ++w) {
      gpx += gpx_w[w][0][lane];
      gpy += gpx_w[w][1][lane];
      gpz += gpx_w[w][2][lane];
    }
    float* out = gp_part + (int64_t)by * 3 * P + p;
    out[0] = gpx;
    out[P] = gpy;
    out[2 * P] = gpz;
  }
  for (int j = threadIdx.x; j < s1 - s0; j += SHV_BLOCK) gs_part[bx * S + s0 + j] = red[j];
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_pair_bwd(const float* __restrict__ Wg, const float* __restrict__ pts,
                                                        int64_t P, const float4* __restrict__ sph, int S, int chunk,
                                                        float* __restrict__ gp_part, float4* __restrict__ gs_part) {
  __shared__ PairBwdShared sh;
  pair_bwd_item<NB>(Wg, pts, P, sph, S, chunk, gp_part, gs_part, blockIdx.x, blockIdx.y, sh);
}

// ---------------------------------------------------------------------------
// Launchers for one band count (instantiated per band count in shv_nb.hip).

template <int NB>
hipError_t pair_fwd_nb(const float* pts, int64_t P, const float* sph, int S, Split sp, float* Fpart,
                       const float* light, float* M, hipStream_t st) {
  dim3 grid((unsigned)pair_blocks(P), (unsigned)sp.nchunks);
  k_pair_fwd<NB><<<grid, SHV_BLOCK, 0, st>>>(pts, P, (const float4*)sph, S, sp.chunk, Fpart, light, M);
  return hipGetLastError();
}

template <int NB>
hipError_t pair_bwd_nb(const float* W, const float* pts, int64_t P, const float* sph, int S, Split sp, float* gp_part,
                       float* gs_part, hipStream_t st) {
  dim3 grid((unsigned)pair_blocks(P), (unsigned)sp.nchunks);
  k_pair_bwd<NB><<<grid, SHV_BLOCK, 0, st>>>(W, pts, P, (const float4*)sph, S, sp.chunk, gp_part, (float4*)gs_part);
  return hipGetLastError();
}

// Batched pair phases over the scenes with NB bands, one block per item.
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_batch_pair_fwd(const char* __restrict__ table) {
  __shared__ PairFwdShared<NB> sh;
  const BatchView v(table);
  const int64_t item = blockIdx.x;
  if (item >= v.h->total_pair_f[NB]) return;
  const BatchScene S = in_global(v.scene_of_pair_fwd(NB, item));
  const int64_t local = item - S.off_pair_f;
  const int64_t tile = local % S.range_tiles;
  const int by = (int)(local / S.range_tiles);
  pair_fwd_item<NB>(S.points, S.P, reinterpret_cast<const float4*>(S.spheres), (int)S.S, S.chunk_f, S.Fpart, S.light,
                    S.M, S.tile0 + tile, by, tile, S.range_tiles, sh);
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_batch_pair_bwd(const char* __restrict__ table) {
  __shared__ PairBwdShared sh;
  const BatchView v(table);
  const int64_t item = blockIdx.x;
  if (item >= v.h->total_pair_b[NB]) return;
  const BatchScene S = in_global(v.scene_of_pair_bwd(NB, item));
  if (!S.grad_radiance || (!S.grad_points && !S.grad_spheres)) return;  // uniform: nothing to do
  const int64_t local = item - S.off_pair_b;
  const int64_t bx = S.tile0 + local % S.range_tiles;
  const int by = (int)(local / S.range_tiles);
  pair_bwd_item<NB>(S.W, S.points, S.P, reinterpret_cast<const float4*>(S.spheres), (int)S.S, S.chunk_b, S.gp,
                    reinterpret_cast<float4*>(S.gs), bx, by, sh);
}

template <int NB>
hipError_t batch_pair_fwd_nb(const void* table, int64_t blocks, hipStream_t st) {
  k_batch_pair_fwd<NB><<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  return hipGetLastError();
}

template <int NB>
hipError_t batch_pair_bwd_nb(const void* table, int64_t blocks, hipStream_t st) {
  k_batch_pair_bwd<NB><<<(unsigned)blocks, SHV_BLOCK, 0, st>>>((const char*)table);
  return hipGetLastError();
}

}  // namespace shv
