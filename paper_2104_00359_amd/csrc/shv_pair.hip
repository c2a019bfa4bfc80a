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
// Receiver gradients stay in registers; sphere gradients are summed over the
// wave (butterfly), then over the block's waves in LDS, in a fixed order, and
// written as per-block partials reduced by a second deterministic pass.
//
// Layout: one receiver per lane, 256 receivers per block; grid.y splits the
// sphere set into chunks so that small receiver sets still fill 256 CUs.
// Sphere records are read with wave-uniform addresses (scalar loads).

#include "shv_device.h"
#include "shv_launch.h"

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

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_pair_fwd(const float* __restrict__ pts, int64_t P,
                                                        const float4* __restrict__ sph, int S, int chunk,
                                                        float* __restrict__ Fpart) {
  constexpr int N = NB * NB;
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const bool ok = p < P;
  const int s0 = blockIdx.y * chunk;
  const int s1 = min(S, s0 + chunk);
  const float px = ok ? pts[p] : 0.0f;
  const float py = ok ? pts[P + p] : 0.0f;
  const float pz = ok ? pts[2 * P + p] : 0.0f;

  float acc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) acc[i] = 0.0f;
  // The DC coefficient sets V's overall scale through exp(F_0 / sqrt(4 pi)),
  // so its sum over spheres is compensated (Kahan).
  float dc_comp = 0.0f;

  for (int s = s0; s < s1; ++s) {
    const PairGeom G = pair_geom(px, py, pz, sph[s]);
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
  if (ok) {
    float* out = Fpart + (int64_t)blockIdx.y * N * P + p;
#pragma unroll
    for (int i = 0; i < N; ++i) out[(int64_t)i * P] = acc[i];
  }
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_pair_bwd(const float* __restrict__ Wg, const float* __restrict__ pts,
                                                        int64_t P, const float4* __restrict__ sph, int S, int chunk,
                                                        float* __restrict__ gp_part, float4* __restrict__ gs_part) {
  constexpr int N = NB * NB;
  __shared__ float4 red[SHV_WAVES_PER_BLOCK][SHV_MAX_CHUNK];
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const bool ok = p < P;
  const int s0 = blockIdx.y * chunk;
  const int s1 = min(S, s0 + chunk);
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const float px = ok ? pts[p] : 0.0f;
  const float py = ok ? pts[P + p] : 0.0f;
  const float pz = ok ? pts[2 * P + p] : 0.0f;

  // W_lm and its z-derivative weights RHO[l][|m|] W_lm (zero on tail lanes,
  // so they contribute nothing to the sphere sums).
  float W[N], Wz[N];
#pragma unroll
  for (int l = 0; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const float w = ok ? Wg[(int64_t)idx(l, m) * P + p] : 0.0f;
      W[idx(l, m)] = w;
      Wz[idx(l, m)] = w * SHV_RHO[l][m < 0 ? -m : m];
    }
  }

  float gpx = 0.0f, gpy = 0.0f, gpz = 0.0f;
  for (int s = s0; s < s1; ++s) {
    const PairGeom G = pair_geom(px, py, pz, sph[s]);
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
    float gvx = (Gx - sd * G.x) * G.inv;
    float gvy = (Gy - sd * G.y) * G.inv;
    float gvz = (Gz - sd * G.z) * G.inv;
    float gr = 0.0f;
    if (G.t > 0.0f) {
      const float k = Gt * G.rs / G.t * G.inv;  // dLoss/dt * (-dt/dr)
      const float kd = k * G.rs;                // dLoss/dt * dt/d|v|
      gvx = fmaf(kd, G.x, gvx);
      gvy = fmaf(kd, G.y, gvy);
      gvz = fmaf(kd, G.z, gvz);
      gr = -k;
    }
    gpx -= gvx;
    gpy -= gvy;
    gpz -= gvz;
    const float4 tot = make_float4(wave_sum(gvx), wave_sum(gvy), wave_sum(gvz), wave_sum(gr));
    if (lane == 0) red[wave][s - s0] = tot;
  }
  if (ok) {
    float* out = gp_part + (int64_t)blockIdx.y * 3 * P + p;
    out[0] = gpx;
    out[P] = gpy;
    out[2 * P] = gpz;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < s1 - s0; j += SHV_BLOCK) {
    float4 a = red[0][j];
#pragma unroll
    for (int w = 1; w < SHV_WAVES_PER_BLOCK; ++w) {
      const float4 b = red[w][j];
      a.x += b.x;
      a.y += b.y;
      a.z += b.z;
      a.w += b.w;
    }
    gs_part[(int64_t)blockIdx.x * S + s0 + j] = a;
  }
}

Split choose_split(int64_t P, int64_t S) {
  Split sp{1, (int)(S > 0 ? S : 1)};
  if (S <= 0) return sp;
  const int64_t waves = (P + 63) / 64;
  const int64_t target_waves = 4096;  // 4 waves per SIMD on 256 CUs x 4 SIMDs
  int64_t n = waves > 0 ? (target_waves + waves - 1) / waves : 1;
  const int64_t max_by_size = (S + 15) / 16;  // keep >= 16 spheres per chunk
  if (n > max_by_size) n = max_by_size;
  const int64_t min_by_lds = (S + SHV_MAX_CHUNK - 1) / SHV_MAX_CHUNK;
  if (n < min_by_lds) n = min_by_lds;
  if (n < 1) n = 1;
  const int64_t chunk = (S + n - 1) / n;
  sp.chunk = (int)chunk;
  sp.nchunks = (int)((S + chunk - 1) / chunk);
  return sp;
}

int64_t point_blocks(int64_t P) { return (P + SHV_BLOCK - 1) / SHV_BLOCK; }

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

hipError_t launch_pair_fwd(int nb, const float* pts, int64_t P, const float* sph, int S, Split sp, float* Fpart,
                           hipStream_t st) {
  dim3 grid((unsigned)point_blocks(P), (unsigned)sp.nchunks);
  SHV_DISPATCH(nb, k_pair_fwd, grid, SHV_BLOCK, 0, st>>>(pts, P, (const float4*)sph, S, sp.chunk, Fpart))
  return hipGetLastError();
}

hipError_t launch_pair_bwd(int nb, const float* W, const float* pts, int64_t P, const float* sph, int S, Split sp,
                           float* gp_part, float* gs_part, hipStream_t st) {
  dim3 grid((unsigned)point_blocks(P), (unsigned)sp.nchunks);
  SHV_DISPATCH(nb, k_pair_bwd, grid, SHV_BLOCK, 0,
               st>>>(W, pts, P, (const float4*)sph, S, sp.chunk, gp_part, (float4*)gs_part))
  return hipGetLastError();
}

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
__global__ __launch_bounds__(SHV_BLOCK) void k_sum_chunks(const float* __restrict__ part, int nchunks, int64_t len,
                                                          float* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (j >= len) return;
  float a = part[j];
  for (int c = 1; c < nchunks; ++c) a += part[(int64_t)c * len + j];
  out[j] = a;
}

hipError_t launch_sum_chunks(const float* part, int nchunks, int64_t len, float* out, hipStream_t st) {
  if (len <= 0) return hipSuccess;
  k_sum_chunks<<<(unsigned)((len + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(part, nchunks, len, out);
  return hipGetLastError();
}

// out[c] = sum_r part[r * cols + c] for every column c: one block per column,
// each thread sums a fixed stride of rows, then a fixed-shape tree in LDS.
__global__ __launch_bounds__(SHV_BLOCK) void k_reduce_rows(const float* __restrict__ part, int rows, int cols,
                                                           float* __restrict__ out) {
  __shared__ float buf[SHV_BLOCK];
  const int c = blockIdx.x;
  float a = 0.0f;
  for (int r = threadIdx.x; r < rows; r += SHV_BLOCK) a += part[(int64_t)r * cols + c];
  buf[threadIdx.x] = a;
  __syncthreads();
#pragma unroll
  for (int w = SHV_BLOCK / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = buf[0];
}

hipError_t launch_reduce_rows(const float* part, int rows, int cols, float* out, hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  k_reduce_rows<<<(unsigned)cols, SHV_BLOCK, 0, st>>>(part, rows, cols, out);
  return hipGetLastError();
}

}  // namespace shv
