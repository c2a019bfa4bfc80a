// The SH exponential as the projection of the pointwise exponential (the
// function-space quantity that the scaling and squaring scheme stands in for),
// taken with a fixed quadrature on MFMA.  A selectable accuracy mode; it
// changes the result.
//
//   F = eps * lambda * (sum of the sphere-chunk partials)   (as in the squaring path)
//   c = F_0 / sqrt(4 pi),  f_q = sum_{i >= 1} F_i y_i(w_q)
//   V = exp(c) sum_q w_q exp(f_q) y(w_q)
// over the product rule of degree 8n - 1: 4n Gauss-Legendre nodes in z times
// 8n uniform azimuths (weights wz * 2 pi / 8n), padded to a multiple of 64
// nodes with zero weights.
//
// For a block of 64 receivers and a tile of 64 nodes the two sums are GEMMs:
//   f [64 rec x 64 nodes] = Fhat [64 x 64 coef] * Y [64 coef x 64 nodes]
//   V [64 rec x 64 coef] += (w exp f) [64 x 64 nodes] * Y^T [64 nodes x 64 coef]
// (coefficients padded to 64).  Four waves each own one 32 x 32 quadrant of
// both and run them on v_mfma_f32_32x32x2f32; the tile's Y is evaluated in LDS
// from the node directions, and w exp f goes through LDS between the GEMMs.
//
// Adjoint for Vbar: Fbar_0 = (sum_j Vbar_j V_j) / sqrt(4 pi) and, for i >= 1,
//   Fbar_i = exp(c) sum_q w_q exp(f_q) g_q y_i(w_q),  g_q = sum_j Vbar_j y_j(w_q)
// (three GEMMs per tile); W = eps * lambda * Fbar feeds the pair adjoint.
#pragma once

#include "shv_exp_impl.h"

namespace shv {

typedef float mfma_f32x16 __attribute__((ext_vector_type(16)));

constexpr int kQuadPitch = 65;  // LDS row pitch of the 64 x 64 tiles (no bank conflicts down a column)

template <int NB>
struct QuadTab;
#define SHV_QTAB(n)                                                                         \
  template <>                                                                               \
  struct QuadTab<n> {                                                                       \
    static __device__ __forceinline__ float z(int i) { return shv_quad_z_##n[i]; }          \
    static __device__ __forceinline__ float w(int i) { return shv_quad_w_##n[i]; }          \
  };
SHV_QTAB(1)
SHV_QTAB(2)
SHV_QTAB(3)
SHV_QTAB(4)
SHV_QTAB(5)
SHV_QTAB(6)
SHV_QTAB(7)
SHV_QTAB(8)
#undef SHV_QTAB

template <int NB>
struct QuadRule {
  static constexpr int NZ = 4 * NB;           // Gauss-Legendre nodes in z
  static constexpr int NPHI = 8 * NB;         // uniform azimuths
  static constexpr int Q = NZ * NPHI;         // real nodes
  static constexpr int QP = (Q + 63) / 64 * 64;
};

// Node q of the rule: direction and weight (weight 0 for the padding nodes).
template <int NB>
__device__ __forceinline__ void quad_node(int q, float& x, float& y, float& z, float& w) {
  constexpr int NPHI = QuadRule<NB>::NPHI;
  if (q >= QuadRule<NB>::Q) {
    x = 0.0f;
    y = 0.0f;
    z = 1.0f;
    w = 0.0f;
    return;
  }
  const int zi = q / NPHI, mi = q - zi * NPHI;
  z = QuadTab<NB>::z(zi);
  const float st = sqrtf(fmaxf(0.0f, 1.0f - z * z));
  float s, c;
  sincosf(((float)mi + 0.5f) * (SHV_TWO_PI / (float)NPHI), &s, &c);
  x = st * c;
  y = st * s;
  w = QuadTab<NB>::w(zi) * (SHV_TWO_PI / (float)NPHI);
}

struct QuadShared {
  float Yt[64 * kQuadPitch];  // Yt[coef * pitch + node]
  float Et[64 * kQuadPitch];  // Et[rec * pitch + node]
  float wq[64];
  float cs[64];               // c of each receiver
};

// The rule's basis table: Ytab[q * 64 + t] = y_t(w_q) (0 for t >= N) and
// wtab[q], one thread per node (once per call; every block then reads it).
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_quad_table(float* __restrict__ Ytab, float* __restrict__ wtab) {
  constexpr int N = NB * NB;
  const int q = blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (q >= QuadRule<NB>::QP) return;
  float x, y, z, w;
  quad_node<NB>(q, x, y, z, w);
  float Y[N];
  sh_eval<NB>(x, y, z, Y);
#pragma unroll
  for (int t = 0; t < 64; ++t) Ytab[(int64_t)q * 64 + t] = t < N ? Y[t < N ? t : 0] : 0.0f;
  wtab[q] = w;
}

// The tile's 64 nodes from the table into Yt [coef][node] and wq: thread t
// copies 16 coefficients (t % 4) of node t / 4 (float4 loads).
__device__ __forceinline__ void quad_tile_load(QuadShared& sh, const float* __restrict__ Ytab,
                                               const float* __restrict__ wtab, int q0) {
  const int node = threadIdx.x >> 2, part = threadIdx.x & 3;
  const float4* src = reinterpret_cast<const float4*>(Ytab + (int64_t)(q0 + node) * 64 + 16 * part);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float4 y = src[v];
    const int c = 16 * part + 4 * v;
    sh.Yt[(c + 0) * kQuadPitch + node] = y.x;
    sh.Yt[(c + 1) * kQuadPitch + node] = y.y;
    sh.Yt[(c + 2) * kQuadPitch + node] = y.z;
    sh.Yt[(c + 3) * kQuadPitch + node] = y.w;
  }
  if (part == 0) sh.wq[node] = wtab[q0 + node];
}

// 32 x 32 quadrant (rows ra.., cols cb..) of A [64 x 64 K] * B [64 K x 64]
// with A taken from the lane's registers a[32] (A[ra + l % 32][2s + l / 32])
// and B from LDS as Bsrc[(2s + l / 32) * bk + (cb + l % 32) * bn].
__device__ __forceinline__ mfma_f32x16 quad_gemm_regA(const float (&a)[32], const float* Bsrc, int bk, int bn,
                                                     int cb, mfma_f32x16 acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const float b = Bsrc[(2 * s + (lane >> 5)) * bk + (cb + (lane & 31)) * bn];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], b, acc, 0, 0, 0);
  }
  return acc;
}

// Both operands from LDS: A as Asrc[(ra + l % 32) * ak + (2s + l / 32)].
__device__ __forceinline__ mfma_f32x16 quad_gemm_lds(const float* Asrc, int ak, int ra, const float* Bsrc, int bk,
                                                    int bn, int cb, mfma_f32x16 acc) {
  const int lane = threadIdx.x & 63;
#pragma unroll 8
  for (int s = 0; s < 32; ++s) {
    const float a = Asrc[(ra + (lane & 31)) * ak + 2 * s + (lane >> 5)];
    const float b = Bsrc[(2 * s + (lane >> 5)) * bk + (cb + (lane & 31)) * bn];
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Row (within the 32 x 32 quadrant) of accumulator element r of this lane.
__device__ __forceinline__ int quad_row(int r) { return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3); }

// The lane's A operand rows of F-like data: a[s] = X[coef 2s + l / 32][rec ra + l % 32]
// for a row-major [N][P] array (0 past N or P), summed over `chunks` arrays `stride` apart.
template <int NB>
__device__ __forceinline__ void quad_load_rows(const float* __restrict__ X, int chunks, int64_t stride, int64_t P,
                                               int64_t p, bool ok, float (&a)[32]) {
  constexpr int N = NB * NB;
  const int half = (threadIdx.x & 63) >> 5;
  const int64_t q = ok ? p : 0;
  // Chunk by chunk, each chunk's 32 loads issued together (the sum per row
  // is still taken in chunk order).
#pragma unroll
  for (int s = 0; s < 32; ++s) {
    const int coef = 2 * s + half;
    a[s] = X[(int64_t)(coef < N ? coef : N - 1) * P + q];
  }
  for (int c = 1; c < chunks; ++c) {
    const float* src = X + c * stride + q;
    float t[32];
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const int coef = 2 * s + half;
      t[s] = src[(int64_t)(coef < N ? coef : N - 1) * P];
    }
#pragma unroll
    for (int s = 0; s < 32; ++s) a[s] += t[s];
  }
#pragma unroll
  for (int s = 0; s < 32; ++s) a[s] = (ok && 2 * s + half < N) ? a[s] : 0.0f;
}

// Forward: Fpart [nchunks][N][P] -> vis [gridDim.y][N][P], the partial sums of
// V over the node tiles y, y + gridDim.y, ... (added afterwards in order);
// saved (may be NULL) <- F [N][P].
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_quad_fwd(const float* __restrict__ Fpart, int nchunks, int64_t P,
                                                            float eps, float* __restrict__ vis,
                                                            float* __restrict__ saved,
                                                            const float* __restrict__ Ytab,
                                                            const float* __restrict__ wtab) {
  constexpr int N = NB * NB;
  __shared__ QuadShared sh;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ra = 32 * (wave & 1), cb = 32 * (wave >> 1);
  const int half = lane >> 5;
  const int64_t p = (int64_t)blockIdx.x * 64 + ra + (lane & 31);
  const bool ok = p < P;
  float a[32];
  quad_load_rows<NB>(Fpart, nchunks, (int64_t)N * P, P, p, ok, a);
#pragma unroll
  for (int s = 0; s < 32; ++s) a[s] *= eps * coef_lambda(2 * s + half < N ? 2 * s + half : 0);
  if (cb == 0 && ok && saved && blockIdx.y == 0) {
#pragma unroll
    for (int s = 0; s < 32; ++s)
      if (2 * s + half < N) saved[(int64_t)(2 * s + half) * P + p] = a[s];
  }
  if (cb == 0 && half == 0) sh.cs[ra + (lane & 31)] = a[0] * SHV_INV_SQRT_4PI;
  if (half == 0) a[0] = 0.0f;  // the DC term is split off exactly
  mfma_f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int q0 = 64 * blockIdx.y; q0 < QuadRule<NB>::QP; q0 += 64 * gridDim.y) {
    quad_tile_load(sh, Ytab, wtab, q0);
    __syncthreads();
    mfma_f32x16 f;
#pragma unroll
    for (int r = 0; r < 16; ++r) f[r] = 0.0f;
    f = quad_gemm_regA(a, sh.Yt, kQuadPitch, 1, cb, f);  // rows: receivers ra.., cols: nodes cb..
    const float w = sh.wq[cb + (lane & 31)];
#pragma unroll
    for (int r = 0; r < 16; ++r) sh.Et[(ra + quad_row(r)) * kQuadPitch + cb + (lane & 31)] = w * expf(f[r]);
    __syncthreads();
    // rows: receivers ra.., cols: coefficients cb.., K: the tile's nodes
    acc = quad_gemm_lds(sh.Et, kQuadPitch, ra, sh.Yt, 1, kQuadPitch, cb, acc);
    __syncthreads();
  }
  const int coef = cb + (lane & 31);
  if (coef >= N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rec = ra + quad_row(r);
    const int64_t pr = (int64_t)blockIdx.x * 64 + rec;
    if (pr < P) vis[blockIdx.y * (int64_t)N * P + (int64_t)coef * P + pr] = expf(sh.cs[rec]) * acc[r];
  }
}

// Adjoint: gV, vis, saved F [N][P] -> W [gridDim.y][N][P], partial sums of
// eps lambda Fbar over the node tiles as in the forward.
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_quad_bwd(const float* __restrict__ gV,
                                                            const float* __restrict__ vis,
                                                            const float* __restrict__ saved, int64_t P, float eps,
                                                            float* __restrict__ W, const float* __restrict__ Ytab,
                                                            const float* __restrict__ wtab) {
  constexpr int N = NB * NB;
  __shared__ QuadShared sh;
  __shared__ float cbar[64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ra = 32 * (wave & 1), cb = 32 * (wave >> 1);
  const int half = lane >> 5;
  const int64_t p = (int64_t)blockIdx.x * 64 + ra + (lane & 31);
  const bool ok = p < P;
  float a[32], g[32];
  quad_load_rows<NB>(saved, 1, 0, P, p, ok, a);
  quad_load_rows<NB>(gV, 1, 0, P, p, ok, g);
  if (cb == 0 && half == 0) sh.cs[ra + (lane & 31)] = a[0] * SHV_INV_SQRT_4PI;
  if (half == 0) a[0] = 0.0f;
  if (threadIdx.x < 64) {  // sum_j Vbar_j V_j per receiver, j in index order
    const int64_t pr = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int64_t q = pr < P ? pr : 0;
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < N; ++j) s = fmaf(gV[(int64_t)j * P + q], vis[(int64_t)j * P + q], s);
    cbar[threadIdx.x] = pr < P ? s : 0.0f;
  }
  mfma_f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int q0 = 64 * blockIdx.y; q0 < QuadRule<NB>::QP; q0 += 64 * gridDim.y) {
    quad_tile_load(sh, Ytab, wtab, q0);
    __syncthreads();
    mfma_f32x16 f, gq;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      f[r] = 0.0f;
      gq[r] = 0.0f;
    }
    f = quad_gemm_regA(a, sh.Yt, kQuadPitch, 1, cb, f);
    gq = quad_gemm_regA(g, sh.Yt, kQuadPitch, 1, cb, gq);
    const float w = sh.wq[cb + (lane & 31)];
#pragma unroll
    for (int r = 0; r < 16; ++r)
      sh.Et[(ra + quad_row(r)) * kQuadPitch + cb + (lane & 31)] = w * expf(f[r]) * gq[r];
    __syncthreads();
    acc = quad_gemm_lds(sh.Et, kQuadPitch, ra, sh.Yt, 1, kQuadPitch, cb, acc);
    __syncthreads();
  }
  const int coef = cb + (lane & 31);
  if (coef >= N) return;
  const float lam = eps * coef_lambda(coef);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int rec = ra + quad_row(r);
    const int64_t pr = (int64_t)blockIdx.x * 64 + rec;
    if (pr >= P) continue;
    const float fb = coef == 0 ? (blockIdx.y == 0 ? cbar[rec] * SHV_INV_SQRT_4PI : 0.0f) : expf(sh.cs[rec]) * acc[r];
    W[blockIdx.y * (int64_t)N * P + (int64_t)coef * P + pr] = lam * fb;
  }
}

// table: QuadRule<NB>::QP * 65 floats (the basis, then the weights); part:
// kQuadSplits * N * P floats, the per-split partial sums added in split order.
constexpr int kQuadSplits = 2;  // blocks per 64-receiver tile (node tiles interleaved)

template <int NB>
hipError_t exp_quad_fwd_nb(const float* Fpart, int nchunks, int64_t P, float eps, float* vis, float* saved,
                           float* table, float* part, hipStream_t st) {
  constexpr int QP = QuadRule<NB>::QP, N = NB * NB;
  float* Ytab = table;
  float* wtab = table + (int64_t)QP * 64;
  k_quad_table<NB><<<(QP + SHV_BLOCK - 1) / SHV_BLOCK, SHV_BLOCK, 0, st>>>(Ytab, wtab);
  k_exp_quad_fwd<NB><<<dim3((unsigned)pair_blocks(P), kQuadSplits), SHV_BLOCK, 0, st>>>(Fpart, nchunks, P, eps, part,
                                                                                        saved, Ytab, wtab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_chunks(part, kQuadSplits, (int64_t)N * P, vis, st);
}

template <int NB>
hipError_t exp_quad_bwd_nb(const float* gV, const float* vis, const float* saved, int64_t P, float eps, float* W,
                           float* table, float* part, hipStream_t st) {
  constexpr int QP = QuadRule<NB>::QP, N = NB * NB;
  float* Ytab = table;
  float* wtab = table + (int64_t)QP * 64;
  k_quad_table<NB><<<(QP + SHV_BLOCK - 1) / SHV_BLOCK, SHV_BLOCK, 0, st>>>(Ytab, wtab);
  k_exp_quad_bwd<NB><<<dim3((unsigned)pair_blocks(P), kQuadSplits), SHV_BLOCK, 0, st>>>(gV, vis, saved, P, eps, part,
                                                                                        Ytab, wtab);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum_chunks(part, kQuadSplits, (int64_t)N * P, W, st);
}

}  // namespace shv
