// Shading pieces shared by the separate shading kernels and the fused render
// kernels (Eq. 8 with the clamped-cosine transfer of Eqs. 10-11).
//
// M(L) is read from a block-local LDS copy of its transfer-support columns
// (stage_M), so the many uniform reads of the shading products are LDS
// broadcasts rather than scalar-cache loads.
//
// Canonical summation orders (every kernel uses these, so the separate and
// fused paths and all kernel variants give bit-identical results):
//   * B = a * sum_{g=0..3} ( sum over support columns kk = g, g+4, ... of
//     H_k t_k ), t_k = sum_j M_jk V_j in index order, the four partials
//     added as ((p0 + p1) + p2) + p3;
//   * the lighting gradient is formed per tile of 64 receivers: Q_jk summed
//     over the tile's receivers in order, contracted with C, and the tile
//     partials summed in tile order afterwards.
//
// The dense sums over M (t = M^T V, Vbar = w M H, and the tile GEMM Q) run on
// the matrix cores as chains of FP32 MFMA steps.  Each step of
// v_mfma_f32_4x4x1f32 and of v_mfma_f32_16x16x4f32 (one K index after the
// other) is one fused multiply-add rounded once, so a chain gives the bits of
// the fmaf chain that adds the same terms in the same order (checked on the
// device over 64-step chains: every bit equal); the orders above are those
// chains' step orders.
#pragma once

#include "shv_device.h"

namespace shv {

template <int NB>
struct MTab;
#define SHV_MTAB(n)                                                                            \
  template <>                                                                                  \
  struct MTab<n> {                                                                             \
    static __device__ __forceinline__ const int* ptr() { return shv_mtab_ptr_##n; }            \
    static __device__ __forceinline__ const unsigned char* ind() { return shv_mtab_idx_##n; }  \
    static __device__ __forceinline__ const float* val() { return shv_mtab_val_##n; }          \
    static __device__ __forceinline__ const int* lcnt() { return shv_ltab_cnt_##n; }           \
    static __device__ __forceinline__ const unsigned short* lent() { return shv_ltab_pent_##n; }\
    static __device__ __forceinline__ const float* lval() { return shv_ltab_pval_##n; }        \
    static constexpr int LSLOTS = SHV_LTAB_SLOTS_##n;                                          \
    static __device__ __forceinline__ int supp(int kk) { return SHV_HSUPP_##n[kk]; }           \
    static constexpr int HS = SHV_HSUPP_COUNT_##n;                                             \
  };
SHV_MTAB(1)
SHV_MTAB(2)
SHV_MTAB(3)
SHV_MTAB(4)
SHV_MTAB(5)
SHV_MTAB(6)
SHV_MTAB(7)
SHV_MTAB(8)
#undef SHV_MTAB

// M[j * N + k] = sum_i L_i C_ijk for jk = begin, begin + stride, ...
template <int NB>
__device__ __forceinline__ void build_M_range(const float* __restrict__ L, float* __restrict__ M, int begin,
                                              int stride) {
  constexpr int N = NB * NB;
  const int* ptr = MTab<NB>::ptr();
  const unsigned char* ind = MTab<NB>::ind();
  const float* val = MTab<NB>::val();
  for (int jk = begin; jk < N * N; jk += stride) {
    float a = 0.0f;
    for (int e = ptr[jk]; e < ptr[jk + 1]; ++e) a = fmaf(L[ind[e]], val[e], a);
    M[jk] = a;
  }
}

// LDS copy of the support columns of M: support column kk = 4c + g of row j
// at Ms[(g * N + j) * CPG + c], so wave group g's columns are contiguous.
template <int NB>
struct MSupp {
  static constexpr int N = NB * NB;
  static constexpr int CPG = (MTab<NB>::HS + 3) / 4;
  static constexpr int SIZE = 4 * N * CPG;
  static __device__ __forceinline__ constexpr int at(int j, int kk) { return ((kk & 3) * N + j) * CPG + (kk >> 2); }
};

// The clamped cosine's odd bands above 1 vanish.
__device__ __forceinline__ constexpr bool h_support(int l) { return l <= 2 || (l % 2) == 0; }

// The coefficient index k of support column kk of the clamped cosine (its
// bands l <= 2 and even l, each in m order), by arithmetic rather than a
// table lookup.
template <int NB>
__device__ __forceinline__ int support_index(int kk) {
  int k = 0, base = 0;
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (!h_support(l)) continue;
    const int w = 2 * l + 1;
    k = (kk >= base && kk < base + w) ? l * l + (kk - base) : k;
    base += w;
  }
  return k;
}

// Fill Ms from M (global) with the SHV_BLOCK threads tid of a block; the
// caller synchronises before reading it.  Every thread computes all of its
// source addresses first and then issues all of its loads (no per-element
// branch), so their latencies overlap.
template <int NB>
__device__ __forceinline__ void stage_M(const float* __restrict__ M, float* Ms, int tid) {
  constexpr int N = NB * NB, CPG = MSupp<NB>::CPG, HS = MTab<NB>::HS, SIZE = MSupp<NB>::SIZE;
  constexpr int IT = (SIZE + SHV_BLOCK - 1) / SHV_BLOCK;
  int src[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e0 = tid + it * SHV_BLOCK;
    const int e = e0 < SIZE ? e0 : SIZE - 1;
    const int c = e % CPG, j = (e / CPG) % N, g = e / (CPG * N);
    const int kk = 4 * c + g;
    src[it] = j * N + support_index<NB>(kk < HS ? kk : HS - 1);
  }
  float v[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) v[it] = M[src[it]];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = tid + it * SHV_BLOCK;
    if (e < SIZE) Ms[e] = (4 * (e % CPG) + e / (CPG * N)) < HS ? v[it] : 0.0f;
  }
}

// H_lm = A_l y_lm(n_hat) on the support (0 elsewhere); returns 1/|n|.
// n / |n| and 1 / |n|.
__device__ __forceinline__ float unit_normal(float nx, float ny, float nz, float& ux, float& uy, float& uz) {
  const float n2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
  const float inv = fast_rsqrt(n2);
  ux = nx * inv;
  uy = ny * inv;
  uz = nz * inv;
  return inv;
}

template <int NB>
__device__ __forceinline__ float transfer(float nx, float ny, float nz, float (&H)[NB * NB], float& ux, float& uy,
                                          float& uz) {
  const float inv = unit_normal(nx, ny, nz, ux, uy, uz);
  sh_eval<NB>(ux, uy, uz, H);
#pragma unroll
  for (int l = 0; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) H[idx(l, m)] = h_support(l) ? H[idx(l, m)] * SHV_AHAT[l] : 0.0f;
  }
  return inv;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One v_mfma_f32_4x4x1f32 step.  The wave's lanes form 16 blocks of four
// (lanes 4b .. 4b + 3); accumulator i of lane 4b + c gains coef(lane 4b + i)
// * own(lane 4b + c).  With own the lane's operand of its receiver and coef
// the coefficient that output slot (lane & 3) needs, each lane's four
// accumulators are four sums over its own receiver.  All 64 lanes must be
// active: a lane's coefficient feeds its whole block.
__device__ __forceinline__ f32x4 mfma_own4(float coef, float own, f32x4 acc) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(coef, own, acc, 0, 0, 0);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.0f, 0.0f, 0.0f, 0.0f}; }

// t[ch][c] = sum_j M_jk V_j over j in index order for the wave group's
// support columns kk = 4c + G (c < NC) of CH channels (channel ch's staged M
// at Ms + ch * SZ); vj(j) gives the lane's V_j.  Columns c = 4q .. 4q + 3 form
// one four-slot chain.
template <int NB, int G, int CH, typename VF>
__device__ __forceinline__ void col_sums(VF vj, const float* Ms, float (&t)[CH][MSupp<NB>::CPG]) {
  constexpr int N = NB * NB;
  constexpr int CPG = MSupp<NB>::CPG;
  constexpr int SZ = MSupp<NB>::SIZE;
  constexpr int NC = (MTab<NB>::HS - G + 3) / 4;
  constexpr int NQ = NC > 0 ? (NC + 3) / 4 : 1;  // a group has no column at 1 band
  const int slot = threadIdx.x & 3;
  int col[NQ];  // this lane's column in chain q (clamped into the row; that slot is then unused)
#pragma unroll
  for (int q = 0; q < NQ; ++q) col[q] = G * N * CPG + (4 * q + slot < CPG ? 4 * q + slot : CPG - 1);
  f32x4 acc[CH][NQ];
#pragma unroll
  for (int ch = 0; ch < CH; ++ch)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[ch][q] = zero4();
  if constexpr (NC > 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const float v = vj(j);
#pragma unroll
      for (int ch = 0; ch < CH; ++ch)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[ch][q] = mfma_own4(Ms[ch * SZ + col[q] + j * CPG], v, acc[ch][q]);
    }
  }
#pragma unroll
  for (int ch = 0; ch < CH; ++ch)
#pragma unroll
    for (int c = 0; c < CPG; ++c) t[ch][c] = c < NC ? acc[ch][c >> 2][c & 3] : 0.0f;
}

// Partial g of sum_k H_k t_k over support columns kk = g, g + 4, ... from the
// column sums t of col_sums; also Hb_k = w t_k A_l for those columns (the
// cotangent of y_k(n_hat)).
template <int NB, int G, bool ADJ, bool ACC = false>
__device__ __forceinline__ float shade_from_cols(const float (&t)[MSupp<NB>::CPG], const float (&H)[NB * NB], float w,
                                                 float (&Hb)[NB * NB]) {
  float s = 0.0f;
  int kk = 0;
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (!h_support(l)) continue;
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const int k = idx(l, m);
      const int col = kk++;
      if ((col & 3) != G) continue;
      const float tc = t[col >> 2];
      s = fmaf(H[k], tc, s);
      if (ADJ && ACC) Hb[k] += w * tc * SHV_AHAT[l];
      if (ADJ && !ACC) Hb[k] = w * tc * SHV_AHAT[l];
    }
  }
  return s;
}

// Partial g of sum_k H_k t_k (t_k = sum_j M_jk V_j) over support columns
// kk = g, g + 4, ..., with the Hb of shade_from_cols.  Ms is the staged copy
// of M (stage_M).  Called by all 64 lanes of the wave.
template <int NB, int G, bool ADJ, bool ACC = false>
__device__ __forceinline__ float shade_partial(const float (&V)[NB * NB], const float (&H)[NB * NB],
                                               const float* Ms, float w, float (&Hb)[NB * NB]) {
  float t[1][MSupp<NB>::CPG];
  col_sums<NB, G, 1>([&](int j) { return V[j]; }, Ms, t);
  return shade_from_cols<NB, G, ADJ, ACC>(t[0], H, w, Hb);
}

// V^T M H in the canonical order (and the y_k cotangents when ADJ), all four
// column groups in one pass over j (their chains interleave).  Called by all
// 64 lanes of the wave.
template <int NB, bool ADJ>
__device__ __forceinline__ float shade_value(const float (&V)[NB * NB], const float (&H)[NB * NB],
                                             const float* Ms, float w, float (&Hb)[NB * NB]) {
  constexpr int N = NB * NB;
  constexpr int CPG = MSupp<NB>::CPG;
  constexpr int NQ = (CPG + 3) / 4;
  if (ADJ) {
#pragma unroll
    for (int i = 0; i < N; ++i) Hb[i] = 0.0f;
  }
  const int slot = threadIdx.x & 3;
  int col[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) col[q] = 4 * q + slot < CPG ? 4 * q + slot : CPG - 1;
  f32x4 acc[4][NQ];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[g][q] = zero4();
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[g][q] = mfma_own4(Ms[(g * N + j) * CPG + col[q]], V[j], acc[g][q]);
  }
  float t[4][CPG];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int c = 0; c < CPG; ++c) t[g][c] = acc[g][c >> 2][c & 3];
  const float s0 = shade_from_cols<NB, 0, ADJ>(t[0], H, w, Hb);
  const float s1 = shade_from_cols<NB, 1, ADJ>(t[1], H, w, Hb);
  const float s2 = shade_from_cols<NB, 2, ADJ>(t[2], H, w, Hb);
  const float s3 = shade_from_cols<NB, 3, ADJ>(t[3], H, w, Hb);
  return ((s0 + s1) + s2) + s3;
}

// Vbar_j = w sum_k M_jk H_k over the support (k in index order; Ms staged)
// for the R rows j = row(0), ..., row(R - 1): out[r] for row(r).  Four rows
// form one four-slot chain, and up to four chains share a pass over the
// support.  Called by all 64 lanes of the wave.
template <int NB, int R, typename RowF>
__device__ __forceinline__ void vbar_rows(RowF row, const float (&H)[NB * NB], const float* Ms, float w,
                                          float (&out)[R]) {
  constexpr int N = NB * NB;
  constexpr int CPG = MSupp<NB>::CPG;
  constexpr int NQ = (R + 3) / 4;
  const int slot = threadIdx.x & 3;
#pragma unroll
  for (int q0 = 0; q0 < NQ; q0 += 4) {
    constexpr int PASS = 4;
    int base[PASS];
    f32x4 acc[PASS];
#pragma unroll
    for (int u = 0; u < PASS; ++u) {
      const int q = q0 + u < NQ ? q0 + u : NQ - 1;
      int j = row(4 * q);
#pragma unroll
      for (int sl = 1; sl < 4; ++sl)
        if (4 * q + sl < R) j = slot == sl ? row(4 * q + sl) : j;
      base[u] = j * CPG;
      acc[u] = zero4();
    }
    int kk = 0;
#pragma unroll
    for (int l = 0; l < NB; ++l) {
      if (!h_support(l)) continue;
#pragma unroll
      for (int m = -l; m <= l; ++m) {
        const int off = (kk & 3) * N * CPG + (kk >> 2);  // MSupp::at(j, kk) - j * CPG
        ++kk;
#pragma unroll
        for (int u = 0; u < PASS; ++u)
          if (q0 + u < NQ) acc[u] = mfma_own4(Ms[base[u] + off], H[idx(l, m)], acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < PASS; ++u)
#pragma unroll
      for (int sl = 0; sl < 4; ++sl)
        if (4 * (q0 + u) + sl < R) out[4 * (q0 + u) + sl] = w * acc[u][sl];
  }
}

// Normal cotangent from Hb (tangential gradient of the SH polynomial / |n|).
template <int NB>
__device__ __forceinline__ void normal_grad(const float (&Hb)[NB * NB], float ux, float uy, float uz, float inv,
                                            float& gx, float& gy, float& gz) {
  sh_grad<NB>(ux, uy, uz, Hb, gx, gy, gz);
  const float sd = fmaf(gx, ux, fmaf(gy, uy, gz * uz));
  gx = (gx - sd * ux) * inv;
  gy = (gy - sd * uy) * inv;
  gz = (gz - sd * uz) * inv;
}

// LDS tile of 64 receivers for the lighting-gradient GEMM.
constexpr int kTileVS = 66;   // pitch of the V rows (8-byte aligned float2 reads)
constexpr int kTileHS = 36;   // pitch of the w H rows (16-byte aligned float4 reads)
struct alignas(16) LightTile {
  float Vt[64 * kTileVS];  // Vt[x * kTileVS + j] = V_j of receiver x
  float Ht[64 * kTileHS];  // Ht[x * kTileHS + kk] = w H_k of receiver x, kk the support index
  float Lp[4][64];
};

// Called by all 256 threads of a block once the tile is filled and synced:
// Q[j][kk] = sum_x Vt[x][j] Ht[x][kk] (x in order) as 16 x 16 output tiles of
// v_mfma_f32_16x16x4f32 chains (tile t to wave t mod 4; each step adds four
// receivers, one K index after the other), then the Lbar partial
// out[i] = sum_{(j,kk)} C_{i j k} Q[j][kk] (4 strided partials per i).
// Ends with a barrier, so the tile may be refilled afterwards.  Q is staged
// in the V rows unless a separate Qbuf (N x 32 floats) is given, in which
// case the V rows are left intact.
template <int NB>
__device__ __forceinline__ void tile_light_partial(LightTile& T, float* __restrict__ out, float* Qbuf = nullptr) {
  constexpr int N = NB * NB;
  constexpr int HS = MTab<NB>::HS;
  constexpr int RT = (N + 15) / 16, CT = (HS + 15) / 16;  // output tiles (rows j, columns kk)
  constexpr int TPW = (RT * CT + 3) / 4;                    // tiles per wave
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int r16 = lane & 15, kq = lane >> 4;
  f32x4 acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    acc[u] = zero4();
    const int t = wave + 4 * u;
    if (t < RT * CT) {  // uniform over the wave
      // A row j0 + r16 and B column k0 + r16 stay inside the tile's pitches
      // (j < 64 <= kTileVS, kk < 32 <= kTileHS); rows and columns past N and
      // HS only reach outputs that are not stored.
      const int j0 = 16 * (t / CT), k0 = 16 * (t % CT);
#pragma unroll 4
      for (int s4 = 0; s4 < 16; ++s4) {
        const int x = 4 * s4 + kq;
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(T.Vt[x * kTileVS + j0 + r16], T.Ht[x * kTileHS + k0 + r16],
                                                      acc[u], 0, 0, 0);
      }
    }
  }
  __syncthreads();
  float* Qs = Qbuf ? Qbuf : T.Vt;  // N x 32
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = wave + 4 * u;
    if (t < RT * CT) {
      const int kk = 16 * (t % CT) + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = 16 * (t / CT) + 4 * kq + i;  // output row of accumulator i
        if (j < N && kk < HS) Qs[j * 32 + kk] = acc[u][i];
      }
    }
  }
  __syncthreads();
  {
    const int i = tid >> 2, part = tid & 3;
    if (i < N) {
      // this thread's entries of row i (every 4th, in order), all loaded first
      constexpr int SL = MTab<NB>::LSLOTS;
      const int cnt = MTab<NB>::lcnt()[tid];
      const unsigned short* ent = MTab<NB>::lent() + tid * SL;
      const float* val = MTab<NB>::lval() + tid * SL;
      int e[SL];
      float v[SL];
#pragma unroll
      for (int t = 0; t < SL; ++t) {
        e[t] = ent[t];
        v[t] = val[t];
      }
      float acc = 0.0f;
#pragma unroll
      for (int t = 0; t < SL; ++t) {
        const float f = fmaf(v[t], Qs[e[t]], acc);
        acc = t < cnt ? f : acc;
      }
      T.Lp[part][i] = acc;
    }
  }
  __syncthreads();
  if (tid < N && out) out[tid] = ((T.Lp[0][tid] + T.Lp[1][tid]) + T.Lp[2][tid]) + T.Lp[3][tid];
  __syncthreads();
}

// Tile row writers: receiver x = lane of the calling wave.
template <int NB>
__device__ __forceinline__ void tile_put_v(LightTile& T, int x, const float (&V)[NB * NB]) {
#pragma unroll
  for (int j = 0; j < NB * NB; ++j) T.Vt[x * kTileVS + j] = V[j];
}
template <int NB>
__device__ __forceinline__ void tile_put_wh(LightTile& T, int x, const float (&H)[NB * NB], float w) {
  int kk = 0;
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (!h_support(l)) continue;
#pragma unroll
    for (int m = -l; m <= l; ++m) T.Ht[x * kTileHS + (kk++)] = w * H[idx(l, m)];
  }
}

}  // namespace shv
