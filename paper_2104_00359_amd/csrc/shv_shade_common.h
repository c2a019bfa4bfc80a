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

// Partial g of sum_k H_k t_k over support columns kk = g, g + 4, ...; also
// Hb_k = w t_k A_l for those columns (the cotangent of y_k(n_hat)).  Ms is
// the staged copy of M (stage_M).
template <int NB, int G, bool ADJ, bool ACC = false>
__device__ __forceinline__ float shade_partial(const float (&V)[NB * NB], const float (&H)[NB * NB],
                                               const float* Ms, float w, float (&Hb)[NB * NB]) {
  constexpr int N = NB * NB;
  constexpr int CPG = MSupp<NB>::CPG;
  constexpr int NC = (MTab<NB>::HS - G + 3) / 4;  // this group's columns kk = G, G + 4, ...
  // t_kk = sum_j M_jk V_j, j in index order for every column; the group's
  // columns of one row are contiguous in Ms (vector LDS reads)
  float t[CPG];
#pragma unroll
  for (int c = 0; c < CPG; ++c) t[c] = 0.0f;
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int c = 0; c < NC; ++c) t[c] = fmaf(Ms[MSupp<NB>::at(j, 4 * c + G)], V[j], t[c]);
  }
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

// V^T M H in the canonical order (and the y_k cotangents when ADJ).
template <int NB, bool ADJ>
__device__ __forceinline__ float shade_value(const float (&V)[NB * NB], const float (&H)[NB * NB],
                                             const float* M, float w, float (&Hb)[NB * NB]) {
  if (ADJ) {
#pragma unroll
    for (int i = 0; i < NB * NB; ++i) Hb[i] = 0.0f;
  }
  const float s0 = shade_partial<NB, 0, ADJ>(V, H, M, w, Hb);
  const float s1 = shade_partial<NB, 1, ADJ>(V, H, M, w, Hb);
  const float s2 = shade_partial<NB, 2, ADJ>(V, H, M, w, Hb);
  const float s3 = shade_partial<NB, 3, ADJ>(V, H, M, w, Hb);
  return ((s0 + s1) + s2) + s3;
}

// As shade_value<NB, true>, but adding this channel's y_k cotangents to Hb
// (several colour channels that share V and H, Eq. 8 per channel).
template <int NB>
__device__ __forceinline__ float shade_value_acc(const float (&V)[NB * NB], const float (&H)[NB * NB],
                                                 const float* M, float w, float (&Hb)[NB * NB]) {
  const float s0 = shade_partial<NB, 0, true, true>(V, H, M, w, Hb);
  const float s1 = shade_partial<NB, 1, true, true>(V, H, M, w, Hb);
  const float s2 = shade_partial<NB, 2, true, true>(V, H, M, w, Hb);
  const float s3 = shade_partial<NB, 3, true, true>(V, H, M, w, Hb);
  return ((s0 + s1) + s2) + s3;
}

// Vbar_j = w sum_k M_jk H_k over the support (k in index order; Ms staged).
template <int NB>
__device__ __forceinline__ float vbar_entry(int j, const float (&H)[NB * NB], const float* Ms, float w) {
  float t = 0.0f;
  int kk = 0;
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (!h_support(l)) continue;
#pragma unroll
    for (int m = -l; m <= l; ++m) t = fmaf(Ms[MSupp<NB>::at(j, kk++)], H[idx(l, m)], t);
  }
  return w * t;
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
// Q[j][kk] = sum_x Vt[x][j] Ht[x][kk] (x in order; thread (jj, kq) owns
// j = 2jj, 2jj+1 and kk = 4kq .. 4kq+3), then Lbar partial
// out[i] = sum_{(j,kk)} C_{i j k} Q[j][kk] (4 strided partials per i).
// Ends with a barrier, so the tile may be refilled afterwards.  Q is staged
// in the V rows unless a separate Qbuf (N x 32 floats) is given, in which
// case the V rows are left intact.
template <int NB>
__device__ __forceinline__ void tile_light_partial(LightTile& T, float* __restrict__ out, float* Qbuf = nullptr) {
  constexpr int N = NB * NB;
  constexpr int HS = MTab<NB>::HS;
  const int tid = threadIdx.x;
  const int jj = tid & 31, kq = tid >> 5;
  float q[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) q[i] = 0.0f;
  if (2 * jj < N && 4 * kq < HS) {
#pragma unroll 8
    for (int x = 0; x < 64; ++x) {
      const float2 v = *reinterpret_cast<const float2*>(&T.Vt[x * kTileVS + 2 * jj]);
      const float4 h = *reinterpret_cast<const float4*>(&T.Ht[x * kTileHS + 4 * kq]);
      q[0] = fmaf(v.x, h.x, q[0]);
      q[1] = fmaf(v.x, h.y, q[1]);
      q[2] = fmaf(v.x, h.z, q[2]);
      q[3] = fmaf(v.x, h.w, q[3]);
      q[4] = fmaf(v.y, h.x, q[4]);
      q[5] = fmaf(v.y, h.y, q[5]);
      q[6] = fmaf(v.y, h.z, q[6]);
      q[7] = fmaf(v.y, h.w, q[7]);
    }
  }
  __syncthreads();
  float* Qs = Qbuf ? Qbuf : T.Vt;  // N x 32
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = 2 * jj + a, kk = 4 * kq + c;
      if (j < N && kk < HS) Qs[j * 32 + kk] = q[a * 4 + c];
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
