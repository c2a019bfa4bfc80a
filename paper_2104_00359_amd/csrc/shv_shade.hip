// Diffuse SH shading B = a (L . (V * H)) (Eq. 8) and its adjoint.
//
// With the lit transfer matrix M(L)_jk = sum_i L_i C_ijk (symmetric, built once
// per call from L), B = a V^T M H.  The clamped-cosine transfer is
// H_lm = A_l y_lm(n / |n|) (Eqs. 10-11): its odd bands above 1 vanish, so only
// the columns of M on H's support are ever read (31 of 64 at n = 8).
// M is read with wave-uniform addresses, so it is served by scalar loads.
//
// Adjoint for the cotangent Bbar, w = Bbar a:
//   abar = Bbar (V^T M H),  Vbar = w M H,  Hbar = w M V  -> nbar through the
//   gradient of the SH polynomial (tangential part / |n|),
//   Lbar_i = sum_x w(x) (V(x) * H(x))_i   (per-lane accumulation over a
//   grid-stride set of receivers, then wave / block sums in a fixed order).

#include "shv_device.h"
#include "shv_launch.h"

namespace shv {

template <int NB>
struct MTab;
#define SHV_MTAB(n)                                                          \
  template <>                                                                \
  struct MTab<n> {                                                           \
    static __device__ __forceinline__ const int* ptr() { return shv_mtab_ptr_##n; }            \
    static __device__ __forceinline__ const unsigned char* ind() { return shv_mtab_idx_##n; }  \
    static __device__ __forceinline__ const float* val() { return shv_mtab_val_##n; }          \
    static __device__ __forceinline__ void vh(const float* v, const float* h, float* acc) {    \
      shv_vh_acc_##n(v, h, acc);                                                               \
    }                                                                                          \
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

// M[j * N + k] = sum_i L_i C_ijk, one thread per (j, k).
template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_build_M(const float* __restrict__ L, float* __restrict__ M) {
  constexpr int N = NB * NB;
  const int jk = blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (jk >= N * N) return;
  const int* ptr = MTab<NB>::ptr();
  const unsigned char* ind = MTab<NB>::ind();
  const float* val = MTab<NB>::val();
  float a = 0.0f;
  for (int e = ptr[jk]; e < ptr[jk + 1]; ++e) a = fmaf(L[ind[e]], val[e], a);
  M[jk] = a;
}

__device__ __forceinline__ constexpr bool h_support(int l) { return l <= 2 || (l % 2) == 0; }

// H_lm = A_l y_lm(n_hat) on the support (0 elsewhere); returns 1/|n|.
template <int NB>
__device__ __forceinline__ float transfer(float nx, float ny, float nz, float (&H)[NB * NB], float& ux, float& uy,
                                          float& uz) {
  const float n2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
  const float inv = fast_rsqrt(n2);
  ux = nx * inv;
  uy = ny * inv;
  uz = nz * inv;
  sh_eval<NB>(ux, uy, uz, H);
#pragma unroll
  for (int l = 0; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) H[idx(l, m)] = h_support(l) ? H[idx(l, m)] * SHV_AHAT[l] : 0.0f;
  }
  return inv;
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_shade_fwd(const float* __restrict__ vis, const float* __restrict__ nrm,
                                                         const float* __restrict__ alb, const float* __restrict__ M,
                                                         int64_t P, float* __restrict__ rad) {
  constexpr int N = NB * NB;
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (p >= P) return;
  float V[N], H[N];
#pragma unroll
  for (int i = 0; i < N; ++i) V[i] = vis[(int64_t)i * P + p];
  float ux, uy, uz;
  transfer<NB>(nrm[p], nrm[P + p], nrm[2 * P + p], H, ux, uy, uz);
  float B = 0.0f;
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    if (!h_support(l)) continue;
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const int k = idx(l, m);
      float t = 0.0f;
#pragma unroll
      for (int j = 0; j < N; ++j) t = fmaf(M[j * N + k], V[j], t);
      B = fmaf(H[k], t, B);
    }
  }
  rad[p] = alb[p] * B;
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_shade_bwd(const float* __restrict__ gB, const float* __restrict__ vis,
                                                         const float* __restrict__ nrm, const float* __restrict__ alb,
                                                         const float* __restrict__ M, int64_t P,
                                                         float* __restrict__ gV, float* __restrict__ gN,
                                                         float* __restrict__ gA, float* __restrict__ Lpart) {
  constexpr int N = NB * NB;
  __shared__ float red[SHV_WAVES_PER_BLOCK][N];
  float Lacc[N];
#pragma unroll
  for (int i = 0; i < N; ++i) Lacc[i] = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * SHV_BLOCK;
  for (int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x; p < P; p += stride) {
    float V[N], H[N];
#pragma unroll
    for (int i = 0; i < N; ++i) V[i] = vis[(int64_t)i * P + p];
    float ux, uy, uz;
    const float inv = transfer<NB>(nrm[p], nrm[P + p], nrm[2 * P + p], H, ux, uy, uz);
    const float a = alb[p];
    const float bb = gB[p];
    const float w = bb * a;
    // t_k = (M V)_k on H's support; s = H . t
    float Hb[N];
    float s = 0.0f;
#pragma unroll
    for (int l = 0; l < NB; ++l) {
#pragma unroll
      for (int m = -l; m <= l; ++m) {
        const int k = idx(l, m);
        if (!h_support(l)) {
          Hb[k] = 0.0f;
          continue;
        }
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < N; ++j) t = fmaf(M[j * N + k], V[j], t);
        s = fmaf(H[k], t, s);
        Hb[k] = w * t * SHV_AHAT[l];  // dLoss/d y_k(n_hat) = Hbar_k A_l
      }
    }
    if (gA) gA[p] = bb * s;
    if (gV) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        float t = 0.0f;
#pragma unroll
        for (int l = 0; l < NB; ++l) {
          if (!h_support(l)) continue;
#pragma unroll
          for (int m = -l; m <= l; ++m) t = fmaf(M[j * N + idx(l, m)], H[idx(l, m)], t);
        }
        gV[(int64_t)j * P + p] = w * t;
      }
    }
    if (gN) {
      float gx, gy, gz;
      sh_grad<NB>(ux, uy, uz, Hb, gx, gy, gz);
      const float sd = fmaf(gx, ux, fmaf(gy, uy, gz * uz));
      gN[p] = (gx - sd * ux) * inv;
      gN[P + p] = (gy - sd * uy) * inv;
      gN[2 * P + p] = (gz - sd * uz) * inv;
    }
    if (Lpart) {
#pragma unroll
      for (int k = 0; k < N; ++k) H[k] *= w;
      MTab<NB>::vh(V, H, Lacc);
    }
  }
  if (Lpart) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const float v = wave_sum(Lacc[i]);
      if (lane == 0) red[wave][i] = v;
    }
    __syncthreads();
    if (threadIdx.x < N) {
      float a = red[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < SHV_WAVES_PER_BLOCK; ++w) a += red[w][threadIdx.x];
      Lpart[(int64_t)blockIdx.x * N + threadIdx.x] = a;
    }
  }
}

int shade_blocks(int64_t P) {
  const int64_t b = (P + SHV_BLOCK - 1) / SHV_BLOCK;
  return (int)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

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

hipError_t launch_build_M(int nb, const float* light, float* M, hipStream_t st) {
  const int NN = nb * nb * nb * nb;
  const unsigned grid = (unsigned)((NN + SHV_BLOCK - 1) / SHV_BLOCK);
  SHV_DISPATCH(nb, k_build_M, grid, SHV_BLOCK, 0, st>>>(light, M))
  return hipGetLastError();
}

hipError_t launch_shade_fwd(int nb, const float* vis, const float* nrm, const float* alb, const float* M, int64_t P,
                            float* rad, hipStream_t st) {
  const unsigned grid = (unsigned)point_blocks(P);
  SHV_DISPATCH(nb, k_shade_fwd, grid, SHV_BLOCK, 0, st>>>(vis, nrm, alb, M, P, rad))
  return hipGetLastError();
}

hipError_t launch_shade_bwd(int nb, const float* gB, const float* vis, const float* nrm, const float* alb,
                            const float* M, int64_t P, float* gV, float* gN, float* gA, float* Lpart,
                            hipStream_t st) {
  const unsigned grid = (unsigned)shade_blocks(P);
  SHV_DISPATCH(nb, k_shade_bwd, grid, SHV_BLOCK, 0, st>>>(gB, vis, nrm, alb, M, P, gV, gN, gA, Lpart))
  return hipGetLastError();
}

}  // namespace shv
