// SH exponential V = exp*(F) and its adjoint, one receiver per lane.
//
// The paper replaces the product of blocker vectors (Eq. 12) by the
// exponential of the summed log-blockers and adopts Ren et al.'s scaling,
// squaring and optimal linear approximation.  With N = n^2 coefficients:
//   c   = F_0 / sqrt(4 pi)                 (the constant value of the DC part)
//   G   = (F with F_0 := 0) * 2^-k
//   E_0 = a (sqrt(4 pi) e_0 + G),  a = exp(|G|^2 / (8 pi))
//         (least-squares line a + b g through exp(g) when g's values over the
//          sphere are Gaussian with variance |G|^2 / (4 pi); it gives a = b)
//   E_{j+1} = E_j * E_j  (k truncated triple-product squarings, Eqs. 6-7)
//   V   = exp(c) E_k
// The squaring is straight-line generated code (coefficients are literals).
// Saved for the adjoint, coefficient-major: row 0 = c, rows 1 + j*N + i = E_j[i].
//
// The first kernel also sums the sphere-chunk partials of F' in a fixed order
// and applies F_lm = eps * LAMBDA[l][|m|] * F'_lm.  The adjoint writes
// W = eps * LAMBDA * dLoss/dF, the weights the pair adjoint consumes.

#include "shv_device.h"
#include "shv_launch.h"

namespace shv {

template <int NB>
__device__ __forceinline__ void square(const float* e, float* o);
template <int NB>
__device__ __forceinline__ void square_adj(const float* ob, const float* e, float* eb);

#define SHV_SQ(n)                                                                                    \
  template <>                                                                                        \
  __device__ __forceinline__ void square<n>(const float* e, float* o) { shv_square_##n(e, o); }      \
  template <>                                                                                        \
  __device__ __forceinline__ void square_adj<n>(const float* ob, const float* e, float* eb) {        \
    shv_square_adj_##n(ob, e, eb);                                                                   \
  }
SHV_SQ(1)
SHV_SQ(2)
SHV_SQ(3)
SHV_SQ(4)
SHV_SQ(5)
SHV_SQ(6)
SHV_SQ(7)
SHV_SQ(8)
#undef SHV_SQ

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_fwd(const float* __restrict__ Fpart, int nchunks, int64_t P,
                                                       float eps, int k, float* __restrict__ vis,
                                                       float* __restrict__ saved) {
  constexpr int N = NB * NB;
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (p >= P) return;
  float E[N], O[N];
#pragma unroll
  for (int i = 0; i < N; ++i) E[i] = Fpart[(int64_t)i * P + p];
  for (int c = 1; c < nchunks; ++c) {
    const float* src = Fpart + (int64_t)c * N * P + p;
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] += src[(int64_t)i * P];
  }
  // F = eps * LAMBDA * F'
#pragma unroll
  for (int l = 0; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) E[idx(l, m)] *= eps * SHV_LAMBDA[l][m < 0 ? -m : m];
  }
  const float c = E[0] * SHV_INV_SQRT_4PI;
  const float scale = __builtin_ldexpf(1.0f, -k);
  float sig = 0.0f;
#pragma unroll
  for (int i = 1; i < N; ++i) {
    E[i] *= scale;
    sig = fmaf(E[i], E[i], sig);
  }
  const float a = expf(sig * SHV_INV_8PI);
  E[0] = a * SHV_SQRT_4PI;
#pragma unroll
  for (int i = 1; i < N; ++i) E[i] *= a;
  if (saved) saved[p] = c;
  for (int j = 0; j < k; ++j) {
    if (saved) {
      float* dst = saved + (int64_t)(1 + j * N) * P + p;
#pragma unroll
      for (int i = 0; i < N; ++i) dst[(int64_t)i * P] = E[i];
    }
    square<NB>(E, O);
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = O[i];
  }
  const float ec = expf(c);
#pragma unroll
  for (int i = 0; i < N; ++i) vis[(int64_t)i * P + p] = ec * E[i];
}

template <int NB>
__global__ __launch_bounds__(SHV_BLOCK) void k_exp_bwd(const float* __restrict__ gV, const float* __restrict__ vis,
                                                       const float* __restrict__ saved, int64_t P, float eps, int k,
                                                       float* __restrict__ Wout) {
  constexpr int N = NB * NB;
  const int64_t p = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (p >= P) return;
  const float c = saved[p];
  const float ec = expf(c);
  float Eb[N], E[N], T[N];
  float cbar = 0.0f;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const float vb = gV[(int64_t)i * P + p];
    const float v = vis[(int64_t)i * P + p];
    cbar = fmaf(vb, v, cbar);  // d/dc of exp(c) E_k . Vbar = V . Vbar
    Eb[i] = ec * vb;
    if (k == 0) E[i] = v / ec;  // E_0 itself when there is no squaring
  }
  for (int j = k - 1; j >= 0; --j) {
    const float* src = saved + (int64_t)(1 + j * N) * P + p;
#pragma unroll
    for (int i = 0; i < N; ++i) E[i] = src[(int64_t)i * P];
    square_adj<NB>(Eb, E, T);  // Ebar_j = 2 (Ebar_{j+1} * E_j)
#pragma unroll
    for (int i = 0; i < N; ++i) Eb[i] = T[i];
  }
  // E holds E_0 = a (sqrt(4 pi) e_0 + G).  Adjoint of the linear approximation:
  // Gbar_i = a (Ebar_i + G_i / (4 pi) (sqrt(4 pi) Ebar_0 + sum_j Ebar_j G_j)).
  const float a = E[0] * SHV_INV_SQRT_4PI;
  const float inva = 1.0f / a;
  float dot = SHV_SQRT_4PI * Eb[0];
#pragma unroll
  for (int i = 1; i < N; ++i) {
    E[i] *= inva;  // G_i
    dot = fmaf(Eb[i], E[i], dot);
  }
  const float scale = __builtin_ldexpf(1.0f, -k);
  const float kdot = dot * SHV_INV_4PI;
  // W = eps * LAMBDA * Fbar, Fbar_i = 2^-k Gbar_i (i > 0), Fbar_0 = cbar / sqrt(4 pi)
  Wout[p] = eps * SHV_LAMBDA[0][0] * cbar * SHV_INV_SQRT_4PI;
#pragma unroll
  for (int l = 1; l < NB; ++l) {
#pragma unroll
    for (int m = -l; m <= l; ++m) {
      const int i = idx(l, m);
      const float gb = a * fmaf(E[i], kdot, Eb[i]);
      Wout[(int64_t)i * P + p] = eps * SHV_LAMBDA[l][m < 0 ? -m : m] * scale * gb;
    }
  }
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

hipError_t launch_exp_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k, float* vis,
                          float* saved, hipStream_t st) {
  const unsigned grid = (unsigned)point_blocks(P);
  SHV_DISPATCH(nb, k_exp_fwd, grid, SHV_BLOCK, 0, st>>>(Fpart, nchunks, P, eps, k, vis, saved))
  return hipGetLastError();
}

hipError_t launch_exp_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P, float eps,
                          int k, float* W, hipStream_t st) {
  const unsigned grid = (unsigned)point_blocks(P);
  SHV_DISPATCH(nb, k_exp_bwd, grid, SHV_BLOCK, 0, st>>>(gV, vis, saved, P, eps, k, W))
  return hipGetLastError();
}

}  // namespace shv
