// FP32 MFMA probe (a measurement tool built beside the library, not part of
// it), two parts:
//
// 1. Rounding and lane layout.  One wave runs 64-step chains of
//    v_mfma_f32_4x4x1f32 and of v_mfma_f32_16x16x4f32 on seeded operands
//    (magnitudes over 2^-6 .. 2^6), and beside them the fmaf chains that add
//    the same products in the same order under the lane layout the shading
//    code assumes:
//      4x4x1 (16 blocks): accumulator i of lane 4b + c gains
//        A(lane 4b + i) * B(lane 4b + c);
//      16x16x4: lane l supplies A[row l % 16][k l / 16] and B[k l / 16][col
//        l % 16]; accumulator i of lane l is D[4 (l / 16) + i][l % 16], and
//        the four k of one step are added one after the other.
//    It prints how many of the 256 outputs of each chain are bit-identical.
// 2. Issue rate.  8,192 blocks of 256 threads each run independent chains of
//    one instruction (4x4x1 MFMA, 16x16x4 MFMA, or a plain FMA for
//    comparison); the best of ten timed launches gives FP32 TFLOP/s
//    (2 flops per multiply-add).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int K = 64;

__global__ __launch_bounds__(64) void k_layout(const float* A, const float* B, const float* C0, float* D4,
                                                float* V4, float* D16, float* V16) {
  const int l = threadIdx.x;
  f32x4 d = {C0[l * 4 + 0], C0[l * 4 + 1], C0[l * 4 + 2], C0[l * 4 + 3]};
  f32x4 e = d;
  for (int k = 0; k < K; ++k) {
    d = __builtin_amdgcn_mfma_f32_4x4x1f32(A[k * 64 + l], B[k * 64 + l], d, 0, 0, 0);
    e = __builtin_amdgcn_mfma_f32_16x16x4f32(A[k * 64 + l], B[k * 64 + l], e, 0, 0, 0);
  }
  const int b = l / 4, c = l % 4, row0 = 4 * (l / 16), col = l % 16;
  for (int i = 0; i < 4; ++i) {
    D4[l * 4 + i] = d[i];
    D16[l * 4 + i] = e[i];
    float v = C0[l * 4 + i], w = C0[l * 4 + i];
    for (int k = 0; k < K; ++k) {
      v = fmaf(A[k * 64 + 4 * b + i], B[k * 64 + 4 * b + c], v);
      for (int kk = 0; kk < 4; ++kk) w = fmaf(A[k * 64 + kk * 16 + row0 + i], B[k * 64 + kk * 16 + col], w);
    }
    V4[l * 4 + i] = v;
    V16[l * 4 + i] = w;
  }
}

template <int OP>
__global__ __launch_bounds__(256) void k_rate(float* out, float a0, float b0, int iters) {
  const float a = a0 + threadIdx.x * 1e-9f, b = b0 - threadIdx.x * 1e-9f;
  f32x4 acc[8];
  float f[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    f[i] = threadIdx.x * 1e-3f + i;
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (OP == 0) acc[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[i], 0, 0, 0);
      if (OP == 1) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
      if (OP == 2) f[i] = fmaf(f[i], a, b);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3] + f[i];
  if (s == 12345.678f) out[0] = s;  // keeps the chains live
}

template <int OP>
static double rate(float* out, int iters, double macs_per_lane_op) {
  const int blocks = 8192;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1;
  double best = 0;
  for (int rep = 0; rep < 12; ++rep) {
    if (hipEventRecord(e0) != hipSuccess) return -1;
    k_rate<OP><<<blocks, 256>>>(out, 1.0001f, 0.9999f, iters);
    if (hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1;
    const double flops = 2.0 * macs_per_lane_op * 8.0 * iters * blocks * 256.0;
    if (rep >= 2) best = std::max(best, flops / (ms * 1e-3) / 1e12);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

int main() {
  std::mt19937 rng(7);
  std::normal_distribution<float> nd(0.f, 1.f);
  std::uniform_int_distribution<int> ex(-6, 6);
  std::vector<float> A(K * 64), B(K * 64), C0(256), D4(256), V4(256), D16(256), V16(256);
  for (auto& x : A) x = std::ldexp(nd(rng), ex(rng));
  for (auto& x : B) x = std::ldexp(nd(rng), ex(rng));
  for (auto& x : C0) x = nd(rng);
  float *dA, *dB, *dC, *dD4, *dV4, *dD16, *dV16, *dout;
  if (hipMalloc(&dA, A.size() * 4) != hipSuccess || hipMalloc(&dB, B.size() * 4) != hipSuccess ||
      hipMalloc(&dC, 1024) != hipSuccess || hipMalloc(&dD4, 1024) != hipSuccess || hipMalloc(&dV4, 1024) != hipSuccess ||
      hipMalloc(&dD16, 1024) != hipSuccess || hipMalloc(&dV16, 1024) != hipSuccess || hipMalloc(&dout, 64) != hipSuccess) {
    printf("allocation failed\n");
    return 1;
  }
  if (hipMemcpy(dA, A.data(), A.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dB, B.data(), B.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dC, C0.data(), 1024, hipMemcpyHostToDevice) != hipSuccess) {
    printf("copy failed\n");
    return 1;
  }
  k_layout<<<1, 64>>>(dA, dB, dC, dD4, dV4, dD16, dV16);
  if (hipDeviceSynchronize() != hipSuccess) {
    printf("launch failed\n");
    return 1;
  }
  if (hipMemcpy(D4.data(), dD4, 1024, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(V4.data(), dV4, 1024, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(D16.data(), dD16, 1024, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(V16.data(), dV16, 1024, hipMemcpyDeviceToHost) != hipSuccess) {
    printf("copy back failed\n");
    return 1;
  }
  int same4 = 0, same16 = 0;
  for (int t = 0; t < 256; ++t) {
    same4 += std::memcmp(&D4[t], &V4[t], 4) == 0;
    same16 += std::memcmp(&D16[t], &V16[t], 4) == 0;
  }
  printf("mfma_4x4x1_bitwise_equal_to_fmaf %d of 256\n", same4);
  printf("mfma_16x16x4_bitwise_equal_to_fmaf %d of 256\n", same16);
  const int iters = 2048;
  printf("mfma_4x4x1_tflops %.1f\n", rate<0>(dout, iters, 4.0));     // 4 multiply-adds per lane per instruction
  printf("mfma_16x16x4_tflops %.1f\n", rate<1>(dout, iters, 16.0));  // 16 per lane per instruction
  printf("valu_fma_tflops %.1f\n", rate<2>(dout, iters, 1.0));
  return 0;
}
