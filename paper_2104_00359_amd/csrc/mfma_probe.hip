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
// 3. One wave alone.  A single wave runs 1, 2, 4 or 8 interleaved dependent
//    chains of the same instructions; the shader clock read before and after
//    gives the cycles per instruction (the best of five launches; the loop
//    is unrolled eight times, so its compare and branch come once per 8 C
//    instructions): the dependent latency with one chain, the one-wave issue
//    interval with eight.
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

template <int C, int OP>
__global__ __launch_bounds__(64) void k_one_wave(float* out, long long* cyc, float a0, float b0, int iters) {
  const float a = a0 + threadIdx.x * 1e-9f, b = b0 - threadIdx.x * 1e-9f;
  f32x4 acc[C];
  float f[C];
#pragma unroll
  for (int i = 0; i < C; ++i) {
    acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    f[i] = threadIdx.x * 1e-3f + i;
  }
  const long long t0 = clock64(), w0 = wall_clock64();
  for (int it = 0; it < iters; it += 8) {  // iters is a multiple of 8
#pragma unroll
    for (int u = 0; u < 8; ++u) {
#pragma unroll
      for (int i = 0; i < C; ++i) {
        if (OP == 0) acc[i] = __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, acc[i], 0, 0, 0);
        if (OP == 1) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
        if (OP == 2) f[i] = fmaf(f[i], a, b);
      }
    }
  }
  const long long t1 = clock64(), w1 = wall_clock64();
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < C; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3] + f[i];
  out[threadIdx.x] = s;  // keeps the chains live (out holds one float per lane)
  if (threadIdx.x == 0) {
    cyc[0] = t1 - t0;
    cyc[1] = w1 - w0;
  }
}

// Shader-clock cycles per instruction; *ghz gets the shader clock's rate
// against the constant-rate wall clock over the same launch.
template <int C, int OP>
static double one_wave_cycles(float* out, long long* cyc, double* ghz) {
  const int iters = 4096;
  long long best = -1, wall = 0;
  for (int rep = 0; rep < 5; ++rep) {
    k_one_wave<C, OP><<<1, 64>>>(out, cyc, 1.0001f, 0.9999f, iters);
    long long h[2] = {0, 0};
    if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(h, cyc, 16, hipMemcpyDeviceToHost) != hipSuccess) return -1;
    if (best < 0 || h[0] < best) {
      best = h[0];
      wall = h[1];
    }
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0) == hipSuccess && khz > 0 && wall > 0)
    *ghz = (double)best / ((double)wall / (khz * 1e3) * 1e9);
  return (double)best / ((double)iters * C);
}

template <int OP>
static void one_wave_line(float* out, long long* cyc, const char* name) {
  double ghz = 0;
  const double c1 = one_wave_cycles<1, OP>(out, cyc, &ghz), c2 = one_wave_cycles<2, OP>(out, cyc, &ghz);
  const double c4 = one_wave_cycles<4, OP>(out, cyc, &ghz), c8 = one_wave_cycles<8, OP>(out, cyc, &ghz);
  printf("one_wave_%s_cycles_per_instruction chains 1 %.1f  2 %.1f  4 %.1f  8 %.1f  (shader clock %.2f GHz)\n", name,
         c1, c2, c4, c8, ghz);
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
  long long* dcyc = nullptr;
  float* dwave = nullptr;  // one float per lane of the single wave
  if (hipMalloc(&dcyc, 2 * sizeof(long long)) != hipSuccess || hipMalloc(&dwave, 64 * sizeof(float)) != hipSuccess) {
    printf("allocation failed\n");
    return 1;
  }
  one_wave_line<0>(dwave, dcyc, "mfma_4x4x1");
  one_wave_line<1>(dwave, dcyc, "mfma_16x16x4");
  one_wave_line<2>(dwave, dcyc, "valu_fma");
  return 0;
}
