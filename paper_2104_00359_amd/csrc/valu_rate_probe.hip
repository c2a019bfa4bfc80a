// FP32 VALU issue-rate probe (a measurement tool built beside the library,
// not part of it): eight independent chains per thread of one FP32 operation
// with operands of a given kind, 8,192 blocks of 256 threads, each launch
// timed with HIP events; prints the best of ten launches (after two) in lane
// operations per second.  Kinds: FMA with two scalar-register operands, FMA
// with register operands, FMA with a literal, multiply, and FMA whose second
// factor is another chain.
#include <hip/hip_runtime.h>

#include <cstdio>

template <int OP>
__global__ __launch_bounds__(256) void k_rate(float* out, float b, float c, int iters) {
  float a[8];
  const float bv = b + threadIdx.x * 1e-9f, cv = c + threadIdx.x * 1e-9f;  // per-lane values
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = threadIdx.x * 1e-3f + i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if (OP == 0) a[i] = fmaf(a[i], b, c);
      if (OP == 1) a[i] = fmaf(a[i], bv, cv);
      if (OP == 2) a[i] = fmaf(a[i], bv, 0.3711f);
      if (OP == 3) a[i] = a[i] * bv;
      if (OP == 4) a[i] = fmaf(a[i], a[(i + 1) & 7], cv);
    }
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += a[i];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
static int run(float* out, const char* name) {
  const int blocks = 256 * 32, iters = 16384;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
  float best = 1e30f;
  for (int rep = 0; rep < 12; ++rep) {
    if (hipEventRecord(e0) != hipSuccess) return 1;
    k_rate<OP><<<blocks, 256>>>(out, 0.999f, 1e-4f, iters);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return 1;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 1;
    if (rep >= 2 && ms < best) best = ms;
  }
  const double ops = 8.0 * iters * (double)blocks * 256;
  std::printf("%-24s %.3f ms  %.1f T lane-ops/s  (%.1f TFLOP/s if each were an FMA)\n", name, best, ops / best / 1e9,
              2.0 * ops / best / 1e9);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return 0;
}

int main() {
  float* out = nullptr;
  if (hipMalloc(&out, (size_t)256 * 32 * 256 * 4) != hipSuccess) return 1;
  int rc = run<0>(out, "fma(a, sgpr, sgpr)");
  rc |= run<1>(out, "fma(a, vgpr, vgpr)");
  rc |= run<2>(out, "fma(a, vgpr, literal)");
  rc |= run<3>(out, "mul(a, vgpr)");
  rc |= run<4>(out, "fma(a, a_next, vgpr)");
  (void)hipFree(out);
  return rc;
}
