// Internal launcher declarations (host side).  Every launcher enqueues one
// kernel on `st` and returns the launch status; none allocates or syncs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shv {

// Split of the sphere set into chunks for the pair kernels ("split-S"): the
// log-visibility is a sum over spheres (Sec. 3.3.2), so partial sums from
// sphere chunks add up.  A pure function of (P, S): the same scene is always
// reduced in the same order.
struct Split {
  int nchunks;
  int chunk;
};
Split choose_split(int64_t P, int64_t S);

int64_t point_blocks(int64_t P);  // ceil(P / 256)
int shade_blocks(int64_t P);      // grid of the shading adjoint

hipError_t launch_pair_fwd(int nb, const float* pts, int64_t P, const float* sph, int S, Split sp,
                           float* Fpart, hipStream_t st);
hipError_t launch_exp_fwd(int nb, const float* Fpart, int nchunks, int64_t P, float eps, int k,
                          float* vis, float* saved, hipStream_t st);
hipError_t launch_build_M(int nb, const float* light, float* M, hipStream_t st);
hipError_t launch_shade_fwd(int nb, const float* vis, const float* nrm, const float* alb, const float* M,
                            int64_t P, float* rad, hipStream_t st);
hipError_t launch_shade_bwd(int nb, const float* gB, const float* vis, const float* nrm, const float* alb,
                            const float* M, int64_t P, float* gV, float* gN, float* gA, float* Lpart,
                            hipStream_t st);
hipError_t launch_reduce_rows(const float* part, int rows, int cols, float* out, hipStream_t st);
hipError_t launch_exp_bwd(int nb, const float* gV, const float* vis, const float* saved, int64_t P,
                          float eps, int k, float* W, hipStream_t st);
hipError_t launch_pair_bwd(int nb, const float* W, const float* pts, int64_t P, const float* sph, int S,
                           Split sp, float* gp_part, float* gs_part, hipStream_t st);
// Zero n floats with a plain kernel (safe inside captured graphs).
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t st);
hipError_t launch_sum_chunks(const float* part, int nchunks, int64_t len, float* out, hipStream_t st);

}  // namespace shv
