// Every kernel that depends on the number of SH bands, instantiated for one
// band count (SHV_NB) and one part of the library (SHV_PART), both set on the
// compiler command line: many translation units of moderate size that build
// in parallel, instead of one very large one.

#include "shv_exp_impl.h"
#include "shv_pair_impl.h"
#include "shv_prod_impl.h"
#include "shv_quad_impl.h"
#include "shv_shade_impl.h"
#include "shv_taylor_impl.h"

#if !defined(SHV_NB) || !defined(SHV_PART)
#error "compile with -DSHV_NB=<1..8> -DSHV_PART=<0..8>"
#endif

namespace shv {

#if SHV_PART == 0
template hipError_t pair_fwd_nb<SHV_NB>(const float*, int64_t, const float*, int, Split, float*, const float*, float*,
                                        hipStream_t);
template hipError_t pair_bwd_nb<SHV_NB>(const float*, const float*, int64_t, const float*, int, Split, float*, float*,
                                        hipStream_t);
template hipError_t build_M_nb<SHV_NB>(const float*, float*, int, hipStream_t);
template hipError_t shade_ch_fwd_nb<SHV_NB>(const float*, const float*, const float*, const float*, int, int64_t,
                                            float*, hipStream_t);
template hipError_t shade_ch_bwd_nb<SHV_NB>(const float*, const float*, const float*, const float*, const float*, int,
                                            int64_t, float*, float*, float*, float*, hipStream_t);
template hipError_t envmap_rows_nb<SHV_NB>(const float*, int, int64_t, int64_t, float*, hipStream_t);
template hipError_t batch_pair_fwd_nb<SHV_NB>(const void*, int64_t, hipStream_t);
template hipError_t batch_pair_bwd_nb<SHV_NB>(const void*, int64_t, hipStream_t);
#elif SHV_PART == 1
template hipError_t exp_fwd_nb<SHV_NB, false>(const float*, int, int64_t, float, int, float*, float*, const float*,
                                              const float*, const float*, float*, uint32_t, hipStream_t);
template hipError_t exp_fwd_nb<SHV_NB, true>(const float*, int, int64_t, float, int, float*, float*, const float*,
                                             const float*, const float*, float*, uint32_t, hipStream_t);
#elif SHV_PART == 2
template hipError_t exp_bwd_nb<SHV_NB, false>(const float*, const float*, const float*, int64_t, float, int, float*,
                                              const float*, const float*, const float*, float*, float*, float*,
                                              uint32_t, hipStream_t);
#elif SHV_PART == 3
template hipError_t exp_bwd_nb<SHV_NB, true>(const float*, const float*, const float*, int64_t, float, int, float*,
                                             const float*, const float*, const float*, float*, float*, float*,
                                             uint32_t, hipStream_t);
#elif SHV_PART == 4
template hipError_t batch_exp_fwd_nb<SHV_NB>(const void*, bool, int64_t, hipStream_t);
#elif SHV_PART == 5
template hipError_t batch_exp_bwd_nb<SHV_NB>(const void*, bool, int64_t, hipStream_t);
#elif SHV_PART == 6
template hipError_t exp_quad_fwd_nb<SHV_NB>(const float*, int, int64_t, float, float*, float*, float*, float*,
                                            hipStream_t);
template hipError_t exp_quad_bwd_nb<SHV_NB>(const float*, const float*, const float*, int64_t, float, float*, float*,
                                            float*, hipStream_t);
#elif SHV_PART == 7
template hipError_t prod_fwd_nb<SHV_NB>(const float*, int64_t, const float*, int, float, float*, float*, hipStream_t);
template hipError_t prod_bwd_nb<SHV_NB>(const float*, const float*, const float*, int64_t, const float*, int, float,
                                        float*, float*, hipStream_t);
#elif SHV_PART == 8
template hipError_t exp_taylor_fwd_nb<SHV_NB>(const float*, int, int64_t, float, int, int, float*, float*,
                                              hipStream_t);
template hipError_t exp_taylor_bwd_nb<SHV_NB>(const float*, const float*, const float*, int64_t, float, int, int,
                                              float*, hipStream_t);
#endif

}  // namespace shv
