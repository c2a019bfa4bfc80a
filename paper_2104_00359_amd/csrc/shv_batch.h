// Device-side work table of the batched (multi-scene) render path.
//
// The host packs a BatchHeader, one BatchScene record per scene and two index
// arrays that list the scenes grouped by band count (pair phases) and by
// exponential layout and band count (exponential phases).  Every phase of a
// batched forward or backward runs as one launch per group present, whose
// blocks cover that group's item space (item = one block's worth of work of
// one scene, exactly a block of the single-scene kernel; the scene is found by
// binary search over the group's offsets, and blocks past the end exit); the
// closing reductions run as one launch over all scenes.  Scene
// records carry the split decisions of the single-scene entry points, so every
// scene's results are bit-identical to a single-scene call.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shvis.h"

namespace shv {

struct BatchScene {
  // inputs
  const float* points;         // [3][P]
  const float* normals;        // [3][P]
  const float* albedo;         // [P]
  const float* spheres;        // [S][4]
  const float* light;          // [N]
  const float* grad_radiance;  // [P] (backward)
  // outputs
  float* vis;                  // [N][P]
  float* radiance;             // [P]
  float* saved;                // render saved state (M(L) at its end)
  float* grad_points;          // [3][P] or NULL
  float* grad_normals;         // [3][P] or NULL
  float* grad_albedo;          // [P] or NULL
  float* grad_spheres;         // [S][4] or NULL (NULL when S = 0)
  float* grad_light;           // [N] or NULL
  // workspace regions
  float* Fpart;
  float* M;
  float* W;
  float* gp;
  float* gs;
  float* lp;
  int64_t P, S;
  int32_t nb, k;
  float eps;
  uint32_t flags;
  int32_t nchunks_f, chunk_f;  // sphere split of the pair forward
  int32_t nchunks_b, chunk_b;  // sphere split of the pair adjoint
  int32_t four_waves;          // exponential layout
  int32_t fin_pts, fin_cols_s, fin_cols_l;  // closing reductions: point blocks, sphere / lighting columns
  int64_t pair_tiles;          // ceil(P / 64): receiver tiles of the whole scene
  int64_t exp_blocks;          // exponential blocks of the whole scene
  int64_t tile0, range_tiles;  // receiver tiles of this call's range
  int64_t exp_block0;          // first exponential block of the range
  int64_t n_pair_f, n_pair_b, n_exp, n_fin;  // items per phase
  int64_t off_pair_f;          // first pair-forward item within the band count's item space
  int64_t off_pair_b;          // first pair-adjoint item within the band count's item space
  int64_t off_exp;             // first exponential item within the (layout, band count) item space
  int64_t off_fin;             // first item of the closing reductions (all scenes)
};

struct BatchHeader {
  int32_t n_scenes;
  int64_t total_fin;
  int64_t total_pair_f[SHV_MAX_BANDS_API + 1];   // pair-forward items per band count
  int64_t total_pair_b[SHV_MAX_BANDS_API + 1];   // pair-adjoint items per band count
  int32_t grp_begin[SHV_MAX_BANDS_API + 1];      // slice of `order` per band count
  int32_t grp_count[SHV_MAX_BANDS_API + 1];
  int64_t total_exp[2][SHV_MAX_BANDS_API + 1];   // exponential items per (layout, band count)
  int32_t egrp_begin[2][SHV_MAX_BANDS_API + 1];  // slice of `eorder` per (layout, band count)
  int32_t egrp_count[2][SHV_MAX_BANDS_API + 1];
};


// Layout: header, n scene records, `order` (scene ids grouped by band count),
// `eorder` (scene ids grouped by exponential layout, then band count).
inline size_t batch_table_bytes(int32_t n) {
  return sizeof(BatchHeader) + (size_t)n * sizeof(BatchScene) + 2 * (size_t)n * sizeof(int32_t);
}

// Read-only view of a device table.
struct BatchView {
  const BatchHeader* h;
  const BatchScene* sc;
  const int32_t* order;
  const int32_t* eorder;
  __device__ explicit BatchView(const char* t)
      : h(reinterpret_cast<const BatchHeader*>(t)),
        sc(reinterpret_cast<const BatchScene*>(t + sizeof(BatchHeader))),
        order(reinterpret_cast<const int32_t*>(t + sizeof(BatchHeader) + h->n_scenes * sizeof(BatchScene))),
        eorder(order + h->n_scenes) {}

  // Scene of a group owning `item`: the last one whose offset is <= item.
  template <class Off>
  __device__ const BatchScene& find(const int32_t* g, int count, int64_t item, Off off) const {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off(sc[g[mid]]) <= item) lo = mid;
      else hi = mid - 1;
    }
    return sc[g[lo]];
  }

  __device__ const BatchScene& scene_of_pair_fwd(int nb, int64_t item) const {
    return find(order + h->grp_begin[nb], h->grp_count[nb], item, [](const BatchScene& s) { return s.off_pair_f; });
  }

  __device__ const BatchScene& scene_of_pair_bwd(int nb, int64_t item) const {
    return find(order + h->grp_begin[nb], h->grp_count[nb], item, [](const BatchScene& s) { return s.off_pair_b; });
  }

  __device__ const BatchScene& scene_of_exp(int four, int nb, int64_t item) const {
    return find(eorder + h->egrp_begin[four][nb], h->egrp_count[four][nb], item,
                [](const BatchScene& s) { return s.off_exp; });
  }

  __device__ const BatchScene& scene_of_fin(int64_t item) const {
    int lo = 0, hi = h->n_scenes - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sc[mid].off_fin <= item) lo = mid;
      else hi = mid - 1;
    }
    return sc[lo];
  }
};

// Pointers read from the table have no known address space, so the compiler
// would address them with flat instructions and 64-bit per-lane addresses.
// Every buffer of a scene is global device memory: read each pointer field
// from the table as a pointer to global memory.
template <class T>
__device__ __forceinline__ T* load_global_ptr(T* const& field) {
  const void* addr = &field;
  return (T*)*static_cast<T __attribute__((address_space(1)))* const*>(addr);
}

// Copy of a scene record (a reference into the table) with global pointers.
__device__ __forceinline__ BatchScene in_global(const BatchScene& s) {
  BatchScene r = s;
  r.points = load_global_ptr(s.points);
  r.normals = load_global_ptr(s.normals);
  r.albedo = load_global_ptr(s.albedo);
  r.spheres = load_global_ptr(s.spheres);
  r.light = load_global_ptr(s.light);
  r.grad_radiance = load_global_ptr(s.grad_radiance);
  r.vis = load_global_ptr(s.vis);
  r.radiance = load_global_ptr(s.radiance);
  r.saved = load_global_ptr(s.saved);
  r.grad_points = load_global_ptr(s.grad_points);
  r.grad_normals = load_global_ptr(s.grad_normals);
  r.grad_albedo = load_global_ptr(s.grad_albedo);
  r.grad_spheres = load_global_ptr(s.grad_spheres);
  r.grad_light = load_global_ptr(s.grad_light);
  r.Fpart = load_global_ptr(s.Fpart);
  r.M = load_global_ptr(s.M);
  r.W = load_global_ptr(s.W);
  r.gp = load_global_ptr(s.gp);
  r.gs = load_global_ptr(s.gs);
  r.lp = load_global_ptr(s.lp);
  return r;
}

}  // namespace shv
