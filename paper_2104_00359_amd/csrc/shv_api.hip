// C ABI: validation, workspace carving, launch sequencing and per-launch timing.
// Declarations and the contract of every entry point are in include/shvis.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "shvis.h"
#include "shv_batch.h"
#include "shv_config.h"
#include "shv_launch.h"

namespace {

thread_local std::string g_last_error;

shv_status set_error(shv_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

std::mutex g_init_mu;
bool g_init[64] = {false};

}  // namespace

// Scratch of sh_render_forward_noalloc: a static device array, one copy per
// device.  Host code never passes its name to a kernel (on the host it is a
// stand-in, not a device address): shv_init looks up each device's address
// with hipGetSymbolAddress and keeps it in g_scratch.
static __device__ __align__(256) unsigned char scratch[SHV_NOALLOC_SCRATCH_BYTES];

namespace {

void* g_scratch[64] = {nullptr};   // device address of `scratch`, per device (under g_init_mu)

shv_status check_device() {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(SHV_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (dev < 0 || dev >= 64 || !g_init[dev])
    return set_error(SHV_ERR_NOT_INITIALIZED, "shv_init() has not been called for device %d", dev);
  return SHV_OK;
}

// ------------------------------------------------------------------ profiling

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;      // event pool
int64_t g_prof_used = 0;          // records filled
std::map<std::string, int64_t> g_prof_untimed;

// Set while a graph is being captured on this thread: event records would
// become graph nodes, so launches are not timed then.
thread_local bool g_capturing = false;

struct ProfScope {
  ProfRec* rec = nullptr;
  hipStream_t st;
  ProfScope(const char* name, hipStream_t s) : st(s) {
    if (g_capturing) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on) return;
    if (g_prof_used < (int64_t)g_prof.size()) {
      rec = &g_prof[g_prof_used++];
      rec->name = name;
      (void)hipEventRecord(rec->a, st);
    } else {
      g_prof_untimed[name] += 1;
    }
  }
  ~ProfScope() {
    if (rec) (void)hipEventRecord(rec->b, st);
  }
};

template <class F>
shv_status launch(const char* name, hipStream_t st, F&& f) {
  hipError_t e;
  {
    ProfScope ps(name, st);
    e = f();
  }
  if (e != hipSuccess) return set_error(SHV_ERR_HIP, "%s launch failed: %s", name, hipGetErrorString(e));
  return SHV_OK;
}

// ------------------------------------------------------------------ validation

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

shv_status check_params(const shv_params* prm) {
  if (!prm) return set_error(SHV_ERR_INVALID_ARG, "params is NULL");
  if (prm->n_bands < 1 || prm->n_bands > SHV_MAX_BANDS_API)
    return set_error(SHV_ERR_UNSUPPORTED, "n_bands=%d outside [1, %d]", prm->n_bands, SHV_MAX_BANDS_API);
  if (prm->n_squarings < 0 || prm->n_squarings > SHV_MAX_SQUARINGS)
    return set_error(SHV_ERR_UNSUPPORTED, "n_squarings=%d outside [0, %d]", prm->n_squarings, SHV_MAX_SQUARINGS);
  if (!(prm->eps == prm->eps) || prm->eps < 0.0f)
    return set_error(SHV_ERR_INVALID_ARG, "eps must be a non-negative number");
  const uint32_t layouts = SHV_FLAG_EXP_ONE_WAVE | SHV_FLAG_EXP_FOUR_WAVES;
  const uint32_t known = layouts | SHV_FLAG_EXP_QUADRATURE | SHV_FLAG_EXP_PRODUCT | SHV_FLAG_EXP_TAYLOR |
                         SHV_FLAG_EXP_TAYLOR_ORDER(15);
  if (prm->flags & ~known) return set_error(SHV_ERR_INVALID_ARG, "unknown flags 0x%x", prm->flags);
  if ((prm->flags & layouts) == layouts)
    return set_error(SHV_ERR_INVALID_ARG, "SHV_FLAG_EXP_ONE_WAVE and SHV_FLAG_EXP_FOUR_WAVES are exclusive");
  if ((prm->flags & SHV_FLAG_EXP_QUADRATURE) && (prm->flags & layouts))
    return set_error(SHV_ERR_INVALID_ARG, "SHV_FLAG_EXP_QUADRATURE takes no layout flag");
  if ((prm->flags & SHV_FLAG_EXP_PRODUCT) && (prm->flags & ~SHV_FLAG_EXP_PRODUCT))
    return set_error(SHV_ERR_INVALID_ARG, "SHV_FLAG_EXP_PRODUCT takes no other flag");
  const uint32_t order = (prm->flags >> 8) & 15u;
  if (prm->flags & SHV_FLAG_EXP_TAYLOR) {
    if (prm->flags & ~(SHV_FLAG_EXP_TAYLOR | SHV_FLAG_EXP_TAYLOR_ORDER(15)))
      return set_error(SHV_ERR_INVALID_ARG, "SHV_FLAG_EXP_TAYLOR takes no other flag");
    if (order < 1 || order > SHV_MAX_TAYLOR_ORDER)
      return set_error(SHV_ERR_INVALID_ARG, "Taylor order %u outside [1, %d]", order, SHV_MAX_TAYLOR_ORDER);
  } else if (order) {
    return set_error(SHV_ERR_INVALID_ARG, "a Taylor order is set without SHV_FLAG_EXP_TAYLOR");
  }
  return SHV_OK;
}

bool quadrature(const shv_params* prm) { return (prm->flags & SHV_FLAG_EXP_QUADRATURE) != 0; }
bool product(const shv_params* prm) { return (prm->flags & SHV_FLAG_EXP_PRODUCT) != 0; }
bool taylor(const shv_params* prm) { return (prm->flags & SHV_FLAG_EXP_TAYLOR) != 0; }
int taylor_order(const shv_params* prm) { return (int)((prm->flags >> 8) & 15u); }

// Entry points built on the squaring exponential with its linear
// approximation only.
shv_status no_quadrature(const shv_params* prm) {
  if (quadrature(prm) || product(prm) || taylor(prm))
    return set_error(SHV_ERR_UNSUPPORTED, "%s is supported by sh_visibility_forward / sh_visibility_backward only",
                     quadrature(prm) ? "SHV_FLAG_EXP_QUADRATURE"
                                     : (product(prm) ? "SHV_FLAG_EXP_PRODUCT" : "SHV_FLAG_EXP_TAYLOR"));
  return SHV_OK;
}

shv_status check_sizes(int64_t P, int64_t S) {
  if (P < 0 || S < 0) return set_error(SHV_ERR_INVALID_ARG, "negative size (P=%lld, S=%lld)", (long long)P, (long long)S);
  if (P > ((int64_t)1 << 31) - 256 || S > ((int64_t)1 << 24))
    return set_error(SHV_ERR_INVALID_ARG, "size too large (P=%lld, S=%lld)", (long long)P, (long long)S);
  return SHV_OK;
}

shv_status need(const void* p, const char* what) {
  if (!p) return set_error(SHV_ERR_INVALID_ARG, "%s is NULL", what);
  return SHV_OK;
}

shv_status aligned16(const void* p, const char* what) {
  if (((uintptr_t)p) & 15u) return set_error(SHV_ERR_INVALID_ARG, "%s must be 16-byte aligned", what);
  return SHV_OK;
}

#define SHV_TRY(x)                 \
  do {                             \
    shv_status _s = (x);           \
    if (_s != SHV_OK) return _s;   \
  } while (0)

// Workspace carving, one region per phase; phases run in stream order, so
// they reuse the same bytes.
struct FwdWs {
  size_t fpart;
};
struct ShadeWs {
  size_t M, lpart;
};
struct VisBwdWs {
  size_t W, gp, gs;
};

size_t fwd_bytes(int64_t P, int64_t S, int nb, FwdWs* o = nullptr) {
  const shv::Split sp = shv::fwd_split(P, S);
  const size_t fpart = align_up((size_t)sp.nchunks * nb * nb * (size_t)P * 4);
  if (o) o->fpart = 0;
  return fpart;
}
// The quadrature exponential's basis table and partial sums (after the
// phase's own workspace).
size_t quad_table_bytes(int nb) { return align_up((size_t)shv::quad_table_floats(nb) * 4); }
size_t quad_bytes(int nb, int64_t P) {
  return quad_table_bytes(nb) + align_up((size_t)shv::quad_part_floats(nb, P) * 4);
}

// The direct product chain's adjoint: every step's input [S][N][P] and the
// sphere-gradient partials, one row per (block, wave).
struct ProdWs {
  size_t states, gs;
};
size_t prod_bytes(int64_t P, int64_t S, int nb, ProdWs* o = nullptr) {
  const size_t st = align_up((size_t)S * nb * nb * (size_t)P * 4);
  const size_t gs = align_up((size_t)4 * shv::pair_blocks(P) * (size_t)S * 16);
  if (o) {
    o->states = 0;
    o->gs = st;
  }
  return st + gs;
}
// The chain's saved states must stay addressable (below 2^50 bytes).
shv_status check_product_size(int64_t P, int64_t S, int nb) {
  if ((double)P * (double)S * nb * nb * 4.0 > 1125899906842624.0)
    return set_error(SHV_ERR_INVALID_ARG, "P * S too large for SHV_FLAG_EXP_PRODUCT (P=%lld, S=%lld)", (long long)P,
                     (long long)S);
  return SHV_OK;
}

size_t shade_bytes(int64_t P, int nb, ShadeWs* o = nullptr) {
  const size_t N = (size_t)nb * nb;
  const size_t m = align_up(N * N * 4);
  const size_t lp = align_up((size_t)shv::pair_blocks(P) * N * 4);
  if (o) {
    o->M = 0;
    o->lpart = m;
  }
  return m + lp;
}
size_t visbwd_bytes(int64_t P, int64_t S, int nb, VisBwdWs* o = nullptr) {
  const shv::Split sp = shv::bwd_split(P, S);
  const size_t N = (size_t)nb * nb;
  const size_t w = align_up(N * (size_t)P * 4);
  const size_t gp = align_up((size_t)sp.nchunks * 3 * (size_t)P * 4);
  const size_t gs = align_up((size_t)shv::pair_blocks(P) * (size_t)S * 16);
  if (o) {
    o->W = 0;
    o->gp = w;
    o->gs = w + gp;
  }
  return w + gp + gs;
}

struct RenderBwdWs {
  size_t W, gp, gs, lp;
};
// The render backward's W ([N][P]) may alias the forward's sphere-chunk
// partials ([nchunks][N][P], from offset 0): both are indexed by receiver
// column, and a call (or receiver range of a batched call) only touches its
// own receivers' columns.  The receiver-gradient partials and the per-tile
// sphere and lighting partials must outlive later ranges' forwards until the
// closing reductions, so they start after the forward's region.
size_t render_bwd_bytes(int64_t P, int64_t S, int nb, RenderBwdWs* o = nullptr) {
  const shv::Split sp = shv::bwd_split(P, S);
  const size_t N = (size_t)nb * nb;
  const size_t w = align_up(N * (size_t)P * 4);
  const size_t base = std::max(w, fwd_bytes(P, S, nb));
  const size_t gp = align_up((size_t)sp.nchunks * 3 * (size_t)P * 4);
  const size_t gs = align_up((size_t)shv::pair_blocks(P) * (size_t)S * 16);
  const size_t lp = align_up((size_t)shv::pair_blocks(P) * N * 4);
  if (o) {
    o->W = 0;
    o->gp = base;
    o->gs = base + gp;
    o->lp = base + gp + gs;
  }
  return base + gp + gs + lp;
}
// Forward: the F' partials, then M(L) when it is not kept in `saved`.
size_t render_fwd_bytes(int64_t P, int64_t S, int nb) {
  return fwd_bytes(P, S, nb) + align_up((size_t)nb * nb * nb * nb * 4);
}

// Several channels: every channel's M(L_c), then the per-channel tile
// partials of the lighting gradient.
struct ChannelWs {
  size_t M, lpart;
};
size_t channels_bytes(int64_t P, int channels, int nb, ChannelWs* o = nullptr) {
  const size_t N = (size_t)nb * nb;
  const size_t m = align_up((size_t)channels * N * N * 4);
  const size_t lp = align_up((size_t)channels * (size_t)shv::pair_blocks(P) * N * 4);
  if (o) {
    o->M = 0;
    o->lpart = m;
  }
  return m + lp;
}
// Environment map: the per-row-block partial sums [channels][row blocks][N]
// (at most one block per row).
size_t envmap_bytes(int channels, int64_t H, int nb) {
  return align_up((size_t)channels * (size_t)H * nb * nb * 4);
}

shv_status check_channels(int channels) {
  if (channels < 1 || channels > SHV_MAX_CHANNELS)
    return set_error(SHV_ERR_INVALID_ARG, "channels must be in [1, %d] (got %d)", SHV_MAX_CHANNELS, channels);
  return SHV_OK;
}

// Deformation: rotation matrices, the cotangents ybar / zbar, the global
// partials and their sum.
struct DeformWs {
  size_t rm, yb, gpart, g;
};
size_t deform_bytes(int64_t P, int64_t S, DeformWs* o = nullptr) {
  const size_t rm = align_up((size_t)(S + 1) * 9 * 4);
  const size_t yb = align_up((size_t)6 * P * 4);
  const size_t gp = align_up((size_t)(shv::deform_vert_blocks(P) + S) * 12 * 4);
  const size_t g = align_up(12 * 4);
  if (o) {
    o->rm = 0;
    o->yb = rm;
    o->gpart = rm + yb;
    o->g = rm + yb + gp;
  }
  return rm + yb + gp + g;
}

shv_status check_graph(const shv_deform_graph* gr, shv::DeformGraphDev* g) {
  if (!gr) return set_error(SHV_ERR_INVALID_ARG, "graph is NULL");
  if (gr->P < 1 || gr->S < 1 || gr->K < 1 || gr->K > gr->P || gr->P > ((int64_t)1 << 31) - 256 ||
      gr->S * (int64_t)gr->K >= ((int64_t)1 << 31))
    return set_error(SHV_ERR_INVALID_ARG, "invalid graph sizes (P=%lld, S=%lld, K=%d)", (long long)gr->P,
                     (long long)gr->S, gr->K);
  if (!gr->vertices || !gr->normals || !gr->spheres || !gr->vert_ptr || !gr->vert_sph || !gr->vert_w ||
      !gr->sph_vert || !gr->sph_w)
    return set_error(SHV_ERR_INVALID_ARG, "graph has a NULL array");
  *g = shv::DeformGraphDev{gr->vertices, gr->normals, gr->spheres, gr->vert_ptr, gr->vert_sph, gr->vert_w,
                           gr->sph_vert, gr->sph_w, gr->P, gr->S, gr->K};
  return SHV_OK;
}

shv_status check_ws(void* ws, size_t ws_bytes, size_t needed) {
  if (needed == 0) return SHV_OK;
  if (!ws) return set_error(SHV_ERR_WORKSPACE, "workspace is NULL (need %zu bytes)", needed);
  if (((uintptr_t)ws) % kAlign) return set_error(SHV_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
  if (ws_bytes < needed) return set_error(SHV_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, needed);
  return SHV_OK;
}

// The forward's saved state: `floats` FP32 values in a buffer of `bytes`
// bytes.  A NULL buffer is accepted where the state is optional (a forward
// with no backward to follow) or empty.
shv_status check_saved(const void* saved, size_t bytes, int64_t floats, bool required) {
  if (!saved) {
    if (required && floats > 0) return set_error(SHV_ERR_INVALID_ARG, "saved is NULL (need %lld floats)",
                                                 (long long)floats);
    return SHV_OK;
  }
  if (((uintptr_t)saved) & 3u) return set_error(SHV_ERR_INVALID_ARG, "saved must be 4-byte aligned");
  if (bytes / 4 < (size_t)floats)
    return set_error(SHV_ERR_WORKSPACE, "saved has %zu bytes, needs %lld (%lld floats)", bytes,
                     (long long)floats * 4, (long long)floats);
  return SHV_OK;
}

shv_status check_camera(const shv_camera* cam, shv::RasterCam& rc) {
  if (!cam) return set_error(SHV_ERR_INVALID_ARG, "camera is NULL");
  if (cam->width < 1 || cam->height < 1 || cam->width > SHV_MAX_IMAGE_SIDE || cam->height > SHV_MAX_IMAGE_SIDE)
    return set_error(SHV_ERR_INVALID_ARG, "image size %d x %d outside [1, %d]", cam->width, cam->height,
                     SHV_MAX_IMAGE_SIDE);
  for (int i = 0; i < 12; ++i) {
    if (!std::isfinite(cam->P[i])) return set_error(SHV_ERR_INVALID_ARG, "camera matrix has a non-finite entry");
    rc.P[i] = cam->P[i];
  }
  rc.width = cam->width;
  rc.height = cam->height;
  return SHV_OK;
}

// The tile lists hold up to 16 entries per face in 32-bit offsets.
bool mesh_size_ok(int64_t V, int64_t T) {
  return V >= 0 && T >= 0 && V < ((int64_t)1 << 31) && 32 * T < ((int64_t)1 << 31);
}

shv_status check_mesh(int64_t V, int64_t T) {
  if (!mesh_size_ok(V, T))
    return set_error(SHV_ERR_INVALID_ARG, "mesh size out of range (V=%lld, T=%lld; T < 2^26)", (long long)V,
                     (long long)T);
  return SHV_OK;
}

}  // namespace

extern "C" {

shv_status shv_init(int device) {
  if (device < 0 || device >= 64) return set_error(SHV_ERR_INVALID_ARG, "device %d out of range", device);
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return set_error(SHV_ERR_HIP, "hipSetDevice(%d): %s", device, hipGetErrorString(e));
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return set_error(SHV_ERR_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return set_error(SHV_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(SHV_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
    g_scratch[device] = ptr;
  }
  g_init[device] = true;
  return SHV_OK;
}

const char* shv_status_string(shv_status s) {
  switch (s) {
    case SHV_OK: return "ok";
    case SHV_ERR_INVALID_ARG: return "invalid argument";
    case SHV_ERR_UNSUPPORTED: return "unsupported parameters";
    case SHV_ERR_WORKSPACE: return "workspace too small";
    case SHV_ERR_NOT_INITIALIZED: return "library not initialised for this device";
    case SHV_ERR_HIP: return "HIP error";
    default: return "unknown status";
  }
}

const char* shv_last_error(void) { return g_last_error.c_str(); }

int64_t shv_saved_floats(int64_t P, const shv_params* prm) {
  if (!prm || prm->n_bands < 1 || prm->n_bands > SHV_MAX_BANDS_API || prm->n_squarings < 0 || P < 0) return 0;
  const int64_t N = (int64_t)prm->n_bands * prm->n_bands;
  const int64_t squaring = (1 + (int64_t)prm->n_squarings * N) * P;
  if (prm->flags & SHV_FLAG_EXP_PRODUCT) return 0;
  if (prm->flags & SHV_FLAG_EXP_TAYLOR) return (1 + ((int64_t)prm->n_squarings + ((prm->flags >> 8) & 15u)) * N) * P;
  return (prm->flags & SHV_FLAG_EXP_QUADRATURE) ? std::max(squaring, N * P) : squaring;
}

size_t shv_workspace_bytes(int64_t P, int64_t S, const shv_params* prm) {
  if (!prm || prm->n_bands < 1 || prm->n_bands > SHV_MAX_BANDS_API || P < 0 || S < 0) return 0;
  const int nb = prm->n_bands;
  size_t b = fwd_bytes(P, S, nb);
  b = std::max(b, shade_bytes(P, nb));
  b = std::max(b, visbwd_bytes(P, S, nb));
  b = std::max(b, render_fwd_bytes(P, S, nb));
  b = std::max(b, render_bwd_bytes(P, S, nb));
  if (prm->flags & SHV_FLAG_EXP_QUADRATURE) {
    b = std::max(b, fwd_bytes(P, S, nb) + quad_bytes(nb, P));
    b = std::max(b, visbwd_bytes(P, S, nb) + quad_bytes(nb, P));
  }
  if (prm->flags & SHV_FLAG_EXP_PRODUCT) b = std::max(b, prod_bytes(P, S, nb));
  return b;
}

int64_t shv_render_saved_floats(int64_t P, const shv_params* prm) {
  if (!prm || prm->n_bands < 1 || prm->n_bands > SHV_MAX_BANDS_API || prm->n_squarings < 0 || P < 0) return 0;
  const int64_t N = (int64_t)prm->n_bands * prm->n_bands;
  return (1 + (int64_t)prm->n_squarings * N) * P + N * N;
}

shv_status sh_render_forward(const float* points, const float* normals, const float* albedo, const float* spheres,
                             const float* light, int64_t P, int64_t S, const shv_params* prm, float* vis,
                             float* radiance, float* saved, size_t saved_bytes, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(no_quadrature(prm));
  SHV_TRY(check_sizes(P, S));
  if (P == 0) return check_device();
  SHV_TRY(need(points, "points"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(albedo, "albedo"));
  SHV_TRY(need(light, "light"));
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(radiance, "radiance"));
  if (S > 0) {
    SHV_TRY(need(spheres, "spheres"));
    SHV_TRY(aligned16(spheres, "spheres"));
  }
  const int nb = prm->n_bands;
  SHV_TRY(check_saved(saved, saved_bytes, shv_render_saved_floats(P, prm), false));
  SHV_TRY(check_ws(ws, ws_bytes, render_fwd_bytes(P, S, nb)));
  SHV_TRY(check_device());
  float* Fpart = (float*)ws;
  const int64_t N = (int64_t)nb * nb;
  float* M = saved ? saved + (1 + (int64_t)prm->n_squarings * N) * P : (float*)((char*)ws + fwd_bytes(P, S, nb));
  const shv::Split sp = shv::fwd_split(P, S);
  SHV_TRY(launch("pair_fwd", stream, [&] {
    return shv::launch_pair_fwd(nb, points, P, spheres, (int)S, sp, Fpart, light, M, stream);
  }));
  SHV_TRY(launch("exp_shade_fwd", stream, [&] {
    return shv::launch_render_exp_fwd(nb, Fpart, sp.nchunks, P, prm->eps, prm->n_squarings, vis, saved, normals,
                                      albedo, M, radiance, prm->flags, stream);
  }));
  return SHV_OK;
}

shv_status sh_render_forward_noalloc(const float* points, const float* normals, const float* albedo,
                                     const float* spheres, const float* light, int64_t P, int64_t S,
                                     const shv_params* prm, float* vis, float* radiance, float* saved,
                                     size_t saved_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(no_quadrature(prm));
  SHV_TRY(check_sizes(P, S));
  const size_t need_bytes = render_fwd_bytes(P, S, prm->n_bands);
  if (need_bytes > SHV_NOALLOC_SCRATCH_BYTES)
    return set_error(SHV_ERR_WORKSPACE,
                     "sh_render_forward_noalloc: P=%lld, S=%lld, n_bands=%d needs %zu bytes of scratch; the static "
                     "scratch holds %zu (use sh_render_forward with a workspace)",
                     (long long)P, (long long)S, prm->n_bands, need_bytes, (size_t)SHV_NOALLOC_SCRATCH_BYTES);
  if (P == 0) return check_device();
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(SHV_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_init_mu);
    if (dev >= 0 && dev < 64) ws = g_scratch[dev];
  }
  if (!ws) return set_error(SHV_ERR_NOT_INITIALIZED, "shv_init() has not been called for device %d", dev);
  return sh_render_forward(points, normals, albedo, spheres, light, P, S, prm, vis, radiance, saved, saved_bytes,
                           ws, SHV_NOALLOC_SCRATCH_BYTES, stream);
}

shv_status sh_render_backward(const float* grad_radiance, const float* points, const float* normals,
                              const float* albedo, const float* spheres, int64_t P, int64_t S, const shv_params* prm,
                              const float* vis, const float* saved, size_t saved_bytes, float* grad_points,
                              float* grad_normals, float* grad_albedo, float* grad_spheres, float* grad_light,
                              void* ws, size_t ws_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(no_quadrature(prm));
  SHV_TRY(check_sizes(P, S));
  const int nb = prm->n_bands;
  const int N = nb * nb;
  if (P == 0) {
    SHV_TRY(check_device());
    if (grad_light)
      SHV_TRY(launch("fill_zero", stream, [&] { return shv::launch_fill_zero(grad_light, N, stream); }));
    if (grad_spheres && S > 0)
      SHV_TRY(launch("fill_zero", stream, [&] { return shv::launch_fill_zero(grad_spheres, 4 * S, stream); }));
    return SHV_OK;
  }
  SHV_TRY(need(grad_radiance, "grad_radiance"));
  SHV_TRY(need(points, "points"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(albedo, "albedo"));
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(saved, "saved"));
  if (S > 0) {
    SHV_TRY(need(spheres, "spheres"));
    SHV_TRY(aligned16(spheres, "spheres"));
  }
  SHV_TRY(check_saved(saved, saved_bytes, shv_render_saved_floats(P, prm), true));
  RenderBwdWs L;
  SHV_TRY(check_ws(ws, ws_bytes, render_bwd_bytes(P, S, nb, &L)));
  SHV_TRY(check_device());
  float* W = (float*)((char*)ws + L.W);
  float* gp = (float*)((char*)ws + L.gp);
  float* gs = (float*)((char*)ws + L.gs);
  float* lp = (float*)((char*)ws + L.lp);
  const float* M = saved + (1 + (int64_t)prm->n_squarings * N) * P;
  const shv::Split sp = shv::bwd_split(P, S);
  SHV_TRY(launch("exp_shade_bwd", stream, [&] {
    return shv::launch_render_exp_bwd(nb, grad_radiance, vis, saved, P, prm->eps, prm->n_squarings, W, normals,
                                      albedo, M, grad_normals, grad_albedo, grad_light ? lp : nullptr, prm->flags,
                                      stream);
  }));
  const bool need_pair = grad_points || (grad_spheres && S > 0);
  if (need_pair) {
    SHV_TRY(launch("pair_bwd", stream, [&] {
      return shv::launch_pair_bwd(nb, W, points, P, spheres, (int)S, sp, gp, gs, stream);
    }));
  }
  if (grad_spheres && S == 0) grad_spheres = nullptr;
  SHV_TRY(launch("finalize", stream, [&] {
    return shv::launch_finalize(gp, sp.nchunks, P, need_pair ? grad_points : nullptr, gs,
                                (int)shv::pair_blocks(P), S, grad_spheres, lp, (int)shv::pair_blocks(P), N, grad_light,
                                stream);
  }));
  return SHV_OK;
}

shv_status sh_visibility_forward(const float* points, int64_t P, const float* spheres, int64_t S,
                                 const shv_params* prm, float* vis, float* saved, size_t saved_bytes, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_sizes(P, S));
  if (P == 0) return check_device();
  SHV_TRY(need(points, "points"));
  SHV_TRY(need(vis, "vis"));
  if (S > 0) {
    SHV_TRY(need(spheres, "spheres"));
    SHV_TRY(aligned16(spheres, "spheres"));
  }
  const int nb = prm->n_bands;
  SHV_TRY(check_saved(saved, saved_bytes, shv_saved_floats(P, prm), false));
  if (product(prm)) {
    SHV_TRY(check_product_size(P, S, nb));
    SHV_TRY(check_device());
    SHV_TRY(launch("prod_fwd", stream, [&] {
      return shv::launch_prod_fwd(nb, points, P, spheres, (int)S, prm->eps, vis, nullptr, stream);
    }));
    return SHV_OK;
  }
  const size_t base = fwd_bytes(P, S, nb);
  SHV_TRY(check_ws(ws, ws_bytes, base + (quadrature(prm) ? quad_bytes(nb, P) : 0)));
  SHV_TRY(check_device());
  float* Fpart = (float*)ws;
  const shv::Split sp = shv::fwd_split(P, S);
  SHV_TRY(launch("pair_fwd", stream, [&] {
    return shv::launch_pair_fwd(nb, points, P, spheres, (int)S, sp, Fpart, nullptr, nullptr, stream);
  }));
  if (quadrature(prm)) {
    SHV_TRY(launch("exp_quad_fwd", stream, [&] {
      return shv::launch_exp_quad_fwd(nb, Fpart, sp.nchunks, P, prm->eps, vis, saved, (float*)((char*)ws + base),
                                      (float*)((char*)ws + base + quad_table_bytes(nb)), stream);
    }));
    return SHV_OK;
  }
  if (taylor(prm)) {
    SHV_TRY(launch("exp_taylor_fwd", stream, [&] {
      return shv::launch_exp_taylor_fwd(nb, Fpart, sp.nchunks, P, prm->eps, prm->n_squarings, taylor_order(prm), vis,
                                        saved, stream);
    }));
    return SHV_OK;
  }
  SHV_TRY(launch("exp_fwd", stream, [&] {
    return shv::launch_exp_fwd(nb, Fpart, sp.nchunks, P, prm->eps, prm->n_squarings, vis, saved, prm->flags,
                               stream);
  }));
  return SHV_OK;
}

shv_status sh_shade(const float* vis, const float* normals, const float* albedo, const float* light, int64_t P,
                    const shv_params* prm, float* radiance, void* ws, size_t ws_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_sizes(P, 0));
  SHV_TRY(check_device());
  if (P == 0) return SHV_OK;
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(albedo, "albedo"));
  SHV_TRY(need(light, "light"));
  SHV_TRY(need(radiance, "radiance"));
  const int nb = prm->n_bands;
  ShadeWs L;
  SHV_TRY(check_ws(ws, ws_bytes, shade_bytes(P, nb, &L)));
  float* M = (float*)((char*)ws + L.M);
  SHV_TRY(launch("build_M", stream, [&] { return shv::launch_build_M(nb, light, M, stream); }));
  SHV_TRY(launch("shade_fwd", stream, [&] {
    return shv::launch_shade_ch_fwd(nb, vis, normals, albedo, M, 1, P, radiance, stream);
  }));
  return SHV_OK;
}

shv_status sh_shade_backward(const float* grad_radiance, const float* vis, const float* normals, const float* albedo,
                             const float* light, int64_t P, const shv_params* prm, float* grad_vis,
                             float* grad_normals, float* grad_albedo, float* grad_light, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_sizes(P, 0));
  SHV_TRY(check_device());
  const int nb = prm->n_bands;
  const int N = nb * nb;
  if (P == 0) {
    if (grad_light)
      SHV_TRY(launch("fill_zero", stream, [&] { return shv::launch_fill_zero(grad_light, N, stream); }));
    return SHV_OK;
  }
  SHV_TRY(need(grad_radiance, "grad_radiance"));
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(albedo, "albedo"));
  SHV_TRY(need(light, "light"));
  ShadeWs L;
  SHV_TRY(check_ws(ws, ws_bytes, shade_bytes(P, nb, &L)));
  float* M = (float*)((char*)ws + L.M);
  float* Lpart = grad_light ? (float*)((char*)ws + L.lpart) : nullptr;
  SHV_TRY(launch("build_M", stream, [&] { return shv::launch_build_M(nb, light, M, stream); }));
  SHV_TRY(launch("shade_bwd", stream, [&] {
    return shv::launch_shade_ch_bwd(nb, grad_radiance, vis, normals, albedo, M, 1, P, grad_vis, grad_normals,
                                    grad_albedo, Lpart, stream);
  }));
  if (grad_light) {
    SHV_TRY(launch("reduce_light", stream, [&] {
      return shv::launch_reduce_rows(Lpart, (int)shv::pair_blocks(P), N, grad_light, stream);
    }));
  }
  return SHV_OK;
}

size_t shv_channels_workspace_bytes(int64_t P, int channels, const shv_params* prm) {
  if (!prm || prm->n_bands < 1 || prm->n_bands > SHV_MAX_BANDS_API || P < 0 || channels < 1 ||
      channels > SHV_MAX_CHANNELS)
    return 0;
  return channels_bytes(P, channels, prm->n_bands);
}

shv_status sh_shade_channels(const float* vis, const float* normals, const float* albedo, const float* light,
                             int channels, int64_t P, const shv_params* prm, float* radiance, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_sizes(P, 0));
  SHV_TRY(check_channels(channels));
  SHV_TRY(check_device());
  if (P == 0) return SHV_OK;
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(albedo, "albedo"));
  SHV_TRY(need(light, "light"));
  SHV_TRY(need(radiance, "radiance"));
  const int nb = prm->n_bands;
  ChannelWs L;
  SHV_TRY(check_ws(ws, ws_bytes, channels_bytes(P, channels, nb, &L)));
  float* M = (float*)((char*)ws + L.M);
  SHV_TRY(launch("build_M", stream, [&] { return shv::launch_build_M(nb, light, M, stream, channels); }));
  SHV_TRY(launch("shade_ch_fwd", stream, [&] {
    return shv::launch_shade_ch_fwd(nb, vis, normals, albedo, M, channels, P, radiance, stream);
  }));
  return SHV_OK;
}

shv_status sh_shade_channels_backward(const float* grad_radiance, const float* vis, const float* normals,
                                      const float* albedo, const float* light, int channels, int64_t P,
                                      const shv_params* prm, float* grad_vis, float* grad_normals,
                                      float* grad_albedo, float* grad_light, void* ws, size_t ws_bytes,
                                      hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_sizes(P, 0));
  SHV_TRY(check_channels(channels));
  SHV_TRY(check_device());
  const int nb = prm->n_bands;
  const int N = nb * nb;
  if (P == 0) {
    if (grad_light)
      SHV_TRY(launch("fill_zero", stream,
                     [&] { return shv::launch_fill_zero(grad_light, (int64_t)channels * N, stream); }));
    return SHV_OK;
  }
  SHV_TRY(need(grad_radiance, "grad_radiance"));
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(albedo, "albedo"));
  SHV_TRY(need(light, "light"));
  ChannelWs L;
  SHV_TRY(check_ws(ws, ws_bytes, channels_bytes(P, channels, nb, &L)));
  float* M = (float*)((char*)ws + L.M);
  float* Lpart = grad_light ? (float*)((char*)ws + L.lpart) : nullptr;
  SHV_TRY(launch("build_M", stream, [&] { return shv::launch_build_M(nb, light, M, stream, channels); }));
  SHV_TRY(launch("shade_ch_bwd", stream, [&] {
    return shv::launch_shade_ch_bwd(nb, grad_radiance, vis, normals, albedo, M, channels, P, grad_vis,
                                    grad_normals, grad_albedo, Lpart, stream);
  }));
  if (grad_light) {
    SHV_TRY(launch("reduce_light", stream, [&] {
      return shv::launch_reduce_rows(Lpart, (int)shv::pair_blocks(P), N, grad_light, stream, channels);
    }));
  }
  return SHV_OK;
}

size_t shv_envmap_workspace_bytes(int channels, int64_t H, int64_t W, const shv_params* prm) {
  if (!prm || prm->n_bands < 1 || prm->n_bands > SHV_MAX_BANDS_API || channels < 1 ||
      channels > SHV_MAX_CHANNELS || H < 0 || W < 0 || H > SHV_MAX_ENVMAP_ROWS || W > SHV_MAX_ENVMAP_COLS)
    return 0;
  return envmap_bytes(channels, H, prm->n_bands);
}

shv_status sh_envmap_project(const float* image, int channels, int64_t H, int64_t W, const shv_params* prm,
                             float* light, void* ws, size_t ws_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_channels(channels));
  if (H < 0 || W < 0) return set_error(SHV_ERR_INVALID_ARG, "negative map size (H=%lld, W=%lld)", (long long)H,
                                       (long long)W);
  if (H > SHV_MAX_ENVMAP_ROWS || W > SHV_MAX_ENVMAP_COLS)
    return set_error(SHV_ERR_INVALID_ARG, "map too large (H=%lld, W=%lld)", (long long)H, (long long)W);
  SHV_TRY(check_device());
  SHV_TRY(need(light, "light"));
  const int nb = prm->n_bands;
  const int N = nb * nb;
  if (H == 0 || W == 0)
    return launch("fill_zero", stream,
                  [&] { return shv::launch_fill_zero(light, (int64_t)channels * N, stream); });
  SHV_TRY(need(image, "image"));
  SHV_TRY(check_ws(ws, ws_bytes, envmap_bytes(channels, H, nb)));
  float* part = (float*)ws;
  SHV_TRY(launch("envmap_rows", stream,
                 [&] { return shv::launch_envmap_rows(nb, image, channels, H, W, part, stream); }));
  SHV_TRY(launch("reduce_envmap", stream, [&] {
    return shv::launch_reduce_rows(part, (int)shv::envmap_row_blocks(H, W), N, light, stream, channels);
  }));
  return SHV_OK;
}

// ------------------------------------------------------------------ rasteriser

shv_status shv_raster_incidence_build(const int32_t* faces, int64_t T, int64_t V, int32_t* ptr, int32_t* idx) {
  if (T < 0 || V < 0 || 3 * T >= ((int64_t)1 << 31) || V >= ((int64_t)1 << 31))
    return set_error(SHV_ERR_INVALID_ARG, "mesh size out of range (T=%lld, V=%lld)", (long long)T, (long long)V);
  if ((T > 0 && (!faces || !idx)) || !ptr) return set_error(SHV_ERR_INVALID_ARG, "NULL array");
  std::vector<int32_t> count(V + 1, 0);
  for (int64_t c = 0; c < 3 * T; ++c) {
    const int32_t v = faces[c];
    if (v < 0 || v >= V)
      return set_error(SHV_ERR_INVALID_ARG, "face %lld has vertex index %d outside [0, %lld)", (long long)(c / 3), v,
                       (long long)V);
    ++count[v + 1];
  }
  for (int64_t v = 0; v < V; ++v) count[v + 1] += count[v];
  for (int64_t v = 0; v <= V; ++v) ptr[v] = count[v];
  for (int64_t c = 0; c < 3 * T; ++c) idx[count[faces[c]]++] = (int32_t)c;
  return SHV_OK;
}

size_t shv_raster_workspace_bytes(int64_t V, int64_t T, int32_t width, int32_t height) {
  if (!mesh_size_ok(V, T) || width < 1 || height < 1 || width > SHV_MAX_IMAGE_SIDE || height > SHV_MAX_IMAGE_SIDE)
    return 0;
  return align_up(shv::raster_record_bytes(T)) +
         std::max(align_up((size_t)T * 12 * 4), align_up(shv::raster_bin_bytes(T, width, height)));
}

shv_status sh_raster_forward(const float* vertices, int64_t V, const int32_t* faces, int64_t T, const float* radiance,
                             const shv_camera* camera, float* image, int32_t* face_id, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  shv::RasterCam rc;
  SHV_TRY(check_camera(camera, rc));
  SHV_TRY(check_mesh(V, T));
  SHV_TRY(check_device());
  SHV_TRY(need(image, "image"));
  SHV_TRY(need(face_id, "face_id"));
  if (T > 0) {
    SHV_TRY(need(vertices, "vertices"));
    SHV_TRY(need(faces, "faces"));
    SHV_TRY(need(radiance, "radiance"));
  }
  SHV_TRY(check_ws(ws, ws_bytes, shv_raster_workspace_bytes(V, T, rc.width, rc.height)));
  void* bins = (char*)ws + align_up(shv::raster_record_bytes(T));
  SHV_TRY(launch("raster_fwd", stream, [&] {
    return shv::launch_raster_forward(vertices, V, faces, T, radiance, rc, image, face_id, ws, bins, stream);
  }));
  return SHV_OK;
}

shv_status sh_raster_backward(const float* grad_image, const float* vertices, int64_t V, const int32_t* faces,
                              int64_t T, const float* radiance, const shv_camera* camera, const int32_t* face_id,
                              const int32_t* inc_ptr, const int32_t* inc_idx, float* grad_radiance,
                              float* grad_vertices, void* ws, size_t ws_bytes, hipStream_t stream) {
  shv::RasterCam rc;
  SHV_TRY(check_camera(camera, rc));
  SHV_TRY(check_mesh(V, T));
  SHV_TRY(check_device());
  if (V == 0 || (!grad_radiance && !grad_vertices)) return SHV_OK;
  SHV_TRY(need(vertices, "vertices"));
  SHV_TRY(need(inc_ptr, "inc_ptr"));
  if (T > 0) {
    SHV_TRY(need(grad_image, "grad_image"));
    SHV_TRY(need(faces, "faces"));
    SHV_TRY(need(radiance, "radiance"));
    SHV_TRY(need(face_id, "face_id"));
    SHV_TRY(need(inc_idx, "inc_idx"));
  }
  SHV_TRY(check_ws(ws, ws_bytes, shv_raster_workspace_bytes(V, T, rc.width, rc.height)));
  float* part = (float*)((char*)ws + align_up(shv::raster_record_bytes(T)));
  SHV_TRY(launch("raster_bwd", stream, [&] {
    return shv::launch_raster_backward(grad_image, vertices, V, faces, T, radiance, rc, face_id, inc_ptr, inc_idx,
                                       grad_radiance, grad_vertices, ws, part, stream);
  }));
  return SHV_OK;
}

shv_status shv_deform_graph_build(const float* vertices, int64_t P, const float* spheres, int64_t S, int32_t K,
                                  int32_t* vert_ptr, int32_t* vert_sph, float* vert_w, int32_t* sph_vert,
                                  float* sph_w) {
  if (P < 1 || S < 1 || K < 1 || K > P || P > ((int64_t)1 << 31) - 256 || S * (int64_t)K >= ((int64_t)1 << 31))
    return set_error(SHV_ERR_INVALID_ARG, "invalid attachment sizes (P=%lld, S=%lld, K=%d)", (long long)P,
                     (long long)S, K);
  SHV_TRY(need(vertices, "vertices"));
  SHV_TRY(need(spheres, "spheres"));
  SHV_TRY(need(vert_ptr, "vert_ptr"));
  SHV_TRY(need(vert_sph, "vert_sph"));
  SHV_TRY(need(vert_w, "vert_w"));
  SHV_TRY(need(sph_vert, "sph_vert"));
  SHV_TRY(need(sph_w, "sph_w"));
  shv::deform_graph_build(vertices, P, spheres, S, K, vert_ptr, vert_sph, vert_w, sph_vert, sph_w);
  return SHV_OK;
}

size_t shv_deform_workspace_bytes(int64_t P, int64_t S) {
  if (P < 1 || S < 1) return 0;
  DeformWs L;
  return deform_bytes(P, S, &L);
}

shv_status sh_deform_forward(const shv_deform_graph* graph, const float* params, float* points, float* normals,
                             float* spheres, void* ws, size_t ws_bytes, hipStream_t stream) {
  shv::DeformGraphDev g;
  SHV_TRY(check_graph(graph, &g));
  SHV_TRY(check_device());
  SHV_TRY(need(params, "params"));
  SHV_TRY(need(points, "points"));
  SHV_TRY(need(normals, "normals"));
  SHV_TRY(need(spheres, "spheres"));
  DeformWs L;
  SHV_TRY(check_ws(ws, ws_bytes, deform_bytes(g.P, g.S, &L)));
  float* Rm = (float*)((char*)ws + L.rm);
  return launch("deform_fwd", stream,
                [&] { return shv::launch_deform_forward(g, params, Rm, points, normals, spheres, stream); });
}

shv_status sh_deform_backward(const shv_deform_graph* graph, const float* params, const float* grad_points,
                              const float* grad_normals, const float* grad_spheres, float* grad_params, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  shv::DeformGraphDev g;
  SHV_TRY(check_graph(graph, &g));
  SHV_TRY(check_device());
  SHV_TRY(need(params, "params"));
  SHV_TRY(need(grad_params, "grad_params"));
  DeformWs L;
  SHV_TRY(check_ws(ws, ws_bytes, deform_bytes(g.P, g.S, &L)));
  char* b = (char*)ws;
  return launch("deform_bwd", stream, [&] {
    return shv::launch_deform_backward(g, params, grad_points, grad_normals, grad_spheres, (float*)(b + L.rm),
                                       (float*)(b + L.yb), (float*)(b + L.gpart), (float*)(b + L.g), grad_params,
                                       stream);
  });
}

size_t shv_l2_workspace_bytes(int64_t n) {
  if (n < 1) return 0;
  return align_up((size_t)((n + SHV_BLOCK - 1) / SHV_BLOCK) * 4);
}

shv_status sh_l2_loss(const float* value, const float* target, int64_t n, float* grad, float* loss, void* ws,
                      size_t ws_bytes, hipStream_t stream) {
  if (n < 1 || n > ((int64_t)1 << 31) - 256) return set_error(SHV_ERR_INVALID_ARG, "invalid size n=%lld", (long long)n);
  SHV_TRY(check_device());
  SHV_TRY(need(value, "value"));
  SHV_TRY(need(target, "target"));
  SHV_TRY(need(loss, "loss"));
  SHV_TRY(check_ws(ws, ws_bytes, shv_l2_workspace_bytes(n)));
  return launch("l2_loss", stream, [&] { return shv::launch_l2(value, target, n, grad, (float*)ws, loss, stream); });
}

shv_status sh_sgd_step(float* x, const float* grad, int64_t n, float lr, hipStream_t stream) {
  if (n < 0) return set_error(SHV_ERR_INVALID_ARG, "negative size");
  if (!(lr == lr)) return set_error(SHV_ERR_INVALID_ARG, "lr is NaN");
  SHV_TRY(check_device());
  if (n == 0) return SHV_OK;
  SHV_TRY(need(x, "x"));
  SHV_TRY(need(grad, "grad"));
  return launch("sgd", stream, [&] { return shv::launch_sgd(x, grad, n, lr, stream); });
}

shv_status sh_visibility_backward(const float* grad_vis, const float* vis, const float* points, int64_t P,
                                  const float* spheres, int64_t S, const shv_params* prm, const float* saved,
                                  size_t saved_bytes, float* grad_points, float* grad_spheres, void* ws,
                                  size_t ws_bytes, hipStream_t stream) {
  SHV_TRY(check_params(prm));
  SHV_TRY(check_sizes(P, S));
  if (P == 0 || (!grad_points && !grad_spheres)) {
    SHV_TRY(check_device());
    if (grad_spheres && S > 0)
      SHV_TRY(launch("fill_zero", stream, [&] { return shv::launch_fill_zero(grad_spheres, 4 * S, stream); }));
    return SHV_OK;
  }
  SHV_TRY(need(grad_vis, "grad_vis"));
  SHV_TRY(need(vis, "vis"));
  SHV_TRY(need(points, "points"));
  SHV_TRY(check_saved(saved, saved_bytes, shv_saved_floats(P, prm), true));
  if (S > 0) {
    SHV_TRY(need(spheres, "spheres"));
    SHV_TRY(aligned16(spheres, "spheres"));
  }
  const int nb = prm->n_bands;
  if (product(prm)) {
    // The chain is run again, recording each step's input, then reversed.
    SHV_TRY(check_product_size(P, S, nb));
    ProdWs L;
    SHV_TRY(check_ws(ws, ws_bytes, prod_bytes(P, S, nb, &L)));
    SHV_TRY(check_device());
    float* states = (float*)((char*)ws + L.states);
    float* gs = (float*)((char*)ws + L.gs);
    if (S > 0) {
      SHV_TRY(launch("prod_fwd_states", stream, [&] {
        return shv::launch_prod_fwd(nb, points, P, spheres, (int)S, prm->eps, nullptr, states, stream);
      }));
    }
    SHV_TRY(launch("prod_bwd", stream, [&] {
      return shv::launch_prod_bwd(nb, grad_vis, states, points, P, spheres, (int)S, prm->eps, grad_points, gs,
                                  stream);
    }));
    if (grad_spheres && S > 0) {
      SHV_TRY(launch("reduce_spheres", stream, [&] {
        return shv::launch_reduce_rows(gs, (int)(4 * shv::pair_blocks(P)), (int)(4 * S), grad_spheres, stream);
      }));
    }
    return SHV_OK;
  }
  VisBwdWs L;
  const size_t base = visbwd_bytes(P, S, nb, &L);
  SHV_TRY(check_ws(ws, ws_bytes, base + (quadrature(prm) ? quad_bytes(nb, P) : 0)));
  SHV_TRY(check_device());
  float* W = (float*)((char*)ws + L.W);
  float* gp = (float*)((char*)ws + L.gp);
  float* gs = (float*)((char*)ws + L.gs);
  const shv::Split sp = shv::bwd_split(P, S);
  if (quadrature(prm)) {
    SHV_TRY(launch("exp_quad_bwd", stream, [&] {
      return shv::launch_exp_quad_bwd(nb, grad_vis, vis, saved, P, prm->eps, W, (float*)((char*)ws + base),
                                      (float*)((char*)ws + base + quad_table_bytes(nb)), stream);
    }));
  } else if (taylor(prm)) {
    SHV_TRY(launch("exp_taylor_bwd", stream, [&] {
      return shv::launch_exp_taylor_bwd(nb, grad_vis, vis, saved, P, prm->eps, prm->n_squarings, taylor_order(prm), W,
                                        stream);
    }));
  } else {
    SHV_TRY(launch("exp_bwd", stream, [&] {
      return shv::launch_exp_bwd(nb, grad_vis, vis, saved, P, prm->eps, prm->n_squarings, W, prm->flags, stream);
    }));
  }
  SHV_TRY(launch("pair_bwd", stream, [&] {
    return shv::launch_pair_bwd(nb, W, points, P, spheres, (int)S, sp, gp, gs, stream);
  }));
  if (grad_points) {
    SHV_TRY(launch("sum_point_chunks", stream, [&] {
      return shv::launch_sum_chunks(gp, sp.nchunks, 3 * P, grad_points, stream);
    }));
  }
  if (grad_spheres && S > 0) {
    SHV_TRY(launch("reduce_spheres", stream, [&] {
      return shv::launch_reduce_rows(gs, (int)shv::pair_blocks(P), (int)(4 * S), grad_spheres, stream);
    }));
  }
  return SHV_OK;
}

size_t shv_batch_table_bytes(int32_t n_scenes) {
  if (n_scenes < 0) return 0;
  return shv::batch_table_bytes(n_scenes);
}

shv_status shv_batch_table_build(const shv_scene* scenes, int32_t n_scenes, void* table, size_t table_bytes) {
  if (n_scenes < 0) return set_error(SHV_ERR_INVALID_ARG, "negative scene count");
  if (n_scenes > 0 && !scenes) return set_error(SHV_ERR_INVALID_ARG, "scenes is NULL");
  if (!table) return set_error(SHV_ERR_INVALID_ARG, "table is NULL");
  if (table_bytes < shv_batch_table_bytes(n_scenes))
    return set_error(SHV_ERR_WORKSPACE, "table has %zu bytes, needs %zu", table_bytes, shv_batch_table_bytes(n_scenes));
  shv::BatchHeader h{};
  h.n_scenes = n_scenes;
  shv::BatchScene* out = (shv::BatchScene*)((char*)table + sizeof(shv::BatchHeader));
  int32_t* order = (int32_t*)((char*)table + sizeof(shv::BatchHeader) + (size_t)n_scenes * sizeof(shv::BatchScene));
  int32_t* eorder = order + n_scenes;
  int64_t tf = 0;
  for (int32_t i = 0; i < n_scenes; ++i) {
    const shv_scene& in = scenes[i];
    const shv_params* prm = &in.params;
    shv_status st = check_params(prm);
    if (st == SHV_OK) st = no_quadrature(prm);
    if (st == SHV_OK) st = check_sizes(in.P, in.S);
    const char* what = nullptr;
    if (st == SHV_OK && in.P > 0) {
      if (!in.points) what = "points";
      else if (!in.normals) what = "normals";
      else if (!in.albedo) what = "albedo";
      else if (!in.light) what = "light";
      else if (!in.vis) what = "vis";
      else if (!in.radiance) what = "radiance";
      else if (!in.saved) what = "saved";
      else if (in.S > 0 && !in.spheres) what = "spheres";
      if (what) st = set_error(SHV_ERR_INVALID_ARG, "%s is NULL", what);
      else if (in.S > 0 && (((uintptr_t)in.spheres) & 15u)) st = set_error(SHV_ERR_INVALID_ARG, "spheres misaligned");
    }
    if (st == SHV_OK && in.P > 0) st = check_saved(in.saved, in.saved_bytes, shv_render_saved_floats(in.P, prm), true);
    if (st == SHV_OK) st = check_ws(in.ws, in.ws_bytes, in.P > 0 ? shv_workspace_bytes(in.P, in.S, prm) : 0);
    if (st == SHV_OK && !(in.range_begin == 0 && in.range_end == 0)) {
      const int64_t a = in.range_begin, e = in.range_end;
      if (a < 0 || a > e || e > in.P || a % SHV_RANGE_ALIGN || (e != in.P && e % SHV_RANGE_ALIGN))
        st = set_error(SHV_ERR_INVALID_ARG,
                       "receiver range [%lld, %lld) invalid for P = %lld (ends must be multiples of %d or P)",
                       (long long)a, (long long)e, (long long)in.P, SHV_RANGE_ALIGN);
    }
    if (st != SHV_OK) {
      const std::string msg = g_last_error;
      return set_error(st, "scene %d: %s", (int)i, msg.c_str());
    }
    shv::BatchScene b{};
    const int nb = prm->n_bands;
    const int64_t N = (int64_t)nb * nb;
    b.points = in.points;
    b.normals = in.normals;
    b.albedo = in.albedo;
    b.spheres = in.spheres;
    b.light = in.light;
    b.grad_radiance = in.grad_radiance;
    b.vis = in.vis;
    b.radiance = in.radiance;
    b.saved = in.saved;
    b.grad_points = in.grad_points;
    b.grad_normals = in.grad_normals;
    b.grad_albedo = in.grad_albedo;
    b.grad_spheres = in.S > 0 ? in.grad_spheres : nullptr;
    b.grad_light = in.grad_light;
    b.P = in.P;
    b.S = in.S;
    b.nb = nb;
    b.k = prm->n_squarings;
    b.eps = prm->eps;
    b.flags = prm->flags;
    const shv::Split spf = shv::fwd_split(in.P, in.S), spb = shv::bwd_split(in.P, in.S);
    b.nchunks_f = spf.nchunks;
    b.chunk_f = spf.chunk;
    b.nchunks_b = spb.nchunks;
    b.chunk_b = spb.chunk;
    b.four_waves = shv::exp_four_waves(nb, in.P, prm->flags, true) ? 1 : 0;
    b.pair_tiles = shv::pair_blocks(in.P);
    b.exp_blocks = b.four_waves ? (in.P + 63) / 64 : shv::point_blocks(in.P);
    // receiver range of this call (whole scene by default)
    const int64_t r0 = in.range_begin, r1 = (in.range_begin == 0 && in.range_end == 0) ? in.P : in.range_end;
    const int64_t eb = b.four_waves ? 64 : SHV_BLOCK;  // receivers per exponential block
    b.tile0 = r0 / 64;
    b.range_tiles = (r1 + 63) / 64 - r0 / 64;
    b.exp_block0 = r0 / eb;
    // the same workspace carving as the single-scene render entry points
    RenderBwdWs L;
    render_bwd_bytes(in.P, in.S, nb, &L);
    char* ws = (char*)in.ws;
    b.Fpart = (float*)ws;
    b.M = in.saved ? in.saved + (1 + (int64_t)prm->n_squarings * N) * in.P : nullptr;
    b.W = (float*)(ws + L.W);
    b.gp = (float*)(ws + L.gp);
    b.gs = (float*)(ws + L.gs);
    b.lp = (float*)(ws + L.lp);
    const bool need_pair = in.P > 0 && (in.grad_points || b.grad_spheres);
    b.fin_pts = (need_pair && in.grad_points) ? (int32_t)((3 * in.P + SHV_BLOCK - 1) / SHV_BLOCK) : 0;
    b.fin_cols_s = b.grad_spheres ? (int32_t)(4 * in.S) : 0;
    b.fin_cols_l = in.grad_light ? (int32_t)N : 0;
    b.n_pair_f = in.P > 0 ? b.range_tiles * spf.nchunks : 0;
    b.n_pair_b = in.P > 0 ? b.range_tiles * spb.nchunks : 0;
    b.n_exp = in.P > 0 ? (r1 + eb - 1) / eb - b.exp_block0 : 0;
    b.n_fin = in.defer_reductions ? 0 : (int64_t)b.fin_pts + (b.fin_cols_s + 15) / 16 + (b.fin_cols_l + 15) / 16;
    const int lay = b.four_waves;
    b.off_pair_f = h.total_pair_f[nb];
    b.off_pair_b = h.total_pair_b[nb];
    b.off_exp = h.total_exp[lay][nb];
    b.off_fin = tf;
    h.total_pair_f[nb] += b.n_pair_f;
    h.total_pair_b[nb] += b.n_pair_b;
    h.total_exp[lay][nb] += b.n_exp;
    tf += b.n_fin;
    h.grp_count[nb] += 1;
    h.egrp_count[lay][nb] += 1;
    out[i] = b;
  }
  h.total_fin = tf;
  int32_t pos = 0, epos = 0;
  for (int nb = 0; nb <= SHV_MAX_BANDS_API; ++nb) {
    h.grp_begin[nb] = pos;
    for (int32_t i = 0; i < n_scenes; ++i)
      if (out[i].nb == nb) order[pos++] = i;
  }
  for (int lay = 0; lay < 2; ++lay) {
    for (int nb = 0; nb <= SHV_MAX_BANDS_API; ++nb) {
      h.egrp_begin[lay][nb] = epos;
      for (int32_t i = 0; i < n_scenes; ++i)
        if (out[i].nb == nb && out[i].four_waves == lay) eorder[epos++] = i;
    }
  }
  *(shv::BatchHeader*)table = h;
  return SHV_OK;
}

shv_status shv_batch_table_grid(const void* table, shv_batch_grid* grid) {
  if (!table) return set_error(SHV_ERR_INVALID_ARG, "table is NULL");
  if (!grid) return set_error(SHV_ERR_INVALID_ARG, "grid is NULL");
  const shv::BatchHeader& h = *(const shv::BatchHeader*)table;
  shv_batch_grid g{};
  for (int nb = 1; nb <= SHV_MAX_BANDS_API; ++nb) {
    g.pair_fwd[nb] = h.total_pair_f[nb];
    g.pair_bwd[nb] = h.total_pair_b[nb];
    g.exp[0][nb] = h.total_exp[0][nb];
    g.exp[1][nb] = h.total_exp[1][nb];
  }
  g.finalize = h.total_fin;
  *grid = g;
  return SHV_OK;
}

static shv_status check_grid(const shv_batch_grid* g) {
  SHV_TRY(need(g, "grid"));
  const int64_t lim = 0x7fffffff;
  auto bad = [&](int64_t x) { return x < 0 || x > lim; };
  if (g->pair_fwd[0] || g->pair_bwd[0] || g->exp[0][0] || g->exp[1][0])
    return set_error(SHV_ERR_INVALID_ARG, "grid entries for 0 bands must be 0");
  for (int nb = 1; nb <= SHV_MAX_BANDS_API; ++nb)
    if (bad(g->pair_fwd[nb]) || bad(g->pair_bwd[nb]) || bad(g->exp[0][nb]) || bad(g->exp[1][nb]))
      return set_error(SHV_ERR_INVALID_ARG, "grid entry for %d bands outside [0, 2^31)", nb);
  if (bad(g->finalize)) return set_error(SHV_ERR_INVALID_ARG, "finalize grid outside [0, 2^31)");
  return SHV_OK;
}

// Timing name of a batched launch: phase, band count and (exponential
// phases) the one-wave layout, e.g. "batch_pair_bwd/n8",
// "batch_exp_shade_fwd/n4/one".
static const char* batch_name(int phase, int nb, int lay) {
  static const std::vector<std::string> table = [] {
    static const char* base[4] = {"batch_pair_fwd", "batch_exp_shade_fwd", "batch_exp_shade_bwd", "batch_pair_bwd"};
    std::vector<std::string> t;
    for (int p = 0; p < 4; ++p)
      for (int n = 0; n <= SHV_MAX_BANDS_API; ++n)
        for (int l = 0; l < 2; ++l)
          t.push_back(std::string(base[p]) + "/n" + std::to_string(n) + ((p == 1 || p == 2) && l == 0 ? "/one" : ""));
    return t;
  }();
  return table[((size_t)phase * (SHV_MAX_BANDS_API + 1) + nb) * 2 + lay].c_str();
}

// Launches of one phase for every group with a non-empty grid.
static shv_status batched_phase(int phase, const shv_batch_grid* g, const void* table, hipStream_t stream) {
  for (int nb = 1; nb <= SHV_MAX_BANDS_API; ++nb) {
    if (phase == 0 || phase == 3) {
      const int64_t blocks = phase == 0 ? g->pair_fwd[nb] : g->pair_bwd[nb];
      if (blocks > 0)
        SHV_TRY(launch(batch_name(phase, nb, 1), stream,
                       [&] { return shv::launch_batch_nb(nb, phase, false, table, blocks, stream); }));
      continue;
    }
    for (int lay = 1; lay >= 0; --lay) {
      const int64_t blocks = g->exp[lay][nb];
      if (blocks > 0)
        SHV_TRY(launch(batch_name(phase, nb, lay), stream,
                       [&] { return shv::launch_batch_nb(nb, phase, lay == 1, table, blocks, stream); }));
    }
  }
  return SHV_OK;
}

shv_status sh_render_batched_forward(const void* table, const shv_batch_grid* grid, hipStream_t stream) {
  SHV_TRY(check_device());
  SHV_TRY(need(table, "table"));
  SHV_TRY(check_grid(grid));
  SHV_TRY(batched_phase(0, grid, table, stream));
  SHV_TRY(batched_phase(1, grid, table, stream));
  return SHV_OK;
}

shv_status sh_render_batched_backward(const void* table, const shv_batch_grid* grid, hipStream_t stream) {
  SHV_TRY(check_device());
  SHV_TRY(need(table, "table"));
  SHV_TRY(check_grid(grid));
  SHV_TRY(batched_phase(2, grid, table, stream));
  SHV_TRY(batched_phase(3, grid, table, stream));
  if (grid->finalize > 0)
    SHV_TRY(launch("batch_finalize", stream,
                   [&] { return shv::launch_batch_finalize(table, grid->finalize, stream); }));
  return SHV_OK;
}

shv_status sh_solve_batched(const void* table, const shv_batch_grid* grid, hipStream_t stream) {
  SHV_TRY(need(table, "table"));
  SHV_TRY(check_grid(grid));
  SHV_TRY(check_device());
  for (int phase = 0; phase < 4; ++phase) SHV_TRY(batched_phase(phase, grid, table, stream));
  if (grid->finalize > 0)
    SHV_TRY(launch("batch_finalize", stream,
                   [&] { return shv::launch_batch_finalize(table, grid->finalize, stream); }));
  return SHV_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ graphs

struct shv_graph {
  static constexpr int kSlots = 4;
  int device = -1;
  int32_t max_scenes = 0;
  uint32_t flags = 0;
  size_t table_bytes = 0;
  void* table_dev = nullptr;            // device copy of the table the graph reads
  void* staging[kSlots] = {};           // pinned host tables
  hipEvent_t staged[kSlots] = {};       // recorded after each slot's copy
  bool slot_pending[kSlots] = {};
  int next_slot = 0;
  hipEvent_t done = nullptr;            // recorded after the last launch
  bool launched = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  shv_batch_grid captured{};            // block counts the graph was captured with
  // one entry per launch, in launch order: its group and its node
  struct Node {
    int kind;   // 0..3 batched phase, 4 finalize
    int nb;
    int lay;
    hipGraphNode_t node;
    hipKernelNodeParams params;
    bool enabled = true;  // disabled while a launch's batch has no work in the node's group
  };
  std::vector<Node> nodes;
  const void* arg_table = nullptr;      // storage of the kernels' one argument
  void* args[1] = {nullptr};
};

namespace {

int64_t grid_entry(const shv_batch_grid& g, int kind, int nb, int lay) {
  if (kind == 4) return g.finalize;
  if (kind == 0) return g.pair_fwd[nb];
  if (kind == 3) return g.pair_bwd[nb];
  return g.exp[lay][nb];
}

void graph_free(shv_graph* g) {
  if (!g) return;
  if (g->done) (void)hipEventSynchronize(g->done);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (int i = 0; i < shv_graph::kSlots; ++i) {
    if (g->staged[i]) (void)hipEventDestroy(g->staged[i]);
    if (g->staging[i]) (void)hipHostFree(g->staging[i]);
  }
  if (g->done) (void)hipEventDestroy(g->done);
  if (g->table_dev) (void)hipFree(g->table_dev);
  delete g;
}

#define SHV_HIP(call, what)                                                                    \
  do {                                                                                         \
    hipError_t _e = (call);                                                                    \
    if (_e != hipSuccess) return set_error(SHV_ERR_HIP, "%s: %s", what, hipGetErrorString(_e)); \
  } while (0)

// Captures the launches of sh_solve_batched for the groups of g->captured,
// in the order sh_solve_batched issues them, and pairs each launch with its
// node by walking the captured chain from its root.
shv_status graph_capture(shv_graph* g) {
  hipStream_t cs = nullptr;
  SHV_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  std::vector<shv_graph::Node> order;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  shv_status st = SHV_OK;
  if (e == hipSuccess) {
    g_capturing = true;
    const shv_batch_grid& cap = g->captured;
    for (int phase = 0; phase < 4 && st == SHV_OK; ++phase) {
      for (int nb = 1; nb <= SHV_MAX_BANDS_API && st == SHV_OK; ++nb) {
        if (phase == 0 || phase == 3) {
          const int64_t blocks = phase == 0 ? cap.pair_fwd[nb] : cap.pair_bwd[nb];
          if (blocks > 0) {
            st = launch("graph", cs, [&] { return shv::launch_batch_nb(nb, phase, false, g->table_dev, blocks, cs); });
            order.push_back({phase, nb, 0, nullptr, {}});
          }
          continue;
        }
        for (int lay = 1; lay >= 0 && st == SHV_OK; --lay) {
          if (cap.exp[lay][nb] > 0) {
            st = launch("graph", cs,
                        [&] { return shv::launch_batch_nb(nb, phase, lay == 1, g->table_dev, cap.exp[lay][nb], cs); });
            order.push_back({phase, nb, lay, nullptr, {}});
          }
        }
      }
    }
    if (st == SHV_OK && cap.finalize > 0) {
      st = launch("graph", cs, [&] { return shv::launch_batch_finalize(g->table_dev, cap.finalize, cs); });
      order.push_back({4, 0, 0, nullptr, {}});
    }
    g_capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    g->graph = graph;
    if (st == SHV_OK && e2 != hipSuccess)
      st = set_error(SHV_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e2));
  } else {
    st = set_error(SHV_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  }
  (void)hipStreamDestroy(cs);
  SHV_TRY(st);
  if (!g->graph) return set_error(SHV_ERR_HIP, "capture produced no graph");
  // walk the chain: one root, each node with at most one dependent
  hipGraphNode_t cur = nullptr;
  size_t nroot = 1;
  SHV_HIP(hipGraphGetRootNodes(g->graph, &cur, &nroot), "hipGraphGetRootNodes");
  if (nroot != 1) return set_error(SHV_ERR_HIP, "captured graph has %zu roots, expected 1", nroot);
  for (size_t i = 0; i < order.size(); ++i) {
    if (!cur) return set_error(SHV_ERR_HIP, "captured graph has %zu nodes, expected %zu", i, order.size());
    hipGraphNodeType ty;
    SHV_HIP(hipGraphNodeGetType(cur, &ty), "hipGraphNodeGetType");
    if (ty != hipGraphNodeTypeKernel) return set_error(SHV_ERR_HIP, "captured node %zu is not a kernel", i);
    order[i].node = cur;
    SHV_HIP(hipGraphKernelNodeGetParams(cur, &order[i].params), "hipGraphKernelNodeGetParams");
    size_t ndep = 0;
    SHV_HIP(hipGraphNodeGetDependentNodes(cur, nullptr, &ndep), "hipGraphNodeGetDependentNodes");
    if (ndep > 1) return set_error(SHV_ERR_HIP, "captured node %zu has %zu dependents", i, ndep);
    hipGraphNode_t nxt = nullptr;
    if (ndep == 1) {
      size_t one = 1;
      SHV_HIP(hipGraphNodeGetDependentNodes(cur, &nxt, &one), "hipGraphNodeGetDependentNodes");
    }
    cur = nxt;
  }
  if (cur) return set_error(SHV_ERR_HIP, "captured graph has more nodes than launches");
  g->arg_table = g->table_dev;
  g->args[0] = &g->arg_table;
  for (auto& n : order) {
    n.params.kernelParams = g->args;
    n.params.extra = nullptr;
  }
  g->nodes = std::move(order);
  SHV_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  return SHV_OK;
}

}  // namespace

extern "C" {

shv_status shv_graph_create(const shv_batch_grid* groups, int32_t max_scenes, uint32_t flags, shv_graph** out) {
  SHV_TRY(need(out, "graph"));
  *out = nullptr;
  SHV_TRY(check_grid(groups));
  if (max_scenes < 1 || max_scenes > (1 << 20))
    return set_error(SHV_ERR_INVALID_ARG, "max_scenes=%d outside [1, 2^20]", max_scenes);
  if (flags & ~SHV_GRAPH_FIXED_GRID) return set_error(SHV_ERR_INVALID_ARG, "unknown graph flags 0x%x", flags);
  bool any = groups->finalize > 0;
  for (int nb = 1; nb <= SHV_MAX_BANDS_API; ++nb)
    any = any || groups->pair_fwd[nb] > 0 || groups->pair_bwd[nb] > 0 || groups->exp[0][nb] > 0 ||
          groups->exp[1][nb] > 0;
  if (!any) return set_error(SHV_ERR_INVALID_ARG, "groups selects no launch");
  SHV_TRY(check_device());
  shv_graph* g = new shv_graph();
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  g->device = dev;
  g->max_scenes = max_scenes;
  g->flags = flags;
  g->captured = *groups;
  g->table_bytes = shv::batch_table_bytes(max_scenes);
  if (e == hipSuccess) e = hipMalloc(&g->table_dev, g->table_bytes);
  for (int i = 0; i < shv_graph::kSlots && e == hipSuccess; ++i) {
    e = hipHostMalloc(&g->staging[i], g->table_bytes, hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->staged[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->done, hipEventDisableTiming);
  if (e == hipSuccess) {
    // an empty table until the first launch writes one
    shv::BatchHeader h{};
    e = hipMemcpy(g->table_dev, &h, sizeof(h), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    const shv_status st = set_error(SHV_ERR_HIP, "shv_graph_create: %s", hipGetErrorString(e));
    graph_free(g);
    return st;
  }
  const shv_status st = graph_capture(g);
  if (st != SHV_OK) {
    const std::string msg = g_last_error;
    graph_free(g);
    return set_error(st, "shv_graph_create: %s", msg.c_str());
  }
  *out = g;
  return SHV_OK;
}

shv_status shv_graph_launch(shv_graph* g, const shv_scene* scenes, int32_t n_scenes, hipStream_t stream) {
  SHV_TRY(need(g, "graph"));
  if (n_scenes < 0 || n_scenes > g->max_scenes)
    return set_error(SHV_ERR_INVALID_ARG, "n_scenes=%d outside [0, %d]", n_scenes, g->max_scenes);
  int dev = -1;
  SHV_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != g->device) return set_error(SHV_ERR_INVALID_ARG, "graph belongs to device %d, current is %d", g->device, dev);
  const int slot = g->next_slot;
  if (g->slot_pending[slot]) SHV_HIP(hipEventSynchronize(g->staged[slot]), "hipEventSynchronize");
  g->slot_pending[slot] = false;
  SHV_TRY(shv_batch_table_build(scenes, n_scenes, g->staging[slot], g->table_bytes));
  shv_batch_grid need_grid;
  SHV_TRY(shv_batch_table_grid(g->staging[slot], &need_grid));
  const bool fixed = (g->flags & SHV_GRAPH_FIXED_GRID) != 0;
  // every group with work must be in the graph (and fit it with fixed grids)
  struct Group {
    const char* name;
    int kind, lay;  // as in grid_entry
  };
  static const Group kGroups[4] = {
      {"pair forward", 0, 0}, {"one-wave exponential", 1, 0}, {"four-wave exponential", 1, 1}, {"pair adjoint", 3, 0}};
  for (int nb = 0; nb <= SHV_MAX_BANDS_API; ++nb) {
    for (const Group& gr : kGroups) {
      const int64_t want = grid_entry(need_grid, gr.kind, nb, gr.lay);
      const int64_t have = grid_entry(g->captured, gr.kind, nb, gr.lay);
      if (want > 0 && (have <= 0 || (fixed && want > have)))
        return set_error(SHV_ERR_UNSUPPORTED, "batch needs %lld blocks in the %s group of %d bands; the graph holds %lld",
                         (long long)want, gr.name, nb, (long long)have);
    }
  }
  if (need_grid.finalize > 0 && (g->captured.finalize <= 0 || (fixed && need_grid.finalize > g->captured.finalize)))
    return set_error(SHV_ERR_UNSUPPORTED, "batch needs %lld finalize blocks; the graph holds %lld",
                     (long long)need_grid.finalize, (long long)g->captured.finalize);
  // Nodes of groups without work are disabled (a disabled node is an empty
  // node: it keeps its place in the chain and launches nothing), the others
  // are set to their exact block counts unless the grids are fixed.
  bool any = false;
  for (auto& n : g->nodes) {
    const int64_t want = grid_entry(need_grid, n.kind, n.nb, n.lay);
    const bool on = want > 0;
    if (on != n.enabled) {
      SHV_HIP(hipGraphNodeSetEnabled(g->exec, n.node, on ? 1u : 0u), "hipGraphNodeSetEnabled");
      n.enabled = on;
    }
    any = any || on;
    if (on && !fixed && n.params.gridDim.x != (unsigned)want) {
      n.params.gridDim = dim3((unsigned)want, 1, 1);
      SHV_HIP(hipGraphExecKernelNodeSetParams(g->exec, n.node, &n.params), "hipGraphExecKernelNodeSetParams");
    }
  }
  if (!any) return SHV_OK;  // an empty batch: nothing to enqueue
  if (g->launched) SHV_HIP(hipStreamWaitEvent(stream, g->done, 0), "hipStreamWaitEvent");
  const size_t bytes = shv::batch_table_bytes(n_scenes);
  SHV_HIP(hipMemcpyAsync(g->table_dev, g->staging[slot], bytes, hipMemcpyHostToDevice, stream), "hipMemcpyAsync");
  SHV_HIP(hipEventRecord(g->staged[slot], stream), "hipEventRecord");
  g->slot_pending[slot] = true;
  g->next_slot = (slot + 1) % shv_graph::kSlots;
  SHV_TRY(launch("graph_solve", stream, [&] { return hipGraphLaunch(g->exec, stream); }));
  SHV_HIP(hipEventRecord(g->done, stream), "hipEventRecord");
  g->launched = true;
  return SHV_OK;
}

shv_status shv_graph_destroy(shv_graph* g) {
  graph_free(g);
  return SHV_OK;
}

shv_status shv_profile_enable(int enable, int32_t capacity) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!enable) {
    g_prof_on = false;
    return SHV_OK;
  }
  if (capacity < 0) return set_error(SHV_ERR_INVALID_ARG, "negative capacity");
  // Resuming (2) never grows the pool: creating events inside a timed region
  // would be timed with it.
  while (enable != 2 && (int64_t)g_prof.size() < capacity) {
    ProfRec r{nullptr, nullptr, nullptr};
    hipError_t e1 = hipEventCreate(&r.a);
    hipError_t e2 = hipEventCreate(&r.b);
    if (e1 != hipSuccess || e2 != hipSuccess) return set_error(SHV_ERR_HIP, "hipEventCreate failed");
    g_prof.push_back(r);
  }
  if (enable != 2) {  // 2 resumes the current collection
    g_prof_used = 0;
    g_prof_untimed.clear();
  }
  g_prof_on = true;
  return SHV_OK;
}

int64_t shv_profile_report(char* buf, int64_t len) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  std::map<std::string, std::pair<int64_t, double>> agg;
  for (int64_t i = 0; i < g_prof_used; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, g_prof[i].a, g_prof[i].b) != hipSuccess) ms = -1.0f;
    auto& a = agg[g_prof[i].name];
    a.first += 1;
    a.second += ms;
  }
  std::string out;
  char line[256];
  for (auto& kv : agg) {
    snprintf(line, sizeof(line), "%s %lld %.6f\n", kv.first.c_str(), (long long)kv.second.first, kv.second.second);
    out += line;
  }
  for (auto& kv : g_prof_untimed) {
    snprintf(line, sizeof(line), "%s:untimed %lld 0\n", kv.first.c_str(), (long long)kv.second);
    out += line;
  }
  if (buf && len > 0) {
    const int64_t n = std::min<int64_t>(len - 1, (int64_t)out.size());
    std::memcpy(buf, out.data(), (size_t)n);
    buf[n] = '\0';
  }
  return (int64_t)out.size() + 1;
}

}  // extern "C"
