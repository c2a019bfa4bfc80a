// Rasterisation of the shaded mesh (Sec. 3.4, Eq. 14) and its adjoint.
//
// I_R = R(B(x_0), ..., B(x_n), P): the vertices are projected by the 3 x 4
// camera matrix P ((u, v, w) = P [x; 1], pixel coordinates (u / w, v / w),
// depth w); each pixel centre (i + 0.5, j + 0.5) takes the nearest triangle
// covering it (edge functions over the doubled signed area all >= 0, depth
// 1 / sum_k lambda_k / w_k, ties to the lower face index) and interpolates
// the vertices' radiance with the perspective-correct weights
// b_k = (lambda_k / w_k) / sum_j (lambda_j / w_j).  Uncovered pixels are 0.
//
// The coverage and depth decisions pick integers from floating-point values,
// so they are taken with one rounding per operation (no contraction into
// FMAs, correctly rounded division) in a fixed order; the same decisions can
// then be reproduced exactly in FP32 elsewhere.
//
// Forward: a setup pass writes one record per face (projected corners,
// depths, area, pixel bounding box; faces behind the camera, degenerate or
// with an index outside [0, V) get an empty box) and counts, per 8 x 8
// pixel tile, the faces whose box meets it; faces meeting more than
// kMaxBinTiles tiles go to one shared list instead.  The counting atomics
// also give each face its slot in each tile's list; a scan turns the counts
// into offsets and a binning pass scatters the faces to their slots (the
// order within a list varies from run to run).  Then one wave
// per (tile, chunk of kChunk entries of its list and the shared list) tests its
// 8 x 8 pixels against the chunk's faces, staged in LDS, and merges each
// pixel's smallest (depth, face index) pair into a 64-bit depth buffer with
// an atomic; the result does not depend on the order of the lists or of the
// merges.  A per-pixel pass then writes the face and the interpolated
// radiance.
//
// Adjoint (through the winning triangle's weights; which triangle wins is
// piecewise constant): sixteen lanes per face walk the face's bounding box, takes
// the pixels that face won, and sums their contributions to the face's three
// corners (radiance, pixel x, pixel y, depth) in a fixed order; a per-vertex
// pass then sums the corners of its incident faces in the incidence list's
// order and chains through the projection.  No atomics: every sum has a
// fixed order.

#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "shv_config.h"
#include "shv_launch.h"

namespace shv {

constexpr float kRasterMinW = 1e-6f;
constexpr int kTile = 8;                 // one wave per 8 x 8 tile
constexpr int kTileThreads = kTile * kTile;
// Entries of a tile's list (and the shared list after it) per wave of the
// depth-buffer pass: short chunks give many short waves, which hide the
// latency of the per-pixel divisions better than few long ones.
constexpr int kChunk = 8;
constexpr int kMaxBinTiles = 16;

struct alignas(16) FaceRec {
  float x[3], y[3], w[3], area;
  int32_t i0, i1, j0, j1;
  int32_t pad[2];
};
static_assert(sizeof(FaceRec) == 64, "face record is one 64-byte line");

// (u, v, w) of one vertex, each ((P_r0 x + P_r1 y) + P_r2 z) + P_r3.
__device__ __forceinline__ void project_vertex(const float* __restrict__ P, float x, float y, float z, float& u,
                                               float& v, float& w) {
  u = ((P[0] * x + P[1] * y) + P[2] * z) + P[3];
  v = ((P[4] * x + P[5] * y) + P[6] * z) + P[7];
  w = ((P[8] * x + P[9] * y) + P[10] * z) + P[11];
}

__device__ __forceinline__ float edge_fn(float ax, float ay, float bx, float by, float px, float py) {
  return (ax - px) * (by - py) - (bx - px) * (ay - py);
}

__device__ __forceinline__ int clamp_floor(float v, int lo, int hi) {
  if (!(v > (float)lo)) return lo;  // also NaN
  if (v >= (float)hi) return hi;
  return (int)floorf(v);
}

// Tile range of a record's box; false for an empty box.
__device__ __forceinline__ bool tile_range(const FaceRec& r, int& tx0, int& tx1, int& ty0, int& ty1) {
  if (r.i0 > r.i1 || r.j0 > r.j1) return false;
  tx0 = r.i0 / kTile;
  tx1 = r.i1 / kTile;
  ty0 = r.j0 / kTile;
  ty1 = r.j1 / kTile;
  return true;
}

// With counts != NULL also bins: counts[tile] += 1 for each tile a binned
// face meets, and the face gets a distinct slot in that tile's list
// (slots[kMaxBinTiles f + k] for its k-th tile, row by row); a face meeting
// more tiles is appended to big_list.  The block first counts its faces'
// tiles in an LDS hash table (a block's faces are usually neighbours and meet
// few tiles), then reserves each tile's run of slots with one global atomic;
// when the table is full a face's tile takes its slot from the global counter
// directly.
constexpr int kBinHash = 1024;  // LDS hash slots per block

__device__ __forceinline__ int bin_hash(int tile) { return (int)(((uint32_t)tile * 0x9E3779B1u) >> 22); }

struct SetupShared {
  int32_t key[kBinHash];  // tile + 1, 0 = empty
  int32_t cnt[kBinHash];
  int32_t base[kBinHash];
};
__global__ __launch_bounds__(SHV_BLOCK) void k_raster_setup(const float* __restrict__ verts, int64_t V,
                                                            const int32_t* __restrict__ faces, int64_t T,
                                                            RasterCam cam, FaceRec* __restrict__ rec,
                                                            int tiles_x, int32_t* __restrict__ counts,
                                                            int32_t* __restrict__ slots,
                                                            int32_t* __restrict__ big_count,
                                                            int32_t* __restrict__ big_list) {
  __shared__ SetupShared sh;
  const int64_t f = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  const bool live = f < T;
  FaceRec r;
  r.i0 = 0;
  r.i1 = -1;
  r.j0 = 0;
  r.j1 = -1;
  r.pad[0] = r.pad[1] = 0;
  r.area = 0.0f;
  if (live) {
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      const int32_t vi = faces[3 * f + k];
      if (vi < 0 || vi >= V) {
        ok = false;
        r.x[k] = r.y[k] = r.w[k] = 0.0f;
        continue;
      }
      float u, v, w;
      project_vertex(cam.P, verts[vi], verts[V + vi], verts[2 * V + vi], u, v, w);
      r.x[k] = u / w;
      r.y[k] = v / w;
      r.w[k] = w;
      ok = ok && (w > kRasterMinW);
    }
    r.area = (r.x[1] - r.x[0]) * (r.y[2] - r.y[0]) - (r.x[2] - r.x[0]) * (r.y[1] - r.y[0]);
    ok = ok && (r.area != 0.0f) && isfinite(r.area);
    if (ok) {
      const float xmin = fminf(fminf(r.x[0], r.x[1]), r.x[2]), xmax = fmaxf(fmaxf(r.x[0], r.x[1]), r.x[2]);
      const float ymin = fminf(fminf(r.y[0], r.y[1]), r.y[2]), ymax = fmaxf(fmaxf(r.y[0], r.y[1]), r.y[2]);
      // pixel i is a candidate when xmin - 1 <= i <= xmax (a superset of the
      // centres i + 0.5 inside [xmin, xmax]); the coverage test decides.
      r.i0 = clamp_floor(xmin - 1.0f, 0, cam.width - 1);
      r.i1 = clamp_floor(xmax, -1, cam.width - 1);
      r.j0 = clamp_floor(ymin - 1.0f, 0, cam.height - 1);
      r.j1 = clamp_floor(ymax, -1, cam.height - 1);
      if (xmax < -1.0f || ymax < -1.0f) r.i1 = -1;
    }
    rec[f] = r;
  }
  if (!counts) return;  // the adjoint's setup: records only (uniform over the grid)
  for (int h = threadIdx.x; h < kBinHash; h += SHV_BLOCK) {
    sh.key[h] = 0;
    sh.cnt[h] = 0;
  }
  __syncthreads();
  int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1;
  bool binned = false;
  if (live && tile_range(r, tx0, tx1, ty0, ty1)) {
    if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) > kMaxBinTiles) {
      big_list[atomicAdd(big_count, 1)] = (int32_t)f;
    } else {
      binned = true;
      // per tile: the rank within the block's count (>= 0), or, with the
      // table full, -1 - the slot taken from the global counter
      int k = 0;
      for (int ty = ty0; ty <= ty1; ++ty) {
        for (int tx = tx0; tx <= tx1; ++tx) {
          const int tile = ty * tiles_x + tx;
          int h = bin_hash(tile), found = -1;
          for (int probe = 0; probe < kBinHash; ++probe) {
            const int prev = atomicCAS(&sh.key[h], 0, tile + 1);
            if (prev == 0 || prev == tile + 1) {
              found = h;
              break;
            }
            h = (h + 1) & (kBinHash - 1);
          }
          slots[kMaxBinTiles * f + k++] =
              found >= 0 ? atomicAdd(&sh.cnt[found], 1) : -1 - atomicAdd(&counts[tile], 1);
        }
      }
    }
  }
  __syncthreads();
  for (int h = threadIdx.x; h < kBinHash; h += SHV_BLOCK) {
    const int key = sh.key[h];
    if (key != 0) sh.base[h] = atomicAdd(&counts[key - 1], sh.cnt[h]);
  }
  __syncthreads();
  if (!binned) return;
  int k = 0;
  for (int ty = ty0; ty <= ty1; ++ty) {
    for (int tx = tx0; tx <= tx1; ++tx) {
      int32_t* sl = &slots[kMaxBinTiles * f + k++];
      const int v = *sl;
      if (v < 0) {
        *sl = -1 - v;
        continue;
      }
      const int tile = ty * tiles_x + tx;
      int h = bin_hash(tile);
      for (int probe = 0; probe < kBinHash && sh.key[h] != tile + 1; ++probe) h = (h + 1) & (kBinHash - 1);
      *sl = sh.base[h] + v;
    }
  }
}

// Exclusive scans, one block: the tile counts into offsets[0 .. n], and the
// tiles' chunk counts (kChunk entries of the tile's list and the shared list per
// chunk) into chunk_off[0 .. n].  The chunk offsets are 64-bit: every tile
// scans the whole shared list, so their total grows as tiles x shared-list
// length and passes 2^31 on large images with many large faces.  The counts
// go through LDS in segments of kScanSeg with a running carry: a coalesced
// load of the segment, a run of kScanPer consecutive counts summed by each
// thread, the run totals scanned in log2 steps, each thread's run of offsets
// back into LDS, and a coalesced store of the segment.  Entry t of a segment
// sits at t + t / kScanPer in LDS, so that the runs' accesses (stride
// kScanPer + 1 words) fall in distinct banks.
constexpr int kScanPer = 16;
constexpr int kScanSeg = kScanPer * SHV_BLOCK;

__global__ __launch_bounds__(SHV_BLOCK) void k_raster_scan(const int32_t* __restrict__ counts, int n,
                                                           const int32_t* __restrict__ big_count,
                                                           int32_t* __restrict__ offsets,
                                                           int64_t* __restrict__ chunk_off) {
  __shared__ int32_t seg[kScanSeg + kScanSeg / kScanPer];
  __shared__ int64_t cseg[kScanSeg + kScanSeg / kScanPer];
  __shared__ int32_t part[2][SHV_BLOCK];
  __shared__ int64_t cpart[2][SHV_BLOCK];
  const int nbig = *big_count;
  const int x = threadIdx.x;
  int32_t carry = 0;
  int64_t ccarry = 0;
  for (int base = 0; base < n; base += kScanSeg) {
    const int m = min(kScanSeg, n - base);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int t = k * SHV_BLOCK + x;
      seg[t + t / kScanPer] = t < m ? counts[base + t] : 0;
    }
    __syncthreads();
    int32_t v[kScanPer];
    int32_t sum = 0;
    int64_t csum = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = seg[x * (kScanPer + 1) + k];
      sum += v[k];
      csum += x * kScanPer + k < m ? ((int64_t)v[k] + nbig + kChunk - 1) / kChunk : 0;
    }
    int cur = 0;
    part[0][x] = sum;
    cpart[0][x] = csum;
    __syncthreads();
    for (int d = 1; d < SHV_BLOCK; d <<= 1) {
      const bool has = x >= d;
      const int32_t a = part[cur][x] + (has ? part[cur][x - d] : 0);
      const int64_t b = cpart[cur][x] + (has ? cpart[cur][x - d] : 0);
      part[cur ^ 1][x] = a;
      cpart[cur ^ 1][x] = b;
      cur ^= 1;
      __syncthreads();
    }
    int32_t run = carry + part[cur][x] - sum;  // exclusive prefixes of this thread's run
    int64_t crun = ccarry + cpart[cur][x] - csum;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      seg[x * (kScanPer + 1) + k] = run;
      cseg[x * (kScanPer + 1) + k] = crun;
      run += v[k];
      crun += x * kScanPer + k < m ? ((int64_t)v[k] + nbig + kChunk - 1) / kChunk : 0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      const int t = k * SHV_BLOCK + x;
      if (t < m) {
        offsets[base + t] = seg[t + t / kScanPer];
        chunk_off[base + t] = cseg[t + t / kScanPer];
      }
    }
    carry += part[cur][SHV_BLOCK - 1];
    ccarry += cpart[cur][SHV_BLOCK - 1];
    __syncthreads();  // seg and part are rewritten by the next segment
  }
  if (x == 0) {
    offsets[n] = carry;
    chunk_off[n] = ccarry;
  }
}

__global__ __launch_bounds__(SHV_BLOCK) void k_raster_bin(const FaceRec* __restrict__ rec, int64_t T, int tiles_x,
                                                          const int32_t* __restrict__ offsets,
                                                          const int32_t* __restrict__ slots,
                                                          int32_t* __restrict__ list) {
  const int64_t f = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (f >= T) return;
  const FaceRec r = rec[f];
  int tx0, tx1, ty0, ty1;
  if (!tile_range(r, tx0, tx1, ty0, ty1) || (tx1 - tx0 + 1) * (ty1 - ty0 + 1) > kMaxBinTiles) return;
  const int64_t cap = (int64_t)kMaxBinTiles * T;
  int k = 0;
  for (int ty = ty0; ty <= ty1; ++ty) {
    for (int tx = tx0; tx <= tx1; ++tx) {
      const int64_t pos = (int64_t)offsets[ty * tiles_x + tx] + slots[kMaxBinTiles * f + k++];
      if (pos >= 0 && pos < cap) list[pos] = (int32_t)f;  // always true; checked all the same
    }
  }
}

struct RasterShared {
  FaceRec recs[kChunk];
  int32_t ids[kChunk];
};

// Coverage and depth of one pixel centre for one face: false if the face does
// not cover it; else its weights' numerators l0, l1, l2 and the depth z.
__device__ __forceinline__ bool cover(const FaceRec& r, int i, int j, float px, float py, float& l0, float& l1,
                                      float& l2, float& z) {
  if (i < r.i0 || i > r.i1 || j < r.j0 || j > r.j1) return false;
  const float e0 = edge_fn(r.x[1], r.y[1], r.x[2], r.y[2], px, py);
  const float e1 = edge_fn(r.x[2], r.y[2], r.x[0], r.y[0], px, py);
  const float e2 = edge_fn(r.x[0], r.y[0], r.x[1], r.y[1], px, py);
  // Exact early rejection: an edge value of the opposite sign to the area and
  // above 2^-100 |area| in magnitude has a quotient by the area below
  // -2^-101, strictly negative (no underflow to -0), so the coverage test
  // below fails for it too.
  const float sg = r.area > 0.0f ? 1.0f : -1.0f;
  const float thr = -(fabsf(r.area) * 0x1p-100f);
  if (sg * e0 < thr || sg * e1 < thr || sg * e2 < thr) return false;
  l0 = e0 / r.area;
  l1 = e1 / r.area;
  l2 = e2 / r.area;
  if (!(l0 >= 0.0f && l1 >= 0.0f && l2 >= 0.0f)) return false;
  z = 1.0f / ((l0 / r.w[0] + l1 / r.w[1]) + l2 / r.w[2]);
  return true;
}

// Waves stride over the chunks of all tiles (chunk_off: the scan of the
// tiles' chunk counts); a chunk is kChunk entries of its tile's list followed by
// the shared list.  Its tile is the last t with chunk_off[t] <= c, found by a
// 64-way search: the wave's lanes probe 64 evenly spaced offsets of the
// interval at once, and the count of probes at or below c (they form a
// prefix, the offsets being non-decreasing) picks the sub-interval.  Each
// round shrinks the interval to at most a 64th, so 4,097 offsets take two
// rounds of dependent loads where a binary search takes twelve.  Each lane keeps
// its pixel's smallest (depth, face) over the chunk and merges it into zbuf
// with one atomic max of the bit-inverted key (depth bits above the face
// index: positive floats order like their bits), which is the lexicographic
// minimum whatever the order of the merges.
__global__ __launch_bounds__(kTileThreads) void k_raster_zbuf(const FaceRec* __restrict__ rec, int64_t T,
                                                              const int32_t* __restrict__ offsets,
                                                              const int64_t* __restrict__ chunk_off,
                                                              const int32_t* __restrict__ list,
                                                              const int32_t* __restrict__ big_count,
                                                              const int32_t* __restrict__ big_list, int width,
                                                              int height, int tiles_x, int tiles,
                                                              unsigned long long* __restrict__ zbuf) {
  __shared__ RasterShared sh;
  const int lane = threadIdx.x;
  const int64_t total = chunk_off[tiles];
  const int nbig = *big_count;
  for (int64_t c = blockIdx.x; c < total; c += gridDim.x) {
    int lo = 0, hi = tiles;  // chunk_off[lo] <= c < chunk_off[hi]
    for (int round = 0; round < 8 && hi - lo > 1; ++round) {  // tiles < 2^24: four rounds suffice
      const int64_t span = hi - lo;
      const int probe = lo + (int)(((int64_t)(lane + 1) * span) >> 6);  // lane 63 probes hi
      const bool le = probe < hi && chunk_off[probe] <= c;
      const int k = __popcll(__ballot(le));  // probes of lanes 0 .. k-1 are <= c, that of lane k is not
      const int nlo = k > 0 ? lo + (int)(((int64_t)k * span) >> 6) : lo;
      hi = lo + (int)(((int64_t)(k + 1) * span) >> 6);
      lo = nlo;
    }
    const int tile = lo;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int ti0 = tx * kTile, tj0 = ty * kTile;
    const int ti1 = min(ti0 + kTile, width) - 1, tj1 = min(tj0 + kTile, height) - 1;
    const int i = ti0 + (lane % kTile), j = tj0 + (lane / kTile);
    const float px = (float)i + 0.5f, py = (float)j + 0.5f;
    const int b0 = offsets[tile], nb = offsets[tile + 1] - b0;
    const int n = nb + nbig;
    // below (nb + nbig) + kChunk <= 17 T + kChunk < 2^31 for T < 2^26
    const int e = (int)(c - chunk_off[tile]) * kChunk + lane;
    bool meets = false;
    if (lane < kChunk && e < n) {
      const int32_t f = e < nb ? list[b0 + e] : big_list[e - nb];
      if (f >= 0 && (int64_t)f < T) {  // every list entry is a face index; checked all the same
        const FaceRec r = rec[f];
        sh.ids[lane] = f;
        sh.recs[lane] = r;
        meets = r.i0 <= ti1 && r.i1 >= ti0 && r.j0 <= tj1 && r.j1 >= tj0;
      }
    }
    uint64_t mask = __ballot(meets);
    __syncthreads();
    unsigned long long best = 0ull;  // inverted key: 0 = nothing
    while (mask) {
      const int k = __ffsll((unsigned long long)mask) - 1;
      mask &= mask - 1;
      float l0, l1, l2, z;
      if (!cover(sh.recs[k], i, j, px, py, l0, l1, l2, z)) continue;
      const unsigned long long key =
          ~(((unsigned long long)__float_as_uint(z) << 32) | (unsigned long long)(uint32_t)sh.ids[k]);
      best = key > best ? key : best;
    }
    if (best != 0ull && i <= ti1 && j <= tj1) atomicMax(&zbuf[(int64_t)j * width + i], best);
    __syncthreads();  // the chunk's records are no longer read
  }
}

// Per pixel: the winning face from the depth buffer, its weights again (the
// same operations as the coverage test) and the interpolated radiance.
__global__ __launch_bounds__(SHV_BLOCK) void k_raster_resolve(const FaceRec* __restrict__ rec,
                                                              const unsigned long long* __restrict__ zbuf,
                                                              const int32_t* __restrict__ faces,
                                                              const float* __restrict__ radiance, int width,
                                                              int64_t npix, float* __restrict__ image,
                                                              int32_t* __restrict__ face_id) {
  const int64_t pix = (int64_t)blockIdx.x * SHV_BLOCK + threadIdx.x;
  if (pix >= npix) return;
  const unsigned long long key = zbuf[pix];
  int32_t f = -1;
  float val = 0.0f;
  if (key != 0ull) {
    f = (int32_t)(uint32_t)(~key & 0xffffffffull);
    const int i = (int)(pix % width), j = (int)(pix / width);
    const FaceRec r = rec[f];
    float l0 = 0.0f, l1 = 0.0f, l2 = 0.0f, z;
    cover(r, i, j, (float)i + 0.5f, (float)j + 0.5f, l0, l1, l2, z);
    const float q0 = l0 / r.w[0], q1 = l1 / r.w[1], q2 = l2 / r.w[2];
    const float Q = (q0 + q1) + q2;
    const int32_t* fv = faces + 3 * (int64_t)f;
    val = ((q0 * radiance[fv[0]] + q1 * radiance[fv[1]]) + q2 * radiance[fv[2]]) / Q;
  }
  face_id[pix] = f;
  image[pix] = val;
}

// Contributions of one pixel won by face r to its corners: radiance
// cotangent, pixel-coordinate and depth cotangents (see the header).
__device__ __forceinline__ void pixel_adjoint(const FaceRec& r, float px, float py, float gI, const float (&B)[3],
                                              float (&gB)[3], float (&gx)[3], float (&gy)[3], float (&gw)[3]) {
  const float dx[3] = {r.x[0] - px, r.x[1] - px, r.x[2] - px};
  const float dy[3] = {r.y[0] - py, r.y[1] - py, r.y[2] - py};
  const float E[3] = {dx[1] * dy[2] - dx[2] * dy[1], dx[2] * dy[0] - dx[0] * dy[2], dx[0] * dy[1] - dx[1] * dy[0]};
  const float inv_a = 1.0f / r.area;
  float lam[3], q[3];
  for (int k = 0; k < 3; ++k) {
    lam[k] = E[k] * inv_a;
    q[k] = lam[k] / r.w[k];
  }
  const float Q = (q[0] + q[1]) + q[2];
  const float invQ = 1.0f / Q;
  const float I = ((q[0] * B[0] + q[1] * B[1]) + q[2] * B[2]) * invQ;
  float gl[3], gA = 0.0f;
  for (int k = 0; k < 3; ++k) {
    gB[k] = gI * (q[k] * invQ);
    const float gq = gI * (B[k] - I) * invQ;
    gw[k] = -gq * q[k] / r.w[k];
    gl[k] = gq / r.w[k];
    gA -= gl[k] * lam[k];
  }
  const float gE0 = gl[0] * inv_a, gE1 = gl[1] * inv_a, gE2 = gl[2] * inv_a;
  gA *= inv_a;
  gx[0] = -gE1 * dy[2] + gE2 * dy[1] + gA * (r.y[1] - r.y[2]);
  gx[1] = gE0 * dy[2] - gE2 * dy[0] + gA * (r.y[2] - r.y[0]);
  gx[2] = -gE0 * dy[1] + gE1 * dy[0] + gA * (r.y[0] - r.y[1]);
  gy[0] = gE1 * dx[2] - gE2 * dx[1] + gA * (r.x[2] - r.x[1]);
  gy[1] = -gE0 * dx[2] + gE2 * dx[0] + gA * (r.x[0] - r.x[2]);
  gy[2] = gE0 * dx[1] - gE1 * dx[0] + gA * (r.x[1] - r.x[0]);
}

// Sum over a group of 16 lanes by a butterfly: every lane of the group ends
// with the same, fixed-order sum.
__device__ __forceinline__ float group16_sum(float v) {
  for (int o = 8; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

constexpr int kFaceLanes = 16;                 // lanes per face in the adjoint
constexpr int kFacesPerBlock = SHV_BLOCK / kFaceLanes;

// Sixteen lanes per face: part[f][k][c] for corner k and c = (radiance, x, y,
// w).  The lanes stride over the face's box; each lane sums its pixels in
// order, then the group's butterfly adds the lanes in a fixed order.
__global__ __launch_bounds__(SHV_BLOCK) void k_raster_face_grads(const FaceRec* __restrict__ rec, int64_t T,
                                                                 const int32_t* __restrict__ faces,
                                                                 const float* __restrict__ radiance,
                                                                 const float* __restrict__ grad_image,
                                                                 const int32_t* __restrict__ face_id, int width,
                                                                 float* __restrict__ part) {
  const int sub = threadIdx.x % kFaceLanes;
  const int64_t f = (int64_t)blockIdx.x * kFacesPerBlock + threadIdx.x / kFaceLanes;
  const bool live = f < T;  // whole groups of 16 lanes are live or not
  const FaceRec r = rec[live ? f : 0];
  float acc[12];
  for (int c = 0; c < 12; ++c) acc[c] = 0.0f;
  if (live && r.i0 <= r.i1 && r.j0 <= r.j1) {
    const int32_t* fv = faces + 3 * f;
    const float B[3] = {radiance[fv[0]], radiance[fv[1]], radiance[fv[2]]};
    // the box is clamped to the image: at most 2^14 x 2^14 pixels, so 32-bit
    // indices (and divisions) suffice
    const int bw = r.i1 - r.i0 + 1;
    const int n = bw * (r.j1 - r.j0 + 1);
    for (int t = sub; t < n; t += kFaceLanes) {
      const int i = r.i0 + t % bw, j = r.j0 + t / bw;
      const int64_t pix = (int64_t)j * width + i;
      if (face_id[pix] != (int32_t)f) continue;
      float gB[3], gx[3], gy[3], gw[3];
      pixel_adjoint(r, (float)i + 0.5f, (float)j + 0.5f, grad_image[pix], B, gB, gx, gy, gw);
      for (int k = 0; k < 3; ++k) {
        acc[4 * k + 0] += gB[k];
        acc[4 * k + 1] += gx[k];
        acc[4 * k + 2] += gy[k];
        acc[4 * k + 3] += gw[k];
      }
    }
  }
  for (int c = 0; c < 12; ++c) acc[c] = group16_sum(acc[c]);
  if (live && sub < 12) {
    float v = acc[0];
    for (int c = 1; c < 12; ++c)
      if (sub == c) v = acc[c];
    part[12 * f + sub] = v;
  }
}

// Per vertex: the corners of its incident faces in incidence order, then the
// projection's adjoint.  inc holds 3 f + k for corner k of face f.
constexpr int kVertThreads = 64;  // small blocks: V / 64 blocks spread over all CUs
constexpr int kIncBatch = 8;      // incident corners whose loads are issued together

__global__ __launch_bounds__(kVertThreads) void k_raster_vertex_grads(const float* __restrict__ verts, int64_t V,
                                                                   int64_t T, RasterCam cam,
                                                                   const int32_t* __restrict__ inc_ptr,
                                                                   const int32_t* __restrict__ inc,
                                                                   const float* __restrict__ part,
                                                                   float* __restrict__ grad_radiance,
                                                                   float* __restrict__ grad_verts) {
  const int64_t v = (int64_t)blockIdx.x * kVertThreads + threadIdx.x;
  if (v >= V) return;
  const int64_t lim = 3 * T;
  int64_t b = inc_ptr[v], e = inc_ptr[v + 1];
  b = b < 0 ? 0 : (b > lim ? lim : b);
  e = e < b ? b : (e > lim ? lim : e);
  float gB = 0.0f, gx = 0.0f, gy = 0.0f, gw = 0.0f;
  // The corners' sums in incidence order; each batch issues its index loads,
  // then its 16-byte partial loads, together.
  for (int64_t t0 = b; t0 < e; t0 += kIncBatch) {
    int64_t cs[kIncBatch];
#pragma unroll
    for (int k = 0; k < kIncBatch; ++k) cs[k] = t0 + k < e ? (int64_t)inc[t0 + k] : -1;
    float4 q[kIncBatch];
#pragma unroll
    for (int k = 0; k < kIncBatch; ++k)
      q[k] = cs[k] >= 0 && cs[k] < lim ? *reinterpret_cast<const float4*>(part + 4 * cs[k])
                                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int k = 0; k < kIncBatch; ++k) {
      if (cs[k] >= 0 && cs[k] < lim) {
        gB += q[k].x;
        gx += q[k].y;
        gy += q[k].z;
        gw += q[k].w;
      }
    }
  }
  if (grad_radiance) grad_radiance[v] = gB;
  if (grad_verts) {
    const float x = verts[v], y = verts[V + v], z = verts[2 * V + v];
    float u, vv, w;
    project_vertex(cam.P, x, y, z, u, vv, w);
    const float gu = gx / w, gv = gy / w;
    const float gww = gw - (gu * u + gv * vv) / w;
    const float* P = cam.P;
    grad_verts[v] = (P[0] * gu + P[4] * gv) + P[8] * gww;
    grad_verts[V + v] = (P[1] * gu + P[5] * gv) + P[9] * gww;
    grad_verts[2 * V + v] = (P[2] * gu + P[6] * gv) + P[10] * gww;
  }
}

// ---------------------------------------------------------------------------

int64_t raster_tiles(int width, int height) {
  return (int64_t)((width + kTile - 1) / kTile) * ((height + kTile - 1) / kTile);
}

// Forward scratch after the face records: the depth buffer (one 64-bit key
// per pixel), the tile counts ([tiles + 1]), the shared-list count and one
// pad word (the three cleared together), the tile offsets ([tiles + 1]), the
// chunk offsets ([tiles + 1], 64-bit; 2 npix + 2 tiles + 4 words precede
// them, an even number, so they are 8-byte aligned),
// the faces' slots (kMaxBinTiles per face), the tile lists (kMaxBinTiles
// entries per face at most) and the shared list (one per face at most).
size_t raster_bin_bytes(int64_t T, int width, int height) {
  const int64_t tiles = raster_tiles(width, height);
  return (size_t)width * height * 8 + (size_t)(tiles + 1) * 8 +
         (size_t)(2 * (tiles + 1) + 2 + (2 * kMaxBinTiles + 1) * T) * 4;
}

constexpr int kZbufWaves = 8192;  // waves of the depth-buffer pass (32 per CU), striding over the chunks

hipError_t launch_raster_forward(const float* verts, int64_t V, const int32_t* faces, int64_t T, const float* radiance,
                                 const RasterCam& cam, float* image, int32_t* face_id, void* rec, void* bins,
                                 hipStream_t st) {
  const int tiles_x = (cam.width + kTile - 1) / kTile;
  const int64_t tiles = raster_tiles(cam.width, cam.height);
  const int64_t npix = (int64_t)cam.width * cam.height;
  unsigned long long* zbuf = (unsigned long long*)bins;
  int32_t* counts = (int32_t*)(zbuf + npix);
  int32_t* big_count = counts + (tiles + 1);
  int32_t* offsets = big_count + 2;
  int64_t* chunk_off = (int64_t*)(offsets + (tiles + 1));  // 2 npix + 2 tiles + 4 words in
  int32_t* slots = (int32_t*)(chunk_off + (tiles + 1));
  int32_t* list = slots + kMaxBinTiles * T;
  int32_t* big_list = list + kMaxBinTiles * T;
  // zero the depth buffer, the counts and the shared-list count (a fill
  // kernel, also under stream capture)
  hipError_t e = launch_fill_zero((float*)zbuf, 2 * npix + (tiles + 1) + 1, st);
  if (e != hipSuccess) return e;
  if (T > 0) {
    k_raster_setup<<<(unsigned)((T + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(
        verts, V, faces, T, cam, (FaceRec*)rec, tiles_x, counts, slots, big_count, big_list);
    k_raster_scan<<<1, SHV_BLOCK, 0, st>>>(counts, (int)tiles, big_count, offsets, chunk_off);
    k_raster_bin<<<(unsigned)((T + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>((const FaceRec*)rec, T, tiles_x,
                                                                                    offsets, slots, list);
    k_raster_zbuf<<<kZbufWaves, kTileThreads, 0, st>>>((const FaceRec*)rec, T, offsets, chunk_off, list, big_count,
                                                       big_list, cam.width, cam.height, tiles_x, (int)tiles, zbuf);
  }
  k_raster_resolve<<<(unsigned)((npix + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(
      (const FaceRec*)rec, zbuf, faces, radiance, cam.width, npix, image, face_id);
  return hipGetLastError();
}

hipError_t launch_raster_backward(const float* grad_image, const float* verts, int64_t V, const int32_t* faces,
                                  int64_t T, const float* radiance, const RasterCam& cam, const int32_t* face_id,
                                  const int32_t* inc_ptr, const int32_t* inc, float* grad_radiance,
                                  float* grad_verts, void* rec, float* part, hipStream_t st) {
  if (T > 0) {
    k_raster_setup<<<(unsigned)((T + SHV_BLOCK - 1) / SHV_BLOCK), SHV_BLOCK, 0, st>>>(
        verts, V, faces, T, cam, (FaceRec*)rec, 0, nullptr, nullptr, nullptr, nullptr);
    k_raster_face_grads<<<(unsigned)((T + kFacesPerBlock - 1) / kFacesPerBlock), SHV_BLOCK, 0, st>>>(
        (const FaceRec*)rec, T, faces, radiance, grad_image, face_id, cam.width, part);
  }
  if (V > 0) {
    k_raster_vertex_grads<<<(unsigned)((V + kVertThreads - 1) / kVertThreads), kVertThreads, 0, st>>>(
        verts, V, T, cam, inc_ptr, inc, part, grad_radiance, grad_verts);
  }
  return hipGetLastError();
}

size_t raster_record_bytes(int64_t T) { return (size_t)T * sizeof(FaceRec); }

}  // namespace shv
