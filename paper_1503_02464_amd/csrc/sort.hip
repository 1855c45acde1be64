// Counting sort of a species by tile, with the particles of each tile laid
// out level by level: a particle's level is its rank among the particles
// sharing its nearest grid node (its cell, for the linear shape), and the
// particles of one tile are ordered by (level, arrival).  Within a level no
// two particles share a node, so the 64 lanes of a wavefront of the fused
// kernel deposit into disjoint LDS windows and its atomics never collide on
// one address (on gfx950 such collisions serialise the LDS).
//
// Passes: (1) node ranks from per-node counters; bucket (tile, level) slots
// from per-bucket counters, one atomic per distinct bucket per wavefront;
// (2) exclusive scan of the bucket counters (multi-block), which also yields
// the tile starts; (3) every particle copied to its slot in the second set.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {
namespace {

struct SortGeom {
  int bits0, bits1;
  int mask0, mask1, mask2;
  int n[3];
  int L[3];
  int ntile0, ntile1;
  int dims;
};

__device__ __forceinline__ void unpack_cell(int32_t packed, const SortGeom &g, int c[3]) {
  const uint32_t p = static_cast<uint32_t>(packed);
  c[0] = static_cast<int>(p & g.mask0);
  c[1] = static_cast<int>((p >> g.bits0) & g.mask1);
  c[2] = static_cast<int>((p >> (g.bits0 + g.bits1)) & g.mask2);
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = c[d] >= g.n[d] ? c[d] - g.n[d] : c[d];  // fields hold < 2^bits < 2n
}

// Rank of each lane's key among the active lanes of its wavefront holding the
// same key, and one atomicAdd per distinct key on counts[]: returns the slot.
__device__ __forceinline__ int wave_slot(bool active, int key, int32_t *counts) {
  const int lane = __lane_id();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t remaining = __ballot(active);
  int slot = 0;
  while (remaining) {
    const int leader = __ffsll(static_cast<unsigned long long>(remaining)) - 1;
    const int lk = __shfl(key, leader);
    const uint64_t grp = __ballot(active && key == lk);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[lk], __popcll(grp));
    base = __shfl(base, leader);
    if (active && key == lk) slot = base + __popcll(grp & below);
    remaining &= ~grp;
  }
  return slot;
}

template <typename T, int M>
__global__ void __launch_bounds__(256) k_sort_count(const int32_t *cell, const T *o0, const T *o1, const T *o2,
                                                    int64_t np, SortGeom g, int levels, int32_t *node_count,
                                                    int32_t *key, int32_t *rank, int32_t *bucket_count) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = p < np;
  int bucket = -1;
  if (active) {
    int c[3];
    unpack_cell(cell[p], g, c);
    const int tile = c[0] / g.L[0] + g.ntile0 * (c[1] / g.L[1] + g.ntile1 * (c[2] / g.L[2]));
    // nearest node (quadratic shape) or cell (linear shape), periodic
    int nd[3] = {c[0], c[1], c[2]};
    if (M == 2) {
      const T o[3] = {o0[p], o1[p], g.dims == 3 ? o2[p] : T(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (d < g.dims && o[d] >= T(0.5)) nd[d] = (nd[d] + 1 == g.n[d]) ? 0 : nd[d] + 1;
      }
    }
    const int64_t node = nd[0] + (int64_t)g.n[0] * (nd[1] + (int64_t)g.n[1] * nd[2]);
    int level = atomicAdd(&node_count[node], 1);
    level = level < levels - 1 ? level : levels - 1;
    bucket = tile * levels + level;
  }
  const int slot = wave_slot(active, bucket, bucket_count);
  if (active) {
    key[p] = bucket;
    rank[p] = slot;
  }
}

// Multi-block exclusive scan of n counters into start[0..n]; every `levels`
// entries the running offset is also the start of a tile.
constexpr int kScanBlock = 1024;
constexpr int kScanItems = 8;  // per thread
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *sh, int64_t &total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    const int64_t a = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[kScanBlock - 1];
  const int64_t incl = sh[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_partials(const int32_t *counts, int64_t n, int64_t *partials) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += counts[base + i];
  int64_t total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_partials_top(int64_t *partials, int64_t nblocks) {
  __shared__ int64_t sh[kScanBlock];
  // nblocks <= kScanBlock * kScanItems (checked on the host)
  const int64_t base = (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < nblocks ? partials[base + i] : 0;
    s += v[i];
  }
  int64_t total;
  int64_t run = block_exclusive_scan(s, sh, total);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < nblocks) partials[base + i] = run;
    run += v[i];
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const int32_t *counts, int64_t n, const int64_t *partials,
                                                          int levels, int32_t *start, int32_t *tile_start,
                                                          int64_t ntiles) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? counts[base + i] : 0;
    s += v[i];
  }
  int64_t total;
  int64_t run = block_exclusive_scan(s, sh, total) + partials[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < n) {
      start[idx] = static_cast<int32_t>(run);
      if (idx % levels == 0) tile_start[idx / levels] = static_cast<int32_t>(run);
    }
    run += v[i];
  }
  if (base <= n - 1 && n - 1 < base + kScanItems) {  // the thread holding the last entry writes the totals
    start[n] = static_cast<int32_t>(run);
    tile_start[ntiles] = static_cast<int32_t>(run);
  }
}

template <typename T, int D>
__global__ void __launch_bounds__(256) k_sort_scatter(int64_t np, const int32_t *key, const int32_t *rank,
                                                      const int32_t *start, const int32_t *cell, const T *o0,
                                                      const T *o1, const T *o2, const T *u0, const T *u1,
                                                      const T *u2, const T *w, int32_t *cell_d, T *o0d, T *o1d,
                                                      T *o2d, T *u0d, T *u1d, T *u2d, T *wd) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int64_t q = start[key[p]] + rank[p];
  cell_d[q] = cell[p];
  o0d[q] = o0[p];
  o1d[q] = o1[p];
  if (D == 3) o2d[q] = o2[p];
  u0d[q] = u0[p];
  u1d[q] = u1[p];
  u2d[q] = u2[p];
  wd[q] = w[p];
}

template <typename T>
void count(const pic_ctx &c, const pic_species &sp, const SortGeom &g, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
  const auto *o0 = static_cast<const T *>(sp.off[0]);
  const auto *o1 = static_cast<const T *>(sp.off[1]);
  const auto *o2 = static_cast<const T *>(c.p.dims == 3 ? sp.off[2] : sp.off[0]);
  int32_t *nodes = c.wsp<int32_t>(c.ws.node_count);
  int32_t *keys = c.wsp<int32_t>(c.ws.sort_key);
  int32_t *ranks = c.wsp<int32_t>(c.ws.sort_rank);
  int32_t *buckets = c.wsp<int32_t>(c.ws.tile_count);
  if (c.p.shape_order == 2)
    hipLaunchKernelGGL((k_sort_count<T, 2>), dim3(blocks), dim3(256), 0, s, sp.cell, o0, o1, o2, sp.np, g,
                       c.levels, nodes, keys, ranks, buckets);
  else
    hipLaunchKernelGGL((k_sort_count<T, 1>), dim3(blocks), dim3(256), 0, s, sp.cell, o0, o1, o2, sp.np, g,
                       c.levels, nodes, keys, ranks, buckets);
}

template <typename T, int D>
void scatter(const pic_ctx &c, const pic_species &sp, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
  hipLaunchKernelGGL((k_sort_scatter<T, D>), dim3(blocks), dim3(256), 0, s, sp.np, c.wsp<int32_t>(c.ws.sort_key),
                     c.wsp<int32_t>(c.ws.sort_rank), c.wsp<int32_t>(c.ws.bucket_start), sp.cell,
                     static_cast<const T *>(sp.off[0]), static_cast<const T *>(sp.off[1]),
                     static_cast<const T *>(sp.off[2]), static_cast<const T *>(sp.u[0]),
                     static_cast<const T *>(sp.u[1]), static_cast<const T *>(sp.u[2]),
                     static_cast<const T *>(sp.w), sp.cell_alt, static_cast<T *>(sp.off_alt[0]),
                     static_cast<T *>(sp.off_alt[1]), static_cast<T *>(sp.off_alt[2]),
                     static_cast<T *>(sp.u_alt[0]), static_cast<T *>(sp.u_alt[1]), static_cast<T *>(sp.u_alt[2]),
                     static_cast<T *>(sp.w_alt));
}

}  // namespace

int64_t sort_scan_blocks(int64_t nbuckets) { return (nbuckets + kScanTile - 1) / kScanTile; }
int64_t sort_scan_capacity() { return static_cast<int64_t>(kScanBlock) * kScanItems; }

hipError_t launch_sort(const pic_ctx &c, pic_species &sp, hipStream_t s) {
  const int64_t nb = c.ntiles * c.levels;
  int32_t *buckets = c.wsp<int32_t>(c.ws.tile_count);
  hipError_t e = launch_fill_zero(buckets, nb, 4, s);
  if (e == hipSuccess) e = launch_fill_zero(c.wsp<int32_t>(c.ws.node_count), c.ncells, 4, s);
  if (e != hipSuccess) return e;
  if (sp.np > 0) {
    SortGeom g{};
    g.bits0 = c.bits[0];
    g.bits1 = c.bits[1];
    g.mask0 = (1 << c.bits[0]) - 1;
    g.mask1 = (1 << c.bits[1]) - 1;
    g.mask2 = (1 << c.bits[2]) - 1;
    for (int d = 0; d < 3; ++d) {
      g.L[d] = c.p.tile[d];
      g.n[d] = static_cast<int>(c.n[d]);
    }
    g.ntile0 = c.ntile[0];
    g.ntile1 = c.ntile[1];
    g.dims = c.p.dims;
    if (c.p.precision == PIC_FP64)
      count<double>(c, sp, g, s);
    else
      count<float>(c, sp, g, s);
  }
  const int64_t nblk = sort_scan_blocks(nb);
  int64_t *partials = c.wsp<int64_t>(c.ws.scan_partials);
  hipLaunchKernelGGL(k_scan_partials, dim3(static_cast<unsigned>(nblk)), dim3(kScanBlock), 0, s, buckets, nb,
                     partials);
  hipLaunchKernelGGL(k_scan_partials_top, dim3(1), dim3(kScanBlock), 0, s, partials, nblk);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nblk)), dim3(kScanBlock), 0, s, buckets, nb, partials,
                     c.levels, c.wsp<int32_t>(c.ws.bucket_start), sp.tile_start, c.ntiles);
  if (sp.np > 0) {
    const bool f64 = c.p.precision == PIC_FP64;
    if (f64)
      (c.p.dims == 3) ? scatter<double, 3>(c, sp, s) : scatter<double, 2>(c, sp, s);
    else
      (c.p.dims == 3) ? scatter<float, 3>(c, sp, s) : scatter<float, 2>(c, sp, s);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the sorted data now lives in the second set: swap the sets
  std::swap(sp.cell, sp.cell_alt);
  for (int d = 0; d < 3; ++d) {
    std::swap(sp.off[d], sp.off_alt[d]);
    std::swap(sp.u[d], sp.u_alt[d]);
  }
  std::swap(sp.w, sp.w_alt);
  sp.sorted = 1;
  return hipSuccess;
}

}  // namespace pic
