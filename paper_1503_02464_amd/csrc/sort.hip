// Counting sort of a species by tile, with the particles of each tile laid
// out level by level: particles sharing a nearest grid node (a cell, for the
// linear shape) get distinct levels, and a tile's particles are ordered by
// level, then by node.  The 64 lanes of a wavefront of the fused kernel then
// hold particles of distinct nodes, so their LDS atomics never collide on one
// address (on gfx950 such collisions serialise the LDS), and neighbouring
// lanes hold neighbouring nodes, so their LDS reads spread over the banks.
//
// Passes: (1) one workgroup per run of particles that the previous sort put in
// one tile (or per fixed chunk when the species is not sorted yet) assigns
// levels and ranks with LDS counters and bitmaps (see k_sort_count); (2) an
// exclusive scan of the bucket counts (multi-block) gives the bucket starts
// and the tile starts; (3) every particle's slot is found, then every array
// is copied into the second set in slot order.  Particles removed at an open
// face go to one last bucket behind every tile.
#include <hip/hip_runtime.h>

#include <cstdint>

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
// The groups are found with ballots first, then every group's lowest lane
// issues its atomic in the same instruction, so a wavefront waits for one
// atomic round trip however many distinct keys it holds.
__device__ __forceinline__ int wave_slot(bool active, int key, int32_t *counts) {
  const int lane = __lane_id();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t remaining = __ballot(active);
  if (!remaining) return 0;
  uint64_t mine = 0;  // the lanes sharing this lane's key
  int leader = lane;
  while (remaining) {
    const int lead = __ffsll(static_cast<unsigned long long>(remaining)) - 1;
    const int lk = __shfl(key, lead);
    const uint64_t grp = __ballot(active && key == lk);
    if (active && key == lk) {
      mine = grp;
      leader = lead;
    }
    remaining &= ~grp;
  }
  int base = 0;
  if (active && lane == leader) base = atomicAdd(&counts[key], __popcll(mine));
  base = __shfl(base, leader);
  return active ? base + __popcll(mine & below) : 0;
}

// LDS rank counters of the count pass: nodes hash to kRankSlots counters by
// the low bits of their coordinates, enough bits per dimension to keep every
// node a run can reach apart (a collision only merges two nodes' levels).
constexpr int kRankBits = 12;
constexpr int kRankSlots = 1 << kRankBits;
constexpr int kCountBlock = 1024;
constexpr int64_t kCountChunk = 4096;  // particles per workgroup when not sorted
constexpr int kCountRegs = 5;          // runs up to kCountRegs * kCountBlock particles rank in registers
// LDS words of the per-level bitmaps over a tile's nodes (and of their prefix
// counts) that order the particles staying in their tile by node.
constexpr int kOrderWords = 4096;
constexpr int kLevelShift = 20;  // stayer rank word: level << 20 | local node

struct RankGeom {
  int hbits[3], hmask[3];  // node hash
  int nl[3];               // nodes per dimension a tile's particles can be nearest to
  int words;               // bitmap words per level; 0 disables the node order
};

// Pass 1.  Workgroup b ranks the particles of run b (those the previous sort
// put in tile b), or of chunk b when the species is not sorted yet.
//  * Chunk: a particle's level is its rank among the chunk's particles of its
//    node (LDS counters); every particle takes a slot in its bucket from an
//    HBM counter (an "arrival": its key is stored as -bucket-1).
//  * Run: a particle still in tile b (a "stayer") keeps the level it had
//    (the segment of the previous sort's buckets it sits in) unless another
//    stayer of its node claimed that level first; then it takes the node's
//    lowest free level.  Claims are bits of per-level bitmaps over the tile's
//    nodes.  Stayers are then ranked inside their (tile, level) bucket by node,
//    so a bucket holds its stayers in node order and a particle whose node and
//    level did not change keeps its place: the permutation stays close to a
//    shift, and the copy's reads stay mostly contiguous.  A particle that left
//    the tile keeps its level and arrives after the stayers of its new bucket.
constexpr int kMaxLevels = kMaxSortLevels;
constexpr int32_t kDeferred = INT32_MIN;  // a stayer whose previous level was taken

struct CountLds {
  int32_t counter[kRankSlots];
  uint32_t bits[kOrderWords];
  int32_t prefix[kOrderWords];
  int64_t seg[kMaxLevels + 1];
  int64_t raw[kMaxLevels];
};

// One run (or chunk) b, by the whole workgroup.
template <typename T, int M>
__device__ __forceinline__ void count_run(int64_t b, CountLds &sh, const int32_t *cell, const T *o0, const T *o1,
                                          const T *o2, const T *w, int open, int64_t np, const SortGeom &g,
                                          const RankGeom &rg, int levels, const int32_t *runs, const int32_t *hints,
                                          int64_t nruns, int32_t *key, int32_t *rank, int32_t *stay_count,
                                          int32_t *arrive_count) {
  int32_t *counter = sh.counter;
  uint32_t *bits = sh.bits;
  int32_t *prefix = sh.prefix;
  int64_t *seg = sh.seg;
  int64_t *raw = sh.raw;
  const bool order = runs != nullptr && hints != nullptr && b < nruns && rg.words > 0;
  int64_t lo, hi;
  if (runs) {  // run b of the previous sort; the extra last workgroup takes any tail
    lo = b < nruns ? runs[b] : runs[nruns];
    hi = b < nruns ? runs[b + 1] : np;
  } else {
    lo = b * kCountChunk;
    hi = lo + kCountChunk;
  }
  lo = lo < 0 ? 0 : (lo > np ? np : lo);
  hi = hi < lo ? lo : (hi > np ? np : hi);
  if (lo >= hi) return;  // an empty run: its stayer counts are already zero
  if (order) {
    for (int i = threadIdx.x; i < levels * rg.words; i += kCountBlock) bits[i] = 0u;
    // previous level segments, clamped to partition [lo, hi): segment l
    // starts at the largest of the first l + 1 hinted starts (the first is
    // lo), at most hi
    const int t = static_cast<int>(threadIdx.x);
    if (t < levels) raw[t] = t == 0 ? lo : hints[b * levels + t];
    __syncthreads();
    if (t <= levels) {
      int64_t v = lo;
      if (t < levels)
        for (int l = 0; l <= t; ++l) v = raw[l] > v ? raw[l] : v;
      seg[t] = t < levels && v < hi ? v : hi;
    }
  } else {
    for (int i = threadIdx.x; i < kRankSlots; i += kCountBlock) counter[i] = 0;
  }
  __syncthreads();
  int T0[3] = {0, 0, 0};
  if (order) {
    T0[0] = static_cast<int>(b % g.ntile0) * g.L[0];
    T0[1] = static_cast<int>((b / g.ntile0) % g.ntile1) * g.L[1];
    T0[2] = static_cast<int>(b / ((int64_t)g.ntile0 * g.ntile1)) * g.L[2];
  }
  const int64_t dead = (int64_t)g.ntile0 * g.ntile1 * (g.n[2] / g.L[2]) * levels;  // bucket of removed particles
  // What the count pass reads of particle p: its packed cell, its nearest
  // node's step per dimension (quadratic shape), and whether it was removed.
  struct Seen {
    int32_t cell;
    bool up[3];
    bool removed;
  };
  auto look = [&](int64_t p, bool active) {
    Seen v{0, {false, false, false}, false};
    if (active) {
      v.cell = cell[p];
      v.removed = open && w[p] == T(0);
      if (M == 2) {
        v.up[0] = o0[p] >= T(0.5);
        v.up[1] = o1[p] >= T(0.5);
        v.up[2] = g.dims == 3 && o2[p] >= T(0.5);
      }
    }
    return v;
  };
  // First look at particle p (inactive lanes still take part in the ballots):
  // its key and rank, or a deferred stayer's node.
  auto first = [&](int64_t p, bool active, const Seen &sv, int32_t &k, int32_t &r) {
    int bucket = -1;
    int kind = 0;  // 0 arrival, 1 stayer with its level, 2 stayer deferred
    int word = 0;
    if (active && sv.removed) {  // removed at an open face: to the end, out of every tile
      bucket = static_cast<int>(dead);
    } else if (active) {
      int c[3];
      unpack_cell(sv.cell, g, c);
      const int tile = c[0] / g.L[0] + g.ntile0 * (c[1] / g.L[1] + g.ntile1 * (c[2] / g.L[2]));
      // nearest node (quadratic shape) or cell (linear shape), unwrapped
      int nd[3] = {c[0], c[1], c[2]};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (sv.up[d]) nd[d] += 1;
      int level;
      if (order) {
        // previous level: the last segment starting at or before p (the
        // starts are non-decreasing and seg[0] = lo <= p)
        int l0 = 0, l1 = levels - 1;
        while (l0 < l1) {
          const int mid = (l0 + l1 + 1) >> 1;
          if (seg[mid] <= p) l0 = mid;
          else l1 = mid - 1;
        }
        level = l0;
        if (tile == b) {  // a stayer's nearest node lies in [T0, T0 + L] per dimension
          const int v = (nd[0] - T0[0]) + rg.nl[0] * ((nd[1] - T0[1]) + rg.nl[1] * (nd[2] - T0[2]));
          const uint32_t m = 1u << (v & 31);
          if (l0 < levels - 1 && !(atomicOr(&bits[l0 * rg.words + (v >> 5)], m) & m)) {
            kind = 1;
            word = (l0 << kLevelShift) | v;
          } else {
            kind = 2;
            word = v;
          }
        }
      } else {
        const int hs = (nd[0] & rg.hmask[0]) | ((nd[1] & rg.hmask[1]) << rg.hbits[0]) |
                       ((nd[2] & rg.hmask[2]) << (rg.hbits[0] + rg.hbits[1]));
        level = atomicAdd(&counter[hs], 1);
        level = level < levels - 1 ? level : levels - 1;
      }
      bucket = tile * levels + level;
    }
    const int slot = wave_slot(active && kind == 0, bucket, arrive_count);
    if (active) {
      k = kind == 1 ? bucket : (kind == 2 ? kDeferred : -bucket - 1);
      r = kind == 0 ? slot : word;
    }
  };
  // A deferred stayer takes its node's lowest free level (or overflows into
  // the last level as an arrival).
  auto defer = [&](bool deferred, int32_t &k, int32_t &r) {
    int v = 0, level = levels - 1;
    bool got = false;
    if (deferred) {
      v = r;
      const uint32_t m = 1u << (v & 31);
      for (int l = 0; l < levels - 1 && !got; ++l) {
        if (!(atomicOr(&bits[l * rg.words + (v >> 5)], m) & m)) {
          got = true;
          level = l;
        }
      }
    }
    const int bucket = static_cast<int>(b) * levels + level;
    const int slot = wave_slot(deferred && !got, bucket, arrive_count);
    if (deferred) {
      k = got ? bucket : -bucket - 1;
      r = got ? ((level << kLevelShift) | v) : slot;
    }
  };
  // Per level: prefix popcounts of the claim bitmaps and the stayer count.
  auto level_counts = [&]() {
    for (int l = threadIdx.x; l < levels; l += kCountBlock) {
      int run = 0;
      for (int wd = 0; wd < rg.words; ++wd) {
        prefix[l * rg.words + wd] = run;
        run += __popc(bits[l * rg.words + wd]);
      }
      stay_count[b * levels + l] = run;
    }
  };
  // A stayer's rank in its bucket: the claimed nodes below it in its level.
  auto node_rank = [&](int32_t r) {
    const int v = r & ((1 << kLevelShift) - 1);
    const int wi = (r >> kLevelShift) * rg.words + (v >> 5);
    return prefix[wi] + __popc(bits[wi] & ((1u << (v & 31)) - 1u));
  };

  if (hi - lo <= static_cast<int64_t>(kCountBlock) * kCountRegs) {
    // A run of at most kCountRegs particles per thread keeps its keys and
    // ranks in registers and stores them once.  The guards on `it` are
    // uniform over the workgroup.
    int32_t kk[kCountRegs], rr[kCountRegs];
    Seen sv[kCountRegs];
#pragma unroll
    for (int it = 0; it < kCountRegs; ++it) {  // every load first, then the ranking
      const int64_t p = lo + static_cast<int64_t>(it) * kCountBlock + threadIdx.x;
      sv[it] = look(p, p < hi);
    }
#pragma unroll
    for (int it = 0; it < kCountRegs; ++it) {
      kk[it] = 0;
      rr[it] = 0;
      const int64_t p = lo + static_cast<int64_t>(it) * kCountBlock + threadIdx.x;
      if (lo + static_cast<int64_t>(it) * kCountBlock < hi) first(p, p < hi, sv[it], kk[it], rr[it]);
    }
    if (order) {
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kCountRegs; ++it) {
        const int64_t p = lo + static_cast<int64_t>(it) * kCountBlock + threadIdx.x;
        if (lo + static_cast<int64_t>(it) * kCountBlock < hi) defer(p < hi && kk[it] == kDeferred, kk[it], rr[it]);
      }
      __syncthreads();
      level_counts();
      __syncthreads();
#pragma unroll
      for (int it = 0; it < kCountRegs; ++it) {
        const int64_t p = lo + static_cast<int64_t>(it) * kCountBlock + threadIdx.x;
        if (p < hi && kk[it] >= 0) rr[it] = node_rank(rr[it]);
      }
    }
#pragma unroll
    for (int it = 0; it < kCountRegs; ++it) {
      const int64_t p = lo + static_cast<int64_t>(it) * kCountBlock + threadIdx.x;
      if (p < hi) {
        key[p] = kk[it];
        rank[p] = rr[it];
      }
    }
    return;
  }

  // Longer runs go through key[] and rank[] in HBM.
  for (int64_t base = lo; base < hi; base += kCountBlock) {  // uniform trip count per workgroup
    const int64_t p = base + threadIdx.x;
    int32_t k = 0, r = 0;
    first(p, p < hi, look(p, p < hi), k, r);
    if (p < hi) {
      key[p] = k;
      rank[p] = r;
    }
  }
  if (!order) return;
  __syncthreads();
  for (int64_t base = lo; base < hi; base += kCountBlock) {
    const int64_t p = base + threadIdx.x;
    const bool deferred = p < hi && key[p] == kDeferred;
    int32_t k = 0, r = deferred ? rank[p] : 0;
    defer(deferred, k, r);
    if (deferred) {
      key[p] = k;
      rank[p] = r;
    }
  }
  __syncthreads();
  level_counts();
  __syncthreads();
  for (int64_t base = lo; base < hi; base += kCountBlock) {
    const int64_t p = base + threadIdx.x;
    if (p < hi && key[p] >= 0) rank[p] = node_rank(rank[p]);
  }
}

// One workgroup per run (or chunk).  Runs are taken in the order of the
// previous sort's list of non-empty tiles: dealing the blocks of a sparse box
// by tile index would pile the busy ones onto a few XCDs and CUs.
// Eight waves per SIMD let two workgroups share a CU (the pass waits on
// memory more than it computes).
template <typename T, int M>
__global__ void __launch_bounds__(kCountBlock) __attribute__((amdgpu_waves_per_eu(8)))
    k_sort_count(const int32_t *cell, const T *o0, const T *o1, const T *o2, const T *w, int open, int64_t np,
                 SortGeom g, RankGeom rg, int levels, const int32_t *runs, const int32_t *hints, int64_t nruns,
                 const int32_t *live, int64_t nitems, int32_t *key, int32_t *rank, int32_t *stay_count,
                 int32_t *arrive_count) {
  __shared__ CountLds sh;
  int64_t b = blockIdx.x;
  if (live) {  // the previous sort's non-empty runs first (balanced over the CUs), then the tail
    int64_t nlive = live[nruns];
    nlive = nlive < 0 ? 0 : (nlive > nruns ? nruns : nlive);
    if (b > nlive) return;
    b = b < nlive ? live[b] : nruns;
    if (b < 0 || b > nruns) return;
  } else if (b >= nitems) {
    return;
  }
  count_run<T, M>(b, sh, cell, o0, o1, o2, w, open, np, g, rg, levels, runs, hints, nruns, key, rank, stay_count,
                  arrive_count);
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

__global__ void __launch_bounds__(kScanBlock) k_scan_partials(const int32_t *ca, const int32_t *cb, int64_t n,
                                                              int64_t *partials) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += (int64_t)ca[base + i] + cb[base + i];
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

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const int32_t *ca, const int32_t *cb, int64_t n,
                                                          const int64_t *partials, int levels, int32_t *start,
                                                          int32_t *tile_start, int64_t ntiles) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? (int64_t)ca[base + i] + cb[base + i] : 0;
    s += v[i];
  }
  int64_t total;
  int64_t run = block_exclusive_scan(s, sh, total) + partials[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i;
    if (idx < n) {
      start[idx] = static_cast<int32_t>(run);
      // entry ntiles * levels is the bucket of removed particles: its start
      // closes the last tile
      if (idx % levels == 0 && idx / levels <= ntiles) tile_start[idx / levels] = static_cast<int32_t>(run);
    }
    run += v[i];
  }
  if (base <= n - 1 && n - 1 < base + kScanItems)  // the thread holding the last entry writes the total
    start[n] = static_cast<int32_t>(run);
}

// The tiles left non-empty, in tile order, and their count at [ntiles]: each
// thread counts a contiguous chunk, one block scan places the chunks.  The
// same for the non-empty tiles with at least `sparse` particles (dense) and
// with fewer (sparse); sparse = 0 makes every live tile dense.
__global__ void __launch_bounds__(kScanBlock) k_list_tiles(const int32_t *tile_start, int64_t ntiles, int32_t sparse,
                                                          int32_t *live, int32_t *dense, int32_t *few) {
  __shared__ int64_t sh[kScanBlock];
  const int64_t per = (ntiles + kScanBlock - 1) / kScanBlock;
  const int64_t a = threadIdx.x * per;
  const int64_t e = a + per < ntiles ? a + per : ntiles;
  int64_t cnt = 0, cnt_few = 0;
#pragma unroll 8
  for (int64_t t = a; t < e; ++t) {
    const int32_t n = tile_start[t + 1] - tile_start[t];
    cnt += n > 0 ? 1 : 0;
    cnt_few += n > 0 && n < sparse ? 1 : 0;
  }
  int64_t total, total_few;
  int64_t pos = block_exclusive_scan(cnt, sh, total);
  __syncthreads();  // sh is reused
  int64_t pos_few = block_exclusive_scan(cnt_few, sh, total_few);
  int64_t pos_dense = pos - pos_few;
  for (int64_t t = a; t < e; ++t) {
    const int32_t n = tile_start[t + 1] - tile_start[t];
    if (n > 0) live[pos++] = static_cast<int32_t>(t);
    if (n > 0 && n < sparse) few[pos_few++] = static_cast<int32_t>(t);
    else if (n > 0) dense[pos_dense++] = static_cast<int32_t>(t);
  }
  if (threadIdx.x == 0) {
    live[ntiles] = static_cast<int32_t>(total);
    dense[ntiles] = static_cast<int32_t>(total - total_few);
    few[ntiles] = static_cast<int32_t>(total_few);
  }
}

// Workgroups are dealt to the 8 XCDs round-robin.  The copy passes launch a
// multiple of 8 workgroups and give XCD x the x-th contiguous eighth of the
// particles, so the lines that neighbouring workgroups share (the reads of a
// shifted run, the writes of a permuted one) meet in one XCD's L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_block() {
  const int64_t per = gridDim.x / kXcds;
  return (blockIdx.x % kXcds) * per + blockIdx.x / kXcds;
}

unsigned xcd_grid(int64_t nblocks) { return static_cast<unsigned>((nblocks + kXcds - 1) / kXcds * kXcds); }

// Pass 3a.  Each particle's slot: a stayer goes to start[bucket] + its node
// rank, an arrival after the bucket's stayers.  src[slot] = particle.
__global__ void __launch_bounds__(256) k_sort_slots(int64_t np, const int32_t *key, const int32_t *rank,
                                                   const int32_t *start, const int32_t *stay, int64_t nbuckets,
                                                   int32_t *src, int32_t *flags) {
  const int64_t p = xcd_block() * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const int32_t k = key[p];
  const int64_t bk = k >= 0 ? k : -(int64_t)k - 1;
  int64_t q = -1;
  if (bk < nbuckets) q = (int64_t)start[bk] + rank[p] + (k >= 0 ? 0 : stay[bk]);
  if (q < 0 || q >= np || (bk < nbuckets && q >= start[bk + 1])) {
    // the runs handed to the count pass did not partition the particles
    atomicOr(&flags[0], kFlagSort);
    return;
  }
  src[q] = static_cast<int32_t>(p);
}

// Pass 3b.  Every array is copied into the second set in destination order
// (coalesced writes; the reads follow the permutation, which keeps most
// neighbours together).
template <typename T, int D>
__global__ void __launch_bounds__(256) k_sort_gather(int64_t np, const int32_t *src, const int32_t *cell,
                                                    const T *o0, const T *o1, const T *o2, const T *u0, const T *u1,
                                                    const T *u2, const T *w, int32_t *cell_d, T *o0d, T *o1d,
                                                    T *o2d, T *u0d, T *u1d, T *u2d, T *wd) {
  const int64_t q = xcd_block() * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const int64_t p = src[q];
  if (p < 0 || p >= np) return;  // only after a flagged inconsistency
  cell_d[q] = cell[p];
  o0d[q] = o0[p];
  o1d[q] = o1[p];
  if (D == 3) o2d[q] = o2[p];
  u0d[q] = u0[p];
  u1d[q] = u1[p];
  u2d[q] = u2[p];
  wd[q] = w[p];
}

RankGeom rank_geom(const pic_ctx &c) {
  // a run's nodes span at most tile + 2 slack + 1 per dimension
  RankGeom h{};
  int total = 0;
  for (int d = 0; d < 3; ++d) {
    int span = d < c.p.dims ? c.p.tile[d] + 2 * c.p.slack + 1 : 1;
    int b = 0;
    while ((1 << b) < span) ++b;
    h.hbits[d] = b;
    total += b;
  }
  while (total > kRankBits) {  // trim the widest dimension; collisions only cost conflicts
    int dmax = 0;
    for (int d = 1; d < 3; ++d)
      if (h.hbits[d] > h.hbits[dmax]) dmax = d;
    --h.hbits[dmax];
    --total;
  }
  int64_t vol = 1;
  for (int d = 0; d < 3; ++d) {
    h.hmask[d] = (1 << h.hbits[d]) - 1;
    h.nl[d] = d < c.p.dims ? c.p.tile[d] + (c.p.shape_order == 2 ? 1 : 0) : 1;
    vol *= h.nl[d];
  }
  const int64_t words = (vol + 31) / 32;
  h.words = (words * c.levels <= kOrderWords && vol < (1 << kLevelShift) && c.levels <= kMaxLevels)
                ? static_cast<int>(words)
                : 0;
  return h;
}

template <typename T>
void count(const pic_ctx &c, const pic_species &sp, const SortGeom &g, bool by_runs, const int32_t *hints,
           const int32_t *live, hipStream_t s) {
  const auto *o0 = static_cast<const T *>(sp.off[0]);
  const auto *o1 = static_cast<const T *>(sp.off[1]);
  const auto *o2 = static_cast<const T *>(c.p.dims == 3 ? sp.off[2] : sp.off[0]);
  int32_t *keys = c.wsp<int32_t>(c.ws.sort_key);
  int32_t *ranks = c.wsp<int32_t>(c.ws.sort_rank);
  int32_t *stay = c.wsp<int32_t>(c.ws.stay_count);
  int32_t *arrive = c.wsp<int32_t>(c.ws.arrive_count);
  const int32_t *runs = by_runs ? sp.tile_start : nullptr;
  const int64_t nruns = by_runs ? c.ntiles : 0;
  const int64_t items = by_runs ? c.ntiles + 1 : (sp.np + kCountChunk - 1) / kCountChunk;
  const unsigned blocks = static_cast<unsigned>(items);
  const RankGeom rg = rank_geom(c);
  const auto *w = static_cast<const T *>(sp.w);
  const int open = c.p.open_x;
  if (c.p.shape_order == 2)
    hipLaunchKernelGGL((k_sort_count<T, 2>), dim3(blocks), dim3(kCountBlock), 0, s, sp.cell, o0, o1, o2, w, open,
                       sp.np, g, rg, c.levels, runs, hints, nruns, by_runs ? live : nullptr, items, keys, ranks, stay,
                       arrive);
  else
    hipLaunchKernelGGL((k_sort_count<T, 1>), dim3(blocks), dim3(kCountBlock), 0, s, sp.cell, o0, o1, o2, w, open,
                       sp.np, g, rg, c.levels, runs, hints, nruns, by_runs ? live : nullptr, items, keys, ranks, stay,
                       arrive);
}

// Slots, then (copy) the gather into the second set.
template <typename T, int D>
void reorder(const pic_ctx &c, const pic_species &sp, const int32_t *start, bool copy, hipStream_t s) {
  const unsigned blocks = xcd_grid((sp.np + 255) / 256);
  int32_t *src = c.wsp<int32_t>(c.ws.sort_src);
  hipLaunchKernelGGL(k_sort_slots, dim3(blocks), dim3(256), 0, s, sp.np, c.wsp<int32_t>(c.ws.sort_key),
                     c.wsp<int32_t>(c.ws.sort_rank), start, c.wsp<int32_t>(c.ws.stay_count),
                     c.ntiles * c.levels + 1, src, c.wsp<int32_t>(c.ws.flags));
  if (!copy) return;
  hipLaunchKernelGGL((k_sort_gather<T, D>), dim3(blocks), dim3(256), 0, s, sp.np, src, sp.cell,
                     static_cast<const T *>(sp.off[0]), static_cast<const T *>(sp.off[1]),
                     static_cast<const T *>(sp.off[2]), static_cast<const T *>(sp.u[0]),
                     static_cast<const T *>(sp.u[1]), static_cast<const T *>(sp.u[2]),
                     static_cast<const T *>(sp.w), sp.cell_alt, static_cast<T *>(sp.off_alt[0]),
                     static_cast<T *>(sp.off_alt[1]), static_cast<T *>(sp.off_alt[2]),
                     static_cast<T *>(sp.u_alt[0]), static_cast<T *>(sp.u_alt[1]), static_cast<T *>(sp.u_alt[2]),
                     static_cast<T *>(sp.w_alt));
}

}  // namespace

void swap_sets(pic_species &sp) {
  std::swap(sp.cell, sp.cell_alt);
  for (int d = 0; d < 3; ++d) {
    std::swap(sp.off[d], sp.off_alt[d]);
    std::swap(sp.u[d], sp.u_alt[d]);
  }
  std::swap(sp.w, sp.w_alt);
}

int64_t sort_scan_blocks(int64_t nbuckets) { return (nbuckets + kScanTile - 1) / kScanTile; }
int64_t sort_scan_capacity() { return static_cast<int64_t>(kScanBlock) * kScanItems; }

hipError_t launch_sort(pic_ctx &c, pic_species &sp, hipStream_t s, const int32_t **fold_src, bool wait) {
  // buckets: (tile, level) for every tile, then one for removed particles
  const int64_t nb = c.ntiles * c.levels + 1;
  int32_t *stay = c.wsp<int32_t>(c.ws.stay_count);
  int32_t *arrive = c.wsp<int32_t>(c.ws.arrive_count);
  void *const counts[2] = {stay, arrive};
  hipError_t e = launch_fill_zero_n(counts, 2, nb, 4, s);
  if (e != hipSuccess) return e;
  // The previous sort's tile runs (and its bucket starts, kept in the
  // species' slot) stay valid while the particle set is the one this context
  // sorted last into this tile_start array.
  int slot = -1;
  bool by_runs = false;
  for (size_t i = 0; i < c.sorted_runs.size(); ++i)
    if (c.sorted_runs[i].first == sp.tile_start) {
      slot = static_cast<int>(i);
      by_runs = c.sorted_runs[i].second == sp.np && sp.sorted;
    }
  if (slot >= 0 && c.live_pending[slot]) {
    // The previous sort left the removed particles behind its tiles, from
    // its live count on; pushes since then kept that order.  Drop them if the
    // count has arrived (never wait for it) and the species is still that
    // sort's particle set.
    const hipError_t q = hipEventQuery(c.live_event[slot]);
    if (q == hipSuccess) {
      c.live_pending[slot] = false;
      const int64_t nlive = c.live_host[slot];
      if (by_runs && nlive >= 0 && nlive < sp.np) {
        sp.np = nlive;
        c.sorted_runs[slot].second = sp.np;
      }
    } else if (q != hipErrorNotReady) {
      return q;
    }
    if (!by_runs) c.live_pending[slot] = false;
  }
  if (slot < 0) {
    if (c.sorted_runs.size() < static_cast<size_t>(kMaxSpecies)) {
      slot = static_cast<int>(c.sorted_runs.size());
      c.sorted_runs.emplace_back(sp.tile_start, -1);
    } else {  // more species than slots: share the last one, without hints
      slot = kMaxSpecies - 1;
      by_runs = false;
      c.sorted_runs[slot].first = sp.tile_start;
    }
  }
  int32_t *start = c.wsp<int32_t>(c.ws.bucket_start) + static_cast<size_t>(slot) * (nb + 1);
  c.wmax_known[slot] = false;  // the tiles change: the next fused launch finds their weight bounds again
  int32_t *live = c.wsp<int32_t>(c.ws.live_tiles) + static_cast<size_t>(slot) * (c.ntiles + 1);
  int32_t *dense = c.wsp<int32_t>(c.ws.dense_tiles) + static_cast<size_t>(slot) * (c.ntiles + 1);
  int32_t *few = c.wsp<int32_t>(c.ws.sparse_tiles) + static_cast<size_t>(slot) * (c.ntiles + 1);
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
    const int32_t *hints = by_runs ? start : nullptr;
    if (c.p.precision == PIC_FP64)
      count<double>(c, sp, g, by_runs, hints, live, s);
    else
      count<float>(c, sp, g, by_runs, hints, live, s);
  }
  const int64_t nblk = sort_scan_blocks(nb);
  int64_t *partials = c.wsp<int64_t>(c.ws.scan_partials);
  hipLaunchKernelGGL(k_scan_partials, dim3(static_cast<unsigned>(nblk)), dim3(kScanBlock), 0, s, stay, arrive, nb,
                     partials);
  hipLaunchKernelGGL(k_scan_partials_top, dim3(1), dim3(kScanBlock), 0, s, partials, nblk);
  hipLaunchKernelGGL(k_scan_apply, dim3(static_cast<unsigned>(nblk)), dim3(kScanBlock), 0, s, stay, arrive, nb,
                     partials, c.levels, start, sp.tile_start, c.ntiles);
  hipLaunchKernelGGL(k_list_tiles, dim3(1), dim3(kScanBlock), 0, s, sp.tile_start, c.ntiles,
                     c.p.dims == 3 ? kSparseTile : 0, live, dense, few);
  const bool copy = fold_src == nullptr || sp.np == 0;
  if (sp.np > 0) {
    const bool f64 = c.p.precision == PIC_FP64;
    if (f64)
      (c.p.dims == 3) ? reorder<double, 3>(c, sp, start, copy, s) : reorder<double, 2>(c, sp, start, copy, s);
    else
      (c.p.dims == 3) ? reorder<float, 3>(c, sp, start, copy, s) : reorder<float, 2>(c, sp, start, copy, s);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (copy) {
    if (fold_src) *fold_src = nullptr;
    swap_sets(sp);  // the sorted data now lives in the second set
  } else {
    *fold_src = c.wsp<int32_t>(c.ws.sort_src);  // the caller's push copies, then swaps
  }
  sp.sorted = 1;
  if (c.p.open_x && sp.np > 0 && wait) {
    // The removed particles now sit behind every tile, from tile_start[ntiles]
    // on: the species keeps only the live ones (a folded copy then never
    // reads the removed ones, and later sorts never rank them).
    int32_t nlive = 0;
    e = hipMemcpyAsync(&nlive, sp.tile_start + c.ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (nlive >= 0 && nlive < sp.np) sp.np = nlive;
    c.live_pending[slot] = false;
  } else if (c.p.open_x && sp.np > 0) {
    // the live count goes to pinned host memory behind the sort; the next
    // sort of this species applies it
    if (!c.live_host) {
      void *h = nullptr;
      e = hipHostMalloc(&h, sizeof(int32_t) * kMaxSpecies, hipHostMallocDefault);
      if (e != hipSuccess) return e;
      c.live_host = static_cast<int32_t *>(h);
    }
    if (!c.live_event[slot]) {
      e = hipEventCreateWithFlags(&c.live_event[slot], hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    e = hipMemcpyAsync(c.live_host + slot, sp.tile_start + c.ntiles, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(c.live_event[slot], s);
    if (e != hipSuccess) return e;
    c.live_pending[slot] = true;
  }
  c.sorted_runs[slot].second = sp.np;
  return hipSuccess;
}

int sorted_slot(const pic_ctx &c, const pic_species &sp) {
  for (size_t i = 0; i < c.sorted_runs.size(); ++i)
    if (c.sorted_runs[i].first == sp.tile_start && c.sorted_runs[i].second == sp.np) return static_cast<int>(i);
  return -1;
}

namespace {
const int32_t *tile_list(const pic_ctx &c, const pic_species &sp, size_t base) {
  const int i = sorted_slot(c, sp);
  return i < 0 ? nullptr : c.wsp<int32_t>(base) + static_cast<size_t>(i) * (c.ntiles + 1);
}
}  // namespace

const int32_t *live_tiles(const pic_ctx &c, const pic_species &sp) { return tile_list(c, sp, c.ws.live_tiles); }
const int32_t *dense_tiles(const pic_ctx &c, const pic_species &sp) { return tile_list(c, sp, c.ws.dense_tiles); }
const int32_t *sparse_tiles(const pic_ctx &c, const pic_species &sp) { return tile_list(c, sp, c.ws.sparse_tiles); }

}  // namespace pic
