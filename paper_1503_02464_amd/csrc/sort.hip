// Counting sort of a species by tile: (1) each particle finds its tile and
// takes a slot in that tile's counter with one atomic per distinct tile per
// wavefront (particles already close to sorted hit one or two tiles per wave);
// (2) one workgroup turns the counters into tile start offsets; (3) every
// particle is copied to start[tile] + slot in the second buffer set.
#include <hip/hip_runtime.h>

#include "pic_internal.h"

namespace pic {
namespace {

struct TileKey {
  int bits0, bits1;
  int mask0, mask1, mask2;
  int n[3];
  int L[3];
  int ntile0, ntile1;
  __device__ __forceinline__ int operator()(int32_t packed) const {
    const uint32_t p = static_cast<uint32_t>(packed);
    int ix = static_cast<int>(p & mask0);
    int iy = static_cast<int>((p >> bits0) & mask1);
    int iz = static_cast<int>((p >> (bits0 + bits1)) & mask2);
    ix = ix >= n[0] ? ix - n[0] : ix;  // fields hold values below 2^bits < 2n
    iy = iy >= n[1] ? iy - n[1] : iy;
    iz = iz >= n[2] ? iz - n[2] : iz;
    return ix / L[0] + ntile0 * (iy / L[1] + ntile1 * (iz / L[2]));
  }
};

__global__ void __launch_bounds__(256) k_sort_count(const int32_t *cell, int64_t np, TileKey tk, int32_t *key,
                                                    int32_t *rank, int32_t *counts) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = p < np;
  const int k = active ? tk(cell[p]) : -1;
  const int lane = __lane_id();
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t remaining = __ballot(active);
  int my_rank = 0;
  while (remaining) {
    const int leader = __ffsll(static_cast<unsigned long long>(remaining)) - 1;
    const int lk = __shfl(k, leader);
    const uint64_t grp = __ballot(active && k == lk);
    int base = 0;
    if (lane == leader) base = atomicAdd(&counts[lk], __popcll(grp));
    base = __shfl(base, leader);
    if (active && k == lk) my_rank = base + __popcll(grp & below);
    remaining &= ~grp;
  }
  if (active) {
    key[p] = k;
    rank[p] = my_rank;
  }
}

// Exclusive scan of n counters into start[0..n] with one workgroup.
__global__ void __launch_bounds__(1024) k_scan(const int32_t *counts, int64_t n, int32_t *start) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
  const int64_t b = t * chunk, e = (b + chunk < n) ? b + chunk : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;  // exclusive prefix of this chunk
  for (int64_t i = b; i < e; ++i) {
    start[i] = static_cast<int32_t>(run);
    run += counts[i];
  }
  if (t == blockDim.x - 1) start[n] = static_cast<int32_t>(part[t]);
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

template <typename T, int D>
void scatter(const pic_ctx &c, const pic_species &sp, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
  hipLaunchKernelGGL((k_sort_scatter<T, D>), dim3(blocks), dim3(256), 0, s, sp.np, c.wsp<int32_t>(c.ws.sort_key),
                     c.wsp<int32_t>(c.ws.sort_rank), sp.tile_start, sp.cell, static_cast<const T *>(sp.off[0]),
                     static_cast<const T *>(sp.off[1]), static_cast<const T *>(sp.off[2]),
                     static_cast<const T *>(sp.u[0]), static_cast<const T *>(sp.u[1]),
                     static_cast<const T *>(sp.u[2]), static_cast<const T *>(sp.w), sp.cell_alt,
                     static_cast<T *>(sp.off_alt[0]), static_cast<T *>(sp.off_alt[1]),
                     static_cast<T *>(sp.off_alt[2]), static_cast<T *>(sp.u_alt[0]), static_cast<T *>(sp.u_alt[1]),
                     static_cast<T *>(sp.u_alt[2]), static_cast<T *>(sp.w_alt));
}

}  // namespace

hipError_t launch_sort(const pic_ctx &c, pic_species &sp, hipStream_t s) {
  int32_t *counts = c.wsp<int32_t>(c.ws.tile_count);
  hipError_t e = launch_fill_zero(counts, c.ntiles + 1, 4, s);
  if (e != hipSuccess) return e;
  if (sp.np > 0) {
    TileKey tk{};
    tk.bits0 = c.bits[0];
    tk.bits1 = c.bits[1];
    tk.mask0 = (1 << c.bits[0]) - 1;
    tk.mask1 = (1 << c.bits[1]) - 1;
    tk.mask2 = (1 << c.bits[2]) - 1;
    for (int d = 0; d < 3; ++d) {
      tk.L[d] = c.p.tile[d];
      tk.n[d] = static_cast<int>(c.n[d]);
    }
    tk.ntile0 = c.ntile[0];
    tk.ntile1 = c.ntile[1];
    const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
    hipLaunchKernelGGL(k_sort_count, dim3(blocks), dim3(256), 0, s, sp.cell, sp.np, tk,
                       c.wsp<int32_t>(c.ws.sort_key), c.wsp<int32_t>(c.ws.sort_rank), counts);
  }
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, c.ntiles, sp.tile_start);
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
