// Output extraction on the device (paper Sec. 3.1: reduced-dimension and
// subdomain outputs of the grid data and of the particles' phase space).
//
// Grid extraction copies the values of a strided box of points out of up to
// kMaxExtractGrids grids into one dense buffer, bit for bit (4- or 8-byte
// elements): a plane is a box one point thick along one axis, a line one
// thick along two.  Particle extraction keeps, in storage order, the
// particles whose cell lies in a box of cells and whose storage index is a
// multiple of a subsampling stride, and writes one record per particle:
// the absolute position along each dimension, the three momenta and the
// weight.  The order is the storage order because each block writes at the
// exclusive prefix of the counts of the blocks before it (count, scan,
// write), so the output is a deterministic function of the state.
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kExtractThreads = 256;
constexpr int kSelThreads = 256;
constexpr int kSelRounds = kSelectChunk / kSelThreads;
constexpr int kScanThreads = 1024;

struct GridBox {
  const void *g[kMaxExtractGrids];
  int32_t ngrids;
  int64_t n0, n01;   // source strides of y and z
  int32_t lo[3], st[3];
  int64_t m0, m1, m2;  // selected points per axis
  int64_t total;       // ngrids m0 m1 m2
};

template <typename E, typename I>
__global__ void __launch_bounds__(kExtractThreads) k_extract_grid(GridBox b, E *__restrict__ dst) {
  const I m0 = static_cast<I>(b.m0), m1 = static_cast<I>(b.m1), m2 = static_cast<I>(b.m2);
  const I total = static_cast<I>(b.total);
  for (I t = static_cast<I>(blockIdx.x) * kExtractThreads + threadIdx.x; t < total;
       t += static_cast<I>(gridDim.x) * kExtractThreads) {
    I r = t / m0;
    const I a = t - r * m0;
    I q = r / m1;
    const I bb = r - q * m1;
    const I g = q / m2;
    const I c = q - g * m2;
    const int64_t i = b.lo[0] + static_cast<int64_t>(a) * b.st[0];
    const int64_t j = b.lo[1] + static_cast<int64_t>(bb) * b.st[1];
    const int64_t k = b.lo[2] + static_cast<int64_t>(c) * b.st[2];
    const E *src = static_cast<const E *>(b.g[g]);
    dst[t] = src[i + b.n0 * j + b.n01 * k];
  }
}

struct SelArgs {
  const int32_t *cell;
  const void *off[3];
  const void *u[3];
  const void *w;
  int64_t np, every;
  int32_t lo[3], hi[3];
  int32_t shift[3];
  int32_t mask[3];
  double dx[3];
  int32_t dims;
  int32_t skip_weightless;  // open x faces: weight-0 particles are removed ones
  int64_t nblocks;
  int64_t *block_base;  // nblocks counts, turned into exclusive offsets by the scan
  int64_t *count;       // total selected
  void *dst;
  int64_t capacity;     // records dst holds
};

template <typename T>
__device__ __forceinline__ bool selected(const SelArgs &a, int64_t i, int32_t *cd) {
  if (i >= a.np || (a.every != 1 && i % a.every != 0)) return false;
  const int32_t cell = a.cell[i];
  bool in = true;
  for (int d = 0; d < 3; ++d) {
    cd[d] = d < a.dims ? (cell >> a.shift[d]) & a.mask[d] : 0;
    in = in && cd[d] >= a.lo[d] && cd[d] < a.hi[d];
  }
  if (in && a.skip_weightless) in = static_cast<const T *>(a.w)[i] != T(0);
  return in;
}

// Selected particles of each chunk of kSelectChunk storage slots.
template <typename T>
__global__ void __launch_bounds__(kSelThreads) k_select_count(SelArgs a) {
  __shared__ int32_t total;
  if (threadIdx.x == 0) total = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSelectChunk;
  int32_t mine = 0;
  for (int r = 0; r < kSelRounds; ++r) {
    int32_t cd[3];
    mine += selected<T>(a, base + r * kSelThreads + threadIdx.x, cd) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o);
  if ((threadIdx.x & 63) == 0) atomicAdd(&total, mine);
  __syncthreads();
  if (threadIdx.x == 0) a.block_base[blockIdx.x] = total;
}

// One workgroup: exclusive prefix of the chunk counts in place, and the total.
__global__ void __launch_bounds__(kScanThreads) k_select_scan(int64_t *v, int64_t n, int64_t *count) {
  __shared__ int64_t part[kScanThreads / 64];
  int64_t carry = 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t b = 0; b < n; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    const int64_t x = i < n ? v[i] : 0;
    int64_t incl = x;  // inclusive scan inside the wave
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) part[wave] = incl;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
      before += k < wave ? part[k] : 0;
      all += part[k];
    }
    if (i < n) v[i] = carry + before + incl - x;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = carry;
}

template <typename T>
__global__ void __launch_bounds__(kSelThreads) k_select_write(SelArgs a) {
  __shared__ int32_t wave_sum[kSelThreads / 64];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kSelectChunk;
  int64_t out = a.block_base[blockIdx.x];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rec = a.dims + 4;
  T *dst = static_cast<T *>(a.dst);
  for (int r = 0; r < kSelRounds; ++r) {
    const int64_t i = base + r * kSelThreads + threadIdx.x;
    int32_t cd[3];
    const bool take = selected<T>(a, i, cd);
    const uint64_t m = __ballot(take);
    const int32_t below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wave_sum[wave] = __popcll(m);
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int k = 0; k < kSelThreads / 64; ++k) {
      before += k < wave ? wave_sum[k] : 0;
      all += wave_sum[k];
    }
    const int64_t slot = out + before + below;
    if (take && slot < a.capacity) {
      T *o = dst + slot * rec;
      for (int d = 0; d < a.dims; ++d) {
        const double x = static_cast<double>(cd[d]) + static_cast<double>(static_cast<const T *>(a.off[d])[i]);
        o[d] = static_cast<T>(x * a.dx[d]);
      }
      for (int d = 0; d < 3; ++d) o[a.dims + d] = static_cast<const T *>(a.u[d])[i];
      o[a.dims + 3] = static_cast<const T *>(a.w)[i];
    }
    out += all;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_extract_grid(const pic_ctx &c, const void *const *grids, int32_t ngrids, int32_t elem_bytes,
                               const pic_box &box, void *dst, hipStream_t s) {
  GridBox b{};
  for (int g = 0; g < ngrids; ++g) b.g[g] = grids[g];
  b.ngrids = ngrids;
  b.n0 = c.n[0];
  b.n01 = c.n[0] * c.n[1];
  for (int d = 0; d < 3; ++d) {
    b.lo[d] = box.lo[d];
    b.st[d] = box.stride[d];
  }
  b.m0 = box_points(box, 0);
  b.m1 = box_points(box, 1);
  b.m2 = box_points(box, 2);
  b.total = ngrids * b.m0 * b.m1 * b.m2;
  if (b.total == 0) return hipSuccess;
  const int64_t want = (b.total + kExtractThreads - 1) / kExtractThreads;
  const unsigned blocks = static_cast<unsigned>(want < 65536 ? want : 65536);
  const bool small = b.total < (int64_t(1) << 31);
  if (elem_bytes == 4) {
    if (small)
      hipLaunchKernelGGL((k_extract_grid<uint32_t, uint32_t>), dim3(blocks), dim3(kExtractThreads), 0, s, b,
                         static_cast<uint32_t *>(dst));
    else
      hipLaunchKernelGGL((k_extract_grid<uint32_t, uint64_t>), dim3(blocks), dim3(kExtractThreads), 0, s, b,
                         static_cast<uint32_t *>(dst));
  } else {
    if (small)
      hipLaunchKernelGGL((k_extract_grid<uint64_t, uint32_t>), dim3(blocks), dim3(kExtractThreads), 0, s, b,
                         static_cast<uint64_t *>(dst));
    else
      hipLaunchKernelGGL((k_extract_grid<uint64_t, uint64_t>), dim3(blocks), dim3(kExtractThreads), 0, s, b,
                         static_cast<uint64_t *>(dst));
  }
  return hipGetLastError();
}

hipError_t launch_extract_particles(const pic_ctx &c, const pic_species &sp, const pic_box &cells, int64_t every,
                                    void *dst, int64_t capacity, int64_t *count, hipStream_t s) {
  SelArgs a{};
  a.cell = sp.cell;
  for (int d = 0; d < 3; ++d) {
    a.off[d] = sp.off[d];
    a.u[d] = sp.u[d];
    a.lo[d] = cells.lo[d];
    a.hi[d] = cells.hi[d];
    a.dx[d] = c.p.dx[d];
  }
  a.w = sp.w;
  a.np = sp.np;
  a.every = every;
  int shift = 0;
  for (int d = 0; d < 3; ++d) {
    a.shift[d] = shift;
    a.mask[d] = static_cast<int32_t>((int64_t(1) << c.bits[d]) - 1);
    shift += c.bits[d];
  }
  a.dims = c.p.dims;
  a.skip_weightless = c.p.open_x ? 1 : 0;
  a.nblocks = (sp.np + kSelectChunk - 1) / kSelectChunk;
  a.block_base = c.wsp<int64_t>(c.ws.select_base);
  a.count = count;
  a.dst = dst;
  a.capacity = capacity;
  const dim3 grid(static_cast<unsigned>(a.nblocks));
  if (a.nblocks > 0) {
    if (c.p.precision == PIC_FP32)
      hipLaunchKernelGGL(k_select_count<float>, grid, dim3(kSelThreads), 0, s, a);
    else
      hipLaunchKernelGGL(k_select_count<double>, grid, dim3(kSelThreads), 0, s, a);
  }
  // also writes the zero count of an empty species
  hipLaunchKernelGGL(k_select_scan, dim3(1), dim3(kScanThreads), 0, s, a.block_base, a.nblocks, count);
  if (a.nblocks == 0) return hipGetLastError();
  if (c.p.precision == PIC_FP32)
    hipLaunchKernelGGL(k_select_write<float>, grid, dim3(kSelThreads), 0, s, a);
  else
    hipLaunchKernelGGL(k_select_write<double>, grid, dim3(kSelThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace pic
