// FP64 diagnostics: field and kinetic energy, total charge, the charge density
// on nodes and the residuals of Gauss's law and of the continuity equation.
// Sums run in double whatever the state precision; partial results go to
// fixed slots and one workgroup reduces them in a fixed order, so the result
// does not depend on scheduling (the charge grid itself is built with double
// atomics, whose order does vary at round-off level).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "particle_math.h"
#include "pic_internal.h"

namespace pic {
namespace {

constexpr int kB = 256;
constexpr int kStride = kMaxSpecies * kDiagBlocks;  // entries per slot

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < static_cast<int>(blockDim.x / 64); ++i) r += sh[i];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double block_max(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o));
  const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < static_cast<int>(blockDim.x / 64); ++i) r = fmax(r, sh[i]);
  __syncthreads();
  return r;
}

// Slots 0, 1: sum |E|^2, sum |B|^2 (scaled to energies by the final pass).
template <typename T>
__global__ void __launch_bounds__(kB) k_field_sq(const T *e0, const T *e1, const T *e2, const T *b0, const T *b1,
                                                 const T *b2, int64_t n, double *partials) {
  __shared__ double sh[16];
  double se = 0.0, sb = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double x = e0[i], y = e1[i], z = e2[i];
    se += x * x + y * y + z * z;
    const double a = b0[i], b = b1[i], c = b2[i];
    sb += a * a + b * b + c * c;
  }
  se = block_sum(se, sh);
  sb = block_sum(sb, sh);
  if (threadIdx.x == 0) {
    partials[0 * kStride + blockIdx.x] = se;
    partials[1 * kStride + blockIdx.x] = sb;
  }
}

// Slots 2, 3: sum w m (gamma - 1), sum q w for one species (block range by species).
template <typename T>
__global__ void __launch_bounds__(kB) k_particle_sums(const T *u0, const T *u1, const T *u2, const T *w, int64_t np,
                                                      double q, double m, double *partials, int slot0) {
  __shared__ double sh[16];
  double k = 0.0, qs = 0.0;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
    const double a = u0[p], b = u1[p], c = u2[p];
    const double usq = a * a + b * b + c * c;
    // gamma - 1 written without cancellation for slow particles
    const double gm1 = usq / (sqrt(1.0 + usq) + 1.0);
    k += static_cast<double>(w[p]) * m * gm1;
    qs += q * static_cast<double>(w[p]);
  }
  k = block_sum(k, sh);
  qs = block_sum(qs, sh);
  if (threadIdx.x == 0) {
    partials[2 * kStride + slot0 + blockIdx.x] = k;
    partials[3 * kStride + slot0 + blockIdx.x] = qs;
  }
}

// Charge density on nodes: rho(node) += q w / dV * S(x - node), in double.
template <typename T, int D, int M>
__global__ void __launch_bounds__(kB) k_rho(const int32_t *cell, const T *o0, const T *o1, const T *o2, const T *w,
                                            int64_t np, double qdv, int b0, int b1, int m0, int m1, int m2, int n0,
                                            int n1, int n2, double *rho) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  const uint32_t pk = static_cast<uint32_t>(cell[p]);
  int c[3] = {static_cast<int>(pk & m0), static_cast<int>((pk >> b0) & m1),
              static_cast<int>((pk >> (b0 + b1)) & m2)};
  c[0] = c[0] >= n0 ? c[0] - n0 : c[0];
  c[1] = c[1] >= n1 ? c[1] - n1 : c[1];
  c[2] = c[2] >= n2 ? c[2] - n2 : c[2];
  const double o[3] = {static_cast<double>(o0[p]), static_cast<double>(o1[p]), D == 3 ? static_cast<double>(o2[p]) : 0.0};
  double wx[M + 1], wy[M + 1], wz[M + 1];
  int bx, by, bz = 0;
  node_weights<double, M>(c[0], o[0], wx, bx);
  node_weights<double, M>(c[1], o[1], wy, by);
  if (D == 3) node_weights<double, M>(c[2], o[2], wz, bz);
  const double a = qdv * static_cast<double>(w[p]);
  const int kmax = D == 3 ? M : 0;
  for (int k = 0; k <= kmax; ++k) {
    const int gk = D == 3 ? wrap_near(bz + k, n2) : 0;
    const double fz = D == 3 ? wz[k] : 1.0;
    for (int j = 0; j <= M; ++j) {
      const int gj = wrap_near(by + j, n1);
      for (int i = 0; i <= M; ++i) {
        const int gi = wrap_near(bx + i, n0);
        unsafeAtomicAdd(&rho[gi + (int64_t)n0 * (gj + (int64_t)n1 * gk)], a * wx[i] * wy[j] * fz);
      }
    }
  }
}

// The same on sorted particles, one workgroup per tile: the tile's charge is
// accumulated in an LDS box (double) and added to HBM once.  Particles whose
// cell lies more than `slack` cells outside their tile add to HBM directly.
// With `live` (the non-empty tiles of the species' last sort, their count at
// [ntiles]) workgroup b takes the b-th non-empty tile, so that the busy tiles
// of a sparse box (a foil) are dealt over every XCD rather than the few that
// tile-index order maps them to.
template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_rho_tiled(const int32_t *cell, const T *o0, const T *o1, const T *o2,
                                                   const T *w, const int32_t *tile_start, const int32_t *live,
                                                   int64_t ntiles, int64_t np, double qdv,
                                                   int b0, int b1, int m0, int m1, int m2, int n0, int n1, int n2,
                                                   int L0, int L1, int L2, int nt0, int nt1, int slack, double *rho) {
  extern __shared__ double box[];
  int64_t tile = blockIdx.x;
  if (live) {
    if (tile >= live[ntiles]) return;
    tile = live[tile];
  }
  int64_t pbeg = tile_start[tile], pend = tile_start[tile + 1];
  pbeg = pbeg < 0 ? 0 : (pbeg > np ? np : pbeg);
  pend = pend > np ? np : pend;
  if (pbeg >= pend) return;
  const int T0[3] = {static_cast<int>(tile % nt0) * L0, static_cast<int>((tile / nt0) % nt1) * L1,
                     static_cast<int>(tile / ((int64_t)nt0 * nt1)) * L2};
  const int lo = 1 + slack;
  const int bx = L0 + 2 * slack + 3, by = L1 + 2 * slack + 3, bz = D == 3 ? L2 + 2 * slack + 3 : 1;
  const int vol = bx * by * bz;
  for (int i = threadIdx.x; i < vol; i += blockDim.x) box[i] = 0.0;
  __syncthreads();
  const int n[3] = {n0, n1, n2};
  for (int64_t p = pbeg + threadIdx.x; p < pend; p += blockDim.x) {
    const uint32_t pk = static_cast<uint32_t>(cell[p]);
    int c[3] = {static_cast<int>(pk & m0), static_cast<int>((pk >> b0) & m1), static_cast<int>((pk >> (b0 + b1)) & m2)};
    bool inside = true;
    int lc[3] = {0, 0, 0};
    for (int d = 0; d < D; ++d) {
      c[d] = c[d] >= n[d] ? c[d] - n[d] : c[d];
      int l = c[d] - T0[d];
      if (l > n[d] / 2) l -= n[d];
      if (l < -n[d] / 2) l += n[d];
      lc[d] = l;
      const int L = d == 0 ? L0 : (d == 1 ? L1 : L2);
      inside = inside && l >= -slack && l < L + slack;
    }
    const double o[3] = {static_cast<double>(o0[p]), static_cast<double>(o1[p]), D == 3 ? static_cast<double>(o2[p]) : 0.0};
    double wx[M + 1], wy[M + 1], wz[M + 1];
    int ix, iy, iz = 0;
    node_weights<double, M>(inside ? lc[0] : c[0], o[0], wx, ix);
    node_weights<double, M>(inside ? lc[1] : c[1], o[1], wy, iy);
    if (D == 3) node_weights<double, M>(inside ? lc[2] : c[2], o[2], wz, iz);
    const double a = qdv * static_cast<double>(w[p]);
    const int kmax = D == 3 ? M : 0;
    for (int k = 0; k <= kmax; ++k) {
      const double fz = D == 3 ? wz[k] : 1.0;
      for (int j = 0; j <= M; ++j)
        for (int i = 0; i <= M; ++i) {
          const double v = a * wx[i] * wy[j] * fz;
          if (inside) {
            atomicAdd(&box[(ix + i + lo) + bx * ((iy + j + lo) + by * (D == 3 ? iz + k + lo : 0))], v);
          } else {
            const int gi = wrap_near(ix + i, n0), gj = wrap_near(iy + j, n1), gk = D == 3 ? wrap_near(iz + k, n2) : 0;
            unsafeAtomicAdd(&rho[gi + (int64_t)n0 * (gj + (int64_t)n1 * gk)], v);
          }
        }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < vol; idx += blockDim.x) {
    const double v = box[idx];
    if (v == 0.0) continue;
    const int li = idx % bx, lj = (idx / bx) % by, lk = idx / (bx * by);
    int gi = (T0[0] - lo + li) % n0, gj = (T0[1] - lo + lj) % n1, gk = D == 3 ? (T0[2] - lo + lk) % n2 : 0;
    gi = gi < 0 ? gi + n0 : gi;
    gj = gj < 0 ? gj + n1 : gj;
    gk = gk < 0 ? gk + n2 : gk;
    unsafeAtomicAdd(&rho[gi + (int64_t)n0 * (gj + (int64_t)n1 * gk)], v);
  }
}

// Slots 4..7 per node: |rho|, |div E - rho|, |G - G_prev|, |(rho - rho_prev)/dt + div J|;
// then the current rho and G become the previous ones.
// history = 0: rho_prev and g_prev are neither read nor written (may be null).
template <typename T, int D>
__global__ void __launch_bounds__(kB) k_gauss(const T *ex, const T *ey, const T *ez, const T *jx, const T *jy,
                                              const T *jz, const double *rho, double *rho_prev, double *g_prev,
                                              int n0, int n1, int n2, double idx, double idy, double idz, double idt,
                                              int history, int have_prev, int have_cont, double *partials) {
  __shared__ double sh[16];
  const int64_t n = (int64_t)n0 * n1 * n2;
  double mr = 0.0, mg = 0.0, mdg = 0.0, mc = 0.0;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    const int i = static_cast<int>(o % n0);
    const int j = static_cast<int>((o / n0) % n1);
    const int k = static_cast<int>(o / ((int64_t)n0 * n1));
    const int64_t im = i == 0 ? o + (n0 - 1) : o - 1;
    const int64_t jm = j == 0 ? o + (int64_t)n0 * (n1 - 1) : o - n0;
    const int64_t km = k == 0 ? o + (int64_t)n0 * n1 * (n2 - 1) : o - (int64_t)n0 * n1;
    double dE = (static_cast<double>(ex[o]) - ex[im]) * idx + (static_cast<double>(ey[o]) - ey[jm]) * idy;
    double dJ = (static_cast<double>(jx[o]) - jx[im]) * idx + (static_cast<double>(jy[o]) - jy[jm]) * idy;
    if (D == 3) {
      dE += (static_cast<double>(ez[o]) - ez[km]) * idz;
      dJ += (static_cast<double>(jz[o]) - jz[km]) * idz;
    }
    const double r = rho[o];
    const double g = dE - r;
    mr = fmax(mr, fabs(r));
    mg = fmax(mg, fabs(g));
    if (history) {
      if (have_prev) mdg = fmax(mdg, fabs(g - g_prev[o]));
      if (have_cont) mc = fmax(mc, fabs((r - rho_prev[o]) * idt + dJ));
      rho_prev[o] = r;
      g_prev[o] = g;
    }
  }
  mr = block_max(mr, sh);
  mg = block_max(mg, sh);
  mdg = block_max(mdg, sh);
  mc = block_max(mc, sh);
  if (threadIdx.x == 0) {
    partials[4 * kStride + blockIdx.x] = mr;
    partials[5 * kStride + blockIdx.x] = mg;
    partials[6 * kStride + blockIdx.x] = mdg;
    partials[7 * kStride + blockIdx.x] = mc;
  }
}

// G = div E - rho per node (the uniform background excluded), backward
// differences from the E points onto the nodes.
template <typename T, int D>
__global__ void __launch_bounds__(kB) k_gauss_grid(const T *ex, const T *ey, const T *ez, const double *rho, int n0,
                                                   int n1, int n2, double idx, double idy, double idz, double *out) {
  const int64_t n = (int64_t)n0 * n1 * n2;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    const int i = static_cast<int>(o % n0);
    const int j = static_cast<int>((o / n0) % n1);
    const int k = static_cast<int>(o / ((int64_t)n0 * n1));
    const int64_t im = i == 0 ? o + (n0 - 1) : o - 1;
    const int64_t jm = j == 0 ? o + (int64_t)n0 * (n1 - 1) : o - n0;
    const int64_t km = k == 0 ? o + (int64_t)n0 * n1 * (n2 - 1) : o - (int64_t)n0 * n1;
    double dE = (static_cast<double>(ex[o]) - ex[im]) * idx + (static_cast<double>(ey[o]) - ey[jm]) * idy;
    if (D == 3) dE += (static_cast<double>(ez[o]) - ez[km]) * idz;
    out[o] = dE - rho[o];
  }
}

// One workgroup: reduce slot s over cnt[s] entries (sum for 0..3, max for 4..7).
__global__ void __launch_bounds__(1024) k_final(const double *partials, int cnt_fields, int cnt_particles,
                                                int cnt_grid, double dv, double *result) {
  __shared__ double sh[16];
  for (int s = 0; s < kDiagSlots; ++s) {
    const int cnt = s < 2 ? cnt_fields : (s < 4 ? cnt_particles : cnt_grid);
    double v = 0.0;
    if (s < 4) {
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) v += partials[s * kStride + i];
      v = block_sum(v, sh);
    } else {
      for (int i = threadIdx.x; i < cnt; i += blockDim.x) v = fmax(v, partials[s * kStride + i]);
      v = block_max(v, sh);
    }
    if (threadIdx.x == 0) result[s] = s < 2 ? 0.5 * v * dv : v;
  }
}

// Where one diagnostics pass keeps its partial sums, charge grid and result,
// and whether it reads and renews the previous call's rho and G.
struct DiagBufs {
  double *partials;  // [kDiagSlots][kStride]
  double *rho;       // [ncells]
  double *rho_prev;  // [ncells] (history only)
  double *g_prev;    // [ncells] (history only)
  double *result;    // [kDiagSlots]
  bool history, have_prev, have_cont;
};

// rho(node) = sum over the species' particles of q w / dV S(x - node), into
// rho (cleared first): per tile in LDS for sorted species whose tile box
// fits, else one thread per particle with HBM atomics.
template <typename T, int D, int M>
hipError_t charge_grid(const pic_ctx &c, const pic_species *sp, int nsp, double *rho, hipStream_t s) {
  const int64_t n = c.ncells;
  double dV = 1.0;
  for (int d = 0; d < c.p.dims; ++d) dV *= c.p.dx[d];
  hipError_t e = launch_fill_zero(rho, n, 8, s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < nsp; ++i) {
    const pic_species &q = sp[i];
    if (q.np == 0) continue;
    if (q.sorted && q.tile_start) {
      const int sl = c.p.slack;
      size_t box = static_cast<size_t>(c.p.tile[0] + 2 * sl + 3) * (c.p.tile[1] + 2 * sl + 3) *
                   (D == 3 ? c.p.tile[2] + 2 * sl + 3 : 1) * sizeof(double);
      if (box <= 64 * 1024) {
        hipLaunchKernelGGL((k_rho_tiled<T, D, M>), dim3(static_cast<unsigned>(c.ntiles)), dim3(kB), box, s, q.cell,
                           static_cast<const T *>(q.off[0]), static_cast<const T *>(q.off[1]),
                           static_cast<const T *>(q.off[2]), static_cast<const T *>(q.w), q.tile_start,
                           live_tiles(c, q), c.ntiles, q.np,
                           q.q / dV, c.bits[0], c.bits[1], (1 << c.bits[0]) - 1, (1 << c.bits[1]) - 1, (1 << c.bits[2]) - 1,
                           static_cast<int>(c.n[0]), static_cast<int>(c.n[1]), static_cast<int>(c.n[2]),
                           c.p.tile[0], c.p.tile[1], c.p.tile[2], c.ntile[0], c.ntile[1], sl, rho);
        continue;
      }
    }
    const unsigned rb = static_cast<unsigned>((q.np + kB - 1) / kB);
    hipLaunchKernelGGL((k_rho<T, D, M>), dim3(rb), dim3(kB), 0, s, q.cell, static_cast<const T *>(q.off[0]),
                       static_cast<const T *>(q.off[1]), static_cast<const T *>(q.off[2]),
                       static_cast<const T *>(q.w), q.np, q.q / dV, c.bits[0], c.bits[1], (1 << c.bits[0]) - 1,
                       (1 << c.bits[1]) - 1, (1 << c.bits[2]) - 1, static_cast<int>(c.n[0]),
                       static_cast<int>(c.n[1]), static_cast<int>(c.n[2]), rho);
  }
  return hipGetLastError();
}

int grid_blocks(const pic_ctx &c) {
  int gblocks = static_cast<int>((c.ncells + kB - 1) / kB);
  return gblocks > kDiagBlocks ? kDiagBlocks : gblocks;
}

template <typename T, int D, int M>
hipError_t run(const pic_ctx &c, const pic_species *sp, int nsp, const pic_fields &f, const DiagBufs &b,
               hipStream_t s) {
  const int64_t n = c.ncells;
  double dV = 1.0;
  for (int d = 0; d < c.p.dims; ++d) dV *= c.p.dx[d];
  const int gblocks = grid_blocks(c);
  hipLaunchKernelGGL(k_field_sq<T>, dim3(gblocks), dim3(kB), 0, s, static_cast<const T *>(f.E[0]),
                     static_cast<const T *>(f.E[1]), static_cast<const T *>(f.E[2]), static_cast<const T *>(f.B[0]),
                     static_cast<const T *>(f.B[1]), static_cast<const T *>(f.B[2]), n, b.partials);
  // clear the particle slots (species that are empty leave their blocks unused)
  hipError_t e = launch_fill_zero(b.partials + 2 * kStride, 2 * kStride, 8, s);
  if (e != hipSuccess) return e;
  for (int i = 0; i < nsp; ++i) {
    const pic_species &q = sp[i];
    if (q.np == 0) continue;
    int pb = static_cast<int>((q.np + kB - 1) / kB);
    if (pb > kDiagBlocks) pb = kDiagBlocks;
    hipLaunchKernelGGL(k_particle_sums<T>, dim3(pb), dim3(kB), 0, s, static_cast<const T *>(q.u[0]),
                       static_cast<const T *>(q.u[1]), static_cast<const T *>(q.u[2]), static_cast<const T *>(q.w),
                       q.np, q.q, q.m, b.partials, i * kDiagBlocks);
  }
  e = charge_grid<T, D, M>(c, sp, nsp, b.rho, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gauss<T, D>), dim3(gblocks), dim3(kB), 0, s, static_cast<const T *>(f.E[0]),
                     static_cast<const T *>(f.E[1]), static_cast<const T *>(f.E[2]), static_cast<const T *>(f.J[0]),
                     static_cast<const T *>(f.J[1]), static_cast<const T *>(f.J[2]), b.rho, b.rho_prev, b.g_prev,
                     static_cast<int>(c.n[0]), static_cast<int>(c.n[1]), static_cast<int>(c.n[2]), 1.0 / c.p.dx[0],
                     1.0 / c.p.dx[1], c.p.dims == 3 ? 1.0 / c.p.dx[2] : 0.0, 1.0 / c.p.dt, b.history ? 1 : 0,
                     b.have_prev ? 1 : 0, b.have_cont ? 1 : 0, b.partials);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(1024), 0, s, b.partials, gblocks, kMaxSpecies * kDiagBlocks, gblocks, dV,
                     b.result);
  return hipGetLastError();
}

template <typename T, int D, int M>
hipError_t density(const pic_ctx &c, const pic_species *sp, int nsp, const pic_fields *f, double *rho, double *gauss,
                   hipStream_t s) {
  hipError_t e = charge_grid<T, D, M>(c, sp, nsp, rho, s);
  if (e != hipSuccess || !gauss) return e;
  hipLaunchKernelGGL((k_gauss_grid<T, D>), dim3(grid_blocks(c)), dim3(kB), 0, s, static_cast<const T *>(f->E[0]),
                     static_cast<const T *>(f->E[1]), static_cast<const T *>(f->E[2]), rho, static_cast<int>(c.n[0]),
                     static_cast<int>(c.n[1]), static_cast<int>(c.n[2]), 1.0 / c.p.dx[0], 1.0 / c.p.dx[1],
                     c.p.dims == 3 ? 1.0 / c.p.dx[2] : 0.0, gauss);
  return hipGetLastError();
}

#define PIC_DIAG_DISPATCH(F, ...)                                                     \
  do {                                                                                \
    const bool f64 = c.p.precision == PIC_FP64;                                       \
    const int key = (f64 ? 4 : 0) + (c.p.dims == 3 ? 2 : 0) + (c.p.shape_order - 1); \
    switch (key) {                                                                    \
      case 0: return F<float, 2, 1>(__VA_ARGS__);                                    \
      case 1: return F<float, 2, 2>(__VA_ARGS__);                                    \
      case 2: return F<float, 3, 1>(__VA_ARGS__);                                    \
      case 3: return F<float, 3, 2>(__VA_ARGS__);                                    \
      case 4: return F<double, 2, 1>(__VA_ARGS__);                                   \
      case 5: return F<double, 2, 2>(__VA_ARGS__);                                   \
      case 6: return F<double, 3, 1>(__VA_ARGS__);                                   \
      default: return F<double, 3, 2>(__VA_ARGS__);                                  \
    }                                                                                 \
  } while (0)

// Scratch of the allocation-free diagnostics (pic_diagnostics_noalloc): the
// partial sums, the result and a charge grid of at most kScratchCells nodes,
// one copy per GPU, held from module load to process exit.  In host code the
// symbol's name is not a device address; hipGetSymbolAddress gives each
// device's own copy, and only that address is ever passed to a kernel.
constexpr size_t kScratchPartials = static_cast<size_t>(kDiagSlots) * kStride;
constexpr size_t kScratchResult = 16;
static __device__ __align__(256) double scratch[kScratchPartials + kScratchResult + kScratchCells];

}  // namespace

hipError_t launch_diagnostics(const pic_ctx &c, const pic_species *sp, int nspecies, const pic_fields &f,
                              bool have_prev, bool have_cont, hipStream_t s) {
  DiagBufs b{c.wsp<double>(c.ws.partials), c.wsp<double>(c.ws.rho), c.wsp<double>(c.ws.rho_prev),
             c.wsp<double>(c.ws.gauss_prev), c.wsp<double>(c.ws.result), true, have_prev, have_cont};
  PIC_DIAG_DISPATCH(run, c, sp, nspecies, f, b, s);
}

hipError_t launch_charge_density(const pic_ctx &c, const pic_species *sp, int nspecies, const pic_fields *f,
                                 double *rho, double *gauss, hipStream_t s) {
  PIC_DIAG_DISPATCH(density, c, sp, nspecies, f, rho, gauss, s);
}

hipError_t scratch_address(double **out) {
  // one address per device, looked up once with that device current
  static std::mutex mu;
  static double *addr[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = static_cast<double *>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

hipError_t launch_diagnostics_noalloc(const pic_ctx &c, const pic_species *sp, int nspecies, const pic_fields &f,
                                      double *scratch_ptr, hipStream_t s) {
  if (c.ncells > kScratchCells) return hipErrorInvalidValue;
  DiagBufs b{scratch_ptr, scratch_ptr + kScratchPartials + kScratchResult, nullptr, nullptr,
             scratch_ptr + kScratchPartials, false, false, false};
  PIC_DIAG_DISPATCH(run, c, sp, nspecies, f, b, s);
}

size_t scratch_result_offset() { return kScratchPartials; }

}  // namespace pic
