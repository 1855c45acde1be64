// Particle kernels: the unfused gather+push and deposit pair (particles in any
// order, fields and current in HBM), and the fused per-tile kernel that
// stages the tile's E and B in LDS, accumulates J in LDS and merges it into
// HBM once.  Dispatch over precision x dimensions x shape order.
#include <hip/hip_runtime.h>

#include "particle_math.h"
#include "pic_internal.h"

namespace pic {
namespace {

template <typename T>
struct SpeciesArgs {
  int64_t np;
  int32_t *cell;
  T *off[3];
  T *u[3];
  const T *w;
  T h;          // q dt / (2 m)
  T dtdx[3];    // dt / dx_d
  T jc[3];      // (q / dV)(dx_d / dt), times w per particle
  T jz;         // q / dV (2D J_z), times w v_z per particle
};

struct GridArgs {
  int n[3];
  int bits[3];
  int mask[3];
};

// Packed cell -> per-dimension cells, each reduced into [0, n) (a field
// holds values below 2^bits < 2n, so one subtraction suffices).
__device__ __forceinline__ void unpack(int32_t packed, const GridArgs &g, int c[3]) {
  const uint32_t p = static_cast<uint32_t>(packed);
  c[0] = static_cast<int>(p & g.mask[0]);
  c[1] = static_cast<int>((p >> g.bits[0]) & g.mask[1]);
  c[2] = static_cast<int>((p >> (g.bits[0] + g.bits[1])) & g.mask[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) c[d] = c[d] >= g.n[d] ? c[d] - g.n[d] : c[d];
}

// Full periodic reduction (tile staging, where guard boxes may exceed n).
__device__ __forceinline__ int wrap_full(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int32_t pack(const int c[3], const GridArgs &g) {
  return static_cast<int32_t>(static_cast<uint32_t>(c[0]) | (static_cast<uint32_t>(c[1]) << g.bits[0]) |
                              (static_cast<uint32_t>(c[2]) << (g.bits[0] + g.bits[1])));
}

template <typename T, int D>
__device__ __forceinline__ void load_particle(const SpeciesArgs<T> &s, int64_t p, T o[3], T u[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) o[d] = d < D ? s.off[d][p] : T(0);
  u[0] = s.u[0][p];
  u[1] = s.u[1][p];
  u[2] = s.u[2][p];
}

// ---------------------------------------------------------------------------
// Unfused: gather + Boris + move, old position saved for the deposit.
// ---------------------------------------------------------------------------
template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_gather_push(SpeciesArgs<T> s, GridArgs g, GlobalFields<T> f,
                                                     int32_t *save_cell, T *save_off0, T *save_off1, T *save_off2,
                                                     int32_t *flags) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= s.np) return;
  int c[3];
  const int32_t packed = s.cell[p];
  unpack(packed, g, c);
  T o[3], u[3];
  load_particle<T, D>(s, p, o, u);
  save_cell[p] = packed;
  save_off0[p] = o[0];
  save_off1[p] = o[1];
  if (D == 3) save_off2[p] = o[2];
  T eb[6];
  gather_eb<T, D, M>(f, c, o, eb);
  boris<T>(u, eb, s.h);
  const T ig = rsqrt_t<T>(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  T on[3] = {T(0), T(0), T(0)};
  int dc[3] = {0, 0, 0};
  if (!move<T, D>(u, ig, s.dtdx, o, on, dc)) {
    atomicOr(&flags[0], kFlagCross);
    save_cell[p] = -1;  // packed cells are non-negative: -1 tells the deposit to skip
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    c[d] = wrap_near(c[d] + dc[d], g.n[d]);
    s.off[d][p] = on[d];
  }
  s.cell[p] = pack(c, g);
  s.u[0][p] = u[0];
  s.u[1][p] = u[1];
  s.u[2][p] = u[2];
}

// Unfused: Esirkepov deposit of the move recorded by k_gather_push.
template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_deposit(SpeciesArgs<T> s, GridArgs g, GlobalCurrent<T> J,
                                                 const int32_t *save_cell, const T *save_off0, const T *save_off1,
                                                 const T *save_off2) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= s.np) return;
  const int32_t saved = save_cell[p];
  if (saved < 0) return;  // frozen by the push (displacement of a cell or more, or non-finite)
  int c0[3], c1[3];
  unpack(saved, g, c0);
  unpack(s.cell[p], g, c1);
  T o0[3] = {save_off0[p], save_off1[p], D == 3 ? save_off2[p] : T(0)};
  T o1[3], u[3];
  load_particle<T, D>(s, p, o1, u);
  int dc[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < D; ++d) {
    int k = c1[d] - c0[d];
    if (k > 1) k -= g.n[d];
    if (k < -1) k += g.n[d];
    dc[d] = k;
  }
  const T w = s.w[p];
  const T jc[3] = {w * s.jc[0], w * s.jc[1], w * s.jc[2]};
  const T ig = rsqrt_t<T>(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  T jz = T(0);
  if (D == 2) jz = w * s.jz * u[2] * ig;
  deposit<T, D, M>(J, c0, o0, dc, o1, jc, jz);
}

// ---------------------------------------------------------------------------
// Fused per-tile kernel.
// ---------------------------------------------------------------------------
struct TileArgs {
  const int32_t *tile_start;
  int L[3];       // tile size
  int ntile[3];   // tiles per dimension
  int slack;
  int rf[3], rj[3];        // LDS field / current box sizes
  int gf_lo[3], gj_lo[3];  // box origins below the tile origin
  int remap;               // 1: spread consecutive tiles over XCDs in blocks
};

template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_push_deposit_tiled(SpeciesArgs<T> s, GridArgs g, GlobalFields<T> gf,
                                                            GlobalCurrent<T> gj, TileArgs t, int32_t *flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *smem = reinterpret_cast<T *>(smem_raw);
  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous range of tiles so neighbouring tiles share its L2.
  int64_t tile = blockIdx.x;
  if (t.remap) {
    const int64_t per = gridDim.x / 8;
    tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
  }
  const int64_t pbeg = t.tile_start[tile], pend = t.tile_start[tile + 1];
  if (pbeg >= pend) return;
  const int tx = static_cast<int>(tile % t.ntile[0]);
  const int ty = static_cast<int>((tile / t.ntile[0]) % t.ntile[1]);
  const int tz = static_cast<int>(tile / ((int64_t)t.ntile[0] * t.ntile[1]));
  const int T0[3] = {tx * t.L[0], ty * t.L[1], tz * t.L[2]};

  const int fvol = t.rf[0] * t.rf[1] * t.rf[2];
  const int jvol = t.rj[0] * t.rj[1] * t.rj[2];
  T *fl = smem;
  T *jl = smem + 6 * fvol;

  // stage E, B of the tile plus guards (periodic wrap)
  for (int idx = threadIdx.x; idx < fvol; idx += blockDim.x) {
    const int li = idx % t.rf[0];
    const int lj = (idx / t.rf[0]) % t.rf[1];
    const int lk = idx / (t.rf[0] * t.rf[1]);
    int gi = T0[0] - t.gf_lo[0] + li, gjj = T0[1] - t.gf_lo[1] + lj, gk = T0[2] - t.gf_lo[2] + lk;
    gi = wrap_full(gi, g.n[0]);
    gjj = wrap_full(gjj, g.n[1]);
    gk = D == 3 ? wrap_full(gk, g.n[2]) : 0;
    const int64_t gidx = gi + (int64_t)g.n[0] * (gjj + (int64_t)g.n[1] * gk);
#pragma unroll
    for (int c = 0; c < 6; ++c) fl[c * fvol + idx] = gf.F[c][gidx];
  }
  for (int idx = threadIdx.x; idx < 3 * jvol; idx += blockDim.x) jl[idx] = T(0);
  __syncthreads();

  // local frames: the tile origin is (0,0,0)
  const LdsFields<T> lf{fl, t.rf[0], t.rf[0] * t.rf[1], fvol, -t.gf_lo[0], -t.gf_lo[1], D == 3 ? -t.gf_lo[2] : 0};
  const LdsCurrent<T> lj{jl, t.rj[0], t.rj[0] * t.rj[1], jvol, -t.gj_lo[0], -t.gj_lo[1], D == 3 ? -t.gj_lo[2] : 0};

  for (int64_t p = pbeg + threadIdx.x; p < pend; p += blockDim.x) {
    int c[3];
    unpack(s.cell[p], g, c);
    T o[3], u[3];
    load_particle<T, D>(s, p, o, u);
    // cell relative to the tile origin, unwrapped across the periodic seam
    int lc[3] = {0, 0, 0};
    bool inside = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      int l = c[d] - T0[d];
      if (l > g.n[d] / 2) l -= g.n[d];
      if (l < -g.n[d] / 2) l += g.n[d];
      lc[d] = l;
      inside = inside && (l >= -t.slack) && (l < t.L[d] + t.slack);
    }
    T eb[6];
    if (inside)
      gather_eb<T, D, M>(lf, lc, o, eb);
    else
      gather_eb<T, D, M>(gf, c, o, eb);
    boris<T>(u, eb, s.h);
    const T ig = rsqrt_t<T>(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    T on[3] = {T(0), T(0), T(0)};
    int dc[3] = {0, 0, 0};
    const bool ok = move<T, D>(u, ig, s.dtdx, o, on, dc);
    if (!ok) atomicOr(&flags[0], kFlagCross);
    const T w = s.w[p];
    const T jc[3] = {w * s.jc[0], w * s.jc[1], w * s.jc[2]};
    const T jz = D == 2 ? w * s.jz * u[2] * ig : T(0);
    if (ok) {
      if (inside)
        deposit<T, D, M>(lj, lc, o, dc, on, jc, jz);
      else
        deposit<T, D, M>(gj, c, o, dc, on, jc, jz);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      c[d] = wrap_near(c[d] + dc[d], g.n[d]);
      s.off[d][p] = on[d];
    }
    s.cell[p] = pack(c, g);
    s.u[0][p] = u[0];
    s.u[1][p] = u[1];
    s.u[2][p] = u[2];
  }
  __syncthreads();

  // merge the current tile into HBM (skipping cells nothing touched)
  for (int idx = threadIdx.x; idx < jvol; idx += blockDim.x) {
    const int li = idx % t.rj[0];
    const int lj2 = (idx / t.rj[0]) % t.rj[1];
    const int lk = idx / (t.rj[0] * t.rj[1]);
    const int gi = wrap_full(T0[0] - t.gj_lo[0] + li, g.n[0]);
    const int gjj = wrap_full(T0[1] - t.gj_lo[1] + lj2, g.n[1]);
    const int gk = D == 3 ? wrap_full(T0[2] - t.gj_lo[2] + lk, g.n[2]) : 0;
    const int64_t gidx = gi + (int64_t)g.n[0] * (gjj + (int64_t)g.n[1] * gk);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const T v = jl[c * jvol + idx];
      if (v != T(0)) unsafeAtomicAdd(&gj.J[c][gidx], v);
    }
  }
}

// ---------------------------------------------------------------------------
// Host-side argument assembly and dispatch.
// ---------------------------------------------------------------------------
template <typename T>
SpeciesArgs<T> species_args(const pic_ctx &c, const pic_species &sp) {
  SpeciesArgs<T> s{};
  s.np = sp.np;
  s.cell = sp.cell;
  for (int d = 0; d < 3; ++d) {
    s.off[d] = static_cast<T *>(sp.off[d]);
    s.u[d] = static_cast<T *>(sp.u[d]);
  }
  s.w = static_cast<const T *>(sp.w);
  const double dt = c.p.dt;
  double dV = 1.0;
  for (int d = 0; d < c.p.dims; ++d) dV *= c.p.dx[d];
  s.h = static_cast<T>(sp.q * dt / (2.0 * sp.m));
  for (int d = 0; d < 3; ++d) {
    s.dtdx[d] = static_cast<T>(d < c.p.dims ? dt / c.p.dx[d] : 0.0);
    s.jc[d] = static_cast<T>(d < c.p.dims ? sp.q / dV * c.p.dx[d] / dt : 0.0);
  }
  s.jz = static_cast<T>(sp.q / dV);
  return s;
}

GridArgs grid_args(const pic_ctx &c) {
  GridArgs g{};
  for (int d = 0; d < 3; ++d) {
    g.n[d] = static_cast<int>(c.n[d]);
    g.bits[d] = c.bits[d];
    g.mask[d] = (1 << c.bits[d]) - 1;
  }
  return g;
}

template <typename T>
GlobalFields<T> global_fields(const pic_ctx &c, const pic_fields &f) {
  GlobalFields<T> g{};
  for (int d = 0; d < 3; ++d) {
    g.F[d] = static_cast<const T *>(f.E[d]);
    g.F[3 + d] = static_cast<const T *>(f.B[d]);
    g.n[d] = static_cast<int>(c.n[d]);
  }
  return g;
}

template <typename T>
GlobalCurrent<T> global_current(const pic_ctx &c, const pic_fields &f) {
  GlobalCurrent<T> g{};
  for (int d = 0; d < 3; ++d) {
    g.J[d] = static_cast<T *>(f.J[d]);
    g.n[d] = static_cast<int>(c.n[d]);
  }
  return g;
}

template <typename T, int D, int M>
hipError_t gather_push_impl(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  const int64_t mp = c.p.max_particles;
  T *so = c.wsp<T>(c.ws.save_off);
  const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
  hipLaunchKernelGGL((k_gather_push<T, D, M>), dim3(blocks), dim3(256), 0, st, species_args<T>(c, sp), grid_args(c),
                     global_fields<T>(c, f), c.wsp<int32_t>(c.ws.save_cell), so, so + mp, so + 2 * mp,
                     c.wsp<int32_t>(c.ws.flags));
  return hipGetLastError();
}

template <typename T, int D, int M>
hipError_t deposit_impl(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  const int64_t mp = c.p.max_particles;
  const T *so = c.wsp<T>(c.ws.save_off);
  const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
  hipLaunchKernelGGL((k_deposit<T, D, M>), dim3(blocks), dim3(256), 0, st, species_args<T>(c, sp), grid_args(c),
                     global_current<T>(c, f), c.wsp<int32_t>(c.ws.save_cell), so, so + mp, so + 2 * mp);
  return hipGetLastError();
}

template <typename T, int D, int M>
hipError_t tiled_impl(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  TileArgs t{};
  t.tile_start = sp.tile_start;
  for (int d = 0; d < 3; ++d) {
    t.L[d] = c.p.tile[d];
    t.ntile[d] = c.ntile[d];
    t.rf[d] = c.rf[d];
    t.rj[d] = c.rj[d];
    t.gf_lo[d] = c.gf_lo[d];
    t.gj_lo[d] = c.gj_lo[d];
  }
  t.slack = c.p.slack;
  t.remap = (c.ntiles % 8 == 0 && c.ntiles >= 64) ? 1 : 0;
  const auto kern = k_push_deposit_tiled<T, D, M>;
  const size_t lds = c.lds_bytes;
  static size_t lds_set = 0;  // largest dynamic LDS size granted to this instantiation
  if (lds > 65536 && lds > lds_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    lds_set = lds;
  }
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(c.ntiles)), dim3(c.block), lds, st, species_args<T>(c, sp),
                     grid_args(c), global_fields<T>(c, f), global_current<T>(c, f), t, c.wsp<int32_t>(c.ws.flags));
  return hipGetLastError();
}

template <template <typename, int, int> class F, typename... A>
hipError_t dispatch(const pic_ctx &c, A &&...a);

#define PIC_DISPATCH(IMPL, ...)                                                     \
  do {                                                                              \
    const bool f64 = c.p.precision == PIC_FP64;                                     \
    const int key = (f64 ? 4 : 0) + (c.p.dims == 3 ? 2 : 0) + (c.p.shape_order - 1); \
    switch (key) {                                                                  \
      case 0: return IMPL<float, 2, 1>(__VA_ARGS__);                               \
      case 1: return IMPL<float, 2, 2>(__VA_ARGS__);                               \
      case 2: return IMPL<float, 3, 1>(__VA_ARGS__);                               \
      case 3: return IMPL<float, 3, 2>(__VA_ARGS__);                               \
      case 4: return IMPL<double, 2, 1>(__VA_ARGS__);                              \
      case 5: return IMPL<double, 2, 2>(__VA_ARGS__);                              \
      case 6: return IMPL<double, 3, 1>(__VA_ARGS__);                              \
      default: return IMPL<double, 3, 2>(__VA_ARGS__);                             \
    }                                                                               \
  } while (0)

}  // namespace

hipError_t launch_gather_push(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t s) {
  PIC_DISPATCH(gather_push_impl, c, sp, f, s);
}

hipError_t launch_deposit(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t s) {
  PIC_DISPATCH(deposit_impl, c, sp, f, s);
}

hipError_t launch_push_deposit_tiled(const pic_ctx &c, const pic_species &sp, const pic_fields &f, hipStream_t s) {
  PIC_DISPATCH(tiled_impl, c, sp, f, s);
}

}  // namespace pic
