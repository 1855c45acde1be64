// Particle kernels: the unfused gather+push and deposit pair (particles in any
// order, fields and current in HBM), and the fused per-tile kernel that
// stages the tile's E and B in LDS, accumulates J in LDS and merges it into
// HBM once.  Dispatch over precision x dimensions x shape order.
#include <hip/hip_runtime.h>

#include <type_traits>

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
  T *w;         // written only to remove a particle at an open x face
  int open;     // 1: open x faces; weight-0 particles are inert
  int xlo, xhi; // live x cells [xlo, xhi) when open
  T h;          // q dt / (2 m)
  T dtdx[3];    // dt / dx_d
  T jc[3];      // (q / dV)(dx_d / dt), times w per particle
  T jz;         // q / dV (2D J_z), times w v_z per particle
  // The fused kernel reads particle q at src[q] when src is set (a sort whose
  // copy it takes over) and writes it to the *_o arrays, which otherwise are
  // the arrays above.
  const int32_t *src;
  int64_t np_src;  // particles in the arrays src indexes (a sort may have dropped removed ones since)
  int32_t *cell_o;
  T *off_o[3];
  T *u_o[3];
  T *w_o;
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

// After a move: remove the particle (weight 0) if its x cell left the live
// range of an open box.  Its current for this move is already deposited.
template <typename T>
__device__ __forceinline__ void absorb_if_out(const SpeciesArgs<T> &s, int64_t p, int cx) {
  if (s.open && (cx < s.xlo || cx >= s.xhi)) s.w[p] = T(0);
}

// Deal each wavefront's particles to lanes by the bank residue of their
// deposit window (the fused kernel in 3D, where the deposit's 54 FP64 LDS
// atomics per particle weigh most; in 2D, with 21, the exchange costs more
// than it saves).
constexpr bool kDealLanes = true;

// A value sent from this lane to lane to/4 of the wavefront.
__device__ __forceinline__ int32_t lane_push(int to, int32_t v) { return __builtin_amdgcn_ds_permute(to, v); }
__device__ __forceinline__ float lane_push(int to, float v) {
  return __int_as_float(__builtin_amdgcn_ds_permute(to, __float_as_int(v)));
}
__device__ __forceinline__ double lane_push(int to, double v) {
  const int lo = __builtin_amdgcn_ds_permute(to, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_permute(to, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

// The Esirkepov deposit (3D) of a particle whose nearest node (cell, for the
// linear shape) changed along at least one axis, into the LDS current box
// jl (origin -jlo, strides 1, jx, jxy, component stride jvol).  The current
// along each axis depends symmetrically on the two axes across it, so a
// cyclic relabelling of the axes leaves it unchanged.  Each lane relabels
// its axes so that one it crossed comes first: that axis takes the wide
// window (M + 2 nodes) in every lane, the other two take M + 1 nodes, or
// M + 2 where they crossed as well (rare).  A wavefront of such particles
// then runs one set of loops: 75 adds per particle for the quadratic shape
// (20 for the linear one) where the general form issues 144 (54) divergent,
// zero-tested slots.  The nodes it skips carry exact zeros.  Every add goes
// through per-lane strides.
template <typename T, int M, typename S>
__device__ __forceinline__ void esirkepov_rotated(S *jl, int jx, int jxy, int jvol, int jlo, const int c0[3],
                                                  const T o0[3], const int dc[3], const T o1[3], const T jc[3]) {
  constexpr int WN = M + 1, WW = M + 2;  // narrow and wide node counts
  bool cr[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if constexpr (M == 2) {
      const int n0 = o0[d] >= T(0.5) ? 1 : 0;
      cr[d] = dc[d] + (o1[d] >= T(0.5) ? 1 : 0) != n0;
    } else {
      cr[d] = dc[d] != 0;
    }
  }
  const int a = cr[0] ? 0 : (cr[1] ? 1 : 2);  // the leading axis: one that was crossed
  const int ax[3] = {a, a == 2 ? 0 : a + 1, a == 0 ? 2 : a - 1};
  T p0[3], p1[3], pc[3];
  int pdc[3], st[3], cb[3];
  bool wide[3];
  int org = 0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int d = ax[r];
    p0[r] = d == 0 ? o0[0] : (d == 1 ? o0[1] : o0[2]);
    p1[r] = d == 0 ? o1[0] : (d == 1 ? o1[1] : o1[2]);
    pdc[r] = d == 0 ? dc[0] : (d == 1 ? dc[1] : dc[2]);
    pc[r] = d == 0 ? jc[0] : (d == 1 ? jc[1] : jc[2]);
    st[r] = d == 0 ? 1 : (d == 1 ? jx : jxy);
    cb[r] = d * jvol;
    wide[r] = d == 0 ? cr[0] : (d == 1 ? cr[1] : cr[2]);
  }
  Esirk<T, M> e;
  esirkepov_factors<T, 3, M>(p0, pdc, p1, e);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int d = ax[r];
    org += st[r] * ((d == 0 ? c0[0] : (d == 1 ? c0[1] : c0[2])) + e.b[r] + jlo);
  }
  // along the leading axis: its M + 1 edges, nodes across
#pragma unroll
  for (int k = 0; k < WW; ++k)
    if (k < WN || wide[2])
#pragma unroll
      for (int j = 0; j < WW; ++j)
        if (j < WN || wide[1]) {
          const T t = e.A[1][j] * e.S0[2][k] + e.Bf[1][j] * e.DS[2][k];
#pragma unroll
          for (int i = 0; i < WW - 1; ++i)
            lds_add(&jl[cb[0] + org + i * st[0] + j * st[1] + k * st[2]], -pc[0] * e.CDS[0][i] * t);
        }
  // along the second axis
#pragma unroll
  for (int k = 0; k < WW; ++k)
    if (k < WN || wide[2])
#pragma unroll
      for (int i = 0; i < WW; ++i) {
        const T t = e.A[0][i] * e.S0[2][k] + e.Bf[0][i] * e.DS[2][k];
#pragma unroll
        for (int j = 0; j < WW - 1; ++j)
          if (j < WN - 1 || wide[1])
            lds_add(&jl[cb[1] + org + i * st[0] + j * st[1] + k * st[2]], -pc[1] * e.CDS[1][j] * t);
      }
  // along the third axis
#pragma unroll
  for (int j = 0; j < WW; ++j)
    if (j < WN || wide[1])
#pragma unroll
      for (int i = 0; i < WW; ++i) {
        const T t = e.A[0][i] * e.S0[1][j] + e.Bf[0][i] * e.DS[1][j];
#pragma unroll
        for (int k = 0; k < WW - 1; ++k)
          if (k < WN - 1 || wide[2])
            lds_add(&jl[cb[2] + org + i * st[0] + j * st[1] + k * st[2]], -pc[2] * e.CDS[2][k] * t);
      }
}

// The same in 2D3V: the axes x and y swap when only y was crossed.  J_z,
// the time-averaged shape product times v_z, is symmetric in them too.  29
// adds per particle for the quadratic shape (12 for the linear one) where the
// general form issues 40 (21) zero-tested slots.
template <typename T, int M, typename S>
__device__ __forceinline__ void esirkepov_rotated_2d(S *jl, int jx, int jvol, int jlo, const int c0[3],
                                                     const T o0[3], const int dc[3], const T o1[3], const T jc[3],
                                                     T jzc) {
  constexpr int WN = M + 1, WW = M + 2;
  bool cr[2];
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    if constexpr (M == 2) {
      const int n0 = o0[d] >= T(0.5) ? 1 : 0;
      cr[d] = dc[d] + (o1[d] >= T(0.5) ? 1 : 0) != n0;
    } else {
      cr[d] = dc[d] != 0;
    }
  }
  const bool sw = !cr[0];  // lead with y
  const T p0[3] = {sw ? o0[1] : o0[0], sw ? o0[0] : o0[1], T(0)};
  const T p1[3] = {sw ? o1[1] : o1[0], sw ? o1[0] : o1[1], T(0)};
  const int pdc[3] = {sw ? dc[1] : dc[0], sw ? dc[0] : dc[1], 0};
  const T pc[2] = {sw ? jc[1] : jc[0], sw ? jc[0] : jc[1]};
  const int st[2] = {sw ? jx : 1, sw ? 1 : jx};
  const int cb[2] = {sw ? jvol : 0, sw ? 0 : jvol};
  const bool wide1 = sw ? cr[0] : cr[1];
  Esirk<T, M> e;
  esirkepov_factors<T, 2, M>(p0, pdc, p1, e);
  const int org = st[0] * ((sw ? c0[1] : c0[0]) + e.b[0] + jlo) + st[1] * ((sw ? c0[0] : c0[1]) + e.b[1] + jlo);
  // along the leading axis
#pragma unroll
  for (int j = 0; j < WW; ++j)
    if (j < WN || wide1) {
      const T t = e.A[1][j];
#pragma unroll
      for (int i = 0; i < WW - 1; ++i)
        lds_add(&jl[cb[0] + org + i * st[0] + j * st[1]], -pc[0] * e.CDS[0][i] * t);
    }
  // along the other in-plane axis
#pragma unroll
  for (int i = 0; i < WW; ++i) {
    const T t = e.A[0][i];
#pragma unroll
    for (int j = 0; j < WW - 1; ++j)
      if (j < WN - 1 || wide1)
        lds_add(&jl[cb[1] + org + i * st[0] + j * st[1]], -pc[1] * e.CDS[1][j] * t);
  }
  // out of the plane
  if (jzc != T(0))
#pragma unroll
    for (int j = 0; j < WW; ++j)
      if (j < WN || wide1)
#pragma unroll
        for (int i = 0; i < WW; ++i)
          lds_add(&jl[2 * jvol + org + i * st[0] + j * st[1]], jzc * (e.A[0][i] * e.S0[1][j] + e.Bf[0][i] * e.DS[1][j]));
}

// Element i of a particle array.  With SMALL (index times element size
// below 2^32) the byte offset is formed in 32 bits, so the arrays of one
// particle share a single offset register against their scalar bases instead
// of a 64-bit address each.
template <bool SMALL, typename P>
__device__ __forceinline__ P &elem(P *base, int64_t i) {
  if constexpr (SMALL) {
    using B = std::conditional_t<std::is_const<P>::value, const char, char>;
    return *reinterpret_cast<P *>(reinterpret_cast<B *>(base) +
                                  static_cast<uint32_t>(i) * static_cast<uint32_t>(sizeof(P)));
  } else {
    return base[i];
  }
}

template <typename T, int D, bool SMALL = false>
__device__ __forceinline__ void load_particle(const SpeciesArgs<T> &s, int64_t p, T o[3], T u[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) o[d] = d < D ? elem<SMALL>(s.off[d], p) : T(0);
  u[0] = elem<SMALL>(s.u[0], p);
  u[1] = elem<SMALL>(s.u[1], p);
  u[2] = elem<SMALL>(s.u[2], p);
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
  if (s.open && s.w[p] == T(0)) {  // removed: inert, and the deposit skips it
    save_cell[p] = -1;
    return;
  }
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
  absorb_if_out(s, p, c1[0]);
}

// ---------------------------------------------------------------------------
// Fused per-tile kernel.
// ---------------------------------------------------------------------------
// Local cell (within [-32, 32) of the tile origin) and cell change per axis in one int.
__device__ __forceinline__ int32_t pack_local(const int lc[3], const int dc[3]) {
  int32_t v = 0;
#pragma unroll
  for (int d = 0; d < 3; ++d) v |= (((lc[d] + 32) & 63) | ((dc[d] + 1) << 6)) << (8 * d);
  return v;
}

__device__ __forceinline__ void unpack_local(int32_t v, int lc[3], int dc[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int b = (v >> (8 * d)) & 255;
    lc[d] = (b & 63) - 32;
    dc[d] = (b >> 6) - 1;
  }
}

struct TileArgs {
  const int32_t *tile_start;
  int L[3];       // tile size
  int ntile[3];   // tiles per dimension
  int slack;
  int rf[3], rj[3];        // LDS field / current box sizes
  int jxy;                 // plane stride of the current box (padded in 3D)
  int gf_lo[3], gj_lo[3];  // box origins below the tile origin
  int remap;               // 1: spread consecutive tiles over XCDs in blocks
  const int32_t *live;     // non-empty tiles in order, count at [ntiles] (null: every tile)
  int64_t ntiles;
  int32_t *stray_count;    // particles left outside their LDS box (handled by k_stragglers)
  int32_t *stray_list;
  int32_t *queue;          // [8]: next item of each XCD's range, zero at launch
  int cross_cap;           // entries of the LDS list of wide-window particles
  uint32_t *wcache;        // [ntiles]: per tile, the bits of its largest |w| (fixed-point current)
  int wmode;               // 0: find each tile's bound; 1: find and store it in wcache; 2: take it from wcache
};

__device__ __forceinline__ float scale2(float x, int e) { return ldexpf(x, e); }
__device__ __forceinline__ double scale2(double x, int e) { return ldexp(x, e); }

// The power-of-two shift of a tile's fixed-point current: every contribution
// is bounded by max_d |jc_d| w_max (2D J_z: |jz| w_max, since |v_z| < 1),
// w_max the largest |w| among the tile's particles, and the shift brings that
// bound to at most 2^30.
template <typename T>
__device__ __forceinline__ int fixed_shift(const SpeciesArgs<T> &s, float wmax, int dims) {
  float c = fmaxf(fabsf(static_cast<float>(s.jc[0])), fabsf(static_cast<float>(s.jc[1])));
  c = fmaxf(c, fabsf(static_cast<float>(dims == 3 ? s.jc[2] : s.jz)));
  c *= wmax;
  if (!(c > 0.f) || !isfinite(c)) return 0;
  int e = 0;
  frexpf(c, &e);  // c < 2^e
  return 30 - e;
}

// Tile geometry known at compile time: LDS offsets fold into immediates.
template <int D, int M, int LX, int LY, int LZ, int SL>
struct FixedGeom {
  static constexpr int L0 = LX, L1 = LY, L2 = D == 3 ? LZ : 1, S = SL;
  static constexpr int FLO = 1 + SL, JLO = M + SL;
  // the field box's rows are padded to an even length (pair reads in the gather)
  static constexpr int FX = (LX + 1 + M + 2 * SL + 1) / 2 * 2, FY = LY + 1 + M + 2 * SL,
                       FZ = D == 3 ? LZ + 1 + M + 2 * SL : 1;
  static constexpr int JX = LX + 2 * M + 1 + 2 * SL, JY = LY + 2 * M + 1 + 2 * SL,
                       JZ = D == 3 ? LZ + 2 * M + 1 + 2 * SL : 1;
  static constexpr int JXY = current_plane_stride(JX, JY, D);
  static constexpr int FVOL = FX * FY * FZ, JVOL = JXY * JZ;
  __device__ explicit FixedGeom(const TileArgs &) {}
};

// Tile geometry from the launch arguments (any tile shape).
struct RuntimeGeom {
  int L0, L1, L2, S, FLO, JLO, FX, FY, FZ, JX, JY, JZ, JXY, FVOL, JVOL;
  __device__ explicit RuntimeGeom(const TileArgs &t)
      : L0(t.L[0]), L1(t.L[1]), L2(t.L[2]), S(t.slack), FLO(t.gf_lo[0]), JLO(t.gj_lo[0]), FX(t.rf[0]), FY(t.rf[1]),
        FZ(t.rf[2]), JX(t.rj[0]), JY(t.rj[1]), JZ(t.rj[2]), JXY(t.jxy), FVOL(t.rf[0] * t.rf[1] * t.rf[2]),
        JVOL(t.jxy * t.rj[2]) {}
};

template <typename T, class G, int D>
struct FieldBox;
template <typename T, class G, int D>
struct CurrentBox;

template <typename T, int D, int M, int LX, int LY, int LZ, int SL, int DD>
struct FieldBox<T, FixedGeom<D, M, LX, LY, LZ, SL>, DD> {
  using G = FixedGeom<D, M, LX, LY, LZ, SL>;
  using type = LdsBox<T, G::FX, G::FX * G::FY, G::FVOL, G::FLO, G::FLO, D == 3 ? G::FLO : 0>;
  __device__ static type make(T *base, const G &) { return type{base}; }
};
template <typename T, int D, int M, int LX, int LY, int LZ, int SL, int DD>
struct CurrentBox<T, FixedGeom<D, M, LX, LY, LZ, SL>, DD> {
  using G = FixedGeom<D, M, LX, LY, LZ, SL>;
  using type = LdsBox<T, G::JX, G::JXY, G::JVOL, G::JLO, G::JLO, D == 3 ? G::JLO : 0>;
  __device__ static type make(T *base, const G &) { return type{base}; }
};
template <typename T, int DD>
struct FieldBox<T, RuntimeGeom, DD> {
  using type = LdsFields<T>;
  __device__ static type make(T *base, const RuntimeGeom &g) {
    return type{base, g.FX, g.FX * g.FY, g.FVOL, -g.FLO, -g.FLO, DD == 3 ? -g.FLO : 0};
  }
};
template <typename T, int DD>
struct CurrentBox<T, RuntimeGeom, DD> {
  using type = LdsCurrent<T>;
  __device__ static type make(T *base, const RuntimeGeom &g) {
    return type{base, g.JX, g.JXY, g.JVOL, -g.JLO, -g.JLO, DD == 3 ? -g.JLO : 0};
  }
};

// Persistent workgroups, each taking one tile of sorted particles at a time:
// stage E and B of the tile plus guards in LDS, push every particle whose
// cell lies within the slack of the tile (gather from LDS, Boris, move,
// Esirkepov into an LDS current box held in TJ), then add the current box
// into J in HBM.  Particles further out are listed for k_stragglers.
// FOLD: the launch takes over a sort's copy (reads through s.src, writes the
// *_o arrays); otherwise it updates the particles in place and never touches
// those pointers, which keeps them out of the registers.
// SMALL: every byte offset into a particle array of the launch (the
// particles it reads, through src or not, and writes) fits in 32 bits.
template <typename T, int D, int M, class G, int BLOCK, typename TJ, bool FOLD, bool SMALL>
__global__ void __launch_bounds__(BLOCK) k_push_deposit_tiled(SpeciesArgs<T> s, GridArgs g, GlobalFields<T> gf,
                                                              GlobalCurrent<T> gj, TileArgs t, int32_t *flags) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *smem = reinterpret_cast<T *>(smem_raw);
  const G geo(t);
  int32_t *const cell_o = FOLD ? s.cell_o : s.cell;
  T *const off_o[3] = {FOLD ? s.off_o[0] : s.off[0], FOLD ? s.off_o[1] : s.off[1], FOLD ? s.off_o[2] : s.off[2]};
  T *const u_o[3] = {FOLD ? s.u_o[0] : s.u[0], FOLD ? s.u_o[1] : s.u[1], FOLD ? s.u_o[2] : s.u[2]};
  T *const w_o = FOLD ? s.w_o : s.w;
  // Work items are the non-empty tiles (all tiles when no list is known).
  // Workgroups are dealt to the 8 XCDs round-robin.  Each XCD owns a
  // contiguous range of items, so that neighbouring tiles share its L2.  A
  // workgroup's first item is the j-th of its XCD's range (j = its index
  // among that XCD's workgroups), which spreads a sparse box over every CU;
  // items beyond the first round come from the XCD's queue, and a workgroup
  // whose queue is empty takes from the next ones.
  int64_t items = t.live ? t.live[t.ntiles] : t.ntiles;
  items = items < 0 ? 0 : (items > t.ntiles ? t.ntiles : items);
  const int nq = t.remap ? 8 : 1;
  const int64_t per = (items + nq - 1) / nq;
  const int home = static_cast<int>(blockIdx.x % nq);
  // the first item, and the workgroups per XCD (the items dealt before any queue)
  int64_t first = static_cast<int64_t>(blockIdx.x / nq);
  first = first < per && home * per + first < items ? home * per + first : -1;
  const int64_t nb = gridDim.x;

  T *fl = smem;
  TJ *jl = reinterpret_cast<TJ *>(smem + 6 * geo.FVOL);  // 6 * FVOL * sizeof(T) is a multiple of 8
  // Particles whose nearest node changes are deposited after the main loop,
  // all together, so that the wide-window path runs with full wavefronts.
  const int CAP = t.cross_cap;
  T *xo = reinterpret_cast<T *>(jl + 3 * geo.JVOL);  // [6][CAP]: old then new offsets
  T *xw = xo + 6 * CAP;                               // [2][CAP]: weight, 2D v_z factor
  int32_t *xk = reinterpret_cast<int32_t *>(xw + 2 * CAP);  // [CAP]: local cell and cell change
  int32_t *xn = xk + CAP;                                    // list length
  int32_t *slot = xn + 1;                                    // the item this workgroup takes next
  uint32_t *wbits = reinterpret_cast<uint32_t *>(slot + 1);  // bits of the tile's largest |w| (fixed point)
  constexpr bool kFixed = sizeof(TJ) == 8 && !std::is_floating_point<TJ>::value;
  // the merge clears the box behind it, so it is zeroed once here
  for (int idx = threadIdx.x; idx < 3 * geo.JVOL; idx += BLOCK) jl[idx] = TJ(0);
  // A box index T0 - lo + l (0 <= l < X, lo < X, T0 <= n - L) lies in
  // [-X, n + X).  Where the grid is at least as wide as both boxes along every
  // axis that is within one period of [0, n), and one conditional add or
  // subtract wraps it; narrower grids keep the integer modulo.
  const bool once = g.n[0] >= (geo.FX > geo.JX ? geo.FX : geo.JX) && g.n[1] >= (geo.FY > geo.JY ? geo.FY : geo.JY) &&
                    (D < 3 || g.n[2] >= (geo.FZ > geo.JZ ? geo.FZ : geo.JZ));
  const auto near_wrap = [](int i, int n) { return wrap_near(i, n); };
  const auto full_wrap = [](int i, int n) { return wrap_full(i, n); };

  for (int round = 0;; ++round) {
    if (threadIdx.x == 0) {
      int64_t it = round == 0 ? first : -1;
      for (int k = 0; k < nq && it < 0; ++k) {
        const int q = (home + k) % nq;
        const int64_t lo = q * per, hi = lo + per < items ? lo + per : items;
        const int64_t dealt = (nb - q + nq - 1) / nq;  // items of queue q taken in the first round
        if (lo + dealt >= hi) continue;
        const int64_t v = atomicAdd(&t.queue[q], 1);
        if (lo + dealt + v < hi) it = lo + dealt + v;
      }
      *slot = static_cast<int32_t>(it);
      *xn = 0;
      *wbits = 0u;
    }
    __syncthreads();
    const int64_t item = *slot;
    __syncthreads();  // every thread has its item before thread 0 writes the next one
    if (item < 0) break;
    const int64_t tile = t.live ? t.live[item] : item;
    if (tile < 0 || tile >= t.ntiles) continue;
    // clamp to the species: ranges that a failed sort left beyond np are ignored
    int64_t pbeg = t.tile_start[tile], pend = t.tile_start[tile + 1];
    pbeg = pbeg < 0 ? 0 : (pbeg > s.np ? s.np : pbeg);
    pend = pend > s.np ? s.np : pend;
    if (pbeg >= pend) continue;
    const int tx = static_cast<int>(tile % t.ntile[0]);
    const int ty = static_cast<int>((tile / t.ntile[0]) % t.ntile[1]);
    const int tz = static_cast<int>(tile / ((int64_t)t.ntile[0] * t.ntile[1]));
    const int T0[3] = {tx * geo.L0, ty * geo.L1, tz * geo.L2};

    // stage E, B of the tile plus guards (periodic wrap)
    auto stage = [&](auto wrap) {
      for (int idx = threadIdx.x; idx < geo.FVOL; idx += BLOCK) {
        const int li = idx % geo.FX;
        const int lj = (idx / geo.FX) % geo.FY;
        const int lk = idx / (geo.FX * geo.FY);
        const int gi = wrap(T0[0] - geo.FLO + li, g.n[0]);
        const int gjj = wrap(T0[1] - geo.FLO + lj, g.n[1]);
        const int gk = D == 3 ? wrap(T0[2] - geo.FLO + lk, g.n[2]) : 0;
        const int64_t gidx = gi + (int64_t)g.n[0] * (gjj + (int64_t)g.n[1] * gk);
#pragma unroll
        for (int c = 0; c < 6; ++c) fl[c * geo.FVOL + idx] = gf.F[c][gidx];
      }
    };
    if (once) stage(near_wrap);
    else stage(full_wrap);
    // the tile's largest |w| sets the fixed-point scale of its current box
    // (the main loop then reads the weights again, from the L2); after the
    // first launch since a sort it comes from the cache of that launch, and a
    // particle heavier than it (its weight changed since) takes the HBM path
    if constexpr (kFixed) {
      if (t.wmode == 2) {
        if (threadIdx.x == 0) *wbits = t.wcache[tile];
      } else {
      float wm = 0.f;
      for (int64_t q = pbeg + threadIdx.x; q < pend; q += BLOCK) {
        int64_t r = q;
        if constexpr (FOLD) {
          r = elem<SMALL>(s.src, q);
          r = r >= 0 && r < s.np_src ? r : -1;
        }
        if (r >= 0) wm = fmaxf(wm, fabsf(static_cast<float>(elem<SMALL>(s.w, r))));
      }
      for (int o = 32; o > 0; o >>= 1) wm = fmaxf(wm, __shfl_xor(wm, o));
      if (__lane_id() == 0) atomicMax(wbits, __float_as_uint(wm));
      }
    }
    __syncthreads();
    const float wbound = kFixed ? __uint_as_float(*wbits) : 0.f;
    if (kFixed && t.wmode == 1 && threadIdx.x == 0) t.wcache[tile] = __float_as_uint(wbound);
    const bool wcheck = kFixed && t.wmode == 2;
    const int shift = kFixed ? fixed_shift<T>(s, wbound, D) : 0;
    // the current's coefficients, in the fixed-point box's units (2^shift)
    const T tjc[3] = {scale2(s.jc[0], shift), scale2(s.jc[1], shift), scale2(s.jc[2], shift)};
    const T tjz = scale2(s.jz, shift);

    // local frames: the tile origin is (0,0,0)
    const auto lf = FieldBox<T, G, D>::make(fl, geo);
    const auto lj = CurrentBox<TJ, G, D>::make(jl, geo);
    const int lane = __lane_id();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    // The next particle's data is loaded before the current one is processed,
    // so its HBM latency hides behind the gather, push and deposit.  The trip
    // count is the same for every thread: lanes without a particle still take
    // part in the wavefront's exchange below.
    const int64_t trips = (pend - pbeg + BLOCK - 1) / BLOCK;
    int64_t pn = pbeg + threadIdx.x;
    int32_t n_cell = 0;
    T n_w = T(0), n_o[3] = {T(0), T(0), T(0)}, n_u[3] = {T(0), T(0), T(0)};
    // FOLD: particle q of the sorted order is read at src[q] (-1: a slot the
    // sort left inconsistent, which it flagged)
    auto from = [&](int64_t q) -> int64_t {
      const int64_t r = elem<SMALL>(s.src, q);
      return r >= 0 && r < s.np_src ? r : -1;
    };
    int64_t n_r = -1;
    if constexpr (FOLD) {
      n_r = pn < pend ? from(pn) : -1;
      if (n_r >= 0) {
        n_cell = elem<SMALL>(s.cell, n_r);
        n_w = elem<SMALL>(s.w, n_r);
        load_particle<T, D, SMALL>(s, n_r, n_o, n_u);
      }
    } else if (pn < pend) {
      n_cell = elem<SMALL>(s.cell, pn);
      n_w = elem<SMALL>(s.w, pn);
      load_particle<T, D, SMALL>(s, pn, n_o, n_u);
    }
    for (int64_t trip = 0; trip < trips; ++trip, pn += BLOCK) {
      const int32_t p_cell = n_cell;
      const T w = n_w;
      T o[3] = {n_o[0], n_o[1], n_o[2]}, u[3] = {n_u[0], n_u[1], n_u[2]};
      bool have = pn < pend;
      if constexpr (FOLD) {
        have = have && n_r >= 0;
        n_r = pn + BLOCK < pend ? from(pn + BLOCK) : -1;
        if (n_r >= 0) {
          n_cell = elem<SMALL>(s.cell, n_r);
          n_w = elem<SMALL>(s.w, n_r);
          load_particle<T, D, SMALL>(s, n_r, n_o, n_u);
        }
      } else if (pn + BLOCK < pend) {
        n_cell = elem<SMALL>(s.cell, pn + BLOCK);
        n_w = elem<SMALL>(s.w, pn + BLOCK);
        load_particle<T, D, SMALL>(s, pn + BLOCK, n_o, n_u);
      }
      const int64_t p = pn;
      int c[3] = {0, 0, 0};
      // cell relative to the tile origin, unwrapped across the periodic seam
      int lc[3] = {0, 0, 0};
      bool inside = true;
      if (have) {
        unpack(p_cell, g, c);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          int l = c[d] - T0[d];
          if (l > g.n[d] / 2) l -= g.n[d];
          if (l < -g.n[d] / 2) l += g.n[d];
          lc[d] = l;
          const int L = d == 0 ? geo.L0 : (d == 1 ? geo.L1 : geo.L2);
          inside = inside && (l >= -geo.S) && (l < L + geo.S);
        }
        if (wcheck) inside = inside && !(fabsf(static_cast<float>(w)) > wbound);
      }
      const bool stray = have && !inside;
      const uint64_t out = __ballot(stray);
      if (out) {  // list the particles outside the box for the HBM path
        const int leader = __ffsll(static_cast<unsigned long long>(out)) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(t.stray_count, __popcll(out));
        base = __shfl(base, leader);
        if (stray) t.stray_list[base + __popcll(out & below)] = static_cast<int32_t>(p);
      }
      // removed at an open face: skipped until the next sort drops it
      const bool live = have && inside && !(s.open && w == T(0));
      T on[3] = {T(0), T(0), T(0)};
      int dc[3] = {0, 0, 0};
      T jz = T(0);
      bool wide = false, fast = false;
      if (live) {
        T eb[6];
        gather_eb<T, D, M>(lf, lc, o, eb);
        boris<T>(u, eb, s.h);
        const T ig = rsqrt_t<T>(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const bool ok = move<T, D>(u, ig, s.dtdx, o, on, dc);
        if (!ok) atomicOr(&flags[0], kFlagCross);
        jz = D == 2 ? tjz * u[2] * ig : T(0);
        wide = ok && crosses<T, D, M>(o, dc, on);
        fast = ok && !wide;
      }
      if constexpr (kDealLanes && D == 3) {
        // The LDS unit serves a wavefront's 8-byte atomics 16 lanes at a time
        // and replays a group once per repeat of (element index mod 16)
        // within it.  Every deposit atomic of a particle sits at a fixed
        // offset from its window base, so that residue of the base decides.
        // The wavefront sorts its fast deposits by it and deals them
        // round-robin over its four 16-lane groups: copies of one residue
        // land in different groups as long as there are at most four.  Only
        // the deposit's inputs move; gather, push and stores stay in the
        // particles' own lanes, where neighbouring lanes hold neighbouring
        // nodes and the field reads spread over the banks.
        int key = 16;  // lanes without a fast deposit sort last
        if (fast) {
          const int stride[3] = {1, geo.JX, geo.JXY};
          int idx = 0;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const int b = lc[d] + (M == 2 ? (o[d] >= T(0.5) ? 0 : -1) : 0);
            idx += stride[d] * (b + geo.JLO);
          }
          key = idx & 15;
        }
        int k = 0, run = 0;
#pragma unroll
        for (int r = 0; r <= 16; ++r) {
          const uint64_t m = __ballot(key == r);
          const int t = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
              static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), static_cast<uint32_t>(run))));
          k = key == r ? t : k;
          run += __popcll(m);
        }
        const int to = ((k & 3) * 16 + (k >> 2)) * 4;
        T so[3], sn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          so[d] = lane_push(to, o[d]);
          sn[d] = lane_push(to, on[d]);
        }
        // the packed local cell (24 bits, so never negative) doubles as the flag
        const int32_t sk = lane_push(to, fast ? pack_local(lc, dc) : int32_t(-1));
        const T sw = lane_push(to, w);
        if (sk >= 0) {
          int slc[3], sdc[3];
          unpack_local(sk, slc, sdc);
          Esirk<T, M> e;
          esirkepov_factors_fast<T, D, M>(so, sn, e);
          const T jc[3] = {sw * tjc[0], sw * tjc[1], sw * tjc[2]};
          esirkepov_accumulate<T, D, M, true>(lj, slc, e, jc, T(0));
        }
      } else {
        if (fast) {
          Esirk<T, M> e;
          esirkepov_factors_fast<T, D, M>(o, on, e);
          const T jc[3] = {w * tjc[0], w * tjc[1], w * tjc[2]};
          esirkepov_accumulate<T, D, M, true>(lj, lc, e, jc, w * jz);
        }
      }
      // one LDS atomic per wavefront reserves list slots for the wide ones
      const uint64_t wm = __ballot(wide);
      if (wm) {
        const int leader = __ffsll(static_cast<unsigned long long>(wm)) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(xn, __popcll(wm));
        base = __shfl(base, leader);
        if (wide) {
          const int k = base + __popcll(wm & below);
          if (k < CAP) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
              xo[d * CAP + k] = o[d];
              xo[(3 + d) * CAP + k] = on[d];
            }
            xw[k] = w;
            xw[CAP + k] = jz;
            xk[k] = pack_local(lc, dc);
          } else {  // list full: deposit here, in the drain's form
            const T jc[3] = {w * tjc[0], w * tjc[1], w * tjc[2]};
            if constexpr (D == 3)
              esirkepov_rotated<T, M>(jl, geo.JX, geo.JXY, geo.JVOL, geo.JLO, lc, o, dc, on, jc);
            else
              esirkepov_rotated_2d<T, M>(jl, geo.JX, geo.JVOL, geo.JLO, lc, o, dc, on, jc, w * jz);
          }
        }
      }
      if (live) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          c[d] = wrap_near(c[d] + dc[d], g.n[d]);
          elem<SMALL>(off_o[d], p) = on[d];
        }
        elem<SMALL>(cell_o, p) = pack(c, g);
        elem<SMALL>(u_o[0], p) = u[0];
        elem<SMALL>(u_o[1], p) = u[1];
        elem<SMALL>(u_o[2], p) = u[2];
        if (s.open && (c[0] < s.xlo || c[0] >= s.xhi)) elem<SMALL>(w_o, p) = T(0);  // removed at an open face
        else if (FOLD) elem<SMALL>(w_o, p) = w;
      } else if (FOLD && have) {  // a straggler or a removed particle moves unchanged
#pragma unroll
        for (int d = 0; d < D; ++d) elem<SMALL>(off_o[d], p) = o[d];
        elem<SMALL>(cell_o, p) = p_cell;
        elem<SMALL>(u_o[0], p) = u[0];
        elem<SMALL>(u_o[1], p) = u[1];
        elem<SMALL>(u_o[2], p) = u[2];
        elem<SMALL>(w_o, p) = w;
      }
    }
    __syncthreads();

    // the listed particles, with every lane busy
    const int nx = *xn < CAP ? *xn : CAP;
    for (int k = threadIdx.x; k < nx; k += BLOCK) {
      T o0[3], o1[3];
      int lc[3], dc[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        o0[d] = xo[d * CAP + k];
        o1[d] = xo[(3 + d) * CAP + k];
      }
      unpack_local(xk[k], lc, dc);
      const T w = xw[k];
      const T jc[3] = {w * tjc[0], w * tjc[1], w * tjc[2]};
      if constexpr (D == 3)
        esirkepov_rotated<T, M>(jl, geo.JX, geo.JXY, geo.JVOL, geo.JLO, lc, o0, dc, o1, jc);
      else
        esirkepov_rotated_2d<T, M>(jl, geo.JX, geo.JVOL, geo.JLO, lc, o0, dc, o1, jc, w * xw[CAP + k]);
    }
    __syncthreads();

    // add the current box into HBM (skipping cells nothing touched)
    auto merge = [&](auto wrap) {
      for (int cell = threadIdx.x; cell < geo.JX * geo.JY * geo.JZ; cell += BLOCK) {
        const int li = cell % geo.JX;
        const int lj2 = (cell / geo.JX) % geo.JY;
        const int lk = cell / (geo.JX * geo.JY);
        const int idx = li + geo.JX * lj2 + geo.JXY * lk;  // the plane stride may be padded
        const int gi = wrap(T0[0] - geo.JLO + li, g.n[0]);
        const int gjj = wrap(T0[1] - geo.JLO + lj2, g.n[1]);
        const int gk = D == 3 ? wrap(T0[2] - geo.JLO + lk, g.n[2]) : 0;
        const int64_t gidx = gi + (int64_t)g.n[0] * (gjj + (int64_t)g.n[1] * gk);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T v = lds_value<T>(jl[c * geo.JVOL + idx], shift);
          jl[c * geo.JVOL + idx] = TJ(0);  // ready for the next tile
          if (v != T(0)) unsafeAtomicAdd(&gj.J[c][gidx], v);
        }
      }
    };
    if (once) merge(near_wrap);
    else merge(full_wrap);
  }
}

// One particle's full step with the fields and current in HBM, updated in
// place (particle p of the species' arrays): gather, Boris, move, deposit
// with global atomics, removal at an open face.
template <typename T, int D, int M>
__device__ __forceinline__ void push_hbm(const SpeciesArgs<T> &s, const GridArgs &g, const GlobalFields<T> &gf,
                                         const GlobalCurrent<T> &gj, int64_t p, int32_t *flags) {
  const T w = s.w[p];
  if (s.open && w == T(0)) return;  // removed at an open face
  int c[3];
  unpack(s.cell[p], g, c);
  T o[3], u[3];
  load_particle<T, D>(s, p, o, u);
  T eb[6];
  gather_eb<T, D, M>(gf, c, o, eb);
  boris<T>(u, eb, s.h);
  const T ig = rsqrt_t<T>(T(1) + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  T on[3] = {T(0), T(0), T(0)};
  int dc[3] = {0, 0, 0};
  const bool ok = move<T, D>(u, ig, s.dtdx, o, on, dc);
  if (!ok) atomicOr(&flags[0], kFlagCross);
  const T jc[3] = {w * s.jc[0], w * s.jc[1], w * s.jc[2]};
  const T jz = D == 2 ? w * s.jz * u[2] * ig : T(0);
  if (ok) deposit<T, D, M>(gj, c, o, dc, on, jc, jz);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    c[d] = wrap_near(c[d] + dc[d], g.n[d]);
    s.off[d][p] = on[d];
  }
  s.cell[p] = pack(c, g);
  s.u[0][p] = u[0];
  s.u[1][p] = u[1];
  s.u[2][p] = u[2];
  absorb_if_out(s, p, c[0]);
}

// The particles a tiled launch left outside their LDS box, then (when few is
// given) every particle of the tiles the launch skipped for having few
// particles, one wavefront per tile: full step with fields and current in HBM.
template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_stragglers(SpeciesArgs<T> s, GridArgs g, GlobalFields<T> gf,
                                                    GlobalCurrent<T> gj, const int32_t *count, const int32_t *list,
                                                    const int32_t *few, const int32_t *tile_start, int64_t ntiles,
                                                    int32_t *flags, int32_t *clear_next) {
  // the other counter bank, which the next fused launch takes (this launch
  // does not read it)
  if (clear_next && blockIdx.x == 0 && threadIdx.x < 9) clear_next[threadIdx.x] = 0;
  const int64_t n = *count;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    push_hbm<T, D, M>(s, g, gf, gj, list[k], flags);
  if (!few) return;
  int64_t nfew = few[ntiles];
  nfew = nfew < 0 ? 0 : (nfew > ntiles ? ntiles : nfew);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  const int lane = __lane_id();
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / 64) + threadIdx.x / 64; i < nfew; i += waves) {
    const int64_t tile = few[i];
    if (tile < 0 || tile >= ntiles) continue;
    // clamp to the species, as the fused kernel does
    int64_t pbeg = tile_start[tile], pend = tile_start[tile + 1];
    pbeg = pbeg < 0 ? 0 : (pbeg > s.np ? s.np : pbeg);
    pend = pend > s.np ? s.np : pend;
    for (int64_t q = pbeg + lane; q < pend; q += 64) push_hbm<T, D, M>(s, g, gf, gj, q, flags);
  }
}

// After a fused launch that took over a sort's copy: the particles behind
// every tile (the bucket of removed ones, [tile_start[ntiles], np)) move to
// the second set unchanged.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_fold_tail(SpeciesArgs<T> s, const int32_t *tile_start, int64_t ntiles) {
  int64_t lo = tile_start[ntiles];
  lo = lo < 0 ? 0 : lo;
  for (int64_t q = lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < s.np; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = s.src[q];
    if (r < 0 || r >= s.np_src) continue;  // only after a flagged inconsistency
    s.cell_o[q] = s.cell[r];
#pragma unroll
    for (int d = 0; d < D; ++d) s.off_o[d][q] = s.off[d][r];
#pragma unroll
    for (int d = 0; d < 3; ++d) s.u_o[d][q] = s.u[d][r];
    s.w_o[q] = s.w[r];
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
  s.w = static_cast<T *>(sp.w);
  s.src = nullptr;
  s.np_src = sp.np;
  s.cell_o = s.cell;
  for (int d = 0; d < 3; ++d) {
    s.off_o[d] = s.off[d];
    s.u_o[d] = s.u[d];
  }
  s.w_o = s.w;
  s.open = c.p.open_x;
  s.xlo = c.p.open_x ? c.p.absorb : 0;
  s.xhi = c.p.open_x ? static_cast<int>(c.n[0]) - c.p.absorb : static_cast<int>(c.n[0]);
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

template <typename T, int D, int M, class G, int BLOCK, typename TJ>
hipError_t launch_tiled_acc(const pic_ctx &c, const SpeciesArgs<T> &sa, const pic_fields &f, const TileArgs &t,
                            hipStream_t st) {
  // only 3D launches fold a sort's copy; 32-bit byte offsets while every
  // particle array (elements of sizeof(T) at most) spans at most 2^32 bytes
  const bool fold = D == 3 && sa.src;
  const int64_t nmax = sa.np > sa.np_src ? sa.np : sa.np_src;
  const bool small = nmax * static_cast<int64_t>(sizeof(T)) <= (int64_t(1) << 32);
  const auto kern = fold ? (small ? k_push_deposit_tiled<T, D, M, G, BLOCK, TJ, D == 3, true>
                                  : k_push_deposit_tiled<T, D, M, G, BLOCK, TJ, D == 3, false>)
                         : (small ? k_push_deposit_tiled<T, D, M, G, BLOCK, TJ, false, true>
                                  : k_push_deposit_tiled<T, D, M, G, BLOCK, TJ, false, false>);
  const size_t lds = c.lds_bytes;
  // granted on every launch (idempotent, and valid for whichever device is current)
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  // persistent workgroups: as many as the device holds at once, at most one per tile
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, BLOCK, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int64_t blocks = static_cast<int64_t>(ncu) * per_cu;
  if (blocks > c.ntiles) blocks = c.ntiles;
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(blocks)), dim3(BLOCK), lds, st, sa, grid_args(c),
                     global_fields<T>(c, f), global_current<T>(c, f), t, c.wsp<int32_t>(c.ws.flags));
  return hipGetLastError();
}

// The LDS current box of an FP32 state is accumulated in 64-bit fixed point
// (default), double or float; an FP64 state's in double.
template <typename T, int D, int M, class G, int BLOCK>
hipError_t launch_tiled(const pic_ctx &c, const SpeciesArgs<T> &sa, const pic_fields &f, const TileArgs &t,
                        hipStream_t st) {
  if constexpr (sizeof(T) == 4) {
    if (c.accfix) return launch_tiled_acc<T, D, M, G, BLOCK, unsigned long long>(c, sa, f, t, st);
    if (!c.acc64) return launch_tiled_acc<T, D, M, G, BLOCK, float>(c, sa, f, t, st);
  }
  return launch_tiled_acc<T, D, M, G, BLOCK, double>(c, sa, f, t, st);
}

// Tile shapes with a compile-time instantiation; other shapes use the
// runtime-geometry kernel.
template <typename T, int D, int M>
hipError_t tiled_impl(const pic_ctx &c, pic_species &sp, const pic_fields &f, hipStream_t st, const int32_t *src,
                      int64_t np_src) {
  if (sp.np == 0) return hipSuccess;
  if (D != 3 && src) return hipErrorInvalidValue;  // only 3D launches fold a sort's copy
  SpeciesArgs<T> sa = species_args<T>(c, sp);
  if (src) {  // read through the sort's slots, write the second set
    sa.src = src;
    sa.np_src = np_src;
    sa.cell_o = sp.cell_alt;
    for (int d = 0; d < 3; ++d) {
      sa.off_o[d] = static_cast<T *>(sp.off_alt[d]);
      sa.u_o[d] = static_cast<T *>(sp.u_alt[d]);
    }
    sa.w_o = static_cast<T *>(sp.w_alt);
  }
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
  t.jxy = c.jxy;
  t.remap = c.ntiles >= 64 ? 1 : 0;
  // a launch that folds a sort's copy takes every non-empty tile; the in-place
  // ones leave the tiles with few particles to the straggler kernel
  t.live = src ? live_tiles(c, sp) : dense_tiles(c, sp);
  const int32_t *few = src ? nullptr : sparse_tiles(c, sp);
  // the fixed-point current's tile bounds: found by the first launch after
  // the species' sort, taken from it by the later ones
  const int slot = c.accfix ? sorted_slot(c, sp) : -1;
  t.wcache = slot < 0 ? nullptr : c.wsp<uint32_t>(c.ws.wmax_tiles) + static_cast<size_t>(slot) * c.ntiles;
  t.wmode = slot < 0 ? 0 : (c.wmax_known[slot] ? 2 : 1);
  t.ntiles = c.ntiles;
  // the straggler count and the 8 queues, in this launch's bank: zero if the
  // previous launch's straggler kernel cleared it, else cleared here
  const int bank = c.stray_bank;
  int32_t *banks = c.wsp<int32_t>(c.ws.stray_count);
  t.stray_count = banks + 16 * bank;
  t.stray_list = c.wsp<int32_t>(c.ws.stray_list);
  t.queue = t.stray_count + 1;
  t.cross_cap = c.cross_cap;
  hipError_t e = hipSuccess;
  if (!c.stray_clean) e = launch_fill_zero(t.stray_count, 9, 4, st);
  c.stray_clean = false;  // until this launch's straggler kernel has gone out
  if (e != hipSuccess) return e;
  const int *L = c.p.tile;
  const int sl = c.p.slack;
  // threads per workgroup of the fixed-shape kernels: in 3D 16 waves in FP32
  // and 12 in FP64, whose kernel needs up to 168 registers (3 waves per SIMD);
  // in 2D 16 waves in FP32 and 8 in FP64
  constexpr int BIG = sizeof(T) == 4 ? 1024 : 768;
  constexpr int DENSE = sizeof(T) == 4 ? 1024 : 512;
  if constexpr (D == 3) {
    if (sizeof(T) == 4 && L[0] == 8 && L[1] == 8 && L[2] == 8 && sl == 1 && c.rf[0] == FixedGeom<D, M, 8, 8, 8, 1>::FX)
      e = launch_tiled<T, D, M, FixedGeom<D, M, 8, 8, 8, 1>, BIG>(c, sa, f, t, st);
    else if (L[0] == 8 && L[1] == 8 && L[2] == 4 && sl == 1 && c.rf[0] == FixedGeom<D, M, 8, 8, 4, 1>::FX)
      e = launch_tiled<T, D, M, FixedGeom<D, M, 8, 8, 4, 1>, BIG>(c, sa, f, t, st);
    else
      e = launch_tiled<T, D, M, RuntimeGeom, 256>(c, sa, f, t, st);
  } else {
    if (L[0] == 16 && L[1] == 16 && sl == 1 && c.rf[0] == FixedGeom<D, M, 16, 16, 1, 1>::FX)
      e = launch_tiled<T, D, M, FixedGeom<D, M, 16, 16, 1, 1>, DENSE>(c, sa, f, t, st);
    else if (L[0] == 8 && L[1] == 8 && sl == 1 && c.rf[0] == FixedGeom<D, M, 8, 8, 1, 1>::FX)  // dense foils
      e = launch_tiled<T, D, M, FixedGeom<D, M, 8, 8, 1, 1>, DENSE>(c, sa, f, t, st);
    else if (L[0] == 16 && L[1] == 16 && sl == 2 && c.rf[0] == FixedGeom<D, M, 16, 16, 1, 2>::FX)  // the rollout
      e = launch_tiled<T, D, M, FixedGeom<D, M, 16, 16, 1, 2>, DENSE>(c, sa, f, t, st);
    else
      e = launch_tiled<T, D, M, RuntimeGeom, 256>(c, sa, f, t, st);
  }
  if (e != hipSuccess) return e;
  if (slot >= 0) c.wmax_known[slot] = true;
  // up to 4096 workgroups of four wavefronts: the straggler kernel gives each
  // sparse tile a wavefront, and a box of many such tiles keeps them in flight
  int64_t blocks = (sp.np + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (src) {  // the removed particles behind every tile, then the sets swap
    hipLaunchKernelGGL((k_fold_tail<T, D>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, sa,
                       sp.tile_start, c.ntiles);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    swap_sets(sp);
  }
  hipLaunchKernelGGL((k_stragglers<T, D, M>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                     species_args<T>(c, sp), grid_args(c), global_fields<T>(c, f), global_current<T>(c, f),
                     t.stray_count, t.stray_list, few, sp.tile_start, c.ntiles, c.wsp<int32_t>(c.ws.flags),
                     banks + 16 * (1 - bank));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  c.stray_last = bank;
  c.stray_bank = 1 - bank;
  c.stray_clean = true;
  return hipSuccess;
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

hipError_t launch_push_deposit_tiled(const pic_ctx &c, pic_species &sp, const pic_fields &f, hipStream_t s,
                                     const int32_t *src, int64_t np_src) {
  PIC_DISPATCH(tiled_impl, c, sp, f, s, src, np_src);
}

}  // namespace pic
