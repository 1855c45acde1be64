// Device arithmetic of one particle for one step: B-spline weights, the
// staggered gather, the relativistic Boris rotation, the leap-frog move in
// (cell, offset) form and the Esirkepov current.  Everything is templated on
// the floating type T, the number of dimensions D and the shape order M, and
// reads fields / writes current through accessors, so the same code runs
// against LDS tiles and against HBM.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace pic {

template <typename T>
__device__ __forceinline__ T rsqrt_t(T x);
template <>
__device__ __forceinline__ float rsqrt_t<float>(float x) { return rsqrtf(x); }
template <>
__device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

__device__ __forceinline__ int wrap_near(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Quadratic B-spline weights of the three nodes nearest to a point at
// distance d in [-1/2, 1/2) from the middle node.
template <typename T>
__device__ __forceinline__ void quad_weights(T d, T w[3]) {
  const T a = T(0.5) - d, b = T(0.5) + d;
  w[0] = T(0.5) * a * a;
  w[1] = T(0.75) - d * d;
  w[2] = T(0.5) * b * b;
}

// Weights on the integer nodes (components not staggered along this axis):
// w[0..M] belong to nodes base..base+M.
template <typename T, int M>
__device__ __forceinline__ void node_weights(int c, T o, T w[M + 1], int &base) {
  if constexpr (M == 1) {
    base = c;
    w[0] = T(1) - o;
    w[1] = o;
  } else {
    const bool up = o >= T(0.5);
    base = up ? c : c - 1;
    quad_weights<T>(up ? o - T(1) : o, w);
  }
}

// Weights on the half-integer points (components staggered along this axis):
// w[0..M] belong to array indices base..base+M (positions index + 1/2).
template <typename T, int M>
__device__ __forceinline__ void half_weights(int c, T o, T w[M + 1], int &base) {
  if constexpr (M == 1) {
    const bool up = o >= T(0.5);
    const T f = up ? o - T(0.5) : o + T(0.5);
    base = up ? c : c - 1;
    w[0] = T(1) - f;
    w[1] = f;
  } else {
    base = c - 1;
    quad_weights<T>(o - T(0.5), w);
  }
}

// Accessors whose x runs can be read as aligned pairs (see interp).
template <class A, class = void>
struct HasPairs : std::false_type {};
template <class A>
struct HasPairs<A, std::void_t<decltype(A::kPairs)>> : std::bool_constant<A::kPairs> {};

template <typename T>
struct Pair;
template <>
struct Pair<float> {
  using type = float2;
};
template <>
struct Pair<double> {
  using type = double2;
};

// Sum over the (M+1)^D points of one component with per-axis weights.
template <typename T, int D, int M, class Acc>
__device__ __forceinline__ T interp(const Acc &acc, int comp, const T *wx, int bx, const T *wy, int by, const T *wz,
                                    int bz) {
  T s = T(0);
  if constexpr (M == 2 && HasPairs<Acc>::value) {
    // Every row of the box starts at an even element, so each run of three
    // values is one aligned pair and one single: (v0 v1 | v2) when the run
    // starts at an even element, (v0 | v1 v2) when odd.  The weights are
    // rotated once to match, and every row takes one read of two values and
    // one of one value, where three single reads cost the LDS about twice as
    // much (its cost follows the number of addresses more than the bytes).
    static_assert(sizeof(typename Acc::value_type) == sizeof(T), "pair reads need the state's type");
    using P2 = typename Pair<T>::type;
    const int e0 = acc.index(comp, bx, by, D == 3 ? bz : 0);
    const bool odd = (e0 & 1) != 0;
    const T a = odd ? wx[1] : wx[0], b = odd ? wx[2] : wx[1], c = odd ? wx[0] : wx[2];
    const P2 *pr = reinterpret_cast<const P2 *>(acc.base) + ((e0 + 1) >> 1);
    const T *sg = acc.base + (odd ? e0 : e0 + 2);
#pragma unroll
    for (int k = 0; k <= (D == 3 ? M : 0); ++k) {
      T sy = T(0);
#pragma unroll
      for (int j = 0; j <= M; ++j) {
        const int off = Acc::kSX * j + Acc::kSXY * k;
        const P2 p = pr[off >> 1];
        sy += wy[j] * (a * p.x + b * p.y + c * sg[off]);
      }
      if constexpr (D == 3) s += wz[k] * sy;
      else s = sy;
    }
  } else if constexpr (D == 3) {
#pragma unroll
    for (int k = 0; k <= M; ++k) {
      T sy = T(0);
#pragma unroll
      for (int j = 0; j <= M; ++j) {
        T row = T(0);
#pragma unroll
        for (int i = 0; i <= M; ++i) row += wx[i] * acc.load(comp, bx + i, by + j, bz + k);
        sy += wy[j] * row;
      }
      s += wz[k] * sy;
    }
  } else {
#pragma unroll
    for (int j = 0; j <= M; ++j) {
      T row = T(0);
#pragma unroll
      for (int i = 0; i <= M; ++i) row += wx[i] * acc.load(comp, bx + i, by + j, 0);
      s += wy[j] * row;
    }
  }
  return s;
}

// E and B at the particle: each component weighted on its own staggered grid
// (Ex: half in x; Ey: half in y; Ez: half in z; Bx: half in y,z; By: half in
// x,z; Bz: half in x,y).  c[] is the cell in the accessor's frame.
template <typename T, int D, int M, class Acc>
__device__ __forceinline__ void gather_eb(const Acc &acc, const int c[3], const T o[3], T eb[6]) {
  T wn[3][M + 1], wh[3][M + 1];
  int bn[3] = {0, 0, 0}, bh[3] = {0, 0, 0};
#pragma unroll
  for (int d = 0; d < D; ++d) {
    node_weights<T, M>(c[d], o[d], wn[d], bn[d]);
    half_weights<T, M>(c[d], o[d], wh[d], bh[d]);
  }
  if constexpr (D == 2) {
#pragma unroll
    for (int i = 0; i <= M; ++i) wn[2][i] = wh[2][i] = T(0);
  }
  eb[0] = interp<T, D, M>(acc, 0, wh[0], bh[0], wn[1], bn[1], wn[2], bn[2]);
  eb[1] = interp<T, D, M>(acc, 1, wn[0], bn[0], wh[1], bh[1], wn[2], bn[2]);
  eb[2] = interp<T, D, M>(acc, 2, wn[0], bn[0], wn[1], bn[1], wh[2], bh[2]);
  eb[3] = interp<T, D, M>(acc, 3, wn[0], bn[0], wh[1], bh[1], wh[2], bh[2]);
  eb[4] = interp<T, D, M>(acc, 4, wh[0], bh[0], wn[1], bn[1], wh[2], bh[2]);
  eb[5] = interp<T, D, M>(acc, 5, wh[0], bh[0], wh[1], bh[1], wn[2], bn[2]);
}

// Relativistic Boris rotation, u^{n-1/2} -> u^{n+1/2}; h = q dt / (2 m).
template <typename T>
__device__ __forceinline__ void boris(T u[3], const T eb[6], T h) {
  const T um0 = u[0] + h * eb[0], um1 = u[1] + h * eb[1], um2 = u[2] + h * eb[2];
  const T ig = rsqrt_t<T>(T(1) + um0 * um0 + um1 * um1 + um2 * um2);
  const T t0 = h * ig * eb[3], t1 = h * ig * eb[4], t2 = h * ig * eb[5];
  const T f = T(2) / (T(1) + t0 * t0 + t1 * t1 + t2 * t2);
  const T s0 = f * t0, s1 = f * t1, s2 = f * t2;
  const T up0 = um0 + (um1 * t2 - um2 * t1);
  const T up1 = um1 + (um2 * t0 - um0 * t2);
  const T up2 = um2 + (um0 * t1 - um1 * t0);
  u[0] = um0 + (up1 * s2 - up2 * s1) + h * eb[0];
  u[1] = um1 + (up2 * s0 - up0 * s2) + h * eb[1];
  u[2] = um2 + (up0 * s1 - up1 * s0) + h * eb[2];
}

// Leap-frog move in cell units with floor renormalisation: on[d] in [0,1),
// dc[d] in {-1,0,1}.  Returns false (and moves nothing) when a displacement
// reaches a full cell or is not finite.
template <typename T, int D>
__device__ __forceinline__ bool move(const T u[3], T ig, const T dtdx[3], const T o[3], T on[3], int dc[3]) {
  bool ok = true;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const T disp = u[d] * ig * dtdx[d];
    ok = ok && (fabs(disp) < T(1));
    const T x = o[d] + disp;
    const T fl = floor(x);
    T r = x - fl;
    int k = static_cast<int>(fl);
    if (r >= T(1)) {  // a tiny negative x rounds up to 1 after the shift
      r = T(0);
      k += 1;
    }
    on[d] = r;
    dc[d] = k;
  }
  if (!ok) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      on[d] = o[d];
      dc[d] = 0;
    }
  }
  return ok;
}

// Per-axis Esirkepov factors over a window of W = M + 2 nodes starting at
// node (old cell + base): S0 = old shape, DS = new shape - old shape.
// When the nearest node (M = 2) or the cell (M = 1) does not change, DS is
// taken from the displacement directly, which keeps FP32 results accurate
// for tiny moves.  cross tells whether it changed.
template <typename T, int M>
__device__ __forceinline__ void esirkepov_axis(T o0, int dc, T o1, int &base, T S0[M + 2], T DS[M + 2], bool &cross) {
  if constexpr (M == 2) {
    const bool u0 = o0 >= T(0.5), u1 = o1 >= T(0.5);
    const int n0 = u0 ? 1 : 0, n1 = dc + (u1 ? 1 : 0);
    const T d0 = u0 ? o0 - T(1) : o0, d1 = u1 ? o1 - T(1) : o1;
    T q0[3];
    quad_weights<T>(d0, q0);
    const int b = (n0 < n1 ? n0 : n1) - 1;
    base = b;
    const bool sh0 = (n0 - 1 - b) == 1;
    S0[0] = sh0 ? T(0) : q0[0];
    S0[1] = sh0 ? q0[0] : q0[1];
    S0[2] = sh0 ? q0[1] : q0[2];
    S0[3] = sh0 ? q0[2] : T(0);
    cross = n1 != n0;
    if (!cross) {
      const T dd = d1 - d0, s = T(2) * d0 + dd;
      DS[0] = T(-0.5) * dd * (T(1) - s);
      DS[1] = -dd * s;
      DS[2] = T(0.5) * dd * (T(1) + s);
      DS[3] = T(0);
    } else {
      T q1[3];
      quad_weights<T>(d1, q1);
      const bool sh1 = (n1 - 1 - b) == 1;
      DS[0] = (sh1 ? T(0) : q1[0]) - S0[0];
      DS[1] = (sh1 ? q1[0] : q1[1]) - S0[1];
      DS[2] = (sh1 ? q1[1] : q1[2]) - S0[2];
      DS[3] = (sh1 ? q1[2] : T(0)) - S0[3];
    }
  } else {
    const int b = dc < 0 ? dc : 0;
    base = b;
    const bool sh0 = b == -1;
    S0[0] = sh0 ? T(0) : T(1) - o0;
    S0[1] = sh0 ? T(1) - o0 : o0;
    S0[2] = sh0 ? o0 : T(0);
    cross = dc != 0;
    if (!cross) {
      const T dd = o1 - o0;
      DS[0] = -dd;
      DS[1] = dd;
      DS[2] = T(0);
    } else {
      const bool sh1 = (dc - b) == 1;
      DS[0] = (sh1 ? T(0) : T(1) - o1) - S0[0];
      DS[1] = (sh1 ? T(1) - o1 : o1) - S0[1];
      DS[2] = (sh1 ? o1 : T(0)) - S0[2];
    }
  }
}

// Whether a move from (o0) to (dc + o1) changes the nearest node (M = 2) or
// the cell (M = 1) on some axis: such a particle needs the M + 2 wide window.
template <typename T, int D, int M>
__device__ __forceinline__ bool crosses(const T o0[3], const int dc[3], const T o1[3]) {
  bool c = false;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if constexpr (M == 2) {
      const int n0 = o0[d] >= T(0.5) ? 1 : 0;
      const int n1 = dc[d] + (o1[d] >= T(0.5) ? 1 : 0);
      c = c || n1 != n0;
    } else {
      c = c || dc[d] != 0;
    }
  }
  return c;
}

// Per-particle Esirkepov factors on all axes (window of W = M + 2 nodes per
// axis starting at node old cell + b[d]): the old shape S0, DS = new - old,
// CDS = running sum of DS, A = S0 + DS/2, Bf = S0/2 + DS/3.  cross is true
// when the nearest node (M = 2) or the cell (M = 1) changed on some axis;
// otherwise every factor vanishes beyond the first M + 1 window slots.
template <typename T, int M>
struct Esirk {
  static constexpr int W = M + 2;
  T S0[3][W], DS[3][W], CDS[3][W - 1], A[3][W], Bf[3][W];
  int b[3];
  bool cross;
};

template <typename T, int D, int M>
__device__ __forceinline__ void esirkepov_factors(const T o0[3], const int dc[3], const T o1[3], Esirk<T, M> &e) {
  constexpr int W = M + 2;
  e.cross = false;
  e.b[0] = e.b[1] = e.b[2] = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    bool cross;
    esirkepov_axis<T, M>(o0[d], dc[d], o1[d], e.b[d], e.S0[d], e.DS[d], cross);
    e.cross = e.cross || cross;
    T run = T(0);
#pragma unroll
    for (int i = 0; i < W - 1; ++i) {
      run += e.DS[d][i];
      e.CDS[d][i] = run;
    }
    if (!cross) e.CDS[d][W - 2] = T(0);  // the sum of DS over the window vanishes
#pragma unroll
    for (int i = 0; i < W; ++i) {
      e.A[d][i] = e.S0[d][i] + T(0.5) * e.DS[d][i];
      e.Bf[d][i] = T(0.5) * e.S0[d][i] + e.DS[d][i] * T(1.0 / 3.0);
    }
  }
}

// The same factors for a particle whose nearest node (M = 2) or cell (M = 1)
// did not change on any axis (the caller knows it): the window is M + 1 nodes
// from the old nearest node's lower neighbour (M = 2) or the cell (M = 1),
// and only the first M + 1 entries (M for CDS) are filled, which are all that
// the FAST accumulation reads.
template <typename T, int D, int M>
__device__ __forceinline__ void esirkepov_factors_fast(const T o0[3], const T o1[3], Esirk<T, M> &e) {
  e.cross = false;
  e.b[0] = e.b[1] = e.b[2] = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    if constexpr (M == 2) {
      const bool u0 = o0[d] >= T(0.5), u1 = o1[d] >= T(0.5);
      const T d0 = u0 ? o0[d] - T(1) : o0[d], d1 = u1 ? o1[d] - T(1) : o1[d];
      e.b[d] = u0 ? 0 : -1;
      quad_weights<T>(d0, e.S0[d]);
      const T dd = d1 - d0, sm = T(2) * d0 + dd;
      e.DS[d][0] = T(-0.5) * dd * (T(1) - sm);
      e.DS[d][1] = -dd * sm;
      e.DS[d][2] = T(0.5) * dd * (T(1) + sm);
    } else {
      const T dd = o1[d] - o0[d];
      e.S0[d][0] = T(1) - o0[d];
      e.S0[d][1] = o0[d];
      e.DS[d][0] = -dd;
      e.DS[d][1] = dd;
    }
    T run = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) {
      run += e.DS[d][i];
      e.CDS[d][i] = run;
    }
#pragma unroll
    for (int i = 0; i <= M; ++i) {
      e.A[d][i] = e.S0[d][i] + T(0.5) * e.DS[d][i];
      e.Bf[d][i] = T(0.5) * e.S0[d][i] + e.DS[d][i] * T(1.0 / 3.0);
    }
  }
}

// Esirkepov current of one particle:
//   J_x(i+1/2) - J_x(i-1/2) = -(q w / dV)(dx/dt) W_x(i), and in 3D
//   W_x = DS_x (S0_y S0_z + DS_y S0_z / 2 + S0_y DS_z / 2 + DS_y DS_z / 3)
// so J_x over the window is -(q w/dV)(dx/dt) * CDS_x[i] * T_x[j][k] with
// T_x[j][k] = A_y[j] S0_z[k] + Bf_y[j] DS_z[k] (cyclic for y and z).  In 2D3V
// J_z is the time average of the shape product times v_z.  jc[d] = (q w/dV)(dx_d/dt),
// jzc = q w v_z / dV.  FAST (no axis crossed a node): the window is M + 1
// nodes per axis and every add is issued; otherwise M + 2 nodes and exact
// zeros are skipped.
template <typename T, int D, int M, bool FAST, class Acc>
__device__ __forceinline__ void esirkepov_accumulate(const Acc &acc, const int c0[3], const Esirk<T, M> &e,
                                                     const T jc[3], T jzc) {
  constexpr int WJ = FAST ? M + 1 : M + 2;  // nodes across
  constexpr int WI = WJ - 1;                // staggered points along
  const int x0 = c0[0] + e.b[0], y0 = c0[1] + e.b[1], z0 = (D == 3) ? c0[2] + e.b[2] : 0;
  if constexpr (D == 3) {
#pragma unroll
    for (int k = 0; k < WJ; ++k)
#pragma unroll
      for (int j = 0; j < WJ; ++j) {
        const T t = e.A[1][j] * e.S0[2][k] + e.Bf[1][j] * e.DS[2][k];
        if (FAST || t != T(0)) {
#pragma unroll
          for (int i = 0; i < WI; ++i) {
            const T v = -jc[0] * e.CDS[0][i] * t;
            if (FAST || v != T(0)) acc.add(0, x0 + i, y0 + j, z0 + k, v);
          }
        }
      }
#pragma unroll
    for (int k = 0; k < WJ; ++k)
#pragma unroll
      for (int i = 0; i < WJ; ++i) {
        const T t = e.A[0][i] * e.S0[2][k] + e.Bf[0][i] * e.DS[2][k];
        if (FAST || t != T(0)) {
#pragma unroll
          for (int j = 0; j < WI; ++j) {
            const T v = -jc[1] * e.CDS[1][j] * t;
            if (FAST || v != T(0)) acc.add(1, x0 + i, y0 + j, z0 + k, v);
          }
        }
      }
#pragma unroll
    for (int j = 0; j < WJ; ++j)
#pragma unroll
      for (int i = 0; i < WJ; ++i) {
        const T t = e.A[0][i] * e.S0[1][j] + e.Bf[0][i] * e.DS[1][j];
        if (FAST || t != T(0)) {
#pragma unroll
          for (int k = 0; k < WI; ++k) {
            const T v = -jc[2] * e.CDS[2][k] * t;
            if (FAST || v != T(0)) acc.add(2, x0 + i, y0 + j, z0 + k, v);
          }
        }
      }
  } else {
#pragma unroll
    for (int j = 0; j < WJ; ++j) {
      const T t = e.A[1][j];
      if (FAST || t != T(0)) {
#pragma unroll
        for (int i = 0; i < WI; ++i) {
          const T v = -jc[0] * e.CDS[0][i] * t;
          if (FAST || v != T(0)) acc.add(0, x0 + i, y0 + j, 0, v);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < WJ; ++i) {
      const T t = e.A[0][i];
      if (FAST || t != T(0)) {
#pragma unroll
        for (int j = 0; j < WI; ++j) {
          const T v = -jc[1] * e.CDS[1][j] * t;
          if (FAST || v != T(0)) acc.add(1, x0 + i, y0 + j, 0, v);
        }
      }
    }
    if (FAST || jzc != T(0)) {
#pragma unroll
      for (int j = 0; j < WJ; ++j)
#pragma unroll
        for (int i = 0; i < WJ; ++i) {
          const T v = jzc * (e.A[0][i] * e.S0[1][j] + e.Bf[0][i] * e.DS[1][j]);
          if (FAST || v != T(0)) acc.add(2, x0 + i, y0 + j, 0, v);
        }
    }
  }
}

// Esirkepov current of one particle moving from (c0 + o0) to (c0 + dc + o1).
template <typename T, int D, int M, class Acc>
__device__ __forceinline__ void deposit(const Acc &acc, const int c0[3], const T o0[3], const int dc[3], const T o1[3],
                                        const T jc[3], T jzc) {
  Esirk<T, M> e;
  esirkepov_factors<T, D, M>(o0, dc, o1, e);
  if (!e.cross)
    esirkepov_accumulate<T, D, M, true>(acc, c0, e, jc, jzc);
  else
    esirkepov_accumulate<T, D, M, false>(acc, c0, e, jc, jzc);
}

// ---- accessors ------------------------------------------------------------

// One addition into an on-chip current accumulator of type S.  Floating
// accumulators add the value; the 64-bit fixed-point one (unsigned long long,
// two's complement) adds v truncated to an integer (toward zero: one
// conversion, no rounding step): its callers pass contributions already
// scaled by 2^shift (the coefficients of the current carry the factor), which
// keeps every one within 2^30, so the truncation is below 2^-30 of the bound.
template <typename S, typename V>
__device__ __forceinline__ void lds_add(S *p, V v) {
  atomicAdd(p, static_cast<S>(v));
}
template <typename V>
__device__ __forceinline__ void lds_add(unsigned long long *p, V v) {
  const int k = static_cast<int>(static_cast<float>(v));
  atomicAdd(p, static_cast<unsigned long long>(static_cast<long long>(k)));
}

// The value an accumulator holds, in the state's type T (the fixed-point sum
// scaled back by 2^-shift).
template <typename T, typename S>
__device__ __forceinline__ T lds_value(S a, int) {
  return static_cast<T>(a);
}
template <typename T>
__device__ __forceinline__ T lds_value(unsigned long long a, int shift) {
  return static_cast<T>(ldexp(static_cast<double>(static_cast<long long>(a)), -shift));
}

// Fields in HBM with periodic wrap (indices at most a few cells outside).
template <typename T>
struct GlobalFields {
  const T *F[6];
  int n[3];
  __device__ __forceinline__ T load(int comp, int i, int j, int k) const {
    i = wrap_near(i, n[0]);
    j = wrap_near(j, n[1]);
    k = wrap_near(k, n[2]);
    return F[comp][i + (int64_t)n[0] * (j + (int64_t)n[1] * k)];
  }
};

// Current in HBM with periodic wrap; atomic adds.
template <typename T>
struct GlobalCurrent {
  T *J[3];
  int n[3];
  __device__ __forceinline__ void add(int comp, int i, int j, int k, T v) const {
    i = wrap_near(i, n[0]);
    j = wrap_near(j, n[1]);
    k = wrap_near(k, n[2]);
    unsafeAtomicAdd(&J[comp][i + (int64_t)n[0] * (j + (int64_t)n[1] * k)], v);
  }
};

// A box of a field or current tile in LDS: index (i - o0) + sx (j - o1) + sxy (k - o2).
template <typename T>
struct LdsFields {
  const T *base;
  int sx, sxy, vol, o0, o1, o2;
  __device__ __forceinline__ T load(int comp, int i, int j, int k) const {
    return base[comp * vol + (i - o0) + sx * (j - o1) + sxy * (k - o2)];
  }
};

// The same with compile-time strides and origin, so every offset of the
// (M+1)^D stencil folds into the LDS instruction's immediate offset.  S is
// the stored type; values added are converted to it.
template <typename S, int SX, int SXY, int VOL, int OX, int OY, int OZ>
struct LdsBox {
  using value_type = S;
  S *base;
  static constexpr int kSX = SX, kSXY = SXY;
  // floating values with even strides: x runs read as aligned pairs (interp)
  static constexpr bool kPairs = std::is_floating_point<S>::value && SX % 2 == 0 && SXY % 2 == 0 && VOL % 2 == 0;
  __device__ __forceinline__ int index(int comp, int i, int j, int k) const {
    return comp * VOL + (i + OX) + SX * (j + OY) + SXY * (k + OZ);
  }
  __device__ __forceinline__ S load(int comp, int i, int j, int k) const {
    return base[comp * VOL + (i + OX) + SX * (j + OY) + SXY * (k + OZ)];
  }
  template <typename V>
  __device__ __forceinline__ void add(int comp, int i, int j, int k, V v) const {
    lds_add(&base[comp * VOL + (i + OX) + SX * (j + OY) + SXY * (k + OZ)], v);
  }
};

template <typename S>
struct LdsCurrent {
  S *base;
  int sx, sxy, vol, o0, o1, o2;
  template <typename V>
  __device__ __forceinline__ void add(int comp, int i, int j, int k, V v) const {
    lds_add(&base[comp * vol + (i - o0) + sx * (j - o1) + sxy * (k - o2)], v);
  }
};

}  // namespace pic
