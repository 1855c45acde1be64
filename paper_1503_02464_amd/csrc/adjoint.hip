// Hand-written reverse mode of one PIC step.
//
// Field part (Yee): the forward update is B' = B - dt/2 C_E E, E' = E + dt
// (C_B B' - J), B'' = B' - dt/2 C_E E' with C_B = C_E^T, so its transpose
// maps (lamE, lamB) of step n+1 to step n by the same stencils with other
// coefficients: lamE -= dt/2 C_B lamB; lamJ = -dt lamE; lamB += dt C_E lamE;
// lamE -= dt/2 C_B lamB.
//
// Particle part, one thread per particle: recompute the forward step from the
// state at step n (gather, Boris, move, Esirkepov shapes), then propagate
// (lamX^{n+1}, lamU^{n+1/2}, lamJ) back through the deposit, the move, the
// Boris rotation and the gather, adding the gather's transpose to lamE and
// lamB (atomics) and writing (lamX^n, lamU^{n-1/2}).  Positions are
// differentiated through the offsets (cell units); the integer cell is a
// constant of the map.
#include <hip/hip_runtime.h>

#include "particle_math.h"
#include "pic_internal.h"

namespace pic {
namespace {

template <typename T, int M>
__device__ __forceinline__ T bspline(T r) {
  const T a = fabs(r);
  if constexpr (M == 1) return a < T(1) ? T(1) - a : T(0);
  if (a <= T(0.5)) return T(0.75) - r * r;
  if (a < T(1.5)) return T(0.5) * (T(1.5) - a) * (T(1.5) - a);
  return T(0);
}

template <typename T, int M>
__device__ __forceinline__ T bspline_d(T r) {
  const T a = fabs(r);
  const T sg = r < T(0) ? T(-1) : T(1);
  if constexpr (M == 1) return a < T(1) ? -sg : T(0);
  if (a <= T(0.5)) return T(-2) * r;
  if (a < T(1.5)) return -(T(1.5) - a) * sg;
  return T(0);
}

// Gather weights and their derivatives along one axis (see node_weights / half_weights).
template <typename T, int M>
__device__ __forceinline__ void weights_d(int c, T o, bool half, T w[M + 1], T dw[M + 1], int &base) {
  if constexpr (M == 1) {
    if (half) {
      const bool up = o >= T(0.5);
      const T f = up ? o - T(0.5) : o + T(0.5);
      base = up ? c : c - 1;
      w[0] = T(1) - f;
      w[1] = f;
    } else {
      base = c;
      w[0] = T(1) - o;
      w[1] = o;
    }
    dw[0] = T(-1);
    dw[1] = T(1);
  } else {
    T d;
    if (half) {
      base = c - 1;
      d = o - T(0.5);
    } else {
      const bool up = o >= T(0.5);
      base = up ? c : c - 1;
      d = up ? o - T(1) : o;
    }
    quad_weights<T>(d, w);
    dw[0] = -(T(0.5) - d);
    dw[1] = T(-2) * d;
    dw[2] = T(0.5) + d;
  }
}

template <typename T>
struct AdjArgs {
  int64_t np;
  const int32_t *cell;
  const T *off[3];
  const T *u[3];
  const T *w;
  const T *F[6];  // E, B at step n
  T *LF[6];       // lamE, lamB (accumulated)
  const T *LJ[3]; // lamJ
  T *lx[3];       // in lamX^{n+1}, out lamX^n
  T *lu[3];       // in lamU^{n+1/2}, out lamU^{n-1/2}
  int n[3], bits[3], mask[3];
  T h, dtdx[3], jc[3], jz;
  int32_t *flags;
};

__device__ __forceinline__ int64_t gidx(const int n[3], int i, int j, int k) {
  return wrap_near(i, n[0]) + (int64_t)n[0] * (wrap_near(j, n[1]) + (int64_t)n[1] * wrap_near(k, n[2]));
}

// staggering (half = true) of Ex Ey Ez Bx By Bz along x, y, z
__device__ __forceinline__ bool stag(int comp, int d) {
  const int bits[6] = {0b001, 0b010, 0b100, 0b110, 0b101, 0b011};
  return (bits[comp] >> d) & 1;
}

// Fields, lamJ and lamE/lamB in HBM (periodic wrap); lamE/lamB by atomics.
template <typename T>
struct AdjGlobalF {
  const AdjArgs<T> &a;
  __device__ __forceinline__ T load(int comp, int i, int j, int k) const { return a.F[comp][gidx(a.n, i, j, k)]; }
};
template <typename T>
struct AdjGlobalJ {
  const AdjArgs<T> &a;
  __device__ __forceinline__ T load(int comp, int i, int j, int k) const { return a.LJ[comp][gidx(a.n, i, j, k)]; }
};
template <typename T>
struct AdjGlobalL {
  const AdjArgs<T> &a;
  __device__ __forceinline__ void add(int comp, int i, int j, int k, T v) const {
    if (v != T(0)) unsafeAtomicAdd(&a.LF[comp][gidx(a.n, i, j, k)], v);
  }
};

// The reverse of one particle's step.  c is the particle's cell in the frame
// of the accessors (global cell for the HBM ones, cell relative to the tile
// origin for the LDS ones); Fa reads E, B at step n, LJa reads lamJ, LFa adds
// to lamE, lamB.
template <typename T, int D, int M, class FA, class JA, class LA>
__device__ __forceinline__ void adjoint_one(const AdjArgs<T> &a, int64_t p, const int c[3], const T o[3],
                                            const T u0[3], const T w, const FA &Fa, const JA &LJa, const LA &LFa) {
  constexpr int K = M + 1;  // gather stencil per axis
  constexpr int W = M + 2;  // Esirkepov window per axis
  // ---- forward recompute: gather
  T eb[6];
#pragma unroll
  for (int comp = 0; comp < 6; ++comp) {
    T wt[3][K], dw[3][K];
    int b[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < D) {
        weights_d<T, M>(c[d], o[d], stag(comp, d), wt[d], dw[d], b[d]);
      } else {
#pragma unroll
        for (int i = 0; i < K; ++i) wt[d][i] = dw[d][i] = T(0);
        wt[d][0] = T(1);
      }
    }
    T v = T(0);
    const int kmax = D == 3 ? K : 1;
    for (int k = 0; k < kmax; ++k)
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int i = 0; i < K; ++i) v += Fa.load(comp, b[0] + i, b[1] + j, b[2] + k) * wt[0][i] * wt[1][j] * wt[2][k];
    eb[comp] = v;
  }
  // ---- forward recompute: Boris with intermediates
  const T h = a.h;
  T um[3], t[3], s[3], up[3], uh[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) um[d] = u0[d] + h * eb[d];
  const T gm = sqrt(T(1) + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) t[d] = h * eb[3 + d] / gm;
  const T f = T(2) / (T(1) + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) s[d] = f * t[d];
  up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
  up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
  up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
  uh[0] = um[0] + (up[1] * s[2] - up[2] * s[1]) + h * eb[0];
  uh[1] = um[1] + (up[2] * s[0] - up[0] * s[2]) + h * eb[1];
  uh[2] = um[2] + (up[0] * s[1] - up[1] * s[0]) + h * eb[2];
  const T ig = T(1) / sqrt(T(1) + uh[0] * uh[0] + uh[1] * uh[1] + uh[2] * uh[2]);
  T o1[3] = {T(0), T(0), T(0)};
  int dc[3] = {0, 0, 0};
  const bool ok = move<T, D>(uh, ig, a.dtdx, o, o1, dc);
  if (!ok) atomicOr(&a.flags[0], kFlagCross);

  T lx[3] = {T(0), T(0), T(0)}, lx1[3] = {T(0), T(0), T(0)}, luh[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < D) lx1[d] = a.lx[d][p];
    luh[d] = a.lu[d][p];
  }
  T gvz = T(0);
  if (ok) {
    // ---- deposit adjoint: gradients with respect to the old and new shapes
    T S0[3][W], S1[3][W], gS0[3][W], gS1[3][W], dS0[3][W], dS1[3][W];
    int b[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < D) {
        int lo;
        if constexpr (M == 2) {
          const int n0 = o[d] >= T(0.5) ? 1 : 0, n1 = dc[d] + (o1[d] >= T(0.5) ? 1 : 0);
          lo = (n0 < n1 ? n0 : n1) - 1;
        } else {
          lo = dc[d] < 0 ? dc[d] : 0;
        }
        b[d] = lo;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const T r0 = o[d] - T(lo + i), r1 = (T(dc[d]) + o1[d]) - T(lo + i);
          S0[d][i] = bspline<T, M>(r0);
          S1[d][i] = bspline<T, M>(r1);
          dS0[d][i] = bspline_d<T, M>(r0);
          dS1[d][i] = bspline_d<T, M>(r1);
        }
      } else {
#pragma unroll
        for (int i = 0; i < W; ++i) S0[d][i] = S1[d][i] = dS0[d][i] = dS1[d][i] = T(0);
        S0[d][0] = S1[d][0] = T(1);
      }
#pragma unroll
      for (int i = 0; i < W; ++i) gS0[d][i] = gS1[d][i] = T(0);
    }
    const T third = T(1.0 / 3.0), sixth = T(1.0 / 6.0);
    if constexpr (D == 3) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const int bb = ax == 0 ? 1 : 0, cc = ax == 2 ? 1 : 2;  // transverse axes, ascending
        const T JC = w * a.jc[ax];
        T gC[W - 1], gT[W][W];
#pragma unroll
        for (int i = 0; i < W - 1; ++i) gC[i] = T(0);
#pragma unroll
        for (int j = 0; j < W; ++j)
#pragma unroll
          for (int k = 0; k < W; ++k) gT[j][k] = T(0);
        T cds = T(0);
#pragma unroll
        for (int i = 0; i < W - 1; ++i) {
          cds += S1[ax][i] - S0[ax][i];
#pragma unroll
          for (int j = 0; j < W; ++j)
#pragma unroll
            for (int k = 0; k < W; ++k) {
              int nd[3];
              nd[ax] = c[ax] + b[ax] + i;
              nd[bb] = c[bb] + b[bb] + j;
              nd[cc] = c[cc] + b[cc] + k;
              const T L = LJa.load(ax, nd[0], nd[1], nd[2]);
              const T Tt = third * (S0[bb][j] * S0[cc][k] + S1[bb][j] * S1[cc][k]) +
                           sixth * (S0[bb][j] * S1[cc][k] + S1[bb][j] * S0[cc][k]);
              gC[i] += -JC * L * Tt;
              gT[j][k] += -JC * L * cds;
            }
        }
        T run = T(0);
#pragma unroll
        for (int i = W - 2; i >= 0; --i) {
          run += gC[i];
          gS1[ax][i] += run;
          gS0[ax][i] -= run;
        }
#pragma unroll
        for (int j = 0; j < W; ++j)
#pragma unroll
          for (int k = 0; k < W; ++k) {
            const T g = gT[j][k];
            gS0[bb][j] += g * (third * S0[cc][k] + sixth * S1[cc][k]);
            gS1[bb][j] += g * (third * S1[cc][k] + sixth * S0[cc][k]);
            gS0[cc][k] += g * (third * S0[bb][j] + sixth * S1[bb][j]);
            gS1[cc][k] += g * (third * S1[bb][j] + sixth * S0[bb][j]);
          }
      }
    } else {
#pragma unroll
      for (int ax = 0; ax < 2; ++ax) {
        const int bb = 1 - ax;
        const T JC = w * a.jc[ax];
        T gC[W - 1], gA[W];
#pragma unroll
        for (int i = 0; i < W - 1; ++i) gC[i] = T(0);
#pragma unroll
        for (int j = 0; j < W; ++j) gA[j] = T(0);
        T cds = T(0);
#pragma unroll
        for (int i = 0; i < W - 1; ++i) {
          cds += S1[ax][i] - S0[ax][i];
#pragma unroll
          for (int j = 0; j < W; ++j) {
            int nd[2];
            nd[ax] = c[ax] + b[ax] + i;
            nd[bb] = c[bb] + b[bb] + j;
            const T L = LJa.load(ax, nd[0], nd[1], 0);
            const T A = T(0.5) * (S0[bb][j] + S1[bb][j]);
            gC[i] += -JC * L * A;
            gA[j] += -JC * L * cds;
          }
        }
        T run = T(0);
#pragma unroll
        for (int i = W - 2; i >= 0; --i) {
          run += gC[i];
          gS1[ax][i] += run;
          gS0[ax][i] -= run;
        }
#pragma unroll
        for (int j = 0; j < W; ++j) {
          gS0[bb][j] += T(0.5) * gA[j];
          gS1[bb][j] += T(0.5) * gA[j];
        }
      }
      // J_z = (q w / dA) v_z Tz
      const T vz = uh[2] * ig;
      const T JZ = w * a.jz;
#pragma unroll
      for (int i = 0; i < W; ++i)
#pragma unroll
        for (int j = 0; j < W; ++j) {
          const T L = LJa.load(2, c[0] + b[0] + i, c[1] + b[1] + j, 0);
          const T Tz = third * (S0[0][i] * S0[1][j] + S1[0][i] * S1[1][j]) +
                       sixth * (S0[0][i] * S1[1][j] + S1[0][i] * S0[1][j]);
          gvz += JZ * L * Tz;
          const T g = JZ * vz * L;
          gS0[0][i] += g * (third * S0[1][j] + sixth * S1[1][j]);
          gS1[0][i] += g * (third * S1[1][j] + sixth * S0[1][j]);
          gS0[1][j] += g * (third * S0[0][i] + sixth * S1[0][i]);
          gS1[1][j] += g * (third * S1[0][i] + sixth * S0[0][i]);
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      T g0 = T(0), g1 = T(0);
#pragma unroll
      for (int i = 0; i < W; ++i) {
        g0 += gS0[d][i] * dS0[d][i];
        g1 += gS1[d][i] * dS1[d][i];
      }
      lx1[d] += g1;  // the new position also feeds the deposit
      lx[d] = lx1[d] + g0;
    }
    // ---- move adjoint: x^{n+1} = x^n + dt/dx u/gamma
    T av[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int d = 0; d < D; ++d) av[d] = lx1[d] * a.dtdx[d];
    const T adu = av[0] * uh[0] + av[1] * uh[1] + av[2] * uh[2];
    const T ig3 = ig * ig * ig;
#pragma unroll
    for (int d = 0; d < 3; ++d) luh[d] += ig * av[d] - ig3 * uh[d] * adu;
    if (D == 2) {  // v_z = u_z / gamma in J_z
#pragma unroll
      for (int d = 0; d < 3; ++d) luh[d] += gvz * ((d == 2 ? ig : T(0)) - uh[2] * uh[d] * ig3);
    }
  } else {
#pragma unroll
    for (int d = 0; d < D; ++d) lx[d] = lx1[d];
  }
  // ---- Boris adjoint
  T lE[3], lB[3], lum[3], lup[3], ls[3], lt[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) lE[d] = h * luh[d];
  // u+ = um + up x s
  lup[0] = s[1] * luh[2] - s[2] * luh[1];
  lup[1] = s[2] * luh[0] - s[0] * luh[2];
  lup[2] = s[0] * luh[1] - s[1] * luh[0];
  ls[0] = luh[1] * up[2] - luh[2] * up[1];
  ls[1] = luh[2] * up[0] - luh[0] * up[2];
  ls[2] = luh[0] * up[1] - luh[1] * up[0];
  // up = um + um x t
  lum[0] = luh[0] + lup[0] + (t[1] * lup[2] - t[2] * lup[1]);
  lum[1] = luh[1] + lup[1] + (t[2] * lup[0] - t[0] * lup[2]);
  lum[2] = luh[2] + lup[2] + (t[0] * lup[1] - t[1] * lup[0]);
  lt[0] = lup[1] * um[2] - lup[2] * um[1];
  lt[1] = lup[2] * um[0] - lup[0] * um[2];
  lt[2] = lup[0] * um[1] - lup[1] * um[0];
  // s = f t, f = 2 / (1 + t.t)
  const T tls = t[0] * ls[0] + t[1] * ls[1] + t[2] * ls[2];
#pragma unroll
  for (int d = 0; d < 3; ++d) lt[d] += f * ls[d] - f * f * t[d] * tls;
  // t = h B / gm
#pragma unroll
  for (int d = 0; d < 3; ++d) lB[d] = h / gm * lt[d];
  const T lgm = -(t[0] * lt[0] + t[1] * lt[1] + t[2] * lt[2]) / gm;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lum[d] += lgm * um[d] / gm;
    lE[d] += h * lum[d];
  }
  // ---- gather adjoint: scatter lamEB with the shape, and position gradient
  const T leb[6] = {lE[0], lE[1], lE[2], lB[0], lB[1], lB[2]};
#pragma unroll
  for (int comp = 0; comp < 6; ++comp) {
    T wt[3][K], dw[3][K];
    int b[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d < D) {
        weights_d<T, M>(c[d], o[d], stag(comp, d), wt[d], dw[d], b[d]);
      } else {
#pragma unroll
        for (int i = 0; i < K; ++i) wt[d][i] = dw[d][i] = T(0);
        wt[d][0] = T(1);
      }
    }
    const int kmax = D == 3 ? K : 1;
    for (int k = 0; k < kmax; ++k)
#pragma unroll
      for (int j = 0; j < K; ++j)
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const T Fv = Fa.load(comp, b[0] + i, b[1] + j, b[2] + k);
          lx[0] += leb[comp] * Fv * dw[0][i] * wt[1][j] * wt[2][k];
          lx[1] += leb[comp] * Fv * wt[0][i] * dw[1][j] * wt[2][k];
          if (D == 3) lx[2] += leb[comp] * Fv * wt[0][i] * wt[1][j] * dw[2][k];
          const T v = leb[comp] * wt[0][i] * wt[1][j] * wt[2][k];
          LFa.add(comp, b[0] + i, b[1] + j, b[2] + k, v);
        }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (d < D) a.lx[d][p] = lx[d];
    a.lu[d][p] = lum[d];
  }
}

// One thread per particle, fields in HBM: every particle (list null) or the
// listed ones (the stragglers of the tiled pass).
template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_particle_adjoint(AdjArgs<T> a, const int32_t *list, const int32_t *count) {
  const int64_t n = list ? *count : a.np;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = list ? list[k] : k;
    if (p < 0 || p >= a.np) continue;
    const uint32_t pk = static_cast<uint32_t>(a.cell[p]);
    int c[3] = {static_cast<int>(pk & a.mask[0]), static_cast<int>((pk >> a.bits[0]) & a.mask[1]),
                static_cast<int>((pk >> (a.bits[0] + a.bits[1])) & a.mask[2])};
#pragma unroll
    for (int d = 0; d < 3; ++d) c[d] = c[d] >= a.n[d] ? c[d] - a.n[d] : c[d];
    T o[3], u0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      o[d] = d < D ? a.off[d][p] : T(0);
      u0[d] = a.u[d][p];
    }
    adjoint_one<T, D, M>(a, p, c, o, u0, a.w[p], AdjGlobalF<T>{a}, AdjGlobalJ<T>{a}, AdjGlobalL<T>{a});
  }
}

// Tile geometry of the tiled adjoint (the fused forward kernel's boxes).
struct AdjTile {
  const int32_t *tile_start;  // ranges of the last sort of these particles, in this order
  int L[3], ntile[3], slack;
  int rf[3], rj[3];           // field and current box sizes
  int gf_lo[3], gj_lo[3];     // box origins below the tile origin
  int32_t *stray_count, *stray_list;
};

// Full periodic reduction (guard boxes may exceed n on small grids).
__device__ __forceinline__ int adj_wrap(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// One workgroup per tile of sorted particles: stage E, B (step n) and lamJ of
// the tile plus guards in LDS, run the reverse step of every particle within
// the slack against them, accumulate the gather's transpose in an FP64 LDS
// box, and add that box to lamE, lamB in HBM.  Particles further out are
// listed for the HBM kernel.
template <typename T, int D, int M>
__global__ void __launch_bounds__(256) k_particle_adjoint_tiled(AdjArgs<T> a, AdjTile t) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t tile = blockIdx.x;
  int64_t pbeg = t.tile_start[tile], pend = t.tile_start[tile + 1];
  pbeg = pbeg < 0 ? 0 : (pbeg > a.np ? a.np : pbeg);
  pend = pend > a.np ? a.np : pend;
  if (pbeg >= pend) return;
  const int T0[3] = {static_cast<int>(tile % t.ntile[0]) * t.L[0],
                     static_cast<int>((tile / t.ntile[0]) % t.ntile[1]) * t.L[1],
                     static_cast<int>(tile / ((int64_t)t.ntile[0] * t.ntile[1])) * t.L[2]};
  const int FX = t.rf[0], FY = t.rf[1], FVOL = t.rf[0] * t.rf[1] * t.rf[2];
  const int JX = t.rj[0], JY = t.rj[1], JVOL = t.rj[0] * t.rj[1] * t.rj[2];
  double *lfb = reinterpret_cast<double *>(smem_raw);  // [6][FVOL] lamE, lamB
  T *fb = reinterpret_cast<T *>(lfb + 6 * FVOL);       // [6][FVOL] E, B
  T *jb = fb + 6 * FVOL;                               // [3][JVOL] lamJ
  for (int idx = threadIdx.x; idx < FVOL; idx += 256) {
    const int li = idx % FX, lj = (idx / FX) % FY, lk = idx / (FX * FY);
    const int64_t g = adj_wrap(T0[0] - t.gf_lo[0] + li, a.n[0]) +
                      (int64_t)a.n[0] * (adj_wrap(T0[1] - t.gf_lo[1] + lj, a.n[1]) +
                                         (int64_t)a.n[1] * adj_wrap(T0[2] - t.gf_lo[2] + lk, a.n[2]));
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      fb[c * FVOL + idx] = a.F[c][g];
      lfb[c * FVOL + idx] = 0.0;
    }
  }
  for (int idx = threadIdx.x; idx < JVOL; idx += 256) {
    const int li = idx % JX, lj = (idx / JX) % JY, lk = idx / (JX * JY);
    const int64_t g = adj_wrap(T0[0] - t.gj_lo[0] + li, a.n[0]) +
                      (int64_t)a.n[0] * (adj_wrap(T0[1] - t.gj_lo[1] + lj, a.n[1]) +
                                         (int64_t)a.n[1] * adj_wrap(T0[2] - t.gj_lo[2] + lk, a.n[2]));
#pragma unroll
    for (int c = 0; c < 3; ++c) jb[c * JVOL + idx] = a.LJ[c][g];
  }
  __syncthreads();
  const LdsFields<T> Fa{fb, FX, FX * FY, FVOL, -t.gf_lo[0], -t.gf_lo[1], -t.gf_lo[2]};
  const LdsFields<T> Ja{jb, JX, JX * JY, JVOL, -t.gj_lo[0], -t.gj_lo[1], -t.gj_lo[2]};
  const LdsCurrent<double> La{lfb, FX, FX * FY, FVOL, -t.gf_lo[0], -t.gf_lo[1], -t.gf_lo[2]};
  for (int64_t p = pbeg + threadIdx.x; p < pend; p += 256) {
    const uint32_t pk = static_cast<uint32_t>(a.cell[p]);
    int c[3] = {static_cast<int>(pk & a.mask[0]), static_cast<int>((pk >> a.bits[0]) & a.mask[1]),
                static_cast<int>((pk >> (a.bits[0] + a.bits[1])) & a.mask[2])};
    // cell relative to the tile origin, unwrapped across the periodic seam
    int lc[3] = {0, 0, 0};
    bool inside = true;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      c[d] = c[d] >= a.n[d] ? c[d] - a.n[d] : c[d];
      int l = c[d] - T0[d];
      if (l > a.n[d] / 2) l -= a.n[d];
      if (l < -a.n[d] / 2) l += a.n[d];
      lc[d] = l;
      inside = inside && l >= -t.slack && l < t.L[d] + t.slack;
    }
    if (!inside) {
      t.stray_list[atomicAdd(t.stray_count, 1)] = static_cast<int32_t>(p);
      continue;
    }
    T o[3], u0[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      o[d] = d < D ? a.off[d][p] : T(0);
      u0[d] = a.u[d][p];
    }
    adjoint_one<T, D, M>(a, p, lc, o, u0, a.w[p], Fa, Ja, La);
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < FVOL; idx += 256) {
    const int li = idx % FX, lj = (idx / FX) % FY, lk = idx / (FX * FY);
    const int64_t g = adj_wrap(T0[0] - t.gf_lo[0] + li, a.n[0]) +
                      (int64_t)a.n[0] * (adj_wrap(T0[1] - t.gf_lo[1] + lj, a.n[1]) +
                                         (int64_t)a.n[1] * adj_wrap(T0[2] - t.gf_lo[2] + lk, a.n[2]));
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const T v = static_cast<T>(lfb[c * FVOL + idx]);
      if (v != T(0)) unsafeAtomicAdd(&a.LF[c][g], v);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_scale_copy(T *d0, T *d1, T *d2, const T *s0, const T *s1, const T *s2,
                                                    int64_t n, T scale) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    d0[i] = scale * s0[i];
    d1[i] = scale * s1[i];
    d2[i] = scale * s2[i];
  }
}

template <typename T, int D, int M>
hipError_t particle_adjoint_impl(const pic_ctx &c, const pic_species &sp, const pic_fields &f,
                                 const pic_fields &lam, const pic_species_adjoint &lsp, hipStream_t st) {
  if (sp.np == 0) return hipSuccess;
  AdjArgs<T> a{};
  a.np = sp.np;
  a.cell = sp.cell;
  for (int d = 0; d < 3; ++d) {
    a.off[d] = static_cast<const T *>(d < c.p.dims ? sp.off[d] : sp.off[0]);
    a.u[d] = static_cast<const T *>(sp.u[d]);
    a.F[d] = static_cast<const T *>(f.E[d]);
    a.F[3 + d] = static_cast<const T *>(f.B[d]);
    a.LF[d] = static_cast<T *>(lam.E[d]);
    a.LF[3 + d] = static_cast<T *>(lam.B[d]);
    a.LJ[d] = static_cast<const T *>(lam.J[d]);
    a.lx[d] = static_cast<T *>(d < c.p.dims ? lsp.x[d] : lsp.x[0]);
    a.lu[d] = static_cast<T *>(lsp.u[d]);
    a.n[d] = static_cast<int>(c.n[d]);
    a.bits[d] = c.bits[d];
    a.mask[d] = (1 << c.bits[d]) - 1;
  }
  a.w = static_cast<const T *>(sp.w);
  double dV = 1.0;
  for (int d = 0; d < c.p.dims; ++d) dV *= c.p.dx[d];
  a.h = static_cast<T>(sp.q * c.p.dt / (2.0 * sp.m));
  for (int d = 0; d < 3; ++d) {
    a.dtdx[d] = static_cast<T>(d < c.p.dims ? c.p.dt / c.p.dx[d] : 0.0);
    a.jc[d] = static_cast<T>(d < c.p.dims ? sp.q / dV * c.p.dx[d] / c.p.dt : 0.0);
  }
  a.jz = static_cast<T>(sp.q / dV);
  a.flags = c.wsp<int32_t>(c.ws.flags);
  // per tile when the particles' tile ranges are known and the boxes fit in LDS
  const size_t fvol = static_cast<size_t>(c.rf[0]) * c.rf[1] * c.rf[2];
  const size_t lds = 6 * fvol * 8 + 6 * fvol * sizeof(T) + 3 * static_cast<size_t>(c.rj[0]) * c.rj[1] * c.rj[2] * sizeof(T);
  if (sp.tile_start && lds <= kLdsLimit) {
    AdjTile t{};
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
    // the count goes to the bank the next fused launch takes, which then
    // clears that bank itself; the straggler count reads this call's
    t.stray_count = c.wsp<int32_t>(c.ws.stray_count) + 16 * c.stray_bank;
    t.stray_list = c.wsp<int32_t>(c.ws.stray_list);
    const auto kern = k_particle_adjoint_tiled<T, D, M>;
    c.stray_clean = false;
    c.stray_last = c.stray_bank;
    hipError_t e = launch_fill_zero(t.stray_count, 1, 4, st);
    if (e == hipSuccess && lds > 65536)
      e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(c.ntiles)), dim3(256), lds, st, a, t);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int64_t sblocks = (sp.np + 255) / 256;
    if (sblocks > 1024) sblocks = 1024;
    hipLaunchKernelGGL((k_particle_adjoint<T, D, M>), dim3(static_cast<unsigned>(sblocks)), dim3(256), 0, st, a,
                       t.stray_list, t.stray_count);
    return hipGetLastError();
  }
  const unsigned blocks = static_cast<unsigned>((sp.np + 255) / 256);
  hipLaunchKernelGGL((k_particle_adjoint<T, D, M>), dim3(blocks), dim3(256), 0, st, a, nullptr, nullptr);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_particle_adjoint(const pic_ctx &c, const pic_species &sp, const pic_fields &f,
                                   const pic_fields &lam, const pic_species_adjoint &lsp, hipStream_t s) {
  const bool f64 = c.p.precision == PIC_FP64;
  const int key = (f64 ? 4 : 0) + (c.p.dims == 3 ? 2 : 0) + (c.p.shape_order - 1);
  switch (key) {
    case 0: return particle_adjoint_impl<float, 2, 1>(c, sp, f, lam, lsp, s);
    case 1: return particle_adjoint_impl<float, 2, 2>(c, sp, f, lam, lsp, s);
    case 2: return particle_adjoint_impl<float, 3, 1>(c, sp, f, lam, lsp, s);
    case 3: return particle_adjoint_impl<float, 3, 2>(c, sp, f, lam, lsp, s);
    case 4: return particle_adjoint_impl<double, 2, 1>(c, sp, f, lam, lsp, s);
    case 5: return particle_adjoint_impl<double, 2, 2>(c, sp, f, lam, lsp, s);
    case 6: return particle_adjoint_impl<double, 3, 1>(c, sp, f, lam, lsp, s);
    default: return particle_adjoint_impl<double, 3, 2>(c, sp, f, lam, lsp, s);
  }
}

hipError_t launch_scale_copy(const pic_ctx &c, void *const dst[3], const void *const src[3], double scale,
                             hipStream_t s) {
  int64_t blocks = (c.ncells + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (c.p.precision == PIC_FP64)
    hipLaunchKernelGGL(k_scale_copy<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<double *>(dst[0]), static_cast<double *>(dst[1]), static_cast<double *>(dst[2]),
                       static_cast<const double *>(src[0]), static_cast<const double *>(src[1]),
                       static_cast<const double *>(src[2]), c.ncells, scale);
  else
    hipLaunchKernelGGL(k_scale_copy<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<float *>(dst[0]), static_cast<float *>(dst[1]), static_cast<float *>(dst[2]),
                       static_cast<const float *>(src[0]), static_cast<const float *>(src[1]),
                       static_cast<const float *>(src[2]), c.ncells, static_cast<float>(scale));
  return hipGetLastError();
}

}  // namespace pic
