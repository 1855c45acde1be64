// Field kernels: the Yee curl updates (paper Sec. 2, FDTD on the Yee lattice)
// and a zero fill.  One thread per cell, x fastest so loads and stores are
// coalesced; neighbours along y and z come from rows that neighbouring
// workgroups also read, so they are served mostly from L2.
#include <hip/hip_runtime.h>

#include <cmath>

#include "pic_internal.h"

namespace pic {
namespace {

template <typename T>
struct Yee {
  const T *E[3];
  T *B[3];
  T *Eo[3];
  const T *Bi[3];
  const T *J[3];
  int n[3];
  T cx, cy, cz;  // dt/dx_d (times the half-step fraction for B)
  T cj;          // dt
  int use_j;     // 0: E += frac dt curl B only (J is not read)
};

// B -= f dt curl E, forward differences onto the B points.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_yee_b(Yee<T> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n[0]) return;
  const int j = blockIdx.y, k = blockIdx.z;
  const int64_t sx = a.n[0], sxy = (int64_t)a.n[0] * a.n[1];
  const int64_t o = i + sx * j + sxy * k;
  const int64_t ip = (i + 1 == a.n[0]) ? o - i : o + 1;
  const int64_t jp = (j + 1 == a.n[1]) ? o - sx * j : o + sx;
  const T ex = a.E[0][o], ey = a.E[1][o], ez = a.E[2][o];
  const T dEz_dy = a.cy * (a.E[2][jp] - ez), dEx_dy = a.cy * (a.E[0][jp] - ex);
  const T dEz_dx = a.cx * (a.E[2][ip] - ez), dEy_dx = a.cx * (a.E[1][ip] - ey);
  T dEy_dz = T(0), dEx_dz = T(0);
  if constexpr (D == 3) {
    const int64_t kp = (k + 1 == a.n[2]) ? o - sxy * k : o + sxy;
    dEy_dz = a.cz * (a.E[1][kp] - ey);
    dEx_dz = a.cz * (a.E[0][kp] - ex);
  }
  a.B[0][o] -= dEz_dy - dEy_dz;
  a.B[1][o] -= dEx_dz - dEz_dx;
  a.B[2][o] -= dEy_dx - dEx_dy;
}

// E += dt (curl B - J), backward differences onto the E points.
template <typename T, int D>
__global__ void __launch_bounds__(256) k_yee_e(Yee<T> a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n[0]) return;
  const int j = blockIdx.y, k = blockIdx.z;
  const int64_t sx = a.n[0], sxy = (int64_t)a.n[0] * a.n[1];
  const int64_t o = i + sx * j + sxy * k;
  const int64_t im = (i == 0) ? o + (a.n[0] - 1) : o - 1;
  const int64_t jm = (j == 0) ? o + sx * (a.n[1] - 1) : o - sx;
  const T bx = a.Bi[0][o], by = a.Bi[1][o], bz = a.Bi[2][o];
  const T dBz_dy = a.cy * (bz - a.Bi[2][jm]), dBx_dy = a.cy * (bx - a.Bi[0][jm]);
  const T dBz_dx = a.cx * (bz - a.Bi[2][im]), dBy_dx = a.cx * (by - a.Bi[1][im]);
  T dBy_dz = T(0), dBx_dz = T(0);
  if constexpr (D == 3) {
    const int64_t km = (k == 0) ? o + sxy * (a.n[2] - 1) : o - sxy;
    dBy_dz = a.cz * (by - a.Bi[1][km]);
    dBx_dz = a.cz * (bx - a.Bi[0][km]);
  }
  const T jx = a.use_j ? a.cj * a.J[0][o] : T(0);
  const T jy = a.use_j ? a.cj * a.J[1][o] : T(0);
  const T jz = a.use_j ? a.cj * a.J[2][o] : T(0);
  a.Eo[0][o] += (dBz_dy - dBy_dz) - jx;
  a.Eo[1][o] += (dBx_dz - dBz_dx) - jy;
  a.Eo[2][o] += (dBy_dx - dBx_dy) - jz;
}

// ---------------------------------------------------------------------------
// One-pass Yee step (3D): B^{n+1/2} = B^n - dt/2 curl E^n, E^{n+1} = E^n +
// dt (curl B^{n+1/2} - J), B^{n+1} = B^{n+1/2} - dt/2 curl E^{n+1}, reading
// E^n, B^n, J once and writing E^{n+1}, B^{n+1} into the second field set.
//
// A workgroup owns an xy tile of YX x YY cells and marches up through a chunk
// of z planes.  Each thread owns one column of the tile plus its halo (x from
// x0 - 1 to x0 + YX + 2, y from y0 - 1 to y0 + YY + 1) and keeps its own
// column's values of the planes z and z +- 1 in registers; the x and y
// differences read the neighbours' values of the current plane from LDS.
// Per plane z the workgroup computes B^{n+1/2}(z) on the tile plus one
// layer, E^{n+1}(z) on the tile plus one layer above (two in x, where the
// Mur update of a wrapped face needs the point inside it), and B^{n+1}(z-1)
// on the tile.  A chunk starts one plane early (B^{n+1/2} below it) and ends
// one plane late (E^{n+1} above it), so chunks overlap by two planes of
// recomputed values and read each input plane at most three times more.
// With open x faces, E_y and E_z on the node planes i = 0 and i = n0 - 1
// take the first-order Mur update from E^n of the face and the plane inside
// it and E^{n+1} of the plane inside, before B^{n+1} uses them.
// ---------------------------------------------------------------------------
constexpr int kYX = 64, kYY = 8;                  // tile of output columns
constexpr int kYPX = kYX + 4, kYPY = kYY + 3;     // columns a workgroup holds
constexpr int kYPlane = kYPX * kYPY;              // 748
constexpr int kYThreads = (kYPlane + 63) / 64 * 64;  // 768

template <typename T>
struct YeeFused {
  const T *E[3], *B[3], *J[3];
  T *Eo[3], *Bo[3];
  int n[3];
  int ntx, nty, nch, chunk;  // xy tiles per dimension, z chunks, planes per chunk
  T hx, hy, hz;              // dt/2 / dx_d
  T fx, fy, fz;              // dt / dx_d
  T dt;
  int open;                  // Mur on the x faces
  T mur;                     // (dt - dx) / (dt + dx)
};

template <typename T>
__global__ void __launch_bounds__(kYThreads) k_yee_fused(YeeFused<T> a) {
  __shared__ T sE[3][kYPlane];      // E^n(z)
  __shared__ T sH[3][kYPlane];      // B^{n+1/2}(z)
  __shared__ T sN[2][3][kYPlane];   // E^{n+1}(z - 1), E^{n+1}(z), by parity of the plane
  // XCD-aware work order: the 8 XCDs take contiguous ranges of (xy tile,
  // chunk) items, so the tiles whose halos overlap run on one XCD's L2.
  const int nwork = a.ntx * a.nty * a.nch;
  const int per = (nwork + 7) / 8;
  const int w = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (w >= nwork) return;
  const int ch = w % a.nch, tx = (w / a.nch) % a.ntx, ty = w / (a.nch * a.ntx);
  const int lx = threadIdx.x % kYPX, ly = threadIdx.x / kYPX;
  const bool mine = threadIdx.x < kYPlane;
  const int n0 = a.n[0], n1 = a.n[1], n2 = a.n[2];
  // global column (periodic wrap)
  int gx = tx * kYX - 1 + lx, gy = ty * kYY - 1 + ly;
  gx = gx < 0 ? gx + n0 : (gx >= n0 ? gx - n0 : gx);
  gy = gy < 0 ? gy + n1 : (gy >= n1 ? gy - n1 : gy);
  const int64_t col = gx + (int64_t)n0 * gy, plane = (int64_t)n0 * n1;
  // regions in local column coordinates
  const bool r2 = mine && lx < kYX + 3 && ly < kYY + 2;                                    // B^{n+1/2}
  const bool r1 = mine && lx >= 1 && lx < kYX + 3 && ly >= 1 && ly < kYY + 2;              // E^{n+1}
  const bool out = mine && lx >= 1 && lx < kYX + 1 && ly >= 1 && ly < kYY + 1;             // written
  const int me = ly * kYPX + lx;
  const int zs = ch * a.chunk, ze = zs + a.chunk < n2 ? zs + a.chunk : n2;
  auto zw = [&](int z) { return z < 0 ? z + n2 : (z >= n2 ? z - n2 : z); };
  auto ld = [&](const T *const F[3], int z, T v[3], bool on) {
    const int64_t o = col + plane * zw(z);
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = on ? F[c][o] : T(0);
  };
  // Mur: which face this column is (0 none, 1 low, 2 high) and the column inside it
  const int face = (a.open && r1) ? (gx == 0 ? 1 : (gx == n0 - 1 ? 2 : 0)) : 0;
  const int inner = face == 1 ? me + 1 : (face == 2 ? me - 1 : me);

  T E0[3], E1[3], Bn[3], Jn[3], pE[3], pB[3], pJ[3], H0[3], H1[3], N0[3], N1[3];
  ld(a.E, zs - 1, E0, mine);
  ld(a.E, zs, E1, mine);
  ld(a.B, zs - 1, Bn, r2);
#pragma unroll
  for (int c = 0; c < 3; ++c) Jn[c] = H0[c] = H1[c] = N0[c] = N1[c] = T(0);
  ld(a.E, zs + 1, pE, mine);
  ld(a.B, zs, pB, r2);
  ld(a.J, zs, pJ, r1);
  for (int z = zs - 1; z <= ze; ++z) {
    // E^n(z) to LDS
    if (mine) {
#pragma unroll
      for (int c = 0; c < 3; ++c) sE[c][me] = E0[c];
    }
    __syncthreads();
    // B^{n+1/2}(z) = B^n(z) - dt/2 curl E^n (forward differences)
    if (r2) {
      const T dEz_dy = sE[2][me + kYPX] - E0[2], dEx_dy = sE[0][me + kYPX] - E0[0];
      const T dEz_dx = sE[2][me + 1] - E0[2], dEy_dx = sE[1][me + 1] - E0[1];
      const T dEy_dz = E1[1] - E0[1], dEx_dz = E1[0] - E0[0];
      H1[0] = Bn[0] - (a.hy * dEz_dy - a.hz * dEy_dz);
      H1[1] = Bn[1] - (a.hz * dEx_dz - a.hx * dEz_dx);
      H1[2] = Bn[2] - (a.hx * dEy_dx - a.hy * dEx_dy);
#pragma unroll
      for (int c = 0; c < 3; ++c) sH[c][me] = H1[c];
    }
    __syncthreads();
    // E^{n+1}(z) = E^n(z) + dt (curl B^{n+1/2} - J) (backward differences)
    const int cur = z & 1;
    if (z >= zs) {
      if (r1) {
        const T dBz_dy = H1[2] - sH[2][me - kYPX], dBx_dy = H1[0] - sH[0][me - kYPX];
        const T dBz_dx = H1[2] - sH[2][me - 1], dBy_dx = H1[1] - sH[1][me - 1];
        const T dBy_dz = H1[1] - H0[1], dBx_dz = H1[0] - H0[0];
        N1[0] = E0[0] + ((a.fy * dBz_dy - a.fz * dBy_dz) - a.dt * Jn[0]);
        N1[1] = E0[1] + ((a.fz * dBx_dz - a.fx * dBz_dx) - a.dt * Jn[1]);
        N1[2] = E0[2] + ((a.fx * dBy_dx - a.fy * dBx_dy) - a.dt * Jn[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) sN[cur][c][me] = N1[c];
      }
      if (a.open) {  // uniform over the workgroup
        __syncthreads();
        if (face) {
#pragma unroll
          for (int c = 1; c < 3; ++c) {
            N1[c] = sE[c][inner] + a.mur * (sN[cur][c][inner] - E0[c]);
          }
        }
        __syncthreads();
        if (face) {
#pragma unroll
          for (int c = 1; c < 3; ++c) sN[cur][c][me] = N1[c];
        }
      }
    }
    __syncthreads();
    // B^{n+1}(z - 1) = B^{n+1/2}(z - 1) - dt/2 curl E^{n+1}, and E^{n+1}(z - 1), out
    if (z >= zs + 1 && out) {
      const int prv = cur ^ 1;
      const T dEz_dy = sN[prv][2][me + kYPX] - N0[2], dEx_dy = sN[prv][0][me + kYPX] - N0[0];
      const T dEz_dx = sN[prv][2][me + 1] - N0[2], dEy_dx = sN[prv][1][me + 1] - N0[1];
      const T dEy_dz = N1[1] - N0[1], dEx_dz = N1[0] - N0[0];
      const int64_t o = col + plane * zw(z - 1);
      a.Bo[0][o] = H0[0] - (a.hy * dEz_dy - a.hz * dEy_dz);
      a.Bo[1][o] = H0[1] - (a.hz * dEx_dz - a.hx * dEz_dx);
      a.Bo[2][o] = H0[2] - (a.hx * dEy_dx - a.hy * dEx_dy);
#pragma unroll
      for (int c = 0; c < 3; ++c) a.Eo[c][o] = N0[c];
    }
    // next plane
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      E0[c] = E1[c];
      E1[c] = pE[c];
      Bn[c] = pB[c];
      Jn[c] = pJ[c];
      H0[c] = H1[c];
      N0[c] = N1[c];
    }
    if (z + 1 < ze) {  // the planes iteration z + 2 needs (the last one, ze, needs none beyond)
      ld(a.E, z + 3, pE, mine);
      ld(a.B, z + 2, pB, r2);
      ld(a.J, z + 2, pJ, r1);
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill_zero(T *p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = T(0);
}

// Up to kFillArrays arrays of n elements in one launch (grid y picks the array).
template <typename T>
struct FillArrays {
  T *p[kFillArrays];
};
template <typename T>
__global__ void __launch_bounds__(256) k_fill_zero_n(FillArrays<T> a, int64_t n) {
  T *p = a.p[blockIdx.y];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) p[i] = T(0);
}

template <typename T>
Yee<T> yee_args(const pic_ctx &c, const pic_fields &f, double frac) {
  Yee<T> a{};
  for (int d = 0; d < 3; ++d) {
    a.E[d] = static_cast<const T *>(f.E[d]);
    a.B[d] = static_cast<T *>(f.B[d]);
    a.Eo[d] = static_cast<T *>(f.E[d]);
    a.Bi[d] = static_cast<const T *>(f.B[d]);
    a.J[d] = static_cast<const T *>(f.J[d]);
    a.n[d] = static_cast<int>(c.n[d]);
  }
  a.cx = static_cast<T>(frac * c.p.dt / c.p.dx[0]);
  a.cy = static_cast<T>(frac * c.p.dt / c.p.dx[1]);
  a.cz = static_cast<T>(c.p.dims == 3 ? frac * c.p.dt / c.p.dx[2] : 0.0);
  a.cj = static_cast<T>(c.p.dt);
  a.use_j = 1;
  return a;
}

dim3 yee_grid(const pic_ctx &c, int block) {
  return dim3(static_cast<unsigned>((c.n[0] + block - 1) / block), static_cast<unsigned>(c.n[1]),
              static_cast<unsigned>(c.n[2]));
}

int yee_block(const pic_ctx &c) { return c.n[0] >= 256 ? 256 : static_cast<int>((c.n[0] + 63) / 64 * 64); }

// Open x faces (first-order Mur on the tangential E of the face planes
// i = 0 and i = n0-1).  k_mur_save keeps E_y, E_z^n of the planes
// {0, 1, n0-2, n0-1} before the E update; k_mur_apply then replaces the
// faces: E_face^{n+1} = E_next^n + a (E_next^{n+1} - E_face^n),
// a = (dt - dx)/(dt + dx), "next" one plane inside.
template <typename T>
__global__ void __launch_bounds__(256) k_mur_save(const T *__restrict__ Ey, const T *__restrict__ Ez, T *old, int n0,
                                                  int64_t nyz) {
  const int64_t jk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (jk >= nyz) return;
  const int plane[4] = {0, 1, n0 - 2, n0 - 1};
  const int64_t row = (int64_t)n0 * jk;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    old[q * nyz + jk] = Ey[row + plane[q]];
    old[(4 + q) * nyz + jk] = Ez[row + plane[q]];
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_mur_apply(T *Ey, T *Ez, const T *__restrict__ old, int n0, int64_t nyz,
                                                   T a) {
  const int64_t jk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (jk >= nyz) return;
  const int64_t row = (int64_t)n0 * jk;
  T *F[2] = {Ey, Ez};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const T *o = old + 4 * c * nyz;
    T *f = F[c] + row;
    const T lo = o[nyz + jk] + a * (f[1] - o[jk]);
    const T hi = o[2 * nyz + jk] + a * (f[n0 - 2] - o[3 * nyz + jk]);
    f[0] = lo;
    f[n0 - 1] = hi;
  }
}

// Laser sheet: J[plane, j, k] += amp exp(-r^2 / w0^2), r from the axis at
// the J component's staggered point; amp carries the time dependence.
template <typename T>
__global__ void __launch_bounds__(256) k_laser(T *J, int plane, int n0, int n1, int64_t nyz, int dims, double dy,
                                               double dz, double sy, double sz, double amp, double inv_w02, double yc,
                                               double zc) {
  const int64_t jk = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (jk >= nyz) return;
  const int j = static_cast<int>(jk % n1);
  const int k = static_cast<int>(jk / n1);
  const double y = (j + sy) * dy - yc;
  const double z = dims == 3 ? (k + sz) * dz - zc : 0.0;
  J[plane + (int64_t)n0 * jk] += static_cast<T>(amp * exp(-(y * y + z * z) * inv_w02));
}


bool yee_fused_supported(const pic_ctx &c) {
  return c.p.dims == 3 && c.n[0] % kYX == 0 && c.n[1] % kYY == 0 && c.n[2] >= 2;
}

template <typename T>
hipError_t yee_fused_impl(const pic_ctx &c, const pic_fields &f, hipStream_t s) {
  YeeFused<T> a{};
  for (int d = 0; d < 3; ++d) {
    a.E[d] = static_cast<const T *>(f.E[d]);
    a.B[d] = static_cast<const T *>(f.B[d]);
    a.J[d] = static_cast<const T *>(f.J[d]);
    a.Eo[d] = static_cast<T *>(f.E_alt[d]);
    a.Bo[d] = static_cast<T *>(f.B_alt[d]);
    a.n[d] = static_cast<int>(c.n[d]);
  }
  a.ntx = static_cast<int>(c.n[0] / kYX);
  a.nty = static_cast<int>(c.n[1] / kYY);
  // enough (tile, chunk) items for two workgroups per CU, chunks of at least 4 planes
  int nch = (512 + a.ntx * a.nty - 1) / (a.ntx * a.nty);
  const int most = static_cast<int>(c.n[2] / 4) > 1 ? static_cast<int>(c.n[2] / 4) : 1;
  nch = nch < 1 ? 1 : (nch > most ? most : nch);
  a.chunk = static_cast<int>((c.n[2] + nch - 1) / nch);
  a.nch = static_cast<int>((c.n[2] + a.chunk - 1) / a.chunk);
  const double dt = c.p.dt;
  a.hx = static_cast<T>(0.5 * dt / c.p.dx[0]);
  a.hy = static_cast<T>(0.5 * dt / c.p.dx[1]);
  a.hz = static_cast<T>(0.5 * dt / c.p.dx[2]);
  a.fx = static_cast<T>(dt / c.p.dx[0]);
  a.fy = static_cast<T>(dt / c.p.dx[1]);
  a.fz = static_cast<T>(dt / c.p.dx[2]);
  a.dt = static_cast<T>(dt);
  a.open = c.p.open_x;
  a.mur = static_cast<T>((dt - c.p.dx[0]) / (dt + c.p.dx[0]));
  const int64_t nwork = static_cast<int64_t>(a.ntx) * a.nty * a.nch;
  const unsigned blocks = static_cast<unsigned>((nwork + 7) / 8 * 8);
  hipLaunchKernelGGL(k_yee_fused<T>, dim3(blocks), dim3(kYThreads), 0, s, a);
  return hipGetLastError();
}
}  // namespace

bool yee_fused_ok(const pic_ctx &c, const pic_fields &f) {
  if (!yee_fused_supported(c)) return false;
  for (int d = 0; d < 3; ++d)
    if (!f.E_alt[d] || !f.B_alt[d]) return false;
  return true;
}

hipError_t launch_yee_fused(const pic_ctx &c, const pic_fields &f, hipStream_t s) {
  if (!yee_fused_ok(c, f)) return hipErrorInvalidValue;
  return c.p.precision == PIC_FP64 ? yee_fused_impl<double>(c, f, s) : yee_fused_impl<float>(c, f, s);
}

hipError_t launch_yee_b(const pic_ctx &c, const pic_fields &f, double frac, hipStream_t s) {
  const int bs = yee_block(c);
  const dim3 grid = yee_grid(c, bs);
  const bool f64 = c.p.precision == PIC_FP64;
  if (f64) {
    if (c.p.dims == 3)
      hipLaunchKernelGGL((k_yee_b<double, 3>), grid, dim3(bs), 0, s, yee_args<double>(c, f, frac));
    else
      hipLaunchKernelGGL((k_yee_b<double, 2>), grid, dim3(bs), 0, s, yee_args<double>(c, f, frac));
  } else {
    if (c.p.dims == 3)
      hipLaunchKernelGGL((k_yee_b<float, 3>), grid, dim3(bs), 0, s, yee_args<float>(c, f, frac));
    else
      hipLaunchKernelGGL((k_yee_b<float, 2>), grid, dim3(bs), 0, s, yee_args<float>(c, f, frac));
  }
  return hipGetLastError();
}

hipError_t launch_yee_e(const pic_ctx &c, const pic_fields &f, hipStream_t s, double frac, bool with_j) {
  const int bs = yee_block(c);
  const dim3 grid = yee_grid(c, bs);
  const bool f64 = c.p.precision == PIC_FP64;
  if (f64) {
    auto a = yee_args<double>(c, f, frac);
    a.use_j = with_j ? 1 : 0;
    if (c.p.dims == 3)
      hipLaunchKernelGGL((k_yee_e<double, 3>), grid, dim3(bs), 0, s, a);
    else
      hipLaunchKernelGGL((k_yee_e<double, 2>), grid, dim3(bs), 0, s, a);
  } else {
    auto a = yee_args<float>(c, f, frac);
    a.use_j = with_j ? 1 : 0;
    if (c.p.dims == 3)
      hipLaunchKernelGGL((k_yee_e<float, 3>), grid, dim3(bs), 0, s, a);
    else
      hipLaunchKernelGGL((k_yee_e<float, 2>), grid, dim3(bs), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *ptr, int64_t n, size_t elem, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (elem == 8)
    hipLaunchKernelGGL(k_fill_zero<double>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<double *>(ptr), n);
  else if (elem == 4)
    hipLaunchKernelGGL(k_fill_zero<float>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<float *>(ptr), n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fill_zero_n(void *const *ptrs, int count, int64_t n, size_t elem, hipStream_t s) {
  if (count < 1 || count > kFillArrays) return hipErrorInvalidValue;
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;  // writes stream best with many workgroups in flight
  const dim3 grid(static_cast<unsigned>(blocks), static_cast<unsigned>(count));
  if (elem == 8) {
    FillArrays<double> a{};
    for (int i = 0; i < count; ++i) a.p[i] = static_cast<double *>(ptrs[i]);
    hipLaunchKernelGGL(k_fill_zero_n<double>, grid, dim3(256), 0, s, a, n);
  } else if (elem == 4) {
    FillArrays<float> a{};
    for (int i = 0; i < count; ++i) a.p[i] = static_cast<float *>(ptrs[i]);
    hipLaunchKernelGGL(k_fill_zero_n<float>, grid, dim3(256), 0, s, a, n);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mur(const pic_ctx &c, const pic_fields &f, bool save, hipStream_t s) {
  const int64_t nyz = c.n[1] * c.n[2];
  const unsigned blocks = static_cast<unsigned>((nyz + 255) / 256);
  const int n0 = static_cast<int>(c.n[0]);
  const double a = (c.p.dt - c.p.dx[0]) / (c.p.dt + c.p.dx[0]);
  if (c.p.precision == PIC_FP64) {
    auto *old = c.wsp<double>(c.ws.mur_old);
    if (save)
      hipLaunchKernelGGL(k_mur_save<double>, dim3(blocks), dim3(256), 0, s, static_cast<const double *>(f.E[1]),
                         static_cast<const double *>(f.E[2]), old, n0, nyz);
    else
      hipLaunchKernelGGL(k_mur_apply<double>, dim3(blocks), dim3(256), 0, s, static_cast<double *>(f.E[1]),
                         static_cast<double *>(f.E[2]), old, n0, nyz, a);
  } else {
    auto *old = c.wsp<float>(c.ws.mur_old);
    if (save)
      hipLaunchKernelGGL(k_mur_save<float>, dim3(blocks), dim3(256), 0, s, static_cast<const float *>(f.E[1]),
                         static_cast<const float *>(f.E[2]), old, n0, nyz);
    else
      hipLaunchKernelGGL(k_mur_apply<float>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(f.E[1]),
                         static_cast<float *>(f.E[2]), old, n0, nyz, static_cast<float>(a));
  }
  return hipGetLastError();
}

hipError_t launch_laser(const pic_ctx &c, const pic_fields &f, double t, hipStream_t s) {
  const pic_laser &L = c.laser;
  const double env = std::exp(-2.0 * std::log(2.0) * (t - L.t0) * (t - L.t0) / (L.tau * L.tau));
  const double amp = c.laser_j0 * env * std::sin(L.omega * (t - L.t0));
  const int64_t nyz = c.n[1] * c.n[2];
  const unsigned blocks = static_cast<unsigned>((nyz + 255) / 256);
  const double sy = L.pol == 1 ? 0.5 : 0.0, sz = L.pol == 2 ? 0.5 : 0.0;
  const double dz = c.p.dims == 3 ? c.p.dx[2] : 0.0;
  void *J = f.J[L.pol];
  if (c.p.precision == PIC_FP64)
    hipLaunchKernelGGL(k_laser<double>, dim3(blocks), dim3(256), 0, s, static_cast<double *>(J), L.plane,
                       static_cast<int>(c.n[0]), static_cast<int>(c.n[1]), nyz, c.p.dims, c.p.dx[1], dz, sy, sz, amp,
                       1.0 / (L.w0 * L.w0), L.yc, L.zc);
  else
    hipLaunchKernelGGL(k_laser<float>, dim3(blocks), dim3(256), 0, s, static_cast<float *>(J), L.plane,
                       static_cast<int>(c.n[0]), static_cast<int>(c.n[1]), nyz, c.p.dims, c.p.dx[1], dz, sy, sz, amp,
                       1.0 / (L.w0 * L.w0), L.yc, L.zc);
  return hipGetLastError();
}

}  // namespace pic
