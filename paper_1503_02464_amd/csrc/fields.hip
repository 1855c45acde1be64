// Field kernels: the Yee curl updates (paper Sec. 2, FDTD on the Yee lattice)
// and a zero fill.  One thread per cell, x fastest so loads and stores are
// coalesced; neighbours along y and z come from rows that neighbouring
// workgroups also read, so they are served mostly from L2.
#include <hip/hip_runtime.h>

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

template <typename T>
__global__ void __launch_bounds__(256) k_fill_zero(T *p, int64_t n) {
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

}  // namespace

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

}  // namespace pic
