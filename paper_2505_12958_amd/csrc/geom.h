// Canonical minimum-image displacement shared by every kernel that visits a
// bond.  Operation order is fixed and nothing is contracted into fused
// multiply-adds, so the neighbour test r^2 < rc^2 is bit-exact against any
// implementation of the same recipe (see the ap_systems comment in ap.h).
#pragma once
#include <hip/hip_runtime.h>

namespace ap {

__device__ __forceinline__ void frac3(const double* Hi, double x, double y, double z, double& s0,
                                      double& s1, double& s2) {
#pragma clang fp contract(off)
  s0 = (x * Hi[0] + y * Hi[3]) + z * Hi[6];
  s1 = (x * Hi[1] + y * Hi[4]) + z * Hi[7];
  s2 = (x * Hi[2] + y * Hi[5]) + z * Hi[8];
}

__device__ __forceinline__ double wrap_half(double d, double L) {
#pragma clang fp contract(off)
  const double half = 0.5 * L;
  return d > half ? d - L : (d < -half ? d + L : d);
}

__device__ __forceinline__ double wrap_unit(double d) {
#pragma clang fp contract(off)
  return d > 0.5 ? d - 1.0 : (d < -0.5 ? d + 1.0 : d);
}

// d = r_j - r_i in an orthorhombic box of edge lengths (Lx, Ly, Lz).
__device__ __forceinline__ void displacement_ortho(const int32_t* per, double Lx, double Ly,
                                                   double Lz, double xi, double yi, double zi,
                                                   double xj, double yj, double zj, double& dx,
                                                   double& dy, double& dz) {
#pragma clang fp contract(off)
  dx = xj - xi;
  dy = yj - yi;
  dz = zj - zi;
  if (per[0]) dx = wrap_half(dx, Lx);
  if (per[1]) dy = wrap_half(dy, Ly);
  if (per[2]) dz = wrap_half(dz, Lz);
}

// d = r_j - r_i for system box H (row-major rows = lattice vectors).
__device__ __forceinline__ void displacement(bool ortho, const double* H, const double* Hi,
                                             const int32_t* per, double xi, double yi, double zi,
                                             double xj, double yj, double zj, double& dx,
                                             double& dy, double& dz) {
#pragma clang fp contract(off)
  if (ortho) {
    displacement_ortho(per, H[0], H[4], H[8], xi, yi, zi, xj, yj, zj, dx, dy, dz);
  } else {
    double si0, si1, si2, sj0, sj1, sj2;
    frac3(Hi, xi, yi, zi, si0, si1, si2);
    frac3(Hi, xj, yj, zj, sj0, sj1, sj2);
    const double a = wrap_unit(sj0 - si0);
    const double b = wrap_unit(sj1 - si1);
    const double c = wrap_unit(sj2 - si2);
    dx = (a * H[0] + b * H[3]) + c * H[6];
    dy = (a * H[1] + b * H[4]) + c * H[7];
    dz = (a * H[2] + b * H[5]) + c * H[8];
  }
}

__device__ __forceinline__ double norm2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return (dx * dx + dy * dy) + dz * dz;
}


}  // namespace ap
