// Per-bond ACE basis on the device: Chebyshev radial functions with the
// cosine cutoff, real spherical harmonics by recurrence, and their
// derivatives.  Templated on the arithmetic type (double for the FP64 path,
// float for the mixed path).
//
// Radial: g_k(r) = T_k(x) fc(r), x = 2r/rc - 1, fc = (1 + cos(pi r/rc))/2,
// with T_{k+1} = 2x T_k - T_{k-1} and T'_{k+1} = 2 T_k + 2x T'_k - T'_{k-1};
// R_nl = sum_k W_nlk g_k.
// Harmonics for a unit vector u = (x, y, z): Q_l^m = d^m P_l/dz^m from the
// three-term recurrence (l-m) Q_l^m = (2l-1) z Q_{l-1}^m - (l+m-1) Q_{l-2}^m
// with Q_m^m = (2m-1)!!, and (x + iy)^m = C_m + i S_m:
// Y_l0 = N_l0 Q_l^0, Y_{l,m} = sqrt2 N_lm Q_l^m C_m, Y_{l,-m} = sqrt2 N_lm Q_l^m S_m.
// Gradient with respect to the bond vector d: tangential part of the
// polynomial gradient (dQ_l^m/dz = Q_l^{m+1}), divided by |d|.
#pragma once
#include <hip/hip_runtime.h>

#include "ap_internal.h"

namespace ap {

template <typename T>
__device__ __forceinline__ T t_cos(T x);
template <>
__device__ __forceinline__ double t_cos<double>(double x) { return cos(x); }
template <>
__device__ __forceinline__ float t_cos<float>(float x) { return cosf(x); }
template <typename T>
__device__ __forceinline__ T t_sin(T x);
template <>
__device__ __forceinline__ double t_sin<double>(double x) { return sin(x); }
template <>
__device__ __forceinline__ float t_sin<float>(float x) { return sinf(x); }

// Chebyshev-times-cutoff basis g[k] and dg/dr for k < K
template <typename T>
__device__ __forceinline__ void cheb_basis(int K, T rc, T r, T* g, T* dg) {
  const T pi = (T)3.14159265358979323846;
  const T x = (T)2 * r / rc - (T)1;
  const T arg = pi * r / rc;
  const T fc = (T)0.5 * ((T)1 + t_cos<T>(arg));
  const T dfc = (T)-0.5 * pi / rc * t_sin<T>(arg);
  T t0 = 1, t1 = x, d0 = 0, d1 = 1;
  const T s = (T)2 / rc;
  g[0] = fc;
  dg[0] = dfc;
  g[1] = x * fc;
  dg[1] = d1 * s * fc + x * dfc;
#pragma unroll
  for (int k = 2; k < kMaxK; ++k) {
    const T t2 = (T)2 * x * t1 - t0;
    const T d2 = (T)2 * t1 + (T)2 * x * d1 - d0;
    g[k] = t2 * fc;
    dg[k] = d2 * s * fc + t2 * dfc;
    t0 = t1; t1 = t2; d0 = d1; d1 = d2;
  }
  (void)K;
}

// Q[l][m] = d^m P_l / dz^m for 0 <= m <= l+1 (zero for m = l+1), l <= lmax
template <typename T>
__device__ __forceinline__ void legendre_derivs(int lmax, T z, T Q[kMaxL + 1][kMaxL + 2]) {
  (void)lmax;
#pragma unroll
  for (int m = 0; m <= kMaxL; ++m) {
    T dfact = 1;
#pragma unroll
    for (int k = 1; k <= 2 * m - 1; k += 2) dfact *= (T)k;
    Q[m][m] = dfact;
    if (m + 1 <= kMaxL) Q[m + 1][m] = (T)(2 * m + 1) * z * dfact;
#pragma unroll
    for (int l = m + 2; l <= kMaxL; ++l)
      Q[l][m] = ((T)(2 * l - 1) * z * Q[l - 1][m] - (T)(l + m - 1) * Q[l - 2][m]) / (T)(l - m);
  }
#pragma unroll
  for (int l = 0; l <= kMaxL; ++l) Q[l][l + 1] = 0;
}

// Y[lm] (lm = l*l + l + m) of the unit vector (x, y, z); with dY != nullptr
// also dY[lm][3] = dY/dd for a bond of length r.
template <typename T>
__device__ __forceinline__ void real_ylm(int lmax, const double* ynorm, T x, T y, T z, T r, T* Y,
                                         T (*dY)[3]) {
  T Q[kMaxL + 1][kMaxL + 2];
  legendre_derivs<T>(lmax, z, Q);
  T C[kMaxL + 1], S[kMaxL + 1];
  C[0] = 1;
  S[0] = 0;
#pragma unroll
  for (int m = 1; m <= kMaxL; ++m) {
    C[m] = x * C[m - 1] - y * S[m - 1];
    S[m] = x * S[m - 1] + y * C[m - 1];
  }
  const T ir = (T)1 / r;
#pragma unroll
  for (int l = 0; l <= kMaxL; ++l) {
    if (l > lmax) break;
    const int c0 = l * l + l;
    {
      const T nrm = (T)ynorm[c0];
      Y[c0] = nrm * Q[l][0];
      if (dY) {
        T gx = 0, gy = 0, gz = nrm * Q[l][1];
        const T ug = z * gz;
        dY[c0][0] = (gx - ug * x) * ir;
        dY[c0][1] = (gy - ug * y) * ir;
        dY[c0][2] = (gz - ug * z) * ir;
      }
    }
#pragma unroll
    for (int m = 1; m <= l; ++m) {
      const T nrm = (T)ynorm[c0 + m];
      Y[c0 + m] = nrm * Q[l][m] * C[m];
      Y[c0 - m] = nrm * Q[l][m] * S[m];
      if (dY) {
        const T q = nrm * Q[l][m] * (T)m, dq = nrm * Q[l][m + 1];
        T gx = q * C[m - 1], gy = -q * S[m - 1], gz = dq * C[m];
        T ug = x * gx + y * gy + z * gz;
        dY[c0 + m][0] = (gx - ug * x) * ir;
        dY[c0 + m][1] = (gy - ug * y) * ir;
        dY[c0 + m][2] = (gz - ug * z) * ir;
        gx = q * S[m - 1];
        gy = q * C[m - 1];
        gz = dq * S[m];
        ug = x * gx + y * gy + z * gz;
        dY[c0 - m][0] = (gx - ug * x) * ir;
        dY[c0 - m][1] = (gy - ug * y) * ir;
        dY[c0 - m][2] = (gz - ug * z) * ir;
      }
    }
  }
}

// sum_lm b[lm] Y_lm and sum_lm a[lm] dY_lm/dd without storing dY
template <typename T>
__device__ __forceinline__ void ylm_contract(int lmax, const double* ynorm, T x, T y, T z, T r,
                                             const T* a, const T* b, T& yb, T& gx_o, T& gy_o,
                                             T& gz_o) {
  T Q[kMaxL + 1][kMaxL + 2];
  legendre_derivs<T>(lmax, z, Q);
  T C[kMaxL + 1], S[kMaxL + 1];
  C[0] = 1;
  S[0] = 0;
#pragma unroll
  for (int m = 1; m <= kMaxL; ++m) {
    C[m] = x * C[m - 1] - y * S[m - 1];
    S[m] = x * S[m - 1] + y * C[m - 1];
  }
  T sb = 0, gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int l = 0; l <= kMaxL; ++l) {
    if (l > lmax) break;
    const int c0 = l * l + l;
    {
      const T nrm = (T)ynorm[c0];
      sb += b[c0] * nrm * Q[l][0];
      gz += a[c0] * nrm * Q[l][1];
    }
#pragma unroll
    for (int m = 1; m <= l; ++m) {
      const T nrm = (T)ynorm[c0 + m];
      const T ap = a[c0 + m], am = a[c0 - m];
      sb += nrm * Q[l][m] * (b[c0 + m] * C[m] + b[c0 - m] * S[m]);
      const T q = nrm * Q[l][m] * (T)m, dq = nrm * Q[l][m + 1];
      gx += q * (ap * C[m - 1] + am * S[m - 1]);
      gy += q * (-ap * S[m - 1] + am * C[m - 1]);
      gz += dq * (ap * C[m] + am * S[m]);
    }
  }
  // tangential projection of the polynomial gradient, divided by r
  const T ir = (T)1 / r;
  const T ug = x * gx + y * gy + z * gz;
  yb = sb;
  gx_o = (gx - ug * x) * ir;
  gy_o = (gy - ug * y) * ir;
  gz_o = (gz - ug * z) * ir;
}

}  // namespace ap
