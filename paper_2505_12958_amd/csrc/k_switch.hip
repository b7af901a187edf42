// Dynamic switching parameter (paper: section "Adaptive-precision potential"
// and the appendix "Switching function" with the table of the adaptive-
// precision model's parameters), in the ACE-weight convention
// mu = 1 - lambda_paper:
//
//  1. CSP_i: the n/2 smallest |d_a + d_b|^2 over the pairs of the n nearest
//     neighbours (n = 14 for BCC), summed in ascending order; fewer than n
//     neighbours within the cutoff: (n/2) (2 r_c)^2;
//  2. time average c_i <- c_i + (CSP_i - c_i)/N_csp; detection mu0_i: 0 below
//     CSP_lo, 1 above CSP_hi, a cosine ramp between; 1 inside the precise
//     ball, 0 for surface atoms outside it;
//  3. spatial transition mu_i = max_j mu0_j g(r_ij), g = 1 up to r_lo, a
//     cosine down to 0 at r_hi;
//  4. time average m_i <- m_i + (mu_i - m_i)/N_lambda; lambda_i = m_i snapped
//     to 0 / 1 within dlambda_min; the ascending list of atoms with
//     lambda_i > 0.
//
// Every decision (which neighbours, which pair sums, inside or outside a
// zone or the transition range) is taken on FP64 values computed in a fixed
// operation order with nothing contracted, so it is bit-exact against any
// implementation of the same recipe; the max of step 3 does not depend on
// the order in which sources are combined.
#include "ap_internal.h"
#include "geom.h"
#include "scan.h"

#include <algorithm>

namespace ap {

constexpr int kCspWaves = 4;
constexpr int kMaxCsp = 16;

// (key, index) order: smaller key first, equal keys by index
__device__ __forceinline__ bool before(double a, int ia, double b, int ib) {
  return a < b || (a == b && ia < ib);
}

// ---- 1. CSP, one wavefront per atom
__global__ __launch_bounds__(64 * kCspWaves) void k_csp(SysView sv, const double* __restrict__ pos,
                                                        const int32_t* __restrict__ nbr,
                                                        const int32_t* __restrict__ count, int cap,
                                                        int n_csp, double csp_full,
                                                        double* __restrict__ csp) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n = sv.n_atoms;
  const int i = blockIdx.x * kCspWaves + wave;
  if (i >= n) return;  // whole wavefront
  const int per_wave = cap + 3 * kMaxCsp + kMaxCsp * (kMaxCsp - 1) / 2 + kMaxCsp;
  double* r2s = reinterpret_cast<double*>(lds) + (size_t)wave * per_wave;  // [cap]
  double* sel = r2s + cap;                                                  // [n][3]
  double* sums = sel + 3 * kMaxCsp;                                         // [n(n-1)/2]
  double* low = sums + kMaxCsp * (kMaxCsp - 1) / 2;                         // [n/2]
  const int c = count[i];
  if (c < n_csp) {
    if (lane == 0) csp[i] = csp_full;
    return;
  }
  const int s = sv.sys_of[i];
  const bool ortho = sv.ortho[s] != 0;
  const double* H = sv.H + 9 * s;
  const double* Hi = sv.Hi + 9 * s;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  auto disp = [&](int slot, double& dx, double& dy, double& dz) {
    const int j = nbr[(int64_t)slot * n + i];
    displacement(ortho, H, Hi, sv.per, xi, yi, zi, pos[j], pos[n + j], pos[2 * n + j], dx, dy, dz);
  };
  for (int k = lane; k < c; k += 64) {
    double dx, dy, dz;
    disp(k, dx, dy, dz);
    r2s[k] = norm2(dx, dy, dz);
  }
  __syncwarp_ap();
  // the n nearest: each candidate's rank in (r^2, slot) order; slots are in
  // ascending neighbour index, so equal distances keep that order
  for (int k = lane; k < c; k += 64) {
    const double v = r2s[k];
    int rank = 0;
    for (int m = 0; m < c; ++m) rank += before(r2s[m], m, v, k) ? 1 : 0;
    if (rank < n_csp) {
      double dx, dy, dz;
      disp(k, dx, dy, dz);
      sel[3 * rank] = dx;
      sel[3 * rank + 1] = dy;
      sel[3 * rank + 2] = dz;
    }
  }
  __syncwarp_ap();
  // pair sums |d_a + d_b|^2, a < b
  const int np = n_csp * (n_csp - 1) / 2;
  for (int q = lane; q < np; q += 64) {
    int a = 0, rem = q;
    while (rem >= n_csp - 1 - a) {
      rem -= n_csp - 1 - a;
      ++a;
    }
    const int b = a + 1 + rem;
    const double sx = sel[3 * a] + sel[3 * b];
    const double sy = sel[3 * a + 1] + sel[3 * b + 1];
    const double sz = sel[3 * a + 2] + sel[3 * b + 2];
    sums[q] = norm2(sx, sy, sz);
  }
  __syncwarp_ap();
  // the n/2 smallest, in ascending order (equal values are interchangeable)
  const int half = n_csp / 2;
  for (int q = lane; q < np; q += 64) {
    const double v = sums[q];
    int rank = 0;
    for (int m = 0; m < np; ++m) rank += before(sums[m], m, v, q) ? 1 : 0;
    if (rank < half) low[rank] = v;
  }
  __syncwarp_ap();
  if (lane == 0) {
    double t = 0.0;
    for (int k = 0; k < half; ++k) t += low[k];
    csp[i] = t;
  }
}

struct SwitchArgs {
  double csp_lo, csp_hi, r_lo, r_hi, n_csp_avg, n_lam_avg, dmin;
  double cx, cy, cz, r_precise, zsurf;
  int32_t init;
};

__device__ __forceinline__ double ramp_csp(double c, double lo, double hi) {
#pragma clang fp contract(off)
  if (c <= lo) return 0.0;
  if (c >= hi) return 1.0;
  return 0.5 * (1.0 - cos(M_PI * ((c - lo) / (hi - lo))));
}

// ---- 2. averaged CSP, detection value and fixed zones; flags of the sources
__global__ void k_switch_detect(int n, const double* __restrict__ pos, const double* __restrict__ csp,
                                double* __restrict__ c_avg, SwitchArgs a, double* __restrict__ mu0,
                                int32_t* __restrict__ flag) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double c = csp[i];
  const double ca = a.init ? c : c_avg[i] + (c - c_avg[i]) / a.n_csp_avg;
  c_avg[i] = ca;
  double m = ramp_csp(ca, a.csp_lo, a.csp_hi);
  const double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
  bool inside = false;
  if (a.r_precise > 0.0) {
    const double dx = x - a.cx, dy = y - a.cy, dz = z - a.cz;
    inside = norm2(dx, dy, dz) <= a.r_precise * a.r_precise;
  }
  if (inside) m = 1.0;
  else if (z >= a.zsurf) m = 0.0;
  mu0[i] = m;
  flag[i] = m > 0.0 ? 1 : 0;
}

// ---- 3. spatial transition: one wavefront per source, the cells within
// r_hi of it (cell edge >= cutoff), max-combined into mu (FP64 bit patterns
// of non-negative values order like unsigned integers)
__global__ __launch_bounds__(256) void k_switch_spread(
    SysView sv, const double* __restrict__ pos, const int32_t* __restrict__ cell_of,
    const int32_t* __restrict__ cell_start, const int32_t* __restrict__ cell_count,
    const int32_t* __restrict__ cell_atoms, const double4* __restrict__ cell_pos,
    const int32_t* __restrict__ src, const int32_t* __restrict__ n_src_p,
    const double* __restrict__ mu0, SwitchArgs a, unsigned long long* __restrict__ mu_bits) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int n_src = *n_src_p;
  const int n = sv.n_atoms;
  const double rh2 = a.r_hi * a.r_hi;
  for (int w = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); w < n_src;
       w += gridDim.x * (blockDim.x >> 6)) {
    const int j = src[w];
    const double mj = mu0[j];
    const int s = sv.sys_of[j];
    const int* g = sv.grid + 3 * s;
    const double* H = sv.H + 9 * s;
    const int local = cell_of[j] - sv.cell_base[s];
    const int c0 = local / (g[1] * g[2]), c1 = (local / g[2]) % g[1], c2 = local % g[2];
    int R[3], lo[3], cnt[3];
    const int cc[3] = {c0, c1, c2};
    for (int k = 0; k < 3; ++k) {
      const double edge = H[4 * k] / g[k];
      R[k] = (int)ceil(a.r_hi / edge);
      if (sv.per[k] && 2 * R[k] + 1 >= g[k]) {
        lo[k] = 0;
        cnt[k] = g[k];
      } else {
        lo[k] = cc[k] - R[k];
        cnt[k] = 2 * R[k] + 1;
      }
    }
    const double xj = pos[j], yj = pos[n + j], zj = pos[2 * n + j];
    const int ncell = cnt[0] * cnt[1] * cnt[2];
    for (int q = lane; q < ncell; q += 64) {
      int o0 = lo[0] + q / (cnt[1] * cnt[2]);
      int o1 = lo[1] + (q / cnt[2]) % cnt[1];
      int o2 = lo[2] + q % cnt[2];
      const int o[3] = {o0, o1, o2};
      bool ok = true;
      int w3[3];
      for (int k = 0; k < 3; ++k) {
        int v = o[k];
        if (sv.per[k]) v = ((v % g[k]) + g[k]) % g[k];
        else if (v < 0 || v >= g[k]) ok = false;
        w3[k] = v;
      }
      if (!ok) continue;
      const int cell = sv.cell_base[s] + (w3[0] * g[1] + w3[1]) * g[2] + w3[2];
      const int b = cell_start[cell], e = b + cell_count[cell];
      for (int t = b; t < e; ++t) {
        const double4 p = cell_pos[t];
        double dx, dy, dz;
        displacement_ortho(sv.per, H[0], H[4], H[8], xj, yj, zj, p.x, p.y, p.z, dx, dy, dz);
        const double r2 = norm2(dx, dy, dz);
        if (r2 < rh2) {
          const double r = sqrt(r2);
          const double gr =
              r <= a.r_lo ? 1.0 : 0.5 * (1.0 + cos((M_PI * (r - a.r_lo)) / (a.r_hi - a.r_lo)));
          const double v = mj * gr;
          if (v > 0.0) atomicMax(&mu_bits[cell_atoms[t]], (unsigned long long)__double_as_longlong(v));
        }
      }
    }
  }
}

// ---- 4. averaged mu, snapping, flags of the ACE list
__global__ void k_switch_finish(int n, const unsigned long long* __restrict__ mu_bits,
                                double* __restrict__ m_avg, SwitchArgs a, double* __restrict__ lambda,
                                int32_t* __restrict__ flag) {
#pragma clang fp contract(off)
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double mu = __longlong_as_double((long long)mu_bits[i]);
  const double m = a.init ? mu : m_avg[i] + (mu - m_avg[i]) / a.n_lam_avg;
  m_avg[i] = m;
  const double l = m < a.dmin ? 0.0 : (m > 1.0 - a.dmin ? 1.0 : m);
  lambda[i] = l;
  flag[i] = l > 0.0 ? 1 : 0;
}

hipError_t launch_switching(const SysView& sv, const double* pos, const int32_t* nbr,
                            const int32_t* count, int32_t cap, const int32_t* cell_of,
                            const int32_t* cell_start, const int32_t* cell_count,
                            const int32_t* cell_atoms, const double4* cell_pos,
                            const ap_switching& sw, double csp_full, double* csp, double* mu0,
                            unsigned long long* mu_bits, int32_t* flag, int32_t* src, int32_t* n_src,
                            int32_t* scan_tmp, double* lambda, int32_t* ace_list, int32_t* n_ace,
                            hipStream_t s) {
  const int n = sv.n_atoms;
  SwitchArgs a;
  a.csp_lo = sw.csp_lo;
  a.csp_hi = sw.csp_hi;
  a.r_lo = sw.r_lo;
  a.r_hi = sw.r_hi;
  a.n_csp_avg = (double)sw.n_csp_avg;
  a.n_lam_avg = (double)sw.n_lambda_avg;
  a.dmin = sw.dlambda_min;
  a.cx = sw.centre[0];
  a.cy = sw.centre[1];
  a.cz = sw.centre[2];
  a.r_precise = sw.r_precise;
  a.zsurf = sw.z_surface_min;
  a.init = sw.initialised ? 0 : 1;
  if (n > 0) {
    const size_t lds = (size_t)kCspWaves * (cap + 3 * kMaxCsp + kMaxCsp * (kMaxCsp - 1) / 2 + kMaxCsp) * 8;
    hipLaunchKernelGGL(k_csp, dim3((n + kCspWaves - 1) / kCspWaves), dim3(64 * kCspWaves), lds, s, sv,
                       pos, nbr, count, cap, sw.n_csp, csp_full, csp);
    hipLaunchKernelGGL(k_switch_detect, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, csp, sw.csp_avg,
                       a, mu0, flag);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = launch_compact(n, flag, src, n_src, scan_tmp, s)) != hipSuccess) return e;
  if ((e = launch_fill_i32(reinterpret_cast<int32_t*>(mu_bits), 0, 2 * (int64_t)n, s)) != hipSuccess) return e;
  if (n > 0) {
    const int blocks = std::min((n + 3) / 4, 65536);
    hipLaunchKernelGGL(k_switch_spread, dim3(blocks), dim3(256), 0, s, sv, pos, cell_of, cell_start,
                       cell_count, cell_atoms, cell_pos, src, n_src, mu0, a, mu_bits);
    hipLaunchKernelGGL(k_switch_finish, dim3((n + 255) / 256), dim3(256), 0, s, n, mu_bits,
                       sw.lambda_avg, a, lambda, flag);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return launch_compact(n, flag, ace_list, n_ace, scan_tmp, s);
}

}  // namespace ap
