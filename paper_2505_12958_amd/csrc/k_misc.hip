// Switching parameter, ordered compaction and prefix sums, deterministic
// per-system reductions, indenter, velocity-Verlet, finiteness check.
#include "ap_internal.h"
#include "scan.h"

namespace ap {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

// --------------------------------------------------------------------------
// three-pass multi-block exclusive scan of int32 (tile sums, scan of tile
// sums in one block, tile-local scan + offset).  mode 0 writes the prefix
// sums; mode 1 writes, for every i with in[i] != 0, i at out[prefix(i)] and
// the total at *out_n (ordered compaction of a 0/1 flag array).
__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t* __restrict__ in, int n,
                                                            int32_t* __restrict__ sums) {
  __shared__ int ws[kScanThreads / 64];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int t = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = base + k;
    if (i < n) t += in[i];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
  if (lane == 0) ws[w] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) s += ws[k];
    sums[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(1024) void k_scan_sums(int32_t* __restrict__ sums, int nt,
                                                    int32_t* __restrict__ total) {
  // single block, sequential chunks of 1024 with a running carry
  __shared__ int ws[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int b = 0; b < nt; b += 1024) {
    const int i = b + threadIdx.x;
    const int v = i < nt ? sums[i] : 0;
    int incl = wave_incl_scan_i32(v, lane);
    if (lane == 63) ws[w] = incl;
    __syncthreads();
    int off = carry;
    for (int k = 0; k < w; ++k) off += ws[k];
    if (i < nt) sums[i] = off + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = off + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <int MODE>
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t* __restrict__ in, int n,
                                                            const int32_t* __restrict__ offs,
                                                            int32_t* __restrict__ out,
                                                            int32_t* __restrict__ out2) {
  __shared__ int ws[kScanThreads / 64];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int v[kScanItems];
  int t = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = base + k;
    v[k] = i < n ? in[i] : 0;
    t += v[k];
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int incl = wave_incl_scan_i32(t, lane);
  if (lane == 63) ws[w] = incl;
  __syncthreads();
  int off = offs[blockIdx.x];
  for (int k = 0; k < w; ++k) off += ws[k];
  int run = off + incl - t;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int i = base + k;
    if (i < n) {
      if (MODE == 0) {
        out[i] = run;
        if (out2) out2[i] = run;
      } else if (v[k]) {
        out[run] = i;
      }
    }
    run += v[k];
  }
}

static hipError_t scan_impl(const int32_t* in, int32_t n, int32_t* out, int32_t* total,
                            int32_t* tmp, int mode, hipStream_t s, int32_t* out2 = nullptr) {
  const int nt = (n + kScanTile - 1) / kScanTile;
  if (nt == 0) {
    if (total) {
      hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, 0, total);
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tmp, nt, total);
  if (mode == 0)
    hipLaunchKernelGGL(k_tile_scan<0>, dim3(nt), dim3(kScanThreads), 0, s, in, n, tmp, out, out2);
  else
    hipLaunchKernelGGL(k_tile_scan<1>, dim3(nt), dim3(kScanThreads), 0, s, in, n, tmp, out,
                       (int32_t*)nullptr);
  return hipGetLastError();
}

// tmp must hold ceil(n / 4096) + 1 ints; out2 (optional) receives a second
// copy of the scan
hipError_t launch_scan_exclusive(const int32_t* in, int32_t* out, int32_t n, int32_t* tmp,
                                 hipStream_t s, int32_t* out2) {
  return scan_impl(in, n, out, nullptr, tmp, 0, s, out2);
}

hipError_t launch_compact(int32_t n, const int32_t* flag, int32_t* out_list, int32_t* out_n,
                          int32_t* tmp, hipStream_t s) {
  return scan_impl(flag, n, out_list, out_n, tmp, 1, s);
}

__global__ void k_seq(int n, int32_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = i;
}

hipError_t launch_seq(int32_t n, int32_t* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_seq, dim3((n + 255) / 256), dim3(256), 0, s, n, out);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// switching parameter (ACE weight) from the rule
__global__ void k_blend(int n, const double* __restrict__ pos, ap_lambda_rule rule,
                        double* __restrict__ lambda, int32_t* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double lam;
  if (rule.kind == AP_LAMBDA_GIVEN) {
    lam = lambda[i];
  } else if (rule.kind == AP_LAMBDA_CONST) {
    lam = rule.value;
  } else {
    const double x = pos[i] - rule.centre[0];
    const double y = pos[n + i] - rule.centre[1];
    const double z = pos[2 * n + i] - rule.centre[2];
    const double d = sqrt(x * x + y * y + z * z);
    double geo = 0.0;
    if (d <= rule.r_full) {
      geo = 1.0;
    } else if (d < rule.r_full + rule.taper) {
      geo = 0.5 * (1.0 + cos(M_PI * (d - rule.r_full) / rule.taper));
    }
    lam = geo;
    if (rule.kind == AP_LAMBDA_MASK && rule.mask[i]) lam = 1.0;
    if (geo == 0.0 && pos[2 * n + i] >= rule.z_surface_min) lam = 0.0;
  }
  if (rule.kind != AP_LAMBDA_GIVEN) lambda[i] = lam;
  flag[i] = lam > 0.0 ? 1 : 0;
}

hipError_t launch_blend(int32_t n, const double* pos, const ap_lambda_rule& rule, double* lambda,
                        int32_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_blend, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, rule, lambda, flag);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Deterministic per-system sums of m arrays vals[k*stride + i]: one block per
// (chunk of at most kReduceChunk atoms of one system, k) in a fixed
// thread-strided order and fixed tree, then one thread per (system, k) adds
// the chunk partials of its system in chunk order.
__global__ __launch_bounds__(256) void k_reduce_chunks(const int64_t* __restrict__ lo,
                                                       const int64_t* __restrict__ hi,
                                                       const double* __restrict__ vals, int m,
                                                       int64_t stride,
                                                       double* __restrict__ partials) {
  __shared__ double ws[4];
  const int c = blockIdx.x, k = blockIdx.y;  // one workgroup per (chunk, component)
  const int64_t a = lo[c], b = hi[c];
  double t = 0.0;
  for (int64_t i = a + threadIdx.x; i < b; i += 256) t += vals[k * stride + i];
  t = block_sum_f64<4>(t, ws);
  if (threadIdx.x == 0) partials[(int64_t)c * m + k] = t;
}

__global__ void k_reduce_systems(int n_sys, const int32_t* __restrict__ sys_chunk, int m,
                                 const double* __restrict__ partials, double* __restrict__ out,
                                 int accumulate, double* __restrict__ copy0,
                                 double* __restrict__ copy1) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_sys * m) return;
  const int s = t / m, k = t % m;
  double v = 0.0;
  for (int c = sys_chunk[s]; c < sys_chunk[s + 1]; ++c) v += partials[(int64_t)c * m + k];
  const double r = accumulate ? out[t] + v : v;
  out[t] = r;
  if (t == 0 && copy0) *copy0 = r;
  if (t == 1 && copy1) *copy1 = r;
}

hipError_t launch_reduce(const SysView& sv, int32_t n_chunks, const int64_t* chunk_lo,
                         const int64_t* chunk_hi, const int32_t* sys_chunk, const double* vals,
                         int32_t m, int64_t stride, double* partials, double* out, bool accumulate,
                         hipStream_t s, double* copy0, double* copy1) {
  if (n_chunks > 0)
    hipLaunchKernelGGL(k_reduce_chunks, dim3(n_chunks, m), dim3(256), 0, s, chunk_lo, chunk_hi,
                       vals, m, stride, partials);
  const int nt = sv.n_sys * m;
  hipLaunchKernelGGL(k_reduce_systems, dim3((nt + 255) / 256), dim3(256), 0, s, sv.n_sys,
                     sys_chunk, m, partials, out, accumulate ? 1 : 0, copy0, copy1);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// indenter: per-atom energy and load into e2[i], e2[n + i] (reduced later)
__global__ void k_indenter(int n, const double* __restrict__ pos, const uint8_t* __restrict__ fixed,
                           double cx, double cy, double cz, double R, double K, double ux,
                           double uy, double uz, double* __restrict__ force,
                           double* __restrict__ e2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e = 0.0, ld = 0.0;
  if (!(fixed && fixed[i])) {
    const double x = pos[i] - cx, y = pos[n + i] - cy, z = pos[2 * n + i] - cz;
    const double d = sqrt(x * x + y * y + z * z);
    if (d < R) {
      const double p = R - d;
      e = K / 3.0 * p * p * p;
      const double f = K * p * p / d;
      force[i] += f * x;
      force[n + i] += f * y;
      force[2 * n + i] += f * z;
      ld = f * x * ux + f * y * uy + f * z * uz;
    }
  }
  if (e2) {
    e2[i] = e;
    e2[n + i] = ld;
  }
}

hipError_t launch_indenter(int32_t n, const double* pos, const uint8_t* fixed, const double* c,
                           double R, double K, const double* dir, double* force, double* e2,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_indenter, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, fixed, c[0], c[1],
                     c[2], R, K, dir[0], dir[1], dir[2], force, e2);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// velocity Verlet: half kick, optional drift with periodic wrap
constexpr double kAcc = 9.648533212e-3;  // (eV/A/amu) -> A/fs^2
constexpr double kKb = 8.617333262e-5;   // Boltzmann constant, eV/K

__global__ void k_kick_drift(int n, SysView sv, double* __restrict__ pos, double* __restrict__ vel,
                             const double* __restrict__ force, const double* __restrict__ mass,
                             const uint8_t* __restrict__ fixed, const uint8_t* __restrict__ nvt,
                             const double* __restrict__ nvt_fac, double dt, int drift) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (fixed && fixed[i]) {
    vel[i] = 0.0;
    vel[n + i] = 0.0;
    vel[2 * n + i] = 0.0;
    return;
  }
  const double a = 0.5 * dt * kAcc / mass[i];
  const int s = sv.sys_of[i];
  const double* H = sv.H + 9 * s;
  // thermostat scaling of the layer's velocities, applied before the kick
  const double f = (nvt_fac && nvt[i]) ? nvt_fac[s] : 1.0;
  for (int k = 0; k < 3; ++k) {
    double v = f * vel[k * n + i] + a * force[k * n + i];
    vel[k * n + i] = v;
    if (drift) {
      double x = pos[k * n + i] + dt * v;
      if (sv.per[k] && sv.ortho[s]) {
        const double L = H[4 * k];
        x = x >= L ? x - L : (x < 0.0 ? x + L : x);
      }
      pos[k * n + i] = x;
    }
  }
}

hipError_t launch_kick_drift(int32_t n, const SysView& sv, double* pos, double* vel,
                             const double* force, const double* mass, const uint8_t* fixed,
                             const uint8_t* nvt, const double* nvt_fac, double dt, bool drift,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_kick_drift, dim3((n + 255) / 256), dim3(256), 0, s, n, sv, pos, vel, force,
                     mass, fixed, nvt, nvt_fac, dt, drift ? 1 : 0);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Nose-Hoover layer (section "Nanoindentation": the NVT region between the
// fixed bottom and the NVE top).  Per system s: xi_s, its integral eta_s, and
// dv/dt = F/m - xi_s v on the layer's atoms with dxi/dt = (T/T0 - 1)/tau^2.

// out[i] = m v^2 of a (non-fixed) layer atom, out[n + i] = 1 for it; zero
// elsewhere (reduced per system in a fixed order).
__global__ void k_nvt_ke(int n, const double* __restrict__ vel, const double* __restrict__ mass,
                         const uint8_t* __restrict__ nvt, const uint8_t* __restrict__ fixed,
                         double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool on = nvt[i] && !(fixed && fixed[i]);
  const double vx = vel[i], vy = vel[n + i], vz = vel[2 * n + i];
  out[i] = on ? mass[i] * (vx * vx + vy * vy + vz * vz) : 0.0;
  out[n + i] = on ? 1.0 : 0.0;
}

// Half a thermostat step per system: xi += dt/4 G(T), eta += xi dt/2,
// f = exp(-xi dt/2), T *= f^2, xi += dt/4 G(T).  sums[2s] holds the layer's
// sum of m v^2 (updated to the scaled value), sums[2s + 1] its atom count.
__global__ void k_nvt_half(int n_sys, double* __restrict__ sums, double* __restrict__ xi,
                           double* __restrict__ fac, double T0, double tau, double dt) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  const double cnt = sums[2 * s + 1];
  if (!(cnt > 0.0)) {
    fac[s] = 1.0;
    return;
  }
  const double gkt = 3.0 * cnt * kKb * T0;       // g k_B T0, eV
  const double c = 0.25 * dt / (tau * tau);
  double twok = sums[2 * s] / kAcc;              // 2K, eV
  double x = xi[2 * s];
  x += c * (twok / gkt - 1.0);
  const double eta = xi[2 * s + 1] + 0.5 * dt * x;
  const double f = exp(-0.5 * dt * x);
  twok *= f * f;
  x += c * (twok / gkt - 1.0);
  xi[2 * s] = x;
  xi[2 * s + 1] = eta;
  fac[s] = f;
  sums[2 * s] = twok * kAcc;
}

__global__ void k_nvt_scale(int n, const int32_t* __restrict__ sys_of, double* __restrict__ vel,
                            const uint8_t* __restrict__ nvt, const uint8_t* __restrict__ fixed,
                            const double* __restrict__ fac) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !nvt[i] || (fixed && fixed[i])) return;
  const double f = fac[sys_of[i]];
  vel[i] *= f;
  vel[n + i] *= f;
  vel[2 * n + i] *= f;
}

hipError_t launch_nvt_ke(int32_t n, const double* vel, const double* mass, const uint8_t* nvt,
                         const uint8_t* fixed, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nvt_ke, dim3((n + 255) / 256), dim3(256), 0, s, n, vel, mass, nvt, fixed, out);
  return hipGetLastError();
}

hipError_t launch_nvt_half(int32_t n_sys, double* sums, double* xi, double* fac, double T0,
                           double tau, double dt, hipStream_t s) {
  hipLaunchKernelGGL(k_nvt_half, dim3((n_sys + 63) / 64), dim3(64), 0, s, n_sys, sums, xi, fac, T0,
                     tau, dt);
  return hipGetLastError();
}

hipError_t launch_nvt_scale(int32_t n, const SysView& sv, double* vel, const uint8_t* nvt,
                            const uint8_t* fixed, const double* fac, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_nvt_scale, dim3((n + 255) / 256), dim3(256), 0, s, n, sv.sys_of, vel, nvt,
                     fixed, fac);
  return hipGetLastError();
}

// Force of a position-dependent geometric switching parameter: atoms of the
// cosine band (0 < lambda < 1 under rule kinds 1-3; masked and surface atoms
// have lambda 0 or 1) get -(E^ACE - E^EAM) d lambda/d r, and their virial
// -(r - centre) (x) (E^ACE - E^EAM) d lambda/d r (nine per-atom entries,
// zero elsewhere, for the deterministic per-system reduction).
__global__ void k_lambda_grad(int n, const double* __restrict__ pos, ap_lambda_rule rule,
                              const double* __restrict__ lambda, const double* __restrict__ e_ace,
                              const double* __restrict__ e_eam, double* __restrict__ force,
                              double* __restrict__ vir) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lam = lambda[i];
  const bool geo = rule.kind == AP_LAMBDA_SPHERE || rule.kind == AP_LAMBDA_HEMISPHERE ||
                   rule.kind == AP_LAMBDA_MASK;
  double d3[3] = {0.0, 0.0, 0.0}, g[3] = {0.0, 0.0, 0.0};
  if (geo && lam > 0.0 && lam < 1.0) {
    for (int k = 0; k < 3; ++k) d3[k] = pos[(int64_t)k * n + i] - rule.centre[k];
    const double d = sqrt(d3[0] * d3[0] + d3[1] * d3[1] + d3[2] * d3[2]);
    const double dl = -0.5 * M_PI / rule.taper * sin(M_PI * (d - rule.r_full) / rule.taper);
    const double c = (e_ace[i] - e_eam[i]) * dl / d;
    for (int k = 0; k < 3; ++k) {
      g[k] = c * d3[k];
      force[(int64_t)k * n + i] -= g[k];
    }
  }
  if (vir)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) vir[(int64_t)(3 * a + b) * n + i] = -d3[a] * g[b];
}

hipError_t launch_lambda_grad(int32_t n, const double* pos, const ap_lambda_rule& rule,
                              const double* lambda, const double* e_ace, const double* e_eam,
                              double* force, double* vir_atom, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lambda_grad, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, rule, lambda,
                     e_ace, e_eam, force, vir_atom);
  return hipGetLastError();
}

__global__ void k_check_finite(int n, const double* __restrict__ f, int32_t* __restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = f[i], b = f[n + i], c = f[2 * n + i];
  if (!(isfinite(a) && isfinite(b) && isfinite(c))) atomicOr(flag, 1);
}

hipError_t launch_check_finite(int32_t n, const double* force, int32_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_finite, dim3((n + 255) / 256), dim3(256), 0, s, n, force, flag);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// positions as one 32-byte record per atom: a neighbour's position is one
// gathered load instead of three
__global__ void k_pack_pos(int n, const double* __restrict__ pos, double4* __restrict__ p4) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p4[i] = make_double4(pos[i], pos[n + i], pos[2 * n + i], 0.0);
}

hipError_t launch_pack_pos(int32_t n, const double* pos, double4* p4, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_pos, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, p4);
  return hipGetLastError();
}

}  // namespace ap
