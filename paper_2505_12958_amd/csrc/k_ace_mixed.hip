// ACE part of the AP force, mixed-precision path: bond basis (kernel 1),
// embedding and bond gradients (kernel 3) and the launcher of the three
// phases; the rank kernels (phase 1) are in ace_rank.h / k_ace_rank.hip.
#include "ace_basis.h"
#include "ap_internal.h"
#include "geom.h"
#include "scan.h"

namespace ap {

// ---- kernel 1: bond basis and atomic basis A, one wavefront per ACE atom
constexpr int kBasisWaves = 4;

// NM, LM, KK > 0: model shape fixed at compile time (n_max, l_max, K), so
// every loop over radial and angular indices unrolls with constant trip
// counts and the radial weights are read as scalar loads at constant
// offsets; NM = 0: the shape is read from the model at run time.
template <int NM, int LM, int KK>
__global__ __launch_bounds__(64 * kBasisWaves) void k_ace_basis(
    SysView sv, MixDev m, const double* __restrict__ pos, const double4* __restrict__ pos4,
    const int32_t* __restrict__ nbr, const int32_t* __restrict__ count, int cap,
    const int32_t* __restrict__ ace_list,
    const int32_t* __restrict__ n_ace_p, int n_all, float* __restrict__ A_out,
    float* __restrict__ bn_out, int32_t* __restrict__ nbr_ace, int32_t* __restrict__ halo,
    int32_t stamp) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int n_max = NM ? NM : m.n_max, l_max = NM ? LM : m.l_max, K = NM ? KK : m.K;
  const int lp1 = l_max + 1, nlm = lp1 * lp1, nnl = n_max * lp1, nA = n_max * nlm;
  // per bond the Chebyshev values g_k and the harmonics Y_lm go to LDS; the
  // wavefront sums B[k][lm] = sum_j g_k(r_j) Y_lm(u_j) and contracts with the
  // radial weights once per atom: A_nlm = sum_k W_nlk B[k][lm]
  const int nB = K * nlm;
  const int stride = K + nlm;
  float* RY = reinterpret_cast<float*>(lds) + wave * 64 * stride;
  const int n = sv.n_atoms;
  const int n_items = ace_list ? *n_ace_p : n_all;
  const int item = blockIdx.x * kBasisWaves + wave;
  if (item >= n_items) return;  // whole wavefront
  const int a = ace_list ? ace_list[item] : item;
  const int c = count[a];
  const int sy = sv.sys_of[a];
  const float rc = (float)m.rc;
  float acc[(kMaxN * kMaxLM + 63) / 64];
#pragma unroll
  for (int q = 0; q < (kMaxN * kMaxLM + 63) / 64; ++q) acc[q] = 0.f;
  // the atom and its neighbours carry an ACE force term: stamped for the gather
  if (lane == 0) halo[a] = stamp;
  for (int base = 0; base < c; base += 64) {
    const int s = base + lane;
    float* o = RY + lane * stride;
    if (s < c) {
      const int j = nbr[(int64_t)s * n + a];
      nbr_ace[(int64_t)item * cap + s] = j;  // the row again, atom-major, for the force gather
      halo[j] = stamp;
      double dx, dy, dz;
      displacement(sv.ortho[sy] != 0, sv.H + 9 * sy, sv.Hi + 9 * sy, sv.per, pos[a], pos[n + a],
                   pos[2 * n + a], pos4[j].x, pos4[j].y, pos4[j].z, dx, dy, dz);
      const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
      const float r = sqrtf(fx * fx + fy * fy + fz * fz);
      float g[kMaxK], dg[kMaxK];
      cheb_basis<float>(K, rc, r, g, dg);
#pragma unroll
      for (int k = 0; k < kMaxK; ++k)
        if (k < K) o[k] = g[k];
      float Y[kMaxLM];
      const float ir = 1.f / r;
      real_ylm<float>(l_max, m.ynorm, fx * ir, fy * ir, fz * ir, r, Y, nullptr);
#pragma unroll
      for (int q = 0; q < kMaxLM; ++q)
        if (q < nlm) o[K + q] = Y[q];
    } else {
      for (int q = 0; q < stride; ++q) o[q] = 0.f;
    }
    __syncwarp_ap();
    const int nb = min(64, c - base);
#pragma unroll
    for (int r = 0; r < (kMaxN * kMaxLM + 63) / 64; ++r) {
      const int e = lane + 64 * r;
      if (e >= nB) break;
      const int k = e / nlm, lm = e - k * nlm;
      float v = 0.f;
      const float* ga = RY + k;
      const float* ya = RY + K + lm;
#pragma unroll 4
      for (int s2 = 0; s2 < nb; ++s2) v += ga[s2 * stride] * ya[s2 * stride];
      acc[r] += v;
    }
    __syncwarp_ap();
  }
  // B through LDS (the staging area is free now), then A = W B
  float* B = RY;
  float Asq[(kMaxN * kMaxLM + 63) / 64];
#pragma unroll
  for (int r = 0; r < (kMaxN * kMaxLM + 63) / 64; ++r) Asq[r] = 0.f;
#pragma unroll
  for (int r = 0; r < (kMaxN * kMaxLM + 63) / 64; ++r) {
    const int e = lane + 64 * r;
    if (e < nB) B[e] = acc[r];
  }
  __syncwarp_ap();
#pragma unroll
  for (int r = 0; r < (kMaxN * kMaxLM + 63) / 64; ++r) {
    const int e = lane + 64 * r;
    if (e >= nA) continue;
    const int nn = e / nlm, lm = e - nn * nlm;
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    const float* w = m.Wf + (nn * lp1 + l) * K;
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k)
      if (k < K) v += w[k] * B[k * nlm + lm];
    A_out[(int64_t)item * nA + e] = v;
    Asq[r] = v * v;
  }
  // largest |A_(n,l)|^2 over the atom's single indices: it bounds every entry
  // of the coupled operand and fixes the atom's power-of-two scale there
  float* Q = RY + nB;
  __syncwarp_ap();
#pragma unroll
  for (int r = 0; r < (kMaxN * kMaxLM + 63) / 64; ++r) {
    const int e = lane + 64 * r;
    if (e < nA) Q[e] = Asq[r];
  }
  __syncwarp_ap();
  float bq = 0.f;
  if (lane < nnl) {
    const int nn = lane / lp1, l = lane - nn * lp1;
    for (int q = 0; q <= 2 * l; ++q) bq += Q[nn * nlm + l * l + q];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) bq = fmaxf(bq, __shfl_xor(bq, d, 64));
  if (lane == 0) bn_out[item] = bq;
}

// ---- kernel 3: embedding (FP64), bond gradients and virial, one wavefront per atom
template <int NM, int LM, int KK>
__global__ __launch_bounds__(64 * kBasisWaves) void k_ace_grad(
    SysView sv, MixDev m, const double* __restrict__ pos, const double4* __restrict__ pos4,
    const int32_t* __restrict__ nbr, const int32_t* __restrict__ count, int cap,
    const double* __restrict__ lambda,
    const int32_t* __restrict__ ace_list, const int32_t* __restrict__ n_ace_p, int n_all,
    const float* __restrict__ A_in, const float* __restrict__ om_in,
    const float* __restrict__ phi_in, float* __restrict__ pair_g, double* __restrict__ e_atom,
    double* __restrict__ vir, double* __restrict__ e_raw, int vir_acc) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float* om = reinterpret_cast<float*>(lds) + wave * (m.apad + kMaxLM * kMaxK);
  float* Om = om + m.apad;  // [nlm][K]
  const int n = sv.n_atoms;
  const int n_items = ace_list ? *n_ace_p : n_all;
  const int item = blockIdx.x * kBasisWaves + wave;
  if (item >= n_items) return;  // whole wavefront
  const int a = ace_list ? ace_list[item] : item;
  const double lam = lambda ? lambda[a] : 1.0;
  // phi_p = X.Z/2 summed over L.  X rows are homogeneous in A of degree 2
  // (coupled channels), 1 (A rows) and 0 (constant row); by Euler's theorem
  // phi_p = (A . dphi_p/dA + S_A + 2 Z_1)/4 with S_A = A.Z over the A rows and
  // Z_1 the constant row, accumulated in phi_in.
  double d1 = 0.0, d2 = 0.0;
  for (int e = lane; e < m.nA; e += 64) {
    const int64_t o = (int64_t)item * m.nA + e;
    const double av = (double)A_in[o];
    d1 += av * (double)om_in[2 * o];
    d2 += av * (double)om_in[2 * o + 1];
  }
  d1 = wave_sum_f64(d1);
  d2 = wave_sum_f64(d2);
  const double p1 = 0.25 * (d1 + (double)phi_in[2 * (int64_t)item]);
  const double p2 = 0.25 * (d2 + (double)phi_in[2 * (int64_t)item + 1]);
  const double root = sqrt(fabs(p2) + 1e-6);
  const double E = p1 + root;
  const double sp = (p2 >= 0.0 ? 1.0 : -1.0) / (2.0 * root);
  for (int e = lane; e < m.nA; e += 64) {
    const int64_t o = (int64_t)item * m.nA + e;
    om[e] = (float)(lam * ((double)om_in[2 * o] + sp * (double)om_in[2 * o + 1]));
  }
  __syncwarp_ap();
  const int c = count[a];
  const int sy = sv.sys_of[a];
  const int n_max = NM ? NM : m.n_max, l_max = NM ? LM : m.l_max, K = NM ? KK : m.K;
  const int lp1 = l_max + 1, nlm = lp1 * lp1;
  const float rc = (float)m.rc;
  // omega contracted with the radial weights once per atom:
  // Om[lm][k] = sum_n omega_nlm W_nlk, so that for every bond
  // sum_n omega_nlm R_nl = sum_k Om[lm][k] g_k (and likewise with g_k')
  for (int e = lane; e < nlm * K; e += 64) {
    const int q = e / K, k = e - q * K;
    int l = 0;
    while ((l + 1) * (l + 1) <= q) ++l;
    float acc = 0.f;
    for (int nn = 0; nn < n_max; ++nn) acc += om[nn * nlm + q] * m.Wf[(nn * lp1 + l) * K + k];
    Om[e] = acc;
  }
  __syncwarp_ap();
  double w9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int s = lane; s < c; s += 64) {
    const int j = nbr[(int64_t)s * n + a];
    double dx, dy, dz;
    displacement(sv.ortho[sy] != 0, sv.H + 9 * sy, sv.Hi + 9 * sy, sv.per, pos[a], pos[n + a],
                 pos[2 * n + a], pos4[j].x, pos4[j].y, pos4[j].z, dx, dy, dz);
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
    const float r = sqrtf(fx * fx + fy * fy + fz * fz);
    const float ir = 1.f / r;
    float g[kMaxK], dg[kMaxK];
    cheb_basis<float>(K, rc, r, g, dg);
    float ca[kMaxLM], cb[kMaxLM];
#pragma unroll
    for (int q = 0; q < kMaxLM; ++q) {
      ca[q] = 0.f;
      cb[q] = 0.f;
      if (q < nlm) {
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K) {
            const float w = Om[q * K + k];
            ca[q] += w * g[k];
            cb[q] += w * dg[k];
          }
      }
      // compiler barrier: the loads of one row stay with it, so the row's
      // weights are the only ones live at a time
      asm volatile("" ::: "memory");
    }
    float rad, gx, gy, gz;
    ylm_contract<float>(l_max, m.ynorm, fx * ir, fy * ir, fz * ir, r, ca, cb, rad, gx, gy, gz);
    gx += rad * fx * ir;
    gy += rad * fy * ir;
    gz += rad * fz * ir;
    float* o = pair_g + ((int64_t)item * cap + s) * 3;
    o[0] = gx; o[1] = gy; o[2] = gz;
    w9[0] -= dx * gx; w9[1] -= dx * gy; w9[2] -= dx * gz;
    w9[3] -= dy * gx; w9[4] -= dy * gy; w9[5] -= dy * gz;
    w9[6] -= dz * gx; w9[7] -= dz * gy; w9[8] -= dz * gz;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) w9[k] = wave_sum_f64(w9[k]);
  if (lane == 0) {
    if (vir)
      for (int k = 0; k < 9; ++k) {
        double* v = vir + (int64_t)k * n + a;
        *v = vir_acc ? *v + w9[k] : w9[k];
      }
    e_atom[a] += lam * E;
    if (e_raw) e_raw[a] = E;
  }
}

size_t ace_mixed_lds_bytes(const MixDev& m) { return m.big_off + m.big_bytes; }

uint32_t rank_xomask(const MixDev& m) {
  uint32_t x = 0;
  for (int L = 0; L <= m.L_max; ++L)
    if (m.lv[L].xonce) x |= 1u << L;
  return x;
}

hipError_t launch_ace_mixed(const Ctx& c, const SysView& sv, const double* pos, const double4* pos4,
                            const int32_t* nbr,
                            const int32_t* count, int32_t cap, int32_t n_atoms, const double* lambda,
                            const int32_t* ace_list, const int32_t* n_ace, int32_t* counter,
                            float* pair_g, float* A_buf, float* om_buf, float* phi_buf,
                            float* bn_buf, double* e_atom, double* vir_atom, hipStream_t s,
                            int phase, int rank_mode, double* e_raw, int32_t* nbr_ace,
                            int32_t* halo, int32_t stamp, bool vir_acc) {
  const MixDev& m = c.mix;
  // grids are sized for every atom; wavefronts past *n_ace leave at once
  const int blocks = (n_atoms + kBasisWaves - 1) / kBasisWaves;
  if (phase == 0) {
    if (n_atoms == 0) return hipSuccess;
    const size_t lds = (size_t)kBasisWaves * 64 * (m.K + m.nlm) * 4;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * kBasisWaves), lds, s, sv, m, pos, pos4, nbr,
                         count, cap, ace_list, n_ace, n_atoms, A_buf, bn_buf, nbr_ace, halo, stamp);
    };
    if (m.n_max == 8 && m.l_max == 4 && m.K == 8) go(k_ace_basis<8, 4, 8>);
    else if (m.n_max == 6 && m.l_max == 3 && m.K == 6) go(k_ace_basis<6, 3, 6>);
    else go(k_ace_basis<0, 0, 0>);
  } else if (phase == 1) {
    int dev = 0, n_cu = 256;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t lds = ace_mixed_lds_bytes(m);
    const int32_t* na = ace_list ? n_ace : nullptr;
    if (rank_mode != AP_RANK_PER_L) {
      // one persistent launch over all coupled ranks; the work counter was
      // reset on the stream before this phase
      const void* fn = rank_kernel_fused(rank_mode == AP_RANK_FUSED_QUEUE, rank_xomask(m), m.L_max);
      if (!fn) return hipErrorInvalidDeviceFunction;
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      void* args[] = {(void*)&m, (void*)&na, (void*)&n_atoms, (void*)&A_buf, (void*)&om_buf,
                      (void*)&phi_buf, (void*)&bn_buf, (void*)&counter};
      e = hipLaunchKernel(fn, dim3(n_cu), dim3(64 * kMixWaves), args, lds, s);
      if (e != hipSuccess) return e;
      return hipGetLastError();
    }
    for (int L = 0; L <= m.L_max; ++L) {
      const void* fn = nullptr;
      // X_L kept for both sets when it fits beside Z_L (decided with the LDS layout)
      const bool xo = m.lv[L].xonce != 0;
      switch (L) {
        case 0: fn = rank_kernel<0>(xo); break;
        case 1: fn = rank_kernel<1>(xo); break;
        case 2: fn = rank_kernel<2>(xo); break;
        case 3: fn = rank_kernel<3>(xo); break;
        case 4: fn = rank_kernel<4>(xo); break;
        case 5: fn = rank_kernel<5>(xo); break;
        case 6: fn = rank_kernel<6>(xo); break;
        case 7: fn = rank_kernel<7>(xo); break;
        default: fn = rank_kernel<8>(xo); break;
      }
      e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
      void* args[] = {(void*)&m, (void*)&na, (void*)&n_atoms, (void*)&A_buf, (void*)&om_buf,
                      (void*)&phi_buf, (void*)&bn_buf};
      e = hipLaunchKernel(fn, dim3(n_cu), dim3(64 * kMixWaves), args, lds, s);
      if (e != hipSuccess) return e;
    }
  } else {
    if (n_atoms == 0) return hipSuccess;
    const size_t lds = (size_t)kBasisWaves * (m.apad + kMaxLM * kMaxK) * 4;
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * kBasisWaves), lds, s, sv, m, pos, pos4, nbr,
                         count, cap, lambda, ace_list, n_ace, n_atoms, A_buf, om_buf, phi_buf,
                         pair_g, e_atom, vir_atom, e_raw, vir_acc ? 1 : 0);
    };
    if (m.n_max == 8 && m.l_max == 4 && m.K == 8) go(k_ace_grad<8, 4, 8>);
    else if (m.n_max == 6 && m.l_max == 3 && m.K == 6) go(k_ace_grad<6, 3, 6>);
    else go(k_ace_grad<0, 0, 0>);
  }
  return hipGetLastError();
}

}  // namespace ap
