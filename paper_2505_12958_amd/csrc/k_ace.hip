// ACE part of the AP force, FP64 path, and the gather that turns per-bond
// gradients into forces.
//
// Per ACE-active atom i (one workgroup, persistent loop over a global atom
// counter):
//   A_nlm = sum_j R_nl(r_ij) Y_lm(u_ij)                    (LDS, 64 bonds at a time)
//   for each coupled rank L:
//     X_L = [AA_{c,M} over coupled channels c | A_{n,L,M} | 1 (L = 0)]
//     Z_L^(p) = C_L^(p) X_L   (folded, symmetric coefficient matrix; sparse rows)
//     phi^(p) += X_L . Z_L^(p) / 2,   dphi^(p)/dA += (dX_L/dA)^T Z_L^(p)
//   E_i = phi1 + sqrt(|phi2| + 1e-6)                  (embedding, FP64)
//   omega = lambda_i (dphi1/dA + sgn(phi2)/(2 sqrt(..)) dphi2/dA)
//   g_ij = sum_nlm omega_nlm d(R_nl Y_lm)/dd_ij        (per bond, stored)
// The folded matrix C_L collects every product-basis function: nu=4 terms
// sit in the channel-channel block, nu=3 in the channel-A block, nu=2 and
// nu=1 against the constant row, so one quadratic form per L gives phi.
#include <algorithm>

#include "ace_basis.h"
#include "ap_internal.h"
#include "geom.h"
#include "scan.h"

namespace ap {

constexpr int kAceThreads = 256;
constexpr int kBondChunk = 64;


// Z^(p) = C^(p) X for both coefficient sets, one folded row per thread with
// all 2L+1 components: each stored coefficient is read once per row and used
// for every component.  The sum over a row runs in storage order.
template <int W>
__device__ __forceinline__ void contract_rows(const int* __restrict__ cptr,
                                              const int* __restrict__ ccol,
                                              const double2* __restrict__ cval, const double* X,
                                              double* Z1, double* Z2, int nr, int tid, double& p1,
                                              double& p2) {
  for (int row = tid; row < nr; row += kAceThreads) {
    double z1[W], z2[W];
#pragma unroll
    for (int M = 0; M < W; ++M) { z1[M] = 0.0; z2[M] = 0.0; }
    const int q1 = cptr[row + 1];
    // unrolled so that several coefficient loads are in flight at once
#pragma unroll 4
    for (int q = cptr[row]; q < q1; ++q) {
      const double2 cv = cval[q];
      const double* xc = X + ccol[q] * W;
#pragma unroll
      for (int M = 0; M < W; ++M) {
        const double x = xc[M];
        z1[M] += cv.x * x;
        z2[M] += cv.y * x;
      }
    }
#pragma unroll
    for (int M = 0; M < W; ++M) {
      Z1[row * W + M] = z1[M];
      Z2[row * W + M] = z2[M];
      p1 += 0.5 * X[row * W + M] * z1[M];
      p2 += 0.5 * X[row * W + M] * z2[M];
    }
  }
}

__global__ __launch_bounds__(kAceThreads) void k_ace_fp64(
    SysView sv, AceDev a, const double* __restrict__ pos, const double4* __restrict__ pos4,
    const int32_t* __restrict__ nbr,
    const int32_t* __restrict__ count, int cap, const double* __restrict__ lambda,
    const int32_t* __restrict__ ace_list, const int32_t* __restrict__ n_ace_p, int n_all,
    int32_t* __restrict__ counter, double* __restrict__ pair_g, double* __restrict__ e_atom,
    double* __restrict__ vir, double* __restrict__ e_raw, int32_t* __restrict__ nbr_ace,
    int vir_acc) {
  extern __shared__ double lds[];
  const int nnl = a.nnl, nlm = a.nlm, nA = a.nA, xs = a.max_xsize;
  double* A = lds;                               // [nA]
  double* om1 = A + nA;                          // [nA]
  double* om2 = om1 + nA;                        // [nA]
  double* red = om2 + nA;                        // [16]
  // the bond staging of the A phase and the rank buffers share one region:
  // the two phases never overlap, so the workgroup's LDS (and with it the
  // number of resident workgroups per CU) is set by the larger of the two
  double* Rs = red + 16;                         // [64][nnl]
  double* Ys = Rs + kBondChunk * nnl;            // [64][nlm]
  double* X = red + 16;                          // [xs]
  double* Z1 = X + xs;                           // [xs]
  double* Z2 = Z1 + xs;                          // [xs]
  __shared__ int s_item;
  const int tid = threadIdx.x;
  const int n = sv.n_atoms;
  const int n_items = ace_list ? *n_ace_p : n_all;
  const int lp1 = a.l_max + 1;

  for (;;) {
    if (tid == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= n_items) break;
    const int i = ace_list ? ace_list[item] : item;
    const double lam = lambda ? lambda[i] : 1.0;
    const int s = sv.sys_of[i];
    const bool ortho = sv.ortho[s] != 0;
    const double* H = sv.H + 9 * s;
    const double* Hi = sv.Hi + 9 * s;
    const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
    const int c = count[i];

    // ---- atomic basis A
    for (int e = tid; e < nA; e += kAceThreads) { A[e] = 0.0; om1[e] = 0.0; om2[e] = 0.0; }
    for (int base = 0; base < c; base += kBondChunk) {
      const int nb = min(kBondChunk, c - base);
      if (tid < nb) {
        const int j = nbr[(int64_t)(base + tid) * n + i];
        nbr_ace[(int64_t)item * cap + base + tid] = j;  // the row again, atom-major, for the force gather
        const double4 pj = pos4[j];
        double dx, dy, dz;
        displacement(ortho, H, Hi, sv.per, xi, yi, zi, pj.x, pj.y, pj.z, dx, dy, dz);
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        double g[kMaxK], dg[kMaxK];
        cheb_basis<double>(a.K, a.rc, r, g, dg);
        for (int nl = 0; nl < nnl; ++nl) {
          double v = 0.0;
          for (int k = 0; k < a.K; ++k) v += a.W[nl * a.K + k] * g[k];
          Rs[tid * nnl + nl] = v;
        }
        double Y[kMaxLM];
        const double ir = 1.0 / r;
        real_ylm<double>(a.l_max, a.ynorm, dx * ir, dy * ir, dz * ir, r, Y, nullptr);
        for (int q = 0; q < nlm; ++q) Ys[tid * nlm + q] = Y[q];
      }
      __syncthreads();
      for (int e = tid; e < nA; e += kAceThreads) {
        const int nn = e / nlm, q = e % nlm;
        int l = 0;
        while ((l + 1) * (l + 1) <= q) ++l;
        const int col = nn * lp1 + l;
        double acc = A[e];
        for (int t = 0; t < nb; ++t) acc += Rs[t * nnl + col] * Ys[t * nlm + q];
        A[e] = acc;
      }
      __syncthreads();
    }

    // ---- folded contraction per coupled rank L
    double p1 = 0.0, p2 = 0.0;
    for (int L = 0; L <= a.L_max; ++L) {
      const int w = 2 * L + 1;
      const int nr = a.nrow[L], nch = a.nch[L];
      const int* xptr = a.xb_ptr + a.xb_off[L];
      for (int e = tid; e < nr * w; e += kAceThreads) {
        const int row = e / w, M = e % w;
        double v;
        if (row < nch) {
          v = 0.0;
#pragma unroll 4
          for (int q = xptr[e]; q < xptr[e + 1]; ++q) {
            const PairTerm u = a.xb_t[q];
            v += u.c * A[u.i] * A[u.j];
          }
        } else if (a.has_arow[L] && row < nch + a.n_max) {
          v = A[(row - nch) * nlm + L * L + M];
        } else {
          v = 1.0;  // constant row (L = 0 only)
        }
        X[e] = v;
      }
      __syncthreads();
      const int* cptr = a.cx_ptr + a.cx_off[L];
      switch (L) {
#define AP_CONTRACT_CASE(LL) \
  case LL: contract_rows<2 * LL + 1>(cptr, a.cx_col, a.cx_val, X, Z1, Z2, nr, tid, p1, p2); break;
        AP_CONTRACT_CASE(0) AP_CONTRACT_CASE(1) AP_CONTRACT_CASE(2) AP_CONTRACT_CASE(3)
        AP_CONTRACT_CASE(4) AP_CONTRACT_CASE(5) AP_CONTRACT_CASE(6) AP_CONTRACT_CASE(7)
        AP_CONTRACT_CASE(8)
#undef AP_CONTRACT_CASE
        default: break;
      }
      __syncthreads();
      const int* aptr = a.ad_ptr + a.ad_off[L];
      for (int t = tid; t < nA; t += kAceThreads) {
        double g1 = om1[t], g2 = om2[t];
#pragma unroll 4
        for (int q = aptr[t]; q < aptr[t + 1]; ++q) {
          const PairTerm u = a.ad_t[q];
          const double f = u.c * A[u.i];
          g1 += f * Z1[u.j];
          g2 += f * Z2[u.j];
        }
        const int q = t % nlm;
        if (a.has_arow[L] && q >= L * L && q < (L + 1) * (L + 1)) {
          const int z = (nch + t / nlm) * w + (q - L * L);
          g1 += Z1[z];
          g2 += Z2[z];
        }
        om1[t] = g1;
        om2[t] = g2;
      }
      __syncthreads();
    }
    p1 = block_sum_f64<kAceThreads / 64>(p1, red);
    p2 = block_sum_f64<kAceThreads / 64>(p2, red + 4);
    const double root = sqrt(fabs(p2) + 1e-6);
    const double E = p1 + root;
    const double sp = (p2 >= 0.0 ? 1.0 : -1.0) / (2.0 * root);
    for (int t = tid; t < nA; t += kAceThreads) om1[t] = lam * (om1[t] + sp * om2[t]);
    __syncthreads();

    // ---- per-bond gradients and the atom's virial
    double w9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int sl = tid; sl < c; sl += kAceThreads) {
      const int j = nbr[(int64_t)sl * n + i];
      const double4 pj = pos4[j];
      double dx, dy, dz;
      displacement(ortho, H, Hi, sv.per, xi, yi, zi, pj.x, pj.y, pj.z, dx, dy, dz);
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double ir = 1.0 / r;
      double g[kMaxK], dg[kMaxK];
      cheb_basis<double>(a.K, a.rc, r, g, dg);
      double ca[kMaxLM], cb[kMaxLM];
      for (int q = 0; q < nlm; ++q) { ca[q] = 0.0; cb[q] = 0.0; }
      for (int nn = 0; nn < a.n_max; ++nn) {
        for (int l = 0; l <= a.l_max; ++l) {
          double R = 0.0, dR = 0.0;
          const double* Wr = a.W + (nn * lp1 + l) * a.K;
          for (int k = 0; k < a.K; ++k) { R += Wr[k] * g[k]; dR += Wr[k] * dg[k]; }
          const double* om = om1 + nn * nlm;
          for (int q = l * l; q < (l + 1) * (l + 1); ++q) {
            ca[q] += om[q] * R;
            cb[q] += om[q] * dR;
          }
        }
      }
      double rad, gx, gy, gz;
      ylm_contract<double>(a.l_max, a.ynorm, dx * ir, dy * ir, dz * ir, r, ca, cb, rad, gx, gy, gz);
      gx += rad * dx * ir;
      gy += rad * dy * ir;
      gz += rad * dz * ir;
      double* o = pair_g + ((int64_t)item * cap + sl) * 3;
      o[0] = gx; o[1] = gy; o[2] = gz;
      w9[0] -= dx * gx; w9[1] -= dx * gy; w9[2] -= dx * gz;
      w9[3] -= dy * gx; w9[4] -= dy * gy; w9[5] -= dy * gz;
      w9[6] -= dz * gx; w9[7] -= dz * gy; w9[8] -= dz * gz;
    }
    for (int k = 0; k < 9; ++k) {
      const double v = block_sum_f64<kAceThreads / 64>(w9[k], red + 8);
      if (tid == 0 && vir) vir[(int64_t)k * n + i] = vir_acc ? vir[(int64_t)k * n + i] + v : v;
    }
    if (tid == 0) {
      e_atom[i] += lam * E;
      if (e_raw) e_raw[i] = E;
    }
    __syncthreads();
  }
}

size_t ace_lds_bytes(const AceDev& a, int precision) {
  (void)precision;
  const size_t shared = std::max((size_t)kBondChunk * (a.nnl + a.nlm), 3 * (size_t)a.max_xsize);
  return sizeof(double) * (3 * (size_t)a.nA + 16 + shared);
}

// Stamps the listed atoms and their neighbours (the atoms the force gather
// visits) for the FP64 path; the mixed path stamps them in its basis pass.
// Stamping inside k_ace_fp64 slowed that kernel by 7 %, so it has a pass of
// its own: one wavefront per listed atom, one lane per slot.
__global__ void k_ace_stamp(int n, const int32_t* __restrict__ nbr, const int32_t* __restrict__ count,
                            const int32_t* __restrict__ ace_list, const int32_t* __restrict__ n_ace,
                            int32_t* __restrict__ halo, int32_t stamp) {
  const int lane = threadIdx.x & 63;
  const int waves = (int)((gridDim.x * (int64_t)blockDim.x) >> 6);
  const int m = ace_list ? *n_ace : n;
  for (int item = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6); item < m;
       item += waves) {
    const int j = ace_list ? ace_list[item] : item;
    const int cj = count[j];
    if (lane == 0) halo[j] = stamp;
    for (int r = lane; r < cj; r += 64) halo[nbr[(int64_t)r * n + j]] = stamp;
  }
}

__global__ void k_ace_rows(int n, const int32_t* __restrict__ ace_list,
                           const int32_t* __restrict__ n_ace, int32_t* __restrict__ row) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = ace_list ? *n_ace : n;
  if (t < m) row[ace_list ? ace_list[t] : t] = t;
}

hipError_t launch_ace_rows(int32_t n_atoms, const int32_t* ace_list, const int32_t* n_ace,
                           int32_t* ace_row, hipStream_t s) {
  hipError_t e = launch_fill_i32(ace_row, -1, n_atoms, s);
  if (e != hipSuccess || n_atoms == 0) return e;
  hipLaunchKernelGGL(k_ace_rows, dim3((n_atoms + 255) / 256), dim3(256), 0, s, n_atoms, ace_list,
                     n_ace, ace_row);
  return hipGetLastError();
}

hipError_t launch_ace_reset(int32_t* counter, hipStream_t s) {
  return launch_fill_i32(counter, 0, 1, s);
}

hipError_t launch_ace(const Ctx& c, const SysView& sv, const double* pos, const double4* pos4,
                      const int32_t* nbr,
                      const int32_t* count, int32_t cap, int32_t n_atoms, const double* lambda,
                      const int32_t* ace_list, const int32_t* n_ace, int32_t* ace_row,
                      int32_t* counter, void* pair_g, double* e_atom, double* vir_atom,
                      double* e_raw, int32_t* nbr_ace, int32_t* halo, int32_t stamp,
                      bool vir_acc, hipStream_t s) {
  (void)ace_row;
  hipError_t e = hipSuccess;
  int dev = 0, n_cu = 256;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t lds = ace_lds_bytes(c.ace, c.precision);
  const int blocks = n_cu * 2;
  if (n_atoms > 0) {
    // enough wavefronts to fill the chip several times over the list
    const int64_t threads = std::min<int64_t>(n_atoms, 65536) * 64;
    hipLaunchKernelGGL(k_ace_stamp, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, n_atoms,
                       nbr, count, ace_list, n_ace, halo, stamp);
  }
  if (lds > 65536) {
    e = hipFuncSetAttribute((const void*)k_ace_fp64, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_ace_fp64, dim3(blocks), dim3(kAceThreads), lds, s, sv, c.ace, pos, pos4, nbr,
                     count, cap, lambda, ace_list, n_ace, n_atoms, counter, (double*)pair_g, e_atom,
                     vir_atom, e_raw, nbr_ace, vir_acc ? 1 : 0);
  return hipGetLastError();
}

// F_k = sum_s g(k, s) - sum_s g(j_s, r_s) over the slots s of k, j_s = nbr(k, s),
// where g(i, s) is the gradient of the ACE energy of listed atom i with
// respect to its bond s and r_s is the slot of k in the row of j_s: read from
// the full reverse index when the list has one (REV), else found by binary
// search of j_s's ascending row in the atom-major copy the ACE kernels wrote
// (nbr_ace, one row of cap entries per listed atom, so a search stays within
// a few cache lines); both give the same value.  kGatherLanes lanes per atom,
// lane l taking the slots s = l (mod kGatherLanes); the lanes' partial sums are
// combined by a fixed butterfly, so the result is the same in every run and
// with or without the reverse index.  Atoms not stamped for this evaluation
// (the ACE kernels stamp every listed atom and its neighbours) have no ACE
// term: zero, or unchanged when accumulating.
constexpr int kGatherLanes = 4;

template <typename G, bool REV>
__global__ __launch_bounds__(256) void k_ace_gather(int n, const int32_t* __restrict__ nbr,
                                                    const int32_t* __restrict__ count,
                                                    const int32_t* __restrict__ rev,
                                                    const int32_t* __restrict__ nbr_ace, int cap,
                                                    const int32_t* __restrict__ row,
                                                    const int32_t* __restrict__ halo, int32_t stamp,
                                                    const G* __restrict__ g,
                                                    double* __restrict__ force, int accumulate) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int k = (int)(t / kGatherLanes);
  const int l = (int)(t % kGatherLanes);
  // whole groups leave together: the butterfly below reads only lanes of its group
  if (k >= n) return;
  if (halo[k] != stamp) {
    if (!accumulate && l == 0) { force[k] = 0.0; force[n + k] = 0.0; force[2 * n + k] = 0.0; }
    return;
  }
  const int rk = row[k];
  const int c = count[k];
  double fx = 0, fy = 0, fz = 0;
  for (int s = l; s < c; s += kGatherLanes) {
    if (rk >= 0) {
      const G* o = g + ((int64_t)rk * cap + s) * 3;
      fx += (double)o[0]; fy += (double)o[1]; fz += (double)o[2];
    }
    const int j = nbr[(int64_t)s * n + k];
    const int rj = row[j];
    if (rj >= 0) {
      int r = -1;
      if constexpr (REV) {
        r = rev[(int64_t)s * n + k];
      } else {
        const int32_t* rowj = nbr_ace + (int64_t)rj * cap;
        int lo = 0, hi = count[j] - 1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int v = rowj[mid];
          if (v == k) { r = mid; break; }
          if (v < k) lo = mid + 1; else hi = mid - 1;
        }
      }
      if (r >= 0) {
        const G* o = g + ((int64_t)rj * cap + r) * 3;
        fx -= (double)o[0]; fy -= (double)o[1]; fz -= (double)o[2];
      }
    }
  }
#pragma unroll
  for (int d = kGatherLanes / 2; d >= 1; d >>= 1) {
    fx += __shfl_xor(fx, d, kGatherLanes);
    fy += __shfl_xor(fy, d, kGatherLanes);
    fz += __shfl_xor(fz, d, kGatherLanes);
  }
  if (l != 0) return;
  if (accumulate) {
    force[k] += fx; force[n + k] += fy; force[2 * n + k] += fz;
  } else {
    force[k] = fx; force[n + k] = fy; force[2 * n + k] = fz;
  }
}

hipError_t launch_ace_gather(const Ctx& c, int32_t n_atoms, const int32_t* nbr, const int32_t* count,
                             const int32_t* rev, const int32_t* nbr_ace, int32_t cap,
                             const int32_t* ace_row, const int32_t* halo, int32_t stamp,
                             const void* pair_g, double* force, bool accumulate, hipStream_t s) {
  if (n_atoms == 0) return hipSuccess;
  const int64_t threads = (int64_t)n_atoms * kGatherLanes;
  const dim3 g((unsigned)((threads + 255) / 256)), b(256);
  const int acc = accumulate ? 1 : 0;
  const bool fp64 = c.precision == AP_PREC_FP64;
  if (fp64 && rev)
    hipLaunchKernelGGL((k_ace_gather<double, true>), g, b, 0, s, n_atoms, nbr, count, rev, nbr_ace,
                       cap, ace_row, halo, stamp, (const double*)pair_g, force, acc);
  else if (fp64)
    hipLaunchKernelGGL((k_ace_gather<double, false>), g, b, 0, s, n_atoms, nbr, count, rev, nbr_ace,
                       cap, ace_row, halo, stamp, (const double*)pair_g, force, acc);
  else if (rev)
    hipLaunchKernelGGL((k_ace_gather<float, true>), g, b, 0, s, n_atoms, nbr, count, rev, nbr_ace,
                       cap, ace_row, halo, stamp, (const float*)pair_g, force, acc);
  else
    hipLaunchKernelGGL((k_ace_gather<float, false>), g, b, 0, s, n_atoms, nbr, count, rev, nbr_ace,
                       cap, ace_row, halo, stamp, (const float*)pair_g, force, acc);
  return hipGetLastError();
}

}  // namespace ap
