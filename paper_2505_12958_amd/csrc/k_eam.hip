// EAM part of the AP force: two gather passes over the full ELL lists, no
// atomics.  Paper, section "EAM potential": E_i = xi(sum_j zeta(r_ij)) +
// 1/2 sum_j Phi(r_ij); with weights w_i = 1 - lambda_i the force on atom k is
// F_k = sum_j [(w_k xi'_k + w_j xi'_j) zeta'(r) + (w_k + w_j) Phi'(r)/2] d_kj/r.
#include "ap_internal.h"
#include "geom.h"

namespace ap {

// coef: the table's (n-1) double4 coefficients, in global memory or staged in LDS
__device__ __forceinline__ void tab_eval(const TableDev& t, const double4* coef, double x,
                                         bool linear_beyond, double& v, double& dv) {
  int k = (int)floor((x - t.x0) * t.inv_dx);
  k = k < 0 ? 0 : (k > t.n - 2 ? t.n - 2 : k);
  const double u = x - (t.x0 + k * t.dx);
  const double4 c = coef[k];
  v = c.x + u * (c.y + u * (c.z + u * c.w));
  dv = c.y + u * (2.0 * c.z + u * 3.0 * c.w);
  const double x_end = t.x0 + (t.n - 1) * t.dx;
  if (x > x_end) {
    if (linear_beyond) {
      const double4 e = coef[t.n - 2];
      const double h = t.dx;
      const double ve = e.x + h * (e.y + h * (e.z + h * e.w));
      const double de = e.y + h * (2.0 * e.z + h * 3.0 * e.w);
      v = ve + de * (x - x_end);
      dv = de;
    } else {
      v = 0.0;
      dv = 0.0;
    }
  }
}

// ---- the paper's W EAM in closed form (appendix "AP potential for tungsten":
// equations eam_F_Marinica, eam_Phi_Marinica, eam_rho_Marinica,
// tungsten_rho_up, tungsten_F_up, tungsten_Phi_up), FP64.
__device__ __forceinline__ void an_knots(const double* a, const double* d, int n, double r, double& v,
                                         double& dv) {
  v = 0.0;
  dv = 0.0;
  for (int i = 0; i < n; ++i) {
    const double t = d[i] - r;
    if (t >= 0.0) {
      const double t2 = t * t;
      v += a[i] * t2 * t;
      dv -= 3.0 * a[i] * t2;
    }
  }
}

// zeta(r) = zeta_0(max(r, r_cut))
__device__ __forceinline__ void an_density(const EamAnalyticDev& p, double r, double& v, double& dv) {
  if (r <= p.r_cut_rho) {
    v = p.zeta_cut;
    dv = 0.0;
  } else {
    an_knots(p.a_rho, p.d_rho, p.n_rho, r, v, dv);
  }
}

// Phi^Fit(r): screened Coulomb below r_lo, quintic bridge up to r_hi, knot sum above
__device__ __forceinline__ void an_pair(const EamAnalyticDev& p, double r, double& v, double& dv) {
  if (r < p.r_lo) {
    const double x = r / p.a_zbl;
    double s = 0.0, ds = 0.0;
    for (int k = 0; k < 4; ++k) {
      const double e = exp(-p.zbl_q[k] * x);
      s += p.zbl_c[k] * e;
      ds -= p.zbl_c[k] * p.zbl_q[k] / p.a_zbl * e;
    }
    v = p.zbl_pref * s / r;
    dv = p.zbl_pref * (ds / r - s / (r * r));
  } else if (r <= p.r_hi) {
    const double* b = p.b_phi;
    v = b[0] + r * (b[1] + r * (b[2] + r * (b[3] + r * (b[4] + r * b[5]))));
    dv = b[1] + r * (2.0 * b[2] + r * (3.0 * b[3] + r * (4.0 * b[4] + r * 5.0 * b[5])));
  } else {
    an_knots(p.a_phi, p.d_phi, p.n_phi, r, v, dv);
  }
}

// xi^Fit(x) = a1 sqrt(x) + a2 x^2 + Delta xi (the square root dropped for x <= 0)
__device__ __forceinline__ void an_embed(const EamAnalyticDev& p, double x, double& v, double& dv) {
  const double s = x > 0.0 ? sqrt(x) : 0.0;
  v = p.a_xi1 * s + p.a_xi2 * x * x + p.d_xi;
  dv = (x > 0.0 ? 0.5 * p.a_xi1 / s : 0.0) + 2.0 * p.a_xi2 * x;
}

// Copies a table's coefficients into LDS (whole workgroup, before any thread
// leaves); returns where the bond loop reads them from.
__device__ __forceinline__ const double4* stage_table(const TableDev& t, double4* lds, bool use) {
  const double4* g = reinterpret_cast<const double4*>(t.c);
  if (!use) return g;
  for (int q = threadIdx.x; q < t.n - 1; q += blockDim.x) lds[q] = g[q];
  return lds;
}

// kOrtho: every system is orthorhombic, so the box edges are hoisted out of
// the bond loop (same arithmetic as the general displacement).  kLds: the
// pair tables are staged in LDS (dynamic shared memory sized by the host).
template <bool kOrtho, bool kLds, bool kAn>
__global__ __launch_bounds__(256) void k_eam_density(SysView sv, TableDev rho_t, TableDev F_t,
                                                     EamAnalyticDev an,
                                                     const double4* __restrict__ pos4,
                                                     const int32_t* __restrict__ nbr,
                                                     const int32_t* __restrict__ count,
                                                     const double* __restrict__ lambda,
                                                     double* __restrict__ wfp,
                                                     double* __restrict__ eF,
                                                     double* __restrict__ wgt) {
  extern __shared__ double4 tab_lds[];
  const double4* rho_c = stage_table(rho_t, tab_lds, kLds);
  if (kLds) __syncthreads();
  const int n = sv.n_atoms;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double w = lambda ? 1.0 - lambda[i] : 1.0;
  wgt[i] = w;
  if (!(w > 0.0)) {
    wfp[i] = 0.0;
    eF[i] = 0.0;
    return;
  }
  const int s = sv.sys_of[i];
  const bool ortho = sv.ortho[s] != 0;
  const double* H = sv.H + 9 * s;
  const double* Hi = sv.Hi + 9 * s;
  const double Lx = H[0], Ly = H[4], Lz = H[8];
  const double4 pi = pos4[i];
  const int c = count[i];
  double rho = 0.0;
#pragma unroll 2
  for (int q = 0; q < c; ++q) {
    const int j = nbr[(int64_t)q * n + i];
    const double4 pj = pos4[j];
    double dx, dy, dz;
    if (kOrtho)
      displacement_ortho(sv.per, Lx, Ly, Lz, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
    else
      displacement(ortho, H, Hi, sv.per, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    double v, dv;
    if constexpr (kAn) an_density(an, r, v, dv);
    else tab_eval(rho_t, rho_c, r, false, v, dv);
    rho += v;
  }
  double Fv, Fp;
  if constexpr (kAn) an_embed(an, rho, Fv, Fp);
  else tab_eval(F_t, reinterpret_cast<const double4*>(F_t.c), rho, true, Fv, Fp);
  wfp[i] = w * Fp;
  eF[i] = Fv;
}

template <bool kOrtho, bool kLds, bool kAn>
__global__ __launch_bounds__(256) void k_eam_force(SysView sv, TableDev rho_t, TableDev phi_t,
                                                   EamAnalyticDev an,
                                                   const double4* __restrict__ pos4,
                                                   const int32_t* __restrict__ nbr,
                                                   const int32_t* __restrict__ count,
                                                   const double* __restrict__ wfp,
                                                   const double* __restrict__ eF,
                                                   const double* __restrict__ wgt,
                                                   double* __restrict__ e_atom,
                                                   double* __restrict__ force,
                                                   double* __restrict__ vir, int accumulate,
                                                   double* __restrict__ e_raw) {
  extern __shared__ double4 tab_lds[];
  const double4* rho_c = stage_table(rho_t, tab_lds, kLds);
  const double4* phi_c = stage_table(phi_t, tab_lds + (rho_t.n - 1), kLds);
  if (kLds) __syncthreads();
  const int n = sv.n_atoms;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int s = sv.sys_of[k];
  const bool ortho = sv.ortho[s] != 0;
  const double* H = sv.H + 9 * s;
  const double* Hi = sv.Hi + 9 * s;
  const double Lx = H[0], Ly = H[4], Lz = H[8];
  const double4 pk = pos4[k];
  const double wk = wgt[k], fk = wfp[k];
  const int c = count[k];
  double fx = 0, fy = 0, fz = 0, ephi = 0;
  // atom k's bond gradients are parallel to the bonds, so its virial
  // -sum_j d (x) G_kj is symmetric: six sums
  double v00 = 0, v01 = 0, v02 = 0, v11 = 0, v12 = 0, v22 = 0;
#pragma unroll 2
  for (int q = 0; q < c; ++q) {
    const int j = nbr[(int64_t)q * n + k];
    const double wj = wgt[j], fj = wfp[j];
    if (wk == 0.0 && wj == 0.0) continue;
    const double4 pj = pos4[j];
    double dx, dy, dz;
    if (kOrtho)
      displacement_ortho(sv.per, Lx, Ly, Lz, pk.x, pk.y, pk.z, pj.x, pj.y, pj.z, dx, dy, dz);
    else
      displacement(ortho, H, Hi, sv.per, pk.x, pk.y, pk.z, pj.x, pj.y, pj.z, dx, dy, dz);
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double ir = 1.0 / r;
    double z, dzr, p, dp;
    if constexpr (kAn) {
      an_density(an, r, z, dzr);
      an_pair(an, r, p, dp);
    } else {
      tab_eval(rho_t, rho_c, r, false, z, dzr);
      tab_eval(phi_t, phi_c, r, false, p, dp);
    }
    const double a = ((fk + fj) * dzr + 0.5 * (wk + wj) * dp) * ir;
    fx += a * dx;
    fy += a * dy;
    fz += a * dz;
    ephi += p;
    // virial of atom k's own bond gradient G_kj = (w_k xi'_k zeta' + w_k Phi'/2) d/r
    const double g = (fk * dzr + 0.5 * wk * dp) * ir;
    const double gx = g * dx, gy = g * dy, gz = g * dz;
    v00 -= dx * gx; v01 -= dx * gy; v02 -= dx * gz;
    v11 -= dy * gy; v12 -= dy * gz;
    v22 -= dz * gz;
  }
  const double e_un = wk > 0.0 ? eF[k] + 0.5 * ephi : 0.0;  // E_k^EAM, unweighted
  const double e = wk > 0.0 ? wk * e_un : 0.0;
  if (e_raw) e_raw[k] = e_un;
  if (accumulate) {
    e_atom[k] += e;
    force[k] += fx;
    force[n + k] += fy;
    force[2 * n + k] += fz;
  } else {
    e_atom[k] = e;
    force[k] = fx;
    force[n + k] = fy;
    force[2 * n + k] = fz;
  }
  if (vir) {
    vir[0 * (int64_t)n + k] = v00; vir[1 * (int64_t)n + k] = v01; vir[2 * (int64_t)n + k] = v02;
    vir[3 * (int64_t)n + k] = v01; vir[4 * (int64_t)n + k] = v11; vir[5 * (int64_t)n + k] = v12;
    vir[6 * (int64_t)n + k] = v02; vir[7 * (int64_t)n + k] = v12; vir[8 * (int64_t)n + k] = v22;
  }
}

hipError_t launch_eam(const Ctx& c, const SysView& sv, const double* pos, const double4* pos4,
                      const int32_t* nbr,
                      const int32_t* count, int32_t n_atoms, const double* lambda, double* wfp,
                      double* eF, double* wgt, double* e_atom, double* force, double* vir_atom,
                      bool accumulate, double* e_raw, hipStream_t s) {
  if (n_atoms == 0) return hipSuccess;
  const dim3 g((n_atoms + 255) / 256), b(256);
  (void)pos;
  // pair tables in LDS when both fit in a quarter of a CU's LDS (four
  // resident workgroups); otherwise they are read through the caches
  const size_t rho_b = c.eam_analytic ? 0 : 32 * (size_t)(c.rho.n - 1);
  const size_t phi_b = c.eam_analytic ? 0 : 32 * (size_t)(c.phi.n - 1);
  const bool lds = !c.eam_analytic && rho_b + phi_b <= 40 * 1024;
  auto go = [&](auto dens, auto frc) {
    hipLaunchKernelGGL(dens, g, b, lds ? rho_b : 0, s, sv, c.rho, c.F, c.ean, pos4, nbr, count, lambda,
                       wfp, eF, wgt);
    hipLaunchKernelGGL(frc, g, b, lds ? rho_b + phi_b : 0, s, sv, c.rho, c.phi, c.ean, pos4, nbr, count,
                       wfp, eF, wgt, e_atom, force, vir_atom, accumulate ? 1 : 0, e_raw);
  };
  if (c.eam_analytic) {
    if (sv.all_ortho) go(k_eam_density<true, false, true>, k_eam_force<true, false, true>);
    else go(k_eam_density<false, false, true>, k_eam_force<false, false, true>);
  } else if (sv.all_ortho) {
    if (lds) go(k_eam_density<true, true, false>, k_eam_force<true, true, false>);
    else go(k_eam_density<true, false, false>, k_eam_force<true, false, false>);
  } else {
    if (lds) go(k_eam_density<false, true, false>, k_eam_force<false, true, false>);
    else go(k_eam_density<false, false, false>, k_eam_force<false, false, false>);
  }
  return hipGetLastError();
}

}  // namespace ap
