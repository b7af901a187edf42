// Rank kernels of the mixed-precision ACE path (coupling, folded
// contraction and adjoint per coupled rank L), shared by the translation
// units k_ace_rank.hip (one per L).
//
// ACE part of the AP force, mixed-precision path.
//
// One workgroup (512 threads, 8 wavefronts, two per SIMD) evaluates tiles of 8 ACE-active
// atoms (persistent loop, tiles assigned round-robin: every tile costs the same), on chip:
//
//  1. bond basis in FP32 from the FP64 minimum-image displacement; the
//     atomic basis A_nlm of the 8 atoms is accumulated in LDS;
//  2. per coupled rank L:
//     a. coupling X_L = [AA_{c,M} | A_{n,L,M} | 1] for the 8 atoms (VALU;
//        one lane per (channel, atom), channels grouped by (l_a, l_b) so the
//        Clebsch-Gordan entries are wavefront-uniform), scaled per atom by a
//        power of two and written to LDS as an fp16 hi/lo split (x = hi + lo
//        to ~22 bits);
//     b. folded contraction Z_L = C_L X_L for both coefficient sets with
//        v_mfma_f32_16x16x32_f16: the 16x32 tiles of C_L are stored dense,
//        each row scaled by a power of two and pre-split into fp16 hi/lo;
//        each product is taken as hi*hi + hi*lo + lo*hi with FP32
//        accumulation and the two scales are undone exactly on the result;
//     c. Z_L of each set goes to LDS (over the dead X_L) and the adjoint
//        dphi/dA = (dX_L/dA)^T Z_L is formed per (channel, atom) and added
//        to the atom's gradient; phi itself follows from Euler's theorem
//        for homogeneous functions (see the end of the tile loop);
//  3. embedding E = phi1 + sqrt(|phi2| + 1e-6) and its derivative in FP64;
//  4. per-bond gradients g_ij (FP32) and the atom's virial (FP64 sums).
#pragma once

#include "ace_basis.h"
#include "ap_internal.h"
#include "geom.h"
#include "scan.h"

#include <utility>

namespace ap {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMT = 8;
constexpr int kMWaves = kMixWaves;
constexpr int kMThreads = 64 * kMWaves;

__device__ __forceinline__ f16x8 as_f16x8(uint4 v) { return __builtin_bit_cast(f16x8, v); }

// Values the compiler cannot prove uniform (loads next to stores) are made
// wavefront-uniform explicitly so they live in scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Read-only model tables are read through the constant address space, so
// wavefront-uniform indices become scalar loads (the kernel never writes them).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> as_const(const T* p) { return (cptr<T>)p; }

__device__ __forceinline__ MixL load_level(const MixL* p) {
  static_assert(sizeof(MixL) == 15 * sizeof(int32_t), "MixL is 15 int32 fields");
  cptr<int32_t> q = as_const(reinterpret_cast<const int32_t*>(p));
  MixL P;
  P.nrow = uni(q[0]); P.nrow16 = uni(q[1]); P.nch = uni(q[2]); P.arow = uni(q[3]);
  P.rt = uni(q[4]); P.ct = uni(q[5]); P.kt = uni(q[6]); P.kstr = uni(q[7]); P.zstr = uni(q[8]);
  P.grp0 = uni(q[9]); P.ngrp = uni(q[10]); P.bt0 = uni(q[11]); P.xonce = uni(q[12]);
  P.zoff = uni(q[13]); P.rs0 = uni(q[14]);
  return P;
}

// The same fields from the copy the fused kernel stages in LDS (kLevelInts
// int32 per rank): LDS reads are not hoisted across the tile loop's LDS
// stores, so the parameters of all ranks are never held in registers at once.
__device__ __forceinline__ MixL load_level_lds(const int32_t* q) {
  MixL P;
  P.nrow = uni(q[0]); P.nrow16 = uni(q[1]); P.nch = uni(q[2]); P.arow = uni(q[3]);
  P.rt = uni(q[4]); P.ct = uni(q[5]); P.kt = uni(q[6]); P.kstr = uni(q[7]); P.zstr = uni(q[8]);
  P.grp0 = uni(q[9]); P.ngrp = uni(q[10]); P.bt0 = uni(q[11]); P.xonce = uni(q[12]);
  P.zoff = uni(q[13]); P.rs0 = uni(q[14]);
  return P;
}

__device__ __forceinline__ CgEnt load_ent(const CgEnt* p) {
  const int2 raw = *reinterpret_cast<const int2*>(p);
  const int w0 = uni(raw.x);
  CgEnt e;
  e.m1 = (int8_t)(w0 & 0xff);
  e.m2 = (int8_t)((w0 >> 8) & 0xff);
  e.M = (int8_t)((w0 >> 16) & 0xff);
  e.pad = 0;
  e.c = __int_as_float(uni(raw.y));
  return e;
}

// x (already scaled so that |x| < 2^13) as hi + lo in fp16: hi is x rounded
// to 11 significant bits, lo the exact fp32 residual x - hi rounded again
__device__ __forceinline__ void split_f16(float x, _Float16& hi, _Float16& lo) {
  hi = (_Float16)x;
  lo = (_Float16)(x - (float)hi);
}

// Power-of-two scale of an atom's entries of X_L.  With B2 the largest
// squared norm |A_(n,l)|^2 over the atom's single indices, every coupled
// entry obeys |AA_{c,M}| <= |A_a| |A_b| <= B2 (the real coupling
// coefficients of one rank are orthonormal over (m1, m2)), every A row
// |A_{n,L,M}| <= sqrt(B2), and L = 0 holds the constant 1.  The scale puts
// the bound just below 2^13: fp16 keeps its full 11 bits in hi and in lo for
// all but negligibly small entries, and no product can overflow.
__device__ __forceinline__ int xscale_exp(float b2, int L) {
  float bound = fmaxf(b2, sqrtf(b2));
  if (L == 0) bound = fmaxf(bound, 1.f);
  int ex = 0;
  (void)frexpf(bound, &ex);
  return 13 - ex;
}

// GEMM of one L for N owned row tiles (rt = wave + kMWaves i, i < N): N and
// CTN are compile-time, so the k loop has no branches and the coefficient
// loads of the next k tile stay in flight under this tile's MFMAs.  X is read
// from LDS (column-major, k contiguous); the coefficient tiles stream from L2.
template <int N, int RTW, int CTN>
__device__ __forceinline__ void gemm_owned(const MixL& P, const uint4* base, const _Float16* xh,
                                           const _Float16* xl, f32x4 (&acc)[RTW][CTN], int lane) {
  static_assert(N >= 1 && N <= RTW, "owned row tiles");
  const uint4* tp[N];
#pragma unroll
  for (int i = 0; i < N; ++i) tp[i] = base + (size_t)2 * 64 * kMWaves * i * P.kt;
  const int col_l = lane & 15;
  const int k_l = 8 * (lane >> 4);
  // two register buffers of coefficient tiles (hi, lo), ping-pong: the tiles
  // of k tile kt + 1 load while those of kt feed the MFMAs
  uint4 ah[N], al[N], bh[N], bl[N];
  auto load = [&](uint4 (&h)[N], uint4 (&l)[N], int kt) {
    const int k = min(kt, P.kt - 1);  // past the end: reload the last tile (harmless)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      h[i] = tp[i][128 * k];
      l[i] = tp[i][128 * k + 64];
    }
    // compiler barrier: keep the loads here, ahead of their use
    asm volatile("" ::: "memory");
  };
  auto compute = [&](const uint4 (&h)[N], const uint4 (&l)[N], int kt) {
#pragma unroll
    for (int c = 0; c < CTN; ++c) {
      const int off = (c * 16 + col_l) * P.kstr + kt * 32 + k_l;
      const f16x8 xbh = as_f16x8(*reinterpret_cast<const uint4*>(xh + off));
      const f16x8 xbl = as_f16x8(*reinterpret_cast<const uint4*>(xl + off));
      // the three split products, interleaved over independent accumulators
#pragma unroll
      for (int sp = 0; sp < 3; ++sp) {
#pragma unroll
        for (int i = 0; i < N; ++i) {
          const f16x8 a = as_f16x8(sp == 2 ? l[i] : h[i]);
          acc[i][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, sp == 1 ? xbl : xbh, acc[i][c], 0, 0, 0);
        }
      }
    }
  };
  load(ah, al, 0);
  for (int kt = 0; kt < P.kt; kt += 2) {
    load(bh, bl, kt + 1);
    compute(ah, al, kt);
    if (kt + 1 < P.kt) {
      load(ah, al, kt + 2);
      compute(bh, bl, kt + 1);
    }
  }
}

// GEMM of one L: accumulators of the wavefront's row tiles for all column tiles.
template <int RTW, int CTN>
__device__ __forceinline__ void gemm_tiles(const MixDev& m, const MixL& P, const _Float16* xh,
                                           const _Float16* xl, f32x4 (&acc)[RTW][CTN], int wave,
                                           int lane, int p) {
  const int rt_set = P.nrow16 / 16;
#pragma unroll
  for (int i = 0; i < RTW; ++i)
#pragma unroll
    for (int c = 0; c < CTN; ++c) acc[i][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nown = uni(min(RTW, max(0, (rt_set - wave + kMWaves - 1) / kMWaves)));
  const uint4* base = m.ctile + (size_t)2 * 64 * ((size_t)P.bt0 + (size_t)(p * rt_set + wave) * P.kt) + lane;
  if (nown == 1) gemm_owned<1, RTW, CTN>(P, base, xh, xl, acc, lane);
  if constexpr (RTW >= 2)
    if (nown == 2) gemm_owned<(RTW >= 2 ? 2 : 1), RTW, CTN>(P, base, xh, xl, acc, lane);
  if constexpr (RTW >= 3)
    if (nown == 3) gemm_owned<(RTW >= 3 ? 3 : 1), RTW, CTN>(P, base, xh, xl, acc, lane);
}

// Write the accumulators of coefficient set p (rows [p*nrow16, (p+1)*nrow16))
// as FP32 Z[row][col] into LDS, undoing the row scale of the coefficients
// (staged in LDS with the rank's tables, so that no per-lane load of them can
// be hoisted out of the tile loop and held in registers) and the column
// (atom) scale of X_L; both are powers of two, so this is exact.
template <int RTW, int CTN>
__device__ __forceinline__ void store_z(const MixL& P, const f32x4 (&acc)[RTW][CTN], float* Z,
                                        const float* bn2, const float* rs_lds, int L, int p, int wave,
                                        int lane, int ncols) {
  const int col_l = lane & 15;
  const int r_l = 4 * (lane >> 4);
  const int w = 2 * L + 1;
  const float* rs = rs_lds + p * P.nrow16;
  int cex[CTN];
#pragma unroll
  for (int c = 0; c < CTN; ++c) {
    const int col = c * 16 + col_l;
    cex[c] = col < ncols ? -xscale_exp(bn2[col / w], L) : 0;
  }
#pragma unroll
  for (int i = 0; i < RTW; ++i) {
    const int rt = wave + kMWaves * i;
    if (rt >= P.nrow16 / 16) continue;
    const int row0 = rt * 16 + r_l;
    float rinv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) rinv[q] = rs[row0 + q];
#pragma unroll
    for (int c = 0; c < CTN; ++c) {
      const int col = c * 16 + col_l;
      if (col >= ncols) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + q;
        if (row >= 0 && row < P.nrow) Z[row * P.zstr + col] = ldexpf(acc[i][c][q] * rinv[q], cex[c]);
      }
    }
  }
}

// Selection rule of the real coupling coefficients C^{la lb L}_{m1 m2 M}
// (l_a + l_b + L even): the M-type (cosine for M >= 0, sine for M < 0) is the
// product of the m1- and m2-types and |M| is |m1| + |m2| or ||m1| - |m2||.
// Every non-zero entry satisfies it; the library's coefficient table holds
// one value per entry of this superset, in (m1, m2, M) order.
__device__ constexpr int iabs_c(int v) { return v < 0 ? -v : v; }
__device__ constexpr bool cg_rule(int m1, int m2, int M) {
  return ((M < 0) == ((m1 < 0) != (m2 < 0))) &&
         (iabs_c(M) == iabs_c(m1) + iabs_c(m2) || iabs_c(M) == iabs_c(iabs_c(m1) - iabs_c(m2)));
}

// ---- coupling coefficients as compile-time constants
// Complex <j1 m1 j2 m2 | J M> from Racah's closed form and the change of
// basis to the real harmonics (real Y_m = sum_mu U_{m mu} Y^mu with
// U_{0,0} = 1; m > 0: U_{m,m} = (-1)^m/sqrt2, U_{m,-m} = 1/sqrt2; m < 0, k = |m|:
// U_{m,k} = -i(-1)^k/sqrt2, U_{m,-k} = i/sqrt2), evaluated by the compiler.
constexpr double ce_fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}
constexpr double ce_sqrt(double x) {
  if (x <= 0.0) return 0.0;
  double r = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 200; ++i) {
    const double n = 0.5 * (r + x / r);
    if (n == r) break;
    r = n;
  }
  return r;
}
constexpr double ce_cg(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || iabs_c(m1) > j1 || iabs_c(m2) > j2 || iabs_c(M) > J) return 0.0;
  if (J < iabs_c(j1 - j2) || J > j1 + j2) return 0.0;
  const double pre = (2 * J + 1) * ce_fact(J + j1 - j2) * ce_fact(J - j1 + j2) * ce_fact(j1 + j2 - J) /
                     ce_fact(j1 + j2 + J + 1) * ce_fact(J + M) * ce_fact(J - M) * ce_fact(j1 - m1) *
                     ce_fact(j1 + m1) * ce_fact(j2 - m2) * ce_fact(j2 + m2);
  double sum = 0.0;
  for (int k = 0; k <= j1 + j2 - J; ++k) {
    const int a0 = k, a1 = j1 + j2 - J - k, a2 = j1 - m1 - k, a3 = j2 + m2 - k, a4 = J - j2 + m1 + k,
              a5 = J - j1 - m2 + k;
    if (a0 < 0 || a1 < 0 || a2 < 0 || a3 < 0 || a4 < 0 || a5 < 0) continue;
    const double den = ce_fact(a0) * ce_fact(a1) * ce_fact(a2) * ce_fact(a3) * ce_fact(a4) * ce_fact(a5);
    sum += ((k & 1) ? -1.0 : 1.0) / den;
  }
  return ce_sqrt(pre) * sum;
}
// U_{m, mu} as (re, im); zero unless mu = +-m
struct ce_c2 { double re, im; };
constexpr ce_c2 ce_u(int m, int mu) {
  const double s = 0.70710678118654752440;
  if (m == 0) return mu == 0 ? ce_c2{1.0, 0.0} : ce_c2{0.0, 0.0};
  if (m > 0) {
    if (mu == m) return ce_c2{(m & 1) ? -s : s, 0.0};
    if (mu == -m) return ce_c2{s, 0.0};
    return ce_c2{0.0, 0.0};
  }
  const int k = -m;
  if (mu == k) return ce_c2{0.0, (k & 1) ? s : -s};
  if (mu == -k) return ce_c2{0.0, s};
  return ce_c2{0.0, 0.0};
}
constexpr ce_c2 ce_mul(ce_c2 a, ce_c2 b) { return ce_c2{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
constexpr ce_c2 ce_conj(ce_c2 a) { return ce_c2{a.re, -a.im}; }
// real coupling coefficient C^{l1 l2 L}_{m1 m2 M}
constexpr double ce_real_cg(int l1, int l2, int L, int m1, int m2, int M) {
  double acc = 0.0;
  const int mu1s[2] = {iabs_c(m1), -iabs_c(m1)};
  const int mu2s[2] = {iabs_c(m2), -iabs_c(m2)};
  for (int a = 0; a < (m1 == 0 ? 1 : 2); ++a)
    for (int b = 0; b < (m2 == 0 ? 1 : 2); ++b) {
      const int mu1 = mu1s[a], mu2 = mu2s[b], mu = mu1 + mu2;
      if (iabs_c(mu) > L) continue;
      const ce_c2 u = ce_mul(ce_mul(ce_u(M, mu), ce_conj(ce_u(m1, mu1))), ce_conj(ce_u(m2, mu2)));
      acc += u.re * ce_cg(l1, mu1, l2, mu2, L, mu);
    }
  return acc;
}

// one entry of the coupling of (LA, m1 index I1) with (LB, m2 index I2) to
// (L, M index Q), flat index E = (I1 * (2LB+1) + I2) * (2L+1) + Q
template <int LA, int LB, int L, int E>
__device__ __forceinline__ void xb_entry(const float* Aa, const float* Ab, float* X) {
  constexpr int q = E % (2 * L + 1), i2 = (E / (2 * L + 1)) % (2 * LB + 1),
                i1 = E / ((2 * L + 1) * (2 * LB + 1));
  if constexpr (cg_rule(i1 - LA, i2 - LB, q - L)) {
    constexpr float c = (float)ce_real_cg(LA, LB, L, i1 - LA, i2 - LB, q - L);
    if constexpr (c != 0.0f) X[q] = fmaf(c * Aa[i1], Ab[i2], X[q]);
  }
}
template <int LA, int LB, int L, int... E>
__device__ __forceinline__ void xb_all(std::integer_sequence<int, E...>, const float* Aa,
                                       const float* Ab, float* X) {
  (xb_entry<LA, LB, L, E>(Aa, Ab, X), ...);
}

// One group of X_L: lane = (member j = lane/8, atom t = lane%8), all members
// coupling (n, LA) with (n', LB) to rank L.  Register indices and coupling
// coefficients are compile-time constants.
template <int LA, int LB, int L>
__device__ __forceinline__ void xbuild_group(const float* At, int4 mem, _Float16* xh, _Float16* xl,
                                             int kstr, int t, int sx) {
  float Aa[2 * LA + 1], Ab[2 * LB + 1], X[2 * L + 1];
#pragma unroll
  for (int q = 0; q <= 2 * LA; ++q) Aa[q] = At[mem.y + q];
#pragma unroll
  for (int q = 0; q <= 2 * LB; ++q) Ab[q] = At[mem.z + q];
#pragma unroll
  for (int q = 0; q <= 2 * L; ++q) X[q] = 0.f;
  xb_all<LA, LB, L>(std::make_integer_sequence<int, (2 * LA + 1) * (2 * LB + 1) * (2 * L + 1)>{}, Aa,
                    Ab, X);
  const int col0 = t * (2 * L + 1);
#pragma unroll
  for (int q = 0; q <= 2 * L; ++q) {
    _Float16 hi, lo;
    split_f16(ldexpf(X[q], sx), hi, lo);
    xh[(col0 + q) * kstr + mem.x] = hi;
    xl[(col0 + q) * kstr + mem.x] = lo;
  }
}

// Adjoint of one coupled pattern (LT, LP, L) for the components [I0, I1) of
// the target: lane = (target n = lane/8, atom t = lane%8), target index
// a = (n, LT), partners (n', LP) for every n'.  Every coupled channel {a, p}
// of this L is visited from both of its indices (the coupled value is
// symmetric in them), so the lane owns its sums.  The partner sum is taken
// first, W[m2][M] = sum_n' f A_(n',LP,m2) Z_({a,p},M), so the coupling
// coefficients enter once per target instead of once per partner:
// dphi/dA_(a,m1) += sum_(m2,M) C^{LT LP L}_{m1 m2 M} W[m2][M].
template <int LT, int LP, int L, int I0, int I1, int E>
__device__ __forceinline__ void adw_entry(const float* Wv, float* ga) {
  constexpr int w = 2 * L + 1;
  constexpr int q = E % w, i2 = (E / w) % (2 * LP + 1), i1 = E / (w * (2 * LP + 1));
  if constexpr (i1 >= I0 && i1 < I1 && cg_rule(i1 - LT, i2 - LP, q - L)) {
    constexpr float c = (float)ce_real_cg(LT, LP, L, i1 - LT, i2 - LP, q - L);
    if constexpr (c != 0.0f) ga[i1 - I0] = fmaf(c, Wv[i2 * w + q], ga[i1 - I0]);
  }
}
template <int LT, int LP, int L, int I0, int I1, int... E>
__device__ __forceinline__ void adw_all(std::integer_sequence<int, E...>, const float* Wv, float* ga) {
  (adw_entry<LT, LP, L, I0, I1, E>(Wv, ga), ...);
}
// (i2, q) is used by some component of [I0, I1)
template <int LT, int LP, int L, int I0, int I1>
__device__ constexpr bool adw_used(int i2, int q) {
  for (int i1 = I0; i1 < I1; ++i1)
    if (cg_rule(i1 - LT, i2 - LP, q - L) && ce_real_cg(LT, LP, L, i1 - LT, i2 - LP, q - L) != 0.0)
      return true;
  return false;
}
template <int LT, int LP, int L, int I0, int I1, int E>
__device__ __forceinline__ void adw_acc(const float* Ap, const float* Zv, float* Wv) {
  constexpr int w = 2 * L + 1;
  constexpr int q = E % w, i2 = E / w;
  if constexpr (adw_used<LT, LP, L, I0, I1>(i2, q)) Wv[E] = fmaf(Ap[i2], Zv[q], Wv[E]);
}
template <int LT, int LP, int L, int I0, int I1, int... E>
__device__ __forceinline__ void adw_acc_all(std::integer_sequence<int, E...>, const float* Ap,
                                            const float* Zv, float* Wv) {
  (adw_acc<LT, LP, L, I0, I1, E>(Ap, Zv, Wv), ...);
}

template <int LT, int LP, int L, int I0, int I1>
__device__ __forceinline__ void adjoint_partners(const MixDev& m, const MixL& P, const float* At,
                                                 const float* Z, const int16_t* rows_lds, int j,
                                                 int t, float* ga) {
  constexpr int w = 2 * L + 1, w2 = 2 * LP + 1;
  const int lp1 = m.l_max + 1;
  const int nidx = m.n_max * lp1;
  const bool act = j < m.n_max;
  const int a = j * lp1 + LT;
  // the channel row of the next partner is fetched one partner ahead
  const int16_t* rp = rows_lds + a * nidx + LP;
  int row_next = act ? rp[0] : -1;
  float Wv[w2 * w];
#pragma unroll
  for (int e = 0; e < w2 * w; ++e) Wv[e] = 0.f;
#pragma unroll 1
  for (int np = 0; np < m.n_max; ++np) {
    const int pidx = np * lp1 + LP;
    const int row = row_next;
    row_next = (act && np + 1 < m.n_max) ? rp[(np + 1) * lp1] : -1;
    float Ap[w2], Zv[w];
    const float f = row < 0 ? 0.f : (pidx == a ? 2.f : 1.f);
#pragma unroll
    for (int q = 0; q < w2; ++q) Ap[q] = f * At[np * m.nlm + LP * LP + q];
    const int zb = (row < 0 ? 0 : row) * P.zstr + t * w;
#pragma unroll
    for (int q = 0; q < w; ++q) Zv[q] = Z[zb + q];
    adw_acc_all<LT, LP, L, I0, I1>(std::make_integer_sequence<int, w2 * w>{}, Ap, Zv, Wv);
  }
  adw_all<LT, LP, L, I0, I1>(std::make_integer_sequence<int, (2 * LT + 1) * w2 * w>{}, Wv, ga);
}

template <int LT, int L, int I0, int I1, int LP>
__device__ __forceinline__ void adjoint_lp(const MixDev& m, const MixL& P, const float* At,
                                           const float* Z, const int16_t* rows_lds, int j, int t,
                                           float* ga) {
  if constexpr (LP <= kMaxL) {
    if constexpr (iabs_c(LT - LP) <= L && L <= LT + LP && ((LT + LP + L) & 1) == 0) {
      if (LP <= m.l_max) adjoint_partners<LT, LP, L, I0, I1>(m, P, At, Z, rows_lds, j, t, ga);
    }
    adjoint_lp<LT, L, I0, I1, LP + 1>(m, P, At, Z, rows_lds, j, t, ga);
  }
}

// One adjoint job: the components [K (2LT+1)/NP, (K+1)(2LT+1)/NP) of every
// target (n, LT), summed over all partner patterns; jobs write disjoint
// gradient entries, so the sums are stored without atomics.  The job with
// LT = L also takes the A rows of X_L: dphi/dA_{n,L,M} gets Z of row (n, L)
// and its part K of A.Z (summed over n for each atom) goes to slot K of the
// atom's partial phi sums, which the rank adds up in a fixed order.
template <int LT, int L, int NP, int K>
__device__ __forceinline__ void adjoint_job(const MixDev& m, const MixL& P, const float* At,
                                            const float* Z, float* omt, float* phi_t,
                                            const int16_t* rows_lds, int j, int t) {
  constexpr int w = 2 * L + 1;
  constexpr int I0 = K * (2 * LT + 1) / NP, I1 = (K + 1) * (2 * LT + 1) / NP;
  const bool act = j < m.n_max;
  float ga[I1 - I0 > 0 ? I1 - I0 : 1];
#pragma unroll
  for (int q = 0; q < I1 - I0; ++q) ga[q] = 0.f;
  adjoint_lp<LT, L, I0, I1, 0>(m, P, At, Z, rows_lds, j, t, ga);
  if constexpr (LT == L) {
    if (P.arow) {
      const int zb = (P.nch + (act ? j : 0)) * P.zstr + t * w;
      float sa = 0.f;
#pragma unroll
      for (int q = I0; q < I1; ++q) {
        const float z = act ? Z[zb + q] : 0.f;
        ga[q - I0] += z;
        sa = fmaf(At[(act ? j : 0) * m.nlm + L * L + q], z, sa);
      }
      // sum over the 8 lanes of atom t (lanes t, t + 8, ..., t + 56)
      sa += __shfl_xor(sa, 8);
      sa += __shfl_xor(sa, 16);
      sa += __shfl_xor(sa, 32);
      if (j == 0) phi_t[K * kMT] = sa;
    }
  }
  if (act) {
#pragma unroll
    for (int q = I0; q < I1; ++q) omt[q] += ga[q - I0];
  }
}

#define AP_XB_CASE(la, lb)                                                           \
  case (la) * 5 + (lb):                                                              \
    if constexpr (iabs_c((la) - (lb)) <= L && L <= (la) + (lb) && (((la) + (lb) + L) & 1) == 0) \
      xbuild_group<la, lb, L>(At, mem, xh, xl, kstr, t, sx);                          \
    break;
#define AP_AD_CASE(lt, np, k)                                                        \
  case (lt) * 16 + (np) * 4 + (k):                                                   \
    if constexpr ((k) < (np) && (np) <= 2 * (lt) + 1)                                \
      adjoint_job<lt, L, np, k>(m, P, At, Z, omt, phi_t, rows_lds, j, t);            \
    break;
#define AP_AD_LT(lt) AP_AD_CASE(lt, 1, 0) AP_AD_CASE(lt, 2, 0) AP_AD_CASE(lt, 2, 1) \
  AP_AD_CASE(lt, 3, 0) AP_AD_CASE(lt, 3, 1) AP_AD_CASE(lt, 3, 2)
#define AP_ALL_CASES(X) \
  X(0, 0) X(0, 1) X(0, 2) X(0, 3) X(0, 4) X(1, 0) X(1, 1) X(1, 2) X(1, 3) X(1, 4) \
  X(2, 0) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(3, 0) X(3, 1) X(3, 2) X(3, 3) X(3, 4) \
  X(4, 0) X(4, 1) X(4, 2) X(4, 3) X(4, 4)

// Build the channel rows of X_L (fp16 hi/lo) for the 8 atoms of the tile.
// Group g of this L: members {row, A offset of a, A offset of b, la*5+lb}.
template <int L>
__device__ __forceinline__ void xbuild(const MixDev& m, const MixL& P, const float* A, _Float16* xh,
                                       _Float16* xl, const int4* mem_lds, const float* bn2, int wave,
                                       int lane) {
  const int t = lane & 7, j = lane >> 3;
  const float* At = A + t * m.apad;
  const int sx = xscale_exp(bn2[t], L);
  const int kstr = P.kstr;
  for (int g = wave; g < P.ngrp; g += kMWaves) {
    const int4 mem = mem_lds[g * 8 + j];
    const int key = uni(mem.w);
    if (mem.x < 0) continue;
    switch (key) {
      AP_ALL_CASES(AP_XB_CASE)
      default: break;
    }
  }
}

// Gradient of phi_p with respect to A from the coupled channels of X_L.  The
// wavefront's jobs (target l, component part) come from a schedule the
// library balanced over the workgroup's wavefronts.  part_p: the set's
// partial phi sums, [4 slots][8 atoms].
template <int L>
__device__ __forceinline__ void adjoint(const MixDev& m, const MixL& P, const float* A,
                                        const float* Z, float* om, float* part_p,
                                        const int16_t* rows_lds, int wave, int lane) {
  const int j = lane >> 3, t = lane & 7;
  float* phi_t = part_p + t;
  const float* At = A + t * m.apad;
  cptr<int32_t> ptr = as_const(m.adj_ptr) + L * (kMWaves + 1);
  const int u0 = uni(ptr[wave]), u1 = uni(ptr[wave + 1]);
  cptr<int32_t> units = as_const(reinterpret_cast<const int32_t*>(m.adj_units));
  for (int u = u0; u < u1; ++u) {
    const int key = uni(units[4 * u]), lt = uni(units[4 * u + 3]);
    float* omt = om + t * m.apad + j * m.nlm + lt * lt;
    switch (key) {
      AP_AD_LT(0) AP_AD_LT(1) AP_AD_LT(2) AP_AD_LT(3) AP_AD_LT(4)
      default: break;
    }
  }
}
#undef AP_XB_CASE
#undef AP_AD_CASE
#undef AP_AD_LT
#undef AP_ALL_CASES

template <int L, int RTW, int CTN, bool XO>
__device__ __forceinline__ void rank_L(const MixDev& m, const MixL& P, float* A, float* om1,
                                       float* om2, unsigned char* big, float* phi_lds,
                                       const float* bn2, const int16_t* rows_lds,
                                       const int4* mem_lds, const float* rs_lds, int wave, int lane,
                                       int tid) {
  const int w = 2 * L + 1;
  const int ncols = kMT * w;
  // X_L column-major (k contiguous), hi then lo.  Where Z_L shares the LDS
  // region (XO), only the tile's ncols columns are stored: the contraction's
  // reads of the padding columns of the last column tile then fall on lo
  // (or, for lo, on Z) and feed only result columns that are never stored.
  const int xcols = XO ? ncols : P.ct * 16;
  _Float16* xh = reinterpret_cast<_Float16*>(big);
  _Float16* xl = xh + (size_t)xcols * P.kstr;
  // coupled operand X_L: zero padding (rows past nrow up to the k tiles, and
  // the padding columns where they are stored), channel rows, A rows, constant row
  auto build_x = [&]() {
    const int kpad = P.kt * 32;
    const int padr = kpad - P.nrow;
    for (int q = tid; q < ncols * padr; q += kMThreads) {
      const int o = (q / padr) * P.kstr + P.nrow + q % padr;
      xh[o] = (_Float16)0.0f;
      xl[o] = (_Float16)0.0f;
    }
    if constexpr (!XO) {
      const int padc = P.ct * 16 - ncols;
      for (int q = tid; q < padc * kpad; q += kMThreads) {
        const int o = (ncols + q / kpad) * P.kstr + q % kpad;
        xh[o] = (_Float16)0.0f;
        xl[o] = (_Float16)0.0f;
      }
    }
    xbuild<L>(m, P, A, xh, xl, mem_lds, bn2, wave, lane);
    if (P.arow) {
      for (int q = tid; q < m.n_max * ncols; q += kMThreads) {
        const int n = q / ncols, col = q % ncols, t = col / w, M = col % w;
        const float v = A[t * m.apad + n * m.nlm + L * L + M];
        _Float16 hi, lo;
        split_f16(ldexpf(v, xscale_exp(bn2[t], L)), hi, lo);
        xh[col * P.kstr + P.nch + n] = hi;
        xl[col * P.kstr + P.nch + n] = lo;
      }
    }
    if (L == 0 && tid < kMT) {
      // the constant 1, scaled like the atom's column (a power of two <= 2^12)
      xh[tid * P.kstr + P.nch + m.n_max] = (_Float16)ldexpf(1.f, xscale_exp(bn2[tid], 0));
      xl[tid * P.kstr + P.nch + m.n_max] = (_Float16)0.0f;
    }
  };
  // partial phi sums of this rank, [set][slot][atom]: slots 0-2 the parts of
  // the A-row job, slot 3 the constant row (L = 0); every slot is written by
  // one lane and the slots are added to the atom's phi in a fixed order once
  // the rank is done, so the mixed path's sums do not depend on timing
  float* part = phi_lds + 3 * kMT;
  if (tid < 8 * kMT) part[tid] = 0.f;
  auto adjoint_set = [&](const float* Z, int p) {
    float* om = p == 0 ? om1 : om2;
    adjoint<L>(m, P, A, Z, om, part + p * 4 * kMT, rows_lds, wave, lane);
    if (L == 0 && tid < kMT) part[(p * 4 + 3) * kMT + tid] = 2.f * Z[(P.nch + m.n_max) * P.zstr + tid];
  };
  auto add_parts = [&]() {
    if (tid < 2 * kMT) {
      const float* q = part + (tid & 1) * 4 * kMT + (tid >> 1);
      phi_lds[tid] += ((q[0] + q[kMT]) + q[2 * kMT]) + q[3 * kMT];
    }
  };
  f32x4 acc[RTW][CTN];
  if constexpr (XO) {
    // X_L built once; Z_L beside it.  The contraction of set 1 reads only X,
    // so wavefronts may start it while others finish the adjoint of set 0.
    float* Z = reinterpret_cast<float*>(big + P.zoff);
    build_x();
    __syncthreads();
    gemm_tiles<RTW, CTN>(m, P, xh, xl, acc, wave, lane, 0);
    store_z<RTW, CTN>(P, acc, Z, bn2, rs_lds, L, 0, wave, lane, ncols);
    __syncthreads();
    adjoint_set(Z, 0);
    gemm_tiles<RTW, CTN>(m, P, xh, xl, acc, wave, lane, 1);
    __syncthreads();  // every wavefront is done with Z of set 0
    store_z<RTW, CTN>(P, acc, Z, bn2, rs_lds, L, 1, wave, lane, ncols);
    __syncthreads();
    adjoint_set(Z, 1);
    __syncthreads();
    add_parts();
  } else {
    float* Z = reinterpret_cast<float*>(big);
    for (int p = 0; p < 2; ++p) {
      build_x();
      __syncthreads();
      // Z_L of coefficient set p
      gemm_tiles<RTW, CTN>(m, P, xh, xl, acc, wave, lane, p);
      __syncthreads();  // X is dead from here on
      store_z<RTW, CTN>(P, acc, Z, bn2, rs_lds, L, p, wave, lane, ncols);
      __syncthreads();
      adjoint_set(Z, p);
      __syncthreads();
    }
    add_parts();
  }
}


// ---- kernel 2 (one instance per coupled rank L): coupling, folded
// contraction and adjoint for tiles of 8 atoms; adds the tile's gradient
// and phi terms of this L to the per-atom buffers (first rank: writes).
template <int L, int RTW, int CTN, bool XO>
__global__ __launch_bounds__(kMThreads, 1) void k_ace_rank(
    MixDev m, const int32_t* __restrict__ n_ace_p, int n_all, const float* __restrict__ A_in,
    float* __restrict__ om_buf, float* __restrict__ phi_buf, const float* __restrict__ bn_in) {
  extern __shared__ __align__(16) unsigned char lds[];
  float* A = reinterpret_cast<float*>(lds);
  float* om1 = A + kMT * m.apad;
  float* om2 = om1 + kMT * m.apad;
  float* phi_lds = om2 + kMT * m.apad;                  // [kMT][2], then [2][4][kMT] partial sums
  float* bn_lds = phi_lds + 2 * kMT;                    // [kMT]
  unsigned char* big = lds + m.big_off;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront-uniform
  const int n_items = n_ace_p ? *n_ace_p : n_all;
  const int n_tiles = (n_items + kMT - 1) / kMT;
  const MixL P = load_level(m.lv_d + L);
  // stage this rank's channel tables in LDS (read by every tile)
  const int nidx = m.n_max * (m.l_max + 1);
  int16_t* rows_lds = reinterpret_cast<int16_t*>(lds + m.tab_off);
  int4* mem_lds = reinterpret_cast<int4*>(lds + m.tab_off + (nidx * nidx * 2 + 15) / 16 * 16);
  for (int q = tid; q < nidx * nidx; q += kMThreads)
    rows_lds[q] = (int16_t)m.rowtab[(size_t)L * nidx * nidx + q];
  for (int q = tid; q < P.ngrp * 8; q += kMThreads) mem_lds[q] = m.grp_mem[(size_t)P.grp0 * 8 + q];
  float* rs_lds = reinterpret_cast<float*>(mem_lds + P.ngrp * 8);
  for (int q = tid; q < 2 * P.nrow16; q += kMThreads) rs_lds[q] = m.rscale[P.rs0 + q];
  // A of a tile's atoms and the gradient and phi sums of the lower ranks are
  // loaded into registers ahead of the tile that uses them
  constexpr int kPf = (kMT * (8 * kMaxLM + 1) + kMThreads - 1) / kMThreads;
  float pa[kPf];
  float2 po[kPf];
  float pphi = 0.f, pbn = 0.f;
  auto fetch = [&](int tile) {
    const int nt = min(kMT, n_items - tile * kMT);
    const int64_t base = (int64_t)tile * kMT * m.nA;
    // the index arithmetic below is redone per tile rather than kept live
    // across the whole tile loop (registers are scarce in rank_L)
    int tq = tid;
    asm volatile("" : "+v"(tq));
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
      const int q = tq + r * kMThreads;
      const int t = q / m.apad, e = q - t * m.apad;
      const bool ok = q < kMT * m.apad && t < nt && e < m.nA;
      const int64_t o = base + (int64_t)t * m.nA + e;
      pa[r] = ok ? A_in[o] : 0.f;
      po[r] = (L > 0 && ok) ? reinterpret_cast<const float2*>(om_buf)[o] : make_float2(0.f, 0.f);
    }
    if (tid < 2 * kMT) pphi = (L > 0 && tid < 2 * nt) ? phi_buf[(int64_t)tile * kMT * 2 + tid] : 0.f;
    if (tid < kMT) pbn = tid < nt ? bn_in[(int64_t)tile * kMT + tid] : 0.f;
  };
  auto stage = [&]() {
    int tq = tid;
    asm volatile("" : "+v"(tq));
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
      const int q = tq + r * kMThreads;
      if (q < kMT * m.apad) {
        A[q] = pa[r];
        om1[q] = po[r].x;
        om2[q] = po[r].y;
      }
    }
    if (tid < 2 * kMT) phi_lds[tid] = pphi;
    if (tid < kMT) bn_lds[tid] = pbn;
  };
  if ((int)blockIdx.x < n_tiles) {
    fetch(blockIdx.x);
    stage();
  }
  __syncthreads();
  // ranks with spare registers fetch the next tile before this tile's work,
  // the others just before this tile's stores
  constexpr bool kEarly = L <= 1 || L >= 7;
  for (int tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int nt = min(kMT, n_items - tile * kMT);
    const int64_t base = (int64_t)tile * kMT * m.nA;
    const int next = tile + (int)gridDim.x;
    if (kEarly && next < n_tiles) fetch(next);
    rank_L<L, RTW, CTN, XO>(m, P, A, om1, om2, big, phi_lds, bn_lds, rows_lds, mem_lds, rs_lds, wave,
                            lane, tid);
    __syncthreads();
    if (!kEarly && next < n_tiles) fetch(next);
    for (int q = tid; q < nt * m.nA; q += kMThreads) {
      const int t = q / m.nA, e = q - t * m.nA;
      reinterpret_cast<float2*>(om_buf)[base + q] = make_float2(om1[t * m.apad + e], om2[t * m.apad + e]);
    }
    if (tid < 2 * nt) phi_buf[(int64_t)tile * kMT * 2 + tid] = phi_lds[tid];
    __syncthreads();
    if (next < n_tiles) stage();
    __syncthreads();
  }
}

}  // namespace ap
