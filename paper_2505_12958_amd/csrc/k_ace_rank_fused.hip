// All coupled ranks of the mixed-precision ACE path in one persistent launch.
//
// A workgroup takes a tile of 8 ACE atoms, stages their atomic basis A and
// the per-atom bound of the coupled operand once, and runs every coupled
// rank L = 0..L_max on it (coupling, split-fp16 contraction, adjoint) with
// the adjoints dphi_p/dA and the phi sums of both coefficient sets held in
// LDS throughout; only the finished adjoints and sums go back to HBM.  Each
// rank stages its own channel tables (from L2) before its body runs.
//
// Tiles come either round-robin (tile = workgroup + k * grid) or from a
// device work counter (one atomic per tile, taken one tile ahead), chosen by
// the library's tuner.  Every tile costs the same in this phase (the work per
// atom does not depend on its neighbour count), so the counter only matters
// when the workgroups do not run in lockstep.
#include "ace_rank.h"

namespace ap {

// coupled rank L of the current tile: its channel tables and row scales into
// LDS, then the
// rank body (which ends with a workgroup barrier).  Whether rank L keeps X_L
// for both coefficient sets (bit L of XOMASK) is fixed at compile time, so
// only the variant the model's LDS layout chose is generated.
template <int L, uint32_t XOMASK>
__device__ __forceinline__ void fused_rank(const MixDev& m, float* A, float* om1, float* om2,
                                           unsigned char* big, float* phi_lds, const float* bn_lds,
                                           const int32_t* lv_lds, int16_t* rows_lds, int4* mem_lds,
                                           int wave, int lane, int tid) {
  const MixL P = load_level_lds(lv_lds + L * kLevelInts);
  const int nidx = m.n_max * (m.l_max + 1);
  for (int q = tid; q < nidx * nidx; q += kMThreads)
    rows_lds[q] = (int16_t)m.rowtab[(size_t)L * nidx * nidx + q];
  for (int q = tid; q < P.ngrp * 8; q += kMThreads) mem_lds[q] = m.grp_mem[(size_t)P.grp0 * 8 + q];
  float* rs_lds = reinterpret_cast<float*>(mem_lds + P.ngrp * 8);
  for (int q = tid; q < 2 * P.nrow16; q += kMThreads) rs_lds[q] = m.rscale[P.rs0 + q];
  __syncthreads();
  rank_L<L, kMixRtw[L], L + 1, ((XOMASK >> L) & 1u) != 0>(m, P, A, om1, om2, big, phi_lds, bn_lds,
                                                          rows_lds, mem_lds, rs_lds, wave, lane, tid);
}

// ranks L..LMAX of the tile in order; the next tile's A is loaded into
// registers ahead of the last two (the lightest) ranks
template <int L, int LMAX, uint32_t XOMASK, typename Fetch>
__device__ __forceinline__ void fused_ranks(const MixDev& m, float* A, float* om1, float* om2,
                                            unsigned char* big, float* phi_lds, const float* bn_lds,
                                            const int32_t* lv_lds, int16_t* rows_lds, int4* mem_lds,
                                            int wave, int lane, int tid, Fetch&& fetch_next) {
  if constexpr (L <= LMAX) {
    if constexpr (L == (LMAX > 0 ? LMAX - 1 : 0)) fetch_next();
    fused_rank<L, XOMASK>(m, A, om1, om2, big, phi_lds, bn_lds, lv_lds, rows_lds, mem_lds, wave, lane,
                          tid);
    fused_ranks<L + 1, LMAX, XOMASK>(m, A, om1, om2, big, phi_lds, bn_lds, lv_lds, rows_lds, mem_lds,
                                     wave, lane, tid, fetch_next);
  }
}

template <bool QUEUE, uint32_t XOMASK, int LMAX>
__global__ __launch_bounds__(kMThreads, 1) void k_ace_rank_fused(
    MixDev m, const int32_t* __restrict__ n_ace_p, int n_all, const float* __restrict__ A_in,
    float* __restrict__ om_buf, float* __restrict__ phi_buf, const float* __restrict__ bn_in,
    int32_t* __restrict__ queue) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int next_s;
  float* A = reinterpret_cast<float*>(lds);
  float* om1 = A + kMT * m.apad;
  float* om2 = om1 + kMT * m.apad;
  float* phi_lds = om2 + kMT * m.apad;                  // [kMT][2], then [2][4][kMT] partial sums
  float* bn_lds = phi_lds + 2 * kMT;                    // [kMT]
  unsigned char* big = lds + m.big_off;
  const int nidx = m.n_max * (m.l_max + 1);
  int16_t* rows_lds = reinterpret_cast<int16_t*>(lds + m.tab_off);
  int4* mem_lds = reinterpret_cast<int4*>(lds + m.tab_off + (nidx * nidx * 2 + 15) / 16 * 16);
  int32_t* lv_lds = reinterpret_cast<int32_t*>(lds + m.tab_off) - (2 * kMaxL + 1) * kLevelInts;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int q = tid; q < (LMAX + 1) * kLevelInts; q += kMThreads) {
    const int L = q / kLevelInts, f = q % kLevelInts;
    lv_lds[q] = f < 15 ? reinterpret_cast<const int32_t*>(m.lv_d + L)[f] : 0;
  }
  const int n_items = n_ace_p ? *n_ace_p : n_all;
  const int n_tiles = (n_items + kMT - 1) / kMT;
  constexpr int kPf = (kMT * (8 * kMaxLM + 1) + kMThreads - 1) / kMThreads;
  float pa[kPf];
  float pbn = 0.f;
  auto fetch = [&](int tile) {
    const int nt = min(kMT, n_items - tile * kMT);
    const int64_t base = (int64_t)tile * kMT * m.nA;
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
      const int q = tid + r * kMThreads;
      const int t = q / m.apad, e = q - t * m.apad;
      const bool ok = q < kMT * m.apad && t < nt && e < m.nA;
      pa[r] = ok ? A_in[base + (int64_t)t * m.nA + e] : 0.f;
    }
    if (tid < kMT) pbn = tid < nt ? bn_in[(int64_t)tile * kMT + tid] : 0.f;
  };
  // A and the bound of the next tile; the adjoints and phi sums start at zero
  auto stage = [&]() {
#pragma unroll
    for (int r = 0; r < kPf; ++r) {
      const int q = tid + r * kMThreads;
      if (q < kMT * m.apad) {
        A[q] = pa[r];
        om1[q] = 0.f;
        om2[q] = 0.f;
      }
    }
    if (tid < 2 * kMT) phi_lds[tid] = 0.f;
    if (tid < kMT) bn_lds[tid] = pbn;
  };
  auto take = [&](int fallback) {
    if constexpr (QUEUE) {
      if (tid == 0) next_s = atomicAdd(queue, 1);
      __syncthreads();
      const int t = next_s;
      __syncthreads();
      return t;
    } else {
      return fallback;
    }
  };
  int tile = take((int)blockIdx.x);
  if (tile < n_tiles) {
    fetch(tile);
    stage();
  }
  __syncthreads();
  while (tile < n_tiles) {
    const int nt = min(kMT, n_items - tile * kMT);
    const int64_t base = (int64_t)tile * kMT * m.nA;
    const int next = take(tile + (int)gridDim.x);
    fused_ranks<0, LMAX, XOMASK>(m, A, om1, om2, big, phi_lds, bn_lds, lv_lds, rows_lds, mem_lds, wave,
                                 lane, tid, [&]() {
                                   if (next < n_tiles) fetch(next);
                                 });
    for (int q = tid; q < nt * m.nA; q += kMThreads) {
      const int t = q / m.nA, e = q - t * m.nA;
      reinterpret_cast<float2*>(om_buf)[base + q] = make_float2(om1[t * m.apad + e], om2[t * m.apad + e]);
    }
    if (tid < 2 * nt) phi_buf[(int64_t)tile * kMT * 2 + tid] = phi_lds[tid];
    __syncthreads();
    if (next < n_tiles) stage();
    __syncthreads();
    tile = next;
  }
}

// Instances for the rank layouts of the two model shapes of the workloads:
// (n_max 8, l_max 4, nu <= 4): L_max 8, X_L kept at L = 0, 1, 2, 6, 7, 8;
// (n_max 6, l_max 3, nu <= 3): L_max 3, X_L kept at every L.
// Other layouts run one kernel per rank.
const void* rank_kernel_fused(bool queue, uint32_t xomask, int lmax) {
  if (xomask == 0x1c7u && lmax == 8)
    return queue ? (const void*)k_ace_rank_fused<true, 0x1c7u, 8> : (const void*)k_ace_rank_fused<false, 0x1c7u, 8>;
  if (xomask == 0xfu && lmax == 3)
    return queue ? (const void*)k_ace_rank_fused<true, 0xfu, 3> : (const void*)k_ace_rank_fused<false, 0xfu, 3>;
  return nullptr;
}

}  // namespace ap
