// Cell-list neighbour build: binning (counting sort), 27-cell stencil with
// the canonical FP64 test, ascending-order ELL lists and the reverse-slot
// index.  Also the generic fill and scan primitives.
#include <algorithm>

#include "ap_internal.h"
#include "geom.h"
#include "scan.h"

namespace ap {

// --------------------------------------------------------------------------
template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, T v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) { return fill(p, v, n, s); }

// --------------------------------------------------------------------------
// cell of atom i: orthorhombic boxes bin Cartesian coordinates (clamped into
// the grid in free dimensions), triclinic boxes bin wrapped fractional ones.
__device__ __forceinline__ int cell_coords(const SysView& sv, int s, double x, double y, double z,
                                           int& cx, int& cy, int& cz) {
  const int* g = sv.grid + 3 * s;
  const double* H = sv.H + 9 * s;
  double f0, f1, f2;
  if (sv.ortho[s]) {
    f0 = x / H[0];
    f1 = y / H[4];
    f2 = z / H[8];
  } else {
    frac3(sv.Hi + 9 * s, x, y, z, f0, f1, f2);
    f0 -= floor(f0);
    f1 -= floor(f1);
    f2 -= floor(f2);
  }
  // non-finite coordinates land in cell 0 (the force check reports them)
  cx = isfinite(f0) ? (int)fmax(-1.0, fmin(floor(f0 * g[0]), (double)g[0])) : 0;
  cy = isfinite(f1) ? (int)fmax(-1.0, fmin(floor(f1 * g[1]), (double)g[1])) : 0;
  cz = isfinite(f2) ? (int)fmax(-1.0, fmin(floor(f2 * g[2]), (double)g[2])) : 0;
  cx = cx < 0 ? 0 : (cx >= g[0] ? g[0] - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= g[1] ? g[1] - 1 : cy);
  cz = cz < 0 ? 0 : (cz >= g[2] ? g[2] - 1 : cz);
  return sv.cell_base[s] + (cx * g[1] + cy) * g[2] + cz;
}

__global__ void k_bin(SysView sv, const double* __restrict__ pos, int32_t* __restrict__ cell_of,
                      int32_t* __restrict__ cell_count) {
  const int n = sv.n_atoms;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int cx, cy, cz;
  int c = cell_coords(sv, sv.sys_of[i], pos[i], pos[n + i], pos[2 * n + i], cx, cy, cz);
  cell_of[i] = c;
  atomicAdd(&cell_count[c], 1);
}

hipError_t launch_bin(const SysView& sv, const double* pos, int32_t* cell_of, int32_t* cell_count,
                      hipStream_t s) {
  if (sv.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin, dim3((sv.n_atoms + 255) / 256), dim3(256), 0, s, sv, pos, cell_of,
                     cell_count);
  return hipGetLastError();
}

__global__ void k_scatter(int n, const double* __restrict__ pos, const int32_t* __restrict__ cell_of,
                          int32_t* __restrict__ cursor, int32_t* __restrict__ cell_atoms,
                          double4* __restrict__ cell_pos) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int slot = atomicAdd(&cursor[cell_of[i]], 1);
  cell_atoms[slot] = i;
  cell_pos[slot] = make_double4(pos[i], pos[n + i], pos[2 * n + i], (double)i);
}

hipError_t launch_scatter(const SysView& sv, const double* pos, const int32_t* cell_of,
                          int32_t* cursor, int32_t* cell_atoms, double4* cell_pos, hipStream_t s) {
  if (sv.n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((sv.n_atoms + 255) / 256), dim3(256), 0, s, sv.n_atoms, pos,
                     cell_of, cursor, cell_atoms, cell_pos);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// One wavefront per atom.  The (at most 27, deduplicated) stencil cells are
// laid end to end; lanes walk the concatenated candidates 64 at a time,
// accepted indices are compacted into LDS with a ballot, then each lane
// ranks its entries (indices are unique) and stores them in ascending order.
constexpr int kWavesPerBlock = 4;
constexpr int kListLds = kMaxCap;

__device__ __forceinline__ void atom_list_direct(const SysView& sv, const double* __restrict__ pos,
                                                 const int32_t* __restrict__ cell_of,
                                                 const int32_t* __restrict__ cell_start,
                                                 const int32_t* __restrict__ cell_count,
                                                 const double4* __restrict__ cell_pos,
                                                 int32_t* __restrict__ nbr,
                                                 int32_t* __restrict__ count, int cap,
                                                 int32_t* __restrict__ overflow, int i,
                                                 int (&list)[kWavesPerBlock][kListLds],
                                                 int (&st_cell)[kWavesPerBlock][32],
                                                 int (&st_pre)[kWavesPerBlock][33]) {
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int n = sv.n_atoms;
  const int s = sv.sys_of[i];
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int* g = sv.grid + 3 * s;
  const int ci = cell_of[i] - sv.cell_base[s];
  const int c0 = ci / (g[1] * g[2]);
  const int c1 = (ci / g[2]) % g[1];
  const int c2 = ci % g[2];
  const int cc[3] = {c0, c1, c2};
  // stencil: lane k < 27 owns offset (k/9, k/3%3, k%3) of the per-axis lists
  int my_cell = -1, my_cnt = 0;
  if (lane < 27) {
    int idx[3] = {lane / 9, (lane / 3) % 3, lane % 3};
    int co[3];
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
      const int gk = g[k];
      if (sv.per[k] && gk < 3) {
        if (idx[k] >= gk) ok = false;
        co[k] = idx[k];
      } else {
        int v = cc[k] + idx[k] - 1;
        if (sv.per[k]) {
          v = v < 0 ? v + gk : (v >= gk ? v - gk : v);
        } else if (v < 0 || v >= gk) {
          ok = false;
        }
        co[k] = v;
      }
    }
    if (ok) {
      my_cell = sv.cell_base[s] + (co[0] * g[1] + co[1]) * g[2] + co[2];
      my_cnt = cell_count[my_cell];
    }
  }
  const int incl = wave_incl_scan_i32(my_cnt, lane);
  const int total = __shfl(incl, 63);
  if (lane < 27) {
    st_cell[w][lane] = my_cell;
    st_pre[w][lane] = incl - my_cnt;
  }
  if (lane == 27) st_pre[w][27] = total;
  __syncwarp_ap();
  const bool ortho = sv.ortho[s] != 0;
  const double* H = sv.H + 9 * s;
  const double* Hi = sv.Hi + 9 * s;
  int cnt = 0;
  for (int base = 0; base < total; base += 64) {
    const int c = base + lane;
    bool acc = false;
    int j = -1;
    if (c < total) {
      int k = 0;
      while (k < 26 && st_pre[w][k + 1] <= c) ++k;
      const int slot = cell_start[st_cell[w][k]] + (c - st_pre[w][k]);
      const double4 q = cell_pos[slot];
      j = (int)q.w;
      if (j != i) {
        double dx, dy, dz;
        displacement(ortho, H, Hi, sv.per, xi, yi, zi, q.x, q.y, q.z, dx, dy, dz);
        acc = norm2(dx, dy, dz) < sv.rc2;
      }
    }
    const unsigned long long b = __ballot(acc);
    if (acc) {
      const int p = cnt + __popcll(b & ((1ull << lane) - 1ull));
      if (p < kListLds) list[w][p] = j;
    }
    cnt += __popcll(b);
  }
  __syncwarp_ap();
  if (cnt > cap && lane == 0) atomicMax(overflow, cnt);
  const int m = cnt < kListLds ? cnt : kListLds;
  for (int e = lane; e < m; e += 64) {
    const int v = list[w][e];
    int rank = 0;
    for (int q = 0; q < m; ++q) rank += list[w][q] < v;
    if (rank < cap) nbr[(int64_t)rank * n + i] = v;
  }
  if (lane == 0) count[i] = cnt < cap ? cnt : cap;
}

__global__ __launch_bounds__(256) void k_fill_nbr(SysView sv, const double* __restrict__ pos,
                                                  const int32_t* __restrict__ cell_of,
                                                  const int32_t* __restrict__ cell_start,
                                                  const int32_t* __restrict__ cell_count,
                                                  const double4* __restrict__ cell_pos,
                                                  int32_t* __restrict__ nbr,
                                                  int32_t* __restrict__ count, int cap,
                                                  int32_t* __restrict__ overflow) {
  __shared__ int list[kWavesPerBlock][kListLds];
  __shared__ int st_cell[kWavesPerBlock][32];
  __shared__ int st_pre[kWavesPerBlock][33];
  const int i = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
  if (i >= sv.n_atoms) return;  // whole wavefront leaves together
  atom_list_direct(sv, pos, cell_of, cell_start, cell_count, cell_pos, nbr, count, cap, overflow, i,
                   list, st_cell, st_pre);
}

__global__ __launch_bounds__(256) void k_fill_nbr_big(SysView sv, const double* __restrict__ pos,
                                                      const int32_t* __restrict__ cell_of,
                                                      const int32_t* __restrict__ cell_start,
                                                      const int32_t* __restrict__ cell_count,
                                                      const double4* __restrict__ cell_pos,
                                                      int32_t* __restrict__ nbr,
                                                      int32_t* __restrict__ count, int cap,
                                                      int32_t* __restrict__ overflow,
                                                      const int32_t* __restrict__ big_atoms) {
  __shared__ int list[kWavesPerBlock][kListLds];
  __shared__ int st_cell[kWavesPerBlock][32];
  __shared__ int st_pre[kWavesPerBlock][33];
  // big_atoms = [m, atom_0, ..., atom_{m-1}]: one wavefront per listed atom,
  // grid-stride (the loop only holds wavefront-level synchronisation)
  const int m = big_atoms[0];
  const int waves = gridDim.x * kWavesPerBlock;
  for (int w = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6); w < m; w += waves)
    atom_list_direct(sv, pos, cell_of, cell_start, cell_count, cell_pos, nbr, count, cap, overflow,
                     big_atoms[1 + w], list, st_cell, st_pre);
}

hipError_t launch_fill_nbr(const SysView& sv, const double* pos, const int32_t* cell_of,
                           const int32_t* cell_start, const int32_t* cell_count,
                           const double4* cell_pos, int32_t* nbr, int32_t* count, int32_t cap,
                           int32_t* overflow, hipStream_t s) {
  if (sv.n_atoms == 0) return hipSuccess;
  const int blocks = (sv.n_atoms + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL(k_fill_nbr, dim3(blocks), dim3(64 * kWavesPerBlock), 0, s, sv, pos, cell_of,
                     cell_start, cell_count, cell_pos, nbr, count, cap, overflow);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// One workgroup per cell.  The candidates of the cell's stencil (at most 27
// deduplicated cells) are gathered into LDS once (as FP32 coordinates) and
// shared by the cell's atoms, one wavefront per atom: lanes screen 64
// candidates at a time in FP32 with a 0.05 A margin and compact the
// survivors (about a quarter); the survivors are tested with the canonical
// FP64 rule, accepted indices are compacted into a per-wavefront LDS list
// with a ballot, then each lane ranks its entries (indices are unique) and
// stores them in ascending order.  A cell whose stencil holds more than
// kMaxCand candidates falls back to the kernel above for its atoms.
constexpr int kCellThreads = 256;
constexpr int kCellWaves = kCellThreads / 64;
constexpr int kMaxCand = 512;

__global__ __launch_bounds__(kCellThreads) void k_fill_nbr_cell(
    SysView sv, const int32_t* __restrict__ cell_start, const int32_t* __restrict__ cell_count,
    const double4* __restrict__ cell_pos, int32_t* __restrict__ nbr, int32_t* __restrict__ count,
    int cap, int32_t* __restrict__ overflow, int32_t* __restrict__ big_atoms) {
  // candidates as float (x, y, z) plus their cell-order index: the screen;
  // the exact FP64 test reads the survivors' positions from cell_pos
  __shared__ float4 cposf[kMaxCand];
  __shared__ int cand[kCellWaves][kMaxCand];
  __shared__ __align__(16) int list[kCellWaves][kListLds + 4];
  __shared__ int st_src[32];   // first cell-ordered atom of each stencil cell
  __shared__ int st_pre[33];   // exclusive prefix of the stencil cells' counts
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = blockIdx.x;
  const int n_here = cell_count[c];
  if (n_here == 0) return;  // whole workgroup
  // system of this cell
  int lo = 0, hi = sv.n_sys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sv.cell_base[mid] <= c) lo = mid; else hi = mid - 1;
  }
  const int s = lo;
  const int* g = sv.grid + 3 * s;
  const int ci = c - sv.cell_base[s];
  const int cc[3] = {ci / (g[1] * g[2]), (ci / g[2]) % g[1], ci % g[2]};
  if (wave == 0) {
    int my_cell = -1, my_cnt = 0, my_src = 0;
    if (lane < 27) {
      const int idx[3] = {lane / 9, (lane / 3) % 3, lane % 3};
      int co[3];
      bool ok = true;
      for (int k = 0; k < 3; ++k) {
        const int gk = g[k];
        if (sv.per[k] && gk < 3) {
          if (idx[k] >= gk) ok = false;
          co[k] = idx[k];
        } else {
          int v = cc[k] + idx[k] - 1;
          if (sv.per[k]) {
            v = v < 0 ? v + gk : (v >= gk ? v - gk : v);
          } else if (v < 0 || v >= gk) {
            ok = false;
          }
          co[k] = v;
        }
      }
      if (ok) {
        my_cell = sv.cell_base[s] + (co[0] * g[1] + co[1]) * g[2] + co[2];
        my_cnt = cell_count[my_cell];
        my_src = cell_start[my_cell];
      }
    }
    const int incl = wave_incl_scan_i32(my_cnt, lane);
    if (lane < 27) {
      st_src[lane] = my_src;
      st_pre[lane] = incl - my_cnt;
    }
    if (lane == 26) st_pre[27] = incl;
  }
  __syncthreads();
  const int total = st_pre[27];
  const int n = sv.n_atoms;
  const int first = cell_start[c];
  if (total > kMaxCand) {
    // too many candidates for LDS: the cell's atoms go to the fallback
    // kernel's list (their order there does not matter, every row is
    // computed on its own)
    __shared__ int s_base;
    if (tid == 0) s_base = atomicAdd(big_atoms, n_here);
    __syncthreads();
    for (int a = tid; a < n_here; a += kCellThreads)
      big_atoms[1 + s_base + a] = (int)cell_pos[first + a].w;
    return;
  }
  // candidates of the stencil, cell after cell, all loads of the workgroup in
  // one pass: candidate q belongs to the last stencil cell k with
  // st_pre[k] <= q (that cell is not empty, as st_pre[k + 1] > q)
  for (int q = tid; q < total; q += kCellThreads) {
    int lo = 0, hi = 26;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (st_pre[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const int src = st_src[lo] + (q - st_pre[lo]);
    const double4 p = cell_pos[src];
    cposf[q] = make_float4((float)p.x, (float)p.y, (float)p.z, __int_as_float(src));
  }
  __syncthreads();
  const bool ortho = sv.ortho[s] != 0;
  const double* H = sv.H + 9 * s;
  const double* Hi = sv.Hi + 9 * s;
  // screen in FP32 on orthorhombic boxes: the minimum-image distance of the
  // rounded positions is within 0.02 A of the exact one for coordinates below
  // 1e5 A, so every pair with r < r_c passes r < r_c + 0.05 A; the exact
  // canonical FP64 test then decides (triclinic boxes: every candidate goes on)
  const float Lf[3] = {(float)H[0], (float)H[4], (float)H[8]};
  const float iLf[3] = {1.f / Lf[0], 1.f / Lf[1], 1.f / Lf[2]};
  const float rs = (float)sqrt(sv.rc2) + 0.05f;
  const float rs2 = rs * rs;
  int* lw = list[wave];
  int* cw = cand[wave];
  for (int a = wave; a < n_here; a += kCellWaves) {
    const double4 pi = cell_pos[first + a];
    const int i = (int)pi.w;
    const float xf = (float)pi.x, yf = (float)pi.y, zf = (float)pi.z;
    int npass = 0;
    for (int base = 0; base < total; base += 64) {
      const int q = base + lane;
      bool pass = false;
      int src = 0;
      if (q < total) {
        const float4 pf = cposf[q];
        src = __float_as_int(pf.w);
        if (ortho) {
          float d[3] = {pf.x - xf, pf.y - yf, pf.z - zf};
#pragma unroll
          for (int k = 0; k < 3; ++k)
            if (sv.per[k]) d[k] -= Lf[k] * rintf(d[k] * iLf[k]);
          pass = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rs2;
        } else {
          pass = true;
        }
      }
      const unsigned long long b = __ballot(pass);
      if (pass) cw[npass + __popcll(b & ((1ull << lane) - 1ull))] = src;
      npass += __popcll(b);
    }
    __syncwarp_ap();
    int cnt = 0;
    for (int base = 0; base < npass; base += 64) {
      const int q = base + lane;
      bool acc = false;
      int j = -1;
      if (q < npass) {
        const double4 pj = cell_pos[cw[q]];
        j = (int)pj.w;
        if (j != i) {
          double dx, dy, dz;
          displacement(ortho, H, Hi, sv.per, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
          acc = norm2(dx, dy, dz) < sv.rc2;
        }
      }
      const unsigned long long b = __ballot(acc);
      if (acc) {
        const int p = cnt + __popcll(b & ((1ull << lane) - 1ull));
        if (p < kListLds) lw[p] = j;
      }
      cnt += __popcll(b);
    }
    const int m = cnt < kListLds ? cnt : kListLds;
    if (lane < 4) lw[m + lane] = 0x7fffffff;  // sentinels: the rank loop reads whole int4
    __syncwarp_ap();
    for (int e = lane; e < m; e += 64) {
      const int v = lw[e];
      int rank = 0;
      for (int q = 0; q < m; q += 4) {
        const int4 u = *reinterpret_cast<const int4*>(lw + q);
        rank += (u.x < v) + (u.y < v) + (u.z < v) + (u.w < v);
      }
      if (rank < cap) nbr[(int64_t)rank * n + i] = v;
    }
    if (lane == 0) {
      count[i] = cnt < cap ? cnt : cap;
      if (cnt > cap) atomicMax(overflow, cnt);
    }
    __syncwarp_ap();
  }
}

hipError_t launch_fill_nbr_cells(const SysView& sv, int32_t n_cells, const double* pos,
                                 const int32_t* cell_of, const int32_t* cell_start,
                                 const int32_t* cell_count, const double4* cell_pos, int32_t* nbr,
                                 int32_t* count, int32_t cap, int32_t* overflow, int32_t* big_atoms,
                                 hipStream_t s) {
  if (sv.n_atoms == 0 || n_cells == 0) return hipSuccess;
  hipError_t e = launch_fill_i32(big_atoms, 0, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_fill_nbr_cell, dim3(n_cells), dim3(kCellThreads), 0, s, sv, cell_start,
                     cell_count, cell_pos, nbr, count, cap, overflow, big_atoms);
  const int blocks = std::min((sv.n_atoms + kWavesPerBlock - 1) / kWavesPerBlock, 1024);
  hipLaunchKernelGGL(k_fill_nbr_big, dim3(blocks), dim3(64 * kWavesPerBlock), 0, s, sv, pos, cell_of,
                     cell_start, cell_count, cell_pos, nbr, count, cap, overflow, big_atoms);
  return hipGetLastError();
}

// rev[s][i] = slot of i in the (ascending) list of j = nbr[s][i]
__global__ void k_rev(int n, const int32_t* __restrict__ nbr, const int32_t* __restrict__ count,
                      int32_t* __restrict__ rev) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ci = count[i];
  for (int s = 0; s < ci; ++s) {
    const int j = nbr[(int64_t)s * n + i];
    int lo = 0, hi = count[j] - 1, r = -1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = nbr[(int64_t)mid * n + j];
      if (v == i) { r = mid; break; }
      if (v < i) lo = mid + 1; else hi = mid - 1;
    }
    rev[(int64_t)s * n + i] = r;
  }
}

hipError_t launch_rev(int32_t n_atoms, const int32_t* nbr, const int32_t* count, int32_t* rev,
                      hipStream_t s) {
  if (n_atoms == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rev, dim3((n_atoms + 255) / 256), dim3(256), 0, s, n_atoms, nbr, count, rev);
  return hipGetLastError();
}

}  // namespace ap
