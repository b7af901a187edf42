// Internal declarations of the AP library: context, device-side model
// tables, kernel launchers.  Not part of the public ABI (include/ap.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/ap.h"

namespace ap {

constexpr int kMaxSys = 1 << 20;
constexpr int kMaxL = 4;                   // l_max limit of the ACE model
constexpr int kMaxLM = (kMaxL + 1) * (kMaxL + 1);
constexpr int kMaxN = 16;
constexpr int kMaxK = 16;
constexpr int kMaxCap = 256;               // neighbour-list capacity limit
constexpr int kReduceChunk = 4096;         // atoms per deterministic partial sum

#define AP_HIP(call)                                                    \
  do {                                                                  \
    hipError_t e_ = (call);                                             \
    if (e_ != hipSuccess) return fail_hip(ctx, e_, #call, __FILE__, __LINE__); \
  } while (0)

// --------------------------------------------------------------------------
// device view of the systems of one call
struct SysView {
  int32_t n_sys;
  int32_t n_atoms;
  const int64_t* off;      // n_sys+1
  const double* H;         // 9 per system
  const double* Hi;        // 9 per system (triclinic inverse; unused for orthorhombic)
  const uint8_t* ortho;    // per system
  const int32_t* grid;     // 3 per system: cells along each axis
  const int32_t* cell_base;// n_sys+1: first global cell of each system
  const int32_t* sys_of;   // per atom
  int32_t per[3];
  int32_t all_ortho;        // every system orthorhombic (kernels may specialise)
  double rc2;
};

// piecewise-cubic table on device (4 coefficients per interval)
struct TableDev {
  double x0, dx, inv_dx;
  int32_t n;                // knots
  const double* c;          // (n-1)*4
  const float* cf;          // same, float
};

// the paper's W EAM in closed form (passed to the EAM kernels by value)
constexpr int kMaxEamKnots = 32;
struct EamAnalyticDev {
  int32_t n_phi, n_rho;
  double a_phi[kMaxEamKnots], d_phi[kMaxEamKnots];
  double a_rho[kMaxEamKnots], d_rho[kMaxEamKnots];
  double r_cut_rho, zeta_cut;       // zeta = zeta_0(max(r, r_cut)); zeta_cut = zeta_0(r_cut)
  double a_xi1, a_xi2, d_xi;
  double zbl_pref, a_zbl;           // Z^2 / (4 pi eps0), screening length
  double zbl_c[4], zbl_q[4];
  double r_lo, r_hi, b_phi[6];
};

// ACE model folded for the device
// one term of the FP64 path's sparse sums, read as a single 16-byte load:
// coefficient c and the two operand indices i, j
struct alignas(16) PairTerm {
  double c;
  int32_t i, j;
};

struct AceDev {
  int32_t n_max, l_max, K, nlm, nA, nnl;
  int32_t L_max;            // largest coupled L
  double rc;
  const double* W;          // [n_max][l_max+1][K]
  const float* Wf;
  const double* ynorm;      // N_lm for m >= 0 at l*l + l + m (sqrt2 folded in for m > 0)
  // per L (0..L_max): X_L rows = [channels | A rows (n, l=L) | one-row (L=0)]
  int32_t nrow[2 * kMaxL + 1];
  int32_t nch[2 * kMaxL + 1];
  int32_t has_arow[2 * kMaxL + 1];
  // CSR building X: entry e of (channel row r, M) at dst = r*(2L+1)+M
  int32_t xb_off[2 * kMaxL + 2];    // offset of the L block in xb_ptr (size nch*(2L+1)+1 each)
  const int32_t* xb_ptr;
  const PairTerm* xb_t;             // c A[i] A[j]
  // Cext_L CSR over rows (symmetric, both coefficient sets)
  int32_t cx_off[2 * kMaxL + 2];    // offset of the L block in cx_ptr (nrow+1 each)
  const int32_t* cx_ptr;
  const int32_t* cx_col;
  const double2* cx_val;
  // adjoint CSR over A targets: terms (z index, partner A index, coef)
  int32_t ad_off[2 * kMaxL + 2];    // offset of the L block in ad_ptr (nA+1 each)
  const int32_t* ad_ptr;
  const PairTerm* ad_t;             // c A[i] Z[j]
  int32_t max_xsize;        // max_L nrow*(2L+1)
};

// ---- mixed-precision ACE model: per-L tiling, dense split-fp16 tiles,
// channel groups of equal (l_a, l_b) with their coupling entries
struct CgEnt {
  int8_t m1, m2, M, pad;
  float c;
};

// Work-group shape of the mixed rank kernels: kMixWaves wavefronts; each
// owns at most kMixRtw[L] 16-row tiles of one coefficient set of C_L
// (row tile rt = wave + kMixWaves * i).
constexpr int kMixWaves = 8;
// int32 slots per rank of the level parameters the fused rank kernel stages in
// LDS (the 15 fields of MixL, padded)
constexpr int kLevelInts = 16;
constexpr int kMixRtw[2 * kMaxL + 1] = {2, 3, 3, 3, 3, 2, 2, 1, 1};
// launch modes of the rank phase: one kernel per coupled rank; all ranks in
// one persistent launch with tiles round-robin; the same with tiles from a
// device work counter
enum { AP_RANK_PER_L = 0, AP_RANK_FUSED = 1, AP_RANK_FUSED_QUEUE = 2, AP_RANK_N_MODES = 3 };

struct MixL {
  int32_t nrow, nrow16, nch, arow;  // rows of X_L, padded to 16, channel rows, has A rows
  int32_t rt, ct, kt;               // row tiles (both sets), column tiles, k tiles
  int32_t kstr, zstr;               // LDS strides of the operand (fp16) and of Z (floats)
  int32_t grp0, ngrp;               // channel groups of this L
  int32_t bt0;                      // first coefficient tile of this L; tile (rt, kt) is bt0 + rt * kt_n + kt
  int32_t xonce;                    // X_L stays in LDS for both sets (Z stored beside it at zoff)
  int32_t zoff;                     // byte offset of Z within the big LDS region when xonce
  int32_t rs0;                      // first row scale of this L in MixDev::rscale (set p at rs0 + p * nrow16)
};

struct MixDev {
  int32_t n_max, l_max, K, nlm, nA, apad, nnl, L_max;
  double rc;
  const float* Wf;
  const double* ynorm;
  MixL lv[2 * kMaxL + 1];   // host copy
  const MixL* lv_d;         // device copy (indexed by L in the kernel)
  const uint4* ctile;      // dense tiles: (2 * tile + split) * 64 + lane, 8 fp16 per lane
  const float* rscale;     // per coefficient row: 2^-e, the inverse of the row's power-of-two scale
  const int32_t* grp_pat;  // pattern of each group
  const int4* grp_mem;     // 8 members per group: {row, A offset of a, A offset of b, la*5+lb}
  const int32_t* pat_hdr;  // 5 ints per pattern: la, lb, L, switch key, first coefficient
  const CgEnt* pat_ent;
  const float* pat_coef;   // coefficients per pattern over the selection-rule superset
  const int32_t* pat_off;  // first coefficient of pattern key la*45 + lb*9 + L (-1: invalid)
  const int32_t* rowtab;   // [L][a][p]: row of the coupled channel {a, p} in X_L, or -1
  const int32_t* adj_ptr;  // [L][kMixWaves + 1]: each wavefront's adjoint units
  const int4* adj_units;   // {l_t * 16 + parts * 4 + part, 0, 0, l_t}
  int32_t tab_off;             // LDS: staged channel tables of one L (rows, groups)
  int32_t big_off, big_bytes;  // LDS layout
};

struct Buffer {
  void* p = nullptr;
  size_t bytes = 0;
};

struct SysCache {
  bool valid = false;
  std::vector<int64_t> off;
  std::vector<double> box;
  uint8_t periodic[3] = {0, 0, 0};
  double cutoff = 0;
  int32_t n_cells = 0;
  int32_t n_chunks = 0;
  bool all_ortho = false;
  // device
  Buffer off_d, H_d, Hi_d, ortho_d, grid_d, cell_base_d, sys_of_d;
  Buffer chunk_lo_d, chunk_hi_d, sys_chunk_d;  // reduction chunks
};

struct Ctx {
  int device = 0;
  int precision = AP_PREC_FP64;
  std::string err;
  bool has_eam = false, has_ace = false;
  TableDev phi{}, rho{}, F{};
  bool eam_analytic = false;            // EAM in closed form (ean) instead of the tables
  EamAnalyticDev ean{};
  AceDev ace{};
  MixDev mix{};
  std::vector<Buffer> owned;            // model tables
  SysCache sys;
  // scratch, grown on demand
  Buffer cell_big, pos4;               // cell_big: [m, atoms of the cells too big for LDS]
  Buffer cell_count, cell_start, cell_cursor, cell_atoms, cell_pos, cell_of;
  Buffer scan_tmp;
  Buffer wfp, eF, wgt, vir_atom, e_tmp;
  Buffer ace_row, pair_g, ace_counter, ace_rows_list, ace_halo, nbr_ace;
  int32_t halo_stamp = 0;           // last stamp written into ace_halo (0: cleared)
  Buffer mix_A, mix_om, mix_phi;        // mixed path: A, adjoint (2 sets), phi per ACE atom
  Buffer mix_bn;                        // mixed path: largest |A_(n,l)|^2 per ACE atom (X scale)
  Buffer partials, flags;               // flags: [0] nbr overflow max count, [1] nonfinite
  Buffer ind_atom;
  Buffer nvt_ke, nvt_sums, nvt_fac;      // Nose-Hoover layer: per-atom m v^2, per-system sums, scale
  Buffer sw_csp, sw_mu0, sw_mu, sw_flag, sw_src, sw_nsrc;   // dynamic switching scratch
  Buffer e_eam_raw, e_ace_raw;          // unweighted per-atom energies of the last force calls
  int64_t cells_n_atoms = -1;           // atoms of the last neighbour build (its cell list)
  void* static_scratch = nullptr;      // this device's address of the static scratch array
  // launch mode of the mixed rank phase: forced (AP_RANK_MODE, >= 0) or tuned
  // per bucket of the atom count (timed on first use, optionally cached in
  // the JSON file named by AP_AUTOTUNE_CACHE)
  int rank_mode_forced = -1;
  std::map<int, int> rank_mode_tuned;
  std::string tune_key;                 // device and model shape, prefix of the cache keys
  std::string tune_cache;               // cache file path ("" = none)
  int last_rank_mode = -1;
  size_t ace_lds = 0;
  // set by ap_step's force evaluation, whose EAM and ACE calls see the same
  // positions: the ACE call reuses the positions the EAM call packed, and with
  // a virial the EAM call leaves its per-atom virial unreduced and the ACE call
  // adds to it and reduces both at once
  bool fused_eval = false;
  // algorithmic work counts (ap_info)
  double flops_atom = 0, flops_contract = 0, flops_bond = 0, nnz = 0, x_rows = 0;
  double mix_tiles = 0;        // stored 16x32 coefficient tiles (mixed path)
  double mix_mfma_flops = 0;   // executed MFMA FLOPs per ACE atom (3 split products)
  // per-phase event timing (ap_profile)
  bool prof = false;
  struct Ev { int phase; hipEvent_t a, b; };
  std::vector<Ev> evs;
  double prof_ms[AP_N_PHASES] = {0};
  int64_t prof_calls[AP_N_PHASES] = {0};
};

// Records a HIP event pair around a phase when profiling is on.
struct PhaseTimer {
  Ctx* c;
  int ph;
  hipStream_t s;
  hipEvent_t a = nullptr;
  PhaseTimer(Ctx* c_, int ph_, hipStream_t s_) : c(c_), ph(ph_), s(s_) {
    if (c->prof && hipEventCreate(&a) == hipSuccess) hipEventRecord(a, s);
  }
  ~PhaseTimer() {
    if (!a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) == hipSuccess) {
      hipEventRecord(b, s);
      c->evs.push_back({ph, a, b});
    }
  }
};

// error helpers (ap_api.hip)
ap_status fail(Ctx* ctx, ap_status s, const std::string& msg);
ap_status fail_hip(Ctx* ctx, hipError_t e, const char* what, const char* file, int line);
ap_status ensure(Ctx* ctx, Buffer& b, size_t bytes);

// launchers ---------------------------------------------------------------
// neighbours (k_nbr.hip)
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);
hipError_t launch_bin(const SysView& sv, const double* pos, int32_t* cell_of, int32_t* cell_count,
                      hipStream_t s);
hipError_t launch_scan_exclusive(const int32_t* in, int32_t* out, int32_t n, int32_t* tmp,
                                 hipStream_t s, int32_t* out2 = nullptr);
hipError_t launch_scatter(const SysView& sv, const double* pos, const int32_t* cell_of,
                          int32_t* cursor, int32_t* cell_atoms, double4* cell_pos, hipStream_t s);
hipError_t launch_fill_nbr_cells(const SysView& sv, int32_t n_cells, const double* pos,
                                 const int32_t* cell_of, const int32_t* cell_start,
                                 const int32_t* cell_count, const double4* cell_pos, int32_t* nbr,
                                 int32_t* count, int32_t cap, int32_t* overflow, int32_t* big_atoms,
                                 hipStream_t s);
hipError_t launch_fill_nbr(const SysView& sv, const double* pos, const int32_t* cell_of,
                           const int32_t* cell_start, const int32_t* cell_count,
                           const double4* cell_pos, int32_t* nbr, int32_t* count, int32_t cap,
                           int32_t* overflow, hipStream_t s);
hipError_t launch_rev(int32_t n_atoms, const int32_t* nbr, const int32_t* count, int32_t* rev,
                      hipStream_t s);
// switching and compaction (k_misc.hip)
hipError_t launch_blend(int32_t n, const double* pos, const ap_lambda_rule& rule, double* lambda,
                        int32_t* flag, hipStream_t s);
hipError_t launch_compact(int32_t n, const int32_t* flag, int32_t* out_list, int32_t* out_n,
                          int32_t* tmp, hipStream_t s);
hipError_t launch_seq(int32_t n, int32_t* out, hipStream_t s);
// reductions
hipError_t launch_reduce(const SysView& sv, int32_t n_chunks, const int64_t* chunk_lo,
                         const int64_t* chunk_hi, const int32_t* sys_chunk, const double* vals,
                         int32_t m, int64_t stride, double* partials, double* out, bool accumulate,
                         hipStream_t s, double* copy0 = nullptr, double* copy1 = nullptr);
// indenter / integration / checks
hipError_t launch_indenter(int32_t n, const double* pos, const uint8_t* fixed, const double* c,
                           double R, double K, const double* dir, double* force, double* e_atom2,
                           hipStream_t s);
hipError_t launch_kick_drift(int32_t n, const SysView& sv, double* pos, double* vel,
                             const double* force, const double* mass, const uint8_t* fixed,
                             const uint8_t* nvt, const double* nvt_fac, double dt, bool drift,
                             hipStream_t s);
hipError_t launch_nvt_ke(int32_t n, const double* vel, const double* mass, const uint8_t* nvt,
                         const uint8_t* fixed, double* out, hipStream_t s);
hipError_t launch_nvt_half(int32_t n_sys, double* sums, double* xi, double* fac, double T0,
                           double tau, double dt, hipStream_t s);
hipError_t launch_nvt_scale(int32_t n, const SysView& sv, double* vel, const uint8_t* nvt,
                            const uint8_t* fixed, const double* fac, hipStream_t s);
hipError_t launch_check_finite(int32_t n, const double* force, int32_t* flag, hipStream_t s);
hipError_t launch_lambda_grad(int32_t n, const double* pos, const ap_lambda_rule& rule,
                              const double* lambda, const double* e_ace, const double* e_eam,
                              double* force, double* vir_atom, hipStream_t s);
// dynamic switching (k_switch.hip)
hipError_t launch_switching(const SysView& sv, const double* pos, const int32_t* nbr,
                            const int32_t* count, int32_t cap, const int32_t* cell_of,
                            const int32_t* cell_start, const int32_t* cell_count,
                            const int32_t* cell_atoms, const double4* cell_pos,
                            const ap_switching& sw, double csp_full, double* csp, double* mu0,
                            unsigned long long* mu_bits, int32_t* flag, int32_t* src, int32_t* n_src,
                            int32_t* scan_tmp, double* lambda, int32_t* ace_list, int32_t* n_ace,
                            hipStream_t s);
// EAM (k_eam.hip)
hipError_t launch_pack_pos(int32_t n, const double* pos, double4* p4, hipStream_t s);
hipError_t launch_eam(const Ctx& c, const SysView& sv, const double* pos, const double4* pos4,
                      const int32_t* nbr,
                      const int32_t* count, int32_t n_atoms, const double* lambda, double* wfp,
                      double* eF, double* wgt, double* e_atom, double* force, double* vir_atom,
                      bool accumulate, double* e_raw, hipStream_t s);
// ACE (k_ace.hip)
size_t ace_lds_bytes(const AceDev& a, int precision);
hipError_t launch_ace_reset(int32_t* counter, hipStream_t s);
hipError_t launch_ace(const Ctx& c, const SysView& sv, const double* pos, const double4* pos4,
                      const int32_t* nbr,
                      const int32_t* count, int32_t cap, int32_t n_atoms, const double* lambda,
                      const int32_t* ace_list, const int32_t* n_ace, int32_t* ace_row,
                      int32_t* counter, void* pair_g, double* e_atom, double* vir_atom,
                      double* e_raw, int32_t* nbr_ace, int32_t* halo, int32_t stamp,
                      bool vir_acc, hipStream_t s);
// phase 0: bond basis -> A (and the listed atoms' rows, atom-major, ->
// nbr_ace; the listed atoms and their neighbours stamped in halo); 1:
// coupling/contraction/adjoint -> om, phi; 2: embedding, bond gradients, virial
hipError_t launch_ace_mixed(const Ctx& c, const SysView& sv, const double* pos, const double4* pos4,
                            const int32_t* nbr,
                            const int32_t* count, int32_t cap, int32_t n_atoms, const double* lambda,
                            const int32_t* ace_list, const int32_t* n_ace, int32_t* counter,
                            float* pair_g, float* A_buf, float* om_buf, float* phi_buf,
                            float* bn_buf, double* e_atom, double* vir_atom, hipStream_t s,
                            int phase, int rank_mode, double* e_raw, int32_t* nbr_ace,
                            int32_t* halo, int32_t stamp, bool vir_acc);
size_t ace_mixed_lds_bytes(const MixDev& m);
// the rank kernel of coupled rank L (k_ace_rank.hip, one translation unit
// per L); xo: the variant that keeps X_L in LDS for both coefficient sets
template <int L>
const void* rank_kernel(bool xo);
// all coupled ranks in one persistent launch (k_ace_rank_fused.hip) for the
// rank layout (bit L of xomask: X_L kept for both sets; lmax: largest rank),
// or NULL when no instance exists for that layout; queue: tiles from the
// device work counter instead of round-robin
const void* rank_kernel_fused(bool queue, uint32_t xomask, int lmax);
uint32_t rank_xomask(const MixDev& m);
hipError_t launch_ace_gather(const Ctx& c, int32_t n_atoms, const int32_t* nbr, const int32_t* count,
                             const int32_t* rev, const int32_t* nbr_ace, int32_t cap,
                             const int32_t* ace_row, const int32_t* halo, int32_t stamp,
                             const void* pair_g, double* force, bool accumulate, hipStream_t s);
hipError_t launch_ace_rows(int32_t n_atoms, const int32_t* ace_list, const int32_t* n_ace,
                           int32_t* ace_row, hipStream_t s);

}  // namespace ap
