// Host side of the AP library: the extern "C" entry points of include/ap.h,
// argument validation, model folding (coupling coefficients, folded
// coefficient matrices, adjoint lists), system geometry, scratch management.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <map>
#include <mutex>
#include <tuple>

#include "ap_internal.h"

namespace ap {

static thread_local std::string g_create_err;

// --------------------------------------------------------------------------
// Static device scratch of the entry point that allocates nothing
// (ap_blend_noalloc): the per-atom flags of the switching pass and the
// partial sums of the compaction scan.  Every GPU the library runs on holds
// its own copy of this array until the process ends.  In host code the name
// only stands in for the device symbol; host code uses the address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device when the first context on that device is created.
constexpr int64_t kNoallocMaxAtoms = AP_BLEND_NOALLOC_MAX_ATOMS;
constexpr size_t kNoallocFlagBytes = (size_t)4 * kNoallocMaxAtoms;            // int32 per atom
constexpr size_t kNoallocScanBytes = (size_t)4 * (kNoallocMaxAtoms / 4096 + 2);  // scan partial sums
constexpr size_t kStaticScratchBytes = kNoallocFlagBytes + 256 + kNoallocScanBytes;
static_assert(kNoallocFlagBytes % 256 == 0, "scan sums start 256-byte aligned");
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

ap_status fail(Ctx* ctx, ap_status s, const std::string& msg) {
  if (ctx) ctx->err = msg; else g_create_err = msg;
  return s;
}

ap_status fail_hip(Ctx* ctx, hipError_t e, const char* what, const char* file, int line) {
  char buf[512];
  snprintf(buf, sizeof buf, "HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what,
           file, line);
  return fail(ctx, e == hipErrorOutOfMemory ? AP_ERR_NOMEM : AP_ERR_HIP, buf);
}

ap_status ensure(Ctx* ctx, Buffer& b, size_t bytes) {
  if (bytes <= b.bytes && b.p) return AP_OK;
  if (b.p) {
    AP_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, 256);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    b.p = nullptr;
    return fail_hip(ctx, e, "hipMalloc(scratch)", __FILE__, __LINE__);
  }
  b.bytes = want;
  return AP_OK;
}

static void release(Buffer& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

template <typename T>
static ap_status upload(Ctx* ctx, Buffer& b, const std::vector<T>& v) {
  ap_status st = ensure(ctx, b, std::max<size_t>(1, v.size()) * sizeof(T));
  if (st != AP_OK) return st;
  if (!v.empty()) AP_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return AP_OK;
}

template <typename T>
static ap_status upload_owned(Ctx* ctx, const std::vector<T>& v, const T** out) {
  ctx->owned.emplace_back();
  ap_status st = upload(ctx, ctx->owned.back(), v);
  *out = (const T*)ctx->owned.back().p;
  return st;
}

// --------------------------------------------------------------------------
// box geometry (scalar FP64, no contraction: the inverse must equal the
// cofactor formula bit for bit)
static void box_inverse(const double* H, double* Hi) {
#pragma clang fp contract(off)
  const double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7],
               i = H[8];
  const double det = a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
  Hi[0] = (e * i - f * h) / det;
  Hi[1] = (c * h - b * i) / det;
  Hi[2] = (b * f - c * e) / det;
  Hi[3] = (f * g - d * i) / det;
  Hi[4] = (a * i - c * g) / det;
  Hi[5] = (c * d - a * f) / det;
  Hi[6] = (d * h - e * g) / det;
  Hi[7] = (b * g - a * h) / det;
  Hi[8] = (a * e - b * d) / det;
}

static ap_status prepare_systems(Ctx* ctx, const ap_systems* sys, SysView* sv) {
  if (!sys) return fail(ctx, AP_ERR_ARG, "sys is NULL");
  if (sys->n_systems < 1 || sys->n_systems > kMaxSys) return fail(ctx, AP_ERR_ARG, "n_systems out of range");
  if (sys->n_atoms < 0 || sys->n_atoms > (int64_t)INT32_MAX / 2)
    return fail(ctx, AP_ERR_ARG, "n_atoms out of range");
  if (!sys->sys_offset || !sys->box) return fail(ctx, AP_ERR_ARG, "sys_offset/box is NULL");
  if (!(sys->cutoff > 0.0) || !std::isfinite(sys->cutoff)) return fail(ctx, AP_ERR_ARG, "cutoff must be > 0");
  const int ns = sys->n_systems;
  SysCache& C = ctx->sys;
  bool same = C.valid && (int)C.off.size() == ns + 1 && C.cutoff == sys->cutoff &&
              !memcmp(C.periodic, sys->periodic, 3) &&
              !memcmp(C.off.data(), sys->sys_offset, sizeof(int64_t) * (ns + 1)) &&
              !memcmp(C.box.data(), sys->box, sizeof(double) * 9 * ns);
  if (!same) {
    C.valid = false;
    if (sys->sys_offset[0] != 0 || sys->sys_offset[ns] != sys->n_atoms)
      return fail(ctx, AP_ERR_ARG, "sys_offset must run from 0 to n_atoms");
    for (int s = 0; s < ns; ++s)
      if (sys->sys_offset[s + 1] < sys->sys_offset[s]) return fail(ctx, AP_ERR_ARG, "sys_offset not monotone");
    const double rc = sys->cutoff;
    std::vector<double> Hi(9 * ns, 0.0);
    std::vector<uint8_t> ortho(ns);
    std::vector<int32_t> grid(3 * ns), base(ns + 1, 0);
    int64_t cells = 0;
    for (int s = 0; s < ns; ++s) {
      const double* H = sys->box + 9 * s;
      for (int k = 0; k < 9; ++k)
        if (!std::isfinite(H[k])) return fail(ctx, AP_ERR_BOX, "box has non-finite entries");
      const bool o = H[1] == 0 && H[2] == 0 && H[3] == 0 && H[5] == 0 && H[6] == 0 && H[7] == 0;
      ortho[s] = o;
      double width[3];
      if (o) {
        for (int k = 0; k < 3; ++k) {
          width[k] = H[4 * k];
          if (!(width[k] > 0)) return fail(ctx, AP_ERR_BOX, "box diagonal must be positive");
        }
      } else {
        if (!(sys->periodic[0] && sys->periodic[1] && sys->periodic[2]))
          return fail(ctx, AP_ERR_UNSUPPORTED, "triclinic boxes must be periodic in x, y and z");
        const double* a = H;
        const double* b = H + 3;
        const double* c = H + 6;
        auto cross = [](const double* u, const double* v, double* w) {
          w[0] = u[1] * v[2] - u[2] * v[1];
          w[1] = u[2] * v[0] - u[0] * v[2];
          w[2] = u[0] * v[1] - u[1] * v[0];
        };
        double bc[3], ca[3], ab[3];
        cross(b, c, bc);
        cross(c, a, ca);
        cross(a, b, ab);
        const double vol = std::fabs(a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2]);
        if (!(vol > 0)) return fail(ctx, AP_ERR_BOX, "degenerate box");
        width[0] = vol / std::sqrt(bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
        width[1] = vol / std::sqrt(ca[0] * ca[0] + ca[1] * ca[1] + ca[2] * ca[2]);
        width[2] = vol / std::sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
        box_inverse(H, &Hi[9 * s]);
      }
      for (int k = 0; k < 3; ++k) {
        if (sys->periodic[k] && width[k] < 2.0 * rc)
          return fail(ctx, AP_ERR_BOX, "a periodic cell is narrower than twice the cutoff");
        int g = (int)std::floor(width[k] / (rc * (1.0 + 1e-9)));
        grid[3 * s + k] = std::max(1, std::min(g, 1024));
      }
      cells += (int64_t)grid[3 * s] * grid[3 * s + 1] * grid[3 * s + 2];
      if (cells > (1 << 28)) return fail(ctx, AP_ERR_BOX, "too many cells");
      base[s + 1] = (int32_t)cells;
    }
    std::vector<int32_t> sys_of(sys->n_atoms);
    std::vector<int64_t> lo, hi;
    std::vector<int32_t> sc(ns + 1, 0);
    for (int s = 0; s < ns; ++s) {
      for (int64_t i = sys->sys_offset[s]; i < sys->sys_offset[s + 1]; ++i) sys_of[i] = s;
      for (int64_t a = sys->sys_offset[s]; a < sys->sys_offset[s + 1]; a += kReduceChunk) {
        lo.push_back(a);
        hi.push_back(std::min<int64_t>(a + kReduceChunk, sys->sys_offset[s + 1]));
      }
      sc[s + 1] = (int32_t)lo.size();
    }
    std::vector<int64_t> off(sys->sys_offset, sys->sys_offset + ns + 1);
    std::vector<double> box(sys->box, sys->box + 9 * ns);
    ap_status st;
    if ((st = upload(ctx, C.off_d, off)) || (st = upload(ctx, C.H_d, box)) ||
        (st = upload(ctx, C.Hi_d, Hi)) || (st = upload(ctx, C.ortho_d, ortho)) ||
        (st = upload(ctx, C.grid_d, grid)) || (st = upload(ctx, C.cell_base_d, base)) ||
        (st = upload(ctx, C.sys_of_d, sys_of)) || (st = upload(ctx, C.chunk_lo_d, lo)) ||
        (st = upload(ctx, C.chunk_hi_d, hi)) || (st = upload(ctx, C.sys_chunk_d, sc)))
      return st;
    C.off = off;
    C.box = box;
    memcpy(C.periodic, sys->periodic, 3);
    C.cutoff = sys->cutoff;
    C.n_cells = (int32_t)cells;
    C.n_chunks = (int32_t)lo.size();
    C.all_ortho = std::all_of(ortho.begin(), ortho.end(), [](uint8_t o) { return o != 0; });
    C.valid = true;
  }
  sv->n_sys = ns;
  sv->n_atoms = (int32_t)sys->n_atoms;
  sv->off = (const int64_t*)C.off_d.p;
  sv->H = (const double*)C.H_d.p;
  sv->Hi = (const double*)C.Hi_d.p;
  sv->ortho = (const uint8_t*)C.ortho_d.p;
  sv->grid = (const int32_t*)C.grid_d.p;
  sv->cell_base = (const int32_t*)C.cell_base_d.p;
  sv->sys_of = (const int32_t*)C.sys_of_d.p;
  for (int k = 0; k < 3; ++k) sv->per[k] = sys->periodic[k] ? 1 : 0;
  sv->all_ortho = C.all_ortho ? 1 : 0;
  sv->rc2 = sys->cutoff * sys->cutoff;
  return AP_OK;
}

// --------------------------------------------------------------------------
// Clebsch-Gordan coefficients: Racah's closed form (complex basis), then the
// change of basis to the real harmonics of ace_basis.h.
static double fact(int n) {
  static double f[41] = {0};
  if (f[0] == 0) {
    f[0] = 1;
    for (int k = 1; k <= 40; ++k) f[k] = f[k - 1] * k;
  }
  return f[n];
}

static double cg_complex(int j1, int m1, int j2, int m2, int J, int M) {
  if (m1 + m2 != M || std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(M) > J) return 0.0;
  if (J < std::abs(j1 - j2) || J > j1 + j2) return 0.0;
  const double pre = (2 * J + 1) * fact(J + j1 - j2) * fact(J - j1 + j2) * fact(j1 + j2 - J) /
                     fact(j1 + j2 + J + 1) * fact(J + M) * fact(J - M) * fact(j1 - m1) *
                     fact(j1 + m1) * fact(j2 - m2) * fact(j2 + m2);
  double sum = 0.0;
  for (int k = 0; k <= j1 + j2 - J; ++k) {
    const int a[6] = {k, j1 + j2 - J - k, j1 - m1 - k, j2 + m2 - k, J - j2 + m1 + k, J - j1 - m2 + k};
    bool ok = true;
    double den = 1.0;
    for (int t = 0; t < 6; ++t) {
      if (a[t] < 0) { ok = false; break; }
      den *= fact(a[t]);
    }
    if (ok) sum += ((k & 1) ? -1.0 : 1.0) / den;
  }
  return std::sqrt(pre) * sum;
}

using cplx = std::complex<double>;
// U[m][mu] (offset by l): real Y_m = sum_mu U[m][mu] Y^mu
static std::vector<cplx> umat(int l) {
  const int w = 2 * l + 1;
  std::vector<cplx> U(w * w, 0.0);
  const double s = 1.0 / std::sqrt(2.0);
  for (int m = -l; m <= l; ++m) {
    const int r = m + l;
    if (m == 0) {
      U[r * w + l] = 1.0;
    } else if (m > 0) {
      U[r * w + m + l] = ((m & 1) ? -1.0 : 1.0) * s;
      U[r * w - m + l] = s;
    } else {
      const int k = -m;
      U[r * w + k + l] = cplx(0.0, -((k & 1) ? -1.0 : 1.0) * s);
      U[r * w - k + l] = cplx(0.0, s);
    }
  }
  return U;
}

// real coupling tensor C[(m1+l1)][(m2+l2)][(M+L)]
static bool real_cg(int l1, int l2, int L, std::vector<double>& out) {
  const int w1 = 2 * l1 + 1, w2 = 2 * l2 + 1, wL = 2 * L + 1;
  auto U1 = umat(l1), U2 = umat(l2), UL = umat(L);
  out.assign((size_t)w1 * w2 * wL, 0.0);
  for (int a = 0; a < w1; ++a)
    for (int b = 0; b < w2; ++b)
      for (int c = 0; c < wL; ++c) {
        cplx acc = 0.0;
        for (int mu1 = -l1; mu1 <= l1; ++mu1) {
          const cplx u1 = std::conj(U1[a * w1 + mu1 + l1]);
          if (u1 == 0.0) continue;
          for (int mu2 = -l2; mu2 <= l2; ++mu2) {
            const int mu = mu1 + mu2;
            if (std::abs(mu) > L) continue;
            const cplx u2 = std::conj(U2[b * w2 + mu2 + l2]);
            const cplx uL = UL[c * wL + mu + L];
            if (u2 == 0.0 || uL == 0.0) continue;
            acc += uL * u1 * u2 * cg_complex(l1, mu1, l2, mu2, L, mu);
          }
        }
        if (std::fabs(acc.imag()) > 1e-12) return false;
        out[((size_t)a * w2 + b) * wL + c] = std::fabs(acc.real()) < 1e-15 ? 0.0 : acc.real();
      }
  return true;
}

// --------------------------------------------------------------------------
static ap_status fold_ace(Ctx* ctx, const ap_ace_model* m) {
  const int nmax = m->n_max, lmax = m->l_max, K = m->K;
  if (lmax < 0 || lmax > kMaxL) return fail(ctx, AP_ERR_ARG, "ACE l_max must be in [0, 4]");
  if (nmax < 1 || nmax > kMaxN) return fail(ctx, AP_ERR_ARG, "ACE n_max must be in [1, 16]");
  if (K < 1 || K > kMaxK) return fail(ctx, AP_ERR_ARG, "ACE K must be in [1, 16]");
  if (m->nu_max < 1 || m->nu_max > 4) return fail(ctx, AP_ERR_ARG, "ACE nu_max must be in [1, 4]");
  if (!(m->r_c > 0)) return fail(ctx, AP_ERR_ARG, "ACE r_c must be > 0");
  if (m->n_funcs < 0 || (m->n_funcs > 0 && (!m->funcs || !m->c1 || !m->c2)) || !m->W)
    return fail(ctx, AP_ERR_ARG, "ACE model arrays missing");
  const int lp1 = lmax + 1, nlm = lp1 * lp1, nA = nmax * nlm;
  AceDev& a = ctx->ace;
  a.n_max = nmax;
  a.l_max = lmax;
  a.K = K;
  a.nlm = nlm;
  a.nA = nA;
  a.nnl = nmax * lp1;
  a.rc = m->r_c;
  // normalisation of the real harmonics (sqrt2 folded in for m > 0)
  std::vector<double> yn(nlm, 0.0);
  for (int l = 0; l <= lmax; ++l)
    for (int mm = 0; mm <= l; ++mm) {
      double v = std::sqrt((2 * l + 1) / (4.0 * M_PI) * fact(l - mm) / fact(l + mm));
      yn[l * l + l + mm] = mm ? std::sqrt(2.0) * v : v;
    }
  std::vector<double> W(m->W, m->W + (size_t)nmax * lp1 * K);
  std::vector<float> Wf(W.begin(), W.end());
  ap_status st;
  if ((st = upload_owned(ctx, yn, &a.ynorm)) || (st = upload_owned(ctx, W, &a.W)) ||
      (st = upload_owned(ctx, Wf, &a.Wf)))
    return st;

  // channels (a <= b, L) used by the function list
  auto sidx = [&](int n, int l) { return n * lp1 + l; };
  auto ok_nl = [&](int n, int l) { return n >= 0 && n < nmax && l >= 0 && l <= lmax; };
  auto coupl = [](int l1, int l2, int L) { return std::abs(l1 - l2) <= L && L <= l1 + l2 && ((l1 + l2 + L) % 2 == 0); };
  std::map<std::tuple<int, int, int>, int> chan;  // (L, a, b) -> row
  struct Term { int L, r1, r2; double c1, c2; };
  std::vector<std::tuple<int, int, int, int, int, int, double, double>> raw;  // kind data
  auto chan_key = [&](int n1, int l1, int n2, int l2, int L) {
    int x = sidx(n1, l1), y = sidx(n2, l2);
    if (x > y) std::swap(x, y);
    chan[{L, x, y}] = 0;
    return std::make_tuple(L, x, y);
  };
  const int32_t* F = m->funcs;
  int Lmax = lmax;
  for (int v = 0; v < m->n_funcs; ++v) {
    const int32_t* f = F + 10 * v;
    const int nu = f[0];
    if (nu < 1 || nu > m->nu_max) return fail(ctx, AP_ERR_ARG, "ACE function has invalid nu");
    for (int k = 0; k < nu; ++k)
      if (!ok_nl(f[1 + 2 * k], f[2 + 2 * k])) return fail(ctx, AP_ERR_ARG, "ACE function index out of range");
    if (nu == 1 && f[2] != 0) return fail(ctx, AP_ERR_ARG, "nu=1 function needs l=0");
    if (nu == 2 && f[2] != f[4]) return fail(ctx, AP_ERR_ARG, "nu=2 function needs equal l");
    if (nu == 3 && (f[9] != f[6] || !coupl(f[2], f[4], f[9])))
      return fail(ctx, AP_ERR_ARG, "nu=3 function: L must equal l3 and couple (l1, l2) with an even sum");
    if (nu == 4 && (!coupl(f[2], f[4], f[9]) || !coupl(f[6], f[8], f[9])))
      return fail(ctx, AP_ERR_ARG, "nu=4 function: L must couple (l1,l2) and (l3,l4) with even sums");
    if (nu == 2) chan_key(f[1], f[2], f[3], f[4], 0);
    if (nu == 3) chan_key(f[1], f[2], f[3], f[4], f[9]);
    if (nu == 4) {
      chan_key(f[1], f[2], f[3], f[4], f[9]);
      chan_key(f[5], f[6], f[7], f[8], f[9]);
    }
    if (nu >= 3) Lmax = std::max(Lmax, (int)f[9]);
  }
  a.L_max = Lmax;
  int nch[2 * kMaxL + 1] = {0};
  for (auto& kv : chan) kv.second = nch[std::get<0>(kv.first)]++;
  int max_xsize = 0;
  for (int L = 0; L <= Lmax; ++L) {
    a.nch[L] = nch[L];
    a.has_arow[L] = L <= lmax ? 1 : 0;
    a.nrow[L] = nch[L] + (L <= lmax ? nmax : 0) + (L == 0 ? 1 : 0);
    max_xsize = std::max(max_xsize, a.nrow[L] * (2 * L + 1));
  }
  a.max_xsize = max_xsize;
  auto arow = [&](int n, int L) { return nch[L] + n; };
  auto one_row = [&]() { return nch[0] + nmax; };

  // X-building CSR and adjoint lists per L
  std::vector<int32_t> xb_ptr, ad_ptr;
  std::vector<PairTerm> xb_t, ad_t;
  std::map<std::tuple<int, int, int>, std::vector<double>> cgcache;
  for (int L = 0; L <= Lmax; ++L) {
    const int w = 2 * L + 1;
    a.xb_off[L] = (int32_t)xb_ptr.size();
    std::vector<std::vector<std::tuple<int, int, double>>> rows(nch[L] * w);
    std::vector<std::vector<std::tuple<int, int, double>>> adj(nA);
    for (auto& kv : chan) {
      if (std::get<0>(kv.first) != L) continue;
      const int x = std::get<1>(kv.first), y = std::get<2>(kv.first);
      const int n1 = x / lp1, l1 = x % lp1, n2 = y / lp1, l2 = y % lp1;
      auto key = std::make_tuple(l1, l2, L);
      if (!cgcache.count(key)) {
        std::vector<double> c;
        if (!real_cg(l1, l2, L, c)) return fail(ctx, AP_ERR_ARG, "complex coupling coefficient");
        cgcache[key] = c;
      }
      const auto& C = cgcache[key];
      const int w1 = 2 * l1 + 1, w2 = 2 * l2 + 1;
      for (int M = 0; M < w; ++M)
        for (int p = 0; p < w1; ++p)
          for (int q = 0; q < w2; ++q) {
            const double c = C[((size_t)p * w2 + q) * w + M];
            if (c == 0.0) continue;
            const int s1 = n1 * nlm + l1 * l1 + p, s2 = n2 * nlm + l2 * l2 + q;
            const int dst = kv.second * w + M;
            rows[dst].emplace_back(s1, s2, c);
            adj[s1].emplace_back(dst, s2, c);
            adj[s2].emplace_back(dst, s1, c);
          }
    }
    xb_ptr.push_back((int32_t)xb_t.size());
    for (auto& r : rows) {
      for (auto& t : r) xb_t.push_back(PairTerm{std::get<2>(t), std::get<0>(t), std::get<1>(t)});
      xb_ptr.push_back((int32_t)xb_t.size());
    }
    a.ad_off[L] = (int32_t)ad_ptr.size();
    ad_ptr.push_back((int32_t)ad_t.size());
    for (auto& r : adj) {
      for (auto& t : r) ad_t.push_back(PairTerm{std::get<2>(t), std::get<1>(t), std::get<0>(t)});
      ad_ptr.push_back((int32_t)ad_t.size());
    }
  }
  // folded coefficient matrices: phi^(p) = 1/2 sum_L sum_M X_L[:,M]^T C_L^(p) X_L[:,M]
  std::vector<std::map<std::pair<int, int>, std::pair<double, double>>> Cm(Lmax + 1);
  auto add = [&](int L, int r, int c, double v1, double v2) {
    auto& e = Cm[L][{r, c}];
    e.first += v1;
    e.second += v2;
  };
  auto sym = [&](int L, int r, int c, double v1, double v2) {
    if (r == c) {
      add(L, r, r, 2 * v1, 2 * v2);
    } else {
      add(L, r, c, v1, v2);
      add(L, c, r, v1, v2);
    }
  };
  auto ch = [&](int n1, int l1, int n2, int l2, int L) {
    int x = sidx(n1, l1), y = sidx(n2, l2);
    if (x > y) std::swap(x, y);
    return chan[{L, x, y}];
  };
  for (int v = 0; v < m->n_funcs; ++v) {
    const int32_t* f = F + 10 * v;
    const double c1 = m->c1[v], c2 = m->c2[v];
    switch (f[0]) {
      case 1: sym(0, arow(f[1], 0), one_row(), c1, c2); break;
      case 2: sym(0, ch(f[1], f[2], f[3], f[4], 0), one_row(), c1, c2); break;
      case 3: sym(f[9], ch(f[1], f[2], f[3], f[4], f[9]), arow(f[5], f[9]), c1, c2); break;
      case 4: sym(f[9], ch(f[1], f[2], f[3], f[4], f[9]), ch(f[5], f[6], f[7], f[8], f[9]), c1, c2); break;
    }
  }
  std::vector<int32_t> cx_ptr, cx_col;
  std::vector<double2> cx_val;
  for (int L = 0; L <= Lmax; ++L) {
    a.cx_off[L] = (int32_t)cx_ptr.size();
    std::vector<std::vector<std::pair<int, std::pair<double, double>>>> rows(a.nrow[L]);
    for (auto& kv : Cm[L]) rows[kv.first.first].push_back({kv.first.second, kv.second});
    cx_ptr.push_back((int32_t)cx_col.size());
    for (auto& r : rows) {
      for (auto& t : r) {
        cx_col.push_back(t.first);
        cx_val.push_back(make_double2(t.second.first, t.second.second));
      }
      cx_ptr.push_back((int32_t)cx_col.size());
    }
  }
  if ((st = upload_owned(ctx, xb_ptr, &a.xb_ptr)) || (st = upload_owned(ctx, xb_t, &a.xb_t)) ||
      (st = upload_owned(ctx, ad_ptr, &a.ad_ptr)) || (st = upload_owned(ctx, ad_t, &a.ad_t)) ||
      (st = upload_owned(ctx, cx_ptr, &a.cx_ptr)) || (st = upload_owned(ctx, cx_col, &a.cx_col)) ||
      (st = upload_owned(ctx, cx_val, &a.cx_val)))
    return st;
  {
    double contract = 0, xrows = 0;
    for (int L = 0; L <= Lmax; ++L) {
      const int w = 2 * L + 1;
      const int nnzL = cx_ptr[a.cx_off[L] + a.nrow[L]] - cx_ptr[a.cx_off[L]];
      contract += 4.0 * nnzL * w + 4.0 * a.nrow[L] * w;
      xrows += a.nrow[L];
    }
    ctx->flops_contract = contract;
    ctx->flops_atom = contract + 3.0 * xb_t.size() + 5.0 * ad_t.size();
    ctx->nnz = (double)cx_col.size();
    ctx->x_rows = xrows;
    ctx->flops_bond = 12.0 * K + 6.0 * a.nnl * K + 6.0 * nA + 20.0 * nlm + 40.0;
  }
  ctx->ace_lds = ace_lds_bytes(a, ctx->precision);
  if (ctx->precision == AP_PREC_FP64) {
    if (ctx->ace_lds > 160 * 1024) return fail(ctx, AP_ERR_UNSUPPORTED, "ACE model too large for LDS");
    return AP_OK;
  }

  // ---- mixed path: dense split-fp16 tiles with power-of-two row scales, channel groups
  MixDev& x = ctx->mix;
  x.n_max = nmax; x.l_max = lmax; x.K = K; x.nlm = nlm; x.nA = nA; x.nnl = a.nnl;
  x.apad = nA | 1;
  x.L_max = Lmax;
  x.rc = m->r_c;
  x.Wf = a.Wf;
  x.ynorm = a.ynorm;
  double mfma_flops = 0;
  std::vector<int32_t> pat_off(225, -1);

  std::vector<int32_t> grp_pat, pat_hdr;
  std::vector<int4> grp_mem;
  std::vector<CgEnt> pat_ent;
  std::vector<float> pat_coef;
  auto rule = [](int m1, int m2, int M) {
    return ((M < 0) == ((m1 < 0) != (m2 < 0))) &&
           (std::abs(M) == std::abs(m1) + std::abs(m2) || std::abs(M) == std::abs(std::abs(m1) - std::abs(m2)));
  };
  std::vector<uint4> ctile;
  std::map<std::tuple<int, int, int>, int> pat_id;
  size_t big = (size_t)4 * 64 * (a.nnl + nlm) * 4;
  std::vector<size_t> xbytes(Lmax + 1, 0), zbytes(Lmax + 1, 0);
  // fp16 round-to-nearest-even of a float and back
  auto f16_bits = [](float f) -> uint16_t {
    const _Float16 h = (_Float16)f;
    uint16_t u;
    memcpy(&u, &h, 2);
    return u;
  };
  auto f16_val = [](uint16_t b) -> float {
    _Float16 h;
    memcpy(&h, &b, 2);
    return (float)h;
  };
  std::vector<float> rscale;
  // coupling coefficients of every valid (la, lb, L), over the selection-rule
  // superset in (m1, m2, M) order, addressed by key la*45 + lb*9 + L
  for (int la = 0; la <= lmax; ++la)
    for (int lb = 0; lb <= lmax; ++lb)
      for (int L = std::abs(la - lb); L <= std::min(la + lb, Lmax); ++L) {
        if ((la + lb + L) & 1) continue;
        auto key = std::make_tuple(la, lb, L);
        if (!cgcache.count(key)) {
          std::vector<double> c;
          if (!real_cg(la, lb, L, c)) return fail(ctx, AP_ERR_ARG, "complex coupling coefficient");
          cgcache[key] = c;
        }
        const auto& C = cgcache[key];
        const int w1 = 2 * la + 1, w2 = 2 * lb + 1, w = 2 * L + 1;
        pat_off[la * 45 + lb * 9 + L] = (int32_t)pat_coef.size();
        for (int p = 0; p < w1; ++p)
          for (int q = 0; q < w2; ++q)
            for (int M = 0; M < w; ++M) {
              const double c = C[((size_t)p * w2 + q) * w + M];
              if (rule(p - la, q - lb, M - L)) {
                pat_coef.push_back((float)c);
              } else if (c != 0.0) {
                return fail(ctx, AP_ERR_ARG, "coupling coefficient outside the selection rule");
              }
            }
      }
  // channel rows by unordered pair, for the adjoint gather
  const int nidx = nmax * lp1;
  std::vector<int32_t> rowtab((size_t)(Lmax + 1) * nidx * nidx, -1);
  for (auto& kv : chan) {
    const int L = std::get<0>(kv.first), xa = std::get<1>(kv.first), xb = std::get<2>(kv.first);
    rowtab[((size_t)L * nidx + xa) * nidx + xb] = kv.second;
    rowtab[((size_t)L * nidx + xb) * nidx + xa] = kv.second;
  }
  for (int L = 0; L <= Lmax; ++L) {
    MixL& P = x.lv[L];
    const int w = 2 * L + 1;
    P.nrow = a.nrow[L];
    P.nrow16 = (P.nrow + 15) / 16 * 16;
    P.nch = nch[L];
    P.arow = a.has_arow[L];
    const int kpad = (P.nrow + 31) / 32 * 32;
    P.kt = kpad / 32;
    // column stride of the operand in LDS: kpad/2 is a multiple of 16 dwords,
    // so the stride is 4 or 20 dwords mod 32 banks (an odd multiple of 4) and
    // the 16-byte operand reads of 8 consecutive columns hit distinct banks
    P.kstr = kpad + 8;
    P.ct = (8 * w + 15) / 16;
    P.rt = 2 * P.nrow16 / 16;
    P.zstr = 8 * w + 1;
    if ((P.nrow16 / 16 + kMixWaves - 1) / kMixWaves > kMixRtw[L] || P.ct != L + 1 || nmax > 8)
      return fail(ctx, AP_ERR_UNSUPPORTED, "ACE model outside the mixed kernels' tiling (n_max <= 8, rows per rank)");
    xbytes[L] = ((size_t)P.ct * 16 * P.kstr * 2 * 2 + 15) / 16 * 16;
    zbytes[L] = (size_t)P.nrow * P.zstr * 4;
    big = std::max(big, xbytes[L]);
    big = std::max(big, zbytes[L]);
    // dense folded matrix of this L (both sets)
    std::vector<double> D((size_t)P.nrow * P.nrow * 2, 0.0);
    for (auto& kv : Cm[L]) {
      D[((size_t)kv.first.first * P.nrow + kv.first.second) * 2] = kv.second.first;
      D[((size_t)kv.first.first * P.nrow + kv.first.second) * 2 + 1] = kv.second.second;
    }
    P.bt0 = (int32_t)(ctile.size() / 128);
    // each row of each set is scaled by 2^e so that its largest entry lies
    // in [2^12, 2^13): the fp16 hi/lo pieces then keep 22 significant bits of
    // every entry that matters and no product overflows; the kernel
    // multiplies the row's results by 2^-e (exact)
    P.rs0 = (int32_t)rscale.size();
    std::vector<int> rexp(2 * P.nrow16, 0);
    for (int p = 0; p < 2; ++p)
      for (int rr = 0; rr < P.nrow16; ++rr) {
        double mx = 0.0;
        if (rr < P.nrow)
          for (int k = 0; k < P.nrow; ++k) mx = std::max(mx, std::fabs(D[((size_t)rr * P.nrow + k) * 2 + p]));
        int ex = 0;
        if (mx > 0.0) (void)std::frexp((double)(float)mx, &ex);
        rexp[p * P.nrow16 + rr] = mx > 0.0 ? 13 - ex : 0;
        rscale.push_back(std::ldexp(1.0f, -rexp[p * P.nrow16 + rr]));
      }
    for (int rt = 0; rt < P.rt; ++rt) {
      for (int kt = 0; kt < P.kt; ++kt) {
        double v[16][32];
        bool any = false;
        for (int i = 0; i < 16; ++i)
          for (int kk = 0; kk < 32; ++kk) {
            const int r = rt * 16 + i, k = kt * 32 + kk;
            const int p = r / P.nrow16, rr = r % P.nrow16;
            double val = 0.0;
            if (rr < P.nrow && k < P.nrow) val = D[((size_t)rr * P.nrow + k) * 2 + p];
            v[i][kk] = std::ldexp(val, rexp[r]);
            any = any || val != 0.0;
          }
        (void)any;  // all tiles are stored (the folded matrices are almost dense)
        mfma_flops += 3.0 * 2.0 * 16 * 16 * 32 * P.ct / 8.0;  // per atom (tile of 8 atoms)
        const int idx = (int)(ctile.size() / 128);
        ctile.resize(ctile.size() + 128);
        for (int lane = 0; lane < 64; ++lane) {
          uint16_t hi[8], lo[8];
          for (int j = 0; j < 8; ++j) {
            const double val = v[lane % 16][8 * (lane / 16) + j];
            hi[j] = f16_bits((float)val);
            lo[j] = f16_bits((float)(val - (double)f16_val(hi[j])));
          }
          uint4 h4, l4;
          memcpy(&h4, hi, 16);
          memcpy(&l4, lo, 16);
          ctile[(size_t)idx * 128 + lane] = h4;
          ctile[(size_t)idx * 128 + 64 + lane] = l4;
        }
      }
    }
    // channel groups of equal (la, lb)
    std::map<std::pair<int, int>, std::vector<int4>> by_pat;
    for (auto& kv : chan) {
      if (std::get<0>(kv.first) != L) continue;
      const int xa = std::get<1>(kv.first), xb = std::get<2>(kv.first);
      const int na = xa / lp1, la = xa % lp1, nb = xb / lp1, lb = xb % lp1;
      by_pat[{la, lb}].push_back(make_int4(kv.second, na * nlm + la * la, nb * nlm + lb * lb, la * 5 + lb));
    }
    P.grp0 = (int32_t)grp_pat.size();
    for (auto& kv : by_pat) {
      const int la = kv.first.first, lb = kv.first.second;
      auto key = std::make_tuple(la, lb, L);
      if (!pat_id.count(key)) {
        const auto& C = cgcache[key];
        const int e0 = (int)pat_ent.size();
        const int w1 = 2 * la + 1, w2 = 2 * lb + 1;
        for (int M = 0; M < w; ++M)
          for (int p = 0; p < w1; ++p)
            for (int q = 0; q < w2; ++q) {
              const double c = C[((size_t)p * w2 + q) * w + M];
              if (c != 0.0) pat_ent.push_back(CgEnt{(int8_t)p, (int8_t)q, (int8_t)M, 0, (float)c});
            }
        (void)e0;
        pat_id[key] = (int)pat_hdr.size() / 5;
        pat_hdr.insert(pat_hdr.end(), {la, lb, L, la * 45 + lb * 9 + L, pat_off[la * 45 + lb * 9 + L]});
      }
      const int pid = pat_id[key];
      const auto& mem = kv.second;
      // members of a group are taken with stride n_groups from the (a, b)
      // ordered list, so they rarely share a single index
      const size_t ng = (mem.size() + 7) / 8;
      for (size_t g = 0; g < ng; ++g) {
        grp_pat.push_back(pid);
        for (size_t q = 0; q < 8; ++q) {
          const size_t src = g + q * ng;
          grp_mem.push_back(src < mem.size() ? mem[src] : make_int4(-1, 0, 0, la * 5 + lb));
        }
      }
    }
    P.ngrp = (int32_t)grp_pat.size() - P.grp0;
  }
  // adjoint jobs per L: (target l, component part K of NP) - every job owns
  // its gradient entries, so no two wavefronts write the same entry.  The
  // part counts and the assignment to wavefronts balance an estimated cost
  // (largest job first onto the least-loaded wavefront).
  std::vector<int32_t> adj_ptr;
  std::vector<int4> adj_units;
  for (int L = 0; L <= Lmax; ++L) {
    const int w = 2 * L + 1;
    // cost of the components [i0, i1) of target l = lt
    auto job_cost = [&](int lt, int i0, int i1) {
      double c = 0;
      for (int lp = 0; lp <= lmax; ++lp) {
        if (!(std::abs(lt - lp) <= L && L <= lt + lp && ((lt + lp + L) & 1) == 0)) continue;
        const auto& C = cgcache[std::make_tuple(lt, lp, L)];
        const int w2 = 2 * lp + 1;
        // the partner sum W[m2][M] over the entries some component uses,
        // then one pass over the coupling coefficients
        int nnz = 0, used = 0;
        for (int q = 0; q < w2; ++q)
          for (int M = 0; M < w; ++M) {
            bool u = false;
            for (int p1 = i0; p1 < i1; ++p1)
              if (C[((size_t)p1 * w2 + q) * w + M] != 0.0) {
                ++nnz;
                u = true;
              }
            used += u;
          }
        c += nmax * (used + w + 2.0 * w2 + 8.0) + nnz;
      }
      if (lt == L) c += 3.0 * (i1 - i0) + 12.0;
      return c;
    };
    std::vector<int> np(lmax + 1, 1);
    std::vector<bool> live(lmax + 1, false);
    for (int lt = 0; lt <= lmax; ++lt) {
      bool any = lt == L;
      for (int lp = 0; lp <= lmax && !any; ++lp)
        if (std::abs(lt - lp) <= L && L <= lt + lp && ((lt + lp + L) & 1) == 0) any = true;
      live[lt] = any;
    }
    struct Job { int lt, npart, k; double cost; };
    auto schedule = [&](std::vector<std::vector<Job>>& per) {
      std::vector<Job> jobs;
      for (int lt = 0; lt <= lmax; ++lt) {
        if (!live[lt]) continue;
        const int nc = 2 * lt + 1;
        for (int k = 0; k < np[lt]; ++k)
          jobs.push_back(Job{lt, np[lt], k, job_cost(lt, k * nc / np[lt], (k + 1) * nc / np[lt])});
      }
      std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& b) { return a.cost > b.cost; });
      per.assign(kMixWaves, {});
      std::vector<double> load(kMixWaves, 0.0);
      for (auto& jb : jobs) {
        const int wv = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        per[wv].push_back(jb);
        load[wv] += jb.cost;
      }
      return *std::max_element(load.begin(), load.end());
    };
    std::vector<std::vector<Job>> per;
    double best = schedule(per);
    for (;;) {
      // split further the target whose job sits on the most loaded wavefront
      int wmax = 0;
      double lmax_w = -1;
      for (int wv = 0; wv < kMixWaves; ++wv) {
        double l = 0;
        for (auto& jb : per[wv]) l += jb.cost;
        if (l > lmax_w) { lmax_w = l; wmax = wv; }
      }
      int cand = -1;
      double cc = -1;
      for (auto& jb : per[wmax])
        if (np[jb.lt] < 3 && np[jb.lt] < 2 * jb.lt + 1 && jb.cost > cc) { cc = jb.cost; cand = jb.lt; }
      if (cand < 0) break;
      ++np[cand];
      std::vector<std::vector<Job>> trial;
      const double t = schedule(trial);
      if (t < best) {
        best = t;
        per = trial;
      } else {
        --np[cand];
        break;
      }
    }
    for (int wv = 0; wv < kMixWaves; ++wv) {
      adj_ptr.push_back((int32_t)adj_units.size());
      for (auto& jb : per[wv]) adj_units.push_back(make_int4(jb.lt * 16 + jb.npart * 4 + jb.k, 0, 0, jb.lt));
    }
    adj_ptr.push_back((int32_t)adj_units.size());
  }
  // LDS head: A, omega of both sets, phi [8][2], per-atom norm bound [8], the
  // rank's partial phi sums [2][4][8], and the level parameters of every rank
  // (fused kernel)
  x.tab_off = (int32_t)(((size_t)(3 * 8 * x.apad + 16 + 8 + 64) * 4 + 15) / 16 * 16 +
                        (size_t)(2 * kMaxL + 1) * kLevelInts * 4);
  // the channel row table is staged as int16 (rows < 2^15)
  for (int L = 0; L <= Lmax; ++L)
    if (x.lv[L].nrow >= 32768) return fail(ctx, AP_ERR_UNSUPPORTED, "too many coupled rows for one rank");
  const size_t rows_bytes = ((size_t)nidx * nidx * 2 + 15) / 16 * 16;
  size_t tab = rows_bytes;
  // per rank: the channel rows, the coupling groups and the row scales of both sets
  for (int L = 0; L <= Lmax; ++L)
    tab = std::max(tab, rows_bytes + (size_t)x.lv[L].ngrp * 8 * 16 + (size_t)x.lv[L].nrow16 * 2 * 4);
  x.big_off = (int32_t)((x.tab_off + tab + 15) / 16 * 16);
  // room the kernels' own static LDS needs beside the dynamic allocation
  constexpr size_t kLdsReserve = 256;
  // ranks whose X_L and Z_L fit in LDS together keep X_L for both sets
  for (int L = 0; L <= Lmax; ++L) {
    MixL& P = x.lv[L];
    // Z_L's row stride: 8w + 4 floats puts the rows r and r + 4 that one store
    // instruction writes (the MFMA result layout) 16 banks apart; 8w + 1 only
    // where that is what lets X_L and Z_L fit together
    const int w = 2 * L + 1;
    // beside Z_L, X_L holds only the tile's 8w columns (hi, then lo); the
    // contraction's reads of the last column tile's padding run on into the
    // next region, which must cover them
    const size_t x_tight = ((size_t)8 * w * P.kstr * 2 * 2 + 15) / 16 * 16;
    const size_t overread = (size_t)(P.ct * 16 - 8 * w) * P.kstr * 2;
    auto fits = [&](int zstr) {
      const size_t zb = (size_t)P.nrow * zstr * 4;
      return zb >= overread && (size_t)x.big_off + x_tight + zb + kLdsReserve <= 160 * 1024;
    };
    P.zstr = fits(8 * w + 4) || !fits(8 * w + 1) ? 8 * w + 4 : 8 * w + 1;
    zbytes[L] = (size_t)P.nrow * P.zstr * 4;
    P.xonce = fits(P.zstr) ? 1 : 0;
    P.zoff = P.xonce ? (int32_t)x_tight : 0;
    big = std::max(big, P.xonce ? x_tight + zbytes[L] : std::max(xbytes[L], zbytes[L]));
  }
  x.big_bytes = (int32_t)big;
  if (ace_mixed_lds_bytes(x) + kLdsReserve > 160 * 1024)
    return fail(ctx, AP_ERR_UNSUPPORTED, "ACE model too large for the mixed kernel's LDS");
  if ((st = upload_owned(ctx, ctile, &x.ctile)) || (st = upload_owned(ctx, rscale, &x.rscale)) ||
      (st = upload_owned(ctx, grp_pat, &x.grp_pat)) || (st = upload_owned(ctx, grp_mem, &x.grp_mem)) ||
      (st = upload_owned(ctx, pat_hdr, &x.pat_hdr)) || (st = upload_owned(ctx, pat_ent, &x.pat_ent)) ||
      (st = upload_owned(ctx, pat_coef, &x.pat_coef)) || (st = upload_owned(ctx, pat_off, &x.pat_off)) ||
      (st = upload_owned(ctx, rowtab, &x.rowtab)) || (st = upload_owned(ctx, adj_ptr, &x.adj_ptr)) ||
      (st = upload_owned(ctx, adj_units, &x.adj_units)))
    return st;
  {
    std::vector<MixL> lv(x.lv, x.lv + Lmax + 1);
    if ((st = upload_owned(ctx, lv, &x.lv_d))) return st;
  }
  ctx->mix_tiles = (double)(ctile.size() / 128);
  ctx->mix_mfma_flops = mfma_flops;
  return AP_OK;
}

// --------------------------------------------------------------------------
// Launch-mode tuner of the mixed rank phase.  The three modes (one kernel per
// coupled rank; all ranks in one persistent launch, tiles round-robin; the
// same with a device work counter) are timed with HIP events on the first
// call of a context for each bucket of the atom count (powers of two), on that
// call's own inputs, and the fastest is kept.  AP_RANK_MODE=0/1/2 forces a
// mode; AP_AUTOTUNE=0 turns the tuner off (mode 1); AP_AUTOTUNE_CACHE names a
// JSON file {"<device>|<model shape>|b<bucket>": mode, ...} that is read when
// a context is created and updated after each tuning.
static int size_bucket(int64_t n) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= std::max<int64_t>(n, 1)) ++b;
  return b;
}

static std::map<std::string, int> read_tune_cache(const std::string& path) {
  std::map<std::string, int> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t a = line.find('"');
    if (a == std::string::npos) continue;
    const size_t b = line.find('"', a + 1);
    const size_t c = b == std::string::npos ? b : line.find(':', b);
    if (c == std::string::npos) continue;
    char* end = nullptr;
    const long v = std::strtol(line.c_str() + c + 1, &end, 10);
    if (end != line.c_str() + c + 1) out[line.substr(a + 1, b - a - 1)] = (int)v;
  }
  return out;
}

static void write_tune_cache(const std::string& path, const std::string& key, int mode) {
  std::map<std::string, int> all = read_tune_cache(path);
  all[key] = mode;
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp, std::ios::trunc);
    if (!f) return;
    f << "{\n";
    size_t k = 0;
    for (auto& kv : all) f << "  \"" << kv.first << "\": " << kv.second << (++k < all.size() ? ",\n" : "\n");
    f << "}\n";
  }
  std::rename(tmp.c_str(), path.c_str());
}

static void setup_tuner(Ctx* ctx, const ap_ace_model* m) {
  hipDeviceProp_t prop;
  std::string dev = "hip";
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) dev = std::string(prop.gcnArchName) + " " + prop.name;
  std::ostringstream k;
  k << dev << "|ace " << m->n_max << " " << m->l_max << " " << m->K << " " << m->nu_max << " "
    << ctx->ace.L_max << " " << m->n_funcs;
  ctx->tune_key = k.str();
  if (const char* f = std::getenv("AP_RANK_MODE")) {
    const int v = std::atoi(f);
    if (v >= 0 && v < AP_RANK_N_MODES) ctx->rank_mode_forced = v;
  }
  if (const char* f = std::getenv("AP_AUTOTUNE"))
    if (std::string(f) == "0" && ctx->rank_mode_forced < 0) ctx->rank_mode_forced = AP_RANK_FUSED;
  if (const char* f = std::getenv("AP_AUTOTUNE_CACHE")) {
    ctx->tune_cache = f;
    const std::string pre = ctx->tune_key + "|b";
    for (auto& kv : read_tune_cache(ctx->tune_cache))
      if (kv.first.compare(0, pre.size(), pre) == 0 && kv.second >= 0 && kv.second < AP_RANK_N_MODES)
        ctx->rank_mode_tuned[std::atoi(kv.first.c_str() + pre.size())] = kv.second;
  }
}

// Address of `scratch` on the context's device (current when called).
static ap_status static_scratch(Ctx* ctx) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, AP_ERR_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(ctx, e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    if (!p) return fail(ctx, AP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[ctx->device] = p;
  }
  ctx->static_scratch = g_scratch_ptr[ctx->device];
  return AP_OK;
}

static ap_status upload_table(Ctx* ctx, const ap_table& t, TableDev* d, const char* name) {
  if (t.n_knots < 2 || !(t.dx > 0) || !t.coef)
    return fail(ctx, AP_ERR_ARG, std::string("invalid EAM table ") + name);
  std::vector<double> c(t.coef, t.coef + (size_t)(t.n_knots - 1) * 4);
  std::vector<float> cf(c.begin(), c.end());
  d->x0 = t.x0;
  d->dx = t.dx;
  d->inv_dx = 1.0 / t.dx;
  d->n = t.n_knots;
  ap_status st;
  if ((st = upload_owned(ctx, c, &d->c)) || (st = upload_owned(ctx, cf, &d->cf))) return st;
  return AP_OK;
}

static ap_status check_nl(Ctx* ctx, const ap_nlist* nl) {
  if (!nl || !nl->nbr || !nl->count) return fail(ctx, AP_ERR_ARG, "neighbour list arrays missing");
  if (nl->capacity < 1 || nl->capacity > kMaxCap) return fail(ctx, AP_ERR_ARG, "capacity must be in [1, 256]");
  return AP_OK;
}

}  // namespace ap

using namespace ap;

// ============================================================================
extern "C" {

const char* ap_version(void) { return "ap 0.1 gfx950"; }

const char* ap_last_error(const ap_ctx* c) {
  const Ctx* ctx = (const Ctx*)c;
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

ap_status ap_create(ap_ctx** out, int32_t device, int32_t precision, const ap_eam_tables* eam,
                    const ap_ace_model* ace) {
  if (!out) return fail(nullptr, AP_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (precision != AP_PREC_FP64 && precision != AP_PREC_MIXED)
    return fail(nullptr, AP_ERR_ARG, "precision must be AP_PREC_FP64 or AP_PREC_MIXED");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || device < 0 || device >= ndev)
    return fail(nullptr, AP_ERR_HIP, "no such HIP device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return fail(nullptr, AP_ERR_HIP, "hipSetDevice failed");
  Ctx* ctx = new Ctx();
  ctx->device = device;
  ctx->precision = precision;
  ap_status st = static_scratch(ctx);
  if (st != AP_OK) {
    g_create_err = ctx->err;
    ap_destroy((ap_ctx*)ctx);
    return st;
  }
  if (eam) {
    if ((st = upload_table(ctx, eam->phi, &ctx->phi, "phi")) ||
        (st = upload_table(ctx, eam->rho, &ctx->rho, "rho")) ||
        (st = upload_table(ctx, eam->F, &ctx->F, "F"))) {
      g_create_err = ctx->err;
      ap_destroy((ap_ctx*)ctx);
      return st;
    }
    ctx->has_eam = true;
  }
  if (ace) {
    if ((st = fold_ace(ctx, ace)) != AP_OK) {
      g_create_err = ctx->err;
      ap_destroy((ap_ctx*)ctx);
      return st;
    }
    ctx->has_ace = true;
    setup_tuner(ctx, ace);
  }
  if ((st = ensure(ctx, ctx->flags, 64)) != AP_OK) {
    g_create_err = ctx->err;
    ap_destroy((ap_ctx*)ctx);
    return st;
  }
  hipMemset(ctx->flags.p, 0, 64);
  hipDeviceSynchronize();
  *out = (ap_ctx*)ctx;
  return AP_OK;
}

ap_status ap_destroy(ap_ctx* c) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return AP_OK;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto& b : ctx->owned) release(b);
  SysCache& C = ctx->sys;
  for (Buffer* b : {&C.off_d, &C.H_d, &C.Hi_d, &C.ortho_d, &C.grid_d, &C.cell_base_d, &C.sys_of_d,
                    &C.chunk_lo_d, &C.chunk_hi_d, &C.sys_chunk_d})
    release(*b);
  for (Buffer* b : {&ctx->cell_big, &ctx->pos4, &ctx->cell_count, &ctx->cell_start, &ctx->cell_cursor, &ctx->cell_atoms,
                    &ctx->cell_pos, &ctx->cell_of, &ctx->scan_tmp, &ctx->wfp, &ctx->eF, &ctx->wgt,
                    &ctx->vir_atom, &ctx->e_tmp, &ctx->ace_row, &ctx->pair_g, &ctx->ace_counter,
                    &ctx->ace_rows_list, &ctx->ace_halo, &ctx->nbr_ace, &ctx->partials, &ctx->flags, &ctx->ind_atom, &ctx->mix_A,
                    &ctx->mix_om, &ctx->mix_phi, &ctx->mix_bn, &ctx->sw_csp, &ctx->sw_mu0,
                    &ctx->sw_mu, &ctx->sw_flag, &ctx->sw_src, &ctx->sw_nsrc,
                    &ctx->e_eam_raw, &ctx->e_ace_raw, &ctx->nvt_ke, &ctx->nvt_sums, &ctx->nvt_fac})
    release(*b);
  delete ctx;
  return AP_OK;
}

static ap_status scratch_reduce(Ctx* ctx, int m) {
  return ensure(ctx, ctx->partials, sizeof(double) * (size_t)std::max(1, ctx->sys.n_chunks) * m);
}

ap_status ap_build_neighbors(ap_ctx* c, const ap_systems* sys, const double* pos, const ap_nlist* nl,
                             int32_t* needed_capacity, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if ((st = check_nl(ctx, nl))) return st;
  if (!pos && sys && sys->n_atoms > 0) return fail(ctx, AP_ERR_ARG, "pos is NULL");
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  const int64_t N = sv.n_atoms;
  const int nc = ctx->sys.n_cells;
  if ((st = ensure(ctx, ctx->cell_count, 4 * (size_t)nc)) ||
      (st = ensure(ctx, ctx->cell_start, 4 * (size_t)nc)) ||
      (st = ensure(ctx, ctx->cell_cursor, 4 * (size_t)nc)) ||
      (st = ensure(ctx, ctx->cell_big, 4 * ((size_t)N + 1))) ||
      (st = ensure(ctx, ctx->cell_of, 4 * (size_t)N)) ||
      (st = ensure(ctx, ctx->cell_atoms, 4 * (size_t)N)) ||
      (st = ensure(ctx, ctx->cell_pos, 32 * (size_t)N)) ||
      (st = ensure(ctx, ctx->scan_tmp, 4 * ((size_t)std::max<int64_t>(nc, N) / 4096 + 2))))
    return st;
  int32_t* flags = (int32_t*)ctx->flags.p;
  PhaseTimer timer(ctx, AP_PHASE_NEIGHBORS, s);
  if (needed_capacity) AP_HIP(launch_fill_i32(flags, 0, 1, s));
  AP_HIP(launch_fill_i32((int32_t*)ctx->cell_count.p, 0, nc, s));
  AP_HIP(launch_bin(sv, pos, (int32_t*)ctx->cell_of.p, (int32_t*)ctx->cell_count.p, s));
  // the scan also writes the scatter's cursors (a copy of the cell starts)
  AP_HIP(launch_scan_exclusive((const int32_t*)ctx->cell_count.p, (int32_t*)ctx->cell_start.p, nc,
                               (int32_t*)ctx->scan_tmp.p, s, (int32_t*)ctx->cell_cursor.p));
  AP_HIP(launch_scatter(sv, pos, (const int32_t*)ctx->cell_of.p, (int32_t*)ctx->cell_cursor.p,
                        (int32_t*)ctx->cell_atoms.p, (double4*)ctx->cell_pos.p, s));
  AP_HIP(launch_fill_nbr_cells(sv, nc, pos, (const int32_t*)ctx->cell_of.p,
                               (const int32_t*)ctx->cell_start.p, (const int32_t*)ctx->cell_count.p,
                               (const double4*)ctx->cell_pos.p, nl->nbr, nl->count, nl->capacity,
                               flags, (int32_t*)ctx->cell_big.p, s));
  if (nl->rev) AP_HIP(launch_rev((int32_t)N, nl->nbr, nl->count, nl->rev, s));
  ctx->cells_n_atoms = N;
  if (needed_capacity) {
    int32_t need = 0;
    AP_HIP(hipMemcpyAsync(&need, flags, 4, hipMemcpyDeviceToHost, s));
    AP_HIP(hipStreamSynchronize(s));
    if (need > nl->capacity) {
      *needed_capacity = need;
      AP_HIP(launch_fill_i32(flags, 0, 1, s));
      return fail(ctx, AP_ERR_NBR_CAPACITY, "neighbour list capacity exceeded");
    }
  }
  return AP_OK;
}

static ap_status check_blend_args(Ctx* ctx, const ap_lambda_rule* rule, const double* lambda,
                                  const int32_t* ace_list, const int32_t* n_ace) {
  if (!rule || !lambda || !ace_list || !n_ace) return fail(ctx, AP_ERR_ARG, "blend arguments missing");
  if (rule->kind < AP_LAMBDA_CONST || rule->kind > AP_LAMBDA_GIVEN) return fail(ctx, AP_ERR_ARG, "bad rule kind");
  if (rule->kind == AP_LAMBDA_CONST && !(rule->value >= 0.0 && rule->value <= 1.0))
    return fail(ctx, AP_ERR_ARG, "constant lambda must be in [0, 1]");
  if (rule->kind != AP_LAMBDA_CONST && rule->kind != AP_LAMBDA_GIVEN &&
      (!(rule->r_full >= 0) || !(rule->taper > 0)))
    return fail(ctx, AP_ERR_ARG, "rule needs r_full >= 0 and taper > 0");
  if (rule->kind == AP_LAMBDA_MASK && !rule->mask) return fail(ctx, AP_ERR_ARG, "mask rule needs a mask");
  return AP_OK;
}

ap_status ap_blend(ap_ctx* c, const ap_systems* sys, const double* pos, const ap_lambda_rule* rule,
                   double* lambda, int32_t* ace_list, int32_t* n_ace, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if ((st = check_blend_args(ctx, rule, lambda, ace_list, n_ace))) return st;
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  if (!pos && sv.n_atoms > 0) return fail(ctx, AP_ERR_ARG, "pos is NULL");
  const int64_t N = sv.n_atoms;
  if ((st = ensure(ctx, ctx->e_tmp, 8 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->scan_tmp, 4 * ((size_t)N / 4096 + 2))))
    return st;
  int32_t* flag = (int32_t*)ctx->e_tmp.p;
  PhaseTimer timer(ctx, AP_PHASE_BLEND, s);
  AP_HIP(launch_blend((int32_t)N, pos, *rule, lambda, flag, s));
  AP_HIP(launch_compact((int32_t)N, flag, ace_list, n_ace, (int32_t*)ctx->scan_tmp.p, s));
  return AP_OK;
}

// copy0/copy1 (optional) receive system 0's first and second sums as well
static ap_status reduce_into(Ctx* ctx, const SysView& sv, const double* vals, int m, double* out,
                             bool accumulate, hipStream_t s, double* copy0 = nullptr,
                             double* copy1 = nullptr) {
  ap_status st;
  PhaseTimer timer(ctx, AP_PHASE_REDUCE, s);
  if ((st = scratch_reduce(ctx, m))) return st;
  AP_HIP(launch_reduce(sv, ctx->sys.n_chunks, (const int64_t*)ctx->sys.chunk_lo_d.p,
                       (const int64_t*)ctx->sys.chunk_hi_d.p, (const int32_t*)ctx->sys.sys_chunk_d.p,
                       vals, m, sv.n_atoms, (double*)ctx->partials.p, out, accumulate, s, copy0,
                       copy1));
  return AP_OK;
}

ap_status ap_eam_forces(ap_ctx* c, const ap_systems* sys, const double* pos, const ap_nlist* nl,
                        const double* lambda, double* e_atom, double* force, double* virial,
                        uint32_t flags, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (!ctx->has_eam) return fail(ctx, AP_ERR_ARG, "context has no EAM tables");
  if (flags > 1u) return fail(ctx, AP_ERR_ARG, "flags must be AP_OVERWRITE or AP_ACCUMULATE");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if ((st = check_nl(ctx, nl))) return st;
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  const int64_t N = sv.n_atoms;
  if (N > 0 && (!pos || !e_atom || !force)) return fail(ctx, AP_ERR_ARG, "pos/e_atom/force is NULL");
  if ((st = ensure(ctx, ctx->wfp, 8 * (size_t)N)) || (st = ensure(ctx, ctx->eF, 8 * (size_t)N)) ||
      (st = ensure(ctx, ctx->wgt, 8 * (size_t)N)) || (st = ensure(ctx, ctx->e_eam_raw, 8 * (size_t)N)) ||
      (virial && (st = ensure(ctx, ctx->vir_atom, 72 * (size_t)N))))
    return st;
  const bool acc = flags == AP_ACCUMULATE;
  double* vir = virial ? (double*)ctx->vir_atom.p : nullptr;
  {
  PhaseTimer timer(ctx, AP_PHASE_EAM, s);
  if ((st = ensure(ctx, ctx->pos4, 32 * (size_t)std::max<int64_t>(N, 1)))) return st;
  AP_HIP(launch_pack_pos((int32_t)N, pos, (double4*)ctx->pos4.p, s));
  AP_HIP(launch_eam(*ctx, sv, pos, (const double4*)ctx->pos4.p, nl->nbr, nl->count, (int32_t)N,
                    lambda, (double*)ctx->wfp.p, (double*)ctx->eF.p, (double*)ctx->wgt.p, e_atom,
                    force, vir, acc, (double*)ctx->e_eam_raw.p, s));
  }
  // in a fused evaluation the ACE call reduces the EAM and ACE per-atom virials together
  if (virial && !ctx->fused_eval && (st = reduce_into(ctx, sv, vir, 9, virial, acc, s))) return st;
  return AP_OK;
}

ap_status ap_ace_forces(ap_ctx* c, const ap_systems* sys, const double* pos, const ap_nlist* nl,
                        const double* lambda, const int32_t* ace_list, const int32_t* n_ace,
                        double* e_atom, double* force, double* virial, uint32_t flags,
                        void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (!ctx->has_ace) return fail(ctx, AP_ERR_ARG, "context has no ACE model");
  if (flags > 1u) return fail(ctx, AP_ERR_ARG, "flags must be AP_OVERWRITE or AP_ACCUMULATE");
  if (ace_list && !n_ace) return fail(ctx, AP_ERR_ARG, "n_ace is NULL");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if ((st = check_nl(ctx, nl))) return st;
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  const int64_t N = sv.n_atoms;
  if (N > 0 && (!pos || !e_atom || !force)) return fail(ctx, AP_ERR_ARG, "pos/e_atom/force is NULL");
  const size_t gsz = ctx->precision == AP_PREC_FP64 ? 8 : 4;
  if ((st = ensure(ctx, ctx->ace_row, 4 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->ace_counter, 256)) ||
      (st = ensure(ctx, ctx->pair_g, gsz * 3 * (size_t)nl->capacity * std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->nbr_ace, 4 * (size_t)nl->capacity * std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->e_ace_raw, 8 * (size_t)std::max<int64_t>(N, 1))) ||
      (virial && (st = ensure(ctx, ctx->vir_atom, 72 * (size_t)N))))
    return st;
  const bool acc = flags == AP_ACCUMULATE;
  double* vir = virial ? (double*)ctx->vir_atom.p : nullptr;
  if (!acc) AP_HIP(launch_fill_f64(e_atom, 0.0, N, s));
  // a fused evaluation adds the ACE per-atom virial to the EAM call's
  const bool vir_acc = vir && ctx->fused_eval;
  if (vir && !vir_acc) AP_HIP(launch_fill_f64(vir, 0.0, 9 * N, s));
  if ((st = ensure(ctx, ctx->pos4, 32 * (size_t)std::max<int64_t>(N, 1)))) return st;
  // a fused evaluation's EAM call packed these positions already
  if (!ctx->fused_eval) AP_HIP(launch_pack_pos((int32_t)N, pos, (double4*)ctx->pos4.p, s));
  AP_HIP(launch_ace_rows((int32_t)N, ace_list, n_ace, (int32_t*)ctx->ace_row.p, s));
  // the ACE kernels stamp the listed atoms and their neighbours (the atoms the
  // gather visits) in the halo array with a fresh stamp per evaluation; a new
  // allocation, or the stamp running out of range, clears it once.  A stale
  // entry equal to the current stamp would only make the gather visit an atom
  // whose ACE sum is zero, so correctness never depends on the clear.
  const void* halo_before = ctx->ace_halo.p;
  if ((st = ensure(ctx, ctx->ace_halo, 4 * (size_t)std::max<int64_t>(N, 1)))) return st;
  if (ctx->ace_halo.p != halo_before || ctx->halo_stamp == INT32_MAX) {
    AP_HIP(launch_fill_i32((int32_t*)ctx->ace_halo.p, 0, (int32_t)(ctx->ace_halo.bytes / 4), s));
    ctx->halo_stamp = 0;
  }
  const int32_t stamp = ++ctx->halo_stamp;
  int32_t* halo = (int32_t*)ctx->ace_halo.p;
  if (ctx->precision == AP_PREC_FP64) {
    PhaseTimer timer(ctx, AP_PHASE_ACE, s);
    // the FP64 kernel takes atoms from a work counter
    AP_HIP(launch_ace_reset((int32_t*)ctx->ace_counter.p, s));
    AP_HIP(launch_ace(*ctx, sv, pos, (const double4*)ctx->pos4.p, nl->nbr, nl->count, nl->capacity,
                      (int32_t)N, lambda, ace_list, n_ace, (int32_t*)ctx->ace_row.p,
                      (int32_t*)ctx->ace_counter.p, ctx->pair_g.p, e_atom, vir,
                      (double*)ctx->e_ace_raw.p, (int32_t*)ctx->nbr_ace.p, halo, stamp, vir_acc, s));
  } else {
    const MixDev& mx = ctx->mix;
    const size_t rows = (size_t)std::max<int64_t>(N, 1) + 8;
    if ((st = ensure(ctx, ctx->mix_A, 4 * rows * mx.nA)) ||
        (st = ensure(ctx, ctx->mix_om, 8 * rows * mx.nA)) ||
        (st = ensure(ctx, ctx->mix_phi, 8 * rows)) || (st = ensure(ctx, ctx->mix_bn, 4 * rows)))
      return st;
    auto phase_run = [&](int phase, int mode) -> hipError_t {
      if (phase == 1 && mode == AP_RANK_FUSED_QUEUE) {
        const hipError_t e = launch_ace_reset((int32_t*)ctx->ace_counter.p, s);
        if (e != hipSuccess) return e;
      }
      return launch_ace_mixed(*ctx, sv, pos, (const double4*)ctx->pos4.p, nl->nbr, nl->count,
                              nl->capacity, (int32_t)N, lambda, ace_list, n_ace,
                              (int32_t*)ctx->ace_counter.p, (float*)ctx->pair_g.p, (float*)ctx->mix_A.p,
                              (float*)ctx->mix_om.p, (float*)ctx->mix_phi.p, (float*)ctx->mix_bn.p, e_atom,
                              vir, s, phase, mode, (double*)ctx->e_ace_raw.p, (int32_t*)ctx->nbr_ace.p,
                              halo, stamp, vir_acc);
    };
    {
      PhaseTimer timer(ctx, AP_PHASE_ACE_BOND, s);
      AP_HIP(phase_run(0, 0));
    }
    int mode = ctx->rank_mode_forced;
    if (mode > AP_RANK_PER_L && !rank_kernel_fused(false, rank_xomask(ctx->mix), ctx->mix.L_max))
      mode = AP_RANK_PER_L;
    if (mode < 0) {
      const int bucket = size_bucket(N);
      auto it = ctx->rank_mode_tuned.find(bucket);
      if (it != ctx->rank_mode_tuned.end()) {
        mode = it->second;
      } else {
        // time every mode twice on these inputs (the first round warms up);
        // each run rewrites the phase's outputs completely
        // (the fused modes exist for the rank layouts with an instance)
        const int n_modes = rank_kernel_fused(false, rank_xomask(ctx->mix), ctx->mix.L_max) ? AP_RANK_N_MODES : 1;
        hipEvent_t ev[2 * AP_RANK_N_MODES];
        for (auto& e : ev) AP_HIP(hipEventCreate(&e));
        for (int rep = 0; rep < 2; ++rep)
          for (int md = 0; md < n_modes; ++md) {
            if (rep == 1) AP_HIP(hipEventRecord(ev[2 * md], s));
            AP_HIP(phase_run(1, md));
            if (rep == 1) AP_HIP(hipEventRecord(ev[2 * md + 1], s));
          }
        AP_HIP(hipEventSynchronize(ev[2 * n_modes - 1]));
        float best = 0.f;
        for (int md = 0; md < n_modes; ++md) {
          float ms = 0.f;
          AP_HIP(hipEventElapsedTime(&ms, ev[2 * md], ev[2 * md + 1]));
          if (mode < 0 || ms < best) {
            best = ms;
            mode = md;
          }
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        ctx->rank_mode_tuned[bucket] = mode;
        if (!ctx->tune_cache.empty())
          write_tune_cache(ctx->tune_cache, ctx->tune_key + "|b" + std::to_string(bucket), mode);
      }
    }
    ctx->last_rank_mode = mode;
    {
      PhaseTimer timer(ctx, AP_PHASE_ACE, s);
      AP_HIP(phase_run(1, mode));
    }
    {
      PhaseTimer timer(ctx, AP_PHASE_ACE_BOND, s);
      AP_HIP(phase_run(2, 0));
    }
  }
  {
    PhaseTimer timer(ctx, AP_PHASE_ACE_GATHER, s);
    const int32_t* rev = nl->rev;
    // without a full reverse index the gather finds each reverse slot by
    // binary search of the (ascending) neighbour row, in the atom-major copy
    // of the listed atoms' rows that the ACE kernels wrote
    AP_HIP(launch_ace_gather(*ctx, (int32_t)N, nl->nbr, nl->count, rev,
                             (const int32_t*)ctx->nbr_ace.p, nl->capacity, (const int32_t*)ctx->ace_row.p, halo, stamp, ctx->pair_g.p, force, acc, s));
  }
  // fused: the per-atom virial holds EAM + ACE and the system virial is written afresh
  if (virial && (st = reduce_into(ctx, sv, vir, 9, virial, vir_acc ? false : acc, s))) return st;
  return AP_OK;
}

ap_status ap_indenter(ap_ctx* c, const ap_systems* sys, const double* pos, const uint8_t* fixed,
                      const double* centre, double R, double K, const double* dir, double* force,
                      double* e_ind, double* load, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (!centre || !dir) return fail(ctx, AP_ERR_ARG, "centre/dir is NULL");
  if (!(R > 0) || !(K >= 0)) return fail(ctx, AP_ERR_ARG, "indenter needs R > 0 and K >= 0");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  if (sv.n_sys != 1) return fail(ctx, AP_ERR_UNSUPPORTED, "the indenter acts on a single system");
  const int64_t N = sv.n_atoms;
  if (N > 0 && (!pos || !force)) return fail(ctx, AP_ERR_ARG, "pos/force is NULL");
  const bool want = e_ind || load;
  if (want && (st = ensure(ctx, ctx->ind_atom, 16 * (size_t)N + 64))) return st;
  double* e2 = want ? (double*)ctx->ind_atom.p : nullptr;
  PhaseTimer timer(ctx, AP_PHASE_INDENTER, s);
  AP_HIP(launch_indenter((int32_t)N, pos, fixed, centre, R, K, dir, force, e2, s));
  if (want) {
    double* out = (double*)ctx->ind_atom.p + 2 * N;
    if ((st = reduce_into(ctx, sv, e2, 2, out, false, s, e_ind, load))) return st;
  }
  return AP_OK;
}

ap_status ap_switching_update(ap_ctx* c, const ap_systems* sys, const double* pos,
                              const ap_nlist* nl, ap_switching* sw, double* lambda,
                              int32_t* ace_list, int32_t* n_ace, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if (!sw || !lambda || !ace_list || !n_ace) return fail(ctx, AP_ERR_ARG, "switching arguments missing");
  if (!(sw->csp_lo < sw->csp_hi) || sw->n_csp < 2 || sw->n_csp > 16 || (sw->n_csp & 1) ||
      sw->n_csp_avg < 1 || sw->n_lambda_avg < 1 || !(sw->r_lo >= 0.0) || !(sw->r_lo < sw->r_hi) ||
      !(sw->dlambda_min >= 0.0 && sw->dlambda_min < 0.5) || !std::isfinite(sw->r_hi))
    return fail(ctx, AP_ERR_ARG, "switching parameters out of range");
  if ((st = check_nl(ctx, nl))) return st;
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  const int64_t N = sv.n_atoms;
  if (N > 0 && (!pos || !sw->csp_avg || !sw->lambda_avg)) return fail(ctx, AP_ERR_ARG, "pos or switching state is NULL");
  if (!ctx->sys.all_ortho) return fail(ctx, AP_ERR_UNSUPPORTED, "dynamic switching needs orthorhombic systems");
  for (int k = 0; k < 3; ++k)
    if (sys->periodic[k])
      for (int q = 0; q < sys->n_systems; ++q)
        if (sys->box[9 * q + 4 * k] < 2.0 * sw->r_hi)
          return fail(ctx, AP_ERR_BOX, "a periodic width is below twice the transition range r_hi");
  if (ctx->cells_n_atoms != N) return fail(ctx, AP_ERR_ARG, "build the neighbour list on this context first");
  if ((st = ensure(ctx, ctx->sw_csp, 8 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->sw_mu0, 8 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->sw_mu, 8 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->sw_flag, 4 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->sw_src, 4 * (size_t)std::max<int64_t>(N, 1))) ||
      (st = ensure(ctx, ctx->sw_nsrc, 256)) ||
      (st = ensure(ctx, ctx->scan_tmp, 4 * ((size_t)std::max<int64_t>(ctx->sys.n_cells, N) / 4096 + 2))))
    return st;
  const double full = (sw->n_csp / 2) * (2.0 * sys->cutoff) * (2.0 * sys->cutoff);
  PhaseTimer timer(ctx, AP_PHASE_BLEND, s);
  AP_HIP(launch_switching(sv, pos, nl->nbr, nl->count, nl->capacity, (const int32_t*)ctx->cell_of.p,
                          (const int32_t*)ctx->cell_start.p, (const int32_t*)ctx->cell_count.p,
                          (const int32_t*)ctx->cell_atoms.p, (const double4*)ctx->cell_pos.p, *sw, full,
                          (double*)ctx->sw_csp.p, (double*)ctx->sw_mu0.p,
                          (unsigned long long*)ctx->sw_mu.p, (int32_t*)ctx->sw_flag.p,
                          (int32_t*)ctx->sw_src.p, (int32_t*)ctx->sw_nsrc.p, (int32_t*)ctx->scan_tmp.p,
                          lambda, ace_list, n_ace, s));
  sw->initialised = 1;
  return AP_OK;
}

ap_status ap_set_eam_analytic(ap_ctx* c, const ap_eam_analytic* e) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (!e) return fail(ctx, AP_ERR_ARG, "eam is NULL");
  if (e->n_phi < 0 || e->n_phi > kMaxEamKnots || e->n_rho < 0 || e->n_rho > kMaxEamKnots ||
      (e->n_phi > 0 && (!e->a_phi || !e->d_phi)) || (e->n_rho > 0 && (!e->a_rho || !e->d_rho)))
    return fail(ctx, AP_ERR_ARG, "analytic EAM: knot arrays missing or more than 32 knots");
  if (!(e->a_zbl > 0) || !(e->eps0 > 0) || !(e->r_lo > 0) || !(e->r_lo <= e->r_hi))
    return fail(ctx, AP_ERR_ARG, "analytic EAM: need a_zbl, eps0 > 0 and 0 < r_lo <= r_hi");
  EamAnalyticDev& p = ctx->ean;
  p = EamAnalyticDev{};
  p.n_phi = e->n_phi;
  p.n_rho = e->n_rho;
  for (int i = 0; i < e->n_phi; ++i) {
    p.a_phi[i] = e->a_phi[i];
    p.d_phi[i] = e->d_phi[i];
  }
  for (int i = 0; i < e->n_rho; ++i) {
    p.a_rho[i] = e->a_rho[i];
    p.d_rho[i] = e->d_rho[i];
  }
  p.r_cut_rho = e->r_cut_rho;
  double zc = 0.0;
  for (int i = 0; i < e->n_rho; ++i) {
    const double t = e->d_rho[i] - e->r_cut_rho;
    if (t >= 0.0) zc += e->a_rho[i] * t * t * t;
  }
  p.zeta_cut = zc;
  p.a_xi1 = e->a_xi1;
  p.a_xi2 = e->a_xi2;
  p.d_xi = e->d_xi;
  p.zbl_pref = e->z * e->z / (4.0 * M_PI * e->eps0);
  p.a_zbl = e->a_zbl;
  for (int k = 0; k < 4; ++k) {
    p.zbl_c[k] = e->zbl_c[k];
    p.zbl_q[k] = e->zbl_q[k];
  }
  p.r_lo = e->r_lo;
  p.r_hi = e->r_hi;
  for (int m = 0; m < 6; ++m) p.b_phi[m] = e->b_phi[m];
  ctx->eam_analytic = true;
  ctx->has_eam = true;
  return AP_OK;
}

ap_status ap_lambda_gradient(ap_ctx* c, const ap_systems* sys, const double* pos,
                             const ap_lambda_rule* rule, const double* lambda, double* force,
                             double* virial, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if (!rule || !lambda || !force) return fail(ctx, AP_ERR_ARG, "lambda-gradient arguments missing");
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  const int64_t N = sv.n_atoms;
  if (N > 0 && !pos) return fail(ctx, AP_ERR_ARG, "pos is NULL");
  const bool geo = rule->kind == AP_LAMBDA_SPHERE || rule->kind == AP_LAMBDA_HEMISPHERE ||
                   rule->kind == AP_LAMBDA_MASK;
  if (!geo || N == 0) return AP_OK;  // lambda does not follow the positions
  if (!(rule->taper > 0)) return fail(ctx, AP_ERR_ARG, "rule needs taper > 0");
  if (!ctx->has_eam || !ctx->has_ace || ctx->e_eam_raw.bytes < 8 * (size_t)N ||
      ctx->e_ace_raw.bytes < 8 * (size_t)N)
    return fail(ctx, AP_ERR_ARG, "call ap_eam_forces and ap_ace_forces on this context first");
  if (virial && (st = ensure(ctx, ctx->vir_atom, 72 * (size_t)N))) return st;
  double* vir = virial ? (double*)ctx->vir_atom.p : nullptr;
  {
    PhaseTimer timer(ctx, AP_PHASE_BLEND, s);
    AP_HIP(launch_lambda_grad((int32_t)N, pos, *rule, lambda, (const double*)ctx->e_ace_raw.p,
                              (const double*)ctx->e_eam_raw.p, force, vir, s));
  }
  if (virial && (st = reduce_into(ctx, sv, vir, 9, virial, true, s))) return st;
  return AP_OK;
}

ap_status ap_blend_noalloc(ap_ctx* c, const ap_systems* sys, const double* pos,
                           const ap_lambda_rule* rule, double* lambda, int32_t* ace_list,
                           int32_t* n_ace, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  ap_status st;
  if ((st = check_blend_args(ctx, rule, lambda, ace_list, n_ace))) return st;
  // the systems are only validated: the switching pass needs no geometry, so
  // nothing is uploaded (the systems cache of the other calls may allocate)
  if (!sys || !sys->sys_offset || sys->n_systems < 1 || sys->n_systems > kMaxSys)
    return fail(ctx, AP_ERR_ARG, "sys is NULL or has no systems");
  const int64_t N = sys->n_atoms;
  if (N < 0 || sys->sys_offset[0] != 0 || sys->sys_offset[sys->n_systems] != N)
    return fail(ctx, AP_ERR_ARG, "sys_offset must run from 0 to n_atoms");
  if (N > kNoallocMaxAtoms) {
    char buf[160];
    snprintf(buf, sizeof buf, "ap_blend_noalloc: %lld atoms exceed its static scratch (at most %lld)",
             (long long)N, (long long)kNoallocMaxAtoms);
    return fail(ctx, AP_ERR_ARG, buf);
  }
  if (!pos && N > 0) return fail(ctx, AP_ERR_ARG, "pos is NULL");
  int cur = -1;
  AP_HIP(hipGetDevice(&cur));
  if (cur != ctx->device) return fail(ctx, AP_ERR_ARG, "ap_blend_noalloc: the context's device is not current");
  if (!ctx->static_scratch) return fail(ctx, AP_ERR_HIP, "static scratch address not set up");
  // flags [0, 4 N) and the scan's partial sums: both written before they are
  // read, so nothing is cleared; no timer events (creating one may allocate)
  int32_t* flag = (int32_t*)ctx->static_scratch;
  int32_t* tmp = (int32_t*)((unsigned char*)ctx->static_scratch + kNoallocFlagBytes + 256);
  AP_HIP(launch_blend((int32_t)N, pos, *rule, lambda, flag, s));
  AP_HIP(launch_compact((int32_t)N, flag, ace_list, n_ace, tmp, s));
  return AP_OK;
}

ap_status ap_reduce_energy(ap_ctx* c, const ap_systems* sys, const double* e_atom, double* e_sys,
                           void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (!e_sys || (!e_atom && sys && sys->n_atoms > 0)) return fail(ctx, AP_ERR_ARG, "e_atom/e_sys is NULL");
  ap_status st;
  SysView sv;
  if ((st = prepare_systems(ctx, sys, &sv))) return st;
  return reduce_into(ctx, sv, e_atom, 1, e_sys, false, (hipStream_t)stream);
}

ap_status ap_check(ap_ctx* c, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  hipStream_t s = (hipStream_t)stream;
  int32_t f[2] = {0, 0};
  AP_HIP(hipMemcpyAsync(f, ctx->flags.p, 8, hipMemcpyDeviceToHost, s));
  AP_HIP(hipStreamSynchronize(s));
  AP_HIP(hipGetLastError());
  if (f[0] || f[1]) {
    AP_HIP(launch_fill_i32((int32_t*)ctx->flags.p, 0, 2, s));
    AP_HIP(hipStreamSynchronize(s));
  }
  if (f[0]) {
    char buf[128];
    snprintf(buf, sizeof buf, "neighbour list capacity exceeded (needed %d)", f[0]);
    return fail(ctx, AP_ERR_NBR_CAPACITY, buf);
  }
  if (f[1]) return fail(ctx, AP_ERR_NONFINITE, "non-finite force detected");
  return AP_OK;
}

static ap_status force_eval(Ctx* ctx, const ap_systems* sys, ap_md_state* st, hipStream_t s) {
  ap_status r;
  const int64_t N = sys->n_atoms;
  if (st->switching) {
    // the dynamic rule needs the neighbour list (and its cells) of these positions
    if ((r = ap_build_neighbors((ap_ctx*)ctx, sys, st->pos, &st->nl, nullptr, s))) return r;
    if ((r = ap_switching_update((ap_ctx*)ctx, sys, st->pos, &st->nl, st->switching, st->lambda,
                                 st->ace_list, st->n_ace, s)))
      return r;
  } else {
    if ((r = ap_blend((ap_ctx*)ctx, sys, st->pos, &st->rule, st->lambda, st->ace_list, st->n_ace, s)))
      return r;
    if ((r = ap_build_neighbors((ap_ctx*)ctx, sys, st->pos, &st->nl, nullptr, s))) return r;
  }
  bool written = false;
  {
    // EAM then ACE on the same positions: the positions are packed once and,
    // with a virial, the summed per-atom virials are reduced once
    struct Unfuse {
      Ctx* c;
      ~Unfuse() { c->fused_eval = false; }
    } unfuse{ctx};
    ctx->fused_eval = ctx->has_eam && ctx->has_ace;
    if (ctx->has_eam) {
      if ((r = ap_eam_forces((ap_ctx*)ctx, sys, st->pos, &st->nl, st->lambda, st->e_atom, st->force,
                             st->virial, AP_OVERWRITE, s)))
        return r;
      written = true;
    }
    if (ctx->has_ace) {
      if ((r = ap_ace_forces((ap_ctx*)ctx, sys, st->pos, &st->nl, st->lambda, st->ace_list, st->n_ace,
                             st->e_atom, st->force, st->virial, written ? AP_ACCUMULATE : AP_OVERWRITE,
                             s)))
        return r;
      written = true;
    }
  }
  if (!written) {
    AP_HIP(launch_fill_f64(st->force, 0.0, 3 * N, s));
    AP_HIP(launch_fill_f64(st->e_atom, 0.0, N, s));
  }
  if (st->lambda_gradient && !st->switching && ctx->has_eam && ctx->has_ace) {
    if ((r = ap_lambda_gradient((ap_ctx*)ctx, sys, st->pos, &st->rule, st->lambda, st->force,
                                st->virial, s)))
      return r;
  }
  if (st->ind_K > 0) {
    if ((r = ap_indenter((ap_ctx*)ctx, sys, st->pos, st->fixed, st->ind_centre, st->ind_R, st->ind_K,
                         st->ind_dir, st->force, st->e_ind, st->load, s)))
      return r;
  }
  return AP_OK;
}

ap_status ap_step(ap_ctx* c, const ap_systems* sys, ap_md_state* st, int32_t n_steps, void* stream) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (!st || n_steps < 0) return fail(ctx, AP_ERR_ARG, "state is NULL or n_steps < 0");
  if (!st->pos || !st->vel || !st->force || !st->e_atom || !st->lambda || !st->mass ||
      !st->ace_list || !st->n_ace)
    return fail(ctx, AP_ERR_ARG, "md state arrays missing");
  if (n_steps > 0 && !(st->dt > 0)) return fail(ctx, AP_ERR_ARG, "dt must be > 0");
  hipStream_t s = (hipStream_t)stream;
  ap_status r;
  SysView sv;
  if ((r = prepare_systems(ctx, sys, &sv))) return r;
  const int64_t N = sv.n_atoms;
  const bool nvt = st->nvt != nullptr && n_steps > 0;
  if (nvt) {
    if (!(st->nvt_T > 0) || !(st->nvt_tau > 0) || !st->nvt_xi)
      return fail(ctx, AP_ERR_ARG, "Nose-Hoover layer needs nvt_T > 0, nvt_tau > 0 and nvt_xi");
    if ((r = ensure(ctx, ctx->nvt_ke, 16 * (size_t)std::max<int64_t>(N, 1))) ||
        (r = ensure(ctx, ctx->nvt_sums, 16 * (size_t)sv.n_sys)) ||
        (r = ensure(ctx, ctx->nvt_fac, 8 * (size_t)sv.n_sys)))
      return r;
  }
  double* nvt_sums = (double*)ctx->nvt_sums.p;
  double* nvt_fac = (double*)ctx->nvt_fac.p;
  // layer sums of m v^2 and atom counts of the current velocities
  auto layer_sums = [&]() -> ap_status {
    {
      PhaseTimer timer(ctx, AP_PHASE_INTEGRATE, s);
      AP_HIP(launch_nvt_ke((int32_t)N, st->vel, st->mass, st->nvt, st->fixed, (double*)ctx->nvt_ke.p, s));
    }
    return reduce_into(ctx, sv, (const double*)ctx->nvt_ke.p, 2, nvt_sums, false, s);
  };
  if (n_steps == 0) {
    if ((r = force_eval(ctx, sys, st, s))) return r;
  }
  if (nvt && (r = layer_sums())) return r;
  for (int step = 0; step < n_steps; ++step) {
    {
      PhaseTimer timer(ctx, AP_PHASE_INTEGRATE, s);
      if (nvt) AP_HIP(launch_nvt_half(sv.n_sys, nvt_sums, st->nvt_xi, nvt_fac, st->nvt_T, st->nvt_tau,
                                      st->dt, s));
      AP_HIP(launch_kick_drift((int32_t)N, sv, st->pos, st->vel, st->force, st->mass, st->fixed,
                               st->nvt, nvt ? nvt_fac : nullptr, st->dt, true, s));
    }
    for (int k = 0; k < 3; ++k) st->ind_centre[k] += st->dt * st->ind_vel[k];
    if ((r = force_eval(ctx, sys, st, s))) return r;
    {
      PhaseTimer timer(ctx, AP_PHASE_INTEGRATE, s);
      AP_HIP(launch_kick_drift((int32_t)N, sv, st->pos, st->vel, st->force, st->mass, st->fixed,
                               nullptr, nullptr, st->dt, false, s));
    }
    if (nvt) {
      if ((r = layer_sums())) return r;
      PhaseTimer timer(ctx, AP_PHASE_INTEGRATE, s);
      AP_HIP(launch_nvt_half(sv.n_sys, nvt_sums, st->nvt_xi, nvt_fac, st->nvt_T, st->nvt_tau, st->dt, s));
      AP_HIP(launch_nvt_scale((int32_t)N, sv, st->vel, st->nvt, st->fixed, nvt_fac, s));
    }
    if (st->check_every > 0 && (step + 1) % st->check_every == 0) {
      AP_HIP(launch_check_finite((int32_t)N, st->force, (int32_t*)ctx->flags.p + 1, s));
      if ((r = ap_check(c, s))) return r;
    }
  }
  if (st->e_sys && (r = ap_reduce_energy(c, sys, st->e_atom, st->e_sys, s))) return r;
  return AP_OK;
}

static void prof_drain(Ctx* ctx) {
  for (auto& e : ctx->evs) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      ctx->prof_ms[e.phase] += ms;
      ctx->prof_calls[e.phase] += 1;
    }
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  ctx->evs.clear();
}

ap_status ap_profile(ap_ctx* c, int32_t enable) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  prof_drain(ctx);
  if (enable) {
    for (int k = 0; k < AP_N_PHASES; ++k) {
      ctx->prof_ms[k] = 0;
      ctx->prof_calls[k] = 0;
    }
  }
  ctx->prof = enable != 0;
  return AP_OK;
}

ap_status ap_profile_read(ap_ctx* c, double* ms, int64_t* calls, int32_t n) {
  Ctx* ctx = (Ctx*)c;
  if (!ctx) return fail(nullptr, AP_ERR_ARG, "ctx is NULL");
  if (n < 0 || n > AP_N_PHASES) return fail(ctx, AP_ERR_ARG, "n must be in [0, AP_N_PHASES]");
  prof_drain(ctx);
  for (int k = 0; k < n; ++k) {
    if (ms) ms[k] = ctx->prof_ms[k];
    if (calls) calls[k] = ctx->prof_calls[k];
  }
  return AP_OK;
}

ap_status ap_info(const ap_ctx* c, const char* key, double* value) {
  const Ctx* ctx = (const Ctx*)c;
  if (!ctx || !key || !value) return fail(nullptr, AP_ERR_ARG, "ctx/key/value is NULL");
  const std::string k(key);
  if (k == "ace.flops_atom") *value = ctx->flops_atom;
  else if (k == "ace.flops_contract") *value = ctx->flops_contract;
  else if (k == "ace.flops_bond") *value = ctx->flops_bond;
  else if (k == "ace.nnz") *value = ctx->nnz;
  else if (k == "ace.x_rows") *value = ctx->x_rows;
  else if (k == "ace.a_size") *value = ctx->ace.nA;
  else if (k == "eam.flops_bond") *value = 80.0;
  else if (k == "ace.mfma_tiles") *value = ctx->mix_tiles;
  else if (k == "ace.mfma_flops_atom") *value = ctx->mix_mfma_flops;
  else if (k == "ace.rank_mode") *value = ctx->last_rank_mode;
  else return fail(const_cast<Ctx*>(ctx), AP_ERR_ARG, "unknown info key");
  return AP_OK;
}

}  // extern "C"
