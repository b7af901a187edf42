/*
 * ap.h - C ABI of the adaptive-precision (AP) EAM/ACE force path on AMD
 * MI355X (gfx950).
 *
 * The method (Immel, Mrovec, Drautz, Sutmann, arXiv 2505.12958, section
 * "Adaptive-precision potential", equation for E_i of the AP potential):
 *
 *     E = sum_i [ lambda_i E_i^ACE + (1 - lambda_i) E_i^EAM ]   (+ indenter)
 *
 * with a per-atom switching parameter lambda_i in [0, 1].  NOTE: in this ABI
 * lambda is the weight of the *accurate* ACE potential (lambda = 1: pure
 * ACE); the paper's switching parameter is 1 - lambda.  Forces are
 * F = -dE/dr at fixed lambda (lambda is an input of each evaluation).
 *
 * EAM per-atom energy: section "EAM potential", E_i^EAM = xi(sum_j zeta(r_ij))
 * + 1/2 sum_j Phi(r_ij), the three functions given as tables (ap_table).
 * ACE per-atom energy: section "Atomic cluster expansion", E_i^ACE =
 * phi^(1) + sqrt(phi^(2)), evaluated as phi^(1) + sqrt(|phi^(2)| + 1e-6)
 * (finite for phi^(2) <= 0), with phi^(p) = sum_v c_v^(p) B_v over the
 * product basis of ap_ace_model.
 * Indenter: section "Nanoindentation", V_ind = K/3 (R - delta)^3 for
 * delta = |r - r_ind| < R; load = sum of indenter forces along `dir`.
 *
 * Units: Angstrom, eV, amu, fs; forces eV/A; virial eV.
 *
 * Memory: every pointer is a DEVICE pointer owned by the caller unless
 * marked [host].  Arrays of atoms are structure-of-arrays: pos[3][n_atoms]
 * (x block, then y, then z), force[3][n_atoms], vel[3][n_atoms].  The
 * library owns only what ap_create allocates (model tables, scratch space
 * that grows on demand; it is freed by ap_destroy).
 *
 * Streams: `stream` is a hipStream_t (NULL = default stream).  Calls enqueue
 * work on it and return without waiting, except where a host out-parameter
 * needs a device value (needed_capacity, ap_check) - those synchronise the
 * stream.  A context is not thread safe; use one context per stream.
 *
 * Errors: every call returns ap_status; nothing throws across the ABI.
 * Arguments are validated on the host before anything is enqueued; on error
 * the outputs are unspecified (except needed_capacity) and ap_last_error()
 * holds a message.  Device-side conditions (neighbour-list overflow,
 * non-finite forces) are latched in the context and reported by the next
 * synchronising call (ap_check, ap_build_neighbors with needed_capacity,
 * ap_step with check_every > 0).  An asynchronous HIP fault surfaces as
 * AP_ERR_HIP from the next call that synchronises.
 *
 * Determinism: no floating-point atomics in either precision; forces are
 * gathered with a reverse-slot index and every sum has a fixed order (the
 * mixed path's partial phi sums of a rank are added slot by slot), so results
 * are bitwise reproducible run to run.  Integer atomics (work queues, cell
 * counts, overflow maxima, the switching spread's maximum over FP64 bit
 * patterns of non-negative values) do not affect results.
 */
#ifndef AP_H
#define AP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ap_ctx ap_ctx;

typedef enum {
  AP_OK = 0,
  AP_ERR_ARG = 1,          /* null pointer, negative size, bad enum, inconsistent sizes */
  AP_ERR_NBR_CAPACITY = 2, /* a neighbour list holds more than nl->capacity entries */
  AP_ERR_BOX = 3,          /* a periodic cell is narrower than 2*cutoff, or bad geometry */
  AP_ERR_NONFINITE = 4,    /* a non-finite energy or force was detected */
  AP_ERR_HIP = 5,          /* a HIP runtime call failed */
  AP_ERR_NOMEM = 6,        /* device allocation failed */
  AP_ERR_UNSUPPORTED = 7   /* valid request that this build does not implement */
} ap_status;

typedef enum { AP_PREC_FP64 = 0, AP_PREC_MIXED = 1 } ap_precision;

#define AP_OVERWRITE 0u   /* outputs (e_atom, force, virial) are written */
#define AP_ACCUMULATE 1u  /* outputs are added to, in stream order */

/* A batch of independent systems whose atoms are concatenated.
 * Atoms of system s are [sys_offset[s], sys_offset[s+1]).  Each box is a
 * 3x3 matrix whose ROWS are the lattice vectors a, b, c (r = s_frac * H).
 * Orthorhombic boxes (all off-diagonals exactly 0) may be periodic in any
 * subset of dimensions; positions in a periodic dimension must lie in
 * [0, L).  Triclinic boxes must be periodic in all three dimensions.
 * Canonical displacement d = r_j - r_i (bit-exact neighbour lists):
 *   orthorhombic: d = x_j - x_i; periodic dim: if d > L/2 then d -= L else
 *     if d < -L/2 then d += L;
 *   triclinic: s = r H^-1 with s_k = (x Hi[0][k] + y Hi[1][k]) + z Hi[2][k]
 *     (Hi from the cofactor formula, scalar FP64), ds = s_j - s_i wrapped at
 *     +-0.5 the same way, d_k = (ds0 H[0][k] + ds1 H[1][k]) + ds2 H[2][k];
 *   r^2 = (dx dx + dy dy) + dz dz, every operation rounded separately.
 *   j != i is a neighbour iff r^2 < cutoff*cutoff.
 * Every periodic cell must be at least 2*cutoff wide (AP_ERR_BOX). */
typedef struct {
  int32_t n_systems;
  int64_t n_atoms;
  const int64_t* sys_offset; /* [host] n_systems + 1 */
  const double* box;         /* [host] n_systems * 9, row-major, rows = lattice vectors */
  uint8_t periodic[3];
  double cutoff;
} ap_systems;

/* Full neighbour lists in slot-major ELL layout: the s-th neighbour of atom
 * i is nbr[s * n_atoms + i] (s < count[i]), sorted by ascending index;
 * rev[s * n_atoms + i] is the slot of i in the list of nbr[s * n_atoms + i].
 * nbr and rev hold capacity * n_atoms int32 each, count n_atoms.
 * rev is optional (NULL): ap_build_neighbors then does not build it, and
 * ap_ace_forces derives the reverse slots it needs (pairs whose first atom
 * is ACE-listed) in library scratch; results are identical either way. */
typedef struct {
  int32_t* nbr;
  int32_t* count;
  int32_t* rev;
  int32_t capacity;
} ap_nlist;

/* A function tabulated on uniform knots x_k = x0 + k*dx, k = 0..n_knots-1,
 * stored as one cubic per interval: coef[4k + p], value = sum_p coef[4k+p]
 * t^p with t = x - x_k.  Interval k = clamp(floor((x - x0)/dx), 0, n-2);
 * below x0 the first cubic is used; beyond the last knot Phi and zeta are 0
 * and F continues linearly with its end slope. */
typedef struct {
  double x0, dx;
  int32_t n_knots;
  const double* coef; /* [host] (n_knots - 1) * 4 */
} ap_table;

typedef struct {
  ap_table phi; /* pair potential Phi(r) */
  ap_table rho; /* density zeta(r) */
  ap_table F;   /* embedding xi(rho) */
} ap_eam_tables;

/* Single-species ACE model.
 * Radial basis g_k(r) = T_k(2r/r_c - 1) (1 + cos(pi r/r_c))/2, k < K;
 * R_nl(r) = sum_k W[(n*(l_max+1) + l)*K + k] g_k(r).
 * A_nlm = sum_j R_nl(r_ij) Y_lm(unit d_ij), real orthonormal Y_lm
 * (Y_l0 = Y_l^0, Y_{l,m>0} = sqrt2 (-1)^m Re Y_l^m, Y_{l,m<0} = sqrt2 (-1)^m
 * Im Y_l^|m|, Condon-Shortley phase in Y_l^m).
 * Coupled pairs AA_{(a,b),L,M} = sum C^{la lb L}_{m1 m2 M} A_{a m1} A_{b m2}
 * with the real-basis Clebsch-Gordan coefficients (l_a + l_b + L even).
 * funcs[10*v ..] = nu, n1,l1, n2,l2, n3,l3, n4,l4, L (unused = -1):
 *   nu=1: B = A_{n1 0 0}; nu=2: B = AA_{(1,2),0,0};
 *   nu=3: B = sum_M AA_{(1,2),L,M} A_{(n3,l3),M} with L = l3;
 *   nu=4: B = sum_M AA_{(1,2),L,M} AA_{(3,4),L,M}.
 * Single indices (n,l) are ordered by n then l, and each function lists
 * them in non-decreasing order.  Limits: l_max <= 4, n_max <= 16, K <= 16,
 * nu_max <= 4. */
typedef struct {
  int32_t n_max, l_max, nu_max, K;
  double r_c;
  const double* W;      /* [host] n_max * (l_max+1) * K */
  int32_t n_funcs;
  const int32_t* funcs; /* [host] n_funcs * 10 */
  const double* c1;     /* [host] n_funcs, coefficients of phi^(1) */
  const double* c2;     /* [host] n_funcs, coefficients of phi^(2) */
} ap_ace_model;

typedef enum {
  AP_LAMBDA_CONST = 0,      /* lambda = value */
  AP_LAMBDA_SPHERE = 1,     /* cosine-tapered ball */
  AP_LAMBDA_HEMISPHERE = 2, /* ball centred on the first-contact surface point */
  AP_LAMBDA_MASK = 3,       /* hemisphere, raised to 1 where mask[i] != 0 */
  AP_LAMBDA_GIVEN = 4       /* lambda is an input (values in [0, 1]); only the list is built */
} ap_lambda_kind;

/* Switching rule (section "Adaptive-precision potential": precise region
 * under the indenter, fast surface outside it, detector-selected atoms).
 * Geometric part: delta = |r - centre| (plain Euclidean), lambda = 1 for
 * delta <= r_full, (1 + cos(pi (delta - r_full)/taper))/2 below
 * r_full + taper, 0 beyond.  For kinds 1-3, atoms with z >= z_surface_min
 * whose geometric lambda is 0 get lambda = 0 (also overriding the mask). */
typedef struct {
  int32_t kind;
  double value;
  double centre[3];
  double r_full, taper;
  double z_surface_min;
  const uint8_t* mask; /* device, n_atoms, kind 3 only */
} ap_lambda_rule;

/* Dynamic switching (section "Adaptive-precision potential": the switching
 * parameter follows the centro-symmetry parameter (CSP) during the run, with
 * fixed zones; appendix "Switching function" and the table of the
 * adaptive-precision model's parameters).  One update, in this order, with
 * mu = the ACE weight (1 - the paper's lambda):
 *   CSP_i = sum of the n_csp/2 smallest |d_a + d_b|^2 over the pairs of the
 *     n_csp nearest neighbours (ranked by the canonical r^2, ties by index),
 *     summed in ascending order; (n_csp/2) (2 cutoff)^2 for atoms with fewer
 *     than n_csp neighbours;
 *   csp_avg_i <- csp_avg_i + (CSP_i - csp_avg_i) / n_csp_avg;
 *   mu0_i = 0 for csp_avg_i <= csp_lo, 1 for >= csp_hi, between
 *     (1 - cos(pi (csp_avg_i - csp_lo)/(csp_hi - csp_lo)))/2; then 1 inside
 *     the precise ball (|r_i - centre|^2 <= r_precise^2), else 0 for atoms
 *     with z_i >= z_surface_min (fast surface);
 *   mu_i = max over j with r_ij^2 < r_hi^2 of mu0_j g(r_ij), g = 1 for
 *     r <= r_lo, (1 + cos(pi (r - r_lo)/(r_hi - r_lo)))/2 below r_hi;
 *   lambda_avg_i <- lambda_avg_i + (mu_i - lambda_avg_i) / n_lambda_avg;
 *   lambda_i = lambda_avg_i, set to 0 below dlambda_min and to 1 above
 *     1 - dlambda_min.
 * The first update (initialised == 0) sets both averages to the current
 * values.  The paper's values for W: n_csp 14, csp_lo 1.5, csp_hi 1.6 A^2,
 * n_csp_avg = n_lambda_avg = 110, r_lo 4, r_hi 12 A, dlambda_min 0.01. */
typedef struct {
  double csp_lo, csp_hi;   /* A^2, csp_lo < csp_hi */
  int32_t n_csp;           /* neighbours in the CSP: even, 2..16 */
  int32_t n_csp_avg;       /* length of the CSP time average (updates), >= 1 */
  double r_lo, r_hi;       /* spatial transition zone (A), 0 <= r_lo < r_hi */
  int32_t n_lambda_avg;    /* length of the time average of mu, >= 1 */
  double dlambda_min;      /* snapping width, in [0, 0.5) */
  double centre[3];        /* centre of the precise ball (first-contact point) */
  double r_precise;        /* its radius; <= 0: no precise ball */
  double z_surface_min;    /* surface zone outside the ball: z >= this */
  double* csp_avg;         /* device [n_atoms]: state, caller-owned */
  double* lambda_avg;      /* device [n_atoms]: state, caller-owned */
  int32_t initialised;     /* [host] 0 before the first update; set to 1 by it */
} ap_switching;

/* The paper's W EAM in closed form (appendix "AP potential for tungsten":
 * equations eam_F_Marinica, eam_Phi_Marinica, eam_rho_Marinica,
 * tungsten_rho_up, tungsten_F_up, tungsten_Phi_up and the table of optimised
 * parameters), evaluated in FP64 by the EAM kernels instead of tables:
 *   xi(x)    = a_xi1 sqrt(x) + a_xi2 x^2 + d_xi   (x <= 0: a_xi2 x^2 + d_xi);
 *   zeta(r)  = zeta_0(max(r, r_cut_rho)), zeta_0(r) = sum_i a_rho[i] (d_rho[i] - r)^3
 *              over the knots with d_rho[i] >= r;
 *   Phi(r)   = z^2 / (4 pi eps0 r) sum_k zbl_c[k] exp(-zbl_q[k] r / a_zbl) for
 *              r < r_lo; sum_m b_phi[m] r^m for r_lo <= r <= r_hi; the knot sum
 *              of (a_phi, d_phi) above r_hi.
 * Units: eps0 in e^2/(eV A).  Pair terms end at the neighbour-list cutoff. */
typedef struct {
  int32_t n_phi;               /* knots of the pair sum, <= 32 */
  const double* a_phi;         /* [host] n_phi */
  const double* d_phi;         /* [host] n_phi */
  int32_t n_rho;               /* knots of the density sum, <= 32 */
  const double* a_rho;         /* [host] n_rho */
  const double* d_rho;         /* [host] n_rho */
  double r_cut_rho;
  double a_xi1, a_xi2, d_xi;
  double z, eps0, a_zbl;
  double zbl_c[4], zbl_q[4];
  double r_lo, r_hi;
  double b_phi[6];
} ap_eam_analytic;

/* Create a context on HIP device `device`.  eam and/or ace may be NULL (the
 * matching force call then returns AP_ERR_ARG).  The model is copied and
 * folded into device tables; host arrays may be freed afterwards. */
ap_status ap_create(ap_ctx** out, int32_t device, int32_t precision,
                    const ap_eam_tables* eam, const ap_ace_model* ace);
ap_status ap_destroy(ap_ctx* ctx);
/* Message of the last failing call on ctx (or of ap_create when ctx is NULL);
 * never NULL. */
const char* ap_last_error(const ap_ctx* ctx);

/* Cell-list neighbour build (27-cell stencil, FP64 canonical test).  If
 * needed_capacity is non-NULL the call synchronises and, on overflow,
 * returns AP_ERR_NBR_CAPACITY with *needed_capacity = the largest count;
 * if it is NULL an overflow is latched and reported by ap_check. */
ap_status ap_build_neighbors(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                             const ap_nlist* nl, int32_t* needed_capacity, void* stream);

/* Switching parameter lambda[n_atoms] (ACE weight) from the rule, and the
 * ascending list of atoms with lambda > 0: ace_list[0 .. *n_ace).  With
 * AP_LAMBDA_GIVEN, lambda is read (not written) and only the list is built. */
ap_status ap_blend(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                   const ap_lambda_rule* rule, double* lambda, int32_t* ace_list,
                   int32_t* n_ace, void* stream);

/* Use the closed-form EAM (ap_eam_analytic) in ctx instead of tables: it
 * replaces the tables given to ap_create, or adds EAM to a context created
 * without them.  The parameters are copied. */
ap_status ap_set_eam_analytic(ap_ctx* ctx, const ap_eam_analytic* eam);

/* Forces of a switching parameter that follows the positions (section
 * "Adaptive-precision potential": E = sum_i [lambda_i E_i^ACE + (1 - lambda_i)
 * E_i^EAM] with lambda_i = lambda(r_i) of a geometric rule).  For the rule
 * kinds 1-3 it adds -(E_i^ACE - E_i^EAM) d lambda_i / d r_i to force[3][n]
 * on every atom of the cosine band (0 < lambda_i < 1; masked and surface
 * atoms have lambda 0 or 1 and no gradient), using the unweighted per-atom
 * energies of the last ap_eam_forces and ap_ace_forces calls on this context
 * (same positions and lambda); virial (NULL: skipped) gets
 * -sum_i (r_i - centre) (x) (E_i^ACE - E_i^EAM) d lambda_i / d r_i added.
 * With it the forces are the full -dE/dr of that energy.  Other rule kinds
 * add nothing. */
ap_status ap_lambda_gradient(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                             const ap_lambda_rule* rule, const double* lambda, double* force,
                             double* virial, void* stream);

/* One update of the dynamic switching rule (ap_switching): lambda[n_atoms]
 * (ACE weight) and the ascending list ace_list[0 .. *n_ace) of atoms with
 * lambda > 0.  nl must be the list ap_build_neighbors built on this context
 * at these positions (its cell list is reused for the transition zone).
 * Orthorhombic systems only (else AP_ERR_UNSUPPORTED); r_hi and every
 * periodic width must satisfy 2 r_hi <= width (else AP_ERR_BOX).
 * Deterministic: every decision is taken on FP64 values in a fixed order and
 * the transition zone is a maximum. */
ap_status ap_switching_update(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                              const ap_nlist* nl, ap_switching* sw, double* lambda,
                              int32_t* ace_list, int32_t* n_ace, void* stream);

/* ap_blend for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as ap_blend; it allocates nothing and
 * uploads nothing.  Its per-atom flags and the compaction's partial sums live
 * in a static device array of the library (one copy per GPU, about 16 MB,
 * held until the process ends), so n_atoms <= AP_BLEND_NOALLOC_MAX_ATOMS
 * (larger systems: AP_ERR_ARG, nothing enqueued).  The context's device must
 * be current (else AP_ERR_ARG).  Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (on different streams or host threads) race;
 * calls ordered on one stream do not. */
#define AP_BLEND_NOALLOC_MAX_ATOMS 4000000
ap_status ap_blend_noalloc(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                           const ap_lambda_rule* rule, double* lambda, int32_t* ace_list,
                           int32_t* n_ace, void* stream);

/* EAM part weighted by w_i = 1 - lambda_i (lambda NULL: w = 1).
 * e_atom[i] = w_i E_i^EAM; force = -dE/dr of sum_i w_i E_i^EAM;
 * virial[s*9 + 3a + b] = -sum_{i in s} sum_j d_ij,a G_ij,b (NULL: skipped). */
ap_status ap_eam_forces(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                        const ap_nlist* nl, const double* lambda, double* e_atom, double* force,
                        double* virial, uint32_t flags, void* stream);

/* ACE part weighted by lambda_i over atoms ace_list[0 .. *n_ace) (ace_list
 * NULL: every atom, n_ace ignored; lambda NULL: lambda = 1).  Atoms outside
 * the list contribute nothing but still receive forces from listed
 * neighbours.  Outputs as ap_eam_forces. */
ap_status ap_ace_forces(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                        const ap_nlist* nl, const double* lambda, const int32_t* ace_list,
                        const int32_t* n_ace, double* e_atom, double* force, double* virial,
                        uint32_t flags, void* stream);

/* Spherical indenter on every atom with fixed[i] == 0 (fixed NULL: all).
 * Adds its forces to force; e_ind and load (device scalars, may be NULL)
 * receive the energy and the load along unit vector dir[3] (host). */
ap_status ap_indenter(ap_ctx* ctx, const ap_systems* sys, const double* pos,
                      const uint8_t* fixed, const double* centre, double R, double K,
                      const double* dir, double* force, double* e_ind, double* load,
                      void* stream);

/* e_sys[s] = sum of e_atom over system s in a fixed order (bitwise
 * reproducible). */
ap_status ap_reduce_energy(ap_ctx* ctx, const ap_systems* sys, const double* e_atom,
                           double* e_sys, void* stream);

/* Molecular-dynamics state for ap_step.  Device arrays are caller-owned;
 * ind_* are host values that ap_step advances. */
typedef struct {
  double* pos;            /* [3][n_atoms] */
  double* vel;            /* [3][n_atoms] A/fs */
  double* force;          /* [3][n_atoms] */
  double* e_atom;         /* [n_atoms] */
  double* lambda;         /* [n_atoms] */
  const double* mass;     /* [n_atoms] amu */
  const uint8_t* fixed;   /* [n_atoms] or NULL (nothing fixed) */
  int32_t* ace_list;      /* [n_atoms] */
  int32_t* n_ace;         /* device scalar */
  ap_nlist nl;
  ap_lambda_rule rule;
  double dt;              /* fs */
  double ind_centre[3];   /* [host] indenter centre, advanced by ind_vel*dt per step */
  double ind_vel[3];      /* [host] A/fs */
  double ind_dir[3];      /* [host] unit vector of the load */
  double ind_R, ind_K;    /* K <= 0: no indenter */
  double* virial;         /* [n_systems*9] or NULL */
  double* e_sys;          /* [n_systems] or NULL (reduced after the last step) */
  double* e_ind;          /* device scalar or NULL */
  double* load;           /* device scalar or NULL */
  int32_t check_every;    /* > 0: synchronise and check overflow / finiteness every k steps */
  ap_switching* switching;/* [host] non-NULL: lambda from ap_switching_update every evaluation
                             (after the neighbour build) instead of `rule` */
  int32_t lambda_gradient;/* nonzero (geometric rule, EAM and ACE): forces include the
                             term of ap_lambda_gradient */
  const uint8_t* nvt;     /* [n_atoms] or NULL: nonzero marks the atoms of the Nose-Hoover layer
                             (section "Nanoindentation"); an atom also marked fixed stays fixed
                             and is not counted */
  double nvt_T;           /* layer target temperature, K (> 0 when nvt is set) */
  double nvt_tau;         /* thermostat time constant, fs (> 0 when nvt is set) */
  double* nvt_xi;         /* [n_systems][2] device, caller-owned: the thermostat rate xi (1/fs)
                             and its time integral eta; zero them before the first step.  The
                             conserved quantity is K + U + 3 n_layer k_B T0 (tau^2 xi^2/2 + eta). */
} ap_md_state;

/* n_steps == 0: one force evaluation at the current positions
 * (blend, neighbours, EAM, ACE, indenter, reductions).  n_steps > 0:
 * velocity-Verlet steps (half kick, drift with periodic wrap, indenter move,
 * force evaluation, half kick; fixed atoms never move and keep v = 0).
 * With a Nose-Hoover layer (st->nvt) each step is thermostat(dt/2), kick,
 * drift, forces, kick, thermostat(dt/2), one thermostat per system: its half
 * step advances xi by dt/4 (T/T0 - 1)/tau^2, eta by xi dt/2, scales the
 * layer's velocities by exp(-xi dt/2) and advances xi again with the scaled
 * temperature T = sum m v^2 / (3 n_layer k_B) (deterministic sums).
 * The forces in st->force must be those of the current positions when
 * n_steps > 0 (call once with n_steps = 0 first). */
ap_status ap_step(ap_ctx* ctx, const ap_systems* sys, ap_md_state* st, int32_t n_steps,
                  void* stream);

/* Synchronise the stream and report latched device conditions
 * (AP_ERR_NBR_CAPACITY, AP_ERR_NONFINITE) or an asynchronous HIP error;
 * clears the latch. */
ap_status ap_check(ap_ctx* ctx, void* stream);

/* Per-phase GPU timing with HIP events recorded on each call's stream around
 * the kernels of a phase (AP_PHASE_ACE brackets exactly the launch of the
 * kernel that does the ACE contraction).  ap_profile(ctx, 1) clears the totals and starts recording,
 * ap_profile(ctx, 0) stops.  ap_profile_read synchronises the device and
 * returns, for the first n phases, the accumulated milliseconds (ms[n]) and
 * the number of timed launches (calls[n]); either pointer may be NULL. */
enum {
  AP_PHASE_NEIGHBORS = 0,
  AP_PHASE_BLEND = 1,
  AP_PHASE_EAM = 2,
  AP_PHASE_ACE = 3,
  AP_PHASE_ACE_GATHER = 4,
  AP_PHASE_INDENTER = 5,
  AP_PHASE_INTEGRATE = 6,
  AP_PHASE_REDUCE = 7,
  AP_PHASE_ACE_BOND = 8, /* mixed path: bond basis and bond-gradient kernels */
  AP_N_PHASES = 9
};
ap_status ap_profile(ap_ctx* ctx, int32_t enable);
ap_status ap_profile_read(ap_ctx* ctx, double* ms, int64_t* calls, int32_t n);

/* Algorithmic work counts of the loaded model, by key:
 *   "ace.flops_atom"     FLOPs per ACE-active atom of the coupling, folded
 *                        contraction (both coefficient sets) and adjoint;
 *   "ace.flops_contract" the folded-contraction part of ace.flops_atom;
 *   "ace.flops_bond"     FLOPs per bond of the radial/harmonic basis, the A
 *                        accumulation and the bond gradient;
 *   "ace.nnz"            non-zeros of the folded coefficient matrices;
 *   "ace.x_rows"         rows of the coupled vectors X_L summed over L;
 *   "ace.a_size"         length of the atomic basis A;
 *   "eam.flops_bond"     FLOPs per bond of the two EAM passes;
 *   "ace.mfma_tiles"     stored 16x32 coefficient tiles of the mixed path;
 *   "ace.mfma_flops_atom" executed MFMA FLOPs per ACE atom of the mixed path
 *                        (three split products over the dense tiles);
 *   "ace.rank_mode"      launch mode of the last mixed rank phase (-1: none).
 * Returns AP_ERR_ARG for an unknown key. */
ap_status ap_info(const ap_ctx* ctx, const char* key, double* value);

/* Library version string, e.g. "ap 0.1 gfx950". */
const char* ap_version(void);

#ifdef __cplusplus
}
#endif
#endif /* AP_H */
