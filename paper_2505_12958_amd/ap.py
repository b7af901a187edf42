"""Python binding of the AP C ABI (include/ap.h): argument marshalling only.

Every step of the path runs in the HIP kernels of ``libap.so``; this module
only converts torch device tensors and numpy model arrays into the C
structs and calls the library on the current HIP stream.  There is no CPU
fallback: if the library or a GPU is missing, loading fails loudly.

Layout: positions, velocities and forces are (3, N) float64 device tensors
(structure of arrays); lambda and per-atom energies are (N,) float64; the
virial is (n_systems, 9) float64 with entry 3a+b = -sum d_a G_b.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libap.so")

AP_OK, AP_ERR_ARG, AP_ERR_NBR_CAPACITY, AP_ERR_BOX, AP_ERR_NONFINITE, AP_ERR_HIP, AP_ERR_NOMEM, \
    AP_ERR_UNSUPPORTED = range(8)
AP_PREC_FP64, AP_PREC_MIXED = 0, 1
AP_OVERWRITE, AP_ACCUMULATE = 0, 1
STATUS = {0: "AP_OK", 1: "AP_ERR_ARG", 2: "AP_ERR_NBR_CAPACITY", 3: "AP_ERR_BOX",
          4: "AP_ERR_NONFINITE", 5: "AP_ERR_HIP", 6: "AP_ERR_NOMEM", 7: "AP_ERR_UNSUPPORTED"}


class APError(RuntimeError):
    def __init__(self, status, msg, needed=None):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.needed = needed


class Systems(C.Structure):
    _fields_ = [("n_systems", C.c_int32), ("n_atoms", C.c_int64), ("sys_offset", C.POINTER(C.c_int64)),
                ("box", C.POINTER(C.c_double)), ("periodic", C.c_uint8 * 3), ("cutoff", C.c_double)]


class NList(C.Structure):
    _fields_ = [("nbr", C.c_void_p), ("count", C.c_void_p), ("rev", C.c_void_p), ("capacity", C.c_int32)]


class Table(C.Structure):
    _fields_ = [("x0", C.c_double), ("dx", C.c_double), ("n_knots", C.c_int32),
                ("coef", C.POINTER(C.c_double))]


class EamTables(C.Structure):
    _fields_ = [("phi", Table), ("rho", Table), ("F", Table)]


class AceModel(C.Structure):
    _fields_ = [("n_max", C.c_int32), ("l_max", C.c_int32), ("nu_max", C.c_int32), ("K", C.c_int32),
                ("r_c", C.c_double), ("W", C.POINTER(C.c_double)), ("n_funcs", C.c_int32),
                ("funcs", C.POINTER(C.c_int32)), ("c1", C.POINTER(C.c_double)),
                ("c2", C.POINTER(C.c_double))]


class LambdaRule(C.Structure):
    _fields_ = [("kind", C.c_int32), ("value", C.c_double), ("centre", C.c_double * 3),
                ("r_full", C.c_double), ("taper", C.c_double), ("z_surface_min", C.c_double),
                ("mask", C.c_void_p)]


class EamAnalytic(C.Structure):
    _fields_ = [("n_phi", C.c_int32), ("a_phi", C.POINTER(C.c_double)), ("d_phi", C.POINTER(C.c_double)),
                ("n_rho", C.c_int32), ("a_rho", C.POINTER(C.c_double)), ("d_rho", C.POINTER(C.c_double)),
                ("r_cut_rho", C.c_double), ("a_xi1", C.c_double), ("a_xi2", C.c_double),
                ("d_xi", C.c_double), ("z", C.c_double), ("eps0", C.c_double), ("a_zbl", C.c_double),
                ("zbl_c", C.c_double * 4), ("zbl_q", C.c_double * 4), ("r_lo", C.c_double),
                ("r_hi", C.c_double), ("b_phi", C.c_double * 6)]


class Switching(C.Structure):
    _fields_ = [("csp_lo", C.c_double), ("csp_hi", C.c_double), ("n_csp", C.c_int32),
                ("n_csp_avg", C.c_int32), ("r_lo", C.c_double), ("r_hi", C.c_double),
                ("n_lambda_avg", C.c_int32), ("dlambda_min", C.c_double),
                ("centre", C.c_double * 3), ("r_precise", C.c_double), ("z_surface_min", C.c_double),
                ("csp_avg", C.c_void_p), ("lambda_avg", C.c_void_p), ("initialised", C.c_int32)]


class MDState(C.Structure):
    _fields_ = [("pos", C.c_void_p), ("vel", C.c_void_p), ("force", C.c_void_p),
                ("e_atom", C.c_void_p), ("lambda_", C.c_void_p), ("mass", C.c_void_p),
                ("fixed", C.c_void_p), ("ace_list", C.c_void_p), ("n_ace", C.c_void_p),
                ("nl", NList), ("rule", LambdaRule), ("dt", C.c_double),
                ("ind_centre", C.c_double * 3), ("ind_vel", C.c_double * 3),
                ("ind_dir", C.c_double * 3), ("ind_R", C.c_double), ("ind_K", C.c_double),
                ("virial", C.c_void_p), ("e_sys", C.c_void_p), ("e_ind", C.c_void_p),
                ("load", C.c_void_p), ("check_every", C.c_int32),
                ("switching", C.POINTER(Switching)), ("lambda_gradient", C.c_int32),
                ("nvt", C.c_void_p), ("nvt_T", C.c_double), ("nvt_tau", C.c_double),
                ("nvt_xi", C.c_void_p)]


_lib = None


def lib():
    """Load libap.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.ap_create.argtypes = [C.POINTER(vp), i32, i32, C.POINTER(EamTables), C.POINTER(AceModel)]
        L.ap_destroy.argtypes = [vp]
        L.ap_last_error.argtypes = [vp]
        L.ap_last_error.restype = C.c_char_p
        L.ap_version.restype = C.c_char_p
        L.ap_build_neighbors.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(NList),
                                         C.POINTER(i32), vp]
        L.ap_blend.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(LambdaRule), vp, vp, vp, vp]
        L.ap_blend_noalloc.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(LambdaRule), vp, vp,
                                       vp, vp]
        L.ap_eam_forces.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(NList), vp, vp, vp, vp,
                                    C.c_uint32, vp]
        L.ap_ace_forces.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(NList), vp, vp, vp, vp, vp,
                                    vp, C.c_uint32, vp]
        L.ap_indenter.argtypes = [vp, C.POINTER(Systems), vp, vp, C.POINTER(d), d, d, C.POINTER(d),
                                  vp, vp, vp, vp]
        L.ap_reduce_energy.argtypes = [vp, C.POINTER(Systems), vp, vp, vp]
        L.ap_step.argtypes = [vp, C.POINTER(Systems), C.POINTER(MDState), i32, vp]
        L.ap_switching_update.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(NList),
                                          C.POINTER(Switching), vp, vp, vp, vp]
        L.ap_lambda_gradient.argtypes = [vp, C.POINTER(Systems), vp, C.POINTER(LambdaRule), vp, vp,
                                         vp, vp]
        L.ap_set_eam_analytic.argtypes = [vp, C.POINTER(EamAnalytic)]
        L.ap_check.argtypes = [vp, vp]
        L.ap_profile.argtypes = [vp, i32]
        L.ap_profile_read.argtypes = [vp, C.POINTER(d), C.POINTER(i64), i32]
        L.ap_info.argtypes = [vp, C.c_char_p, C.POINTER(d)]
        for f in ("ap_profile", "ap_profile_read", "ap_info", "ap_create", "ap_destroy", "ap_build_neighbors", "ap_blend", "ap_blend_noalloc",
                  "ap_switching_update", "ap_lambda_gradient", "ap_set_eam_analytic",
                  "ap_eam_forces", "ap_ace_forces", "ap_indenter", "ap_reduce_energy", "ap_step", "ap_check"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


EXPORTS = ("ap_create", "ap_destroy", "ap_last_error", "ap_build_neighbors", "ap_blend",
           "ap_blend_noalloc", "ap_switching_update", "ap_lambda_gradient", "ap_set_eam_analytic",
           "ap_eam_forces", "ap_ace_forces", "ap_indenter", "ap_reduce_energy", "ap_step",
           "ap_check", "ap_version", "ap_profile", "ap_profile_read", "ap_info")
PHASES = ("neighbors", "blend", "eam", "ace", "ace_gather", "indenter", "integrate", "reduce",
          "ace_bond")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class SystemsArg:
    """Host-side ap_systems with the arrays it points to kept alive."""

    def __init__(self, box, sys_offset, periodic, cutoff):
        self.box = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(-1, 9))
        self.off = np.ascontiguousarray(np.asarray(sys_offset, dtype=np.int64))
        self.c = Systems()
        self.c.n_systems = len(self.box)
        self.c.n_atoms = int(self.off[-1])
        self.c.sys_offset = self.off.ctypes.data_as(C.POINTER(C.c_int64))
        self.c.box = _dptr(self.box)
        for k in range(3):
            self.c.periodic[k] = 1 if periodic[k] else 0
        self.c.cutoff = float(cutoff)

    @classmethod
    def from_workload(cls, wl):
        return cls(wl.box, wl.sys_offset, wl.periodic, wl.cutoff)

    @property
    def n_atoms(self):
        return int(self.off[-1])

    @property
    def n_systems(self):
        return len(self.box)


def rule_struct(rule, mask_dev=None):
    r = LambdaRule()
    r.kind = int(rule.kind)
    r.value = float(rule.value)
    for k in range(3):
        r.centre[k] = float(rule.centre[k])
    r.r_full = float(rule.r_full)
    r.taper = float(rule.taper) if rule.taper else 1.0
    r.z_surface_min = float(rule.z_surface_min)
    r.mask = None if mask_dev is None else mask_dev.data_ptr()
    return r


class NeighbourList:
    """Caller-owned device arrays of an ap_nlist."""

    def __init__(self, n_atoms, capacity=64, device="cuda", with_rev=True):
        self.capacity = int(capacity)
        self.n_atoms = int(n_atoms)
        self.nbr = torch.empty(self.capacity * max(1, n_atoms), dtype=torch.int32, device=device)
        self.rev = torch.empty_like(self.nbr) if with_rev else None
        self.count = torch.empty(max(1, n_atoms), dtype=torch.int32, device=device)

    def struct(self):
        s = NList()
        s.nbr = self.nbr.data_ptr()
        s.count = self.count.data_ptr()
        s.rev = self.rev.data_ptr() if self.rev is not None else None
        s.capacity = self.capacity
        return s

    def rows(self):
        """Host copy: list of neighbour index arrays (ascending)."""
        cnt = self.count.cpu().numpy()[: self.n_atoms]
        nb = self.nbr.cpu().numpy().reshape(self.capacity, -1)[:, : self.n_atoms]
        return [nb[: cnt[i], i].copy() for i in range(self.n_atoms)]


class Context:
    """An ap_ctx with a model (EAM tables and/or ACE model) on one device."""

    def __init__(self, eam=None, ace=None, precision=AP_PREC_FP64, device=0):
        L = lib()
        self.has_eam = eam is not None
        self.has_ace = ace is not None
        self._keep = []
        eam_s = None
        if eam is not None:
            eam_s = EamTables()
            for name, t in (("phi", eam.phi), ("rho", eam.rho), ("F", eam.F)):
                coef = np.ascontiguousarray(t.coef, dtype=np.float64)
                self._keep.append(coef)
                tab = getattr(eam_s, name)
                tab.x0, tab.dx, tab.n_knots = float(t.x0), float(t.dx), int(t.n_knots)
                tab.coef = _dptr(coef)
        ace_s = None
        if ace is not None:
            W = np.ascontiguousarray(ace.W, dtype=np.float64)
            funcs = np.ascontiguousarray(ace.funcs, dtype=np.int32)
            c1 = np.ascontiguousarray(ace.c1, dtype=np.float64)
            c2 = np.ascontiguousarray(ace.c2, dtype=np.float64)
            self._keep += [W, funcs, c1, c2]
            ace_s = AceModel(int(ace.n_max), int(ace.l_max), int(ace.nu_max), int(ace.K), float(ace.r_c),
                             _dptr(W), len(funcs), funcs.ctypes.data_as(C.POINTER(C.c_int32)),
                             _dptr(c1), _dptr(c2))
        h = C.c_void_p()
        st = L.ap_create(C.byref(h), int(device), int(precision),
                         C.byref(eam_s) if eam_s is not None else None,
                         C.byref(ace_s) if ace_s is not None else None)
        if st != AP_OK:
            raise APError(st, L.ap_last_error(None).decode())
        self.h = h
        self.precision = precision
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            lib().ap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, needed=None):
        if st != AP_OK:
            raise APError(st, lib().ap_last_error(self.h).decode(), needed)

    # ---- entry points -------------------------------------------------
    def build_neighbors(self, sysarg, pos, nl, check=True):
        need = C.c_int32(0)
        st = lib().ap_build_neighbors(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(nl.struct()),
                                      C.byref(need) if check else None, _stream())
        self._check(st, need.value)

    def blend(self, sysarg, pos, rule, lam, ace_list, n_ace, mask=None):
        r = rule_struct(rule, mask)
        st = lib().ap_blend(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(r), _ptr(lam),
                            _ptr(ace_list), _ptr(n_ace), _stream())
        self._check(st)

    def set_eam_analytic(self, p):
        """Closed-form EAM from a parameter dict (keys as workloads.W_EAM plus
        zbl = [(c, q)] * 4)."""
        arrs = {k: np.ascontiguousarray(p[k], dtype=np.float64) for k in ("a_phi", "d_phi", "a_rho", "d_rho")}
        e = EamAnalytic()
        e.n_phi, e.a_phi, e.d_phi = len(arrs["a_phi"]), _dptr(arrs["a_phi"]), _dptr(arrs["d_phi"])
        e.n_rho, e.a_rho, e.d_rho = len(arrs["a_rho"]), _dptr(arrs["a_rho"]), _dptr(arrs["d_rho"])
        e.r_cut_rho = p["r_cut_rho"]
        e.a_xi1, e.a_xi2 = p["a_xi"]
        e.d_xi, e.z, e.eps0, e.a_zbl = p["d_xi"], p["Z"], p["eps0"], p["a_zbl"]
        for k, (c, q) in enumerate(p["zbl"]):
            e.zbl_c[k], e.zbl_q[k] = c, q
        e.r_lo, e.r_hi = p["r_lo"], p["r_hi"]
        for m in range(6):
            e.b_phi[m] = p["b_phi"][m]
        self._check(lib().ap_set_eam_analytic(self.h, C.byref(e)))
        self.has_eam = True

    def lambda_gradient(self, sysarg, pos, rule, lam, force, virial=None, mask=None):
        """Add the force (and virial) of a position-dependent geometric lambda."""
        r = rule_struct(rule, mask)
        st = lib().ap_lambda_gradient(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(r), _ptr(lam),
                                      _ptr(force), _ptr(virial), _stream())
        self._check(st)

    def switching_update(self, sysarg, pos, nl, sw, lam, ace_list, n_ace):
        """One update of the dynamic switching rule (sw: DynamicSwitching)."""
        st = lib().ap_switching_update(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(nl.struct()),
                                       C.byref(sw.c), _ptr(lam), _ptr(ace_list), _ptr(n_ace),
                                       _stream())
        self._check(st)

    def blend_noalloc(self, sysarg, pos, rule, lam, ace_list, n_ace, mask=None):
        r = rule_struct(rule, mask)
        st = lib().ap_blend_noalloc(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(r), _ptr(lam),
                                    _ptr(ace_list), _ptr(n_ace), _stream())
        self._check(st)

    def eam_forces(self, sysarg, pos, nl, lam, e_atom, force, virial=None, accumulate=False):
        st = lib().ap_eam_forces(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(nl.struct()), _ptr(lam),
                                 _ptr(e_atom), _ptr(force), _ptr(virial),
                                 AP_ACCUMULATE if accumulate else AP_OVERWRITE, _stream())
        self._check(st)

    def ace_forces(self, sysarg, pos, nl, lam, ace_list, n_ace, e_atom, force, virial=None,
                   accumulate=False):
        st = lib().ap_ace_forces(self.h, C.byref(sysarg.c), _ptr(pos), C.byref(nl.struct()), _ptr(lam),
                                 _ptr(ace_list), _ptr(n_ace), _ptr(e_atom), _ptr(force), _ptr(virial),
                                 AP_ACCUMULATE if accumulate else AP_OVERWRITE, _stream())
        self._check(st)

    def indenter(self, sysarg, pos, fixed, centre, R, K, force, e_ind=None, load=None,
                 direction=(0.0, 0.0, -1.0)):
        c = (C.c_double * 3)(*[float(x) for x in centre])
        dvec = (C.c_double * 3)(*[float(x) for x in direction])
        st = lib().ap_indenter(self.h, C.byref(sysarg.c), _ptr(pos), _ptr(fixed), c, float(R), float(K),
                               dvec, _ptr(force), _ptr(e_ind), _ptr(load), _stream())
        self._check(st)

    def reduce_energy(self, sysarg, e_atom, e_sys):
        st = lib().ap_reduce_energy(self.h, C.byref(sysarg.c), _ptr(e_atom), _ptr(e_sys), _stream())
        self._check(st)

    def step(self, sysarg, state, n_steps):
        st = lib().ap_step(self.h, C.byref(sysarg.c), C.byref(state.c), int(n_steps), _stream())
        self._check(st)
        state.pull_indenter()

    def check(self):
        self._check(lib().ap_check(self.h, _stream()))

    def profile(self, enable):
        self._check(lib().ap_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """{phase: (total_ms, timed_calls)} accumulated since profile(True)."""
        n = len(PHASES)
        ms = (C.c_double * n)()
        calls = (C.c_int64 * n)()
        self._check(lib().ap_profile_read(self.h, ms, calls, n))
        return {PHASES[k]: (ms[k], calls[k]) for k in range(n)}

    def info(self, key):
        v = C.c_double()
        self._check(lib().ap_info(self.h, key.encode(), C.byref(v)))
        return v.value


class MD:
    """Device-resident MD state (ap_md_state) for a workload."""

    def __init__(self, wl, capacity=64, device="cuda", with_rev=False):
        N = wl.n_atoms
        f64 = dict(dtype=torch.float64, device=device)
        self.sys = SystemsArg.from_workload(wl)
        self.pos = torch.tensor(np.ascontiguousarray(wl.pos.T), **f64)
        self.vel = torch.tensor(np.ascontiguousarray(wl.vel.T), **f64)
        self.force = torch.zeros((3, N), **f64)
        self.e_atom = torch.zeros(N, **f64)
        self.lam = torch.zeros(N, **f64)
        self.mass = torch.tensor(wl.masses, **f64)
        self.fixed = torch.tensor(wl.fixed, dtype=torch.uint8, device=device)
        self.ace_list = torch.zeros(max(1, N), dtype=torch.int32, device=device)
        self.n_ace = torch.zeros(1, dtype=torch.int32, device=device)
        self.nl = NeighbourList(N, capacity, device, with_rev)
        self.virial = torch.zeros((wl.n_systems, 9), **f64)
        self.e_sys = torch.zeros(wl.n_systems, **f64)
        self.e_ind = torch.zeros(1, **f64)
        self.load = torch.zeros(1, **f64)
        self.mask = (torch.tensor(wl.rule.mask, dtype=torch.uint8, device=device)
                     if wl.rule.mask is not None else None)
        c = MDState()
        c.pos, c.vel, c.force = self.pos.data_ptr(), self.vel.data_ptr(), self.force.data_ptr()
        c.e_atom, c.lambda_, c.mass = self.e_atom.data_ptr(), self.lam.data_ptr(), self.mass.data_ptr()
        c.fixed = self.fixed.data_ptr()
        c.ace_list, c.n_ace = self.ace_list.data_ptr(), self.n_ace.data_ptr()
        c.nl = self.nl.struct()
        c.rule = rule_struct(wl.rule, self.mask)
        c.dt = float(wl.dt)
        ind = wl.indenter or {}
        K = float(ind.get("K", 0.0))
        for k in range(3):
            c.ind_centre[k] = float(ind["centre"][k]) if K > 0 else 0.0
            c.ind_vel[k] = float(ind["vel"][k]) if K > 0 else 0.0
            c.ind_dir[k] = (0.0, 0.0, -1.0)[k]
        c.ind_R = float(ind.get("R", 1.0)) if K > 0 else 1.0
        c.ind_K = K
        c.virial, c.e_sys = self.virial.data_ptr(), self.e_sys.data_ptr()
        c.e_ind, c.load = self.e_ind.data_ptr(), self.load.data_ptr()
        c.check_every = 0
        c.switching = None
        c.lambda_gradient = 0
        c.nvt, c.nvt_T, c.nvt_tau, c.nvt_xi = None, 0.0, 0.0, None
        self.c = c
        self.switching = None
        self.nvt = None
        self.nvt_xi = None
        self.ind_centre = np.array(c.ind_centre[:])
        self._device = device
        self._n_sys = wl.n_systems

    def use_nvt(self, layer, T, tau):
        """Nose-Hoover thermostat at temperature T (K) with time constant tau
        (fs) on the atoms where `layer` (N booleans) is true; xi and eta
        start at zero (self.nvt_xi, [n_systems][2])."""
        self.nvt = torch.tensor(np.asarray(layer, dtype=np.uint8), device=self._device)
        self.nvt_xi = torch.zeros((self._n_sys, 2), dtype=torch.float64, device=self._device)
        self.c.nvt, self.c.nvt_xi = self.nvt.data_ptr(), self.nvt_xi.data_ptr()
        self.c.nvt_T, self.c.nvt_tau = float(T), float(tau)

    def use_switching(self, sw):
        """Take lambda from the dynamic switching rule sw (DynamicSwitching)
        in every force evaluation of ap_step."""
        self.switching = sw
        self.c.switching = C.pointer(sw.c)

    def pull_indenter(self):
        self.ind_centre = np.array(self.c.ind_centre[:])


AP_LAMBDA_GIVEN = 4


class DynamicSwitching:
    """ap_switching with its device state (time averages) kept alive.

    The paper's values for W (table of the adaptive-precision model's
    parameters) are the defaults; `centre`/`r_precise` give the precise ball
    and `z_surface_min` the fast surface zone."""

    def __init__(self, n_atoms, *, csp_lo=1.5, csp_hi=1.6, n_csp=14, n_csp_avg=110, r_lo=4.0,
                 r_hi=12.0, n_lambda_avg=110, dlambda_min=0.01, centre=(0.0, 0.0, 0.0),
                 r_precise=-1.0, z_surface_min=float("inf"), device="cuda"):
        self.csp_avg = torch.zeros(max(1, n_atoms), dtype=torch.float64, device=device)
        self.lambda_avg = torch.zeros(max(1, n_atoms), dtype=torch.float64, device=device)
        c = Switching()
        c.csp_lo, c.csp_hi, c.n_csp, c.n_csp_avg = csp_lo, csp_hi, n_csp, n_csp_avg
        c.r_lo, c.r_hi, c.n_lambda_avg, c.dlambda_min = r_lo, r_hi, n_lambda_avg, dlambda_min
        for k in range(3):
            c.centre[k] = float(centre[k])
        c.r_precise, c.z_surface_min = float(r_precise), float(z_surface_min)
        c.csp_avg, c.lambda_avg = self.csp_avg.data_ptr(), self.lambda_avg.data_ptr()
        c.initialised = 0
        self.c = c


def given_rule():
    """ap_lambda_rule that takes lambda as an input (only the ACE list is built)."""
    r = LambdaRule()
    r.kind = AP_LAMBDA_GIVEN
    return r


class Evaluator:
    """AP energy, forces and virial at a given (frozen) lambda through the C
    ABI: neighbour build, list of lambda > 0, EAM, ACE, per-system sums.  The
    device buffers are kept between calls (sized for one system layout)."""

    def __init__(self, ctx, sysarg, capacity=64, device="cuda"):
        self.ctx, self.sys = ctx, sysarg
        N = sysarg.n_atoms
        f64 = dict(dtype=torch.float64, device=device)
        self.nl = NeighbourList(N, capacity, device, with_rev=False)
        self.ace_list = torch.zeros(max(1, N), dtype=torch.int32, device=device)
        self.n_ace = torch.zeros(1, dtype=torch.int32, device=device)
        self.e_atom = torch.zeros(N, **f64)
        self.e_sys = torch.zeros(sysarg.n_systems, **f64)
        self.virial = torch.zeros((sysarg.n_systems, 9), **f64)
        self.rule = given_rule()

    def __call__(self, pos_T, lam):
        """pos_T: (3, N) float64, lam: (N,) float64 in [0, 1] (ACE weight).
        Returns (e_sys (n_sys,), force (3, N), virial (n_sys, 9)) as new tensors."""
        ctx, S = self.ctx, self.sys
        pos_T = pos_T.contiguous()
        lam = lam.contiguous()
        N = S.n_atoms
        force = torch.zeros((3, N), dtype=torch.float64, device=pos_T.device)
        ctx.build_neighbors(S, pos_T, self.nl)
        st = lib().ap_blend(ctx.h, C.byref(S.c), _ptr(pos_T), C.byref(self.rule), _ptr(lam),
                            _ptr(self.ace_list), _ptr(self.n_ace), _stream())
        ctx._check(st)
        written = False
        if ctx.has_eam:
            ctx.eam_forces(S, pos_T, self.nl, lam, self.e_atom, force, self.virial)
            written = True
        if ctx.has_ace:
            ctx.ace_forces(S, pos_T, self.nl, lam, self.ace_list, self.n_ace, self.e_atom, force,
                           self.virial, accumulate=written)
        ctx.reduce_energy(S, self.e_atom, self.e_sys)
        return self.e_sys.clone(), force, self.virial.clone()


class APEnergy(torch.autograd.Function):
    """Total AP energy sum_s E_s as a differentiable function of the positions
    (lambda frozen): APEnergy.apply(pos_T, lam, evaluator) -> E.  The backward
    pass returns -F * dL/dE; the forces come from the library's adjoint."""

    @staticmethod
    def forward(fctx, pos_T, lam, evaluator):
        e_sys, force, _ = evaluator(pos_T.detach(), lam.detach())
        fctx.save_for_backward(force)
        return e_sys.sum()

    @staticmethod
    def backward(fctx, grad_e):
        (force,) = fctx.saved_tensors
        return -force * grad_e, None, None
