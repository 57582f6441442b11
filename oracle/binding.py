"""ctypes binding of the CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from . import build as _build

_LIB = None

I32, I64, U32, U64, F64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
PD, PI64, PI32, PU8 = C.POINTER(F64), C.POINTER(I64), C.POINTER(I32), C.POINTER(C.c_uint8)

NCLASS = 6
HIST_KE, HIST_TEFF, HIST_R = 202, 202, 102
CLASS_NAMES = ("active", "transmitted", "electrode", "radial", "axial", "numeric")


class Ion(C.Structure):
    _fields_ = [("mass_da", F64), ("charge_z", I32), ("ccs_m2", F64), ("n_atoms", I32), ("theta_e", F64),
                ("alpha", F64), ("t_eff0", F64), ("act_kind", I32), ("act_p1", F64), ("act_p2", F64)]


class Source(C.Structure):
    _fields_ = [("kind", I32), ("ion", I32), ("current_a", F64), ("weight", F64), ("packs_per_step", I64),
                ("n_total", I64), ("sigma_r", F64), ("r_trunc", F64), ("z_inj", F64), ("step_start", I64)]


class Operating(C.Structure):
    _fields_ = [("dt", F64), ("v_rf", F64), ("f_rf", F64), ("phase_rf", F64), ("v_off", F64),
                ("gas_mass_da", F64), ("collisions_on", I32), ("sc_on", I32), ("sc_every", I32),
                ("z_det", F64), ("r_det", F64), ("d_hit", F64), ("exit_bin_dt", F64), ("n_exit_bins", I32),
                ("langevin_on", I32), ("lv_z_lo", F64), ("lv_z_hi", F64), ("lv_switch", F64), ("sc_mask", I32),
                ("sample_every", I32), ("sample_stride", I32),
                ("adaptive", I32), ("lv_dt_max", F64)]


class Packs(C.Structure):
    _fields_ = [("n", I64)] + [(f, PD) for f in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w")] + \
               [("id", PI64), ("q", PI64), ("tag", PI32), ("status", PI32)]


class Tallies(C.Structure):
    _fields_ = [("emitted_n", I64), ("emitted_w", I64), ("class_n", I64 * NCLASS), ("class_w", I64 * NCLASS),
                ("n_cand", I64), ("n_coll", I64), ("n_cap", I64), ("n_clamp", I64), ("exit_overflow", I64), ("n_langevin", I64),
                ("n_exchange", I64), ("sum_w_ke_active", F64), ("sum_w_eint_active", F64), ("sum_w_dissoc_terminal", F64),
                ("exit_bins", PI64), ("loss_map", PI64), ("hist_ke", PI64), ("hist_teff", PI64), ("hist_r", PI64),
                ("act_hist_ke", PI64), ("act_hist_teff", PI64)]


SAMPLE_DTYPE = np.dtype([("id", np.int64), ("step", np.int64), ("tag", np.int32), ("pad", np.int32)] +
                        [(f, np.float64) for f in ("x", "y", "z", "vx", "vy", "vz", "ke_ev", "t_eff", "h", "w")])


class Exit(C.Structure):
    _fields_ = [("id", I64), ("step", I64), ("cls", I32), ("inode", I32), ("jnode", I32), ("tag", I32)] + \
               [(f, F64) for f in ("x", "y", "z", "vx", "vy", "vz", "t_cross", "r_cross", "ke_ev", "t_eff",
                                   "h", "w")]


class Probe(C.Structure):
    _fields_ = [("n_cand", I64), ("n_acc", I64), ("sum_g", F64), ("sum_g2", F64)]


def lib():
    """Load (building first if absent) the oracle shared library.  The
    environment variable MC_ORACLE_LIB names another build of the oracle to
    load instead (the mutation tests load copies with a planted mistake)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.environ.get("MC_ORACLE_LIB")
    if not path:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
    L = C.CDLL(path)
    sig = {
        "orc_philox4x32_10": (None, [C.POINTER(U32), C.POINTER(U32), C.POINTER(U32)]),
        "orc_bake": (None, [PD, I32, I32, F64, F64, PD, PD]),
        "orc_gather": (F64, [PD, I32, I32, F64, F64, F64, F64]),
        "orc_einstein_u": (F64, [F64, I32, F64]),
        "orc_einstein_t": (F64, [F64, I32, F64]),
        "orc_rate": (F64, [I32, F64, F64, F64]),
        "orc_dst1": (None, [PD, I32, PD]),
        "orc_poisson": (None, [I32, I32, F64, F64, PD, PD]),
        "orc_poisson_residual": (F64, [I32, I32, F64, F64, PD, PD]),
        "orc_poisson_masked": (I32, [I32, I32, F64, F64, PD, PU8, F64, I32, PD]),
        "orc_rho_from_charge": (None, [I32, I32, F64, F64, PI64, PD]),
        "orc_iict_update": (None, [F64, F64, PD, PD, F64, F64, F64, PD, PD, PD, PD, PI32, PI32]),
        "orc_collision_probe": (I32, [F64, F64, F64, F64, F64, PD, PD, F64, I64, U64, C.POINTER(Probe)]),
        "orc_create": (C.c_void_p, [U64]),
        "orc_destroy": (None, [C.c_void_p]),
        "orc_load_fields": (I32, [C.c_void_p, I32, I32, F64, F64, PD, PD, PD, PD, PD, PD, PD, PU8]),
        "orc_define_ion": (I32, [C.c_void_p, C.POINTER(Ion)]),
        "orc_define_source": (I32, [C.c_void_p, C.POINTER(Source)]),
        "orc_set_operating": (I32, [C.c_void_p, C.POINTER(Operating)]),
        "orc_inject": (I32, [C.c_void_p, I32, I64]),
        "orc_step": (I32, [C.c_void_p, I64]),
        "orc_num_packs": (I64, [C.c_void_p]),
        "orc_num_threads": (I32, []),
        "orc_current_step": (I64, [C.c_void_p]),
        "orc_read_packs": (I32, [C.c_void_p, C.POINTER(Packs)]),
        "orc_write_packs": (I32, [C.c_void_p, C.POINTER(Packs)]),
        "orc_read_tallies": (I32, [C.c_void_p, C.POINTER(Tallies)]),
        "orc_read_exits": (I64, [C.c_void_p, C.POINTER(Exit), I64]),
        "orc_read_samples": (I64, [C.c_void_p, C.c_void_p, I64]),
        "orc_read_charge": (I32, [C.c_void_p, PI64]),
        "orc_read_sc": (I32, [C.c_void_p, PD, PD, PD]),
        "orc_read_hit": (I32, [C.c_void_p, PU8]),
        "orc_pic_update": (I32, [C.c_void_p]),
        "orc_deposit": (I32, [C.c_void_p]),
        "orc_current_time": (F64, [C.c_void_p]),
        "orc_last_dt": (F64, [C.c_void_p]),
        "orc_langevin_gamma": (F64, [F64, F64, F64, F64]),
        "orc_langevin_relax": (None, [F64, F64, F64, PD, F64, PD, PD]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --- unit-level functions -------------------------------------------------

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c, U32), _p(k, U32), _p(o, U32))
    return o


def bake(phi: np.ndarray, dr: float, dz: float):
    phi = _f64(phi)
    nz, nr = phi.shape
    er, ez = np.zeros_like(phi), np.zeros_like(phi)
    lib().orc_bake(_p(phi, F64), nr, nz, dr, dz, _p(er, F64), _p(ez, F64))
    return er, ez


def gather(tab: np.ndarray, dr: float, dz: float, r: float, z: float) -> float:
    tab = _f64(tab)
    nz, nr = tab.shape
    return lib().orc_gather(_p(tab, F64), nr, nz, dr, dz, r, z)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def einstein_u(t, n_atoms, theta=1100.0):
    return lib().orc_einstein_u(float(t), int(n_atoms), float(theta))


def einstein_t(e, n_atoms, theta=1100.0):
    return lib().orc_einstein_t(float(e), int(n_atoms), float(theta))


def rate(kind, p1, p2, t):
    return lib().orc_rate(int(kind), float(p1), float(p2), float(t))


def dst1(x) -> np.ndarray:
    x = _f64(x)
    o = np.zeros_like(x)
    lib().orc_dst1(_p(x, F64), x.size, _p(o, F64))
    return o


def poisson(rho: np.ndarray, dr: float, dz: float) -> np.ndarray:
    rho = _f64(rho)
    nz, nr = rho.shape
    phi = np.zeros_like(rho)
    lib().orc_poisson(nr, nz, dr, dz, _p(rho, F64), _p(phi, F64))
    return phi


def poisson_masked(rho: np.ndarray, mask: np.ndarray, dr: float, dz: float, tol: float = 1e-13,
                   max_iter: int = 2000):
    """Phi with Phi = 0 on the mask nodes; returns (phi, iterations)."""
    nz, nr = rho.shape
    rho = _f64(rho)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    phi = np.zeros((nz, nr))
    it = lib().orc_poisson_masked(nr, nz, dr, dz, _p(rho, F64), _p(m, C.c_uint8), tol, max_iter, _p(phi, F64))
    return phi, it


def poisson_residual(rho, phi, dr, dz) -> float:
    rho, phi = _f64(rho), _f64(phi)
    nz, nr = rho.shape
    return lib().orc_poisson_residual(nr, nz, dr, dz, _p(rho, F64), _p(phi, F64))


def rho_from_charge(q: np.ndarray, dr: float, dz: float) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.int64)
    nz, nr = q.shape
    rho = np.zeros(q.shape)
    lib().orc_rho_from_charge(nr, nz, dr, dz, _p(q, I64), _p(rho, F64))
    return rho


def iict_update(m, mg, v, vgas, e_int, t_eff, alpha, uniforms):
    v, vg = _f64(v), _f64(vgas)
    w = _f64(uniforms).copy()
    vo, vgo, eo, cl = np.zeros(3), np.zeros(3), np.zeros(1), np.zeros(2, dtype=np.int32)
    lib().orc_iict_update(m, mg, _p(v, F64), _p(vg, F64), e_int, t_eff, alpha, _p(w, F64), _p(vo, F64),
                          _p(vgo, F64), _p(eo, F64), _p(cl[:1], I32), _p(cl[1:], I32))
    return vo, vgo, float(eo[0]), int(cl[0]), int(cl[1])


def langevin_gamma(m: float, mg: float, n_sigma: float, t_gas: float) -> float:
    return lib().orc_langevin_gamma(m, mg, n_sigma, t_gas)


def langevin_relax(m, gamma, t_gas, u, dt, xi, v) -> np.ndarray:
    u, xi, v = _f64(u), _f64(xi), _f64(v).copy()
    lib().orc_langevin_relax(m, gamma, t_gas, _p(u, F64), dt, _p(xi, F64), _p(v, F64))
    return v


def collision_probe(m_da, ccs, mg_da, p, t_gas, u, v, dt, n_steps, seed):
    pr = Probe()
    uu, vv = _f64(u), _f64(v)
    lib().orc_collision_probe(m_da, ccs, mg_da, p, t_gas, _p(uu, F64), _p(vv, F64), dt, n_steps, seed, C.byref(pr))
    return dict(n_cand=pr.n_cand, n_acc=pr.n_acc, sum_g=pr.sum_g, sum_g2=pr.sum_g2)


# --- simulation --------------------------------------------------------------

def _struct(cls, obj):
    s = cls()
    for name, _ in cls._fields_:
        setattr(s, name, getattr(obj, name))
    return s


class OracleSim:
    """One oracle simulation: fields, ions, sources, operating point, packs."""

    def __init__(self, seed: int):
        self._h = lib().orc_create(seed)
        self.nr = self.nz = 0
        self.n_exit_bins = 0

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _chk(rc, what):
        if rc < 0:
            raise RuntimeError(f"oracle {what} failed ({rc})")
        return rc

    def load_fields(self, f):
        g = f.grid
        self.nr, self.nz, self.dr, self.dz = g.nr, g.nz, g.dr, g.dz
        self._keep = [_f64(a) for a in (f.phi_dc, f.phi_off, f.phi_rf, f.gas_ur, f.gas_uz, f.gas_p, f.gas_t)]
        m = np.ascontiguousarray(f.mask, dtype=np.uint8)
        a = self._keep
        self._chk(lib().orc_load_fields(self._h, g.nr, g.nz, g.dr, g.dz, *[_p(x, F64) for x in a], _p(m, C.c_uint8)),
                  "load_fields")

    def define_ion(self, ion) -> int:
        return self._chk(lib().orc_define_ion(self._h, C.byref(_struct(Ion, ion))), "define_ion")

    def define_source(self, src) -> int:
        return self._chk(lib().orc_define_source(self._h, C.byref(_struct(Source, src))), "define_source")

    def set_operating(self, op):
        self.n_exit_bins = op.n_exit_bins
        self._chk(lib().orc_set_operating(self._h, C.byref(_struct(Operating, op))), "set_operating")

    def setup(self, fields, ions, sources, op):
        self.load_fields(fields)
        for i in ions:
            self.define_ion(i)
        self.set_operating(op)
        for s in sources:
            self.define_source(s)

    def inject(self, src: int, n: int):
        self._chk(lib().orc_inject(self._h, src, n), "inject")

    def step(self, n: int = 1):
        self._chk(lib().orc_step(self._h, n), "step")

    def pic_update(self):
        self._chk(lib().orc_pic_update(self._h), "pic_update")

    @property
    def time(self) -> float:
        return lib().orc_current_time(self._h)

    @property
    def last_dt(self) -> float:
        return lib().orc_last_dt(self._h)

    def deposit(self):
        self._chk(lib().orc_deposit(self._h), "deposit")

    @property
    def n_packs(self) -> int:
        return lib().orc_num_packs(self._h)

    @property
    def current_step(self) -> int:
        return lib().orc_current_step(self._h)

    def read_packs(self) -> Dict[str, np.ndarray]:
        n = self.n_packs
        out = {f: np.zeros(n) for f in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w")}
        out.update(id=np.zeros(n, np.int64), q=np.zeros(n, np.int64), tag=np.zeros(n, np.int32),
                   status=np.zeros(n, np.int32))
        P = Packs()
        P.n = n
        for k, a in out.items():
            setattr(P, k, _p(a, {np.float64: F64, np.int64: I64, np.int32: I32}[a.dtype.type]))
        self._chk(lib().orc_read_packs(self._h, C.byref(P)), "read_packs")
        return out

    def write_packs(self, snap: Dict[str, np.ndarray]):
        n = len(snap["x"])
        arrs = {f: _f64(snap[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w")}
        arrs["id"] = np.ascontiguousarray(snap["id"], dtype=np.int64)
        arrs["tag"] = np.ascontiguousarray(snap["tag"], dtype=np.int32)
        P = Packs()
        P.n = n
        for k, a in arrs.items():
            setattr(P, k, _p(a, {np.float64: F64, np.int64: I64, np.int32: I32}[a.dtype.type]))
        self._chk(lib().orc_write_packs(self._h, C.byref(P)), "write_packs")

    def read_tallies(self) -> Dict[str, object]:
        T = Tallies()
        bufs = dict(exit_bins=np.zeros(self.n_exit_bins, np.int64), loss_map=np.zeros((self.nz, self.nr), np.int64),
                    hist_ke=np.zeros(HIST_KE, np.int64), hist_teff=np.zeros(HIST_TEFF, np.int64),
                    hist_r=np.zeros(HIST_R, np.int64), act_hist_ke=np.zeros(HIST_KE, np.int64),
                    act_hist_teff=np.zeros(HIST_TEFF, np.int64))
        for k, a in bufs.items():
            setattr(T, k, _p(a, I64))
        self._chk(lib().orc_read_tallies(self._h, C.byref(T)), "read_tallies")
        out = dict(bufs)
        for k in ("emitted_n", "emitted_w", "n_cand", "n_coll", "n_cap", "n_clamp", "exit_overflow", "n_langevin",
                  "n_exchange", "sum_w_ke_active", "sum_w_eint_active", "sum_w_dissoc_terminal"):
            out[k] = getattr(T, k)
        out["class_n"] = np.array(list(T.class_n), np.int64)
        out["class_w"] = np.array(list(T.class_w), np.int64)
        return out

    def read_samples(self) -> np.ndarray:
        n = lib().orc_read_samples(self._h, None, 0)
        buf = np.zeros(max(n, 1), dtype=SAMPLE_DTYPE)
        lib().orc_read_samples(self._h, buf.ctypes.data_as(C.c_void_p), n)
        return buf[:n]

    def read_exits(self) -> np.ndarray:
        n = lib().orc_read_exits(self._h, None, 0)
        buf = (Exit * max(n, 1))()
        lib().orc_read_exits(self._h, buf, n)
        names = [f for f, _ in Exit._fields_]
        dt = [(f, np.int64 if t is I64 else (np.int32 if t is I32 else np.float64)) for f, t in Exit._fields_]
        out = np.zeros(n, dtype=dt)
        for k in range(n):
            out[k] = tuple(getattr(buf[k], f) for f in names)
        return np.sort(out, order="id")

    def read_charge(self) -> np.ndarray:
        q = np.zeros((self.nz, self.nr), np.int64)
        lib().orc_read_charge(self._h, _p(q, I64))
        return q

    def read_sc(self):
        phi, er, ez = (np.zeros((self.nz, self.nr)) for _ in range(3))
        lib().orc_read_sc(self._h, _p(phi, F64), _p(er, F64), _p(ez, F64))
        return phi, er, ez

    def read_hit(self) -> np.ndarray:
        h = np.zeros((self.nz, self.nr), np.uint8)
        self._chk(lib().orc_read_hit(self._h, _p(h, C.c_uint8)), "read_hit")
        return h
