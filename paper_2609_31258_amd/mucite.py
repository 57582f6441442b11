"""ctypes binding of the HIP ion-pack library (include/mucite.h).

Argument marshalling only: every step of the path runs in the library's
kernels.  PyTorch is used for device memory (the library's allocator
callbacks draw from torch's caching allocator) and for the stream the
library enqueues on.  The library must have been built
(``python -m paper_2609_31258_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmucite.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mucite.h")

I32, I64, U64, F64 = C.c_int32, C.c_int64, C.c_uint64, C.c_double
PD, PI64, PI32, PU8 = C.POINTER(F64), C.POINTER(I64), C.POINTER(I32), C.POINTER(C.c_uint8)

MC_OK, MC_EINVAL, MC_ESTATE, MC_ENOMEM, MC_EBUDGET, MC_EDEVICE, MC_ENUMERIC, MC_EINTERNAL = 0, -1, -2, -3, -4, -5, -6, -7
PREC_FP64, PREC_FP32 = 0, 1
ABI_VERSION = 6
NCLASS = 6
HIST_KE, HIST_TEFF, HIST_R = 202, 202, 102
K_EMIT, K_STEP, K_DEPOSIT, K_POISSON, K_FIELD, K_TALLY, K_SORT = range(7)
KERNEL_NAMES = ("emit", "step", "deposit", "poisson", "field", "tally", "sort")
NKERNEL = len(KERNEL_NAMES)

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Options(C.Structure):
    _fields_ = [("precision", I32), ("device", I32), ("seed", U64), ("pack_capacity", I64), ("exit_capacity", I64),
                ("hbm_budget", I64), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p), ("timing", I32), ("fp32_tables", I32), ("sample_capacity", I64)]


class Grid(C.Structure):
    _fields_ = [("nr", I32), ("nz", I32), ("dr", F64), ("dz", F64)]


class FieldTables(C.Structure):
    _fields_ = [(f, PD) for f in ("phi_dc", "phi_off", "phi_rf", "gas_ur", "gas_uz", "gas_p", "gas_t")] + \
               [("mask", PU8)]


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
                ("sample_every", I32), ("sample_stride", I32), ("adaptive", I32), ("lv_dt_max", F64),
                ("sort_every", I32)]


class Packs(C.Structure):
    _fields_ = [("n", I64)] + [(f, PD) for f in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w")] + \
               [("id", PI64), ("q", PI64), ("tag", PI32), ("status", PI32)]


class Tallies(C.Structure):
    _fields_ = [("emitted_n", I64), ("emitted_w", I64), ("class_n", I64 * NCLASS), ("class_w", I64 * NCLASS),
                ("n_cand", I64), ("n_coll", I64), ("n_cap", I64), ("n_clamp", I64), ("pack_steps", I64),
                ("exit_overflow", I64), ("exit_dropped", I64), ("n_langevin", I64), ("n_exchange", I64),
                ("sum_w_ke_active", F64), ("sum_w_eint_active", F64), ("sum_w_dissoc_terminal", F64),
                ("exit_bins", PI64), ("loss_map", PI64), ("hist_ke", PI64), ("hist_teff", PI64), ("hist_r", PI64),
                ("act_hist_ke", PI64), ("act_hist_teff", PI64)]


class TallyLayout(C.Structure):
    _fields_ = [("n_classes", I32), ("n_exit_bins", I32), ("exit_bin_dt", F64), ("nr", I32), ("nz", I32),
                ("loss_map_len", I64), ("hist_ke_len", I32), ("ke_bins", I32), ("ke_log10_lo", F64),
                ("ke_log10_hi", F64), ("hist_teff_len", I32), ("teff_bins", I32), ("teff_lo", F64),
                ("teff_hi", F64), ("hist_r_len", I32), ("r_bins", I32), ("r_lo", F64), ("r_hi", F64),
                ("exit_capacity", I64), ("sample_capacity", I64), ("charge_grid_len", I64)]


class ExitRec(C.Structure):
    _fields_ = [("id", I64), ("step", I64), ("cls", I32), ("inode", I32), ("jnode", I32), ("tag", I32)] + \
               [(f, F64) for f in ("x", "y", "z", "vx", "vy", "vz", "t_cross", "r_cross", "ke_ev", "t_eff",
                                   "h", "w")]


class SampleRec(C.Structure):
    _fields_ = [("id", I64), ("step", I64), ("tag", I32), ("reserved", I32)] + \
               [(f, F64) for f in ("x", "y", "z", "vx", "vy", "vz", "ke_ev", "t_eff", "h", "w")]


class Info(C.Structure):
    _fields_ = [("step", I64), ("n_slots", I64), ("capacity", I64), ("exit_capacity", I64), ("device_bytes", I64),
                ("nr", I32), ("nz", I32), ("n_exit_bins", I32), ("precision", I32), ("n_ions", I32),
                ("n_sources", I32), ("time", F64), ("last_dt", F64)]


class Timing(C.Structure):
    _fields_ = [("ms", F64 * NKERNEL), ("launches", I64 * NKERNEL), ("pack_steps", I64)]


class ServerOptions(C.Structure):
    _fields_ = [("precision", I32), ("device", I32), ("hbm_budget", I64), ("max_resident", I32),
                ("steps_per_sync", I32), ("stream", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN),
                ("alloc_user", C.c_void_p), ("fp32_tables", I32), ("reserved", I32), ("d_hit", F64),
                ("gas_mass_da", F64)]


class Query(C.Structure):
    _fields_ = [("ion", Ion), ("source", Source), ("op", Operating), ("n_steps", I64), ("seed", U64),
                ("exit_capacity", I64), ("sample_capacity", I64)]


class QueryResult(C.Structure):
    _fields_ = [("state", I32), ("error", I32), ("t_submit", F64), ("t_admit", F64), ("t_done", F64),
                ("device_bytes", I64), ("tallies", Tallies), ("exits", C.c_void_p), ("exits_len", I64),
                ("n_exits", I64), ("samples", C.c_void_p), ("samples_len", I64), ("n_samples", I64)]


class ServerStats(C.Structure):
    _fields_ = [(f, I64) for f in ("submitted", "admitted", "completed", "failed", "resident", "pending",
                                   "pool_bytes", "pool_in_use", "pool_peak", "shared_bytes", "co_steps",
                                   "pack_steps", "max_resident_seen")] + [("busy_s", F64), ("wall_s", F64)]


class CicPacks(C.Structure):
    _fields_ = [("n", I64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p), ("q", C.c_void_p),
                ("status", C.c_void_p)]


Q_PENDING, Q_RUNNING, Q_DONE, Q_FAILED = 0, 1, 2, 3

EXIT_DTYPE = np.dtype([(f, np.int64 if t is I64 else (np.int32 if t is I32 else np.float64))
                       for f, t in ExitRec._fields_])
assert EXIT_DTYPE.itemsize == C.sizeof(ExitRec)
SAMPLE_DTYPE = np.dtype([(f, np.int64 if t is I64 else (np.int32 if t is I32 else np.float64))
                         for f, t in SampleRec._fields_])
assert SAMPLE_DTYPE.itemsize == C.sizeof(SampleRec)

_SIGS = {
    "mc_abi_version": (I32, []),
    "mc_create": (I32, [C.POINTER(Options), C.POINTER(C.c_void_p)]),
    "mc_destroy": (None, [C.c_void_p]),
    "mc_last_error": (C.c_char_p, [C.c_void_p]),
    "mc_load_fields": (I32, [C.c_void_p, C.POINTER(Grid), C.POINTER(FieldTables)]),
    "mc_define_ion": (I32, [C.c_void_p, C.POINTER(Ion), PI32]),
    "mc_set_operating": (I32, [C.c_void_p, C.POINTER(Operating)]),
    "mc_define_source": (I32, [C.c_void_p, C.POINTER(Source), PI32]),
    "mc_inject": (I32, [C.c_void_p, I32, I64]),
    "mc_step": (I32, [C.c_void_p, I64]),
    "mc_pic_update": (I32, [C.c_void_p]),
    "mc_synchronize": (I32, [C.c_void_p]),
    "mc_get_info": (I32, [C.c_void_p, C.POINTER(Info)]),
    "mc_get_tally_layout": (I32, [C.c_void_p, C.POINTER(TallyLayout)]),
    "mc_read_tallies": (I32, [C.c_void_p, C.POINTER(Tallies)]),
    "mc_read_exits": (I32, [C.c_void_p, C.c_void_p, I64, PI64]),
    "mc_read_samples": (I32, [C.c_void_p, C.c_void_p, I64, PI64]),
    "mc_save_state": (I32, [C.c_void_p, C.c_char_p]),
    "mc_load_state": (I32, [C.c_void_p, C.c_char_p]),
    "mc_read_packs": (I32, [C.c_void_p, C.POINTER(Packs)]),
    "mc_write_packs": (I32, [C.c_void_p, C.POINTER(Packs)]),
    "mc_read_charge": (I32, [C.c_void_p, PI64]),
    "mc_read_sc": (I32, [C.c_void_p, PD, PD, PD]),
    "mc_read_hit": (I32, [C.c_void_p, PU8]),
    "mc_read_timing": (I32, [C.c_void_p, C.POINTER(Timing)]),
    "mc_reset_timing": (I32, [C.c_void_p]),
    "mc_set_timing": (I32, [C.c_void_p, I32]),
    "mc_deposit_cic": (I32, [C.POINTER(CicPacks), C.POINTER(Grid), C.c_void_p, C.c_void_p]),
    "mc_deposit_cic_noalloc": (I32, [C.POINTER(CicPacks), C.POINTER(Grid), C.c_void_p, C.c_void_p]),
    "mc_server_create": (I32, [C.POINTER(ServerOptions), C.POINTER(Grid), C.POINTER(FieldTables),
                               C.POINTER(C.c_void_p)]),
    "mc_server_destroy": (None, [C.c_void_p]),
    "mc_server_last_error": (C.c_char_p, [C.c_void_p]),
    "mc_server_submit": (I32, [C.c_void_p, C.POINTER(Query), C.POINTER(U64)]),
    "mc_server_poll": (I32, [C.c_void_p, U64, C.POINTER(QueryResult)]),
    "mc_server_wait": (I32, [C.c_void_p, U64, F64, C.POINTER(QueryResult)]),
    "mc_server_release": (I32, [C.c_void_p, U64]),
    "mc_server_get_stats": (I32, [C.c_void_p, C.POINTER(ServerStats)]),
}

_LIB = None


def load_library():
    """Load libmucite.so; raise if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run `python -m paper_2609_31258_amd.build`")
    try:
        # torch carries its own HIP runtime under the same soname; loading it
        # first makes the library bind to that one copy instead of a second
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.mc_abi_version() != ABI_VERSION:
        raise RuntimeError("ABI version mismatch")
    _LIB = L
    return L


class MucateError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where} failed ({code}): {msg}")
        self.code = code


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _struct(cls, obj):
    s = cls()
    for name, _ in cls._fields_:
        setattr(s, name, getattr(obj, name))
    return s


class _TorchMemory:
    """Device memory from torch's caching allocator, one stream."""

    def __init__(self, device: int):
        import torch
        self.torch = torch
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self.live: Dict[int, int] = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, stream, user):
        try:
            ptr = self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:
            return None
        self.live[int(ptr)] = int(nbytes)
        return ptr

    def _free(self, ptr, stream, user):
        if ptr and int(ptr) in self.live:
            del self.live[int(ptr)]
            self.torch.cuda.caching_allocator_delete(int(ptr))


class Sim:
    """One simulation context on one GPU (see include/mucite.h)."""

    def __init__(self, *, seed: int = 7, pack_capacity: int, precision: int = PREC_FP64, device: int = 0,
                 exit_capacity: int = 0, hbm_budget: int = 0, timing: bool = False, fp32_tables: bool = False,
                 sample_capacity: int = 0, use_torch: bool = True):
        self.L = load_library()
        self._mem = _TorchMemory(device) if use_torch else None
        o = Options()
        o.precision = precision
        o.device = device
        o.seed = seed
        o.pack_capacity = pack_capacity
        o.exit_capacity = exit_capacity
        o.hbm_budget = hbm_budget
        o.timing = int(timing)
        o.fp32_tables = int(fp32_tables)
        o.sample_capacity = sample_capacity
        self.sample_capacity = sample_capacity
        if self._mem is not None:
            o.stream = self._mem.stream.cuda_stream
            o.alloc = self._mem.alloc_cb
            o.free = self._mem.free_cb
        self._h = C.c_void_p()
        rc = self.L.mc_create(C.byref(o), C.byref(self._h))
        if rc != MC_OK:
            raise MucateError(rc, "mc_create", "context creation failed")
        self.precision = precision
        self.nr = self.nz = 0
        self.n_exit_bins = 0

    def close(self):
        if getattr(self, "_h", None):
            self.L.mc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, rc: int, where: str) -> None:
        if rc != MC_OK:
            raise MucateError(rc, where, (self.L.mc_last_error(self._h) or b"").decode())

    # -- setup --------------------------------------------------------------
    def load_fields(self, f) -> None:
        g = f.grid
        self.nr, self.nz = g.nr, g.nz
        arrs = [_f64(a) for a in (f.phi_dc, f.phi_off, f.phi_rf, f.gas_ur, f.gas_uz, f.gas_p, f.gas_t)]
        mask = np.ascontiguousarray(f.mask, dtype=np.uint8)
        t = FieldTables(*[_p(a, F64) for a in arrs], _p(mask, C.c_uint8))
        self._chk(self.L.mc_load_fields(self._h, C.byref(Grid(g.nr, g.nz, g.dr, g.dz)), C.byref(t)), "mc_load_fields")

    def define_ion(self, ion) -> int:
        out = I32()
        self._chk(self.L.mc_define_ion(self._h, C.byref(_struct(Ion, ion)), C.byref(out)), "mc_define_ion")
        return out.value

    def set_operating(self, op) -> None:
        self.n_exit_bins = op.n_exit_bins
        self._chk(self.L.mc_set_operating(self._h, C.byref(_struct(Operating, op))), "mc_set_operating")

    def define_source(self, src) -> int:
        out = I32()
        self._chk(self.L.mc_define_source(self._h, C.byref(_struct(Source, src)), C.byref(out)), "mc_define_source")
        return out.value

    def setup(self, fields, ions, sources, op) -> None:
        self.load_fields(fields)
        for i in ions:
            self.define_ion(i)
        self.set_operating(op)
        for s in sources:
            self.define_source(s)

    # -- run ----------------------------------------------------------------
    def inject(self, src: int, n: int) -> None:
        self._chk(self.L.mc_inject(self._h, src, n), "mc_inject")

    def step(self, n: int = 1) -> None:
        self._chk(self.L.mc_step(self._h, n), "mc_step")

    def pic_update(self) -> None:
        self._chk(self.L.mc_pic_update(self._h), "mc_pic_update")

    def synchronize(self) -> None:
        self._chk(self.L.mc_synchronize(self._h), "mc_synchronize")

    def info(self) -> Dict[str, int]:
        i = Info()
        self._chk(self.L.mc_get_info(self._h, C.byref(i)), "mc_get_info")
        return {f: getattr(i, f) for f, _ in Info._fields_}

    # -- read/write ------------------------------------------------------------
    def read_packs(self) -> Dict[str, np.ndarray]:
        n = self.info()["n_slots"]
        out = {f: np.zeros(n) for f in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w")}
        out.update(id=np.zeros(n, np.int64), q=np.zeros(n, np.int64), tag=np.zeros(n, np.int32),
                   status=np.zeros(n, np.int32))
        P = Packs()
        P.n = n
        for k, a in out.items():
            setattr(P, k, _p(a, {np.float64: F64, np.int64: I64, np.int32: I32}[a.dtype.type]))
        self._chk(self.L.mc_read_packs(self._h, C.byref(P)), "mc_read_packs")
        return out

    def write_packs(self, snap: Dict[str, np.ndarray]) -> None:
        n = len(snap["x"])
        arrs = {f: _f64(snap[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w")}
        arrs["id"] = np.ascontiguousarray(snap["id"], dtype=np.int64)
        arrs["tag"] = np.ascontiguousarray(snap["tag"], dtype=np.int32)
        P = Packs()
        P.n = n
        for k, a in arrs.items():
            setattr(P, k, _p(a, {np.float64: F64, np.int64: I64, np.int32: I32}[a.dtype.type]))
        self._chk(self.L.mc_write_packs(self._h, C.byref(P)), "mc_write_packs")

    def tally_layout(self) -> Dict[str, object]:
        L = TallyLayout()
        self._chk(self.L.mc_get_tally_layout(self._h, C.byref(L)), "mc_get_tally_layout")
        return {f: getattr(L, f) for f, _ in TallyLayout._fields_}

    def read_tallies(self) -> Dict[str, object]:
        T = Tallies()
        L = self.tally_layout()  # buffer sizes from the library's own layout
        bufs = dict(exit_bins=np.zeros(L["n_exit_bins"], np.int64),
                    loss_map=np.zeros(L["loss_map_len"], np.int64).reshape(L["nz"], L["nr"]),
                    hist_ke=np.zeros(L["hist_ke_len"], np.int64), hist_teff=np.zeros(L["hist_teff_len"], np.int64),
                    hist_r=np.zeros(L["hist_r_len"], np.int64), act_hist_ke=np.zeros(L["hist_ke_len"], np.int64),
                    act_hist_teff=np.zeros(L["hist_teff_len"], np.int64))
        for k, a in bufs.items():
            setattr(T, k, _p(a, I64))
        self._chk(self.L.mc_read_tallies(self._h, C.byref(T)), "mc_read_tallies")
        out = dict(bufs)
        for k in ("emitted_n", "emitted_w", "n_cand", "n_coll", "n_cap", "n_clamp", "pack_steps", "exit_overflow",
                  "exit_dropped", "n_langevin", "n_exchange", "sum_w_ke_active", "sum_w_eint_active", "sum_w_dissoc_terminal"):
            out[k] = getattr(T, k)
        out["class_n"] = np.array(list(T.class_n), np.int64)
        out["class_w"] = np.array(list(T.class_w), np.int64)
        return out

    def read_exits(self) -> np.ndarray:
        n = I64()
        self._chk(self.L.mc_read_exits(self._h, None, 0, C.byref(n)), "mc_read_exits")
        buf = np.zeros(max(n.value, 1), dtype=EXIT_DTYPE)
        self._chk(self.L.mc_read_exits(self._h, buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(n)),
                  "mc_read_exits")
        return buf[: min(n.value, buf.size, self.info()["exit_capacity"])]  # records beyond the buffer were dropped

    def save_state(self, path: str) -> None:
        self._chk(self.L.mc_save_state(self._h, os.fsencode(path)), "mc_save_state")

    def load_state(self, path: str) -> None:
        self._chk(self.L.mc_load_state(self._h, os.fsencode(path)), "mc_load_state")

    def read_samples(self) -> np.ndarray:
        n = I64()
        self._chk(self.L.mc_read_samples(self._h, None, 0, C.byref(n)), "mc_read_samples")
        buf = np.zeros(max(n.value, 1), dtype=SAMPLE_DTYPE)
        self._chk(self.L.mc_read_samples(self._h, buf.ctypes.data_as(C.c_void_p), buf.size, C.byref(n)),
                  "mc_read_samples")
        return buf[: min(n.value, buf.size, self.sample_capacity)]  # records beyond the buffer were dropped

    def read_charge(self) -> np.ndarray:
        q = np.zeros((self.nz, self.nr), np.int64)
        self._chk(self.L.mc_read_charge(self._h, _p(q, I64)), "mc_read_charge")
        return q

    def read_sc(self):
        phi, er, ez = (np.zeros((self.nz, self.nr)) for _ in range(3))
        self._chk(self.L.mc_read_sc(self._h, _p(phi, F64), _p(er, F64), _p(ez, F64)), "mc_read_sc")
        return phi, er, ez

    def read_hit(self) -> np.ndarray:
        h = np.zeros((self.nz, self.nr), np.uint8)
        self._chk(self.L.mc_read_hit(self._h, _p(h, C.c_uint8)), "mc_read_hit")
        return h

    def read_timing(self) -> Dict[str, object]:
        t = Timing()
        self._chk(self.L.mc_read_timing(self._h, C.byref(t)), "mc_read_timing")
        return {"ms": dict(zip(KERNEL_NAMES, list(t.ms))), "launches": dict(zip(KERNEL_NAMES, list(t.launches))),
                "pack_steps": t.pack_steps}

    def reset_timing(self) -> None:
        self._chk(self.L.mc_reset_timing(self._h), "mc_reset_timing")

    def set_timing(self, on: bool) -> None:
        self._chk(self.L.mc_set_timing(self._h, 1 if on else 0), "mc_set_timing")


def _tally_buffers(nz: int, nr: int, n_exit_bins: int):
    return dict(exit_bins=np.zeros(n_exit_bins, np.int64), loss_map=np.zeros((nz, nr), np.int64),
                hist_ke=np.zeros(HIST_KE, np.int64), hist_teff=np.zeros(HIST_TEFF, np.int64),
                hist_r=np.zeros(HIST_R, np.int64), act_hist_ke=np.zeros(HIST_KE, np.int64),
                act_hist_teff=np.zeros(HIST_TEFF, np.int64))


class Server:
    """Continuous-batching server of design queries over one field set."""

    def __init__(self, fields, *, hbm_budget: int, precision: int = PREC_FP32, max_resident: int = 64,
                 steps_per_sync: int = 20, d_hit: float = 1e-5, gas_mass_da: float = 28.0134, device: int = 0,
                 fp32_tables: bool = False, use_torch: bool = True):
        self.L = load_library()
        self._mem = _TorchMemory(device) if use_torch else None
        o = ServerOptions()
        o.precision = precision
        o.device = device
        o.hbm_budget = hbm_budget
        o.max_resident = max_resident
        o.steps_per_sync = steps_per_sync
        o.fp32_tables = int(fp32_tables)
        o.d_hit = d_hit
        o.gas_mass_da = gas_mass_da
        if self._mem is not None:
            o.stream = self._mem.stream.cuda_stream
            o.alloc = self._mem.alloc_cb
            o.free = self._mem.free_cb
        g = fields.grid
        self.nr, self.nz = g.nr, g.nz
        arrs = [_f64(a) for a in (fields.phi_dc, fields.phi_off, fields.phi_rf, fields.gas_ur, fields.gas_uz,
                                  fields.gas_p, fields.gas_t)]
        mask = np.ascontiguousarray(fields.mask, dtype=np.uint8)
        t = FieldTables(*[_p(a, F64) for a in arrs], _p(mask, C.c_uint8))
        self._h = C.c_void_p()
        rc = self.L.mc_server_create(C.byref(o), C.byref(Grid(g.nr, g.nz, g.dr, g.dz)), C.byref(t),
                                     C.byref(self._h))
        if rc != MC_OK:
            raise MucateError(rc, "mc_server_create", "server creation failed")
        self._bins: Dict[int, int] = {}
        self._caps: Dict[int, tuple] = {}

    def close(self):
        if getattr(self, "_h", None):
            self.L.mc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, rc, where):
        if rc != MC_OK:
            raise MucateError(rc, where, (self.L.mc_server_last_error(self._h) or b"").decode())

    def submit(self, ion, source, op, n_steps: int, seed: int, exit_capacity: int = 0,
               sample_capacity: int = 0) -> int:
        q = Query()
        q.ion = _struct(Ion, ion)
        q.source = _struct(Source, source)
        q.op = _struct(Operating, op)
        q.n_steps = n_steps
        q.seed = seed
        q.exit_capacity = exit_capacity
        q.sample_capacity = sample_capacity
        out = U64()
        self._chk(self.L.mc_server_submit(self._h, C.byref(q), C.byref(out)), "mc_server_submit")
        self._bins[out.value] = op.n_exit_bins
        self._caps[out.value] = (exit_capacity, sample_capacity)
        return out.value

    def _result(self, qid: int, fn, *args):
        r = QueryResult()
        bufs = _tally_buffers(self.nz, self.nr, self._bins.get(qid, 1))
        for k, a in bufs.items():
            setattr(r.tallies, k, _p(a, I64))
        ecap, scap = self._caps.get(qid, (0, 0))
        exits = np.zeros(max(ecap, 1), dtype=EXIT_DTYPE)
        samples = np.zeros(max(scap, 1), dtype=SAMPLE_DTYPE)
        r.exits, r.exits_len = exits.ctypes.data, ecap
        r.samples, r.samples_len = samples.ctypes.data, scap
        self._chk(fn(self._h, qid, *args, C.byref(r)), fn.__name__)
        out = dict(state=r.state, error=r.error, t_submit=r.t_submit, t_admit=r.t_admit, t_done=r.t_done,
                   device_bytes=r.device_bytes)
        if r.state == Q_DONE:
            T = r.tallies
            tal = dict(bufs)
            for k in ("emitted_n", "emitted_w", "n_cand", "n_coll", "n_cap", "n_clamp", "pack_steps",
                      "exit_overflow", "exit_dropped", "n_langevin", "n_exchange", "sum_w_ke_active", "sum_w_eint_active",
                      "sum_w_dissoc_terminal"):
                tal[k] = getattr(T, k)
            tal["class_n"] = np.array(list(T.class_n), np.int64)
            tal["class_w"] = np.array(list(T.class_w), np.int64)
            out["tallies"] = tal
            out["exits"] = exits[: min(r.n_exits, ecap)]
            out["samples"] = samples[: min(r.n_samples, scap)]
        return out

    def poll(self, qid: int) -> Dict[str, object]:
        return self._result(qid, self.L.mc_server_poll)

    def wait(self, qid: int, timeout_s: float = 600.0) -> Dict[str, object]:
        return self._result(qid, self.L.mc_server_wait, F64(timeout_s))

    def release(self, qid: int) -> None:
        self._chk(self.L.mc_server_release(self._h, qid), "mc_server_release")

    def stats(self) -> Dict[str, float]:
        st = ServerStats()
        self._chk(self.L.mc_server_get_stats(self._h, C.byref(st)), "mc_server_get_stats")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}


def deposit_cic(x, y, z, q, status, grid, out, *, noalloc: bool = False, stream=None) -> None:
    """CIC deposit of device tensors (x, y, z float64; q int64; status int32;
    one GPU) onto `out` (int64 tensor of nz * nr on the same device) through
    mc_deposit_cic, or mc_deposit_cic_noalloc with noalloc=True.  `grid` has
    nr, nz, dr, dz.  Runs on `stream` (a torch stream; default: the current
    one)."""
    import torch
    n = int(x.numel())
    for t, dt in ((x, torch.float64), (y, torch.float64), (z, torch.float64), (q, torch.int64),
                  (status, torch.int32)):
        if t.dtype != dt or not t.is_contiguous() or t.numel() != n or not t.is_cuda:
            raise ValueError("deposit_cic: x, y, z float64, q int64, status int32, contiguous, on the GPU, same length")
    if out.dtype != torch.int64 or not out.is_contiguous() or out.numel() != grid.nr * grid.nz:
        raise ValueError("deposit_cic: out must be a contiguous int64 tensor of nz * nr")
    L = load_library()
    P = CicPacks(n, x.data_ptr(), y.data_ptr(), z.data_ptr(), q.data_ptr(), status.data_ptr())
    G = Grid(grid.nr, grid.nz, grid.dr, grid.dz)
    s = (stream or torch.cuda.current_stream(out.device)).cuda_stream
    fn = L.mc_deposit_cic_noalloc if noalloc else L.mc_deposit_cic
    with torch.cuda.device(out.device):
        rc = fn(C.byref(P), C.byref(G), C.c_void_p(out.data_ptr()), C.c_void_p(s))
    if rc != MC_OK:
        raise MucateError(rc, fn.__name__, "deposit failed")


def declared_symbols(header: str = HEADER):
    """Names of the functions declared in include/mucite.h."""
    import re
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:int32_t|void|const char \*)\s*\*?\s*(mc_[a-z_0-9]+)\s*\(", text, re.M)))
