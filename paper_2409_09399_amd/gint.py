"""Thin ctypes binding of libgint.so (include/gint.h).

Argument marshalling only: every step of grid integration runs in the HIP
library.  PyTorch supplies device memory and the current stream.  There is no
CPU fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgint.so")

GINT_OK, GINT_EINVAL, GINT_EPATTERN, GINT_ENOMEM, GINT_EHIP, GINT_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GINT_FP64, GINT_MIXED_FP16X3, GINT_MIXED_BF16X3 = 0, 1, 2
GINT_DECOMP_DEFAULT, GINT_DECOMP_CLUSTER_PAIRS, GINT_DECOMP_BIGCELL, GINT_DECOMP_BIGCELL_RHO_FORCE = 0, 1, 2, 3


class GintError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib.gint_strerror(code).decode() if _lib is not None else str(code)
        if code == GINT_EHIP:
            msg += f" (hip error {_lib.gint_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]" if what else f"{msg} [{code}]")


class gint_species(C.Structure):
    _fields_ = [("rcut", C.c_double), ("dr", C.c_double), ("nknots", C.c_int), ("nchan", C.c_int),
                ("chan_l", C.c_void_p), ("f", C.c_void_p), ("fp", C.c_void_p)]


class gint_system(C.Structure):
    _fields_ = [("cell", C.c_double * 9), ("natom", C.c_int), ("pos", C.c_void_p), ("species", C.c_void_p),
                ("nspecies", C.c_int), ("species_list", C.c_void_p), ("grid", C.c_int * 3),
                ("nblk", C.c_int), ("blk_i", C.c_void_p), ("blk_j", C.c_void_p), ("blk_r", C.c_void_p),
                ("blk_off", C.c_void_p)]


class gint_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("cluster_atoms", C.c_int), ("max_bigcells_per_item", C.c_int),
                ("device_mib_cap", C.c_int), ("brick", C.c_int * 3), ("decomposition", C.c_int)]


class gint_sizes(C.Structure):
    _fields_ = [("ngrid", C.c_int64), ("nnz", C.c_int64), ("natom", C.c_int), ("ncluster", C.c_int),
                ("npairs", C.c_int64), ("nitems", C.c_int64), ("nbigcells", C.c_int64),
                ("work_units", C.c_double), ("volume", C.c_double), ("device_bytes", C.c_int64),
                ("precision", C.c_int), ("build_seconds", C.c_double), ("n_sys", C.c_int),
                ("decomposition", C.c_int), ("brick", C.c_int * 3), ("nbricks", C.c_int64),
                ("brick_images", C.c_int64)]


class gint_system_sizes(C.Structure):
    _fields_ = [("g_off", C.c_int64), ("ngrid", C.c_int64), ("nnz_off", C.c_int64), ("nnz", C.c_int64),
                ("atom_off", C.c_int), ("natom", C.c_int), ("grid", C.c_int * 3), ("volume", C.c_double)]


GINT_TUNE_MAX = 16


class gint_pipeline_stats(C.Structure):
    _fields_ = [("n_slabs", C.c_int), ("slabs_built", C.c_int), ("steps", C.c_int), ("build_seconds", C.c_double),
                ("first_step_seconds", C.c_double), ("wait_seconds", C.c_double),
                ("shared_device_bytes", C.c_int64), ("slot_device_bytes", C.c_int64),
                ("largest_slab_bytes", C.c_int64), ("all_slabs_bytes", C.c_int64), ("copied_bytes", C.c_int64)]


class gint_tune_report(C.Structure):
    _fields_ = [("ntrials", C.c_int), ("best", C.c_int), ("best_brick", C.c_int),
                ("cluster_atoms", C.c_int * GINT_TUNE_MAX), ("max_bigcells_per_item", C.c_int * GINT_TUNE_MAX),
                ("brick", (C.c_int * 3) * GINT_TUNE_MAX), ("vlocal_ms", C.c_double * GINT_TUNE_MAX),
                ("rho_force_ms", C.c_double * GINT_TUNE_MAX), ("step_ms", C.c_double * GINT_TUNE_MAX),
                ("seconds", C.c_double), ("cached", C.c_int)]


EXPORTED = ["gint_plan_create", "gint_vlocal", "gint_rho", "gint_force_stress", "gint_work_units",
            "gint_check_symmetry", "gint_energy", "gint_energy_noalloc",
            "gint_rho_force_stress", "gint_graph_create", "gint_graph_launch", "gint_graph_destroy", "gint_autotune", "gint_autotune_forget",
            "gint_plan_query", "gint_plan_query_system", "gint_plan_destroy", "gint_strerror",
            "gint_last_hip_error", "gint_peaks_measure",
            "gint_scf_create", "gint_scf_solve", "gint_scf_fold_gamma", "gint_scf_destroy",
            "gint_pipeline_create", "gint_pipeline_step", "gint_pipeline_query", "gint_pipeline_destroy"]


def _hip_runtimes():
    """Files of libamdhip64 mapped into this process."""
    found = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                p = line.split()[-1] if line.strip() else ""
                if "libamdhip64.so" in os.path.basename(p):
                    found.add(os.path.realpath(p))
    except OSError:
        pass
    return found


def _load():
    # PyTorch-ROCm ships its own HIP runtime (soname libamdhip64.so.7).  Load
    # it first so that libgint.so binds to the same runtime that owns the
    # tensors and streams it is handed; two runtimes in one process do not
    # share devices, memory or streams.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    rts = _hip_runtimes()
    if len(rts) > 1:
        raise ImportError(f"two HIP runtimes are loaded ({sorted(rts)}); libgint.so must share torch's")
    P = C.c_void_p
    lib.gint_plan_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(gint_system), C.c_int,
                                     C.POINTER(gint_options), P]
    lib.gint_plan_create.restype = C.c_int
    for name in ("gint_vlocal",):
        getattr(lib, name).argtypes = [P, P, P, P]
    lib.gint_rho.argtypes = [P, P, P, P, P]
    lib.gint_force_stress.argtypes = [P, P, P, P, P, P, P]
    lib.gint_rho_force_stress.argtypes = [P] * 9
    lib.gint_work_units.argtypes = [P, P, P]
    lib.gint_energy.argtypes = [P, P, P, P, P]
    lib.gint_energy_noalloc.argtypes = [P, P, P, P, P]
    lib.gint_peaks_measure.argtypes = [C.POINTER(C.c_double), P]
    lib.gint_check_symmetry.argtypes = [P, P, P, P]
    lib.gint_scf_create.argtypes = [C.POINTER(C.c_void_p), P, C.POINTER(C.c_int64)]
    lib.gint_pipeline_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(gint_system), C.POINTER(gint_options),
                                         C.c_int]
    lib.gint_pipeline_step.argtypes = [P] * 10
    lib.gint_pipeline_query.argtypes = [P, C.POINTER(gint_pipeline_stats)]
    lib.gint_pipeline_destroy.argtypes = [P]
    lib.gint_pipeline_destroy.restype = None
    lib.gint_scf_solve.argtypes = [P, P, P, C.c_double, C.c_double, P, P, P, P, P]
    lib.gint_scf_fold_gamma.argtypes = [P, P, P, P]
    lib.gint_scf_destroy.argtypes = [P]
    lib.gint_scf_destroy.restype = None
    lib.gint_plan_query.argtypes = [P, C.POINTER(gint_sizes)]
    lib.gint_plan_query_system.argtypes = [P, C.c_int, C.POINTER(gint_system_sizes)]
    lib.gint_plan_destroy.argtypes = [P]
    lib.gint_plan_destroy.restype = None
    lib.gint_graph_create.argtypes = [C.POINTER(C.c_void_p)] + [P] * 9
    lib.gint_graph_launch.argtypes = [P, P]
    lib.gint_graph_destroy.argtypes = [P]
    lib.gint_graph_destroy.restype = None
    lib.gint_autotune.argtypes = [C.POINTER(gint_system), C.c_int, C.POINTER(gint_options), C.c_double, P,
                                  C.POINTER(gint_tune_report)]
    lib.gint_autotune_forget.argtypes = []
    lib.gint_autotune_forget.restype = None
    lib.gint_strerror.argtypes = [C.c_int]
    lib.gint_strerror.restype = C.c_char_p
    lib.gint_last_hip_error.argtypes = []
    for name in EXPORTED:
        if name not in ("gint_plan_destroy", "gint_strerror", "gint_graph_destroy"):
            getattr(lib, name).restype = C.c_int
    return lib


_lib = _load()


def _check(rc: int, what: str):
    if rc != GINT_OK:
        raise GintError(rc, what)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t, n: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return C.c_void_p(t.data_ptr())


def _marshal_system(s, keep):
    def arr(x, dt):
        a = np.ascontiguousarray(np.asarray(x), dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(C.c_void_p)

    sps = (gint_species * len(s.species_list))()
    keep.append(sps)
    for k, sp in enumerate(s.species_list):
        sps[k].rcut = sp.rcut
        sps[k].dr = sp.dr
        sps[k].nknots = sp.nknots
        sps[k].nchan = sp.nchan
        sps[k].chan_l = arr(sp.ls, np.int32)
        sps[k].f = arr(sp.f, np.float64)
        sps[k].fp = arr(sp.fp, np.float64)
    st = gint_system()
    cell = np.ascontiguousarray(s.cell, dtype=np.float64).ravel()
    for k in range(9):
        st.cell[k] = float(cell[k])
    st.natom = int(s.pos.shape[0])
    st.pos = arr(s.pos, np.float64)
    st.species = arr(s.species, np.int32)
    st.nspecies = len(s.species_list)
    st.species_list = C.cast(sps, C.c_void_p)
    for k in range(3):
        st.grid[k] = int(s.grid[k])
    st.nblk = int(s.blk_i.shape[0])
    st.blk_i = arr(s.blk_i, np.int32)
    st.blk_j = arr(s.blk_j, np.int32)
    st.blk_r = arr(s.blk_r, np.int32)
    st.blk_off = arr(s.blk_off, np.int64)
    return st


def _marshal_batch(system):
    batch = list(system) if isinstance(system, (list, tuple)) else [system]
    if not batch:
        raise ValueError("empty batch")
    keep = []
    sts = (gint_system * len(batch))()
    for i, s in enumerate(batch):
        sts[i] = _marshal_system(s, keep)
    return sts, keep, len(batch)


class Plan:
    """A gint plan for one system or a batch of systems
    (paper_2409_09399_amd.inputs.System or any object with the same fields),
    built on the current HIP device.  A batch uses packed buffers; the slices
    of system i are given by `systems[i]` (dicts of offsets and sizes)."""

    def __init__(self, system, cluster_atoms: int = 0, max_bigcells_per_item: int = 0,
                 precision: int = GINT_FP64, stream=None, device_mib_cap: int = 0, brick=(0, 0, 0),
                 decomposition: int = GINT_DECOMP_DEFAULT):
        sts, keep, n = _marshal_batch(system)
        opt = gint_options()
        opt.precision = precision
        opt.cluster_atoms = cluster_atoms
        opt.max_bigcells_per_item = max_bigcells_per_item
        opt.device_mib_cap = device_mib_cap
        for k in range(3):
            opt.brick[k] = int(brick[k])
        opt.decomposition = decomposition
        ptr = C.c_void_p()
        rc = _lib.gint_plan_create(C.byref(ptr), sts, n, C.byref(opt),
                                   _stream(stream) if stream is not None else None)
        _check(rc, "gint_plan_create")
        self._p = ptr
        q = gint_sizes()
        _check(_lib.gint_plan_query(self._p, C.byref(q)), "gint_plan_query")
        self.sizes = q
        self.n_sys = int(q.n_sys)
        self.natom = int(q.natom)
        self.ngrid = int(q.ngrid)
        self.nnz = int(q.nnz)
        self.volume = float(q.volume)
        self.systems = []
        for i in range(self.n_sys):
            ss = gint_system_sizes()
            _check(_lib.gint_plan_query_system(self._p, i, C.byref(ss)), "gint_plan_query_system")
            self.systems.append({"g_off": int(ss.g_off), "ngrid": int(ss.ngrid), "nnz_off": int(ss.nnz_off),
                                 "nnz": int(ss.nnz), "atom_off": int(ss.atom_off), "natom": int(ss.natom),
                                 "grid": tuple(int(x) for x in ss.grid), "volume": float(ss.volume)})

    def close(self):
        if getattr(self, "_p", None):
            _lib.gint_plan_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        q = self.sizes
        out = {}
        for f, _ in gint_sizes._fields_:
            v = getattr(q, f)
            out[f] = tuple(v) if f == "brick" else v
        return out


def gint_vlocal(plan: Plan, v_loc, h_vals, stream=None):
    _check(_lib.gint_vlocal(plan._p, _dev_ptr(v_loc, plan.ngrid, "v_loc"), _dev_ptr(h_vals, plan.nnz, "h_vals"),
                            _stream(stream)), "gint_vlocal")


def gint_rho(plan: Plan, d_vals, rho, n_elec=None, stream=None):
    ne = _dev_ptr(n_elec, plan.n_sys, "n_elec") if n_elec is not None else None
    _check(_lib.gint_rho(plan._p, _dev_ptr(d_vals, plan.nnz, "d_vals"), _dev_ptr(rho, plan.ngrid, "rho"), ne,
                         _stream(stream)), "gint_rho")


def gint_force_stress(plan: Plan, v_loc, d_vals, force, stress, energy=None, stream=None):
    en = _dev_ptr(energy, plan.n_sys, "energy") if energy is not None else None
    _check(_lib.gint_force_stress(plan._p, _dev_ptr(v_loc, plan.ngrid, "v_loc"),
                                  _dev_ptr(d_vals, plan.nnz, "d_vals"), _dev_ptr(force, 3 * plan.natom, "force"),
                                  _dev_ptr(stress, 9 * plan.n_sys, "stress"), en, _stream(stream)), "gint_force_stress")


def gint_energy(plan: Plan, v_loc, rho, energy, stream=None):
    """E = w sum_g V_g rho_g per system into energy (device, n_sys)."""
    _check(_lib.gint_energy(plan._p, _dev_ptr(v_loc, plan.ngrid, "v_loc"), _dev_ptr(rho, plan.ngrid, "rho"),
                            _dev_ptr(energy, plan.n_sys, "energy"), _stream(stream)), "gint_energy")


def gint_energy_noalloc(plan: Plan, v_loc, rho, energy, stream=None):
    """gint_energy with its partial sums in the library's static device
    scratch (no allocation, no plan workspace; calls on one GPU must not
    overlap)."""
    _check(_lib.gint_energy_noalloc(plan._p, _dev_ptr(v_loc, plan.ngrid, "v_loc"), _dev_ptr(rho, plan.ngrid, "rho"),
                                    _dev_ptr(energy, plan.n_sys, "energy"), _stream(stream)), "gint_energy_noalloc")


class Scf:
    """One SCF step at the Gamma point on the device (include/gint_scf.h):
    H(R), S(R) -> H^G c = e S^G c (rocSOLVER) -> occupations -> D(R)."""

    def __init__(self, plan: Plan):
        ptr = C.c_void_p()
        n = C.c_int64()
        _check(_lib.gint_scf_create(C.byref(ptr), plan._p, C.byref(n)), "gint_scf_create")
        self._p = ptr
        self.plan = plan
        self.n = int(n.value)

    def solve(self, h_vals, s_vals, n_electrons: float, kT: float, eigvals, occupations, d_vals, info=None,
              stream=None):
        p = self.plan
        inf = info.data_ptr() if info is not None else None
        _check(_lib.gint_scf_solve(self._p, _dev_ptr(h_vals, p.nnz, "h_vals"), _dev_ptr(s_vals, p.nnz, "s_vals"),
                                   float(n_electrons), float(kT), _dev_ptr(eigvals, self.n, "eigvals"),
                                   _dev_ptr(occupations, self.n, "occupations"), _dev_ptr(d_vals, p.nnz, "d_vals"),
                                   inf, _stream(stream)), "gint_scf_solve")

    def fold_gamma(self, vals, dense, stream=None):
        _check(_lib.gint_scf_fold_gamma(self._p, _dev_ptr(vals, self.plan.nnz, "vals"),
                                        _dev_ptr(dense, self.n * self.n, "dense"), _stream(stream)),
               "gint_scf_fold_gamma")

    def close(self):
        if getattr(self, "_p", None):
            _lib.gint_scf_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pipeline:
    """Streaming pipeline of one system (include/gint_pipeline.h): its grid
    cut into n_slabs slabs along a1, slab plans built on a host thread and
    streamed to the device while earlier slabs compute."""

    def __init__(self, system, n_slabs: int, precision: int = GINT_FP64, decomposition: int = GINT_DECOMP_DEFAULT,
                 cluster_atoms: int = 0, max_bigcells_per_item: int = 0, brick=(0, 0, 0)):
        sts, keep, n = _marshal_batch(system)
        if n != 1:
            raise ValueError("a pipeline holds one system")
        opt = gint_options()
        opt.precision = precision
        opt.decomposition = decomposition
        opt.cluster_atoms = cluster_atoms
        opt.max_bigcells_per_item = max_bigcells_per_item
        for k in range(3):
            opt.brick[k] = int(brick[k])
        ptr = C.c_void_p()
        _check(_lib.gint_pipeline_create(C.byref(ptr), sts, C.byref(opt), int(n_slabs)), "gint_pipeline_create")
        self._p = ptr
        s = system[0] if isinstance(system, (list, tuple)) else system
        self.natom = int(s.natom)
        self.ngrid = int(np.prod(s.grid))
        self.nnz = int(s.nnz)

    def step(self, v_loc, d_vals, h_vals, rho, force, stress, n_elec=None, energy=None, stream=None):
        ne = _dev_ptr(n_elec, 1, "n_elec") if n_elec is not None else None
        en = _dev_ptr(energy, 1, "energy") if energy is not None else None
        _check(_lib.gint_pipeline_step(self._p, _dev_ptr(v_loc, self.ngrid, "v_loc"),
                                       _dev_ptr(d_vals, self.nnz, "d_vals"), _dev_ptr(h_vals, self.nnz, "h_vals"),
                                       _dev_ptr(rho, self.ngrid, "rho"), ne, _dev_ptr(force, 3 * self.natom, "force"),
                                       _dev_ptr(stress, 9, "stress"), en, _stream(stream)), "gint_pipeline_step")

    def stats(self) -> dict:
        q = gint_pipeline_stats()
        _check(_lib.gint_pipeline_query(self._p, C.byref(q)), "gint_pipeline_query")
        return {k: getattr(q, k) for k, _ in gint_pipeline_stats._fields_}

    def close(self):
        if getattr(self, "_p", None):
            _lib.gint_pipeline_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def measure_peaks(stream=None) -> dict:
    """Achievable TFLOP/s of FP64 MFMA, FP16 MFMA, FP32 and FP64 vector FMA
    on the current device (gint_peaks_measure; synchronous)."""
    out = (C.c_double * 4)()
    rc = _lib.gint_peaks_measure(out, _stream(stream))
    if rc != 0:
        raise RuntimeError(f"gint_peaks_measure failed ({rc})")
    return {"mfma_f64": out[0], "mfma_f16": out[1], "valu_f32": out[2], "valu_f64": out[3]}


def gint_work_units(plan: Plan, w_out, stream=None):
    _check(_lib.gint_work_units(plan._p, _dev_ptr(w_out, plan.n_sys, "w_out"), _stream(stream)), "gint_work_units")


def gint_check_symmetry(plan: Plan, d_vals, max_asym, stream=None):
    """max |D_IJR[mu,nu] - D_JI(-R)[nu,mu]| per system into max_asym (device, n_sys)."""
    _check(_lib.gint_check_symmetry(plan._p, _dev_ptr(d_vals, plan.nnz, "d_vals"),
                                    _dev_ptr(max_asym, plan.n_sys, "max_asym"), _stream(stream)),
           "gint_check_symmetry")


class Graph:
    """One captured step of a plan (gint_graph_create): Vlocal into h_vals,
    rho (and n_elec) into rho, force/stress (and energy) into force/stress,
    each stage present when its output is given.  Keeps the buffers alive."""

    def __init__(self, plan: Plan, v_loc=None, d_vals=None, h_vals=None, rho=None, n_elec=None, force=None,
                 stress=None, energy=None):
        n = plan.n_sys
        args = [_dev_ptr(v_loc, plan.ngrid, "v_loc") if v_loc is not None else None,
                _dev_ptr(d_vals, plan.nnz, "d_vals") if d_vals is not None else None,
                _dev_ptr(h_vals, plan.nnz, "h_vals") if h_vals is not None else None,
                _dev_ptr(rho, plan.ngrid, "rho") if rho is not None else None,
                _dev_ptr(n_elec, n, "n_elec") if n_elec is not None else None,
                _dev_ptr(force, 3 * plan.natom, "force") if force is not None else None,
                _dev_ptr(stress, 9 * n, "stress") if stress is not None else None,
                _dev_ptr(energy, n, "energy") if energy is not None else None]
        self._keep = (plan, v_loc, d_vals, h_vals, rho, n_elec, force, stress, energy)
        ptr = C.c_void_p()
        _check(_lib.gint_graph_create(C.byref(ptr), plan._p, *args), "gint_graph_create")
        self._g = ptr

    def launch(self, stream=None):
        _check(_lib.gint_graph_launch(self._g, _stream(stream)), "gint_graph_launch")

    def close(self):
        if getattr(self, "_g", None):
            _lib.gint_graph_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(system, precision: int = GINT_FP64, budget_seconds: float = 2.0, stream=None,
             decomposition: int = GINT_DECOMP_DEFAULT):
    """Pick the Vlocal cluster tile (cluster_atoms, max_bigcells_per_item) and
    the rho/force brick shape by timed trials (gint_autotune).  Returns
    (options dict for Plan, report dict)."""
    sts, keep, n = _marshal_batch(system)
    opt = gint_options()
    opt.precision = precision
    opt.decomposition = decomposition
    rep = gint_tune_report()
    _check(_lib.gint_autotune(sts, n, C.byref(opt), float(budget_seconds), _stream(stream), C.byref(rep)),
           "gint_autotune")
    trials = [{"cluster_atoms": rep.cluster_atoms[k], "max_bigcells_per_item": rep.max_bigcells_per_item[k],
               "brick": tuple(rep.brick[k]), "vlocal_ms": rep.vlocal_ms[k], "rho_force_ms": rep.rho_force_ms[k],
               "step_ms": rep.step_ms[k]} for k in range(rep.ntrials)]
    return ({"cluster_atoms": int(opt.cluster_atoms), "max_bigcells_per_item": int(opt.max_bigcells_per_item),
             "brick": tuple(int(x) for x in opt.brick), "decomposition": decomposition, "precision": precision},
            {"trials": trials, "best": int(rep.best), "best_brick": int(rep.best_brick),
             "seconds": float(rep.seconds), "cached": bool(rep.cached)})


def autotune_forget():
    """Empty the tuner's per-process cache (gint_autotune_forget)."""
    _lib.gint_autotune_forget()


def gint_rho_force_stress(plan: Plan, v_loc, d_vals, rho, force, stress, n_elec=None, energy=None, stream=None):
    ne = _dev_ptr(n_elec, plan.n_sys, "n_elec") if n_elec is not None else None
    en = _dev_ptr(energy, plan.n_sys, "energy") if energy is not None else None
    _check(_lib.gint_rho_force_stress(plan._p, _dev_ptr(v_loc, plan.ngrid, "v_loc"),
                                      _dev_ptr(d_vals, plan.nnz, "d_vals"), _dev_ptr(rho, plan.ngrid, "rho"), ne,
                                      _dev_ptr(force, 3 * plan.natom, "force"),
                                      _dev_ptr(stress, 9 * plan.n_sys, "stress"), en, _stream(stream)),
           "gint_rho_force_stress")
