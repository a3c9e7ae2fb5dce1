"""ctypes binding of libcube (include/cube.h): argument marshalling only.

Every step of the particle-mesh path runs in the HIP kernels of libcube.so; this module only
converts numpy arrays and parameters, supplies PyTorch's stream and (optionally) PyTorch's
caching allocator for device memory, and raises ``CubeError`` for non-zero status codes.
The library must have been built in-tree (``python -m paper_1712_06121_amd.build``); there is no
fallback of any kind when it is missing.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from ctypes import (CFUNCTYPE, POINTER, Structure, byref, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_uint32,
                    c_size_t, c_uint64, c_void_p)

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libcube.so")

CUBE_OK, CUBE_DONE = 0, 1
ERRORS = {-1: "CUBE_E_INVALID", -2: "CUBE_E_NOMEM", -3: "CUBE_E_DEVICE", -4: "CUBE_E_CAPACITY", -5: "CUBE_E_CFL",
          -6: "CUBE_E_NONFINITE", -7: "CUBE_E_OVERFLOW", -8: "CUBE_E_STATE"}
SIGMA_GLOBAL, SIGMA_PER_CELL = 0, 1

EXPORTED = [
    "cube_create", "cube_destroy", "cube_last_error", "cube_init_ic", "cube_load_particles", "cube_step",
    "cube_scale_factor", "cube_steps_done", "cube_num_particles", "cube_get_density", "cube_get_power",
    "cube_get_state", "cube_set_state", "cube_get_counts", "cube_stage_deposit", "cube_stage_solve", "cube_stage_move",
    "cube_get_mesh", "cube_set_mesh", "cube_get_ic_displacement", "cube_get_tables", "cube_get_schedule",
    "cube_device_bytes", "cube_set_profiling", "cube_get_timings", "cube_autotune", "cube_get_variant",
    "cube_set_variant", "cube_batch_create", "cube_batch_destroy", "cube_batch_last_error", "cube_batch_size",
    "cube_batch_box", "cube_batch_init_ic", "cube_batch_autotune", "cube_batch_step", "cube_batch_set_mode",
    "cube_footprint", "cube_get_cross_power", "cube_enable_pids", "cube_get_pids", "cube_set_pids",
    "cube_get_counts_u8", "cube_counts_from_u8", "cube_set_ic_parent", "cube_set_adaptive",
    "cube_get_adaptive_log", "cube_get_last_maxima", "cube_debug_inject_flag", "cube_debug_set_turn_limit",
    "cube_get_power_noalloc", "cube_autotune_report", "cube_set_two_level",
    "cube_server_create", "cube_server_destroy", "cube_server_last_error", "cube_server_submit", "cube_server_poll",
    "cube_server_status", "cube_server_job_error", "cube_server_job", "cube_server_release", "cube_server_stats",
]


class CubeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class CubeParams(Structure):
    _fields_ = [("np_side", c_int32), ("nm_side", c_int32), ("nc_side", c_int32), ("x_bytes", c_int32),
                ("v_bytes", c_int32), ("sigma_mode", c_int32), ("n_steps", c_int32), ("spacing", c_int32),
                ("box", c_double), ("omega_m", c_double), ("omega_l", c_double), ("h", c_double),
                ("sigma8", c_double), ("n_s", c_double), ("a_init", c_double), ("a_final", c_double),
                ("seed", c_uint64), ("capacity", c_int64)]


class CubeVariant(Structure):
    _fields_ = [("move_variant", c_int32), ("fft_col_width", c_int32), ("fft_z_order", c_int32),
                ("deposit_variant", c_int32), ("fft_z_layout", c_int32), ("fft_z_width", c_int32)]


ALLOC_FN = CFUNCTYPE(c_void_p, c_size_t, c_void_p)
FREE_FN = CFUNCTYPE(None, c_void_p, c_void_p)


class CubeAllocator(Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


class CubeStateView(Structure):
    _fields_ = [("cnt", c_void_p), ("chi", c_void_p), ("nu", c_void_p), ("vc", c_void_p), ("vs", c_void_p),
                ("n", c_int64), ("a", c_double), ("steps_done", c_int32)]


_lib = None

# Handles still open at interpreter exit are closed before PyTorch (whose allocator frees their
# device memory) is torn down.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcube.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcube.so not found at {path}: build it with `python -m paper_1712_06121_amd.build`")
    # PyTorch bundles its own HIP runtime with the same soname as the system one libcube links
    # against. Import it first so the process holds a single runtime (the one that owns the
    # streams and device memory PyTorch hands to the library).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    sim_p = c_void_p
    lib.cube_create.argtypes = [POINTER(CubeParams), c_void_p, POINTER(CubeAllocator), POINTER(c_void_p)]
    lib.cube_destroy.argtypes = [sim_p]
    lib.cube_destroy.restype = None
    lib.cube_last_error.argtypes = [sim_p]
    lib.cube_last_error.restype = c_char_p
    for name in ("cube_init_ic", "cube_stage_deposit", "cube_stage_solve"):
        getattr(lib, name).argtypes = [sim_p]
    lib.cube_load_particles.argtypes = [sim_p, c_void_p, c_void_p, c_int64]
    lib.cube_step.argtypes = [sim_p, c_int32]
    lib.cube_debug_inject_flag.argtypes = [sim_p, c_int32, c_uint32]
    lib.cube_debug_set_turn_limit.argtypes = [sim_p, c_uint32]
    lib.cube_set_two_level.argtypes = [sim_p, c_double]
    lib.cube_scale_factor.argtypes = [sim_p]
    lib.cube_scale_factor.restype = c_double
    lib.cube_steps_done.argtypes = [sim_p]
    lib.cube_steps_done.restype = c_int32
    lib.cube_num_particles.argtypes = [sim_p]
    lib.cube_num_particles.restype = c_int64
    lib.cube_get_density.argtypes = [sim_p, c_void_p, c_int]
    lib.cube_get_power.argtypes = [sim_p, c_int32, c_void_p, c_void_p, c_void_p]
    lib.cube_get_power_noalloc.argtypes = [sim_p, c_int32, c_void_p, c_void_p, c_void_p]
    lib.cube_get_cross_power.argtypes = [sim_p, sim_p, c_int32] + [c_void_p] * 5
    lib.cube_enable_pids.argtypes = [sim_p, c_int32]
    lib.cube_set_ic_parent.argtypes = [sim_p, c_int32]
    lib.cube_set_adaptive.argtypes = [sim_p, c_double, c_double, c_double]
    lib.cube_get_adaptive_log.argtypes = [sim_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.cube_get_last_maxima.argtypes = [sim_p, c_void_p, c_void_p]
    lib.cube_get_counts_u8.argtypes = [sim_p, c_void_p, c_void_p, c_int64, c_void_p]
    lib.cube_counts_from_u8.argtypes = [c_void_p, c_int64, c_void_p, c_int64, c_void_p]
    lib.cube_get_pids.argtypes = [sim_p, c_void_p]
    lib.cube_set_pids.argtypes = [sim_p, c_void_p]
    lib.cube_get_state.argtypes = [sim_p, POINTER(CubeStateView)]
    lib.cube_set_state.argtypes = [sim_p, POINTER(CubeStateView)]
    lib.cube_get_counts.argtypes = [sim_p, c_void_p]
    lib.cube_stage_move.argtypes = [sim_p, c_float, c_float]
    lib.cube_get_mesh.argtypes = [sim_p, c_void_p]
    lib.cube_set_mesh.argtypes = [sim_p, c_void_p]
    lib.cube_get_ic_displacement.argtypes = [sim_p, c_void_p]
    lib.cube_get_tables.argtypes = [sim_p, c_void_p, c_void_p]
    lib.cube_get_schedule.argtypes = [sim_p, c_void_p, c_void_p, c_void_p]
    lib.cube_device_bytes.argtypes = [sim_p]
    lib.cube_device_bytes.restype = c_int64
    lib.cube_set_profiling.argtypes = [sim_p, c_int]
    lib.cube_get_timings.argtypes = [sim_p, c_void_p]
    lib.cube_autotune.argtypes = [sim_p]
    lib.cube_autotune_report.argtypes = [sim_p]
    lib.cube_autotune_report.restype = c_char_p
    lib.cube_get_variant.argtypes = [sim_p, POINTER(CubeVariant)]
    lib.cube_set_variant.argtypes = [sim_p, POINTER(CubeVariant)]
    batch_p = c_void_p
    lib.cube_batch_create.argtypes = [POINTER(CubeParams), c_int32, c_void_p, POINTER(CubeAllocator), POINTER(c_void_p)]
    lib.cube_batch_destroy.argtypes = [batch_p]
    lib.cube_batch_destroy.restype = None
    lib.cube_batch_last_error.argtypes = [batch_p]
    lib.cube_batch_last_error.restype = c_char_p
    lib.cube_batch_size.argtypes = [batch_p]
    lib.cube_batch_size.restype = c_int32
    lib.cube_batch_box.argtypes = [batch_p, c_int32]
    lib.cube_batch_box.restype = c_void_p
    for name in ("cube_batch_init_ic", "cube_batch_autotune"):
        getattr(lib, name).argtypes = [batch_p]
    lib.cube_batch_step.argtypes = [batch_p, c_int32]
    lib.cube_batch_set_mode.argtypes = [batch_p, c_int32]
    lib.cube_footprint.argtypes = [POINTER(CubeParams)]
    lib.cube_footprint.restype = c_int64
    srv_p = c_void_p
    lib.cube_server_create.argtypes = [c_int64, c_int32, c_int32, POINTER(CubeAllocator), POINTER(c_void_p)]
    lib.cube_server_destroy.argtypes = [srv_p]
    lib.cube_server_destroy.restype = None
    lib.cube_server_last_error.argtypes = [srv_p]
    lib.cube_server_last_error.restype = c_char_p
    lib.cube_server_submit.argtypes = [srv_p, POINTER(CubeParams), c_int64]
    lib.cube_server_poll.argtypes = [srv_p, c_void_p, c_int32, POINTER(c_int32)]
    lib.cube_server_status.argtypes = [srv_p, c_int64, POINTER(c_int32), POINTER(c_int32)]
    lib.cube_server_job_error.argtypes = [srv_p, c_int64]
    lib.cube_server_job_error.restype = c_char_p
    lib.cube_server_job.argtypes = [srv_p, c_int64]
    lib.cube_server_job.restype = c_void_p
    lib.cube_server_release.argtypes = [srv_p, c_int64]
    lib.cube_server_stats.argtypes = [srv_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int64)]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> c_void_p:
    return c_void_p(a.ctypes.data)


def make_params(np_side: int, nm_side: int, box: float, nc_side: int | None = None, x_bytes: int = 1,
                v_bytes: int = 1, sigma_mode: int = SIGMA_PER_CELL, omega_m: float = 0.3, omega_l: float | None = None,
                h: float = 0.7, sigma8: float = 0.8, n_s: float = 1.0, a_init: float = 0.02, a_final: float = 1.0,
                n_steps: int = 50, spacing: int = 0, seed: int = 1, capacity: int = 0, **_ignored) -> CubeParams:
    """``cube_params`` from keyword arguments (omega_l defaults to a flat universe)."""
    return CubeParams(np_side, nm_side, nc_side or nm_side // 4, x_bytes, v_bytes, sigma_mode, n_steps, spacing, box,
                      omega_m, 1.0 - omega_m if omega_l is None else omega_l, h, sigma8, n_s, a_init, a_final, seed,
                      capacity)


def _torch_env(torch_memory: bool):
    """PyTorch's current HIP stream and (optionally) its caching allocator as a cube_allocator.
    Returns (stream, allocator pointer or None, objects to keep alive)."""
    keep, stream, alloc_p = [], c_void_p(0), None
    try:
        import torch
        if torch.cuda.is_available():
            stream = c_void_p(torch.cuda.current_stream().cuda_stream)
            if torch_memory:
                dev = torch.cuda.current_device()
                tstream = torch.cuda.current_stream()

                t_alloc, t_delete = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

                def _alloc(nbytes, _user):
                    try:
                        return t_alloc(int(nbytes), dev, tstream)
                    except Exception:  # out of memory: the library reports CUBE_E_NOMEM
                        return None

                def _free(ptr, _user):
                    t_delete(ptr)

                a = CubeAllocator(ALLOC_FN(_alloc), FREE_FN(_free), None)
                keep.append(a)
                alloc_p = byref(a)
    except ImportError:
        pass
    return stream, alloc_p, keep


class Sim:
    """One simulation box. Parameters as in ``cube_params`` (include/cube.h)."""

    def __init__(self, np_side: int, nm_side: int, box: float, nc_side: int | None = None, x_bytes: int = 1,
                 v_bytes: int = 1, sigma_mode: int = SIGMA_PER_CELL, omega_m: float = 0.3, omega_l: float | None = None,
                 h: float = 0.7, sigma8: float = 0.8, n_s: float = 1.0, a_init: float = 0.02, a_final: float = 1.0,
                 n_steps: int = 50, spacing: int = 0, seed: int = 1, capacity: int = 0, torch_memory: bool = True,
                 _handle: c_void_p | None = None, **_ignored):
        self._lib = load_library()
        self.params = make_params(np_side, nm_side, box, nc_side, x_bytes, v_bytes, sigma_mode, omega_m, omega_l, h,
                                  sigma8, n_s, a_init, a_final, n_steps, spacing, seed, capacity)
        self._set_shape(self.params)
        self.pid_bytes = 0
        self._owned = _handle is None
        if _handle is not None:  # a box owned by a Batch
            self._h = _handle
            self._keep = []
            return
        stream, alloc_p, self._keep = _torch_env(torch_memory)
        self._stream = stream
        self._h = c_void_p()
        rc = self._lib.cube_create(byref(self.params), stream, alloc_p, byref(self._h))
        if rc != CUBE_OK:
            raise CubeError(rc, "cube_create: " + self._lib.cube_last_error(None).decode())
        _live.add(self)

    def _set_shape(self, p: CubeParams):
        self.np_side, self.nm, self.nc = p.np_side, p.nm_side, p.nc_side
        self.x_bytes, self.v_bytes, self.n_steps = p.x_bytes, p.v_bytes, p.n_steps
        self.box = p.box

    # ---- helpers -----------------------------------------------------------------------------
    def _check(self, rc: int) -> int:
        if rc < 0:
            raise CubeError(rc, self._lib.cube_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            if self._owned:
                self._lib.cube_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def chi_dtype(self):
        return np.uint8 if self.x_bytes == 1 else np.uint16

    @property
    def nu_dtype(self):
        return np.int8 if self.v_bytes == 1 else np.int16

    # ---- calls -------------------------------------------------------------------------------
    def init_ic(self):
        self._check(self._lib.cube_init_ic(self._h))

    def load_particles(self, x, v):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        assert x.shape == v.shape and x.ndim == 2 and x.shape[1] == 3
        self._check(self._lib.cube_load_particles(self._h, _ptr(x), _ptr(v), x.shape[0]))

    def step(self, k: int = 1) -> int:
        return self._check(self._lib.cube_step(self._h, k))

    @property
    def a(self) -> float:
        return self._lib.cube_scale_factor(self._h)

    @property
    def steps_done(self) -> int:
        return self._lib.cube_steps_done(self._h)

    @property
    def n(self) -> int:
        return self._lib.cube_num_particles(self._h)

    def get_density(self, device: bool = False):
        """CIC density contrast [z, y, x]: a numpy array, or with device=True a torch tensor on the
        simulation's GPU that the library writes directly (device-to-device)."""
        if device:
            import torch
            out = torch.empty((self.nm,) * 3, dtype=torch.float32, device="cuda")
            self._check(self._lib.cube_get_density(self._h, c_void_p(out.data_ptr()), 1))
            return out
        out = np.empty((self.nm,) * 3, dtype=np.float32)
        self._check(self._lib.cube_get_density(self._h, _ptr(out), 0))
        return out

    def get_power_noalloc(self, k, pk, nmodes, nbins: int | None = None):
        """cube_get_power_noalloc into caller-provided device tensors (float64, nbins each); the
        library allocates nothing and does not synchronise."""
        nb = nbins or self.nm // 2
        for t in (k, pk, nmodes):
            assert t.is_cuda and t.is_contiguous() and t.numel() >= nb and str(t.dtype) == "torch.float64"
        self._check(self._lib.cube_get_power_noalloc(self._h, nb, c_void_p(k.data_ptr()), c_void_p(pk.data_ptr()),
                                                     c_void_p(nmodes.data_ptr())))

    def set_two_level(self, r_s: float):
        """Two-level force with split radius r_s (fine cells); 0 returns to the single-level solve."""
        self._check(self._lib.cube_set_two_level(self._h, float(r_s)))

    def debug_inject_flag(self, step: int, flag: int):
        """Raise device error bits before the move of `step` (tests of the error path); -1: off."""
        self._check(self._lib.cube_debug_inject_flag(self._h, step, flag))

    def debug_set_turn_limit(self, polls: int):
        """Polls after which a gradient-tile scatter chunk stops waiting for its turn and raises
        the count error (tests of that path); the default is 2^22."""
        self._check(self._lib.cube_debug_set_turn_limit(self._h, polls))

    def get_power(self, nbins: int | None = None):
        nb = nbins or self.nm // 2
        k, pk, nm = (np.empty(nb) for _ in range(3))
        self._check(self._lib.cube_get_power(self._h, nb, _ptr(k), _ptr(pk), _ptr(nm)))
        return k, pk, nm

    def set_adaptive(self, eta_v: float, eta_a: float, eta_e: float):
        """Adaptive time steps bounded by the largest drift (eta_v fine cells), the drift of the
        largest velocity change (eta_a fine cells) and the expansion (Delta a / a <= eta_e)."""
        self._check(self._lib.cube_set_adaptive(self._h, eta_v, eta_a, eta_e))

    def get_adaptive_log(self):
        """(a_int, vmax, gmax) of the adaptive schedule so far."""
        m = self.n_steps + 8
        a, v, g = np.empty(m), np.empty(m), np.empty(m)
        na, nv = np.zeros(1, np.int32), np.zeros(1, np.int32)
        self._check(self._lib.cube_get_adaptive_log(self._h, m, _ptr(a), _ptr(v), _ptr(g), _ptr(na), _ptr(nv)))
        return a[: na[0]].copy(), v[: nv[0]].copy(), g[: nv[0]].copy()

    def get_last_maxima(self):
        v, g = np.zeros(1), np.zeros(1)
        self._check(self._lib.cube_get_last_maxima(self._h, _ptr(v), _ptr(g)))
        return float(v[0]), float(g[0])

    def set_ic_parent(self, parent_np: int):
        """Refine the initial conditions from a parent_np^3 lattice of the same seed (0: off)."""
        self._check(self._lib.cube_set_ic_parent(self._h, parent_np))

    def enable_pids(self, pid_bytes: int = 8):
        """Carry a particle ID of pid_bytes (4 or 8; 0 drops them) through every step."""
        self._check(self._lib.cube_enable_pids(self._h, pid_bytes))
        self.pid_bytes = pid_bytes

    def get_pids(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.uint64 if self.pid_bytes == 8 else np.uint32)
        self._check(self._lib.cube_get_pids(self._h, _ptr(out)))
        return out

    def set_pids(self, ids):
        dt = np.uint64 if self.pid_bytes == 8 else np.uint32
        ids = np.ascontiguousarray(ids, dtype=dt)
        if ids.shape != (self.n,):
            raise ValueError(f"expected {self.n} IDs")
        self._check(self._lib.cube_set_pids(self._h, _ptr(ids)))

    def get_cross_power(self, other: "Sim", nbins: int | None = None):
        """(k, P_aa, P_bb, P_ab, n_modes) of this state (a) and `other` (b) over the same box; the
        cross-correlation coefficient is P_ab / sqrt(P_aa P_bb)."""
        nb = nbins or min(self.nm, other.nm) // 2
        out = [np.empty(nb) for _ in range(5)]
        self._check(self._lib.cube_get_cross_power(self._h, other._h, nb, *(_ptr(x) for x in out)))
        return tuple(out)

    def get_state(self, device: bool = False) -> dict:
        """The disjoint state as numpy arrays, or with device=True as torch tensors on the
        simulation's GPU (cnt and the codes as int32 / uint8 / int8 / int16 tensors of the same bits)."""
        n = self.n
        nc3 = self.nc**3
        if device:
            import torch
            tdt = {np.dtype(np.uint8): torch.uint8, np.dtype(np.int8): torch.int8, np.dtype(np.uint16): torch.int16,
                   np.dtype(np.int16): torch.int16}
            st = dict(cnt=torch.empty(nc3, dtype=torch.int32, device="cuda"),
                      chi=torch.empty((3, n), dtype=tdt[np.dtype(self.chi_dtype)], device="cuda"),
                      nu=torch.empty((3, n), dtype=tdt[np.dtype(self.nu_dtype)], device="cuda"),
                      vc=torch.empty((3, nc3), dtype=torch.float32, device="cuda"),
                      vs=torch.empty(nc3, dtype=torch.float32, device="cuda"))
            ptr = {k: c_void_p(t.data_ptr()) for k, t in st.items()}
        else:
            st = dict(cnt=np.empty(nc3, np.uint32), chi=np.empty((3, n), self.chi_dtype),
                      nu=np.empty((3, n), self.nu_dtype), vc=np.empty((3, nc3), np.float32), vs=np.empty(nc3, np.float32))
            ptr = {k: _ptr(a) for k, a in st.items()}
        view = CubeStateView(ptr["cnt"], ptr["chi"], ptr["nu"], ptr["vc"], ptr["vs"], n, 0.0, 0)
        self._check(self._lib.cube_get_state(self._h, byref(view)))
        st["a"] = view.a
        st["steps_done"] = view.steps_done
        return st

    def get_counts(self) -> np.ndarray:
        out = np.empty(self.nc**3, np.uint32)
        self._check(self._lib.cube_get_counts(self._h, _ptr(out)))
        return out

    def get_counts_u8(self):
        """(rho1 uint8[nc^3], overflow uint32[...]): the 1-byte count export of Sec. 2.1."""
        rho1 = np.empty(self.nc**3, np.uint8)
        nov = np.zeros(1, np.int64)
        over = np.empty(1024, np.uint32)
        rc = self._lib.cube_get_counts_u8(self._h, _ptr(rho1), _ptr(over), len(over), _ptr(nov))
        if rc == -4:  # CUBE_E_CAPACITY: the overflow list is longer
            over = np.empty(int(nov[0]), np.uint32)
            rc = self._lib.cube_get_counts_u8(self._h, _ptr(rho1), _ptr(over), len(over), _ptr(nov))
        self._check(rc)
        return rho1, over[: int(nov[0])].copy()

    def set_state(self, cnt, chi, nu, vc, vs, steps_done: int = 0):
        cnt = np.ascontiguousarray(cnt, np.uint32)
        chi = np.ascontiguousarray(chi, self.chi_dtype)
        nu = np.ascontiguousarray(nu, self.nu_dtype)
        vc = np.ascontiguousarray(vc, np.float32)
        vs = np.ascontiguousarray(vs, np.float32)
        view = CubeStateView(_ptr(cnt), _ptr(chi), _ptr(nu), _ptr(vc), _ptr(vs), chi.shape[1], 0.0, steps_done)
        self._check(self._lib.cube_set_state(self._h, byref(view)))

    def stage_deposit(self):
        self._check(self._lib.cube_stage_deposit(self._h))

    def stage_solve(self):
        self._check(self._lib.cube_stage_solve(self._h))

    def stage_move(self, kfac: float, dfac: float):
        self._check(self._lib.cube_stage_move(self._h, c_float(kfac), c_float(dfac)))

    def get_mesh(self, device: bool = False):
        """The real-space mesh [z, y, x]: numpy, or with device=True a torch tensor on the GPU."""
        if device:
            import torch
            out = torch.empty((self.nm,) * 3, dtype=torch.float32, device="cuda")
            self._check(self._lib.cube_get_mesh(self._h, c_void_p(out.data_ptr())))
            return out
        out = np.empty((self.nm,) * 3, dtype=np.float32)
        self._check(self._lib.cube_get_mesh(self._h, _ptr(out)))
        return out

    def set_mesh(self, field):
        f = np.ascontiguousarray(field, dtype=np.float32)
        assert f.shape == (self.nm,) * 3
        self._check(self._lib.cube_set_mesh(self._h, _ptr(f)))

    def get_ic_displacement(self) -> np.ndarray:
        out = np.empty((3,) + (self.np_side,) * 3, dtype=np.float32)
        self._check(self._lib.cube_get_ic_displacement(self._h, _ptr(out)))
        return out

    def get_tables(self):
        m = (1 << (8 * self.v_bytes)) - 1
        dec, edg = np.empty(m, np.float32), np.empty(m - 1, np.float32)
        self._check(self._lib.cube_get_tables(self._h, _ptr(dec), _ptr(edg)))
        return dec, edg

    def get_schedule(self):
        d0 = c_double()
        k, d = np.empty(self.n_steps), np.empty(self.n_steps)
        self._check(self._lib.cube_get_schedule(self._h, byref(d0), _ptr(k), _ptr(d)))
        return d0.value, k, d

    @property
    def device_bytes(self) -> int:
        return self._lib.cube_device_bytes(self._h)

    def set_profiling(self, on: bool = True):
        self._check(self._lib.cube_set_profiling(self._h, int(on)))

    TIMING_NAMES = ("deposit", "fft_x", "fft_y", "fft_z_green", "fft_y_inv", "fft_x_inv", "move_count",
                    "link_scan", "move_scatter")

    def get_timings(self) -> np.ndarray:
        """Average milliseconds per step of each kernel (order of TIMING_NAMES)."""
        out = np.empty(9)
        self._check(self._lib.cube_get_timings(self._h, _ptr(out)))
        return out

    # ---- kernel variants ---------------------------------------------------------------------
    def autotune(self):
        """Time the equivalent kernel variants on the current state and keep the fastest."""
        self._check(self._lib.cube_autotune(self._h))

    @property
    def autotune_report(self) -> str:
        """The per-variant times of the last autotune (text)."""
        return self._lib.cube_autotune_report(self._h).decode()

    @property
    def variant(self) -> dict:
        """The kernel variants in use (``cube_variant``): move_variant, fft_col_width, fft_z_order,
        deposit_variant."""
        v = CubeVariant()
        self._check(self._lib.cube_get_variant(self._h, byref(v)))
        return {name: getattr(v, name) for name, _ in CubeVariant._fields_}

    def set_variant(self, **changes):
        """Change some of the variants (keyword arguments named as the fields of ``variant``)."""
        cur = self.variant
        unknown = set(changes) - set(cur)
        if unknown:
            raise TypeError(f"unknown variant fields {sorted(unknown)}")
        if "fft_col_width" in changes and "fft_z_width" not in changes:
            cur["fft_z_width"] = changes["fft_col_width"]
        cur.update(changes)
        self._check(self._lib.cube_set_variant(self._h, byref(CubeVariant(**cur))))


class Batch:
    """An ensemble of independent boxes stepped together (``cube_batch_*``): one HIP graph launch
    per step for all boxes, each box on its own stream. ``boxes[i]`` is a ``Sim`` view of box i
    (owned by the batch) for every single-box call."""

    def __init__(self, configs: list[dict], torch_memory: bool = True):
        self._lib = load_library()
        n = len(configs)
        arr = (CubeParams * n)(*[make_params(**c) for c in configs])
        stream, alloc_p, self._keep = _torch_env(torch_memory)
        self._h = c_void_p()
        rc = self._lib.cube_batch_create(arr, n, stream, alloc_p, byref(self._h))
        if rc != CUBE_OK:
            raise CubeError(rc, "cube_batch_create: " + self._lib.cube_batch_last_error(None).decode())
        _live.add(self)
        self.boxes = [Sim(**c, _handle=c_void_p(self._lib.cube_batch_box(self._h, i))) for i, c in enumerate(configs)]

    def _check(self, rc: int) -> int:
        if rc < 0:
            raise CubeError(rc, self._lib.cube_batch_last_error(self._h).decode())
        return rc

    def __len__(self):
        return len(self.boxes)

    def init_ic(self):
        self._check(self._lib.cube_batch_init_ic(self._h))

    def autotune(self):
        self._check(self._lib.cube_batch_autotune(self._h))

    def step(self, k: int = 1) -> int:
        return self._check(self._lib.cube_batch_step(self._h, k))

    # 0: graph with a branch per box; 1: each box's kernels on its own stream; 2: graph with one
    # launch per stage over all boxes
    GRAPH, STREAMS, ENSEMBLE = 0, 1, 2

    def set_mode(self, mode: int):
        self._check(self._lib.cube_batch_set_mode(self._h, mode))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            for b in self.boxes:
                b._h = c_void_p()
            self._lib.cube_batch_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def counts_from_u8(rho1, overflow) -> np.ndarray:
    """Counts from the 1-byte export (host only, no GPU)."""
    lib = load_library()
    rho1 = np.ascontiguousarray(rho1, np.uint8)
    overflow = np.ascontiguousarray(overflow, np.uint32)
    out = np.empty(len(rho1), np.uint32)
    rc = lib.cube_counts_from_u8(_ptr(rho1), len(rho1), _ptr(overflow), len(overflow), _ptr(out))
    if rc != CUBE_OK:
        raise CubeError(rc, "overflow list does not match the cells marked 255")
    return out


def footprint(**cfg) -> int:
    """Device bytes a simulation of these parameters allocates at most (``cube_footprint``)."""
    lib = load_library()
    fp = lib.cube_footprint(byref(make_params(**cfg)))
    if fp < 0:
        raise CubeError(fp, "cube_footprint: invalid parameters")
    return fp


class Server:
    """Continuous-batching simulation server (``cube_server_*``): submit jobs at any time, call
    ``poll()`` repeatedly; it returns the ids of jobs that finished (or failed) since the last
    poll. ``job(id)`` is a ``Sim`` view of a finished job until ``release(id)``."""

    QUEUED, ACTIVE, FINISHED, FAILED = 0, 1, 2, 3

    def __init__(self, mem_budget_bytes: int, max_active: int = 16, slice_steps: int = 1, torch_memory: bool = True):
        self._lib = load_library()
        _, alloc_p, self._keep = _torch_env(torch_memory)
        self._h = c_void_p()
        rc = self._lib.cube_server_create(int(mem_budget_bytes), max_active, slice_steps, alloc_p, byref(self._h))
        if rc != CUBE_OK:
            raise CubeError(rc, "cube_server_create")
        _live.add(self)
        self._cfg = {}
        self._buf = np.empty(1024, np.int64)

    def _check(self, rc: int) -> int:
        if rc < 0:
            raise CubeError(rc, self._lib.cube_server_last_error(self._h).decode())
        return rc

    def submit(self, cfg: dict, job_id: int):
        self._check(self._lib.cube_server_submit(self._h, byref(make_params(**cfg)), job_id))
        self._cfg[job_id] = cfg

    def poll(self) -> list[int]:
        n = c_int32()
        self._check(self._lib.cube_server_poll(self._h, _ptr(self._buf), len(self._buf), byref(n)))
        return [int(x) for x in self._buf[: n.value]]

    def status(self, job_id: int) -> tuple[int, int]:
        st, rc = c_int32(), c_int32()
        self._check(self._lib.cube_server_status(self._h, job_id, byref(st), byref(rc)))
        return st.value, rc.value

    def job_error(self, job_id: int) -> str:
        return self._lib.cube_server_job_error(self._h, job_id).decode()

    def job(self, job_id: int) -> Sim:
        h = self._lib.cube_server_job(self._h, job_id)
        if not h:
            raise CubeError(-8, f"job {job_id} is not finished")
        return Sim(**self._cfg[job_id], _handle=c_void_p(h))

    def release(self, job_id: int):
        self._check(self._lib.cube_server_release(self._h, job_id))
        self._cfg.pop(job_id, None)

    def stats(self) -> tuple[int, int, int]:
        q, a, b = c_int32(), c_int32(), c_int64()
        self._check(self._lib.cube_server_stats(self._h, byref(q), byref(a), byref(b)))
        return q.value, a.value, b.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.cube_server_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
