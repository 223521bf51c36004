"""Crowd-of-walkers particle-by-particle QMC move on MI355X (gfx950).

Thin ctypes binding of ``libcrowdqmc.so`` (C ABI in ``include/cq.h``): argument
marshalling only, every step of the move runs in the library's HIP kernels.
PyTorch is optional plumbing: a torch CUDA tensor may be passed wherever a
device buffer is accepted and a torch stream as the crowd's stream.

The method is the batched particle-by-particle move of Luo, Doak and Kent,
arXiv 2209.14487 (the move and local-energy steps of Alg. 1 applied to every walker of a crowd in lock-step,
Sec. III "crowds", Alg. 4).
"""
import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrowdqmc.so")

CQ_OK, CQ_EINVAL, CQ_ENOMEM, CQ_EDEVICE, CQ_ESINGULAR, CQ_ESTATE, CQ_EIO = range(7)
CQ_FP64, CQ_MIXED = 0, 1
PATHS = {"auto": 0, "multi": 1, "window": 2, "batch": 3, "sweep": 4}
KERNEL_VGL, KERNEL_RESOLVE, KERNEL_UPDATE, KERNEL_ENERGY, KERNEL_INVERSE, KERNEL_PROPOSE, KERNEL_VIRTUAL = range(7)
KERNEL_NAMES = {"vgl": KERNEL_VGL, "resolve": KERNEL_RESOLVE, "update": KERNEL_UPDATE,
                "energy": KERNEL_ENERGY, "inverse": KERNEL_INVERSE, "propose": KERNEL_PROPOSE,
                "virtual": KERNEL_VIRTUAL}

_STATUS_NAMES = {1: "CQ_EINVAL", 2: "CQ_ENOMEM", 3: "CQ_EDEVICE", 4: "CQ_ESINGULAR", 5: "CQ_ESTATE", 6: "CQ_EIO"}


class CqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class CrowdDesc(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("delay_rank", ctypes.c_int), ("recompute_every", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("first_uid", ctypes.c_uint32), ("hip_stream", ctypes.c_void_p),
                ("use_graph", ctypes.c_int), ("kernel_path", ctypes.c_int), ("max_walkers", ctypes.c_int),
                ("streams", ctypes.c_int)]


class Tiles(ctypes.Structure):
    """cq_tiles: candidates per round (Q), gather workgroups per CU beside the update, and the
    FP64 update kernel (1 vector units, 2 matrix cores; 0 default)."""
    _fields_ = [("candidates", ctypes.c_int), ("gather_blocks_per_cu", ctypes.c_int), ("update_kernel", ctypes.c_int)]


def _tiles_dict(t):
    return dict(candidates=t.candidates, gather_blocks_per_cu=t.gather_blocks_per_cu, update_kernel=t.update_kernel)


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "cq_system_create": [_I, _I, ctypes.c_double, _P],
    "cq_system_load_bspline": [_P, _P, _I, _I, _I, _I, _I, _I],
    "cq_system_fill_bspline_philox": [_P, ctypes.c_uint64, _I, _I, _I],
    "cq_system_load_pade_j2": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "cq_system_load_pade_j1": [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double],
    "cq_system_set_coulomb": [_P, _I],
    "cq_system_destroy": [_P],
    "cq_crowd_create": [_P, _P, _I, _P, _P],
    "cq_crowd_set_positions": [_P, _P, _I, ctypes.c_uint32],
    "cq_crowd_run_vmc": [_P, _I, ctypes.c_double],
    "cq_crowd_run_dmc": [_P, _I, ctypes.c_double, ctypes.c_double, _I, _P],
    "cq_crowd_run_dmc_systems": [_P, _I, ctypes.c_double, _P, _P, _P],
    "cq_crowd_get_population": [_P, _P],
    "cq_crowd_virtual_ratios": [_P, _P, _I, _P, _P, _P, _I],
    "cq_crowd_autotune": [_P, _I, _P],
    "cq_crowd_get_delay_rank": [_P, _P],
    "cq_crowd_get_path": [_P, _P],
    "cq_crowd_set_round_plan": [_P, ctypes.c_int],
    "cq_crowd_set_tiles": [_P, _P],
    "cq_crowd_get_tiles": [_P, _P],
    "cq_crowd_autotune_tiles": [_P, _I, ctypes.c_char_p, _P, _P],
    "cq_tile_cache_find": [ctypes.c_char_p, ctypes.c_char_p, _I, _I, _I, _I, _P, _P],
    "cq_tile_cache_store": [ctypes.c_char_p, ctypes.c_char_p, _I, _I, _I, _I, _P, ctypes.c_double],
    "cq_crowd_get_round_plan": [_P, _P],
    "cq_crowd_get_uids": [_P, _P],
    "cq_crowd_recompute": [_P, _P],
    "cq_crowd_get_drift": [_P, _P, _P, _P],
    "cq_crowd_get_logdet": [_P, _P, _P],
    "cq_crowd_get_acceptance": [_P, _P, _P],
    "cq_crowd_get_local_energy": [_P, _P],
    "cq_crowd_get_positions": [_P, _P, _P],
    "cq_crowd_get_inverse": [_P, _P],
    "cq_crowd_set_forced_decisions": [_P, _P, _I],
    "cq_crowd_set_forced_branching": [_P, _P, _I],
    "cq_crowd_get_dmc_moves": [_P, _P, _P],
    "cq_crowd_record_moves": [_P, _I],
    "cq_crowd_get_move_records": [_P, _P, _P, _P, _P],
    "cq_crowd_get_move_proposals": [_P, _P],
    "cq_crowd_set_kernel_timing": [_P, _I],
    "cq_crowd_get_kernel_timing": [_P, _I, _P, _P],
    "cq_crowd_synchronize": [_P],
    "cq_device_copy": [_P, _P, ctypes.c_uint64, _P],
    "cq_slater_inverse": [_P, _I, _I, _I, _P, _P, _P, _P],
    "cq_slater_inverse_static": [_P, _I, _I, _I, _P, _P, _P, _P],
    "cq_crowd_destroy": [_P],
    "cq_csystem_create": [_I, _P, _P, _P],
    "cq_csystem_load_bspline": [_P, _P, _I, _I, _I, _I],
    "cq_csystem_load_pade_j2": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    "cq_csystem_destroy": [_P],
    "cq_ccrowd_create": [_P, _I, _I, ctypes.c_uint64, ctypes.c_uint32, _P, _P],
    "cq_ccrowd_set_positions": [_P, _P, ctypes.c_uint32],
    "cq_ccrowd_run_vmc": [_P, _I, ctypes.c_double],
    "cq_ccrowd_recompute": [_P, _P],
    "cq_ccrowd_get_logdet": [_P, _P, _P],
    "cq_ccrowd_get_local_energy": [_P, _P],
    "cq_ccrowd_get_positions": [_P, _P],
    "cq_ccrowd_get_acceptance": [_P, _P, _P],
    "cq_ccrowd_get_inverse": [_P, _I, _I, _P],
    "cq_ccrowd_record_moves": [_P, _I],
    "cq_ccrowd_get_move_records": [_P, _P, _P, _P, _P],
    "cq_ccrowd_set_timing": [_P, _I],
    "cq_ccrowd_get_timing": [_P, _P, _P],
    "cq_ccrowd_synchronize": [_P],
    "cq_ccrowd_destroy": [_P],
    "cq_last_error": [],
}
_VOID = {"cq_system_destroy", "cq_crowd_destroy", "cq_csystem_destroy", "cq_ccrowd_destroy"}


def lib():
    """Load the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcrowdqmc.so is not built; run __graft_entry__.build() "
                              "(hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name in _VOID else (ctypes.c_char_p if name == "cq_last_error" else ctypes.c_int)
        _lib = L
    return _lib


def exported_names():
    return list(_SIGS)


def _check(st):
    if st != CQ_OK:
        raise CqError(st, lib().cq_last_error().decode())


def _prec(precision) -> int:
    return CQ_FP64 if precision in ("fp64", CQ_FP64) else CQ_MIXED


def tile_cache_find(path, device: str, n: int, walkers: int, precision, delay_rank: int):
    """The tile cache's last entry for the key (cq_tile_cache_find; host only), or None."""
    t, found = Tiles(), ctypes.c_int()
    _check(lib().cq_tile_cache_find(os.fsencode(path), device.encode(), int(n), int(walkers), _prec(precision),
                                    int(delay_rank), ctypes.byref(t), ctypes.byref(found)))
    return _tiles_dict(t) if found.value else None


def tile_cache_store(path, device: str, n: int, walkers: int, precision, delay_rank: int, candidates: int,
                     gather_blocks_per_cu: int, ms_per_sweep: float, update_kernel: int = 0):
    """Append an entry to the tile cache (cq_tile_cache_store; host only)."""
    t = Tiles(int(candidates), int(gather_blocks_per_cu), int(update_kernel))
    _check(lib().cq_tile_cache_store(os.fsencode(path), device.encode(), int(n), int(walkers), _prec(precision),
                                     int(delay_rank), ctypes.byref(t), float(ms_per_sweep)))


_hip = None


def _hiprt():
    """The HIP runtime the library is linked against (already loaded with it)."""
    global _hip
    if _hip is None:
        lib()
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        h.hipFree.argtypes = [ctypes.c_void_p]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipDeviceSynchronize.argtypes = []
        for f in (h.hipMalloc, h.hipFree, h.hipMemcpy, h.hipDeviceSynchronize):
            f.restype = ctypes.c_int
        _hip = h
    return _hip


class DeviceArray:
    """A device buffer of the library's HIP runtime holding an array (plumbing for callers
    that pass device pointers): created from a numpy array (copied in) or zeros of a shape and
    dtype; ``ptr`` is the device address, ``numpy()`` copies the contents back."""

    def __init__(self, arr=None, shape=None, dtype=None):
        if arr is not None:
            arr = np.ascontiguousarray(arr)
            shape, dtype = arr.shape, arr.dtype
        self.shape, self.dtype = tuple(shape), np.dtype(dtype)
        self.nbytes = int(np.prod(self.shape)) * self.dtype.itemsize
        p = ctypes.c_void_p()
        h = _hiprt()
        if h.hipMalloc(ctypes.byref(p), max(self.nbytes, 16)) != 0:
            raise MemoryError("hipMalloc of %d bytes failed" % self.nbytes)
        self.ptr = p.value
        src = arr if arr is not None else np.zeros(self.shape, self.dtype)
        if self.nbytes and h.hipMemcpy(self.ptr, src.ctypes.data, self.nbytes, 1) != 0:
            raise RuntimeError("hipMemcpy to the device failed")

    @property
    def itemsize(self):
        return self.dtype.itemsize

    def numpy(self):
        out = np.empty(self.shape, self.dtype)
        if self.nbytes and _hiprt().hipMemcpy(out.ctypes.data, self.ptr, self.nbytes, 2) != 0:
            raise RuntimeError("hipMemcpy from the device failed")
        return out

    def free(self):
        if self.ptr:
            _hiprt().hipFree(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def device_copy(dst, src, nbytes: int, stream=None):
    """Library streaming copy between device buffers (traffic-counter calibration)."""
    _check(lib().cq_device_copy(_ptr(dst), _ptr(src), nbytes, _stream_handle(stream)))


def slater_inverse(A, Minv, logdet, sign, stream=None):
    """FP64 Gauss-Jordan inverses of device matrices A [nmat][n][n] (DeviceArray or torch CUDA
    tensors, float32 or float64): Minv[m][a][j] = (A_m^-1)[j][a], logdet [nmat] float64, sign
    [nmat] int32."""
    nmat, n = A.shape[0], A.shape[1]
    _check(lib().cq_slater_inverse(_ptr(A), _itemsize(A), n, nmat, _ptr(Minv), _ptr(logdet), _ptr(sign),
                                   _stream_handle(stream)))


def slater_inverse_static(A, Minv, logdet, sign, stream=None):
    """slater_inverse on the library's static workspace (no device allocation)."""
    nmat, n = A.shape[0], A.shape[1]
    _check(lib().cq_slater_inverse_static(_ptr(A), _itemsize(A), n, nmat, _ptr(Minv), _ptr(logdet), _ptr(sign),
                                          _stream_handle(stream)))


def _itemsize(x):
    return x.itemsize if isinstance(x, DeviceArray) else x.element_size()


def _ptr(x):
    """Device or host address of a numpy array, a torch tensor or an int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    if isinstance(x, DeviceArray):
        return x.ptr
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    raise TypeError("unsupported buffer type %r" % type(x))


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


class System:
    """Electrons, box, B-spline orbitals and Pade J2 of one system (cq_system)."""

    def __init__(self, n_per_spin: int, box_L: float):
        h = ctypes.c_void_p()
        _check(lib().cq_system_create(n_per_spin, n_per_spin, box_L, ctypes.byref(h)))
        self._h = h
        self.n = n_per_spin
        self.L = box_L
        self._keep = []

    def fill_philox(self, seed: int, elem_bytes: int, grid: int):
        _check(lib().cq_system_fill_bspline_philox(self._h, seed, elem_bytes, grid, self.n))

    def load_table(self, table, elem_bytes: Optional[int] = None):
        """table [G][G][G][N]: numpy (copied) or a torch CUDA tensor (borrowed, kept alive here)."""
        G = table.shape[0]
        if isinstance(table, np.ndarray):
            eb = table.dtype.itemsize if elem_bytes is None else elem_bytes
            arr = np.ascontiguousarray(table, dtype=np.float32 if eb == 4 else np.float64)
            _check(lib().cq_system_load_bspline(self._h, arr.ctypes.data, eb, G, G, G, table.shape[3], 0))
        else:
            assert table.is_contiguous()
            eb = table.element_size()
            self._keep.append(table)
            _check(lib().cq_system_load_bspline(self._h, table.data_ptr(), eb, G, G, G, table.shape[3], 1))

    def load_j2(self, a_par=0.25, a_anti=0.5, b=1.0):
        _check(lib().cq_system_load_pade_j2(self._h, a_par, a_anti, b))

    def load_j1(self, centres, a, b):
        """One-body Pade Jastrow a r / (1 + b r) around the centres [n][3] (n = 0 removes it)."""
        c = np.ascontiguousarray(np.asarray(centres, dtype=np.float64).reshape(-1, 3))
        _check(lib().cq_system_load_pade_j1(self._h, c.ctypes.data if c.size else None, c.shape[0], a, b))

    def set_coulomb(self, enable: bool = True):
        """Include the Ewald electron-electron energy in E_L of crowds created afterwards."""
        _check(lib().cq_system_set_coulomb(self._h, int(enable)))

    def close(self):
        if self._h:
            lib().cq_system_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Crowd:
    """A crowd of walkers moved in lock-step (cq_crowd): of one system, or of several systems
    (pass lists of systems and walker counts) whose DMC generations share their launches."""

    def __init__(self, system, n_walkers, precision: str = "mixed", delay_rank: int = 1,
                 recompute_every: int = 0, seed: int = 0, first_uid: int = 0, stream=None,
                 use_graph: bool = True, path: str = "auto", max_walkers: int = 0, streams: int = 2):
        systems = list(system) if isinstance(system, (list, tuple)) else [system]
        counts = list(n_walkers) if isinstance(n_walkers, (list, tuple)) else [n_walkers]
        assert len(systems) == len(counts)
        self.group = len(systems) > 1
        self.systems = systems
        self.system = systems[0]
        self.Ws = counts
        self.W = sum(counts)
        self._w0 = self.W
        self.Wcap = max(self.W, max_walkers)  # walker stride of the parity-mode buffers
        self.n = systems[0].n
        self.ne = 2 * systems[0].n
        desc = CrowdDesc(CQ_MIXED if precision == "mixed" else CQ_FP64, delay_rank, recompute_every, seed,
                         first_uid, _stream_handle(stream), int(use_graph), PATHS[path], max_walkers, streams)
        hs = (ctypes.c_void_p * len(systems))(*[x._h.value for x in systems])
        cs = (ctypes.c_int * len(counts))(*counts)
        h = ctypes.c_void_p()
        _check(lib().cq_crowd_create(hs, cs, len(systems), ctypes.byref(desc), ctypes.byref(h)))
        self._h = h
        self._rec = 0

    def _refresh_counts(self):
        counts = (ctypes.c_int * len(self.systems))()
        _check(lib().cq_crowd_get_positions(self._h, None, counts))
        self.Ws = list(counts)
        self.W = sum(self.Ws)

    def run_dmc_systems(self, n_generations: int, tau: float, e_trial=None, n_target=None):
        """DMC generations of every system (one launch per step serves the walkers of all of
        them); returns the history [n_generations][n_systems][4] (population, sum of weights,
        E_est, E_T).  e_trial, n_target: per system (None: continue / the starting counts)."""
        S = len(self.systems)
        h = np.zeros((n_generations, S, 4))
        et = None if e_trial is None else np.ascontiguousarray(e_trial, dtype=np.float64)
        nt = None if n_target is None else np.ascontiguousarray(n_target, dtype=np.int32)
        try:
            _check(lib().cq_crowd_run_dmc_systems(self._h, n_generations, tau, None if et is None else et.ctypes.data,
                                                  None if nt is None else nt.ctypes.data, h.ctypes.data))
        finally:
            self._refresh_counts()
        return h

    def set_positions(self, R, first_step: int = 0):
        if self.group:  # one array [W_s][Ne_s][3] per system
            flat = np.concatenate([np.ascontiguousarray(r, dtype=np.float64).ravel() for r in R])
            _check(lib().cq_crowd_set_positions(self._h, flat.ctypes.data, 0, first_step))
            return
        if isinstance(R, np.ndarray):
            R = np.ascontiguousarray(R, dtype=np.float64)
            assert R.shape == (self.W, self.ne, 3)
            _check(lib().cq_crowd_set_positions(self._h, R.ctypes.data, 0, first_step))
        else:
            _check(lib().cq_crowd_set_positions(self._h, R.data_ptr(), 1, first_step))

    def run_vmc(self, n_sweeps: int, sigma: float = 0.5):
        _check(lib().cq_crowd_run_vmc(self._h, n_sweeps, sigma))

    def run_dmc(self, n_generations: int, tau: float, e_trial: float = float("nan"), n_target: int = 0):
        """DMC generations; returns the history [n_generations][4] (population, sum of
        weights, E_est, E_T).  n_target 0: the initial walker count."""
        h = np.zeros((n_generations, 4))
        if n_target <= 0:
            n_target = self._w0
        try:
            _check(lib().cq_crowd_run_dmc(self._h, n_generations, tau, e_trial, n_target, h.ctypes.data))
        finally:
            self.W = self.population()
        return h

    def autotune(self, sweeps_per_candidate: int = 1) -> int:
        k = ctypes.c_int()
        _check(lib().cq_crowd_autotune(self._h, sweeps_per_candidate, ctypes.byref(k)))
        return k.value

    def delay_rank(self) -> int:
        k = ctypes.c_int()
        _check(lib().cq_crowd_get_delay_rank(self._h, ctypes.byref(k)))
        return k.value

    def set_round_plan(self, rounds: int):
        """Rounds per spin block of the batched path before the tail kernel (0: learned)."""
        _check(lib().cq_crowd_set_round_plan(self._h, int(rounds)))

    def round_plan(self):
        r = np.zeros(2, np.int32)
        _check(lib().cq_crowd_get_round_plan(self._h, r.ctypes.data))
        return r

    def set_tiles(self, candidates: int = 0, gather_blocks_per_cu: int = 0, update_kernel: int = 0):
        """Launch shapes of the batched path (0: default); see cq_crowd_set_tiles."""
        t = Tiles(int(candidates), int(gather_blocks_per_cu), int(update_kernel))
        _check(lib().cq_crowd_set_tiles(self._h, ctypes.byref(t)))

    def tiles(self) -> dict:
        t = Tiles()
        _check(lib().cq_crowd_get_tiles(self._h, ctypes.byref(t)))
        return _tiles_dict(t)

    def autotune_tiles(self, sweeps_per_candidate: int = 1, cache_path=None):
        """Time the candidate launch shapes (or take them from the JSON cache); returns
        (tiles dict, from_cache)."""
        t, hit = Tiles(), ctypes.c_int()
        path = None if cache_path is None else os.fsencode(cache_path)
        _check(lib().cq_crowd_autotune_tiles(self._h, int(sweeps_per_candidate), path, ctypes.byref(t),
                                             ctypes.byref(hit)))
        return _tiles_dict(t), bool(hit.value)

    def path(self) -> str:
        """The kernel path in use ("multi", "window", "batch" or "sweep")."""
        p = ctypes.c_int()
        _check(lib().cq_crowd_get_path(self._h, ctypes.byref(p)))
        return {v: k for k, v in PATHS.items()}[p.value]

    def virtual_ratios(self, offsets, out=None):
        """Ratio-only virtual moves of every electron to r_e + offsets[q] ([n_q][3]): returns
        (ratio, rho_D, dlnJ) host arrays [W][Ne][n_q]; with out = (ratio, rho, dlnj) device
        buffers (DeviceArray or None each) the call only enqueues the kernel."""
        off = np.ascontiguousarray(offsets, dtype=np.float64).reshape(-1, 3)
        nq = off.shape[0]
        if out is not None:
            _check(lib().cq_crowd_virtual_ratios(self._h, off.ctypes.data, nq, *[_ptr(o) for o in out], 1))
            return None
        res = [np.zeros((self.W, self.ne, nq)) for _ in range(3)]
        _check(lib().cq_crowd_virtual_ratios(self._h, off.ctypes.data, nq, *[r.ctypes.data for r in res], 0))
        return tuple(res)

    def population(self) -> int:
        n = ctypes.c_int()
        _check(lib().cq_crowd_get_population(self._h, ctypes.byref(n)))
        return n.value

    def uids(self):
        u = np.zeros(self.W, np.uint32)
        _check(lib().cq_crowd_get_uids(self._h, u.ctypes.data))
        return u

    def recompute(self) -> float:
        d = ctypes.c_double()
        _check(lib().cq_crowd_recompute(self._h, ctypes.byref(d)))
        return d.value

    def drift(self):
        """(drift [W][2] at the last inversion, largest drift of any recompute since the positions
        were set, number of recomputes since then); drift = |log|det| kept - log|det| recomputed|."""
        last = np.zeros((self.W, 2))
        m = ctypes.c_double()
        k = ctypes.c_int()
        _check(lib().cq_crowd_get_drift(self._h, last.ctypes.data, ctypes.byref(m), ctypes.byref(k)))
        return last, m.value, k.value

    def logdet(self):
        ld = np.zeros((self.W, 2))
        sg = np.zeros((self.W, 2), np.int32)
        _check(lib().cq_crowd_get_logdet(self._h, ld.ctypes.data, sg.ctypes.data))
        return ld, sg

    def acceptance(self):
        a = np.zeros(self.W, np.int64)
        p = np.zeros(self.W, np.int64)
        _check(lib().cq_crowd_get_acceptance(self._h, a.ctypes.data, p.ctypes.data))
        return a, p

    def local_energy(self):
        e = np.zeros(self.W)
        _check(lib().cq_crowd_get_local_energy(self._h, e.ctypes.data))
        return e

    def positions(self):
        """[W][Ne][3]; with several systems a list of [W_s][Ne_s][3]."""
        if self.group:
            self._refresh_counts()
            sizes = [w * 2 * x.n * 3 for w, x in zip(self.Ws, self.systems)]
            flat = np.zeros(sum(sizes))
            _check(lib().cq_crowd_get_positions(self._h, flat.ctypes.data, None))
            out, o = [], 0
            for w, x, k in zip(self.Ws, self.systems, sizes):
                out.append(flat[o:o + k].reshape(w, 2 * x.n, 3))
                o += k
            return out
        R = np.zeros((self.W, self.ne, 3))
        _check(lib().cq_crowd_get_positions(self._h, R.ctypes.data, None))
        return R

    def inverse(self):
        """A^-1 per walker and spin, [W][2][N][N] FP64 (row = orbital, column = electron)."""
        a = np.zeros((self.W, 2, self.n, self.n))
        _check(lib().cq_crowd_get_inverse(self._h, a.ctypes.data))
        return a

    def set_forced(self, flags: Optional[np.ndarray]):
        if flags is None:
            _check(lib().cq_crowd_set_forced_decisions(self._h, None, 0))
        else:
            f = np.ascontiguousarray(flags, dtype=np.uint8)
            if f.shape[1:] != (self.ne, self.Wcap):  # [sweeps][Ne][W] padded with own decisions
                assert f.shape[1] == self.ne and f.shape[2] <= self.Wcap
                g = np.full((f.shape[0], self.ne, self.Wcap), 2, np.uint8)
                g[:, :, :f.shape[2]] = f
                f = g
            _check(lib().cq_crowd_set_forced_decisions(self._h, f.ctypes.data, f.shape[0]))

    def set_forced_branching(self, mult: Optional[np.ndarray]):
        """DMC parity mode: multiplicities [generations][<= Wcap] to follow (None: off)."""
        if mult is None:
            _check(lib().cq_crowd_set_forced_branching(self._h, None, 0))
        else:
            m = np.zeros((mult.shape[0], self.Wcap), np.int32)
            m[:, :mult.shape[1]] = mult
            _check(lib().cq_crowd_set_forced_branching(self._h, m.ctypes.data, m.shape[0]))

    def dmc_moves(self):
        """(accepted, proposed) drift-diffusion moves over every DMC generation run so far."""
        a = ctypes.c_int64()
        p = ctypes.c_int64()
        _check(lib().cq_crowd_get_dmc_moves(self._h, ctypes.byref(a), ctypes.byref(p)))
        return a.value, p.value

    def record(self, n_sweeps: int):
        _check(lib().cq_crowd_record_moves(self._h, n_sweeps))
        self._rec = n_sweeps

    def records(self, all_slots: bool = False):
        """Per-move records [sweeps][Ne][W] (all_slots: [sweeps][Ne][Wcap], every walker slot)."""
        shp = (self._rec, self.ne, self.Wcap)
        rho, dl, pr = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        acc = np.zeros(shp, np.uint8)
        _check(lib().cq_crowd_get_move_records(self._h, rho.ctypes.data, dl.ctypes.data, pr.ctypes.data,
                                               acc.ctypes.data))
        out = dict(rho=rho, dlnj=dl, prob=pr, acc=acc)
        rn = np.zeros(shp + (3,))
        _check(lib().cq_crowd_get_move_proposals(self._h, rn.ctypes.data))
        out["rnew"] = rn  # DMC proposals (NaN for VMC sweeps)
        if not all_slots:
            out = {k: v[:, :, :self.W] for k, v in out.items()}
        return out

    def set_timing(self, kinds=()):
        """Time the given kernel kinds (names or ids) with HIP events; () switches timing off."""
        mask = 0
        for k in kinds:
            mask |= 1 << (KERNEL_NAMES[k] if isinstance(k, str) else k)
        _check(lib().cq_crowd_set_kernel_timing(self._h, mask))

    def kernel_timing(self, kind):
        k = KERNEL_NAMES[kind] if isinstance(kind, str) else kind
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().cq_crowd_get_kernel_timing(self._h, k, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def synchronize(self):
        _check(lib().cq_crowd_synchronize(self._h))

    def close(self):
        if self._h:
            lib().cq_crowd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ComplexSystem:
    """Complex (Bloch) orbitals with a twist in a general cell (cq_csystem); FP64."""

    def __init__(self, n_per_spin: int, lattice, twist=(0.0, 0.0, 0.0)):
        lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(3, 3))
        k = np.ascontiguousarray(np.asarray(twist, dtype=np.float64).reshape(3))
        h = ctypes.c_void_p()
        _check(lib().cq_csystem_create(n_per_spin, lat.ctypes.data, k.ctypes.data, ctypes.byref(h)))
        self._h = h
        self.n = n_per_spin
        self._keep = []

    def load_table(self, table):
        """table [G][G][G][N] complex128 (FP64 crowds) or complex64 (mixed crowds): numpy (copied)
        or a torch CUDA tensor of that type (borrowed, kept alive here)."""
        G = table.shape[0]
        if isinstance(table, np.ndarray):
            eb = 8 if table.dtype == np.complex64 else 16
            arr = np.ascontiguousarray(table, dtype=np.complex64 if eb == 8 else np.complex128)
            _check(lib().cq_csystem_load_bspline(self._h, arr.ctypes.data, eb, G, table.shape[3], 0))
        else:
            assert table.is_contiguous() and table.element_size() in (8, 16)
            self._keep.append(table)
            _check(lib().cq_csystem_load_bspline(self._h, table.data_ptr(), table.element_size(), G,
                                                 table.shape[3], 1))

    def load_j2(self, a_par=0.25, a_anti=0.5, b=1.0):
        _check(lib().cq_csystem_load_pade_j2(self._h, a_par, a_anti, b))

    def close(self):
        if self._h:
            lib().cq_csystem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ComplexCrowd:
    """Walkers of a ComplexSystem moved by one sweep kernel per sweep (cq_ccrowd)."""

    def __init__(self, system: ComplexSystem, walkers: int, seed: int = 0, first_uid: int = 0, stream=None,
                 precision: str = "fp64"):
        """precision "fp64": complex128 table; "mixed": complex64 table, FP64 arithmetic."""
        h = ctypes.c_void_p()
        _check(lib().cq_ccrowd_create(system._h, walkers, _prec(precision), seed, first_uid, stream,
                                      ctypes.byref(h)))
        self._h = h
        self.sys = system
        self.W = walkers
        self.n = system.n
        self._rec = 0

    def set_positions(self, R, first_step: int = 0):
        R = np.ascontiguousarray(R, dtype=np.float64)
        assert R.shape == (self.W, 2 * self.n, 3)
        _check(lib().cq_ccrowd_set_positions(self._h, R.ctypes.data, first_step))

    def run_vmc(self, n_sweeps: int, sigma: float = 0.5):
        _check(lib().cq_ccrowd_run_vmc(self._h, n_sweeps, sigma))

    def recompute(self) -> float:
        d = ctypes.c_double()
        _check(lib().cq_ccrowd_recompute(self._h, ctypes.byref(d)))
        return d.value

    def logdet(self):
        """(log|det| [W][2], phase [W][2])."""
        ld = np.zeros((self.W, 2))
        ph = np.zeros((self.W, 2))
        _check(lib().cq_ccrowd_get_logdet(self._h, ld.ctypes.data, ph.ctypes.data))
        return ld, ph

    def local_energy(self):
        el = np.zeros((self.W, 2))
        _check(lib().cq_ccrowd_get_local_energy(self._h, el.ctypes.data))
        return el[:, 0] + 1j * el[:, 1]

    def positions(self):
        R = np.zeros((self.W, 2 * self.n, 3))
        _check(lib().cq_ccrowd_get_positions(self._h, R.ctypes.data))
        return R

    def acceptance(self):
        a = np.zeros(self.W, np.int64)
        p = np.zeros(self.W, np.int64)
        _check(lib().cq_ccrowd_get_acceptance(self._h, a.ctypes.data, p.ctypes.data))
        return a, p

    def inverse(self, walker: int, spin: int):
        """A^-1 [n][n] complex (row j orbital, column i electron)."""
        out = np.zeros((self.n, self.n, 2))
        _check(lib().cq_ccrowd_get_inverse(self._h, walker, spin, out.ctypes.data))
        return out[..., 0] + 1j * out[..., 1]

    def record(self, n_sweeps: int):
        _check(lib().cq_ccrowd_record_moves(self._h, n_sweeps))
        self._rec = n_sweeps

    def records(self):
        """rho [S][Ne][W] complex, dlnj, prob [S][Ne][W], acc [S][Ne][W] uint8."""
        shp = (self._rec, 2 * self.n, self.W)
        rho = np.zeros(shp + (2,))
        dj = np.zeros(shp)
        pr = np.zeros(shp)
        acc = np.zeros(shp, np.uint8)
        _check(lib().cq_ccrowd_get_move_records(self._h, rho.ctypes.data, dj.ctypes.data, pr.ctypes.data,
                                                acc.ctypes.data))
        return dict(rho=rho[..., 0] + 1j * rho[..., 1], dlnj=dj, prob=pr, acc=acc)

    def set_timing(self, on: bool = True):
        _check(lib().cq_ccrowd_set_timing(self._h, int(on)))

    def timing(self):
        """(device ms, launches) of the sweep kernel since timing was switched on or last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().cq_ccrowd_get_timing(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def synchronize(self):
        _check(lib().cq_ccrowd_synchronize(self._h))

    def close(self):
        if self._h:
            lib().cq_ccrowd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
