"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every computation runs in the gfx950 kernels of ``liblbm.so``; this module
only converts arguments.  PyTorch supplies device memory and streams when a
caller wants to pass device buffers (``tensor.data_ptr()``) or a stream
(``torch.cuda.current_stream().cuda_stream``).  There is no fallback: if the
library is not built, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # load torch's HIP runtime first so the library and torch share it
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is optional for the binding
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EUNSUPPORTED, LBM_EUNSTABLE, LBM_EDEVICE = 0, -1, -2, -3, -4, -5
LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_BGK, LBM_RR, LBM_HRR = 0, 1, 2
LBM_FP64, LBM_FP32_DEV = 0, 1
LBM_HOST, LBM_DEVICE = 0, 1
LBM_C_MIDDLE, LBM_C_TF, LBM_C_TN, LBM_C_COVERED = 0, 1, 2, 3
LBM_F_MIDDLE, LBM_F_TF, LBM_F_IE, LBM_F_IE_FACE, LBM_F_TN = 0, 1, 2, 3, 4
LBM_N_VARIANTS = 4

EXPORTS = (
    "lbm_create_grid", "lbm_destroy", "lbm_set_state", "lbm_step", "lbm_get_macros",
    "lbm_set_populations", "lbm_get_populations", "lbm_get_totals", "lbm_get_totals_noalloc", "lbm_sensors_enable", "lbm_sensors",
    "lbm_set_dynamic_sigma", "lbm_create_nested",
    "lbm_probe_enable", "lbm_probe_read", "lbm_get_index_maps",
    "lbm_level_dims", "lbm_lattice_info", "lbm_interface_counts", "lbm_interface_tables",
    "lbm_updates_per_step", "lbm_profile_enable", "lbm_kernel_time", "lbm_tune", "lbm_set_variants",
    "lbm_last_error", "lbm_batch_create", "lbm_batch_destroy", "lbm_batch_add", "lbm_batch_remove",
    "lbm_batch_set_state", "lbm_batch_get_macros", "lbm_batch_get_populations", "lbm_batch_step",
    "lbm_batch_use_graph", "lbm_batch_tune", "lbm_batch_set_variants", "lbm_batch_info", "lbm_batch_slot_steps", "lbm_footprint", "lbm_copy_probe",
    "lbm_batch_last_error",
)


class lbm_grid_desc(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("collision", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3), ("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3),
        ("tau_coarse", ctypes.c_double), ("sigma", ctypes.c_double),
        ("device", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Loads liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.lbm_create_grid.argtypes = [ctypes.POINTER(lbm_grid_desc), ctypes.POINTER(vp)]
    L.lbm_create_nested.argtypes = [ctypes.POINTER(lbm_grid_desc), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(vp)]
    L.lbm_destroy.argtypes = [vp]
    L.lbm_set_state.argtypes = [vp, ip, vp, vp, ip]
    L.lbm_step.argtypes = [vp, ip, vp]
    L.lbm_get_macros.argtypes = [vp, ip, vp, vp, ip]
    L.lbm_set_populations.argtypes = [vp, ip, vp, ip]
    L.lbm_get_populations.argtypes = [vp, ip, vp, ip]
    L.lbm_get_totals.argtypes = [vp, dp, dp]
    L.lbm_get_totals_noalloc.argtypes = [vp, dp, dp]
    L.lbm_sensors_enable.argtypes = [vp, ip]
    L.lbm_sensors.argtypes = [vp, ip, ctypes.c_double, vp, vp, ip]
    L.lbm_set_dynamic_sigma.argtypes = [vp, ip, ctypes.c_double, ctypes.c_double]
    L.lbm_probe_enable.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64]
    L.lbm_probe_read.argtypes = [vp, dp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_get_index_maps.argtypes = [vp, ip, vp, ip]
    L.lbm_level_dims.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int32)]
    L.lbm_lattice_info.argtypes = [ip, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), dp]
    L.lbm_interface_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_interface_tables.argtypes = [vp, vp, vp, vp, vp]
    L.lbm_updates_per_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_profile_enable.argtypes = [vp, ip]
    L.lbm_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), dp, ctypes.POINTER(ctypes.c_int64)]
    L.lbm_tune.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int32)]
    L.lbm_set_variants.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.lbm_last_error.argtypes = [vp]
    L.lbm_last_error.restype = ctypes.c_char_p
    i32p, i64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
    L.lbm_batch_create.argtypes = [ip, ip, ip, ip, ip, ctypes.POINTER(vp)]
    L.lbm_batch_destroy.argtypes = [vp]
    L.lbm_batch_add.argtypes = [vp, ctypes.POINTER(lbm_grid_desc), i32p]
    L.lbm_batch_remove.argtypes = [vp, ip]
    L.lbm_batch_set_state.argtypes = [vp, ip, ip, vp, vp, ip]
    L.lbm_batch_get_macros.argtypes = [vp, ip, ip, vp, vp, ip]
    L.lbm_batch_get_populations.argtypes = [vp, ip, ip, vp, ip]
    L.lbm_batch_step.argtypes = [vp, ip, vp]
    L.lbm_batch_use_graph.argtypes = [vp, ip]
    L.lbm_batch_tune.argtypes = [vp, ip, i32p]
    L.lbm_batch_set_variants.argtypes = [vp, i32p]
    L.lbm_batch_info.argtypes = [vp, i64p]
    L.lbm_batch_slot_steps.argtypes = [vp, ip, i64p]
    L.lbm_footprint.argtypes = [ctypes.POINTER(lbm_grid_desc), i64p]
    L.lbm_copy_probe.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    L.lbm_batch_last_error.argtypes = [vp]
    L.lbm_batch_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc, h=None):
    if rc != LBM_OK:
        msg = load().lbm_last_error(h)
        raise LbmError(rc, msg.decode() if msg else "")


def _ptr(a):
    """Host numpy array or device torch tensor -> (pointer, mem)."""
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data), LBM_HOST
    if torch is not None and isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr()), (LBM_DEVICE if a.is_cuda else LBM_HOST)
    raise TypeError(type(a))


def lbm_lattice_info(lattice: int):
    D = ctypes.c_int32()
    Q = ctypes.c_int32()
    xi = (ctypes.c_int32 * 57)()
    w = (ctypes.c_double * 19)()
    _check(load().lbm_lattice_info(lattice, ctypes.byref(D), ctypes.byref(Q), xi, w))
    q = Q.value
    return D.value, q, np.array(xi[: 3 * q], np.int32).reshape(q, 3), np.array(w[:q])


def make_desc(lattice, collision, precision, n, lo=None, hi=None, tau_coarse=0.51, sigma=0.995, device=0):
    d = lbm_grid_desc()
    d.lattice, d.collision, d.precision = lattice, collision, precision
    D = 2 if lattice == LBM_D2Q9 else 3
    nn = list(n) + [1] * (3 - len(n))
    lo = list(lo if lo is not None else [0] * D) + [0] * (3 - D)
    hi = list(hi if hi is not None else [0] * D) + [0] * (3 - D)
    for k in range(3):
        d.n[k], d.lo[k], d.hi[k] = int(nn[k]), int(lo[k]), int(hi[k])
    d.tau_coarse, d.sigma, d.device, d.reserved = float(tau_coarse), float(sigma), int(device), 0
    return d


def lbm_copy_probe(bytes_, reps=10, device=0):
    """GB/s (read + written) of the library's streaming device copy."""
    v = ctypes.c_double()
    rc = load().lbm_copy_probe(int(device), int(bytes_), int(reps), ctypes.byref(v))
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return v.value


def lbm_footprint(desc):
    v = ctypes.c_int64()
    rc = load().lbm_footprint(ctypes.byref(desc), ctypes.byref(v))
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return v.value


def make_desc_(lattice, collision, precision, n, lo, hi, tau_coarse, sigma, device):
    d = lbm_grid_desc()
    d.lattice, d.collision, d.precision = lattice, collision, precision
    D = 2 if lattice == LBM_D2Q9 else 3
    nn = list(n) + [1] * (3 - len(n))
    lo = list(lo if lo is not None else [0] * D) + [0] * (3 - D)
    hi = list(hi if hi is not None else [0] * D) + [0] * (3 - D)
    for k in range(3):
        d.n[k], d.lo[k], d.hi[k] = int(nn[k]), int(lo[k]), int(hi[k])
    d.tau_coarse, d.sigma, d.device, d.reserved = float(tau_coarse), float(sigma), int(device), 0
    return d


def lbm_create_nested(lattice, collision, precision, n, lo, hi, lo2, hi2, tau_coarse=0.51, sigma=0.995, device=0):
    """Three nested levels: the patch [lo, hi] of coarse vertices carries the
    patch [lo2, hi2] of its own vertices (BGK, RR, H-RR)."""
    d = make_desc_(lattice, collision, precision, n, lo, hi, tau_coarse, sigma, device)
    D = 2 if lattice == LBM_D2Q9 else 3
    l2 = (ctypes.c_int32 * 3)(*[int(x) for x in (list(lo2)[:D] + [0] * (3 - D))])
    h2 = (ctypes.c_int32 * 3)(*[int(x) for x in (list(hi2)[:D] + [0] * (3 - D))])
    h = ctypes.c_void_p()
    rc = load().lbm_create_nested(ctypes.byref(d), l2, h2, ctypes.byref(h))
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return h


def lbm_create_grid(lattice, collision, precision, n, lo=None, hi=None, tau_coarse=0.51, sigma=0.995, device=0):
    d = lbm_grid_desc()
    d.lattice, d.collision, d.precision = lattice, collision, precision
    D = 2 if lattice == LBM_D2Q9 else 3
    nn = list(n) + [1] * (3 - len(n))
    lo = list(lo if lo is not None else [0] * D) + [0] * (3 - D)
    hi = list(hi if hi is not None else [0] * D) + [0] * (3 - D)
    for k in range(3):
        d.n[k], d.lo[k], d.hi[k] = int(nn[k]), int(lo[k]), int(hi[k])
    d.tau_coarse, d.sigma, d.device, d.reserved = float(tau_coarse), float(sigma), int(device), 0
    h = ctypes.c_void_p()
    rc = load().lbm_create_grid(ctypes.byref(d), ctypes.byref(h))
    if rc != LBM_OK:
        raise LbmError(rc, load().lbm_last_error(None).decode())
    return h


def lbm_destroy(h):
    _check(load().lbm_destroy(h))


def lbm_level_dims(h, level):
    d = (ctypes.c_int32 * 3)()
    _check(load().lbm_level_dims(h, level, d), h)
    return tuple(d)


def lbm_set_state(h, level, rho, u):
    pr, m1 = _ptr(rho)
    pu, m2 = _ptr(u)
    assert m1 == m2
    _check(load().lbm_set_state(h, level, pr, pu, m1), h)


def lbm_step(h, n, stream=None):
    _check(load().lbm_step(h, int(n), ctypes.c_void_p(stream) if stream else None), h)


def lbm_get_macros(h, level, rho, u):
    pr, m1 = _ptr(rho)
    pu, m2 = _ptr(u)
    assert m1 == m2
    _check(load().lbm_get_macros(h, level, pr, pu, m1), h)


def lbm_set_populations(h, level, f):
    p, m = _ptr(f)
    _check(load().lbm_set_populations(h, level, p, m), h)


def lbm_get_populations(h, level, f):
    p, m = _ptr(f)
    _check(load().lbm_get_populations(h, level, p, m), h)


def lbm_get_totals(h):
    mass = (ctypes.c_double * 2)()
    mom = (ctypes.c_double * 6)()
    _check(load().lbm_get_totals(h, mass, mom), h)
    return np.array(mass[:]), np.array(mom[:]).reshape(2, 3)


def lbm_get_totals_noalloc(h):
    mass = (ctypes.c_double * 2)()
    mom = (ctypes.c_double * 6)()
    _check(load().lbm_get_totals_noalloc(h, mass, mom), h)
    return np.array(mass[:]), np.array(mom[:]).reshape(2, 3)


def lbm_sensors_enable(h, on=True):
    _check(load().lbm_sensors_enable(h, 1 if on else 0), h)


def lbm_sensors(h, level, threshold, flags, diag=None):
    """NH-sensor flags of a level after the last step into `flags` (uint8 per
    node, host numpy array or device tensor); `diag` optionally receives
    [3][N] doubles (divergence product, curl product, ghost norm)."""
    p, m = _ptr(flags)
    dptr = None if diag is None else _ptr(diag)[0]
    _check(load().lbm_sensors(h, level, float(threshold), p, dptr, m), h)


def lbm_set_dynamic_sigma(h, on=True, sigma_dyn=0.0, threshold=0.0):
    """H-RR with sigma_dyn at nodes whose divergence or curl product (sensor
    tests between consecutive collisions) falls below -threshold."""
    _check(load().lbm_set_dynamic_sigma(h, 1 if on else 0, float(sigma_dyn), float(threshold)), h)


def lbm_probe_enable(h, level, node=(0, 0, 0), capacity=1):
    nd = (ctypes.c_int32 * 3)(*[int(x) for x in (list(node) + [0, 0, 0])[:3]])
    _check(load().lbm_probe_enable(h, int(level), nd, int(capacity)), h)


def lbm_probe_read(h, max_values):
    out = np.zeros(int(max_values))
    cnt = ctypes.c_int64()
    _check(load().lbm_probe_read(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(max_values),
                                 ctypes.byref(cnt)), h)
    return out[: min(cnt.value, int(max_values))], cnt.value


def lbm_get_index_maps(h, level, out):
    p, m = _ptr(out)
    _check(load().lbm_get_index_maps(h, level, p, m), h)


def lbm_interface_counts(h):
    c = (ctypes.c_int64 * 3)()
    _check(load().lbm_interface_counts(h, c), h)
    return tuple(c)


def lbm_interface_tables(h):
    nh, nr, _ = lbm_interface_counts(h)
    hn = np.zeros(nh, np.int64)
    rn = np.zeros(nr, np.int64)
    rnp = np.zeros(nr, np.int32)
    rpt = np.zeros((nr, 16), np.int64)
    _check(load().lbm_interface_tables(h, hn.ctypes.data, rn.ctypes.data, rnp.ctypes.data, rpt.ctypes.data), h)
    return hn, rn, rnp, rpt


def lbm_updates_per_step(h):
    v = ctypes.c_int64()
    _check(load().lbm_updates_per_step(h, ctypes.byref(v)), h)
    return v.value


def lbm_profile_enable(h, on=True):
    _check(load().lbm_profile_enable(h, 1 if on else 0), h)


def lbm_kernel_time(h):
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    nodes = ctypes.c_int64()
    _check(load().lbm_kernel_time(h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(nodes)), h)
    return n.value, ms.value, nodes.value


def lbm_tune(h, reps=5):
    v = (ctypes.c_int32 * 4)()
    _check(load().lbm_tune(h, int(reps), v), h)
    return list(v)


def lbm_set_variants(h, variants):
    v = (ctypes.c_int32 * 4)(*[int(x) for x in variants])
    _check(load().lbm_set_variants(h, v), h)


class Grid:
    """Convenience wrapper over one handle (host numpy arrays in and out)."""

    def __init__(self, lattice, collision, precision, n, lo=None, hi=None, tau_coarse=0.51, sigma=0.995, device=0):
        self.h = lbm_create_grid(lattice, collision, precision, n, lo, hi, tau_coarse, sigma, device)
        self.D, self.Q, self.xi, self.w = lbm_lattice_info(lattice)
        self.lattice, self.collision, self.precision = lattice, collision, precision
        D = self.D
        self.shape = (tuple(int(x) for x in list(n)[:D]), None if lo is None else tuple(int(x) for x in list(lo)[:D]),
                      None if hi is None else tuple(int(x) for x in list(hi)[:D]))
        self.device = device

    def close(self):
        if self.h:
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dims(self, level):
        return lbm_level_dims(self.h, level)

    def nodes(self, level):
        a, b, c = self.dims(level)
        return a * b * c

    def set_state(self, level, rho, u):
        N = self.nodes(level)
        lbm_set_state(self.h, level, np.ascontiguousarray(rho, np.float64).reshape(N),
                      np.ascontiguousarray(u, np.float64).reshape(self.D, N))

    def step(self, n=1, stream=None):
        lbm_step(self.h, n, stream)

    def get_macros(self, level):
        N = self.nodes(level)
        rho = np.zeros(N)
        u = np.zeros((self.D, N))
        lbm_get_macros(self.h, level, rho, u)
        return rho, u

    def set_populations(self, level, f):
        lbm_set_populations(self.h, level, np.ascontiguousarray(f, np.float64).reshape(self.Q, self.nodes(level)))

    def get_populations(self, level):
        f = np.zeros((self.Q, self.nodes(level)))
        lbm_get_populations(self.h, level, f)
        return f

    def totals(self):
        return lbm_get_totals(self.h)

    def sensors(self, level, threshold):
        """(flags[N] uint8, diag[3, N]) of the NH sensors after the last step
        (sensors must have been enabled before that step)."""
        N = self.nodes(level)
        flags = np.zeros(N, np.uint8)
        diag = np.zeros((3, N))
        lbm_sensors(self.h, level, threshold, flags, diag)
        return flags, diag

    def set_dynamic_sigma(self, on=True, sigma_dyn=0.0, threshold=0.0):
        lbm_set_dynamic_sigma(self.h, on, sigma_dyn, threshold)

    def class_map(self, level):
        out = np.zeros(self.nodes(level), np.uint8)
        lbm_get_index_maps(self.h, level, out)
        return out

    def updates_per_step(self):
        return lbm_updates_per_step(self.h)

    def tune(self, reps=5):
        return lbm_tune(self.h, reps)

    def set_variants(self, variants):
        lbm_set_variants(self.h, variants)


# ---------------------------------------------------------------------------
# Batches


def _bcheck(rc, b):
    if rc != LBM_OK:
        msg = load().lbm_batch_last_error(b)
        raise LbmError(rc, msg.decode() if msg else "")


class Batch:
    """Many grids of one lattice / collision model / precision, stepped
    together by one launch per phase, replayed from a hipGraph."""

    def __init__(self, lattice, collision, precision, capacity, device=0):
        self.b = ctypes.c_void_p()
        rc = load().lbm_batch_create(lattice, collision, precision, device, capacity, ctypes.byref(self.b))
        if rc != LBM_OK:
            raise LbmError(rc, load().lbm_batch_last_error(None).decode())
        self.D, self.Q, self.xi, self.w = lbm_lattice_info(lattice)
        self.lattice, self.collision, self.precision = lattice, collision, precision
        self.device = device
        self.dims = {}
        self.shapes = {}

    def close(self):
        if self.b:
            load().lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, n, lo=None, hi=None, tau_coarse=0.51, sigma=0.995):
        d = make_desc(self.lattice, self.collision, self.precision, n, lo, hi, tau_coarse, sigma)
        slot = ctypes.c_int32()
        _bcheck(load().lbm_batch_add(self.b, ctypes.byref(d), ctypes.byref(slot)), self.b)
        D = self.D
        nc = [int(x) for x in list(n)[:D]]
        nf = None
        if lo is not None and any(int(a) != int(b) for a, b in zip(lo, hi)):
            nf = [2 * (int(h) - int(l)) + 1 for l, h in zip(list(lo)[:D], list(hi)[:D])]
        self.dims[slot.value] = (nc, nf)
        self.shapes[slot.value] = (tuple(nc), None if lo is None else tuple(int(x) for x in list(lo)[:D]),
                                   None if hi is None else tuple(int(x) for x in list(hi)[:D]))
        return slot.value

    def remove(self, slot):
        _bcheck(load().lbm_batch_remove(self.b, slot), self.b)
        self.dims.pop(slot, None)
        self.shapes.pop(slot, None)

    def nodes(self, slot, level):
        nc, nf = self.dims[slot]
        return int(np.prod(nc if level == 0 else nf))

    def set_state(self, slot, level, rho, u):
        N = self.nodes(slot, level)
        rho = np.ascontiguousarray(rho, np.float64).reshape(N)
        u = np.ascontiguousarray(u, np.float64).reshape(self.D, N)
        _bcheck(load().lbm_batch_set_state(self.b, slot, level, rho.ctypes.data, u.ctypes.data, LBM_HOST), self.b)

    def get_macros(self, slot, level):
        N = self.nodes(slot, level)
        rho = np.zeros(N)
        u = np.zeros((self.D, N))
        _bcheck(load().lbm_batch_get_macros(self.b, slot, level, rho.ctypes.data, u.ctypes.data, LBM_HOST), self.b)
        return rho, u

    def get_populations(self, slot, level):
        f = np.zeros((self.Q, self.nodes(slot, level)))
        _bcheck(load().lbm_batch_get_populations(self.b, slot, level, f.ctypes.data, LBM_HOST), self.b)
        return f

    def step(self, n=1, stream=None):
        _bcheck(load().lbm_batch_step(self.b, int(n), ctypes.c_void_p(stream) if stream else None), self.b)

    def use_graph(self, on=True):
        _bcheck(load().lbm_batch_use_graph(self.b, 1 if on else 0), self.b)

    def tune(self, reps=3):
        v = (ctypes.c_int32 * 2)()
        _bcheck(load().lbm_batch_tune(self.b, int(reps), v), self.b)
        return list(v)

    def set_variants(self, variants):
        v = (ctypes.c_int32 * 2)(*[int(x) for x in variants])
        _bcheck(load().lbm_batch_set_variants(self.b, v), self.b)

    def info(self):
        v = (ctypes.c_int64 * 3)()
        _bcheck(load().lbm_batch_info(self.b, v), self.b)
        return {"grids": v[0], "updates_per_step": v[1], "bytes": v[2]}

    def slot_steps(self, slot):
        v = ctypes.c_int64()
        _bcheck(load().lbm_batch_slot_steps(self.b, slot, ctypes.byref(v)), self.b)
        return v.value


class Nested(Grid):
    """Three nested levels (levels 0, 1, 2) over one handle: the coarse
    periodic grid, its patch [lo, hi], and the patch [lo2, hi2] of level-1
    vertices.  BGK, RR and H-RR."""

    def __init__(self, lattice, collision, precision, n, lo, hi, lo2, hi2, tau_coarse=0.51, sigma=0.995, device=0):
        self.h = lbm_create_nested(lattice, collision, precision, n, lo, hi, lo2, hi2, tau_coarse, sigma, device)
        self.D, self.Q, self.xi, self.w = lbm_lattice_info(lattice)
        self.lattice, self.collision, self.precision = lattice, collision, precision
        D = self.D
        self.shape = (tuple(int(x) for x in list(n)[:D]), tuple(int(x) for x in list(lo)[:D]),
                      tuple(int(x) for x in list(hi)[:D]))
        self.device = device
