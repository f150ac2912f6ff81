"""Python binding of the MI355X three-site TEBD library (``libptebd.so``).

Argument marshalling only: every step of the evolution and of the
measurement runs in the library's HIP kernels.  The functions carry the
names of the C ABI in ``include/ptebd.h``.  Importing this package fails
loudly if the library has not been built (``python -m
paper_2401_05301_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptebd.so")

TEBD_OK, TEBD_EINVAL, TEBD_ENOMEM, TEBD_EDEVICE, TEBD_ENOCONV, TEBD_ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32, FP32_SPLIT = 0, 1, 2
SVD_JACOBI, SVD_GRAM_EIG, SVD_RANDOMIZED = 0, 1, 2
GRAM_EPS_MIN = 1e-6   # TEBD_GRAM_EPS_MIN: smallest trunc_rel the Gram route accepts

EXPORTS = [
    "tebd_opts_default", "mps_init_cdw", "mps_init_product", "mps_init_state", "tebd_layer", "tebd_step",
    "tebd_step4",
    "tebd_step_many", "measure_local", "mps_set_model", "mps_bond_dims", "mps_lambda", "mps_site",
    "mps_discarded_weight", "mps_sweep_stats", "mps_footprint", "mps_sync", "mps_free", "tebd_last_error",
    "tebd_prepare", "mps_profile", "mps_profile_read", "mps_canonicalize", "tebd_serve", "measure_quasi_local",
    "mps_bond_charges", "mps_trunc_stats", "mps_profile_busy", "mps_checkpoint", "mps_restore",
]
KERNEL_CLASSES = {"gemm_fp64": 0, "gemm_fp32": 1, "herm_eig": 2, "herm_apply": 3, "jac_gram": 4, "jac_rotate": 5}


class TebdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class Model(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("d", ctypes.c_int32), ("U", ctypes.c_double), ("J", ctypes.c_double),
                ("Jnnn", ctypes.c_double), ("K", ctypes.c_double), ("jc", ctypes.c_double)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Opts(ctypes.Structure):
    _fields_ = [("chi_max", ctypes.c_int32), ("trunc_weight", ctypes.c_double), ("trunc_rel", ctypes.c_double),
                ("prec", ctypes.c_int32), ("svd", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN),
                ("alloc_ctx", ctypes.c_void_p), ("workers", ctypes.c_int32), ("supersite", ctypes.c_int32),
                ("u1", ctypes.c_int32), ("fuse", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("model", Model), ("chi_max", ctypes.c_int32), ("dt", ctypes.c_double), ("steps", ctypes.c_int32),
                ("arrival", ctypes.c_double), ("first_occupied", ctypes.c_int32)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("hbm_budget", ctypes.c_double), ("prec", ctypes.c_int32),
                ("svd", ctypes.c_int32), ("trunc_weight", ctypes.c_double), ("trunc_rel", ctypes.c_double),
                ("workers_per_request", ctypes.c_int32), ("measure_every", ctypes.c_int32), ("u1", ctypes.c_int32),
                ("batched", ctypes.c_int32)]


class ServeResult(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("admitted", ctypes.c_double), ("finished", ctypes.c_double),
                ("discarded_weight", ctypes.c_double), ("gate_updates", ctypes.c_int64), ("status", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2401_05301_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    P = ctypes.POINTER
    st = ctypes.c_int
    sig = {
        "tebd_opts_default": (None, [P(Opts)]),
        "mps_init_cdw": (st, [P(Model), P(Opts), ctypes.c_int32, P(H)]),
        "mps_init_product": (st, [P(Model), P(Opts), P(ctypes.c_int32), P(H)]),
        "mps_init_state": (st, [P(Model), P(Opts), P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double), P(H)]),
        "tebd_layer": (st, [H, ctypes.c_int32, ctypes.c_double]),
        "tebd_step": (st, [H, ctypes.c_double]),
        "tebd_step4": (st, [H, ctypes.c_double]),
        "tebd_step_many": (st, [P(H), ctypes.c_int32, P(ctypes.c_double)]),
        "measure_local": (st, [H, P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_double)]),
        "mps_set_model": (st, [H, P(Model)]),
        "mps_bond_dims": (st, [H, P(ctypes.c_int32)]),
        "mps_lambda": (st, [H, ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32, P(ctypes.c_int32)]),
        "mps_bond_charges": (st, [H, ctypes.c_int32, P(ctypes.c_int32), ctypes.c_int32, P(ctypes.c_int32)]),
        "mps_site": (st, [H, ctypes.c_int32, P(ctypes.c_double), ctypes.c_int64]),
        "mps_discarded_weight": (st, [H, P(ctypes.c_double)]),
        "mps_checkpoint": (st, [H, ctypes.c_void_p, ctypes.c_size_t, P(ctypes.c_size_t)]),
        "mps_restore": (st, [P(Model), P(Opts), ctypes.c_void_p, ctypes.c_size_t, P(H)]),
        "mps_sweep_stats": (st, [H, P(ctypes.c_int64), P(ctypes.c_int64)]),
        "mps_trunc_stats": (st, [H, P(ctypes.c_int64)]),
        "mps_footprint": (st, [P(Model), P(Opts), P(ctypes.c_size_t)]),
        "mps_sync": (st, [H]),
        "mps_free": (st, [H]),
        "tebd_last_error": (ctypes.c_char_p, []),
        "tebd_prepare": (st, [H, ctypes.c_double]),
        "mps_canonicalize": (st, [H]),
        "mps_profile": (st, [H, ctypes.c_int32]),
        "mps_profile_read": (st, [H, ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int64), P(ctypes.c_double)]),
        "mps_profile_busy": (st, [H, ctypes.c_int32, P(ctypes.c_double)]),
        "tebd_serve": (st, [P(Request), ctypes.c_int32, P(ServeOpts), P(ServeResult), P(ctypes.c_double),
                            P(ctypes.c_double), P(ctypes.c_double)]),
        "measure_quasi_local": (st, [H, ctypes.c_int32, P(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def _check(status: int):
    if status != TEBD_OK:
        raise TebdError(status, _lib.tebd_last_error().decode())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_model(L: int, d: int, U: float, J: float = 1.0, Jnnn: float = 0.0, K: float = 0.0,
               jc: Optional[float] = None) -> Model:
    """Eq. (1) parameters; jc is the 1-based trap centre (default (L+1)/2)."""
    return Model(L, d, U, J, Jnnn, K, (L + 1) / 2.0 if jc is None else jc)


def make_opts(chi_max: int, w_max: float = 1e-12, eps: float = 1e-12, prec: int = FP64, svd: int = SVD_JACOBI,
              max_sweeps: int = 80, stream: Optional[int] = None, workers: int = 0, supersite: bool = False,
              u1: bool = False, fuse: bool = False) -> Opts:
    o = Opts()
    _lib.tebd_opts_default(ctypes.byref(o))
    o.chi_max, o.trunc_weight, o.trunc_rel = chi_max, w_max, eps
    o.prec, o.svd, o.max_sweeps = prec, svd, max_sweeps
    o.stream = stream
    o.workers = workers
    o.supersite = int(bool(supersite))
    o.u1 = int(bool(u1))
    o.fuse = int(bool(fuse))
    return o


def torch_allocator(opts: Opts, stream: Optional[int] = None):
    """Route the library's device allocations through torch's caching allocator.

    Returns the callback objects, which the caller must keep alive as long as
    any handle created with these options exists."""
    import torch

    def _alloc(nbytes, _ctx):
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream)

    def _free(ptr, _ctx):
        torch.cuda.caching_allocator_delete(ptr)

    keep = (ALLOC_FN(_alloc), FREE_FN(_free))
    opts.dev_alloc, opts.dev_free = keep
    return keep


def mps_init_cdw(model: Model, opts: Opts, first_occupied: int = 1):
    h = ctypes.c_void_p()
    _check(_lib.mps_init_cdw(ctypes.byref(model), ctypes.byref(opts), first_occupied, ctypes.byref(h)))
    return h


def mps_init_product(model: Model, opts: Opts, occ: Sequence[int]):
    a = np.ascontiguousarray(occ, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(_lib.mps_init_product(ctypes.byref(model), ctypes.byref(opts),
                                 a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(h)))
    return h


def mps_init_state(model: Model, opts: Opts, B: Sequence[np.ndarray], lam: Sequence[np.ndarray]):
    """State in stored form: B[i] complex (chi_i, d, chi_{i+1}), lam[b] real (chi_b)."""
    chi = np.array([1] + [b.shape[2] for b in B], dtype=np.int32)
    flat = []
    for b in B:
        b = np.ascontiguousarray(b, dtype=np.complex128)
        flat.append(b.real.ravel())
        flat.append(b.imag.ravel())
    Bf = np.ascontiguousarray(np.concatenate(flat), dtype=np.float64)
    Lf = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64) for x in lam]))
    h = ctypes.c_void_p()
    _check(_lib.mps_init_state(ctypes.byref(model), ctypes.byref(opts),
                               chi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(Bf), _dptr(Lf),
                               ctypes.byref(h)))
    return h


def tebd_layer(h, group: int, tau: float):
    _check(_lib.tebd_layer(h, group, tau))


def tebd_step(h, dt: float):
    _check(_lib.tebd_step(h, dt))


def tebd_step4(h, dt: float):
    _check(_lib.tebd_step4(h, dt))


def tebd_step_many(handles, dts):
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[x.value if isinstance(x, ctypes.c_void_p) else x for x in handles])
    d = np.ascontiguousarray(dts, dtype=np.float64)
    _check(_lib.tebd_step_many(arr, n, _dptr(d)))


def measure_local(h, L: int):
    """Returns (n[L], C[L-1] complex, D[L-2] complex)."""
    n = np.zeros(L)
    c = np.zeros(2 * max(L - 1, 1))
    dd = np.zeros(2 * max(L - 2, 1))
    _check(_lib.measure_local(h, _dptr(n), _dptr(c), _dptr(dd)))
    C = c[0:2 * (L - 1):2] + 1j * c[1:2 * (L - 1):2]
    D = dd[0:2 * (L - 2):2] + 1j * dd[1:2 * (L - 2):2]
    return n, C, D


def measure_quasi_local(h, centre: int):
    """Quasi-local observables (see ptebd.h) as a dict."""
    out = np.zeros(8)
    _check(_lib.measure_quasi_local(h, int(centre), _dptr(out)))
    return dict(N=out[0], n_odd=out[1], n_even=out[2], C_even=complex(out[3], out[4]), A=out[5], phi=out[6],
                nu=out[7])


def mps_set_model(h, model: Model):
    _check(_lib.mps_set_model(h, ctypes.byref(model)))


def mps_bond_dims(h, L: int):
    a = np.zeros(L + 1, dtype=np.int32)
    _check(_lib.mps_bond_dims(h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return [int(x) for x in a]


def mps_lambda(h, bond: int, cap: int = 16384):
    s = np.zeros(cap)
    n = ctypes.c_int32()
    _check(_lib.mps_lambda(h, bond, _dptr(s), cap, ctypes.byref(n)))
    return s[:n.value].copy()


def mps_bond_charges(h, bond: int, cap: int = 16384):
    q = np.zeros(cap, dtype=np.int32)
    n = ctypes.c_int32()
    _check(_lib.mps_bond_charges(h, bond, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap, ctypes.byref(n)))
    return q[:n.value].astype(np.int64)


def mps_site(h, site: int, shape):
    cl, d, cr = shape
    n = cl * d * cr
    buf = np.zeros(2 * n)
    _check(_lib.mps_site(h, site, _dptr(buf), 2 * n))
    return (buf[:n] + 1j * buf[n:]).reshape(cl, d, cr)


def mps_discarded_weight(h) -> float:
    w = ctypes.c_double()
    _check(_lib.mps_discarded_weight(h, ctypes.byref(w)))
    return w.value


def mps_checkpoint(h) -> np.ndarray:
    """Checkpoint image of the handle's state and ledger (uint8 array)."""
    n = ctypes.c_size_t()
    _check(_lib.mps_checkpoint(h, None, 0, ctypes.byref(n)))
    buf = np.empty(n.value, dtype=np.uint8)
    _check(_lib.mps_checkpoint(h, buf.ctypes.data, buf.nbytes, ctypes.byref(n)))
    return buf


def mps_restore(model: Model, opts: Opts, image) -> ctypes.c_void_p:
    """New handle from a checkpoint image (bytes-like or uint8 array)."""
    buf = np.ascontiguousarray(np.frombuffer(image, dtype=np.uint8))
    h = ctypes.c_void_p()
    _check(_lib.mps_restore(ctypes.byref(model), ctypes.byref(opts), buf.ctypes.data, buf.nbytes,
                            ctypes.byref(h)))
    return h


def mps_sweep_stats(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.mps_sweep_stats(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def mps_trunc_stats(h):
    """Truncations so far by the part of the rule that set k:
    {"chi_max": .., "w_max": .., "eps": .., "none": ..}."""
    a = (ctypes.c_int64 * 4)()
    _check(_lib.mps_trunc_stats(h, a))
    return {"chi_max": a[0], "w_max": a[1], "eps": a[2], "none": a[3]}


def mps_footprint(model: Model, opts: Opts) -> int:
    b = ctypes.c_size_t()
    _check(_lib.mps_footprint(ctypes.byref(model), ctypes.byref(opts), ctypes.byref(b)))
    return b.value


def tebd_prepare(h, dt: float):
    _check(_lib.tebd_prepare(h, dt))


def mps_canonicalize(h):
    _check(_lib.mps_canonicalize(h))


def mps_profile(h, enable: bool):
    _check(_lib.mps_profile(h, 1 if enable else 0))


def mps_profile_read(h, kclass: int):
    """(device ms, launches, algorithmic flops) of one kernel class."""
    ms, n, fl = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    _check(_lib.mps_profile_read(h, kclass, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(fl)))
    return ms.value, n.value, fl.value


def mps_profile_busy(h, kclass: int) -> float:
    """Wall ms during which at least one launch of the class ran."""
    b = ctypes.c_double()
    _check(_lib.mps_profile_busy(h, kclass, ctypes.byref(b)))
    return b.value


def mps_sync(h):
    _check(_lib.mps_sync(h))


def mps_free(h):
    _check(_lib.mps_free(h))


def tebd_serve(requests, max_active: int = 8, hbm_budget: float = 0.0, prec: int = FP64, svd: int = SVD_JACOBI,
               w_max: float = 1e-12, eps: float = 1e-12, workers_per_request: int = 1, measure_every: int = 0,
               u1: bool = False, batched: bool = False):
    """Serve quench requests concurrently (see tebd_serve in ptebd.h).

    ``requests`` are dicts with keys model (a Model), chi_max, dt, steps,
    arrival (s) and optionally first_occupied.  ``batched`` serves them by
    continuous batching (Jacobi route, dense tensors).  Returns one dict per
    request with arrival/admitted/finished times, discarded weight, gate
    updates, status and the observables n, c_nn, c_nnn at the horizon."""
    n = len(requests)
    req = (Request * n)()
    for i, r in enumerate(requests):
        req[i] = Request(r["model"], int(r["chi_max"]), float(r["dt"]), int(r["steps"]), float(r["arrival"]),
                         int(r.get("first_occupied", 1)))
    so = ServeOpts(max_active, hbm_budget, prec, svd, w_max, eps, workers_per_request, measure_every, int(bool(u1)),
                   int(bool(batched)))
    res = (ServeResult * n)()
    Ls = [r["model"].L for r in requests]
    nn = np.zeros(sum(Ls))
    cn = np.zeros(sum(2 * (L - 1) for L in Ls))
    dn = np.zeros(sum(2 * (L - 2) for L in Ls))
    st = _lib.tebd_serve(req, n, ctypes.byref(so), res, _dptr(nn), _dptr(cn), _dptr(dn))
    out = []
    o_n = o_c = o_d = 0
    for i, L in enumerate(Ls):
        c = cn[o_c:o_c + 2 * (L - 1)]
        d = dn[o_d:o_d + 2 * (L - 2)]
        out.append(dict(arrival=res[i].arrival, admitted=res[i].admitted, finished=res[i].finished,
                        discarded_weight=res[i].discarded_weight, gate_updates=res[i].gate_updates,
                        status=res[i].status, n=nn[o_n:o_n + L].copy(), c_nn=c[0::2] + 1j * c[1::2],
                        c_nnn=d[0::2] + 1j * d[1::2]))
        o_n, o_c, o_d = o_n + L, o_c + 2 * (L - 1), o_d + 2 * (L - 2)
    if st not in (TEBD_OK,) and all(r["status"] == TEBD_OK for r in out):
        _check(st)
    return out


class MPS:
    """Owning wrapper of a handle (frees it on close / garbage collection)."""

    def __init__(self, handle, model: Model, keep=None, supersite: bool = False):
        self.h = handle
        self.model = model
        self.L = model.L                  # physical sites (observables)
        self.supersite = bool(supersite)
        # sites and local dimension of the chain the MPS lives on
        self.sites = model.L // 2 if supersite else model.L
        self.d = model.d * model.d if supersite else model.d
        self._keep = keep

    @classmethod
    def cdw(cls, model: Model, opts: Opts, first_occupied: int = 1):
        return cls(mps_init_cdw(model, opts, first_occupied), model, supersite=opts.supersite)

    @classmethod
    def from_tensors(cls, model: Model, opts: Opts, B, lam):
        return cls(mps_init_state(model, opts, B, lam), model, supersite=opts.supersite)

    def layer(self, group: int, tau: float):
        tebd_layer(self.h, group, tau)

    def step(self, dt: float):
        tebd_step(self.h, dt)

    def step4(self, dt: float):
        tebd_step4(self.h, dt)

    def measure(self):
        return measure_local(self.h, self.L)

    def quasi_local(self, centre: int):
        return measure_quasi_local(self.h, centre)

    @classmethod
    def product(cls, model: Model, opts: Opts, occ):
        return cls(mps_init_product(model, opts, occ), model, supersite=opts.supersite)

    def bond_dims(self):
        return mps_bond_dims(self.h, self.sites)

    def lam(self, bond: int):
        return mps_lambda(self.h, bond)

    def charges(self, bond: int):
        return mps_bond_charges(self.h, bond)

    def site(self, i: int):
        chi = self.bond_dims()
        return mps_site(self.h, i, (chi[i], self.d, chi[i + 1]))

    def discarded_weight(self):
        return mps_discarded_weight(self.h)

    def checkpoint(self) -> np.ndarray:
        return mps_checkpoint(self.h)

    @classmethod
    def restore(cls, model: Model, opts: Opts, image):
        return cls(mps_restore(model, opts, image), model, supersite=opts.supersite)

    def save(self, path: str):
        """Write the checkpoint image to a file."""
        self.checkpoint().tofile(path)

    @classmethod
    def load(cls, path: str, model: Model, opts: Opts):
        """Handle from a checkpoint file written by save()."""
        return cls.restore(model, opts, np.fromfile(path, dtype=np.uint8))

    def sweeps(self):
        return mps_sweep_stats(self.h)

    def trunc_stats(self):
        return mps_trunc_stats(self.h)

    def sync(self):
        mps_sync(self.h)

    def canonicalize(self):
        mps_canonicalize(self.h)

    def prepare(self, dt: float):
        tebd_prepare(self.h, dt)

    def profile(self, enable: bool = True):
        mps_profile(self.h, enable)

    def profile_read(self):
        return {name: mps_profile_read(self.h, k) for name, k in KERNEL_CLASSES.items()}

    def profile_sites(self):
        return tebd_diag_profile_sites(self.h)

    def tile_tuner(self):
        return tebd_diag_tile_tuner()

    def profile_busy(self):
        return {name: mps_profile_busy(self.h, k) for name, k in KERNEL_CLASSES.items()}

    def close(self):
        if self.h is not None and self.h.value:
            mps_free(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ diagnostics
def _load_diag():
    P = ctypes.POINTER
    _lib.tebd_diag_zgemm.restype = ctypes.c_int
    _lib.tebd_diag_zgemm.argtypes = [ctypes.c_int32] * 6 + [P(ctypes.c_double)] * 5 + [ctypes.c_int32, P(ctypes.c_double)]
    for name in ("tebd_diag_svd", "tebd_diag_svd_noalloc"):
        f = getattr(_lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double), ctypes.c_int32,
                      ctypes.c_double, ctypes.c_double, P(ctypes.c_int32), P(ctypes.c_double), P(ctypes.c_double),
                      P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int32)]
    _lib.tebd_diag_profile_sites.restype = ctypes.c_int
    _lib.tebd_diag_profile_sites.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64]
    _lib.tebd_diag_tile_tuner.restype = ctypes.c_int
    _lib.tebd_diag_tile_tuner.argtypes = [P(ctypes.c_int64)]
    _lib.tebd_diag_zgemm_time.restype = ctypes.c_int
    _lib.tebd_diag_zgemm_time.argtypes = [ctypes.c_int32] * 5 + [P(ctypes.c_double)]
    _lib.tebd_diag_gate.restype = ctypes.c_int
    _lib.tebd_diag_gate.argtypes = [P(Model), ctypes.c_int32, ctypes.c_int32, ctypes.c_double, P(ctypes.c_double)]
    _lib.tebd_diag_bond_charges.restype = ctypes.c_int
    _lib.tebd_diag_bond_charges.argtypes = [ctypes.c_int32, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_double),
                                            P(ctypes.c_int32)]


_load_diag()
EXPORTS += ["tebd_diag_zgemm", "tebd_diag_svd", "tebd_diag_svd_noalloc", "tebd_diag_zgemm_time", "tebd_diag_gate",
            "tebd_diag_bond_charges", "tebd_diag_profile_sites", "tebd_diag_tile_tuner"]


def tebd_diag_tile_tuner() -> dict:
    """The process-wide theta/gate tile tuner: shapes timed and later launches per tile."""
    c = (ctypes.c_int64 * 3)()
    _check(_lib.tebd_diag_tile_tuner(c))
    return {"shapes_tuned": int(c[0]), "launches_64": int(c[1]), "launches_128": int(c[2])}


def tebd_diag_profile_sites(h) -> dict:
    """Per-call-site GEMM totals since profiling was enabled:
    {site: (launches, device ms, algorithmic flops)}."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(_lib.tebd_diag_profile_sites(h, buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms, fl = line.split()
        out[name] = (int(n), float(ms), float(fl))
    return out


def tebd_diag_gate(model: Model, j: int, tau: float, supersite: bool = False) -> np.ndarray:
    """The library's host-built gate exp(-i h tau) of window j (super sites
    (j, j+1) with supersite=True) as a complex n x n array."""
    n = model.d ** (4 if supersite else 3)
    g = np.zeros(2 * n * n)
    _check(_lib.tebd_diag_gate(ctypes.byref(model), int(bool(supersite)), j, tau, _dptr(g)))
    return (g[:n * n] + 1j * g[n * n:]).reshape(n, n)


def tebd_diag_bond_charges(B: Sequence[np.ndarray]):
    """Particle numbers of every bond index as the library infers them from
    the tensors B[i] (chi_i, d, chi_{i+1}) of a three-site chain."""
    L, d = len(B), B[0].shape[1]
    chi = np.array([1] + [b.shape[2] for b in B], dtype=np.int32)
    flat = []
    for b in B:
        b = np.ascontiguousarray(b, dtype=np.complex128)
        flat.append(b.real.ravel())
        flat.append(b.imag.ravel())
    Bf = np.ascontiguousarray(np.concatenate(flat), dtype=np.float64)
    q = np.zeros(int(chi.sum()), dtype=np.int32)
    _check(_lib.tebd_diag_bond_charges(L, d, chi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(Bf),
                                       q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return np.split(q.astype(np.int64), np.cumsum(chi)[:-1])


def tebd_diag_zgemm_time(m: int, n: int, k: int, prec: int = FP64, reps: int = 5) -> float:
    """Average device milliseconds of one m x n x k complex GEMM launch."""
    ms = ctypes.c_double()
    _check(_lib.tebd_diag_zgemm_time(prec, m, n, k, reps, ctypes.byref(ms)))
    return ms.value


def _planar(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.complex128)
    return np.ascontiguousarray(np.concatenate([a.real.ravel(), a.imag.ravel()]))


def _opt(a):
    if a is None:
        return None
    return _dptr(np.ascontiguousarray(a, dtype=np.float64))


def tebd_diag_zgemm(A: np.ndarray, B: np.ndarray, transA: int = 0, transB: int = 0, prec: int = FP64,
                    k_scale=None, row_scale=None, col_scale=None, herm: bool = False) -> np.ndarray:
    """op(A) diag(k_scale) op(B) scaled by row/col vectors, computed on the GPU.
    A and B are given in their stored shapes.  herm declares the product
    Hermitian (lower tiles computed and mirrored)."""
    m, k = (A.shape if not transA else A.shape[::-1])
    n = B.shape[1] if not transB else B.shape[0]
    pa, pb = _planar(A), _planar(B)
    keep = [None if x is None else np.ascontiguousarray(x, dtype=np.float64) for x in (k_scale, row_scale, col_scale)]
    c = np.zeros(2 * m * n)
    _check(_lib.tebd_diag_zgemm(prec, m, n, k, transA, transB, _dptr(pa), _dptr(pb),
                                *[None if x is None else _dptr(x) for x in keep], int(bool(herm)), _dptr(c)))
    return (c[:m * n] + 1j * c[m * n:]).reshape(m, n)


def tebd_diag_svd(A: np.ndarray, variant: int = SVD_JACOBI, chi_max: int = 1 << 30, w_max: float = 0.0,
                  eps: float = 0.0, noalloc: bool = False):
    """Truncated SVD on the GPU: returns (s_normalised, vh, nrm, w, sweeps).
    noalloc selects tebd_diag_svd_noalloc (no device allocation; m, n <= 512,
    m * n <= 65536)."""
    m, n = A.shape
    r = min(m, n)
    pa = _planar(A)
    s = np.zeros(r)
    vh = np.zeros(2 * r * n)
    k = ctypes.c_int32()
    nrm, w = ctypes.c_double(), ctypes.c_double()
    sw = ctypes.c_int32()
    fn = _lib.tebd_diag_svd_noalloc if noalloc else _lib.tebd_diag_svd
    _check(fn(variant, m, n, _dptr(pa), min(chi_max, 2 ** 31 - 1), w_max, eps, ctypes.byref(k),
              _dptr(s), _dptr(vh), ctypes.byref(nrm), ctypes.byref(w), ctypes.byref(sw)))
    kk = k.value
    V = (vh[:kk * n] + 1j * vh[kk * n:2 * kk * n]).reshape(kk, n)
    return s[:kk].copy(), V, nrm.value, w.value, sw.value
