"""Python binding of the 2d U(1) workload of libwdmg (argument marshalling only).

Every operation runs in the HIP library (``include/wdmg_2d.h``); this module
turns torch tensors into device pointers, fills the C parameter structs and
raises on error codes.  Device memory comes from torch's caching allocator and
the kernels run on the torch stream current at context creation.  There is no
CPU fallback: without ``libwdmg.so`` every entry point raises.
"""
from __future__ import annotations

import ctypes

import torch

from . import wdmg

MAX_LEVELS = 3
METHODS = {"mg-bicgstab": 0, "mg-cg": 1, "cg": 2}


class MgParams2d(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("block", ctypes.c_int * 2), ("nv", ctypes.c_int * (MAX_LEVELS - 1)),
                ("setup_iters", ctypes.c_int), ("vectors", ctypes.c_void_p * (MAX_LEVELS - 1)),
                ("normal", ctypes.c_int), ("omega", ctypes.c_double), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("use_alpha", ctypes.c_int), ("coarse_cycles", ctypes.c_int),
                ("blocking", ctypes.c_int)]


class Stats2d(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("true_res", ctypes.c_double),
                ("wilson", ctypes.c_longlong), ("coarse_applies", ctypes.c_longlong * MAX_LEVELS),
                ("flops", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "converged": bool(self.converged), "true_res": self.true_res,
                "wilson": self.wilson, "coarse_applies": list(self.coarse_applies), "flops": self.flops,
                "seconds": self.seconds}


_SIGS_DONE = False


def load() -> ctypes.CDLL:
    global _SIGS_DONE
    lib = wdmg.load()
    if _SIGS_DONE:
        return lib
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "wdmg_2d_create": (ip, [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(wdmg.AllocStruct),
                                vp]),
        "wdmg_2d_destroy": (None, [vp]),
        "wdmg_2d_last_error": (ctypes.c_char_p, [vp]),
        "wdmg_2d_set_gauge": (ip, [vp, vp, ip]),
        "wdmg_2d_set_mass": (ip, [vp, dp]),
        "wdmg_2d_apply_D": (ip, [vp, vp, vp, ip, ip]),
        "wdmg_2d_mg_setup": (ip, [vp, ctypes.POINTER(MgParams2d)]),
        "wdmg_2d_get_prolongator": (ip, [vp, ip, vp]),
        "wdmg_2d_apply_coarse": (ip, [vp, ip, vp, vp, ip]),
        "wdmg_2d_restrict": (ip, [vp, ip, vp, vp, ip]),
        "wdmg_2d_prolong": (ip, [vp, ip, vp, vp, ip]),
        "wdmg_2d_get_coarse_operator": (ip, [vp, ip, vp]),
        "wdmg_2d_vcycle": (ip, [vp, vp, vp]),
        "wdmg_2d_solve": (ip, [vp, vp, vp, ip, dp, ip, ctypes.POINTER(Stats2d)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _SIGS_DONE = True
    return lib


def _c128(t: torch.Tensor, what: str) -> int:
    return wdmg._ptr(t, torch.complex128, what)


class Context2d:
    """One Lx x Lt lattice, its U(1) links, mass and multigrid hierarchy."""

    def __init__(self, dims, device: str | int = "cuda:0"):
        self.lib = load()
        self.lx, self.lt = (int(d) for d in dims)
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        dev_index = self.device.index if self.device.index is not None else 0
        _alloc, _free = wdmg._torch_allocator(torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete,
                                              dev_index, self.stream)
        self._alloc_cb = wdmg._ALLOC_FN(_alloc)
        self._free_cb = wdmg._FREE_FN(_free)
        self._alloc = wdmg.AllocStruct(self._alloc_cb, self._free_cb, None)
        h = ctypes.c_void_p()
        d = (ctypes.c_int * 2)(self.lx, self.lt)
        rc = self.lib.wdmg_2d_create(ctypes.byref(h), d, ctypes.byref(self._alloc),
                                     ctypes.c_void_p(self.stream.cuda_stream))
        if rc != wdmg.WDMG_OK:
            raise wdmg.WdmgError(rc, "wdmg_2d_create failed")
        self.h = h
        self.levels = []  # (lt, lx, g, n) per level after setup
        self.normal = False

    def _check(self, rc: int, allow_not_converged: bool = False) -> int:
        if rc == wdmg.WDMG_OK or (allow_not_converged and rc == wdmg.WDMG_NOT_CONVERGED):
            return rc
        msg = self.lib.wdmg_2d_last_error(self.h)
        raise wdmg.WdmgError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.wdmg_2d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fine_shape(self):
        return (self.lt, self.lx, 2)

    def level_shape(self, level):
        lt, lx, g, n = self.levels[level]
        return (lt, lx, g, n)

    def set_gauge(self, U: torch.Tensor, t_bc: int = -1):
        if tuple(U.shape) != (self.lt, self.lx, 2):
            raise ValueError(f"link field shape {tuple(U.shape)} != {(self.lt, self.lx, 2)}")
        self._check(self.lib.wdmg_2d_set_gauge(self.h, _c128(U, "U"), int(t_bc)))
        self.levels = []

    def set_mass(self, m: float):
        self._check(self.lib.wdmg_2d_set_mass(self.h, float(m)))
        self.levels = []

    def apply_D(self, psi: torch.Tensor, dagger: bool = False):
        nrhs = 1 if psi.dim() == 3 else int(psi.shape[0])
        if tuple(psi.shape[-3:]) != self.fine_shape():
            raise ValueError("fine field shape mismatch")
        out = torch.empty_like(psi)
        self._check(self.lib.wdmg_2d_apply_D(self.h, _c128(out, "out"), _c128(psi, "in"), nrhs, 1 if dagger else 0))
        return out

    def mg_setup(self, nvs, vectors, *, block=(4, 4), setup_iters=100, normal=False, omega=0.8, nu_pre=2,
                 nu_post=2, use_alpha=True, coarse_cycles=1, blocking=0):
        """``nvs[l]`` candidates per coarsening, ``vectors[l]`` their complex128
        device starting vectors ``[nv, Tl, Xl, 2, n_l]`` (the fine level as
        ``[nv, T, X, 2, 1]`` in every case); ``blocking`` 1 or 2 selects the
        spin-blocked control (two levels of D)."""
        p = MgParams2d()
        p.n_levels = len(nvs) + 1
        p.block = (ctypes.c_int * 2)(*[int(b) for b in block])
        g = 1 if blocking else 2
        levels = [(self.lt, self.lx, g, 2 // g)]
        for i, (nv, v) in enumerate(zip(nvs, vectors)):
            lt, lx, _, n = levels[-1]
            want = (nv, lt, lx, 2, 1) if i == 0 else (nv, lt, lx, g, n)
            if tuple(v.shape) != want:
                raise ValueError(f"level {i} vectors: shape {tuple(v.shape)} != {want}")
            p.nv[i] = int(nv)
            p.vectors[i] = _c128(v, f"level {i} vectors")
            levels.append((lt // block[1], lx // block[0], g, int(nv)))
        p.setup_iters = int(setup_iters)
        p.normal = 1 if normal else 0
        p.omega, p.nu_pre, p.nu_post = float(omega), int(nu_pre), int(nu_post)
        p.use_alpha = 1 if use_alpha else 0
        p.coarse_cycles = int(coarse_cycles)
        p.blocking = int(blocking)
        self._check(self.lib.wdmg_2d_mg_setup(self.h, ctypes.byref(p)))
        self.levels = levels
        self.normal = bool(normal)

    def get_prolongator(self, level: int):
        lt, lx, g, n = self.levels[level]
        nv = self.levels[level + 1][3]
        out = torch.empty((nv, lt, lx, g, n), dtype=torch.complex128, device=self.device)
        self._check(self.lib.wdmg_2d_get_prolongator(self.h, int(level), out.data_ptr()))
        return out

    def get_coarse_operator(self, level: int):
        lt, lx, g, n = self.levels[level]
        S = 9 if self.normal else 5
        out = torch.empty((S, lt, lx, g * n, g * n), dtype=torch.complex128, device=self.device)
        self._check(self.lib.wdmg_2d_get_coarse_operator(self.h, int(level), out.data_ptr()))
        return out

    def _nrhs(self, t, level):
        base = 3 if level == 0 else 4
        return 1 if t.dim() == base else int(t.shape[0])

    def apply_coarse(self, level: int, c: torch.Tensor):
        out = torch.empty_like(c)
        self._check(self.lib.wdmg_2d_apply_coarse(self.h, int(level), _c128(out, "out"), _c128(c, "in"),
                                                  self._nrhs(c, level)))
        return out

    def restrict(self, level: int, f: torch.Tensor):
        nrhs = self._nrhs(f, level)
        shp = self.level_shape(level + 1)
        out = torch.empty(((nrhs,) if f.dim() > (3 if level == 0 else 4) else ()) + shp,
                          dtype=torch.complex128, device=self.device)
        self._check(self.lib.wdmg_2d_restrict(self.h, int(level), _c128(out, "out"), _c128(f, "in"), nrhs))
        return out

    def prolong(self, level: int, c: torch.Tensor):
        nrhs = self._nrhs(c, level + 1)
        shp = self.fine_shape() if level == 0 else self.level_shape(level)
        out = torch.empty(((nrhs,) if c.dim() > 4 else ()) + shp, dtype=torch.complex128, device=self.device)
        self._check(self.lib.wdmg_2d_prolong(self.h, int(level), _c128(out, "out"), _c128(c, "in"), nrhs))
        return out

    def vcycle(self, r: torch.Tensor):
        x = torch.empty_like(r)
        self._check(self.lib.wdmg_2d_vcycle(self.h, _c128(x, "x"), _c128(r, "r")))
        return x

    def solve(self, b: torch.Tensor, method: str = "mg-bicgstab", tol: float = 1e-10, maxit: int = 10000):
        """Returns ``(x, stats)``; ``method``: "mg-bicgstab", "mg-cg" or "cg"."""
        if tuple(b.shape) != self.fine_shape():
            raise ValueError("one fine field expected")
        x = torch.empty_like(b)
        st = Stats2d()
        self._check(self.lib.wdmg_2d_solve(self.h, _c128(x, "x"), _c128(b, "b"), METHODS[method], float(tol),
                                           int(maxit), ctypes.byref(st)), allow_not_converged=True)
        return x, st.as_dict()
