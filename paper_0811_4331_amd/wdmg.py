"""Python binding of libwdmg (argument marshalling only).

Every operation runs in the HIP library; this module converts torch tensors
to device pointers, fills the C parameter structs and turns return codes into
exceptions.  PyTorch provides the device memory (the library allocates
through torch's caching allocator) and the stream (the current stream at
context creation).

There is no fallback: if ``libwdmg.so`` is missing or cannot be loaded, every
entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import re
import sys
from typing import Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwdmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "wdmg.h")

WDMG_OK = 0
WDMG_NOT_CONVERGED = 1
ERRORS = {-1: "WDMG_ERR_ARG", -2: "WDMG_ERR_DIMS", -3: "WDMG_ERR_OOM", -4: "WDMG_ERR_HIP",
          -5: "WDMG_ERR_NOT_SETUP", -6: "WDMG_ERR_NAN", -7: "WDMG_ERR_RANK_DEFICIENT"}
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
KERNELS = ["dslash_f64", "dslash_f32", "dc_f64", "dc_f32", "restrict_f64", "restrict_f32",
           "prolong_f64", "prolong_f32", "dc_build", "block_qr", "dc_mfma_f64", "dc_mfma_f32",
           "dslash_f16", "dslash_bf16", "restrict_h", "prolong_h", "dc_h", "dc_mfma_h", "coarse_gcr"]
MAX_LEVELS = 4


class WdmgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class LevelParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int * 4), ("nv", ctypes.c_int), ("setup_iters", ctypes.c_int),
                ("vectors", ctypes.c_void_p), ("setup_prec", ctypes.c_int), ("adapt_iters", ctypes.c_int)]


class MgParams(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int), ("level", LevelParams * (MAX_LEVELS - 1)),
                ("omega", ctypes.c_double), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("coarse_cycles", ctypes.c_int), ("coarse_tol", ctypes.c_double),
                ("coarse_maxit", ctypes.c_int), ("coarse_restart", ctypes.c_int),
                ("use_alpha", ctypes.c_int), ("normal", ctypes.c_int)]


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("precond", ctypes.c_int), ("mg_prec", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("outer", ctypes.c_int), ("in_place", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("true_res", ctypes.c_double), ("n_D", ctypes.c_longlong),
                ("n_Dc", ctypes.c_longlong * MAX_LEVELS), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {"iters": self.iters, "restarts": self.restarts, "converged": bool(self.converged),
                "true_res": self.true_res, "n_D": self.n_D, "n_Dc": list(self.n_Dc),
                "seconds": self.seconds}


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class AllocStruct(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


def _torch_allocator(alloc_fn, delete_fn, dev_index, stream):
    """The library's device-memory callbacks on torch's caching allocator.

    An exception must not leave a ctypes callback: ctypes would print it and
    hand the library an undefined pointer.  A failed allocation returns None
    (NULL), which the library reports as WDMG_ERR_OOM; a failed release is
    reported on stderr and otherwise ignored."""
    def _alloc(nbytes, _user):
        try:
            return alloc_fn(int(nbytes), dev_index, stream)
        except Exception:  # out of memory, or any allocator error
            return None

    def _free(ptr, _user):
        try:
            delete_fn(ptr)
        except Exception as e:  # never unwind into the library
            print(f"wdmg: releasing device memory at {ptr:#x} failed: {e}", file=sys.stderr)

    return _alloc, _free


_LIB = None


HEADERS = [HEADER, os.path.join(os.path.dirname(HERE), "include", "wdmg_2d.h")]


def header_symbols() -> list[str]:
    """Entry points declared in include/wdmg.h and include/wdmg_2d.h."""
    text = ""
    for path in HEADERS:
        with open(path) as fh:
            text += fh.read()
    return sorted(set(re.findall(r"\b(wdmg_[a-z_A-Z0-9]+)\s*\(", text)))


def load() -> ctypes.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0811_4331_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    sig = {
        "wdmg_create": (ip, [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(AllocStruct), vp]),
        "wdmg_destroy": (None, [vp]),
        "wdmg_last_error": (ctypes.c_char_p, [vp]),
        "wdmg_default_mg_params": (None, [ctypes.POINTER(MgParams)]),
        "wdmg_default_solve_params": (None, [ctypes.POINTER(SolveParams)]),
        "wdmg_set_gauge": (ip, [vp, vp, ip]),
        "wdmg_set_mass": (ip, [vp, dp]),
        "wdmg_apply_D": (ip, [vp, vp, vp, ip, ip]),
        "wdmg_apply_D_noalloc": (ip, [vp, vp, vp, ip, ip]),
        "wdmg_roundtrip": (ip, [vp, vp, vp, ip, ip]),
        "wdmg_mg_setup": (ip, [vp, ctypes.POINTER(MgParams)]),
        "wdmg_get_prolongator": (ip, [vp, ip, vp]),
        "wdmg_release_unused": (ip, [vp, ip]),
        "wdmg_apply_Dc": (ip, [vp, ip, vp, vp, ip, ip]),
        "wdmg_apply_Nc": (ip, [vp, ip, vp, vp, ip]),
        "wdmg_restrict": (ip, [vp, ip, vp, vp, ip, ip]),
        "wdmg_prolong": (ip, [vp, ip, vp, vp, ip, ip]),
        "wdmg_smooth": (ip, [vp, ip, vp, vp, ip, ip, ip]),
        "wdmg_solve": (ip, [vp, vp, vp, ip, ctypes.POINTER(SolveParams), ctypes.POINTER(SolveStats)]),
        "wdmg_solve_bicgstab": (ip, [vp, vp, vp, ip, dp, ip, ctypes.POINTER(SolveStats)]),
        "wdmg_profile": (ip, [vp, ip]),
        "wdmg_set_tuning": (ip, [vp, ip, ip]),
        "wdmg_get_tuning": (ip, [vp, ip, ip, ip, ctypes.POINTER(ctypes.c_int)]),
        "wdmg_profile_read": (ip, [vp, ip, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                   ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _ptr(t: torch.Tensor, dtype, what: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what}: expected a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: tensor must be contiguous")
    return t.data_ptr()


def _cdtype(prec: str):
    return torch.complex128 if prec == "f64" else torch.complex64


class Context:
    """One lattice, one gauge field, one multigrid hierarchy (libwdmg context)."""

    def __init__(self, dims: Sequence[int], device: str | int = "cuda:0"):
        self.lib = load()
        self.dims = tuple(int(d) for d in dims)
        self.device = torch.device(device)
        lx, ly, lz, lt = self.dims
        self.site_shape = (lt, lz, ly, lx)
        self.vol = lx * ly * lz * lt
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        dev_index = self.device.index if self.device.index is not None else 0
        stream = self.stream

        _alloc, _free = _torch_allocator(torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete,
                                         dev_index, stream)
        self._alloc_cb = _ALLOC_FN(_alloc)
        self._free_cb = _FREE_FN(_free)
        self._alloc = AllocStruct(self._alloc_cb, self._free_cb, None)
        h = ctypes.c_void_p()
        d = (ctypes.c_int * 4)(*self.dims)
        rc = self.lib.wdmg_create(ctypes.byref(h), d, ctypes.byref(self._alloc),
                                  ctypes.c_void_p(self.stream.cuda_stream))
        if rc != WDMG_OK:
            raise WdmgError(rc, "wdmg_create failed")
        self.h = h
        self.levels = []  # coarse site shapes and dof per level (after setup)
        self._keep = []

    # -- helpers -----------------------------------------------------------
    def _check(self, rc: int, allow_not_converged: bool = False) -> int:
        if rc == WDMG_OK or (allow_not_converged and rc == WDMG_NOT_CONVERGED):
            return rc
        msg = self.lib.wdmg_last_error(self.h)
        raise WdmgError(rc, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.lib.wdmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fine_shape(self, nrhs=None):
        shp = self.site_shape + (4, 3)
        return shp if nrhs is None else (nrhs,) + shp

    def coarse_shape(self, level, nrhs=None):
        shp, nv = self.levels[level - 1]
        out = tuple(shp) + (2, nv)
        return out if nrhs is None else (nrhs,) + out

    def level_shape(self, level, nrhs=None):
        return self.fine_shape(nrhs) if level == 0 else self.coarse_shape(level, nrhs)

    @staticmethod
    def _nrhs(t: torch.Tensor, base_ndim: int) -> int:
        return 1 if t.dim() == base_ndim else int(t.shape[0])

    # -- entry points ---------------------------------------------------------
    def set_gauge(self, U: torch.Tensor, t_bc: int = -1):
        if tuple(U.shape) != self.site_shape + (4, 3, 3):
            raise ValueError(f"gauge field shape {tuple(U.shape)} != {self.site_shape + (4, 3, 3)}")
        self._check(self.lib.wdmg_set_gauge(self.h, _ptr(U, torch.complex128, "U"), int(t_bc)))
        self.levels = []

    def set_mass(self, m: float):
        self._check(self.lib.wdmg_set_mass(self.h, float(m)))

    def apply_D(self, psi: torch.Tensor, prec: str = "f64", out: torch.Tensor | None = None):
        nrhs = self._nrhs(psi, 6)
        if tuple(psi.shape[-6:]) != self.fine_shape():
            raise ValueError("fine field shape mismatch")
        out = torch.empty_like(psi) if out is None else out
        self._check(self.lib.wdmg_apply_D(self.h, _ptr(out, _cdtype(prec), "out"),
                                          _ptr(psi, _cdtype(prec), "in"), nrhs, PREC[prec]))
        return out

    def apply_D_noalloc(self, psi: torch.Tensor, out: torch.Tensor, prec: str = "f64"):
        """``out = D psi`` through the entry point that allocates nothing (its
        work fields sit in the library's fixed 64 MiB device scratch); the
        caller provides ``out``."""
        nrhs = self._nrhs(psi, 6)
        if tuple(psi.shape[-6:]) != self.fine_shape() or out.shape != psi.shape:
            raise ValueError("fine field shape mismatch")
        self._check(self.lib.wdmg_apply_D_noalloc(self.h, _ptr(out, _cdtype(prec), "out"),
                                                  _ptr(psi, _cdtype(prec), "in"), nrhs, PREC[prec]))
        return out

    def roundtrip(self, psi: torch.Tensor, prec: str = "f32"):
        """``psi`` converted into the internal fine-field storage of ``prec`` and back."""
        nrhs = self._nrhs(psi, 6)
        if tuple(psi.shape[-6:]) != self.fine_shape():
            raise ValueError("fine field shape mismatch")
        out = torch.empty_like(psi)
        self._check(self.lib.wdmg_roundtrip(self.h, _ptr(out, _cdtype(prec), "out"),
                                            _ptr(psi, _cdtype(prec), "in"), nrhs, PREC[prec]))
        return out

    def mg_setup(self, levels, *, omega=0.8, nu_pre=2, nu_post=2, coarse_cycles=4,
                 coarse_tol=1e-1, coarse_maxit=200, coarse_restart=32, use_alpha=True, normal=False):
        """``levels``: list of dicts ``{block, nv, setup_iters, vectors[, setup_prec, adapt_iters]}`` per coarsening;
        ``vectors`` is a complex128 device tensor ``[nv, <level l field shape>]``."""
        p = MgParams()
        self.lib.wdmg_default_mg_params(ctypes.byref(p))
        p.n_levels = len(levels) + 1
        keep = []
        shape = self.site_shape
        new_levels = []
        for i, lv in enumerate(levels):
            blk = tuple(int(b) for b in lv["block"])
            nv = int(lv["nv"])
            vec = lv["vectors"]
            if vec.shape[0] != nv:
                raise ValueError("vectors must hold nv fields")
            keep.append(vec)
            p.level[i].block = (ctypes.c_int * 4)(*blk)
            p.level[i].nv = nv
            p.level[i].setup_iters = int(lv.get("setup_iters", 0))
            p.level[i].setup_prec = PREC[lv.get("setup_prec", "f64")]
            p.level[i].adapt_iters = int(lv.get("adapt_iters", 0))
            p.level[i].vectors = _ptr(vec, torch.complex128, f"level {i} vectors")
            lt, lz, ly, lx = shape
            shape = (lt // blk[3], lz // blk[2], ly // blk[1], lx // blk[0])
            new_levels.append((shape, nv))
        p.omega, p.nu_pre, p.nu_post = float(omega), int(nu_pre), int(nu_post)
        p.coarse_cycles, p.coarse_tol = int(coarse_cycles), float(coarse_tol)
        p.coarse_maxit, p.coarse_restart = int(coarse_maxit), int(coarse_restart)
        p.use_alpha = 1 if use_alpha else 0
        p.normal = 1 if normal else 0
        self._check(self.lib.wdmg_mg_setup(self.h, ctypes.byref(p)))
        self.levels = new_levels
        del keep

    def release_unused(self, mg_prec: str):
        """Free the FP64/FP32 copies of P and D_c that a V-cycle in 16-bit storage
        (``mg_prec`` "f16" or "bf16") does not read, until the next mg_setup."""
        self._check(self.lib.wdmg_release_unused(self.h, PREC[mg_prec]))

    def get_prolongator(self, level: int):
        nv = self.levels[level][1]
        out = torch.empty((nv,) + self.level_shape(level), dtype=torch.complex128, device=self.device)
        self._check(self.lib.wdmg_get_prolongator(self.h, int(level), out.data_ptr()))
        return out

    def apply_Dc(self, level: int, c: torch.Tensor, prec: str = "f64"):
        base = len(self.coarse_shape(level))
        nrhs = self._nrhs(c, base)
        out = torch.empty_like(c)
        self._check(self.lib.wdmg_apply_Dc(self.h, int(level), _ptr(out, _cdtype(prec), "out"),
                                           _ptr(c, _cdtype(prec), "in"), nrhs, PREC[prec]))
        return out

    def apply_Nc(self, level: int, c: torch.Tensor):
        """(D^dagger D)_c of a normal-equation hierarchy on coarse level ``level``."""
        base = len(self.coarse_shape(level))
        nrhs = self._nrhs(c, base)
        out = torch.empty_like(c)
        self._check(self.lib.wdmg_apply_Nc(self.h, int(level), _ptr(out, torch.complex128, "out"),
                                           _ptr(c, torch.complex128, "in"), nrhs))
        return out

    def restrict(self, level: int, f: torch.Tensor, prec: str = "f64"):
        base = len(self.level_shape(level))
        nrhs = self._nrhs(f, base)
        shp = self.coarse_shape(level + 1, nrhs if f.dim() > base else None)
        out = torch.empty(shp, dtype=_cdtype(prec), device=self.device)
        self._check(self.lib.wdmg_restrict(self.h, int(level), out.data_ptr(),
                                           _ptr(f, _cdtype(prec), "f"), nrhs, PREC[prec]))
        return out

    def prolong(self, level: int, c: torch.Tensor, prec: str = "f64"):
        base = len(self.coarse_shape(level + 1))
        nrhs = self._nrhs(c, base)
        shp = self.level_shape(level, nrhs if c.dim() > base else None)
        out = torch.empty(shp, dtype=_cdtype(prec), device=self.device)
        self._check(self.lib.wdmg_prolong(self.h, int(level), out.data_ptr(),
                                          _ptr(c, _cdtype(prec), "c"), nrhs, PREC[prec]))
        return out

    def smooth(self, level: int, x: torch.Tensor, b: torch.Tensor, iters: int, prec: str = "f64"):
        base = len(self.level_shape(level))
        nrhs = self._nrhs(b, base)
        self._check(self.lib.wdmg_smooth(self.h, int(level), _ptr(x, _cdtype(prec), "x"),
                                         _ptr(b, _cdtype(prec), "b"), nrhs, int(iters), PREC[prec]))
        return x

    def solve(self, b: torch.Tensor, x0: torch.Tensor | None = None, *, tol=1e-10, restart=50,
              maxit=1000, precond=True, mg_prec="f64", graph=False, outer="fgcr", in_place=False):
        """MG-preconditioned solve; ``outer`` is "fgcr" (flexible GCR(restart)),
        "bicgstab" (BiCGStab with the V-cycle as right preconditioner, x0 = 0),
        "cgnr" (CG on the normal equations) or "mgcg" (flexible CG on the normal
        equations with the normal-equation V-cycle).  ``in_place``: FGCR from
        x = 0 with the solution written over ``b`` (which is returned), no
        internal copy of b kept; for the largest batches."""
        nrhs = self._nrhs(b, 6)
        if in_place:
            if x0 is not None:
                raise ValueError("an in-place solve starts from x = 0")
            x = b
        else:
            x = torch.zeros_like(b) if x0 is None else x0.clone()
        p = SolveParams(float(tol), int(restart), int(maxit), 1 if precond else 0, PREC[mg_prec],
                        1 if graph else 0, {"fgcr": 0, "bicgstab": 1, "cgnr": 2, "mgcg": 3}[outer],
                        1 if in_place else 0)
        stats = (SolveStats * nrhs)()
        rc = self.lib.wdmg_solve(self.h, _ptr(x, torch.complex128, "x"), _ptr(b, torch.complex128, "b"),
                                 nrhs, ctypes.byref(p), stats)
        self._check(rc, allow_not_converged=True)
        return x, [s.as_dict() for s in stats]

    TUNE = {"dslash": 0, "dslash_group": 1, "coarse_apply": 2}

    def set_tuning(self, key: str, value: int | None):
        """Force a kernel form (0, 1, ...) or let the autotuner pick (None)."""
        self._check(self.lib.wdmg_set_tuning(self.h, self.TUNE[key], -1 if value is None else int(value)))

    def set_tuning_for(self, key: str, prec: str, nrhs: int, value: int | None):
        """Pin the autotuner's choice of ``key`` ("dslash" or "dslash_group") for one
        precision and batch size (None clears it)."""
        self._check(self.lib.wdmg_set_tuning_for(self.h, self.TUNE[key], PREC[prec], int(nrhs),
                                                 -1 if value is None else int(value)))

    def get_tuning(self, key: str, prec: str = "f64", nrhs: int = 1):
        v = ctypes.c_int()
        self._check(self.lib.wdmg_get_tuning(self.h, self.TUNE[key], PREC[prec], int(nrhs), ctypes.byref(v)))
        return None if v.value < 0 else v.value

    def profile(self, enable: bool):
        """Start (clearing earlier records) or stop HIP-event timing of the main kernels."""
        self._check(self.lib.wdmg_profile(self.h, 1 if enable else 0))

    def profile_read(self):
        """{kernel: (launches, units, ms)} since the last profile(True)."""
        out = {}
        for k, name in enumerate(KERNELS):
            n, u, ms = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_double()
            self._check(self.lib.wdmg_profile_read(self.h, k, ctypes.byref(n), ctypes.byref(u), ctypes.byref(ms)))
            out[name] = (n.value, u.value, ms.value)
        return out

    def solve_bicgstab(self, b: torch.Tensor, *, tol=1e-10, maxit=100000):
        nrhs = self._nrhs(b, 6)
        x = torch.zeros_like(b)
        stats = (SolveStats * nrhs)()
        rc = self.lib.wdmg_solve_bicgstab(self.h, _ptr(x, torch.complex128, "x"),
                                          _ptr(b, torch.complex128, "b"), nrhs, float(tol), int(maxit), stats)
        self._check(rc, allow_not_converged=True)
        return x, [s.as_dict() for s in stats]
