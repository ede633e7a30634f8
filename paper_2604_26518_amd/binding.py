"""ctypes binding of libgmt (include/gmt.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Torch tensors supply device memory and the current HIP stream.  Each
method validates device, dtype, contiguity and element counts on the host
before a pointer crosses the ABI, so a wrong shape raises here instead of
reaching a kernel.
"""

from __future__ import annotations

import ctypes as ct
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmt.so")

GMT_OK, GMT_E_INVAL, GMT_E_NOMEM, GMT_E_HIP, GMT_E_NOCONV, GMT_E_SINGULAR, GMT_E_STATE = range(7)
GMT_ELASTIC, GMT_THERMAL = 0, 1
GMT_F64, GMT_F32 = 0, 1
GMT_SMOOTH_CHEBYSHEV, GMT_SMOOTH_JACOBI, GMT_SMOOTH_GS = 0, 1, 2
GMT_CYCLE_V, GMT_CYCLE_W, GMT_CYCLE_F = 0, 1, 2
_SMOOTHERS = {"chebyshev": GMT_SMOOTH_CHEBYSHEV, "jacobi": GMT_SMOOTH_JACOBI, "gs": GMT_SMOOTH_GS}
_SCHEDULES = {"V": GMT_CYCLE_V, "W": GMT_CYCLE_W, "F": GMT_CYCLE_F}

_STATUS = {1: "GMT_E_INVAL", 2: "GMT_E_NOMEM", 3: "GMT_E_HIP", 4: "GMT_E_NOCONV",
           5: "GMT_E_SINGULAR", 6: "GMT_E_STATE"}

ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
RELEASE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class GmtParams(ct.Structure):
    _fields_ = [("physics", ct.c_int32), ("E", ct.c_double), ("nu", ct.c_double),
                ("kappa", ct.c_double), ("levels", ct.c_int32), ("power_iters", ct.c_int32),
                ("seed", ct.c_uint64), ("alloc", ALLOC_FN), ("release", RELEASE_FN),
                ("alloc_ctx", ct.c_void_p), ("gauge", ct.c_int32)]


class GmtSimpParams(ct.Structure):
    _fields_ = [("p", ct.c_double), ("rho_min", ct.c_double), ("prune", ct.c_double)]


class GmtLevelDesc(ct.Structure):
    _fields_ = [("N", ct.c_int32), ("n_e", ct.c_int32), ("n_n", ct.c_int32),
                ("c", ct.c_int32), ("d", ct.c_int32), ("lambda_max", ct.c_double),
                ("sweep_variant", ct.c_int32 * 2), ("sweep_block", ct.c_int32 * 2), ("sweep_xcd", ct.c_int32 * 2)]


class GmtCycleOpts(ct.Structure):
    _fields_ = [("nu1", ct.c_int32), ("nu2", ct.c_int32), ("smoother", ct.c_int32),
                ("omega", ct.POINTER(ct.c_double)), ("lo", ct.POINTER(ct.c_double)),
                ("hi", ct.POINTER(ct.c_double)), ("schedule", ct.c_int32)]


class GmtSolveOpts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("max_iter", ct.c_int32), ("precision", ct.c_int32),
                ("max_outer", ct.c_int32), ("check_every", ct.c_int32), ("cycle", GmtCycleOpts),
                ("graph", ct.c_int32), ("zero_start", ct.c_int32)]


class GmtSolveReport(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("outer", ct.c_int32), ("converged", ct.c_int32),
                ("c", ct.c_int32), ("rel_res", ct.c_double * 6), ("rel_res_init", ct.c_double * 6)]


NN_MAX_LEVELS = 8


class GmtNNConfig(ct.Structure):
    _fields_ = [("levels", ct.c_int32), ("channels", ct.c_int32 * NN_MAX_LEVELS), ("head", ct.c_int32),
                ("attention", ct.c_int32)]


def nn_config(levels, channels, head=32, attention=False):
    cfg = GmtNNConfig()
    cfg.levels = levels
    for l, c in enumerate(channels):
        cfg.channels[l] = c
    cfg.head = head
    cfg.attention = 1 if attention else 0
    return cfg


class GmtError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

# exported symbols and their argument types (must match include/gmt.h)
_P = ct.c_void_p
_I = ct.c_int32
SIGNATURES = {
    "gmt_build_hierarchy": (_P, _I, ct.POINTER(GmtParams), _P, ct.POINTER(_P)),
    "gmt_destroy": (_P,),
    "gmt_level_info": (_P, _I, ct.POINTER(GmtLevelDesc)),
    "gmt_export_maps": (_P, _I, _P, _P, _P, _P, _P, _P, _P),
    "gmt_export_element_matrices": (_P, _I, _P, _P),
    "gmt_export_diagonal": (_P, _I, _P, _P),
    "gmt_load_vector": (_P, _P, _I, _P),
    "gmt_apply_K": (_P, _I, _P, _P, _I, _P),
    "gmt_residual": (_P, _I, _P, _P, _P, _I, _P),
    "gmt_smooth": (_P, _I, _P, _P, _I, _I, ct.c_double, ct.c_double, _I, _P),
    "gmt_restrict": (_P, _I, _P, _P, _I, _P),
    "gmt_prolong_add": (_P, _I, _P, _P, _I, _P),
    "gmt_coarse_solve": (_P, _P, _P, _I, _P),
    "gmt_vcycle": (_P, _P, _P, _P, ct.POINTER(GmtCycleOpts), _I, _P),
    "gmt_solve": (_P, _P, _P, ct.POINTER(GmtSolveOpts), ct.POINTER(GmtSolveReport), _P),
    "gmt_solve_batch": (_P, _I, _P, _P, ct.POINTER(GmtSolveOpts), _I, ct.POINTER(GmtSolveReport),
                        ct.POINTER(ct.c_int32), _P),
    "gmt_relative_residual": (_P, _P, _P, _I, ct.POINTER(ct.c_double), _P),
    "gmt_homogenize": (_P, _P, _I, ct.POINTER(ct.c_double), _P),
    "gmt_time_sweep": (_P, _I, _I, _I, ct.POINTER(ct.c_double), _P),
    "gmt_nn_param_count": (ct.POINTER(GmtNNConfig), _I, ct.POINTER(ct.c_size_t)),
    "gmt_nn_setup": (_P, ct.POINTER(GmtNNConfig), _P),
    "gmt_nn_forward": (_P, _P, _P, _P),
    "gmt_nn_backward": (_P, _P, _P, _P),
    "gmt_nn_activation": (_P, _I, _I, _P, ct.POINTER(ct.c_int32), _P),
    "gmt_nn_serialization": (_P, _I, _P, _P),
    "gmt_nn_time_attention": (_P, _I, _I, ct.POINTER(ct.c_double), _P),
    "gmt_nn_supervised_loss": (_P, _P, _P, ct.c_double, _P, ct.POINTER(ct.c_double), _P),
    "gmt_nn_adamw": (_P, _P, _P, _P, ct.c_size_t, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                     ct.c_double, _I, ct.c_double, _P),
    "gmt_nn_norm2": (_P, ct.c_size_t, ct.POINTER(ct.c_double), _P),
    "gmt_nn_ema": (_P, _P, ct.c_size_t, ct.c_double, _P),
    "gmt_nn_norm2_noalloc": (_P, ct.c_size_t, ct.POINTER(ct.c_double), _P),
    "gmt_vcycle_loss": (_P, _P, ct.POINTER(GmtCycleOpts), ct.c_double, _P, ct.POINTER(ct.c_double), _P, _P),
    "gmt_build_density_hierarchy": (_P, _I, ct.c_void_p, ct.POINTER(GmtParams), _P, ct.POINTER(_P)),
    "gmt_simp_sensitivity": (_P, _P, _P, _P, _P, _P),
    "gmt_simp_objective": (_P, _I, ct.POINTER(ct.c_double), _P),
    "gmt_simp_filter": (_P, _P, _I, ct.c_double, _P, _P),
    "gmt_simp_oc": (_P, _P, ct.c_size_t, ct.c_double, ct.c_double, ct.c_double, ct.c_double, _P,
                    ct.POINTER(ct.c_double), _P),
    "gmt_last_error": (),
}


def lib():
    """Load libgmt.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2604_26518_amd.build`")
        L = ct.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = list(args)
            fn.restype = ct.c_char_p if name == "gmt_last_error" else (None if name == "gmt_destroy" else ct.c_int)
        _lib = L
    return _lib


def _check(status):
    if status != GMT_OK:
        raise GmtError(status, lib().gmt_last_error().decode())


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


_DT = {torch.float64: GMT_F64, torch.float32: GMT_F32}


def _dbl_array(vals):
    if vals is None:
        return None
    arr = (ct.c_double * len(vals))(*[float(v) for v in vals])
    return ct.cast(arr, ct.POINTER(ct.c_double)), arr


class _TorchArena:
    """Device memory for the library's internal buffers from torch's caching allocator."""

    def __init__(self, device):
        self.device = torch.device(device)
        self.live = {}
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.release_cb = RELEASE_FN(self._release)

    def _alloc(self, nbytes, ctx):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _release(self, ptr, ctx):
        self.live.pop(ptr, None)


class Hierarchy:
    """One periodic cell: its sparse GMG hierarchy and operators on the GPU."""

    def __init__(self, voxels, levels: int, physics: str = "elastic", E: float = 1.0,
                 nu: float = 0.3, kappa: float = 1.0, power_iters: int = 20, seed: int = 0,
                 device="cuda", torch_memory: bool = True, density=None, p: float = 3.0,
                 rho_min: float = 1e-3, prune: float = 0.0, gauge: str = "pin"):
        """voxels: binary N^3 cell; or voxels=None and density = an N^3 field rho for the
        SIMP cell problem (App. F.3) with penalization p, floor rho_min and pruning threshold.
        gauge: 'pin' (node 0 fixed, the default) or 'mean' (zero mean per component) for the
        solutions that solve() reports."""
        if physics not in ("elastic", "thermal"):
            raise ValueError(physics)
        self.density = None
        if density is not None:
            if isinstance(density, np.ndarray):
                density = torch.from_numpy(np.ascontiguousarray(density, dtype=np.float64))
            self.density = density.to(device=device, dtype=torch.float64).contiguous()
            voxels = (self.density > prune).to(torch.uint8)
            self.simp = (p, rho_min, prune)
        if isinstance(voxels, np.ndarray):
            voxels = torch.from_numpy(np.ascontiguousarray(voxels, dtype=np.uint8))
        N = int(voxels.shape[0])
        if tuple(voxels.shape) != (N, N, N):
            raise ValueError("voxels must be N^3")
        self._vox = voxels.to(device=device, dtype=torch.uint8).contiguous()
        self.N = N
        self.physics = physics
        self.c, self.d = (6, 3) if physics == "elastic" else (3, 1)
        p = GmtParams()
        p.physics = GMT_ELASTIC if physics == "elastic" else GMT_THERMAL
        p.E, p.nu, p.kappa = E, nu, kappa
        p.levels = levels
        p.power_iters = power_iters
        p.seed = seed
        if gauge not in ("pin", "mean"):
            raise ValueError("gauge is 'pin' (node 0 fixed) or 'mean' (zero mean per component)")
        p.gauge = 1 if gauge == "mean" else 0
        self._arena = None
        if torch_memory:
            self._arena = _TorchArena(self._vox.device)
            p.alloc = self._arena.alloc_cb
            p.release = self._arena.release_cb
        h = ct.c_void_p()
        if self.density is not None:
            sp = GmtSimpParams(*self.simp)
            _check(lib().gmt_build_density_hierarchy(_ptr(self.density), N, ct.byref(sp), ct.byref(p), _stream(),
                                                     ct.byref(h)))
        else:
            _check(lib().gmt_build_hierarchy(_ptr(self._vox), N, ct.byref(p), _stream(), ct.byref(h)))
        self._h = h
        self.L = levels
        self.levels = [self.level_info(l) for l in range(1, levels + 1)]

    def close(self):
        if getattr(self, "_h", None):
            lib().gmt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- shapes
    def level_info(self, level: int) -> dict:
        d = GmtLevelDesc()
        _check(lib().gmt_level_info(self._h, level, ct.byref(d)))
        return {"N": d.N, "n_e": d.n_e, "n_n": d.n_n, "c": d.c, "d": d.d, "lambda_max": d.lambda_max,
                "sweep_variant": tuple(d.sweep_variant), "sweep_block": tuple(d.sweep_block),
                "sweep_xcd": tuple(d.sweep_xcd)}

    def n_n(self, level: int = 1) -> int:
        return self.levels[level - 1]["n_n"]

    def n_e(self, level: int = 1) -> int:
        return self.levels[level - 1]["n_e"]

    def vec(self, level: int = 1, dtype=torch.float64, fill=0.0):
        return torch.full((self.n_n(level), self.c, self.d), fill, dtype=dtype, device=self._vox.device)

    def _v(self, t, level, dtype=None, name="vector"):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if dtype is not None and t.dtype != dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
        if t.dtype not in _DT:
            raise TypeError(f"{name} must be float32 or float64")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        want = self.n_n(level) * self.c * self.d
        if t.numel() != want:
            raise ValueError(f"{name} has {t.numel()} elements, level {level} needs {want}")
        return t

    def _level(self, level):
        if not 1 <= level <= self.L:
            raise ValueError(f"level {level} outside 1..{self.L}")

    # -- maps and operators (exports)
    def export_maps(self, level: int):
        self._level(level)
        info = self.levels[level - 1]
        dev = self._vox.device
        out = {
            "elem_lin": torch.empty(info["n_e"], dtype=torch.int32, device=dev),
            "node_lin": torch.empty(info["n_n"], dtype=torch.int32, device=dev),
            "occ8": torch.empty(info["n_n"], dtype=torch.uint8, device=dev),
            "elem_nodes": torch.empty(info["n_e"], 8, dtype=torch.int32, device=dev),
        }
        if level < self.L:
            out["prol_idx"] = torch.empty(info["n_n"], 8, dtype=torch.int32, device=dev)
            out["prol_w"] = torch.empty(info["n_n"], 8, dtype=torch.float64, device=dev)
        _check(lib().gmt_export_maps(self._h, level, _ptr(out["elem_lin"]), _ptr(out["node_lin"]),
                                     _ptr(out["occ8"]), _ptr(out["elem_nodes"]),
                                     _ptr(out.get("prol_idx")), _ptr(out.get("prol_w")), _stream()))
        return out

    def export_element_matrices(self, level: int):
        self._level(level)
        M = 8 * self.d
        K = torch.empty(self.n_e(level), M, M, dtype=torch.float64, device=self._vox.device)
        _check(lib().gmt_export_element_matrices(self._h, level, _ptr(K), _stream()))
        return K

    def export_diagonal(self, level: int):
        self._level(level)
        D = torch.empty(self.n_n(level), self.d, dtype=torch.float64, device=self._vox.device)
        _check(lib().gmt_export_diagonal(self._h, level, _ptr(D), _stream()))
        return D

    def load_vector(self, dtype=torch.float64):
        f = self.vec(1, dtype)
        _check(lib().gmt_load_vector(self._h, _ptr(f), _DT[dtype], _stream()))
        return f

    def apply_K(self, u, level: int = 1, out=None):
        self._level(level)
        self._v(u, level, name="u")
        y = torch.empty_like(u) if out is None else self._v(out, level, u.dtype, "out")
        _check(lib().gmt_apply_K(self._h, level, _ptr(u), _ptr(y), _DT[u.dtype], _stream()))
        return y

    def residual(self, f, u, level: int = 1):
        self._level(level)
        self._v(u, level, name="u")
        self._v(f, level, u.dtype, "f")
        r = torch.empty_like(u)
        _check(lib().gmt_residual(self._h, level, _ptr(f), _ptr(u), _ptr(r), _DT[u.dtype], _stream()))
        return r

    def smooth(self, f, u, nu: int, smoother: str = "chebyshev", p1: float = 0.0, p2: float = 0.0,
               level: int = 1):
        """nu smoothing steps in place on u: Jacobi (omega = p1), Chebyshev on [p1, p2], or
        8-colour Gauss-Seidel / SOR (omega = p1; colours 0..7 for p2 = 0, 7..0 for p2 = 1)."""
        self._level(level)
        self._v(u, level, name="u")
        self._v(f, level, u.dtype, "f")
        sm = _SMOOTHERS[smoother]
        _check(lib().gmt_smooth(self._h, level, _ptr(f), _ptr(u), nu, sm, p1, p2, _DT[u.dtype], _stream()))
        return u

    def restrict(self, rf, level: int = 1):
        self._level(level)
        if level == self.L:
            raise ValueError("no level below the coarsest")
        self._v(rf, level, name="rf")
        fc = self.vec(level + 1, rf.dtype)
        _check(lib().gmt_restrict(self._h, level, _ptr(rf), _ptr(fc), _DT[rf.dtype], _stream()))
        return fc

    def prolong_add(self, uc, uf, level: int = 1):
        self._level(level)
        if level == self.L:
            raise ValueError("no level below the coarsest")
        self._v(uf, level, name="uf")
        self._v(uc, level + 1, uf.dtype, "uc")
        _check(lib().gmt_prolong_add(self._h, level, _ptr(uc), _ptr(uf), _DT[uf.dtype], _stream()))
        return uf

    def coarse_solve(self, f):
        self._v(f, self.L, name="f")
        u = torch.empty_like(f)
        _check(lib().gmt_coarse_solve(self._h, _ptr(f), _ptr(u), _DT[f.dtype], _stream()))
        return u

    def _cycle(self, nu1=2, nu2=2, smoother="chebyshev", omega=None, lo=None, hi=None, schedule="V"):
        o = GmtCycleOpts()
        o.nu1, o.nu2 = nu1, nu2
        o.smoother = _SMOOTHERS[smoother]
        o.schedule = _SCHEDULES[schedule]
        keep = []
        for name, vals in (("omega", omega), ("lo", lo), ("hi", hi)):
            if vals is not None:
                if len(vals) != self.L:
                    raise ValueError(f"{name} needs {self.L} entries")
                p, arr = _dbl_array(vals)
                setattr(o, name, p)
                keep.append(arr)
        return o, keep

    def vcycle(self, f, u, e_init=None, nu1=2, nu2=2, smoother="chebyshev", omega=None, lo=None, hi=None,
               schedule="V"):
        """One cycle (Alg. 2; schedule V, W or F) in place on u; e_init: list indexed by level-1 of
        corrections or None."""
        self._v(u, 1, name="u")
        self._v(f, 1, u.dtype, "f")
        o, keep = self._cycle(nu1, nu2, smoother, omega, lo, hi, schedule)
        arr = None
        if e_init is not None:
            if len(e_init) != self.L:
                raise ValueError(f"e_init needs {self.L} entries")
            ptrs = []
            for l, e in enumerate(e_init, start=1):
                if e is None or l == 1 or l == self.L:
                    ptrs.append(None)
                else:
                    self._v(e, l, u.dtype, f"e_init[{l}]")
                    ptrs.append(e.data_ptr())
            arr = (ct.c_void_p * self.L)(*ptrs)
        _check(lib().gmt_vcycle(self._h, _ptr(f), _ptr(u), arr, ct.byref(o), _DT[u.dtype], _stream()))
        return u

    def solve_opts(self, tol=1e-5, max_iter=500, precision="f64", max_outer=8, check_every=1, nu1=2, nu2=2,
                   smoother="chebyshev", omega=None, lo=None, hi=None, graph=True, schedule="V"):
        """(gmt_solve_opts, buffers to keep alive during the call)."""
        o = GmtSolveOpts()
        o.tol, o.max_iter, o.max_outer, o.check_every = tol, max_iter, max_outer, check_every
        o.precision = GMT_F64 if precision == "f64" else GMT_F32
        o.cycle, keep = self._cycle(nu1, nu2, smoother, omega, lo, hi, schedule)
        o.graph = 1 if graph else 0
        return o, keep

    def solve(self, f, u=None, tol=1e-5, max_iter=500, precision="f64", max_outer=8, check_every=1,
              nu1=2, nu2=2, smoother="chebyshev", omega=None, lo=None, hi=None, raise_on_noconv=True,
              graph=True, schedule="V"):
        self._v(f, 1, torch.float64, "f")
        zero = u is None
        if zero:
            u = torch.empty_like(f)  # output only: the solve starts from zero
        self._v(u, 1, torch.float64, "u")
        o, keep = self.solve_opts(tol, max_iter, precision, max_outer, check_every, nu1, nu2, smoother, omega, lo,
                                  hi, graph, schedule)
        o.zero_start = 1 if zero else 0
        rep = GmtSolveReport()
        st = lib().gmt_solve(self._h, _ptr(f), _ptr(u), ct.byref(o), ct.byref(rep), _stream())
        report = _report(rep, self.c, st)
        if st != GMT_OK and (st != GMT_E_NOCONV or raise_on_noconv):
            _check(st)
        return u, report

    def relative_residual(self, f, u):
        self._v(u, 1, name="u")
        self._v(f, 1, u.dtype, "f")
        out = (ct.c_double * 6)()
        _check(lib().gmt_relative_residual(self._h, _ptr(f), _ptr(u), _DT[u.dtype], out, _stream()))
        return np.array(out[:self.c])

    # -- learned initializer
    def nn_setup(self, channels, head=32, attention=False):
        """Network on levels 1..len(channels) (at most the hierarchy's L levels), with an
        attention block per level if `attention`."""
        if not 2 <= len(channels) <= self.L:
            raise ValueError(f"need 2..{self.L} channel counts")
        self.nn_levels = len(channels)
        self.nn_attention = bool(attention)
        self._nn_cfg = nn_config(self.nn_levels, channels, head, attention)
        self.n_params = nn_param_count(self.nn_levels, channels, head, self.physics, attention)
        _check(lib().gmt_nn_setup(self._h, ct.byref(self._nn_cfg), _stream()))

    def _check_params(self, params):
        if not (isinstance(params, torch.Tensor) and params.is_cuda and params.dtype == torch.float32
                and params.is_contiguous() and params.numel() == self.n_params):
            raise ValueError(f"params must be a contiguous float32 CUDA tensor of {self.n_params} values")

    def nn_forward(self, params):
        """Predictions [u_hat^1, e_hat^2, ..., e_hat^{L-1}] as float32 [n_l][c][d] tensors."""
        self._check_params(params)
        outs = [self.vec(l, torch.float32) for l in range(1, self.nn_levels)] + [None]
        _check(lib().gmt_nn_forward(self._h, _ptr(params), _ptr_array(outs), _stream()))
        return outs[:-1]

    def nn_backward(self, gouts, grad):
        """grad += d/dparams sum_l <gouts[l], outs[l]> for the last forward."""
        self._check_params(grad)
        gl = (list(gouts) + [None] * self.nn_levels)[:self.nn_levels]
        for l, g in enumerate(gl[:self.nn_levels - 1], start=1):
            if g is not None:
                self._v(g, l, torch.float32, f"gout[{l}]")
        _check(lib().gmt_nn_backward(self._h, _ptr_array(gl), _ptr(grad), _stream()))

    def nn_activation(self, level: int, which: int):
        """Stored activation of the last forward as float32 [n_l][width]: 0 h, 1 a, 2 t, 3 d, 4 z1,
        5 z2, 6 s (attention block output, or a); with attention, in serialization order, 7 q,
        8 k, 9 v and 10 the attention output before its BF16 rounding."""
        self._level(level)
        w = ct.c_int32()
        _check(lib().gmt_nn_activation(self._h, level, which, None, ct.byref(w), _stream()))
        out = torch.empty(self.n_n(level), w.value, dtype=torch.float32, device=self._vox.device)
        _check(lib().gmt_nn_activation(self._h, level, which, _ptr(out), ct.byref(w), _stream()))
        return out

    def nn_serialization(self, level: int):
        """Node ids of level `level` in its serialization order (int32 [n_l]; attention only)."""
        self._level(level)
        out = torch.empty(self.n_n(level), dtype=torch.int32, device=self._vox.device)
        _check(lib().gmt_nn_serialization(self._h, level, _ptr(out), _stream()))
        return out

    def nn_supervised_loss(self, pred, target, alpha=1.0, grad=None) -> float:
        """alpha |pred - target_c|^2 / |target_c|^2 (target centred per column); grad += its gradient."""
        self._v(pred, 1, torch.float32, "pred")
        self._v(target, 1, torch.float32, "target")
        if grad is not None:
            self._v(grad, 1, torch.float32, "grad")
        out = ct.c_double()
        _check(lib().gmt_nn_supervised_loss(self._h, _ptr(pred), _ptr(target), float(alpha),
                                            _ptr(grad) if grad is not None else None, ct.byref(out), _stream()))
        return out.value

    def nn_time_attention(self, level: int, reps: int = 10) -> float:
        """Mean ms of one launch of level `level`'s attention forward kernel (after a forward)."""
        self._level(level)
        out = ct.c_double()
        _check(lib().gmt_nn_time_attention(self._h, level, reps, ct.byref(out), _stream()))
        return out.value

    def vcycle_loss(self, preds, lam=0.0, want_grad=True, want_u1=False, nu1=2, nu2=2, smoother="chebyshev",
                    omega=None, lo=None, hi=None):
        """Alg. 2 V-cycle from network outputs + the physics loss and its gradient.

        preds: [u_hat^1, e_hat^2 or None, ...] float32.  Returns (loss, ||r||, rel[c], u1, grads).
        """
        pl = list(preds) + [None] * (self.L - len(preds))
        self._v(pl[0], 1, torch.float32, "u_hat")
        for l in range(2, self.L):
            if pl[l - 1] is not None:
                self._v(pl[l - 1], l, torch.float32, f"e_hat[{l}]")
        pl[self.L - 1] = None
        o, keep = self._cycle(nu1, nu2, smoother, omega, lo, hi)
        u1 = self.vec(1, torch.float32) if want_u1 else None
        grads = None
        if want_grad:
            grads = [torch.empty_like(p) if p is not None else None for p in pl[:self.L - 1]] + [None]
        out = (ct.c_double * (2 + self.c))()
        _check(lib().gmt_vcycle_loss(self._h, _ptr_array(pl), ct.byref(o), lam,
                                     _ptr(u1) if u1 is not None else None, out,
                                     _ptr_array(grads) if grads is not None else None, _stream()))
        return out[0], out[1], np.array(out[2:2 + self.c]), u1, (grads[:-1] if grads is not None else None)

    def time_sweep(self, level: int = 1, reps: int = 50, dtype=torch.float32) -> float:
        """Mean milliseconds of one fused Chebyshev sweep of a level (HIP events)."""
        self._level(level)
        out = ct.c_double()
        _check(lib().gmt_time_sweep(self._h, level, reps, _DT[dtype], ct.byref(out), _stream()))
        return out.value

    def simp_sensitivity(self, u, G=None, want_dC=False):
        """(dJ [N^3] or None, dC [N^3][c][c] or None) of App. F.3 for a density hierarchy."""
        self._v(u, 1, torch.float64, "u")
        dev = self._vox.device
        n3 = self.N ** 3
        dJ = torch.empty(n3, dtype=torch.float64, device=dev) if G is not None else None
        dC = torch.empty(n3, self.c, self.c, dtype=torch.float64, device=dev) if want_dC else None
        g = None
        if G is not None:
            g = np.ascontiguousarray(G, dtype=np.float64).reshape(self.c * self.c)
        _check(lib().gmt_simp_sensitivity(self._h, _ptr(u), g.ctypes.data if g is not None else None,
                                          _ptr(dJ) if dJ is not None else None,
                                          _ptr(dC) if dC is not None else None, _stream()))
        return dJ, dC

    def homogenize(self, u):
        self._v(u, 1, name="u")
        out = (ct.c_double * 36)()
        _check(lib().gmt_homogenize(self._h, _ptr(u), _DT[u.dtype], out, _stream()))
        return np.array(out[:self.c * self.c]).reshape(self.c, self.c)


def _report(rep, c, st):
    return {"iterations": rep.iterations, "outer": rep.outer, "converged": bool(rep.converged),
            "rel_res": list(rep.rel_res)[:c], "rel_res_init": list(rep.rel_res_init)[:c], "status": st}


def solve_batch(hs, fs, us=None, n_workers=4, raise_on_noconv=True, **opts):
    """gmt_solve_batch over hierarchies hs with FP64 loads fs (initial guesses us, zeros if None).

    All cells share one option set (tol, precision, ...; Chebyshev bounds default per cell).
    Returns (us, reports)."""
    n = len(hs)
    if len(fs) != n or (us is not None and len(us) != n):
        raise ValueError("hs, fs and us must have the same length")
    zero = us is None
    if zero:
        us = [torch.empty_like(f) for f in fs]  # outputs only: every cell starts from zero
    for H, f, u in zip(hs, fs, us):
        H._v(f, 1, torch.float64, "f")
        H._v(u, 1, torch.float64, "u")
    for k in ("omega", "lo", "hi"):
        if opts.get(k) is not None:
            raise ValueError(f"{k} is per cell; the batch uses each cell's defaults")
    o, keep = hs[0].solve_opts(**opts) if n else (GmtSolveOpts(), [])
    o.zero_start = 1 if zero else 0
    harr = (ct.c_void_p * max(n, 1))(*[H._h for H in hs])
    farr = (ct.c_void_p * max(n, 1))(*[f.data_ptr() for f in fs])
    uarr = (ct.c_void_p * max(n, 1))(*[u.data_ptr() for u in us])
    reps = (GmtSolveReport * max(n, 1))()
    stat = (ct.c_int32 * max(n, 1))()
    st = lib().gmt_solve_batch(harr, n, farr, uarr, ct.byref(o), n_workers, reps, stat, _stream())
    reports = [_report(reps[i], hs[i].c, stat[i]) for i in range(n)]
    if st != GMT_OK and (st != GMT_E_NOCONV or raise_on_noconv):
        _check(st)
    return us, reports


SIMP_OBJECTIVES = {"young": 0, "shear": 1, "bulk": 2}


def simp_objective(CH, kind: str):
    """(J, G = dJ/dC_H) of an App. F.3 target on the 6x6 C_H (host, in the library)."""
    c = np.ascontiguousarray(CH, dtype=np.float64).reshape(36)
    J = ct.c_double()
    G = np.zeros(36)
    _check(lib().gmt_simp_objective(c.ctypes.data, SIMP_OBJECTIVES[kind], ct.byref(J), G.ctypes.data))
    return J.value, G.reshape(6, 6)


def simp_filter(rho, dc, rmin: float):
    """Sensitivity filter on the dense periodic grid (float64 CUDA tensors of N^3 values)."""
    N = round(rho.numel() ** (1 / 3))
    for t, name in ((rho, "rho"), (dc, "dc")):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == N ** 3):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of N^3 values")
    out = torch.empty_like(dc)
    _check(lib().gmt_simp_filter(_ptr(rho), _ptr(dc), N, rmin, _ptr(out), _stream()))
    return out


def simp_oc(rho, dc, volfrac: float, move: float = 0.2, eta: float = 0.5, rho_lo: float = 1e-3):
    """Optimality-Criteria step with move limits; returns (rho_new, lam)."""
    for t, name in ((rho, "rho"), (dc, "dc")):
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == rho.numel()):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    out = torch.empty_like(rho)
    lam = ct.c_double()
    _check(lib().gmt_simp_oc(_ptr(rho), _ptr(dc), rho.numel(), volfrac, move, eta, rho_lo, _ptr(out),
                             ct.byref(lam), _stream()))
    return out, lam.value


def nn_param_count(levels, channels, head=32, physics="elastic", attention=False) -> int:
    out = ct.c_size_t()
    cfg = nn_config(levels, channels, head, attention)
    _check(lib().gmt_nn_param_count(ct.byref(cfg), GMT_ELASTIC if physics == "elastic" else GMT_THERMAL,
                                    ct.byref(out)))
    return int(out.value)


def adamw(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, wd=1e-2, grad_scale=1.0):
    for t in (params, grad, m, v):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("AdamW buffers must be contiguous float32 CUDA tensors")
        if t.numel() != params.numel():
            raise ValueError("AdamW buffers must have the same size")
    _check(lib().gmt_nn_adamw(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), lr, beta1, beta2,
                              eps, wd, step, grad_scale, _stream()))


def norm2(x) -> float:
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.is_contiguous()):
        raise TypeError("norm2 needs a contiguous float32 CUDA tensor")
    out = ct.c_double()
    _check(lib().gmt_nn_norm2(_ptr(x), x.numel(), ct.byref(out), _stream()))
    return out.value


def ema(e, x, decay):
    for t in (e, x):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("ema needs contiguous float32 CUDA tensors")
    if e.numel() != x.numel():
        raise ValueError("size mismatch")
    _check(lib().gmt_nn_ema(_ptr(e), _ptr(x), x.numel(), decay, _stream()))


def _ptr_array(tensors):
    return (ct.c_void_p * len(tensors))(*[None if t is None else t.data_ptr() for t in tensors])


def default_levels(N: int, coarsest: int = 4) -> int:
    """Levels so that the coarsest grid has ``coarsest`` (or the nearest feasible) voxels per axis."""
    L = 1
    n = N
    while n % 2 == 0 and n // 2 >= coarsest:
        n //= 2
        L += 1
    return L
