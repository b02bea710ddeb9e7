"""Thin ctypes binding of the C ABI in include/sipg.h.

Argument marshalling only: every step of the method runs in the HIP library
(libsipg.so next to this file).  torch supplies device memory and streams;
vectors are contiguous CUDA (HIP) tensors passed by data pointer.  Loading
fails loudly when the library is missing - there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsipg.so")

SIPG_OK = 0
STATUS = {0: "SIPG_OK", 1: "SIPG_ERR_ARG", 2: "SIPG_ERR_UNSUPPORTED", 3: "SIPG_ERR_OOM",
          4: "SIPG_ERR_HIP", 5: "SIPG_ERR_NOT_CONVERGED", 6: "SIPG_ERR_NONFINITE"}
PRECISION = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
UNITS = {"auto": 0, "vector": 1, "matrix": 2}

_lib = None


class SipgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
DEALLOC_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
SMOOTHER = {"multiplicative": 0, "additive": 1, "multiplicative_fused": 2}
VARIANT = {"fgmres": 0, "gmres": 1}


class Config(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("n_cells", ctypes.c_int), ("n_levels", ctypes.c_int),
                ("mg_precision", ctypes.c_int), ("error_correction", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
                ("smoother", ctypes.c_int), ("damping", ctypes.c_double),
                ("penalty_scale", ctypes.c_double),
                ("alloc", ALLOC_FN), ("dealloc", DEALLOC_FN), ("alloc_ctx", ctypes.c_void_p)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("use_learned", ctypes.c_int), ("log_history", ctypes.c_int),
                ("stagnation", ctypes.c_double), ("variant", ctypes.c_int)]


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None


def _torch_dealloc(ptr, stream, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# kept alive for the life of the process: the library calls them from C
TORCH_ALLOC = ALLOC_FN(_torch_alloc)
TORCH_DEALLOC = DEALLOC_FN(_torch_dealloc)


def make_config(k, n_cells, n_levels=0, mg_precision="f64", error_correction=0, nu_pre=2,
                nu_post=2, smoother="multiplicative", damping=0.0, penalty_scale=1.0,
                allocator=None):
    """sipg_config for one problem.  error_correction: 0, 1 (both operands
    split) or 2 (matrix operand split); True means 1.  allocator "torch" routes
    the handle's workspace through torch's caching allocator."""
    cfg = Config(k, n_cells, n_levels, PRECISION[mg_precision], int(error_correction),
                 nu_pre, nu_post, SMOOTHER[smoother], float(damping), float(penalty_scale))
    if allocator == "torch":
        cfg.alloc = TORCH_ALLOC
        cfg.dealloc = TORCH_DEALLOC
    elif allocator is not None:
        raise ValueError("allocator must be None or 'torch'")
    return cfg


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("rel_res_est", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("seconds", ctypes.c_double), ("history", ctypes.c_double * 128)]


class CnnTrainOpts(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int), ("chain_length", ctypes.c_int),
                ("crops_per_pair", ctypes.c_int), ("crop", ctypes.c_int), ("lr", ctypes.c_float),
                ("log_every", ctypes.c_int), ("seed", ctypes.c_uint64), ("loss", ctypes.c_int)]


class CnnTrainInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("loss_first", ctypes.c_float),
                ("loss_last", ctypes.c_float), ("sigma", ctypes.c_float),
                ("seconds", ctypes.c_double), ("seconds_pairs", ctypes.c_double)]


def load_library(path=None):
    """Load libsipg.so (raises if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # torch ships its own HIP runtime with the same soname as the system one;
    # load it first so that the library binds to that single runtime instead
    # of bringing a second HSA runtime into the process.
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise FileNotFoundError(
            f"{p} not found: build it with `python -m paper_2407_09621_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "sipg_create": (i32, [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]),
        "sipg_smooth_lp": (i32, [vp, i32, vp, vp, i32, vp]),
        "sipg_patch_correct_lp": (i32, [vp, i32, i32, vp, vp, vp]),
        "sipg_cnn_save": (i32, [vp, ctypes.c_char_p]),
        "sipg_cnn_load": (i32, [vp, ctypes.c_char_p]),
        "sipg_destroy": (None, [vp]),
        "sipg_num_levels": (i32, [vp]),
        "sipg_level_cells": (i32, [vp, i32]),
        "sipg_n_dofs": (i64, [vp, i32]),
        "sipg_apply": (i32, [vp, i32, vp, vp, vp]),
        "sipg_set_geometry": (i32, [vp, vp, vp]),
        "sipg_apply_units": (i32, [vp, i32, vp, vp, i32, vp]),
        "sipg_apply_patchwise": (i32, [vp, i32, vp, vp, vp]),
        "sipg_residual": (i32, [vp, i32, vp, vp, vp, vp]),
        "sipg_apply_lp": (i32, [vp, i32, vp, vp, i32, i32, vp]),
        "sipg_smooth": (i32, [vp, i32, vp, vp, i32, vp]),
        "sipg_patch_correct": (i32, [vp, i32, i32, vp, vp, vp]),
        "sipg_restrict": (i32, [vp, i32, vp, vp, vp]),
        "sipg_prolongate_add": (i32, [vp, i32, vp, vp, vp]),
        "sipg_coarse_solve": (i32, [vp, vp, vp, vp]),
        "sipg_vcycle": (i32, [vp, i32, vp, vp, vp]),
        "sipg_fgmres": (i32, [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]),
        "sipg_rhs_sines": (i32, [vp, i32, i32, vp, vp, vp, vp]),
        "sipg_l2_error_sines": (i32, [vp, i32, i32, vp, vp, vp, ctypes.POINTER(dbl), vp]),
        "sipg_l2_error_sines_noalloc": (i32, [vp, i32, i32, vp, vp, vp, ctypes.POINTER(dbl), vp]),
        "sipg_last_error": (ctypes.c_char_p, []),
        "sipg_autotune": (i32, [vp, i32, vp, vp, ctypes.POINTER(i32), vp]),
        "sipg_cnn_num_params": (i32, []),
        "sipg_cnn_create": (i32, [ctypes.POINTER(vp)]),
        "sipg_cnn_destroy": (None, [vp]),
        "sipg_cnn_init": (i32, [vp, ctypes.c_uint64]),
        "sipg_cnn_set_params": (i32, [vp, vp, ctypes.c_float]),
        "sipg_cnn_get_params": (i32, [vp, vp, ctypes.POINTER(ctypes.c_float)]),
        "sipg_cnn_forward": (i32, [vp, i32, i32, vp, vp, vp]),
        "sipg_cnn_gradient": (i32, [vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "sipg_cnn_adam_step": (i32, [vp, vp, ctypes.c_float, vp]),
        "sipg_cnn_gradient_residual": (i32, [vp, vp, vp, vp, vp, vp]),
        "sipg_cnn_make_pairs": (i32, [vp, vp, i32, vp, vp, vp, vp]),
        "sipg_cnn_train": (i32, [vp, vp, ctypes.POINTER(CnnTrainOpts), ctypes.POINTER(CnnTrainInfo)]),
        "sipg_cnn_attach": (i32, [vp, vp]),
        "sipg_batch_create": (i32, [ctypes.POINTER(Config), i32, vp, ctypes.POINTER(vp)]),
        "sipg_batch_destroy": (None, [vp]),
        "sipg_batch_count": (i32, [vp]),
        "sipg_batch_problem": (vp, [vp, i32]),
        "sipg_batch_autotune": (i32, [vp, vp]),
        "sipg_batch_apply": (i32, [vp, vp, vp, vp]),
        "sipg_batch_vcycle": (i32, [vp, vp, vp, vp]),
        "sipg_batch_solve": (i32, [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), i32, vp]),
        "sipg_batch_solve_sequential": (i32, [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != SIPG_OK:
        raise SipgError(status, _lib.sipg_last_error().decode())


def _ptr(t, dtype=None):
    """Device pointer of a contiguous CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Problem:
    """A SIPG Poisson problem on n_cells^3 cells of degree k, with its level
    hierarchy (level 0 coarsest, level -1 finest)."""

    def __init__(self, k, n_cells, n_levels=0, mg_precision="f64", error_correction=0,
                 nu_pre=2, nu_post=2, smoother="multiplicative", damping=0.0, penalty_scale=1.0,
                 allocator=None, stream=None):
        lib = load_library()
        cfg = make_config(k, n_cells, n_levels, mg_precision, int(error_correction), nu_pre,
                          nu_post, smoother, damping, penalty_scale, allocator)
        h = ctypes.c_void_p()
        _check(lib.sipg_create(ctypes.byref(cfg), _stream(stream), ctypes.byref(h)))
        self.mg_precision = mg_precision
        self._h = h
        self.k = k
        self.N = k + 1
        self.n_cells = n_cells
        self.num_levels = lib.sipg_num_levels(h)
        self.cells = [lib.sipg_level_cells(h, l) for l in range(self.num_levels)]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sipg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _lvl(self, level):
        return level % self.num_levels

    def n_dofs(self, level=-1):
        return int(_lib.sipg_n_dofs(self._h, self._lvl(level)))

    def new_vector(self, level=-1, dtype=None):
        import torch
        return torch.zeros(self.n_dofs(level), dtype=dtype or torch.float64, device="cuda")

    def set_geometry(self, vertices, stream=None):
        """Trilinear hexahedra through the finest level's vertex positions
        (sipg_set_geometry): a float64 array of shape (n+1, n+1, n+1, 3)
        indexed [vz, vy, vx]; None restores the Cartesian mesh."""
        import numpy as np
        if vertices is None:
            _check(_lib.sipg_set_geometry(self._h, None, _stream(stream)))
            return
        n = self.cells[-1]
        V = np.ascontiguousarray(vertices, dtype=np.float64)
        if V.shape != (n + 1, n + 1, n + 1, 3):
            raise ValueError(f"vertices must have shape {(n + 1,) * 3 + (3,)}")
        _check(_lib.sipg_set_geometry(self._h, V.ctypes.data_as(ctypes.c_void_p), _stream(stream)))

    def apply(self, u, v=None, level=-1, stream=None, units=None):
        """v = A u in FP64; units "vector" or "matrix" picks the execution
        units (sipg_apply_units), None what sipg_apply uses."""
        import torch
        v = torch.empty_like(u) if v is None else v
        if units is None:
            _check(_lib.sipg_apply(self._h, self._lvl(level), _ptr(u, torch.float64),
                                   _ptr(v, torch.float64), _stream(stream)))
        else:
            _check(_lib.sipg_apply_units(self._h, self._lvl(level), _ptr(u, torch.float64),
                                         _ptr(v, torch.float64), UNITS[units], _stream(stream)))
        return v

    def apply_patchwise(self, u, v=None, level=-1, stream=None):
        """v = A u in FP64 evaluated patch by patch (sipg_apply_patchwise)."""
        import torch
        v = torch.empty_like(u) if v is None else v
        _check(_lib.sipg_apply_patchwise(self._h, self._lvl(level), _ptr(u, torch.float64),
                                         _ptr(v, torch.float64), _stream(stream)))
        return v

    def apply_lp(self, u, v=None, precision="f16", ec=False, level=-1, stream=None):
        """v = A u on FP32 vectors in reduced precision ("f32", "f16", "bf16")."""
        import torch
        v = torch.empty_like(u) if v is None else v
        _check(_lib.sipg_apply_lp(self._h, self._lvl(level), _ptr(u, torch.float32),
                                  _ptr(v, torch.float32), PRECISION[precision], int(ec),
                                  _stream(stream)))
        return v

    def autotune(self, level=-1, stream=None):
        """Tile-order autotuner of the apply on `level`; returns the chosen block."""
        u = self.new_vector(level)
        v = self.new_vector(level)
        best = ctypes.c_int()
        _check(_lib.sipg_autotune(self._h, self._lvl(level), _ptr(u), _ptr(v), ctypes.byref(best),
                                  _stream(stream)))
        return best.value

    def residual(self, b, x, r=None, level=-1, stream=None):
        import torch
        r = torch.empty_like(b) if r is None else r
        _check(_lib.sipg_residual(self._h, self._lvl(level), _ptr(b, torch.float64),
                                  _ptr(x, torch.float64), _ptr(r, torch.float64), _stream(stream)))
        return r

    def smooth(self, x, b, sweeps=1, level=-1, stream=None):
        import torch
        _check(_lib.sipg_smooth(self._h, self._lvl(level), _ptr(x, torch.float64),
                                _ptr(b, torch.float64), int(sweeps), _stream(stream)))
        return x

    def smooth_lp(self, x, b, sweeps=1, level=-1, stream=None):
        """Smoother sweeps on FP32 vectors in the handle's mg_precision."""
        import torch
        _check(_lib.sipg_smooth_lp(self._h, self._lvl(level), _ptr(x, torch.float32),
                                   _ptr(b, torch.float32), int(sweeps), _stream(stream)))
        return x

    def patch_correct_lp(self, colour, r, x, level=-1, stream=None):
        import torch
        _check(_lib.sipg_patch_correct_lp(self._h, self._lvl(level), int(colour),
                                          _ptr(r, torch.float32), _ptr(x, torch.float32),
                                          _stream(stream)))
        return x

    def patch_correct(self, colour, r, x, level=-1, stream=None):
        import torch
        _check(_lib.sipg_patch_correct(self._h, self._lvl(level), int(colour),
                                       _ptr(r, torch.float64), _ptr(x, torch.float64),
                                       _stream(stream)))
        return x

    def restrict(self, rf, rc=None, level=-1, stream=None):
        import torch
        lvl = self._lvl(level)
        rc = self.new_vector(lvl - 1) if rc is None else rc
        _check(_lib.sipg_restrict(self._h, lvl, _ptr(rf, torch.float64), _ptr(rc, torch.float64),
                                  _stream(stream)))
        return rc

    def prolongate_add(self, ec, xf, level=-1, stream=None):
        import torch
        _check(_lib.sipg_prolongate_add(self._h, self._lvl(level), _ptr(ec, torch.float64),
                                        _ptr(xf, torch.float64), _stream(stream)))
        return xf

    def coarse_solve(self, b, x=None, stream=None):
        import torch
        x = torch.empty_like(b) if x is None else x
        _check(_lib.sipg_coarse_solve(self._h, _ptr(b, torch.float64), _ptr(x, torch.float64),
                                      _stream(stream)))
        return x

    def vcycle(self, x, b, level=-1, stream=None):
        import torch
        _check(_lib.sipg_vcycle(self._h, self._lvl(level), _ptr(x, torch.float64),
                                _ptr(b, torch.float64), _stream(stream)))
        return x

    def attach(self, network):
        """Use a trained Network as the learned stage (None detaches)."""
        _check(_lib.sipg_cnn_attach(self._h, network._h if network is not None else None))
        self._network = network

    def fgmres(self, b, x=None, rtol=1e-10, restart=30, max_iters=200, log_history=True,
               stream=None, raise_on_nonconvergence=True, use_learned=False, stagnation=0.0,
               variant="fgmres"):
        import torch
        x = torch.zeros_like(b) if x is None else x
        opts = SolveOpts(rtol, restart, max_iters, int(bool(use_learned)), int(log_history),
                         stagnation, VARIANT[variant])
        info = SolveInfo()
        st = _lib.sipg_fgmres(self._h, _ptr(x, torch.float64), _ptr(b, torch.float64),
                              ctypes.byref(opts), ctypes.byref(info), _stream(stream))
        if st != SIPG_OK and (raise_on_nonconvergence or st != 5):
            _check(st)
        out = dict(iterations=info.iterations, fell_back=bool(info.fell_back),
                   rel_res_est=info.rel_res_est, rel_res_true=info.rel_res_true,
                   seconds=info.seconds, status=STATUS[st],
                   history=list(info.history[:min(info.iterations + 1, 128)]))
        return x, out

    def rhs_sines(self, amps, pqr, b=None, level=-1, stream=None):
        import torch
        amps = np.ascontiguousarray(amps, dtype=np.float64).reshape(-1)
        pqr = np.ascontiguousarray(pqr, dtype=np.int32).reshape(-1, 3)
        b = self.new_vector(level) if b is None else b
        _check(_lib.sipg_rhs_sines(self._h, self._lvl(level), len(amps),
                                   amps.ctypes.data_as(ctypes.c_void_p),
                                   pqr.ctypes.data_as(ctypes.c_void_p),
                                   _ptr(b, torch.float64), _stream(stream)))
        return b

    def l2_error_sines(self, amps, pqr, x, level=-1, stream=None, noalloc=False):
        """||u - u_h||_L2 of the sine modes; noalloc=True calls the entry point
        that uses the library's fixed per-device workspace."""
        import torch
        amps = np.ascontiguousarray(amps, dtype=np.float64).reshape(-1)
        pqr = np.ascontiguousarray(pqr, dtype=np.int32).reshape(-1, 3)
        err = ctypes.c_double()
        fn = _lib.sipg_l2_error_sines_noalloc if noalloc else _lib.sipg_l2_error_sines
        _check(fn(self._h, self._lvl(level), len(amps),
                                        amps.ctypes.data_as(ctypes.c_void_p),
                                        pqr.ctypes.data_as(ctypes.c_void_p),
                                        _ptr(x, torch.float64), ctypes.byref(err),
                                        _stream(stream)))
        return err.value


def _ptr_array(ts, dtype, sizes):
    """Host array of device pointers, one vector per problem of the batch."""
    if len(ts) != len(sizes):
        raise ValueError(f"expected {len(sizes)} vectors, got {len(ts)}")
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        if t.numel() != sizes[i]:
            raise ValueError(f"vector {i} has {t.numel()} entries, problem needs {sizes[i]}")
        arr[i] = _ptr(t, dtype).value
    return arr


def _info_dict(info, status):
    return dict(iterations=info.iterations, fell_back=bool(info.fell_back),
                rel_res_est=info.rel_res_est, rel_res_true=info.rel_res_true,
                seconds=info.seconds, status=STATUS[status],
                history=list(info.history[:min(info.iterations + 1, 128)]))


class Batch:
    """Independent problems of uneven degree and size solved together
    (vectors are lists of CUDA tensors, one per problem)."""

    def __init__(self, problems, mg_precision="f64", error_correction=0, nu_pre=2, nu_post=2,
                 allocator=None, stream=None):
        lib = load_library()
        cfgs = (Config * len(problems))()
        for i, (k, n) in enumerate(problems):
            cfgs[i] = make_config(k, n, 0, mg_precision, int(error_correction), nu_pre, nu_post,
                                  allocator=allocator)
        h = ctypes.c_void_p()
        _check(lib.sipg_batch_create(cfgs, len(problems), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.problems = list(problems)
        self.sizes = []
        for i in range(len(problems)):
            ph = lib.sipg_batch_problem(h, i)
            L = lib.sipg_num_levels(ph)
            self.sizes.append(int(lib.sipg_n_dofs(ph, L - 1)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sipg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_vectors(self):
        import torch
        return [torch.zeros(m, dtype=torch.float64, device="cuda") for m in self.sizes]

    def autotune(self, stream=None):
        _check(_lib.sipg_batch_autotune(self._h, _stream(stream)))

    def apply(self, us, vs=None, stream=None):
        import torch
        vs = [torch.empty_like(u) for u in us] if vs is None else vs
        _check(_lib.sipg_batch_apply(self._h, _ptr_array(us, torch.float64, self.sizes),
                                     _ptr_array(vs, torch.float64, self.sizes), _stream(stream)))
        return vs

    def vcycle(self, xs, bs, stream=None):
        import torch
        _check(_lib.sipg_batch_vcycle(self._h, _ptr_array(xs, torch.float64, self.sizes),
                                      _ptr_array(bs, torch.float64, self.sizes), _stream(stream)))
        return xs

    def solve(self, bs, xs=None, rtol=1e-10, restart=30, max_iters=200, use_graph=True,
              sequential=False, stream=None):
        import torch
        xs = [torch.zeros_like(b) for b in bs] if xs is None else xs
        opts = SolveOpts(rtol, restart, max_iters, 0, 1, 0.0, 0)
        infos = (SolveInfo * len(bs))()
        if sequential:
            st = _lib.sipg_batch_solve_sequential(self._h, _ptr_array(xs, torch.float64, self.sizes),
                                                  _ptr_array(bs, torch.float64, self.sizes), ctypes.byref(opts),
                                                  infos, _stream(stream))
        else:
            st = _lib.sipg_batch_solve(self._h, _ptr_array(xs, torch.float64, self.sizes),
                                       _ptr_array(bs, torch.float64, self.sizes), ctypes.byref(opts), infos,
                                       2 if use_graph == "device" else int(bool(use_graph)),
                                       _stream(stream))
        if st not in (SIPG_OK, 5):
            _check(st)
        return xs, [_info_dict(infos[i], st) for i in range(len(bs))]

    def rhs_sines(self, i, amps, pqr):
        """Right-hand side of problem i (through its borrowed handle)."""
        return _BorrowedProblem(self, i).rhs_sines(amps, pqr)

    def l2_error_sines(self, i, amps, pqr, x):
        return _BorrowedProblem(self, i).l2_error_sines(amps, pqr, x)


class _BorrowedProblem(Problem):
    """View of a problem owned by a Batch (never destroyed by Python)."""

    def __init__(self, batch, i):
        lib = load_library()
        self._batch = batch
        self._h = ctypes.c_void_p(lib.sipg_batch_problem(batch._h, i))
        self.k, self.n_cells = batch.problems[i]
        self.N = self.k + 1
        self.num_levels = lib.sipg_num_levels(self._h)
        self.cells = [lib.sipg_level_cells(self._h, l) for l in range(self.num_levels)]

    def close(self):
        self._h = None


class Network:
    """The learned correction stage's network (1 -> 32 -> 32 -> 32 -> 1
    channels, 3x3x3 convolutions, ReLU), FP16 weights and activations with
    FP32 accumulation on the GPU.  Grids are CUDA float32 tensors of shape
    [batch, G, G, G] (indexed [z, y, x]), G a multiple of 16."""

    def __init__(self, seed=None):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.sipg_cnn_create(ctypes.byref(h)))
        self._h = h
        self.n_params = lib.sipg_cnn_num_params()
        if seed is not None:
            _check(lib.sipg_cnn_init(h, ctypes.c_uint64(seed)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().sipg_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        sig = ctypes.c_float()
        _check(_lib.sipg_cnn_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p), ctypes.byref(sig)))
        return p, float(sig.value)

    def set_params(self, params, sigma):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(_lib.sipg_cnn_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p), float(sigma)))

    @staticmethod
    def _grids(t):
        import torch
        if t.dtype != torch.float32 or t.dim() != 4 or not (t.shape[1] == t.shape[2] == t.shape[3]):
            raise ValueError("expected a float32 tensor [batch, G, G, G]")
        return int(t.shape[1]), int(t.shape[0])

    def forward(self, grids, stream=None):
        import torch
        G, nb = self._grids(grids)
        out = torch.empty_like(grids)
        _check(_lib.sipg_cnn_forward(self._h, G, nb, _ptr(grids, torch.float32),
                                     _ptr(out, torch.float32), _stream(stream)))
        return out

    def gradient(self, grids, targets, masks, stream=None):
        """(gradient tensor [n_params], loss) of the masked MSE."""
        import torch
        G, nb = self._grids(grids)
        for t in (targets, masks):
            if t.shape != grids.shape:
                raise ValueError("targets and masks must match the input grids")
        grad = torch.empty(self.n_params, dtype=torch.float32, device=grids.device)
        loss = torch.empty(1, dtype=torch.float32, device=grids.device)
        _check(_lib.sipg_cnn_gradient(self._h, G, nb, _ptr(grids, torch.float32),
                                      _ptr(targets, torch.float32), _ptr(masks, torch.float32),
                                      _ptr(grad, torch.float32), _ptr(loss, torch.float32),
                                      _stream(stream)))
        return grad, loss

    def gradient_residual(self, problem, rho, stream=None):
        """(gradient tensor [n_params], loss) of the residual-aware loss
        min_alpha ||rho - alpha A c||^2 / ||rho||^2, c = sigma net(rho), on the
        problem's finest level (rho: FP64 cell vector)."""
        import torch
        grad = torch.empty(self.n_params, dtype=torch.float32, device=rho.device)
        loss = torch.empty(1, dtype=torch.float32, device=rho.device)
        _check(_lib.sipg_cnn_gradient_residual(self._h, problem._h, _ptr(rho, torch.float64),
                                               _ptr(grad, torch.float32),
                                               _ptr(loss, torch.float32), _stream(stream)))
        return grad, loss

    def adam_step(self, grad, lr, stream=None):
        import torch
        if grad.numel() != self.n_params:
            raise ValueError("gradient has the wrong length")
        _check(_lib.sipg_cnn_adam_step(self._h, _ptr(grad, torch.float32), float(lr),
                                       _stream(stream)))

    @staticmethod
    def make_pairs(problem, x0, count, stream=None):
        """Solver-generated (rho / s, e / s) grids and the scales s."""
        import torch
        G = problem.cells[-1] * problem.N
        rho = torch.empty((count, G, G, G), dtype=torch.float32, device=x0.device)
        err = torch.empty_like(rho)
        sc = np.zeros(count, dtype=np.float64)
        _check(_lib.sipg_cnn_make_pairs(problem._h, _ptr(x0, torch.float64), count,
                                        _ptr(rho, torch.float32), _ptr(err, torch.float32),
                                        sc.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return rho, err, sc

    def train(self, problem, n_chains, chain_length=4, crops_per_pair=8, crop=32, lr=1e-3,
              seed=0, log_every=0, loss="mse"):
        """Train on solver-made pairs (sipg_cnn_train); loss "mse" (error
        target, random crops) or "residual" (the residual the correction
        leaves, whole grid)."""
        o = CnnTrainOpts(n_chains, chain_length, crops_per_pair, crop, lr, log_every, seed,
                         {"mse": 0, "residual": 1}[loss])
        info = CnnTrainInfo()
        _check(_lib.sipg_cnn_train(problem._h, self._h, ctypes.byref(o), ctypes.byref(info)))
        return dict(steps=info.steps, loss_first=info.loss_first, loss_last=info.loss_last,
                    sigma=info.sigma, seconds=info.seconds, seconds_pairs=info.seconds_pairs)

    def save(self, path):
        """Parameters and output scale to `path` (format of sipg_cnn_save)."""
        _check(_lib.sipg_cnn_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path):
        net = cls()
        _check(_lib.sipg_cnn_load(net._h, os.fsencode(path)))
        return net
