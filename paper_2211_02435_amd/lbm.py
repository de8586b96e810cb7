"""ctypes binding of libpaper_lbm.so (include/lbm.h): argument marshalling only.

Every computation runs in the HIP library; this module converts numpy arrays / torch tensors
into pointers, owns the torch allocations handed to the library as population buffers, and
turns status codes into exceptions.  Function names follow the C ABI.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpaper_lbm.so")

LBM_OK, LBM_EINVAL, LBM_EUNSUPPORTED, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE = 0, -1, -2, -3, -4, -5
STENCILS = {"D2Q9": 0, "D3Q19": 1, "D3Q27": 2, "D3Q15": 3}
SPACES = {"raw": 0, "central": 1, "cumulant": 2, "srt": 3}
EQUILIBRIA = {"maxwellian": 0, "swe": 1, "swe_maxwellian": 2}
EQ_FORMS = {"default": 0, "absolute": 1, "delta": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
STREAMING = {"pull": 0, "aa": 1, "esoteric": 2, "twist": 3, "push": 4}
LAYOUTS = {"auto": 0, "planes": 1, "rows": 2}
ARITHMETIC = {"deviation": 0, "literal": 1}
FORCE_MODELS = {"guo": 0, "he": 1}
BASES = {"graded": 0, "weighted_orthogonal": 1, "orthogonal": 2}
Q = {"D2Q9": 9, "D3Q19": 19, "D3Q27": 27, "D3Q15": 15}
# order of every polynomial of the bases documented in lbm.h (one rate per entry of omegas)
BASIS_ORDERS = {
    "D2Q9": [0, 1, 1, 2, 2, 2, 3, 3, 4],
    "D3Q19": [0, 1, 1, 1] + [2] * 6 + [3] * 6 + [4] * 3,
    "D3Q27": [0, 1, 1, 1] + [2] * 6 + [3] * 6 + [3] + [4] * 3 + [4] * 3 + [5] * 3 + [6],
    "D3Q15": [0, 1, 1, 1] + [2] * 6 + [3] * 4 + [4],
}
# positions of the shear polynomials (xy, xz, yz, x2-y2, x2-z2) and of the trace x2+y2(+z2)
SHEAR = {"D2Q9": [3, 4], "D3Q19": [4, 5, 6, 7, 8], "D3Q27": [4, 5, 6, 7, 8], "D3Q15": [4, 5, 6, 7, 8]}
TRACE = {"D2Q9": 5, "D3Q19": 9, "D3Q27": 9, "D3Q15": 9}


def regularized_rates(stencil, omega_shear, omega_bulk=1.0):
    """Rates of an "R-" method (sec. 4.3) in the basis order of lbm.h: omega_shear on the shear
    polynomials, omega_bulk on the trace, 1 on every higher-order polynomial, 0 on the conserved
    ones (ignored by the library)."""
    om = np.ones(Q[stencil])
    om[[k for k, o in enumerate(BASIS_ORDERS[stencil]) if o < 2]] = 0.0
    om[SHEAR[stencil]] = omega_shear
    om[TRACE[stencil]] = omega_bulk
    return om
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}


class LbmParams(ctypes.Structure):
    _fields_ = [("stencil", c_int), ("space", c_int), ("equilibrium", c_int), ("eq_form", c_int),
                ("zero_centered", c_int), ("omegas", POINTER(c_double)), ("n_omegas", c_int),
                ("gravity", c_double), ("nx", c_int64), ("ny", c_int64), ("nz", c_int64),
                ("periodic", c_int * 3), ("storage", c_int), ("streaming", c_int),
                ("buffers", c_void_p * 2), ("buffer_bytes", c_size_t), ("stream", c_void_p),
                ("layout", c_int), ("arithmetic", c_int), ("force", c_double * 3), ("force_model", c_int),
                ("basis", c_int)]


class LbmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("lbm status %d: %s" % (status, message))
        self.status = status


# name -> (restype, argtypes); every symbol declared in include/lbm.h
SIGNATURES = {
    "lbm_params_default": (c_int, [POINTER(LbmParams)]),
    "lbm_validate": (c_int, [POINTER(LbmParams)]),
    "lbm_required_bytes": (c_int, [POINTER(LbmParams), POINTER(c_size_t)]),
    "lbm_create": (c_int, [POINTER(LbmParams), POINTER(c_void_p)]),
    "lbm_destroy": (None, [c_void_p]),
    "lbm_init_equilibrium": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lbm_step": (c_int, [c_void_p, c_int64]),
    "lbm_graph_prepare": (c_int, [c_void_p, c_int64]),
    "lbm_macroscopic": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lbm_get_populations": (c_int, [c_void_p, c_void_p]),
    "lbm_set_populations": (c_int, [c_void_p, c_void_p]),
    "lbm_set_force_field": (c_int, [c_void_p, c_void_p]),
    "lbm_diagnostics": (c_int, [c_void_p, POINTER(c_double)]),
    "lbm_diagnostics_noalloc": (c_int, [c_void_p, c_void_p]),
    "lbm_synchronize": (c_int, [c_void_p]),
    "lbm_time": (c_int64, [c_void_p]),
    "lbm_set_time": (c_int, [c_void_p, c_int64]),
    "lbm_set_launch": (c_int, [c_void_p, c_int, c_int, c_int]),
    "lbm_get_launch": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
    "lbm_set_vectorized": (c_int, [c_void_p, c_int]),
    "lbm_get_vectorized": (c_int, [c_void_p]),
    "lbm_set_staged": (c_int, [c_void_p, c_int]),
    "lbm_get_staged": (c_int, [c_void_p]),
    "lbm_set_transform": (c_int, [c_void_p, c_int]),
    "lbm_get_transform": (c_int, [c_void_p]),
    "lbm_get_layout": (c_int, [c_void_p]),
    "lbm_set_lds_reserve": (c_int, [c_void_p, c_int]),
    "lbm_get_lds_reserve": (c_int, [c_void_p]),
    "lbm_autotune": (c_int, [c_void_p]),
    "lbm_set_graphs": (c_int, [c_void_p, c_int]),
    "lbm_buffer": (c_int, [c_void_p, c_int, POINTER(c_void_p), POINTER(c_size_t)]),
    "lbm_time_steps": (c_int, [c_void_p, c_int64, POINTER(c_double)]),
    "lbm_last_error": (c_char_p, []),
    "lbm_version": (c_char_p, []),
    "lbm_batch_create": (c_int, [POINTER(LbmParams), c_int, c_void_p, c_void_p, POINTER(c_void_p)]),
    "lbm_batch_destroy": (None, [c_void_p]),
    "lbm_batch_init_equilibrium": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lbm_batch_step": (c_int, [c_void_p, c_int64]),
    "lbm_batch_graph_prepare": (c_int, [c_void_p, c_int64]),
    "lbm_batch_macroscopic": (c_int, [c_void_p, c_void_p, c_void_p]),
    "lbm_batch_get_populations": (c_int, [c_void_p, c_void_p]),
    "lbm_batch_get_box_populations": (c_int, [c_void_p, c_int, c_void_p]),
    "lbm_batch_synchronize": (c_int, [c_void_p]),
    "lbm_batch_cells": (c_int64, [c_void_p]),
    "lbm_batch_set_graphs": (c_int, [c_void_p, c_int]),
    "lbm_batch_time_steps": (c_int, [c_void_p, c_int64, POINTER(c_double)]),
    "lbm_batch_set_launch": (c_int, [c_void_p, c_int, c_int, c_int]),
    "lbm_batch_get_launch": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int), POINTER(c_int)]),
    "lbm_batch_autotune": (c_int, [c_void_p]),
    "lbm_batch_set_persistent": (c_int, [c_void_p, c_int]),
    "lbm_batch_get_persistent": (c_int, [c_void_p]),
    "lbm_copy_bandwidth": (c_int, [c_void_p, c_void_p, c_size_t, c_int, c_void_p, POINTER(c_double)]),
    "lbm_debug_stream_only": (c_int, [c_void_p, c_int64]),
}

_lib = None


def load():
    """Load the HIP library; raises if it has not been built (there is no fallback).

    PyTorch is imported first.  Its ROCm build carries its own HIP runtime, which its libraries
    request under another file name than the library's dependency; loaded first, the library
    would pull in the system runtime and torch would then add its own, leaving two HIP runtimes
    (and two HSA runtimes) in the process, and the one initialised second reports no device.
    Imported first, torch's runtime is the one the library binds to."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libpaper_lbm.so not found at %s; build it with __graft_entry__.build()" % LIB_PATH)
        import torch  # noqa: F401
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def last_error():
    return load().lbm_last_error().decode()


def check(status):
    if status != LBM_OK:
        raise LbmError(status, last_error())


def _dptr(a):
    """Pointer of a numpy array (host) or torch tensor (host or device)."""
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return c_void_p(a.ctypes.data)
    return c_void_p(a.data_ptr())


def make_params(stencil, space, omegas, dims, storage="f32", streaming="pull", equilibrium="maxwellian",
                eq_form="default", gravity=0.0, zero_centered=1, layout="auto", arithmetic="deviation",
                force=(0.0, 0.0, 0.0), force_model="guo", basis="graded"):
    p = LbmParams()
    check(load().lbm_params_default(ctypes.byref(p)))
    p.stencil = STENCILS[stencil]
    p.space = SPACES[space]
    p.equilibrium = EQUILIBRIA[equilibrium]
    p.eq_form = EQ_FORMS[eq_form]
    p.zero_centered = zero_centered
    om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64))
    p._omegas_keep = om
    p.omegas = om.ctypes.data_as(POINTER(c_double))
    p.n_omegas = om.shape[0]
    p.gravity = gravity
    p.nx, p.ny, p.nz = (int(v) for v in dims)
    p.storage = STORAGE[storage]
    p.streaming = STREAMING[streaming]
    p.layout = LAYOUTS[layout]
    p.arithmetic = ARITHMETIC[arithmetic]
    for d in range(3):
        p.force[d] = float(force[d])
    p.force_model = FORCE_MODELS[force_model]
    p.basis = BASES[basis]
    return p


def lbm_validate(p):
    return load().lbm_validate(ctypes.byref(p))


def lbm_required_bytes(p):
    n = c_size_t(0)
    check(load().lbm_required_bytes(ctypes.byref(p), ctypes.byref(n)))
    return n.value


class Lattice:
    """One periodic box advanced by the HIP sweep.

    dims = (nx, ny, nz).  Population buffers are torch CUDA allocations owned by this object
    (torch_buffers=True) or by the library.  Work runs on a torch stream of default priority."""

    def __init__(self, stencil, space, omegas, dims, storage="f32", streaming="pull",
                 equilibrium="maxwellian", eq_form="default", gravity=0.0, torch_buffers=True, layout="auto",
                 zero_centered=True, arithmetic="deviation", force=(0.0, 0.0, 0.0), force_model="guo",
                 basis="graded"):
        import torch
        self.lib = load()
        self.stencil, self.space, self.storage, self.streaming = stencil, space, storage, streaming
        self.q = Q[stencil]
        self.dims = tuple(int(v) for v in dims)
        self.ncells = self.dims[0] * self.dims[1] * self.dims[2]
        p = make_params(stencil, space, omegas, dims, storage, streaming, equilibrium, eq_form, gravity,
                        zero_centered=1 if zero_centered else 0, layout=layout, arithmetic=arithmetic,
                        force=force, force_model=force_model, basis=basis)
        self._torch_stream = torch.cuda.Stream()
        p.stream = c_void_p(self._torch_stream.cuda_stream)
        self._bufs = []
        if torch_buffers:
            total = lbm_required_bytes(p)
            nbuf = 2 if streaming in ("pull", "push") else 1  # the in-place patterns use one array
            per = total // nbuf
            for k in range(nbuf):
                t = torch.empty(per, dtype=torch.uint8, device="cuda")
                self._bufs.append(t)
                p.buffers[k] = t.data_ptr()
            p.buffer_bytes = per
            torch.cuda.synchronize()
        self._params = p
        ctx = c_void_p()
        check(self.lib.lbm_create(ctypes.byref(p), ctypes.byref(ctx)))
        self.ctx = ctx

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            self.lib.lbm_destroy(ctx)
            self.ctx = None

    def close(self):
        self.__del__()

    # --- C ABI, same names ---------------------------------------------------------------
    def lbm_init_equilibrium(self, rho, u):
        rho = np.ascontiguousarray(rho, dtype=np.float64) if isinstance(rho, np.ndarray) else rho
        u = np.ascontiguousarray(u, dtype=np.float64) if isinstance(u, np.ndarray) else u
        check(self.lib.lbm_init_equilibrium(self.ctx, _dptr(rho), _dptr(u)))

    def lbm_step(self, n=1):
        check(self.lib.lbm_step(self.ctx, int(n)))

    def lbm_graph_prepare(self, n):
        check(self.lib.lbm_graph_prepare(self.ctx, int(n)))

    def lbm_debug_stream_only(self, n=1):
        check(self.lib.lbm_debug_stream_only(self.ctx, int(n)))

    def lbm_macroscopic(self):
        nx, ny, nz = self.dims
        rho = np.empty((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        check(self.lib.lbm_macroscopic(self.ctx, _dptr(rho), _dptr(u)))
        return rho, u

    def lbm_get_populations(self):
        nx, ny, nz = self.dims
        df = np.empty((self.q, nz, ny, nx))
        check(self.lib.lbm_get_populations(self.ctx, _dptr(df)))
        return df

    def lbm_set_populations(self, df):
        df = np.ascontiguousarray(df, dtype=np.float64)
        assert df.size == self.q * self.ncells
        check(self.lib.lbm_set_populations(self.ctx, _dptr(df)))

    def lbm_set_force_field(self, F):
        """F: (3, nz, ny, nx) FP64 body force per cell (numpy or torch), or None to remove it."""
        if F is None:
            check(self.lib.lbm_set_force_field(self.ctx, None))
            return
        if isinstance(F, np.ndarray):
            F = np.ascontiguousarray(F, dtype=np.float64)
            assert F.size == 3 * self.ncells
        check(self.lib.lbm_set_force_field(self.ctx, _dptr(F)))

    def lbm_diagnostics(self, allow_nonfinite=False):
        out = (c_double * 6)()
        s = self.lib.lbm_diagnostics(self.ctx, out)
        if not (allow_nonfinite and s == LBM_ENONFINITE):
            check(s)
        return np.array(out[:])

    def lbm_diagnostics_noalloc(self, out=None, allow_nonfinite=False):
        """Allocation-free diagnostics: into `out` (a device tensor of 6 doubles; asynchronous)
        or, without `out`, into a host array (synchronous)."""
        if out is not None:
            check(self.lib.lbm_diagnostics_noalloc(self.ctx, _dptr(out)))
            return out
        host = np.empty(6)
        s = self.lib.lbm_diagnostics_noalloc(self.ctx, _dptr(host))
        if not (allow_nonfinite and s == LBM_ENONFINITE):
            check(s)
        return host

    def lbm_synchronize(self):
        check(self.lib.lbm_synchronize(self.ctx))

    def lbm_time(self):
        return int(self.lib.lbm_time(self.ctx))

    def lbm_set_time(self, t):
        check(self.lib.lbm_set_time(self.ctx, int(t)))

    def lbm_set_launch(self, bx, by, swizzle=0):
        check(self.lib.lbm_set_launch(self.ctx, bx, by, swizzle))

    def lbm_get_launch(self):
        a, b, c = c_int(), c_int(), c_int()
        check(self.lib.lbm_get_launch(self.ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def lbm_set_vectorized(self, enable):
        check(self.lib.lbm_set_vectorized(self.ctx, 1 if enable else 0))

    def lbm_get_vectorized(self):
        return bool(self.lib.lbm_get_vectorized(self.ctx))

    def lbm_set_staged(self, enable):
        check(self.lib.lbm_set_staged(self.ctx, 1 if enable else 0))

    def lbm_get_staged(self):
        return bool(self.lib.lbm_get_staged(self.ctx))

    def lbm_set_transform(self, transform):
        check(self.lib.lbm_set_transform(self.ctx, {"chimera": 0, "dense_mfma": 1}[transform]))

    def lbm_get_layout(self):
        return {1: "planes", 2: "rows"}[int(self.lib.lbm_get_layout(self.ctx))]

    def lbm_get_transform(self):
        return {0: "chimera", 1: "dense_mfma"}[int(self.lib.lbm_get_transform(self.ctx))]

    def lbm_set_lds_reserve(self, nbytes):
        check(self.lib.lbm_set_lds_reserve(self.ctx, int(nbytes)))

    def lbm_get_lds_reserve(self):
        return int(self.lib.lbm_get_lds_reserve(self.ctx))

    def lbm_autotune(self):
        check(self.lib.lbm_autotune(self.ctx))

    def lbm_set_graphs(self, enable):
        check(self.lib.lbm_set_graphs(self.ctx, 1 if enable else 0))

    def lbm_buffer(self, k):
        p, n = c_void_p(), c_size_t()
        check(self.lib.lbm_buffer(self.ctx, k, ctypes.byref(p), ctypes.byref(n)))
        return p.value, n.value

    def lbm_time_steps(self, n):
        ms = c_double()
        check(self.lib.lbm_time_steps(self.ctx, int(n), ctypes.byref(ms)))
        return ms.value


class Batch:
    """Ensemble of independent periodic boxes advanced by one launch per step."""

    def __init__(self, stencil, space, dims_list, omegas_list, storage="f32", equilibrium="maxwellian",
                 eq_form="default"):
        import torch
        self.lib = load()
        self.q = Q[stencil]
        self.dims = [tuple(int(v) for v in d) for d in dims_list]
        self.ncells = [d[0] * d[1] * d[2] for d in self.dims]
        p = make_params(stencil, space, omegas_list[0], self.dims[0], storage, "pull", equilibrium, eq_form)
        self._torch_stream = torch.cuda.Stream()
        p.stream = c_void_p(self._torch_stream.cuda_stream)
        dims = np.ascontiguousarray(np.array(self.dims, dtype=np.int64))
        om = np.ascontiguousarray(np.array(omegas_list, dtype=np.float64))
        assert om.shape == (len(self.dims), self.q)
        b = c_void_p()
        check(self.lib.lbm_batch_create(ctypes.byref(p), len(self.dims), _dptr(dims), _dptr(om), ctypes.byref(b)))
        self.b = b

    def __del__(self):
        b = getattr(self, "b", None)
        if b is not None and b.value:
            self.lib.lbm_batch_destroy(b)
            self.b = None

    def lbm_batch_init_equilibrium(self, rho_cat, u_cat):
        rho_cat = np.ascontiguousarray(rho_cat, dtype=np.float64)
        u_cat = np.ascontiguousarray(u_cat, dtype=np.float64)
        check(self.lib.lbm_batch_init_equilibrium(self.b, _dptr(rho_cat), _dptr(u_cat)))

    def lbm_batch_step(self, n=1):
        check(self.lib.lbm_batch_step(self.b, int(n)))

    def lbm_batch_graph_prepare(self, n):
        check(self.lib.lbm_batch_graph_prepare(self.b, int(n)))

    def lbm_batch_macroscopic(self):
        n = sum(self.ncells)
        rho = np.empty(n)
        u = np.empty(3 * n)
        check(self.lib.lbm_batch_macroscopic(self.b, _dptr(rho), _dptr(u)))
        return rho, u

    def lbm_batch_get_populations(self):
        df = np.empty(self.q * sum(self.ncells))
        check(self.lib.lbm_batch_get_populations(self.b, _dptr(df)))
        return df

    def lbm_batch_get_box_populations(self, k):
        nx, ny, nz = self.dims[k]
        df = np.empty((self.q, nz, ny, nx))
        check(self.lib.lbm_batch_get_box_populations(self.b, int(k), _dptr(df)))
        return df

    def lbm_batch_synchronize(self):
        check(self.lib.lbm_batch_synchronize(self.b))

    def lbm_batch_cells(self):
        return int(self.lib.lbm_batch_cells(self.b))

    def lbm_batch_set_launch(self, threads, swizzle=1, lds_bytes=0):
        check(self.lib.lbm_batch_set_launch(self.b, int(threads), int(swizzle), int(lds_bytes)))

    def lbm_batch_get_launch(self):
        t, s, l = c_int(), c_int(), c_int()
        check(self.lib.lbm_batch_get_launch(self.b, ctypes.byref(t), ctypes.byref(s), ctypes.byref(l)))
        return t.value, s.value, l.value

    def lbm_batch_set_persistent(self, enable):
        check(self.lib.lbm_batch_set_persistent(self.b, 1 if enable else 0))

    def lbm_batch_get_persistent(self):
        return bool(self.lib.lbm_batch_get_persistent(self.b))

    def lbm_batch_autotune(self):
        check(self.lib.lbm_batch_autotune(self.b))
        return self.lbm_batch_get_launch()

    def lbm_batch_set_graphs(self, enable):
        check(self.lib.lbm_batch_set_graphs(self.b, 1 if enable else 0))

    def lbm_batch_time_steps(self, n):
        ms = c_double()
        check(self.lib.lbm_batch_time_steps(self.b, int(n), ctypes.byref(ms)))
        return ms.value


def lbm_copy_bandwidth(dst, src, nbytes, reps, stream=None):
    ms = c_double()
    check(load().lbm_copy_bandwidth(_dptr(dst), _dptr(src), int(nbytes), int(reps),
                                    c_void_p(stream), ctypes.byref(ms)))
    return ms.value
