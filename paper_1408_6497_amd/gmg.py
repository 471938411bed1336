"""Thin ctypes binding of libgmg.so (include/gmg.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  Device buffers are torch tensors on the GPU (passed by data_ptr());
torch is used for device memory and the stream, nothing else.  If the library
is not built, every call raises: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmg.so")

GMG_FP64 = 0
GMG_FP32 = 1

_STATUS = {
    0: "GMG_OK", 1: "GMG_E_ARG", 2: "GMG_E_MESH", 3: "GMG_E_OOM", 4: "GMG_E_HIP",
    5: "GMG_E_NOCONV", 6: "GMG_E_BREAKDOWN", 7: "GMG_E_STATE",
}

EXPORTS = [
    "gmg_setup", "gmg_destroy", "gmg_num_levels", "gmg_num_dofs", "gmg_dof_coords_1d", "gmg_lambda",
    "gmg_diagonal", "gmg_apply", "gmg_mass", "gmg_smooth", "gmg_restrict", "gmg_prolong",
    "gmg_coarse_solve", "gmg_vcycle", "gmg_rhs", "gmg_solve", "gmg_solve_rhs", "gmg_fft_solve", "gmg_dot",
    "gmg_timing_get", "gmg_timing_reset", "gmg_history", "gmg_status_string", "gmg_last_error",
    "gmg_net_set_weights", "gmg_set_learned", "gmg_net_get_weights", "gmg_net_cache_bytes", "gmg_net_forward",
    "gmg_net_backward", "gmg_adam_step", "gmg_net_correction", "gmg_net_loss_grad", "gmg_residual",
    "gmg_octree_refine_gaussians", "gmg_octree_refine_sharp_layer", "gmg_octree_balance", "gmg_level_leaves", "gmg_num_elements", "gmg_dof_coords",
    "gmg_net_get_state", "gmg_net_set_state", "gmg_smooth_zero", "gmg_launch_shape",
    "gmg_dot_noalloc", "gmg_spectral_create", "gmg_spectral_solve", "gmg_spectral_destroy",
]

NET_WEIGHTS = 7776
LOSS_ENERGY, LOSS_RESIDUAL = 0, 1


class GmgMesh(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("n", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_leaves", ctypes.c_int64),
                ("leaf_morton", ctypes.POINTER(ctypes.c_uint64)), ("leaf_level", ctypes.POINTER(ctypes.c_uint8))]


class GmgOptions(ctypes.Structure):
    _fields_ = [
        ("cheb_degree", ctypes.c_int32), ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32),
        ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
        ("lanczos_steps", ctypes.c_int32), ("smoother", ctypes.c_int32), ("jacobi_omega", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("vcycle_prec", ctypes.c_int32), ("krylov", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double), ("max_iters", ctypes.c_int32), ("lambda_override", ctypes.c_double),
        ("timing", ctypes.c_int32), ("no_graphs", ctypes.c_int32),
        ("ir_mode", ctypes.c_int32), ("use_learned", ctypes.c_int32),
        ("learned_depths", ctypes.c_int32), ("no_fused_tail", ctypes.c_int32),
        ("learned_min_depth", ctypes.c_int32), ("no_speculation", ctypes.c_int32),
        ("no_fused_transfer", ctypes.c_int32), ("no_fused_test_norms", ctypes.c_int32),
        ("q4_mfma", ctypes.c_int32),
    ]


class GmgInfo(ctypes.Structure):
    _fields_ = [
        ("outer_iters", ctypes.c_int32), ("inner_iters", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("rel_residual_f64", ctypes.c_double), ("t_setup", ctypes.c_double),
        ("t_solve", ctypes.c_double), ("t_smooth", ctypes.c_double), ("t_transfer", ctypes.c_double),
        ("t_coarse", ctypes.c_double), ("t_learned", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class GmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libgmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "gmg_setup": [ctypes.POINTER(GmgMesh), ctypes.POINTER(GmgOptions), P, ctypes.POINTER(P)],
        "gmg_destroy": [P],
        "gmg_num_levels": [P, ctypes.POINTER(I32)],
        "gmg_num_dofs": [P, I32, ctypes.POINTER(I64)],
        "gmg_dof_coords_1d": [P, I32, P],
        "gmg_lambda": [P, I32, ctypes.POINTER(D)],
        "gmg_diagonal": [P, I32, P],
        "gmg_apply": [P, I32, I32, P, P],
        "gmg_mass": [P, I32, I32, P, P],
        "gmg_smooth": [P, I32, I32, P, P, I32],
        "gmg_restrict": [P, I32, I32, P, P],
        "gmg_prolong": [P, I32, I32, P, P],
        "gmg_coarse_solve": [P, I32, P, P],
        "gmg_vcycle": [P, I32, P, P],
        "gmg_rhs": [P, P, P],
        "gmg_solve": [P, P, P, D, ctypes.POINTER(GmgInfo)],
        "gmg_solve_rhs": [P, P, P, D, ctypes.POINTER(GmgInfo)],
        "gmg_fft_solve": [P, P, P],
        "gmg_dot": [P, I32, I64, P, P, ctypes.POINTER(D)],
        "gmg_timing_get": [P, I32, I32, I32, ctypes.POINTER(I64), ctypes.POINTER(D)],
        "gmg_timing_reset": [P],
        "gmg_history": [P, I32, P, I64, ctypes.POINTER(I64)],
        "gmg_octree_refine_gaussians": [I32, I32, I32, P, P, P, D, P, P, I64, ctypes.POINTER(I64)],
        "gmg_octree_refine_sharp_layer": [I32, I32, P, D, D, D, P, P, I64, ctypes.POINTER(I64)],
        "gmg_octree_balance": [P, P, I64, P, P, I64, ctypes.POINTER(I64)],
        "gmg_level_leaves": [P, I32, P, P, I64, ctypes.POINTER(I64)],
        "gmg_num_elements": [P, I32, ctypes.POINTER(I64)],
        "gmg_dof_coords": [P, I32, P],
        "gmg_net_get_state": [P, I32, P, P, P],
        "gmg_net_set_state": [P, I32, P, P, P],
        "gmg_net_set_weights": [P, I32, P, I64],
        "gmg_set_learned": [P, I32, P, I64],
        "gmg_net_get_weights": [P, I32, P, I64],
        "gmg_net_cache_bytes": [P, I32, ctypes.POINTER(I64)],
        "gmg_net_forward": [P, I32, P, P, P],
        "gmg_net_backward": [P, I32, P, P, P, P],
        "gmg_adam_step": [P, I32, P, ctypes.c_float, I64],
        "gmg_net_correction": [P, I32, P, P],
        "gmg_net_loss_grad": [P, I32, I32, P, P, P, P, ctypes.c_float, ctypes.POINTER(D)],
        "gmg_residual": [P, I32, I32, P, P, P],
        "gmg_smooth_zero": [P, I32, I32, P, P, I32],
        "gmg_launch_shape": [P, I32, I32, I32, P],
        "gmg_dot_noalloc": [P, I32, I64, P, P, P],
        "gmg_spectral_create": [I32, P, ctypes.POINTER(P)],
        "gmg_spectral_solve": [P, P, P],
        "gmg_spectral_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.gmg_status_string.argtypes = [ctypes.c_int]
    lib.gmg_status_string.restype = ctypes.c_char_p
    lib.gmg_last_error.argtypes = [P]
    lib.gmg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Owns one gmg_ctx (a multigrid hierarchy on the current HIP device)."""

    def __init__(self, order, n, levels=0, stream=None, leaves=None, **opts):
        """Uniform mesh of n^3 elements, or (n = 0) the octree leaves = (morton uint64, level uint8)."""
        import numpy as np
        import torch
        self._torch = torch
        self.lib = load()
        mesh = GmgMesh(order=order, n=n, levels=levels, reserved=0)
        if leaves is not None:
            keys = np.ascontiguousarray(leaves[0], dtype=np.uint64)
            lev = np.ascontiguousarray(leaves[1], dtype=np.uint8)
            if n != 0 or keys.shape != lev.shape:
                raise ValueError("octree meshes take n = 0 and equal-length key / level arrays")
            self._leaf_arrays = (keys, lev)
            mesh.n_leaves = keys.size
            mesh.leaf_morton = keys.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
            mesh.leaf_level = lev.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        o = GmgOptions()
        for k, v in opts.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        st = self.lib.gmg_setup(ctypes.byref(mesh), ctypes.byref(o), ctypes.c_void_p(stream.cuda_stream),
                                ctypes.byref(h))
        if st != 0:
            raise GmgError(st, "gmg_setup failed")
        self.h = h
        self.order = order
        self.n = n
        nl = ctypes.c_int32()
        self._check(self.lib.gmg_num_levels(self.h, ctypes.byref(nl)))
        self.levels = nl.value

    def _check(self, st):
        if st != 0:
            msg = self.lib.gmg_last_error(self.h) if getattr(self, "h", None) else b""
            raise GmgError(st, (msg or b"").decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.gmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries
    def num_dofs(self, level=-1):
        level = self._lvl(level)
        v = ctypes.c_int64()
        self._check(self.lib.gmg_num_dofs(self.h, level, ctypes.byref(v)))
        return v.value

    def num_elements(self, level=-1):
        v = ctypes.c_int64()
        self._check(self.lib.gmg_num_elements(self.h, self._lvl(level), ctypes.byref(v)))
        return v.value

    def dof_coords(self, level=-1):
        """(n, 3) DoF coordinates (x, y, z) of a level."""
        import numpy as np
        level = self._lvl(level)
        out = np.zeros((self.num_dofs(level), 3), dtype=np.float64)
        self._check(self.lib.gmg_dof_coords(self.h, level, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def level_leaves(self, level=-1):
        """(morton, level) arrays of an octree level."""
        import numpy as np
        level = self._lvl(level)
        cnt = ctypes.c_int64()
        self.lib.gmg_level_leaves(self.h, level, None, None, 0, ctypes.byref(cnt))
        keys = np.zeros(cnt.value, dtype=np.uint64)
        lev = np.zeros(cnt.value, dtype=np.uint8)
        self._check(self.lib.gmg_level_leaves(self.h, level, keys.ctypes.data_as(ctypes.c_void_p),
                                              lev.ctypes.data_as(ctypes.c_void_p), cnt.value, ctypes.byref(cnt)))
        return keys, lev

    def lattice(self, level=-1):
        return round(self.num_dofs(level) ** (1.0 / 3.0))

    def dof_coords_1d(self, level=-1):
        import numpy as np
        level = self._lvl(level)
        x = np.zeros(self.lattice(level), dtype=np.float64)
        self._check(self.lib.gmg_dof_coords_1d(self.h, level, x.ctypes.data_as(ctypes.c_void_p)))
        return x

    def lam(self, level=-1):
        v = ctypes.c_double()
        self._check(self.lib.gmg_lambda(self.h, self._lvl(level), ctypes.byref(v)))
        return v.value

    def _lvl(self, level):
        return level + self.levels if level < 0 else level

    def _vec(self, t, level, prec=None):
        torch = self._torch
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("expected a contiguous GPU tensor")
        if prec is not None:
            want = torch.float32 if prec == GMG_FP32 else torch.float64
            if t.dtype != want:
                raise ValueError(f"expected dtype {want}, got {t.dtype}")
        if level is not None and t.numel() != self.num_dofs(level):
            raise ValueError(f"expected {self.num_dofs(level)} values, got {t.numel()}")
        return _ptr(t)

    @staticmethod
    def prec_of(t):
        import torch
        return GMG_FP32 if t.dtype == torch.float32 else GMG_FP64

    # -- operations (enqueued on the context stream)
    def diagonal(self, level, d):
        level = self._lvl(level)
        self._check(self.lib.gmg_diagonal(self.h, level, self._vec(d, level, GMG_FP64)))

    def apply(self, level, x, y):
        level = self._lvl(level)
        p = self.prec_of(x)
        self._check(self.lib.gmg_apply(self.h, level, p, self._vec(x, level, p), self._vec(y, level, p)))

    def mass(self, level, x, y):
        level = self._lvl(level)
        p = self.prec_of(x)
        self._check(self.lib.gmg_mass(self.h, level, p, self._vec(x, level, p), self._vec(y, level, p)))

    def smooth(self, level, b, u, nu):
        level = self._lvl(level)
        p = self.prec_of(b)
        self._check(self.lib.gmg_smooth(self.h, level, p, self._vec(b, level, p), self._vec(u, level, p), nu))

    def smooth_zero(self, level, b, u, nu):
        """u = S^nu(0; b): the smoother from a zero initial guess (u is not read)."""
        level = self._lvl(level)
        p = self.prec_of(b)
        self._check(self.lib.gmg_smooth_zero(self.h, level, p, self._vec(b, level, p), self._vec(u, level, p), nu))

    SHAPE_OPS = {"apply": 0, "residual": 1, "smooth": 2, "smooth_zero": 3, "restrict": 4, "prolong": 5}
    SHAPE_KERNELS = {0: "point", 1: "column", 2: "column_preload", 3: "transfer_fused", 4: "transfer_axis",
                     5: "octree", 6: "generic", 7: "column_mfma"}

    def launch_shape(self, level, prec, op):
        """(kernel name, G, TZ, blocks) of the launch an operation takes on a level."""
        level = self._lvl(level)
        out = (ctypes.c_int32 * 4)()
        self._check(self.lib.gmg_launch_shape(self.h, level, prec, self.SHAPE_OPS[op], out))
        return self.SHAPE_KERNELS[out[0]], out[1], out[2], out[3]

    def restrict(self, level, rf, rc):
        level = self._lvl(level)
        p = self.prec_of(rf)
        self._check(self.lib.gmg_restrict(self.h, level, p, self._vec(rf, level, p), self._vec(rc, level - 1, p)))

    def prolong(self, level, ec, uf):
        level = self._lvl(level)
        p = self.prec_of(ec)
        self._check(self.lib.gmg_prolong(self.h, level, p, self._vec(ec, level - 1, p), self._vec(uf, level, p)))

    def coarse_solve(self, b, x):
        p = self.prec_of(b)
        self._check(self.lib.gmg_coarse_solve(self.h, p, self._vec(b, 0, p), self._vec(x, 0, p)))

    def vcycle(self, r, z):
        p = self.prec_of(r)
        lv = self.levels - 1
        self._check(self.lib.gmg_vcycle(self.h, p, self._vec(r, lv, p), self._vec(z, lv, p)))

    def rhs(self, f, b):
        lv = self.levels - 1
        self._check(self.lib.gmg_rhs(self.h, self._vec(f, lv, GMG_FP64), self._vec(b, lv, GMG_FP64)))

    def dot(self, x, y):
        v = ctypes.c_double()
        p = self.prec_of(x)
        self._check(self.lib.gmg_dot(self.h, p, x.numel(), self._vec(x, None, p), self._vec(y, None, p),
                                     ctypes.byref(v)))
        return v.value

    def dot_noalloc(self, x, y, out):
        """out[0] = x . y in FP64 (out: one float64 GPU element), enqueued without allocating."""
        p = self.prec_of(x)
        if out.dtype != self._torch.float64 or out.numel() < 1 or not out.is_cuda:
            raise ValueError("out must be a float64 GPU tensor with at least one element")
        self._check(self.lib.gmg_dot_noalloc(self.h, p, x.numel(), self._vec(x, None, p), self._vec(y, None, p),
                                             _ptr(out)))

    # -- launch timing (needs timing=1 at construction)
    (KIND_APPLY, KIND_RESIDUAL, KIND_SMOOTH0, KIND_SMOOTH, KIND_MASS, KIND_RESTRICT, KIND_PROLONG, KIND_COARSE,
     KIND_LEARNED, KIND_SCALE, KIND_SMOOTHZ, KIND_TAIL) = range(12)

    def timing(self, level, kind, prec):
        """(launches, seconds) of one level / kind / precision since the last reset."""
        cnt, sec = ctypes.c_int64(), ctypes.c_double()
        self._check(self.lib.gmg_timing_get(self.h, self._lvl(level), kind, prec, ctypes.byref(cnt),
                                            ctypes.byref(sec)))
        return cnt.value, sec.value

    def timing_reset(self):
        self._check(self.lib.gmg_timing_reset(self.h))

    def history(self, kind=0):
        """Last solve: kind 0 Krylov residual norms; kind 1 (rho_L, rho_ref, rho_plain) rows."""
        import numpy as np
        cnt = ctypes.c_int64()
        self._check(self.lib.gmg_history(self.h, kind, None, 0, ctypes.byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.float64)
        if cnt.value:
            self._check(self.lib.gmg_history(self.h, kind, out.ctypes.data_as(ctypes.c_void_p), cnt.value,
                                             ctypes.byref(cnt)))
        return out.reshape(-1, 3) if kind == 1 else out

    # -- learned smoother (depth 0 = finest level)
    def net_set_weights(self, depth, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.size != NET_WEIGHTS:
            raise ValueError("expected 7776 weights")
        self._check(self.lib.gmg_net_set_weights(self.h, depth, w.ctypes.data_as(ctypes.c_void_p), w.size))

    def set_learned(self, depth, w_bf16):
        import numpy as np
        w = np.ascontiguousarray(w_bf16, dtype=np.uint16)
        if w.size != NET_WEIGHTS:
            raise ValueError("expected 7776 weights")
        self._check(self.lib.gmg_set_learned(self.h, depth, w.ctypes.data_as(ctypes.c_void_p), w.size))

    def net_get_weights(self, depth):
        import numpy as np
        w = np.zeros(NET_WEIGHTS, dtype=np.float32)
        self._check(self.lib.gmg_net_get_weights(self.h, depth, w.ctypes.data_as(ctypes.c_void_p), w.size))
        return w

    def net_get_state(self, depth):
        """(w, m, v): FP32 master weights and Adam moments of one depth."""
        import numpy as np
        w, m, v = (np.zeros(NET_WEIGHTS, dtype=np.float32) for _ in range(3))
        self._check(self.lib.gmg_net_get_state(self.h, depth, *(a.ctypes.data_as(ctypes.c_void_p) for a in (w, m, v))))
        return w, m, v

    def net_set_state(self, depth, w, m, v):
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (w, m, v)]
        if any(a.size != NET_WEIGHTS for a in arrs):
            raise ValueError("expected 7776 values each")
        self._check(self.lib.gmg_net_set_state(self.h, depth, *(a.ctypes.data_as(ctypes.c_void_p) for a in arrs)))

    def net_cache(self, depth):
        """A device byte buffer large enough for one forward cache at this depth."""
        v = ctypes.c_int64()
        self._check(self.lib.gmg_net_cache_bytes(self.h, depth, ctypes.byref(v)))
        return self._torch.empty(v.value, dtype=self._torch.uint8, device="cuda")

    def net_forward(self, depth, x, y, cache):
        lv = self.levels - 1 - depth
        self._check(self.lib.gmg_net_forward(self.h, depth, self._vec(x, lv, GMG_FP32), self._vec(y, lv, GMG_FP32),
                                             _ptr(cache)))

    def net_backward(self, depth, gy, cache, gw, gin=None):
        lv = self.levels - 1 - depth
        if gw.numel() != NET_WEIGHTS or gw.dtype != self._torch.float32 or not gw.is_cuda:
            raise ValueError("gw must be 7776 FP32 values on the GPU")
        gin_p = self._vec(gin, lv, GMG_FP32) if gin is not None else None
        self._check(self.lib.gmg_net_backward(self.h, depth, self._vec(gy, lv, GMG_FP32), _ptr(cache), _ptr(gw),
                                              gin_p))

    def adam_step(self, depth, gw, lr, step):
        self._check(self.lib.gmg_adam_step(self.h, depth, _ptr(gw), ctypes.c_float(lr), step))

    def net_correction(self, level, r, e):
        level = self._lvl(level)
        self._check(self.lib.gmg_net_correction(self.h, level, self._vec(r, level, GMG_FP32),
                                                self._vec(e, level, GMG_FP32)))

    def net_loss_grad(self, depth, r, e, cache, gw=None, scale=1.0, kind=LOSS_ENERGY):
        """Loss of the pair (r, e) (e unused for LOSS_RESIDUAL); adds scale * dloss/dw into gw."""
        lv = self.levels - 1 - depth
        loss = ctypes.c_double()
        ep = self._vec(e, lv, GMG_FP32) if e is not None else None
        self._check(self.lib.gmg_net_loss_grad(self.h, depth, kind, self._vec(r, lv, GMG_FP32), ep,
                                               _ptr(cache), _ptr(gw) if gw is not None else None,
                                               ctypes.c_float(scale), ctypes.byref(loss)))
        return loss.value

    def residual(self, level, b, u, r):
        level = self._lvl(level)
        p = self.prec_of(b)
        self._check(self.lib.gmg_residual(self.h, level, p, self._vec(b, level, p), self._vec(u, level, p),
                                          self._vec(r, level, p)))

    def solve(self, f, u, rtol, raise_on_noconv=True):
        lv = self.levels - 1
        info = GmgInfo()
        st = self.lib.gmg_solve(self.h, self._vec(f, lv, GMG_FP64), self._vec(u, lv, GMG_FP64), rtol,
                                ctypes.byref(info))
        if st != 0 and (raise_on_noconv or st != 5):
            self._check(st)
        return info

    def fft_solve(self, b, u):
        """Exact FFT solve of the uniform Q1 system A u = b (FP64)."""
        lv = self.levels - 1
        self._check(self.lib.gmg_fft_solve(self.h, self._vec(b, lv, GMG_FP64), self._vec(u, lv, GMG_FP64)))

    def solve_rhs(self, b, u, rtol, raise_on_noconv=True):
        lv = self.levels - 1
        info = GmgInfo()
        st = self.lib.gmg_solve_rhs(self.h, self._vec(b, lv, GMG_FP64), self._vec(u, lv, GMG_FP64), rtol,
                                    ctypes.byref(info))
        if st != 0 and (raise_on_noconv or st != 5):
            self._check(st)
        return info


def _leaves_call(fn, *args):
    """Run an octree-construction call twice: once for the count, once to fill."""
    import numpy as np
    cnt = ctypes.c_int64()
    st = fn(*args, None, None, 0, ctypes.byref(cnt))
    if st not in (0, 1) or cnt.value <= 0:
        raise GmgError(st, "octree construction failed")
    keys = np.zeros(cnt.value, dtype=np.uint64)
    lev = np.zeros(cnt.value, dtype=np.uint8)
    st = fn(*args, keys.ctypes.data_as(ctypes.c_void_p), lev.ctypes.data_as(ctypes.c_void_p), cnt.value,
            ctypes.byref(cnt))
    if st != 0:
        raise GmgError(st, "octree construction failed")
    return keys, lev


def octree_refine_gaussians(base_level, max_level, centres, sigma, amps, tol=1e-2):
    """Leaves (morton, level) of the gradient-refined, 2:1-balanced octree of a Gaussian sum."""
    import numpy as np
    lib = load()
    c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    a = np.ascontiguousarray(amps, dtype=np.float64)
    if not (len(c) == len(s) == len(a)):
        raise ValueError("centres, sigma and amps differ in length")
    vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
    return _leaves_call(lib.gmg_octree_refine_gaussians, base_level, max_level, len(a), vp(c), vp(s), vp(a), tol)


def octree_refine_sharp_layer(base_level, max_level, centre, radius, alpha, tol=1e-2):
    """Leaves (morton, level) of the gradient-refined, 2:1-balanced octree of the source of
    the sharp-layer solution exp(-(r/radius)^alpha) around centre."""
    import numpy as np
    lib = load()
    c = np.ascontiguousarray(centre, dtype=np.float64).reshape(3)
    return _leaves_call(lib.gmg_octree_refine_sharp_layer, base_level, max_level,
                        c.ctypes.data_as(ctypes.c_void_p), float(radius), float(alpha), tol)


def octree_balance(keys, levels):
    """Leaves (morton, level) of the coarsest 2:1-balanced refinement of a complete octree."""
    import numpy as np
    lib = load()
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    l = np.ascontiguousarray(levels, dtype=np.uint8)
    return _leaves_call(lib.gmg_octree_balance, k.ctypes.data_as(ctypes.c_void_p), l.ctypes.data_as(ctypes.c_void_p),
                        k.size)


class SpectralSolver:
    """The paper's FFT Poisson method on the uniform N^3 grid (gmg_spectral_*): u with
    -Laplace(u) = f spectrally, zero mean, f and u FP64 GPU tensors of N^3 values."""

    def __init__(self, N, stream=None):
        import torch
        self._torch = torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.N = N
        h = ctypes.c_void_p()
        st = self.lib.gmg_spectral_create(N, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != 0:
            raise GmgError(st, f"gmg_spectral_create({N}) failed")
        self.h = h

    def solve(self, f, u):
        torch = self._torch
        for t in (f, u):
            if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float64 and t.numel() == self.N ** 3):
                raise ValueError("expected contiguous float64 GPU tensors of N^3 values")
        st = self.lib.gmg_spectral_solve(self.h, _ptr(f), _ptr(u))
        if st != 0:
            raise GmgError(st, "gmg_spectral_solve failed")

    def close(self):
        if getattr(self, "h", None):
            self.lib.gmg_spectral_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
