"""Thin ctypes binding of liboic (include/oic.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; this module only
converts NumPy arrays (host memory) or torch CUDA tensors (device memory) to
pointers and checks return codes.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liboic.so")

OIC_OK = 0
OIC_EINVAL = -1
OIC_ENOMEM = -2
OIC_EDEVICE = -3
OIC_ENOTSPD = -4

OIC_ACT_TANH = 0
OIC_ACT_GELU = 1
OIC_PREC_FP32 = 0
OIC_PREC_BF16 = 1
OIC_PREC_FP8 = 2
OIC_MEM_HOST = 0
OIC_MEM_DEVICE = 1
OIC_MAX_LAYERS = 8
OIC_NOALLOC_SCRATCH_BYTES = 64 << 20

_ERRNAMES = {OIC_EINVAL: "OIC_EINVAL", OIC_ENOMEM: "OIC_ENOMEM", OIC_EDEVICE: "OIC_EDEVICE",
             OIC_ENOTSPD: "OIC_ENOTSPD"}


class OicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class oic_config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("m", ctypes.c_int), ("l", ctypes.c_int),
                ("n_layers", ctypes.c_int), ("channels", ctypes.c_int * (OIC_MAX_LAYERS + 1)),
                ("activation", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_N", ctypes.c_int), ("max_H", ctypes.c_int), ("mem_mode", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


_fp = ctypes.POINTER(ctypes.c_float)


class oic_solve_args(ctypes.Structure):
    _fields_ = [("X0", ctypes.c_void_p), ("reference", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("N", ctypes.c_int), ("horizon", ctypes.c_int),
                ("seed", ctypes.c_uint64), ("U_prev", ctypes.c_void_p),
                ("Z_init", ctypes.c_void_p), ("Z_W", ctypes.c_void_p), ("Z_VX", ctypes.c_void_p),
                ("Z_VU", ctypes.c_void_p), ("U_out", ctypes.c_void_p), ("X_out", ctypes.c_void_p),
                ("Z_VZ", ctypes.c_void_p)]


_lib = None


def lib():
    """Load liboic.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2410_09663_amd.build` (no CPU fallback exists)")
        # One HIP runtime per process.  torch ships its own libamdhip64 under a name that
        # does not match the ROCm runtime's soname, so a library loaded before torch binds
        # to ROCm's copy and torch later adds a second one.  Loading torch first makes the
        # dynamic loader resolve liboic's runtime to torch's copy (same soname).
        try:
            import torch
        except ImportError:
            torch = None
        if torch is not None and torch.cuda.is_available():
            torch.cuda.init()
        L = ctypes.CDLL(LIB_PATH)
        runtimes = _hip_runtimes()
        if len(runtimes) > 1:
            raise RuntimeError("two HIP runtimes are loaded in this process (" + ", ".join(runtimes) +
                               "): load liboic through this module, after torch if torch is used")
        vp, ci, cu64, cs = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t
        sig = {
            "oic_create": (ci, [ctypes.POINTER(oic_config), ctypes.POINTER(vp)]),
            "oic_destroy": (None, [vp]),
            "oic_last_error": (ctypes.c_char_p, [vp]),
            "oic_set_weights": (ci, [vp, vp, ctypes.POINTER(vp), ctypes.POINTER(vp)]),
            "oic_set_u_prev": (ci, [vp, vp]),
            "oic_get_u_prev": (ci, [vp, vp]),
            "oic_solve": (ci, [vp, vp, vp, vp, vp, ci, ci, cu64, vp, vp]),
            "oic_solve_ex": (ci, [vp, ctypes.POINTER(oic_solve_args)]),
            "oic_solve_cov": (ci, [vp, ctypes.POINTER(oic_solve_args), vp, vp]),
            "oic_columns_expand": (ci, [ci, ci, ci, vp, vp, vp]),
            "oic_set_constraint": (ci, [vp, vp, vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float]),
            "oic_columns_project": (ci, [ci, ci, ci, vp, vp, vp]),
            "oic_cnn_forward": (ci, [vp, ci, vp, vp, vp]),
            "oic_cnn_forward_noalloc": (ci, [vp, ci, vp, vp, vp]),
            "oic_plant_step": (ci, [vp, vp, vp, vp]),
            "oic_normals": (ci, [vp, cu64, ci, cs, vp]),
            "oic_timing": (ci, [vp, ci]),
            "oic_kernel_class_count": (ci, []),
            "oic_kernel_stats": (ci, [vp, ci, ctypes.POINTER(ctypes.c_char_p),
                                      ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_double)]),
            "oic_stream": (vp, [vp]),
            "oic_set_graph": (ci, [vp, ci]),
            "oic_server_create": (ci, [cs, ci, ctypes.POINTER(vp)]),
            "oic_server_destroy": (None, [vp]),
            "oic_server_add": (ci, [vp, ctypes.POINTER(oic_config), vp, ctypes.POINTER(vp),
                                    ctypes.POINTER(vp), ci, ci, vp, vp, ctypes.POINTER(ci)]),
            "oic_server_submit": (ci, [vp, ci, vp, vp, cu64, ctypes.POINTER(ctypes.c_longlong)]),
            "oic_server_wait": (ci, [vp, ctypes.c_longlong, vp, vp, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
            "oic_server_stats": (ci, [vp, ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_longlong),
                                      ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
            "oic_server_last_error": (ctypes.c_char_p, [vp]),
            "oic_server_set_group_slots": (ci, [vp, ci]),
            "oic_server_batch_stats": (ci, [vp, ctypes.POINTER(ctypes.c_longlong),
                                            ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
            "oic_footprint_bytes": (cs, [ctypes.POINTER(oic_config)]),
            "oic_stage_cost": (ci, [ci, ci, ci, vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double)]),
            "oic_group_footprint_bytes": (cs, [ctypes.POINTER(oic_config), ci]),
            "oic_group_create": (ci, [ctypes.POINTER(oic_config), ci, ctypes.POINTER(vp)]),
            "oic_group_destroy": (None, [vp]),
            "oic_group_slot": (vp, [vp, ci]),
            "oic_group_solve": (ci, [vp, ci, ctypes.POINTER(ci), ctypes.POINTER(oic_solve_args),
                                     ctypes.POINTER(ci)]),
            "oic_group_last_error": (ctypes.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _hip_runtimes():
    """Distinct files of the HIP runtime (libamdhip64) mapped into this process."""
    try:
        with open("/proc/self/maps") as f:
            paths = {ln.split()[-1] for ln in f if "libamdhip64" in ln}
    except OSError:
        return []
    return sorted({os.path.realpath(p) for p in paths if p.startswith("/")})


EXPORTED = ["oic_create", "oic_destroy", "oic_last_error", "oic_set_weights", "oic_set_u_prev",
            "oic_get_u_prev", "oic_solve", "oic_solve_ex", "oic_solve_cov", "oic_columns_expand", "oic_columns_project", "oic_set_constraint", "oic_cnn_forward", "oic_cnn_forward_noalloc", "oic_plant_step",
            "oic_normals", "oic_timing", "oic_kernel_class_count", "oic_kernel_stats", "oic_stream",
            "oic_set_graph", "oic_server_create", "oic_server_destroy", "oic_server_add",
            "oic_server_submit", "oic_server_wait", "oic_server_stats", "oic_server_last_error",
            "oic_footprint_bytes", "oic_stage_cost", "oic_group_footprint_bytes", "oic_group_create",
            "oic_group_destroy", "oic_group_slot", "oic_group_solve", "oic_group_last_error",
            "oic_server_set_group_slots", "oic_server_batch_stats"]


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class Controller:
    """One handle of liboic.  mem_mode OIC_MEM_HOST takes and returns float32 NumPy
    arrays; OIC_MEM_DEVICE takes float32 torch CUDA tensors (contiguous)."""

    def __init__(self, n: int, m: int, l: int, channels: Sequence[int], activation: int,
                 max_N: int, max_H: int, precision: int = OIC_PREC_FP32,
                 mem_mode: int = OIC_MEM_HOST, stream: Optional[int] = None):
        self._h = None
        cfg = _config(n, m, l, channels, activation, max_N, max_H, precision, mem_mode, stream)
        h = ctypes.c_void_p()
        rc = lib().oic_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OIC_OK:
            raise OicError(rc, "oic_create failed")
        self._h = h
        self._owned = True
        self.n, self.m, self.l = n, m, l
        self.channels = list(channels)
        self.mem_mode = mem_mode
        self.max_N, self.max_H = max_N, max_H

    @classmethod
    def _slot(cls, h, cfg, owner):
        """The handle of a group slot (owned by the group `owner`, kept alive here)."""
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p(h)
        self._owned = False
        self._owner = owner
        self.n, self.m, self.l = cfg.n, cfg.m, cfg.l
        self.channels = [cfg.channels[k] for k in range(cfg.n_layers + 1)]
        self.mem_mode = cfg.mem_mode
        self.max_N, self.max_H = cfg.max_N, cfg.max_H
        return self

    # -- helpers -------------------------------------------------------------
    def _check(self, rc: int):
        if rc != OIC_OK:
            raise OicError(rc, lib().oic_last_error(self._h).decode())

    def _ptr(self, a, shape, writable=False):
        """Pointer to a float32 array/tensor of the given shape (checked)."""
        if a is None:
            return None
        if self.mem_mode == OIC_MEM_DEVICE:
            if not _is_torch(a) or not a.is_cuda:
                raise TypeError("device mode takes torch CUDA tensors")
            import torch
            if a.dtype != torch.float32 or not a.is_contiguous() or tuple(a.shape) != tuple(shape):
                raise ValueError(f"expected contiguous float32 tensor of shape {shape}")
            return a.data_ptr()
        if not isinstance(a, np.ndarray) or a.dtype != np.float32 or not a.flags.c_contiguous:
            raise TypeError("host mode takes C-contiguous float32 NumPy arrays")
        if tuple(a.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        if writable and not a.flags.writeable:
            raise ValueError("output array is read-only")
        return a.ctypes.data

    def _new(self, shape):
        if self.mem_mode == OIC_MEM_DEVICE:
            import torch
            return torch.empty(shape, dtype=torch.float32, device="cuda")
        return np.empty(shape, dtype=np.float32)

    @staticmethod
    def _host(a, shape):
        a = np.ascontiguousarray(a, dtype=np.float32)
        if a.shape != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        return a

    # -- API -----------------------------------------------------------------
    def set_weights(self, B, weights, biases=None):
        B = self._host(B, (self.n, self.l))
        ws = [self._host(w, (co, ci, 3, 3)) for w, ci, co in
              zip(weights, self.channels[:-1], self.channels[1:])]
        if len(ws) != len(self.channels) - 1:
            raise ValueError("one weight tensor per layer")
        wp = (ctypes.c_void_p * len(ws))(*[w.ctypes.data for w in ws])
        bp = None
        keep = [B, ws]
        if biases is not None:
            bs = [None if b is None else self._host(b, (co,)) for b, co in
                  zip(biases, self.channels[1:])]
            keep.append(bs)
            bp = (ctypes.c_void_p * len(bs))(*[None if b is None else b.ctypes.data for b in bs])
        self._check(lib().oic_set_weights(self._h, B.ctypes.data, wp, bp))

    def set_u_prev(self, U):
        self._check(lib().oic_set_u_prev(self._h, self._ptr(U, (self.l, self.m))))

    def get_u_prev(self):
        out = self._new((self.l, self.m))
        self._check(lib().oic_get_u_prev(self._h, self._ptr(out, (self.l, self.m), True)))
        return out

    def solve(self, X0, reference, Q, R, N: int, H: int, seed: int, want_X: bool = False,
              U_out=None, X_out=None):
        """Seeded solve (device-generated Philox noise).  Returns (U_hat, X_hat or None)."""
        Q = self._host(Q, (self.l, self.l))
        R = self._host(R, (self.n, self.n))
        U_out = self._new((H + 1, self.l, self.m)) if U_out is None else U_out
        if want_X and X_out is None:
            X_out = self._new((H + 1, self.n, self.m))
        rc = lib().oic_solve(self._h, self._ptr(X0, (self.n, self.m)),
                             self._ptr(reference, (H + 1, self.n, self.m)), Q.ctypes.data,
                             R.ctypes.data, N, H, seed,
                             self._ptr(U_out, (H + 1, self.l, self.m), True),
                             self._ptr(X_out, (H + 1, self.n, self.m), True))
        self._check(rc)
        return U_out, X_out

    def solve_ex(self, X0, reference, Q, R, N: int, H: int, seed: int = 0, U_prev=None,
                 noise=None, want_X: bool = True, Z_VZ=None, U_out=None, X_out=None):
        """Solve with explicit noise (a workloads.Noise or a 4-tuple) or, if noise is None,
        the seeded stream.  Returns (U_hat, X_hat), written into U_out / X_out if given."""
        a, keep, U_out, X_out = self._args(X0, reference, Q, R, N, H, seed, U_prev, noise, want_X, Z_VZ,
                                           U_out, X_out)
        self._check(lib().oic_solve_ex(self._h, ctypes.byref(a)))
        return U_out, X_out

    def _args(self, X0, reference, Q, R, N, H, seed=0, U_prev=None, noise=None, want_X=True, Z_VZ=None,
              U_out=None, X_out=None):
        """oic_solve_args for one solve on this handle, the arrays it points to (keep them
        alive until the call returns) and the output arrays."""
        Q = self._host(Q, (self.l, self.l))
        R = self._host(R, (self.n, self.n))
        a = oic_solve_args()
        a.X0 = self._ptr(X0, (self.n, self.m))
        a.reference = self._ptr(reference, (H + 1, self.n, self.m))
        a.Q, a.R = Q.ctypes.data, R.ctypes.data
        a.N, a.horizon, a.seed = N, H, seed
        a.U_prev = self._ptr(U_prev, (self.l, self.m))
        if noise is not None:
            z = (noise.Z_init, noise.Z_W, noise.Z_VX, noise.Z_VU) if hasattr(noise, "Z_init") else noise
            a.Z_init = self._ptr(z[0], (N, self.l, self.m))
            a.Z_W = self._ptr(z[1], (H, N, self.l, self.m))
            a.Z_VX = self._ptr(z[2], (H, N, self.n, self.m))
            a.Z_VU = self._ptr(z[3], (H, N, self.l, self.m))
        if Z_VZ is not None:
            a.Z_VZ = self._ptr(Z_VZ, (H, N, 1, self.m))
        U_out = self._new((H + 1, self.l, self.m)) if U_out is None else U_out
        if want_X and X_out is None:
            X_out = self._new((H + 1, self.n, self.m))
        a.U_out = self._ptr(U_out, (H + 1, self.l, self.m), True)
        a.X_out = self._ptr(X_out, (H + 1, self.n, self.m), True) if X_out is not None else None
        return a, (Q, R), U_out, X_out

    def solve_cov(self, X0, reference, Q, R, N: int, H: int, seed: int = 0, U_prev=None, noise=None,
                  Z_VZ=None):
        """oic_solve_cov: returns (U_hat, X_hat, prior, post), where prior[t-1] and post[t-1]
        are the (t+1)(n+l) x (t+1)(n+l) pooled trajectory covariances before and after the
        analysis of horizon step t (FP64)."""
        Q = self._host(Q, (self.l, self.l))
        R = self._host(R, (self.n, self.n))
        a = oic_solve_args()
        a.X0 = self._ptr(X0, (self.n, self.m))
        a.reference = self._ptr(reference, (H + 1, self.n, self.m))
        a.Q, a.R = Q.ctypes.data, R.ctypes.data
        a.N, a.horizon, a.seed = N, H, seed
        a.U_prev = self._ptr(U_prev, (self.l, self.m))
        if noise is not None:
            z = (noise.Z_init, noise.Z_W, noise.Z_VX, noise.Z_VU) if hasattr(noise, "Z_init") else noise
            a.Z_init = self._ptr(z[0], (N, self.l, self.m))
            a.Z_W = self._ptr(z[1], (H, N, self.l, self.m))
            a.Z_VX = self._ptr(z[2], (H, N, self.n, self.m))
            a.Z_VU = self._ptr(z[3], (H, N, self.l, self.m))
        if Z_VZ is not None:
            a.Z_VZ = self._ptr(Z_VZ, (H, N, 1, self.m))
        U_out = self._new((H + 1, self.l, self.m))
        X_out = self._new((H + 1, self.n, self.m))
        a.U_out = self._ptr(U_out, U_out.shape, True)
        a.X_out = self._ptr(X_out, X_out.shape, True)
        rr = self.n + self.l
        sizes = [((t + 1) * rr) ** 2 for t in range(1, H + 1)]
        if self.mem_mode == OIC_MEM_DEVICE:
            import torch
            prior = torch.empty(sum(sizes), dtype=torch.float64, device="cuda")
            post = torch.empty(sum(sizes), dtype=torch.float64, device="cuda")
            pp, qp = prior.data_ptr(), post.data_ptr()
        else:
            prior = np.empty(sum(sizes), np.float64)
            post = np.empty(sum(sizes), np.float64)
            pp, qp = prior.ctypes.data, post.ctypes.data
        self._check(lib().oic_solve_cov(self._h, ctypes.byref(a), pp, qp))
        def split(buf):
            out, off = [], 0
            for t, sz in enumerate(sizes, start=1):
                ma = (t + 1) * rr
                out.append(buf[off:off + sz].reshape(ma, ma))
                off += sz
            return out
        return U_out, X_out, split(prior), split(post)

    def set_constraint(self, aX=None, aU=None, b=0.0, alpha=1.0, beta=1.0, rz=1.0):
        """oic_set_constraint: g_c = aX . X[:, c] + aU . U[:, c] - b <= 0 observed through
        the softplus barrier with noise variance rz; no arguments removes it."""
        if aX is None and aU is None:
            self._check(lib().oic_set_constraint(self._h, None, None, 0.0, 1.0, 1.0, 1.0))
            return
        ax = np.ascontiguousarray(aX, np.float32).reshape(self.n)
        au = np.ascontiguousarray(aU, np.float32).reshape(self.l)
        self._check(lib().oic_set_constraint(self._h, ax.ctypes.data, au.ctypes.data, b, alpha, beta, rz))

    def cnn_forward(self, X, U):
        b = X.shape[0]
        out = self._new((b, self.n, self.m))
        self._check(lib().oic_cnn_forward(self._h, b, self._ptr(X, (b, self.n, self.m)),
                                          self._ptr(U, (b, self.l, self.m)),
                                          self._ptr(out, (b, self.n, self.m), True)))
        return out

    def cnn_forward_noalloc(self, X, U, out=None):
        """oic_cnn_forward_noalloc (device-memory handles): the surrogate with its
        intermediate activations in the library's fixed per-GPU buffer."""
        b = X.shape[0]
        out = self._new((b, self.n, self.m)) if out is None else out
        self._check(lib().oic_cnn_forward_noalloc(self._h, b, self._ptr(X, (b, self.n, self.m)),
                                                  self._ptr(U, (b, self.l, self.m)),
                                                  self._ptr(out, (b, self.n, self.m), True)))
        return out

    def plant_step(self, X, U):
        out = self._new((self.n, self.m))
        self._check(lib().oic_plant_step(self._h, self._ptr(X, (self.n, self.m)),
                                         self._ptr(U, (self.l, self.m)),
                                         self._ptr(out, (self.n, self.m), True)))
        return out

    def normals(self, seed: int, kind: int, count: int):
        out = self._new((count,))
        self._check(lib().oic_normals(self._h, seed, kind, count, self._ptr(out, (count,), True)))
        return out

    def timing(self, enable: bool):
        self._check(lib().oic_timing(self._h, 1 if enable else 0))

    def kernel_stats(self):
        """{class name: (launches, total ms)} since timing was last enabled."""
        out = {}
        for k in range(lib().oic_kernel_class_count()):
            name = ctypes.c_char_p()
            cnt = ctypes.c_longlong()
            ms = ctypes.c_double()
            self._check(lib().oic_kernel_stats(self._h, k, ctypes.byref(name), ctypes.byref(cnt),
                                               ctypes.byref(ms)))
            out[name.value.decode()] = (cnt.value, ms.value)
        return out

    def stream(self) -> int:
        return lib().oic_stream(self._h)

    def set_graph(self, enable: bool):
        self._check(lib().oic_set_graph(self._h, 1 if enable else 0))

    def close(self):
        if self._h is not None:
            if self._owned:
                lib().oic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _config(n, m, l, channels, activation, max_N, max_H, precision, mem_mode, stream) -> oic_config:
    cfg = oic_config()
    cfg.n, cfg.m, cfg.l = n, m, l
    cfg.n_layers = len(channels) - 1
    for k, c in enumerate(channels):
        cfg.channels[k] = c
    cfg.activation, cfg.precision = activation, precision
    cfg.max_N, cfg.max_H, cfg.mem_mode = max_N, max_H, mem_mode
    if stream is None and mem_mode == OIC_MEM_DEVICE:
        # device mode reads caller tensors: order the work after torch's queued kernels
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    cfg.stream = stream
    return cfg


class Group:
    """oic_group: `slots` handles of one configuration whose solves run in shared launches.
    group.slots[i] is slot i's Controller (weights, U_prev, solves of its own)."""

    def __init__(self, n: int, m: int, l: int, channels: Sequence[int], activation: int,
                 max_N: int, max_H: int, slots: int, precision: int = OIC_PREC_BF16,
                 mem_mode: int = OIC_MEM_HOST, stream: Optional[int] = None):
        self._g = None
        cfg = _config(n, m, l, channels, activation, max_N, max_H, precision, mem_mode, stream)
        g = ctypes.c_void_p()
        rc = lib().oic_group_create(ctypes.byref(cfg), slots, ctypes.byref(g))
        if rc != OIC_OK:
            raise OicError(rc, "oic_group_create failed")
        self._g = g
        self.slots = [Controller._slot(lib().oic_group_slot(g, i), cfg, self) for i in range(slots)]

    @staticmethod
    def footprint(problem, N: int, H: int, slots: int, precision: int = OIC_PREC_BF16) -> int:
        p = problem.preset
        cfg = _config(p.n, p.m, p.l, p.channels, p.activation, N, H, precision, OIC_MEM_HOST, None)
        return lib().oic_group_footprint_bytes(ctypes.byref(cfg), slots)

    def solve(self, requests):
        """One batch: requests is a list of (slot, kwargs of Controller.solve_ex).  Returns
        the list of (U_hat, X_hat) in request order; raises OicError if any request failed
        (rc_codes holds each request's status afterwards)."""
        count = len(requests)
        args = (oic_solve_args * count)()
        slots = (ctypes.c_int * count)(*[r[0] for r in requests])
        keep, outs = [], []
        for i, (slot, kw) in enumerate(requests):
            a, k, U_out, X_out = self.slots[slot]._args(**kw)
            args[i] = a
            keep.append(k)
            outs.append((U_out, X_out))
        rcs = (ctypes.c_int * count)()
        rc = lib().oic_group_solve(self._g, count, slots, args, rcs)
        self.rc_codes = list(rcs)
        if rc != OIC_OK:
            raise OicError(rc, lib().oic_group_last_error(self._g).decode())
        return outs

    def close(self):
        if self._g is not None:
            for c in self.slots:
                c._h = None
            lib().oic_group_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def controller_for(problem, max_N=None, max_H=None, precision=None, mem_mode=OIC_MEM_HOST,
                   stream=None) -> Controller:
    """A Controller sized for a workloads.Problem, with its weights set."""
    p = problem.preset
    c = Controller(p.n, p.m, p.l, p.channels, p.activation, max_N or p.N, max_H or p.H,
                   precision=p.precision if precision is None else precision,
                   mem_mode=mem_mode, stream=stream)
    c.set_weights(problem.B, problem.weights)
    return c


def stage_cost(X, Xref, U, dU, Q, R) -> float:
    """Stage cost of the tracking objective (oic_stage_cost), host arrays."""
    f = lambda a: np.ascontiguousarray(a, np.float32)
    X, Xref, U, dU, Q, R = map(f, (X, Xref, U, dU, Q, R))
    n, m = X.shape
    l = U.shape[0]
    out = ctypes.c_double()
    rc = lib().oic_stage_cost(n, m, l, X.ctypes.data, Xref.ctypes.data, U.ctypes.data, dU.ctypes.data,
                              Q.ctypes.data, R.ctypes.data, ctypes.byref(out))
    if rc != OIC_OK:
        raise OicError(rc, "oic_stage_cost failed")
    return out.value


def columns_expand(u, T):
    """U = u T (oic_columns_expand): u (l, q), T (q, m) -> (l, m) float32."""
    u = np.ascontiguousarray(u, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    l, q = u.shape
    m = T.shape[1]
    if T.shape[0] != q:
        raise ValueError("T must be q x m")
    U = np.empty((l, m), np.float32)
    rc = lib().oic_columns_expand(l, q, m, u.ctypes.data, T.ctypes.data, U.ctypes.data)
    if rc != OIC_OK:
        raise OicError(rc, "oic_columns_expand failed")
    return U


def columns_project(U, T):
    """u = U T^T (T T^T)^{-1} (oic_columns_project): U (l, m), T (q, m) -> (l, q) float32."""
    U = np.ascontiguousarray(U, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    l, m = U.shape
    q = T.shape[0]
    if T.shape[1] != m:
        raise ValueError("T must be q x m")
    u = np.empty((l, q), np.float32)
    rc = lib().oic_columns_project(l, m, q, U.ctypes.data, T.ctypes.data, u.ctypes.data)
    if rc != OIC_OK:
        raise OicError(rc, "oic_columns_project failed")
    return u


class Server:
    """Request loop for many controllers (oic_server_*): host NumPy arrays in and out."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 4, group_slots: Optional[int] = None):
        self._s = None
        h = ctypes.c_void_p()
        rc = lib().oic_server_create(int(hbm_budget_bytes), int(max_inflight), ctypes.byref(h))
        if rc != OIC_OK:
            raise OicError(rc, "oic_server_create failed")
        self._s = h
        self._shapes = {}
        if group_slots is not None:
            rc = lib().oic_server_set_group_slots(h, int(group_slots))
            if rc != OIC_OK:
                raise OicError(rc, "oic_server_set_group_slots failed")

    @staticmethod
    def config_for(problem, N: int, H: int, precision: int = None) -> oic_config:
        p = problem.preset
        cfg = oic_config()
        cfg.n, cfg.m, cfg.l = p.n, p.m, p.l
        cfg.n_layers = len(p.channels) - 1
        for k, c in enumerate(p.channels):
            cfg.channels[k] = c
        cfg.activation = p.activation
        cfg.precision = p.precision if precision is None else precision
        cfg.mem_mode = OIC_MEM_HOST
        cfg.max_N, cfg.max_H = N, H
        return cfg

    @staticmethod
    def footprint(problem, N: int, H: int, precision: int = None) -> int:
        cfg = Server.config_for(problem, N, H, precision)
        return int(lib().oic_footprint_bytes(ctypes.byref(cfg)))

    def add(self, problem, N: int, H: int, precision: int = None) -> int:
        """Register a controller for a workloads.Problem; returns its id."""
        p = problem.preset
        cfg = self.config_for(problem, N, H, precision)
        B = np.ascontiguousarray(problem.B, np.float32)
        ws = [np.ascontiguousarray(w, np.float32) for w in problem.weights]
        wp = (ctypes.c_void_p * len(ws))(*[w.ctypes.data for w in ws])
        Q = np.ascontiguousarray(problem.Q, np.float32)
        R = np.ascontiguousarray(problem.R, np.float32)
        cid = ctypes.c_int()
        rc = lib().oic_server_add(self._s, ctypes.byref(cfg), B.ctypes.data, wp, None, N, H,
                                  Q.ctypes.data, R.ctypes.data, ctypes.byref(cid))
        if rc != OIC_OK:
            raise OicError(rc, "oic_server_add failed")
        self._shapes[cid.value] = (p.n, p.m, p.l, H)
        return cid.value

    def submit(self, cid: int, X0, reference, seed: int) -> int:
        n, m, l, H = self._shapes[cid]
        X0 = np.ascontiguousarray(X0, np.float32)
        ref = np.ascontiguousarray(reference, np.float32)
        if X0.shape != (n, m) or ref.shape != (H + 1, n, m):
            raise ValueError("bad X0 or reference shape")
        t = ctypes.c_longlong()
        rc = lib().oic_server_submit(self._s, cid, X0.ctypes.data, ref.ctypes.data, seed, ctypes.byref(t))
        if rc != OIC_OK:
            raise OicError(rc, "oic_server_submit failed")
        return t.value

    def wait(self, cid: int, ticket: int):
        """Returns (U_hat, X_hat, latency_ms, queue_ms)."""
        n, m, l, H = self._shapes[cid]
        U = np.empty((H + 1, l, m), np.float32)
        X = np.empty((H + 1, n, m), np.float32)
        lat, q = ctypes.c_double(), ctypes.c_double()
        rc = lib().oic_server_wait(self._s, ticket, U.ctypes.data, X.ctypes.data, ctypes.byref(lat),
                                   ctypes.byref(q))
        if rc != OIC_OK:
            raise OicError(rc, lib().oic_server_last_error(self._s).decode())
        return U, X, lat.value, q.value

    def stats(self):
        c, a, e, r = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
        u, pk = ctypes.c_size_t(), ctypes.c_size_t()
        lib().oic_server_stats(self._s, ctypes.byref(c), ctypes.byref(a), ctypes.byref(e), ctypes.byref(r),
                               ctypes.byref(u), ctypes.byref(pk))
        b, g, n = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_longlong()
        lib().oic_server_batch_stats(self._s, ctypes.byref(b), ctypes.byref(g), ctypes.byref(n))
        return {"completed": c.value, "admissions": a.value, "evictions": e.value, "recycled": r.value,
                "bytes_in_use": u.value, "peak_bytes": pk.value, "batches": b.value, "grouped": g.value,
                "packs": n.value}

    def close(self):
        if self._s is not None:
            lib().oic_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
