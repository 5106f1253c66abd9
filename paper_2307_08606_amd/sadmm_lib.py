"""ctypes binding of libsadmm.so (the C ABI in include/sadmm.h).

Argument marshalling only: every step of the solver runs in the HIP library.
The functions keep the C names; `Solver` wraps a handle for torch tensors
(device memory and the current HIP stream come from PyTorch).  Importing this
module raises if the shared library has not been built -- there is no other
implementation to fall back to.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsadmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_08606_amd.build`")

# PyTorch ships its own HIP runtime.  Import it before the library so that the
# process holds one HIP runtime (the library then binds to the one already
# loaded); loading the library first would bring in a second runtime.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

SADMM_OK, SADMM_E_ARG, SADMM_E_SHAPE, SADMM_E_STATE = 0, -1, -2, -3
SADMM_E_HIP, SADMM_E_NOMEM, SADMM_E_NUMERIC = -4, -5, -6
SADMM_C128, SADMM_C64 = 0, 1
ST_FP64, ST_FP32, ST_FP16P, ST_BF16P, ST_MATRIX_FREE = 0, 1, 2, 3, 4
STORAGE = {"fp64": ST_FP64, "fp32": ST_FP32, "fp16": ST_FP16P, "bf16": ST_BF16P,
           "mf": ST_MATRIX_FREE}
HIST = {"r": 0, "s": 1, "eps_pri": 2, "eps_dual": 3, "nmse": 4, "max_active_frac": 5,
        "retake_change": 6, "beta": 7, "correction_move": 8}


class sadmm_params(C.Structure):
    _fields_ = [
        ("Q", C.c_int32), ("K", C.c_int32), ("M", C.c_int32), ("N", C.c_int32),
        ("mu", C.c_double), ("beta", C.c_double), ("gamma", C.c_double),
        ("lambda_", C.c_double),
        ("eps_abs", C.c_double), ("eps_rel", C.c_double),
        ("max_iter", C.c_int32), ("stop", C.c_int32), ("check_every", C.c_int32),
        ("prune", C.c_int32), ("Kp", C.c_int32), ("eps_p", C.c_double),
        ("prune_mode", C.c_int32), ("kkt", C.c_int32), ("kkt_tol", C.c_double),
        ("storage", C.c_int32), ("reuse_factor", C.c_int32), ("gram", C.c_int32),
        ("direct", C.c_int32), ("refine_every", C.c_int32), ("nonneg", C.c_int32),
        ("balance_every", C.c_int32), ("balance_mu", C.c_double), ("balance_tau", C.c_double),
        ("stream", C.c_void_p),
    ]


class sadmm_info(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("status", C.c_int32), ("prune_events", C.c_int32),
        ("reinstated", C.c_int32), ("refactors", C.c_int32), ("updates", C.c_int32),
        ("r", C.c_double), ("s", C.c_double), ("eps_pri", C.c_double),
        ("eps_dual", C.c_double), ("max_active_frac", C.c_double), ("nmse", C.c_double),
        ("direct_sensors", C.c_int32), ("pad", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_H = C.c_void_p
_P = C.c_void_p


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


sadmm_default_params = _sig("sadmm_default_params", None, C.POINTER(sadmm_params))
sadmm_create = _sig("sadmm_create", C.c_int, C.POINTER(sadmm_params), C.POINTER(_H))
sadmm_create_shared = _sig("sadmm_create_shared", C.c_int, C.POINTER(sadmm_params), _H, C.POINTER(_H))
sadmm_set_operator = _sig("sadmm_set_operator", C.c_int, _H, C.c_int32, _P, C.c_int32,
                          C.c_int64, C.c_int32)
sadmm_set_operator_geometry = _sig("sadmm_set_operator_geometry", C.c_int, _H, C.c_int32,
                                   _P, _P, _P, C.c_double, C.c_double)
sadmm_set_active_mask = _sig("sadmm_set_active_mask", C.c_int, _H, C.c_int32, _P)
sadmm_set_reference = _sig("sadmm_set_reference", C.c_int, _H, _P, C.c_int32, C.c_int32,
                           C.c_double)
sadmm_solve = _sig("sadmm_solve", C.c_int, _H, _P, C.c_int32, C.c_int32, C.POINTER(sadmm_info))
sadmm_solve_batch = _sig("sadmm_solve_batch", C.c_int, C.POINTER(_H), C.c_int32,
                         C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.POINTER(sadmm_info))
sadmm_get_image = _sig("sadmm_get_image", C.c_int, _H, _P, C.c_int32, C.c_int32)
sadmm_get_sensor_image = _sig("sadmm_get_sensor_image", C.c_int, _H, C.c_int32, _P, C.c_int32,
                              C.c_int32)
sadmm_get_dual = _sig("sadmm_get_dual", C.c_int, _H, _P, C.c_int32, C.c_int32)
sadmm_get_factor = _sig("sadmm_get_factor", C.c_int, _H, C.c_int32, _P, _P)
sadmm_get_active_mask = _sig("sadmm_get_active_mask", C.c_int, _H, C.c_int32, _P)
sadmm_get_active_indices = _sig("sadmm_get_active_indices", C.c_int, _H, C.c_int32, _P, _P)
sadmm_get_history = _sig("sadmm_get_history", C.c_int, _H, C.c_int32, _P, C.c_int32, _P)
sadmm_matched_filter = _sig("sadmm_matched_filter", C.c_int, _H, _P, C.c_int32, C.c_int32, _P)
sadmm_get_timing = _sig("sadmm_get_timing", C.c_int, _H, C.c_int32, C.POINTER(C.c_double))
sadmm_set_profiling = _sig("sadmm_set_profiling", C.c_int, _H, C.c_int32)
sadmm_get_kernel_stats = _sig("sadmm_get_kernel_stats", C.c_int, _H, C.c_int32, _P, _P, _P)
sadmm_destroy = _sig("sadmm_destroy", None, _H)
KERNEL_CLASSES = {"gram": 0, "inverse": 1, "fwd": 2, "wprod": 3, "xupd": 4, "pixel": 5, "cnn": 6,
                  "slice": 7}

sadmm_cnn_create = _sig("sadmm_cnn_create", C.c_int, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                        C.c_void_p, C.POINTER(_H))
sadmm_cnn_param_count = _sig("sadmm_cnn_param_count", C.c_int64, _H)
sadmm_cnn_set_params = _sig("sadmm_cnn_set_params", C.c_int, _H, _P, C.c_int64)
sadmm_cnn_get_params = _sig("sadmm_cnn_get_params", C.c_int, _H, _P, C.c_int64)
sadmm_cnn_forward = _sig("sadmm_cnn_forward", C.c_int, _H, _P, C.c_int32, _P, C.c_int32)
sadmm_cnn_forward_noalloc = _sig("sadmm_cnn_forward_noalloc", C.c_int, _H, _P, C.c_int32, C.c_int32, _P)
sadmm_cnn_set_half = _sig("sadmm_cnn_set_half", C.c_int, _H, C.c_int32)
sadmm_cnn_gradients = _sig("sadmm_cnn_gradients", C.c_int, _H, _P, _P, C.c_int32, C.c_float, _P,
                           C.POINTER(C.c_double))
sadmm_cnn_train_step = _sig("sadmm_cnn_train_step", C.c_int, _H, _P, _P, C.c_int32, C.c_float,
                            C.c_float, C.POINTER(C.c_double))
sadmm_cnn_destroy = _sig("sadmm_cnn_destroy", None, _H)
sadmm_cnn_last_error = _sig("sadmm_cnn_last_error", C.c_char_p, _H)
sadmm_set_pruning_cnn = _sig("sadmm_set_pruning_cnn", C.c_int, _H, _H, C.c_double)
sadmm_last_error = _sig("sadmm_last_error", C.c_char_p, _H)
sadmm_autotune = _sig("sadmm_autotune", C.c_int, _H, _P, C.c_int32, C.c_int32, C.c_int32, _P)
sadmm_back_projection = _sig("sadmm_back_projection", C.c_int, _H, _P, C.c_int32, C.c_int32, _P)
sadmm_stack_real = _sig("sadmm_stack_real", C.c_int, _P, C.c_int32, C.c_int64, C.c_int64, C.c_int64, _P,
                        C.c_void_p)
sadmm_render_db = _sig("sadmm_render_db", C.c_int, _P, C.c_int32, C.c_int64, C.c_double, C.c_int32, _P,
                       C.c_void_p)
sadmm_probe_bandwidth = _sig("sadmm_probe_bandwidth", C.c_int, C.c_int32, _P, _P, C.c_int64, C.c_int32,
                             C.c_void_p, C.POINTER(C.c_double))
sadmm_probe_mfma = _sig("sadmm_probe_mfma", C.c_int, C.c_int32, C.c_int32, C.c_void_p,
                        C.POINTER(C.c_double))

EXPORTED = [n for n in dir() if n.startswith("sadmm_") and callable(globals()[n])
            and n not in ("sadmm_params", "sadmm_info")]


class SadmmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sadmm error {code}: {msg}")
        self.code = code


def _ptr(a) -> int:
    """Address of a numpy array or torch tensor (contiguous)."""
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"] or a.flags["F_CONTIGUOUS"]
        return a.ctypes.data
    return int(a.data_ptr())


def _dtype_code(a) -> int:
    name = str(a.dtype)
    if name in ("complex128", "torch.complex128"):
        return SADMM_C128
    if name in ("complex64", "torch.complex64"):
        return SADMM_C64
    raise TypeError(f"complex128 or complex64 expected, got {a.dtype}")


def _on_device(a) -> int:
    return 0 if isinstance(a, np.ndarray) else int(a.is_cuda)


class Solver:
    """One sadmm handle.  `params` keys follow sadmm_params (lambda as `lam`)."""

    def __init__(self, Q, K, M, N, *, mu=1.0, beta=1.0, gamma=1.0, lam=0.0, eps_abs=0.0,
                 eps_rel=1e-4, max_iter=200, stop=True, check_every=8, prune=False, Kp=5,
                 eps_p=1e-5, prune_mode="freeze", kkt=False, kkt_tol=1e-2, storage="fp32",
                 reuse_factor=True, gram="int8", direct=True, refine_every=0, nonneg=False,
                 balance_every=0, balance_mu=10.0, balance_tau=2.0, stream=None, share=None):
        p = sadmm_params()
        sadmm_default_params(C.byref(p))
        p.Q, p.K, p.M, p.N = Q, K, M, N
        p.mu, p.beta, p.gamma, p.lambda_ = mu, beta, gamma, lam
        p.eps_abs, p.eps_rel = eps_abs, eps_rel
        p.max_iter, p.stop, p.check_every = max_iter, int(bool(stop)), check_every
        p.prune, p.Kp, p.eps_p = int(bool(prune)), Kp, eps_p
        p.prune_mode = {"freeze": 0, "zero": 1}[prune_mode]
        p.kkt, p.kkt_tol = int(bool(kkt)), kkt_tol
        p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        p.reuse_factor = int(bool(reuse_factor))
        p.gram = {"int8": 0, "fp64": 1, "int8_32": 2}[gram]
        p.direct = 0 if direct else 1
        p.refine_every = int(refine_every)
        p.nonneg = int(bool(nonneg))
        p.balance_every, p.balance_mu, p.balance_tau = int(balance_every), balance_mu, balance_tau
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        p.stream = C.c_void_p(int(stream))
        self.params = p
        self.Q, self.K, self.M, self.N = Q, K, M, N
        self._h = _H()
        self._src = share          # a borrowed operator's owner must outlive this handle
        if share is None:
            self._check(sadmm_create(C.byref(p), C.byref(self._h)), create=True)
        else:
            self._check(sadmm_create_shared(C.byref(p), share._h, C.byref(self._h)), create=True)

    def _check(self, rc, create=False):
        if rc != SADMM_OK:
            msg = sadmm_last_error(None if create else self._h).decode()
            raise SadmmError(rc, msg)

    def close(self):
        if self._h:
            sadmm_destroy(self._h)
            self._h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inputs
    def set_operator(self, q, A):
        """A: (KM, N) complex array/tensor; Fortran-ordered numpy (column-major)
        or a torch tensor holding A^T contiguously (shape (N, KM))."""
        if isinstance(A, np.ndarray):
            if A.shape == (self.K * self.M, self.N):
                A = np.asfortranarray(A)
            ld = A.shape[0] if A.shape == (self.K * self.M, self.N) else A.shape[1]
        else:
            assert A.is_contiguous() and A.shape == (self.N, self.K * self.M)
            ld = A.shape[1]
        self._keep = A
        self._check(sadmm_set_operator(self._h, q, _ptr(A), _dtype_code(A), ld, _on_device(A)))

    def set_operator_geometry(self, q, tx, rx, pix, f0, bw):
        tx = np.ascontiguousarray(tx, dtype=np.float64)
        rx = np.ascontiguousarray(rx, dtype=np.float64)
        pix = np.ascontiguousarray(pix, dtype=np.float64)
        self._check(sadmm_set_operator_geometry(self._h, q, _ptr(tx), _ptr(rx), _ptr(pix),
                                                f0, bw))

    def set_active_mask(self, q, mask):
        if mask is None:
            self._check(sadmm_set_active_mask(self._h, q, None))
            return
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        self._check(sadmm_set_active_mask(self._h, q, _ptr(m)))

    def set_reference(self, x_ref, nmse_target=0.0):
        if x_ref is None:
            self._check(sadmm_set_reference(self._h, None, 0, 0, 0.0))
            return
        if isinstance(x_ref, np.ndarray):
            x_ref = np.ascontiguousarray(x_ref)
        self._check(sadmm_set_reference(self._h, _ptr(x_ref), _dtype_code(x_ref),
                                        _on_device(x_ref), nmse_target))

    # -- solve
    def solve(self, y) -> dict:
        if isinstance(y, np.ndarray):
            y = np.ascontiguousarray(y)
        info = sadmm_info()
        self._check(sadmm_solve(self._h, _ptr(y), _dtype_code(y), _on_device(y), C.byref(info)))
        return info.as_dict()

    # -- outputs
    def image(self, dtype=np.complex128) -> np.ndarray:
        out = np.empty(self.N, dtype=dtype)
        self._check(sadmm_get_image(self._h, _ptr(out), _dtype_code(out), 0))
        return out

    def image_into(self, t):
        self._check(sadmm_get_image(self._h, _ptr(t), _dtype_code(t), _on_device(t)))

    def sensor_image(self, q, dtype=np.complex128) -> np.ndarray:
        out = np.empty(self.N, dtype=dtype)
        self._check(sadmm_get_sensor_image(self._h, q, _ptr(out), _dtype_code(out), 0))
        return out

    def dual(self, dtype=np.complex128) -> np.ndarray:
        out = np.empty(self.N, dtype=dtype)
        self._check(sadmm_get_dual(self._h, _ptr(out), _dtype_code(out), 0))
        return out

    def factor(self, q) -> np.ndarray:
        km = self.K * self.M
        out = np.empty((km, km), dtype=np.complex128, order="F")
        n = C.c_int32(0)
        self._check(sadmm_get_factor(self._h, q, _ptr(out), C.addressof(n)))
        return out

    def active_mask(self, q) -> np.ndarray:
        out = np.empty(self.N, dtype=np.uint8)
        self._check(sadmm_get_active_mask(self._h, q, _ptr(out)))
        return out

    def active_indices(self, q) -> np.ndarray:
        out = np.empty(self.N, dtype=np.int32)
        cnt = C.c_int32(0)
        self._check(sadmm_get_active_indices(self._h, q, _ptr(out), C.addressof(cnt)))
        return out[:cnt.value].copy()

    def history(self, which) -> np.ndarray:
        w = HIST[which] if isinstance(which, str) else int(which)
        cap = self.params.max_iter
        out = np.zeros(cap, dtype=np.float64)
        cnt = C.c_int32(0)
        self._check(sadmm_get_history(self._h, w, _ptr(out), cap, C.addressof(cnt)))
        return out[:min(cnt.value, cap)].copy()

    def matched_filter(self, y) -> np.ndarray:
        if isinstance(y, np.ndarray):
            y = np.ascontiguousarray(y)
        out = np.empty((self.Q, self.N), dtype=np.float64)
        self._check(sadmm_matched_filter(self._h, _ptr(y), _dtype_code(y), _on_device(y),
                                         _ptr(out)))
        return out

    def autotune(self, y, iters=8) -> int:
        """Time the forward-product tile widths on this problem, keep the
        fastest (iters = 0: report the current one)."""
        if isinstance(y, np.ndarray):
            y = np.ascontiguousarray(y)
        c = C.c_int32(0)
        self._check(sadmm_autotune(self._h, _ptr(y), _dtype_code(y), _on_device(y), int(iters),
                                   C.addressof(c)))
        return c.value

    def back_projection(self, y) -> np.ndarray:
        """|sum_q A_q^H y_q| (N doubles)."""
        if isinstance(y, np.ndarray):
            y = np.ascontiguousarray(y)
        out = np.empty(self.N, np.float64)
        self._check(sadmm_back_projection(self._h, _ptr(y), _dtype_code(y), _on_device(y), _ptr(out)))
        return out

    def set_pruning_cnn(self, cnn, threshold=0.5):
        self._cnn = cnn
        self._check(sadmm_set_pruning_cnn(self._h, cnn._h if cnn is not None else None, threshold))

    def set_profiling(self, level=1):
        self._check(sadmm_set_profiling(self._h, int(level)))

    def kernel_stats(self) -> dict:
        """{class: (launches, total_ms, work)}; work in flops (gram, inverse) or bytes."""
        out = {}
        for name, k in KERNEL_CLASSES.items():
            n = C.c_int32(0)
            ms = C.c_double(0)
            w = C.c_double(0)
            self._check(sadmm_get_kernel_stats(self._h, k, C.addressof(n), C.addressof(ms),
                                               C.addressof(w)))
            out[name] = (n.value, ms.value, w.value)
        return out

    def timing(self) -> dict:
        v = C.c_double(0)
        out = {}
        for i, k in enumerate(("total_ms", "factor_ms", "iter_ms")):
            self._check(sadmm_get_timing(self._h, i, C.byref(v)))
            out[k] = v.value
        return out


def stack_real(t, stream=None):
    """[Re S; Im S] (complex128, zero imaginary parts) of a complex device
    tensor S: an operator (N, KM) stored column-major as the tensor's rows
    (pixel-major, KM contiguous) gives (N, 2 KM); measurements (Q, KM) give
    (Q, 2 KM)."""
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    assert t.is_cuda and t.is_contiguous() and t.dim() == 2
    cols, rows = int(t.shape[0]), int(t.shape[1])
    out = torch.empty((cols, 2 * rows), dtype=torch.complex128, device=t.device)
    rc = sadmm_stack_real(t.data_ptr(), _dtype_code(t), rows, cols, rows, out.data_ptr(), C_void(stream))
    if rc != SADMM_OK:
        raise SadmmError(rc, "sadmm_stack_real failed")
    return out


def render_db(img, range_db=30.0, stream=None) -> np.ndarray:
    """8-bit levels of |img| on a range_db dynamic range (host array in, host
    array out; real float64 or complex128)."""
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    x = np.ascontiguousarray(img)
    cplx = np.iscomplexobj(x)
    x = np.ascontiguousarray(x.astype(np.complex128 if cplx else np.float64, copy=False).ravel())
    out = np.empty(x.size, np.uint8)
    rc = sadmm_render_db(_ptr(x), 1 if cplx else 0, x.size, float(range_db), 0, _ptr(out), C_void(stream))
    if rc != SADMM_OK:
        raise SadmmError(rc, "sadmm_render_db failed")
    return out


def probe_bandwidth_gbps(kind="copy", nbytes=1 << 30, reps=10, stream=None):
    """Device bandwidth in GB/s over nbytes: 'copy' (read + write bytes per
    second, non-temporal) or 'read' (bytes read per second)."""
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda") if kind == "copy" else None
    ms = C.c_double(0)
    k = {"copy": 0, "read": 1}[kind]
    rc = sadmm_probe_bandwidth(k, a.data_ptr(), b.data_ptr() if b is not None else 0, nbytes, reps,
                               C_void(stream), C.byref(ms))
    if rc != SADMM_OK:
        raise SadmmError(rc, "sadmm_probe_bandwidth failed")
    return (2.0 if k == 0 else 1.0) * nbytes / (ms.value * 1e-3) / 1e9


def probe_mfma_tops(kind, iters=4096, stream=None):
    """Register-only matrix throughput in tera-ops/s: kind 'i8' (16x16x64),
    'f64' (16x16x4) or 'i8_32' (32x32x32)."""
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    ops = C.c_double(0)
    rc = sadmm_probe_mfma({"i8": 0, "f64": 1, "i8_32": 2}[kind], iters, C_void(stream), C.byref(ops))
    if rc != SADMM_OK:
        raise SadmmError(rc, "sadmm_probe_mfma failed")
    return ops.value / 1e12


def solve_batch(solvers, ys):
    """Solve several handles in one batched iteration loop (sadmm_solve_batch).
    ys: list of measurement arrays/tensors (same dtype, all host or all device)."""
    S = len(solvers)
    ys = [np.ascontiguousarray(y) if isinstance(y, np.ndarray) else y for y in ys]
    hs = (_H * S)(*[s._h for s in solvers])
    ptrs = (C.c_void_p * S)(*[_ptr(y) for y in ys])
    infos = (sadmm_info * S)()
    rc = sadmm_solve_batch(hs, S, ptrs, _dtype_code(ys[0]), _on_device(ys[0]), infos)
    if rc != SADMM_OK:
        raise SadmmError(rc, sadmm_last_error(solvers[0]._h).decode())
    return [infos[i].as_dict() for i in range(S)]


# ---------------------------------------------------------------- CNN
CNN_LAYERS = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


class Cnn:
    """Pixel-pruning CNN handle (sadmm_cnn_*).  Parameters are exchanged as a
    dict {W1, b1, ..., W4, b4} of arrays with the shapes of the C header."""

    def __init__(self, Q, channels, H, W, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.Q, self.C, self.H, self.W = Q, channels, H, W
        self._h = _H()
        rc = sadmm_cnn_create(Q, channels, H, W, C_void(stream), C.byref(self._h))
        if rc != SADMM_OK:
            raise SadmmError(rc, "sadmm_cnn_create failed")
        self.n = int(sadmm_cnn_param_count(self._h))

    def shapes(self):
        Q, Cc = self.Q, self.C
        return {"W1": (Cc, Q, 3, 3), "b1": (Cc,), "W2": (Cc, Cc, 3, 3), "b2": (Cc,),
                "W3": (Cc, Cc, 3, 3), "b3": (Cc,), "W4": (1, Cc, 3, 3), "b4": (1,)}

    def flatten(self, params) -> np.ndarray:
        return np.concatenate([np.asarray(params[k], np.float32).reshape(-1) for k in CNN_LAYERS])

    def unflatten(self, flat) -> dict:
        out, o = {}, 0
        for k in CNN_LAYERS:
            shp = self.shapes()[k]
            sz = int(np.prod(shp))
            out[k] = np.asarray(flat[o:o + sz]).reshape(shp)
            o += sz
        return out

    def _check(self, rc):
        if rc != SADMM_OK:
            raise SadmmError(rc, sadmm_cnn_last_error(self._h).decode())

    def set_params(self, params):
        f = np.ascontiguousarray(self.flatten(params) if isinstance(params, dict) else params,
                                 dtype=np.float32)
        assert f.size == self.n
        self._check(sadmm_cnn_set_params(self._h, _ptr(f), self.n))

    def get_params(self) -> dict:
        f = np.empty(self.n, np.float32)
        self._check(sadmm_cnn_get_params(self._h, _ptr(f), self.n))
        return self.unflatten(f)

    def set_half(self, on=True):
        """Inference on FP16 matrix instructions (default) or FP32 direct convolutions."""
        self._check(sadmm_cnn_set_half(self._h, 1 if on else 0))

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        out = np.empty((self.H, self.W), np.float32)
        self._check(sadmm_cnn_forward(self._h, _ptr(x), 0, _ptr(out), 0))
        return out

    def forward_noalloc(self, x, prob):
        """Probability map of a device tensor x (Q x H x W float32, any H x W up
        to 512 x 512) into the device tensor prob (H x W float32), on the
        handle's stream, without allocating; the caller synchronises."""
        assert x.is_cuda and prob.is_cuda and x.dtype == torch.float32 and prob.dtype == torch.float32
        assert x.is_contiguous() and prob.is_contiguous() and x.dim() == 3 and x.shape[0] == self.Q
        H, W = int(x.shape[1]), int(x.shape[2])
        assert tuple(prob.shape) == (H, W)
        self._check(sadmm_cnn_forward_noalloc(self._h, x.data_ptr(), H, W, prob.data_ptr()))

    def gradients(self, x, target, pos_weight):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        g = np.empty(self.n, np.float32)
        loss = C.c_double(0)
        self._check(sadmm_cnn_gradients(self._h, _ptr(x), _ptr(t), 0, pos_weight, _ptr(g),
                                        C.byref(loss)))
        return self.unflatten(g), loss.value

    def train_step(self, x, target, pos_weight, lr) -> float:
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        loss = C.c_double(0)
        self._check(sadmm_cnn_train_step(self._h, _ptr(x), _ptr(t), 0, pos_weight, lr,
                                         C.byref(loss)))
        return loss.value

    def close(self):
        if self._h:
            sadmm_cnn_destroy(self._h)
            self._h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def C_void(v):
    return C.c_void_p(int(v) if v else None)
