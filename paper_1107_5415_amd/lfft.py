"""Thin Python binding of liblfft.so (argument marshalling only).

Every transform runs in the library's HIP kernels; PyTorch is used for device
memory and the current stream.  There is no fallback: if the library is not
built, or a call fails, a RuntimeError is raised.

Names follow the C ABI in include/lfft.h.
"""
import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LFFT_LIBRARY: load another build of the same library (the sanitized host
# build of the CPU tests); default: the in-tree build
LIB_PATH = os.environ.get("LFFT_LIBRARY") or os.path.join(_HERE, "liblfft.so")

LFFT_HOST_ONLY = 0x1
LFFT_SPLIT_BF16 = 0x2
LWT_SINGLE_STREAM = 0x4
LWT_SAMPLES = 0x8
LFFT_SAMPLES_TO_COEFFS = 0
LFFT_COEFFS_TO_SAMPLES = 1
LFFT_IN_NATURAL = 0x0
LFFT_IN_GRID = 0x1
LFFT_OUT_NATURAL = 0x0
LFFT_OUT_GRID = 0x2
LFFT_MAP_SAMPLES = 0
LFFT_MAP_FREQS = 1
LFFT_MAP_SAMPLES_T = 2
LFFT_MAP_FREQS_T = 3
LFFT_POINTS_SAMPLES = 0
LFFT_POINTS_FREQS = 1

EXPORTS = [
    "lfft_plan_create", "lfft_plan_destroy", "lfft_plan_query", "lfft_plan_query_inverse_basis",
    "lfft_plan_info", "lfft_index_map", "lfft_workspace_size", "lfft_forward", "lfft_inverse",
    "lwt_plan_create", "lwt_plan_destroy", "lwt_level_info", "lwt_level_scaling", "lwt_dirichlet_mask",
    "lwt_workspace_size", "lwt_saved_elems", "lwt_decompose", "lwt_reconstruct",
    "lwt_decompose_backward", "lwt_reconstruct_backward", "lfft_trace_begin", "lfft_trace_end",
    "lfft_trace_get", "lfft_strerror", "lfft_batch_create", "lfft_batch_destroy",
    "lfft_batch_offsets", "lfft_batch_workspace_size", "lfft_batch_configure", "lfft_batch_config",
    "lfft_batch_schedule", "lfft_batch_tune", "lfft_batch_execute", "lfft_points",
    "lwt_fiber_map", "lwt_coeff_layout", "lfft_forward_noalloc", "lfft_basis_workspace_size",
    "lfft_basis_change", "lfft_batch_tune_save", "lfft_batch_tune_load", "lfft_batch_tune_clear",
]

LFFT_BATCH_LOOP = 0
LFFT_BATCH_PERSISTENT = 1
LFFT_BATCH_GRAPH = 2

_lib = None
_lock = threading.Lock()

_P = ctypes.c_void_p
_I64P = ctypes.POINTER(ctypes.c_int64)
_I32P = ctypes.POINTER(ctypes.c_int)
_FP = ctypes.POINTER(ctypes.c_float)


class LfftError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__("%s failed: %s (status %d)" % (what, strerror(code), code))


def lib():
    """Load liblfft.so (raises RuntimeError if it is not built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblfft.so is not built (python -m paper_1107_5415_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "lfft_plan_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _I64P, ctypes.c_int64, ctypes.c_uint32]),
            "lfft_plan_destroy": (ctypes.c_int, [_P]),
            "lfft_plan_query": (ctypes.c_int, [_P, _I64P, _I32P, _I64P, _I64P, _I64P, _I64P, _I64P]),
            "lfft_plan_query_inverse_basis": (ctypes.c_int, [_P, _I64P, _I64P]),
            "lfft_plan_info": (ctypes.c_int, [_P, _I32P, _I32P, _I32P]),
            "lfft_index_map": (ctypes.c_int, [_P, ctypes.c_int, _I64P]),
            "lfft_workspace_size": (ctypes.c_size_t, [_P]),
            "lfft_forward": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_uint32, _P]),
            "lfft_inverse": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_uint32, _P]),
            "lwt_plan_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _I64P, _I64P, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32]),
            "lwt_plan_destroy": (ctypes.c_int, [_P]),
            "lwt_level_info": (ctypes.c_int, [_P, ctypes.c_int, _I64P, _I64P, _I64P]),
            "lwt_level_scaling": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                 ctypes.POINTER(ctypes.c_int), _I64P, _I64P]),
            "lwt_dirichlet_mask": (ctypes.c_int, [_P, ctypes.c_int, _FP]),
            "lwt_workspace_size": (ctypes.c_size_t, [_P]),
            "lwt_saved_elems": (ctypes.c_size_t, [_P]),
            "lwt_decompose": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
            "lwt_reconstruct": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P]),
            "lwt_decompose_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
            "lwt_reconstruct_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
            "lfft_trace_begin": (ctypes.c_int, [ctypes.c_int]),
            "lfft_trace_end": (ctypes.c_int, [_I32P]),
            "lfft_trace_get": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p),
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double), _FP]),
            "lfft_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "lfft_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_int, _I64P, ctypes.c_uint32]),
            "lfft_batch_destroy": (ctypes.c_int, [_P]),
            "lfft_batch_offsets": (ctypes.c_int, [_P, _I64P]),
            "lfft_batch_workspace_size": (ctypes.c_size_t, [_P]),
            "lfft_batch_configure": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
            "lfft_batch_config": (ctypes.c_int, [_P, _I32P, _I32P, _I32P]),
            "lfft_batch_schedule": (ctypes.c_int, [_P, ctypes.c_int, _I32P, _I64P, _I64P, _I32P]),
            "lfft_batch_tune": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, _FP, _P]),
            "lfft_batch_execute": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
            "lfft_points": (ctypes.c_int, [_P, ctypes.c_int, _I64P, _I64P]),
            "lfft_forward_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_uint32, _P]),
            "lfft_basis_workspace_size": (ctypes.c_size_t, [_P]),
            "lfft_basis_change": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
            "lwt_fiber_map": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                                             ctypes.c_int64, _I64P, _I64P]),
            "lwt_coeff_layout": (ctypes.c_int, [_P, _I32P, _I32P, _I64P, _I64P, _I32P, _I32P]),
            "lfft_batch_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
            "lfft_batch_tune_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_char_p, _I32P]),
            "lfft_batch_tune_clear": (ctypes.c_int, [_I32P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def strerror(code):
    return lib().lfft_strerror(int(code)).decode()


def _check(code, what):
    if code != 0:
        raise LfftError(code, what)


def _mat(M):
    M = np.asarray(M, dtype=np.int64)
    if M.ndim != 2 or M.shape[0] != M.shape[1]:
        raise ValueError("square integer matrix expected")
    return np.ascontiguousarray(M)


def _ptr64(a):
    return a.ctypes.data_as(_I64P)


def _torch():
    import torch
    return torch


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr())


class LatticePlan:
    """Plan of the lattice FFT on P(M) for `batch` signals (lfft_plan_*)."""

    def __init__(self, M, batch=1, host_only=False, split_bf16=False):
        self.M = _mat(M)
        self.d = self.M.shape[0]
        self.batch = int(batch)
        self.host_only = bool(host_only)
        self.split_bf16 = bool(split_bf16)
        flags = (LFFT_HOST_ONLY if host_only else 0) | (LFFT_SPLIT_BF16 if split_bf16 else 0)
        h = _P()
        _check(lib().lfft_plan_create(ctypes.byref(h), self.d, _ptr64(self.M), self.batch, flags),
               "lfft_plan_create")
        self._h = h
        self._ws = None
        q = self.query()
        self.m = q["m"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lfft_plan_destroy(h)
            self._h = None

    def query(self):
        d = self.d
        m = ctypes.c_int64()
        dM = ctypes.c_int()
        eps = np.zeros(d, np.int64)
        Q = np.zeros((d, d), np.int64)
        R = np.zeros((d, d), np.int64)
        H = np.zeros((d, d), np.int64)
        HT = np.zeros((d, d), np.int64)
        _check(lib().lfft_plan_query(self._h, ctypes.byref(m), ctypes.byref(dM), _ptr64(eps),
                                     _ptr64(Q), _ptr64(R), _ptr64(H), _ptr64(HT)), "lfft_plan_query")
        Qt = np.zeros((d, d), np.int64)
        Rt = np.zeros((d, d), np.int64)
        _check(lib().lfft_plan_query_inverse_basis(self._h, _ptr64(Qt), _ptr64(Rt)),
               "lfft_plan_query_inverse_basis")
        npass = ctypes.c_int()
        af = ctypes.c_int()
        ai = ctypes.c_int()
        _check(lib().lfft_plan_info(self._h, ctypes.byref(npass), ctypes.byref(af), ctypes.byref(ai)),
               "lfft_plan_info")
        return dict(m=m.value, d_M=dM.value, eps=eps, Q=Q, R=R, H_M=H, H_MT=HT, Qt=Qt, Rt=Rt,
                    passes=npass.value, aligned_forward=bool(af.value), aligned_inverse=bool(ai.value))

    def index_map(self, which):
        out = np.zeros(self.m, np.int64)
        _check(lib().lfft_index_map(self._h, int(which), _ptr64(out)), "lfft_index_map")
        return out

    def points(self, which):
        """(keys, sym_num) of lfft_points: int64 arrays (m, d) in natural order."""
        keys = np.zeros((self.m, self.d), np.int64)
        sym = np.zeros((self.m, self.d), np.int64)
        _check(lib().lfft_points(self._h, int(which), _ptr64(keys), _ptr64(sym)), "lfft_points")
        return keys, sym

    def workspace_bytes(self):
        return int(lib().lfft_workspace_size(self._h))

    def _workspace(self, device):
        torch = _torch()
        nb = self.workspace_bytes()
        if nb == 0:
            return None
        if self._ws is None or self._ws.device != device:
            self._ws = torch.empty(nb // 8, dtype=torch.complex64, device=device)
        return self._ws

    def _run(self, fn, x, out, layout, what):
        torch = _torch()
        if not x.is_cuda:
            raise RuntimeError("lattice FFT input must be a HIP device tensor")
        if x.dtype != torch.complex64:
            raise RuntimeError("complex64 expected")
        x = x.contiguous()
        if x.numel() != self.batch * self.m:
            raise RuntimeError("expected %d elements, got %d" % (self.batch * self.m, x.numel()))
        if out is None:
            out = torch.empty_like(x)
        ws = self._workspace(x.device)
        _check(fn(self._h, _dptr(x), _dptr(out), _dptr(ws) if ws is not None else None,
                  int(layout), _stream_handle(x.device)), what)
        return out

    def forward(self, x, out=None, layout=0):
        return self._run(lib().lfft_forward, x, out, layout, "lfft_forward")

    def inverse(self, x, out=None, layout=0):
        return self._run(lib().lfft_inverse, x, out, layout, "lfft_inverse")

    def basis_change(self, x, direction=LFFT_SAMPLES_TO_COEFFS, fourier=False, out=None):
        """lfft_basis_change: point values on P(M) <-> coefficients in the
        orthonormal translates of the Dirichlet kernel (fourier=True: the
        coefficient side is F(M) a in natural G(M^T) order)."""
        torch = _torch()
        if not x.is_cuda or x.dtype != torch.complex64:
            raise RuntimeError("complex64 device tensor expected")
        x = x.contiguous()
        if x.numel() != self.batch * self.m:
            raise RuntimeError("expected %d elements, got %d" % (self.batch * self.m, x.numel()))
        if out is None:
            out = torch.empty_like(x)
        nb = int(lib().lfft_basis_workspace_size(self._h))
        ws = torch.empty(max(nb // 8, 1), dtype=torch.complex64, device=x.device)
        _check(lib().lfft_basis_change(self._h, int(direction), 1 if fourier else 0, _dptr(x),
                                       _dptr(out), _dptr(ws), _stream_handle(x.device)),
               "lfft_basis_change")
        return out

    def forward_noalloc(self, x, out, layout=0):
        """lfft_forward_noalloc: the library allocates nothing; `out` must be
        a preallocated complex64 device tensor like x."""
        torch = _torch()
        if not x.is_cuda or x.dtype != torch.complex64 or not x.is_contiguous():
            raise RuntimeError("contiguous complex64 device tensor expected")
        if x.numel() != self.batch * self.m or out.numel() != x.numel() or not out.is_contiguous():
            raise RuntimeError("expected %d elements in and out" % (self.batch * self.m))
        _check(lib().lfft_forward_noalloc(self._h, _dptr(x), _dptr(out), int(layout),
                                          _stream_handle(x.device)), "lfft_forward_noalloc")
        return out


_plan_cache = {}


def get_plan(M, batch=1):
    key = (tuple(map(tuple, _mat(M).tolist())), int(batch))
    p = _plan_cache.get(key)
    if p is None:
        p = LatticePlan(M, batch)
        _plan_cache[key] = p
    return p


def forward(x, M):
    """Unitary lattice DFT of x (complex64 [..., m], natural sample order)."""
    m = x.shape[-1]
    b = x.numel() // m
    return get_plan(M, b).forward(x).reshape(x.shape)


def inverse(x, M):
    m = x.shape[-1]
    b = x.numel() // m
    return get_plan(M, b).inverse(x).reshape(x.shape)


_wave_cache = {}
_mask_cache = {}


def _wave_key(M, J, levels, batch):
    return (tuple(map(tuple, _mat(M).tolist())), tuple(map(tuple, _mat(J).tolist())), int(levels),
            int(batch))


def get_wavelet_plan(M, J, levels, batch=1):
    key = _wave_key(M, J, levels, batch)
    p = _wave_cache.get(key)
    if p is None:
        p = WaveletPlan(M, J, levels, batch)
        _wave_cache[key] = p
    return p


def _pyramid(x, M, J, levels, masks):
    m = x.shape[-1]
    b = x.numel() // m
    key = _wave_key(M, J, levels, b)
    plan = get_wavelet_plan(M, J, levels, b)
    if masks is None:
        mk = (key, str(x.device))
        if mk not in _mask_cache:
            _mask_cache[mk] = plan.dirichlet_masks(x.device)
        masks = _mask_cache[mk]
    return plan, masks


def decompose(x, M, J, levels, masks=None):
    """Wavelet pyramid coefficients of x (complex64 [..., m], natural sample
    order of M) for `levels` splits M_l = J M_{l+1}; masks: one float32
    device tensor per level in natural G(M_l^T) order (None: the Dirichlet
    masks).  The coefficient layout is WaveletPlan.coeff_blocks()."""
    plan, masks = _pyramid(x, M, J, levels, masks)
    return plan.decompose(x.reshape(-1), masks).reshape(x.shape)


def reconstruct(c, M, J, levels, masks=None):
    """Inverse of decompose (same arguments)."""
    plan, masks = _pyramid(c, M, J, levels, masks)
    return plan.reconstruct(c.reshape(-1), masks).reshape(c.shape)


class WaveletPlan:
    """Plan of the multi-level lattice wavelet pyramid (lwt_plan_*)."""

    def __init__(self, M, J, levels, batch=1, host_only=False, single_stream=False, samples=False):
        self.M = _mat(M)
        self.J = _mat(J)
        self.d = self.M.shape[0]
        self.levels = int(levels)
        self.batch = int(batch)
        h = _P()
        _check(lib().lwt_plan_create(ctypes.byref(h), self.d, _ptr64(self.M), _ptr64(self.J),
                                     self.levels, self.batch,
                                     (LFFT_HOST_ONLY if host_only else 0) |
                                     (LWT_SINGLE_STREAM if single_stream else 0) |
                                     (LWT_SAMPLES if samples else 0)),
               "lwt_plan_create")
        self._h = h
        self._ws = None
        self.level_m = []
        self.level_N = []
        for l in range(self.levels):
            N = np.zeros((self.d, self.d), np.int64)
            ml = ctypes.c_int64()
            eps = np.zeros(self.d, np.int64)
            _check(lib().lwt_level_info(self._h, l, _ptr64(N), ctypes.byref(ml), _ptr64(eps)),
                   "lwt_level_info")
            self.level_m.append(ml.value)
            self.level_N.append(N)
        self.m = self.level_m[0]
        q = ctypes.c_int()
        nb = ctypes.c_int()
        _check(lib().lwt_coeff_layout(self._h, ctypes.byref(q), ctypes.byref(nb), None, None, None,
                                      None), "lwt_coeff_layout")
        self.q = q.value
        off = np.zeros(nb.value, np.int64)
        ln = np.zeros(nb.value, np.int64)
        lv = (ctypes.c_int * nb.value)()
        ch = (ctypes.c_int * nb.value)()
        _check(lib().lwt_coeff_layout(self._h, None, None, _ptr64(off), _ptr64(ln),
                                      ctypes.cast(lv, _I32P), ctypes.cast(ch, _I32P)),
               "lwt_coeff_layout")
        self._blocks = [(int(lv[i]), int(ch[i]), int(off[i]), int(ln[i])) for i in range(nb.value)]

    def coeff_blocks(self):
        """[(level, channel, offset, length)] of the coefficient blocks of one
        signal, as lwt_coeff_layout reports them: channels 1 .. q-1 of every
        level, then channel 0 of the last level."""
        return list(self._blocks)

    def fiber_map(self, level, path=0, k0=0, count=None):
        """(lifts, phase) of lwt_fiber_map for the natural indices k0 ..
        k0+count-1 of G(N_l^T): lifts int64 (count, q); phase int64 (count,)
        for q = 2, None for q > 2."""
        n = self.level_m[level] // self.q
        if count is None:
            count = n - k0
        lifts = np.zeros((count, self.q), np.int64)
        phase = np.zeros(count, np.int64) if self.q == 2 else None
        _check(lib().lwt_fiber_map(self._h, int(level), int(path), int(k0), int(count),
                                   _ptr64(lifts), _ptr64(phase) if phase is not None else None),
               "lwt_fiber_map")
        return lifts, phase

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lwt_plan_destroy(h)
            self._h = None

    def level_scaling(self, level):
        """Theorem 3 report of level l: dict(d_M, d_N, adds, key, grid)."""
        dm, dn = ctypes.c_int(), ctypes.c_int()
        key = np.zeros(self.d, np.int64)
        grid = np.zeros(self.d, np.int64)
        _check(lib().lwt_level_scaling(self._h, int(level), ctypes.byref(dm), ctypes.byref(dn),
                                       _ptr64(key), _ptr64(grid)), "lwt_level_scaling")
        return dict(d_M=dm.value, d_N=dn.value, adds=dm.value - dn.value,
                    key=tuple(int(v) for v in key), grid=tuple(int(v) for v in grid))

    def dirichlet_mask(self, level):
        out = np.zeros(self.level_m[level], np.float32)
        _check(lib().lwt_dirichlet_mask(self._h, int(level), out.ctypes.data_as(_FP)),
               "lwt_dirichlet_mask")
        return out

    def dirichlet_masks(self, device=None):
        torch = _torch()
        ms = [self.dirichlet_mask(l) for l in range(self.levels)]
        if device is None:
            return ms
        return [torch.from_numpy(a).to(device) for a in ms]

    def saved_elems(self):
        return int(lib().lwt_saved_elems(self._h))

    def _workspace(self, device):
        torch = _torch()
        nb = int(lib().lwt_workspace_size(self._h))
        if self._ws is None or self._ws.device != device:
            self._ws = torch.empty(max(nb // 8, 1), dtype=torch.complex64, device=device)
        return self._ws

    def _masks(self, masks):
        torch = _torch()
        if len(masks) != self.levels:
            raise RuntimeError("one mask per level expected")
        ms = []
        for l, mk in enumerate(masks):
            if mk.dtype != torch.float32 or not mk.is_cuda or mk.numel() != self.level_m[l]:
                raise RuntimeError("mask %d must be a float32 device tensor of %d elements" % (l, self.level_m[l]))
            ms.append(mk.contiguous())
        arr = (ctypes.c_void_p * self.levels)(*[m.data_ptr() for m in ms])
        return ms, arr

    def _grad_masks(self, gmasks):
        if gmasks is None:
            return None
        return (ctypes.c_void_p * self.levels)(*[g.data_ptr() for g in gmasks])

    def _check_signal(self, x):
        torch = _torch()
        if not x.is_cuda or x.dtype != torch.complex64 or x.numel() != self.batch * self.m:
            raise RuntimeError("complex64 device tensor of %d elements expected" % (self.batch * self.m))
        return x.contiguous()

    def new_saved(self, device):
        torch = _torch()
        return torch.empty(self.saved_elems(), dtype=torch.complex64, device=device)

    def decompose(self, x, masks, saved=None, out=None):
        torch = _torch()
        x = self._check_signal(x)
        ms, arr = self._masks(masks)
        if out is None:
            out = torch.empty_like(x)
        ws = self._workspace(x.device)
        _check(lib().lwt_decompose(self._h, _dptr(x), ctypes.cast(arr, _P), _dptr(out),
                                   _dptr(saved) if saved is not None else None, _dptr(ws),
                                   _stream_handle(x.device)), "lwt_decompose")
        return out

    def reconstruct(self, c, masks, saved=None, out=None):
        torch = _torch()
        c = self._check_signal(c)
        ms, arr = self._masks(masks)
        if out is None:
            out = torch.empty_like(c)
        ws = self._workspace(c.device)
        _check(lib().lwt_reconstruct(self._h, _dptr(c), ctypes.cast(arr, _P), _dptr(out),
                                     _dptr(saved) if saved is not None else None, _dptr(ws),
                                     _stream_handle(c.device)), "lwt_reconstruct")
        return out

    def decompose_backward(self, grad_c, saved, masks, grad_masks=None):
        torch = _torch()
        g = self._check_signal(grad_c)
        ms, arr = self._masks(masks)
        gx = torch.empty_like(g)
        gm = self._grad_masks(grad_masks)
        ws = self._workspace(g.device)
        _check(lib().lwt_decompose_backward(self._h, _dptr(g), _dptr(saved) if saved is not None else None,
                                            ctypes.cast(arr, _P), _dptr(gx),
                                            ctypes.cast(gm, _P) if gm is not None else None,
                                            _dptr(ws), _stream_handle(g.device)),
               "lwt_decompose_backward")
        return gx

    def reconstruct_backward(self, grad_x, saved, masks, grad_masks=None):
        torch = _torch()
        g = self._check_signal(grad_x)
        ms, arr = self._masks(masks)
        gc = torch.empty_like(g)
        gm = self._grad_masks(grad_masks)
        ws = self._workspace(g.device)
        _check(lib().lwt_reconstruct_backward(self._h, _dptr(g), _dptr(saved) if saved is not None else None,
                                              ctypes.cast(arr, _P), _dptr(gc),
                                              ctypes.cast(gm, _P) if gm is not None else None,
                                              _dptr(ws), _stream_handle(g.device)),
               "lwt_reconstruct_backward")
        return gc


class BatchPlan:
    """Lattice FFTs of signals on patterns of different M in one call
    (lfft_batch_*).  Signals are concatenated: signal i occupies elements
    offsets[i]:offsets[i+1] of a complex64 device tensor."""

    def __init__(self, Ms, host_only=False):
        Ms = [_mat(M) for M in Ms]
        if not Ms:
            raise ValueError("at least one matrix expected")
        self.d = Ms[0].shape[0]
        if any(M.shape != (self.d, self.d) for M in Ms):
            raise ValueError("all matrices must have the same dimension")
        self.count = len(Ms)
        self.Ms = np.ascontiguousarray(np.stack(Ms))
        h = _P()
        _check(lib().lfft_batch_create(ctypes.byref(h), self.count, self.d, _ptr64(self.Ms),
                                       LFFT_HOST_ONLY if host_only else 0), "lfft_batch_create")
        self._h = h
        self._ws = None
        off = np.zeros(self.count + 1, np.int64)
        _check(lib().lfft_batch_offsets(self._h, _ptr64(off)), "lfft_batch_offsets")
        self.offsets = off
        self.total = int(off[-1])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lfft_batch_destroy(h)
            self._h = None

    def configure(self, tile_lg, order=0):
        _check(lib().lfft_batch_configure(self._h, int(tile_lg), int(order)), "lfft_batch_configure")

    def config(self):
        t = ctypes.c_int()
        o = ctypes.c_int()
        e = ctypes.c_int()
        _check(lib().lfft_batch_config(self._h, ctypes.byref(t), ctypes.byref(o), ctypes.byref(e)),
               "lfft_batch_config")
        return dict(tile_lg=t.value, order=o.value, eligible=e.value)

    def schedule(self, i):
        n = ctypes.c_int()
        L = np.zeros(2, np.int64)
        T = np.zeros(2, np.int64)
        post = (ctypes.c_int * 2)()
        _check(lib().lfft_batch_schedule(self._h, int(i), ctypes.byref(n), _ptr64(L), _ptr64(T),
                                         ctypes.cast(post, _I32P)), "lfft_batch_schedule")
        k = n.value
        return dict(passes=k, pencil=L[:k].tolist(), tiles=T[:k].tolist(), post=list(post)[:k])

    def _workspace(self, device):
        torch = _torch()
        nb = int(lib().lfft_batch_workspace_size(self._h))
        if self._ws is None or self._ws.device != device:
            self._ws = torch.empty(max(nb // 8, 1), dtype=torch.complex64, device=device)
        return self._ws

    def _check_signal(self, x):
        torch = _torch()
        if not x.is_cuda or x.dtype != torch.complex64 or x.numel() != self.total:
            raise RuntimeError("complex64 device tensor of %d elements expected" % self.total)
        return x.contiguous()

    def execute(self, x, inverse=False, mode=LFFT_BATCH_GRAPH, out=None):
        torch = _torch()
        x = self._check_signal(x)
        if out is None:
            out = torch.empty_like(x)
        ws = self._workspace(x.device)
        _check(lib().lfft_batch_execute(self._h, 1 if inverse else 0, int(mode), _dptr(x), _dptr(out),
                                        _dptr(ws), _stream_handle(x.device)), "lfft_batch_execute")
        return out

    def tune(self, x, reps=3, out=None):
        """Autotune on x (overwrites out); returns the best time in ms (-1 if
        the choice was already known for these matrices)."""
        torch = _torch()
        x = self._check_signal(x)
        if out is None:
            out = torch.empty_like(x)
        ws = self._workspace(x.device)
        best = ctypes.c_float()
        _check(lib().lfft_batch_tune(self._h, _dptr(x), _dptr(out), _dptr(ws), int(reps),
                                     ctypes.byref(best), _stream_handle(x.device)), "lfft_batch_tune")
        return best.value


def tune_save(path):
    """Write every remembered autotuner choice to `path` (lfft_batch_tune_save)."""
    _check(lib().lfft_batch_tune_save(os.fsencode(path)), "lfft_batch_tune_save")


def tune_load(path, arch=None):
    """Merge the choices for `arch` (None: the current device's) from a file
    written by tune_save; returns how many were taken (lfft_batch_tune_load)."""
    n = ctypes.c_int()
    _check(lib().lfft_batch_tune_load(os.fsencode(path), None if arch is None else arch.encode(),
                                      ctypes.byref(n)), "lfft_batch_tune_load")
    return n.value


def tune_clear():
    """Forget every remembered autotuner choice; returns how many there were."""
    n = ctypes.c_int()
    _check(lib().lfft_batch_tune_clear(ctypes.byref(n)), "lfft_batch_tune_clear")
    return n.value


def trace_begin(capacity=100000):
    """Start per-launch kernel timing (lfft_trace_begin)."""
    _check(lib().lfft_trace_begin(int(capacity)), "lfft_trace_begin")


def trace_end():
    """Stop timing and return [(kernel, method_bytes, pass_bytes, ms), ...]."""
    n = ctypes.c_int()
    _check(lib().lfft_trace_end(ctypes.byref(n)), "lfft_trace_end")
    out = []
    for i in range(n.value):
        name = ctypes.c_char_p()
        b = ctypes.c_double()
        pb = ctypes.c_double()
        ms = ctypes.c_float()
        _check(lib().lfft_trace_get(i, ctypes.byref(name), ctypes.byref(b), ctypes.byref(pb),
                                    ctypes.byref(ms)), "lfft_trace_get")
        out.append((name.value.decode(), b.value, pb.value, ms.value))
    return out
