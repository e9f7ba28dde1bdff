"""Thin Python binding of libgbs (include/gbs.h): argument marshalling only.

Device memory and streams come from PyTorch (ROCm): every context's workspace and every state's
memory are torch tensors (the library never allocates device memory; a call that finds the
workspace too small returns GBS_ENOMEM with the size it needs, and the binding installs a larger
tensor and repeats the call). Every computation runs in the HIP library. There is no CPU fallback:
if libgbs.so is missing or the device is not gfx950, the calls raise.
"""
from __future__ import annotations

import ctypes
import pathlib
from typing import Optional, Tuple

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
LIB_PATH = _HERE / "libgbs.so"

GBS_OK, GBS_EINVAL, GBS_ERANGE, GBS_ENOMEM, GBS_EHIP, GBS_EUNSUPPORTED = range(6)
GBS_N_MAX = 46
GBS_MARGINAL_KMAX = 20
GBS_PREC_FP64, GBS_PREC_DD = 0, 1
GBS_SHAPE_TILE_9_10, GBS_SHAPE_TILE_11_12, GBS_SHAPE_SQT_11_12, GBS_SHAPE_SQT_9_10 = 1, 2, 4, 8
GBS_SHAPE_SQT_13_14 = 16

# Every function declared in include/gbs.h.
EXPORTS = [
    "gbs_ctx_create", "gbs_ctx_destroy", "gbs_ctx_set_workspace", "gbs_ctx_workspace_needed", "gbs_status_str",
    "gbs_last_error", "gbs_ctx_set_exec", "gbs_ctx_set_precision", "gbs_ctx_get_precision", "gbs_debug_fault_inject",
    "gbs_debug_check_symmetry", "gbs_ctx_set_streams", "gbs_ctx_get_streams", "gbs_ctx_set_tuning", "gbs_ctx_get_tuning", "gbs_ctx_set_shape", "gbs_ctx_get_shape", "gbs_haf_flops",
    "haf_batch", "haf_batch_varlen", "haf_batch_noalloc", "gbs_state_bytes", "gbs_state_create", "gbs_state_destroy",
    "gbs_state_info", "gbs_state_copy_B", "gbs_prob_batch", "gbs_subset_count", "gbs_prob_slices",
    "gbs_finalize", "gbs_marginal_batch", "gbs_photon_number_pmf", "gbs_sample_step", "gbs_sweep_count",
    "gbs_prob_sweep", "gbs_sweep_sample",
]

_lib = None


def debug_fault_inject(launch_n: int) -> None:
    """The launch_n-th compute call from now on fails with GBS_EHIP (enqueueing nothing); <= 0: off."""
    lib().gbs_debug_fault_inject(int(launch_n))


def debug_check_symmetry(on: bool) -> None:
    """Check caller-provided matrices for symmetry before the hafnian path (GBS_EINVAL if not)."""
    lib().gbs_debug_check_symmetry(1 if on else 0)


class GBSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class PartialT(ctypes.Structure):
    _fields_ = [("s_re", ctypes.c_double), ("s_im", ctypes.c_double), ("c_re", ctypes.c_double),
                ("c_im", ctypes.c_double)]


def lib() -> ctypes.CDLL:
    """Load the in-tree libgbs.so (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(str(LIB_PATH))
    vp, i32, i64, sz, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p
    sig = {
        "gbs_ctx_create": (ctypes.c_int, [ctypes.c_int, vp, sz, ctypes.POINTER(vp)]),
        "gbs_ctx_destroy": (ctypes.c_int, [vp]),
        "gbs_ctx_set_workspace": (ctypes.c_int, [vp, vp, sz]),
        "gbs_ctx_workspace_needed": (sz, [vp]),
        "gbs_state_bytes": (sz, [i32]),
        "gbs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
        "gbs_last_error": (ctypes.c_char_p, [vp]),
        "gbs_ctx_set_exec": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int]),
        "gbs_ctx_set_precision": (ctypes.c_int, [vp, i32]),
        "gbs_debug_fault_inject": (ctypes.c_int, [i64]),
        "gbs_debug_check_symmetry": (ctypes.c_int, [i32]),
        "gbs_ctx_get_precision": (i32, [vp]),
        "gbs_ctx_set_streams": (ctypes.c_int, [vp, i32]),
        "gbs_ctx_get_streams": (ctypes.c_int, [vp, ctypes.POINTER(i32)]),
        "gbs_ctx_set_tuning": (ctypes.c_int, [vp, i32, i64, i64]),
        "gbs_ctx_get_tuning": (ctypes.c_int, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "gbs_ctx_set_shape": (ctypes.c_int, [vp, i32, i32]),
        "gbs_ctx_get_shape": (ctypes.c_int, [vp, i32, ctypes.POINTER(i32)]),
        "gbs_haf_flops": (ctypes.c_double, [i32]),
        "haf_batch": (ctypes.c_int, [vp, dp, i32, i64, i64, dp, vp]),
        "haf_batch_varlen": (ctypes.c_int, [vp, dp, dp, dp, i64, dp, vp]),
        "haf_batch_noalloc": (ctypes.c_int, [vp, dp, i32, i64, i64, dp, vp]),
        "gbs_state_create": (ctypes.c_int, [vp, dp, i32, dp, dp, sz, vp, ctypes.POINTER(vp)]),
        "gbs_state_destroy": (ctypes.c_int, [vp]),
        "gbs_state_info": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]),
        "gbs_state_copy_B": (ctypes.c_int, [vp, dp, vp]),
        "gbs_prob_batch": (ctypes.c_int, [vp, vp, dp, dp, i64, dp, dp, vp]),
        "gbs_subset_count": (i64, [i32]),
        "gbs_prob_slices": (ctypes.c_int, [vp, vp, dp, dp, dp, dp, i64, dp, dp, vp]),
        "gbs_finalize": (ctypes.c_int, [vp, vp, dp, dp, dp, dp, dp, i64, dp, dp, vp]),  # modes, offsets
        "gbs_marginal_batch": (ctypes.c_int, [vp, vp, i32, dp, dp, i64, dp, vp]),
        "gbs_photon_number_pmf": (ctypes.c_int, [i32, ctypes.c_double, i32, dp]),
        "gbs_sample_step": (ctypes.c_int, [vp, vp, i32, dp, dp, i64, dp, dp, dp, vp]),
        "gbs_sweep_count": (i64, [i32, i32, i32]),
        "gbs_prob_sweep": (ctypes.c_int, [vp, vp, i32, i32, dp, dp, vp]),
        "gbs_sweep_sample": (ctypes.c_int, [vp, dp, i64, dp, i64, dp, dp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def haf_flops(n: int) -> float:
    """Algorithmic FP64 flops of one size-n hafnian as the library schedules it."""
    return float(lib().gbs_haf_flops(int(n)))


def subset_count(n: int) -> int:
    return int(lib().gbs_subset_count(int(n)))


def _np_ptr(a: Optional[np.ndarray]):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _t_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream) -> Optional[ctypes.c_void_p]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def pack_patterns(patterns) -> Tuple[np.ndarray, np.ndarray]:
    """Mode lists (or an (count, n) int array) -> (modes int32, offsets int64)."""
    if isinstance(patterns, tuple) and len(patterns) == 2:
        modes = np.ascontiguousarray(patterns[0], dtype=np.int32)
        offsets = np.ascontiguousarray(patterns[1], dtype=np.int64)
        if offsets.ndim != 1 or len(offsets) < 1 or offsets[-1] > len(modes) or offsets[0] != 0:
            raise ValueError("offsets must start at 0 and end within the modes array")
        return modes, offsets
    if isinstance(patterns, np.ndarray) and patterns.ndim == 2:
        cnt, n = patterns.shape
        return (np.ascontiguousarray(patterns, dtype=np.int32).reshape(-1),
                np.arange(cnt + 1, dtype=np.int64) * n)
    lens = np.fromiter((len(p) for p in patterns), dtype=np.int64, count=len(patterns))
    offsets = np.zeros(len(patterns) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    modes = np.zeros(int(offsets[-1]), dtype=np.int32)
    for i, p in enumerate(patterns):
        modes[offsets[i]:offsets[i + 1]] = p
    return modes, offsets


class State:
    """A resident GBS state: U, B = U diag(tanh r) U^t and 1/prod cosh r on the device."""

    def __init__(self, ctx: "Context", U, r, stream=None):
        import torch
        if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.complex128):
            raise TypeError("U must be a complex128 CUDA tensor")
        U = U.contiguous()
        m = U.shape[0]
        if U.shape != (m, m):
            raise ValueError("U must be square")
        r = np.ascontiguousarray(np.broadcast_to(np.asarray(r, dtype=np.float64), (m,)))
        self._ctx = ctx
        self.m = m
        self._U = U  # read by the state kernel on the stream
        nbytes = int(lib().gbs_state_bytes(m))
        if nbytes == 0:
            raise ValueError(f"m = {m} outside the supported range")
        self._mem = torch.empty(nbytes, dtype=torch.uint8, device=ctx.torch_device)
        h = ctypes.c_void_p()
        ctx._check(lib().gbs_state_create(ctx.handle, _t_ptr(U), m, _np_ptr(r), _t_ptr(self._mem), nbytes,
                                          _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def info(self):
        b = ctypes.c_void_p()
        m = ctypes.c_int32()
        pf = ctypes.c_double()
        rc = lib().gbs_state_info(self.handle, ctypes.byref(b), ctypes.byref(m), ctypes.byref(pf))
        if rc:
            raise GBSError(rc, "gbs_state_info failed")
        return b.value, m.value, pf.value

    def B(self, stream=None):
        """A complex128 CUDA tensor copy of B."""
        import torch
        out = torch.empty((self.m, self.m), dtype=torch.complex128, device=self._ctx.torch_device)
        rc = lib().gbs_state_copy_B(self.handle, _t_ptr(out), _stream_ptr(stream))
        if rc:
            raise GBSError(rc, "gbs_state_copy_B failed")
        return out

    @property
    def prefactor(self) -> float:
        return self.info()[2]

    def close(self):
        if getattr(self, "handle", None):
            lib().gbs_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A libgbs context on one device (staging buffers, workspace, graphs, tuning table)."""

    def __init__(self, device: int = 0, workspace=None, use_graph: bool = True, persistent: bool = True,
                 workspace_bytes: int = 16 << 20, grow: bool = True):
        """workspace: a device tensor to use as the workspace (fixed: calls that need more raise
        GBSError(GBS_ENOMEM)); by default a uint8 tensor of workspace_bytes that grows on demand."""
        import torch
        self.device = int(device)
        self.torch_device = torch.device("cuda", self.device)
        if workspace is None:
            workspace = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=self.torch_device)
        else:
            grow = False
        self._ws = workspace
        self._grow = grow
        h = ctypes.c_void_p()
        rc = lib().gbs_ctx_create(self.device, _t_ptr(workspace), self._ws_bytes(), ctypes.byref(h))
        if rc:
            raise GBSError(rc, f"gbs_ctx_create: {lib().gbs_status_str(rc).decode()}")
        self.handle = h
        self.set_exec(use_graph, persistent)

    def _ws_bytes(self) -> int:
        return self._ws.numel() * self._ws.element_size()

    # -- errors
    def _check(self, rc: int):
        if rc:
            msg = lib().gbs_last_error(self.handle).decode()
            raise GBSError(rc, f"{lib().gbs_status_str(rc).decode()}: {msg}")

    def _run(self, fn, *args):
        """Call fn(handle, *args); on GBS_ENOMEM install a workspace of the size the call needed and
        call once more (the library enqueues nothing on that error)."""
        import torch
        rc = fn(self.handle, *args)
        if rc == GBS_ENOMEM and self._grow:
            need = int(lib().gbs_ctx_workspace_needed(self.handle))
            if need > self._ws_bytes():
                new = torch.empty(need + need // 4, dtype=torch.uint8, device=self.torch_device)
                self._check(lib().gbs_ctx_set_workspace(self.handle, _t_ptr(new), new.numel()))
                self._ws = new
                rc = fn(self.handle, *args)
        self._check(rc)

    def close(self):
        if getattr(self, "handle", None):
            lib().gbs_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- options
    def set_exec(self, use_graph: bool = True, persistent: bool = True):
        self._check(lib().gbs_ctx_set_exec(self.handle, int(use_graph), int(persistent)))

    def set_precision(self, precision):
        """'fp64' (default) or 'dd' (double-double subset sum), or GBS_PREC_FP64 / GBS_PREC_DD."""
        code = {"fp64": GBS_PREC_FP64, "dd": GBS_PREC_DD}.get(precision, precision)
        self._check(lib().gbs_ctx_set_precision(self.handle, int(code)))

    @property
    def precision(self) -> str:
        return "dd" if lib().gbs_ctx_get_precision(self.handle) == GBS_PREC_DD else "fp64"

    def set_streams(self, nstreams: int):
        """Spread a call's engine kernels over nstreams internal streams (1 = all on the call's stream;
        a new context uses 2)."""
        self._check(lib().gbs_ctx_set_streams(self.handle, int(nstreams)))

    @property
    def streams(self) -> int:
        v = ctypes.c_int32()
        self._check(lib().gbs_ctx_get_streams(self.handle, ctypes.byref(v)))
        return v.value

    def set_tuning(self, n: int, chunk_small: int, chunk_large: int):
        self._check(lib().gbs_ctx_set_tuning(self.handle, int(n), int(chunk_small), int(chunk_large)))

    def _copy_tuning_from(self, other: "Context"):
        """The launch-shape table of another context: chunk sizes and engine shape for every n."""
        for n in range(0, GBS_N_MAX + 1):
            self.set_tuning(n, *other.get_tuning(n))
            self.set_shape(n, other.get_shape(n))

    def set_shape(self, n: int, shape: int):
        """Engine shape bits for size-n patterns (GBS_SHAPE_*); -1 restores the built-in choice."""
        self._check(lib().gbs_ctx_set_shape(self.handle, int(n), int(shape)))

    def get_shape(self, n: int) -> int:
        v = ctypes.c_int32()
        self._check(lib().gbs_ctx_get_shape(self.handle, int(n), ctypes.byref(v)))
        return v.value

    def get_tuning(self, n: int) -> Tuple[int, int]:
        a, b = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().gbs_ctx_get_tuning(self.handle, int(n), ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    # -- hafnians
    def haf_batch(self, A, out=None, stream=None):
        """Hafnians of a (batch, n, n) complex128 CUDA tensor -> (batch,) complex128 tensor."""
        import torch
        if not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.complex128 and A.ndim == 3):
            raise TypeError("A must be a (batch, n, n) complex128 CUDA tensor")
        if A.shape[1] != A.shape[2]:
            raise ValueError("matrices must be square")
        A = A.contiguous()
        b, n = A.shape[0], A.shape[1]
        if out is None:
            out = torch.empty(b, dtype=torch.complex128, device=A.device)
        self._run(lib().haf_batch, _t_ptr(A), n, b, n * n, _t_ptr(out), _stream_ptr(stream))
        return out

    def haf_batch_noalloc(self, A, out, stream=None):
        """haf_batch through the entry point that allocates nothing (static device scratch); `out` is
        required, and the binding allocates nothing either."""
        import torch
        if not (isinstance(A, torch.Tensor) and A.is_cuda and A.dtype == torch.complex128 and A.ndim == 3
                and A.is_contiguous() and A.shape[1] == A.shape[2]):
            raise TypeError("A must be a contiguous (batch, n, n) complex128 CUDA tensor")
        if not (out.is_cuda and out.dtype == torch.complex128 and out.is_contiguous() and out.numel() == A.shape[0]):
            raise TypeError("out must be a contiguous complex128 CUDA tensor with one entry per matrix")
        b, n = A.shape[0], A.shape[1]
        self._check(lib().haf_batch_noalloc(self.handle, _t_ptr(A), n, b, n * n, _t_ptr(out), _stream_ptr(stream)))
        return out

    def haf_batch_varlen(self, A_flat, elem_off, ns, out=None, stream=None):
        import torch
        elem_off = np.ascontiguousarray(elem_off, dtype=np.int64)
        ns = np.ascontiguousarray(ns, dtype=np.int32)
        if out is None:
            out = torch.empty(len(ns), dtype=torch.complex128, device=A_flat.device)
        self._run(lib().haf_batch_varlen, _t_ptr(A_flat), _np_ptr(elem_off), _np_ptr(ns), len(ns), _t_ptr(out),
                  _stream_ptr(stream))
        return out

    # -- probabilities
    def state(self, U, r, stream=None) -> State:
        return State(self, U, r, stream)

    def prob_batch(self, state: State, patterns, want_haf: bool = False, prob_out=None, haf_out=None, stream=None):
        """Probabilities (and optionally hafnians) of output patterns against `state`."""
        import torch
        modes, offsets = pack_patterns(patterns)
        b = len(offsets) - 1
        if prob_out is None:
            prob_out = torch.empty(b, dtype=torch.float64, device=self.torch_device)
        if want_haf and haf_out is None:
            haf_out = torch.empty(b, dtype=torch.complex128, device=self.torch_device)
        self._run(lib().gbs_prob_batch, state.handle, _np_ptr(modes), _np_ptr(offsets), b, _t_ptr(prob_out),
                  _t_ptr(haf_out), _stream_ptr(stream))
        return (prob_out, haf_out) if want_haf else prob_out

    def marginal_batch(self, state: State, n: int, prefixes, q_out=None, stream=None):
        """Marginal probabilities q_n(x_1..x_k) of position prefixes for n photons (Theorem 1)."""
        import torch
        modes, offsets = pack_patterns(prefixes)
        b = len(offsets) - 1
        if q_out is None:
            q_out = torch.empty(b, dtype=torch.float64, device=self.torch_device)
        self._run(lib().gbs_marginal_batch, state.handle, int(n), _np_ptr(modes), _np_ptr(offsets), b, _t_ptr(q_out),
                  _stream_ptr(stream))
        return q_out

    def sample_step(self, state: State, n: int, prefixes, uniforms, weights_out=None, stream=None):
        """One chain-rule step: the next position of every prefix, drawn by inverse CDF with the given
        uniforms (a CUDA float64 tensor, one per prefix) -> int32 tensor; optionally the weights."""
        import torch
        modes, offsets = pack_patterns(prefixes)
        b = len(offsets) - 1
        if uniforms.dtype != torch.float64 or not uniforms.is_cuda or uniforms.numel() != b:
            raise ValueError("uniforms must be a CUDA float64 tensor with one value per prefix")
        nxt = torch.empty(b, dtype=torch.int32, device=self.torch_device)
        u = uniforms.contiguous()
        if weights_out is not None and (weights_out.dtype != torch.float64 or not weights_out.is_contiguous()
                                        or weights_out.numel() != b * state.m):
            raise ValueError("weights_out must be a contiguous float64 tensor of prefixes x m")
        self._run(lib().gbs_sample_step, state.handle, int(n), _np_ptr(modes), _np_ptr(offsets), b, _t_ptr(u),
                  _t_ptr(weights_out), _t_ptr(nxt), _stream_ptr(stream))
        return nxt

    def prob_sweep(self, state: State, n: int, collisions: bool = True, want_haf: bool = False, prob_out=None,
                   haf_out=None, stream=None):
        """Probabilities (and optionally hafnians) of every pattern of n photons, in lexicographic order
        of the sorted mode lists (itertools.combinations_with_replacement, or combinations)."""
        import torch
        count = sweep_count(state.m, n, collisions)
        if count < 0:
            raise GBSError(GBS_ERANGE, f"sweep of n = {n} over m = {state.m} modes is too large")
        if prob_out is None:
            prob_out = torch.empty(count, dtype=torch.float64, device=self.torch_device)
        if want_haf and haf_out is None:
            haf_out = torch.empty(count, dtype=torch.complex128, device=self.torch_device)
        self._run(lib().gbs_prob_sweep, state.handle, int(n), int(bool(collisions)), _t_ptr(prob_out), _t_ptr(haf_out),
                  _stream_ptr(stream))
        return (prob_out, haf_out) if want_haf else prob_out

    def sweep_sample(self, prob, uniforms, stream=None):
        """Entries drawn from a probability list (App. I): index_out[s] = the entry whose interval of
        [0, total) holds uniforms[s] * total -> (int64 index tensor, float64 total tensor of one)."""
        import torch
        if prob.dtype != torch.float64 or not prob.is_cuda or not prob.is_contiguous():
            raise TypeError("prob must be a contiguous float64 CUDA tensor")
        if uniforms.dtype != torch.float64 or not uniforms.is_cuda or not uniforms.is_contiguous():
            raise TypeError("uniforms must be a contiguous float64 CUDA tensor")
        idx = torch.empty(uniforms.numel(), dtype=torch.int64, device=self.torch_device)
        total = torch.empty(1, dtype=torch.float64, device=self.torch_device)
        self._run(lib().gbs_sweep_sample, _t_ptr(prob), prob.numel(), _t_ptr(uniforms), uniforms.numel(), _t_ptr(idx),
                  _t_ptr(total), _stream_ptr(stream))
        return idx, total

    def prob_slices(self, state: State, patterns, lo, hi, partials_out=None, out_idx=None, stream=None):
        """Compensated partial sums over subset ranges [lo, hi) -> float64 tensor of (s_re, s_im, c_re, c_im)
        rows; slice b goes to row out_idx[b] (default b)."""
        import torch
        modes, offsets = pack_patterns(patterns)
        b = len(offsets) - 1
        lo = np.ascontiguousarray(lo, dtype=np.int64)
        hi = np.ascontiguousarray(hi, dtype=np.int64)
        if len(lo) != b or len(hi) != b:
            raise ValueError("one (lo, hi) pair per pattern")
        oi = None if out_idx is None else np.ascontiguousarray(out_idx, dtype=np.int64)
        rows = b if oi is None or partials_out is not None else (int(oi.max()) + 1 if len(oi) else 0)
        if partials_out is None:
            partials_out = torch.empty((max(rows, 1), 4), dtype=torch.float64, device=self.torch_device)
        elif oi is not None and len(oi) and (int(oi.max()) >= partials_out.shape[0] or int(oi.min()) < 0):
            raise ValueError("out_idx outside partials_out")
        elif oi is None and partials_out.shape[0] < b:
            raise ValueError("partials_out too small")
        self._run(lib().gbs_prob_slices, state.handle, _np_ptr(modes), _np_ptr(offsets), _np_ptr(lo), _np_ptr(hi), b,
                  _t_ptr(partials_out), _np_ptr(oi), _stream_ptr(stream))
        return partials_out

    def finalize(self, state: Optional[State], partials, part_lo, part_hi, patterns, want_prob=True,
                 prob_out=None, haf_out=None, want_haf=True, stream=None):
        """Pattern b = compensated sum of partials[part_lo[b]:part_hi[b]] -> (prob, haf) tensors; the
        patterns (mode lists) give n and, in the library, the prod_j s_j! divisor."""
        import torch
        lo = np.ascontiguousarray(part_lo, dtype=np.int64)
        hi = np.ascontiguousarray(part_hi, dtype=np.int64)
        modes, offsets = pack_patterns(patterns)
        b = len(offsets) - 1
        if len(lo) != b or len(hi) != b:
            raise ValueError("one partial range per pattern")
        if b and int(hi.max()) > partials.shape[0]:
            raise ValueError("partial range beyond the partials tensor")
        if want_prob and prob_out is None:
            prob_out = torch.empty(b, dtype=torch.float64, device=self.torch_device)
        if want_haf and haf_out is None:
            haf_out = torch.empty(b, dtype=torch.complex128, device=self.torch_device)
        self._run(lib().gbs_finalize, state.handle if state is not None else None, _t_ptr(partials), _np_ptr(lo),
                  _np_ptr(hi), _np_ptr(modes), _np_ptr(offsets), b, _t_ptr(prob_out) if want_prob else None,
                  _t_ptr(haf_out), _stream_ptr(stream))
        return (prob_out if want_prob else None), haf_out


def sweep_count(m: int, n: int, collisions: bool = True) -> int:
    """Number of output patterns of n photons in m modes (-1 if beyond the sweep's limits)."""
    return int(lib().gbs_sweep_count(int(m), int(n), int(bool(collisions))))


def photon_number_pmf(m: int, r: float, nmax: int) -> np.ndarray:
    """P_n for n = 0..nmax (Step 1), computed by the library on the host."""
    out = np.zeros(nmax + 1, dtype=np.float64)
    rc = lib().gbs_photon_number_pmf(int(m), float(r), int(nmax), _np_ptr(out))
    if rc:
        raise GBSError(rc, "gbs_photon_number_pmf failed")
    return out
