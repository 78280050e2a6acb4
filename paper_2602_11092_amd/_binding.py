"""ctypes binding of libslos_hip.so (the C ABI declared in include/slos.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  PyTorch tensors provide device memory and the current stream.  The
library must be built (python -m paper_2602_11092_amd.build_lib); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libslos_hip.so")

SLOS_OK = 0
SLOS_EINVAL = -1
SLOS_ENOMEM = -2
SLOS_EHIP = -3
SLOS_EWORKSPACE = -4
SLOS_EUNSUPPORTED = -5

OP_AMPLITUDES = 0
OP_PROBS = 1
OP_AMPLITUDES_BACKWARD = 2
OP_PROBS_BACKWARD = 3
OP_MODE_EXPECTATIONS = 4
OP_MODE_EXPECTATIONS_BACKWARD = 5
OP_THRESHOLD_PROBS = 6
OP_THRESHOLD_PROBS_BACKWARD = 7
OP_SAMPLE = 8
DETECTOR_PNR = 0
DETECTOR_THRESHOLD = 1

PLAN_DEFAULT = 0
PLAN_FORWARD_ONLY = 1
PLAN_UNBUNCHED = 2
PLAN_DUAL_RAIL = 4
PLAN_THRESHOLD = 8

VARIANT_AUTO = 0
VARIANT_FUSED = 1
VARIANT_LAYERED = 2
VARIANT_FUSED_PAIRS = 3

# every symbol the header declares, with (restype, argtypes)
_c = ctypes
_vp = _c.c_void_p
SIGNATURES = {
    "slos_fock_dim": (_c.c_int64, [_c.c_int, _c.c_int]),
    "slos_unbunched_dim": (_c.c_int64, [_c.c_int, _c.c_int]),
    "slos_space_dim": (_c.c_int64, [_c.c_int, _c.c_int, _c.c_int]),
    "slos_space_unrank": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int, _c.c_int64, _vp]),
    "slos_space_rank": (_c.c_int64, [_c.c_int, _c.c_int, _c.c_int, _vp]),
    "slos_threshold_pattern": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int64, _vp]),
    "slos_fock_unrank": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int64, _vp]),
    "slos_fock_rank": (_c.c_int64, [_c.c_int, _c.c_int, _vp]),
    "slos_last_error": (_c.c_char_p, []),
    "slos_transition_tables": (_c.c_int, [_c.c_int, _c.c_int, _vp, _vp, _vp, _vp]),
    "slos_transition_tables_ex": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int, _vp, _vp, _vp, _vp]),
    "slos_plan_create": (_c.c_int, [_c.c_int, _c.c_int, _c.c_int, _c.POINTER(_vp)]),
    "slos_plan_destroy": (_c.c_int, [_vp]),
    "slos_batch_create": (_c.c_int, [_vp, _c.c_int, _vp, _c.POINTER(_vp)]),
    "slos_batch_destroy": (_c.c_int, [_vp]),
    "slos_batch_out_len": (_c.c_int64, [_vp]),
    "slos_batch_out_offsets": (_c.c_int, [_vp, _vp]),
    "slos_workspace_bytes": (_c.c_int, [_vp, _c.c_int, _c.POINTER(_c.c_size_t)]),
    "slos_batch_set_config": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int]),
    "slos_batch_get_config": (_c.c_int, [_vp, _c.c_int, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)]),
    "slos_batch_set_config_ex": (_c.c_int, [_vp, _c.c_int, _c.c_int, _c.c_int, _c.c_int]),
    "slos_batch_get_config_ex": (_c.c_int, [_vp, _c.c_int, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int),
                                            _c.POINTER(_c.c_int)]),
    "fock_amplitudes": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_probs": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_amplitudes_backward": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_probs_backward": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_mode_expectations": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_mode_expectations_backward": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_mode_expectations_ex": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _c.c_size_t, _vp]),
    "fock_mode_expectations_backward_ex": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_int, _vp, _c.c_size_t, _vp]),
    "slos_threshold_dim": (_c.c_int64, [_c.c_int, _c.c_int]),
    "slos_batch_threshold_len": (_c.c_int64, [_vp]),
    "slos_batch_threshold_offsets": (_c.c_int, [_vp, _vp]),
    "fock_threshold_probs": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_threshold_probs_backward": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "slos_superposition_create": (_c.c_int, [_vp, _c.c_int, _vp, _vp]),
    "slos_superposition_destroy": (_c.c_int, [_vp]),
    "slos_superposition_out_len": (_c.c_int64, [_vp]),
    "slos_superposition_out_offsets": (_c.c_int, [_vp, _vp]),
    "slos_superposition_workspace_bytes": (_c.c_int, [_vp, _c.c_int, _vp]),
    "fock_superposition_amplitudes": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "fock_superposition_amplitudes_backward": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _c.c_size_t, _vp]),
    "slos_shared_superposition_create": (_c.c_int, [_vp, _c.c_int, _vp]),
    "slos_shared_superposition_destroy": (_c.c_int, [_vp]),
    "slos_shared_superposition_dim": (_c.c_int64, [_vp]),
    "fock_shared_superposition_amplitudes": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp]),
    "fock_shared_superposition_amplitudes_backward": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp, _vp, _vp]),
    "fock_probs_from_amplitudes": (_c.c_int, [_vp, _c.c_int64, _vp, _vp]),
    "fock_probs_from_amplitudes_backward": (_c.c_int, [_vp, _vp, _c.c_int64, _vp, _vp]),
    "fock_sample": (_c.c_int, [_vp, _vp, _vp, _c.c_int, _vp, _vp, _c.c_size_t, _vp]),
    "fock_fidelity_kernel": (_c.c_int, [_c.c_int, _vp, _vp, _c.c_int, _vp, _c.c_int, _vp, _vp]),
    "mesh_workspace_bytes": (_c.c_int, [_c.c_int, _c.c_int, _c.POINTER(_c.c_size_t)]),
    "mesh_to_unitary": (_c.c_int, [_c.c_int, _c.c_int, _vp, _vp, _c.c_float, _vp, _vp, _c.c_size_t, _vp]),
    "mesh_to_unitary_backward": (_c.c_int, [_c.c_int, _c.c_int, _vp, _vp, _c.c_float, _vp, _vp, _vp, _vp,
                                            _c.c_size_t, _vp]),
    "mesh_to_unitary_backward_noalloc": (_c.c_int, [_c.c_int, _c.c_int, _vp, _vp, _c.c_float, _vp, _vp, _vp, _vp]),
}

_lib = None


class SlosError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__("%s failed (%d): %s" % (fn, code, msg))
        self.code = code


def lib():
    """Loads the built library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libslos_hip.so is not built; run `python -m paper_2602_11092_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(fn: str, rc: int):
    if rc != SLOS_OK:
        raise SlosError(fn, rc, lib().slos_last_error().decode())


def _stream_ptr(dev: torch.device):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _require(t: torch.Tensor, name: str, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a device (cuda) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.is_conj() or t.is_neg():
        # a lazy conjugate/negative view: its memory holds the unconjugated values
        raise ValueError("%s is a lazy conj/neg view; call resolve_conj()/resolve_neg() first" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


class WorkspaceCache:
    """Device workspaces that the binding hands to compute calls when the
    caller passes none.

    A workspace handed to a call may have been captured into a HIP graph,
    which keeps its raw address.  So a buffer is never freed while its owner
    lives: when a call needs more bytes, the old buffer is retired (kept
    alive) and a larger one, rounded up to a power of two, takes its place.
    Keys include the stream, so calls on different streams never share a
    buffer."""

    def __init__(self):
        self._live = {}
        self._retired = []

    @staticmethod
    def _round(nbytes: int) -> int:
        return 1 << max(8, (max(int(nbytes), 1) - 1).bit_length())

    def get(self, key, nbytes: int, device) -> torch.Tensor:
        dev = torch.device(device)
        full = (key, str(dev))
        ws = self._live.get(full)
        if ws is None or ws.numel() < nbytes:
            if ws is not None:
                self._retired.append(ws)
            ws = torch.empty(self._round(nbytes), dtype=torch.uint8, device=dev)
            self._live[full] = ws
        return ws

    def retired(self) -> int:
        return len(self._retired)


def _stream_key(device) -> int:
    return int(torch.cuda.current_stream(torch.device(device)).cuda_stream)


# ------------------------------------------------------------------ combinatorics

def slos_fock_dim(m: int, n: int) -> int:
    return int(lib().slos_fock_dim(m, n))


def slos_unbunched_dim(m: int, n: int) -> int:
    """C(m, n): states with n photons and at most one per mode (-1 if invalid)."""
    return int(lib().slos_unbunched_dim(m, n))


def space_flags(unbunched: bool = False, dual_rail: bool = False) -> int:
    return (PLAN_UNBUNCHED if unbunched else 0) | (PLAN_DUAL_RAIL if dual_rail else 0)


def slos_space_unrank(m: int, n: int, flags: int, rank: int) -> np.ndarray:
    """Occupation of the state of `rank` in the space of plans with `flags`."""
    occ = np.zeros(m, dtype=np.int32)
    _check("slos_space_unrank", lib().slos_space_unrank(m, n, flags, rank, occ.ctypes.data_as(_vp)))
    return occ


def slos_space_rank(m: int, n: int, flags: int, occ) -> int:
    occ = np.ascontiguousarray(np.asarray(occ, dtype=np.int32))
    return int(lib().slos_space_rank(m, n, flags, occ.ctypes.data_as(_vp)))


def slos_threshold_pattern(m: int, n: int, q: int) -> np.ndarray:
    """0/1 clicks of click pattern q of n photons over m modes."""
    clicks = np.zeros(m, dtype=np.int32)
    _check("slos_threshold_pattern", lib().slos_threshold_pattern(m, n, q, clicks.ctypes.data_as(_vp)))
    return clicks


def slos_threshold_dim(m: int, n: int) -> int:
    """Number of click patterns of n photons over m modes (-1 if invalid)."""
    return int(lib().slos_threshold_dim(m, n))


def slos_space_dim(m: int, n: int, flags: int = PLAN_DEFAULT) -> int:
    """Size of the n-photon layer of the space that plans with `flags` use (-1 if invalid)."""
    return int(lib().slos_space_dim(m, n, flags))


def slos_fock_unrank(m: int, n: int, rank: int) -> np.ndarray:
    occ = np.zeros(m, dtype=np.int32)
    _check("slos_fock_unrank", lib().slos_fock_unrank(m, n, rank, occ.ctypes.data_as(_vp)))
    return occ


def slos_fock_rank(m: int, n: int, occ) -> int:
    o = np.ascontiguousarray(occ, dtype=np.int32)
    return int(lib().slos_fock_rank(m, n, o.ctypes.data_as(_vp)))


# ------------------------------------------------------------------ plan / batch

class Plan:
    """Transition graph for m modes and up to n_max photons (slos_plan_create)."""

    def __init__(self, m: int, n_max: int, forward_only: bool = False, unbunched: bool = False,
                 dual_rail: bool = False, threshold: bool = False):
        h = _vp()
        flags = space_flags(unbunched, dual_rail) | (PLAN_FORWARD_ONLY if forward_only else PLAN_DEFAULT)
        flags |= PLAN_THRESHOLD if threshold else 0
        _check("slos_plan_create", lib().slos_plan_create(m, n_max, flags, ctypes.byref(h)))
        self._h = h
        self.m = m
        self.n_max = n_max
        self.unbunched = unbunched
        self.dual_rail = dual_rail
        self.threshold = threshold

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().slos_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Input states of B samples for one plan (slos_batch_create)."""

    def __init__(self, plan: Plan, occ):
        occ = np.ascontiguousarray(np.asarray(occ, dtype=np.int32).reshape(-1, plan.m))
        h = _vp()
        _check("slos_batch_create", lib().slos_batch_create(plan.handle, occ.shape[0], occ.ctypes.data_as(_vp),
                                                            ctypes.byref(h)))
        self._h = h
        self.plan = plan  # keep the plan alive
        self.m = plan.m
        self.B = occ.shape[0]
        self.occ = occ
        self.n = occ.sum(axis=1)
        self.out_len = int(lib().slos_batch_out_len(h))
        off = np.zeros(self.B + 1, dtype=np.int64)
        _check("slos_batch_out_offsets", lib().slos_batch_out_offsets(h, off.ctypes.data_as(_vp)))
        self.offsets = off
        toff = np.zeros(self.B + 1, dtype=np.int64)
        _check("slos_batch_threshold_offsets", lib().slos_batch_threshold_offsets(h, toff.ctypes.data_as(_vp)))
        self.threshold_offsets = toff
        self.threshold_len = int(toff[-1])
        self._ws = WorkspaceCache()

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, op: int) -> int:
        n = ctypes.c_size_t(0)
        _check("slos_workspace_bytes", lib().slos_workspace_bytes(self._h, op, ctypes.byref(n)))
        return int(n.value)

    def set_config(self, op: int, variant: int, block: int = 0, tile: int = 0):
        _check("slos_batch_set_config_ex", lib().slos_batch_set_config_ex(self._h, op, variant, block, tile))

    def get_config(self, op: int) -> Tuple[int, int]:
        v, b = ctypes.c_int(0), ctypes.c_int(0)
        _check("slos_batch_get_config", lib().slos_batch_get_config(self._h, op, ctypes.byref(v), ctypes.byref(b)))
        return int(v.value), int(b.value)

    def get_config_ex(self, op: int) -> Tuple[int, int, int]:
        """(variant, block, tile) in use for `op`."""
        v, b, t = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        _check("slos_batch_get_config_ex", lib().slos_batch_get_config_ex(self._h, op, ctypes.byref(v),
                                                                          ctypes.byref(b), ctypes.byref(t)))
        return int(v.value), int(b.value), int(t.value)

    def workspace(self, op: int, device) -> Optional[torch.Tensor]:
        """Device workspace for `op` on the current stream, kept by the batch
        (see WorkspaceCache: buffers are retired, never freed, so a captured
        graph's workspace outlives later calls that need more)."""
        need = self.workspace_bytes(op)
        if need == 0:
            return None
        return self._ws.get((op, _stream_key(device)), need, device)

    def close(self):
        if self._h is not None and self._h.value:
            lib().slos_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ws_args(ws: Optional[torch.Tensor]):
    if ws is None:
        return ctypes.c_void_p(0), 0
    return ctypes.c_void_p(ws.data_ptr()), ws.numel()


# ------------------------------------------------------------------ forward / backward

def fock_amplitudes(batch: Batch, U: torch.Tensor, out: Optional[torch.Tensor] = None,
                    ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Amplitudes a_t of every sample, complex64 [out_len] (ragged per sample)."""
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    if out is None:
        out = torch.empty(batch.out_len, dtype=torch.complex64, device=U.device)
    _require(out, "out", torch.complex64, (batch.out_len,))
    if ws is None:
        ws = batch.workspace(OP_AMPLITUDES, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_amplitudes", lib().fock_amplitudes(batch.handle, _ptr(U), _ptr(out), wp, wn, _stream_ptr(U.device)))
    return out


def fock_probs(batch: Batch, U: torch.Tensor, out: Optional[torch.Tensor] = None,
               ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Probabilities |a_t|^2, float32 [out_len]."""
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    if out is None:
        out = torch.empty(batch.out_len, dtype=torch.float32, device=U.device)
    _require(out, "out", torch.float32, (batch.out_len,))
    if ws is None:
        ws = batch.workspace(OP_PROBS, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_probs", lib().fock_probs(batch.handle, _ptr(U), _ptr(out), wp, wn, _stream_ptr(U.device)))
    return out


def fock_amplitudes_backward(batch: Batch, U: torch.Tensor, grad_amps: torch.Tensor,
                             out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    _require(grad_amps, "grad_amps", torch.complex64, (batch.out_len,))
    if out is None:
        out = torch.empty_like(U)
    _require(out, "grad_U", torch.complex64, (batch.B, batch.m, batch.m))
    if ws is None:
        ws = batch.workspace(OP_AMPLITUDES_BACKWARD, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_amplitudes_backward",
           lib().fock_amplitudes_backward(batch.handle, _ptr(U), _ptr(grad_amps), _ptr(out), wp, wn,
                                          _stream_ptr(U.device)))
    return out


def fock_probs_backward(batch: Batch, U: torch.Tensor, grad_probs: torch.Tensor,
                        out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    _require(grad_probs, "grad_probs", torch.float32, (batch.out_len,))
    if out is None:
        out = torch.empty_like(U)
    _require(out, "grad_U", torch.complex64, (batch.B, batch.m, batch.m))
    if ws is None:
        ws = batch.workspace(OP_PROBS_BACKWARD, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_probs_backward",
           lib().fock_probs_backward(batch.handle, _ptr(U), _ptr(grad_probs), _ptr(out), wp, wn,
                                     _stream_ptr(U.device)))
    return out


def _detector(detector) -> int:
    if detector in ("pnr", DETECTOR_PNR):
        return DETECTOR_PNR
    if detector in ("threshold", DETECTOR_THRESHOLD):
        return DETECTOR_THRESHOLD
    raise ValueError("detector must be 'pnr' or 'threshold'")


def fock_mode_expectations(batch: Batch, U: torch.Tensor, out: Optional[torch.Tensor] = None,
                           ws: Optional[torch.Tensor] = None, detector="pnr") -> torch.Tensor:
    """Per-mode photon-number expectations <n_j> = sum_t t_j p_t, float32 [B, m]
    (detector="threshold": click probabilities sum_t [t_j > 0] p_t)."""
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    if out is None:
        out = torch.empty((batch.B, batch.m), dtype=torch.float32, device=U.device)
    _require(out, "out", torch.float32, (batch.B, batch.m))
    if ws is None:
        ws = batch.workspace(OP_MODE_EXPECTATIONS, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_mode_expectations_ex",
           lib().fock_mode_expectations_ex(batch.handle, _ptr(U), _ptr(out), _detector(detector), wp, wn,
                                           _stream_ptr(U.device)))
    return out


def fock_mode_expectations_backward(batch: Batch, U: torch.Tensor, grad_out: torch.Tensor,
                                    out: Optional[torch.Tensor] = None,
                                    ws: Optional[torch.Tensor] = None, detector="pnr") -> torch.Tensor:
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    _require(grad_out, "grad_out", torch.float32, (batch.B, batch.m))
    if out is None:
        out = torch.empty_like(U)
    _require(out, "grad_U", torch.complex64, (batch.B, batch.m, batch.m))
    if ws is None:
        ws = batch.workspace(OP_MODE_EXPECTATIONS_BACKWARD, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_mode_expectations_backward_ex",
           lib().fock_mode_expectations_backward_ex(batch.handle, _ptr(U), _ptr(grad_out), _ptr(out),
                                                    _detector(detector), wp, wn, _stream_ptr(U.device)))
    return out


def fock_threshold_probs(batch: Batch, U: torch.Tensor, out: Optional[torch.Tensor] = None,
                         ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Threshold-detector click probabilities, float32 [threshold_len] (ragged per sample)."""
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    if out is None:
        out = torch.empty(batch.threshold_len, dtype=torch.float32, device=U.device)
    _require(out, "out", torch.float32, (batch.threshold_len,))
    if ws is None:
        ws = batch.workspace(OP_THRESHOLD_PROBS, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_threshold_probs",
           lib().fock_threshold_probs(batch.handle, _ptr(U), _ptr(out), wp, wn, _stream_ptr(U.device)))
    return out


def fock_threshold_probs_backward(batch: Batch, U: torch.Tensor, grad_out: torch.Tensor,
                                  out: Optional[torch.Tensor] = None,
                                  ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    _require(grad_out, "grad_out", torch.float32, (batch.threshold_len,))
    if out is None:
        out = torch.empty_like(U)
    _require(out, "grad_U", torch.complex64, (batch.B, batch.m, batch.m))
    if ws is None:
        ws = batch.workspace(OP_THRESHOLD_PROBS_BACKWARD, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_threshold_probs_backward",
           lib().fock_threshold_probs_backward(batch.handle, _ptr(U), _ptr(grad_out), _ptr(out), wp, wn,
                                               _stream_ptr(U.device)))
    return out


class Superposition:
    """Amplitude-encoded inputs (slos_superposition_create): the batch's samples
    are components; group g holds components [group_off[g], group_off[g+1])."""

    def __init__(self, batch: Batch, group_off):
        off = np.ascontiguousarray(np.asarray(group_off, dtype=np.int64).ravel())
        h = _vp()
        _check("slos_superposition_create",
               lib().slos_superposition_create(batch.handle, off.size - 1, off.ctypes.data_as(_vp), ctypes.byref(h)))
        self._h = h
        self.batch = batch  # keep the batch alive
        self.G = off.size - 1
        self.group_off = off
        self.out_len = int(lib().slos_superposition_out_len(h))
        oo = np.zeros(self.G + 1, dtype=np.int64)
        _check("slos_superposition_out_offsets", lib().slos_superposition_out_offsets(h, oo.ctypes.data_as(_vp)))
        self.out_offsets = oo
        self._ws = WorkspaceCache()

    @property
    def handle(self):
        return self._h

    def workspace(self, backward: bool, device) -> torch.Tensor:
        n = ctypes.c_size_t(0)
        _check("slos_superposition_workspace_bytes",
               lib().slos_superposition_workspace_bytes(self._h, int(backward), ctypes.byref(n)))
        return self._ws.get((bool(backward), _stream_key(device)), int(n.value), device)

    def close(self):
        if self._h is not None and self._h.value:
            lib().slos_superposition_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fock_superposition_amplitudes(sup: Superposition, U: torch.Tensor, x: torch.Tensor,
                                  out: Optional[torch.Tensor] = None,
                                  ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sum_c x_c a(U_g, s_c) per group, complex64 [out_len] (ragged per group)."""
    m = sup.batch.m
    _require(U, "U", torch.complex64, (sup.G, m, m))
    _require(x, "x", torch.complex64, (sup.batch.B,))
    if out is None:
        out = torch.empty(sup.out_len, dtype=torch.complex64, device=U.device)
    _require(out, "out", torch.complex64, (sup.out_len,))
    if ws is None:
        ws = sup.workspace(False, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_superposition_amplitudes",
           lib().fock_superposition_amplitudes(sup.handle, _ptr(U), _ptr(x), _ptr(out), wp, wn, _stream_ptr(U.device)))
    return out


def fock_superposition_amplitudes_backward(sup: Superposition, U: torch.Tensor, x: torch.Tensor,
                                           grad_out: torch.Tensor, need_grad_x: bool = True,
                                           ws: Optional[torch.Tensor] = None):
    """(dL/dU [G, m, m], dL/dx [C] or None) given dL/dout."""
    m = sup.batch.m
    _require(U, "U", torch.complex64, (sup.G, m, m))
    _require(x, "x", torch.complex64, (sup.batch.B,))
    _require(grad_out, "grad_out", torch.complex64, (sup.out_len,))
    gU = torch.empty_like(U)
    gx = torch.empty_like(x) if need_grad_x else None
    if ws is None:
        ws = sup.workspace(True, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_superposition_amplitudes_backward",
           lib().fock_superposition_amplitudes_backward(sup.handle, _ptr(U), _ptr(x), _ptr(grad_out), _ptr(gU),
                                                        _ptr(gx), wp, wn, _stream_ptr(U.device)))
    return gU, gx


class SharedSuperposition:
    """Dense inputs over the n-photon basis that all go through one U
    (slos_shared_superposition_create): out = X Uhat^T by one complex GEMM."""

    def __init__(self, plan: Plan, n: int):
        h = _vp()
        _check("slos_shared_superposition_create", lib().slos_shared_superposition_create(plan.handle, n, ctypes.byref(h)))
        self._h = h
        self.plan = plan
        self.m = plan.m
        self.n = n
        self.N = int(lib().slos_shared_superposition_dim(h))

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().slos_shared_superposition_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fock_shared_superposition_amplitudes(s: SharedSuperposition, U: torch.Tensor, X: torch.Tensor,
                                         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """X [G, N] complex64 -> U's action, complex64 [G, N]."""
    _require(U, "U", torch.complex64, (s.m, s.m))
    _require(X, "X", torch.complex64)
    if X.dim() != 2 or X.shape[1] != s.N:
        raise ValueError("X must be [G, %d]" % s.N)
    G = X.shape[0]
    if out is None:
        out = torch.empty((G, s.N), dtype=torch.complex64, device=U.device)
    _require(out, "out", torch.complex64, (G, s.N))
    _check("fock_shared_superposition_amplitudes",
           lib().fock_shared_superposition_amplitudes(s.handle, _ptr(U), _ptr(X), G, _ptr(out), _stream_ptr(U.device)))
    return out


def fock_shared_superposition_amplitudes_backward(s: SharedSuperposition, U: torch.Tensor, X: torch.Tensor,
                                                  grad_out: torch.Tensor, need_grad_x: bool = True):
    _require(U, "U", torch.complex64, (s.m, s.m))
    _require(X, "X", torch.complex64)
    G = X.shape[0]
    _require(grad_out, "grad_out", torch.complex64, (G, s.N))
    gU = torch.empty_like(U)
    gX = torch.empty_like(X) if need_grad_x else None
    _check("fock_shared_superposition_amplitudes_backward",
           lib().fock_shared_superposition_amplitudes_backward(s.handle, _ptr(U), _ptr(X), G, _ptr(grad_out), _ptr(gU),
                                                               _ptr(gX), _stream_ptr(U.device)))
    return gU, gX


def fock_probs_from_amplitudes(a: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """|a|^2 elementwise (complex64 in, float32 out of the same shape)."""
    _require(a, "amps", torch.complex64)
    if out is None:
        out = torch.empty(a.shape, dtype=torch.float32, device=a.device)
    _require(out, "probs", torch.float32, tuple(a.shape))
    _check("fock_probs_from_amplitudes",
           lib().fock_probs_from_amplitudes(_ptr(a), a.numel(), _ptr(out), _stream_ptr(a.device)))
    return out


def fock_probs_from_amplitudes_backward(a: torch.Tensor, grad_p: torch.Tensor,
                                        out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/da = 2 (dL/dp) a for p = |a|^2."""
    _require(a, "amps", torch.complex64)
    _require(grad_p, "grad_probs", torch.float32, tuple(a.shape))
    if out is None:
        out = torch.empty_like(a)
    _require(out, "grad_amps", torch.complex64, tuple(a.shape))
    _check("fock_probs_from_amplitudes_backward",
           lib().fock_probs_from_amplitudes_backward(_ptr(a), _ptr(grad_p), a.numel(), _ptr(out),
                                                     _stream_ptr(a.device)))
    return out


def fock_sample(batch: Batch, U: torch.Tensor, u: torch.Tensor, out: Optional[torch.Tensor] = None,
                ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Shots drawn from p / sum(p) by inverse transform of the uniforms u
    (float32 [B, S] in [0, 1)): int32 [B, S] state indices within each
    sample's output block."""
    _require(U, "U", torch.complex64, (batch.B, batch.m, batch.m))
    _require(u, "u", torch.float32)
    if u.dim() != 2 or u.shape[0] != batch.B:
        raise ValueError("u must be [B, S]")
    S = u.shape[1]
    if out is None:
        out = torch.empty((batch.B, S), dtype=torch.int32, device=U.device)
    _require(out, "shots", torch.int32, (batch.B, S))
    if ws is None:
        ws = batch.workspace(OP_SAMPLE, U.device)
    wp, wn = _ws_args(ws)
    _check("fock_sample", lib().fock_sample(batch.handle, _ptr(U), _ptr(u), S, _ptr(out), wp, wn,
                                            _stream_ptr(U.device)))
    return out


def fock_fidelity_kernel(occ, U1: torch.Tensor, U2: Optional[torch.Tensor] = None,
                         out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K[a][b] = |<phi(U1_a)|phi(U2_b)>|^2 for input state occ, float32 [B1, B2]
    (U2 = None: the Gram matrix of U1)."""
    occ = np.ascontiguousarray(np.asarray(occ, dtype=np.int32).ravel())
    m = occ.size
    _require(U1, "U1", torch.complex64)
    if U1.dim() != 3 or tuple(U1.shape[1:]) != (m, m):
        raise ValueError("U1 must be [B1, m, m]")
    if U2 is None:
        U2 = U1
    _require(U2, "U2", torch.complex64)
    if U2.dim() != 3 or tuple(U2.shape[1:]) != (m, m):
        raise ValueError("U2 must be [B2, m, m]")
    B1, B2 = U1.shape[0], U2.shape[0]
    if out is None:
        out = torch.empty((B1, B2), dtype=torch.float32, device=U1.device)
    _require(out, "out", torch.float32, (B1, B2))
    _check("fock_fidelity_kernel",
           lib().fock_fidelity_kernel(m, occ.ctypes.data_as(_vp), _ptr(U1), B1, _ptr(U2), B2, _ptr(out),
                                      _stream_ptr(U1.device)))
    return out


# ------------------------------------------------------------------ mesh

_mesh_ws = WorkspaceCache()


def mesh_workspace(m: int, B: int, device) -> torch.Tensor:
    """Workspace of the mesh calls on the current stream, shared by every
    caller on that stream and device; buffers that become too small are
    retired, never freed (WorkspaceCache)."""
    n = ctypes.c_size_t(0)
    _check("mesh_workspace_bytes", lib().mesh_workspace_bytes(m, B, ctypes.byref(n)))
    return _mesh_ws.get(("mesh", _stream_key(device)), int(n.value), device)


def mesh_to_unitary(theta: torch.Tensor, x: Optional[torch.Tensor], enc_scale: float, m: Optional[int] = None,
                    out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """U(x_b, theta) for every row of x (complex64 [B, m, m]); with x = None,
    the plain mesh W2 W1 as [1, m, m]."""
    if x is not None:
        _require(x, "x", torch.float32)
        B, m = x.shape
    else:
        if m is None:
            raise ValueError("m is required when x is None")
        B = 1
    _require(theta, "theta", torch.float32, (m * (m - 1),))
    if out is None:
        out = torch.empty(B, m, m, dtype=torch.complex64, device=theta.device)
    _require(out, "U", torch.complex64, (B, m, m))
    if ws is None:
        ws = mesh_workspace(m, B, theta.device)
    _check("mesh_to_unitary", lib().mesh_to_unitary(m, B, _ptr(theta), _ptr(x), float(enc_scale), _ptr(out),
                                                    _ptr(ws), ws.numel(), _stream_ptr(theta.device)))
    return out


def mesh_to_unitary_backward(theta: torch.Tensor, x: Optional[torch.Tensor], enc_scale: float,
                             grad_U: torch.Tensor, need_grad_x: bool = True,
                             ws: Optional[torch.Tensor] = None, out_theta: Optional[torch.Tensor] = None,
                             out_x: Optional[torch.Tensor] = None):
    """(grad_theta [m(m-1)], grad_x [B, m] or None)."""
    B, m = grad_U.shape[0], grad_U.shape[1]
    _require(grad_U, "grad_U", torch.complex64, (B, m, m))
    _require(theta, "theta", torch.float32, (m * (m - 1),))
    if x is not None:
        _require(x, "x", torch.float32, (B, m))
    gt = out_theta if out_theta is not None else torch.empty_like(theta)
    _require(gt, "grad_theta", torch.float32, (m * (m - 1),))
    gx = None
    if x is not None and need_grad_x:
        gx = out_x if out_x is not None else torch.empty(B, m, dtype=torch.float32, device=theta.device)
        _require(gx, "grad_x", torch.float32, (B, m))
    if ws is None:
        ws = mesh_workspace(m, B, theta.device)
    _check("mesh_to_unitary_backward",
           lib().mesh_to_unitary_backward(m, B, _ptr(theta), _ptr(x), float(enc_scale), _ptr(grad_U), _ptr(gt),
                                          _ptr(gx), _ptr(ws), ws.numel(), _stream_ptr(theta.device)))
    return gt, gx


MESH_NOALLOC_SCRATCH_BYTES = 16 << 20


def mesh_to_unitary_backward_noalloc(theta: torch.Tensor, x: Optional[torch.Tensor], enc_scale: float,
                                     grad_U: torch.Tensor, out_theta: torch.Tensor,
                                     out_x: Optional[torch.Tensor] = None):
    """mesh_to_unitary_backward with the library's static scratch instead of a
    workspace: the caller passes every output, and nothing is allocated."""
    B, m = grad_U.shape[0], grad_U.shape[1]
    _require(grad_U, "grad_U", torch.complex64, (B, m, m))
    _require(theta, "theta", torch.float32, (m * (m - 1),))
    _require(out_theta, "grad_theta", torch.float32, (m * (m - 1),))
    if x is not None:
        _require(x, "x", torch.float32, (B, m))
    if out_x is not None:
        _require(out_x, "grad_x", torch.float32, (B, m))
    _check("mesh_to_unitary_backward_noalloc",
           lib().mesh_to_unitary_backward_noalloc(m, B, _ptr(theta), _ptr(x), float(enc_scale), _ptr(grad_U),
                                                  _ptr(out_theta), _ptr(out_x), _stream_ptr(theta.device)))
    return out_theta, out_x


def slos_transition_tables(m: int, k: int, want_succ: bool = True, unbunched: bool = False,
                           dual_rail: bool = False):
    """Host copy of layer k's transition tables: (pred [k, N_k], succ [m, N_{k-1}]
    or None, nrm [N_k], minoff [m+1]).  With `unbunched` or `dual_rail`, the
    tables of that restricted space."""
    flags = space_flags(unbunched, dual_rail)
    Nk = slos_space_dim(m, k, flags)
    Nkm1 = slos_space_dim(m, k - 1, flags)
    if Nk < 0 or Nkm1 < 0:
        raise SlosError("slos_transition_tables", SLOS_EINVAL, "bad m=%d k=%d" % (m, k))
    pred = np.zeros((k, Nk), dtype=np.int32)
    succ = np.zeros((m, Nkm1), dtype=np.int32) if want_succ else None
    nrm = np.zeros(Nk, dtype=np.float32)
    minoff = np.zeros(m + 1, dtype=np.int32)
    _check("slos_transition_tables_ex",
           lib().slos_transition_tables_ex(m, k, flags,
                                           pred.ctypes.data_as(_vp),
                                           succ.ctypes.data_as(_vp) if succ is not None else None,
                                           nrm.ctypes.data_as(_vp), minoff.ctypes.data_as(_vp)))
    return pred, succ, nrm, minoff
