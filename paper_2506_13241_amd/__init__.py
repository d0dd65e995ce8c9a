"""Thin Python binding of the gfx950 Pauli-propagation library (liborqa_hip.so).

Argument marshalling only: every step of the propagation runs in the HIP
kernels behind the C ABI declared in include/orqa.h.  PyTorch is used only to
obtain the current HIP stream.  Importing this package never falls back to
anything else: if the shared library is missing, every call raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liborqa_hip.so")

PS_OK, PS_ERR_INVALID, PS_ERR_CAPACITY, PS_ERR_HIP, PS_ERR_NONFINITE, PS_ERR_UNSUPPORTED, PS_ERR_DEVICE = (
    0, -1, -2, -3, -4, -5, -6)
PS_F64, PS_F32 = 0, 1
PS_TRUNC_NONE, PS_TRUNC_MAGNITUDE, PS_TRUNC_LEARNED = 0, 1, 2

EXPORTED_SYMBOLS = (
    "pauli_sum_create", "pauli_sum_destroy", "apply_rotation_layer", "pauli_sum_gates_applied",
    "pauli_sum_truncate", "expectation_z", "pauli_sum_size", "pauli_sum_norm2", "pauli_sum_export",
    "pauli_sum_load_scorer", "pauli_sum_set_timing", "pauli_sum_stats", "ps_last_error",
    "ps_scorer_create", "ps_scorer_destroy", "ps_scorer_set_params", "ps_scorer_get_params", "ps_scorer_set_data",
    "ps_scorer_forward", "ps_scorer_loss_grad", "ps_scorer_adam_step", "pauli_sum_set_graphs",
    "pauli_sum_histogram", "pauli_sum_set_sort_config", "pauli_sum_histogram_noalloc",
    "pauli_sum_set_lookback_epoch", "pauli_sum_lookback_epoch", "pauli_sum_set_rx_boundary_prologue",
    "pauli_sum_set_learned",
)
N_SCORER_PARAMS = 37249
SORT_CONFIGS = ((8, 8), (8, 16), (7, 16), (6, 16), (7, 8), (6, 8))  # (digit bits, items per thread)


class PsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class ps_pauli(ctypes.Structure):
    _fields_ = [("x", ctypes.c_uint64 * 2), ("z", ctypes.c_uint64 * 2)]


class ps_stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_double) for name in (
        "updates", "gates", "rx_launches", "rx_in", "rx_out", "rx_ms", "cliff_launches", "cliff_in", "cliff_ms",
        "sort_passes", "sort_elems", "sort_ms", "bytes_per_string", "graph_replays", "graph_captures",
        "score_launches", "score_in", "score_ms",
        "radix_sorts", "sort_digit_bits", "sort_items_per_thread", "run_merges",
        "learned_passes", "learned_fallbacks", "learned_est", "learned_l1")]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liborqa_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library not built: {path} (run python -m paper_2506_13241_amd.build)")
    try:  # share torch's HIP runtime (device memory and streams come from torch)
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover
        pass
    lib = ctypes.CDLL(path)
    P, I, S, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_double
    sig = {
        "pauli_sum_create": (I, [I, I, I, S, P, P, S, P, ctypes.POINTER(P)]),
        "pauli_sum_destroy": (I, [P]),
        "apply_rotation_layer": (I, [P, P, P, S, D, I]),
        "pauli_sum_gates_applied": (I, [P, ctypes.POINTER(S)]),
        "pauli_sum_truncate": (I, [P, D, I]),
        "expectation_z": (I, [P, P]),
        "pauli_sum_size": (I, [P, ctypes.POINTER(S)]),
        "pauli_sum_norm2": (I, [P, P]),
        "pauli_sum_export": (I, [P, P, P, S, ctypes.POINTER(S)]),
        "pauli_sum_load_scorer": (I, [P, P]),
        "pauli_sum_set_timing": (I, [P, I]),
        "pauli_sum_stats": (I, [P, ctypes.POINTER(ps_stats), I]),
        "ps_last_error": (ctypes.c_char_p, []),
        "pauli_sum_set_graphs": (I, [P, I]),
        "pauli_sum_histogram": (I, [P, I, P, I, I, P]),
        "pauli_sum_histogram_noalloc": (I, [P, I, P, I, I, P]),
        "pauli_sum_set_lookback_epoch": (I, [P, ctypes.c_uint32]),
        "pauli_sum_set_rx_boundary_prologue": (I, [P, I]),
        "pauli_sum_set_learned": (I, [P, D, D]),
        "pauli_sum_lookback_epoch": (I, [P, ctypes.POINTER(ctypes.c_uint32)]),
        "pauli_sum_set_sort_config": (I, [P, I, I]),
        "ps_scorer_create": (I, [I, P, P, P, P, ctypes.POINTER(P)]),
        "ps_scorer_destroy": (I, [P]),
        "ps_scorer_set_params": (I, [P, P, S]),
        "ps_scorer_get_params": (I, [P, P, S]),
        "ps_scorer_set_data": (I, [P, P, P, S]),
        "ps_scorer_forward": (I, [P, P, P]),
        "ps_scorer_loss_grad": (I, [P, ctypes.POINTER(D), P]),
        "ps_scorer_adam_step": (I, [P, ctypes.c_float]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != PS_OK:
        raise PsError(rc, load_library().ps_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _words_to_pauli(words: np.ndarray) -> np.ndarray:
    """(m,4) uint64 words (x0,x1,z0,z1) -> (m,4) contiguous array laid out as ps_pauli."""
    return np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, 4)


def current_stream():
    """hipStream_t of torch's current stream (None if torch has no GPU)."""
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch missing
        pass
    return None


class PauliSum:
    """Handle on a GPU-resident Pauli sum (see include/orqa.h for semantics)."""

    def __init__(self, n_qubits: int, terms, coeffs, dtype: int = PS_F64, capacity: int = 0, stream=None):
        lib = load_library()
        terms = _words_to_pauli(terms)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64)
        lanes = coeffs.shape[1] if coeffs.ndim == 2 else 1
        coeffs = coeffs.reshape(terms.shape[0], lanes)
        self.n_qubits = n_qubits
        self.lanes = coeffs.shape[1]
        self.dtype = dtype
        h = ctypes.c_void_p()
        if stream is None:
            stream = current_stream()
        _check(lib.pauli_sum_create(n_qubits, self.lanes, dtype, capacity, _ptr(terms), _ptr(coeffs),
                                    terms.shape[0], stream, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.pauli_sum_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def apply_rotation_layer(self, gates, rel_eps: float = 0.0, trunc_mode: int = PS_TRUNC_MAGNITUDE):
        gens = _words_to_pauli(gates.gens)
        th = np.ascontiguousarray(gates.thetas, dtype=np.float64)
        if th.ndim == 1:
            th = th[:, None]
        if th.shape[1] == 1 and self.lanes > 1:
            th = np.ascontiguousarray(np.repeat(th, self.lanes, axis=1))
        assert th.shape == (gens.shape[0], self.lanes), th.shape
        _check(_lib.apply_rotation_layer(self._h, _ptr(gens), _ptr(th), gens.shape[0], float(rel_eps), trunc_mode))
        return self

    def gates_applied(self) -> int:
        n = ctypes.c_size_t()
        _check(_lib.pauli_sum_gates_applied(self._h, ctypes.byref(n)))
        return int(n.value)

    def truncate(self, rel_eps: float, trunc_mode: int = PS_TRUNC_MAGNITUDE):
        _check(_lib.pauli_sum_truncate(self._h, float(rel_eps), trunc_mode))
        return self

    def expectation_z(self) -> np.ndarray:
        out = np.zeros(self.lanes)
        _check(_lib.expectation_z(self._h, _ptr(out)))
        return out

    def size(self) -> int:
        n = ctypes.c_size_t()
        _check(_lib.pauli_sum_size(self._h, ctypes.byref(n)))
        return int(n.value)

    def norm2(self) -> np.ndarray:
        out = np.zeros(self.lanes)
        _check(_lib.pauli_sum_norm2(self._h, _ptr(out)))
        return out

    def export(self) -> tuple[np.ndarray, np.ndarray]:
        """(terms (m,4) uint64 sorted by (x1,x0,z1,z0), coeffs (m, lanes))."""
        n = self.size()
        keys = np.zeros((max(n, 1), 4), dtype=np.uint64)
        ct = np.float64 if self.dtype == PS_F64 else np.float32
        coeffs = np.zeros((max(n, 1), self.lanes), dtype=ct)
        got = ctypes.c_size_t()
        _check(_lib.pauli_sum_export(self._h, _ptr(keys), _ptr(coeffs), keys.shape[0], ctypes.byref(got)))
        m = int(got.value)
        return keys[:m], coeffs[:m]

    def set_timing(self, enable: bool = True):
        _check(_lib.pauli_sum_set_timing(self._h, int(enable)))
        return self

    def set_graphs(self, enable: bool = True):
        _check(_lib.pauli_sum_set_graphs(self._h, int(enable)))
        return self

    def set_sort_config(self, digit_bits: int = 0, items_per_thread: int = 0):
        """Radix-sort digit width and tile size; (0, 0) tunes online."""
        _check(_lib.pauli_sum_set_sort_config(self._h, int(digit_bits), int(items_per_thread)))
        return self

    def stats(self, reset: bool = False) -> dict:
        st = ps_stats()
        _check(_lib.pauli_sum_stats(self._h, ctypes.byref(st), int(reset)))
        return st.as_dict()

    def as_dict(self) -> dict:
        t, c = self.export()
        return {tuple(int(v) for v in row): c[i].copy() for i, row in enumerate(t)}

    def histogram(self, edges, signed: bool = True, lane: int = 0, noalloc: bool = False) -> np.ndarray:
        """Counts over the bins given by `edges` (relative to max|c|), then the
        counts below and above the range (Pauli-string density, Appendix D).
        noalloc: use pauli_sum_histogram_noalloc (no device allocation)."""
        e = np.ascontiguousarray(edges, dtype=np.float64)
        out = np.zeros(e.size + 1, dtype=np.uint64)
        f = _lib.pauli_sum_histogram_noalloc if noalloc else _lib.pauli_sum_histogram
        _check(f(self._h, lane, _ptr(e), e.size - 1, int(signed), _ptr(out)))
        return out

    def set_learned(self, eps_ratio: float = 1.0, tol: float = 0.0):
        """Learned-rule threshold ratio and fallback tolerance (see include/orqa.h)."""
        _check(_lib.pauli_sum_set_learned(self._h, float(eps_ratio), float(tol)))
        return self

    def set_rx_boundary_prologue(self, enable: bool = True):
        """enable=False: every RX tile finds its own boundaries (tests of that path)."""
        _check(_lib.pauli_sum_set_rx_boundary_prologue(self._h, int(enable)))
        return self

    def set_lookback_epoch(self, epoch: int):
        """Clear the look-back status words and restart their epoch (tests of the wrap guard)."""
        _check(_lib.pauli_sum_set_lookback_epoch(self._h, int(epoch)))
        return self

    def lookback_epoch(self) -> int:
        e = ctypes.c_uint32()
        _check(_lib.pauli_sum_lookback_epoch(self._h, ctypes.byref(e)))
        return int(e.value)

    def load_scorer(self, scorer: "PsScorer"):
        """Copy a scorer's network into this handle (for PS_TRUNC_LEARNED)."""
        _check(_lib.pauli_sum_load_scorer(self._h, scorer._h))
        return self


class PsScorer:
    """Learned truncation scorer: feature table, network and its training set
    on the GPU (semantics in include/orqa.h).  The feature table comes from
    paper_2506_13241_amd.scorer.feature_table."""

    def __init__(self, n_qubits: int, qmask, letters, scales, stream=None):
        lib = load_library()
        qmask = np.ascontiguousarray(qmask, dtype=np.uint64).reshape(160, 2)
        letters = np.ascontiguousarray(letters, dtype=np.uint8).reshape(160)
        scales = np.ascontiguousarray(scales, dtype=np.float32).reshape(160)
        self.n_qubits = n_qubits
        self.n = 0
        h = ctypes.c_void_p()
        if stream is None:
            stream = current_stream()
        _check(lib.ps_scorer_create(n_qubits, _ptr(qmask), _ptr(letters), _ptr(scales), stream, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ps_scorer_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        _check(_lib.ps_scorer_set_params(self._h, _ptr(p), p.size))
        return self

    def get_params(self) -> np.ndarray:
        p = np.empty(N_SCORER_PARAMS, dtype=np.float32)
        _check(_lib.ps_scorer_get_params(self._h, _ptr(p), p.size))
        return p

    def set_data(self, keys, targets):
        k = _words_to_pauli(keys)
        t = np.ascontiguousarray(targets, dtype=np.float32).reshape(-1)
        if t.size != k.shape[0]:
            raise ValueError("one target per key")
        _check(_lib.ps_scorer_set_data(self._h, _ptr(k), _ptr(t), k.shape[0]))
        self.n = k.shape[0]
        return self

    def forward(self, features: bool = False):
        """Network outputs of the training set (and its bf16 features as uint16)."""
        y = np.empty(self.n, dtype=np.float32)
        f = np.empty((self.n, 160), dtype=np.uint16) if features else None
        _check(_lib.ps_scorer_forward(self._h, _ptr(y), _ptr(f) if features else None))
        return (y, f) if features else y

    def loss_grad(self, grad: bool = True):
        loss = ctypes.c_double()
        g = np.empty(N_SCORER_PARAMS, dtype=np.float32) if grad else None
        _check(_lib.ps_scorer_loss_grad(self._h, ctypes.byref(loss), _ptr(g) if grad else None))
        return (loss.value, g) if grad else loss.value

    def adam_step(self, lr: float):
        _check(_lib.ps_scorer_adam_step(self._h, lr))
        return self


# C-ABI names at module level (same names, same meaning).
def pauli_sum_create(n_qubits, terms, coeffs, dtype=PS_F64, capacity=0, stream=None) -> PauliSum:
    return PauliSum(n_qubits, terms, coeffs, dtype=dtype, capacity=capacity, stream=stream)


def pauli_sum_destroy(ps: PauliSum):
    ps.close()


def apply_rotation_layer(ps: PauliSum, gates, rel_eps=0.0, trunc_mode=PS_TRUNC_MAGNITUDE):
    return ps.apply_rotation_layer(gates, rel_eps, trunc_mode)


def pauli_sum_truncate(ps: PauliSum, rel_eps, trunc_mode=PS_TRUNC_MAGNITUDE):
    return ps.truncate(rel_eps, trunc_mode)


truncate = pauli_sum_truncate


def expectation_z(ps: PauliSum):
    return ps.expectation_z()


def pauli_sum_size(ps: PauliSum):
    return ps.size()


def pauli_sum_norm2(ps: PauliSum):
    return ps.norm2()


def pauli_sum_export(ps: PauliSum):
    return ps.export()


def pauli_sum_histogram(ps: PauliSum, edges, signed=True, lane=0):
    return ps.histogram(edges, signed, lane)


def pauli_sum_histogram_noalloc(ps: PauliSum, edges, signed=True, lane=0):
    return ps.histogram(edges, signed, lane, noalloc=True)


def pauli_sum_set_lookback_epoch(ps: PauliSum, epoch: int):
    return ps.set_lookback_epoch(epoch)


def pauli_sum_lookback_epoch(ps: PauliSum) -> int:
    return ps.lookback_epoch()


def pauli_sum_set_rx_boundary_prologue(ps: PauliSum, enable: bool = True):
    return ps.set_rx_boundary_prologue(enable)


def pauli_sum_set_learned(ps: PauliSum, eps_ratio: float = 1.0, tol: float = 0.0):
    return ps.set_learned(eps_ratio, tol)


def pauli_sum_load_scorer(ps: PauliSum, scorer: PsScorer):
    return ps.load_scorer(scorer)


def pauli_sum_set_sort_config(ps: PauliSum, digit_bits=0, items_per_thread=0):
    return ps.set_sort_config(digit_bits, items_per_thread)


def pauli_sum_set_graphs(ps: PauliSum, enable=True):
    return ps.set_graphs(enable)


def pauli_sum_set_timing(ps: PauliSum, enable=True):
    return ps.set_timing(enable)


def pauli_sum_stats(ps: PauliSum, reset=False) -> dict:
    return ps.stats(reset)


def pauli_sum_gates_applied(ps: PauliSum) -> int:
    return ps.gates_applied()


def ps_scorer_create(n_qubits, qmask, letters, scales, stream=None) -> PsScorer:
    return PsScorer(n_qubits, qmask, letters, scales, stream=stream)


def ps_scorer_destroy(s: PsScorer):
    s.close()


def ps_last_error() -> str:
    """Message of the calling thread's last failed library call."""
    return load_library().ps_last_error().decode()


def ps_scorer_set_params(s: PsScorer, params):
    return s.set_params(params)


def ps_scorer_get_params(s: PsScorer) -> np.ndarray:
    return s.get_params()


def ps_scorer_set_data(s: PsScorer, keys, targets):
    return s.set_data(keys, targets)


def ps_scorer_forward(s: PsScorer, features: bool = False):
    return s.forward(features)


def ps_scorer_loss_grad(s: PsScorer, grad: bool = True):
    return s.loss_grad(grad)


def ps_scorer_adam_step(s: PsScorer, lr: float):
    return s.adam_step(lr)
