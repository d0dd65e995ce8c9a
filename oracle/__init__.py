"""Reference oracle for ORQA propagation (test infrastructure only).

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  It shares no code with the HIP library:
the map-based propagator is plain C++ (`orqa_oracle.cpp`), the statevector and
dense Pauli-basis brute forces are numpy (`statevector.py`, `dense.py`), and
the scorer network reference is numpy FP64 (`mlp.py`).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orqa_oracle.cpp")
# ORQA_ORACLE_LIB names another build of the same source (the sanitized one
# of tests/test_oracle_sanitized.py); by default the in-tree library is used.
_LIB = os.environ.get("ORQA_ORACLE_LIB") or os.path.join(_HERE, "liborqa_oracle.so")


def build(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the C++ oracle (g++, FP contraction off) to `out` (default: the
    library this module loads).  sanitize=True adds AddressSanitizer and
    UndefinedBehaviorSanitizer, every report fatal; such a build is loaded
    only by a process that has the ASan runtime preloaded."""
    out = out or _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC"]
        if sanitize:
            cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all"]
        subprocess.check_call(cmd + ["-o", tmp, _SRC])
        os.replace(tmp, out)
    return out


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_size_t, ctypes.POINTER(P)]
        lib.orc_create.restype = ctypes.c_int
        lib.orc_destroy.argtypes = [P]
        lib.orc_destroy.restype = None
        lib.orc_apply.argtypes = [P, P, P, ctypes.c_size_t, ctypes.c_double]
        lib.orc_apply.restype = ctypes.c_int
        lib.orc_truncate.argtypes = [P, ctypes.c_double]
        lib.orc_truncate.restype = ctypes.c_int
        lib.orc_size.argtypes = [P]
        lib.orc_size.restype = ctypes.c_size_t
        lib.orc_updates.argtypes = [P]
        lib.orc_updates.restype = ctypes.c_double
        lib.orc_expectation_z.argtypes = [P, P]
        lib.orc_expectation_z.restype = ctypes.c_int
        lib.orc_norm2.argtypes = [P, P]
        lib.orc_norm2.restype = ctypes.c_int
        lib.orc_export.argtypes = [P, P, P, ctypes.c_size_t]
        lib.orc_export.restype = ctypes.c_size_t
        lib.orc_phase_B.argtypes = [ctypes.c_int, P, P]
        lib.orc_phase_B.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleSum:
    """std::map FP64 Pauli sum.  terms: (m,4) uint64 x/z words; coeffs: (m,L)."""

    def __init__(self, n_qubits: int, terms, coeffs):
        lib = _load()
        terms = np.ascontiguousarray(terms, dtype=np.uint64).reshape(-1, 4)
        coeffs = np.ascontiguousarray(coeffs, dtype=np.float64).reshape(terms.shape[0], -1)
        self.n_qubits = n_qubits
        self.lanes = coeffs.shape[1]
        h = ctypes.c_void_p()
        rc = lib.orc_create(n_qubits, self.lanes, _ptr(terms), _ptr(coeffs), terms.shape[0], ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"orc_create failed ({rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def apply(self, gates, eps0: float = 0.0) -> "OracleSum":
        gens = np.ascontiguousarray(gates.gens, dtype=np.uint64)
        th = np.ascontiguousarray(gates.thetas, dtype=np.float64)
        if th.shape[1] == 1 and self.lanes > 1:
            th = np.ascontiguousarray(np.repeat(th, self.lanes, axis=1))
        assert th.shape == (gens.shape[0], self.lanes)
        rc = _load().orc_apply(self._h, _ptr(gens), _ptr(th), gens.shape[0], float(eps0))
        assert rc == 0
        return self

    def truncate(self, eps0: float) -> "OracleSum":
        _load().orc_truncate(self._h, float(eps0))
        return self

    def size(self) -> int:
        return int(_load().orc_size(self._h))

    def updates(self) -> float:
        return float(_load().orc_updates(self._h))

    def expectation_z(self) -> np.ndarray:
        out = np.zeros(self.lanes)
        _load().orc_expectation_z(self._h, _ptr(out))
        return out

    def norm2(self) -> np.ndarray:
        out = np.zeros(self.lanes)
        _load().orc_norm2(self._h, _ptr(out))
        return out

    def export(self) -> tuple[np.ndarray, np.ndarray]:
        """(terms (m,4) uint64, coeffs (m,L)), sorted by (x1,x0,z1,z0) words."""
        m = self.size()
        terms = np.zeros((m, 4), dtype=np.uint64)
        coeffs = np.zeros((m, self.lanes))
        got = _load().orc_export(self._h, _ptr(terms), _ptr(coeffs), m)
        assert got == m
        order = np.lexsort((terms[:, 2], terms[:, 3], terms[:, 0], terms[:, 1]))
        return terms[order], coeffs[order]

    def as_dict(self) -> dict:
        t, c = self.export()
        return {tuple(int(v) for v in row): c[i].copy() for i, row in enumerate(t)}


def phase_B(n_qubits: int, I_xz, J_xz) -> int:
    a = np.ascontiguousarray(I_xz, dtype=np.uint64)
    b = np.ascontiguousarray(J_xz, dtype=np.uint64)
    return int(_load().orc_phase_B(n_qubits, _ptr(a), _ptr(b)))
