"""CPU oracle for the sparse simulator -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never loads it and the
two share no code; both consume the same op records from the seeded workload
generator.

``Oracle`` wraps ``liboracle.so`` (built from ``sparse_oracle.cpp`` by
``build()``), a std::unordered_map simulation of the sparse method of
arXiv 2105.01533 Sec. 3 -- see the header of ``sparse_oracle.cpp`` for the
operations and the readings it takes where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sparse_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

TRACE_DTYPE = np.dtype([("nnz_in", "<u8"), ("applied", "<i4"), ("outcome", "<i4"),
                        ("p0", "<f8"), ("p1", "<f8")])


class Totals(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_uint64), ("u2_applied", ctypes.c_uint64),
                ("u2_skipped", ctypes.c_uint64), ("measures", ctypes.c_uint64),
                ("mono_gates", ctypes.c_uint64), ("peak_nnz", ctypes.c_uint64),
                ("pruned", ctypes.c_uint64), ("pruned_mass", ctypes.c_double),
                ("parallel_runs", ctypes.c_uint64), ("min_margin", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (no fused multiply-add)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, u64, f64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_double, ctypes.c_int32
        L.orc_create.restype = vp
        L.orc_create.argtypes = [ctypes.c_uint, f64]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_basis.argtypes = [vp, u64, u64]
        L.orc_import.argtypes = [vp, vp, vp, vp, u64]
        L.orc_nnz.restype = u64
        L.orc_nnz.argtypes = [vp]
        L.orc_run.argtypes = [vp, vp, u64, ctypes.c_int, vp, vp, ctypes.POINTER(u64)]
        L.orc_export.restype = u64
        L.orc_export.argtypes = [vp, vp, vp, vp, u64]
        L.orc_probabilities.argtypes = [vp, ctypes.c_uint, ctypes.POINTER(f64), ctypes.POINTER(f64)]
        L.orc_totals.argtypes = [vp, ctypes.POINTER(Totals)]
        L.orc_monomial_samples.argtypes = [vp, u64, vp, vp, vp, u64]
        L.orc_run_commuting.argtypes = [vp, vp, u64, vp, u64, ctypes.POINTER(u64), vp, ctypes.POINTER(u64)]
        L.orc_run_pauli.argtypes = [vp, vp, u64, vp, ctypes.POINTER(u64)]
        L.orc_set_threads.restype = ctypes.c_uint
        L.orc_set_threads.argtypes = [vp, ctypes.c_uint]
        for f in ("orc_set_basis", "orc_import", "orc_run", "orc_probabilities", "orc_monomial_samples",
                  "orc_run_commuting", "orc_run_pauli"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


class Oracle:
    """Sparse state {label: amplitude}; labels are (lo, hi) uint64 pairs."""

    def __init__(self, n_qubits: int, eps: float = 0.0):
        self.n_qubits = n_qubits
        self.eps = eps
        self.h = lib().orc_create(n_qubits, eps)
        if not self.h:
            raise OracleError("bad qubit count")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def set_threads(self, n: int = 0) -> int:
        """Threads for queues of more than 64 gates on more than 4096 entries
        (Sec. 5); 0 = all hardware threads.  Returns the count in use."""
        return int(lib().orc_set_threads(self.h, n))

    def set_basis(self, lo: int = 0, hi: int = 0):
        lib().orc_set_basis(self.h, lo, hi)

    def import_state(self, lo, hi, amp):
        lo = np.ascontiguousarray(lo, dtype=np.uint64)
        hi = np.ascontiguousarray(hi, dtype=np.uint64)
        amp = np.ascontiguousarray(amp, dtype=np.complex128)
        if lib().orc_import(self.h, _ptr(lo), _ptr(hi), _ptr(amp), len(lo)) != 0:
            raise OracleError("duplicate label in import")

    def run(self, ops: np.ndarray, queued: bool = True, trace: bool = False):
        """Apply op records.  Returns (outcomes, trace-or-None)."""
        ops = np.ascontiguousarray(ops)
        assert ops.dtype.itemsize == 48
        n_meas = int(np.count_nonzero(ops["kind"] == 12))
        outcomes = np.full(max(n_meas, 1), -1, dtype=np.int32)
        tr = np.zeros(len(ops), dtype=TRACE_DTYPE) if trace else None
        bad = ctypes.c_uint64(0)
        rc = lib().orc_run(self.h, _ptr(ops), len(ops), int(queued),
                           _ptr(tr) if trace else None, _ptr(outcomes), ctypes.byref(bad))
        if rc == -1:
            raise OracleError(f"invalid op at index {bad.value}")
        if rc == -2:
            raise OracleError(f"zero-probability measurement at index {bad.value}")
        return outcomes[:n_meas], tr

    def run_commuting(self, ops: np.ndarray):
        """Apply op records through the gate-commuting queues (Sec. 3.3).
        Returns (outcomes, log): log holds the op records sent to the state,
        in order (the queues' contents as they were executed)."""
        ops = np.ascontiguousarray(ops)
        assert ops.dtype.itemsize == 48
        n_meas = int(np.count_nonzero(ops["kind"] == 12))
        outcomes = np.full(max(n_meas, 1), -1, dtype=np.int32)
        log = np.zeros(max(len(ops), 1), dtype=ops.dtype)
        n_log = ctypes.c_uint64(0)
        bad = ctypes.c_uint64(0)
        rc = lib().orc_run_commuting(self.h, _ptr(ops), len(ops), _ptr(log), len(log), ctypes.byref(n_log),
                                     _ptr(outcomes), ctypes.byref(bad))
        if rc == -1:
            raise OracleError(f"invalid op at index {bad.value}")
        if rc == -2:
            raise OracleError(f"zero-probability measurement at index {bad.value}")
        assert n_log.value <= len(log), "applied-gate log longer than the input"
        return outcomes[:n_meas], log[:n_log.value]

    def run_pauli(self, terms: np.ndarray, trace: bool = False):
        """Apply Pauli-exponential records exp(-i theta P) in order (64-byte
        records: x, z, ctrl masks as lo/hi pairs, theta, cap).  Returns the
        trace or None."""
        terms = np.ascontiguousarray(terms)
        assert terms.dtype.itemsize == 64
        tr = np.zeros(len(terms), dtype=TRACE_DTYPE) if trace else None
        bad = ctypes.c_uint64(0)
        rc = lib().orc_run_pauli(self.h, _ptr(terms), len(terms), _ptr(tr) if trace else None, ctypes.byref(bad))
        if rc == -1:
            raise OracleError(f"invalid Pauli term at index {bad.value}")
        return tr

    @property
    def nnz(self) -> int:
        return int(lib().orc_nnz(self.h))

    def export(self):
        """Sorted (lo, hi, amp complex128) arrays."""
        n = self.nnz
        lo = np.empty(n, np.uint64)
        hi = np.empty(n, np.uint64)
        amp = np.empty(n, np.complex128)
        got = lib().orc_export(self.h, _ptr(lo), _ptr(hi), _ptr(amp), n)
        assert got == n
        return lo, hi, amp

    def probabilities(self, q: int):
        p0, p1 = ctypes.c_double(), ctypes.c_double()
        if lib().orc_probabilities(self.h, q, ctypes.byref(p0), ctypes.byref(p1)) != 0:
            raise OracleError("bad qubit")
        return p0.value, p1.value

    def totals(self) -> dict:
        t = Totals()
        lib().orc_totals(self.h, ctypes.byref(t))
        return {f: getattr(t, f) for f, _ in Totals._fields_}


def monomial_samples(ops: np.ndarray, lo, hi, amp):
    """Apply a list of phase/permutation op records to independent samples."""
    ops = np.ascontiguousarray(ops)
    lo = np.array(lo, dtype=np.uint64)
    hi = np.array(hi, dtype=np.uint64)
    amp = np.array(amp, dtype=np.complex128)
    if lib().orc_monomial_samples(_ptr(ops), len(ops), _ptr(lo), _ptr(hi), _ptr(amp), len(lo)) != 0:
        raise OracleError("non-monomial op in sample run")
    return lo, hi, amp


def run_workload(w, queued: bool = True, trace: bool = False):
    """Run a workloads.Workload from its basis state; returns (oracle, outcomes, trace)."""
    o = Oracle(w.n_qubits, w.eps)
    o.set_basis(*w.basis)
    outcomes, tr = o.run(w.ops, queued=queued, trace=trace)
    return o, outcomes, tr


def run_pauli_workload(w, trace: bool = False):
    """Run a workloads.PauliWorkload from its basis state; returns (oracle, trace)."""
    o = Oracle(w.n_qubits, w.eps)
    o.set_basis(*w.basis)
    tr = o.run_pauli(w.terms, trace=trace)
    return o, tr
