"""Dense Schrodinger-picture reference (paper Sec. 2.2) used to pin the oracle.

A 2^n complex128 array holds every amplitude; index i is the basis state whose
bit q is qubit q (Sec. 2.1).  Gate matrices are built from their definitions
in Sec. 2.1 with library routines where the definition is an exponential
(R_P(theta) = expm(-i theta P / 2) via scipy), so this file shares neither the
oracle's gate table nor its trigonometric formulas.  A controlled gate acts as
|0><0| (x) 1 + |1><1| (x) U on every control (Sec. 2.1).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

from paper_2105_01533_amd import workloads as W

PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
I2 = np.eye(2, dtype=complex)


def gate_matrix(kind: int, theta: float) -> np.ndarray:
    if kind == W.K_X:
        return PX
    if kind == W.K_Y:
        return PY
    if kind == W.K_Z:
        return PZ
    if kind == W.K_S:
        return np.diag([1, 1j])
    if kind == W.K_SDG:
        return np.diag([1, 1j]).conj().T
    if kind == W.K_T:
        return np.diag([1, np.exp(1j * np.pi / 4)])
    if kind == W.K_TDG:
        return np.diag([1, np.exp(1j * np.pi / 4)]).conj().T
    if kind == W.K_RZ:
        return expm(-0.5j * theta * PZ)
    if kind == W.K_RX:
        return expm(-0.5j * theta * PX)
    if kind == W.K_RY:
        return expm(-0.5j * theta * PY)
    if kind == W.K_PHASE:
        return np.diag([1, np.exp(1j * theta)])
    if kind == W.K_H:
        return np.sqrt(0.5) * np.array([[1, 1], [1, -1]], dtype=complex)
    raise ValueError(kind)


class Dense:
    def __init__(self, n: int, basis: int = 0):
        assert n <= 22
        self.n = n
        self.psi = np.zeros(1 << n, dtype=complex)
        self.psi[basis] = 1.0
        self.idx = np.arange(1 << n, dtype=np.int64)

    def apply(self, U: np.ndarray, target: int, ctrl_mask: int = 0):
        i0 = self.idx[((self.idx >> target) & 1 == 0) & ((self.idx & ctrl_mask) == ctrl_mask)]
        i1 = i0 | (1 << target)
        a0, a1 = self.psi[i0].copy(), self.psi[i1].copy()
        self.psi[i0] = U[0, 0] * a0 + U[0, 1] * a1
        self.psi[i1] = U[1, 0] * a0 + U[1, 1] * a1

    def measure(self, q: int, u: float, forced: int = -1) -> int:
        p = np.abs(self.psi) ** 2
        bit = (self.idx >> q) & 1
        p0, p1 = p[bit == 0].sum(), p[bit == 1].sum()
        o = forced if forced >= 0 else (0 if u < p0 / (p0 + p1) else 1)
        self.psi[bit != o] = 0
        self.psi /= np.sqrt(p1 if o else p0)
        return o

    def run(self, ops: np.ndarray, skip_cap_nnz=None):
        """Apply op records.  Branching gates with cap != 0 consult
        skip_cap_nnz(i) -> bool (whether the sparse run skipped op i)."""
        outs = []
        for i, op in enumerate(ops):
            kind = int(op["kind"])
            if kind == W.K_MEASURE:
                outs.append(self.measure(int(op["target"]), float(op["param"]), int(op["forced"])))
                continue
            if kind in W.BRANCHING_KINDS and int(op["cap"]) and skip_cap_nnz is not None and skip_cap_nnz(i):
                continue
            ctrl = int(op["ctrl_lo"]) | (int(op["ctrl_hi"]) << 64)
            self.apply(gate_matrix(kind, float(op["param"])), int(op["target"]), ctrl)
        return outs

    def as_dict(self, tol: float = 0.0) -> dict:
        nz = np.nonzero(np.abs(self.psi) > tol)[0]
        return {int(i): self.psi[i] for i in nz}


def pauli_string_matrix(n: int, qubits, paulis) -> np.ndarray:
    """Full 2^n x 2^n matrix of a Pauli string (qubit q = bit q of the index)."""
    mats = {"X": PX, "Y": PY, "Z": PZ}
    M = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):       # kron: highest qubit leftmost
        op = mats[paulis[qubits.index(q)]] if q in qubits else I2
        M = np.kron(M, op)
    return M
