"""Seeded synthetic circuit generators.

This module only draws circuits: which gate, on which qubits, with which
angle, and the uniform number each measurement consumes.  It holds none of
the simulation arithmetic (no gate matrices, no state), imports nothing from
the rest of the package, and is the single input source shared by the GPU
library, the CPU oracle and the benchmark.

Circuits are numpy arrays of ``OP_DTYPE`` records ("op records"):

  kind    gate kind (``K_*`` below)
  target  target qubit
  ctrl_lo / ctrl_hi   128-bit control mask (qubit q <-> bit q; q >= 64 in hi)
  param   rotation angle for RZ/RX/RY/PHASE, the uniform u in [0,1) for MEASURE
  cap     branching gates only: skip the gate iff cap != 0 and 2*nnz > cap
  forced  MEASURE only: -1 = sample with u, 0/1 = force that outcome

Randomness is SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014); uniform doubles are (x >> 11) * 2^-53 and
normal deviates use the Box-Muller transform.  Each synthetic workload mirrors
a family the paper benchmarks (Sec. 4): a permutation-heavy random circuit
with sparse branching (the "~60 % permutations" mix of Sec. 5), a ripple-carry
adder on a superposed register (the CDKM arithmetic of Sec. 4.1) and a
Trotter-like product of Pauli exponentials (Sec. 4.4).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --- gate kinds (shared record format) -------------------------------------
K_X, K_Y, K_Z, K_S, K_SDG, K_T, K_TDG, K_RZ, K_PHASE = 0, 1, 2, 3, 4, 5, 6, 7, 8
K_H, K_RX, K_RY = 9, 10, 11
K_MEASURE = 12
KIND_NAMES = {K_X: "X", K_Y: "Y", K_Z: "Z", K_S: "S", K_SDG: "SDG", K_T: "T",
              K_TDG: "TDG", K_RZ: "RZ", K_PHASE: "PHASE", K_H: "H", K_RX: "RX",
              K_RY: "RY", K_MEASURE: "MEASURE"}
MONOMIAL_KINDS = (K_X, K_Y, K_Z, K_S, K_SDG, K_T, K_TDG, K_RZ, K_PHASE)
BRANCHING_KINDS = (K_H, K_RX, K_RY)

OP_DTYPE = np.dtype([
    ("kind", "<u4"), ("target", "<u4"),
    ("ctrl_lo", "<u8"), ("ctrl_hi", "<u8"),
    ("param", "<f8"), ("cap", "<u8"),
    ("forced", "<i4"), ("pad", "<u4"),
])
assert OP_DTYPE.itemsize == 48

# Pauli-exponential records ("Pauli terms"), exp(-i theta P): P acts as X on
# the qubits in x only, Y on those in x and z, Z on those in z only; ctrl as
# for op records; cap skips a term with x != 0 iff cap != 0 and 2*nnz > cap.
PAULI_DTYPE = np.dtype([
    ("x_lo", "<u8"), ("x_hi", "<u8"), ("z_lo", "<u8"), ("z_hi", "<u8"),
    ("ctrl_lo", "<u8"), ("ctrl_hi", "<u8"), ("theta", "<f8"), ("cap", "<u8"),
])
assert PAULI_DTYPE.itemsize == 64

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 stream with the published constants."""

    def __init__(self, seed: int):
        self.s = seed & MASK64

    def next(self) -> int:
        self.s = (self.s + 0x9E3779B97F4A7C15) & MASK64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)

    def randint(self, n: int) -> int:
        return min(int(self.uniform() * n), n - 1)

    def distinct(self, n: int, k: int) -> list[int]:
        out: list[int] = []
        while len(out) < k:
            q = self.randint(n)
            if q not in out:
                out.append(q)
        return out

    def normal(self) -> float:
        u1 = 1.0 - self.uniform()          # (0, 1]
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def seed_for(config: int, run: int = 0) -> int:
    """Run r of config c uses seed 1000*(c+1) + r."""
    return 1000 * (config + 1) + run


# --- circuit builder ---------------------------------------------------------
class Circuit:
    def __init__(self):
        self.rows: list[tuple] = []

    def gate(self, kind, target, controls=(), param=0.0, cap=0):
        lo = hi = 0
        for c in controls:
            if c < 64:
                lo |= 1 << c
            else:
                hi |= 1 << (c - 64)
        self.rows.append((kind, target, lo, hi, float(param), int(cap), -1, 0))

    def measure(self, q, u, forced=-1):
        self.rows.append((K_MEASURE, q, 0, 0, float(u), 0, int(forced), 0))

    # named helpers
    def x(self, t, ctrls=()):
        self.gate(K_X, t, ctrls)

    def h(self, t, ctrls=(), cap=0):
        self.gate(K_H, t, ctrls, cap=cap)

    def array(self) -> np.ndarray:
        return np.array(self.rows, dtype=OP_DTYPE)

    def __len__(self):
        return len(self.rows)


@dataclass
class Workload:
    name: str
    n_qubits: int
    eps: float
    ops: np.ndarray
    capacity: int                 # entries the state may need (upper bound)
    basis: tuple[int, int] = (0, 0)   # initial basis key (lo, hi)
    meta: dict = field(default_factory=dict)


def _random_mono(rng: SplitMix64, c: Circuit, n: int, perm_frac: float, phase_frac: float,
                 h_cap: int):
    """One gate of the random mix: X/CNOT/Toffoli with probability perm_frac,
    Z/S/T/Rz with probability phase_frac, otherwise a capped H."""
    u = rng.uniform()
    if u < perm_frac:
        which = rng.randint(3)               # 0 X, 1 CNOT, 2 Toffoli
        qs = rng.distinct(n, which + 1)
        c.gate(K_X, qs[-1], qs[:-1])
    elif u < perm_frac + phase_frac:
        which = rng.randint(4)               # Z, S, T, Rz
        q = rng.randint(n)
        if which == 3:
            c.gate(K_RZ, q, (), param=rng.uniform() * 2.0 * math.pi)
        else:
            c.gate((K_Z, K_S, K_T)[which], q)
    else:
        c.h(rng.randint(n), cap=h_cap)


def config0(seed: int = seed_for(0), n: int = 24, h_qubits: int = 10, gates: int = 5000,
            cap: int = 1 << 16, measured: int = 4) -> Workload:
    """Plain sparse simulation: |0>, H on q0..q9, 5,000 random gates
    (70 % X/CNOT/Toffoli, 25 % Z/S/T/Rz(theta ~ U[0, 2pi)), 5 % H skipped when
    the state could exceed 2^16 entries), then measure q0..q3 in order."""
    rng = SplitMix64(seed)
    c = Circuit()
    for q in range(h_qubits):
        c.h(q)
    for _ in range(gates):
        _random_mono(rng, c, n, 0.70, 0.25, cap)
    for q in range(measured):
        c.measure(q, rng.uniform())
    return Workload("c0_plain_24q", n, 1e-20, c.array(), capacity=max(cap, 1 << h_qubits),
                    meta={"seed": seed, "gates": gates})


def cdkm_add(c: Circuit, a: list[int], b: list[int], c0: int, z: int):
    """In-place ripple-carry addition a += b (Cuccaro, Draper, Kutin, Moulton,
    quant-ph/0410184), with ancilla c0 (restored) and carry-out z (z ^= carry).
    The running carry lives in b; b and c0 are restored by the UMA half."""
    w = len(a)
    carry = [c0] + b[:-1]
    for i in range(w):                        # MAJ(c_i, a_i, b_i)
        c.x(a[i], (b[i],))
        c.x(carry[i], (b[i],))
        c.x(b[i], (carry[i], a[i]))
    c.x(z, (b[w - 1],))
    for i in reversed(range(w)):              # UMA(c_i, a_i, b_i)
        c.x(b[i], (carry[i], a[i]))
        c.x(carry[i], (b[i],))
        c.x(a[i], (carry[i],))


def config1(seed: int = seed_for(1), w: int = 20, adds: int = 50, n: int = 64) -> Workload:
    """Arithmetic circuit: H on register A (2^w entries), a seeded w-bit constant
    loaded into B with X, `adds` CDKM additions A += B, a controlled-Rz(pi/2^j)
    ladder on A, then a final H layer on A."""
    rng = SplitMix64(seed)
    A = list(range(w))
    B = list(range(w, 2 * w))
    c0, z = 2 * w, 2 * w + 1
    assert z < n
    const = rng.next() & ((1 << w) - 1)
    c = Circuit()
    for q in A:
        c.h(q)
    for i in range(w):
        if (const >> i) & 1:
            c.x(B[i])
    for _ in range(adds):
        cdkm_add(c, A, B, c0, z)
    for i in range(w):
        for j in range(1, w - i):
            c.gate(K_RZ, A[i], (A[i + j],), param=math.pi / (1 << j))
    for q in A:
        c.h(q)
    return Workload(f"c1_adder_{n}q_w{w}", n, 1e-20, c.array(), capacity=2 << w,
                    meta={"seed": seed, "const": const, "w": w, "adds": adds})


def config2(seed: int = seed_for(2), n: int = 100, h_qubits: int = 24, gates: int = 200_000,
            round_gates: int = 20_000, meas_per_round: int = 8, cap: int | None = None) -> Workload:
    """Large sparse random circuit: H on 24 qubits, 200,000 gates (80 % X/CNOT/
    Toffoli, 15 % Z/S/T/Rz, 5 % H capped at 2^24 entries) with 8 distinct random
    qubits measured after every 20,000 gates."""
    if cap is None:
        cap = 1 << h_qubits
    rng = SplitMix64(seed)
    c = Circuit()
    for q in range(h_qubits):
        c.h(q)
    for g in range(1, gates + 1):
        _random_mono(rng, c, n, 0.80, 0.15, cap)
        if g % round_gates == 0:
            for q in rng.distinct(n, meas_per_round):
                c.measure(q, rng.uniform())
    return Workload(f"c2_random_{n}q", n, 1e-20, c.array(), capacity=cap,
                    meta={"seed": seed, "gates": gates, "h_qubits": h_qubits})


def pauli_term(qubits, paulis, theta: float, ctrls=(), cap: int = 0) -> tuple:
    """One PAULI_DTYPE record for exp(-i theta P), P = paulis[k] on qubits[k]
    ("I", "X", "Y" or "Z"), controlled on ctrls."""
    x = z = cm = 0
    for q, p in zip(qubits, paulis):
        if p in ("X", "Y"):
            x |= 1 << q
        if p in ("Z", "Y"):
            z |= 1 << q
    for q in ctrls:
        cm |= 1 << q
    return (x & MASK64, x >> 64, z & MASK64, z >> 64, cm & MASK64, cm >> 64, float(theta), int(cap))


@dataclass
class PauliWorkload:
    name: str
    n_qubits: int
    eps: float
    terms: np.ndarray             # PAULI_DTYPE records
    capacity: int
    basis: tuple[int, int] = (0, 0)
    meta: dict = field(default_factory=dict)


def pauli_exp(c: Circuit, qubits: list[int], paulis: list[str], theta: float):
    """exp(-i theta P) for a Pauli string P on distinct ascending qubits:
    basis change to Z (X: H; Y: S^dagger then H), CNOT parity ladder onto the
    last qubit, Rz(2 theta) there, then the ladder and basis change undone."""
    for q, p in zip(qubits, paulis):
        if p == "X":
            c.h(q)
        elif p == "Y":
            c.gate(K_SDG, q)
            c.h(q)
    for a, b in zip(qubits[:-1], qubits[1:]):
        c.x(b, (a,))
    c.gate(K_RZ, qubits[-1], (), param=2.0 * theta)
    for a, b in reversed(list(zip(qubits[:-1], qubits[1:]))):
        c.x(b, (a,))
    for q, p in zip(qubits, paulis):
        if p == "X":
            c.h(q)
        elif p == "Y":
            c.h(q)
            c.gate(K_S, q)


def phase_oracle_blocks(seed: int = 5151, n: int = 64, superposed: int = 20, blocks: int = 2000,
                        ctrl_max: int = 3, eps: float = 1e-20) -> Workload:
    """H on q0..q(superposed-1), then `blocks` phase-oracle blocks: H on a
    target t, an X on t with 1..ctrl_max controls, H on t (together a
    controlled Z), each followed with probability 1/4 by an X or Z on a random
    qubit.  Targets and controls are uniform over all qubits."""
    rng = SplitMix64(seed)
    c = Circuit()
    for q in range(superposed):
        c.h(q)
    for _ in range(blocks):
        k = 1 + rng.randint(ctrl_max)
        qs = rng.distinct(n, k + 1)
        t, ctrls = qs[-1], qs[:-1]
        c.h(t)
        c.x(t, ctrls)
        c.h(t)
        if rng.randint(4) == 0:
            c.gate((K_X, K_Z)[rng.randint(2)], rng.randint(n))
    return Workload(f"phase_oracle_{n}q_{blocks}b", n, eps, c.array(), capacity=1 << (superposed + 1),
                    meta={"seed": seed, "superposed": superposed, "blocks": blocks})


def config3(seed: int = seed_for(3), n: int = 40, set_bits: int = 20, terms: int = 500,
            locality: int = 4, capacity: int = 1 << 22) -> Workload:
    """Chemistry-like Trotter step: start from the basis state with q0..q19 set,
    apply 500 factors exp(-i theta P) with P a random 4-local Pauli string over
    {X, Y, Z} and theta = 0.01 N(0, 1); prune |a|^2 < 1e-10."""
    c = Circuit()
    for qs, ps, theta in _trotter_terms(seed, n, terms, locality):
        pauli_exp(c, qs, ps, theta)
    basis = (1 << set_bits) - 1
    return Workload(f"c3_trotter_{n}q", n, 1e-10, c.array(), capacity=capacity,
                    basis=(basis & MASK64, basis >> 64), meta={"seed": seed, "terms": terms})


def _trotter_terms(seed: int, n: int, terms: int, locality: int):
    rng = SplitMix64(seed)
    out = []
    for _ in range(terms):
        qs = sorted(rng.distinct(n, locality))
        ps = ["XYZ"[rng.randint(3)] for _ in qs]
        theta = 0.01 * rng.normal()
        out.append((qs, ps, theta))
    return out


def config3_terms(seed: int = seed_for(3), n: int = 40, set_bits: int = 20, terms: int = 500,
                  locality: int = 4, capacity: int = 1 << 22) -> PauliWorkload:
    """The same Trotter step as config3 (same draws), as native Pauli terms
    exp(-i theta P) instead of basis-change / CNOT-ladder / Rz circuits."""
    recs = [pauli_term(qs, ps, theta) for qs, ps, theta in _trotter_terms(seed, n, terms, locality)]
    basis = (1 << set_bits) - 1
    return PauliWorkload(f"c3_trotter_{n}q_native", n, 1e-10, np.array(recs, dtype=PAULI_DTYPE),
                         capacity=capacity, basis=(basis & MASK64, basis >> 64), meta={"seed": seed, "terms": terms})


def random_pauli_terms(seed: int, n: int, count: int, max_weight: int = 4, ctrl_max: int = 2,
                       diag_frac: float = 0.2, ident_frac: float = 0.05, cap: int = 0,
                       theta_scale: float = math.pi) -> np.ndarray:
    """Random Pauli terms for tests: weight 1..max_weight over {X, Y, Z} (a
    diag_frac share Z-only, an ident_frac share the identity), 0..ctrl_max
    controls on other qubits, theta uniform in [-theta_scale, theta_scale)."""
    rng = SplitMix64(seed)
    recs = []
    for _ in range(count):
        u = rng.uniform()
        w = 1 + rng.randint(max_weight)
        nc = rng.randint(ctrl_max + 1)
        qs = rng.distinct(n, min(n, w + nc))
        ctrls, qs = qs[:nc], qs[nc:]
        if u < ident_frac:
            ps = ["I"] * len(qs)
        elif u < ident_frac + diag_frac:
            ps = ["Z"] * len(qs)
        else:
            ps = ["XYZ"[rng.randint(3)] for _ in qs]
        theta = (rng.uniform() * 2.0 - 1.0) * theta_scale
        recs.append(pauli_term(qs, ps, theta, ctrls, cap))
    return np.array(recs, dtype=PAULI_DTYPE)


def random_circuit(seed: int, n: int, gates: int, h_frac: float = 0.1, ctrl_max: int = 2,
                   with_rx_ry: bool = True, measure_frac: float = 0.0, cap: int = 0) -> Workload:
    """Small mixed circuit for tests: every gate kind, random controls."""
    rng = SplitMix64(seed)
    c = Circuit()
    mono = [K_X, K_Y, K_Z, K_S, K_SDG, K_T, K_TDG, K_RZ, K_PHASE]
    branch = [K_H, K_RX, K_RY] if with_rx_ry else [K_H]
    for _ in range(gates):
        u = rng.uniform()
        if u < measure_frac:
            c.measure(rng.randint(n), rng.uniform())
            continue
        nc = rng.randint(ctrl_max + 1)
        qs = rng.distinct(n, nc + 1)
        if u < measure_frac + h_frac:
            kind = branch[rng.randint(len(branch))]
        else:
            kind = mono[rng.randint(len(mono))]
        param = (rng.uniform() * 4.0 - 2.0) * math.pi
        c.gate(kind, qs[-1], qs[:-1], param=param, cap=cap)
    return Workload(f"random_{n}q_{gates}g", n, 0.0, c.array(), capacity=1 << min(n, 20),
                    meta={"seed": seed})


def _serving_request(spec):
    """Build one request of serving_trace from its drawn parameters."""
    r, fam, lg, ng, sub_seed, n_draw = spec
    if fam == 0:
        n = max(16, min(100, lg + 2 + n_draw))
        w = config0(sub_seed, n=n, h_qubits=max(1, lg - 4), gates=ng, cap=1 << lg)
    elif fam == 1:
        wbits = max(2, min(lg - 1, 30))
        n = max(2 * wbits + 2, 16 + n_draw)
        adds = max(1, ng // (6 * wbits + 1))
        w = config1(sub_seed, w=wbits, adds=adds, n=min(n, 128))
    else:
        n = max(16, min(100, lg + 8 + n_draw))
        rg = max(1, ng // 4)
        w = config2(sub_seed, n=n, h_qubits=lg, gates=ng, round_gates=rg,
                    meas_per_round=min(4, lg), cap=1 << lg)
    w.meta.update({"family": fam, "cap_log2": lg, "request": r})
    return w


def _serving_specs(seed, requests, rate, cap_log2, gates_range):
    """Arrival times and per-request parameters of serving_trace, drawn from
    one stream in request order."""
    rng = SplitMix64(seed)
    t = 0.0
    times, specs = [], []
    for r in range(requests):
        t += -math.log(1.0 - rng.uniform()) / rate
        fam = rng.randint(3)
        lg = cap_log2[0] + rng.randint(cap_log2[1] - cap_log2[0] + 1)
        lo, hi = math.log(gates_range[0]), math.log(gates_range[1])
        ng = int(math.exp(lo + rng.uniform() * (hi - lo)))
        sub_seed = rng.next() & 0xFFFFFFFF
        if fam == 0:
            n_draw = rng.randint(100 - lg - 1)
        elif fam == 1:
            n_draw = rng.randint(49)
        else:
            n_draw = rng.randint(100 - lg - 7)
        times.append(t)
        specs.append((r, fam, lg, ng, sub_seed, n_draw))
    return times, specs


def serving_trace(seed: int = 4242, requests: int = 512, rate: float = 100.0,
                  cap_log2: tuple[int, int] = (8, 22), gates_range: tuple[int, int] = (1000, 200_000),
                  workers: int = 1):
    """Poisson-arriving requests drawn from the config-0..2 families with seeded
    sizes: family uniform over {0, 1, 2}, entry cap 2^U{8..22}, gate count
    log-uniform in [1e3, 2e5].  Returns a list of (arrival_s, Workload).

    The arrival times and every request's parameters come from one stream in
    request order; the circuits (each from its own sub-seed) are then built,
    in a pool of `workers` forked processes when workers > 1 -- the same trace
    either way."""
    times, specs = _serving_specs(seed, requests, rate, cap_log2, gates_range)
    if workers > 1 and requests > 1:
        import multiprocessing as mp

        with mp.get_context("fork").Pool(min(workers, requests)) as pool:
            ws = pool.map(_serving_request, specs, chunksize=1)
    else:
        ws = [_serving_request(sp) for sp in specs]
    return list(zip(times, ws))


def serving_request(index: int, seed: int = 4242, requests: int = 512,
                    cap_log2: tuple[int, int] = (8, 22), gates_range: tuple[int, int] = (1000, 200_000)):
    """Request `index` of serving_trace(seed, requests, ...), built alone."""
    _, specs = _serving_specs(seed, requests, 1.0, cap_log2, gates_range)
    return _serving_request(specs[index])


# --- random sparse states (counter-based SplitMix64, vectorised) --------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64_array(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start..start+count-1 of the SplitMix64 stream of `seed`
    (output i mixes seed + (i+1)*gamma), as uint64."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def random_state(seed: int, n_entries: int, n_qubits: int, normalise: bool = True):
    """n_entries distinct random labels below 2^n_qubits with random complex
    amplitudes (re, im uniform in [-1, 1)), returned as (lo, hi, amp)."""
    assert n_qubits >= 64 or n_entries <= (1 << n_qubits)
    lo_mask = np.uint64((1 << min(n_qubits, 64)) - 1)
    hi_mask = np.uint64((1 << max(n_qubits - 64, 0)) - 1)
    keys: dict = {}
    lo = np.empty(0, np.uint64)
    hi = np.empty(0, np.uint64)
    ctr = 0
    while len(lo) < n_entries:
        m = 2 * (n_entries - len(lo)) + 16
        r = splitmix64_array(seed, ctr, 2 * m)
        ctr += 2 * m
        cand_lo = r[0::2] & lo_mask
        cand_hi = r[1::2] & hi_mask
        lo = np.concatenate([lo, cand_lo])
        hi = np.concatenate([hi, cand_hi])
        _, first = np.unique(np.stack([hi, lo], axis=1), axis=0, return_index=True)
        first.sort()
        lo, hi = lo[first], hi[first]
    lo, hi = lo[:n_entries], hi[:n_entries]
    return lo, hi, random_amplitudes(seed, n_entries, normalise)


def random_amplitudes(seed: int, n: int, normalise: bool = True) -> np.ndarray:
    """n random complex amplitudes, re and im uniform in [-1, 1)."""
    r = splitmix64_array(seed ^ 0x5DEECE66D, 0, 2 * n)
    u = (r >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    amp = (2.0 * u[0::2] - 1.0) + 1j * (2.0 * u[1::2] - 1.0)
    if normalise and n:
        amp = amp / np.sqrt(np.sum(np.abs(amp) ** 2))
    return amp
