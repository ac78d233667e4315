"""ctypes binding of libsparsesim (include/sparsesim.h) -- argument marshalling only.

Every step of the simulation runs in the HIP library; this module only
converts numpy arrays and torch device memory/streams into the C-ABI's plain
pointers.  Functions keep the C names.  ``Simulator`` is a small convenience
wrapper that borrows its workspace from torch and runs on torch's current
stream.

The library must be built (``python -m paper_2105_01533_amd.build``); there is
no fallback: a missing library raises ``ImportError`` at load time.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: it loads the HIP runtime that libsparsesim then shares.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsparsesim.so")

SIM_OK, SIM_E_ARG, SIM_E_NOMEM, SIM_E_CAPACITY, SIM_E_BUFFER, SIM_E_HIP, SIM_E_STATE = 0, -1, -2, -3, -4, -5, -6
SIM_OP_MONO, SIM_OP_U2, SIM_OP_MEASURE = 0, 1, 2
SIM_MONO_AUTO, SIM_MONO_DIRECT, SIM_MONO_BITSLICE = 0, 1, 2
SIM_PROFILE_OFF, SIM_PROFILE_ALL, SIM_PROFILE_MONO = 0, 1, 2
SIM_FLAG_U2_TWO_PASS = 1
SIM_FLAG_BS_LDS = 2
SIM_FLAG_U2_GLOBAL_INDEX = 4
SIM_FLAG_COUNT_INDEX = 8
SIM_FLAG_NO_UNIFORM = 16

GATE_DTYPE = np.dtype([
    ("op", "<u4"), ("target", "<u4"), ("ctrl_lo", "<u8"), ("ctrl_hi", "<u8"),
    ("flip", "<u4"), ("forced", "<i4"), ("m", "<c16", (4,)), ("cap", "<u8"), ("u", "<f8"),
    ("reserved", "<u8"), ("x_lo", "<u8"), ("x_hi", "<u8"), ("z_lo", "<u8"), ("z_hi", "<u8"),
])
assert GATE_DTYPE.itemsize == 152
KEY_DTYPE = np.dtype([("lo", "<u8"), ("hi", "<u8")])


class sim_config(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_uint32), ("fuse_max", ctypes.c_uint32), ("capacity", ctypes.c_uint64),
                ("eps", ctypes.c_double), ("load_factor", ctypes.c_double), ("block", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("mono_mode", ctypes.c_uint32), ("bs_min_gates", ctypes.c_uint32)]


class sim_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "gates_applied", "updates", "mono_passes", "u2_applied", "u2_skipped", "measures", "host_syncs",
        "peak_nnz", "pruned", "bitslice_passes")] + [("pruned_mass", ctypes.c_double)] + [
        (f, ctypes.c_uint64) for f in ("index_inserts", "index_cas", "index_lookups", "index_probes", "u2_split")]

    def as_dict(self):
        return {f: (float if t is ctypes.c_double else int)(getattr(self, f)) for f, t in self._fields_}


class sim_key(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class sim_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("alg_bytes", ctypes.c_double), ("updates", ctypes.c_double)]


class SimError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {sim_strerror(code)} ({code}): {sim_last_error()}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2105_01533_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, i32, u32, f64, sz = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32,
                                  ctypes.c_double, ctypes.c_size_t)
    sig = {
        "sim_workspace_bytes": (sz, [vp]),
        "sim_create": (i32, [vp, vp, vp, sz, ctypes.POINTER(vp)]),
        "sim_destroy": (i32, [vp]),
        "sim_set_basis": (i32, [vp, sim_key]),
        "sim_import_state": (i32, [vp, vp, vp, u64]),
        "sim_gates_from_ops": (i32, [vp, sz, vp]),
        "sim_commute_ops": (i32, [vp, sz, ctypes.c_uint32, vp, sz, ctypes.POINTER(sz)]),
        "sim_gates_from_pauli": (i32, [vp, sz, ctypes.c_uint32, vp, sz, ctypes.POINTER(sz)]),
        "sim_apply_pauli": (i32, [vp, vp, sz, vp]),
        "sim_apply_gates": (i32, [vp, vp, sz, vp, vp]),
        "sim_apply_gates_static": (i32, [vp, vp, sz, vp, vp]),
        "sim_apply_ops": (i32, [vp, vp, sz, vp, vp]),
        "sim_measure": (i32, [vp, u32, f64, i32, ctypes.POINTER(i32), ctypes.POINTER(f64)]),
        "sim_nnz": (i32, [vp, ctypes.POINTER(u64)]),
        "sim_sync": (i32, [vp]),
        "sim_export_state": (i32, [vp, vp, vp, u64, ctypes.POINTER(u64)]),
        "sim_export_state_soa": (i32, [vp, vp, vp, vp, u64, ctypes.POINTER(u64)]),
        "sim_device_state": (i32, [vp, vp, vp, vp, vp]),
        "sim_set_tuning": (i32, [vp, vp]),
        "sim_device_copy": (i32, [vp, vp, sz, vp]),
        "sim_set_profiling": (i32, [vp, ctypes.c_int]),
        "sim_kernel_stats": (i32, [vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "sim_kernel_stats_reset": (i32, [vp]),
        "sim_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "sim_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


_lib = _load()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, where: str):
    if rc != SIM_OK:
        raise SimError(rc, where)


# --- C names -----------------------------------------------------------------
def sim_strerror(code: int) -> str:
    return _lib.sim_strerror(code).decode()


def sim_last_error() -> str:
    return _lib.sim_last_error().decode()


def sim_workspace_bytes(cfg: sim_config) -> int:
    return int(_lib.sim_workspace_bytes(ctypes.byref(cfg)))


def sim_create(cfg: sim_config, stream: int | None = None, workspace: int | None = None, ws_bytes: int = 0):
    h = ctypes.c_void_p()
    _check(_lib.sim_create(ctypes.byref(cfg), stream, workspace, ws_bytes, ctypes.byref(h)), "sim_create")
    return h


def sim_destroy(h):
    _check(_lib.sim_destroy(h), "sim_destroy")


def sim_set_basis(h, lo: int = 0, hi: int = 0):
    _check(_lib.sim_set_basis(h, sim_key(lo, hi)), "sim_set_basis")


def sim_import_state(h, lo, hi, amp):
    keys = np.empty(len(lo), KEY_DTYPE)
    keys["lo"], keys["hi"] = lo, hi
    amp = np.ascontiguousarray(amp, dtype=np.complex128)
    _check(_lib.sim_import_state(h, _ptr(keys), _ptr(amp), len(keys)), "sim_import_state")


def sim_gates_from_ops(ops: np.ndarray) -> np.ndarray:
    ops = np.ascontiguousarray(ops)
    assert ops.dtype.itemsize == 48
    out = np.zeros(len(ops), GATE_DTYPE)
    _check(_lib.sim_gates_from_ops(_ptr(ops), len(ops), _ptr(out)), "sim_gates_from_ops")
    return out


def sim_commute_ops(ops: np.ndarray, n_qubits: int) -> np.ndarray:
    """Gate commuting (Sec. 3.3): the op records the per-qubit H/Rx/Ry queues
    send on, in order (at most len(ops) of them)."""
    ops = np.ascontiguousarray(ops)
    assert ops.dtype.itemsize == 48
    out = np.zeros(max(len(ops), 1), ops.dtype)
    n = ctypes.c_size_t(0)
    _check(_lib.sim_commute_ops(_ptr(ops), len(ops), n_qubits, _ptr(out), len(out), ctypes.byref(n)),
           "sim_commute_ops")
    return out[:n.value]


def sim_gates_from_pauli(terms: np.ndarray, n_qubits: int) -> np.ndarray:
    """Pauli-exponential records (64 bytes: x, z, ctrl masks, theta, cap) as
    sim_gate ops: one branching op per term with x != 0, a CNOT-gathered
    parity phase for a diagonal term."""
    terms = np.ascontiguousarray(terms)
    assert terms.dtype.itemsize == 64
    n = ctypes.c_size_t(0)
    rc = _lib.sim_gates_from_pauli(_ptr(terms), len(terms), n_qubits, None, 0, ctypes.byref(n))
    if rc not in (SIM_OK, SIM_E_BUFFER):
        _check(rc, "sim_gates_from_pauli")
    out = np.zeros(max(n.value, 1), GATE_DTYPE)
    _check(_lib.sim_gates_from_pauli(_ptr(terms), len(terms), n_qubits, _ptr(out), len(out), ctypes.byref(n)),
           "sim_gates_from_pauli")
    return out[:n.value]


def sim_apply_pauli(h, terms: np.ndarray, raise_on_error: bool = True):
    """Returns (rc, stats dict)."""
    terms = np.ascontiguousarray(terms)
    assert terms.dtype.itemsize == 64
    st = sim_stats()
    rc = _lib.sim_apply_pauli(h, _ptr(terms), len(terms), ctypes.byref(st))
    if raise_on_error:
        _check(rc, "sim_apply_pauli")
    return rc, st.as_dict()


def _n_meas_gates(gates):
    return int(np.count_nonzero(gates["op"] == SIM_OP_MEASURE))


def sim_apply_gates(h, gates: np.ndarray, raise_on_error: bool = True):
    """Returns (rc, outcomes, stats dict)."""
    gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    outcomes = np.full(max(_n_meas_gates(gates), 1), -1, np.int32)
    st = sim_stats()
    rc = _lib.sim_apply_gates(h, _ptr(gates), len(gates), _ptr(outcomes), ctypes.byref(st))
    if raise_on_error:
        _check(rc, "sim_apply_gates")
    return rc, outcomes[:_n_meas_gates(gates)], st.as_dict()


def sim_apply_gates_static(h, gates: np.ndarray, raise_on_error: bool = True):
    """The allocation-free form of sim_apply_gates (at most 65536 ops per
    call).  Returns (rc, outcomes, stats dict)."""
    gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    outcomes = np.full(max(_n_meas_gates(gates), 1), -1, np.int32)
    st = sim_stats()
    rc = _lib.sim_apply_gates_static(h, _ptr(gates), len(gates), _ptr(outcomes), ctypes.byref(st))
    if raise_on_error:
        _check(rc, "sim_apply_gates_static")
    return rc, outcomes[:_n_meas_gates(gates)], st.as_dict()


def sim_apply_ops(h, ops: np.ndarray, raise_on_error: bool = True):
    """Returns (rc, outcomes, stats dict)."""
    ops = np.ascontiguousarray(ops)
    assert ops.dtype.itemsize == 48
    n_meas = int(np.count_nonzero(ops["kind"] == 12))
    outcomes = np.full(max(n_meas, 1), -1, np.int32)
    st = sim_stats()
    rc = _lib.sim_apply_ops(h, _ptr(ops), len(ops), _ptr(outcomes), ctypes.byref(st))
    if raise_on_error:
        _check(rc, "sim_apply_ops")
    return rc, outcomes[:n_meas], st.as_dict()


def sim_measure(h, qubit: int, u: float, forced: int = -1):
    o, p1 = ctypes.c_int32(), ctypes.c_double()
    _check(_lib.sim_measure(h, qubit, u, forced, ctypes.byref(o), ctypes.byref(p1)), "sim_measure")
    return o.value, p1.value


def sim_nnz(h) -> int:
    n = ctypes.c_uint64()
    _check(_lib.sim_nnz(h, ctypes.byref(n)), "sim_nnz")
    return n.value


def sim_sync(h):
    _check(_lib.sim_sync(h), "sim_sync")


def sim_export_state(h, sort: bool = True):
    """(lo, hi, amp) numpy arrays; sorted ascending by (hi, lo) when sort.
    The arrays are written directly by sim_export_state_soa."""
    return sim_export_state_soa(h, sort)


def sim_export_state_soa(h, sort: bool = True):
    """(lo, hi, amp) numpy arrays; sorted ascending by (hi, lo) when sort."""
    n = sim_nnz(h)
    lo, hi = np.empty(n, np.uint64), np.empty(n, np.uint64)
    amp = np.empty(n, np.complex128)
    got = ctypes.c_uint64()
    _check(_lib.sim_export_state_soa(h, _ptr(lo), _ptr(hi), _ptr(amp), n, ctypes.byref(got)), "sim_export_state_soa")
    assert got.value == n
    if sort:
        order = np.lexsort((lo, hi))
        lo, hi, amp = lo[order], hi[order], amp[order]
    return lo, hi, amp


def sim_device_state(h):
    lo, hi, amp, nnz = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    _check(_lib.sim_device_state(h, ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(amp), ctypes.byref(nnz)),
           "sim_device_state")
    return lo.value, hi.value, amp.value, nnz.value


def sim_set_tuning(h, fuse_max: int = 0, block: int = 0, mono_mode: int = 0, bs_min_gates: int = 0,
                   load_factor: float = 0.0, flags: int = 0):
    t = sim_config(fuse_max=fuse_max, block=block, mono_mode=mono_mode, bs_min_gates=bs_min_gates,
                   load_factor=load_factor, flags=flags)
    _check(_lib.sim_set_tuning(h, ctypes.byref(t)), "sim_set_tuning")


def sim_device_copy(dst: int, src: int, nbytes: int, stream: int | None = None):
    _check(_lib.sim_device_copy(dst, src, nbytes, stream), "sim_device_copy")


def sim_set_profiling(h, on):
    """on: False/True (off / every kernel class) or a SIM_PROFILE_* mode."""
    mode = int(on) if not isinstance(on, bool) else (SIM_PROFILE_ALL if on else SIM_PROFILE_OFF)
    _check(_lib.sim_set_profiling(h, mode), "sim_set_profiling")


def sim_kernel_stats(h) -> dict:
    """{class name: {launches, total_ms, alg_bytes, updates}}."""
    arr = (sim_kernel_stat * 32)()
    n = ctypes.c_int()
    _check(_lib.sim_kernel_stats(h, arr, 32, ctypes.byref(n)), "sim_kernel_stats")
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": arr[i].total_ms,
                                   "alg_bytes": arr[i].alg_bytes, "updates": arr[i].updates}
            for i in range(min(n.value, 32))}


def sim_kernel_stats_reset(h):
    _check(_lib.sim_kernel_stats_reset(h), "sim_kernel_stats_reset")


# --- convenience wrapper -----------------------------------------------------
class Simulator:
    """One sparse state on the current torch device and stream.

    Launch knobs left as None take the committed autotuner table's values for
    this state's bucket (autotune.state_knobs), or the library defaults with
    tuned=False or SPARSESIM_TUNING=off; `knobs` records what was used."""

    def __init__(self, n_qubits: int, capacity: int, eps: float = 0.0, fuse_max: int | None = None,
                 load_factor: float | None = None, block: int | None = None, mono_mode: int | None = None,
                 bs_min_gates: int | None = None, flags: int | None = None, device: str = "cuda",
                 tuned: bool = True):
        from . import autotune
        given = {"fuse_max": fuse_max, "load_factor": load_factor, "block": block, "mono_mode": mono_mode,
                 "bs_min_gates": bs_min_gates, "flags": flags}
        if tuned:
            self.knobs = autotune.state_knobs(n_qubits, capacity, given)
        else:
            self.knobs = {k: (v if v is not None else 0) for k, v in given.items()}
        self.cfg = sim_config(n_qubits=n_qubits, capacity=capacity, eps=eps, **self.knobs)
        nbytes = sim_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise SimError(SIM_E_ARG, "sim_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = torch.cuda.current_stream(self.workspace.device)
        self.h = sim_create(self.cfg, self.stream.cuda_stream, self.workspace.data_ptr(), nbytes)

    def close(self):
        if getattr(self, "h", None):
            sim_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_basis(self, lo=0, hi=0):
        sim_set_basis(self.h, lo, hi)

    def import_state(self, lo, hi, amp):
        sim_import_state(self.h, lo, hi, amp)

    def apply_ops(self, ops, raise_on_error=True):
        return sim_apply_ops(self.h, ops, raise_on_error)

    def apply_gates(self, gates, raise_on_error=True):
        return sim_apply_gates(self.h, gates, raise_on_error)

    def apply_pauli(self, terms, raise_on_error=True):
        return sim_apply_pauli(self.h, terms, raise_on_error)

    def measure(self, q, u, forced=-1):
        return sim_measure(self.h, q, u, forced)

    @property
    def nnz(self):
        return sim_nnz(self.h)

    def export(self, sort=True):
        return sim_export_state(self.h, sort)


def run_workload(w, commute: bool = False, **kw):
    """Simulate a workloads.Workload from its basis state; returns (sim,
    outcomes, stats).  commute: pass the ops through the gate-commuting queues
    first (sim_commute_ops)."""
    s = Simulator(w.n_qubits, w.capacity, w.eps, **kw)
    s.set_basis(*w.basis)
    ops = sim_commute_ops(w.ops, w.n_qubits) if commute else w.ops
    _, outcomes, stats = s.apply_ops(ops)
    return s, outcomes, stats


def run_pauli_workload(w, **kw):
    """Simulate a workloads.PauliWorkload (native exp(-i theta P) terms) from
    its basis state; returns (sim, stats)."""
    s = Simulator(w.n_qubits, w.capacity, w.eps, **kw)
    s.set_basis(*w.basis)
    _, stats = s.apply_pauli(w.terms)
    return s, stats


# --- continuous-batching server (srv_*) -----------------------------------------
SRV_QUEUED, SRV_RUNNING, SRV_DONE, SRV_FAILED = 0, 1, 2, 3
SRV_FLAG_NO_GRAPH = 1
SRV_FLAG_U2_GLOBAL_INDEX = 2
SRV_FLAG_NO_RP = 4
SRV_FLAG_ONE_SEGMENT = 8
SRV_LANE_OFF = 0xFFFFFFFF


class srv_config(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("max_slots", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("tick_updates", ctypes.c_uint64),
                ("grid", ctypes.c_uint32), ("lane_capacity", ctypes.c_uint32),
                ("lane_workers", ctypes.c_uint32), ("max_run_ops", ctypes.c_uint32)]


class srv_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in (
        "submitted", "admitted", "completed", "failed", "ticks", "items", "bitslice_runs",
        "pool_used_bytes", "pool_peak_bytes")] + [(f, ctypes.c_double) for f in ("host_ms", "wait_ms", "group_ms")] + [
        ("lane_completed", ctypes.c_uint64), ("lane_ms", ctypes.c_double), ("ahead_hits", ctypes.c_uint64),
        ("ahead_ms", ctypes.c_double), ("copy_ms", ctypes.c_double), ("rp_runs", ctypes.c_uint64),
        ("paired", ctypes.c_uint64), ("chained", ctypes.c_uint64)]

    def as_dict(self):
        return {f: (round(getattr(self, f), 3) if t is ctypes.c_double else int(getattr(self, f)))
                for f, t in self._fields_}


def _srv_sigs():
    vp, u64, i32, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_size_t
    sig = {
        "srv_footprint": (sz, [vp]),
        "srv_create": (i32, [vp, vp, vp, sz, ctypes.POINTER(vp)]),
        "srv_destroy": (i32, [vp]),
        "srv_submit": (i32, [vp, vp, vp, sz, sim_key, ctypes.POINTER(u64)]),
        "srv_tick": (i32, [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]),
        "srv_run": (i32, [vp]),
        "srv_poll": (i32, [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "srv_result": (i32, [vp, u64, vp, vp, u64, ctypes.POINTER(u64), vp, u64, ctypes.POINTER(u64), vp]),
        "srv_result_soa": (i32, [vp, u64, vp, vp, vp, u64, ctypes.POINTER(u64), vp, u64, ctypes.POINTER(u64), vp]),
        "srv_release": (i32, [vp, u64]),
        "srv_get_stats": (i32, [vp, vp]),
        "srv_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(_lib, name)
        f.restype = res
        f.argtypes = args


_srv_sigs()


class ServerError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {sim_strerror(code)} ({code}): {srv_last_error()}")


def _scheck(rc: int, where: str):
    if rc != SIM_OK:
        raise ServerError(rc, where)


def srv_last_error() -> str:
    return _lib.srv_last_error().decode()


def srv_footprint(cfg: sim_config) -> int:
    return int(_lib.srv_footprint(ctypes.byref(cfg)))


def srv_create(cfg: srv_config, stream=None, pool=None, pool_bytes: int = 0):
    h = ctypes.c_void_p()
    _scheck(_lib.srv_create(ctypes.byref(cfg), stream, pool, pool_bytes, ctypes.byref(h)), "srv_create")
    return h


def srv_destroy(h):
    _scheck(_lib.srv_destroy(h), "srv_destroy")


def srv_submit(h, cfg: sim_config, gates: np.ndarray, basis=(0, 0)) -> int:
    gates = np.ascontiguousarray(gates, dtype=GATE_DTYPE)
    rid = ctypes.c_uint64()
    _scheck(_lib.srv_submit(h, ctypes.byref(cfg), _ptr(gates), len(gates), sim_key(*basis), ctypes.byref(rid)),
            "srv_submit")
    return rid.value


def srv_tick(h):
    r, q = ctypes.c_uint32(), ctypes.c_uint32()
    _scheck(_lib.srv_tick(h, ctypes.byref(r), ctypes.byref(q)), "srv_tick")
    return r.value, q.value


def srv_run(h):
    _scheck(_lib.srv_run(h), "srv_run")


def srv_poll(h, rid: int):
    st, err = ctypes.c_int32(), ctypes.c_int32()
    _scheck(_lib.srv_poll(h, rid, ctypes.byref(st), ctypes.byref(err)), "srv_poll")
    return st.value, err.value


def srv_result(h, rid: int, sort: bool = True):
    """(lo, hi, amp, outcomes, stats dict) of a finished request; the arrays
    are written directly by srv_result_soa."""
    return srv_result_soa(h, rid, sort)


def srv_result_soa(h, rid: int, sort: bool = True):
    """(lo, hi, amp, outcomes, stats dict) of a finished request."""
    nnz, nout = ctypes.c_uint64(), ctypes.c_uint64()
    st = sim_stats()
    rc = _lib.srv_result(h, rid, None, None, 0, ctypes.byref(nnz), None, 0, ctypes.byref(nout), ctypes.byref(st))
    if rc not in (SIM_OK, SIM_E_BUFFER):
        raise ServerError(rc, "srv_result")
    n = nnz.value
    lo, hi = np.empty(n, np.uint64), np.empty(n, np.uint64)
    amp = np.empty(n, np.complex128)
    outs = np.empty(max(nout.value, 1), np.int32)
    _scheck(_lib.srv_result_soa(h, rid, _ptr(lo), _ptr(hi), _ptr(amp), n, ctypes.byref(nnz), _ptr(outs), len(outs),
                                ctypes.byref(nout), ctypes.byref(st)), "srv_result_soa")
    if sort:
        order = np.lexsort((lo, hi))
        lo, hi, amp = lo[order], hi[order], amp[order]
    return lo, hi, amp, outs[:nout.value].copy(), st.as_dict()


def srv_release(h, rid: int):
    _scheck(_lib.srv_release(h, rid), "srv_release")


def srv_get_stats(h) -> dict:
    st = srv_stats()
    _scheck(_lib.srv_get_stats(h, ctypes.byref(st)), "srv_get_stats")
    return st.as_dict()


class Server:
    """Continuous-batching server on one device; states live in a pool of
    budget_bytes borrowed from torch."""

    def __init__(self, budget_bytes: int, max_slots: int = 256, arena_bytes: int = 0, graph: bool = True,
                 tick_updates: int | None = None, grid: int | None = None, lane_capacity: int | None = None,
                 lane_workers: int | None = None, device: str = "cuda", tuned: bool = True, flags: int = 0,
                 max_run_ops: int | None = None):
        """Server knobs left as None take the autotuner table's values (the
        library defaults with tuned=False); `knobs` records what was used.
        submit_workload applies the table's per-state knobs the same way."""
        from . import autotune
        given = {"tick_updates": tick_updates, "grid": grid, "lane_capacity": lane_capacity,
                 "lane_workers": lane_workers, "max_run_ops": max_run_ops}
        self.tuned = tuned
        self.knobs = autotune.server_knobs(given) if tuned else {k: (v or 0) for k, v in given.items()}
        self.cfg = srv_config(budget_bytes=budget_bytes, arena_bytes=arena_bytes, max_slots=max_slots,
                              flags=flags | (0 if graph else SRV_FLAG_NO_GRAPH), **self.knobs)
        self.pool = torch.empty(budget_bytes, dtype=torch.uint8, device=device)
        self.h = srv_create(self.cfg, None, self.pool.data_ptr(), budget_bytes)

    def close(self):
        if getattr(self, "h", None):
            srv_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit_workload(self, w, **tuning) -> int:
        from . import autotune
        knobs = autotune.state_knobs(w.n_qubits, w.capacity, tuning) if self.tuned else tuning
        cfg = sim_config(n_qubits=w.n_qubits, capacity=w.capacity, eps=w.eps, **knobs)
        return srv_submit(self.h, cfg, sim_gates_from_ops(w.ops), w.basis)

    def submit(self, cfg: sim_config, gates: np.ndarray, basis=(0, 0)) -> int:
        return srv_submit(self.h, cfg, gates, basis)

    def tick(self):
        return srv_tick(self.h)

    def run(self):
        srv_run(self.h)

    def poll(self, rid):
        return srv_poll(self.h, rid)

    def result(self, rid, sort=True):
        return srv_result(self.h, rid, sort)

    def release(self, rid):
        srv_release(self.h, rid)

    def stats(self):
        return srv_get_stats(self.h)
