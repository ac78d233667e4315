"""GPU: sim_apply_gates_static, the allocation-free form of sim_apply_gates,
through the C-ABI.  On two handles in the same state it must give bitwise the
same state, outcomes and counters as sim_apply_gates, on two calls in a row
(the second smaller, so the static array keeps the first call's contents);
it must reject lists longer than its limit without touching the state, and a
call must not take device memory."""
import numpy as np
import pytest

from paper_2105_01533_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    from paper_2105_01533_amd import sim
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return sim


def _same(S, A, B, gates, what):
    _, oa, sa = S.sim_apply_gates(A.h, gates)
    _, ob, sb = S.sim_apply_gates_static(B.h, gates)
    ma, mb = sa.pop("pruned_mass"), sb.pop("pruned_mass")
    # CAS attempts and probe lengths depend on the order threads insert in
    for k, base in (("index_cas", "index_inserts"), ("index_probes", "index_lookups")):
        assert sa.pop(k) >= sa[base] and sb.pop(k) >= sb[base], what
    assert list(oa) == list(ob), what
    assert sa == sb, (what, sa, sb)
    assert abs(ma - mb) <= 1e-12 * max(1.0, ma), what
    ga, gb = A.export(), B.export()
    for x, y in zip(ga, gb):
        assert x.tobytes() == y.tobytes(), what
    return sa


@pytest.mark.parametrize("nq", [24, 100])
def test_static_matches_allocating(S, nq):
    if nq == 24:
        big = W.config0(41, n=24, h_qubits=10, gates=6000, cap=1 << 16)
        small = W.config0(42, n=24, h_qubits=5, gates=700, cap=1 << 12)
    else:
        big = W.random_circuit(43, n=100, gates=3000, h_frac=0.05, ctrl_max=3, measure_frac=0.01, cap=1 << 15)
        small = W.random_circuit(44, n=100, gates=500, h_frac=0.05, ctrl_max=2, measure_frac=0.02, cap=1 << 15)
    cap = 1 << 16
    A = S.Simulator(nq, cap, 1e-20)
    B = S.Simulator(nq, cap, 1e-20)
    for k, w in enumerate((big, small)):
        A.set_basis(*w.basis)
        B.set_basis(*w.basis)
        st = _same(S, A, B, S.sim_gates_from_ops(w.ops), f"{w.name} call {k}")
        if k == 0:
            assert st["bitslice_passes"] > 0 and st["u2_applied"] > 0
    A.close()
    B.close()


def test_static_limit_and_memory(S):
    import torch
    w = W.config0(45, n=20, h_qubits=8, gates=60000, cap=1 << 14, measured=4)
    gates = S.sim_gates_from_ops(w.ops)
    assert len(gates) <= 65536
    B = S.Simulator(20, 1 << 14, 1e-20)
    B.set_basis(*w.basis)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    _, _, st = S.sim_apply_gates_static(B.h, gates)
    free1 = torch.cuda.mem_get_info()[0]
    assert st["gates_applied"] == len(gates)
    assert free0 - free1 < (1 << 20), (free0, free1)
    before = B.export()
    too_many = np.concatenate([gates, gates[:65536 - len(gates) + 1]])
    rc, _, _ = S.sim_apply_gates_static(B.h, too_many, raise_on_error=False)
    assert rc == S.SIM_E_ARG
    after = B.export()
    for x, y in zip(before, after):
        assert x.tobytes() == y.tobytes()
    B.close()
