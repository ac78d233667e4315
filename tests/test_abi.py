"""CPU checks of the C-ABI library: it is built, loads, and exports every
function include/sparsesim.h declares; host-only entry points (gate
conversion, workspace sizing, config validation) behave as documented.  No
call here touches a GPU."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sparsesim.h")
LIB = os.path.join(ROOT, "paper_2105_01533_amd", "libsparsesim.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z_]+)\s*\(", text)))


def test_library_built():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"


def test_every_declared_symbol_exported():
    names = declared_functions()
    assert "sim_apply_gates" in names and "sim_create" in names
    out = subprocess.check_output(["nm", "-D", "--defined-only", LIB], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_binding_loads_and_names_match():
    from paper_2105_01533_amd import sim
    for n in declared_functions():
        assert hasattr(sim, n), n
        assert hasattr(sim._lib, n), n


def test_gate_conversion_matches_definitions():
    from paper_2105_01533_amd import sim, workloads as W
    c = W.Circuit()
    c.h(3)
    c.gate(W.K_RZ, 1, (0,), param=0.8)
    c.gate(W.K_Y, 2)
    c.gate(W.K_RY, 0, (), param=-1.1)
    c.gate(W.K_T, 5, (70,))
    c.measure(4, 0.25)
    g = sim.sim_gates_from_ops(c.array())
    s = math.sqrt(0.5)
    assert g["op"].tolist() == [sim.SIM_OP_U2, sim.SIM_OP_MONO, sim.SIM_OP_MONO, sim.SIM_OP_U2, sim.SIM_OP_MONO,
                                sim.SIM_OP_MEASURE]
    assert np.array_equal(g[0]["m"], np.array([s, s, s, -s]))
    assert g[1]["ctrl_lo"] == 1 and g[1]["flip"] == 0
    assert abs(g[1]["m"][0] - np.exp(-0.4j)) < 1e-16 and abs(g[1]["m"][1] - np.exp(0.4j)) < 1e-16
    assert g[2]["flip"] == 1 and g[2]["m"][0] == 1j and g[2]["m"][1] == -1j
    U = g[3]["m"].reshape(2, 2)
    assert np.allclose(U, [[math.cos(-0.55), -math.sin(-0.55)], [math.sin(-0.55), math.cos(-0.55)]], atol=1e-16)
    assert g[4]["ctrl_hi"] == 1 << 6 and g[4]["m"][1] == complex(s, s)
    assert g[5]["u"] == 0.25 and g[5]["forced"] == -1


def test_unknown_kind_rejected():
    from paper_2105_01533_amd import sim, workloads as W
    ops = W.Circuit()
    ops.gate(99, 0)
    with pytest.raises(sim.SimError) as e:
        sim.sim_gates_from_ops(ops.array())
    assert e.value.code == sim.SIM_E_ARG


def test_workspace_bytes_and_config_validation():
    from paper_2105_01533_amd import sim
    cfg = sim.sim_config(n_qubits=100, capacity=1 << 20, eps=0.0, load_factor=0.5, block=256)
    nb = sim.sim_workspace_bytes(cfg)
    # two buffers of 32 B/entry (128-bit labels) + 2^22 index slots + 4 B/entry partner scratch
    assert nb >= 2 * 32 * (1 << 20) + 8 * (1 << 22) + 4 * (1 << 20)
    narrow = sim.sim_config(n_qubits=40, capacity=1 << 20)
    assert sim.sim_workspace_bytes(narrow) < nb            # no high label words below 65 qubits
    two_pass = sim.sim_config(n_qubits=100, capacity=1 << 20, eps=0.0, load_factor=0.5, block=256,
                              flags=sim.SIM_FLAG_U2_TWO_PASS)
    assert sim.sim_workspace_bytes(two_pass) == nb         # a known flag; same layout
    lds = sim.sim_config(n_qubits=100, capacity=1 << 20, eps=0.0, load_factor=0.5, block=256,
                         flags=sim.SIM_FLAG_BS_LDS)
    assert sim.sim_workspace_bytes(lds) == nb
    glob = sim.sim_config(n_qubits=100, capacity=1 << 20, eps=0.0, load_factor=0.5, block=256,
                          flags=sim.SIM_FLAG_U2_GLOBAL_INDEX)
    assert sim.sim_workspace_bytes(glob) == nb
    for bad in [sim.sim_config(n_qubits=0, capacity=10), sim.sim_config(n_qubits=129, capacity=10),
                sim.sim_config(n_qubits=10, capacity=0), sim.sim_config(n_qubits=10, capacity=1 << 31),
                sim.sim_config(n_qubits=10, capacity=10, load_factor=0.95),
                sim.sim_config(n_qubits=10, capacity=10, block=96),
                sim.sim_config(n_qubits=10, capacity=10, flags=32)]:
        assert sim.sim_workspace_bytes(bad) == 0
        with pytest.raises(sim.SimError) as e:
            sim.sim_create(bad)
        assert e.value.code == sim.SIM_E_ARG
