"""Pins of the oracle's amplitudes: two independent codes (state vector and
tensor-network contraction) agree, the state is normalised, a mirror circuit
returns a delta, and summing all slices reproduces the unsliced contraction
(Sec. 2.1.1: slicing yields 2^|S| subtasks whose results are accumulated)."""
import numpy as np
import pytest

from oracle import network as nw
from oracle import planner as pl
from oracle import statevector as sv
from oracle.gates import gate_matrix
from workload import Gate, make_rqc, make_workload


def _tn_amp(circuit, open_q, closed, absorb=True):
    net = nw.circuit_network(circuit, open_q, closed)
    if absorb:
        net = nw.absorb_small(net)
    path = pl.greedy_path(net.indices)
    return nw.contract_path(net, path)


@pytest.mark.parametrize("absorb", [False, True])
def test_sv_equals_tn_rqc12(absorb):
    w = make_workload("rqc12")
    a_sv = sv.amplitudes(w.circuit, w.open_qubits, w.closed_bits)
    a_tn = _tn_amp(w.circuit, w.open_qubits, w.closed_bits, absorb)
    assert np.linalg.norm(a_sv - a_tn) / np.linalg.norm(a_sv) < 1e-12


@pytest.mark.parametrize("rows,cols,cycles,n_open", [(3, 3, 6, 3), (2, 4, 10, 4), (3, 4, 5, 12)])
def test_sv_equals_tn_open(rows, cols, cycles, n_open):
    c = make_rqc(rows, cols, cycles, seed=5)
    n = c.n_qubits
    open_q = tuple(range(n - n_open, n))
    closed = {q: (q * 7 + 1) % 2 for q in range(n - n_open)}
    a_sv = sv.amplitudes(c, open_q, closed)
    a_tn = _tn_amp(c, open_q, closed)
    assert np.linalg.norm(a_sv - a_tn) / np.linalg.norm(a_sv) < 1e-12


def test_normalisation_all_open():
    c = make_rqc(3, 4, 8, seed=0)
    psi = _tn_amp(c, tuple(range(12)), {})
    assert abs(np.sum(np.abs(psi) ** 2) - 1) < 1e-12
    # Porter-Thomas: 2^n |psi|^2 has mean 1 exactly (normalisation) and
    # second moment near 2 for a random circuit
    p = (2 ** 12) * np.abs(psi) ** 2
    assert 1.5 < np.mean(p ** 2) < 2.5


def test_mirror_circuit_gives_delta():
    c = make_rqc(3, 3, 6, seed=9)
    inv = [Gate("matrix", g.qubits, tuple(gate_matrix(g).conj().T.reshape(-1)))
           for g in reversed(c.gates)]
    c.gates = list(c.gates) + inv
    psi = _tn_amp(c, tuple(range(9)), {})
    expect = np.zeros(2 ** 9)
    expect[0] = 1
    np.testing.assert_allclose(psi, expect, atol=1e-12)


def test_identity_circuit_gives_delta():
    c = make_rqc(2, 3, 3, seed=1)
    c.gates = [Gate("matrix", g.qubits, tuple(np.eye(2 ** len(g.qubits)).reshape(-1)))
               for g in c.gates]
    psi = _tn_amp(c, tuple(range(6)), {}, absorb=False)
    expect = np.zeros(64)
    expect[0] = 1
    np.testing.assert_allclose(psi, expect, atol=1e-15)


@pytest.mark.parametrize("open_sliced", [False, True])
def test_sum_over_slices_equals_unsliced(open_sliced):
    c = make_rqc(3, 3, 5, seed=2)
    open_q = (6, 7, 8)
    closed = {q: q % 2 for q in range(6)}
    net = nw.absorb_small(nw.circuit_network(c, open_q, closed))
    path = pl.greedy_path(net.indices)
    full = nw.contract_path(net, path)
    tree = pl.Tree(net.indices, path)
    rng = np.random.default_rng(0)
    closed_ids = sorted(set(range(net.n_indices)) - set(net.open_ids))
    S = [int(x) for x in rng.choice(closed_ids, size=4, replace=False)]
    if open_sliced:
        S.append(net.open_ids[1])
    out = nw.sliced_sum(net, path, S)
    np.testing.assert_allclose(out, full, atol=1e-13)
    # the slice finder's set gives the same result too
    S2 = pl.slice_finder(tree, 4)
    assert tree.space(S2) <= 2 ** 4
    np.testing.assert_allclose(nw.sliced_sum(net, path, S2), full, atol=1e-13)


def test_absorbed_network_conservation():
    """Lemma 1 (Conservation): every closed index lies in exactly two
    tensors, every open index in one."""
    for name in ("rqc12", "rqc30", "rqc20_grad"):
        w = make_workload(name)
        net = nw.absorb_small(nw.circuit_network(w.circuit, w.open_qubits, w.closed_bits))
        count = np.zeros(net.n_indices, dtype=int)
        for ix in net.indices:
            assert len(set(ix)) == len(ix)
            for x in ix:
                count[x] += 1
        opened = np.zeros(net.n_indices, dtype=bool)
        opened[net.open_ids] = True
        assert np.all(count[opened] == 1)
        assert np.all(count[~opened] == 2)
