"""Pins of the oracle's gate definitions and bit order (algebra, closed forms)."""
import numpy as np
import pytest

from oracle import gates as G
from oracle import statevector as sv
from workload import Circuit, Gate


def test_sqrt_gates_square_to_paulis():
    for p in (G.X, G.Y, G.W):
        s = G.sqrt_pauli(p)
        np.testing.assert_allclose(s @ s, p, atol=1e-15)
        np.testing.assert_allclose(s.conj().T @ s, np.eye(2), atol=1e-15)


def test_fsim_entries_and_unitarity():
    f = G.fsim(np.pi / 2, np.pi / 6)
    np.testing.assert_allclose(f.conj().T @ f, np.eye(4), atol=1e-15)
    assert f[0, 0] == 1
    np.testing.assert_allclose(f[1, 2], -1j, atol=1e-15)   # |01> -> -i|10>
    np.testing.assert_allclose(f[2, 1], -1j, atol=1e-15)
    np.testing.assert_allclose(f[1, 1], 0, atol=1e-15)
    np.testing.assert_allclose(f[3, 3], np.exp(-1j * np.pi / 6), atol=1e-15)


def test_u3_composition():
    np.testing.assert_allclose(G.u3(0, 0, 0), np.eye(2), atol=1e-15)
    # Rz(a) Rz(c) at b = 0 is Rz(a + c)
    np.testing.assert_allclose(G.u3(0.3, 0.0, 0.4), G.rz(0.7), atol=1e-15)
    # Ry(pi)|0> = |1>
    np.testing.assert_allclose(G.u3(0, np.pi, 0) @ [1, 0], [0, 1], atol=1e-15)
    u = G.u3(1.1, 2.2, 3.3)
    np.testing.assert_allclose(u.conj().T @ u, np.eye(2), atol=1e-15)


def _circ(n, gates):
    return Circuit(1, n, 0, n, (), "", gates)


def test_single_qubit_closed_form():
    a = sv.final_state(_circ(1, [Gate("sqrt_x", (0,))]))
    np.testing.assert_allclose(a, [(1 + 1j) / 2, (1 - 1j) / 2], atol=1e-15)


def test_qubit_zero_is_most_significant():
    # X on qubit 0 of two qubits -> |10> -> flat index 2
    x = [Gate("sqrt_x", (0,)), Gate("sqrt_x", (0,))]
    psi = sv.final_state(_circ(2, x))
    np.testing.assert_allclose(np.abs(psi), [0, 0, 1, 0], atol=1e-15)


def test_fsim_swaps_excitation_with_phase():
    # |01> (qubit 1 excited) --fsim(pi/2, .)--> -i |10>
    g = [Gate("sqrt_x", (1,)), Gate("sqrt_x", (1,)), Gate("fsim", (0, 1), (np.pi / 2, np.pi / 6))]
    psi = sv.final_state(_circ(2, g))
    # X = sqrt_x^2 carries no extra phase: sqrt_x^2 = X exactly
    np.testing.assert_allclose(psi, [0, 0, -1j, 0], atol=1e-15)
