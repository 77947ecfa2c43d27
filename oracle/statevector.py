"""Brute-force state-vector simulation (complex128).

psi(x) = <x| C |0...0> with C the product of the circuit's gates in order.
The state is held as an n-axis array of shape [2]*n, axis q = qubit q, so the
flat index is x = sum_q b_q 2^(n-1-q) (qubit 0 is the most significant bit).
This is the plain definition of what every contraction in the paper computes
(Introduction: amplitudes of the output state).
"""
import numpy as np

from .gates import gate_matrix


def apply_gate(state: np.ndarray, mat: np.ndarray, qubits) -> np.ndarray:
    """Apply a k-qubit matrix [out][in] to the listed axes of ``state``."""
    k = len(qubits)
    n = state.ndim
    g = mat.reshape([2] * (2 * k))
    # contract the gate's input axes (k..2k-1) with the state's qubit axes
    out = np.tensordot(g, state, axes=(list(range(k, 2 * k)), list(qubits)))
    # tensordot puts the gate's output axes first; move them back in place
    rest = [a for a in range(n) if a not in qubits]
    order = list(qubits) + rest
    inv = np.argsort(order)
    return np.transpose(out, inv)


def final_state(circuit, gates=None) -> np.ndarray:
    """Full output state as a flat complex128 vector of length 2^n."""
    n = circuit.n_qubits
    state = np.zeros([2] * n, dtype=np.complex128)
    state[(0,) * n] = 1.0
    for g in (circuit.gates if gates is None else gates):
        state = apply_gate(state, gate_matrix(g), g.qubits)
    return state.reshape(-1)


def amplitudes(circuit, open_qubits, closed_bits, gates=None) -> np.ndarray:
    """Vector over the open qubits (first open qubit most significant) with
    every closed qubit fixed to its bit."""
    n = circuit.n_qubits
    psi = final_state(circuit, gates).reshape([2] * n)
    idx = []
    for q in range(n):
        idx.append(slice(None) if q in set(open_qubits) else closed_bits[q])
    sub = psi[tuple(idx)]
    # remaining axes are the open qubits in ascending order
    return np.ascontiguousarray(sub).reshape(-1)


def bitstring_amplitudes(circuit, bitstrings, gates=None) -> np.ndarray:
    """psi(x) for each integer x (qubit 0 most significant)."""
    psi = final_state(circuit, gates)
    return psi[np.asarray(bitstrings, dtype=np.int64)]
