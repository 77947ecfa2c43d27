"""Gradient references for the u3 angles (complex128 / float64).

The paper computes no gradients; these are plain definitions used to check
the library's adjoint contraction:

* loss L = sum_b log|psi_b|^2 over the requested bitstrings;
* PyTorch's convention for a complex output: the incoming gradient is
  g = dL/dRe psi + i dL/dIm psi, here g_b = 2 psi_b / |psi_b|^2, and
  dL/dtheta = Re sum_b conj(g_b) dpsi_b/dtheta;
* ``sv_adjoint``: state-vector adjoint sweep (forward state, then the
  backward state |lambda> = sum_b g_b |b> pulled back gate by gate);
* ``parameter_shift``: for a rotation R(x) = exp(-i x P / 2),
  dR/dx = R(x + pi)/2 exactly, so dpsi/dx = psi(x + pi)/2;
* ``finite_difference``: central differences of L with step h.
"""
import numpy as np

from . import statevector as sv
from .gates import rz, ry, gate_matrix


def _u3_parts(a, b, c):
    """U3 and its three partial derivatives."""
    drz = lambda x: np.diag([-0.5j * np.exp(-0.5j * x), 0.5j * np.exp(0.5j * x)])
    dry = lambda x: 0.5 * np.array([[-np.sin(0.5 * x), -np.cos(0.5 * x)],
                                    [np.cos(0.5 * x), -np.sin(0.5 * x)]], dtype=np.complex128)
    U = rz(a) @ ry(b) @ rz(c)
    return U, (drz(a) @ ry(b) @ rz(c), rz(a) @ dry(b) @ rz(c), rz(a) @ ry(b) @ drz(c))


def loss(circuit, bitstrings, gates=None) -> float:
    amp = sv.bitstring_amplitudes(circuit, bitstrings, gates)
    return float(np.sum(np.log(np.abs(amp) ** 2)))


def incoming_gradient(amp: np.ndarray) -> np.ndarray:
    """g_b = dL/dRe psi_b + i dL/dIm psi_b for L = sum log|psi_b|^2."""
    return 2.0 * amp / np.abs(amp) ** 2


def sv_adjoint(circuit, bitstrings):
    """(L, dL/dangles) with angles laid out [u3 gate][a, b, c]."""
    n = circuit.n_qubits
    gates = circuit.gates
    phi = sv.final_state(circuit).reshape([2] * n)
    flat = phi.reshape(-1)
    bs = np.asarray(bitstrings, dtype=np.int64)
    amp = flat[bs]
    g = incoming_gradient(amp)
    lam = np.zeros(2 ** n, dtype=np.complex128)
    np.add.at(lam, bs, g)
    lam = lam.reshape([2] * n)
    n_u3 = sum(1 for x in gates if x.name == "u3")
    grad = np.zeros((n_u3, 3), dtype=np.float64)
    for gate in reversed(gates):
        U = gate_matrix(gate)
        Ud = U.conj().T
        phi = sv.apply_gate(phi, Ud, gate.qubits)      # state before the gate
        if gate.name == "u3":
            _, dU = _u3_parts(*gate.params)
            for j in range(3):
                v = sv.apply_gate(phi, dU[j], gate.qubits)
                grad[gate.param_id, j] = np.real(np.vdot(lam, v))
        lam = sv.apply_gate(lam, Ud, gate.qubits)
    return float(np.sum(np.log(np.abs(amp) ** 2))), grad.reshape(-1)


def _with_angle(circuit, k, delta):
    """Gate list with angle k (flat [gate][a, b, c] numbering) shifted."""
    from dataclasses import replace
    gid, j = divmod(k, 3)
    out = []
    for gate in circuit.gates:
        if gate.name == "u3" and gate.param_id == gid:
            p = list(gate.params)
            p[j] += delta
            gate = replace(gate, params=tuple(p))
        out.append(gate)
    return out


def parameter_shift(circuit, bitstrings, which):
    """dL/dangle_k for k in ``which`` via dpsi/dx = psi(x + pi) / 2."""
    amp = sv.bitstring_amplitudes(circuit, bitstrings)
    g = incoming_gradient(amp)
    out = []
    for k in which:
        dpsi = 0.5 * sv.bitstring_amplitudes(circuit, bitstrings, _with_angle(circuit, k, np.pi))
        out.append(float(np.real(np.sum(np.conj(g) * dpsi))))
    return np.asarray(out)


def finite_difference(circuit, bitstrings, which, h=1e-3):
    out = []
    for k in which:
        lp = loss(circuit, bitstrings, _with_angle(circuit, k, h))
        lm = loss(circuit, bitstrings, _with_angle(circuit, k, -h))
        out.append((lp - lm) / (2 * h))
    return np.asarray(out)
