"""Gate matrices (complex128) of the synthetic random circuits.

The paper simulates Sycamore random circuits (Results) without listing the
gates; these are the standard Sycamore choices:

* sqrt(P) = ((1+i)/2) I + ((1-i)/2) P for P in {X, Y, W}, W = (X+Y)/sqrt(2);
* fsim(theta, phi) on |q1 q2> (q1 the more significant) =
  [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,exp(-i phi)]];
* u3(a, b, c) = Rz(a) Ry(b) Rz(c) with Rz(x) = diag(e^{-ix/2}, e^{ix/2}) and
  Ry(x) = [[cos x/2, -sin x/2], [sin x/2, cos x/2]]; Rz(c) acts first.

Matrices are indexed [out][in].
"""
import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
W = (X + Y) / np.sqrt(2.0)


def sqrt_pauli(p: np.ndarray) -> np.ndarray:
    return 0.5 * (1 + 1j) * I2 + 0.5 * (1 - 1j) * p


def rz(x: float) -> np.ndarray:
    return np.diag([np.exp(-0.5j * x), np.exp(0.5j * x)]).astype(np.complex128)


def ry(x: float) -> np.ndarray:
    c, s = np.cos(0.5 * x), np.sin(0.5 * x)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def u3(a: float, b: float, c: float) -> np.ndarray:
    return rz(a) @ ry(b) @ rz(c)


def fsim(theta: float, phi: float) -> np.ndarray:
    c, s = np.cos(theta), np.sin(theta)
    m = np.zeros((4, 4), dtype=np.complex128)
    m[0, 0] = 1
    m[1, 1] = c
    m[1, 2] = -1j * s
    m[2, 1] = -1j * s
    m[2, 2] = c
    m[3, 3] = np.exp(-1j * phi)
    return m


def gate_matrix(gate) -> np.ndarray:
    """Matrix of a ``workload.Gate``; 'matrix' gates carry their own."""
    name = gate.name
    if name == "sqrt_x":
        return sqrt_pauli(X)
    if name == "sqrt_y":
        return sqrt_pauli(Y)
    if name == "sqrt_w":
        return sqrt_pauli(W)
    if name == "fsim":
        return fsim(*gate.params)
    if name == "u3":
        return u3(*gate.params)
    if name == "matrix":
        k = len(gate.qubits)
        return np.asarray(gate.params, dtype=np.complex128).reshape(2 ** k, 2 ** k)
    raise ValueError(f"unknown gate {name!r}")
