"""Write oracle references of the 20-qubit gradient workload.

Calls only the oracle and the seeded workload generator: amplitudes of the
256 bitstrings (state vector, complex128), the loss sum_b log|psi_b|^2, its
gradient over all 720 u3 angles by the state-vector adjoint, and on a
seeded subset of 48 angles the exact parameter shift and central finite
differences (h = 1e-3). Output: rqc20_grad_reference.npz.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import gradients as gr  # noqa: E402
from oracle import statevector as sv  # noqa: E402
from workload import make_workload  # noqa: E402


def main():
    w = make_workload("rqc20_grad")
    c, bs = w.circuit, w.bitstrings
    t0 = time.time()
    amp = sv.bitstring_amplitudes(c, bs)
    loss, grad = gr.sv_adjoint(c, bs)
    print(f"adjoint {time.time() - t0:.1f}s", flush=True)
    subset = np.sort(np.random.default_rng(4).choice(len(grad), 48, replace=False))
    ps = gr.parameter_shift(c, bs, subset)
    print(f"shift {time.time() - t0:.1f}s", flush=True)
    fd = gr.finite_difference(c, bs, subset, h=1e-3)
    print(f"fd {time.time() - t0:.1f}s", flush=True)
    np.savez(os.path.join(HERE, "rqc20_grad_reference.npz"), bitstrings=bs, amplitudes=amp,
             loss=loss, grad=grad, subset=subset, param_shift=ps, finite_diff=fd)
    print("max |adjoint - shift| on subset:", np.max(np.abs(grad[subset] - ps)))


if __name__ == "__main__":
    main()
