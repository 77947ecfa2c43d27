"""CPU oracle for the sliced tensor-network contraction (test infrastructure).

Plain, slow, obviously correct reference implementations, in complex128 /
float64, written from the paper (Chen et al., "Lifetime-based Optimization
for Simulating Quantum Circuits on a New Sunway Supercomputer", PPoPP'23):

* ``gates``        -- gate matrices of the synthetic circuits;
* ``statevector``  -- brute-force state-vector amplitudes (<= ~24 qubits);
* ``network``      -- circuit -> tensor network (Sec. 2.1.1 notation),
                      rank-1/2 absorption (Sec. 2.1.2), pairwise contraction
                      along a path, slicing by fixing edges (Sec. 2.1.1);
* ``planner``      -- greedy path, contraction tree, Eq. (1), Eq. (2),
                      Eq. (4), stem, lifetimes (Sec. 3.1 Definition) and the
                      slice finder (Algorithm 1);
* ``gradients``    -- state-vector adjoint, exact parameter shift and
                      central finite differences for u3 angles.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU library and never calls
it.
"""
