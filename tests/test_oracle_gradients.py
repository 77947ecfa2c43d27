"""Pins of the oracle's gradient references: the state-vector adjoint
agrees with the exact parameter-shift rule and with central differences."""
import numpy as np

from oracle import gradients as gr
from oracle.gates import u3
from workload import make_rqc, sample_bitstrings


def test_u3_derivatives_match_matrix_differences():
    a, b, c = 0.7, 1.9, 4.1
    _, dU = gr._u3_parts(a, b, c)
    h = 1e-6
    num = [(u3(a + h, b, c) - u3(a - h, b, c)) / (2 * h),
           (u3(a, b + h, c) - u3(a, b - h, c)) / (2 * h),
           (u3(a, b, c + h) - u3(a, b, c - h)) / (2 * h)]
    for x, y in zip(dU, num):
        np.testing.assert_allclose(x, y, atol=1e-9)


def test_adjoint_equals_parameter_shift():
    c = make_rqc(2, 3, 4, u3_seed=2)
    bs = sample_bitstrings(6, 8, 1)
    L, g = gr.sv_adjoint(c, bs)
    assert abs(L - gr.loss(c, bs)) < 1e-12
    which = list(range(len(g)))
    ps = gr.parameter_shift(c, bs, which)
    assert np.max(np.abs(g - ps)) < 1e-10 * max(1.0, np.max(np.abs(g)))


def test_adjoint_matches_finite_differences():
    c = make_rqc(3, 3, 3, u3_seed=4)
    bs = sample_bitstrings(9, 16, 1)
    _, g = gr.sv_adjoint(c, bs)
    which = list(range(0, len(g), 7))
    fd = gr.finite_difference(c, bs, which, h=1e-3)
    assert np.linalg.norm(fd - g[which]) / np.linalg.norm(g[which]) < 1e-5
