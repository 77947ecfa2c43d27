"""Split-precision GEMM against its analytic error bound.

A two-leaf network whose only step is one complex GEMM C = A B (m row bits,
k contracted bits, n column bits) runs in each split mode with every split
tile configuration that fits, in both operand roles, forced through
ltn_set_step_kernel. The exact product of the complex64 inputs (complex128)
is the reference.

Bound (elementwise, R_ij = sum_k |a_ik| |b_kj|). With p significand bits
(fp16 11, bf16 8) and u = 2^-p, each real component x of an operand is held
as hi + u lo (fp16: after an exact power-of-two scale) with
|x - hi - u lo| <= u^2 |x|. The kernel sums hi*hi, hi*lo and lo*hi in FP32
and drops lo*lo (<= u^2 (1 + u)^2 |a| |b|). Products of fp16/bf16 values are
exact in FP32; the sum of the 3 x 2K real terms per output component adds at
most 6K 2^-23 of their absolute sum (2^-23 rather than 2^-24, so as not to
assume round-to-nearest inside the matrix core), and the FP32 result one
more rounding. Hence

    |c_ij - (AB)_ij| <= (3.1 u^2 + 1.5 * 6K * 2^-23 + 2^-23) R_ij + F_ij,

where F_ij = 2^-34 (max|A| sum_k |b_kj| + max|B| sum_k |a_ik|) covers fp16
values below the normal range after scaling (subnormal hi and lo).

The bound alone would not see a dropped cross term at larger K, so each case
also requires the relative Frobenius error to be at most 1/16 of that of the
product of the operands rounded once to the half format (hi only), which a
missing hi*lo or lo*hi term would not meet."""
import numpy as np
import pytest

from tests.gpu_util import banner

pytestmark = pytest.mark.gpu

P_BITS = {"split_f16": 11, "split_bf16": 8}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _operands(m, k, n, seed, wide):
    rng = np.random.default_rng(seed)
    M, K, N = 1 << m, 1 << k, 1 << n
    a = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K)))
    b = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N)))
    if wide:
        # amplitudes of deep circuits are tiny and rows differ in magnitude
        a *= 2.0 ** -rng.integers(0, 17, size=(M, 1)) * 2.0 ** -30
        b *= 2.0 ** -rng.integers(0, 5, size=(1, N)) * 2.0 ** -4
    return a.astype(np.complex64), b.astype(np.complex64)


def _half_only_error(torch, a, b, mode):
    """Relative Frobenius error of the product of the operands rounded once
    to the half format (after a power-of-two scale), in float64."""
    dt = torch.float16 if mode == "split_f16" else torch.bfloat16

    def rnd(x):
        s = 2.0 ** -np.floor(np.log2(np.abs(np.stack([x.real, x.imag])).max()))
        re = torch.from_numpy((x.real * s).astype(np.float32)).to(dt).double().numpy() / s
        im = torch.from_numpy((x.imag * s).astype(np.float32)).to(dt).double().numpy() / s
        return re + 1j * im

    exact = a.astype(np.complex128) @ b.astype(np.complex128)
    approx = rnd(a) @ rnd(b)
    return float(np.linalg.norm(approx - exact) / np.linalg.norm(exact))


@pytest.mark.parametrize("wide", [False, True], ids=["normal", "wide_range"])
@pytest.mark.parametrize("k", [4, 6, 8])
@pytest.mark.parametrize("mode", ["split_f16", "split_bf16"])
def test_split_gemm_within_analytic_bound(torch, mode, k, wide):
    import paper_2205_00393_amd as P
    m, n = 8, 7
    a, b = _operands(m, k, n, seed=100 + k, wide=wide)
    mi = list(range(m))
    ki = list(range(m, m + k))
    ni = list(range(m + k, m + k + n))
    net = P.Network.from_arrays([mi + ki, ki + ni], [a, b], mi + ni, m + k + n)
    plan = P.Plan(net, [(0, 1)], [])
    plan.bind(batch=1, budget_bytes=1 << 28)
    steps = plan.steps()
    assert len(steps) == 1

    exact = a.astype(np.complex128) @ b.astype(np.complex128)
    absa, absb = np.abs(a).astype(np.float64), np.abs(b).astype(np.float64)
    R = absa @ absb
    F = 2.0 ** -34 * (absa.max() * absb.sum(axis=0)[None, :] + absb.max() * absa.sum(axis=1)[:, None])
    u = 2.0 ** -P_BITS[mode]
    K = 1 << k
    bound = (3.1 * u * u + 1.5 * 6 * K * 2.0 ** -23 + 2.0 ** -23) * R + F
    e_half = _half_only_error(torch, a, b, mode)

    ran = 0
    for cfg in range(18):
        for swap in (0, 1):
            try:
                plan.set_step_kernel(0, mode, 2, cfg, swap, 1)
            except P.LtnError:
                continue
            out = plan.execute([0], mode=mode)
            torch.cuda.synchronize()
            got = out.cpu().numpy().reshape(1 << m, 1 << n)
            err = np.abs(got - exact)
            ratio = float((err / bound).max())
            fro = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
            banner(f"{mode} k={k} wide={wide} cfg={cfg} swap={swap}: max err/bound {ratio:.3f}, "
                   f"rel fro {fro:.2e} (half-only {e_half:.2e})")
            assert ratio <= 1.0
            assert fro <= e_half / 16
            ran += 1
    assert ran >= 2, "no split tile fits the step"
