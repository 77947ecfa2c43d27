"""Complex64 GEMM tiles against their analytic rounding bounds.

A two-leaf network whose only step is one complex GEMM C = A B runs in
complex64 mode on every complex64 tile that fits (kind 1: direct tiles 0-9,
three-product tiles 10-15; kind 5: split-K tiles 0-7 for a long sum), in both
operand roles, forced through ltn_set_step_kernel; the exact product of the
complex64 inputs (complex128) is the reference. u = 2^-23 (so as not to
assume round-to-nearest inside the matrix core), sums of L terms add at most
L u of their absolute sum (the order inside an MFMA is not known), and a
factor 1.5 covers the second-order terms.

Direct form (the 2x2 real form: Re c = sum ar br - ai bi, Im c = sum ar bi +
ai br, 2K real products per component): with R = |A| |B| (elementwise
moduli),

    |Re, Im (c - AB)| <= 1.5 (2K + 2) u R.

Three-product form (Gauss's method: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)
(Br + Bi), Re c = P1 - P2, Im c = (P3 - P1) - P2, the sums Ar + Ai and
Br + Bi rounded once): with S1 = |Ar| |Br|, S2 = |Ai| |Bi| and
S3 = (|Ar| + |Ai|)(|Br| + |Bi|),

    |Re (c - AB)| <= 1.5 (K + 2) u (S1 + S2),
    |Im (c - AB)| <= 1.5 (K + 6) u (S1 + S2 + S3)

(P3 carries K u S3 from its sum and 2 u S3 from the rounded operand sums;
the two subtractions add u of their operands each). Split-K sums add one
term per chunk: K is replaced by K + chunks (at most 2^8).

Operands: standard normal parts; wide-range rows and columns (magnitudes
over 2^16, as amplitudes of deep circuits); and B = A^H (Hermitian A A^H,
whose diagonal has no imaginary part, so Im c there is pure rounding error
of terms that cancel exactly)."""
import numpy as np
import pytest

from tests.gpu_util import banner

pytestmark = pytest.mark.gpu

U = 2.0 ** -23


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _operands(m, k, n, seed, kind):
    rng = np.random.default_rng(seed)
    M, K, N = 1 << m, 1 << k, 1 << n
    a = rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))
    if kind == "hermitian":
        assert M == N
        b = a.conj().T.copy()
    else:
        b = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    if kind == "wide":
        a *= 2.0 ** -rng.integers(0, 17, size=(M, 1)) * 2.0 ** -20
        b *= 2.0 ** -rng.integers(0, 9, size=(1, N))
    return a.astype(np.complex64), b.astype(np.complex64)


def _bounds(a, b, K_eff, three):
    """Elementwise bounds on |Re| and |Im| of the error (float64)."""
    ar, ai = np.abs(a.real).astype(np.float64), np.abs(a.imag).astype(np.float64)
    br, bi = np.abs(b.real).astype(np.float64), np.abs(b.imag).astype(np.float64)
    if not three:
        R = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
        e = 1.5 * (2 * K_eff + 2) * U * R
        return e, e
    S1, S2, S3 = ar @ br, ai @ bi, (ar + ai) @ (br + bi)
    return 1.5 * (K_eff + 2) * U * (S1 + S2), 1.5 * (K_eff + 6) * U * (S1 + S2 + S3)


@pytest.mark.parametrize("operands", ["normal", "wide", "hermitian"])
@pytest.mark.parametrize("m,k,n", [(8, 6, 8), (7, 11, 7)])
def test_c64_gemm_within_analytic_bound(torch, m, k, n, operands):
    import paper_2205_00393_amd as P
    a, b = _operands(m, k, n, seed=300 + 10 * k + m, kind=operands)
    mi = list(range(m))
    ki = list(range(m, m + k))
    ni = list(range(m + k, m + k + n))
    net = P.Network.from_arrays([mi + ki, ki + ni], [a, b], mi + ni, m + k + n)
    plan = P.Plan(net, [(0, 1)], [])
    plan.bind(batch=1, budget_bytes=1 << 29)
    assert len(plan.steps()) == 1
    exact = a.astype(np.complex128) @ b.astype(np.complex128)
    K = 1 << k
    ran = {False: 0, True: 0}
    for kind, n_cfg in ((1, 16), (5, 8)):
        for cfg in range(n_cfg):
            for swap in (0, 1):
                try:
                    plan.set_step_kernel(0, "c64", kind, cfg, swap, 1)
                except P.LtnError:
                    continue
                name = P.kernel_name(kind, cfg)
                three = "_3m_" in name
                # split-K: at most 2^8 chunks, each one more term of the sum
                eb_re, eb_im = _bounds(a, b, K + (256 if kind == 5 else 0), three)
                out = plan.execute([0], mode="c64")
                torch.cuda.synchronize()
                got = out.cpu().numpy().reshape(1 << m, 1 << n)
                d = got - exact
                r_re = float((np.abs(d.real) / eb_re).max())
                r_im = float((np.abs(d.imag) / eb_im).max())
                banner(f"c64 ({m},{k},{n}) {operands} {name} swap {swap}: max err/bound re {r_re:.3f} "
                       f"im {r_im:.3f}")
                assert r_re <= 1.0 and r_im <= 1.0
                if operands == "hermitian":
                    # the diagonal's imaginary part is rounding error alone
                    diag = np.abs(np.diagonal(got).imag)
                    assert float((diag / np.diagonal(eb_im)).max()) <= 1.0
                ran[three] += 1
    assert ran[False] >= 1 and ran[True] >= 1, f"tiles run per form: {ran}"
