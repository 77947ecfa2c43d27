"""Every kernel a step can run, forced step by step through
ltn_set_step_kernel: narrow-step kernel (both forms) in both operand roles, generic
kernel with 1, 8 and 64 threads per output, complex64 MFMA tiles, and the
split tiles (register- and DMA-staged) in the split modes. Each forced plan must reproduce the
brute-force state-vector amplitudes (complex64 <= 1e-4, split <= 5e-4).
The split-sum and split-K kernels, whose steps the reduced circuits do
not have, run alone on one-step networks against the exact product."""
import numpy as np
import pytest

from tests.gpu_util import banner, rel_l2
from tests.test_gpu_amplitudes import _reduced, _sv

pytestmark = pytest.mark.gpu

# split tile configurations (register-staged 0-9, DMA-staged 10-17)
N_SPLIT_CFGS = 18
# complex64 tile configurations (direct form 0-9, three-product form 10-15)
N_C64_CFGS = 16

VARIANTS = {
    "narrow_rows_a": [(3, 0, 0, 1)],
    "narrow_rows_b": [(3, 0, 1, 1)],
    # the narrow kernel's one-thread-per-row form (k, n <= 4, m >= 8)
    "narrow_thread_rows_a": [(3, 1, 0, 1)],
    "generic_tk1": [(0, -1, 0, 1)],
    "generic_tk8": [(0, -1, 0, 8)],
    "generic_tk64": [(0, -1, 0, 64)],
    "mfma_c64": [(1, c, s, 1) for s in (0, 1) for c in range(10)],
    # complex64 tiles with three real products per complex product (10-15)
    "mfma_c64_3m": [(1, c, s, 1) for s in (0, 1) for c in range(10, N_C64_CFGS)],
    "mfma_split": [(2, c, s, 1) for s in (0, 1) for c in range(N_SPLIT_CFGS)],
    # split sum over k for few-output steps (m, n <= 3)
    "split_sum": [(4, 0, 0, 1)],
    # split tiles staged by global_load_lds (configurations 10-17)
    "mfma_split_dma": [(2, c, s, 1) for s in (0, 1) for c in range(10, N_SPLIT_CFGS)],
}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


@pytest.fixture(scope="module")
def prepared():
    """Narrow steps of every shape: a reconfigured path at t = 14."""
    import paper_2205_00393_amd as P
    w = _reduced(rows=4, cols=5, cycles=10, n_open=6, t=14)
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3, reconf_k=6)
    return w, pr, _sv(w)


@pytest.fixture(scope="module")
def prepared_fat():
    """Steps large enough for the MFMA tiles: a greedy path at t = 16."""
    import paper_2205_00393_amd as P
    w = _reduced(rows=4, cols=5, cycles=12, n_open=6, t=16)
    pr = P.prepare(w, alphas=(0.5, 1.0), taus=(0.0, 0.3), n_seeds=3)
    return w, pr, _sv(w)


@pytest.mark.parametrize("mode", ["c64", "split_f16", "split_bf16"])
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_forced_kernel_variant(torch, prepared, prepared_fat, mode, variant):
    import paper_2205_00393_amd as P
    if variant.startswith("mfma_split") and mode == "c64":
        pytest.skip("split tiles need a split mode")
    w, pr, ref = prepared_fat if variant.startswith("mfma") else prepared
    plan = pr.plan()
    n = 1 << len(pr.sliced)
    plan.bind(batch=min(n, 4), budget_bytes=1 << 30)
    forced = []
    for k, st in enumerate(plan.steps()):
        for kind, cfg, swap, tk in VARIANTS[variant]:
            try:
                plan.set_step_kernel(k, mode, kind, cfg, swap, tk)
            except P.LtnError:
                continue
            forced.append((k, st["m"], st["k"], st["n"]))
            break
    banner(f"forced {variant} in {mode} on {len(forced)} of {len(plan.steps())} steps")
    assert forced, "no step accepts this kernel"
    out = plan.execute_range(0, n, mode=mode)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    banner(f"forced {variant} {mode}: rel err {err:.3e}")
    assert err < (1e-4 if mode == "c64" else 5e-4)


def test_set_step_kernel_rejects_misfits(torch, prepared):
    import paper_2205_00393_amd as P
    w, pr, ref = prepared
    plan = pr.plan()
    plan.bind(batch=1, budget_bytes=1 << 30)
    with pytest.raises(P.LtnError, match="split"):
        plan.set_step_kernel(0, "c64", 2, 0, 0, 1)
    with pytest.raises(P.LtnError, match="tk"):
        plan.set_step_kernel(0, "c64", 0, -1, 0, 3)
    with pytest.raises(P.LtnError, match="kind"):
        plan.set_step_kernel(0, "c64", 7, 0, 0, 1)
    big = [k for k, st in enumerate(plan.steps()) if st["k"] + st["n"] > 10 and st["k"] + st["m"] > 10]
    for k in big[:1]:
        with pytest.raises(P.LtnError, match="narrow"):
            plan.set_step_kernel(k, "c64", 3, 0, 0, 1)


def _force_kind(P, plan, k, mode, kind):
    for cfg in range(N_SPLIT_CFGS):
        for swap in (0, 1):
            try:
                plan.set_step_kernel(k, mode, kind, cfg, swap, 1)
                return True
            except P.LtnError:
                continue
    return False


@pytest.mark.parametrize("mode", ["split_f16", "split_bf16"])
def test_split_producer_writes_split_layout(torch, prepared_fat, mode):
    """Split modes: a tensor that a matrix-core step produces (complex64 or
    split tile) and a split step consumes is written by the producer in the
    split layout (fp16: scaled by the bound 2 K max|a| max|b| from its
    operands' maxima) and read without a conversion pass. Every step that takes
    a split tile gets one, other matrix-core steps a complex64 tile; then the
    producer of the first split step fed by a split step is switched to a
    complex64 tile, so that both producer kinds feed split consumers. The
    result must match the state vector."""
    import paper_2205_00393_amd as P
    w, pr, ref = prepared_fat
    plan = pr.plan()
    n = 1 << len(pr.sliced)
    plan.bind(batch=min(n, 4), budget_bytes=1 << 30)
    steps = plan.steps()
    kind_of = {}
    for k in range(len(steps)):
        for kind in (2, 1):
            if _force_kind(P, plan, k, mode, kind):
                kind_of[k] = kind
                break
    producer = {st["out"]: k for k, st in enumerate(steps)}

    def feeds():
        pairs = []
        for k, st in enumerate(steps):
            if kind_of.get(k) == 2:
                for t in (st["left"], st["right"]):
                    pk = producer.get(t)
                    if pk is not None and kind_of.get(pk) in (1, 2):
                        pairs.append((pk, k))
        return pairs

    first = next((pk for pk, k in feeds() if kind_of[pk] == 2), None)
    assert first is not None, "no split step is fed by a split step"
    assert _force_kind(P, plan, first, mode, 1)
    kind_of[first] = 1
    kinds = {kind_of[pk] for pk, _ in feeds()}
    banner(f"{mode} direct operands: {len(feeds())} producer->split pairs, producer kinds {sorted(kinds)}")
    assert kinds == {1, 2}
    out = plan.execute_range(0, n, mode=mode)
    torch.cuda.synchronize()
    err = rel_l2(out.cpu().numpy(), ref)
    banner(f"{mode} with direct split operands: rel err {err:.3e}")
    assert err < 5e-4


@pytest.mark.parametrize("m,k,n", [(3, 20, 3), (0, 16, 2), (2, 13, 0), (1, 5, 3), (3, 0, 3), (2, 11, 2)])
def test_split_sum_single_step(torch, m, k, n):
    """The split-sum kernel alone on one-step networks: C = A B with 2^m x
    2^k and 2^k x 2^n complex64 operands (k = 0 is an outer product; k = 20
    runs 512 chunks), in every mode, against the exact product."""
    import paper_2205_00393_amd as P
    rng = np.random.default_rng(1000 + 100 * m + 10 * n + k)
    M, K, N = 1 << m, 1 << k, 1 << n
    a = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))).astype(np.complex64)
    b = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))).astype(np.complex64)
    mi, ki, ni = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    net = P.Network.from_arrays([mi + ki, ki + ni], [a, b], mi + ni, m + k + n)
    plan = P.Plan(net, [(0, 1)], [])
    plan.bind(batch=1, budget_bytes=1 << 30)
    exact = (a.astype(np.complex128) @ b.astype(np.complex128)).reshape(-1)
    for mode in ("c64", "split_f16", "split_bf16"):
        plan.set_step_kernel(0, mode, 4, 0, 0, 1)
        out = plan.execute([0], mode=mode)
        torch.cuda.synchronize()
        err = rel_l2(out.cpu().numpy(), exact)
        banner(f"split sum ({m},{k},{n}) {mode}: rel err {err:.2e}")
        assert err < 1e-5


@pytest.mark.parametrize("m,k,n", [(9, 12, 4), (7, 11, 6), (4, 12, 9), (10, 16, 5), (12, 10, 10), (6, 14, 6)])
def test_splitk_single_step(torch, m, k, n):
    """The split-K complex64 MFMA GEMM (kind 5) alone on one-step networks:
    C = A B with 2^m x 2^k and 2^k x 2^n complex64 operands, every tile
    configuration (direct and three-product form) in both operand roles
    where it fits (from 2 to 256 chunks of the sum), in every mode, against
    the exact product."""
    import paper_2205_00393_amd as P
    rng = np.random.default_rng(2000 + 100 * m + 10 * n + k)
    M, K, N = 1 << m, 1 << k, 1 << n
    a = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))).astype(np.complex64)
    b = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))).astype(np.complex64)
    mi, ki, ni = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    net = P.Network.from_arrays([mi + ki, ki + ni], [a, b], mi + ni, m + k + n)
    plan = P.Plan(net, [(0, 1)], [])
    plan.bind(batch=1, budget_bytes=2 << 30)
    exact = (a.astype(np.complex128) @ b.astype(np.complex128)).reshape(-1)
    runs = 0
    for mode in ("c64", "split_f16", "split_bf16"):
        for swap in (0, 1):
            for cfg in range(8):
                try:
                    plan.set_step_kernel(0, mode, 5, cfg, swap, 1)
                except P.LtnError:
                    continue
                out = plan.execute([0], mode=mode)
                torch.cuda.synchronize()
                err = rel_l2(out.cpu().numpy(), exact)
                banner(f"split-K ({m},{k},{n}) cfg {cfg} swap {swap} {mode}: rel err {err:.2e}")
                assert err < 2e-5
                runs += 1
    assert runs > 0, "no split-K tile fits"


@pytest.mark.parametrize("m,k,n", [(9, 0, 1), (10, 2, 3), (3, 2, 10), (12, 4, 4), (4, 1, 11), (22, 2, 2)])
def test_narrow_rows_single_step(torch, m, k, n):
    """The narrow kernel's one-thread-per-row form alone on one-step
    networks (the plan puts the large operand in the rows role, so (3,2,10)
    and (4,1,11) run as (10,2,3) and (11,1,4)), in every mode, against the
    exact product; at m = 22 the blocks take several 256-row chunks of the
    slice, so the output address is advanced by the masked add."""
    import paper_2205_00393_amd as P
    rng = np.random.default_rng(3000 + 100 * m + 10 * n + k)
    M, K, N = 1 << m, 1 << k, 1 << n
    a = (rng.standard_normal((M, K)) + 1j * rng.standard_normal((M, K))).astype(np.complex64)
    b = (rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))).astype(np.complex64)
    mi, ki, ni = list(range(m)), list(range(m, m + k)), list(range(m + k, m + k + n))
    net = P.Network.from_arrays([mi + ki, ki + ni], [a, b], mi + ni, m + k + n)
    plan = P.Plan(net, [(0, 1)], [])
    plan.bind(batch=1, budget_bytes=2 << 30)
    exact = (a.astype(np.complex128) @ b.astype(np.complex128)).reshape(-1)
    runs = 0
    for mode in ("c64", "split_f16", "split_bf16"):
        for swap in (0, 1):
            try:
                plan.set_step_kernel(0, mode, 3, 1, swap, 1)
            except P.LtnError:
                continue
            out = plan.execute([0], mode=mode)
            torch.cuda.synchronize()
            err = rel_l2(out.cpu().numpy(), exact)
            banner(f"narrow rows ({m},{k},{n}) swap {swap} {mode}: rel err {err:.2e}")
            assert err < 1e-5
            runs += 1
    assert runs == 3, "the rows form must fit one operand role"


@pytest.mark.parametrize("mode", ["c64", "split_f16", "split_bf16"])
def test_mfma_output_layouts(torch, mode):
    """MFMA tiles with the output's lowest bits from either operand: a
    two-step chain T = A B (contract k), C = T^T D (contract j) whose second
    step wants j innermost in T, so the first step writes T with its row
    bits lowest (16-byte epilogue stores) when A holds j (swap 0) and with
    its column bits lowest when the operands are swapped. Every complex64
    (and, in the split modes, every split) tile that fits runs the first
    step; in the split modes the second step is a split tile, so the first
    writes the split layout in its epilogue. Against the exact product."""
    import paper_2205_00393_amd as P
    J, K, M, N = 8, 6, 7, 6
    rng = np.random.default_rng(4000 + len(mode))
    cplx = lambda *s: (rng.standard_normal(s) + 1j * rng.standard_normal(s)).astype(np.complex64)
    a, b, d = cplx(1 << J, 1 << K), cplx(1 << K, 1 << M), cplx(1 << J, 1 << N)
    ji = list(range(J))
    ki = list(range(J, J + K))
    mi = list(range(J + K, J + K + M))
    ni = list(range(J + K + M, J + K + M + N))
    net = P.Network.from_arrays([ji + ki, ki + mi, ji + ni], [a, b, d], mi + ni, J + K + M + N)
    plan = P.Plan(net, [(0, 1), (2, 3)], [])
    plan.bind(batch=1, budget_bytes=1 << 30)
    exact = ((a.astype(np.complex128) @ b).T @ d).reshape(-1)
    st = plan.steps()
    assert (st[0]["m"], st[0]["k"], st[0]["n"]) in ((J, K, M), (M, K, J))
    if mode != "c64":
        assert _force_kind(P, plan, 1, mode, 2), "no split tile fits the second step"
    kinds = [1] if mode == "c64" else [1, 2]
    runs = 0
    for kind in kinds:
        for cfg in range(N_C64_CFGS if kind == 1 else N_SPLIT_CFGS):
            for swap in (0, 1):
                try:
                    plan.set_step_kernel(0, mode, kind, cfg, swap, 1)
                except P.LtnError:
                    continue
                out = plan.execute([0], mode=mode)
                torch.cuda.synchronize()
                err = rel_l2(out.cpu().numpy(), exact)
                banner(f"layout chain {mode} kind {kind} cfg {cfg} swap {swap}: rel err {err:.2e}")
                assert err < (1e-5 if mode == "c64" else 5e-4)
                runs += 1
    assert runs >= 4
