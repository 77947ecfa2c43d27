"""bench.py on the host: more than one GPU is refused with a message before
anything touches a device (slices are independent; the multi-GPU split is
design-only), and the per-step roofline arithmetic that marks matrix-core
steps GEMM-bound."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in (r.stdout + r.stderr)


def test_step_roofline_classification():
    """bench.py's roofline per matrix-core step, worked by hand: the ridge
    is the matrix peak over 8 TB/s (157.3 / 8 = 19.66 flop/B for FP32,
    2516.6 / 8 = 314.6 for FP16/BF16), against executed flops (8, 6 or 24
    per complex MAC on direct, three-product and split tiles) per
    algorithmic byte (A + B + C once, 8 bytes per complex element)."""
    import bench
    # (16,12,12), batch 4, direct complex64 tile: 2^40 MACs per slice
    f, fx, by, bound = bench.step_roofline(1, "c64_128x64x16", 16, 12, 12, 4)
    assert f == 8 * 2 ** 40 * 4 and fx == f
    assert by == 8 * (2 ** 28 + 2 ** 24 + 2 ** 28) * 4 and bound
    # three-product tile: 6 of the 8 flops executed
    f3, fx3, by3, _ = bench.step_roofline(1, "c64_3m_128x64x16", 16, 12, 12, 4)
    assert (f3, by3) == (f, by) and fx3 == 0.75 * f
    # (17,5,13): a short sum and a 2^30-element output; 2^35 / (2^30 + 2^22 +
    # 2^18) = 31.87 MACs per element moved, i.e. 31.87 flop/B on a direct
    # tile (GEMM-bound), 23.9 on a three-product tile (bound), 95.6 executed
    # on a split tile (below 314.6: bound by HBM)
    assert bench.step_roofline(1, "c64_128x64x16", 17, 5, 13, 1)[3]
    assert bench.step_roofline(1, "c64_3m_128x64x16", 17, 5, 13, 1)[3]
    assert not bench.step_roofline(2, "split_dma1x4_128x128x16", 17, 5, 13, 1)[3]
    # (20,4,20): 2^44 / (2^24 + 2^24 + 2^40) = 16.0 flop/B, below the FP32
    # ridge; (20,5,20): 32.0, above it; its three-product executed 24.0, too
    assert not bench.step_roofline(1, "c64_64x32x4", 20, 4, 20, 1)[3]
    assert bench.step_roofline(1, "c64_128x64x16", 20, 5, 20, 1)[3]
    assert bench.step_roofline(1, "c64_3m_128x64x16", 20, 5, 20, 1)[3]
    # (16,12,12) split: 24 * 2^40 / (8 (2^29 + 2^24)) = 5958 executed flop/B
    assert bench.step_roofline(2, "split_dma1x4_128x128x16", 16, 12, 12, 4)[3]
