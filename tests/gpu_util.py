"""Helpers shared by the GPU tests (no arithmetic of the method)."""
import numpy as np


def rel_l2(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
