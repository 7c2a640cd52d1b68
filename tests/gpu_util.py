"""Shared helpers of the GPU parity tests (oracle on the CPU, HIP via the C ABI)."""
import numpy as np

from paper_1610_07522_amd import inputs

# Small boxes that the oracle finishes in seconds: several line tiles, ragged
# state counts (not multiples of the 64-wide GEMM tiles or 32-wide Jacobi
# blocks) and every supported grid size up to 32.
CASES = {
    "n16_8p8": inputs.WORKLOADS["fermi16"],
    "n24_13p7_rod": inputs.small_workload("n24", 24, 13, 7, init="rod", seed=31, noise=0.05),
    "n8_5p3": inputs.small_workload("n8", 8, 5, 3, init="slab", seed=32, noise=0.2),
    "n32_70p33_slab": inputs.small_workload("n32", 32, 70, 33, init="slab", seed=33, noise=0.02),
    # pasta density 0.018 fm^-3: several Cholesky blocks and Jacobi block pairs
    "n24_200p50_rod": inputs.small_workload("n24r", 24, 200, 50, init="rod", seed=2, noise=0.0),
}


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.abs(b).max(), 1e-300)
    return float(np.abs(a - b).max() / den)


def to_dev(x, dev="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def to_host(t):
    return t.detach().cpu().numpy()
