"""Shared helpers for the GPU parity tests (inputs from workloads, expected
values from the oracle, results from libtri through its C ABI)."""
import numpy as np
import torch


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def line_relerr(got, ref, axis):
    """Per-line relative error max_j |x - xref| / max_j |xref| along `axis`;
    returns the worst line's value (complex moduli for complex arrays)."""
    num = np.max(np.abs(got - ref), axis=axis)
    den = np.max(np.abs(ref), axis=axis)
    den = np.where(den == 0, 1.0, den)
    return float(np.max(num / den))


TOL = 1e-12
