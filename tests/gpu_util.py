"""Shared helpers of the GPU tests: device transfer and the parity metric."""
import numpy as np
import torch


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().double().cpu().numpy()


def max_rel(got, ref):
    """max_I |got - ref| / max_I |ref|: the element-wise parity metric."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (scale if scale > 0 else 1.0))


def l2_rel(got, ref):
    return float(np.linalg.norm(np.asarray(got) - np.asarray(ref)) / np.linalg.norm(ref))


def f32(a):
    """Round a float64 array to float32 and back (the values an FP32 field holds)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)
