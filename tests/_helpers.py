"""Shared helpers for the GPU parity tests (comparison metrics and tolerances)."""
import numpy as np

# FP64 path vs FP64 oracle: number density normwise, moments and C per entry
TOL = 1e-10


def rel_inf(got, ref):
    ref = np.asarray(ref)
    scale = np.max(np.abs(ref))
    if scale == 0:
        return float(np.max(np.abs(got)))
    return float(np.max(np.abs(np.asarray(got) - ref)) / scale)


def rel_each(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    den = np.where(ref == 0, 1.0, np.abs(ref))
    return float(np.max(np.abs(got - ref) / den))


def split_packed(flat, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(flat[o:o + n])
        o += n
    return out


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
