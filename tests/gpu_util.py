"""Helpers for the GPU parity tests (device transfer and error metrics)."""
import numpy as np
import torch

DEV = "cuda"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", dtype=torch.float64).numpy()


def relerr(got, ref):
    """Normwise max error: max|got-ref| / max|ref| (per array)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def field_errs(got, ref):
    return [relerr(got[q], ref[q]) for q in range(got.shape[0])]
