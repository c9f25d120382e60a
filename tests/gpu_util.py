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


def l1_relerr(got, ref):
    """L1 relative error: sum|got-ref| / sum|ref| (per array)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).sum()
    return float(np.abs(got - ref).sum() / (den if den > 0 else 1.0))


def field_l1_errs(got, ref):
    return [l1_relerr(got[q], ref[q]) for q in range(got.shape[0])]


def hydro_l1_errs(got, ref):
    """L1 relative errors of the hydro state by physical field: density,
    momentum as a vector (sum over both components of |got-ref|, divided by
    the same sum of |ref|: independent of the orientation of the axes, and
    of how the flow's momentum happens to split between them), energy."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mom = float((np.abs(got[1] - ref[1]).sum() + np.abs(got[2] - ref[2]).sum()) /
                max(np.abs(ref[1]).sum() + np.abs(ref[2]).sum(), 1e-300))
    return {"rho": l1_relerr(got[0], ref[0]), "momentum": mom, "E": l1_relerr(got[3], ref[3])}


def hydro_errs(got, ref):
    """Max-norm relative errors of a hydro state (rho, rho u, rho v, E) by
    physical field: density, momentum as a vector (largest |got-ref| over
    both components divided by the largest |ref| over both components) and
    energy.  The Euler equations are rotation invariant, so the momentum's
    error is measured against the momentum's size, not against one
    component's: a component that is small only because of the axes'
    orientation (the y momentum of a wave running nearly along x) is the
    difference of fluxes of the full size and carries their rounding."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    mden = max(np.abs(ref[1]).max(), np.abs(ref[2]).max())
    mnum = max(np.abs(got[1] - ref[1]).max(), np.abs(got[2] - ref[2]).max())
    return [relerr(got[0], ref[0]), float(mnum / (mden if mden > 0 else 1.0)), relerr(got[3], ref[3])]
