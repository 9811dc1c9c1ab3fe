"""Helpers shared by the GPU parity tests (no simulation arithmetic here)."""
import numpy as np
import torch

C64_MAX_ABS = 1e-5       # complex64 max-abs amplitude error vs FP64
C64_L2 = 1e-4            # complex64 ||psi - psi_ref||_2 (psi is unit-norm)
C128_MAX_ABS = 1e-12
C128_L2 = 1e-12


def to_dev(psi: np.ndarray, dtype=torch.complex64) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(psi)).to(dtype)
    if t.dim() == 1:
        t = t.reshape(1, -1)
    return t.cuda().contiguous()


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def round_c64(psi: np.ndarray) -> np.ndarray:
    """The complex64-representable version of psi (as complex128)."""
    return psi.astype(np.complex64).astype(np.complex128)


def check_close(got: np.ndarray, ref: np.ndarray, dtype, what=""):
    got = got.reshape(ref.shape)
    err = np.abs(got - ref)
    mx = float(err.max()) if err.size else 0.0
    l2 = float(np.sqrt((err ** 2).sum(axis=-1)).max()) if err.size else 0.0
    tol_mx, tol_l2 = (C64_MAX_ABS, C64_L2) if dtype == torch.complex64 else (C128_MAX_ABS, C128_L2)
    assert mx <= tol_mx and l2 <= tol_l2, f"{what}: max-abs {mx:.3e} (tol {tol_mx}), L2 {l2:.3e} (tol {tol_l2})"
    return mx, l2
