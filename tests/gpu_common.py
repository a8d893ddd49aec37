"""Helpers shared by the GPU tests (data movement and error measures only)."""
import numpy as np
import torch

DEV = "cuda:0"


def to_dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).to(DEV)


def to_host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def rel_err(y, y_ref) -> float:
    """Norm-wise relative error |y - y_ref|_2 / |y_ref|_2 (FP64, complex128 when either is complex)."""
    cplx = np.iscomplexobj(y) or np.iscomplexobj(y_ref)
    y = np.asarray(y, dtype=np.complex128 if cplx else np.float64)
    y_ref = np.asarray(y_ref, dtype=np.complex128 if cplx else np.float64)
    den = np.linalg.norm(y_ref)
    return float(np.linalg.norm(y - y_ref) / (den if den > 0 else 1.0))


def say(*a):
    print(*a, flush=True)
