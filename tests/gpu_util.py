"""Helpers of the GPU tests: device transfer and error measures (no method
arithmetic here)."""
import sys

import numpy as np
import torch

DEV = "cuda"
TOL = 1e-11   # relative Frobenius error of the FP64 path against the oracle


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def progress(msg: str):
    """A line on the process's real stderr (not captured by pytest), for the
    long steps of the full-size tests."""
    sys.__stderr__.write(f"[progress] {msg}\n")
    sys.__stderr__.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relf(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b)
    s = np.linalg.norm(b)
    return float(d / s) if s > 0 else float(d)


def with_upper_garbage(A: np.ndarray, seed: int = 0) -> np.ndarray:
    """Copy of A whose strict upper triangle is overwritten with NaN and huge
    values: the library must never read it."""
    B = A.copy()
    iu = np.triu_indices(A.shape[0], 1)
    rng = np.random.default_rng(seed)
    vals = rng.choice([np.nan, 1e300, -1e300], size=len(iu[0]))
    B[iu] = vals
    return B
