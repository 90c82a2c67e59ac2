"""Helpers shared by the GPU tests: host <-> device copies of key arrays."""
import numpy as np
import torch


def to_dev(x: np.ndarray) -> torch.Tensor:
    if x.dtype == np.uint64:
        x = x.view(np.int64)
    if x.dtype == np.uint32:
        x = x.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def to_host(t: torch.Tensor, dtype) -> np.ndarray:
    a = t.detach().cpu().numpy()
    return a.view(dtype)


def banner(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
