"""Helpers for GPU tests: device transfers of unsigned keys held in torch's
signed dtypes (bit patterns), and the GPU-availability gate."""
import numpy as np
import pytest
import torch


def have_gpu() -> bool:
    return torch.cuda.is_available()


def require_gpu():
    if not have_gpu():
        pytest.skip("no GPU")
    import paper_2401_00710_amd._lib as L
    L.load()  # fails loudly if the HIP library is missing


def dev_u32(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def dev_u64(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def say(msg: str):
    print(msg, flush=True)
