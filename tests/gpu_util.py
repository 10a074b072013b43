"""Helpers for GPU tests: move numpy arrays to the device and back with the
C-ABI's integer types (uint32 ids and uint64 offsets travel as int32/int64
tensors with the same bits)."""
from __future__ import annotations

import numpy as np
import torch

NONE = 0xFFFFFFFF


def dev(a: np.ndarray) -> torch.Tensor:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    elif a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a.copy()).cuda()


def host_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def empty_u32(*shape, fill=NONE) -> torch.Tensor:
    t = torch.empty(*shape, dtype=torch.int32, device="cuda")
    t.fill_(np.uint32(fill).view(np.int32).item())
    return t


def say(msg: str) -> None:
    print(msg, flush=True)
