"""Helpers shared by the GPU tests: device buffers from numpy words and back."""
import numpy as np
import torch


def to_dev(words: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(words, dtype=np.uint64).view(np.int64)).cuda()


def to_host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64).copy()


def dev_pool(mats) -> torch.Tensor:
    """Stack equal-length word arrays into one (n, nwords) device tensor."""
    return to_dev(np.stack(mats))


def empty_words(nw: int) -> torch.Tensor:
    # poison the output so unwritten words show up
    return torch.full((max(nw, 1),), 0x5A5A5A5A5A5A5A5A, dtype=torch.int64, device="cuda")


def tail_mask(r_bits: int) -> int:
    rem = r_bits % 64
    return (1 << rem) - 1 if rem else (1 << 64) - 1
