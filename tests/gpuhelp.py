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


def dense_planes(n: int) -> int:
    """Counter planes of the dense kernel for n inputs (bit length of n,
    at least 4, and 16 above 13)."""
    k = max(4, int(n).bit_length())
    return 16 if k > 13 else k


def force_dense_shape(tq, ctx, n: int, nwords: int, wpl: int = 1, split: int = 1, groups: int = 1) -> str:
    """Make every dense query with n inputs over nwords-word bitmaps run the
    given launch shape: tuning entries for all of its shape classes are
    imported and the tuner is switched on (an imported entry is used as
    given, nothing is timed).  Returns the imported text."""
    K = dense_planes(n)
    log_n = int(n).bit_length() - 1
    log_w = int(nwords).bit_length() - 1
    lines = []
    for kind in range(4):
        for pruned in (0, 1):
            for t8 in range(9):
                for a16 in (0, 1):
                    if wpl == 2 and not a16:
                        continue
                    lines.append("1 %d %d %d %d %d %d %d : %d %d %d 0 : 1.000"
                                 % (K, log_n, log_w, kind, pruned, t8, a16, wpl, split, groups))
    text = "\n".join(lines) + "\n"
    tq.tq_tune_import(ctx, text)
    tq.tq_set_option(ctx, tq.TQ_OPTION_AUTOTUNE, 1)
    return text
