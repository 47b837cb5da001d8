"""Shared test helpers: class-map packing (a storage format, not part of the
method) and GPU availability."""
import os

import numpy as np


def class_pitch(W):
    return ((-(-W // 4)) + 3) & ~3


def unpack_classes(packed, H, W):
    """Packed 2-bit class map (H x pitch bytes) -> uint8 (H, W) codes."""
    packed = np.asarray(packed, dtype=np.uint8)[:H]
    x = np.arange(W)
    return ((packed[:, x // 4] >> (2 * (x % 4)).astype(np.uint8)) & 3).astype(np.uint8)


def pack_classes(cls):
    """uint8 (H, W) codes -> packed (H, class_pitch(W)) bytes."""
    H, W = cls.shape
    out = np.zeros((H, class_pitch(W)), np.uint8)
    for k in range(4):
        col = cls[:, k::4].astype(np.uint8)
        out[:, :col.shape[1]] |= (col & 3) << (2 * k)
    return out


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def lib_built():
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return os.path.exists(os.path.join(here, "paper_1710_07745_amd", "libcanny.so"))
