"""Helpers shared by the GPU parity tests (inputs come from synthetic/ and the
oracle; nothing here computes any part of the method)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def verts_np(verts):
    """[3T,4] int32 CUDA records -> (float32 [3T,3], uint32 [3T])."""
    v = verts.cpu().numpy()
    return v[:, :3].view(np.float32).copy(), v[:, 3].view(np.uint32).copy()
