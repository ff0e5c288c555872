"""Marshalling helpers shared by the GPU tests."""
def dev(a, dtype=None):
    """numpy -> contiguous cuda tensor (test marshalling only)."""
    import numpy as np
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()
