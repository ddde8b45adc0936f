"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda:0")


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev())


def normwise(got, ref):
    """max-norm relative error ||got - ref||_inf / ||ref||_inf"""
    return float(np.abs(np.asarray(got) - np.asarray(ref)).max() / np.abs(ref).max())


def say(*a):
    print(*a, flush=True)
