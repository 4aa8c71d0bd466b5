"""Helpers shared by the GPU tests: device tensors and error norms."""

import numpy as np


def dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def zeros(*shape):
    import torch

    return torch.zeros(*shape, dtype=torch.float64, device="cuda")


def relnorm(got, ref):
    return float(np.linalg.norm(np.asarray(got) - np.asarray(ref)) / np.linalg.norm(ref))


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
