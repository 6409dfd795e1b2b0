"""Helpers shared by the GPU tests: building ops from workload parameters and
moving states between NumPy and the device (no arithmetic of the method)."""

import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected without a visible GPU")
    return torch


def to_dev(x, dtype):
    torch = require_gpu()
    t = torch.from_numpy(np.ascontiguousarray(x))
    return t.to(device="cuda", dtype=dtype)


def to_np(t):
    return t.detach().cpu().numpy()


def ki_op(p):
    from paper_2102_05054_amd import kicked_ising
    return kicked_ising(p.L, p.J, p.h, p.g, p.periodic)


def bw_op(p):
    from paper_2102_05054_amd import brickwork
    return brickwork(p.L, p.gates)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def circ_op(p):
    from paper_2102_05054_amd import circuit
    return circuit(p.L, p.sites, p.widths, p.gates)
