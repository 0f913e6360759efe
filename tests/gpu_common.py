"""Helpers shared by the GPU parity tests (they compare the HIP path, called
through the C ABI, with the FP64 oracle on identical seeded inputs)."""
import sys

import numpy as np
import torch

import cgp_inputs as ci
from oracle.grid import Grid
from oracle.model import Physics


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev():
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev()).contiguous()


def to_np(t):
    return t.detach().to("cpu", torch.float64).numpy()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_setup(case):
    g = Grid(case.nx, case.ny, case.lx, case.ly, case.y0)
    phys = Physics(inv_re=case.inv_re, inv_ro=case.inv_ro, f1=case.f1, f2=case.f2, drag=case.drag)
    return g, phys


def random_state(case, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return ci.initial_field(case, rng, scale=scale)
