"""Shared helpers for the GPU tests (torch device plumbing; no likelihood arithmetic)."""
import numpy as np


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def oracle_network(inst, n_det=None):
    """FP64 oracle logL over the first n_det detectors of a synth.Instance."""
    import oracle
    n_det = inst.n_det if n_det is None else n_det
    fs = [oracle.factor(inst.acf, inst.N, inst.masks[k], inst.segments) for k in range(n_det)]
    return oracle.loglik_network(fs, inst.d[:n_det], inst.H), fs
