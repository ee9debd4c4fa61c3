"""Shared helpers for the GPU parity tests (inputs from synth, references from oracle)."""
import numpy as np


def rel_err(y, ref):
    y = np.asarray(y)
    ref = np.asarray(ref)
    return float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel()))


def random_rim_er(prob, seed):
    rng = np.random.default_rng(seed)
    return 0.1 * (rng.standard_normal((prob.N, prob.Nr)) + 1j * rng.standard_normal((prob.N, prob.Nr)))


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def banner(msg):
    print(f"[gpu-case] {msg}", flush=True)
