"""Shared helpers for the GPU parity tests (inputs from synth, references from oracle)."""
import numpy as np


def rel_err(y, ref):
    y = np.asarray(y)
    ref = np.asarray(ref)
    return float(np.linalg.norm((y - ref).ravel()) / np.linalg.norm(ref.ravel()))


def parity_errors(Y, ref, N=None, rows=None):
    """Error measures of Y against ref (both (R, n)): the global relative
    2-norm, the largest entry error over the largest reference entry (a
    per-row bound, so that an error confined to a few rows cannot hide in the
    global norm), and the relative 2-norms of the element rows (< N) and of
    the rim rows (>= N) separately.  rows: the unknown index of each of the n
    entries (default 0..n-1)."""
    Y = np.atleast_2d(np.asarray(Y, dtype=np.complex128))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.complex128))
    assert Y.shape == ref.shape, (Y.shape, ref.shape)
    d = Y - ref
    out = {"global": float(np.linalg.norm(d) / np.linalg.norm(ref)),
           "row_max": float(np.max(np.abs(d)) / np.max(np.abs(ref)))}
    if N is not None:
        idx = np.arange(ref.shape[1]) if rows is None else np.asarray(rows)
        for name, sel in (("element", idx < N), ("rim", idx >= N)):
            if np.any(sel):
                out[name] = float(np.linalg.norm(d[:, sel]) / np.linalg.norm(ref[:, sel]))
    return out


def assert_parity(Y, ref, tol, N=None, rows=None, what=""):
    """Every measure of parity_errors within tol."""
    e = parity_errors(Y, ref, N, rows)
    bad = {k: v for k, v in e.items() if not v <= tol}
    assert not bad, f"{what}: {bad} > {tol} (all: {e})"
    return e


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
