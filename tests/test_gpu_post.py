"""Post-steps on the GPU against the oracle: port scattering matrix and far
field (same inputs on both sides; FP64, relative error <= 1e-10)."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import banner, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tp():
    import torch
    assert torch.cuda.is_available()
    import paper_2506_04710_amd as tp
    tp.load()
    return tp


def port_block(p, Nt, rows, Ihat, rng):
    """X (p, Nt) with random entries off the port rows and X[j, rows[i]] = Ihat[i, j]."""
    X = rng.standard_normal((p, Nt)) + 1j * rng.standard_normal((p, Nt))
    X[:, rows] = Ihat.T
    return X


@pytest.mark.parametrize("p", [1, 5, 64, 65, 200])
def test_smatrix_random_ports(tp, p):
    banner(f"S-matrix random p={p}")
    rng = np.random.default_rng(100 + p)
    Nt = 3 * p + 17
    rows = rng.choice(Nt, size=p, replace=False)
    # a well-conditioned admittance block: diagonal dominance plus a symmetric perturbation
    A = 0.05 * (rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)))
    Ihat = np.eye(p) * (0.02 + 0.01j) + 0.01 * (A + A.T) / np.sqrt(p)
    lens = rng.uniform(0.5, 1.5, size=p)
    X = port_block(p, Nt, rows, Ihat, rng)
    S = tp.port_smatrix(to_dev(X), rows, Z0=50.0, edge_len=lens).cpu().numpy()
    ref = oracle.s_matrix(Ihat, 50.0, edge_len=lens)
    assert rel_err(S, ref) <= 1e-10
    S1 = tp.port_smatrix(to_dev(X), rows, Z0=50.0).cpu().numpy()
    assert rel_err(S1, oracle.s_matrix(Ihat, 50.0)) <= 1e-10


def test_smatrix_matched_and_singular(tp):
    banner("S-matrix matched / singular")
    from paper_2506_04710_amd import _lib
    rng = np.random.default_rng(7)
    p, Nt, Z0 = 9, 40, 50.0
    rows = np.arange(0, 36, 4)
    X = port_block(p, Nt, rows, np.eye(p) / Z0, rng)        # Z_port = Z0 I: every port matched
    S = tp.port_smatrix(to_dev(X), rows, Z0=Z0).cpu().numpy()
    assert np.max(np.abs(S)) <= 1e-14
    X = port_block(p, Nt, rows, -np.eye(p) / 64.0, rng)     # I + Z0 Y = 0 exactly (powers of two)
    with pytest.raises(_lib.ToeplitzError) as ei:
        tp.port_smatrix(to_dev(X), rows, Z0=64.0)
    assert ei.value.status == _lib.TP_E_BREAKDOWN
    with pytest.raises(_lib.ToeplitzError):
        tp.port_smatrix(to_dev(X), np.full(p, Nt), Z0=Z0)  # row outside [0, Nt)


def test_smatrix_config3_ports(tp):
    """81 port excitations of the 9 x 9, b = 96 array solved together, then S."""
    banner("S-matrix 9x9 b96 81 ports")
    import torch
    prob, V = sa.make_config(3)
    p = V.shape[0]
    rows = np.nonzero(V)[1]
    assert rows.size == p
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=p, restart=40, device=torch.device("cuda:0"))
    x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8)
    assert all(i["status"] == 0 for i in info)
    S = tp.port_smatrix(x, rows, Z0=50.0).cpu().numpy()
    Xh = x.cpu().numpy()
    ref = oracle.s_matrix(Xh[:, rows].T, 50.0)
    assert rel_err(S, ref) <= 1e-10
    # a reciprocal operator gives a reciprocal network (to the solve tolerance)
    assert rel_err(S, S.T) <= 1e-6
    plan.close()


def geometry_args(prob):
    N = prob.N
    return (prob.Nx, prob.Ny, prob.b, prob.Nr, prob.d, prob.d, prob.centres[:prob.b], prob.tangents[:prob.b],
            prob.centres[N:], prob.tangents[N:])


@pytest.mark.parametrize("shape", [(5, 3, 7, 5, 2), (4, 6, 16, 0, 1), (1, 1, 3, 2, 3)])
def test_far_field_small(tp, shape):
    Nx, Ny, b, Nr, R = shape
    banner(f"far field {shape}")
    prob = sa.make_problem(Nx, Ny, b, Nr, seed=[11, Nx, Ny, b, Nr])
    rng = np.random.default_rng(5)
    I = rng.standard_normal((R, prob.Nt)) + 1j * rng.standard_normal((R, prob.Nt))
    th = np.linspace(-90, 90, 37)
    ph = np.concatenate([np.zeros(19), np.full(18, 45.0)])
    F = tp.far_field(to_dev(I), *geometry_args(prob), np.deg2rad(th), np.deg2rad(ph), prob.k, oracle.ETA0)
    F = F.cpu().numpy()
    for r in range(R):
        Ft, Fp = oracle.far_field(prob.centres, prob.tangents, I[r], th, ph, k=prob.k)
        assert rel_err(F[r, :, 0], Ft) <= 1e-10
        assert rel_err(F[r, :, 1], Fp) <= 1e-10


def test_far_field_config2_cuts(tp):
    """Far field of the solved 32 x 32, b = 64 array on the E- and H-plane cuts
    (181 angles each)."""
    banner("far field 32x32 b64 cuts")
    import torch
    prob, V = sa.make_config(2)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=40, device=torch.device("cuda:0"))
    x, info = plan.solve(to_dev(V), mode="mixed", tol=1e-8)
    assert info[0]["status"] == 0
    th = np.concatenate([np.arange(-90, 91), np.arange(-90, 91)]).astype(np.float64)
    ph = np.concatenate([np.zeros(181), np.full(181, 90.0)])
    F = tp.far_field(x, *geometry_args(prob), np.deg2rad(th), np.deg2rad(ph), prob.k, oracle.ETA0).cpu().numpy()
    Ft, Fp = oracle.far_field(prob.centres, prob.tangents, x.cpu().numpy()[0], th, ph, k=prob.k)
    assert rel_err(F[0, :, 0], Ft) <= 1e-10
    assert rel_err(F[0, :, 1], Fp) <= 1e-10
    plan.close()
