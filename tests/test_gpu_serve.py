"""Continuous-batching server: every result meets the tolerance (FP64 oracle
residual), and each request's solution is the same alone and in the mix
within the tolerance."""
import numpy as np
import pytest

import oracle
from synth import arrays as sa
from helpers import banner, rel_err

pytestmark = pytest.mark.gpu

GEOMS = {}


def problem(key):
    if key not in GEOMS:
        Nx, Ny, b = key
        GEOMS[key] = sa.serving_geometry(Nx, Ny, b, Nr=0)
    return GEOMS[key]


def geometry(key):
    p = problem(key)
    return p.Nx, p.Ny, p.b, p.Nr, p.gen, p.rim_re, p.rim_rr


def make_requests(n, seed, keys):
    from paper_2506_04710_amd.serve import Request
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for i in range(n):
        key = keys[rng.integers(len(keys))]
        p = problem(key)
        R = int(rng.integers(1, 6))
        elems = np.sort(rng.choice(p.Nx * p.Ny, size=R, replace=False))
        t += float(rng.exponential(0.002))
        reqs.append(Request(id=i, t=t, key=key, V=sa.rhs_ports(p, elems)))
    return reqs


@pytest.fixture(scope="module")
def server_cls():
    import torch
    assert torch.cuda.is_available()
    from paper_2506_04710_amd.serve import Server
    return Server


@pytest.mark.parametrize("mode", ["mixed", "fp64"])
def test_serving_mix_matches_alone(server_cls, mode):
    banner(f"serving mix {mode}")
    keys = [(4, 4, 8), (6, 5, 16), (8, 8, 32)]
    reqs = make_requests(14, 5, keys)
    srv = server_cls(geometry, slots=6, mode=mode, tol=1e-8, restart=20, hbm_budget=8 << 30)
    stats = srv.run(reqs, realtime=True)
    assert stats["all_ok"] and stats["max_relres"] <= 1e-8
    for r in reqs:
        p = GEOMS[r.key]
        X = np.stack([x.cpu().numpy() for x in r.X])
        assert np.all(oracle.relres(p, X, r.V) <= 1e-8), r.id
    # The same requests one at a time on a fresh server with the same slot
    # count: every engine step runs the same kernels on a column whatever
    # the other slots hold and whichever slot it sits in (per-column sums in
    # a fixed order), so each result is the same bit for bit.
    alone = server_cls(geometry, slots=6, mode=mode, tol=1e-8, restart=20, hbm_budget=8 << 30)
    for r in reqs[:8]:
        from paper_2506_04710_amd.serve import Request
        r1 = Request(id=r.id, t=0.0, key=r.key, V=r.V)
        alone.run([r1], realtime=False)
        for c in range(r.R):
            assert np.array_equal(r1.X[c].cpu().numpy(), r.X[c].cpu().numpy()), (r.id, c)
            assert r1.info[c]["iters"] == r.info[c]["iters"], (r.id, c)
    srv.close()
    alone.close()
    print(f"serving {mode}: {stats}")


def test_serving_mix_sample_against_oracle(server_cls):
    """The serving workload's own geometries (Nx, Ny in {8, ..., 48}, b in
    {32, 64}, 1-16 ports, mixed + preconditioner, 16 slots): a seeded sample
    of its request stream, chosen to cover every array size and both b, is
    served in one run, and the first port column of every request is checked
    against the oracle's FP64 residual over all rows."""
    banner("serving mix sample vs oracle")
    from paper_2506_04710_amd.serve import Request
    stream = sa.serving_stream(512)
    pick, seen = [], set()
    for r in stream:
        tags = {("n", r["Nx"]), ("n", r["Ny"]), ("b", r["b"])}
        if not tags <= seen:
            pick.append(r)
            seen |= tags
    assert {t[1] for t in seen if t[0] == "n"} == set(sa.SERVE_SIZES)
    assert {t[1] for t in seen if t[0] == "b"} == set(sa.SERVE_B)
    G = {}

    def geom(key):
        if key not in G:
            G[key] = sa.serving_geometry(*key)
        p = G[key]
        return p.Nx, p.Ny, p.b, p.Nr, p.gen, p.rim_re, p.rim_rr

    reqs = []
    for i, r in enumerate(pick):
        key = (r["Nx"], r["Ny"], r["b"])
        geom(key)
        reqs.append(Request(id=r["id"], t=0.002 * i, key=key, V=sa.rhs_ports(G[key], r["elements"])))
    srv = server_cls(geom, slots=16, mode="mixed", tol=1e-8, restart=40, hbm_budget=64 << 30, precond=True)
    stats = srv.run(reqs, realtime=True)
    assert stats["all_ok"], stats
    for r in reqs:
        rr = oracle.relres(G[r.key], r.X[0].cpu().numpy()[None], r.V[:1])[0]
        print(f"request {r.id} {r.key} R={r.R}: oracle relres {rr:.2e}, library {r.info[0]['relres']:.2e}")
        assert rr <= 1e-8, (r.id, r.key, rr)
    srv.close()


def test_serving_hbm_budget_evicts_idle_plans(server_cls):
    """A budget that holds one plan at a time forces eviction between geometries."""
    banner("serving HBM-bounded admission")
    from paper_2506_04710_amd import plan_bytes
    keys = [(4, 4, 8), (5, 4, 8)]
    need = max(plan_bytes(k[0], k[1], k[2], 0, "mixed", 4, 20, symmetric=True) for k in keys)
    reqs = make_requests(6, 7, keys)
    srv = server_cls(geometry, slots=4, mode="mixed", tol=1e-8, restart=20, hbm_budget=int(need * 1.5))
    stats = srv.run(reqs, realtime=False)
    assert stats["all_ok"] and stats["plans_evicted"] >= 1 and stats["hbm_used"] <= need * 1.5
    for r in reqs:
        X = np.stack([x.cpu().numpy() for x in r.X])
        assert np.all(oracle.relres(GEOMS[r.key], X, r.V) <= 1e-8)
    srv.close()


def test_batch_api_direct():
    """Admit, step, poll and release one column by hand; argument errors and a
    plain solve during an active batch are refused."""
    banner("batch API direct")
    import ctypes
    import torch
    import paper_2506_04710_amd as tp
    from paper_2506_04710_amd import _lib
    L = _lib.lib()
    p = problem((4, 4, 8))
    plan = tp.Plan.from_problem(p, prec="mixed", max_rhs=3, restart=20, device=torch.device("cuda:0"))
    o = _lib.SolveOpts()
    L.toeplitz_solve_opts_default(ctypes.byref(o))
    o.restart, o.mode, o.tol = 20, _lib.PREC["mixed"], 1e-9
    V = sa.rhs_ports(p, [5])
    v = torch.from_numpy(V[0]).cuda()
    x = torch.empty_like(v)
    vp = ctypes.c_void_p
    sh = vp(torch.cuda.current_stream().cuda_stream)
    phases = (ctypes.c_int * 3)()
    infos = (_lib.SolveInfo * 3)()
    # no batch yet
    assert L.toeplitz_batch_admit(plan._h, 0, vp(v.data_ptr()), vp(x.data_ptr()), 1e-9, 0, sh) == _lib.TP_E_INVAL
    assert L.toeplitz_batch_step(plan._h, 1) == _lib.TP_E_INVAL
    _lib.check(L.toeplitz_batch_begin(plan._h, ctypes.byref(o)))
    assert L.toeplitz_batch_poll(plan._h, 0, 1, phases, infos) == _lib.TP_E_INVAL   # nothing stepped
    assert L.toeplitz_batch_admit(plan._h, 3, vp(v.data_ptr()), vp(x.data_ptr()), 1e-9, 0, sh) == _lib.TP_E_INVAL
    assert L.toeplitz_batch_admit(plan._h, 0, None, vp(x.data_ptr()), 1e-9, 0, sh) == _lib.TP_E_INVAL
    assert L.toeplitz_batch_admit(plan._h, 0, vp(v.data_ptr()), vp(x.data_ptr()), 0.0, 0, sh) == _lib.TP_E_INVAL
    assert L.toeplitz_batch_step(plan._h, 0) == _lib.TP_E_INVAL
    with pytest.raises(_lib.ToeplitzError):
        plan.solve(v)
    # applications share the engine's workspace: refused while it runs
    for which in ("fp64", "mixed"):
        with pytest.raises(_lib.ToeplitzError) as ei:
            plan.matvec(v, which=which)
        assert ei.value.status == _lib.TP_E_INVAL
    with pytest.raises(_lib.ToeplitzError) as ei:
        plan.precond_create()
    assert ei.value.status == _lib.TP_E_INVAL
    _lib.check(L.toeplitz_batch_admit(plan._h, 1, vp(v.data_ptr()), vp(x.data_ptr()), 1e-9, 0, sh))
    done = False
    for _ in range(200):
        _lib.check(L.toeplitz_batch_step(plan._h, 1))
        _lib.check(L.toeplitz_batch_poll(plan._h, 0, 1, phases, infos))
        assert phases[0] == 0 and phases[2] == 0            # never admitted: idle
        if phases[1] == 2:
            done = True
            break
        assert phases[1] == 1
    assert done and infos[1].status == 0 and infos[1].relres <= 1e-9
    _lib.check(L.toeplitz_batch_release(plan._h, 1))
    _lib.check(L.toeplitz_batch_step(plan._h, 1))
    _lib.check(L.toeplitz_batch_poll(plan._h, 0, 1, phases, infos))
    assert list(phases) == [0, 0, 0]
    assert oracle.relres(p, x.cpu().numpy()[None], V)[0] <= 1e-9
    _lib.check(L.toeplitz_batch_end(plan._h))
    # after the batch a plain solve works again and agrees
    x2, inf = plan.solve(v, tol=1e-9, restart=20)
    assert inf[0]["status"] == 0
    assert rel_err(x2.cpu().numpy(), x.cpu().numpy()) <= 1e-7
    plan.close()
