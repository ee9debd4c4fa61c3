"""Benchmark: solves per second at relative residual 1e-8 on the 32 x 32 array
(b = 64 basis functions per element, 256 rim functions, N = 65,536 + 256),
broadside plane-wave excitation, on one MI355X.

One step = one complete solve of Z x = v to ||v - Z x|| / ||v|| <= 1e-8
(FP64 residual), in the fastest form (the rim as placed channels of the
element cells, FP32 operator and block-circulant preconditioner inside FP64
iterative refinement, all Krylov arithmetic FP64, launch options tuned), with
the plan (extended generator spectrum, preconditioner) resident in HBM and the
right-hand side on the device.  The same GPU's plain FP64 GMRES is
timed beside it ("vs FP64 plain"), together with the operator's achieved
bandwidth, per-solve latency percentiles, the roofline fraction of the
dominant kernel and the plain FP64 CPU oracle on a bounded sample.  Unless
--quick: the 81-port multi-RHS solve (matrix-core product rate, S-matrix),
the 1e-10 precision workload and the 512-request serving stream.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--quick]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/s at rel-residual 1e-8 (32x32,b=64) vs FP64 plain; matvec GB/s; p99 latency"

# HBM traffic of the dominant kernel per launch, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by the same counters on a plain copy of known size),
# valid only for the kernel source it was measured on.
TRAFFIC = {"source_sha256": "78202dab81867be606c19762180f122cb00569385868bf97884cf975968218cd",
           "bytes": 105737075, "fetch_factor": 0.416678, "write_factor": 1.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--quick", action="store_true",
                    help="headline workload only (no multi-RHS, precision or serving sections)")
    ap.add_argument("--solves-only", action="store_true",
                    help="only the headline solves (warmup + steps), for a kernel trace of the solve alone")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device-to-device copies of MIB MiB (HBM counter calibration)")
    ap.add_argument("--apply-only", choices=["mixed", "fp32", "fp64", "precond", "multi"], default=None,
                    help="only 20 applications of one operator form on the headline plan (precond: the FP32 "
                         "preconditioner on complex128 vectors; multi: the FP32 operator on the 81 port columns "
                         "of the 9x9 array), for kernel traces and counters")
    ap.add_argument("--tune-only", action="store_true",
                    help="only tune the headline plan's launch options (placed rim, preconditioner) into the "
                         "cache, so that later runs, profiled or not, take the same choice")
    ap.add_argument("--placed", action="store_true",
                    help="with --solves-only / --apply-only: the plan with the rim as placed channels")
    return ap.parse_args()


def copy_calibration(mib):
    """Plain copies of known size: the reference for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) read on the operator's kernels."""
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)       # an elementwise kernel: reads n bytes, writes n bytes
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "copies": 5}), flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("tp_matvec.h", "tp_apply_wide.hip", "tp_fft.h", "tp_common.h"):
        with open(os.path.join(ROOT, "paper_2506_04710_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def spectrum_blocks(prob, half):
    """Spectrum blocks a matvec must read, at the minimal embedding
    (2Nx-1)(2Ny-1): all of them, or for symmetric generators (Ghat(-k) =
    Ghat(k)^T) the columns kx < Nx only."""
    return (prob.Nx if half else 2 * prob.Nx - 1) * (2 * prob.Ny - 1)


def algorithmic_bytes(prob, R, s, half):
    """Bytes a matvec must move: spectrum + rim (one pass) + C + vectors in/out."""
    return s * (spectrum_blocks(prob, half) * prob.b ** 2 + prob.Nr * prob.N + prob.Nr ** 2 + 2 * prob.Nt * R)


def spec_rim_bytes(prob, Px, s, half, sv=None):
    """Algorithmic bytes of one launch of the fused spectrum+rim kernel: the
    spectrum stream, the rim block, the x-transformed input grid and the
    output grid (rows iy < Ny), all of s bytes per value, and x_A in and the
    rim term out, of sv bytes per value (the solve's FP32 operator works on
    complex128 vectors: s = 8, sv = 16)."""
    sv = s if sv is None else sv
    grid = prob.Ny * Px * prob.b
    return s * (spectrum_blocks(prob, half) * prob.b ** 2 + prob.Nr * prob.N + 2 * grid) + sv * 2 * prob.N


def cpu_model():
    """CPU model name and the threads this process may use (the GPU machine's host)."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def cpu_baseline(prob, V, lu_shape=(8, 8)):
    """The plain FP64 oracle on the host cores: the headline operator's dense
    matvec (on-the-fly rows, every row) on all threads and on one thread, and
    a dense GEPP solve at the largest size run here (the same generators on an
    lu_shape sub-array, n = lu_shape[0] lu_shape[1] b unknowns).  The oracle
    has no iterative solver: its solve is the LU, so its solves/s at the full
    size is the measured LU time scaled by (Nt / n)^3 (labelled as such)."""
    import oracle
    from synth import arrays as sa
    cores = oracle.max_threads()
    model, nproc = cpu_model()
    t0 = time.perf_counter()
    oracle.matvec(prob, V)
    t_mv = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.matvec(prob, V, nthreads=1)
    t_mv1 = time.perf_counter() - t0
    sub, Vs = sa.make_config(2, reduced=dict(Nx=lu_shape[0], Ny=lu_shape[1], Nr=0))
    Z = oracle.assemble(sub)
    n = Z.shape[0]
    t0 = time.perf_counter()
    oracle.lu_solve(Z, Vs)
    t_lu = time.perf_counter() - t0
    t_full = t_lu * (prob.Nt / n) ** 3
    return {
        "value": 1.0 / t_full, "unit": "solves/s", "cores": cores, "kind": "oracle",
        "sample": f"dense FP64 matvec of the headline operator over all {prob.Nt} rows, measured: {t_mv:.2f} s on "
                  f"{cores} threads, {t_mv1:.2f} s on 1 thread; GEPP LU + solve measured at n={n} (the same "
                  f"generators on a {lu_shape[0]}x{lu_shape[1]} sub-array): {t_lu:.2f} s on {cores} threads; value "
                  f"= that LU time scaled by (Nt/n)^3 to Nt={prob.Nt} ({t_full / 3600:.1f} h per solve, "
                  f"extrapolated, not run)",
        "matvec_s_all_threads": round(t_mv, 3), "matvec_s_1_thread": round(t_mv1, 3),
        "lu_n": n, "lu_s_measured": round(t_lu, 3), "cpu_model": model, "nproc": nproc,
    }


def timed_solves(plan, v, K, W, tol=1e-8, **kw):
    """K timed solves after W warm-up ones; each returns after convergence."""
    import numpy as np
    import torch
    for _ in range(W):
        plan.solve(v, tol=tol, **kw)
    torch.cuda.synchronize()
    lat, last = [], None
    t_start = time.perf_counter()
    for _ in range(K):
        ts = time.perf_counter()
        last = plan.solve(v, tol=tol, **kw)
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    return time.perf_counter() - t_start, np.array(lat), last


def _whole_us(plan, x, which, n=20):
    """Mean microseconds of n operator applications back to back between two events."""
    import torch
    plan.matvec(x, which=which)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n):
        plan.matvec(x, which=which)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n * 1e3


def multi_rhs(dev, K=3):
    """81 port excitations of the 9 x 9, b = 96 array solved together, the
    matrix-core product's rate, the persistent launch, the placed-rim form and
    the S-matrix post-step."""
    import numpy as np
    import torch
    import paper_2506_04710_amd as tp
    from paper_2506_04710_amd import _lib, tune
    from synth import arrays as sa
    prob, V = sa.make_config(3)
    R = V.shape[0]
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=40, device=dev).precond_create()
    tuned = tune.tune(plan, "mixed", R)
    v = torch.from_numpy(V).to(dev)
    total, lat, (x, inf) = timed_solves(plan, v, K, 1, mode="mixed", precond=True)
    assert all(i["status"] == 0 and i["relres"] <= 1e-8 for i in inf), inf
    st = plan.matvec_profile(v.to(torch.complex64), which="fp32", reps=20)
    # algorithmic work at the minimal embedding (2Nx - 1)(2Ny - 1) = 17 x 17,
    # not the padded 18 x 18 grid the kernels run on
    Pa = (2 * prob.Nx - 1) * (2 * prob.Ny - 1)
    flops = 8.0 * Pa * prob.b ** 2 * R
    flops_rim = 16.0 * prob.Nr * prob.N * R + 8.0 * prob.Nr ** 2 * R
    xv = v.to(torch.complex64)
    path = sorted(plan.path("fp32", R))
    whole_us = _whole_us(plan, xv, "fp32")
    # the product launch alone (separate launches), and the persistent launch
    keep_multi = plan.get_option(_lib.TP_OPT_MULTI_FUSED)
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 0)
    prod_us = plan.stage_time(xv, 3, "fp32", reps=50) * 1e3
    sep_us = _whole_us(plan, xv, "fp32")
    keep_lds = plan.get_option(_lib.TP_OPT_PROD_LDS)
    keep_cols = plan.get_option(_lib.TP_OPT_MFMA_COLS)
    plan.set_option(_lib.TP_OPT_PROD_LDS, 0)
    plan.set_option(_lib.TP_OPT_MFMA_COLS, 0)
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, 1)
    persistent_us = _whole_us(plan, xv, "fp32") if "persistent" in plan.path("fp32", R) else None
    plan.set_option(_lib.TP_OPT_MULTI_FUSED, keep_multi)
    plan.set_option(_lib.TP_OPT_PROD_LDS, keep_lds)
    plan.set_option(_lib.TP_OPT_MFMA_COLS, keep_cols)
    rows = np.nonzero(V)[1]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = tp.port_smatrix(x, rows, Z0=50.0)
    t_s = time.perf_counter() - t0
    S = S.cpu().numpy()
    plan.close()
    # the same ports with the rim placed as channels of the element cells
    place, nrc = sa.rim_placement(prob)
    pplan = tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                           max_rhs=R, restart=40, device=dev, rim_place=(place, nrc)).precond_create()
    ptuned = tune.tune(pplan, "mixed", R)
    ptotal, _, (px, pinf) = timed_solves(pplan, v, K, 1, mode="mixed", precond=True)
    assert all(i["status"] == 0 and i["relres"] <= 1e-8 for i in pinf), pinf
    pwhole = _whole_us(pplan, xv, "fp32")
    bc = pplan.info()["bc"]
    pflops = 8.0 * Pa * bc ** 2 * R
    pplan.close()
    out = {"workload": "9x9 array, b=96, 72 rim functions, 81 port excitations (one per element feed), tol 1e-8, "
                       "mixed + preconditioner, one launch sequence for all columns",
           "solves_per_s": round(R * K / total, 1), "ms_per_81": round(1e3 * total / K, 2),
           "iters_max": max(i["iters"] for i in inf), "outer_max": max(i["outer_iters"] for i in inf),
           "fp32_matvec_stages_us": {k: round(t * 1e3, 2) for k, t in st.items()},
           "tuned": {k: tuned[k] for k in ("mfma_cols", "multi_fused", "prod_lds", "fft2_lds", "candidates")},
           "path": path,
           "prod_mfma": {"us": round(prod_us, 2), "tflops": round(flops / (prod_us * 1e-6) / 1e12, 1),
                         "peak_tflops_fp32_mfma": 157.3,
                         "frac": round(flops / (prod_us * 1e-6) / 1e12 / 157.3, 3),
                         "flops_per_launch": flops, "grid": "algorithmic 17x17",
                         "timing": "launch repeated back to back between two events"},
           "whole_matvec": {"us": round(whole_us, 2), "flops": flops + flops_rim,
                            "frac_fp32_mfma": round((flops + flops_rim) / (whole_us * 1e-6) / 1e12 / 157.3, 3),
                            "separate_launches_us": round(sep_us, 2),
                            "persistent_launch_us": None if persistent_us is None else round(persistent_us, 2),
                            "timing": "20 applications back to back between two events"},
           "placed_rim": {"channels_per_cell": bc, "solves_per_s": round(R * K / ptotal, 1),
                          "ms_per_81": round(1e3 * ptotal / K, 2),
                          "iters_max": max(i["iters"] for i in pinf),
                          "whole_matvec_us": round(pwhole, 2), "flops": pflops,
                          "frac_fp32_mfma": round(pflops / (pwhole * 1e-6) / 1e12 / 157.3, 3),
                          "tuned": {k: ptuned[k] for k in ("mfma_cols", "multi_fused", "prod_lds", "fft2_lds")}},
           "smatrix_ms": round(1e3 * t_s, 2), "smatrix_max_asymmetry": float(np.abs(S - S.T).max())}
    return out


def precision(dev, K=2):
    """Eight scan-angle plane waves on the 64 x 64, b = 48 array to 1e-10:
    mixed + preconditioner against the FP64 preconditioned solve."""
    import numpy as np
    import torch
    import paper_2506_04710_amd as tp
    from synth import arrays as sa
    prob, V = sa.make_config(4)
    R = V.shape[0]
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=R, restart=40, device=dev).precond_create()
    v = torch.from_numpy(V).to(dev)
    total, _, (x, inf) = timed_solves(plan, v, K, 1, tol=1e-10, mode="mixed", precond=True)
    assert all(i["status"] == 0 and i["relres"] <= 1e-10 for i in inf), inf
    total64, _, (x64, inf64) = timed_solves(plan, v, K, 1, tol=1e-10, mode="fp64", precond=True)
    err = (torch.linalg.norm(x - x64, dim=1) / torch.linalg.norm(x64, dim=1)).max().item()
    plan.close()
    return {"workload": "64x64 array, b=48, no rim, 8 plane waves (theta in 0..60 deg), tol 1e-10",
            "mixed_solves_per_s": round(R * K / total, 1), "fp64_solves_per_s": round(R * K / total64, 1),
            "iters_max": max(i["iters"] for i in inf), "outer_max": max(i["outer_iters"] for i in inf),
            "max_relres": max(i["relres"] for i in inf), "max_rel_diff_vs_fp64": err}


def headline_plan(tp, prob, placed, max_rhs=1, device="cuda:0"):
    """The headline plan: dense rim blocks, or the rim as placed channels."""
    from synth import arrays as sa
    kw = {"rim_place": sa.rim_placement(prob)} if placed else {}
    return tp.Plan.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, prec="mixed",
                          max_rhs=max_rhs, restart=40, device=device, **kw)


def progress(msg):
    """A progress line on stderr (the JSON result stays the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def tune_only():
    """Tune the headline plan (placed rim, preconditioner, mixed, one column)
    and the multi-RHS plan, and print the records."""
    import torch
    import paper_2506_04710_amd as tp
    from paper_2506_04710_amd import tune
    from synth import arrays as sa
    tp.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob, _ = sa.make_config(2)
    plan = headline_plan(tp, prob, True).precond_create()
    rec = tune.tune(plan, "mixed", 1)
    plan.close()
    # the multi-RHS plan of --apply-only multi (9 x 9, b = 96, 81 columns)
    prob3, V3 = sa.make_config(3)
    plan3 = tp.Plan.from_problem(prob3, prec="mixed", max_rhs=V3.shape[0], restart=4).precond_create()
    rec3 = tune.tune(plan3, "mixed", V3.shape[0])
    plan3.close()
    print(json.dumps({"tune": rec, "tune_multi": rec3}), flush=True)


def apply_only(which, placed, K=20):
    """K applications of one operator form on the headline plan (kernel traces
    and HBM counters of its launches): mixed / fp32 / fp64 operator, the FP32
    preconditioner on complex128 vectors, or the FP32 operator on the 81 port
    columns of the 9 x 9 array (multi)."""
    import torch
    import paper_2506_04710_amd as tp
    from synth import arrays as sa
    tp.load()
    if which == "multi":
        from paper_2506_04710_amd import tune
        prob, V = sa.make_config(3)
        plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=V.shape[0], restart=4).precond_create()
        progress(f"tuning: {tune.tune(plan, 'mixed', V.shape[0])}")
        xv = torch.from_numpy(V).to("cuda:0").to(torch.complex64)
        for _ in range(K):
            plan.matvec(xv, which="fp32")
    else:
        from paper_2506_04710_amd import tune
        prob, V = sa.make_config(2)
        plan = headline_plan(tp, prob, placed)
        dt = torch.complex64 if which == "fp32" else torch.complex128
        xv = torch.from_numpy(V).to("cuda:0").to(dt)
        # the headline plan's preconditioner and launch options (the same
        # tuning key as the headline solve), so the operator runs its kernels
        if placed or which == "precond":
            plan.precond_create()
            progress(f"tuning: {tune.tune(plan, 'mixed', 1)}")
        if which == "precond":
            for _ in range(K):
                plan.precond_apply(xv, which="mixed")
        else:
            for _ in range(K):
                plan.matvec(xv, which=which)
    torch.cuda.synchronize()
    print(json.dumps({"apply_only": which, "placed": placed, "applications": K}), flush=True)
    plan.close()


def solves_only(K, W, placed=False):
    """The headline solve alone (mixed + preconditioner, one RHS), K timed after W."""
    import torch
    import paper_2506_04710_amd as tp
    from synth import arrays as sa
    tp.load()
    prob, V = sa.make_config(2)
    plan = headline_plan(tp, prob, placed).precond_create()
    from paper_2506_04710_amd import tune
    rec = tune.tune(plan, "mixed", 1)
    progress(f"tuning: {rec}")
    v = torch.from_numpy(V).to("cuda:0")
    total, _, (_, inf) = timed_solves(plan, v, K, W, mode="mixed", precond=True)
    assert inf[0]["status"] == 0 and inf[0]["relres"] <= 1e-8, inf
    print(json.dumps({"solves_per_s": round(K / total, 2), "steps": K, "warmup": W, "iters": inf[0]["iters"],
                      "outer": inf[0]["outer_iters"], "placed": placed}), flush=True)
    plan.close()


def schur(dev, K):
    """The headline workload solved through the rim's Schur complement: setup
    (F = A^-1 B_er, S = C - B F, S^-1) once, then K solves of one RHS."""
    import torch
    import paper_2506_04710_amd as tp
    from synth import arrays as sa
    prob, V = sa.make_config(2)
    plan = tp.Plan.from_problem(prob, prec="mixed", max_rhs=1, restart=40, device=dev).precond_create()
    elem = tp.Plan.create(prob.Nx, prob.Ny, prob.b, 0, prob.gen, prec="mixed", max_rhs=16, restart=40,
                          device=dev).precond_create()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.schur_create(elem, mode="mixed", tol=1e-10, precond=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    v = torch.from_numpy(V).to(dev)
    for _ in range(2):
        plan.schur_solve(v, tol=1e-8, precond=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        x, inf = plan.schur_solve(v, tol=1e-8, precond=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    assert inf[0]["status"] == 0 and inf[0]["relres"] <= 1e-8, inf
    xd, _ = plan.solve(v, tol=1e-8, mode="mixed", precond=True)
    diff = (torch.linalg.norm(x - xd) / torch.linalg.norm(xd)).item()
    plan.close()
    elem.close()
    return {"workload": "32x32 array, b=64, 256 rim functions, broadside plane wave, tol 1e-8; rim eliminated "
                        "through C - B A^-1 B_er, element solves mixed + preconditioner",
            "setup_s": round(t_setup, 3), "solves_per_s": round(K / total, 2), "iters": inf[0]["iters"],
            "outer": inf[0]["outer_iters"], "relres": inf[0]["relres"], "rel_diff_vs_direct": diff}


def serving(dev, n_requests=512):
    """Seeded Poisson stream of 512 requests over the serving mix of geometries
    (the arrival rate is not given by the paper): the continuous-batching
    server (mixed + preconditioner, 16 slots per plan) at saturation, then the
    same stream re-timed to 0.5x and 0.9x of that saturation rate; the same
    stream through a plain FP64 single-RHS server (one slot per plan, no
    preconditioner) at saturation; and the batched server under an HBM budget
    small enough to force admission waits and evictions."""
    import torch
    from paper_2506_04710_amd.serve import Server, Request
    from synth import arrays as sa
    base_rate = 100.0
    stream = sa.serving_stream(n_requests, rate_hz=base_rate)
    keys = sorted({(r["Nx"], r["Ny"], r["b"]) for r in stream})
    G = {k: sa.serving_geometry(*k) for k in keys}

    def geometry(k):
        p = G[k]
        return p.Nx, p.Ny, p.b, p.Nr, p.gen, p.rim_re, p.rim_rr

    def reqs(rate=None):
        scale = 1.0 if rate is None else base_rate / rate
        return [Request(id=r["id"], t=r["t"] * scale, key=(r["Nx"], r["Ny"], r["b"]),
                        V=sa.rhs_ports(G[(r["Nx"], r["Ny"], r["b"])], r["elements"])) for r in stream]

    keep = ("requests", "columns", "wall_s", "requests_per_s", "solves_per_s", "p50_ms", "p99_ms", "max_relres",
            "all_ok", "plans_created", "plans_evicted")
    rnd = lambda d: {k: (round(d[k], 4) if isinstance(d.get(k), float) and k != "max_relres" else d.get(k))
                     for k in keep + (("error",) if "error" in d else ())}
    srv = Server(geometry, slots=16, mode="mixed", tol=1e-8, restart=40, hbm_budget=160 << 30, precond=True,
                 device=dev)
    t0 = time.perf_counter()
    srv.warm(keys)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    hbm_all = srv.used
    sat = srv.run(reqs(), realtime=False)
    lam = sat["requests_per_s"]
    progress(f"serving saturation: {lam:.1f} requests/s")
    at = {f"{f}x_saturation": rnd(dict(srv.run(reqs(f * lam), realtime=True), offered_rate=round(f * lam, 1)))
          for f in (0.5, 0.9)}
    srv.close()
    # plain FP64, one right-hand side at a time per geometry
    plain = Server(geometry, slots=1, mode="fp64", tol=1e-8, restart=40, hbm_budget=160 << 30, precond=False,
                   device=dev)
    plain.warm(keys)
    torch.cuda.synchronize()
    sat64 = plain.run(reqs(), realtime=False)
    plain.close()
    progress(f"plain FP64 single-RHS server: {sat64['wall_s']:.1f} s")
    # HBM pressure: a budget of half what every plan warm needs (at least 1.5x
    # the largest single plan, so that every request can be admitted): plans
    # are created on demand, requests wait for memory, idle plans are evicted
    tight = Server(geometry, slots=16, mode="mixed", tol=1e-8, restart=40, hbm_budget=hbm_all // 2, precond=True,
                   device=dev)
    tight.budget = max(tight.budget, int(1.5 * max(tight._need(k) for k in keys)))
    try:
        press = tight.run(reqs(), realtime=False, max_seconds=120.0,
                          progress=lambda d, n, t: progress(f"budgeted serving: {d}/{n} requests at {t:.1f} s, "
                                                            f"{tight.stats['plans_created']} plans created"))
    except RuntimeError as ex:
        press = {k: None for k in keep}
        press["error"] = str(ex)
    tight.close()
    progress("serving under an HBM budget done")
    return {"workload": f"{n_requests} requests, Poisson arrivals (seeded), {len(keys)} geometries (Nx, Ny in "
                        "{8..48}, b in {32, 64}), 1-16 ports each, tol 1e-8",
            "batched": "mixed + preconditioner, 16 slots per plan, continuous batching",
            "plans_warm_s": round(t_warm, 2), "hbm_all_plans_gib": round(hbm_all / 2 ** 30, 2),
            "saturation": rnd(sat), **at,
            "fp64_plain_single_rhs_saturation": rnd(sat64),
            "speedup_vs_fp64_plain_single_rhs": round(sat["solves_per_s"] / sat64["solves_per_s"], 2),
            "hbm_budget_saturation": dict(rnd(press), budget_gib=round(tight.budget / 2 ** 30, 2),
                                          note="plans created on demand, idle plans evicted")}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              f"documented but not built", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.solves_only:
        solves_only(args.steps, args.warmup, args.placed)
        return
    if args.apply_only:
        apply_only(args.apply_only, args.placed)
        return
    if args.tune_only:
        tune_only()
        return
    import numpy as np
    import torch
    import paper_2506_04710_amd as tp
    from synth import arrays as sa

    tp.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    from paper_2506_04710_amd import tune
    prob, V = sa.make_config(2)
    # headline plan: the rim as placed channels of the element cells (one
    # extended spectrum, no dense B or C), its preconditioner, tuned options
    t0 = time.perf_counter()
    plan = headline_plan(tp, prob, True, device=dev)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan.precond_create()
    t_pc = time.perf_counter() - t0
    t0 = time.perf_counter()
    tuned = tune.tune(plan, "mixed", 1)
    t_tune = time.perf_counter() - t0
    progress(f"headline plan, preconditioner and tuning: {tuned}")
    info = plan.info()
    Px, Py, bc = info["Px"], info["Py"], info["bc"]
    half = bool(info["half_spectrum"])       # symmetric generators: half the spectrum is stored
    v = torch.from_numpy(V).to(dev)

    # headline: the fastest form (FP32 operator and preconditioner inside FP64
    # refinement) on the headline plan; then the same GPU's plain FP64 GMRES on
    # a plan with the dense rim blocks (no structure beyond the element
    # Toeplitz blocks, no preconditioner), and intermediate forms
    total, lat, (x, inf) = timed_solves(plan, v, args.steps, args.warmup, mode="mixed", precond=True)
    assert inf[0]["status"] == 0 and inf[0]["relres"] <= 1e-8, inf
    progress(f"headline solves: {args.steps / total:.1f}/s")
    dense = headline_plan(tp, prob, False, device=dev)
    total64, lat64, (_, inf64) = timed_solves(dense, v, args.steps, args.warmup, mode="fp64")
    assert inf64[0]["status"] == 0 and inf64[0]["relres"] <= 1e-8, inf64
    kb = max(3, args.steps // 3)
    dense.precond_create()
    totd, _, (_, infd) = timed_solves(dense, v, kb, 1, mode="mixed", precond=True)
    dense.close()
    del dense
    totm, _, (_, infm) = timed_solves(plan, v, kb, 1, mode="mixed")
    totp, _, (_, infp) = timed_solves(plan, v, kb, 1, mode="fp64", precond=True)
    tot64s, _, (_, inf64s) = timed_solves(plan, v, kb, 1, mode="fp64")

    # operator bandwidth (whole matvec) and the dominant kernel's duration.
    # Every timed application follows a 512 MB read that evicts the operator
    # from the 256 MB MALL with clean lines (a write would leave dirty lines
    # whose write-back lands in the timed region); the back-to-back figure is
    # reported beside it as "warm".
    flush = torch.ones(128 << 20, dtype=torch.float32, device=dev)
    sblk = (prob.Nx if half else 2 * prob.Nx - 1) * (2 * prob.Ny - 1)      # stored blocks at 2N - 1
    gbs = {}
    stage = {}
    stage_warm = {}
    # mixed: the FP32 operator on complex128 vectors, the instance the solve runs
    for which, dt, s, sv in (("mixed", torch.complex128, 8, 16), ("fp32", torch.complex64, 8, 8),
                             ("fp64", torch.complex128, 16, 16)):
        xv = v.to(dt)
        for _ in range(3):
            plan.matvec(xv, which=which)
        torch.cuda.synchronize()
        reps = 30
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            flush.sum()
            e0.record()
            plan.matvec(xv, which=which)
            e1.record()
        torch.cuda.synchronize()
        ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            plan.matvec(xv, which=which)
        ev1.record()
        torch.cuda.synchronize()
        ms_warm = ev0.elapsed_time(ev1) / reps
        # what the placed operator must move: its stored extended spectrum and
        # the vectors in and out
        nb = s * sblk * bc * bc + sv * 2 * prob.Nt
        gbs[which] = {"us": round(ms * 1e3, 2), "GB_s": round(nb / (ms * 1e-3) / 1e9, 1),
                      "us_warm": round(ms_warm * 1e3, 2), "GB_s_warm": round(nb / (ms_warm * 1e-3) / 1e9, 1),
                      "bytes": int(nb)}
        cold = []
        for _ in range(reps):
            flush.sum()
            cold.append(plan.matvec_profile(xv, which=which, reps=1))
        stage[which] = {k: sum(c[k] for c in cold) / reps for k in cold[0]}
        stage_warm[which] = plan.matvec_profile(xv, which=which, reps=50)
    del flush
    progress("operator timings done")
    # dominant kernel of the timed solve: the pair-stream launch of the FP32
    # extended spectrum (k_pair_prod<float>; the preconditioner launches the
    # same kernel on its inverted blocks); its duration from HIP events recorded
    # on the stream it is launched on, after the MALL flush.  Its bytes: the
    # stored blocks and the transformed grid in and out.
    pair = tuned["spectrum_pass"] == 2
    # launch duration: the launch repeated back to back between two events on
    # its stream (no event between the repeats); the per-stage intervals of
    # matvec_profile carry an event's own few microseconds each
    k_ms = plan.stage_time(v, 3, "mixed", reps=100)
    k_ms_cold = stage["mixed"]["prod"]
    k_bytes = 8 * (sblk * bc * bc + 2 * (2 * prob.Nx - 1) * (2 * prob.Ny - 1) * bc)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    sha = kernel_source_sha()
    traffic = TRAFFIC["bytes"] if TRAFFIC["source_sha256"] == sha else None
    plan.close()
    del plan

    line = {
        "metric": METRIC,
        "value": round(args.steps / total, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 operator and preconditioner, f64 refinement/Krylov",
        "data": "synthetic",
        "config": {"workload": "32x32 array, b=64, 256 rim functions (N=65,536, Nt=65,792), broadside plane "
                               "wave, tol 1e-8, one RHS", "Nx": 32, "Ny": 32, "b": 64, "Nr": 256,
                   "grid": [Px, Py], "restart": 40, "rim": f"placed, {bc - prob.b} channels per cell",
                   "solve": "mixed GMRES-IR, right block-circulant preconditioner",
                   "tuned": {k: tuned[k] for k in ("spectrum_pass", "source")}},
        "fp64_plain_solves_per_s": round(args.steps / total64, 2),
        "speedup_vs_fp64_plain": round(total64 / total, 3),
        "other_forms_solves_per_s": {"mixed_no_precond": round(kb / totm, 2), "fp64_precond": round(kb / totp, 2),
                                     "fp64_plain_on_placed_plan": round(kb / tot64s, 2),
                                     "dense_rim_mixed_precond": round(kb / totd, 2)},
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 3),
                       "fp64_plain_p50": round(1e3 * float(np.percentile(lat64, 50)), 3),
                       "fp64_plain_p99": round(1e3 * float(np.percentile(lat64, 99)), 3)},
        "iters": {"mixed_precond": inf[0]["iters"], "mixed_precond_outer": inf[0]["outer_iters"],
                  "fp64_plain": inf64[0]["iters"], "mixed_no_precond": infm[0]["iters"],
                  "fp64_precond": infp[0]["iters"], "dense_rim_mixed_precond": infd[0]["iters"]},
        "relres": {"mixed_precond": inf[0]["relres"], "fp64_plain": inf64[0]["relres"]},
        "matvec": gbs,
        "matvec_stages_us": {w: {k: round(v_ * 1e3, 2) for k, v_ in st.items()} for w, st in stage.items()},
        "matvec_stages_us_warm": {w: {k: round(v_ * 1e3, 2) for k, v_ in st.items()} for w, st in stage_warm.items()},
        "plan_create_s": round(t_plan, 3),
        "precond_create_s": round(t_pc, 3),
        "tune_s": round(t_tune, 3),
        "roofline": {"kernel": ("k_pair_prod<float, 9> (pair stream over the stored half of the extended "
                                "spectrum, 72 x 72 blocks)") if pair else
                               "k_spec_rim<float, cpx<double>, cpx<double>, 9, 1, 0, false, true, 256> (fused "
                               "spectrum-only pass over the extended spectrum)",
                     "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(k_bytes), "launch_us": round(k_ms * 1e3, 2),
                     "launch_us_event_interval_after_mall_flush": round(k_ms_cold * 1e3, 2),
                     "note": "launch_us: the launch repeated 100 times back to back between two HIP events on its "
                             "stream (toeplitz_stage_time); the second figure is the interval between events "
                             "recorded right before and after one launch, after a 512 MB read that evicts the "
                             "256 MB MALL (it includes the events' own overhead)"},
    }
    if not args.quick:
        line["multi_rhs"] = multi_rhs(dev)
        progress("multi-RHS done")
        line["precision"] = precision(dev)
        progress("precision done")
        line["serving"] = serving(dev)
        progress("serving done")
        line["schur"] = schur(dev, args.steps)
        progress("rim elimination done")
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(prob, V)
        progress("CPU oracle done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
