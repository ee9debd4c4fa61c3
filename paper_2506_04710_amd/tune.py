"""Launch-option tuning with a JSON cache.

The library's tuner (toeplitz_tune) times the kernel variants that change a
plan's work at a column count and sets the fastest.  This module keys its
choices by device, ROCm/HIP version, plan shape, precision and a bucket of the
column count, stores them in a JSON file, and on a later plan of the same key
sets the stored options without timing again.

    from paper_2506_04710_amd import tune
    tune.tune(plan, which="mixed", nrhs=1)   # after plan.precond_create(), if any

The cache file is $TOEPLITZ_TUNE_CACHE, else
~/.cache/paper_2506_04710_amd/tune.json.  Tune without a profiler attached: a
kernel-trace profiler adds a cost per dispatch and so favours the variants
with fewer launches; a later profiled run then takes the stored choice.
"""
from __future__ import annotations

import ctypes
import json
import os

from . import _lib
from ._lib import PREC, check

_BUCKETS = (1, 2, 8, 16, 32, 64, 128)


def cache_path() -> str:
    return os.environ.get("TOEPLITZ_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2506_04710_amd", "tune.json")


def _bucket(nrhs: int) -> int:
    b = 1
    for v in _BUCKETS:
        if nrhs >= v:
            b = v
    return b


def device_key(device) -> str:
    """Architecture, compute-unit count and HIP version (not the marketing
    name: it is empty in some environments, e.g. under a profiler)."""
    import torch
    props = torch.cuda.get_device_properties(device)
    arch = getattr(props, "gcnArchName", "")
    return f"{arch}|cu{props.multi_processor_count}|hip {torch.version.hip}"


def plan_key(plan, which: str, nrhs: int) -> str:
    d = plan.info()
    pre = 1 if getattr(plan, "pbuf", None) is not None else 0
    return (f"{d['Nx']}x{d['Ny']} b{d['b']} nr{d['Nr']} nrc{d['nrc']} grid{d['Px']}x{d['Py']} "
            f"half{d['half_spectrum']} prec{d['prec']} pre{pre} {which} R{_bucket(nrhs)}")


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(plan, which: str = "mixed", nrhs: int = 1, reps: int = 10, path: str | None = None,
         force: bool = False) -> dict:
    """Set the plan's launch options for `which` at nrhs columns: from the
    cache when the key is there (unless force), else by timing them on the
    device (toeplitz_tune) and storing the result.  Returns the record."""
    import torch
    path = path or cache_path()
    dev = plan.device
    data = _load(path)
    dkey, pkey = device_key(dev), plan_key(plan, which, nrhs)
    rec = None if force else data.get(dkey, {}).get(pkey)
    if rec is None:
        dt = torch.complex64 if which == "fp32" else torch.complex128
        x = torch.zeros((nrhs, plan.Nt), dtype=dt, device=dev)
        y = torch.empty_like(x)
        r = _lib.TuneResult()
        with torch.cuda.device(dev):
            stream = torch.cuda.current_stream(dev)
            check(_lib.lib().toeplitz_tune(plan._h, PREC[which], ctypes.c_void_p(x.data_ptr()), plan.Nt,
                                           ctypes.c_void_p(y.data_ptr()), plan.Nt, nrhs, reps,
                                           ctypes.c_void_p(stream.cuda_stream), ctypes.byref(r)))
        rec = dict(spectrum_pass=r.spectrum_pass, mfma_cols=r.mfma_cols, fft2_lds=r.fft2_lds,
                   multi_fused=r.multi_fused, prod_lds=r.prod_lds, rim_overlap=r.rim_overlap,
                   candidates=r.candidates,
                   ms=r.ms, ms_default=r.ms_default, nrhs=nrhs, source="measured")
        data.setdefault(dkey, {})[pkey] = rec
        _store(path, data)
    else:
        rec = dict(rec, source="cache")
        if rec["spectrum_pass"]:
            plan.set_option(_lib.TP_OPT_SPECTRUM_PASS, rec["spectrum_pass"])
        if rec["mfma_cols"]:
            plan.set_option(_lib.TP_OPT_MFMA_COLS, rec["mfma_cols"])
        if rec.get("fft2_lds"):
            plan.set_option(_lib.TP_OPT_FFT2_LDS, rec["fft2_lds"])
        if rec.get("multi_fused"):
            plan.set_option(_lib.TP_OPT_MULTI_FUSED, rec["multi_fused"])
        if rec.get("prod_lds"):
            plan.set_option(_lib.TP_OPT_PROD_LDS, rec["prod_lds"])
        if "rim_overlap" in rec:
            plan.set_option(_lib.TP_OPT_RIM_OVERLAP, rec["rim_overlap"])
    return rec
