"""MI355X (gfx950) library for the two-level block-Toeplitz array impedance
operator of arXiv 2506.04710: apply Z and solve Z x = v.

The HIP kernels live in ``libtoeplitz.so`` behind the C ABI of
``include/toeplitz.h``.  This module marshals torch device tensors (memory and
streams only) and numpy host arrays into those calls.

    plan = Plan.create(Nx, Ny, b, Nr, gen, rim_re, rim_rr, prec="mixed", max_rhs=R)
    y = plan.matvec(x)                       # x: complex128 / complex64 cuda tensor (Nt,) or (R, Nt)
    x, info = plan.solve(v, mode="mixed", tol=1e-8)

Vectors are torch tensors of shape (R, Nt): row r is column r of the
column-major Nt x R block that the C ABI takes (leading dimension = row stride).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import PREC, ToeplitzError, check  # noqa: F401

__all__ = ["Plan", "plan_bytes", "plan_bytes_placed", "precond_bytes", "gen_symmetric", "port_smatrix", "far_field", "ToeplitzError",
           "load"]


def load():
    """Load libtoeplitz.so (raises if it is missing)."""
    return _lib.lib()


def plan_bytes(Nx, Ny, b, Nr, prec="mixed", max_rhs=1, restart=40, reciprocal=True, symmetric=False) -> int:
    """Device bytes of a plan.  reciprocal: rim_er will be omitted (B_er = B^T);
    symmetric: the generators are symmetric (gen_symmetric), so the plan keeps
    half the spectrum."""
    n = ctypes.c_size_t(0)
    sym = (_lib.TP_SYM_RIM if reciprocal else 0) | (_lib.TP_SYM_GEN if symmetric else 0)
    check(_lib.lib().toeplitz_plan_bytes(Nx, Ny, b, Nr, sym, PREC[prec], max_rhs, restart, ctypes.byref(n)))
    return n.value


def plan_bytes_placed(Nx, Ny, b, Nr, nrc, prec="mixed", max_rhs=1, restart=40, reciprocal=True,
                      symmetric=False) -> int:
    """Device bytes of a plan with a placed rim of nrc channels per cell;
    symmetric: the extended generators are symmetric (symmetric generators,
    reciprocal rim, symmetric rim_rr)."""
    n = ctypes.c_size_t(0)
    sym = (_lib.TP_SYM_RIM if reciprocal else 0) | (_lib.TP_SYM_GEN if symmetric else 0)
    check(_lib.lib().toeplitz_plan_bytes_placed(Nx, Ny, b, Nr, nrc, sym, PREC[prec], max_rhs, restart,
                                                ctypes.byref(n)))
    return n.value


def placed_symmetric(gen_sym, rim_er, rim_rr) -> bool:
    """Whether a placed plan's extended generators are symmetric (so that it
    keeps half the spectrum): symmetric element generators, a reciprocal rim
    (rim_er None) and rim_rr equal to its transpose bit for bit."""
    if not gen_sym or rim_er is not None:
        return False
    rr = np.ascontiguousarray(rim_rr, dtype=np.complex128)
    bits = rr.view(np.uint64).reshape(rr.shape[0], rr.shape[1], 2)
    return bool(np.array_equal(bits, bits.transpose(1, 0, 2)))


def gen_symmetric(Nx, Ny, b, gen) -> bool:
    """Whether the generators satisfy Z_{-m,-n} = Z_{m,n}^T bit for bit (the
    library's own host check; a plan of such generators stores half the
    spectrum)."""
    g = _host_c128(gen, (2 * Ny - 1, 2 * Nx - 1, b, b))
    out = ctypes.c_int(0)
    check(_lib.lib().toeplitz_gen_symmetric(Nx, Ny, b, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)))
    return bool(out.value)


def precond_bytes(Nx, Ny, b, Nr, prec="mixed", symmetric=False, reciprocal=True) -> int:
    """Device bytes of the block-circulant preconditioner of such a plan (the
    library's own count, toeplitz_precond_bytes_for), for HBM admission before
    the plan exists."""
    n = ctypes.c_size_t(0)
    sym = (_lib.TP_SYM_RIM if reciprocal else 0) | (_lib.TP_SYM_GEN if symmetric else 0)
    check(_lib.lib().toeplitz_precond_bytes_for(Nx, Ny, b, Nr, sym, PREC[prec], ctypes.byref(n)))
    return n.value


def _host_c128(a, shape):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape} elements, got {a.shape}")
    return a


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A plan: the operator's spectrum and rim blocks resident in one device buffer."""

    def __init__(self):
        self._h = None

    @classmethod
    def create(cls, Nx, Ny, b, Nr, gen, rim_re=None, rim_rr=None, rim_er=None, prec="mixed", max_rhs=1,
               restart=40, device="cuda:0", stream=None, rim_place=None):
        """rim_place: None (dense rim blocks), or (place, nrc) for a placed rim:
        place an int array [Nr, 3] of (cell x, cell y, channel), nrc the rim
        channels per cell (toeplitz_plan_create_placed)."""
        import torch
        L = _lib.lib()
        N = Nx * Ny * b
        gen = _host_c128(gen, (2 * Ny - 1, 2 * Nx - 1, b, b))
        rim_re = _host_c128(rim_re, (Nr, N)) if Nr else None
        rim_rr = _host_c128(rim_rr, (Nr, Nr)) if Nr else None
        rim_er = _host_c128(rim_er, (N, Nr)) if (Nr and rim_er is not None) else None
        gsym = gen_symmetric(Nx, Ny, b, gen)
        if rim_place is not None:
            place = np.ascontiguousarray(rim_place[0], dtype=np.int32).reshape(Nr, 3)
            nrc = int(rim_place[1])
            xsym = placed_symmetric(gsym, rim_er, rim_rr)
            nbytes = plan_bytes_placed(Nx, Ny, b, Nr, nrc, prec, max_rhs, restart, reciprocal=rim_er is None,
                                       symmetric=xsym)
        else:
            nbytes = plan_bytes(Nx, Ny, b, Nr, prec, max_rhs, restart, reciprocal=rim_er is None, symmetric=gsym)
        self = cls()
        self.device = torch.device(device)
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.buf.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        with torch.cuda.device(self.device):
            if rim_place is not None:
                check(L.toeplitz_plan_create_placed(Nx, Ny, b, Nr, ptr(gen), ptr(rim_re), ptr(rim_er), ptr(rim_rr),
                                                    ptr(place), nrc, PREC[prec], max_rhs, restart,
                                                    ctypes.c_void_p(base + off), nbytes, _stream_handle(stream),
                                                    ctypes.byref(h)))
            else:
                check(L.toeplitz_plan_create(Nx, Ny, b, Nr, ptr(gen), ptr(rim_re), ptr(rim_er), ptr(rim_rr),
                                             PREC[prec], max_rhs, restart, ctypes.c_void_p(base + off), nbytes,
                                             _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.Nx, self.Ny, self.b, self.Nr = Nx, Ny, b, Nr
        self.N, self.Nt = N, N + Nr
        self.prec, self.max_rhs, self.restart = prec, max_rhs, restart
        return self

    @classmethod
    def from_problem(cls, prob, **kw):
        return cls.create(prob.Nx, prob.Ny, prob.b, prob.Nr, prob.gen, prob.rim_re, prob.rim_rr, **kw)

    def set_option(self, option, value):
        """Launch option (toeplitz_plan_set_option), e.g. spectrum pass."""
        check(_lib.lib().toeplitz_plan_set_option(self._h, option, value))
        return self

    def get_option(self, option) -> int:
        v = ctypes.c_int(0)
        check(_lib.lib().toeplitz_plan_get_option(self._h, option, ctypes.byref(v)))
        return v.value

    def path(self, which="mixed", nrhs=1, precond=False) -> set:
        """Names of the launches an application of the operator (or the
        preconditioner) takes at nrhs columns (toeplitz_plan_path)."""
        v = ctypes.c_int(0)
        check(_lib.lib().toeplitz_plan_path(self._h, PREC[which], int(precond), nrhs, ctypes.byref(v)))
        return {k for k, bit in _lib.PATH_BITS.items() if v.value & bit}

    def info(self) -> dict:
        d = _lib.PlanDesc()
        check(_lib.lib().toeplitz_plan_info(self._h, ctypes.byref(d)))
        return {f: getattr(d, f) for f, _ in _lib.PlanDesc._fields_}

    def _cols(self, t, dtype):
        import torch
        if t.device.type != "cuda":
            raise ValueError("vectors must be device tensors")
        if t.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {t.dtype}")
        if t.dim() == 1:
            t = t.unsqueeze(0)
        if t.dim() != 2 or t.shape[1] != self.Nt or t.stride(1) != 1:
            raise ValueError("vectors must have shape (R, Nt) with unit stride along Nt")
        return t, t.shape[0], t.stride(0) if t.shape[0] > 1 else self.Nt

    def matvec(self, x, which=None, out=None, stream=None):
        """y = Z x on the device.  which: 'fp64' (complex128 x, FP64 operator),
        'fp32' (complex64 x, FP32 operator) or 'mixed' (complex128 x, FP32
        operator: the inner operator of a mixed solve)."""
        import torch
        if which is None:
            which = "fp64" if x.dtype == torch.complex128 else "fp32"
        dt = torch.complex64 if which == "fp32" else torch.complex128
        x2, R, ldx = self._cols(x, dt)
        y = torch.empty((R, self.Nt), dtype=dt, device=x.device) if out is None else out
        y2, Ry, ldy = self._cols(y, dt)
        if Ry != R:
            raise ValueError("out has a different number of columns")
        check(_lib.lib().toeplitz_matvec(self._h, PREC[which], ctypes.c_void_p(x2.data_ptr()), ldx,
                                         ctypes.c_void_p(y2.data_ptr()), ldy, R, _stream_handle(stream)))
        return y.reshape(x.shape) if out is None else out

    def matvec_static(self, x, which=None, out=None, stream=None):
        """y = Z x like matvec, through toeplitz_matvec_static: the workspace is
        the library's static device array (no allocation by the library; calls
        that overlap in time on one device race)."""
        import torch
        if which is None:
            which = "fp64" if x.dtype == torch.complex128 else "fp32"
        dt = torch.complex64 if which == "fp32" else torch.complex128
        x2, R, ldx = self._cols(x, dt)
        y = torch.empty((R, self.Nt), dtype=dt, device=x.device) if out is None else out
        y2, Ry, ldy = self._cols(y, dt)
        if Ry != R:
            raise ValueError("out has a different number of columns")
        with torch.cuda.device(x.device):
            check(_lib.lib().toeplitz_matvec_static(self._h, PREC[which], ctypes.c_void_p(x2.data_ptr()), ldx,
                                                    ctypes.c_void_p(y2.data_ptr()), ldy, R, _stream_handle(stream)))
        return y.reshape(x.shape) if out is None else out

    def precond_create(self, stream=None):
        """Build the block-circulant preconditioner into a second device buffer
        owned by this plan object (needs an FP64 or mixed plan)."""
        import torch
        L = _lib.lib()
        n = ctypes.c_size_t(0)
        check(L.toeplitz_precond_bytes(self._h, ctypes.byref(n)))
        buf = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = buf.data_ptr()
        off = (-base) % 256
        with torch.cuda.device(self.device):
            check(L.toeplitz_precond_create(self._h, ctypes.c_void_p(base + off), n.value, _stream_handle(stream)))
        self.pbuf = buf           # only now: a refused rebuild keeps the old buffer in use
        return self

    def precond_apply(self, x, which=None, stream=None):
        """y = M^-1 x with the plan's preconditioner ('fp64': complex128, 'fp32':
        complex64, 'mixed': complex128 vectors with the FP32 copy)."""
        import torch
        if which is None:
            which = "fp64" if x.dtype == torch.complex128 else "fp32"
        dt = torch.complex64 if which == "fp32" else torch.complex128
        x2, R, ldx = self._cols(x, dt)
        y = torch.empty((R, self.Nt), dtype=dt, device=x.device)
        check(_lib.lib().toeplitz_precond_apply(self._h, PREC[which], ctypes.c_void_p(x2.data_ptr()), ldx,
                                                ctypes.c_void_p(y.data_ptr()), self.Nt, R, _stream_handle(stream)))
        return y.reshape(x.shape)

    STAGES = ("rim_main", "fwd_x", "fwd_y", "prod", "inv_y", "inv_x", "rim_finish")

    def matvec_profile(self, x, which=None, reps=20, stream=None) -> dict:
        """Mean per-stage milliseconds of the operator application (HIP events)."""
        import torch
        if which is None:
            which = "fp64" if x.dtype == torch.complex128 else "fp32"
        dt = torch.complex64 if which == "fp32" else torch.complex128
        x2, R, ldx = self._cols(x, dt)
        y = torch.empty((R, self.Nt), dtype=dt, device=x.device)
        ms = (ctypes.c_double * 7)()
        check(_lib.lib().toeplitz_matvec_profile(self._h, PREC[which], ctypes.c_void_p(x2.data_ptr()), ldx,
                                                 ctypes.c_void_p(y.data_ptr()), self.Nt, R, reps,
                                                 _stream_handle(stream), ms))
        return dict(zip(self.STAGES, list(ms)))

    def stage_time(self, x, stage=3, which=None, reps=50, stream=None) -> float:
        """Mean milliseconds of one stage of the application launched reps
        times back to back (toeplitz_stage_time)."""
        import torch
        if which is None:
            which = "fp64" if x.dtype == torch.complex128 else "fp32"
        dt = torch.complex64 if which == "fp32" else torch.complex128
        x2, R, ldx = self._cols(x, dt)
        y = torch.empty((R, self.Nt), dtype=dt, device=x.device)
        ms = ctypes.c_double(0.0)
        check(_lib.lib().toeplitz_stage_time(self._h, PREC[which], ctypes.c_void_p(x2.data_ptr()), ldx,
                                             ctypes.c_void_p(y.data_ptr()), self.Nt, R, stage, reps,
                                             _stream_handle(stream), ctypes.byref(ms)))
        return ms.value

    def solve(self, v, mode="mixed", tol=1e-8, restart=0, max_iter=2000, max_outer=50, inner_tol=1e-4, x0=None,
              stream=None, raise_on_noconv=False, precond=False):
        """Solve Z x = v for the columns of v (complex128 cuda tensor (Nt,) or (R, Nt))."""
        import torch
        v2, R, ldv = self._cols(v, torch.complex128)
        if x0 is not None:
            x = x0.clone().reshape(R, self.Nt)
        else:
            x = torch.empty((R, self.Nt), dtype=torch.complex128, device=v.device)
        x2, _, ldx = self._cols(x, torch.complex128)
        o = _lib.SolveOpts()
        _lib.lib().toeplitz_solve_opts_default(ctypes.byref(o))
        o.tol, o.restart, o.max_iter, o.max_outer = tol, restart, max_iter, max_outer
        o.mode, o.x0_given, o.inner_tol = PREC[mode], 1 if x0 is not None else 0, inner_tol
        o.precond = 1 if precond else 0
        info = (_lib.SolveInfo * R)()
        st = _lib.lib().toeplitz_solve(self._h, ctypes.c_void_p(v2.data_ptr()), ldv, ctypes.c_void_p(x2.data_ptr()),
                                       ldx, R, ctypes.byref(o), info, _stream_handle(stream))
        if st not in (_lib.TP_OK, _lib.TP_E_NOCONV, _lib.TP_E_BREAKDOWN) or (raise_on_noconv and st != _lib.TP_OK):
            check(st)
        infos = [dict(iters=i.iters, outer_iters=i.outer_iters, status=i.status, relres=i.relres) for i in info]
        return x.reshape(v.shape), infos

    @staticmethod
    def _opts(mode, tol, restart, max_iter, max_outer, inner_tol, precond):
        o = _lib.SolveOpts()
        _lib.lib().toeplitz_solve_opts_default(ctypes.byref(o))
        o.tol, o.restart, o.max_iter, o.max_outer = tol, restart, max_iter, max_outer
        o.mode, o.x0_given, o.inner_tol = PREC[mode], 0, inner_tol
        o.precond = 1 if precond else 0
        return o

    def schur_create(self, element_plan, mode="mixed", tol=1e-10, restart=0, max_iter=2000, max_outer=50,
                     inner_tol=1e-4, precond=False, stream=None):
        """Eliminate the rim through its Schur complement: F = A^-1 B_er and
        (C - B F)^-1 into a device buffer owned by this plan object.
        element_plan: a Plan of the same array (Nx, Ny, b, generators) with
        Nr = 0; it runs the solves with the element operator A (options as
        for solve, applied to those solves)."""
        import torch
        L = _lib.lib()
        n = ctypes.c_size_t(0)
        check(L.toeplitz_schur_bytes(self._h, ctypes.byref(n)))
        self.sbuf = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        base = self.sbuf.data_ptr()
        off = (-base) % 256
        o = self._opts(mode, tol, restart, max_iter, max_outer, inner_tol, precond)
        with torch.cuda.device(self.device):
            check(L.toeplitz_schur_create(self._h, element_plan._h, ctypes.c_void_p(base + off), n.value,
                                          ctypes.byref(o), _stream_handle(stream)))
        self.element = element_plan
        return self

    def schur_solve(self, v, mode="mixed", tol=1e-8, restart=0, max_iter=2000, max_outer=50, inner_tol=1e-4,
                    precond=False, stream=None, raise_on_noconv=False):
        """Solve Z x = v through the rim elimination (schur_create first)."""
        import torch
        v2, R, ldv = self._cols(v, torch.complex128)
        x = torch.empty((R, self.Nt), dtype=torch.complex128, device=v.device)
        x2, _, ldx = self._cols(x, torch.complex128)
        o = self._opts(mode, tol, restart, max_iter, max_outer, inner_tol, precond)
        info = (_lib.SolveInfo * R)()
        el = getattr(self, "element", None)
        st = _lib.lib().toeplitz_schur_solve(self._h, el._h if el is not None else None,
                                             ctypes.c_void_p(v2.data_ptr()), ldv, ctypes.c_void_p(x2.data_ptr()),
                                             ldx, R, ctypes.byref(o), info, _stream_handle(stream))
        if st not in (_lib.TP_OK, _lib.TP_E_NOCONV) or (raise_on_noconv and st != _lib.TP_OK):
            check(st)
        infos = [dict(iters=i.iters, outer_iters=i.outer_iters, status=i.status, relres=i.relres) for i in info]
        return x.reshape(v.shape), infos

    def spectrum(self, kx, ky, which="fp64") -> np.ndarray:
        dt = np.complex128 if which == "fp64" else np.complex64
        bc = self.info()["bc"]               # channels per cell (b, plus a placed rim's)
        out = np.empty((bc, bc), dtype=dt)
        check(_lib.lib().toeplitz_plan_spectrum(self._h, PREC[which], kx, ky, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if self._h is not None:
            _lib.lib().toeplitz_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def port_smatrix(X, port_rows, Z0=50.0, edge_len=None, stream=None):
    """Scattering matrix (p x p complex128 cuda tensor, S[i, j]) from the port
    solutions X (complex128 cuda tensor (p, Nt): row j solves the excitation of
    port j) and the port unknowns port_rows (length p)."""
    import torch
    x2 = X if X.dim() == 2 else X.reshape(1, -1)
    if x2.dtype != torch.complex128 or not x2.is_cuda or x2.stride(1) != 1:
        raise ValueError("X must be a complex128 cuda tensor with contiguous rows")
    p, Nt = x2.shape[0], x2.shape[1]
    rows = np.ascontiguousarray(port_rows, dtype=np.int64)
    if rows.shape != (p,):
        raise ValueError(f"port_rows must have {p} entries")
    lens = None if edge_len is None else np.ascontiguousarray(edge_len, dtype=np.float64)
    if lens is not None and lens.shape != (p,):
        raise ValueError(f"edge_len must have {p} entries")
    wbytes = 32 * p * p + 16 * p + 256
    work = torch.empty(wbytes // 8 + 1, dtype=torch.float64, device=x2.device)
    St = torch.empty((p, p), dtype=torch.complex128, device=x2.device)   # St[j, i] = S[i, j] (column-major S)
    check(_lib.lib().toeplitz_port_smatrix(
        p, Nt, ctypes.c_void_p(x2.data_ptr()), x2.stride(0), rows.ctypes.data_as(ctypes.c_void_p),
        None if lens is None else lens.ctypes.data_as(ctypes.c_void_p), float(Z0), ctypes.c_void_p(St.data_ptr()), p,
        ctypes.c_void_p(work.data_ptr()), work.numel() * 8, _stream_handle(stream)))
    return St.t()


def far_field(I, Nx, Ny, b, Nr, dx, dy, elem_pos, elem_tan, rim_pos, rim_tan, theta, phi, k, eta, stream=None):
    """Far field of the current vectors I (complex128 cuda tensor (R, Nt) or (Nt,))
    in the directions (theta[m], phi[m]) (radians).  Geometry arrays are numpy
    float64: elem_pos / elem_tan [b, 3] (basis offsets in the element and unit
    tangents), rim_pos / rim_tan [Nr, 3].  Returns a complex128 cuda tensor
    (R, nang, 2) of (F_theta, F_phi)."""
    import torch
    i2 = I if I.dim() == 2 else I.reshape(1, -1)
    if i2.dtype != torch.complex128 or not i2.is_cuda or i2.stride(1) != 1:
        raise ValueError("I must be a complex128 cuda tensor with contiguous rows")
    dev = i2.device
    R = i2.shape[0]
    th = np.asarray(theta, dtype=np.float64).reshape(-1)
    ph = np.asarray(phi, dtype=np.float64).reshape(-1)
    if th.shape != ph.shape:
        raise ValueError("theta and phi must pair up")

    def d(a, shape):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if a.shape != shape:
            raise ValueError(f"expected shape {shape}, got {a.shape}")
        return torch.from_numpy(a).to(dev)

    up, ut = d(elem_pos, (b, 3)), d(elem_tan, (b, 3))
    rp = d(rim_pos, (Nr, 3)) if Nr else None
    rt = d(rim_tan, (Nr, 3)) if Nr else None
    dirs = torch.from_numpy(np.stack([th, ph], axis=1).copy()).to(dev)
    F = torch.empty((R, th.size, 2), dtype=torch.complex128, device=dev)
    if stream is not None:
        # the staging tensors were filled on the current stream and are read on `stream`
        stream.wait_stream(torch.cuda.current_stream(dev))
        for t in (up, ut, rp, rt, dirs, F):
            if t is not None:
                t.record_stream(stream)
    ptr = lambda t: None if t is None else ctypes.c_void_p(t.data_ptr())
    check(_lib.lib().toeplitz_far_field(Nx, Ny, b, Nr, float(dx), float(dy), ptr(up), ptr(ut), ptr(rp), ptr(rt),
                                        ptr(i2), i2.stride(0), R, ptr(dirs), th.size, float(k), float(eta), ptr(F),
                                        _stream_handle(stream)))
    return F
