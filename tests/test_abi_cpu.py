"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching a device."""
import ctypes

import numpy as np
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "toeplitz.h")


@pytest.fixture(scope="module")
def L():
    from paper_2506_04710_amd import _lib
    return _lib.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(toeplitz_\w+)\s*\(", src)))


def test_header_declares_expected_api():
    from paper_2506_04710_amd import _lib
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_plan_bytes_matches_layout_accounting(L):
    from paper_2506_04710_amd import plan_bytes
    # spectrum of config 2 at Px = Py = 63: 63*63*64*64 complex128 = 260 MB, and half for complex64
    b64 = plan_bytes(32, 32, 64, 256, "fp64", 1, 40)
    b32 = plan_bytes(32, 32, 64, 256, "fp32", 1, 40)
    bm = plan_bytes(32, 32, 64, 256, "mixed", 1, 40)
    spec = 63 * 63 * 64 * 64 * 16
    rim = (256 * 65536 + 256 * 256) * 16
    assert b64 >= spec + rim and b32 >= (spec + rim) // 2
    assert bm - b64 >= (spec + rim) // 2 - 4096 * 8
    # a non-reciprocal rim stores a second dense block per precision
    nr = plan_bytes(32, 32, 64, 256, "fp64", 1, 40, reciprocal=False)
    assert nr - b64 >= 256 * 65536 * 16
    # more columns and longer restarts need more Krylov workspace (small array: the
    # plan-time scratch does not dominate)
    small = plan_bytes(8, 8, 16, 0, "mixed", 4, 40)
    assert plan_bytes(8, 8, 16, 0, "mixed", 64, 40) > small
    assert plan_bytes(8, 8, 16, 0, "mixed", 4, 200) > small


def test_plan_bytes_half_spectrum(L):
    """Symmetric generators keep the spectrum columns kx <= Px/2: at Px = Py = 63
    that is 32 of 63 columns, 31 * 63 blocks fewer per precision (the
    single-column path's mirror parts, 8 * 32 * 31 * 64 values, come back as
    workspace)."""
    from paper_2506_04710_amd import plan_bytes
    for prec, s in (("fp64", 16), ("mixed", 24)):
        full = plan_bytes(32, 32, 64, 256, prec, 1, 40)
        half = plan_bytes(32, 32, 64, 256, prec, 1, 40, symmetric=True)
        saved = 31 * 63 * 64 * 64 * s
        assert saved - 8 * 32 * 31 * 64 * 16 - 4096 <= full - half <= saved, prec
    n = ctypes.c_size_t(0)
    assert L.toeplitz_plan_bytes(4, 4, 16, 0, 4, 0, 1, 40, ctypes.byref(n)) == 1   # unknown sym bit


def test_gen_symmetric_host_check(L):
    """The library's generator symmetry test: Z_{-m,-n} = Z_{m,n}^T bit for bit."""
    from paper_2506_04710_amd import gen_symmetric
    from synth import arrays as sa
    prob = sa.make_problem(3, 2, 4, 0, 7)
    assert gen_symmetric(3, 2, 4, prob.gen)
    g = prob.gen.copy()
    g[0, 1, 1, 2] += 1.0                 # one entry of Z_{-2,-1} changed
    assert not gen_symmetric(3, 2, 4, g)
    # mirrored blocks equal but not transposed: not the symmetry
    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 5, 4, 4)) + 1j * rng.standard_normal((3, 5, 4, 4))
    assert not gen_symmetric(3, 2, 4, a + a[::-1, ::-1])
    assert gen_symmetric(3, 2, 4, a + a[::-1, ::-1].transpose(0, 1, 3, 2))
    out = ctypes.c_int(5)
    assert L.toeplitz_gen_symmetric(3, 2, 4, None, ctypes.byref(out)) == 1 and out.value == 0
    assert L.toeplitz_gen_symmetric(0, 2, 4, prob.gen.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)) == 1


@pytest.mark.parametrize("args", [
    (0, 4, 16, 0), (4, 0, 16, 0), (4, 4, 0, 0), (4, 4, 16, -1), (257, 4, 4, 0), (4, 4, 257, 0)])
def test_plan_bytes_rejects_bad_shapes(L, args):
    n = ctypes.c_size_t(0)
    assert L.toeplitz_plan_bytes(*args, 1, 2, 1, 40, ctypes.byref(n)) == 1
    assert L.toeplitz_last_error()


def test_plan_bytes_rejects_bad_options(L):
    n = ctypes.c_size_t(0)
    assert L.toeplitz_plan_bytes(4, 4, 16, 0, 1, 7, 1, 40, ctypes.byref(n)) == 1     # precision
    assert L.toeplitz_plan_bytes(4, 4, 16, 0, 1, 0, 0, 40, ctypes.byref(n)) == 1     # max_rhs
    assert L.toeplitz_plan_bytes(4, 4, 16, 0, 1, 0, 1, 0, ctypes.byref(n)) == 1      # restart
    assert L.toeplitz_plan_bytes(4, 4, 16, 0, 1, 0, 1, 40, None) == 1


def test_plan_create_validates_before_device_work(L):
    from paper_2506_04710_amd import _lib
    h = ctypes.c_void_p()
    gen = (ctypes.c_double * (2 * 7 * 7 * 4))()
    fake = ctypes.c_void_p(0x1000)          # never dereferenced: validation fails first
    # NULL generators
    assert L.toeplitz_plan_create(4, 4, 1, 0, None, None, None, None, 0, 1, 8, fake, 1 << 30, None,
                                  ctypes.byref(h)) == _lib.TP_E_INVAL
    # rim blocks missing with Nr > 0
    assert L.toeplitz_plan_create(4, 4, 1, 3, gen, None, None, None, 0, 1, 8, fake, 1 << 30, None,
                                  ctypes.byref(h)) == _lib.TP_E_INVAL
    # misaligned device buffer
    assert L.toeplitz_plan_create(4, 4, 1, 0, gen, None, None, None, 0, 1, 8, ctypes.c_void_p(0x1001),
                                  1 << 30, None, ctypes.byref(h)) == _lib.TP_E_INVAL
    # buffer too small
    assert L.toeplitz_plan_create(4, 4, 1, 0, gen, None, None, None, 0, 1, 8, fake, 16, None,
                                  ctypes.byref(h)) == _lib.TP_E_NOMEM
    assert h.value is None
    # a non-finite generator or rim entry
    for bad in (float("nan"), float("inf")):
        g = np.zeros((7, 7, 1, 1), dtype=np.complex128)
        g[3, 2, 0, 0] = complex(0.0, bad)
        assert L.toeplitz_plan_create(4, 4, 1, 0, g.ctypes.data_as(ctypes.c_void_p), None, None, None, 0, 1, 8, fake,
                                      1 << 30, None, ctypes.byref(h)) == _lib.TP_E_INVAL
        assert b"non-finite" in L.toeplitz_last_error()
        rim = np.zeros((2, 16), dtype=np.complex128)
        rim[1, 5] = bad
        rr = np.eye(2, dtype=np.complex128)
        ok = np.zeros((7, 7, 1, 1), dtype=np.complex128)
        assert L.toeplitz_plan_create(4, 4, 1, 2, ok.ctypes.data_as(ctypes.c_void_p),
                                      rim.ctypes.data_as(ctypes.c_void_p), None, rr.ctypes.data_as(ctypes.c_void_p),
                                      0, 1, 8, fake, 1 << 30, None, ctypes.byref(h)) == _lib.TP_E_INVAL
    assert h.value is None


def test_precond_bytes_for_matches_layout(L):
    """The admission size of the preconditioner before a plan exists: the
    inverted stored spectrum blocks per precision, 1/diag(C) per precision,
    a status word, each region 256-byte aligned."""
    from paper_2506_04710_amd import _lib, precond_bytes
    al = lambda v: (v + 255) // 256 * 256
    for (Nx, Ny, b, Nr), (px, py) in (((32, 32, 64, 256), (63, 63)), ((9, 9, 96, 72), (18, 18)),
                                      ((8, 5, 16, 0), (15, 9))):
        for sym in (False, True):
            nblk = ((px // 2 + 1) if sym else px) * py
            for prec, sizes in (("fp64", (16,)), ("mixed", (16, 8))):
                want = sum(al(nblk * b * b * s) for s in sizes) + (sum(al(Nr * s) for s in sizes) if Nr else 0) + 256
                assert precond_bytes(Nx, Ny, b, Nr, prec, symmetric=sym) == want, (Nx, Ny, b, Nr, sym, prec)
    n = ctypes.c_size_t(0)
    assert L.toeplitz_precond_bytes_for(4, 4, 8, 0, 0, _lib.TP_FP32, ctypes.byref(n)) == _lib.TP_E_UNSUPPORTED
    assert L.toeplitz_precond_bytes_for(4, 4, 8, 0, 8, _lib.TP_FP64, ctypes.byref(n)) == _lib.TP_E_INVAL
    assert L.toeplitz_precond_bytes_for(0, 4, 8, 0, 0, _lib.TP_FP64, ctypes.byref(n)) == _lib.TP_E_INVAL


def test_null_plan_calls_fail_cleanly(L):
    from paper_2506_04710_amd import _lib
    for which in (_lib.TP_FP64, _lib.TP_FP32, _lib.TP_MIXED):
        assert L.toeplitz_matvec(None, which, None, 1, None, 1, 1, None) == _lib.TP_E_INVAL
        assert L.toeplitz_precond_apply(None, which, None, 1, None, 1, 1, None) == _lib.TP_E_INVAL
    assert L.toeplitz_solve(None, None, 1, None, 1, 1, None, None, None) == _lib.TP_E_INVAL
    assert L.toeplitz_plan_info(None, None) == _lib.TP_E_INVAL
    n = ctypes.c_size_t(0)
    assert L.toeplitz_schur_bytes(None, ctypes.byref(n)) == _lib.TP_E_INVAL
    assert L.toeplitz_schur_create(None, None, None, 0, None, None) == _lib.TP_E_INVAL
    assert L.toeplitz_schur_solve(None, None, None, 1, None, 1, 1, None, None, None) == _lib.TP_E_INVAL
    L.toeplitz_plan_destroy(None)


def test_solve_defaults(L):
    from paper_2506_04710_amd import _lib
    o = _lib.SolveOpts()
    L.toeplitz_solve_opts_default(ctypes.byref(o))
    assert o.tol == 1e-8 and o.max_iter == 2000 and o.mode == _lib.TP_FP64 and o.x0_given == 0


def test_port_smatrix_validates_before_device_work(L):
    import numpy as np
    vp = ctypes.c_void_p
    fake = vp(0x100000)          # never dereferenced: every case fails validation first
    rows = np.array([0, 3, 5], dtype=np.int64)
    lens = np.array([1.0, 0.5, 2.0])
    rp = rows.ctypes.data_as(vp)
    need = 32 * 9 + 16 * 3 + 256

    def call(p=3, Nt=10, X=fake, ldx=10, r=rp, ln=None, Z0=50.0, S=fake, lds=3, work=fake, wb=need):
        return L.toeplitz_port_smatrix(p, Nt, X, ldx, r, ln, Z0, S, lds, work, wb, None)

    assert call(p=0) == 1 and call(p=1025) == 1
    assert call(Nt=0) == 1 and call(ldx=9) == 1 and call(lds=2) == 1
    assert call(X=None) == 1 and call(r=None) == 1 and call(S=None) == 1 and call(work=None) == 1
    assert call(work=vp(0x100004)) == 1            # misaligned
    assert call(wb=need - 1) == 1
    assert call(Z0=0.0) == 1 and call(Z0=float("inf")) == 1
    bad = np.array([0, 3, 10], dtype=np.int64)
    assert call(r=bad.ctypes.data_as(vp)) == 1     # row outside [0, Nt)
    neg = np.array([1.0, 0.0, 2.0])
    assert call(ln=neg.ctypes.data_as(vp)) == 1
    assert b"edge" in L.toeplitz_last_error()


def test_far_field_validates_before_device_work(L):
    vp = ctypes.c_void_p
    fake = vp(0x100000)

    def call(Nx=4, Ny=4, b=8, Nr=2, up=fake, ut=fake, rp=fake, rt=fake, I=fake, ldi=130, R=1, dirs=fake, nang=3,
             F=fake, k=6.28):
        return L.toeplitz_far_field(Nx, Ny, b, Nr, 0.5, 0.5, up, ut, rp, rt, I, ldi, R, dirs, nang, k, 376.7, F,
                                    None)

    assert call(Nx=0) == 1 and call(b=0) == 1 and call(Nr=-1) == 1
    assert call(R=0) == 1 and call(nang=0) == 1 and call(ldi=129) == 1
    assert call(up=None) == 1 and call(I=None) == 1 and call(F=None) == 1 and call(dirs=None) == 1
    assert call(rp=None) == 1                      # Nr > 0 needs rim geometry
    assert call(k=float("nan")) == 1
