"""Host-side checks of the C-ABI (no GPU needed, no kernel is launched):
exported symbols, struct layout, argument validation, workspace queries and
the mode-order planner."""
import ctypes
import itertools
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import kp_workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kp.h")


@pytest.fixture(scope="module")
def L():
    from paper_2112_11238_amd import _lib
    return _lib


@pytest.fixture(scope="module")
def lib(L):
    return L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kp_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib, L):
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, f"binding lacks a prototype for {name}"


def test_struct_layout_matches_header(L):
    gcc = shutil.which("gcc")
    if not gcc or not os.path.exists("/opt/rocm/include/hip/hip_runtime_api.h"):
        pytest.skip("gcc or HIP headers missing")
    exe = os.path.join(ROOT, "tests", ".abi_layout_bin")
    r = subprocess.run([gcc, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "abi_layout.c"),
                        "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([exe], capture_output=True, text=True).stdout.split("\n")
    os.remove(exe)
    t = out[0].split()
    assert int(t[1]) == ctypes.sizeof(L.KpTensor)
    for name, off in zip(t[2::2], t[3::2]):
        assert getattr(L.KpTensor, name).offset == int(off), name
    mline = out[1].split()
    assert int(mline[1]) == ctypes.sizeof(L.KpMatrix)
    for name, off in zip(mline[2::2], mline[3::2]):
        assert getattr(L.KpMatrix, name).offset == int(off), name
    codes = [int(x) for x in out[2].split()[1:]]
    assert codes == sorted(L.STATUS, reverse=True)
    p = out[3].split()
    assert [int(p[1]), int(p[2]), int(p[3])] == [L.KP_PREC_NATIVE, L.KP_PREC_BF16X3,
                                                 L.KP_PREC_BF16X6]
    assert [int(p[5]), int(p[6]), int(p[8])] == [L.KP_F64, L.KP_F32, L.KP_MAX_ORDER]
    e = out[4].split()
    assert e[0] == "kp_tune_entry" and int(e[1]) == ctypes.sizeof(L.KpTuneEntry) == 64
    for name, off in zip(e[2::2], e[3::2]):
        assert getattr(L.KpTuneEntry, name).offset == int(off), name


def test_strerror_and_version(lib, L):
    assert lib.kp_version() == 100
    for code in L.STATUS:
        assert lib.kp_strerror(code)
    assert lib.kp_strerror(12345) == b"unknown status"


FAKE = 0x10000  # a non-null address; never dereferenced: validation fails first


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:  # pragma: no cover
        return False


# The argument-error tests hand the library fake device addresses that its
# host-side validation must reject before any launch. They run only where no
# GPU is visible, so that a validation bug can never reach a kernel.
no_device = pytest.mark.skipif(_gpu_visible(), reason="fake-address tests run without a GPU")


def tensor(L, dims, dtype=0, data=FAKE):
    t = L.KpTensor()
    t.d = len(dims)
    t.dtype = dtype
    for k, v in enumerate(dims[:8]):
        t.dims[k] = v
    t.data = data
    return t


def matrix(L, rows, cols, dtype=0, data=FAKE + 0x100000):
    mtx = L.KpMatrix()
    mtx.rows, mtx.cols = rows, cols
    mtx.rs, mtx.cs = cols, 1
    mtx.dtype = dtype
    mtx.data = data
    return mtx


def mlist(L, ms):
    arr = (ctypes.POINTER(L.KpMatrix) * len(ms))()
    for k, x in enumerate(ms):
        arr[k] = ctypes.pointer(x) if x is not None else None
    return arr


@no_device
def test_tucker_noalloc_argument_errors(lib, L):
    """The allocation-free Tucker call rejects, before touching a device,
    argument errors (as kp_tucker) and problems whose intermediates exceed
    the fixed scratch buffer."""
    assert lib.kp_noalloc_scratch_bytes() == 128 << 20
    T = tensor(L, [4, 5, 6], dtype=1)
    S = tensor(L, [3, 2, 5], dtype=1, data=FAKE + 0x300000)
    arr = mlist(L, [matrix(L, 3, 4, 1), matrix(L, 2, 5, 1), matrix(L, 5, 6, 1)])
    bad = mlist(L, [matrix(L, 3, 4, 1), matrix(L, 2, 6, 1), matrix(L, 5, 6, 1)])
    assert lib.kp_tucker_noalloc(ctypes.byref(T), bad, ctypes.byref(S), 0, None) == -4
    assert lib.kp_tucker_noalloc(None, arr, ctypes.byref(S), 0, None) == -1
    # FP64 512^3 -> 512^3: two 1 GiB intermediates, far past 128 MiB
    Tb = tensor(L, [512, 512, 512])
    Sb = tensor(L, [512, 512, 512], data=FAKE + (1 << 34))
    big = mlist(L, [matrix(L, 512, 512, data=FAKE + (1 << 33) + 0x100000 * j) for j in range(3)])
    need = lib.kp_tucker_workspace(ctypes.byref(Tb), big, 0)
    assert need > lib.kp_noalloc_scratch_bytes()
    assert lib.kp_tucker_noalloc(ctypes.byref(Tb), big, ctypes.byref(Sb), 0, None) == -10
    assert lib.kp_strerror(-10) != b"unknown status"


@no_device
def test_mump_argument_errors(lib, L):
    T = tensor(L, [4, 5, 6])
    S = tensor(L, [4, 7, 6], data=FAKE + 0x200000)
    M = matrix(L, 7, 5)
    call = lambda t, m, mu, s, prec=0: lib.kp_mump(t, m, mu, s, prec, 0, None)
    assert call(None, ctypes.byref(M), 2, ctypes.byref(S)) == -1
    assert call(ctypes.byref(T), None, 2, ctypes.byref(S)) == -1
    assert call(ctypes.byref(tensor(L, [])), ctypes.byref(M), 1, ctypes.byref(S)) == -2
    assert call(ctypes.byref(tensor(L, [2] * 9)), ctypes.byref(M), 1, ctypes.byref(S)) == -2
    assert call(ctypes.byref(T), ctypes.byref(M), 0, ctypes.byref(S)) == -3
    assert call(ctypes.byref(T), ctypes.byref(M), 4, ctypes.byref(S)) == -3
    assert call(ctypes.byref(T), ctypes.byref(matrix(L, 7, 6)), 2, ctypes.byref(S)) == -4
    assert call(ctypes.byref(T), ctypes.byref(M), 2, ctypes.byref(tensor(L, [4, 8, 6]))) == -4
    assert call(ctypes.byref(T), ctypes.byref(matrix(L, 7, 5, dtype=1)), 2,
                ctypes.byref(S)) == -5
    # BF16 split forms need FP32 data
    assert call(ctypes.byref(T), ctypes.byref(M), 2, ctypes.byref(S), prec=3) == -5
    assert call(ctypes.byref(T), ctypes.byref(M), 2, ctypes.byref(S), prec=5) == -5
    # output overlapping the input
    S_alias = tensor(L, [4, 7, 6], data=FAKE + 8)
    assert call(ctypes.byref(T), ctypes.byref(M), 2, ctypes.byref(S_alias)) == -6
    # NULL data with a non-empty tensor
    assert call(ctypes.byref(tensor(L, [4, 5, 6], data=None)), ctypes.byref(M), 2,
                ctypes.byref(S)) == -1
    # negative factor strides; a factor spanning 2^31 bytes or more
    Mneg = matrix(L, 7, 5)
    Mneg.rs = -5
    assert call(ctypes.byref(T), ctypes.byref(Mneg), 2, ctypes.byref(S)) == -9
    Mneg.rs, Mneg.cs = 5, -1
    assert call(ctypes.byref(T), ctypes.byref(Mneg), 2, ctypes.byref(S)) == -9
    Mbig = matrix(L, 7, 5)
    Mbig.rs = 1 << 26   # 6 * 2^26 * 8 bytes > 2^31
    assert call(ctypes.byref(T), ctypes.byref(Mbig), 2, ctypes.byref(S)) == -4


@no_device
def test_kronsum_argument_errors(lib, L):
    T = tensor(L, [4, 5, 6])
    S = tensor(L, [4, 5, 6], data=FAKE + 0x200000)
    As = [matrix(L, k, k, data=FAKE + 0x400000 + 0x1000 * j) for j, k in enumerate([4, 5, 6])]
    call = lambda t, arr, s, prec=0: lib.kp_kronsum(t, arr, s, prec, None)
    assert call(None, mlist(L, As), ctypes.byref(S)) == -1
    assert call(ctypes.byref(T), mlist(L, [As[0], None, As[2]]), ctypes.byref(S)) == -1
    assert call(ctypes.byref(T), mlist(L, [As[0], matrix(L, 5, 4), As[2]]),
                ctypes.byref(S)) == -4                                  # not square / wrong size
    assert call(ctypes.byref(T), mlist(L, As), ctypes.byref(tensor(L, [4, 5, 7]))) == -4
    assert call(ctypes.byref(T), mlist(L, As), ctypes.byref(S), prec=3) == -5
    assert call(ctypes.byref(T), mlist(L, As), ctypes.byref(tensor(L, [4, 5, 6], data=FAKE))) == -6


@no_device
def test_tucker_argument_errors(lib, L):
    T = tensor(L, [4, 5, 6], dtype=1)
    Ms = [matrix(L, 3, 4, 1), matrix(L, 2, 5, 1), matrix(L, 5, 6, 1)]
    S = tensor(L, [3, 2, 5], dtype=1, data=FAKE + 0x300000)
    arr = mlist(L, Ms)
    need = lib.kp_tucker_workspace(ctypes.byref(T), arr, 0)
    assert need > 0
    # workspace missing / too small is reported before anything is launched
    assert lib.kp_tucker(ctypes.byref(T), arr, ctypes.byref(S), 0, None, 0, None, 0, None) == -7
    assert lib.kp_tucker(ctypes.byref(T), arr, ctypes.byref(S), 0, FAKE + 0x900000, need - 1,
                         None, 0, None) == -7
    bad = mlist(L, [matrix(L, 3, 4, 1), matrix(L, 2, 6, 1), matrix(L, 5, 6, 1)])
    assert lib.kp_tucker(ctypes.byref(T), bad, ctypes.byref(S), 0, None, 0, None, 0, None) == -4
    assert lib.kp_tucker(ctypes.byref(T), arr, ctypes.byref(tensor(L, [3, 2, 4], dtype=1)), 0,
                         None, 0, None, 0, None) == -4
    # cache smaller than required
    cb = lib.kp_tucker_cache_size(ctypes.byref(T), arr)
    assert cb > 0
    assert lib.kp_tucker(ctypes.byref(T), arr, ctypes.byref(S), 0, None, 0, FAKE + 0x900000,
                         cb - 1, None) == -7


@no_device
def test_backward_argument_errors(lib, L):
    T = tensor(L, [4, 5], dtype=0)
    G = tensor(L, [3, 2], dtype=0, data=FAKE + 0x400000)
    Ms = mlist(L, [matrix(L, 3, 4), matrix(L, 2, 5)])
    need = lib.kp_tucker_backward_workspace(ctypes.byref(T), Ms, 0)
    assert need > 0
    dT = tensor(L, [4, 5], data=FAKE + 0x500000)
    assert lib.kp_tucker_backward(ctypes.byref(G), ctypes.byref(T), Ms, None, 0,
                                  ctypes.byref(dT), None, 0, None, 0, None) == -7
    with_null = mlist(L, [matrix(L, 3, 4), None])
    assert lib.kp_tucker_backward(ctypes.byref(G), ctypes.byref(T), with_null, None, 0,
                                  ctypes.byref(dT), None, 0, None, 0, None) == -1
    assert lib.kp_tucker_backward(ctypes.byref(tensor(L, [3, 3], data=FAKE + 0x400000)),
                                  ctypes.byref(T), Ms, None, 0, ctypes.byref(dT), None, 0,
                                  None, 0, None) == -4
    # dT aliasing T
    assert lib.kp_tucker_backward(ctypes.byref(G), ctypes.byref(T), Ms, None, 0,
                                  ctypes.byref(tensor(L, [4, 5])), None, 0,
                                  FAKE + 0x900000, need, None) == -6


@no_device
def test_tucker_workspace_and_cache_alias_errors(lib, L):
    # T at FAKE (4*5*6 floats), factors at FAKE+0x100000 (matrix default),
    # S at FAKE+0x300000; a buffer the call writes (ws, cache) may overlap none
    # of them, nor each other.
    T = tensor(L, [4, 5, 6], dtype=1)
    Ms = [matrix(L, 3, 4, 1, data=FAKE + 0x100000), matrix(L, 2, 5, 1, data=FAKE + 0x110000),
          matrix(L, 5, 6, 1, data=FAKE + 0x120000)]
    S = tensor(L, [3, 2, 5], dtype=1, data=FAKE + 0x300000)
    arr = mlist(L, Ms)
    need = lib.kp_tucker_workspace(ctypes.byref(T), arr, 0)
    cb = lib.kp_tucker_cache_size(ctypes.byref(T), arr)
    ws_ok, cache_ok = FAKE + 0x900000, FAKE + 0xA00000

    def call(ws=ws_ok, nb=need, cache=None, cbytes=0):
        return lib.kp_tucker(ctypes.byref(T), arr, ctypes.byref(S), 0, ws, nb, cache, cbytes,
                             None)
    for bad in (FAKE + 16, FAKE + 0x300000 + 8, FAKE + 0x110000):    # T, S, a factor
        assert call(ws=bad) == -6, hex(bad)
        assert call(ws=None, nb=0, cache=bad, cbytes=cb) == -6, hex(bad)
    assert call(ws=cache_ok + 64, nb=need, cache=cache_ok, cbytes=cb) == -6   # cache vs ws


@no_device
def test_backward_cache_and_output_alias_errors(lib, L):
    T = tensor(L, [4, 5], dtype=0)
    G = tensor(L, [3, 2], dtype=0, data=FAKE + 0x400000)
    Ms = mlist(L, [matrix(L, 3, 4, data=FAKE + 0x100000), matrix(L, 2, 5, data=FAKE + 0x110000)])
    need = lib.kp_tucker_backward_workspace(ctypes.byref(T), Ms, 0)
    cb = lib.kp_tucker_cache_size(ctypes.byref(T), Ms)
    ws, cache = FAKE + 0x900000, FAKE + 0xA00000
    dT = tensor(L, [4, 5], data=FAKE + 0x500000)

    def dl(a0, a1):
        return mlist(L, [matrix(L, 3, 4, data=a0), matrix(L, 2, 5, data=a1)])
    good = dl(FAKE + 0x600000, FAKE + 0x610000)

    def call(w=ws, c=cache, d_T=dT, d_L=good):
        return lib.kp_tucker_backward(ctypes.byref(G), ctypes.byref(T), Ms, c, cb,
                                      ctypes.byref(d_T) if d_T is not None else None, d_L, 0,
                                      w, need, None)
    # a factor gradient written over the cache, dT, or another gradient
    assert call(d_L=dl(cache + 8, FAKE + 0x610000)) == -6
    assert call(d_L=dl(FAKE + 0x500000, FAKE + 0x610000)) == -6
    assert call(d_L=dl(FAKE + 0x600000, FAKE + 0x600008)) == -6
    # the workspace over an input or the cache
    for bad in (FAKE + 8, FAKE + 0x400000, FAKE + 0x110000, cache + 16):
        assert call(w=bad) == -6, hex(bad)


@no_device
def test_expm_argument_errors(lib):
    ws = lib.kp_expm_workspace(128, 3)
    # eight n x n FP64 slots per matrix, then one int per matrix (256-byte aligned)
    assert ws == 8 * 128 * 128 * 3 * 8 + 256
    assert lib.kp_expm_f64(FAKE, 300, 1, 1.0, FAKE * 2, FAKE * 4, 10 ** 9, None) == -4
    assert lib.kp_expm_f64(None, 4, 1, 1.0, FAKE, FAKE * 4, 10 ** 6, None) == -1
    assert lib.kp_expm_f64(FAKE, 4, 1, float("nan"), FAKE * 2, FAKE * 4, 10 ** 6, None) == -9
    assert lib.kp_expm_f64(FAKE, 4, 1, 1.0, FAKE * 2, FAKE * 4, 10, None) == -7
    assert lib.kp_expm_f64(FAKE, 4, 1, 1.0, FAKE + 8, FAKE * 4, 10 ** 6, None) == -6
    assert lib.kp_expm_f64(FAKE, 0, 1, 1.0, FAKE * 2, None, 0, None) == 0


@no_device
def test_tucker_complex_argument_errors(lib, L):
    T = tensor(L, [2, 4, 5])
    S = tensor(L, [2, 3, 6], data=FAKE + 0x200000)
    Re = [matrix(L, 3, 4, data=FAKE + 0x400000), matrix(L, 6, 5, data=FAKE + 0x401000)]
    Im = [matrix(L, 3, 4, data=FAKE + 0x402000), None]
    ws = FAKE + 0x800000
    wsb = lib.kp_tucker_complex_workspace(ctypes.byref(T), mlist(L, Re), mlist(L, Im), 0, 0)
    assert wsb > 0

    def call(t=T, re=Re, im=Im, s=S, conj=0, prec=0, w=ws, nb=wsb):
        return lib.kp_tucker_complex(ctypes.byref(t), mlist(L, re), mlist(L, im),
                                     ctypes.byref(s), conj, prec, w, nb, None)
    assert call(t=tensor(L, [3, 4, 5])) == -4                       # first mode not 2
    assert call(t=tensor(L, [2])) == -2                             # no complex mode
    assert call(re=[None, Re[1]]) == -1                             # imaginary part alone
    assert call(im=[matrix(L, 3, 5), None]) == -4                   # parts differ in size
    assert call(s=tensor(L, [2, 3, 7], data=FAKE + 0x200000)) == -4
    assert call(conj=1) == -4                                       # L^* would be 4 x 3
    assert call(prec=3) == -5
    assert call(nb=wsb - 1) == -7
    assert call(s=tensor(L, [2, 3, 6], data=FAKE + 8)) == -6


@no_device
def test_tridiag_inverse_argument_errors(lib):
    f = lib.kp_tridiag_inverse_f64
    lo, dg, up, E = FAKE, FAKE + 0x1000, FAKE + 0x2000, FAKE + 0x100000
    assert f(lo, dg, up, 2049, 1, 1.0, -1.0, E, None) == -4
    assert f(lo, dg, up, -1, 1, 1.0, -1.0, E, None) == -4
    assert f(lo, dg, up, 4, 65536, 1.0, -1.0, E, None) == -4
    assert f(None, dg, up, 4, 1, 1.0, -1.0, E, None) == -1
    assert f(lo, dg, up, 4, 1, 1.0, -1.0, None, None) == -1
    assert f(lo, dg, up, 4, 1, float("inf"), -1.0, E, None) == -9
    assert f(lo, dg, up, 4, 1, 1.0, float("nan"), E, None) == -9
    assert f(lo, dg, up, 4, 1, 1.0, -1.0, dg + 8, None) == -6
    assert f(lo, dg, up, 0, 1, 1.0, -1.0, E, None) == 0


@no_device
def test_pcg_argument_errors(lib, L):
    B = tensor(L, [4, 5, 6])
    X = tensor(L, [4, 5, 6], data=FAKE + 0x200000)
    Ms = [matrix(L, k, k, data=FAKE + 0x400000 + 0x1000 * j) for j, k in enumerate([4, 5, 6])]
    Ps = [matrix(L, k, k, data=FAKE + 0x500000 + 0x1000 * j) for j, k in enumerate([4, 5, 6])]
    wsb = lib.kp_pcg_workspace(ctypes.byref(X), mlist(L, Ps))
    assert wsb >= 4 * 120 * 8 and lib.kp_pcg_workspace(ctypes.byref(X), None) < wsb
    ws = FAKE + 0x800000

    def call(b=B, m=Ms, p=Ps, x=X, tol=1e-5, maxit=10, w=ws, nb=wsb):
        return lib.kp_pcg_kronsum(ctypes.byref(b), mlist(L, m), None if p is None else mlist(L, p),
                                  None if x is None else ctypes.byref(x), tol, maxit, w, nb,
                                  None, None, None)
    assert call(x=None) == -1
    assert call(m=[Ms[0], None, Ms[2]]) == -1
    assert call(m=[Ms[0], matrix(L, 5, 4), Ms[2]]) == -4
    assert call(p=[Ps[0], matrix(L, 4, 4), Ps[2]]) == -4
    assert call(x=tensor(L, [4, 5, 7], data=FAKE + 0x200000)) == -4
    assert call(b=tensor(L, [4, 5, 6], dtype=1), x=tensor(L, [4, 5, 6], dtype=1)) == -5
    assert call(tol=-1.0) == -9 and call(tol=float("nan")) == -9 and call(maxit=-1) == -9
    assert call(nb=wsb - 1) == -7 and call(w=None) == -7
    assert call(x=tensor(L, [4, 5, 6], data=FAKE + 8)) == -6          # X overlaps B
    assert call(x=tensor(L, [4, 5, 6], data=ws + 64)) == -6            # X overlaps ws


@no_device
def test_semilinear_argument_errors(lib, L):
    dims = (ctypes.c_int64 * 3)(4, 5, 6)
    wsb = lib.kp_semilinear_workspace(3, dims)
    assert wsb > 0
    assert lib.kp_semilinear_workspace(3, (ctypes.c_int64 * 3)(4, 0, 6)) == 0
    assert lib.kp_semilinear_workspace(3, (ctypes.c_int64 * 3)(4, 3000, 6)) == 0
    ptr = lambda base: (ctypes.c_void_p * 3)(*[base + 0x1000 * k for k in range(3)])
    lo, dg, up = ptr(FAKE + 0x300000), ptr(FAKE + 0x310000), ptr(FAKE + 0x320000)
    h = (ctypes.c_double * 3)(0.2, 1 / 6, 1 / 7)
    ws = FAKE + 0x800000

    def call(u=None, lo=lo, dg=dg, up=up, h=h, tau=0.01, steps=3, tol=1e-5, maxit=10, w=ws,
             nb=wsb):
        u = tensor(L, [4, 5, 6]) if u is None else u
        return lib.kp_semilinear_imex_f64(ctypes.byref(u), lo, dg, up, h, 0.0, tau, steps, tol,
                                          maxit, 1, w, nb, None, None)
    assert call(u=tensor(L, [4, 5, 6], dtype=1)) == -5
    assert call(u=tensor(L, [4, 5, 3000])) == -4
    assert call(lo=(ctypes.c_void_p * 3)(FAKE, None, FAKE)) == -1
    assert call(h=(ctypes.c_double * 3)(0.2, -1.0, 0.1)) == -9
    assert call(tau=float("inf")) == -9 and call(steps=-1) == -9 and call(maxit=-1) == -9
    assert call(nb=wsb - 1) == -7
    assert call(u=tensor(L, [4, 5, 6], data=ws + 8)) == -6


def test_force_tile_argument_errors(lib):
    assert lib.kp_force_tile(4, 0, 16, 0, 0, 0) == -9
    assert lib.kp_force_tile(4, 1, 16, 0, 3, 0) == -9
    assert lib.kp_force_tile(4, 1, 16, 0, 0, 2) == -9
    assert lib.kp_force_tile(0, 0, 0, 0, 0, 0) == 0


def test_workspace_sizes(lib, L):
    # cube200 FP64: two ping-pong buffers of one 8M-entry intermediate each
    T = tensor(L, [200, 200, 200])
    arr = mlist(L, [matrix(L, 200, 200)] * 3)
    assert lib.kp_tucker_workspace(ctypes.byref(T), arr, 0) == 2 * 200 ** 3 * 8
    assert lib.kp_tucker_cache_size(ctypes.byref(T), arr) == 2 * 200 ** 3 * 8
    # interp6d FP32: cache holds P_1..P_5
    T6 = tensor(L, [16] * 6, dtype=1)
    arr6 = mlist(L, [matrix(L, 24, 16, 1)] * 6)
    want = sum(((24 ** k) * 16 ** (6 - k) * 4 + 255) // 256 * 256 for k in range(1, 6))
    assert lib.kp_tucker_cache_size(ctypes.byref(T6), arr6) == want


def test_workspace_counts_split_planes(lib, L):
    # BF16 split forms: after the intermediates, one plane set per factor:
    # ceil(n/16) row blocks x ceil(m/32) k steps x P planes x 1 KB (64 lanes
    # x 8 bf16), each set rounded to 256 bytes; FP32 native counts none
    dims, rows = [181, 200, 197], [204, 185, 200]
    T = tensor(L, dims, dtype=1)
    arr = mlist(L, [matrix(L, rows[k], dims[k], 1) for k in range(3)])
    base = lib.kp_tucker_workspace(ctypes.byref(T), arr, 0)
    assert base > 0
    for prec, planes in ((3, 2), (6, 3)):
        want = sum((((n + 15) // 16) * ((m + 31) // 32) * planes * 1024 + 255) // 256 * 256
                   for n, m in zip(rows, dims))
        assert lib.kp_tucker_workspace(ctypes.byref(T), arr, prec) == base + want
    # a single product still gets its planes (no intermediates)
    T1 = tensor(L, [200, 64], dtype=1)
    arr1 = mlist(L, [matrix(L, 200, 200, 1), None])
    assert lib.kp_tucker_workspace(ctypes.byref(T1), arr1, 0) == 0
    assert lib.kp_tucker_workspace(ctypes.byref(T1), arr1, 6) == 13 * 7 * 3 * 1024


def test_complex_workspace_counts_split_planes(lib, L):
    # BF16 split forms: after the intermediates and the packed factor parts,
    # one plane set per factor part as applied (n x m, also for the conjugate
    # transpose, whose factors are given m x n); FP32 native counts none
    dims, rows = [2, 181, 200, 197], [204, 185, 200]
    for conj in (0, 1):
        shp = [(dims[k + 1], rows[k]) if conj else (rows[k], dims[k + 1]) for k in range(3)]
        Re = mlist(L, [matrix(L, r, c, 1) for r, c in shp])
        Im = mlist(L, [matrix(L, r, c, 1) for r, c in shp[:2]] + [None])
        T = tensor(L, dims, dtype=1)
        base = lib.kp_tucker_complex_workspace(ctypes.byref(T), Re, Im, conj, 0)
        assert base > 0
        for prec, planes in ((3, 2), (6, 3)):
            want = sum(parts * ((((n + 15) // 16) * ((m + 31) // 32) * planes * 1024 + 255)
                                // 256 * 256)
                       for n, m, parts in zip(rows, dims[1:], (2, 2, 1)))
            assert lib.kp_tucker_complex_workspace(ctypes.byref(T), Re, Im, conj, prec) == \
                base + want


@pytest.mark.parametrize("seed", range(8))
def test_planned_order_minimises_flops(lib, L, seed):
    rng = np.random.default_rng(900 + seed)
    d = int(rng.integers(2, 6))
    m = [int(x) for x in rng.integers(1, 40, size=d)]
    n = [int(x) for x in rng.integers(1, 40, size=d)]
    T = tensor(L, m)
    arr = mlist(L, [matrix(L, n[k], m[k]) for k in range(d)])
    order = (ctypes.c_int * 8)()
    cnt = ctypes.c_int()
    assert lib.kp_tucker_order(ctypes.byref(T), arr, order, ctypes.byref(cnt)) == 0
    got = [order[k] for k in range(cnt.value)]
    assert sorted(got) == list(range(1, d + 1))
    best = min(kp_workloads.tucker_flops(m, n, p)
               for p in itertools.permutations(range(1, d + 1)))
    assert kp_workloads.tucker_flops(m, n, got) == best


def test_planned_order_skips_identity_factors(lib, L):
    T = tensor(L, [5, 6, 7])
    arr = mlist(L, [None, matrix(L, 3, 6), None])
    order = (ctypes.c_int * 8)()
    cnt = ctypes.c_int()
    assert lib.kp_tucker_order(ctypes.byref(T), arr, order, ctypes.byref(cnt)) == 0
    assert cnt.value == 1 and order[0] == 2


def test_binding_refuses_cpu_tensors():
    import torch
    import paper_2112_11238_amd as kp
    with pytest.raises(ValueError, match="GPU tensors only"):
        kp.tucker(torch.zeros(3, 3, dtype=torch.float64), [None, None])
    with pytest.raises(ValueError, match="GPU tensors only"):
        kp.mump(torch.zeros(3, 3), torch.zeros(2, 3), 1)
