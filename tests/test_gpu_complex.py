"""Complex Tucker operator and its conjugate-transpose form on the device
(Sec. 2 over C; Sec. 3 spectral transforms) against the oracle and numpy's
FFT, in every form."""
import numpy as np
import pytest
import torch

import kp_workloads
import oracle
from gpu_util import say, unit_error

pytestmark = pytest.mark.gpu

FORMS = [("c128", "native"), ("c64", "native"), ("c64", "bf16x3"), ("c64", "bf16x6")]
CDT = {"c128": torch.complex128, "c64": torch.complex64}
RDT = {"c128": torch.float64, "c64": torch.float32}
CASES = [((7, 5), (4, 9)), ((19, 45, 13), (7, 70, 29)), ((30, 3, 70), (2, 33, 64)),
         ((5, 6, 4, 3), (3, 7, 2, 5))]


@pytest.fixture(scope="module")
def kp():
    import paper_2112_11238_amd as kp
    return kp


def dev(x, cdt):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=cdt)


def seen(x, cdt):
    """The values the device sees, back in complex128."""
    return torch.as_tensor(x).to(cdt).to(torch.complex128).numpy()


def bound(T, Ls, conj, prec, rdt, safety=2.0):
    """Componentwise bound for either part of S: the real Tucker operator on
    |Re| + |Im| of T and of each factor, times the summed per-mode error
    coefficients (two real products of length m and the combining add)."""
    absT = np.abs(T.real) + np.abs(T.imag)
    absL = []
    for L in Ls:
        a = np.abs(L.real) + np.abs(L.imag)
        absL.append(a.T if conj else a)
    u = 2.0 ** -53 if rdt == torch.float64 else 2.0 ** -24
    coef = sum(unit_error(prec, rdt, 2 * T.shape[k]) + 2 * u for k in range(T.ndim))
    return safety * coef * oracle.tucker(absT, absL) + 1e-300


@pytest.mark.parametrize("form,prec", FORMS)
@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("conj", [False, True])
def test_tucker_complex_matches_oracle(kp, form, prec, case, conj):
    m, n = CASES[case]
    T, Ls = kp_workloads.complex_problem(500 + case, m, n, conj)
    say("complex tucker", m, n, form, prec, "conj" if conj else "")
    S = kp.tucker_complex(dev(T, CDT[form]), [dev(L, CDT[form]) for L in Ls], conj=conj,
                          prec=prec)
    torch.cuda.synchronize()
    T64, L64 = seen(T, CDT[form]), [seen(L, CDT[form]) for L in Ls]
    ref = oracle.cttucker(T64, L64) if conj else oracle.ztucker(T64, L64)
    got = S.to(torch.complex128).cpu().numpy()
    assert got.shape == ref.shape
    b = bound(T64, L64, conj, prec, RDT[form])
    assert np.all(np.abs(got.real - ref.real) <= b)
    assert np.all(np.abs(got.imag - ref.imag) <= b)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16x6"])
@pytest.mark.parametrize("conj", [False, True])
def test_complex_presplit_planes_bitwise(kp, prec, conj):
    """Split-form products on wide tiles (n > 176) read bf16 planes of the
    packed factor parts, split once per call. The same call with a
    workspace that holds only the intermediates and the packed parts (each
    tile then splits its rows itself) must agree with it bit for bit, and
    both with the oracle within the form's bound. Ragged: rows past n in the
    last tile, a k tail in the last step; the third mode runs on a k-loop
    tile without planes."""
    import ctypes
    from paper_2112_11238_amd import ops
    m, n = (181, 200, 64), (204, 185, 40)
    T, Ls = kp_workloads.complex_problem(77, m, n, conj)
    Td = dev(T, torch.complex64)
    Ld = [dev(L, torch.complex64) for L in Ls]
    say("complex presplit planes", prec, "conj" if conj else "")
    S_full = kp.tucker_complex(Td, Ld, conj=conj, prec=prec)

    lb = ops.lib()
    td = ops._tdesc(torch.view_as_real(Td), True)
    Lv = [torch.view_as_real(L) for L in Ld]
    rarr = ops._mlist([ops._mdesc(v[..., 0]) for v in Lv][::-1])
    iarr = ops._mlist([ops._mdesc(v[..., 1]) for v in Lv][::-1])
    c = 1 if conj else 0
    full = lb.kp_tucker_complex_workspace(ctypes.byref(td), rarr, iarr, c, ops._prec(prec))
    base = lb.kp_tucker_complex_workspace(ctypes.byref(td), rarr, iarr, c, ops._prec("native"))
    assert 0 < base < full                    # the planes take room of their own
    S_inreg = torch.empty_like(S_full)
    sd = ops._tdesc(torch.view_as_real(S_inreg), True)
    ws = torch.empty(base, dtype=torch.uint8, device="cuda")
    st = lb.kp_tucker_complex(ctypes.byref(td), rarr, iarr, ctypes.byref(sd), c, ops._prec(prec),
                              ws.data_ptr(), base, ops._stream())
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(S_full), torch.view_as_real(S_inreg))

    T64, L64 = seen(T, torch.complex64), [seen(L, torch.complex64) for L in Ls]
    ref = oracle.cttucker(T64, L64) if conj else oracle.ztucker(T64, L64)
    got = S_full.to(torch.complex128).cpu().numpy()
    b = bound(T64, L64, conj, prec, torch.float32)
    assert np.all(np.abs(got.real - ref.real) <= b)
    assert np.all(np.abs(got.imag - ref.imag) <= b)


def test_complex_planes_split_in_two_launches(kp):
    """Wide tiles forced on every mode of an order-5 complex problem: ten
    factor parts read as planes, more than one split launch holds (eight),
    so they are split in two launches. Bit for bit against the same call
    with a workspace without room for planes, and within the bound of the
    oracle. Tiny ragged sizes: every tile is mostly rows past n and k past m."""
    import ctypes
    from paper_2112_11238_amd import ops
    m, n = (5, 7, 6, 4, 9), (6, 5, 8, 3, 7)
    T, Ls = kp_workloads.complex_problem(78, m, n)
    Td = dev(T, torch.complex64)
    Ld = [dev(L, torch.complex64) for L in Ls]
    say("complex planes, two split launches")
    lb = ops.lib()
    td = ops._tdesc(torch.view_as_real(Td), True)
    Lv = [torch.view_as_real(L) for L in Ld]
    rarr = ops._mlist([ops._mdesc(v[..., 0]) for v in Lv][::-1])
    iarr = ops._mlist([ops._mdesc(v[..., 1]) for v in Lv][::-1])
    p = ops._prec("bf16x3")
    full = lb.kp_tucker_complex_workspace(ctypes.byref(td), rarr, iarr, 0, p)
    base = lb.kp_tucker_complex_workspace(ctypes.byref(td), rarr, iarr, 0, ops._prec("native"))
    assert 0 < base < full
    out = []
    kp.force_tile(2, 4, 32, 2, 2, 3)
    try:
        for nbytes in (full, base):
            S = torch.empty(n, dtype=torch.complex64, device="cuda")
            sd = ops._tdesc(torch.view_as_real(S), True)
            ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            st = lb.kp_tucker_complex(ctypes.byref(td), rarr, iarr, ctypes.byref(sd), 0, p,
                                      ws.data_ptr(), nbytes, ops._stream())
            assert st == 0
            torch.cuda.synchronize()
            out.append(S)
    finally:
        kp.force_tile(0)
    assert torch.equal(torch.view_as_real(out[0]), torch.view_as_real(out[1]))
    T64, L64 = seen(T, torch.complex64), [seen(L, torch.complex64) for L in Ls]
    ref = oracle.ztucker(T64, L64)
    got = out[0].to(torch.complex128).cpu().numpy()
    b = bound(T64, L64, False, "bf16x3", torch.float32)
    assert np.all(np.abs(got.real - ref.real) <= b)
    assert np.all(np.abs(got.imag - ref.imag) <= b)


def test_fourier_transform_and_inverse(kp):
    shape = (64, 48, 30)
    rng = np.random.default_rng(9)
    T = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Fs = [dev(kp_workloads.fourier_matrix(k), torch.complex128) for k in shape]
    say("fourier", shape)
    S = kp.tucker_complex(dev(T, torch.complex128), Fs)
    back = kp.tucker_complex(S, Fs, conj=True)
    torch.cuda.synchronize()
    ref = np.fft.fftn(T)
    got = S.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    inv = back.cpu().numpy() / T.size
    assert np.max(np.abs(inv - T)) <= 1e-12 * np.max(np.abs(T))


@pytest.mark.parametrize("form", ["c128", "c64"])
def test_identity_and_real_factors(kp, form):
    rng = np.random.default_rng(10)
    T = rng.standard_normal((6, 5, 7)) + 1j * rng.standard_normal((6, 5, 7))
    Lr = rng.standard_normal((4, 5))
    Lc = rng.standard_normal((3, 7)) + 1j * rng.standard_normal((3, 7))
    rdt = RDT[form]
    say("complex mixed factors", form)
    S = kp.tucker_complex(dev(T, CDT[form]),
                          [None, torch.as_tensor(Lr).to(device="cuda", dtype=rdt),
                           dev(Lc, CDT[form])])
    same = kp.tucker_complex(dev(T, CDT[form]), [None, None, None])
    torch.cuda.synchronize()
    T64 = seen(T, CDT[form])
    L64 = [None, torch.as_tensor(Lr).to(rdt).double().numpy(), seen(Lc, CDT[form])]
    ref = oracle.ztucker(T64, L64)
    b = bound(T64, [np.eye(6), L64[1], L64[2]], False, "native", rdt)
    got = S.to(torch.complex128).cpu().numpy()
    assert np.all(np.abs(got.real - ref.real) <= b) and np.all(np.abs(got.imag - ref.imag) <= b)
    assert torch.equal(same, dev(T, CDT[form]))


def test_order_one_and_transposed_views(kp):
    rng = np.random.default_rng(11)
    v = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    A = rng.standard_normal((40, 25)) + 1j * rng.standard_normal((40, 25))
    # conjugate transpose of a 40 x 25 factor maps length 40 to length 25
    S = kp.tucker_complex(dev(v, torch.complex128), [dev(A, torch.complex128)], conj=True)
    torch.cuda.synchronize()
    ref = A.conj().T @ v
    assert np.max(np.abs(S.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
    # a transposed (non-contiguous) complex factor view
    T = rng.standard_normal((5, 6, 7)) + 1j * rng.standard_normal((5, 6, 7))
    B = rng.standard_normal((6, 4)) + 1j * rng.standard_normal((6, 4))       # B^T is 4 x 6
    S = kp.tucker_complex(dev(T, torch.complex128), [None, dev(B, torch.complex128).t(), None])
    torch.cuda.synchronize()
    ref = oracle.ztucker(T, [None, B.T, None])
    assert np.max(np.abs(S.cpu().numpy() - ref)) <= 1e-13 * np.max(np.abs(ref))
