"""torch-facing binding of the C-ABI: argument marshalling only.

Tensors use the paper's indexing: a tensor T of order d is a torch tensor of
shape (m_1, ..., m_d) whose element T[j_1, ..., j_d] is t_{j_1...j_d}; a
factor L_mu is a torch tensor of shape (n_mu, m_mu), any strides. Every step
of the computation runs in libkp.so's HIP kernels; this module only builds
descriptors, allocates outputs and workspaces through torch, and passes the
current stream.

Layout mapping. The library's tensors are column-major (mode 1 contiguous).
A row-major (C-contiguous) torch tensor of shape (m_1..m_d) holds the same
bytes as the column-major tensor of dims (m_d..m_1); so the binding passes
C-contiguous tensors (making non-contiguous inputs contiguous first), with the
dims and the factor list reversed and mode mu mapped to d+1-mu.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import KpMatrix, KpTensor, check

PRECISIONS = {"native": _lib.KP_PREC_NATIVE, "bf16x3": _lib.KP_PREC_BF16X3,
              "bf16x6": _lib.KP_PREC_BF16X6,
              _lib.KP_PREC_NATIVE: _lib.KP_PREC_NATIVE,
              _lib.KP_PREC_BF16X3: _lib.KP_PREC_BF16X3,
              _lib.KP_PREC_BF16X6: _lib.KP_PREC_BF16X6}


def lib():
    return _lib.load()


def _prec(prec):
    if prec not in PRECISIONS:
        raise ValueError(f"unknown precision {prec!r}; use 'native', 'bf16x3' or 'bf16x6'")
    return PRECISIONS[prec]


def _dtype_code(t):
    if t.dtype == torch.float64:
        return _lib.KP_F64
    if t.dtype == torch.float32:
        return _lib.KP_F32
    raise TypeError(f"unsupported dtype {t.dtype}; use float64 or float32")


def _canon(t):
    """The tensor as a C-contiguous torch tensor (library dims = reversed shape)."""
    if t.dim() == 0:
        raise ValueError("a tensor of order >= 1 is required")
    return t if t.is_contiguous() else t.contiguous()


def _tdesc(t, rev):
    d = t.dim()
    if d > _lib.KP_MAX_ORDER:
        raise ValueError(f"order {d} exceeds {_lib.KP_MAX_ORDER}")
    desc = KpTensor()
    desc.d = d
    desc.dtype = _dtype_code(t)
    dims = list(t.shape)
    if rev:
        dims = dims[::-1]
    for k in range(d):
        desc.dims[k] = dims[k]
    desc.data = t.data_ptr() if t.numel() > 0 else None
    return desc


def _mdesc(L):
    if L.dim() != 2:
        raise ValueError("factors must be matrices")
    desc = KpMatrix()
    desc.rows, desc.cols = L.shape
    desc.rs, desc.cs = L.stride()
    desc.dtype = _dtype_code(L)
    desc.data = L.data_ptr() if L.numel() > 0 else None
    return desc


def _mlist(descs):
    arr = (ctypes.POINTER(KpMatrix) * len(descs))()
    for k, dsc in enumerate(descs):
        arr[k] = ctypes.pointer(dsc) if dsc is not None else None
    return arr


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_device(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("libkp operates on GPU tensors only (no CPU path)")


def mump(T, L, mu, prec="native", out=None, accumulate=False):
    """S = T x_mu L (mu is 1-based, as in the paper)."""
    _check_device(T, L)
    d = T.dim()
    if not 1 <= mu <= d:
        raise ValueError(f"mode {mu} outside 1..{d}")
    Tc = _canon(T)
    shape = list(T.shape)
    shape[mu - 1] = L.shape[0]
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs an output tensor")
        out = torch.empty(shape, dtype=T.dtype, device=T.device)
    elif list(out.shape) != shape or not out.is_contiguous():
        raise ValueError("output must be a contiguous tensor of the result's shape")
    td, sd = _tdesc(Tc, True), _tdesc(out, True)
    st = lib().kp_mump(ctypes.byref(td), ctypes.byref(_mdesc(L)), d + 1 - mu, ctypes.byref(sd),
                       _prec(prec), 1 if accumulate else 0, _stream())
    check(st, "kp_mump")
    return out


def kronsum(T, As, prec="native", out=None):
    """S = T x_1 A_1 + ... + T x_d A_d: the action of the Kronecker sum of the
    square A_mu on vec(T) (kp_kronsum)."""
    _check_device(T, *As)
    d = T.dim()
    if len(As) != d:
        raise ValueError(f"need {d} matrices, got {len(As)}")
    Tc = _canon(T)
    if out is None:
        out = torch.empty_like(Tc)
    elif list(out.shape) != list(T.shape) or not out.is_contiguous():
        raise ValueError("output must be a contiguous tensor of T's shape")
    td, sd = _tdesc(Tc, True), _tdesc(out, True)
    arr = _mlist([_mdesc(A) for A in As][::-1])
    check(lib().kp_kronsum(ctypes.byref(td), arr, ctypes.byref(sd), _prec(prec), _stream()),
          "kp_kronsum")
    return out


def _tucker_call(T, Ls, prec, want_cache):
    _check_device(T, *Ls)
    d = T.dim()
    if len(Ls) != d:
        raise ValueError(f"need {d} factors, got {len(Ls)}")
    Tc = _canon(T)
    shape = [T.shape[k] if Ls[k] is None else Ls[k].shape[0] for k in range(d)]
    out = torch.empty(shape, dtype=T.dtype, device=T.device)
    mds = [None if L is None else _mdesc(L) for L in Ls]
    mds = mds[::-1]
    td, sd = _tdesc(Tc, True), _tdesc(out, True)
    arr = _mlist(mds)
    p = _prec(prec)
    lb = lib()
    ws_bytes = lb.kp_tucker_workspace(ctypes.byref(td), arr, p)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=T.device)
    cache = None
    cache_ptr, cache_bytes = None, 0
    if want_cache:
        cache_bytes = lb.kp_tucker_cache_size(ctypes.byref(td), arr)
        cache = torch.empty(max(cache_bytes, 1), dtype=torch.uint8, device=T.device)
        cache_ptr = cache.data_ptr()
    st = lb.kp_tucker(ctypes.byref(td), arr, ctypes.byref(sd), p, ws.data_ptr(), ws_bytes,
                      cache_ptr, cache_bytes, _stream())
    check(st, "kp_tucker")
    return out, cache


def tucker(T, Ls, prec="native"):
    """S = T x_1 L_1 x_2 ... x_d L_d. ``Ls[k] = None`` is the identity."""
    return _tucker_call(T, Ls, prec, False)[0]


def tucker_noalloc(T, Ls, prec="native", out=None):
    """S = T x_1 L_1 x_2 ... x_d L_d with the intermediates in the library's
    fixed device buffer (kp_tucker_noalloc): no workspace is allocated, and
    with ``out`` given (contiguous, S's shape and dtype) nothing at all.
    Calls that overlap in time on one device race on that buffer."""
    _check_device(T, *Ls)
    d = T.dim()
    if len(Ls) != d:
        raise ValueError(f"need {d} factors, got {len(Ls)}")
    Tc = _canon(T)
    shape = [T.shape[k] if Ls[k] is None else Ls[k].shape[0] for k in range(d)]
    if out is None:
        out = torch.empty(shape, dtype=T.dtype, device=T.device)
    elif list(out.shape) != shape or out.dtype != T.dtype or not out.is_contiguous():
        raise ValueError("output must be a contiguous tensor of S's shape and T's dtype")
    mds = [None if L is None else _mdesc(L) for L in Ls][::-1]
    td, sd = _tdesc(Tc, True), _tdesc(out, True)
    check(lib().kp_tucker_noalloc(ctypes.byref(td), _mlist(mds), ctypes.byref(sd), _prec(prec),
                                  _stream()), "kp_tucker_noalloc")
    return out


def tucker_backward(G, T, Ls, prec="native", cache=None, need_dT=True, need_dL=None):
    """Gradient of <G, tucker(T, Ls)>: returns (dT, [dL_1, ..., dL_d]).

    dT = G x_1 L_1^T ... x_d L_d^T, dL_mu = Q_mu^(mu) P_{mu-1}^(mu)^T (see
    include/kp.h). ``cache`` is the forward cache returned by
    ``tucker_with_cache`` (None: the partial products are recomputed).
    ``need_dL`` is a list of booleans (default: all); skipped entries are None.
    """
    _check_device(G, T, *Ls)
    d = T.dim()
    if len(Ls) != d or any(L is None for L in Ls):
        raise ValueError("the backward needs all d factors")
    if need_dL is None:
        need_dL = [True] * d
    Tc, Gc = _canon(T), _canon(G)
    dT = torch.empty_like(Tc) if need_dT else None
    dLs = [torch.empty(L.shape, dtype=T.dtype, device=T.device) if need_dL[k] else None
           for k, L in enumerate(Ls)]
    td, gd = _tdesc(Tc, True), _tdesc(Gc, True)
    mds = [_mdesc(L) for L in Ls][::-1]
    dls = [None if x is None else _mdesc(x) for x in dLs][::-1]
    arr, darr = _mlist(mds), _mlist(dls)
    p = _prec(prec)
    lb = lib()
    ws_bytes = lb.kp_tucker_backward_workspace(ctypes.byref(td), arr, p)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=T.device)
    dtd = _tdesc(dT, True) if dT is not None else None
    cache_ptr = cache.data_ptr() if cache is not None else None
    cache_bytes = cache.numel() if cache is not None else 0
    st = lb.kp_tucker_backward(ctypes.byref(gd), ctypes.byref(td), arr, cache_ptr, cache_bytes,
                               ctypes.byref(dtd) if dtd is not None else None, darr, p,
                               ws.data_ptr(), ws_bytes, _stream())
    check(st, "kp_tucker_backward")
    return dT, dLs


def tucker_with_cache(T, Ls, prec="native"):
    """Tucker operator that also returns the forward cache of partial
    products P_1..P_{d-1} (a uint8 device buffer) for tucker_backward."""
    return _tucker_call(T, Ls, prec, True)


class TuckerFunction(torch.autograd.Function):
    """S = T x_1 L_1 ... x_d L_d with the hand-written backward.

    forward(T, prec, cache_partials, *Ls); with cache_partials the forward
    keeps P_1..P_{d-1} for the backward, otherwise they are recomputed."""

    @staticmethod
    def forward(ctx, T, prec, cache_partials, *Ls):
        if cache_partials:
            S, cache = tucker_with_cache(T, list(Ls), prec)
        else:
            S, cache = tucker(T, list(Ls), prec), None
        ctx.prec = prec
        ctx.cache = cache
        ctx.save_for_backward(T, *Ls)
        return S

    @staticmethod
    def backward(ctx, G):
        T, *Ls = ctx.saved_tensors
        need = ctx.needs_input_grad
        dT, dLs = tucker_backward(G.contiguous(), T, Ls, ctx.prec, ctx.cache,
                                  need_dT=need[0], need_dL=list(need[3:]))
        ctx.cache = None
        return (dT, None, None, *dLs)


def tucker_autograd(T, Ls, prec="native", cache_partials=True):
    """Differentiable Tucker operator (torch.autograd) over libkp's kernels."""
    return TuckerFunction.apply(T, prec, cache_partials, *Ls)


def expm(A, tau=1.0):
    """exp(tau * A) in FP64 on the device for a square matrix A (n <= 256) or
    a batch of them (shape (count, n, n)). Scaling and squaring with the
    degree-13 Pade approximant, every step on the device (kp_expm_f64)."""
    _check_device(A)
    if A.dtype != torch.float64:
        raise TypeError("expm runs in float64")
    batched = A.dim() == 3
    Ab = A if batched else A.unsqueeze(0)
    if Ab.dim() != 3 or Ab.shape[1] != Ab.shape[2]:
        raise ValueError("expects square matrices")
    count, n = Ab.shape[0], Ab.shape[1]
    # the library reads column-major matrices: pass A^T row-major = A col-major
    Ac = Ab.transpose(1, 2).contiguous()
    E = torch.empty_like(Ac)
    lb = lib()
    ws_bytes = lb.kp_expm_workspace(n, count)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=A.device)
    st = lb.kp_expm_f64(Ac.data_ptr(), n, count, float(tau), E.data_ptr(), ws.data_ptr(),
                        ws_bytes, _stream())
    check(st, "kp_expm_f64")
    E = E.transpose(1, 2)
    return E if batched else E[0]


def tucker_complex(T, Ls, conj=False, prec="native"):
    """Complex Tucker operator S = T x_1 L_1 ... x_d L_d (conj: the conjugate
    transposes L_mu^*, each L_mu then m_mu x n_mu) for complex128 / complex64
    T; a factor may be complex, real (same real dtype) or None (identity).
    Zero-copy: the interleaved storage is passed as real views
    (kp_tucker_complex)."""
    _check_device(T, *Ls)
    if T.dtype not in (torch.complex128, torch.complex64):
        raise TypeError("tucker_complex expects a complex128 or complex64 tensor")
    d = T.dim()
    if len(Ls) != d:
        raise ValueError(f"need {d} factors, got {len(Ls)}")
    rdt = torch.float64 if T.dtype == torch.complex128 else torch.float32
    Tr = torch.view_as_real(T.contiguous())            # (m_1..m_d, 2): (2, m_d..m_1) canonical
    res, ims = [], []
    for L in Ls:
        if L is None:
            res.append(None)
            ims.append(None)
        elif L.is_complex():
            if L.dtype != T.dtype:
                raise TypeError("complex factors must share T's dtype")
            Lv = torch.view_as_real(L)                 # (rows, cols, 2), any strides
            res.append(_mdesc(Lv[..., 0]))
            ims.append(_mdesc(Lv[..., 1]))
        else:
            if L.dtype != rdt:
                raise TypeError("real factors must have T's real dtype")
            res.append(_mdesc(L))
            ims.append(None)
    shape = []
    for k in range(d):
        if Ls[k] is None:
            shape.append(T.shape[k])
        else:
            shape.append(Ls[k].shape[1] if conj else Ls[k].shape[0])
    S = torch.empty(shape, dtype=T.dtype, device=T.device)
    Sr = torch.view_as_real(S)
    td, sd = _tdesc(Tr, True), _tdesc(Sr, True)
    rarr, iarr = _mlist(res[::-1]), _mlist(ims[::-1])
    lb = lib()
    c = 1 if conj else 0
    ws_bytes = lb.kp_tucker_complex_workspace(ctypes.byref(td), rarr, iarr, c, _prec(prec))
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=T.device)
    st = lb.kp_tucker_complex(ctypes.byref(td), rarr, iarr, ctypes.byref(sd), c, _prec(prec),
                              ws.data_ptr(), ws_bytes, _stream())
    check(st, "kp_tucker_complex")
    return S


def _f64_device(*ts):
    _check_device(*ts)
    for t in ts:
        if t is not None and t.dtype != torch.float64:
            raise TypeError("this operation runs in float64")


def tridiag_inverse(lower, diag, upper, shift=0.0, scale=1.0):
    """(shift I + scale T)^{-1} in FP64 on the device for the tridiagonal T
    with T[i, i-1] = lower[i], T[i, i] = diag[i], T[i, i+1] = upper[i]
    (vectors of length n, or (count, n) for a batch); elimination without
    pivoting per identity column (kp_tridiag_inverse_f64). With shift=1,
    scale=-tau this is an ADI factor (I - tau A)^{-1}."""
    _f64_device(lower, diag, upper)
    batched = diag.dim() == 2
    lo, dg, up = [(x if batched else x.unsqueeze(0)).contiguous() for x in (lower, diag, upper)]
    if not (lo.shape == dg.shape == up.shape) or dg.dim() != 2:
        raise ValueError("diagonals must share the shape (n,) or (count, n)")
    count, n = dg.shape
    E = torch.empty((count, n, n), dtype=torch.float64, device=dg.device)
    st = lib().kp_tridiag_inverse_f64(lo.data_ptr(), dg.data_ptr(), up.data_ptr(), n, count,
                                      float(shift), float(scale), E.data_ptr(), _stream())
    check(st, "kp_tridiag_inverse_f64")
    E = E.transpose(1, 2)  # the library writes column-major matrices
    return E if batched else E[0]


def pcg_kronsum(B, Ms, Ps=None, x0=None, tol=1e-5, maxit=1000):
    """Solve (M_d (+) ... (+) M_1) x = b (the Kronecker sum acting on B as
    sum_mu B x_mu M_mu) by preconditioned conjugate gradients in FP64 with the
    preconditioner action R x_1 Ps[0] ... x_d Ps[d-1] (Ps None: plain CG; a
    None entry: identity), from x0 (zeros if None). Returns (X, iterations,
    relative residual). Blocks until done (kp_pcg_kronsum)."""
    _f64_device(B, x0, *Ms, *(Ps or []))
    d = B.dim()
    if len(Ms) != d or (Ps is not None and len(Ps) != d):
        raise ValueError(f"need {d} matrices per list")
    Bc = _canon(B)
    X = torch.zeros_like(Bc) if x0 is None else _canon(x0).clone()
    bd, xd = _tdesc(Bc, True), _tdesc(X, True)
    marr = _mlist([_mdesc(M) for M in Ms][::-1])
    parr = None if Ps is None else _mlist([None if Pm is None else _mdesc(Pm) for Pm in Ps][::-1])
    lb = lib()
    ws_bytes = lb.kp_pcg_workspace(ctypes.byref(xd), parr)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=B.device)
    it, res = ctypes.c_int(0), ctypes.c_double(0.0)
    st = lb.kp_pcg_kronsum(ctypes.byref(bd), marr, parr, ctypes.byref(xd), float(tol), int(maxit),
                           ws.data_ptr(), ws_bytes, ctypes.byref(it), ctypes.byref(res), _stream())
    check(st, "kp_pcg_kronsum")
    return X, it.value, res.value


def semilinear_imex(U, lower, diag, upper, h, tau, steps, t0=0.0, tol=1e-5, maxit=1000,
                    precondition=True):
    """Backward-forward Euler steps of the semilinear experiment on the
    device, in place on U (axis mu-1 = x_mu, interior grid points
    x = (i+1) h[mu]): lower/diag/upper[mu] are the diagonals of the second
    difference of axis mu (device vectors). Returns the PCG iterations of
    each step (kp_semilinear_imex_f64)."""
    _f64_device(U, *lower, *diag, *upper)
    d = U.dim()
    if not (len(lower) == len(diag) == len(upper) == len(h) == d):
        raise ValueError(f"need {d} diagonals and spacings")
    if not U.is_contiguous():
        raise ValueError("U must be contiguous (it is updated in place)")
    ud = _tdesc(U, True)
    vecs = [[v.contiguous() for v in arr][::-1] for arr in (lower, diag, upper)]
    ptrs = [(ctypes.c_void_p * d)(*[v.data_ptr() for v in arr]) for arr in vecs]
    hs = (ctypes.c_double * d)(*[float(x) for x in h][::-1])
    dims = (ctypes.c_int64 * d)(*list(U.shape)[::-1])
    lb = lib()
    ws_bytes = lb.kp_semilinear_workspace(d, dims)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=U.device)
    its = (ctypes.c_int * max(int(steps), 1))()
    st = lb.kp_semilinear_imex_f64(ctypes.byref(ud), ptrs[0], ptrs[1], ptrs[2], hs, float(t0),
                                   float(tau), int(steps), float(tol), int(maxit),
                                   1 if precondition else 0, ws.data_ptr(), ws_bytes, its,
                                   _stream())
    check(st, "kp_semilinear_imex_f64")
    return [its[k] for k in range(int(steps))]


class BatchedTucker:
    """Many independent Tucker operators (and optionally their gradients):
    one persistent launch per dependency level and task type
    (kp_tucker_batched).

    Ts[k] is a tensor of order d_k, Ls[k] its d_k factors (no None); all share
    a dtype. With ``Gs`` (cotangents, shapes of the outputs) the backward runs
    in the same launch: ``dT[k]`` (if need_dT) and ``dL[k][mu]`` (if need_dL).
    Outputs, workspace and the device copy of the plan are allocated once
    here; ``run()`` only enqueues the level launches on the current stream,
    so it can be captured into a CUDA/HIP graph and replayed; the inputs can
    be overwritten in place between runs.
    """

    def __init__(self, Ts, Ls, prec="native", Gs=None, need_dT=True, need_dL=True):
        if len(Ts) != len(Ls):
            raise ValueError("one factor list per tensor")
        _check_device(*Ts)
        self.prec = _prec(prec)
        self.Ts = [_canon(T) for T in Ts]
        self.Ls = [list(L) for L in Ls]
        self.Gs = None if Gs is None else [_canon(G) for G in Gs]
        count = len(Ts)
        dev = Ts[0].device if count else torch.device("cuda")
        self.S = []
        self.dT = [] if Gs is not None and need_dT else None
        self.dL = [] if Gs is not None and need_dL else None
        items = (_lib.KpBatchItem * max(count, 1))()
        self._keep = []
        for k in range(count):
            T, L = self.Ts[k], self.Ls[k]
            d = T.dim()
            if len(L) != d or any(x is None for x in L):
                raise ValueError("each problem needs all d factors")
            S = torch.empty([x.shape[0] for x in L], dtype=T.dtype, device=T.device)
            self.S.append(S)
            it = items[k]
            it.T = _tdesc(T, True)
            it.S = _tdesc(S, True)
            for j, x in enumerate(L[::-1]):
                it.L[j] = _mdesc(x)
            if self.Gs is not None:
                G = self.Gs[k]
                if list(G.shape) != list(S.shape):
                    raise ValueError("cotangent shape must match the output")
                it.G = _tdesc(G, True)
                if self.dT is not None:
                    dT = torch.empty_like(T)
                    self.dT.append(dT)
                    it.dT = _tdesc(dT, True)
                if self.dL is not None:
                    dls = [torch.empty(x.shape, dtype=T.dtype, device=T.device) for x in L]
                    self.dL.append(dls)
                    for j, x in enumerate(dls[::-1]):
                        it.dL[j] = _mdesc(x)
        lb = lib()
        self._items = items
        self.count = count
        ws_bytes = lb.kp_batch_workspace(count, items, self.prec)
        plan_bytes = lb.kp_batch_plan_bytes(count, items, self.prec)
        if count and (ws_bytes == 0 or plan_bytes == 0):
            raise ValueError("invalid batch (see include/kp.h for the limits)")
        self.ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=dev)
        self.plan_host = (ctypes.c_char * max(plan_bytes, 1))()
        check(lb.kp_batch_plan(count, items, self.prec, self.ws.data_ptr(), self.ws.numel(),
                               self.plan_host, plan_bytes), "kp_batch_plan")
        self.plan_bytes = plan_bytes
        self._upload()
        nt = ctypes.c_int64()
        ns = ctypes.c_int()
        nl = ctypes.c_int()
        check(lb.kp_batch_info(self.plan_host, ctypes.byref(nt), ctypes.byref(ns),
                               ctypes.byref(nl)), "kp_batch_info")
        self.ntasks, self.nstages, self.nlevels = nt.value, ns.value, nl.value

    def _upload(self):
        host = torch.frombuffer(bytearray(bytes(self.plan_host)), dtype=torch.uint8)
        self.plan_dev = host.to(self.ws.device)
        torch.cuda.current_stream().synchronize()

    def run(self):
        st = lib().kp_tucker_batched(self.plan_dev.data_ptr(), self.plan_host,
                                     self.ws.data_ptr(), self.ws.numel(), _stream())
        check(st, "kp_tucker_batched")
        return self.S


def force_tile(nb=0, fb=0, bk=0, occ=0, pf=0, kind=0):
    """Force the mode-kernel tile for later launches (nb=0 resets); kind 1
    selects a strip tile (bk = padded contraction length >= m), kind 3 a wide
    tile of the BF16 split forms (nb 16-row blocks per wave, fb 16-fiber
    blocks, bk 32)."""
    check(lib().kp_force_tile(nb, fb, bk, occ, pf, kind), "kp_force_tile")
