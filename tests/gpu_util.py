"""Helpers for the GPU parity tests: error bounds and conversions.

The HIP results are compared with the FP64 oracle on the same inputs (the
low-precision inputs promoted back to float64). Two criteria:

* a componentwise a-priori bound: for a chain of mu-mode products each
  output entry obeys |S - S_ref| <= sum_mu u_mu(m_mu) * Tucker(|T|; |L_mu|),
  the standard bound for inner products of length m evaluated in a
  floating-point format with unit roundoff u, gamma_m = m u / (1 - m u),
  applied mode by mode (first order in u). For the BF16 split forms u_mu
  also carries the truncation of the split products (|a b - sum of kept
  products| <= c 2^-16 |a||b| for x3 with c = 3, c 2^-24 with c = 6 for x6);
* the precision targets stated for the method's forms: max-norm relative
  error <= 1e-13 for FP64 and <= 1e-6 for FP32 and BF16x6 (the paper's own
  error metric is the relative error in maximum norm, Sec. 4.3 and 4.4).
"""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def unit_error(prec, dtype, m):
    """Per-mode relative error coefficient for an inner product of length m."""
    if dtype == torch.float64:
        u = U64
        trunc = 0.0
    else:
        u = U32
        trunc = {"native": 0.0, "bf16x3": 3 * 2.0 ** -16, "bf16x6": 6 * 2.0 ** -24}[prec]
    mu = max(m, 1) + 2
    return trunc + mu * u / (1 - mu * u)


def chain_bound(T, Ls, prec, dtype, safety=2.0):
    """Componentwise bound for S = Tucker(T; Ls) computed in (prec, dtype)."""
    absS = oracle.tucker(np.abs(T), [None if L is None else np.abs(L) for L in Ls])
    coef = sum(unit_error(prec, dtype, T.shape[k]) for k in range(T.ndim) if Ls[k] is not None)
    return safety * coef * absS + 1e-300


def to_dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def cast64(x, dtype):
    """The values the GPU sees (x rounded to dtype), back in float64."""
    return torch.as_tensor(x).to(dtype).to(torch.float64).numpy()


def rel_max(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def say(*args):
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()
