"""Shared test helpers: inputs from the seeded generator, the componentwise
error measure, and small conveniences around torch device buffers."""
from __future__ import annotations

import numpy as np

import sj_inputs as gen

LAYOUTS = gen.LAYOUTS
# FP64 parity bar: |gpu - oracle| <= TOL_F64 * sum_d |L||psi| for every output.
# Any summation order or use of FMA stays within gamma_D = D*u/(1-D*u) of the
# exact sum (u = 2^-53), i.e. 1.1e-14 at D = 96, far below this bar.
TOL_F64 = 1e-12


def componentwise_err(got, ref, scale):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    diff = np.abs(got - ref)
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.where(scale > 0, diff / scale, np.where(diff == 0, 0.0, np.inf))
    return float(rel.max()) if rel.size else 0.0


def contraction_inputs(seed, layout, Z, G, D, NM):
    """(L, Lplus, psi stored in layout, phi input stored in layout), float64 numpy."""
    psi = gen.to_layout(gen.psi_logical(seed, D, G, Z), layout).ravel()
    L = gen.matrix_sym(seed, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(seed, gen.ARR_LPLUS, D, NM)
    phi = gen.to_layout(gen.sym(seed, gen.ARR_PHI, np.arange(NM * G * Z, dtype=np.uint64)).reshape(NM, G, Z),
                        layout).ravel()
    return L, Lp, psi, phi


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
