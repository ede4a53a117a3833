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


def layout_flat_index(layout, A, G, Z, a, g, z):
    """Flat storage offset of logical element (a, g, z) of an (A, G, Z) array
    stored in ``layout`` order (rightmost letter fastest).  Index bookkeeping only."""
    ext = {"D": A, "G": G, "Z": Z}
    val = {"D": np.asarray(a, dtype=np.int64), "G": np.asarray(g, dtype=np.int64),
           "Z": np.asarray(z, dtype=np.int64)}
    idx = np.zeros(np.broadcast(val["D"], val["G"], val["Z"]).shape, dtype=np.int64)
    for c in layout:
        idx = idx * ext[c] + val[c]
    return idx


def sample_columns(seed, G, Z, n):
    """n sampled (g, z) columns, the first and last column always included."""
    rng = np.random.default_rng(seed)
    g = rng.integers(0, G, n)
    z = rng.integers(0, Z, n)
    g[:2], z[:2] = [0, G - 1], [0, Z - 1]
    return g, z


def gather_columns(out_d, layout, A, G, Z, g, z):
    """Rows 0..A-1 of the sampled columns of a device array stored in
    ``layout``: a (A, len(g)) float64 host array (a device gather, then a small copy)."""
    import torch
    idx = layout_flat_index(layout, A, G, Z, np.arange(A)[:, None], g[None, :], z[None, :])
    return host(torch.take(out_d, torch.from_numpy(idx).cuda()))
