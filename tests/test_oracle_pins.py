"""Pins of the FP64 CPU oracle against things other than itself: exact rational
arithmetic, closed forms, invariants and library routines.  CPU only."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import sj_inputs as gen
from sj_inputs import quadrature as quad

U = 2.0 ** -53
LAYOUTS = gen.LAYOUTS


def gamma(n):
    return n * U / (1 - n * U)


def logical_inputs(seed, D, G, Z, NM):
    psi = gen.psi_logical(seed, D, G, Z)
    L = gen.matrix_sym(seed, gen.ARR_L, NM, D)
    Lp = gen.matrix_sym(seed, gen.ARR_LPLUS, D, NM)
    return psi, L, Lp


def exact_ltimes(L, psi_log):
    """Exact rational phi[nm,g,z] = sum_d L[nm,d] psi[d,g,z] (logical arrays)."""
    NM, D = L.shape
    _, G, Z = psi_log.shape
    out = np.empty((NM, G, Z), dtype=object)
    Lf = [[Fraction(float(v)) for v in row] for row in L]
    for g in range(G):
        for z in range(Z):
            col = [Fraction(float(psi_log[d, g, z])) for d in range(D)]
            for nm in range(NM):
                out[nm, g, z] = sum((Lf[nm][d] * col[d] for d in range(D)), Fraction(0))
    return out


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(3, 2, 5, 4), (1, 1, 1, 1), (2, 3, 6, 3), (3, 3, 4, 2)])
def test_ltimes_exact_rational(orc, layout, shape):
    """(i) The oracle is within gamma_D * sum|L||psi| of the exact rational sum,
    for every nesting and shapes where NM != D and G != Z (so a transposed
    operand or swapped axis fails)."""
    Z, G, D, NM = shape
    psi, L, _ = logical_inputs(11, D, G, Z, NM)
    phi = orc.ltimes(layout, Z, G, D, NM, L, gen.to_layout(psi, layout))
    phi_log = gen.from_layout(phi, layout, NM, G, Z)
    ex = exact_ltimes(L, psi)
    scale = np.einsum("nd,dgz->ngz", np.abs(L), np.abs(psi))
    for idx in itertools.product(range(NM), range(G), range(Z)):
        err = abs(Fraction(float(phi_log[idx])) - ex[idx])
        assert err <= Fraction(gamma(D) * scale[idx]) + Fraction(1, 2 ** 1074)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_lplustimes_exact_rational(orc, layout):
    Z, G, D, NM = 4, 3, 5, 4
    _, _, Lp = logical_inputs(12, D, G, Z, NM)
    phi_log = gen.sym(12, gen.ARR_PHI, np.arange(NM * G * Z, dtype=np.uint64)).reshape(NM, G, Z)
    out = orc.lplustimes(layout, Z, G, D, NM, Lp, gen.to_layout(phi_log, layout))
    out_log = gen.from_layout(out, layout, D, G, Z)
    ex = exact_ltimes(Lp, phi_log)  # same contraction shape: [D][NM] x [NM,G,Z]
    scale = np.einsum("dn,ngz->dgz", np.abs(Lp), np.abs(phi_log))
    for idx in itertools.product(range(D), range(G), range(Z)):
        err = abs(Fraction(float(out_log[idx])) - ex[idx])
        assert err <= Fraction(gamma(NM) * scale[idx])


def test_ltimes_midsize_rational(orc):
    """Exact rational check at the benchmark's D and NM on a few columns."""
    Z, G, D, NM = 7, 3, 96, 16
    psi, L, _ = logical_inputs(0, D, G, Z, NM)
    phi = orc.ltimes("DGZ", Z, G, D, NM, L, gen.to_layout(psi, "DGZ")).reshape(NM, G, Z)
    ex = exact_ltimes(L, psi)
    scale = np.einsum("nd,dgz->ngz", np.abs(L), np.abs(psi))
    worst = max(float(abs(Fraction(float(phi[i])) - ex[i])) / scale[i] for i in np.ndindex(NM, G, Z))
    assert worst <= gamma(D)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_onehot_row_gather_bitexact(orc, layout):
    """(ii) L[nm,d] = delta(d, pi(nm)) makes phi a row gather of psi, bit-exact."""
    Z, G, D, NM = 5, 3, 7, 4
    psi = gen.psi_logical(3, D, G, Z)
    pi = np.array([6, 0, 3, 3])
    L = np.zeros((NM, D))
    L[np.arange(NM), pi] = 1.0
    phi = gen.from_layout(orc.ltimes(layout, Z, G, D, NM, L, gen.to_layout(psi, layout)), layout, NM, G, Z)
    assert np.array_equal(phi, psi[pi])
    Lp = np.zeros((D, NM))
    Lp[pi, np.arange(NM)] = 1.0
    phi_in = gen.psi_logical(4, NM, G, Z)
    out = gen.from_layout(orc.lplustimes(layout, Z, G, D, NM, Lp, gen.to_layout(phi_in, layout)), layout, D, G, Z)
    expect = np.zeros((D, G, Z))
    for nm in range(NM):
        expect[pi[nm]] += phi_in[nm]  # rows pi are hit once except the repeated 3
    # d = 3 receives phi[2] + phi[3]: a single add, exact to the last bit in both
    assert np.array_equal(out, expect)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_integer_inputs_bitexact(orc, layout):
    """(iii) integer-valued inputs: every partial sum is an exact integer, so the
    result equals integer arithmetic bit for bit."""
    Z, G, D, NM = 6, 5, 13, 7
    rng = np.random.default_rng(5)
    Li = rng.integers(-4, 5, size=(NM, D))
    pi = rng.integers(0, 8, size=(D, G, Z))
    phi = gen.from_layout(orc.ltimes(layout, Z, G, D, NM, Li.astype(float), gen.to_layout(pi.astype(float), layout)),
                          layout, NM, G, Z)
    assert np.array_equal(phi, np.einsum("nd,dgz->ngz", Li, pi).astype(float))
    Lpi = rng.integers(-4, 5, size=(D, NM))
    phii = rng.integers(-7, 8, size=(NM, G, Z))
    out = gen.from_layout(orc.lplustimes(layout, Z, G, D, NM, Lpi.astype(float), gen.to_layout(phii.astype(float), layout)),
                          layout, D, G, Z)
    assert np.array_equal(out, np.einsum("dn,ngz->dgz", Lpi, phii).astype(float))


def test_assoc_legendre_vs_scipy():
    """The quadrature's Legendre recurrence agrees with scipy's lpmv (which carries
    the Condon-Shortley phase (-1)^m)."""
    from scipy.special import lpmv
    x = np.linspace(-0.99, 0.99, 17)
    P = quad.assoc_legendre(7, x)
    for n in range(8):
        for m in range(n + 1):
            assert np.allclose(P[n, m], (-1) ** m * lpmv(m, n, x), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("DNM", list(quad.SETS))
def test_quadrature_identity_closed_form(orc, DNM):
    """(iv) On a matching quadrature, L*L+ = I_NM, so LTimes(LPlusTimes(phi)) = phi,
    and P = L+ L is idempotent.  The harmonics' orthonormality is checked on a
    finer rule first (independent of the rule under test)."""
    D, NM = DNM
    lmax, n_mu, n_phi = quad.SETS[DNM]
    mu, ph, w = quad.product_quadrature(2 * lmax + 2, 4 * lmax + 3)
    Y = quad.real_sph_harm(lmax, mu, ph)
    assert np.abs((Y * w) @ Y.T - np.eye(NM)).max() < 1e-13
    L, Lp = quad.moment_matrices(lmax, n_mu, n_phi)
    assert L.shape == (NM, D)
    Z, G = 9, 2
    phi = gen.sym(1, gen.ARR_PHI, np.arange(NM * G * Z, dtype=np.uint64))
    for layout in ("DGZ", "ZGD"):
        psi2 = orc.lplustimes(layout, Z, G, D, NM, Lp, phi)
        back = orc.ltimes(layout, Z, G, D, NM, L, psi2)
        assert np.abs(back - phi).max() < 5e-14
    P = Lp @ L
    assert np.abs(P @ P - P).max() < 1e-13


def test_six_layouts_agree_bitwise(orc):
    """(v) all six nestings give bit-identical logical results (same sum order)."""
    Z, G, D, NM = 7, 5, 11, 6
    psi, L, Lp = logical_inputs(2, D, G, Z, NM)
    ref = None
    for layout in LAYOUTS:
        phi = gen.from_layout(orc.ltimes(layout, Z, G, D, NM, L, gen.to_layout(psi, layout)), layout, NM, G, Z)
        out = gen.from_layout(orc.lplustimes(layout, Z, G, D, NM, Lp, gen.to_layout(phi, layout)), layout, D, G, Z)
        if ref is None:
            ref = (phi, out)
        else:
            assert np.array_equal(phi, ref[0]) and np.array_equal(out, ref[1])


def test_column_independence(orc):
    """(vi) a zone slab computed alone equals the same slab of the full run."""
    Z, G, D, NM = 12, 3, 9, 5
    psi, L, _ = logical_inputs(6, D, G, Z, NM)
    full = orc.ltimes("DGZ", Z, G, D, NM, L, psi).reshape(NM, G, Z)
    z0, z1 = 4, 9
    part = orc.ltimes("DGZ", z1 - z0, G, D, NM, L, np.ascontiguousarray(psi[:, :, z0:z1])).reshape(NM, G, z1 - z0)
    assert np.array_equal(part, full[:, :, z0:z1])
    cols = gen.psi_columns(6, D, G, Z, [0, 2, 1], [3, 11, 0])
    samp = orc.ltimes("DGZ", 3, 1, D, NM, L, cols).reshape(NM, 3)
    assert np.array_equal(samp, np.stack([full[:, 0, 3], full[:, 2, 11], full[:, 1, 0]], axis=1))


def test_unknown_layout_rejected(orc):
    with pytest.raises(ValueError):
        orc.ltimes(7, 1, 1, 1, 1, np.zeros(1), np.zeros(1))


def test_absscale_is_sum_of_abs(orc):
    Z, G, D, NM = 3, 2, 5, 3
    psi, L, _ = logical_inputs(8, D, G, Z, NM)
    s = orc.ltimes_absscale("GDZ", Z, G, D, NM, L, gen.to_layout(psi, "GDZ"))
    ref = np.einsum("nd,dgz->ngz", np.abs(L), np.abs(psi))
    assert np.allclose(gen.from_layout(s, "GDZ", NM, G, Z), ref, rtol=1e-14, atol=0)


# ----------------------------------------------------------------- batched


def _batch(seed, count, lo=3, hi=16):
    n = gen.batch_sizes(seed, count, lo, hi)
    off = gen.batch_offsets(n)
    A = gen.batch_normal(seed, gen.ARR_A, int(off[-1]))
    B = gen.batch_normal(seed, gen.ARR_B, int(off[-1]))
    return n, off, A, B


def test_bgemm_exact_rational(orc):
    n, off, A, B = _batch(3, 40, 1, 4)
    C = orc.bgemm(n, off[:-1], A, B)
    for i, s in enumerate(n):
        a = A[off[i]:off[i] + s * s].reshape(s, s)
        b = B[off[i]:off[i] + s * s].reshape(s, s)
        c = C[off[i]:off[i] + s * s].reshape(s, s)
        for r in range(s):
            for col in range(s):
                ex = sum((Fraction(float(a[r, k])) * Fraction(float(b[k, col])) for k in range(s)), Fraction(0))
                bound = gamma(s) * float(np.abs(a[r]) @ np.abs(b[:, col]))
                assert abs(Fraction(float(c[r, col])) - ex) <= Fraction(bound)


def test_bgemm_identity_permutation_integer(orc):
    n = np.array([3, 16, 7, 1, 5], dtype=np.int32)
    off = gen.batch_offsets(n)
    rng = np.random.default_rng(1)
    B = rng.standard_normal(off[-1])
    A = np.zeros(off[-1])
    P = np.zeros(off[-1])
    for i, s in enumerate(n):
        A[off[i]:off[i + 1]] = np.eye(s).ravel()
        P[off[i]:off[i + 1]] = np.eye(s)[rng.permutation(s)].ravel()
    assert np.array_equal(orc.bgemm(n, off[:-1], A, B), B)
    C = orc.bgemm(n, off[:-1], P, B)
    for i, s in enumerate(n):
        p = P[off[i]:off[i + 1]].reshape(s, s)
        assert np.array_equal(C[off[i]:off[i + 1]].reshape(s, s), p @ B[off[i]:off[i + 1]].reshape(s, s))
    Ai = rng.integers(-9, 10, off[-1])
    Bi = rng.integers(-9, 10, off[-1])
    C = orc.bgemm(n, off[:-1], Ai.astype(float), Bi.astype(float))
    for i, s in enumerate(n):
        ref = Ai[off[i]:off[i + 1]].reshape(s, s) @ Bi[off[i]:off[i + 1]].reshape(s, s)
        assert np.array_equal(C[off[i]:off[i + 1]], ref.ravel().astype(float))


def test_bgemm_matches_numpy_within_bound(orc):
    n, off, A, B = _batch(0, 500)
    C = orc.bgemm(n, off[:-1], A, B)
    for i in range(0, 500, 7):
        s = n[i]
        a = A[off[i]:off[i + 1]].reshape(s, s)
        b = B[off[i]:off[i + 1]].reshape(s, s)
        ref = a @ b
        bound = 2 * gamma(s) * (np.abs(a) @ np.abs(b))
        assert np.all(np.abs(C[off[i]:off[i + 1]].reshape(s, s) - ref) <= bound)


# -------------------------------------------------------------------- BF16


def test_bf16_round_vs_torch_and_ties(orc):
    """RNE to bfloat16: agrees with torch's float32 -> bfloat16 conversion on
    float32-representable values; explicit ties go to the even neighbour."""
    import torch
    rng = np.random.default_rng(0)
    x32 = np.concatenate([rng.standard_normal(2000), rng.uniform(-1, 1, 2000) * 1e-5]).astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([orc.bf16_round(float(v)) for v in x32])
    assert np.array_equal(got, ref)
    assert orc.bf16_round(1.0 + 2.0 ** -8) == 1.0               # tie -> even (1.0)
    assert orc.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie -> even (...10)
    assert orc.bf16_round(-(1.0 + 2.0 ** -8 + 2.0 ** -40)) == -(1.0 + 2.0 ** -7)  # just above a tie


def test_bf16_round_fp64_nearest_bruteforce(orc):
    """FP64 inputs round in one step to the nearest 8-bit-significand value."""
    rng = np.random.default_rng(1)
    for x in rng.uniform(-4, 4, 300):
        r = orc.bf16_round(float(x))
        e = math.floor(math.log2(abs(x)))
        step = 2.0 ** (e - 7)
        cands = [math.floor(x / step) * step, math.ceil(x / step) * step]
        best = min(abs(c - x) for c in cands)
        assert abs(r - x) == best


def test_bf16_emulation_bounds(orc):
    """Exactly-bf16 inputs: plain == compensated == FP64 oracle.  Random inputs:
    the emulated error is within the split-product bound."""
    Z, G, D, NM = 8, 2, 32, 6
    psi, L, _ = logical_inputs(4, D, G, Z, NM)
    rb = np.vectorize(orc.bf16_round)
    Lb, pb = rb(L), rb(psi)
    ex = orc.ltimes("DGZ", Z, G, D, NM, Lb, pb)
    for mode in (0, 1):
        assert np.array_equal(orc.ltimes_bf16_emul(mode, "DGZ", Z, G, D, NM, Lb, pb), ex)
    ex = orc.ltimes("DGZ", Z, G, D, NM, L, psi)
    scale = orc.ltimes_absscale("DGZ", Z, G, D, NM, L, psi)
    ub = 2.0 ** -8
    e0 = np.abs(orc.ltimes_bf16_emul(0, "DGZ", Z, G, D, NM, L, psi) - ex) / scale
    e1 = np.abs(orc.ltimes_bf16_emul(1, "DGZ", Z, G, D, NM, L, psi) - ex) / scale
    assert e0.max() <= 2 * ub + ub * ub + gamma(3 * D)
    assert e1.max() <= 3 * ub * ub + gamma(3 * D)
    assert e1.max() < e0.max() / 20


def bf16_exact(x: Fraction) -> Fraction:
    """Nearest value with 8 significant bits, ties to even, on rationals: the
    definition of round-to-nearest-even bfloat16 for normal results."""
    if x == 0:
        return Fraction(0)
    s = -1 if x < 0 else 1
    a = abs(x)
    e = 0
    while a >= 2 ** e:
        e += 1
    while a < 2 ** (e - 1):
        e -= 1
    # 2^(e-1) <= a < 2^e: keep 8 bits, i.e. a multiple of 2^(e-8)
    r = round(a * Fraction(2) ** (8 - e))      # Fraction.__round__ rounds ties to even
    return s * r * Fraction(2) ** (e - 8)


@pytest.mark.parametrize("layout", ["DGZ", "GZD", "ZDG"])
def test_bf16_emulation_exact_split(orc, layout):
    """The split emulation against exact rational arithmetic at a tiny shape:
    hi = RNE_bf16(x), lo = RNE_bf16(x - hi) formed on rationals, every product
    and the sum exact; the oracle (FP64 products and sums) must be within
    gamma_{3D} * sum |terms| of it.  Inputs are not bf16 values, so lo != 0 and
    an unrounded or dropped lo, or a dropped cross term, fails."""
    Z, G, D, NM = 3, 2, 6, 4
    psi, L, _ = logical_inputs(9, D, G, Z, NM)
    for v in np.concatenate([L.ravel(), psi.ravel()]):
        assert Fraction(float(orc.bf16_round(float(v)))) == bf16_exact(Fraction(float(v)))

    def split(v):
        h = bf16_exact(Fraction(float(v)))
        return h, bf16_exact(Fraction(float(v)) - h)
    Ls = [[split(L[nm, d]) for d in range(D)] for nm in range(NM)]
    for mode in (0, 1):
        got = gen.from_layout(orc.ltimes_bf16_emul(mode, layout, Z, G, D, NM, L, gen.to_layout(psi, layout)),
                              layout, NM, G, Z)
        for g, z in itertools.product(range(G), range(Z)):
            ps = [split(psi[d, g, z]) for d in range(D)]
            assert any(lo != 0 for _, lo in ps)
            for nm in range(NM):
                terms = []
                for d in range(D):
                    (lh, ll), (ph, pl) = Ls[nm][d], ps[d]
                    terms.append(lh * ph)
                    if mode == 1:
                        terms += [lh * pl, ll * ph]
                ex = sum(terms, Fraction(0))
                bound = Fraction(gamma(3 * D)) * sum(abs(t) for t in terms)
                assert abs(Fraction(float(got[nm, g, z])) - ex) <= bound


# --------------------------------------------------------------------- MLP


def _mlp_setup(F=9, H=8, R=13, seed=2):
    rng = np.random.default_rng(seed)
    import oracle
    P = oracle.mlp_nparams(F, H)
    theta = rng.standard_normal(P) * 0.5
    X = rng.standard_normal((R, F))
    t = rng.standard_normal(R)
    return F, H, theta, X, t


def test_mlp_forward_vs_numpy(orc):
    F, H, theta, X, t = _mlp_setup()
    W1 = theta[:H * F].reshape(H, F)
    b1 = theta[H * F:H * F + H]
    o = H * F + H
    W2 = theta[o:o + H * H].reshape(H, H)
    b2 = theta[o + H * H:o + H * H + H]
    w3 = theta[o + H * H + H:o + H * H + 2 * H]
    b3 = theta[-1]
    h1 = np.maximum(X @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    ref = h2 @ w3 + b3
    assert np.allclose(orc.mlp_forward(F, H, theta, X), ref, rtol=1e-13, atol=1e-13)


def test_mlp_gradient_finite_differences(orc):
    F, H, theta, X, t = _mlp_setup()
    loss, g = orc.mlp_loss_grad(F, H, theta, X, t)
    y = orc.mlp_forward(F, H, theta, X)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-13
    h = 1e-6
    fd = np.empty_like(theta)
    for p in range(theta.size):
        tp = theta.copy(); tp[p] += h
        tm = theta.copy(); tm[p] -= h
        fd[p] = (orc.mlp_loss_grad(F, H, tp, X, t)[0] - orc.mlp_loss_grad(F, H, tm, X, t)[0]) / (2 * h)
    assert np.linalg.norm(fd - g) <= 1e-6 * np.linalg.norm(g)


def test_adam_first_step_closed_form(orc):
    """At step 1, mh = g and vh = g^2, so p1 = p0 - lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p0 = p.copy()
    m = np.zeros(50)
    v = np.zeros(50)
    orc.adam(p, g, m, v, 1, lr=0.01)
    assert np.allclose(p, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-15)
    # second step against the recurrence written out by hand
    g2 = rng.standard_normal(50)
    m2 = 0.9 * m + 0.1 * g2
    v2 = 0.999 * v + 0.001 * g2 * g2
    exp = p - 0.01 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    orc.adam(p, g2, m, v, 2, lr=0.01)
    assert np.allclose(p, exp, rtol=1e-14, atol=1e-15)


# ----------------------------------------------------------- the generator


def test_generator_reference_values():
    """SplitMix64 from the published definition: seed 0, outputs 1..3 of the
    plain generator (state += GAMMA; mix) as recorded in tests/golden."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "splitmix64.json")) as f:
        gold = json.load(f)
    z = np.array([(k * 0x9E3779B97F4A7C15) % 2 ** 64 for k in (1, 2, 3)], dtype=np.uint64)
    assert [int(v) for v in gen.mix64(z)] == gold["seed0_first3"]


def test_generator_logical_indexing():
    D, G, Z = 4, 3, 5
    full = gen.psi_logical(9, D, G, Z)
    cols = gen.psi_columns(9, D, G, Z, [2, 0], [4, 1])
    assert np.array_equal(cols[:, 0], full[:, 2, 4]) and np.array_equal(cols[:, 1], full[:, 0, 1])
    for layout in LAYOUTS:
        assert np.array_equal(gen.from_layout(gen.to_layout(full, layout), layout, D, G, Z), full)
