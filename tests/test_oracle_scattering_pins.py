"""Pins of the oracle's scattering operator (CPU only):
    phi_out[nm,g,z] = sum_g' S[mat(z)][n(nm)][g][g'] * phi[nm,g',z],  n(nm) = floor(sqrt(nm)).
The operator is a reading (the paper names Kripke's scattering kernel but does
not define it); these checks pin the oracle to that definition by means other
than its own code: exact rational sums, integer arithmetic, closed forms for
diagonal and permutation matrices, and the degree of each moment."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import sj_inputs as gen

U = 2.0 ** -53
LAYOUTS = gen.LAYOUTS


def degrees(NM):
    """Moments ordered by degree: n copies... degree n owns nm = n^2 .. n^2 + 2n."""
    out = []
    n = 0
    while len(out) < NM:
        out += [n] * (2 * n + 1)
        n += 1
    return out[:NM]


def brute(S, mat, phi_log):
    """Exact rational scattering of logical phi [NM][G][Z]."""
    NM, G, Z = phi_log.shape
    deg = degrees(NM)
    out = np.empty((NM, G, Z), dtype=object)
    for nm, g, z in itertools.product(range(NM), range(G), range(Z)):
        Sm = S[mat[z], deg[nm]]
        out[nm, g, z] = sum((Fraction(float(Sm[g, gp])) * Fraction(float(phi_log[nm, gp, z])) for gp in range(G)),
                            Fraction(0))
    return out


def inputs(seed, Z, G, NM, nmat):
    rng = np.random.default_rng(seed)
    nl = math.isqrt(NM - 1) + 1
    S = rng.uniform(-1.0, 1.0, (nmat, nl, G, G))
    mat = rng.integers(0, nmat, Z).astype(np.int32)
    phi = rng.uniform(-1.0, 1.0, (NM, G, Z))
    return S, mat, phi


def test_degree_table():
    assert degrees(16) == [0, 1, 1, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 3]
    assert degrees(10) == [0, 1, 1, 1, 2, 2, 2, 2, 2, 3]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("shape", [(3, 2, 4, 2), (2, 3, 10, 3), (1, 1, 1, 1), (4, 5, 9, 1)])
def test_scattering_exact_rational(orc, layout, shape):
    """Within gamma_G * sum|S||phi| of the exact sum, every nesting; G != Z and
    non-symmetric S, so a transposed S or swapped axis fails."""
    Z, G, NM, nmat = shape
    S, mat, phi = inputs(31, Z, G, NM, nmat)
    got = gen.from_layout(orc.scattering(layout, Z, G, NM, S, mat, gen.to_layout(phi, layout)), layout, NM, G, Z)
    scale = gen.from_layout(orc.scattering(layout, Z, G, NM, S, mat, gen.to_layout(phi, layout), absolute=True),
                            layout, NM, G, Z)
    ex = brute(S, mat, phi)
    gam = G * U / (1 - G * U)
    for idx in itertools.product(range(NM), range(G), range(Z)):
        assert abs(Fraction(float(got[idx])) - ex[idx]) <= Fraction(gam * scale[idx]) + Fraction(1, 2 ** 1074)


@pytest.mark.parametrize("layout", ["DGZ", "ZDG", "GZD"])
def test_scattering_integer_bitexact(orc, layout):
    """Integer S and phi: every partial sum is exact, so the oracle equals the
    brute-force sum bit for bit."""
    Z, G, NM, nmat = 5, 7, 9, 3
    rng = np.random.default_rng(32)
    S = rng.integers(-4, 5, (nmat, 3, G, G)).astype(np.float64)
    mat = rng.integers(0, nmat, Z).astype(np.int32)
    phi = rng.integers(0, 8, (NM, G, Z)).astype(np.float64)
    got = gen.from_layout(orc.scattering(layout, Z, G, NM, S, mat, gen.to_layout(phi, layout)), layout, NM, G, Z)
    ex = brute(S, mat, phi)
    assert all(got[i] == float(ex[i]) for i in itertools.product(range(NM), range(G), range(Z)))


def test_scattering_degree_and_material_closed_form(orc):
    """S[m][n] = (1 + n + 10 m) I: phi_out = (1 + n(nm) + 10 mat(z)) phi exactly,
    which pins the moment-to-degree map and the material lookup."""
    Z, G, NM, nmat = 6, 4, 16, 3
    mat = np.array([0, 2, 1, 1, 0, 2], dtype=np.int32)
    S = np.zeros((nmat, 4, G, G))
    for m, n in itertools.product(range(nmat), range(4)):
        S[m, n] = (1 + n + 10 * m) * np.eye(G)
    phi = np.random.default_rng(33).integers(-50, 50, (NM, G, Z)).astype(np.float64)
    got = gen.from_layout(orc.scattering("GDZ", Z, G, NM, S, mat, gen.to_layout(phi, "GDZ")), "GDZ", NM, G, Z)
    fac = (1 + np.array(degrees(NM))[:, None, None] + 10 * mat[None, None, :])
    assert np.array_equal(got, fac * phi)


def test_scattering_permutation_gather(orc):
    """One 1 per row of S: phi_out[nm, g, z] = phi[nm, p(g), z], bit-exact."""
    Z, G, NM = 7, 6, 4
    perm = np.array([3, 0, 5, 1, 2, 4])
    P1 = np.zeros((G, G))
    P1[np.arange(G), perm] = 1.0
    S = np.broadcast_to(P1, (1, 2, G, G)).copy()
    phi = np.random.default_rng(34).uniform(-1, 1, (NM, G, Z))
    got = gen.from_layout(orc.scattering("ZGD", Z, G, NM, S, np.zeros(Z, np.int32), gen.to_layout(phi, "ZGD")),
                          "ZGD", NM, G, Z)
    assert np.array_equal(got, phi[:, perm, :])


def test_scattering_layouts_agree_bitwise(orc):
    Z, G, NM, nmat = 9, 5, 10, 2
    S, mat, phi = inputs(35, Z, G, NM, nmat)
    ref = None
    for lay in LAYOUTS:
        got = gen.from_layout(orc.scattering(lay, Z, G, NM, S, mat, gen.to_layout(phi, lay)), lay, NM, G, Z)
        if ref is None:
            ref = got
        assert np.array_equal(got, ref)


def test_scattering_rejects_bad_material(orc):
    Z, G, NM = 3, 2, 4
    with pytest.raises(ValueError):
        orc.scattering("DGZ", Z, G, NM, np.ones((1, 2, G, G)), np.array([0, 1, 0], np.int32), np.zeros(NM * G * Z))


def absscale_reference(S, mat, phi):
    """sum_g' |S[mat(z)][n(nm)][g][g']| |phi[nm,g',z]| built with numpy's einsum
    from the degree table and the material map (logical [NM][G][Z])."""
    deg = np.array(degrees(phi.shape[0]))
    Sz = np.abs(S)[mat][:, deg]                    # [Z][NM][G][G'] of the zone's material and moment's degree
    return np.einsum("znab,nbz->naz", Sz, np.abs(phi))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_scattering_absscale_independent(orc, layout):
    """The error scale that every scattering parity bar divides by, against an
    independent einsum over |S| and |phi| (terms are nonnegative, so two
    summation orders differ by at most 2 gamma_G relative); signed S and phi,
    so a scale that drops an absolute value or counts a factor twice fails."""
    Z, G, NM, nmat = 7, 5, 10, 3
    S, mat, phi = inputs(37, Z, G, NM, nmat)
    got = gen.from_layout(orc.scattering(layout, Z, G, NM, S, mat, gen.to_layout(phi, layout), absolute=True),
                          layout, NM, G, Z)
    ref = absscale_reference(S, mat, phi)
    gam = G * U / (1 - G * U)
    assert np.all(np.abs(got - ref) <= 2 * gam * ref)


def test_scattering_absscale_exact_rational(orc):
    """The scale at a tiny shape equals the exact rational sum of |S||phi| to gamma_G."""
    Z, G, NM, nmat = 3, 3, 5, 2
    S, mat, phi = inputs(38, Z, G, NM, nmat)
    got = gen.from_layout(orc.scattering("ZGD", Z, G, NM, S, mat, gen.to_layout(phi, "ZGD"), absolute=True),
                          "ZGD", NM, G, Z)
    ex = brute(np.abs(S), mat, np.abs(phi))
    gam = G * U / (1 - G * U)
    for idx in itertools.product(range(NM), range(G), range(Z)):
        assert ex[idx] > 0
        assert abs(Fraction(float(got[idx])) - ex[idx]) <= Fraction(gam) * ex[idx]
