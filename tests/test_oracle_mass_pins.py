"""Pins of the oracle's tensor-product mass operator (CPU only):
    y_e = B^T diag(D_e) B x_e,  B(q, i) = prod_k B1[q_k][i_k]  (first index component fastest).
The operator is a reading (the paper specializes Laghos' partial-assembly
kernels on the numbers of dofs and quadrature points but does not define
them); these checks pin the oracle to that definition by means other than
its own code: exact rational arithmetic, integer inputs, the Kronecker form
built with numpy, an identity basis, and the symmetry of a mass matrix."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

U = 2.0 ** -53


def exact(dim, D1D, Q1D, B1, Dq, X):
    nd, nq = D1D ** dim, Q1D ** dim
    NE = X.size // nd

    def comp(f, base):
        out = []
        for _ in range(dim):
            out.append(f % base)
            f //= base
        return out
    Bf = [[Fraction(1)] * nd for _ in range(nq)]
    for q, i in itertools.product(range(nq), range(nd)):
        qc, ic = comp(q, Q1D), comp(i, D1D)
        b = Fraction(1)
        for k in range(dim):
            b *= Fraction(float(B1[qc[k], ic[k]]))
        Bf[q][i] = b
    Y = []
    for e in range(NE):
        x = [Fraction(float(v)) for v in X[e * nd:(e + 1) * nd]]
        u = [sum((Bf[q][j] * x[j] for j in range(nd)), Fraction(0)) * Fraction(float(Dq[e * nq + q])) for q in range(nq)]
        Y += [sum((Bf[q][i] * u[q] for q in range(nq)), Fraction(0)) for i in range(nd)]
    return Y


def kron_matrix(dim, B1):
    Bf = B1
    for _ in range(dim - 1):
        Bf = np.kron(B1, Bf)     # flat q = q0 + Q q1 + ..., i likewise: the last component is the outer factor
    return Bf


@pytest.mark.parametrize("dim,D1D,Q1D", [(1, 3, 4), (2, 2, 3), (2, 3, 2), (3, 2, 3), (3, 3, 3)])
def test_mass_exact_rational(orc, dim, D1D, Q1D):
    rng = np.random.default_rng(51)
    NE = 3
    B1 = rng.uniform(-1, 1, (Q1D, D1D))
    Dq = rng.uniform(0.1, 2.0, NE * Q1D ** dim)
    X = rng.uniform(-1, 1, NE * D1D ** dim)
    got = orc.mass(dim, D1D, Q1D, B1, Dq, X)
    scale = orc.mass(dim, D1D, Q1D, B1, Dq, X, absolute=True)
    ex = exact(dim, D1D, Q1D, B1, Dq, X)
    n = D1D ** dim + Q1D ** dim + 2 * dim + 2
    gam = n * U / (1 - n * U)
    for g, e, s in zip(got, ex, scale):
        assert abs(Fraction(float(g)) - e) <= Fraction(gam * s) + Fraction(1, 2 ** 1074)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_mass_integer_bitexact(orc, dim):
    rng = np.random.default_rng(52)
    D1D, Q1D, NE = 3, 4, 5
    B1 = rng.integers(-3, 4, (Q1D, D1D)).astype(np.float64)
    Dq = rng.integers(1, 5, NE * Q1D ** dim).astype(np.float64)
    X = rng.integers(-4, 5, NE * D1D ** dim).astype(np.float64)
    got = orc.mass(dim, D1D, Q1D, B1, Dq, X)
    assert all(g == float(e) for g, e in zip(got, exact(dim, D1D, Q1D, B1, Dq, X)))


@pytest.mark.parametrize("dim,D1D,Q1D", [(2, 4, 6), (3, 3, 5), (2, 5, 3)])
def test_mass_matches_kronecker_form(orc, dim, D1D, Q1D):
    """The Kronecker-product matrix built by numpy: y = Bf^T diag(D) Bf x."""
    rng = np.random.default_rng(53)
    NE = 4
    B1 = rng.uniform(-1, 1, (Q1D, D1D))
    Dq = rng.uniform(0.5, 1.5, (NE, Q1D ** dim))
    X = rng.uniform(-1, 1, (NE, D1D ** dim))
    Bf = kron_matrix(dim, B1)
    ref = np.stack([Bf.T @ (Dq[e] * (Bf @ X[e])) for e in range(NE)])
    got = orc.mass(dim, D1D, Q1D, B1, Dq, X).reshape(NE, -1)
    scale = orc.mass(dim, D1D, Q1D, B1, Dq, X, absolute=True).reshape(NE, -1)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale)


def test_mass_identity_basis(orc):
    """B1 = I (Q1D = D1D): y = D * x exactly."""
    dim, D1D, NE = 3, 4, 6
    rng = np.random.default_rng(54)
    Dq = rng.uniform(-2, 2, NE * D1D ** dim)
    X = rng.uniform(-2, 2, NE * D1D ** dim)
    assert np.array_equal(orc.mass(dim, D1D, D1D, np.eye(D1D), Dq, X), Dq * X)


def test_mass_symmetric(orc):
    """A mass matrix is symmetric: <M x1, x2> = <x1, M x2> to rounding."""
    dim, D1D, Q1D, NE = 2, 4, 5, 3
    rng = np.random.default_rng(55)
    B1 = rng.uniform(-1, 1, (Q1D, D1D))
    Dq = rng.uniform(0.1, 1, NE * Q1D ** dim)
    x1 = rng.uniform(-1, 1, NE * D1D ** dim)
    x2 = rng.uniform(-1, 1, NE * D1D ** dim)
    a = float(np.dot(orc.mass(dim, D1D, Q1D, B1, Dq, x1), x2))
    b = float(np.dot(x1, orc.mass(dim, D1D, Q1D, B1, Dq, x2)))
    assert abs(a - b) <= 1e-13 * (abs(a) + abs(b) + 1.0)


@pytest.mark.parametrize("dim,D1D,Q1D", [(1, 5, 7), (2, 4, 6), (3, 3, 5)])
def test_mass_absscale_kronecker(orc, dim, D1D, Q1D):
    """The error scale every mass parity bar divides by,
    |B|^T diag(|D_e|) |B| |x_e| with |B| = |kron(B1, ..)|, built with numpy; B1, D
    and x all signed, so a scale that drops an absolute value or doubles a factor
    fails.  All terms are nonnegative: the two orders agree to 2 gamma_n relative."""
    rng = np.random.default_rng(56)
    NE = 5
    B1 = rng.uniform(-1, 1, (Q1D, D1D))
    Dq = rng.uniform(-1, 1, (NE, Q1D ** dim))
    X = rng.uniform(-1, 1, (NE, D1D ** dim))
    Ba = np.abs(kron_matrix(dim, B1))
    ref = np.stack([Ba.T @ (np.abs(Dq[e]) * (Ba @ np.abs(X[e]))) for e in range(NE)])
    got = orc.mass(dim, D1D, Q1D, B1, Dq, X, absolute=True).reshape(NE, -1)
    n = D1D ** dim + Q1D ** dim + 2 * dim + 2
    assert np.all(ref > 0)
    assert np.all(np.abs(got - ref) <= 2 * n * U / (1 - n * U) * ref)


def test_mass_large_element_supported(orc):
    """Elements with more than 4096 points (dim 3, Q1D = 17) are computed, not
    skipped: with B1 = I the operator is y = D * x exactly."""
    dim, D1D, NE = 3, 17, 2
    rng = np.random.default_rng(57)
    Dq = rng.uniform(-2, 2, NE * D1D ** dim)
    X = rng.uniform(-2, 2, NE * D1D ** dim)
    assert np.array_equal(orc.mass(dim, D1D, D1D, np.eye(D1D), Dq, X), Dq * X)
