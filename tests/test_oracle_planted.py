"""Planted mistakes in a copy of the oracle (CPU only).

Each case below edits one expression of a copy of ``oracle/oracle.c`` (the
kind of slip a reader could miss: a doubled factor, a missing absolute value,
an unrounded split, a transposed or swapped index, a dropped term), compiles
the copy into a temporary library, and runs the named pins on it: at least
one of them must fail.  This shows the pins constrain the oracle's arithmetic,
including the error scales that every GPU parity bar divides by.  The real
oracle is untouched; the copy lives in pytest's temporary directory.
"""
import importlib.util
import os

import pytest

import test_oracle_mass_pins as mass_pins
import test_oracle_pins as pins
import test_oracle_scattering_pins as scat_pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")

# name -> (expression in oracle.c, replacement, pins that must catch it)
CASES = {
    "scattering scale doubled": (
        "double prod = absolute ? fabs(Sm[g * G + gp]) * fabs(x) : Sm[g * G + gp] * x;",
        "double prod = absolute ? 2.0 * fabs(Sm[g * G + gp]) * fabs(x) : Sm[g * G + gp] * x;",
        [lambda o: scat_pins.test_scattering_absscale_independent(o, "DGZ"),
         lambda o: scat_pins.test_scattering_absscale_exact_rational(o)]),
    "scattering scale without |phi|": (
        "double prod = absolute ? fabs(Sm[g * G + gp]) * fabs(x) : Sm[g * G + gp] * x;",
        "double prod = absolute ? fabs(Sm[g * G + gp]) * x : Sm[g * G + gp] * x;",
        [lambda o: scat_pins.test_scattering_absscale_independent(o, "ZDG")]),
    "scattering degree off by one": (
        "const double *Sm = S + ((int64_t)mat[z] * nl + orc_degree(nm)) * G * G;",
        "const double *Sm = S + ((int64_t)mat[z] * nl + orc_degree(nm + 1 < NM ? nm + 1 : nm)) * G * G;",
        [lambda o: scat_pins.test_scattering_degree_and_material_closed_form(o)]),
    "mass scale doubled": (
        "u[q] = acc * (absolute ? fabs(dq[q]) : dq[q]);",
        "u[q] = acc * (absolute ? 2.0 * fabs(dq[q]) : dq[q]);",
        [lambda o: mass_pins.test_mass_absscale_kronecker(o, 2, 4, 6)]),
    "mass scale without |x|": (
        "(absolute ? fabs(x[j]) : x[j])",
        "(absolute ? x[j] : x[j])",
        [lambda o: mass_pins.test_mass_absscale_kronecker(o, 3, 3, 5)]),
    "mass basis transposed": (
        "double v = B1[(q % Q1D) * D1D + (i % D1D)];",
        "double v = B1[(i % D1D) * Q1D + (q % Q1D)];",
        [lambda o: mass_pins.test_mass_matches_kronecker_form(o, 2, 4, 6)]),
    "bf16 lo not rounded": (
        "double ph = orc_bf16_round(p), pl = orc_bf16_round(p - ph);",
        "double ph = orc_bf16_round(p), pl = p - ph;",
        [lambda o: pins.test_bf16_emulation_exact_split(o, "DGZ")]),
    "bf16 cross term dropped": (
        "if (mode == 1) term = term + lh * pl + ll * ph;",
        "if (mode == 1) term = term + lh * pl;",
        [lambda o: pins.test_bf16_emulation_exact_split(o, "GZD")]),
    "ltimes L transposed": (
        "double prod = L[nm * D + d] * psi[",
        "double prod = L[d * NM + nm] * psi[",
        [lambda o: pins.test_ltimes_exact_rational(o, "DGZ", (3, 2, 5, 4))]),
    "ltimes layout index swapped": (
        "case ORC_GDZ: return (g * A + a) * Z + z;",
        "case ORC_GDZ: return (a * G + g) * Z + z;",
        [lambda o: pins.test_ltimes_exact_rational(o, "GDZ", (3, 2, 5, 4))]),
    "ltimes scale sign kept": (
        "acc = acc + fabs(L[nm * D + d]) * fabs(psi[",
        "acc = acc + (L[nm * D + d]) * fabs(psi[",
        [lambda o: pins.test_absscale_is_sum_of_abs(o)]),
}


def load_mutant(tmp_path, name, old, new):
    with open(os.path.join(ORACLE_DIR, "oracle.c")) as f:
        src = f.read()
    assert src.count(old) == 1, f"{name}: the expression to mutate must occur exactly once"
    d = tmp_path / "mutant"
    d.mkdir()
    (d / "oracle.c").write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle_mutant_" + str(abs(hash(name))),
                                                  os.path.join(ORACLE_DIR, "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._SRC = str(d / "oracle.c")
    mod._LIB = str(d / "liboracle.so")
    mod._lib = None
    mod.build(force=True)
    mod.lib()
    return mod


@pytest.mark.parametrize("name", sorted(CASES))
def test_planted_mistake_fails_a_pin(tmp_path, name):
    old, new, checks = CASES[name]
    mut = load_mutant(tmp_path, name, old, new)
    for check in checks:
        with pytest.raises(AssertionError):
            check(mut)


def test_unmutated_copy_passes(tmp_path, orc):
    """The same loader with no edit: every pin used above passes (so the
    failures above come from the edits)."""
    mut = load_mutant(tmp_path, "none", "int orc_set_threads(int n)", "int orc_set_threads(int n)")
    for _, _, checks in CASES.values():
        for check in checks:
            check(mut)
