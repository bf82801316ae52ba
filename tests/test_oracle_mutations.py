"""Plants plausible mistakes in copies of the plain oracle's C source and of
its generated formulas (on the CPU only) and checks that the pins of
tests/test_oracle_plain.py reject every one of them: evidence that the pins
are not tautological."""
import os

import pytest

import test_oracle_plain as pins
from oracle.build import SRC, build
from oracle.gen_formulas import HEADER
from oracle.plain import PlainOracle

# (description, text in eig3_plain.c or eig3_plain_formulas.h, replacement)
MUTATIONS = [
    ("I1 wrong index", "return A[0] + A[4] + A[8];", "return A[0] + A[4] + A[7];"),
    ("J2 wrong fraction", "(d0 * d0 + d1 * d1 + d2 * d2) / 6.0", "(d0 * d0 + d1 * d1 + d2 * d2) / 3.0"),
    ("J2 transposed operand", "A01 * A10 + A02 * A20 + A12 * A21", "A01 * A10 + A02 * A20 + A12 * A12"),
    ("J3 wrong sign of diag", "return offdiag + mixed - diag;", "return offdiag + mixed + diag;"),
    ("J3 wrong t2", "double t2 = d0 - d2;", "double t2 = d0 + d2;"),
    ("dx factor sign", "r[4] = M01 * M12 * d1 - M01 * M02 * M10", "r[4] = M01 * M12 * d1 + M01 * M02 * M10"),
    ("dx dropped term", "r[11] = M12 * d0 * d1 - M02 * M10 * d1 + M01 * M10 * M12 - M12 * M12 * M21;",
     "r[11] = M12 * d0 * d1 - M02 * M10 * d1 + M01 * M10 * M12;"),
    ("dx printed r10 sign", "r[7] = M01 * d1 * d2 + M02 * M21 * d2", "r[7] = M01 * d1 * d2 - M02 * M21 * d2"),
    ("dx wrong difference", "r[9] = M02 * d0 * d2 + M01 * M12 * d2", "r[9] = M02 * d0 * d1 + M01 * M12 * d2"),
    ("last weight", "{9, 6, 6, 6, 8, 8, 8, 2, 2, 2, 2, 2, 2, 1}", "{9, 6, 6, 6, 8, 8, 8, 2, 2, 2, 2, 2, 2, 2}"),
    ("v from A instead of A^T", "    dx_factors(At, d0, d1, d2, v);\n    double disc",
     "    dx_factors(A, d0, d1, d2, v);\n    double disc"),
    ("plain arctan branch", "atan2(sqrt(27.0 * fmax(disc, 0.0)), 27.0 * J3)",
     "atan(sqrt(27.0 * fmax(disc, 0.0)) / (27.0 * J3))"),
    ("angle step", "(phi + 2.0 * pi * k) / 3.0", "(phi + pi * k) / 3.0"),
    ("backward not transposed", "grad[3 * r + c] += g[k] * E[3 * c + r];", "grad[3 * r + c] += g[k] * E[3 * r + c];"),
]


def _pins(o):
    """The plain-oracle pins, cheapest first."""
    return [
        lambda: pins.test_integer_matrices_aux_vectors_exact(o),
        lambda: pins.test_scaled_identity_exact_zero(o),
        lambda: pins.test_j3_singular_deviator_example(o),
        lambda: pins.test_paper_performance_example(o),
        lambda: pins.test_backward_identities(o),
        lambda: pins.test_ordering_and_spectral_sums(o),
        lambda: pins.test_within_stability_bounds_well_conditioned(o, "Haar-similar batch"),
        lambda: pins.test_within_stability_bounds_well_conditioned(o, "differentiation batch"),
        lambda: pins.test_perturbation_sweep_buckets(o, 1.0, 8.0),
        lambda: pins.test_backward_against_exact_and_eigenvectors(o),
    ]


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutant_is_rejected(tmp_path, desc, old, new):
    texts = {path: open(path).read() for path in (SRC, HEADER)}
    hits = [path for path, t in texts.items() if t.count(old) == 1]
    assert len(hits) == 1 and sum(t.count(old) for t in texts.values()) == 1, \
        f"mutation anchor not unique: {desc}"
    for path, t in texts.items():
        with open(os.path.join(tmp_path, os.path.basename(path)), "w") as f:
            f.write(t.replace(old, new) if path == hits[0] else t)
    mutant = os.path.join(tmp_path, os.path.basename(SRC))
    lib = build(src=mutant, out=os.path.join(tmp_path, "libmutant.so"))
    o = PlainOracle(lib)
    for pin in _pins(o):
        try:
            pin()
        except (AssertionError, ValueError, FloatingPointError):
            return
    pytest.fail(f"no pin rejects the mutation: {desc}")
