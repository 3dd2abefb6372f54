"""The pins have teeth: every planted mistake in the oracle fails one of them.

Each mutant is a build of ``oracle/gpcg_ref.c`` with ``-DORA_MUTANT=k``, which
swaps in one plausible mistake (CPU only; nothing here touches a GPU):

 1  projected gradient at the upper bound uses min instead of max
 2  the decrease model drops the 1/2 of s'As
 3  the CG free set is the complement of the binding set, not the active set
 4  alpha_0 inverted (d'Ad / d'd)
 5  CG beta inverted (rho_old'rho_old / rho_new'rho_new)
 6  CG starts from rho = +g instead of -g
 7  gradient sign flipped (b - Ax)
 8  projection returns l for values above u
 9  binding test with the inequalities reversed
10  CG decrease without the 1/2
11  preconditioned CG updates the direction with rho instead of z = M^{-1} rho
12  the residual CG test compares squared norms against eta
"""
import pytest

import oracle
from tests import oracle_pins

MUTANTS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12]


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("mutants"))


@pytest.mark.parametrize("k", MUTANTS)
def test_mutant_is_caught(k, mutant_dir):
    path = oracle.build_mutant(k, mutant_dir)
    o = oracle.Oracle(path)
    caught = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(o)
        except Exception as e:  # AssertionError, or a crash of the bad oracle
            caught.append((pin.__name__, type(e).__name__))
            break
    assert caught, f"mutant {k} passed every pin"
