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
13  eq. (cgstop1) compares with the first CG decrease, not the largest earlier one
14  eta_1 and eta_2 swapped (pgstop2 with eta_2, the CG phases with eta_1)
15  eq. (cgstop3) repeats CG on the face without reducing eta_2
16  eta_2 not reset to its initial value after a gradient-projection phase
17  the objective drops the 1/2 of x'Ax

Mutants 13-17 must also be caught by the pin written for them.
"""
import pytest

import oracle
from tests import oracle_pins

MUTANTS = list(range(1, 18))

# the pin that each mistake of the stopping rules and the objective is
# written against
DEDICATED = {
    13: oracle_pins.pin_cg_ratio_stop,
    14: oracle_pins.pin_gp_ratio_stop,
    15: oracle_pins.pin_eta2_schedule,
    16: oracle_pins.pin_eta2_schedule,
    17: oracle_pins.pin_objective,
}


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


@pytest.mark.parametrize("k", sorted(DEDICATED))
def test_mutant_caught_by_its_pin(k, mutant_dir):
    o = oracle.Oracle(oracle.build_mutant(k, mutant_dir))
    with pytest.raises(AssertionError):
        DEDICATED[k](o)
