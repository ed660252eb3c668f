"""Plant a mistake in the oracle (on the CPU) and check that the pins catch it.

Each mutation is a plausible slip in one formula: a dropped term of the E
recursion, a sign or operand swap, a sign in the R recursion, a wrong Boys
asymptote, a missing angular factor of the normalisation."""
import numpy as np
import pytest

from oracle import oracle as O

from gauss_ref import Basis
from test_oracle_potential import SHELLS2, XYZ2, flat, rand_sym

MUTATIONS = {1: "E recursion without (t+1) E_{t+1}",
             2: "E recursion with -X_PA",
             3: "E recursion with X_PB for the i index",
             4: "R recursion with the wrong sign at order 1",
             5: "Boys F_0 without erf above T = 30",
             6: "normalisation without (4a)^{l/2}/sqrt(dfact)"}

PTS = [np.array([0.5, 0.4, 0.2]), np.array([12.0, 3.0, -4.0])]


def _pins_pass():
    B = Basis(XYZ2, SHELLS2)
    P = rand_sym(B.nbf, 3)
    for pt in PTS:
        M = B.coulomb(pt)
        ref = float(np.sum(P * M))
        absref = float(np.sum(np.abs(P * M)))
        _, _, Ve, _ = O.potential_raw(XYZ2, np.zeros(2), flat(SHELLS2), P, pt[None])
        if abs(Ve[0] - ref) > 1e-12 * absref:
            return False
    return True


def test_unmutated_passes():
    O.set_mutation(0)
    assert _pins_pass()


@pytest.mark.parametrize("m", sorted(MUTATIONS))
def test_mutation_is_caught(m):
    O.set_mutation(m)
    try:
        assert not _pins_pass(), MUTATIONS[m]
    finally:
        O.set_mutation(0)
