"""Each planted mistake in the oracle (compiled with ORACLE_MUTANT=n) must be
caught by at least one pin: a dropped stencil term, a wrong sign in the
boundary lifting, inverted CG beta and alpha, a wrong sign in the residual
update, a replace-instead-of-add outer update, a periodic instead of zero
block boundary, a residual that skips neighbour blocks (no halo), swapped
boundary faces, an overlap region grown into edges and corners, and overlap
corrections added without the owner weights, GMRES least squares without
the earlier Givens rotations, a Gram-Schmidt step that skips the newest
basis vector, an asynchronous model that ignores its delays, an FP32 inner
CG with beta inverted, and a schedule replay that reads the latest
neighbour versions instead of the scheduled ones."""
import os
import tempfile

import pytest

import oracle
import oracle_pins as P

MUTANTS = {
    1: "stencil drops the +z neighbour",
    2: "+z boundary value subtracted",
    3: "CG beta inverted",
    4: "CG residual update sign",
    5: "outer update replaces x",
    6: "block stencil wraps periodically",
    7: "outer residual without neighbour blocks",
    8: "-x and -y faces exchanged",
    10: "CG alpha inverted",
    11: "overlap region includes edges and corners",
    12: "overlap corrections added without weights",
    13: "GMRES without the earlier Givens rotations",
    14: "GMRES Gram-Schmidt skips the newest vector",
    15: "asynchronous model ignores its delay table",
    16: "FP32 inner CG beta inverted",
    17: "schedule replay reads the latest neighbour version, not the scheduled one",
}


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=lambda m: f"m{m}")
def test_mutant_is_caught(mutant):
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(mutant, out=os.path.join(d, f"liboracle_mut{mutant}.so"))
        o = oracle.Oracle(path)
        caught = []
        for pin in P.FAST_PINS:
            try:
                pin(o)
            except Exception:
                caught.append(pin.__name__)
        assert caught, f"mutant {mutant} ({MUTANTS[mutant]}) passed every pin"
