"""The CPU oracle against facts fixed by the paper and by mathematics."""
import pytest

from oracle.oracle import OracleLib
from tests import pins


@pytest.fixture(scope="module")
def O():
    return OracleLib()


@pytest.mark.parametrize("pin", pins.PINS, ids=lambda f: f.__name__)
def test_pin(O, pin):
    pin(O)


def test_caller_trial_list_is_plumbing_only():
    """The oracle's caller-list mode with the generated list (shared, or the
    same list repeated per shot) gives exactly the generated mode's results."""
    import numpy as np
    from oracle import oracle as O
    from workloads import codes as _codes, shots as _shots
    h = _codes.get_code("bb72").hx
    _, syn = _shots.make_shots(h, 0.07, 300, _shots.stream_key(_shots.MASTER_SEED, 970))
    for prm in (O.Params(k=4), O.Params(k=5, cand_mode=1, w_max=2, select_mode=1)):
        ref = O.bpsf_batch(h, syn, 0.07, prm, threads=4)
        tab = O.trial_masks(prm)
        for masks in (tab, np.tile(tab, (len(syn), 1))):
            got = O.bpsf_batch(h, syn, 0.07, prm, threads=4, masks=masks)
            for f in ("correction", "converged", "iterations", "winner", "main_iterations", "trial_iterations"):
                assert np.array_equal(got[f], ref[f]), f

