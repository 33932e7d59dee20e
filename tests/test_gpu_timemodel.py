"""Per-iteration phase times of a profiled factorization (abft_get_iter_profile)
and the time model's predictions against them."""
import numpy as np
import pytest

from paper_2301_03166_amd import gen, timemodel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["chol", "lu", "qr"])
def test_iter_profile_sums_and_predictions(kind):
    import torch
    from paper_2301_03166_amd import abft
    n, nb = 4096, 256
    A = gen.spd(n, 3) if kind == "chol" else gen.general(n, 3)
    with abft.Handle() as h:
        dA = torch.from_numpy(np.asfortranarray(A)).cuda()
        fn = {"chol": h.potrf, "lu": h.getrf, "qr": h.geqrf}[kind]
        fn(dA, nb, profile=True)
        p = h.profile()
        it = h.iter_profile()
    N = timemodel.iterations(n, nb)
    assert all(len(v) == N for v in it.values())
    assert np.isclose(sum(it["pd"]) + sum(it["pu"]), p["ms_panel"], rtol=1e-6)
    assert np.isclose(sum(it["tmu"]), p["ms_tmu"], rtol=1e-6)
    assert np.isclose(sum(it["verify"]), p["ms_verify"], rtol=1e-6)
    assert it["tmu"][N - 1] == 0.0  # the last iteration has no trailing matrix
    if kind != "lu":
        assert sum(it["pu"]) == 0.0
    v = timemodel.validate(it, kind, n, nb)
    print(kind, {op: (round(r["neighbours_p4"], 3), round(r["first_iteration"], 3)) for op, r in v.items()})
    # the efficiency of the update changes as it shrinks (small late updates
    # run far below peak): the neighbours follow it better than the first
    # iteration does, the reason for the paper's enhanced predictor
    assert v["tmu"]["neighbours_p4"] < v["tmu"]["first_iteration"]
    assert v["tmu"]["neighbours_p4"] < 0.5
