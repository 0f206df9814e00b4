"""GPU check of the kernel-timing groups: with the mask set to the pair-rate group only, a step
records events around the rate kernel alone, and the other groups again once the mask is
cleared; the step's results do not depend on the mask."""
import pytest
import torch

import csph_inputs as ci
import paper_1805_05128_amd as P

pytestmark = pytest.mark.gpu

DEV = "cuda"


def test_profile_groups_select_the_timed_kernels():
    w = ci.config0()
    print(f"[case] profile groups n={w.n}", flush=True)
    params = P.Params.from_workload(w, reorder=False)
    out = {}
    try:
        P.profile_enable(True)
        for groups in (["rates"], None):
            s = P.state_from_workload(w, params, DEV)
            P.profile_groups(groups)
            P.profile_read()
            P.csph_step(s, params, P.StepScalars(DEV), s_out=s)
            torch.cuda.synchronize()
            prof = P.profile_read()
            out[groups is None] = {k: s[k].clone() for k in ("x", "vx", "rho", "E")}
            timed = {g for g, (launches, ms) in prof.items() if launches > 0}
            if groups is None:
                assert {"bin", "pack", "rates", "integrate"} <= timed, timed
            else:
                assert timed == {"rates"}, timed
                assert prof["rates"][0] == 1 and prof["rates"][1] > 0.0
    finally:
        P.profile_groups(None)
        P.profile_enable(False)
    for k in out[True]:
        assert torch.equal(out[True][k], out[False][k]), k
