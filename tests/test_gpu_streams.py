"""A step enqueued on a side stream (its mesh bounds polled through the pinned slot while
that stream, not the default one, runs the kernels) equals the same step on the default
stream bit for bit; so does a CFL step VJP, whose minimum comes back the same way."""
import pytest
import torch

import csph_inputs as ci
import paper_1805_05128_amd as P

pytestmark = pytest.mark.gpu

DEV = "cuda"
F8 = ("x", "y", "z", "vx", "vy", "vz", "rho", "E")


def test_step_and_cfl_vjp_on_a_side_stream():
    w = ci.config0()
    print(f"[case] side stream n={w.n}", flush=True)
    params = P.Params.from_workload(w, reorder=False)
    out = {}
    side = torch.cuda.Stream()
    for name in ("default", "side"):
        s = P.state_from_workload(w, params, DEV)
        sc = P.StepScalars(DEV, t0=0.5)
        gn = {k: torch.linspace(-1.0, 1.0, w.n, dtype=torch.float64, device=DEV) * (i + 1)
              for i, k in enumerate(F8)}
        torch.cuda.synchronize()
        if name == "side":
            with torch.cuda.stream(side):
                P.csph_step(s, params, sc, s_out=s, stream=side)
                gp, ge, dt = P.csph_step_vjp_cfl(s, params, gn, stream=side, t=0.5)
            side.synchronize()
        else:
            P.csph_step(s, params, sc, s_out=s)
            gp, ge, dt = P.csph_step_vjp_cfl(s, params, gn, t=0.5)
        torch.cuda.synchronize()
        out[name] = ({k: s[k].clone() for k in F8}, sc.t.clone(), {k: gp[k].clone() for k in F8},
                     ge.clone(), dt)
    a, b = out["default"], out["side"]
    for k in F8:
        assert torch.equal(a[0][k], b[0][k]), k
        assert torch.equal(a[2][k], b[2][k]), k
    assert torch.equal(a[1], b[1]) and torch.equal(a[3], b[3]) and a[4] == b[4]
