"""Continuous-batching server on the GPU: a short Poisson replay finishes every
request, overlaps requests on the device, every result matches the oracle run
on that request's own seeded input (FP64 bit for bit, FP32 within 1e-5
norm-wise) and equals the same request run alone (bit for bit: both use the
same stage kernel)."""
import numpy as np
import pytest

import oracle as O
from gpu_util import FIELDS, bit_equal, max_rel, need_gpu
from paper_2304_13746_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_served_results_match_oracle_and_alone_runs(precision):
    torch = need_gpu()
    from paper_2304_13746_amd.box import MHDBox
    from paper_2304_13746_amd.serve import GpuBackend, Server, poisson_requests
    reqs = poisson_requests(16, rate=400.0, seed=31, edges=(16, 24, 32, 48), steps=(5, 30))
    be = GpuBackend(precision=precision)
    st = Server(be, budget_bytes=2 << 30, epoch_steps=4).run(reqs, keep_results=True)
    assert len(st.done) == 16 and not st.rejected
    assert all(d.status == 0 for d in st.done)
    s = st.summary()
    assert s["p99_ms"] >= s["p50_ms"] > 0
    by_id = {r.rid: r for r in reqs}
    worst = 0.0
    for d in st.done:
        r = by_id[d.rid]
        state, t, dt = d.result
        print(f"request {r.rid}: edge {r.edge} init {r.init} steps {r.steps} seed {r.seed}",
              flush=True)
        # the oracle on the request's own input (rounded to FP32 for an FP32 run)
        x = I.serving_state(r.edge, r.init, r.seed)
        if precision == "fp32":
            x = I.to_float32_exact(x)
        o = O.copy_state(x)
        to, _, _ = O.step(O.Params(r.edge, r.edge, r.edge), o, 0.0, 0.0, r.steps)
        g = {f: state[f].double().cpu().numpy() for f in FIELDS}
        if precision == "fp64":
            assert bit_equal(g, o) and t == to, r.rid
        else:
            err = max_rel(g, o)
            worst = max(worst, err)
            assert err <= 1e-5, (r.rid, err)
            assert abs(t - to) <= 1e-5 * to
        # the same request alone on a fresh context
        alone = MHDBox(r.edge, r.edge, r.edge, precision=precision)
        alone.set_state(be.initial_state(r))
        alone.step(r.steps)
        a, ta, da, _ = alone.get_state()
        alone.close()
        for f in FIELDS:
            assert torch.equal(a[f], state[f]), (d.rid, f)
        assert ta == t and da == dt
    print(f"served {precision}: worst max rel vs oracle {worst:.3e}")
    # requests of one edge and init differ (their seeds translate the data)
    shifts = {I.request_shift(r.seed, r.edge) for r in reqs}
    assert len(shifts) == len(reqs)
