"""Continuous-batching server on the GPU: a short Poisson replay finishes every
request, overlaps requests on the device, and each result equals the same
request run alone (bit for bit: both use the same stage kernel)."""
import numpy as np
import pytest

from gpu_util import FIELDS, need_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_served_results_equal_alone_runs(precision):
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
    for d in st.done[:8]:
        r = by_id[d.rid]
        state, t, dt = d.result
        alone = MHDBox(r.edge, r.edge, r.edge, precision=precision)
        alone.set_state(be.initial_state(r))
        alone.step(r.steps)
        a, ta, da, _ = alone.get_state()
        for f in FIELDS:
            assert torch.equal(a[f], state[f]), (d.rid, f)
        assert ta == t and da == dt
