"""Scheduler logic of the continuous-batching server, driven by a virtual-time
mock backend (no GPU)."""
import numpy as np
import pytest

from paper_2304_13746_amd.serve import MockBackend, Request, Server, poisson_requests


def test_poisson_generator_statistics():
    reqs = poisson_requests(4000, rate=200.0, seed=1)
    gaps = [b.arrival - a.arrival for a, b in zip(reqs, reqs[1:])]
    assert abs(sum(gaps) / len(gaps) - 1 / 200.0) < 0.1 / 200.0
    assert {r.edge for r in reqs} == {32, 48, 64, 96, 128, 192}
    assert min(r.steps for r in reqs) >= 10 and max(r.steps for r in reqs) <= 200
    assert 0.45 < sum(r.init == "ot" for r in reqs) / len(reqs) < 0.55


def test_every_request_completes_with_its_steps():
    reqs = poisson_requests(200, rate=500.0, seed=3)
    b = MockBackend(rate=5e9)
    st = Server(b, budget_bytes=64 * 192 ** 3 * 128, epoch_steps=7).run(reqs, keep_results=True)
    assert len(st.done) == 200 and not st.rejected
    for d in st.done:
        assert d.result == d.steps  # the mock counts the steps it was given
        assert d.finished >= d.admitted >= d.arrival - 1e-12


def test_budget_is_never_exceeded_and_admission_waits():
    """With room for only two 64^3 boxes at once, at most two are active."""
    reqs = [Request(i, 0.001 * i, 64, 50, "ot", i) for i in range(10)]
    b = MockBackend(rate=1e9)
    budget = 2 * 64 ** 3 * 128
    st = Server(b, budget_bytes=budget, epoch_steps=10).run(reqs)
    assert st.peak_bytes <= budget
    for boxes, _ in b.epochs:
        assert len(boxes) <= 2
    assert len(st.done) == 10


def test_skip_ahead_lets_small_boxes_pass_a_blocked_large_one():
    """A large request that does not fit yet must not block small ones behind it
    (within the skip-ahead window); strict FIFO would."""
    reqs = [Request(0, 0.0, 128, 100, "ot", 0), Request(1, 0.0001, 128, 100, "ot", 1)]
    reqs += [Request(2 + i, 0.0002 + 1e-5 * i, 32, 10, "ot", 2 + i) for i in range(4)]
    budget = 128 ** 3 * 128 + 4 * 32 ** 3 * 128
    b = MockBackend(rate=1e9)
    st = Server(b, budget_bytes=budget, skip_ahead=8).run(reqs)
    adm = {d.rid: d.admitted for d in st.done}
    fin = {d.rid: d.finished for d in st.done}
    assert all(adm[2 + i] < adm[1] for i in range(4))
    assert all(fin[2 + i] < fin[0] for i in range(4))
    b2 = MockBackend(rate=1e9)
    st2 = Server(b2, budget_bytes=budget, skip_ahead=1).run(reqs)
    adm2 = {d.rid: d.admitted for d in st2.done}
    assert all(adm2[2 + i] >= adm2[1] for i in range(4))


def test_oversized_request_is_rejected_not_deadlocked():
    reqs = [Request(0, 0.0, 192, 10, "ot", 0), Request(1, 0.0, 32, 10, "ot", 1)]
    st = Server(MockBackend(), budget_bytes=64 ** 3 * 128).run(reqs)
    assert [r.rid for r in st.rejected] == [0]
    assert [d.rid for d in st.done] == [1]


def test_failed_request_does_not_poison_others():
    reqs = poisson_requests(30, rate=1000.0, seed=9, edges=(32, 48))
    st = Server(MockBackend(fail_rids={5, 7}), budget_bytes=1 << 34).run(reqs)
    assert len(st.done) == 30
    bad = {d.rid for d in st.done if d.status != 0}
    assert bad == {5, 7}
    s = st.summary()
    assert s["failed"] == 2 and s["requests"] == 30


def test_overlap_new_requests_join_running_epochs():
    """A request arriving while a long one runs is admitted and advanced in the
    same epochs (continuous batching, not a queue)."""
    reqs = [Request(0, 0.0, 96, 200, "ot", 0), Request(1, 0.01, 32, 20, "ot", 1)]
    b = MockBackend(rate=2e8)
    st = Server(b, budget_bytes=1 << 34, epoch_steps=10).run(reqs)
    shared = [boxes for boxes, _ in b.epochs if set(boxes) == {0, 1}]
    assert shared, b.epochs
    fin = {d.rid: d.finished for d in st.done}
    assert fin[1] < fin[0]


def test_latency_accounting():
    reqs = [Request(0, 0.5, 32, 10, "ot", 0)]
    b = MockBackend(rate=32 ** 3 * 10 / 0.25)  # the whole job takes 0.25 s
    st = Server(b, budget_bytes=1 << 30, epoch_steps=10).run(reqs)
    d = st.done[0]
    assert d.arrival == 0.5
    assert d.latency == pytest.approx(0.25, rel=0.05)


def test_request_inputs_are_seeded_translations():
    """A served request's initial data is its base field translated by the shift
    of the variant its seed draws: div B stays zero, seeds spread over the
    variants and the variants' shifts differ,
    and (the scheme is translation-invariant on a periodic grid) the oracle's
    cycles on the translated input equal the translated cycles of the base, bit
    for bit, so any request can be checked against the oracle on its own input."""
    import oracle as O
    from paper_2304_13746_amd import inputs as I
    n = 16
    base = I.serving_base(n, "turb")
    assert len({I.request_variant(seed) for seed in range(2304, 2344)}) >= 12
    assert len({I.variant_shift(k, n) for k in range(I.SERVING_VARIANTS)}) >= 12
    s = I.serving_state(n, "turb", 2307)
    sx, sy, sz = I.request_shift(2307, n)
    assert (sx, sy, sz) != (0, 0, 0)
    p = O.Params(n, n, n)
    assert O.diagnostics(p, O.copy_state(s))["divb_max"] <= 1e-13
    a, b = O.copy_state(s), O.copy_state(base)
    ta, _, _ = O.step(p, a, 0.0, 0.0, 3)
    tb, _, _ = O.step(p, b, 0.0, 0.0, 3)
    assert ta == tb
    for f in O.FIELDS:
        assert np.array_equal(a[f], np.roll(b[f], (sz, sy, sx), axis=(0, 1, 2))), f
    assert not np.array_equal(s["mx"], base["mx"])
