"""Serving form: independent FSI steps of different sizes admitted continuously under an
HBM budget.  Each result must be the same alone and in the mix (bitwise: every kernel
is deterministic and slots share no device state), agree with the FP64 oracle to 1e-8 in
every block (the parity runs solve to rtol 1e-10, mixed precision), and a tight budget
must queue requests rather than fail."""
import numpy as np
import pytest

from oracle import step as ostep
from oracle import system
from paper_2301_10041_amd import fsi, inputs, serve

from gpu_helpers import assert_block_parity, torch_dev

RTOL = 1e-10   # parity runs: the solution error stays below 1e-8 per block

pytestmark = pytest.mark.gpu


def small_trace(count=10, seed=7):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / 100.0, count))
    t -= t[0]
    out = []
    for i in range(count):
        n = int(rng.choice([16, 32]))
        ellipse = bool(rng.random() < 0.5)
        cx, cy = rng.uniform(0.35, 0.65, 2)
        r = float(rng.uniform(0.08, 0.2))
        m = int(rng.integers(3, 9))
        axes = (r, r * float(rng.uniform(0.6, 1.0))) if ellipse else None
        wl = inputs.Workload(f"s{i}", n, [inputs.Solid(m, (float(cx), float(cy)), r, axes)], dt=0.01,
                             seed=2000 + i)
        out.append(serve.Request(i, float(t[i]), wl, u_seed=wl.seed))
    return out


@pytest.fixture(scope="module")
def mixed_run():
    torch_dev()
    reqs = small_trace()
    srv = serve.Server(max_slots=4, keep_states=True, rtol=RTOL)
    res = srv.run(reqs)
    stats = dict(max_inflight=srv.max_inflight, slots=len(srv.slots))
    srv.close()
    return reqs, res, stats


def test_all_served_and_converged(mixed_run):
    reqs, res, stats = mixed_run
    print(f"[serve] {serve.summarize(res)} {stats}", flush=True)
    assert len(res) == len(reqs)
    assert all(r.stats["converged"] for r in res)
    assert all(r.latency > 0 for r in res)
    assert stats["max_inflight"] >= 2          # requests overlapped


def test_alone_equals_mix_bitwise(mixed_run):
    reqs, res, _ = mixed_run
    for q, r in zip(reqs, res):
        alone = serve.Server(max_slots=1, keep_states=True, rtol=RTOL)
        [a] = alone.run([serve.Request(q.rid, 0.0, q.workload, q.u_seed)], realtime=False)
        alone.close()
        assert np.array_equal(a.state, r.state), q.rid


def test_mixed_results_match_oracle(mixed_run):
    reqs, res, _ = mixed_run
    for q, r in list(zip(reqs, res))[:3]:
        S = system.FSISystem.from_workload(q.workload)
        u = inputs.uniform(2 * S.lay.N2, q.u_seed)
        x_ref, _ = ostep.step(S, u, S.xy_ref, solver="direct")
        assert_block_parity(S, r.state, x_ref, 1e-8, f"request {q.rid}")


def _footprint(q):
    xy, tri = q.workload.solid_mesh()
    return fsi.footprint(q.workload.n, xy.shape[0], tri.shape[0])


def test_tight_budget_queues():
    """Room for one context: requests of one size run one at a time on one slot."""
    torch_dev()
    reqs = [q for q in small_trace(12, seed=3) if q.workload.n == 32][:4]
    assert len(reqs) >= 2
    srv = serve.Server(hbm_budget=int(1.2 * max(_footprint(q) for q in reqs)), max_slots=4,
                       keep_states=True)
    res = srv.run(reqs)
    assert all(r.stats["converged"] for r in res)
    assert srv.max_inflight == 1
    ref = serve.Server(max_slots=2, keep_states=True)
    res2 = ref.run(reqs, realtime=False)
    for a, b in zip(res, res2):
        assert np.array_equal(a.state, b.state)
    srv.close()
    ref.close()


def test_tight_budget_evicts_other_sizes():
    torch_dev()
    reqs = small_trace(8, seed=11)
    sizes = {q.workload.n for q in reqs}
    assert sizes == {16, 32}
    big = max(_footprint(q) for q in reqs)
    srv = serve.Server(hbm_budget=int(1.1 * big), max_slots=2, keep_states=True)
    res = srv.run(reqs)
    assert all(r.stats["converged"] for r in res)
    assert srv.evictions >= 1
    assert srv.reserved <= srv.budget
    srv.close()


def test_request_larger_than_budget_is_refused():
    torch_dev()
    reqs = small_trace(2, seed=1)
    srv = serve.Server(hbm_budget=1 << 20, max_slots=2)
    with pytest.raises(fsi.FsiError):
        srv.run(reqs, realtime=False)
    srv.close()
