"""Host logic of the request loop (no GPU): admission counts slots that are admitted but not
yet built, so a grid never gets more slots than slots_per_grid allows even while a worker
builds a new slot outside the lock."""
from paper_2301_10041_amd import inputs, serve


def _req(rid, n):
    wl = inputs.Workload(f"r{rid}", n, [inputs.Solid(4, (0.5, 0.5), 0.15)], dt=0.01, seed=rid)
    return serve.Request(rid, 0.0, wl, wl.seed)


def test_pending_new_slots_count_against_slots_per_grid():
    srv = serve.Server(hbm_budget=1 << 40, max_slots=4, slots_per_grid=1)
    a, b, c = _req(0, 32), _req(1, 32), _req(2, 64)
    with srv.cv:
        got, new = srv._try_admit(a)
        assert new and got > 0
        # a second request of the same grid while the first slot is still being built
        assert srv._try_admit(b) == (None, False)
        # another grid is admitted
        got_c, new_c = srv._try_admit(c)
        assert new_c
    assert srv._pending == {serve.grid_key(a.workload): 1, serve.grid_key(c.workload): 1}
    assert srv.reserved == got + got_c
