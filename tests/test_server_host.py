"""Request loop logic on the CPU (dry-run mode: admission, scheduling and
accounting run as on the GPU, device work replaced by a modelled time)."""
import pytest

S = pytest.importorskip("paper_1611_08769_amd.sfft")
from paper_1611_08769_amd import api  # noqa: E402

SHAPES = [(1, 8, 8, 4, False), (1, 16, 12, 6, True), (1, 8, 16, 8, True), (2, 4, 8, 4, False),
          (1, 32, 12, 6, True)]


def _plan_info(sh):
    p = api.size_params(*sh, 1)
    return p, S.sfft_analyze(S.shape(*sh), p)


def _ws_bytes(info, p):
    assert info.ws_bytes >= info.ws_cts * S.sfft_ct_bytes(p)
    return info.ws_bytes


def test_all_requests_complete_and_products_add_up():
    srv = api.Server(1 << 34, dry_run=True)
    total = 0
    tickets = []
    for sh in SHAPES * 3:
        p, info = _plan_info(sh)
        total += info.exec_products
        tickets.append(srv.submit(*sh, p))
    srv.drain()
    st = srv.stats()
    assert st.completed == st.submitted == len(tickets)
    assert st.products == total
    assert st.queued == 0 and st.active == 0
    for t in tickets:
        done, lat = srv.poll(t)
        assert done and lat > 0


def test_max_active_and_fifo():
    srv = api.Server(1 << 34, max_active=2, dry_run=True)
    tickets = [srv.submit(*sh, _plan_info(sh)[0]) for sh in SHAPES]
    seen = 0
    while True:
        pend = srv.step()
        st = srv.stats()
        assert st.active <= 2
        seen = max(seen, st.active)
        if pend == 0:
            break
    assert srv.stats().max_active == 2 == seen
    # single slot: strict arrival order, latencies increase
    srv1 = api.Server(1 << 34, max_active=1, dry_run=True)
    t1 = [srv1.submit(*SHAPES[0], _plan_info(SHAPES[0])[0]) for _ in range(4)]
    srv1.drain()
    lats = [srv1.poll(t)[1] for t in t1]
    assert lats == sorted(lats) and lats[0] < lats[-1]


def test_admission_respects_memory_budget():
    big = (1, 32, 12, 6, True)
    p, info = _plan_info(big)
    ws = _ws_bytes(info, p)
    # room for one such workspace only (plus slack below a second one)
    srv = api.Server(int(ws * 1.5) + 4096, dry_run=True)
    for _ in range(3):
        srv.submit(*big, p)
    while srv.step():
        st = srv.stats()
        assert st.active <= 1
        assert st.peak_ws_bytes <= int(ws * 1.5) + 4096
    assert srv.stats().completed == 3 and srv.stats().max_active == 1


def test_oversized_request_rejected():
    p, info = _plan_info(SHAPES[4])
    srv = api.Server(max(1, _ws_bytes(info, p) // 2), dry_run=True)
    with pytest.raises(S.SfftError) as e:
        srv.submit(*SHAPES[4], p)
    assert e.value.code == S.SFFT_ENOMEM


def test_late_arrivals_join_running_requests():
    """Continuous batching: a request submitted while others run is admitted
    at the next step and overlaps with them."""
    srv = api.Server(1 << 34, dry_run=True)
    long_sh = (1, 32, 12, 6, True)
    t0 = srv.submit(*long_sh, _plan_info(long_sh)[0])
    for _ in range(5):
        srv.step()
    t1 = srv.submit(*SHAPES[0], _plan_info(SHAPES[0])[0])
    srv.step()
    assert srv.stats().active == 2
    srv.drain()
    assert srv.poll(t0)[0] and srv.poll(t1)[0]
    assert srv.poll(t1)[1] < srv.poll(t0)[1]


def test_unknown_ticket():
    srv = api.Server(1 << 20, dry_run=True)
    with pytest.raises(S.SfftError):
        srv.poll(12345)


def test_fill_policy_runs_least_remaining_work_first():
    """With fill_blocks set, a small request submitted behind a large one is
    not held to the large one's pace: it completes first, every request
    still completes and the products add up."""
    big, small = (1, 32, 12, 6, True), (1, 8, 8, 4, False)
    pb, ib = _plan_info(big)
    ps, is_ = _plan_info(small)
    lock = api.Server(1 << 34, dry_run=True)
    fill = api.Server(1 << 34, dry_run=True, fill_blocks=1)
    res = {}
    for name, srv in (("lock", lock), ("fill", fill)):
        tb = srv.submit(*big, pb)
        ts = srv.submit(*small, ps)
        srv.drain()
        st = srv.stats()
        assert st.completed == 2 and st.products == ib.exec_products + is_.exec_products
        res[name] = (srv.poll(tb)[1], srv.poll(ts)[1], st.steps)
    # lockstep: both advance every step; fill (one request per step): the
    # small one runs alone from the start and finishes sooner
    assert res["fill"][1] < res["lock"][1]
    assert res["fill"][1] < res["fill"][0]
    # one request per step here: about as many steps as the two plans have together
    assert res["fill"][2] >= ib.levels + is_.levels


def test_fill_policy_keeps_large_levels_out_of_small_steps():
    """A large request's level (more workgroups than fill_blocks) does not join
    a step that small requests started: small requests run on their own and
    all finish before the large one, which then completes too."""
    big, small = (1, 32, 12, 6, True), (1, 8, 8, 4, False)
    pb, _ = _plan_info(big)
    ps, _ = _plan_info(small)
    srv = api.Server(1 << 34, dry_run=True, fill_blocks=64)
    tb = srv.submit(*big, pb)
    ts = [srv.submit(*small, ps) for _ in range(3)]
    srv.drain()
    lb = srv.poll(tb)[1]
    assert all(srv.poll(t)[0] for t in ts) and srv.poll(tb)[0]
    assert max(srv.poll(t)[1] for t in ts) < lb


def test_fill_policy_admission_skips_a_blocked_head():
    """Under the fill policy a small request queued behind one whose workspace
    does not fit yet is admitted at once; lockstep keeps strict arrival order."""
    big, small = (1, 32, 12, 6, True), (1, 8, 8, 4, False)
    pb, ib = _plan_info(big)
    ps, is_ = _plan_info(small)
    wb, ws = _ws_bytes(ib, pb), _ws_bytes(is_, ps)
    budget = wb + 2 * ws + 4096  # one big at a time, with room left for small ones
    for fill, expect_small_first in ((1, True), (0, False)):
        srv = api.Server(budget, dry_run=True, fill_blocks=fill)
        t1 = srv.submit(*big, pb)
        t2 = srv.submit(*big, pb)   # cannot be admitted while t1 runs
        t3 = srv.submit(*small, ps)
        srv.step()
        st = srv.stats()
        assert st.admitted == (2 if expect_small_first else 1)
        srv.drain()
        assert all(srv.poll(t)[0] for t in (t1, t2, t3))
