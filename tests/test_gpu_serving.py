"""GPU tests of the serving loop (sim_server_* / sim_submit / sim_poll /
sim_wait): every request's result in a mix of concurrently batched
requests is the result of the same request checked alone, bit for bit, and
the oracle's; admission stays within the HBM budget; errors stay with their
request."""
import threading

import numpy as np
import pytest

import oracle
import tracegen
from tracegen import RECORD_DTYPE

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)


@pytest.fixture(scope="module")
def pkg():
    import paper_1905_01833_amd as p

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return p


def request_pool(n_req, seed, log2_max=18):
    """Requests of one to three traces each, sizes log-uniform 2^6..2^log2_max."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n_req):
        k = int(rng.integers(1, 4))
        shapes = []
        for j in range(k):
            n = int(2 ** rng.uniform(6, log2_max))
            nb = max(1, min(256, -(-n // (256 * 64))))
            shapes.append((n, nb, -(-n // (nb * 256)), int(rng.integers(1, 1 << 62))))
        recs, off, tpb, _ = tracegen.batch(shapes, inject_rate=1e-3)
        pool.append((recs, off, tpb))
    return pool


def test_alone_equals_in_mix(pkg):
    pool = request_pool(48, seed=11)
    # an empty request, a request with an empty trace, and one bad request
    pool.append((np.zeros(0, dtype=RECORD_DTYPE), np.array([0], dtype=np.uint64), np.zeros(0, dtype=np.uint32)))
    r0 = pool[0]
    pool.append((r0[0], np.concatenate([[0], r0[1]]).astype(np.uint64), np.concatenate([[7], r0[2]]).astype(np.uint32)))
    bad = pool[1][0].copy()
    bad["action"][len(bad) // 2] = 5
    pool.append((bad, pool[1][1], pool[1][2]))
    bad_index = len(pool) - 1

    say("alone: plain context, one call per request")
    ctx = pkg.Context(0)
    alone = []
    for i, (recs, off, tpb) in enumerate(pool):
        try:
            alone.append(ctx.check_traces(recs, off, tpb))
        except pkg.SimError as e:
            assert i == bad_index
            alone.append(e.code)
    ctx.close()
    for i in range(0, len(pool) - 1, 9):  # the oracle on a sample
        recs, off, tpb = pool[i]
        want, wsum = oracle.closed_form(recs, off, tpb)
        assert alone[i][0].tobytes() == want.tobytes() and alone[i][1].tobytes() == wsum.tobytes(), i

    biggest = max(16 * len(r) for r, _, _ in pool)
    budget = 3 * 2 * 36 * biggest  # about three of the largest requests at once
    say(f"mix: 3 slots, budget {budget >> 20} MiB, two submitting threads")
    srv = pkg.Server(0, hbm_budget_bytes=budget, slots=3, max_batch_requests=16)
    tickets = [None] * len(pool)

    def submit(ids):
        for i in ids:
            recs, off, tpb = pool[i]
            tickets[i] = srv.submit(recs, off, tpb)

    ths = [threading.Thread(target=submit, args=(range(k, len(pool), 2),)) for k in range(2)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    for rep in range(2):  # every request twice: the second round while the first drains
        for i, (recs, off, tpb) in enumerate(pool):
            if rep == 1:
                tickets.append(srv.submit(recs, off, tpb))
    results = {}
    for j, t in enumerate(tickets):
        i = j % len(pool)
        try:
            results[j] = srv.wait(t)
        except pkg.SimError as e:
            results[j] = e.code
    st = srv.stats()
    srv.close()
    for j, got in results.items():
        i = j % len(pool)
        if i == bad_index:
            assert got == pkg.SIM_ERECORD == alone[i]
            continue
        assert got[0].tobytes() == alone[i][0].tobytes(), (j, i)
        assert got[1].tobytes() == alone[i][1].tobytes(), (j, i)
    assert st["completed"] == len(tickets) - 2 and st["failed"] == 2
    assert st["batches"] < st["completed"]  # requests shared launches
    assert st["peak_inflight_bytes"] <= budget
    assert st["device_bytes"] <= budget
    assert 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]


def test_device_requests_alone_equals_in_mix(pkg):
    """Requests whose records live in device memory (read in place by the
    workers), mixed with host requests: every result is the request's alone
    result, and the oracle's on a sample."""
    pool = request_pool(40, seed=21)
    say("device requests: alone")
    ctx = pkg.Context(0)
    devs = [torch.from_numpy(r.view(np.uint8).reshape(-1, 16)).to("cuda:0") for r, _, _ in pool]
    torch.cuda.synchronize()
    alone = [ctx.check_traces_device(d, off, tpb) for d, (_, off, tpb) in zip(devs, pool)]
    ctx.close()
    for i in range(0, len(pool), 7):
        recs, off, tpb = pool[i]
        want, wsum = oracle.closed_form(recs, off, tpb)
        assert alone[i][0].tobytes() == want.tobytes() and alone[i][1].tobytes() == wsum.tobytes(), i
    budget = 256 << 20
    say("device requests: mix of device and host submissions, 3 slots")
    srv = pkg.Server(0, hbm_budget_bytes=budget, slots=3, max_batch_requests=32)
    try:
        tickets = []
        for rep in range(3):
            for i, (recs, off, tpb) in enumerate(pool):
                if (i + rep) % 3:
                    tickets.append((i, srv.submit_device(devs[i], off, tpb)))
                else:
                    tickets.append((i, srv.submit(recs, off, tpb)))
        for i, t in tickets:
            got = srv.wait(t)
            assert got[0].tobytes() == alone[i][0].tobytes(), i
            assert got[1].tobytes() == alone[i][1].tobytes(), i
        st = srv.stats()
        assert st["completed"] == len(tickets) and st["failed"] == 0
        assert st["batches"] < st["completed"]
        assert st["peak_inflight_bytes"] <= budget and st["device_bytes"] <= budget
    finally:
        srv.close()


def test_output_beyond_estimate_is_retried_within_budget(pkg):
    """A request with 150k racing locations outgrows the usual footprint
    (64 Ki entries): it fails within its charge, is queued again charged
    its worst case, and its result equals the alone result; the workers'
    charges stay within the budget throughout."""
    n = 150000
    r = np.zeros(2 * n, dtype=RECORD_DTYPE)
    r["unit"] = np.repeat(np.arange(n, dtype=np.uint64) * 3, 2)
    r["tid"] = np.tile([0, 1], n)
    r["action"] = 1
    off = np.array([0, len(r)], dtype=np.uint64)
    want, wsum = oracle.closed_form(r, off, 2)
    small = request_pool(6, seed=5, log2_max=14)
    budget = 96 << 20
    say("retry: 150k racing locations among small requests, budget 96 MiB")
    srv = pkg.Server(0, hbm_budget_bytes=budget, slots=2)
    try:
        ts = [srv.submit(recs, o, t) for recs, o, t in small[:3]]
        big = srv.submit(r, off, 2)
        ts += [srv.submit(recs, o, t) for recs, o, t in small[3:]]
        got = srv.wait(big)
        assert len(got[0]) == n
        assert got[0].tobytes() == want.tobytes() and got[1].tobytes() == wsum.tobytes()
        for (recs, o, t), tk in zip(small, ts):
            g = srv.wait(tk)
            w, ws = oracle.closed_form(recs, o, t)
            assert g[0].tobytes() == w.tobytes() and g[1].tobytes() == ws.tobytes()
        st = srv.stats()
        assert st["failed"] == 0 and st["requeued"] >= 1
        assert st["peak_inflight_bytes"] <= budget and st["device_bytes"] <= budget
    finally:
        srv.close()


def test_concurrent_waits_on_one_ticket(pkg):
    """Two threads wait on the same ticket: one collects the result, the
    other gets SIM_EINVAL (ticket collected), never freed memory."""
    recs, off, tpb = request_pool(1, seed=4, log2_max=16)[0]
    srv = pkg.Server(0, slots=1)
    try:
        for _ in range(5):
            t = srv.submit(recs, off, tpb)
            out = [None, None]

            def waiter(k):
                try:
                    out[k] = srv.wait(t)
                except pkg.SimError as e:
                    out[k] = e.code

            ths = [threading.Thread(target=waiter, args=(k,)) for k in range(2)]
            for th in ths:
                th.start()
            for th in ths:
                th.join()
            codes = [o for o in out if isinstance(o, int)]
            assert len(codes) == 1 and codes[0] == pkg.SIM_EINVAL
    finally:
        srv.close()


def test_admission_and_tickets(pkg):
    recs, off, tpb = request_pool(1, seed=3, log2_max=16)[0]
    srv = pkg.Server(0, hbm_budget_bytes=1 << 20, slots=1)
    try:
        big = np.zeros(1 << 16, dtype=RECORD_DTYPE)  # 64 Ki records need more than 1 MiB
        with pytest.raises(pkg.SimError) as ei:
            srv.submit(big, None, 32)
        assert ei.value.code == pkg.SIM_ENOMEM
        small = tracegen.c0()[:600]
        t = srv.submit(small, None, 256)
        got = srv.wait(t, timeout_ms=60000)
        want, wsum = oracle.closed_form(small, tpb=256)
        assert got[0].tobytes() == want.tobytes() and got[1].tobytes() == wsum.tobytes()
        with pytest.raises(pkg.SimError) as ei:
            srv.poll(t)  # consumed
        assert ei.value.code == pkg.SIM_EINVAL
        with pytest.raises(pkg.SimError) as ei:
            srv.submit(small, np.array([0, 700, 600], dtype=np.uint64), [256, 256])
        assert ei.value.code == pkg.SIM_EINVAL
    finally:
        srv.close()
    # pending requests are finished by close(); uncollected results are freed
    srv = pkg.Server(0, slots=2)
    for _ in range(20):
        srv.submit(recs, off, tpb)
    srv.close()


def test_reserved_buffers(pkg):
    """Workers allocate their buffers at creation when asked; a reservation
    beyond a worker's budget share is refused."""
    with pytest.raises(pkg.SimError) as ei:
        pkg.Server(0, hbm_budget_bytes=64 << 20, slots=2, reserve_records=1 << 22)
    assert ei.value.code == pkg.SIM_EINVAL
    srv = pkg.Server(0, hbm_budget_bytes=1 << 30, slots=2, reserve_records=1 << 18)
    try:
        st = srv.stats()
        assert st["device_bytes"] >= 2 * (1 << 18) * 32
        recs, off, tpb = request_pool(1, seed=9, log2_max=17)[0]
        want, wsum = oracle.closed_form(recs, off, tpb)
        got = srv.wait(srv.submit(recs, off, tpb))
        assert got[0].tobytes() == want.tobytes() and got[1].tobytes() == wsum.tobytes()
        assert srv.stats()["device_bytes"] == st["device_bytes"]  # nothing grew
    finally:
        srv.close()
    ctx = pkg.Context(0, reserve_records=1 << 18, reserve_traces=8)
    try:
        r = tracegen.c0()
        want, _ = oracle.closed_form(r, tpb=256)
        assert ctx.check_traces(r, None, 256)[0].tobytes() == want.tobytes()
    finally:
        ctx.close()
