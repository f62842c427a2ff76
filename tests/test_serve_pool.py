"""Admission by memory footprint: the workspace pool's accounting (host side)."""
import threading

from paper_2402_09356_amd.serve import Problem, WorkspacePool


class _Plan:
    def __init__(self, n, nb, ws_bytes):
        self.n, self.nb, self.maxrank, self.ws_bytes = n, nb, nb // 2, ws_bytes


def _prob(pid, n, nb, ws):
    return Problem(pid=pid, plan=_Plan(n, nb, ws), locs=None, z=None, tol=1e-7)


def test_budget_blocks_then_reuse():
    pool = WorkspacePool(budget_bytes=1000, device="cpu")
    a, b = _prob(0, 100, 10, 600), _prob(1, 200, 20, 300)
    wa = pool.acquire(a)
    wb = pool.acquire(b)
    assert wa is not None and wb is not None and pool.allocated == 900
    assert pool.acquire(b) is None          # 900 + 300 > 1000: not admitted
    pool.release(b, wb)
    assert pool.acquire(b) is wb            # reused, no new memory
    assert pool.allocated == 900
    pool.release(a, wa)
    c = _prob(2, 100, 10, 600)              # same plan shape as a
    assert pool.acquire(c) is wa


def test_concurrent_acquire_never_exceeds_budget():
    pool = WorkspacePool(budget_bytes=10 * 64, device="cpu")
    probs = [_prob(i, 64 * (i % 3 + 1), 8, 64) for i in range(40)]
    got = []
    lock = threading.Lock()

    def take(p):
        w = pool.acquire(p)
        with lock:
            got.append(w)

    ts = [threading.Thread(target=take, args=(p,)) for p in probs]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert sum(w is not None for w in got) == 10
    assert pool.allocated == 640


def test_idle_workspaces_of_other_shapes_are_evicted():
    pool = WorkspacePool(budget_bytes=1000, device="cpu")
    a, b = _prob(0, 100, 10, 600), _prob(1, 200, 20, 300)
    wa, wb = pool.acquire(a), pool.acquire(b)
    pool.release(a, wa)
    pool.release(b, wb)
    assert pool.allocated == 900
    c = _prob(2, 300, 30, 200)                # a new shape: 900 + 200 > 1000
    wc = pool.acquire(c)
    assert wc is not None
    assert pool.allocated == 500              # a (least recently released) given up
    assert pool.acquire(b) is wb              # b's idle workspace is still there
    d = _prob(3, 400, 40, 900)                # cannot fit while b and c are in use
    assert pool.acquire(d) is None
    pool.release(b, wb)
    pool.release(c, wc)
    assert pool.acquire(d) is not None and pool.allocated == 900
