"""The serving loop under memory pressure and its failure paths (needs an MI355X).

Queries whose trees fit a slot pool alone get the same verdicts when they share a pool too small for
all of them (parked splits and preemption instead of giving up); a query that cannot fit alone ends
UNKNOWN with the memory reason; waiting and live queries time out; impossible queries are rejected at
submission; NaN weights give lb = -inf; a rejected call writes nothing."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00263_amd as P
    P.lib()
    yield


def _queries(n, seed=3, eps=0.05):
    nodes = W.make_net(1, scale="small")
    rng = np.random.default_rng(seed)
    qs = []
    for _ in range(n):
        x0, lo, hi = W.make_input(nodes[0]["shape"], eps, int(rng.integers(0, 2**31)))
        Cm, c0, _ = W.make_spec(nodes, x0, n_spec=1, seed=int(rng.integers(0, 2**31)))
        qs.append((0, lo, hi, Cm, c0))
    return nodes, qs


def test_small_pool_alone_equals_mix():
    """Each query alone within a pool of max_slots slots, then all of them at once in that pool."""
    import paper_2205_00263_amd as P
    nodes, qs = _queries(24)
    net = P.Net(nodes)
    big = P.Server([net], max_batch=64, steps=5)
    alone_free = [big.wait(big.query_submit(*q, timeout_s=120)) for q in qs]
    big.close()
    need = [r["subproblems"] for r in alone_free]
    # queries whose trees branch but stay small; the pool holds one of them at a time comfortably
    pick = [k for k, r in enumerate(alone_free) if 3 <= r["subproblems"] <= 40 and r["verdict"] != "unknown"][:6]
    assert len(pick) >= 3, need
    cap = 48
    srv = P.Server([net], max_batch=64, steps=5, max_slots=cap)
    alone = [srv.wait(srv.query_submit(*qs[k], timeout_s=120)) for k in pick]
    tickets = [srv.query_submit(*qs[k], timeout_s=120) for k in pick]
    mix = [srv.wait(t) for t in tickets]
    srv.close()
    for k, a, m in zip(pick, alone, mix):
        print(k, a["verdict"], m["verdict"], a["subproblems"], m["subproblems"], m["restarts"], flush=True)
        assert a["verdict"] == m["verdict"] == alone_free[k]["verdict"]
        assert abs(a["lb"] - m["lb"]) <= 1e-4 * max(1.0, abs(a["lb"]))


def test_query_too_big_for_its_pool_ends_unknown_memory():
    import paper_2205_00263_amd as P
    nodes, qs = _queries(24)
    net = P.Net(nodes)
    big = P.Server([net], max_batch=64, steps=5)
    free = [big.wait(big.query_submit(*q, timeout_s=120)) for q in qs]
    big.close()
    k = int(np.argmax([r["subproblems"] for r in free]))
    assert free[k]["subproblems"] >= 12, [r["subproblems"] for r in free]
    srv = P.Server([net], max_batch=64, steps=5, max_slots=4)
    r = srv.wait(srv.query_submit(*qs[k], timeout_s=120))
    srv.close()
    assert r["verdict"] in ("unknown", free[k]["verdict"])
    if r["verdict"] == "unknown":
        assert r["reason"] == "memory"


def test_timeouts_of_waiting_and_live_queries():
    import paper_2205_00263_amd as P
    nodes, qs = _queries(4)
    net = P.Net(nodes)
    srv = P.Server([net], max_batch=64, steps=5)
    r = srv.wait(srv.query_submit(*qs[0], timeout_s=1e-9))
    assert r["verdict"] == "timeout" and r["reason"] == "time"
    srv.close()


def test_submit_rejects_a_query_that_cannot_fit():
    import paper_2205_00263_amd as P
    nodes, qs = _queries(1)
    net = P.Net(nodes)
    srv = P.Server([net], max_batch=64, steps=5, mem_budget=1024)
    with pytest.raises(P.MnbError):
        srv.query_submit(*qs[0], timeout_s=10)
    srv.close()


def test_nan_weights_give_minus_infinity():
    """A NaN reaching a bound never yields a finite (possibly unsound) lower bound."""
    import paper_2205_00263_amd as P
    wl = W.make_workload(1, scale="small")
    nodes = [dict(n) for n in wl.nodes]
    W2 = np.array(nodes[3]["W"], dtype=np.float32, copy=True)
    W2[0, 0] = np.nan
    nodes[3]["W"] = W2
    net = P.Net(nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=8)
    rid, lb, ub = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    assert np.all(np.isneginf(lb)), lb
    kids = pb.branch_split([rid], [0], [0])
    lb2, _ = pb.bound_optimize(kids, steps=2)
    assert np.all(np.isneginf(lb2)), lb2


def test_invalid_calls_write_nothing():
    import paper_2205_00263_amd as P
    from paper_2205_00263_amd._lib import MNB_EINVAL
    wl = W.make_workload(1, scale="small")
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=8)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    used0 = pb.usage()[0]
    lo = np.array(wl.lo, copy=True)
    lo[0] = wl.hi[0] + 1.0          # lo > hi
    with pytest.raises(P.MnbError) as e:
        pb.bound_init(lo, wl.hi, wl.C, wl.c0)
    assert e.value.code == MNB_EINVAL and pb.usage()[0] == used0
    with pytest.raises(P.MnbError) as e:
        pb.bound_optimize([rid, rid], steps=1)   # duplicate id
    assert e.value.code == MNB_EINVAL
    with pytest.raises(P.MnbError) as e:
        pb.branch_split([rid], [0], [10 ** 6])   # neuron out of range
    assert e.value.code == MNB_EINVAL and pb.usage()[0] == used0
    l0, u0, _ = pb.get_bounds(rid, 0)
    lb, ub = pb.bound_optimize([rid], steps=0)
    l1, u1, _ = pb.get_bounds(rid, 0)
    assert np.array_equal(l0, l1) and np.array_equal(u0, u1)
