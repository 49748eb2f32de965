"""The allocation-free branching scores (needs an MI355X): mnb_branch_scores_noalloc, called through the
C ABI, against mnb_branch_scores on the same subproblems, bit for bit, on two calls in a row (the second
with fewer subproblems), and its rejection of a call larger than its fixed scratch array."""
import ctypes as C

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


def _call(fn, pb, ids, w, td, fill=0):
    n = len(ids)
    ids = np.ascontiguousarray(ids, np.int64)
    sc = np.full((n, td), fill, np.float32)
    bl = np.full(n, fill, np.int32)
    bn = np.full(n, fill, np.int32)
    wp = w.ctypes.data_as(C.POINTER(C.c_float)) if w is not None else None
    rc = fn(pb.h, ids.ctypes.data_as(C.POINTER(C.c_int64)), n, wp, sc.ctypes.data_as(C.POINTER(C.c_float)),
            bl.ctypes.data_as(C.POINTER(C.c_int32)), bn.ctypes.data_as(C.POINTER(C.c_int32)))
    return rc, sc, bl, bn


def _subproblems(P, cfg, scale, n, cap):
    from bench import make_batch
    wl = W.make_workload(cfg, scale=scale)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=3 * n + 16, max_mnc=cap)   # make_batch holds 3 n at once
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    pb.mnc_generate(rid, cap=cap)
    unstable = []
    for m in range(net.n_relu):
        l, u, _ = pb.get_bounds(rid, m)
        unstable.append(np.nonzero((l < 0) & (u > 0))[0])
    ids = make_batch(P, pb, rid, W.make_split_sets(unstable, n, 1, 3, seed=5))
    return net, pb, ids


def test_noalloc_scores_equal_the_allocating_call():
    import paper_2205_00263_amd as P
    from paper_2205_00263_amd._lib import lib
    L = lib()
    net, pb, ids = _subproblems(P, 3, "small", 12, 60)
    pb.bound_optimize(ids, steps=3)
    rng = np.random.default_rng(11)
    for sid in ids:   # gamma of the spec set, some of it nonzero, so that the scores differ
        _, _, g = pb.get_params(int(sid), 0)
        pb.set_params(int(sid), 0, gamma=(rng.uniform(0, 0.3, g.shape) * (rng.uniform(size=g.shape) < 0.5)))
    td = sum(net.relu_sizes)
    w = np.asarray(1.0 / P.split_costs(net.nodes), np.float32)
    positive = 0
    for sub in (ids[:12], ids[:5]):   # the second call is smaller: stale scratch must not leak into it
        for wt in (None, w):
            rc0, s0, l0, n0 = _call(L.mnb_branch_scores, pb, sub, wt, td)
            rc1, s1, l1, n1 = _call(L.mnb_branch_scores_noalloc, pb, sub, wt, td, fill=7)
            assert rc0 == 0 and rc1 == 0, L.mnb_last_error()
            assert np.array_equal(s0, s1) and np.array_equal(l0, l1) and np.array_equal(n0, n1)
            positive += int(np.isfinite(s0).any() and np.nanmax(np.where(np.isfinite(s0), s0, 0)) > 0)
    assert positive > 0


def test_noalloc_rejects_calls_beyond_its_scratch():
    """ConvBig's 62,464 neurons: 89 subproblems fit the 64 MiB array, 90 do not (MNB_EINVAL, nothing
    written)."""
    import paper_2205_00263_amd as P
    from paper_2205_00263_amd._lib import MNB_EINVAL, lib
    L = lib()
    net, pb, ids = _subproblems(P, 3, "full", 90, 500)
    td = sum(net.relu_sizes)
    rc, s, bl, bn = _call(L.mnb_branch_scores_noalloc, pb, ids, None, td, fill=7)
    assert rc == MNB_EINVAL
    assert np.all(s == 7) and np.all(bl == 7) and np.all(bn == 7)
    rc0, s0, l0, n0 = _call(L.mnb_branch_scores, pb, ids[:89], None, td)
    rc1, s1, l1, n1 = _call(L.mnb_branch_scores_noalloc, pb, ids[:89], None, td)
    assert rc0 == 0 and rc1 == 0, L.mnb_last_error()
    assert np.array_equal(s0, s1) and np.array_equal(l0, l1) and np.array_equal(n0, n1)
