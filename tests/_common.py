"""Shared helpers of the test-suite: build the same query for the oracle and the GPU path."""
import numpy as np

import workloads as W
from oracle import backsub as ob
from oracle import bab as obab
from oracle import mnc as omnc
from oracle import net as onet
from oracle import optimize as oo


def tol(ref):
    """Parity bar: |gpu - oracle| <= 1e-4 max(1, |oracle|)."""
    return 1e-4 * np.maximum(1.0, np.abs(ref))


def assert_parity(gpu, ref, what=""):
    gpu = np.asarray(gpu, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(gpu - ref)
    bad = err > tol(ref)
    assert not np.any(bad), f"{what}: {bad.sum()} of {bad.size} outside 1e-4 rel; worst {err.max():.3e} " \
                            f"at {np.unravel_index(np.argmax(err), err.shape)} gpu={gpu.ravel()[np.argmax(err)]} " \
                            f"ref={ref.ravel()[np.argmax(err)]}"


def oracle_query(wl, mncs=None, margin=0.0):
    net = onet.Net(wl.nodes)
    return net, oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0, mncs, margin)


def mnc_layers(net, mncs):
    """oracle Mnc dict (relu node -> Mnc) -> GPU layer dict (relu layer -> CSR tuple)."""
    from paper_2205_00263_amd import mnc_to_csr
    out = {}
    for i, m in mncs.items():
        if m.e > 0:
            out[net.relus.index(i)] = mnc_to_csr(m.P, m.Phat, m.p)
    return out


def sampled_min(net, wl, n=4000, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(wl.lo, wl.hi, size=(n, len(wl.lo)))
    corners = np.where(rng.integers(0, 2, size=(64, len(wl.lo))) > 0, wl.hi, wl.lo)
    X = np.vstack([X, corners])
    f = onet.forward(net, X) @ np.asarray(wl.C, np.float64).T + wl.c0
    return f.min(0)


def root_unstable(net, sub):
    return [np.nonzero((sub.states[i].l < 0) & (sub.states[i].u > 0))[0] for i in net.relus]


def sampled_min_sub(net, wl, S, n=20000, seed=0):
    """min of the spec over samples that satisfy a subproblem's split constraints (inf if none do).

    S: dict relu-node -> split diagonal (-1: zhat >= 0, +1: zhat <= 0)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(wl.lo, wl.hi, size=(n, len(wl.lo)))
    vals = onet.forward_all(net, X)
    ok = np.ones(len(X), dtype=bool)
    for i, s in S.items():
        zh = vals[net.nodes[i]["src"]]
        for j in np.nonzero(s)[0]:
            ok &= (zh[:, j] >= 0) if s[j] == -1 else (zh[:, j] <= 0)
    if not ok.any():
        return np.full(np.asarray(wl.C).shape[0], np.inf)
    f = vals[-1][ok] @ np.asarray(wl.C, np.float64).T + wl.c0
    return f.min(0)


def make_subproblems(P, pb, rid, net_o, q, root, splits):
    """Create subproblems by chained branch_split on both sides; returns (gpu ids, oracle subproblems)."""
    ids, subs = [], []
    for sp in splits:
        gid, osub = rid, root
        chain = []
        for (m, j, sgn) in sp:
            ch = pb.branch_split([gid], [m], [j])
            pos, neg = obab.branch_split(net_o, osub, m, j)
            keep = 0 if sgn > 0 else 1
            chain.append(int(ch[1 - keep]))
            gid = int(ch[keep])
            osub = pos if sgn > 0 else neg
        if chain:
            pb.release(chain)
        ids.append(gid)
        subs.append(osub)
    return np.array(ids), subs


def make_batch(pb, rid, splits):
    """GPU subproblems of a batch from the root by chained branch_split, one call per split depth
    (the way the benchmark builds its batch); returns the ids in split-set order."""
    cur = np.full(len(splits), rid, np.int64)
    depth = max(len(s) for s in splits)
    for t in range(depth):
        idx = [b for b, s in enumerate(splits) if len(s) > t]
        kids = pb.branch_split(cur[idx], [splits[b][t][0] for b in idx], [splits[b][t][1] for b in idx])
        drop = []
        for k, b in enumerate(idx):
            keep = 0 if splits[b][t][2] > 0 else 1
            if t > 0:
                drop.append(cur[b])
            cur[b] = kids[2 * k + keep]
            drop.append(kids[2 * k + 1 - keep])
        pb.release(drop)
    return cur


def oracle_subproblem(net_o, root, split):
    """The oracle's subproblem for one split set (chained branch_split from the root)."""
    s = root
    for (m, j, sg) in split:
        pos, neg = obab.branch_split(net_o, s, m, j)
        s = pos if sg > 0 else neg
    return s
