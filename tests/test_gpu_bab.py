"""Multi-neuron constraints (gamma), branch-and-bound and serving on the GPU path (needs an MI355X)."""
import numpy as np
import pytest

import workloads as W
from oracle import backsub as ob
from oracle import bab as obab
from oracle import enum as oen
from oracle import mnc as omnc
from oracle import net as onet
from oracle import optimize as oo

from _common import assert_parity, mnc_layers, oracle_query, root_unstable, sampled_min_sub

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00263_amd as P
    P.lib()
    yield


def _P():
    import paper_2205_00263_amd as P
    return P


# --------------------------------------------------------------------------- gamma
@pytest.mark.parametrize("cfg", [3, 1])
def test_mnc_gamma_parity(cfg):
    P = _P()
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    mncs = omnc.generate(net_o, root.states, q.lo, q.hi, cap=60, max_groups=4)
    oo.attach_mncs(q, root, mncs)
    assert sum(m.e for m in mncs.values()) > 0
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=32, max_mnc=60)
    rid, lb0, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0, mncs=mnc_layers(net_o, mncs))
    assert_parity(lb0, root.lb, "root lb with mnc")
    # gamma gradient at random feasible parameters (final set)
    rng = np.random.default_rng(5)
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    gam = np.zeros(net.n_relu * 60, np.float32)
    for t, i in enumerate(net_o.relus):
        e = mncs[i].e
        g = rng.uniform(0, 0.3, e).astype(np.float32)
        gam[t * 60:t * 60 + e] = g
        root.sets["final"][i]["gamma"] = g.astype(np.float64)
    pb.set_params(rid, 0, gamma=gam)
    lbr, ga, gb, gg = pb.bound_grad(rid, 0)
    out = ob.backsub(net_o, ob.spec_start(net_o, q.C), q.c0, root.states, root.sets["final"], q.mncs, q.lo, q.hi)
    assert_parity(lbr, out["lb"], "rows with gamma")
    g = oo.bound_grads(net_o, out, q.mncs)
    ref = np.zeros_like(gam)
    for t, i in enumerate(net_o.relus):
        ref[t * 60:t * 60 + mncs[i].e] = g[i]["gamma"]
    assert np.linalg.norm(gg - ref) <= 1e-3 * max(np.linalg.norm(ref), 1e-6)
    # optimise alpha, beta, gamma on split subproblems
    for t, i in enumerate(net_o.relus):
        root.sets["final"][i]["gamma"] = np.zeros(mncs[i].e)
    pb.set_params(rid, 0, gamma=np.zeros_like(gam))
    unst = root_unstable(net_o, root)
    m0 = 0 if len(unst[0]) else 1
    j0 = int(unst[m0][0])
    kids = pb.branch_split([rid], [m0], [j0])
    okids = obab.branch_split(net_o, root, m0, j0)
    lb, ub = pb.bound_optimize(kids, steps=4)
    for b in range(2):
        ref = oo.bound_optimize(q, okids[b], steps=4).lb
        assert_parity(lb[b], ref, f"child {b} with gamma")
        S = {i: okids[b].states[i].S for i in net_o.relus}
        assert np.all(lb[b] <= sampled_min_sub(net_o, wl, S) + 1e-6)


# --------------------------------------------------------------------------- branching scores
@pytest.mark.parametrize("cfg", [3, 1])
def test_branch_scores_match_oracle(cfg):
    """Active constraint scores (and their cost adjusted form) of a root and two children after
    4 Adam steps and with random feasible gamma, against the oracle evaluated on the GPU's own
    gamma and bounds: the candidate
    sets bit for bit, the scores to 1e-5 of the subproblem's largest, and the chosen neuron a
    candidate whose score is the maximum (to the same tolerance)."""
    from types import SimpleNamespace as NS
    from oracle import branching as obr
    P = _P()
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    mncs = omnc.generate(net_o, root.states, q.lo, q.hi, cap=60, max_groups=4)
    oo.attach_mncs(q, root, mncs)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=32, max_mnc=60)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0, mncs=mnc_layers(net_o, mncs))
    unst = root_unstable(net_o, root)
    m0 = 0 if len(unst[0]) else 1
    kids = pb.branch_split([rid], [m0], [int(unst[m0][0])])
    ids = [rid] + [int(k) for k in kids]
    pb.bound_optimize(ids, steps=4)
    n_mnc = [mncs[i].e if i in mncs else 0 for i in net_o.relus]
    # random feasible gamma in the spec set (the optimiser may leave it at zero on small nets)
    rng = np.random.default_rng(17 + cfg)
    for sid in ids:
        gam = np.zeros(net.n_relu * 60, np.float32)
        for t in range(net.n_relu):
            gam[t * 60:t * 60 + n_mnc[t]] = rng.uniform(0, 0.3, n_mnc[t]) * (rng.uniform(size=n_mnc[t]) < 0.7)
        pb.set_params(sid, 0, gamma=gam)
    costs = P.split_costs(wl.nodes, n_mnc).tolist()
    bl, bn, sc = pb.branch_scores(ids, want_scores=True)
    cbl, cbn, csc = pb.branch_scores(ids, layer_weight=[1.0 / c for c in costs], want_scores=True)
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    positive = 0
    for b, sid in enumerate(ids):
        _, _, g = pb.get_params(sid, 0)
        states, fin = {}, {}
        for t, i in enumerate(net_o.relus):
            l, u, S = pb.get_bounds(sid, t)
            states[i] = ob.ReluState(l.astype(np.float64), u.astype(np.float64), S)
            fin[i] = {"gamma": g[t * 60:t * 60 + n_mnc[t]].astype(np.float64)}
        ref = obr.acs_scores(net_o, NS(states=states, sets={"final": fin}), mncs)
        cref = obr.cab_scores(ref, {i: costs[t] for t, i in enumerate(net_o.relus)})
        for name, got, rr, L, J in (("acs", sc[b], ref, bl[b], bn[b]), ("cab", csc[b], cref, cbl[b], cbn[b])):
            r = np.concatenate([rr[i] for i in net_o.relus])
            fin_r = np.isfinite(r)
            assert np.array_equal(np.isfinite(got), fin_r), (name, b, "candidate sets differ")
            if not fin_r.any():
                assert (L, J) == (-1, -1)
                continue
            top = np.abs(r[fin_r]).max()
            tol = 1e-5 * top + 1e-30
            assert np.all(np.abs(got[fin_r] - r[fin_r]) <= tol), (name, b, np.abs(got[fin_r] - r[fin_r]).max(), top)
            assert L >= 0 and fin_r[offs[L] + J], (name, b, L, J)
            assert r[offs[L] + J] >= r[fin_r].max() - 2 * tol, (name, b, L, J)
            positive += int(top > 0)
    assert positive > 0, "gamma stayed zero: the scores were never exercised"
    # the call needs multi-neuron constraints
    pb2 = P.Problem(net, n_spec=wl.C.shape[0], capacity=4)
    rid2, _, _ = pb2.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    with pytest.raises(P.MnbError):
        pb2.branch_scores([rid2])


# --------------------------------------------------------------------------- BaB soundness / completeness
def _gpu_bab(P, wl, steps=10, max_sub=2000):
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=2 * max_sub + 16)
    rid, lb, ub = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    if np.any(ub < 0):
        return "falsified", 1
    queue = [rid]
    bounded = 1
    while queue:
        lb, ub, bl, bn = pb.bound_optimize(queue, want_branch=True, steps=steps)
        bounded += len(queue)
        if np.any(ub < 0):
            return "falsified", bounded
        par, lay, neu = [], [], []
        for b, sid in enumerate(queue):
            if np.all(lb[b] > 0):
                continue
            if bl[b] < 0:
                return "unknown", bounded
            par.append(sid); lay.append(bl[b]); neu.append(bn[b])
        done = list(queue)
        queue = []
        if par:
            if len(par) * 2 > max_sub:
                return "unknown", bounded
            queue = list(pb.branch_split(par, lay, neu))
        pb.release(done)
    return "verified", bounded


# (seed, eps) of tiny nets whose optimised root bound is negative while the exact minimum is
# positive (found with the oracle), plus a few that resolve at the root.
HARD = [(5, 0.3), (6, 0.5), (8, 0.5), (16, 0.5), (23, 0.5), (28, 0.3), (41, 0.5), (47, 0.3)]
EASY = [(0, 0.25), (1, 0.25), (4, 0.25)]


@pytest.mark.parametrize("seed,eps", HARD + EASY)
def test_bab_is_sound_and_complete_on_tiny_nets(seed, eps):
    P = _P()
    nodes = W.tiny_fc(seed, (3, 6, 5, 2))
    x0, lo, hi = W.make_input(nodes[0]["shape"], eps, 40 + seed)
    Cm, c0, _ = W.make_spec(nodes, x0)
    wl = W.Workload(nodes, x0, lo, hi, Cm, c0, 0, eps)
    net_o = onet.Net(nodes)
    top = len(nodes) - 1
    exact = min(oen.exact_min(net_o, lo, hi, {top: Cm[r].astype(np.float64)}, float(c0[r]))[0]
                for r in range(Cm.shape[0]))
    verdict, n = _gpu_bab(P, wl)
    q = oo.Query(net_o, lo, hi, Cm, c0)
    v_o, st = obab.bab(q, steps=10, batch=8, max_subproblems=400)
    print(seed, eps, "exact", exact, "gpu", verdict, n, "oracle", v_o, st, flush=True)
    if exact < -1e-6:
        assert verdict != "verified"          # soundness
    elif exact > 1e-4:
        assert verdict == "verified"          # completeness on these nets
    if (seed, eps) in HARD:
        assert n > 2                          # the root alone did not decide it


def test_bab_resnet_small_agrees_with_oracle_verdict():
    P = _P()
    wl = W.make_workload(4, scale="small", eps=0.004)
    net_o, q = oracle_query(wl)
    v_o, st = obab.bab(q, steps=10, batch=8, max_subproblems=400)
    v_g, n = _gpu_bab(P, wl, steps=10, max_sub=400)
    print("oracle", v_o, st, "gpu", v_g, n, flush=True)
    if v_o in ("verified", "falsified"):
        assert v_g == v_o


# --------------------------------------------------------------------------- serving
def _queries(n, seed=5000):
    """Tiny-net queries that need branching, plus conv queries of mixed difficulty."""
    rng = np.random.default_rng(seed)
    nets, qs = [], []
    for (sd, eps) in HARD:
        nodes = W.tiny_fc(sd, (3, 6, 5, 2))
        x0, lo, hi = W.make_input(nodes[0]["shape"], eps, 40 + sd)
        Cm, c0, _ = W.make_spec(nodes, x0)
        nets.append(nodes)
        qs.append((len(nets) - 1, lo, hi, Cm, c0))
    nets.append(W.make_net(2, scale="small"))
    ci = len(nets) - 1
    while len(qs) < n:
        eps = float(rng.uniform(0.005, 0.08))
        x0, lo, hi = W.make_input(nets[ci][0]["shape"], eps, int(rng.integers(0, 2**31)))
        Cm, c0, _ = W.make_spec(nets[ci], x0, n_spec=1, seed=int(rng.integers(0, 2**31)))
        qs.append((ci, lo, hi, Cm, c0))
    return nets, qs


def test_serving_alone_equals_mix():
    P = _P()
    nets, qs = _queries(16)
    gnets = [P.Net(n) for n in nets]
    srv = P.Server(gnets, max_batch=64, steps=5)
    alone = []
    for (ni, lo, hi, Cm, c0) in qs:
        t = srv.query_submit(ni, lo, hi, Cm, c0, timeout_s=120)
        alone.append(srv.wait(t))
    tickets = [srv.query_submit(ni, lo, hi, Cm, c0, timeout_s=120) for (ni, lo, hi, Cm, c0) in qs]
    mix = [srv.wait(t) for t in tickets]
    srv.close()
    for a, m in zip(alone, mix):
        print(a["verdict"], m["verdict"], a["lb"], m["lb"], a["subproblems"], m["subproblems"], flush=True)
        assert a["verdict"] == m["verdict"]
        assert abs(a["lb"] - m["lb"]) <= 1e-4 * max(1.0, abs(a["lb"]))
        if a["verdict"] == "verified":
            assert a["subproblems"] == m["subproblems"]
    assert sum(a["subproblems"] > 2 for a in alone) >= 4   # branching happened


def test_serving_with_mnc_is_sound_and_complete():
    """Queries that carry multi-neuron constraints are branched in the server by cost adjusted
    active constraint scores; their verdicts against the exact minimum (activation-pattern
    enumeration) on the tiny nets: never verified below zero nor falsified above it, and most
    positive ones verified (a leaf whose neurons are all split can still end UNKNOWN: its split
    constraints are enforced through beta after a fixed number of Adam steps, not exactly)."""
    P = _P()
    nets, qs = [], []
    for (sd, eps) in HARD[:6]:
        nodes = W.tiny_fc(sd, (3, 6, 5, 2))
        x0, lo, hi = W.make_input(nodes[0]["shape"], eps, 40 + sd)
        Cm, c0, _ = W.make_spec(nodes, x0)
        net_o = onet.Net(nodes)
        q = oo.Query(net_o, lo, hi, Cm, c0)
        root, _ = oo.root_pass(q)
        mncs = omnc.generate(net_o, root.states, q.lo, q.hi, cap=60, max_groups=4)
        top = len(nodes) - 1
        exact = min(oen.exact_min(net_o, lo, hi, {top: Cm[r].astype(np.float64)}, float(c0[r]))[0]
                    for r in range(Cm.shape[0]))
        nets.append(nodes)
        qs.append((len(nets) - 1, lo, hi, Cm, c0, mnc_layers(net_o, mncs), exact, sum(m.e for m in mncs.values())))
    srv = P.Server([P.Net(n) for n in nets], max_batch=64, steps=10)
    tickets = [srv.query_submit(ni, lo, hi, Cm, c0, mncs=mm, timeout_s=120) for (ni, lo, hi, Cm, c0, mm, _, _) in qs]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    with_mnc = positive = verified = 0
    for r, (_, _, _, _, _, _, exact, ne) in zip(res, qs):
        print(r["verdict"], r["subproblems"], exact, ne, flush=True)
        if exact < -1e-6:
            assert r["verdict"] != "verified"
        elif exact > 1e-4:
            assert r["verdict"] != "falsified"
            positive += 1
            verified += r["verdict"] == "verified"
        with_mnc += ne > 0
    assert with_mnc >= 3
    assert verified * 2 >= positive, (verified, positive)


# --------------------------------------------------------------------------- alpha-contribution branching
@pytest.mark.parametrize("cfg,scale", [(1, "small"), (2, "small"), (4, "small"), (2, "full")])
def test_contribution_branching_matches_oracle(cfg, scale):
    """bound_optimize's branching choice (want_branch) against the oracle's alpha-contribution score
    (oracle.bab.branching_score) evaluated on the GPU's own last-evaluation state: the spec rows are
    back-substituted by the oracle with the subproblem's parameters (set 0) and bounds as they stand
    after the call.  The GPU's scores (mnb_contribution_scores, same state) must give the same choice
    as bound_optimize bit for bit, the same candidate sets bit for bit, scores within 1e-5 of the
    subproblem's largest, and the chosen neuron a maximum to that tolerance."""
    from types import SimpleNamespace as NS
    from _common import make_batch
    P = _P()
    wl = W.make_workload(cfg, scale=scale)
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    n_sub = 6 if scale == "small" else 3
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=8 * n_sub + 8)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    splits = W.make_split_sets(root_unstable(net_o, root), n_sub, 1, 3, seed=77 + cfg)
    ids = make_batch(pb, rid, splits)
    _, _, bl, bn = pb.bound_optimize(ids, steps=3, want_branch=True)
    bl2, bn2, sc = pb.contribution_scores(ids)
    assert np.array_equal(bl, bl2) and np.array_equal(bn, bn2), (bl, bl2, bn, bn2)
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    for b, sid in enumerate(ids):
        a_, b_, _ = pb.get_params(int(sid), 0)
        states, params = {}, {}
        for t, i in enumerate(net_o.relus):
            l, u, S = pb.get_bounds(int(sid), t)
            states[i] = ob.ReluState(l.astype(np.float64), u.astype(np.float64), S)
            params[i] = {"alpha": a_[offs[t]:offs[t + 1]].astype(np.float64),
                         "beta": b_[offs[t]:offs[t + 1]].astype(np.float64)}
        out = ob.backsub(net_o, ob.spec_start(net_o, q.C), q.c0, states, params, None, q.lo, q.hi)
        ref = obab.branching_score(net_o, NS(states=states), out["records"])
        r = np.concatenate(ref)
        fin = np.isfinite(r)
        assert np.array_equal(np.isfinite(sc[b]), fin), (b, "candidate sets differ")
        if not fin.any():
            assert (bl[b], bn[b]) == (-1, -1)
            continue
        top = np.abs(r[fin]).max()
        tol = 1e-5 * top + 1e-30
        assert np.all(np.abs(sc[b][fin] - r[fin]) <= tol), (b, np.abs(sc[b][fin] - r[fin]).max(), top)
        assert bl[b] >= 0 and fin[offs[bl[b]] + bn[b]], (b, bl[b], bn[b])
        assert r[offs[bl[b]] + bn[b]] >= r[fin].max() - 2 * tol, (b, bl[b], bn[b])
        om, oj = obab.pick_branch(ref)
        srt = np.sort(r[fin])
        if len(srt) == 1 or srt[-1] > srt[-2] + 2 * tol:   # a clear maximum: the same neuron
            assert (bl[b], bn[b]) == (om, oj), (b, (bl[b], bn[b]), (om, oj))
