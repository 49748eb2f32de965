"""Pins of the FP64 oracle against what the paper and mathematics fix (CPU only).

Each test compares the oracle with something other than itself: printed
values (Figure 1, Table 3), closed forms (Eq. 6), LP duality (Sections 2.5
and 3.1), exhaustive enumeration (Section 3.3), dense sampling, finite
differences and library routines.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import backsub as ob
from oracle import bab as obab
from oracle import cost as ocost
from oracle import enum as oen
from oracle import lp as olp
from oracle import mnc as omnc
from oracle import net as onet
from oracle import optimize as oo

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _query(seed, widths=(3, 6, 5, 3), eps=0.4, mnc=False):
    nodes = W.tiny_fc(seed, widths)
    x0, lo, hi = W.make_input(nodes[0]["shape"], eps, 100 + seed)
    C, c0, _ = W.make_spec(nodes, x0)
    net = onet.Net(nodes)
    q = oo.Query(net, lo, hi, C, c0)
    root, _ = oo.root_pass(q)
    if mnc:
        oo.attach_mncs(q, root, omnc.generate(net, root.states, lo, hi))
    return net, q, root


def _samples(net, lo, hi, n=10000, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(lo, hi, size=(n, len(lo)))
    corners = np.where(rng.integers(0, 2, size=(256, len(lo))) > 0, hi, lo)
    return np.vstack([X, corners])


# --------------------------------------------------------------------------- Figure 1
def test_fig1_relaxation_numbers():
    g = json.load(open(os.path.join(GOLD, "fig1_relaxation.json")))
    st = ob.ReluState([g["l"]], [g["u"]])
    # a < 0 selects the upper chord: D = slope, b-underline = intercept.
    ahat, dc, _ = ob.relu_backsub(np.array([[-1.0]]), st, alpha=[g["alpha"]], beta=[0.0])
    assert ahat[0, 0] == pytest.approx(-g["upper_slope"], abs=1e-15)
    assert dc[0] == pytest.approx(-g["upper_intercept"], abs=1e-15)
    # a >= 0 selects the lower line alpha x, no constant.
    ahat, dc, _ = ob.relu_backsub(np.array([[1.0]]), st, alpha=[g["alpha"]], beta=[0.0])
    assert ahat[0, 0] == pytest.approx(g["alpha"], abs=1e-15)
    assert dc[0] == 0.0


def test_relu_identity_hand_example():
    # f = relu(x), x in [-1, 1]: the bound is 0 with alpha = 0 and -1 with alpha = 1.
    nodes = [{"kind": "input", "shape": (1, 1, 1)},
             {"kind": "fc", "src": 0, "W": np.array([[1.0]], np.float32), "b": np.zeros(1, np.float32)},
             {"kind": "relu", "src": 1},
             {"kind": "fc", "src": 2, "W": np.array([[1.0]], np.float32), "b": np.zeros(1, np.float32)}]
    net = onet.Net(nodes)
    st = {2: ob.ReluState([-1.0], [1.0])}
    for alpha, want in ((0.0, 0.0), (1.0, -1.0), (0.5, -0.5)):
        out = ob.backsub(net, ob.spec_start(net, [[1.0]]), [0.0], st,
                         {2: {"alpha": [alpha], "beta": [0.0]}}, None, [-1.0], [1.0])
        assert out["lb"][0] == pytest.approx(want)
    # the heuristic breaks the tie u = -l towards alpha = 0
    q = oo.Query(net, [-1.0], [1.0], [[1.0]], [0.0])
    root, _ = oo.root_pass(q)
    assert root.lb[0] == pytest.approx(0.0)
    # positive split with beta: f = x on [0, 1]; beta enforces zhat >= 0 and lifts the bound.
    pos, neg = obab.branch_split(net, root, 0, 0)
    out = ob.backsub(net, ob.spec_start(net, [[1.0]]), [0.0], pos.states,
                     {2: {"alpha": [0.0], "beta": [1.0]}}, None, [-1.0], [1.0])
    assert out["lb"][0] == pytest.approx(0.0)
    out = ob.backsub(net, ob.spec_start(net, [[1.0]]), [0.0], pos.states,
                     {2: {"alpha": [0.0], "beta": [0.0]}}, None, [-1.0], [1.0])
    assert out["lb"][0] == pytest.approx(-1.0)


# --------------------------------------------------------------------------- Eq. 6
def test_concretisation_matches_hoelder_without_clipping():
    rng = np.random.default_rng(3)
    a0 = rng.normal(size=(5, 7))
    c = rng.normal(size=5)
    x0 = rng.uniform(0.3, 0.7, size=7)
    eps = 0.1
    lb, xs = ob.concretize(a0, c, x0 - eps, x0 + eps)
    np.testing.assert_allclose(lb, a0 @ x0 - eps * np.abs(a0).sum(1) + c, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.einsum("rj,rj->r", a0, xs) + c, lb, atol=1e-12)


def test_rounding_margin_closed_form():
    """One affine layer under the spec: no intermediate bound, so the root bound is Eq. 6 in closed
    form (a = C W, c = C b + c0) lowered by margin * (sum_j |a_j| max(|lo_j|, |hi_j|) + |c|)."""
    rng = np.random.default_rng(8)
    W1 = rng.normal(size=(3, 6)).astype(np.float32)
    b1 = rng.normal(size=3).astype(np.float32)
    nodes = [{"kind": "input", "shape": (1, 1, 6)}, {"kind": "fc", "src": 0, "W": W1, "b": b1}]
    lo = rng.uniform(-1, 0, 6)
    hi = lo + rng.uniform(0.1, 1, 6)
    C, c0 = rng.normal(size=(2, 3)), rng.normal(size=2)
    m = 2.0 ** -20
    net = onet.Net(nodes)
    root, _ = oo.root_pass(oo.Query(net, lo, hi, C, c0, margin=m))
    a, c = C @ W1.astype(np.float64), C @ b1.astype(np.float64) + c0
    exact = np.minimum(a * lo, a * hi).sum(1) + c
    want = exact - m * (np.abs(a) @ np.maximum(np.abs(lo), np.abs(hi)) + np.abs(c))
    np.testing.assert_allclose(root.lb, want, rtol=0, atol=1e-12)
    assert np.all(root.lb < exact)


def test_rounding_margin_only_loosens():
    """On a residual net the margin touches only the reported spec-row bounds: every intermediate
    bound is the exact pass's bit for bit, and each reported lb is the exact one lowered by the
    closed-form margin of its own final row (Eq. 6 with a^(0), c of the exact pass).  A zero margin
    is the exact pass bit for bit, also through optimisation."""
    wl = W.make_workload(4, scale="small")
    net = onet.Net(wl.nodes)
    ex, out = oo.root_pass(oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0))
    z, _ = oo.root_pass(oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0, margin=0.0))
    m = 2.0 ** -12
    mg, _ = oo.root_pass(oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0, margin=m))
    assert np.array_equal(z.lb, ex.lb)
    for i in net.relus:
        assert np.array_equal(mg.states[i].l, ex.states[i].l) and np.array_equal(mg.states[i].u, ex.states[i].u)
    lo, hi = np.asarray(wl.lo, np.float64), np.asarray(wl.hi, np.float64)
    delta = m * (np.abs(out["a0"]) @ np.maximum(np.abs(lo), np.abs(hi)) + np.abs(out["c"]))
    np.testing.assert_allclose(mg.lb, ex.lb - delta, rtol=0, atol=1e-12)
    assert np.all(mg.lb < ex.lb)
    # through optimisation with splits: intermediate bounds equal, reported bounds only lower
    st0 = ex.states[net.relus[0]]
    j = int(np.nonzero((st0.l < 0) & (st0.u > 0))[0][0])
    qe = oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0)
    qm = oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0, margin=m)
    ce = oo.bound_optimize(qe, obab.branch_split(net, ex.clone(), 0, j)[0], steps=2)
    cm = oo.bound_optimize(qm, obab.branch_split(net, mg.clone(), 0, j)[0], steps=2)
    for i in net.relus:
        assert np.array_equal(ce.states[i].l, cm.states[i].l) and np.array_equal(ce.states[i].u, cm.states[i].u)
    assert np.all(cm.lb <= ce.lb)


@pytest.mark.parametrize("seed", range(4))
def test_exact_when_no_relu_is_unstable(seed):
    nodes = W.tiny_fc(seed, (4, 6, 5, 3))
    x0, lo, hi = W.make_input(nodes[0]["shape"], 1e-4, 50 + seed)
    C, c0, _ = W.make_spec(nodes, x0)
    net = onet.Net(nodes)
    q = oo.Query(net, lo, hi, C, c0)
    root, out = oo.root_pass(q)
    assert all(not np.any((s.l < 0) & (s.u > 0)) for s in root.states.values())
    top = len(net.nodes) - 1
    for r in range(C.shape[0]):
        ex, _ = oen.exact_min(net, lo, hi, {top: q.C[r]}, q.c0[r])
        assert root.lb[r] == pytest.approx(ex, abs=1e-10)
    np.testing.assert_allclose(root.ub, root.lb, atol=1e-10)   # f(x*) attains it


# --------------------------------------------------------------------------- LP duality
@pytest.mark.parametrize("seed", range(5))
def test_lp_duals_reproduce_lp_value(seed):
    net, q, root = _query(seed)
    top = len(net.nodes) - 1
    for r in range(q.n_spec):
        res = olp.lp_bound(net, root.states, {}, q.lo, q.hi, {top: q.C[r]}, q.c0[r])
        out = ob.backsub(net, {top: q.C[r:r + 1]}, q.c0[r:r + 1], root.states, res["params"],
                         None, q.lo, q.hi)
        assert out["lb"][0] == pytest.approx(res["value"], abs=1e-8)
        assert root.lb[r] <= res["value"] + 1e-10
        ex, _ = oen.exact_min(net, q.lo, q.hi, {top: q.C[r]}, q.c0[r])
        assert res["value"] <= ex + 1e-8


@pytest.mark.parametrize("seed", range(3))
def test_weak_duality_random_parameters(seed):
    net, q, root = _query(seed)
    top = len(net.nodes) - 1
    rng = np.random.default_rng(seed)
    res = olp.lp_bound(net, root.states, {}, q.lo, q.hi, {top: q.C[0]}, q.c0[0])
    for _ in range(20):
        params = {i: {"alpha": rng.uniform(0, 1, net.sizes[i]), "beta": np.zeros(net.sizes[i])}
                  for i in net.relus}
        out = ob.backsub(net, {top: q.C[:1]}, q.c0[:1], root.states, params, None, q.lo, q.hi)
        assert out["lb"][0] <= res["value"] + 1e-10


@pytest.mark.parametrize("seed", range(4))
def test_lp_duality_with_splits(seed):
    net, q, root = _query(seed)
    top = len(net.nodes) - 1
    st = root.states[net.relus[0]]
    js = np.nonzero((st.l < 0) & (st.u > 0))[0]
    for ch in obab.branch_split(net, root, 0, int(js[0])):
        oo.bound_optimize(q, ch, steps=0)
        res = olp.lp_bound(net, ch.states, {}, q.lo, q.hi, {top: q.C[0]}, q.c0[0])
        out = ob.backsub(net, {top: q.C[:1]}, q.c0[:1], ch.states, res["params"], None, q.lo, q.hi)
        assert out["lb"][0] == pytest.approx(res["value"], abs=1e-8)
        S = {i: ch.states[i].S for i in net.relus}
        ex, _ = oen.exact_min(net, q.lo, q.hi, {top: q.C[0]}, q.c0[0], S=S)
        assert res["value"] <= ex + 1e-8


@pytest.mark.parametrize("seed", [1, 2])
def test_lp_duality_with_mnc(seed):
    net, q, root = _query(seed, mnc=True)
    top = len(net.nodes) - 1
    assert sum(m.e for m in q.mncs.values()) > 0
    res0 = olp.lp_bound(net, root.states, {}, q.lo, q.hi, {top: q.C[0]}, q.c0[0])
    res = olp.lp_bound(net, root.states, q.mncs, q.lo, q.hi, {top: q.C[0]}, q.c0[0])
    out = ob.backsub(net, {top: q.C[:1]}, q.c0[:1], root.states, res["params"], q.mncs, q.lo, q.hi)
    assert out["lb"][0] == pytest.approx(res["value"], abs=1e-8)
    ex, _ = oen.exact_min(net, q.lo, q.hi, {top: q.C[0]}, q.c0[0])
    assert res0["value"] - 1e-9 <= res["value"] <= ex + 1e-8


def test_mnc_constraints_hold_on_samples():
    net, q, root = _query(2, mnc=True)
    X = _samples(net, q.lo, q.hi, n=3000)
    vals = onet.forward_all(net, X)
    for i, m in q.mncs.items():
        zh, z = vals[net.nodes[i]["src"]], vals[i]
        viol = z @ m.P.T + zh @ m.Phat.T - m.p[None, :]
        assert viol.max() <= 1e-9


def test_mnc_over_plain_box_adds_nothing():
    # Over a box the exact hull is the product of triangles: every facet is single-neuron.
    lb = np.full(len(omnc.DIRS), -1e6)
    box_l, box_u = np.array([-1.0, -0.5, -2.0]), np.array([1.5, 0.7, 0.3])
    for t, s in enumerate(omnc.DIRS):
        # implied bound of s . zhat over the box: keeps Q equal to the box
        lb[t] = np.sum(np.where(s > 0, s * box_l, s * box_u))
    assert omnc.hull_facets(omnc.hull_points(lb)) == []


# --------------------------------------------------------------------------- completeness
def test_fully_split_leaf_reaches_exact_minimum():
    net, q, root = _query(4, widths=(2, 4, 3, 2), eps=0.3)
    top = len(net.nodes) - 1
    rng = np.random.default_rng(0)
    sub = root
    for m, i in enumerate(net.relus):
        st = sub.states[i]
        for j in np.nonzero((st.l < 0) & (st.u > 0))[0]:
            kids = obab.branch_split(net, sub, m, int(j))
            sub = kids[int(rng.integers(0, 2))]
    oo.bound_optimize(q, sub, steps=0)
    S = {i: sub.states[i].S for i in net.relus}
    for r in range(q.n_spec):
        ex, _ = oen.exact_min(net, q.lo, q.hi, {top: q.C[r]}, q.c0[r], S=S)
        res = olp.lp_bound(net, sub.states, {}, q.lo, q.hi, {top: q.C[r]}, q.c0[r])
        if np.isfinite(ex):
            assert res["value"] == pytest.approx(ex, abs=1e-7)
            out = ob.backsub(net, {top: q.C[r:r + 1]}, q.c0[r:r + 1], sub.states, res["params"],
                             None, q.lo, q.hi)
            assert out["lb"][0] == pytest.approx(ex, abs=1e-7)


# --------------------------------------------------------------------------- soundness invariants
@pytest.mark.parametrize("seed", range(3))
def test_soundness_invariants_through_optimisation_and_splits(seed):
    net, q, root = _query(seed, mnc=(seed == 2))
    X = _samples(net, q.lo, q.hi)
    fX = onet.forward(net, X) @ q.C.T + q.c0
    smin = fX.min(0)
    assert np.all(root.lb <= smin + 1e-9)
    heur = root.lb.copy()
    sub = root.clone()
    sub.recompute_from = 1
    oo.bound_optimize(q, sub, steps=20)
    assert np.all(sub.lb >= heur - 1e-12)
    assert np.all(sub.lb <= smin + 1e-9)
    assert np.all(sub.ub >= sub.lb - 1e-9)
    st = sub.states[net.relus[0]]
    js = np.nonzero((st.l < 0) & (st.u > 0))[0]
    if len(js):
        for ch in obab.branch_split(net, sub, 0, int(js[0])):
            oo.bound_optimize(q, ch, steps=10)
            assert np.all(ch.lb >= sub.lb - 1e-12)
            # the child's bound holds on the child's subdomain
            S = {i: ch.states[i].S for i in net.relus}
            top = len(net.nodes) - 1
            ex, _ = oen.exact_min(net, q.lo, q.hi, {top: q.C[0]}, q.c0[0], S=S)
            assert ch.lb[0] <= ex + 1e-8


def test_zero_gamma_leaves_bound_unchanged():
    net, q, root = _query(2, mnc=True)
    top = len(net.nodes) - 1
    params = {i: {"alpha": ob.heuristic_alpha(root.states[i]), "beta": np.zeros(net.sizes[i]),
                  "gamma": np.zeros(q.mncs[i].e)} for i in net.relus}
    a = ob.backsub(net, {top: q.C}, q.c0, root.states, params, q.mncs, q.lo, q.hi)["lb"]
    b = ob.backsub(net, {top: q.C}, q.c0, root.states, params, None, q.lo, q.hi)["lb"]
    np.testing.assert_array_equal(a, b)


def test_intermediate_bounds_sound_on_samples():
    net, q, root = _query(5, widths=(4, 8, 8, 6, 3), eps=0.3)
    X = _samples(net, q.lo, q.hi)
    vals = onet.forward_all(net, X)
    for i in net.relus:
        zh = vals[net.nodes[i]["src"]]
        assert np.all(zh.min(0) >= root.states[i].l - 1e-9)
        assert np.all(zh.max(0) <= root.states[i].u + 1e-9)


# --------------------------------------------------------------------------- gradient
@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_finite_differences(seed):
    net, q, root = _query(seed, mnc=True)
    top = len(net.nodes) - 1
    rng = np.random.default_rng(seed)
    st = root.states
    # make a split so beta has a gradient
    s0 = st[net.relus[0]]
    js = np.nonzero((s0.l < 0) & (s0.u > 0))[0]
    ch, _ = obab.branch_split(net, root, 0, int(js[-1]))
    params = {}
    for i in net.relus:
        params[i] = {"alpha": rng.uniform(0.05, 0.95, net.sizes[i]),
                     "beta": rng.uniform(0.0, 0.5, net.sizes[i]),
                     "gamma": rng.uniform(0.0, 0.2, q.mncs[i].e)}
    f = lambda: ob.backsub(net, {top: q.C}, q.c0, ch.states, params, q.mncs, q.lo, q.hi)
    out = f()
    g = oo.bound_grads(net, out, q.mncs)
    h = 1e-6
    for i in net.relus:
        ap = out["records"][i]["ap"]
        for name in ("alpha", "beta", "gamma"):
            vec = params[i][name]
            for j in range(min(len(vec), 12)):
                if name == "alpha" and np.min(np.abs(ap[:, j])) < 1e-4:
                    continue
                vec[j] += h; up = f()
                vec[j] -= 2 * h; dn = f()
                vec[j] += h
                # skip coordinates where the perturbation flips a sign of a' (a kink)
                if any(np.any(np.sign(up["records"][k]["ap"]) != np.sign(dn["records"][k]["ap"]))
                       for k in net.relus):
                    continue
                if np.any(np.sign(up["a0"]) != np.sign(dn["a0"])):
                    continue
                fd = (up["lb"].sum() - dn["lb"].sum()) / (2 * h)
                assert g[i][name][j] == pytest.approx(fd, rel=1e-5, abs=1e-6), (i, name, j)


# --------------------------------------------------------------------------- conv / residual
def test_conv_matches_library_and_adjoint_identity():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    for (ci, co, h, k, s, p) in [(1, 3, 7, 4, 2, 0), (2, 3, 6, 3, 1, 1), (3, 4, 8, 3, 2, 1),
                                 (2, 2, 5, 1, 2, 0), (2, 3, 8, 4, 2, 1)]:
        Wt = rng.normal(size=(co, ci, k, k))
        ho = (h + 2 * p - k) // s + 1
        z = rng.normal(size=(3, ci * h * h))
        mine = onet.conv_apply(Wt, z, (ci, h, h), (co, ho, ho), s, p)
        ref = torch.nn.functional.conv2d(torch.from_numpy(z.reshape(3, ci, h, h)),
                                         torch.from_numpy(Wt), stride=s, padding=p).numpy()
        np.testing.assert_allclose(mine, ref.reshape(3, -1), atol=1e-12)
        a = rng.normal(size=(3, co * ho * ho))
        lhs = np.einsum("rj,rj->r", a, mine)
        rhs = np.einsum("rj,rj->r", onet.conv_adjoint(Wt, a, (ci, h, h), (co, ho, ho), s, p), z)
        np.testing.assert_allclose(lhs, rhs, atol=1e-10)


def test_bn_and_avgpool_match_library_and_adjoint_identity():
    """Batch normalisation with fixed statistics against torch's batch_norm in evaluation mode, average
    pooling against avg_pool2d (zero padding counted), each with <a, A z> = <A^T a, z>."""
    torch = pytest.importorskip("torch")
    F = torch.nn.functional
    rng = np.random.default_rng(4)
    c, h = 3, 6
    bn = {"kind": "bn", "src": 0, "gamma": rng.uniform(0.5, 1.5, c), "beta": rng.normal(size=c),
          "mean": rng.normal(size=c), "var": rng.uniform(0.5, 2.0, c), "eps": 1e-5}
    for node in (bn, {"kind": "avgpool", "src": 0, "k": 2, "stride": 2, "pad": 0},
                 {"kind": "avgpool", "src": 0, "k": 3, "stride": 2, "pad": 1}):
        net = onet.Net([{"kind": "input", "shape": (c, h, h)}, node])
        z = rng.normal(size=(4, c * h * h))
        mine = onet.affine_apply(net, 1, z) + onet.bias_vector(net, 1)
        zt = torch.from_numpy(z.reshape(4, c, h, h))
        if node["kind"] == "bn":
            ref = F.batch_norm(zt, torch.from_numpy(bn["mean"]), torch.from_numpy(bn["var"]),
                               torch.from_numpy(bn["gamma"]), torch.from_numpy(bn["beta"]), training=False,
                               eps=bn["eps"])
        else:
            ref = F.avg_pool2d(zt, node["k"], node["stride"], node["pad"], count_include_pad=True)
        np.testing.assert_allclose(mine, ref.reshape(4, -1).numpy(), atol=1e-12)
        a = rng.normal(size=(4, net.sizes[1]))
        lhs = np.einsum("rj,rj->r", a, onet.affine_apply(net, 1, z))
        rhs = np.einsum("rj,rj->r", onet.affine_adjoint(net, 1, a), z)
        np.testing.assert_allclose(lhs, rhs, atol=1e-10)


@pytest.mark.parametrize("maker", ["tiny_conv", "tiny_resnet", "tiny_resnet_bn"])
def test_conv_and_residual_nets_lp_duality(maker):
    nodes = getattr(W, maker)(3)
    x0, lo, hi = W.make_input(nodes[0]["shape"], 0.15, 9)
    C, c0, _ = W.make_spec(nodes, x0)
    net = onet.Net(nodes)
    q = oo.Query(net, lo, hi, C, c0)
    root, _ = oo.root_pass(q)
    top = len(net.nodes) - 1
    res = olp.lp_bound(net, root.states, {}, lo, hi, {top: q.C[0]}, q.c0[0])
    out = ob.backsub(net, {top: q.C[:1]}, q.c0[:1], root.states, res["params"], None, lo, hi)
    assert out["lb"][0] == pytest.approx(res["value"], abs=1e-7)
    assert root.lb[0] <= res["value"] + 1e-9
    X = _samples(net, lo, hi, n=4000)
    assert res["value"] <= (onet.forward(net, X) @ q.C[0] + q.c0[0]).min() + 1e-9
    vals = onet.forward_all(net, X)
    for i in net.relus:
        zh = vals[net.nodes[i]["src"]]
        assert np.all(zh.min(0) >= root.states[i].l - 1e-9)
        assert np.all(zh.max(0) <= root.states[i].u + 1e-9)


# --------------------------------------------------------------------------- shapes / cost
def test_table3_activation_counts():
    g = json.load(open(os.path.join(GOLD, "table3_activation_counts.json")))
    count = lambda nodes: sum(int(np.prod(s)) for n, s in zip(nodes, W.node_shapes(nodes))
                              if n["kind"] == "relu")
    assert count(W.convsmall(0)) == g["mnist_convsmall"]
    assert count(W.convsmall(0, in_shape=(3, 32, 32))) == g["cifar_convsmall"]
    assert count(W.convbig(0)) == g["cifar_convbig"]
    assert count(W.resnet6(0)) == g["resnet6"]
    assert count(W.resnet8(0)) == g["resnet8"]


def test_appendix_b_split_cost():
    # layers: fc(3x4) relu(4, p=2) fc(4x2) relu(2) : c = [12, 6, 8, 2]
    layers = [{"kind": "fc", "d": 4, "nW": 12}, {"kind": "relu", "d": 4, "p": 2},
              {"kind": "fc", "d": 2, "nW": 8}, {"kind": "relu", "d": 2}]
    # split in layer 1: i = 2, 3 -> 2*2*(12+6) + 2*2*(12+6+8) = 72 + 104
    assert ocost.split_cost(layers, 1) == 176
    assert ocost.layer_costs([{"kind": "conv", "d": 10, "k": 3}]) == [90]


# --------------------------------------------------------------------------- planted mistakes
def test_planted_mistakes_are_caught(monkeypatch):
    """A dropped intercept or a flipped split sign in the oracle must break the LP pin."""
    net, q, root = _query(2)
    top = len(net.nodes) - 1
    res = olp.lp_bound(net, root.states, {}, q.lo, q.hi, {top: q.C[0]}, q.c0[0])
    good = ob.backsub(net, {top: q.C[:1]}, q.c0[:1], root.states, res["params"], None, q.lo, q.hi)
    assert good["lb"][0] == pytest.approx(res["value"], abs=1e-8)
    orig = ob.relu_backsub

    def no_intercept(a, st, alpha, beta, mnc=None, gamma=None):
        ahat, dc, rec = orig(a, st, alpha, beta, mnc, gamma)
        return ahat, dc * 0.0, rec

    monkeypatch.setattr(ob, "relu_backsub", no_intercept)
    bad = ob.backsub(net, {top: q.C[:1]}, q.c0[:1], root.states, res["params"], None, q.lo, q.hi)
    assert abs(bad["lb"][0] - res["value"]) > 1e-6


# --------------------------------------------------------------------------- branching scores (Section 3.4)
def _acs_case(gamma, S=(0, 0, 0), l=(-1.0, -1.0, -1.0), u=(1.0, 1.0, 1.0)):
    from types import SimpleNamespace as NS
    net = NS(relus=[2], sizes={2: 3})
    m = ob.Mnc(P=[[1.0, -2.0, 0.0], [0.0, 1.0, 0.0]], Phat=[[0.0, 3.0, 0.0], [0.5, 0.0, 0.0]], p=[0.0, 0.0])
    sub = NS(states={2: ob.ReluState(l, u, S)}, sets={"final": {2: {"gamma": np.asarray(gamma, float)}}})
    return net, sub, {2: m}


def test_acs_worked_example():
    from oracle import branching as obr
    # gamma = (0.5, 2): gamma^T P = (0.5, -1 + 2, 0) = (0.5, 1, 0); gamma^T Phat = (1, 1.5, 0)
    net, sub, mncs = _acs_case([0.5, 2.0])
    s = obr.acs_scores(net, sub, mncs)[2]
    assert np.allclose(s, [1.5, 2.5, 0.0], rtol=0, atol=1e-15)
    assert obr.select(net, {2: s}) == (0, 1)
    # a split neuron and a stable one are no candidates
    net, sub, mncs = _acs_case([0.5, 2.0], S=(0, 1, 0), l=(-1.0, -1.0, 0.5))
    s = obr.acs_scores(net, sub, mncs)[2]
    assert s[0] == 1.5 and np.isneginf(s[1]) and np.isneginf(s[2])
    assert obr.select(net, {2: s}) == (0, 0)


def test_acs_invariants():
    from oracle import branching as obr
    # gamma = 0 scores every candidate 0 (the lowest index is chosen); positive scaling of gamma
    # scales every score; the sign of gamma does not matter (absolute values)
    net, sub, mncs = _acs_case([0.0, 0.0])
    s0 = obr.acs_scores(net, sub, mncs)[2]
    assert np.all(s0 == 0.0) and obr.select(net, {2: s0}) == (0, 0)
    base = obr.acs_scores(*_acs_case([0.3, 0.7]))[2]
    assert np.allclose(obr.acs_scores(*_acs_case([0.9, 2.1]))[2], 3.0 * base, rtol=1e-14, atol=0)
    assert np.allclose(obr.acs_scores(*_acs_case([-0.3, -0.7]))[2], base, rtol=1e-14, atol=0)
    # no candidate at all
    net, sub, mncs = _acs_case([1.0, 1.0], l=(0.1, 0.2, 0.3))
    assert obr.select(net, obr.acs_scores(net, sub, mncs)) == (-1, -1)


def test_cab_changes_the_choice_with_cost():
    from types import SimpleNamespace as NS
    from oracle import branching as obr
    net = NS(relus=[2, 4])
    scores = {2: np.array([2.0, -np.inf]), 4: np.array([1.5, 0.5])}
    assert obr.select(net, scores) == (0, 0)
    # 2.0 / 100 = 0.02 < 1.5 / 10 = 0.15
    assert obr.select(net, obr.cab_scores(scores, {2: 100.0, 4: 10.0})) == (1, 0)


# --------------------------------------------------------------------------- Adam (Section 3.1 optimiser)
def test_adam_matches_torch_optim_adam():
    """The oracle's Adam ascent equals torch.optim.Adam(maximize=True) (bias-corrected, eps outside
    the square root) on a fixed gradient sequence, in float64, for several hyper-parameters."""
    import torch
    rng = np.random.default_rng(7)
    for lr, b1, b2, eps in ((0.1, 0.9, 0.999, 1e-8), (0.03, 0.5, 0.9, 1e-3), (1.0, 0.0, 0.99, 1e-6)):
        p0 = {"a": rng.normal(size=5), "b": rng.normal(size=(2, 3))}
        grads = [{k: rng.normal(size=v.shape) * 10.0 ** rng.integers(-3, 3) for k, v in p0.items()}
                 for _ in range(12)]
        params = {k: v.copy() for k, v in p0.items()}
        opt = oo.Adam(lr, b1, b2, eps)
        tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p0.items()}
        topt = torch.optim.Adam(list(tp.values()), lr=lr, betas=(b1, b2), eps=eps, maximize=True)
        for g in grads:
            opt.step(params, g)
            topt.zero_grad()
            for k, t in tp.items():
                t.grad = torch.tensor(g[k], dtype=torch.float64)
            topt.step()
            for k in p0:
                np.testing.assert_allclose(params[k], tp[k].detach().numpy(), rtol=0, atol=1e-12)


def test_adam_first_step_hand_computed():
    """After one step the bias-corrected moments are g and g^2, so the ascent is lr * g / (|g| + eps)."""
    g = np.array([2.0, -0.5, 0.0])
    p = {"x": np.array([1.0, 1.0, 1.0])}
    oo.Adam(lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8).step(p, {"x": g})
    np.testing.assert_allclose(p["x"], [1.0 + 0.1 * 2.0 / (2.0 + 1e-8), 1.0 - 0.1 * 0.5 / (0.5 + 1e-8), 1.0],
                               rtol=0, atol=1e-15)


# --------------------------------------------------------------------------- alpha-contribution branching score
def _score_net():
    """input 2 -> fc 3 -> relu -> fc 2 -> relu -> fc 1, weights chosen so every a' is hand-computable."""
    W1 = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    W2 = np.array([[4.0, 1.0, 10.0], [0.0, 0.0, 0.0]])
    W3 = np.array([[2.0, -4.0]])
    nodes = [{"kind": "input", "shape": (2, 1, 1)},
             {"kind": "fc", "src": 0, "W": W1, "b": np.zeros(3)}, {"kind": "relu", "src": 1},
             {"kind": "fc", "src": 2, "W": W2, "b": np.zeros(2)}, {"kind": "relu", "src": 3},
             {"kind": "fc", "src": 4, "W": W3, "b": np.zeros(1)}]
    net = onet.Net(nodes)
    # ReLU layer 0: all unstable, triangle heights -u l / (u - l) = 0.5, 0.5, 1; neuron 2 split positive
    s0 = ob.ReluState([-1.0, -1.0, 0.0], [1.0, 1.0, 2.0], S=[0, 0, -1])
    # ReLU layer 1: heights 3/4 and 1/2
    s1 = ob.ReluState([-1.0, -1.0], [3.0, 1.0])
    states = {2: s0, 4: s1}
    params = {2: {"alpha": np.full(3, 0.5), "beta": np.zeros(3)}, 4: {"alpha": np.full(2, 0.5), "beta": np.zeros(2)}}
    return net, states, params


def test_branching_score_hand_worked():
    """One spec row C = [1]: a' on ReLU layer 1 is W3 = [2, -4] (scores 2 * 3/4, 4 * 1/2); the row
    crosses it with D = (alpha, chord) = (0.5, 0.5), so a' on ReLU layer 0 is [1, -2] W2 = [4, 1, 10]
    (scores 4 * 0.5, 1 * 0.5, and none for the split neuron whose unsplit score would be 10).  The
    two maxima 2.0 tie between (layer 0, neuron 0) and (layer 1, neuron 1): the lowest layer wins."""
    net, states, params = _score_net()
    sub = oo.Subproblem(states, {}, None, None, recompute_from=2)
    out = ob.backsub(net, ob.spec_start(net, [[1.0]]), [0.0], states, params)
    np.testing.assert_allclose(out["records"][4]["ap"], [[2.0, -4.0]], atol=0)
    np.testing.assert_allclose(out["records"][2]["ap"], [[4.0, 1.0, 10.0]], atol=0)
    sc = obab.branching_score(net, sub, out["records"])
    np.testing.assert_allclose(sc[0], [2.0, 0.5, -np.inf], atol=0)
    np.testing.assert_allclose(sc[1], [1.5, 2.0], atol=0)
    assert obab.pick_branch(sc) == (0, 0)
    # a stable neuron is not a candidate: with l_0 >= 0 in layer 0 the other maximum is chosen
    states[2] = ob.ReluState([0.0, -1.0, 0.0], [1.0, 1.0, 2.0], S=[0, 0, -1])
    out = ob.backsub(net, ob.spec_start(net, [[1.0]]), [0.0], states, params)
    sc = obab.branching_score(net, oo.Subproblem(states, {}, None, None, 2), out["records"])
    assert sc[0][0] == -np.inf and obab.pick_branch(sc) == (1, 1)


def test_branching_score_sums_spec_rows():
    """Two spec rows C = [1], [-1]: the second row has a' = [-2, 4] on ReLU layer 1, crosses it with
    D = (chord 3/4, alpha 0.5), giving a' = [-1.5, 2] W2 = [-6, -1.5, -15] on layer 0.  Scores are
    sums of |a'| over the rows times the height: layer 0 (4+6)/2, (1+1.5)/2; layer 1 (2+2)*3/4, (4+4)/2."""
    net, states, params = _score_net()
    out = ob.backsub(net, ob.spec_start(net, [[1.0], [-1.0]]), [0.0, 0.0], states, params)
    np.testing.assert_allclose(out["records"][2]["ap"][1], [-6.0, -1.5, -15.0], atol=0)
    sc = obab.branching_score(net, oo.Subproblem(states, {}, None, None, 2), out["records"])
    np.testing.assert_allclose(sc[0], [5.0, 1.25, -np.inf], atol=0)
    np.testing.assert_allclose(sc[1], [3.0, 4.0], atol=0)
    assert obab.pick_branch(sc) == (0, 0)
    # nothing eligible: every neuron stable or split
    st = {2: ob.ReluState([0.0, 0.0, 0.0], [1.0, 1.0, 2.0]), 4: ob.ReluState([1.0, -2.0], [3.0, -1.0])}
    out = ob.backsub(net, ob.spec_start(net, [[1.0]]), [0.0], st, params)
    assert obab.pick_branch(obab.branching_score(net, oo.Subproblem(st, {}, None, None, 2), out["records"])) is None
