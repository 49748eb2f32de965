"""GPU path vs the FP64 oracle, element by element, through the C ABI (needs an MI355X)."""
import copy

import numpy as np
import pytest

import workloads as W
from oracle import backsub as ob
from oracle import bab as obab
from oracle import net as onet
from oracle import optimize as oo

from _common import (assert_parity, make_batch, make_subproblems, oracle_query, oracle_subproblem, root_unstable,
                     sampled_min, sampled_min_sub)

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


# --------------------------------------------------------------------------- kernels
def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


CONV_GEOMS = [  # (Ci, H, Co, k, s, p)
    (1, 28, 16, 4, 2, 0), (16, 13, 32, 4, 2, 0),          # ConvSmall
    (3, 32, 32, 3, 1, 1), (32, 32, 32, 4, 2, 1), (32, 16, 64, 3, 1, 1), (64, 16, 64, 4, 2, 1),  # ConvBig
    (16, 16, 32, 3, 2, 1), (32, 8, 32, 3, 1, 1), (16, 16, 32, 1, 2, 0), (3, 32, 16, 3, 2, 1),   # ResNet6
    (5, 7, 17, 3, 2, 1), (20, 9, 24, 4, 2, 1), (18, 6, 40, 2, 1, 0),                        # ragged
    # first layers of receptive-field windows (padding 0) and forward cones (padding 2)
    (3, 16, 32, 3, 1, 0), (3, 16, 32, 3, 1, 2), (3, 10, 32, 3, 1, 2), (3, 6, 32, 3, 1, 0),
    (1, 12, 8, 3, 1, 1), (4, 7, 24, 3, 1, 1), (2, 40, 8, 3, 1, 1),
    # channel counts that leave a partial last stage (direct-staged and register-staged tiles)
    (3, 16, 6, 3, 1, 1), (2, 20, 10, 3, 1, 0),
    # planes so small that a workgroup's windows need more staging passes than the direct form holds
    (2, 4, 8, 3, 1, 1), (1, 3, 4, 3, 1, 1),
    # forward cones of ConvBig's second and third convolutions (padding 2)
    (32, 18, 32, 4, 2, 2), (32, 10, 64, 3, 1, 2),
]


@pytest.mark.parametrize("geom", CONV_GEOMS)
def test_conv_kernels_match_oracle(geom):
    P = _P()
    ci, h, co, k, s, p = geom
    rng = np.random.default_rng(hash(geom) % 2**32)
    nodes = [{"kind": "input", "shape": (ci, h, h)},
             {"kind": "conv", "src": 0, "W": rng.normal(size=(co, ci, k, k)).astype(np.float32),
              "b": rng.normal(size=co).astype(np.float32), "stride": s, "pad": p},
             {"kind": "relu", "src": 1},
             {"kind": "fc", "src": 2, "W": np.ones((2, co * ((h + 2 * p - k) // s + 1) ** 2), np.float32),
              "b": np.zeros(2, np.float32)}]
    net = P.Net(nodes)
    onet_ = onet.Net(nodes)
    din, dout = onet_.sizes[0], onet_.sizes[1]
    for M in (1, 37, 300):
        A = rng.normal(size=(M, dout)).astype(np.float32)
        ref = onet.conv_adjoint(onet_.nodes[1]["W"], A.astype(np.float64), onet_.shapes[0], onet_.shapes[1], s, p)
        a_d, c_d = _dev(A), torch.full((M, din), 7.0, device="cuda")
        torch.cuda.synchronize()
        net.conv_backsub(1, a_d.data_ptr(), c_d.data_ptr(), M)
        net.sync()
        out = c_d.cpu().numpy()
        np.testing.assert_allclose(out, ref, rtol=0, atol=1e-5 * np.abs(ref).max() + 1e-5)
        # accumulate mode
        net.conv_backsub(1, a_d.data_ptr(), c_d.data_ptr(), M, accumulate=True)
        net.sync()
        np.testing.assert_allclose(c_d.cpu().numpy(), 2 * ref, rtol=0, atol=2e-5 * np.abs(ref).max() + 2e-5)
        G = rng.normal(size=(M, din)).astype(np.float32)
        reff = onet.conv_apply(onet_.nodes[1]["W"], G.astype(np.float64), onet_.shapes[0], onet_.shapes[1], s, p) \
            + onet.bias_vector(onet_, 1)
        g_d, o_d = _dev(G), torch.zeros((M, dout), device="cuda")
        torch.cuda.synchronize()
        net.conv_forward(1, g_d.data_ptr(), o_d.data_ptr(), M)
        net.sync()
        np.testing.assert_allclose(o_d.cpu().numpy(), reff, rtol=0, atol=1e-5 * np.abs(reff).max() + 1e-5)


WIN_GEOMS = [  # (Ci, H, Co, k, s, p): input-window kernels, whole tiles and ragged ones
    (32, 32, 32, 4, 2, 1), (32, 16, 64, 3, 1, 1), (64, 16, 64, 4, 2, 1),     # ConvBig, float4 staging
    (32, 18, 32, 4, 2, 2), (32, 16, 32, 4, 2, 2), (32, 10, 64, 3, 1, 2),    # its forward cones
    (16, 13, 32, 4, 2, 0), (8, 20, 96, 3, 1, 1), (8, 24, 128, 3, 1, 0),      # ragged tiles, channel tiles
    (16, 12, 32, 4, 2, 3), (16, 16, 32, 3, 2, 1), (16, 14, 32, 3, 1, 1),      # rows of 2 mod 4 floats
    (64, 32, 32, 4, 2, 1), (32, 40, 64, 4, 2, 1), (32, 16, 32, 3, 1, 1),     # transposed: 2x2 and 3x3 phases
    (32, 6, 64, 3, 1, 1), (32, 6, 96, 3, 1, 1), (32, 5, 96, 3, 1, 1),        # transposed: 3x3 grids of 36, 25
    (32, 4, 96, 3, 1, 1),                                                     # and 16 positions into 32 channels
]


@pytest.mark.parametrize("geom", WIN_GEOMS)
def test_window_conv_matches_oracle(geom):
    """Forward and transposed convolutions through the input-window kernels (the default where they
    apply) against the FP64 convolution and its adjoint (the transposed one also accumulating),
    bitwise the same for a row alone and inside a batch (the lone row also sits at an address that
    is not 16-byte aligned for most shapes, so it is staged element by element), and equal to FP32
    rounding to the gather GEMMs (MNB_VAR_NO_WIN_CONV)."""
    P = _P()
    ci, h, co, k, s, p = geom
    rng = np.random.default_rng(hash(geom) % 2**32)
    ho = (h + 2 * p - k) // s + 1
    nodes = [{"kind": "input", "shape": (ci, h, h)},
             {"kind": "conv", "src": 0, "W": rng.normal(size=(co, ci, k, k)).astype(np.float32),
              "b": rng.normal(size=co).astype(np.float32), "stride": s, "pad": p},
             {"kind": "relu", "src": 1},
             {"kind": "fc", "src": 2, "W": np.ones((2, co * ho * ho), np.float32), "b": np.zeros(2, np.float32)}]
    prev = P.get_kernel_variants()
    try:
        P.set_kernel_variants(prev & ~P.VARIANTS["no_win_conv"])
        net = P.Net(nodes)
        onet_ = onet.Net(nodes)
        din, dout = onet_.sizes[0], onet_.sizes[1]
        M = 203
        G = rng.normal(size=(M, din)).astype(np.float32)
        ref = onet.conv_apply(onet_.nodes[1]["W"], G.astype(np.float64), onet_.shapes[0], onet_.shapes[1], s, p) \
            + onet.bias_vector(onet_, 1)
        A = rng.normal(size=(M, dout)).astype(np.float32)
        refb = onet.conv_adjoint(onet_.nodes[1]["W"], A.astype(np.float64), onet_.shapes[0], onet_.shapes[1], s, p)
        g_d, o_d = _dev(G), torch.zeros((M, dout), device="cuda")
        a_d, c_d = _dev(A), torch.full((M, din), 7.0, device="cuda")
        torch.cuda.synchronize()
        net.conv_forward(1, g_d.data_ptr(), o_d.data_ptr(), M)
        net.conv_backsub(1, a_d.data_ptr(), c_d.data_ptr(), M)
        net.sync()
        out, outb = o_d.cpu().numpy(), c_d.cpu().numpy()
        tol, tolb = 1e-5 * np.abs(ref).max() + 1e-5, 1e-5 * np.abs(refb).max() + 1e-5
        np.testing.assert_allclose(out, ref, rtol=0, atol=tol)
        np.testing.assert_allclose(outb, refb, rtol=0, atol=tolb)
        net.conv_backsub(1, a_d.data_ptr(), c_d.data_ptr(), M, accumulate=True)
        net.sync()
        np.testing.assert_allclose(c_d.cpu().numpy(), 2 * refb, rtol=0, atol=2 * tolb)
        one, oneb = torch.zeros((1, dout), device="cuda"), torch.zeros((1, din), device="cuda")
        net.conv_forward(1, g_d[117:118].data_ptr(), one.data_ptr(), 1)
        net.conv_backsub(1, a_d[117:118].data_ptr(), oneb.data_ptr(), 1)
        net.sync()
        assert np.array_equal(one.cpu().numpy()[0], out[117])
        assert np.array_equal(oneb.cpu().numpy()[0], outb[117])
        P.set_kernel_variants(prev | P.VARIANTS["no_win_conv"])
        o2, c2 = torch.zeros((M, dout), device="cuda"), torch.zeros((M, din), device="cuda")
        net.conv_forward(1, g_d.data_ptr(), o2.data_ptr(), M)
        net.conv_backsub(1, a_d.data_ptr(), c2.data_ptr(), M)
        net.sync()
        np.testing.assert_allclose(o2.cpu().numpy(), out, rtol=0, atol=tol)
        np.testing.assert_allclose(c2.cpu().numpy(), outb, rtol=0, atol=tolb)
    finally:
        P.set_kernel_variants(prev)


@pytest.mark.parametrize("dims", [(1, 10, 100), (37, 100, 784), (576, 100, 100), (300, 512, 4096), (129, 33, 65),
                                  (64, 7, 3)])
def test_fc_kernels_match_numpy(dims):
    P = _P()
    M, dout, din = dims
    rng = np.random.default_rng(M * 7 + dout)
    W = rng.normal(size=(dout, din)).astype(np.float32)
    b = rng.normal(size=dout).astype(np.float32)
    nodes = [{"kind": "input", "shape": (din, 1, 1)}, {"kind": "fc", "src": 0, "W": W, "b": b},
             {"kind": "relu", "src": 1}, {"kind": "fc", "src": 2, "W": np.ones((1, dout), np.float32),
                                          "b": np.zeros(1, np.float32)}]
    net = P.Net(nodes)
    A = rng.normal(size=(M, dout)).astype(np.float32)
    ref = A.astype(np.float64) @ W.astype(np.float64)
    a_d, c_d = _dev(A), torch.zeros((M, din), device="cuda")
    torch.cuda.synchronize()
    net.fc_backsub(1, a_d.data_ptr(), c_d.data_ptr(), M)
    net.sync()
    np.testing.assert_allclose(c_d.cpu().numpy(), ref, rtol=0, atol=2e-5 * np.abs(ref).max() + 1e-5)
    G = rng.normal(size=(M, din)).astype(np.float32)
    reff = G.astype(np.float64) @ W.astype(np.float64).T + b
    g_d, o_d = _dev(G), torch.zeros((M, dout), device="cuda")
    torch.cuda.synchronize()
    net.fc_forward(1, g_d.data_ptr(), o_d.data_ptr(), M)
    net.sync()
    np.testing.assert_allclose(o_d.cpu().numpy(), reff, rtol=0, atol=2e-5 * np.abs(reff).max() + 1e-5)


# --------------------------------------------------------------------------- root pass
ROOT_CASES = [(1, "small"), (2, "small"), (3, "small"), (4, "small"), (1, "full"), (2, "full")]


@pytest.mark.parametrize("cfg,scale", ROOT_CASES)
def test_bound_init_matches_oracle(cfg, scale):
    P = _P()
    wl = W.make_workload(cfg, scale=scale)
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=8)
    rid, lb, ub = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    print(f"cfg{cfg}/{scale}: gpu lb {lb[:3]} oracle {root.lb[:3]}", flush=True)
    assert_parity(lb, root.lb, "root lb")
    assert np.all(lb <= sampled_min(net_o, wl) + 1e-6)
    assert np.all(ub >= lb)
    for m, i in enumerate(net_o.relus):
        l, u, S = pb.get_bounds(rid, m)
        st = root.states[i]
        # compare where both sides agree on the stability class decided by the interval pass
        assert_parity(l, st.l, f"layer {m} l")
        assert_parity(u, st.u, f"layer {m} u")


# --------------------------------------------------------------------------- splits, T = 0 (config 1)
@pytest.mark.parametrize("scale,n_sub", [("small", 16), ("full", 64)])
def test_config1_splits_T0(scale, n_sub):
    P = _P()
    wl = W.make_workload(1, scale=scale)
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=4 * n_sub + 8)
    rid, lb0, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    splits = W.make_split_sets(root_unstable(net_o, root), n_sub, 1, 4, seed=3001)
    ids, subs = make_subproblems(P, pb, rid, net_o, q, root, splits)
    lb, ub = pb.bound_optimize(ids, steps=0)
    ref = np.array([oo.bound_optimize(q, s, steps=0).lb for s in subs])
    assert_parity(lb, ref, "T=0 lb")
    assert np.all(lb >= lb0[None, :] - 1e-6)
    for b in range(len(ids)):
        for m, i in enumerate(net_o.relus):
            l, u, _ = pb.get_bounds(ids[b], m)
            assert_parity(l, subs[b].states[i].l, f"sub {b} layer {m} l")
            assert_parity(u, subs[b].states[i].u, f"sub {b} layer {m} u")


# --------------------------------------------------------------------------- gradient
@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_gradient_matches_oracle(cfg):
    P = _P()
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    unst = root_unstable(net_o, root)
    m0 = 0
    j0 = int(unst[0][0])
    gid = int(pb.branch_split([rid], [m0], [j0])[0])
    osub = obab.branch_split(net_o, root, m0, j0)[0]
    # random feasible parameters on both sides
    rng = np.random.default_rng(cfg)
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    for key in oo.set_keys(net_o):
        si = P.set_index(key)
        alpha = rng.uniform(0, 1, offs[-1]).astype(np.float32)
        beta = rng.uniform(0, 0.5, offs[-1]).astype(np.float32)
        pb.set_params(gid, si, alpha=alpha, beta=beta)
        for t, i in enumerate(net_o.relus):
            if i in osub.sets[key]:
                osub.sets[key][i]["alpha"] = alpha[offs[t]:offs[t + 1]].astype(np.float64)
                osub.sets[key][i]["beta"] = beta[offs[t]:offs[t + 1]].astype(np.float64)
    # recompute intermediate bounds with these parameters (T = 0) on both sides, then compare gradients
    pb.bound_optimize([gid], steps=0)
    oo.bound_optimize(q, osub, steps=0)
    for key in oo.set_keys(net_o):
        si = P.set_index(key)
        lbr, ga, gb, _ = pb.bound_grad(gid, si)
        if key == "final":
            start, c0 = ob.spec_start(net_o, q.C), q.c0
        else:
            m, s = key
            i = net_o.relus[m]
            st = osub.states[i]
            js = np.nonzero((st.l < 0) & (st.u > 0))[0]
            if len(js) == 0:
                assert len(lbr) == 0
                continue
            start, c0 = ob.neuron_start(net_o, i, js, s), np.zeros(len(js))
        out = ob.backsub(net_o, start, c0, osub.states, osub.sets[key], None, q.lo, q.hi)
        assert_parity(lbr, out["lb"], f"{key} rows")
        g = oo.bound_grads(net_o, out)
        ref_a = np.concatenate([g[i]["alpha"] if i in g else np.zeros(net_o.sizes[i]) for i in net_o.relus])
        ref_b = np.concatenate([g[i]["beta"] if i in g else np.zeros(net_o.sizes[i]) for i in net_o.relus])
        for name, gg, rr in (("alpha", ga, ref_a), ("beta", gb, ref_b)):
            nrm = np.linalg.norm(rr)
            assert np.linalg.norm(gg - rr) <= 1e-3 * max(nrm, 1e-6), (key, name, np.linalg.norm(gg - rr), nrm)


# --------------------------------------------------------------------------- optimisation
@pytest.mark.parametrize("cfg,n_sub,steps", [(1, 8, 5), (2, 6, 5), (4, 4, 3)])
def test_optimize_matches_oracle(cfg, n_sub, steps):
    P = _P()
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=4 * n_sub + 8)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    splits = W.make_split_sets(root_unstable(net_o, root), n_sub, 1, 3, seed=77 + cfg)
    ids, subs = make_subproblems(P, pb, rid, net_o, q, root, splits)
    lb, ub = pb.bound_optimize(ids, steps=steps, lr=0.1)
    ref = np.array([oo.bound_optimize(q, s, steps=steps, lr=0.1).lb for s in subs])
    print("gpu", lb[:2], "oracle", ref[:2], flush=True)
    assert_parity(lb, ref, f"T={steps} lb")
    # soundness on each subdomain; ub = f(x*) is a value of the spec at a point of the box
    for b, s in enumerate(subs):
        smin = sampled_min_sub(net_o, wl, {i: s.states[i].S for i in net_o.relus})
        assert np.all(lb[b] <= smin + 1e-6)
    # ub = spec at the best iterate's x*; x* may differ where a coefficient of a^(0) is ~0
    ref_ub = np.array([s.ub for s in subs])
    close = np.abs(ub - ref_ub) <= 1e-3 * np.maximum(1.0, np.abs(ref_ub))
    assert close.mean() >= 0.9, close.mean()


@pytest.mark.parametrize("cfg", [1, 2, 4])
def test_teacher_forced_20_steps_match_oracle(cfg):
    """Fixed-parameter parity along a whole 20-step optimisation: the oracle evaluates the GPU's own
    parameter iterates (read back after bound_optimize with steps = t, t = 0..20, each on a fresh
    copy of the subproblem; the trajectory is deterministic, so these are the iterates of one
    20-step run), with its own intersection of the recomputed intermediate bounds.  Every step
    is then compared at identical parameters, free of Adam's sensitivity to rounding order."""
    P = _P()
    T = 20
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=4 * (T + 1) + 8)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    split = W.make_split_sets(root_unstable(net_o, root), 1, 1, 3, seed=500 + cfg)[0]
    ids = make_batch(pb, rid, [split] * (T + 1))
    osub = oracle_subproblem(net_o, root, split)
    layers = oo.recompute_layers(net_o, osub)
    keys = ["final"] + [(m, s) for m in layers for s in (1, -1)]
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    teacher, lbs = [], []
    for t in range(T + 1):
        lb, _ = pb.bound_optimize([ids[t]], steps=t, lr=0.1)
        lbs.append(lb[0])
        sets = {}
        for k in keys:
            a, b, _ = pb.get_params(ids[t], P.set_index(k))
            sk = copy.deepcopy(osub.sets[k])
            for n, i in enumerate(net_o.relus):
                if i in sk:
                    sk[i]["alpha"] = a[offs[n]:offs[n + 1]].astype(np.float64)
                    sk[i]["beta"] = b[offs[n]:offs[n + 1]].astype(np.float64)
            sets[k] = sk
        teacher.append(sets)
    lb0 = osub.lb.copy()
    trace = []
    oo.bound_optimize(q, osub, steps=T, lr=0.1, trace=trace, teacher=teacher)
    best = np.full(q.n_spec, -np.inf)
    for t in range(T + 1):
        best = np.maximum(best, trace[t]["lb"])
        assert_parity(lbs[t], np.maximum(best, lb0), f"cfg{cfg} after {t} steps")
    for m in layers:
        i = net_o.relus[m]
        l, u, _ = pb.get_bounds(ids[T], m)
        assert_parity(l, trace[T]["l"][i], f"cfg{cfg} layer {m} l after {T} steps")
        assert_parity(u, trace[T]["u"][i], f"cfg{cfg} layer {m} u after {T} steps")
    print(f"cfg{cfg}: split {split}, lb after 0 / {T} steps {lbs[0].min():.5f} / {lbs[T].min():.5f}", flush=True)
    # free-running: the oracle's own 20-step trajectory (these seeds cross no kink of the
    # relaxation, where the two trajectories could part legitimately)
    free = oo.bound_optimize(q, oracle_subproblem(net_o, root, split), steps=T, lr=0.1).lb
    assert_parity(lbs[T], free, f"cfg{cfg} free-running {T} steps")


# --------------------------------------------------------------------------- checkpointed adjoint
@pytest.mark.parametrize("cfg,stride", [(1, 2), (2, 2), (4, 2), (4, 3)])
def test_checkpointed_adjoint_is_bitwise_identical(cfg, stride):
    """Layer-wise recomputation from checkpoints gives exactly the stored-a' result."""
    P = _P()
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    splits = W.make_split_sets(root_unstable(net_o, root), 6, 1, 3, seed=11)
    out = []
    for st in (1, stride):
        net = P.Net(wl.nodes)
        pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=64)
        rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
        ids, _ = make_subproblems(P, pb, rid, net_o, q, root, splits)
        lb, ub = pb.bound_optimize(ids, steps=4, ckpt_stride=st)
        alphas = np.stack([pb.get_params(i, 0)[0] for i in ids])
        out.append((lb, ub, alphas))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])


def test_chunked_passes_are_bitwise_identical():
    """A memory budget that splits passes into chunks does not change any result."""
    P = _P()
    wl = W.make_workload(2, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    splits = W.make_split_sets(root_unstable(net_o, root), 12, 1, 4, seed=12)
    out = []
    for budget in (0, 2 << 20):
        net = P.Net(wl.nodes)
        pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=128)
        rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
        ids, _ = make_subproblems(P, pb, rid, net_o, q, root, splits)
        out.append(pb.bound_optimize(ids, steps=3, mem_budget=budget))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_batch_composition_does_not_change_results():
    """A subproblem bounded alone or inside a larger, permuted batch gives bitwise the same bound."""
    P = _P()
    wl = W.make_workload(4, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    splits = W.make_split_sets(root_unstable(net_o, root), 8, 1, 3, seed=13)
    net = P.Net(wl.nodes)
    res = {}
    for mode in ("alone", "batch"):
        pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=128)
        rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
        ids, _ = make_subproblems(P, pb, rid, net_o, q, root, splits)
        if mode == "alone":
            res[mode] = np.stack([pb.bound_optimize([i], steps=3)[0][0] for i in ids])
        else:
            perm = np.random.default_rng(0).permutation(len(ids))
            lb, _ = pb.bound_optimize(ids[perm], steps=3)
            back = np.empty_like(lb)
            back[perm] = lb
            res[mode] = back
    np.testing.assert_array_equal(res["alone"], res["batch"])


@pytest.mark.parametrize("cfg", [2, 4])
def test_optimize_session_equals_one_shot(cfg):
    """bound_optimize_begin + T steps + end gives bound_optimize's results bit for bit, also with other
    calls on the same problem between the steps (another query's bound_init, splits and a one-shot
    optimisation of other subproblems)."""
    import paper_2205_00263_amd as P
    from _common import make_batch
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=128)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    splits = W.make_split_sets(root_unstable(net_o, root), 8, 1, 4, seed=91 + cfg)
    a = make_batch(pb, rid, splits)
    b = make_batch(pb, rid, splits)
    c = make_batch(pb, rid, splits)
    lb1, ub1, bl1, bn1 = pb.bound_optimize(a, steps=5, lr=0.1, want_branch=True)
    s = pb.optimize_begin(b, steps=5, lr=0.1)
    for t in range(5):
        s.step()
        if t == 2:   # unrelated work on the same problem between two steps
            wl2 = W.make_workload(cfg, scale="small", seed_offset=1)
            rid2, _, _ = pb.bound_init(wl2.lo, wl2.hi, wl2.C, wl2.c0)
            pb.bound_optimize(c[:3], steps=2)
            pb.release([rid2])
    lb2, ub2, bl2, bn2 = s.end(want_branch=True)
    assert np.array_equal(lb1, lb2) and np.array_equal(ub1, ub2)
    assert np.array_equal(bl1, bl2) and np.array_equal(bn1, bn2)
    for sid1, sid2 in zip(a, b):
        for m in range(net.n_relu):
            l1, u1, _ = pb.get_bounds(int(sid1), m)
            l2, u2, _ = pb.get_bounds(int(sid2), m)
            assert np.array_equal(l1, l2) and np.array_equal(u1, u2)
        for si in range(2 * net.n_relu - 1):
            p1, p2 = pb.get_params(int(sid1), si), pb.get_params(int(sid2), si)
            assert all(np.array_equal(x, y) for x, y in zip(p1, p2))
