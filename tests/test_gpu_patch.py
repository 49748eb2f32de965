"""Receptive-field rows (needs an MI355X).

An intermediate-bound row +-e_j on a convolution's output is nonzero below only inside the
window neuron j sees; the library keeps such rows as that window (set bit MNB_VAR_NO_PATCH of
mnb_set_kernel_variants to keep whole layers).  Checked here against the FP64 oracle (which
always back-substitutes whole layers) and against the whole-layer path on a ConvBig-shaped net
whose windows are much smaller than its layers, with and without multi-neuron constraints, and
on the full ConvBig batch of the benchmark."""
import numpy as np
import pytest

import workloads as W
from oracle import optimize as oo

from _common import assert_parity, make_batch, oracle_query, oracle_subproblem, root_unstable

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NO_FUSED, NO_PATCH, NO_CONE = 32, 64, 128


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00263_amd as P
    P.lib()
    prev = P.get_kernel_variants()
    yield
    P.set_kernel_variants(prev)


def _medium(eps=0.03):
    """ConvBig topology on a 3x24x24 input with 4-8 channels: the windows of ReLU layers 1-3 on
    the first layer are 4x4, 8x8 and 14x14 of 24x24."""
    nodes = W.convbig(1103, in_shape=(3, 24, 24), ch=(4, 4, 8, 8), hidden=(16, 16))
    x0, lo, hi = W.make_input(nodes[0]["shape"], eps, 2103)
    C, c0, label = W.make_spec(nodes, x0)
    return W.Workload(nodes, x0, lo, hi, C, c0, label, eps)


def _splits(root_unst, n, seed):
    """Split sets whose first split lies in ReLU layer 0 or 1, so that layers 1-3 (or 2-3) are
    recomputed with receptive-field rows."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        m0 = b % 2
        j0 = int(rng.choice(root_unst[m0]))
        sp = [(m0, j0, int(rng.choice([1, -1])))]
        for _ in range(int(rng.integers(0, 3))):
            m = int(rng.integers(m0, 4))
            j = int(rng.choice(root_unst[m]))
            if all((m, j) != (a, c) for a, c, _ in sp):
                sp.append((m, j, int(rng.choice([1, -1]))))
        out.append(sp)
    return out


def _run(wl, mask, splits, steps, cap=0):
    """Root bounds, optimised batch bounds and every subproblem's intermediate bounds under one
    kernel-variant mask."""
    import paper_2205_00263_amd as P
    P.set_kernel_variants(mask)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=3 * len(splits) + 64, max_mnc=cap)
    rid, rlb, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    root = [pb.get_bounds(rid, m)[:2] for m in range(net.n_relu)]
    if cap:
        pb.mnc_generate(rid, cap=cap)
    ids = make_batch(pb, rid, splits)
    timer = P.KernelTimer(net, kind="fold")
    timer.start()
    lb, ub = pb.bound_optimize(ids, steps=steps, lr=0.1)
    fold = timer.stop()
    inter = [[pb.get_bounds(int(i), m)[:2] for m in range(net.n_relu)] for i in ids]
    return dict(rlb=rlb, root=root, lb=lb, ub=ub, inter=inter, fold_bytes=fold["bytes"], pb=pb, ids=ids, rid=rid)


def _close(a, b, what, rel=2e-5):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    fin = np.isfinite(b)
    assert np.array_equal(np.isfinite(a), fin), what
    err = np.abs(a[fin] - b[fin])
    assert np.all(err <= rel * np.maximum(1.0, np.abs(b[fin]))), f"{what}: worst {err.max():.3e}"


@pytest.mark.parametrize("cone", [True, False])
@pytest.mark.parametrize("cap", [0, 60])
def test_patch_rows_equal_whole_layer_rows(cap, cone):
    """The same batch (16 subproblems, 3 Adam steps) with receptive-field rows (adjoint on forward
    cones, or on whole rows rebuilt from the windows) and with whole-layer rows: root bounds,
    reported lb and every intermediate bound agree to FP32 summation order, and the folds of the
    window path move far fewer bytes."""
    wl = _medium()
    net_o, q = oracle_query(wl)
    root_o, _ = oo.root_pass(q)
    splits = _splits(root_unstable(net_o, root_o), 16, seed=5 + cap)
    a = _run(wl, NO_FUSED if cone else NO_FUSED | NO_CONE, splits, 3, cap)
    b = _run(wl, NO_FUSED | NO_PATCH, splits, 3, cap)
    _close(a["rlb"], b["rlb"], "root lb")
    for m in range(len(a["root"])):
        _close(a["root"][m][0], b["root"][m][0], f"root l layer {m}")
        _close(a["root"][m][1], b["root"][m][1], f"root u layer {m}")
    _close(a["lb"], b["lb"], "batch lb", rel=1e-4)
    for k in range(len(splits)):
        for m in range(len(a["inter"][k])):
            _close(a["inter"][k][m][0], b["inter"][k][m][0], f"sub {k} l layer {m}", rel=1e-4)
            _close(a["inter"][k][m][1], b["inter"][k][m][1], f"sub {k} u layer {m}", rel=1e-4)
    assert a["fold_bytes"] < 0.5 * b["fold_bytes"], (a["fold_bytes"], b["fold_bytes"])


def test_patch_rows_match_oracle():
    """Root pass and optimised children with receptive-field rows against the FP64 oracle: every
    root bound, and 4 sampled subproblems after 3 Adam steps (lb and recomputed bounds)."""
    wl = _medium()
    net_o, q = oracle_query(wl)
    root_o, _ = oo.root_pass(q)
    splits = _splits(root_unstable(net_o, root_o), 8, seed=11)
    a = _run(wl, NO_FUSED, splits, 3)
    for m, i in enumerate(net_o.relus):
        assert_parity(a["root"][m][0], root_o.states[i].l, f"root l layer {m}")
        assert_parity(a["root"][m][1], root_o.states[i].u, f"root u layer {m}")
    for k in (0, 1, 4, 7):
        sub = oracle_subproblem(net_o, root_o, splits[k])
        ref = oo.bound_optimize(q, sub, steps=3)
        assert_parity(a["lb"][k], ref.lb, f"sub {k} lb")
        for m, i in enumerate(net_o.relus):
            assert_parity(a["inter"][k][m][0], ref.states[i].l, f"sub {k} l layer {m}")
            assert_parity(a["inter"][k][m][1], ref.states[i].u, f"sub {k} u layer {m}")


def test_patch_gradients_match_whole_layer():
    """mnb_bound_grad of the lower and upper sets of ReLU layers 1-3 of a split subproblem at the same
    random alpha / beta (beta > 0 on the split neurons, so that the shared rows carry split terms):
    row bounds and alpha / beta gradients, window path against whole layers."""
    import paper_2205_00263_amd as P
    wl = _medium()
    net_o, q = oracle_query(wl)
    root_o, _ = oo.root_pass(q)
    unst = root_unstable(net_o, root_o)
    split = [[(0, int(unst[0][0]), 1), (1, int(unst[1][0]), -1), (0, int(unst[0][5]), -1)]]
    got = {}
    for mask in (NO_FUSED, NO_FUSED | NO_CONE, NO_FUSED | NO_PATCH):
        P.set_kernel_variants(mask)
        net = P.Net(wl.nodes)
        pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
        rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
        sid = int(make_batch(pb, rid, split)[0])
        rng = np.random.default_rng(3)
        got[mask] = []
        for s in range(1, 7):
            pb.set_params(sid, s, alpha=rng.uniform(0, 1, pb.total_d), beta=rng.uniform(0, 0.5, pb.total_d))
            got[mask].append(pb.bound_grad(sid, s))
    for mask in (NO_FUSED, NO_FUSED | NO_CONE):
        for s, (x, y) in enumerate(zip(got[mask], got[NO_FUSED | NO_PATCH])):
            assert len(x[0]) == len(y[0]) > 0, f"set {s + 1} rows"
            for t, name in enumerate(("lb", "g_alpha", "g_beta")):
                xa, ya = np.asarray(x[t], np.float64), np.asarray(y[t], np.float64)
                scale = max(1.0, np.abs(ya).max())
                err = np.abs(xa - ya).max()
                assert err <= 2e-5 * scale, f"mask {mask} set {s + 1} {name}: {err:.3e}"


def test_patch_batch_invariance():
    """A subproblem alone and inside a batch give bitwise the same bounds on the window path."""
    import paper_2205_00263_amd as P
    wl = _medium()
    net_o, q = oracle_query(wl)
    root_o, _ = oo.root_pass(q)
    splits = _splits(root_unstable(net_o, root_o), 6, seed=17)
    P.set_kernel_variants(NO_FUSED)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=64)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    ids = make_batch(pb, rid, splits)
    alone = make_batch(pb, rid, splits[2:3])
    lb_all, _ = pb.bound_optimize(ids, steps=2, lr=0.1)
    lb_one, _ = pb.bound_optimize(alone, steps=2, lr=0.1)
    assert np.array_equal(lb_all[2], lb_one[0])
    for m in range(net.n_relu):
        assert np.array_equal(pb.get_bounds(int(ids[2]), m)[0], pb.get_bounds(int(alone[0]), m)[0])


def test_full_convbig_patch_rows_equal_whole_layer_rows():
    """The full ConvBig net with generated constraints (the benchmark's configuration): 6
    subproblems split in ReLU layers 0-2, 2 Adam steps, window rows against whole-layer rows
    (the default kernels on this net use the window rows)."""
    import paper_2205_00263_amd as P
    wl = W.make_workload(3)
    P.set_kernel_variants(0)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=32, max_mnc=500)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    pb.mnc_generate(rid, cap=500)
    unst = []
    for m in range(net.n_relu):
        l, u, _ = pb.get_bounds(rid, m)
        unst.append(np.nonzero((l < 0) & (u > 0))[0])
    splits = [[(m % 3, int(unst[m % 3][7 * m + 3]), 1 if m % 2 else -1)] for m in range(6)]
    res = {}
    for mask in (0, NO_PATCH):
        P.set_kernel_variants(mask)
        ids = make_batch(pb, rid, splits)
        lb, _ = pb.bound_optimize(ids, steps=2, lr=0.1)
        res[mask] = (lb, [[pb.get_bounds(int(i), m)[:2] for m in range(net.n_relu)] for i in ids])
        pb.release(list(ids))
    P.set_kernel_variants(0)
    _close(res[0][0], res[NO_PATCH][0], "lb", rel=1e-4)
    for k in range(len(splits)):
        for m in range(net.n_relu):
            _close(res[0][1][k][m][0], res[NO_PATCH][1][k][m][0], f"sub {k} l layer {m}", rel=1e-4)
            _close(res[0][1][k][m][1], res[NO_PATCH][1][k][m][1], f"sub {k} u layer {m}", rel=1e-4)
