"""Batch normalisation, average pooling and the ResNet8 shape on the GPU path (needs an MI355X).

The library folds batch normalisation into the preceding affine node and runs average pooling as a
convolution; the oracle applies both layers as written (oracle/net.py).  Small ResNet8-shaped nets
with both layers are compared with the oracle element by element (every intermediate bound, the
root bound, optimised split subproblems); the full ResNet8 shape with batch normalisation is compared
with the same net whose batch normalisation was folded in FP64 beforehand, and checked for soundness
on samples."""
import numpy as np
import pytest

import workloads as W
from oracle import bab as obab
from oracle import net as onet
from oracle import optimize as oo

from _common import assert_parity, oracle_query, root_unstable, sampled_min_sub

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00263_amd as P
    P.lib()
    yield


def _small(seed=11, eps=0.04):
    nodes = W.resnet8(seed, in_shape=(3, 16, 16), ch=(4, 4, 8), hidden=20, bn=True, pool=(2, 2))
    x0, lo, hi = W.make_input(nodes[0]["shape"], eps, seed + 1)
    C, c0, label = W.make_spec(nodes, x0)
    return W.Workload(nodes, x0, lo, hi, C, c0, label, eps)


def test_bn_pool_resnet_root_matches_oracle():
    import paper_2205_00263_amd as P
    wl = _small()
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
    rid, lb, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    assert_parity(lb, root.lb, "root lb")
    for m, i in enumerate(net_o.relus):
        l, u, _ = pb.get_bounds(rid, m)
        assert_parity(l, root.states[i].l, f"l of ReLU layer {m}")
        assert_parity(u, root.states[i].u, f"u of ReLU layer {m}")


def test_bn_pool_resnet_optimised_children_match_oracle():
    import paper_2205_00263_amd as P
    wl = _small()
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    unst = root_unstable(net_o, root)
    m0 = next(t for t in range(len(unst)) if len(unst[t]))
    j0 = int(unst[m0][0])
    kids = pb.branch_split([rid], [m0], [j0])
    okids = obab.branch_split(net_o, root, m0, j0)
    lb, _ = pb.bound_optimize(kids, steps=4)
    for b in range(2):
        ref = oo.bound_optimize(q, okids[b], steps=4)
        assert_parity(lb[b], ref.lb, f"child {b}")
        for m, i in enumerate(net_o.relus):
            l, u, _ = pb.get_bounds(int(kids[b]), m)
            assert_parity(l, ref.states[i].l, f"child {b} l, ReLU layer {m}")
        S = {i: okids[b].states[i].S for i in net_o.relus}
        assert np.all(lb[b] <= sampled_min_sub(net_o, wl, S) + 1e-6)


def _fold_bn(nodes):
    """The node list with every batch normalisation folded into the convolution before it (FP64)."""
    out, remap = [], {}
    for i, n in enumerate(nodes):
        n = dict(n)
        if n["kind"] == "bn":
            a = out[remap[n["src"]]]
            scale = np.asarray(n["gamma"], np.float64) / np.sqrt(np.asarray(n["var"], np.float64) + n["eps"])
            shift = np.asarray(n["beta"], np.float64) - np.asarray(n["mean"], np.float64) * scale
            a["W"] = (np.asarray(a["W"], np.float64) * scale.reshape(-1, *([1] * (a["W"].ndim - 1)))).astype(np.float32)
            a["b"] = (np.asarray(a["b"], np.float64) * scale + shift).astype(np.float32)
            remap[i] = remap[n["src"]]
            continue
        for key in ("src", "src2"):
            if key in n:
                n[key] = remap[n[key]]
        remap[i] = len(out)
        out.append(n)
    return out


def test_full_resnet8_with_bn_equals_prefolded_and_is_sound():
    import paper_2205_00263_amd as P
    nodes = W.resnet8(1008, bn=True)
    assert sum(int(np.prod(s)) for s, n in zip(W.node_shapes(nodes), nodes) if n["kind"] == "relu") == 11364
    x0, lo, hi = W.make_input(nodes[0]["shape"], 1 / 255, 2008)
    Cm, c0, _ = W.make_spec(nodes, x0)
    a = P.Net(nodes)
    b = P.Net(_fold_bn(nodes))
    pa = P.Problem(a, n_spec=Cm.shape[0], capacity=8)
    pbb = P.Problem(b, n_spec=Cm.shape[0], capacity=8)
    ra, lba, _ = pa.bound_init(lo, hi, Cm, c0)
    rb, lbb, _ = pbb.bound_init(lo, hi, Cm, c0)
    np.testing.assert_allclose(lba, lbb, rtol=1e-4, atol=1e-4)
    net_o = onet.Net(nodes)
    rng = np.random.default_rng(3)
    X = rng.uniform(lo, hi, size=(2000, len(lo)))
    f = onet.forward(net_o, X) @ np.asarray(Cm, np.float64).T + c0
    assert np.all(lba <= f.min(0) + 1e-6)
