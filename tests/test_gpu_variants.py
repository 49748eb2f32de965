"""The general kernels behind mnb_set_kernel_variants (needs an MI355X).

For the nets of the benchmarks the library picks specialised kernels (MFMA first layer,
tap-GEMM transposed convolution, paired-wavefront forward convolution, window rows);
the general ones they replace still serve other shapes.  Each variant is forced here on
the ConvSmall- and ResNet6-shaped nets and checked against the FP64 oracle: the
convolution products element by element, the optimised bounds and the gradients to the
same tolerances as the default kernels."""
import numpy as np
import pytest

import workloads as W
from oracle import backsub as ob
from oracle import bab as obab
from oracle import net as onet
from oracle import optimize as oo

from _common import assert_parity, make_subproblems, oracle_query, root_unstable

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00263_amd as P
    P.lib()
    yield


@pytest.fixture
def variants():
    """Set a variant mask for one test and restore the previous one afterwards."""
    import paper_2205_00263_amd as P
    prev = P.get_kernel_variants()
    yield P.set_kernel_variants
    P.set_kernel_variants(prev)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


# (Ci, H, Co, k, s, p): ConvSmall's second convolution and a ResNet block convolution
GEOMS = [(16, 13, 32, 4, 2, 0), (16, 16, 32, 3, 2, 1)]
CONV_MASKS = {"no_tap_convt": 2, "no_pair_conv": 4, "no_row_conv": 8}


@pytest.mark.parametrize("name", list(CONV_MASKS))
@pytest.mark.parametrize("geom", GEOMS)
def test_conv_variants_match_oracle(variants, name, geom):
    import paper_2205_00263_amd as P
    variants(CONV_MASKS[name])
    ci, h, co, k, s, p = geom
    rng = np.random.default_rng(11 + sum(geom))
    nodes = [{"kind": "input", "shape": (ci, h, h)},
             {"kind": "conv", "src": 0, "W": rng.normal(size=(co, ci, k, k)).astype(np.float32),
              "b": rng.normal(size=co).astype(np.float32), "stride": s, "pad": p},
             {"kind": "relu", "src": 1},
             {"kind": "fc", "src": 2, "W": np.ones((2, co * ((h + 2 * p - k) // s + 1) ** 2), np.float32),
              "b": np.zeros(2, np.float32)}]
    net = P.Net(nodes)
    on = onet.Net(nodes)
    din, dout = on.sizes[0], on.sizes[1]
    for M in (1, 37, 300):
        A = rng.normal(size=(M, dout)).astype(np.float32)
        ref = onet.conv_adjoint(on.nodes[1]["W"], A.astype(np.float64), on.shapes[0], on.shapes[1], s, p)
        a_d, c_d = _dev(A), torch.full((M, din), 7.0, device="cuda")
        torch.cuda.synchronize()
        net.conv_backsub(1, a_d.data_ptr(), c_d.data_ptr(), M)
        net.sync()
        np.testing.assert_allclose(c_d.cpu().numpy(), ref, rtol=0, atol=1e-5 * np.abs(ref).max() + 1e-5)
        G = rng.normal(size=(M, din)).astype(np.float32)
        reff = onet.conv_apply(on.nodes[1]["W"], G.astype(np.float64), on.shapes[0], on.shapes[1], s, p) \
            + onet.bias_vector(on, 1)
        g_d, o_d = _dev(G), torch.zeros((M, dout), device="cuda")
        torch.cuda.synchronize()
        net.conv_forward(1, g_d.data_ptr(), o_d.data_ptr(), M)
        net.sync()
        np.testing.assert_allclose(o_d.cpu().numpy(), reff, rtol=0, atol=1e-5 * np.abs(reff).max() + 1e-5)


PASS_MASKS = {"valu_bottom": 1, "no_window": 16, "no_fused_bottom": 32, "valu_bottom+no_window": 17,
              "all_general": 63}


@pytest.mark.parametrize("name", list(PASS_MASKS))
@pytest.mark.parametrize("cfg", [2, 4])
def test_pass_variants_match_oracle(variants, name, cfg):
    """Optimised bounds (T = 3, recompute of the layers after the split) and the final set's
    gradients under each forced variant."""
    import paper_2205_00263_amd as P
    variants(PASS_MASKS[name])
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=32)
    rid, root_lb, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    assert_parity(root_lb, root.lb, "root")
    splits = W.make_split_sets(root_unstable(net_o, root), 4, 1, 3, seed=90 + cfg)
    ids, subs = make_subproblems(P, pb, rid, net_o, q, root, splits)
    lb, _ = pb.bound_optimize(ids, steps=3, lr=0.1)
    ref = np.array([oo.bound_optimize(q, s, steps=3, lr=0.1).lb for s in subs])
    assert_parity(lb, ref, f"{name} T=3 lb")
    # gradients of the spec set on a child split in ReLU layer 0 (fixed random parameters)
    j0 = int(root_unstable(net_o, root)[0][0])
    gid = int(pb.branch_split([rid], [0], [j0])[0])
    osub = obab.branch_split(net_o, root, 0, j0)[0]
    rng = np.random.default_rng(cfg)
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    alpha = rng.uniform(0, 1, offs[-1]).astype(np.float32)
    beta = rng.uniform(0, 0.5, offs[-1]).astype(np.float32)
    si = P.set_index("final")
    pb.set_params(gid, si, alpha=alpha, beta=beta)
    for t, i in enumerate(net_o.relus):
        if i in osub.sets["final"]:
            osub.sets["final"][i]["alpha"] = alpha[offs[t]:offs[t + 1]].astype(np.float64)
            osub.sets["final"][i]["beta"] = beta[offs[t]:offs[t + 1]].astype(np.float64)
    pb.bound_optimize([gid], steps=0)
    oo.bound_optimize(q, osub, steps=0)
    lbr, ga, gb, _ = pb.bound_grad(gid, si)
    out = ob.backsub(net_o, ob.spec_start(net_o, q.C), q.c0, osub.states, osub.sets["final"], None, q.lo, q.hi)
    assert_parity(lbr, out["lb"], f"{name} final rows")
    g = oo.bound_grads(net_o, out)
    for nm, gg, key in (("alpha", ga, "alpha"), ("beta", gb, "beta")):
        rr = np.concatenate([g[i][key] if i in g else np.zeros(net_o.sizes[i]) for i in net_o.relus])
        nrm = np.linalg.norm(rr)
        assert np.linalg.norm(gg - rr) <= 1e-3 * max(nrm, 1e-6), (name, nm, np.linalg.norm(gg - rr), nrm)


def test_variant_mask_roundtrip(variants):
    import paper_2205_00263_amd as P
    variants(5)
    assert P.get_kernel_variants() == 5
    assert P.set_kernel_variants(0) == 5
    assert P.get_kernel_variants() == 0
