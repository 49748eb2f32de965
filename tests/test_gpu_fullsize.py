"""Full-size parity of the batched path (needs an MI355X).

The nets of the benchmarks run kernels that the small test nets never reach: the MFMA first
layer needs 16 first-layer channels (ConvSmall, the ResNet6 stem), the window kernel and the
tap-GEMM transposed convolution ConvSmall's second convolution.  Here the full ConvSmall and
ResNet6 nets run in the launch configuration of the benchmark (a batch of split subproblems,
chunked rows, intermediate recompute, the optimiser with the adjoint), and subproblems
sampled from the batch are recomputed one by one by the FP64 oracle.  Every row of the batch
is also compared with the same batch on the general kernels (VALU first layer, no window
kernel), a second implementation of each step.

The library lowers the bounds it reports (the spec rows) by its FP32 rounding margin, 2^-20
(sum |a| max(|lo|, |hi|) + |c|), about 1e-6 of the bound; intermediate bounds carry no margin.
The samples are compared with the exact FP64 oracle (Eq. 6 without margin) and, beside it,
with the oracle computing the same margin in FP64."""
import numpy as np
import pytest

import workloads as W
from oracle import backsub as ob
from oracle import optimize as oo

from _common import (assert_parity, make_batch, oracle_query, oracle_subproblem, root_unstable)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SPLIT_SEED = 3002   # the benchmark's split sets
MARGIN = 2.0 ** -20  # the library's rounding margin of a reported (spec-row) bound


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


# (configuration, batch, Adam steps, sampled subproblems)
CASES = [(2, 512, 3, [0, 255, 511]), (4, 256, 2, [17])]


@pytest.mark.timeout(900)   # the FP64 oracle's root passes and samples of ResNet6 take minutes
@pytest.mark.parametrize("cfg,n_batch,steps,samples", CASES)
def test_full_batch_matches_oracle_on_samples(cfg, n_batch, steps, samples):
    P = _P()
    wl = W.make_workload(cfg)
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    qm = oo.Query(net_o, wl.lo, wl.hi, wl.C, wl.c0, margin=MARGIN)
    root_m, _ = oo.root_pass(qm)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=4 * n_batch + 64)
    rid, root_lb, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    assert_parity(root_lb, root.lb, "root (exact oracle)")
    assert_parity(root_lb, root_m.lb, "root (oracle with the margin)")
    for m, i in enumerate(net_o.relus):
        l, u, _ = pb.get_bounds(rid, m)
        assert_parity(l, root.states[i].l, f"root l, ReLU layer {m}")
        assert_parity(u, root.states[i].u, f"root u, ReLU layer {m}")
    splits = W.make_split_sets(root_unstable(net_o, root), n_batch, 1, 8, seed=SPLIT_SEED)
    ids = make_batch(pb, rid, splits)
    ids2 = make_batch(pb, rid, splits)
    lb, _ = pb.bound_optimize(ids, steps=steps, lr=0.1)
    print(f"cfg{cfg}: batch {n_batch}, T={steps}, mean min-row lb {lb.min(axis=1).mean():.6f}", flush=True)
    for b in samples:
        osub = oo.bound_optimize(q, oracle_subproblem(net_o, root, splits[b]), steps=steps, lr=0.1)
        assert_parity(lb[b], osub.lb, f"cfg{cfg} subproblem {b} (exact oracle)")
        ref_m = oo.bound_optimize(qm, oracle_subproblem(net_o, root_m, splits[b]), steps=steps, lr=0.1).lb
        assert_parity(lb[b], ref_m, f"cfg{cfg} subproblem {b} (oracle with the margin)")
        for m, i in enumerate(net_o.relus):
            l, u, _ = pb.get_bounds(int(ids[b]), m)
            assert_parity(l, osub.states[i].l, f"cfg{cfg} subproblem {b} l, ReLU layer {m}")
            assert_parity(u, osub.states[i].u, f"cfg{cfg} subproblem {b} u, ReLU layer {m}")
    # the whole batch on the general kernels
    prev = P.get_kernel_variants()
    try:
        P.set_kernel_variants(P.VARIANTS["valu_bottom"] | P.VARIANTS["no_window"])
        lb2, _ = pb.bound_optimize(ids2, steps=steps, lr=0.1)
    finally:
        P.set_kernel_variants(prev)
    assert_parity(lb, lb2, f"cfg{cfg} batch, specialised vs general kernels")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("cfg", [2])
def test_full_size_gradient_matches_oracle(cfg):
    """Gradients of every parameter set of one split subproblem of the full net (random
    feasible parameters, intermediate bounds recomputed with them first)."""
    P = _P()
    wl = W.make_workload(cfg)
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    split = W.make_split_sets(root_unstable(net_o, root), 1, 2, 2, seed=SPLIT_SEED + 1)[0]
    gid = int(make_batch(pb, rid, [split])[0])
    osub = oracle_subproblem(net_o, root, split)
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
        out = ob.backsub(net_o, start, c0, osub.states, osub.sets[key], None, q.lo, q.hi,
                         MARGIN if key == "final" else 0.0)
        assert_parity(lbr, out["lb"], f"{key} rows")
        g = oo.bound_grads(net_o, out)
        for name in ("alpha", "beta"):
            gg = ga if name == "alpha" else gb
            rr = np.concatenate([g[i][name] if i in g else np.zeros(net_o.sizes[i]) for i in net_o.relus])
            nrm = np.linalg.norm(rr)
            assert np.linalg.norm(gg - rr) <= 1e-3 * max(nrm, 1e-6), (key, name, np.linalg.norm(gg - rr), nrm)
