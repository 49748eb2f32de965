"""torch.autograd interface of the hand-written adjoint (needs an MI355X).

The gradient that autograd returns through SetBound is compared with the FP64
oracle's analytic gradient (itself pinned against finite differences), and a
projected Adam run driven by torch.optim through SetBound is compared with the
library's own fused optimiser on an identical subproblem."""
import numpy as np
import pytest

import workloads as W
from oracle import backsub as ob
from oracle import bab as obab
from oracle import optimize as oo

from _common import assert_parity, oracle_query, root_unstable

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_00263_amd as P
    P.lib()
    yield


@pytest.mark.parametrize("cfg", [2, 4])
def test_autograd_gradient_matches_oracle(cfg):
    import paper_2205_00263_amd as P
    from paper_2205_00263_amd.autograd import set_bound
    wl = W.make_workload(cfg, scale="small")
    net_o, q = oracle_query(wl)
    root, _ = oo.root_pass(q)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
    rid, _, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    j0 = int(root_unstable(net_o, root)[0][0])
    gid = int(pb.branch_split([rid], [0], [j0])[0])
    osub = obab.branch_split(net_o, root, 0, j0)[0]
    pb.bound_optimize([gid], steps=0)
    oo.bound_optimize(q, osub, steps=0)
    rng = np.random.default_rng(100 + cfg)
    offs = np.cumsum([0] + [net_o.sizes[i] for i in net_o.relus])
    checked = 0
    for key in oo.set_keys(net_o):
        si = P.set_index(key)
        alpha = torch.tensor(rng.uniform(0, 1, offs[-1]).astype(np.float32), device="cuda", requires_grad=True)
        beta = torch.tensor(rng.uniform(0, 0.5, offs[-1]).astype(np.float32), device="cuda", requires_grad=True)
        obj, lb = set_bound(pb, gid, si, alpha, beta)
        if key == "final":
            start, c0 = ob.spec_start(net_o, q.C), q.c0
        else:
            m, s = key
            st = osub.states[net_o.relus[m]]
            js = np.nonzero((st.l < 0) & (st.u > 0))[0]
            if len(js) == 0:
                assert lb.numel() == 0
                continue
            start, c0 = ob.neuron_start(net_o, net_o.relus[m], js, s), np.zeros(len(js))
        params = {}
        a_h, b_h = alpha.detach().cpu().numpy(), beta.detach().cpu().numpy()
        for t, i in enumerate(net_o.relus):
            if i in osub.sets[key]:
                params[i] = dict(osub.sets[key][i])
                params[i]["alpha"] = a_h[offs[t]:offs[t + 1]].astype(np.float64)
                params[i]["beta"] = b_h[offs[t]:offs[t + 1]].astype(np.float64)
        out = ob.backsub(net_o, start, c0, osub.states, params, None, q.lo, q.hi)
        assert_parity(lb.cpu().numpy(), out["lb"], f"{key} rows")
        (2.0 * obj).backward()   # chain rule through the scalar objective
        g = oo.bound_grads(net_o, out)
        for name, tt in (("alpha", alpha), ("beta", beta)):
            ref = 2.0 * np.concatenate([g[i][name] if i in g else np.zeros(net_o.sizes[i]) for i in net_o.relus])
            got = tt.grad.cpu().numpy()
            nrm = np.linalg.norm(ref)
            assert np.linalg.norm(got - ref) <= 1e-3 * max(nrm, 1e-6), (key, name, np.linalg.norm(got - ref), nrm)
        checked += 1
    assert checked >= 2


@pytest.mark.parametrize("cfg", [1, 2])
def test_autograd_adam_matches_fused_optimiser(cfg):
    """torch.optim.Adam on SetBound (spec set, intermediate bounds fixed) == bound_optimize with
    recompute_intermediate off, on two identical children of the root."""
    import paper_2205_00263_amd as P
    from paper_2205_00263_amd.autograd import optimize_set
    wl = W.make_workload(cfg, scale="small")
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=16)
    rid, root_lb, _ = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    l, u, _ = pb.get_bounds(rid, 0)
    j0 = int(np.nonzero((l < 0) & (u > 0))[0][0])
    kids = pb.branch_split([rid, rid], [0, 0], [j0, j0])
    a_id, b_id = int(kids[0]), int(kids[2])
    steps = 6
    lb_fused, _ = pb.bound_optimize([a_id], steps=steps, lr=0.1, recompute_intermediate=False)
    best = optimize_set(pb, b_id, 0, steps=steps, lr=0.1).cpu().numpy()
    lb_auto = np.maximum(best, root_lb)
    print("fused", lb_fused[0][:3], "autograd", lb_auto[:3], flush=True)
    assert_parity(lb_auto, lb_fused[0].astype(np.float64), "autograd Adam vs fused Adam")
    assert np.all(lb_auto >= root_lb - 1e-6)
