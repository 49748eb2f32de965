"""Benchmark: BaB subproblems bounded per second on one MI355X.

Workload (default, --config 3): the ConvBig-shaped network (3x32x32 -> conv 32
3x3/1/1 -> conv 32 4x4/2/1 -> conv 64 3x3/1/1 -> conv 64 4x4/2/1 -> FC 512 ->
FC 512 -> FC 10, He-normal FP32, seeded), eps = 2/255, 9 spec rows, multi-neuron
constraints generated on the device for the root (groups of three unstable
neurons, <= 500 per ReLU layer), and a batch of 1024 subproblems with 1-8 random
splits among the root-unstable neurons.  A subproblem is bounded by 20 Adam
steps on (alpha, beta, gamma) through the hand-written adjoint, each step
recomputing the intermediate bounds of the layers after its earliest split and
then bounding the spec rows.  One timed step is one such Adam iteration over the
whole batch (bound_optimize_step of a session); value = batch / (20 x step time
+ the final evaluation), with inputs and state resident in HBM.  A short Poisson
stream of verification queries through the continuous-batching server gives the
p50/p99 query latency in the same line.

--config 2 measures the ConvSmall-shaped network instead (1x28x28 -> conv 16
4x4/2 -> conv 32 4x4/2 -> FC 100 -> FC 10, eps = 0.03, 512 subproblems, alpha and
beta), one step being one whole bound_optimize of the batch, beside two
per-subproblem loops on the same subproblems (the library one subproblem at a
time, and a plain PyTorch loop with autograd and torch.optim.Adam).

--serving runs the full query stream instead: Poisson arrivals of queries on
the FC / ConvSmall / ConvBig nets (one spec row, eps ~ U[0.005, 0.03]) through
the continuous-batching server, with p50/p99 query latency, subproblems/s and
the verdict mix, and the same stream served one query at a time by a
per-subproblem loop for comparison.

Prints one JSON line (see the repository's measurement notes).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SPLIT_SEED_CS = 3002   # ConvSmall split sets
SPLIT_SEED_CB = 3003   # ConvBig split sets
MNC_CAP = 500          # multi-neuron constraints per ReLU layer (ConvBig)
# counter runs (FETCH_SIZE / WRITE_SIZE) of the roofline kernel of each workload, and the sources that
# fix that kernel and the rows each of its launches gets
TRAFFIC = {
    ("convsmall", "bottom", None): ("bottom_convsmall_traffic.json",
               ("bottom_mf.hip", "bottom.hip", "bottom.h", "common.h", "engine.hip")),
    ("convbig", "conv_forward", 3): ("conv2_forward_convbig_traffic.json",
                     ("conv_win.hip", "gemm.hip", "kernels.h", "common.h", "engine.hip", "engine_calls.inc",
                      "patch.hip")),
}


def kernel_sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2205_00263_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def measured_traffic(workload, kernel, node=None):
    """HBM bytes per launch from the committed counter runs, or None if absent or the kernel changed since."""
    if (workload, kernel, node) not in TRAFFIC:
        return None
    name, files = TRAFFIC[(workload, kernel, node)]
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return d.get("bytes_per_launch") if d.get("kernel_source_sha256") == kernel_sources_sha256(files) else None


def make_batch(P, pb, rid, splits):
    """Create one batch of subproblems from the root by chained branch_split (untimed setup)."""
    cur = np.full(len(splits), rid, np.int64)
    depth = max(len(s) for s in splits)
    for t in range(depth):
        idx = [b for b, s in enumerate(splits) if len(s) > t]
        par = cur[idx]
        lay = [splits[b][t][0] for b in idx]
        neu = [splits[b][t][1] for b in idx]
        kids = pb.branch_split(par, lay, neu)
        drop = []
        for k, b in enumerate(idx):
            keep = 0 if splits[b][t][2] > 0 else 1
            if t > 0:
                drop.append(cur[b])
            cur[b] = kids[2 * k + keep]
            drop.append(kids[2 * k + 1 - keep])
        pb.release(drop)
    return cur


def cpu_baseline(wl, splits, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the same workload (subproblems of the same split sets)."""
    from oracle import bab as obab
    from oracle import net as onet
    from oracle import optimize as oo
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = 1
    net = onet.Net(wl.nodes)
    q = oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0)
    root, _ = oo.root_pass(q)
    done, t0 = 0, time.perf_counter()
    for sp in splits:
        s = root
        for (m, j, sg) in sp:
            a, b = obab.branch_split(net, s, m, j)
            s = a if sg > 0 else b
        oo.bound_optimize(q, s, steps=20, lr=0.1)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "subproblems/s", "cores": int(cores), "kind": "oracle",
            "sample": f"first {done} of the {len(splits)} subproblems (same split sets, T=20), "
                      f"{el:.1f} s FP64 numpy"}


# --------------------------------------------------------------------------- per-subproblem loops
def engine_loop(pb, ids, kw, budget_s):
    """The same library, one subproblem per bound_optimize call (no batching)."""
    import torch
    lat, lbs = [], []
    t0 = time.perf_counter()
    for sid in ids:
        ts = time.perf_counter()
        lb, _ = pb.bound_optimize([int(sid)], **kw)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        lbs.append(lb[0])
        if time.perf_counter() - t0 > budget_s:
            break
    return len(lbs) / (time.perf_counter() - t0), lat, np.array(lbs)


class TorchLoop:
    """The plain per-subproblem loop on the same GPU, written with PyTorch ops.

    One subproblem at a time: the back-substitution (Eq. 2, conv layers as
    transposed convolutions), the ReLU rule of Eq. 5 with alpha and beta, box
    concretisation (Eq. 6) and the intermediate-bound recompute of the layers
    after the subproblem's earliest split, with gradients by autograd and
    torch.optim.Adam (projected), T + 1 evaluations and the best bound per row
    kept -- the schedule bound_optimize runs, without batching or the
    hand-written adjoint."""

    def __init__(self, wl, dev="cuda"):
        import torch
        from workloads import node_shapes
        self.torch = torch
        self.nodes = wl.nodes
        self.shapes = node_shapes(wl.nodes)
        self.relus = [i for i, n in enumerate(wl.nodes) if n["kind"] == "relu"]
        self.sizes = [int(np.prod(self.shapes[i])) for i in self.relus]
        self.offs = np.cumsum([0] + self.sizes)
        self.dev = dev
        self.W, self.bias = {}, {}
        for i, n in enumerate(wl.nodes):
            if n["kind"] in ("fc", "conv"):
                self.W[i] = torch.tensor(np.asarray(n["W"], np.float32), device=dev)
                b = torch.tensor(np.asarray(n["b"], np.float32), device=dev)
                c, h, w = self.shapes[i]
                self.bias[i] = b.repeat_interleave(h * w) if n["kind"] == "conv" else b
        self.lo = torch.tensor(np.asarray(wl.lo, np.float32), device=dev)
        self.hi = torch.tensor(np.asarray(wl.hi, np.float32), device=dev)
        self.C = torch.tensor(np.asarray(wl.C, np.float32), device=dev)
        self.c0 = torch.tensor(np.asarray(wl.c0, np.float32), device=dev)

    def _adjoint(self, i, a):
        import torch.nn.functional as F
        n = self.nodes[i]
        if n["kind"] == "fc":
            return a @ self.W[i]
        ci, hi, wi = self.shapes[n["src"]]
        co, ho, wo = self.shapes[i]
        s, p, k = n["stride"], n["pad"], self.W[i].shape[2]
        op = hi - ((ho - 1) * s - 2 * p + k)
        out = F.conv_transpose2d(a.reshape(-1, co, ho, wo), self.W[i], stride=s, padding=p, output_padding=op)
        return out.reshape(a.shape[0], -1)

    def _bound(self, start_node, a, c, st, par):
        torch = self.torch
        coef = {start_node: a}
        for i in range(start_node, 0, -1):
            if i not in coef:
                continue
            a = coef.pop(i)
            n = self.nodes[i]
            if n["kind"] in ("fc", "conv"):
                c = c + a @ self.bias[i]
                v = self._adjoint(i, a)
                coef[n["src"]] = coef[n["src"]] + v if n["src"] in coef else v
            elif n["kind"] == "relu":
                m = self.relus.index(i)
                l, u, S = st[m]
                al, be = par[m]
                pos, neg = S < 0, S > 0
                act = ~pos & ~neg & (l >= 0)
                ina = ~pos & ~neg & ~act & (u <= 0)
                uns = ~pos & ~neg & ~act & ~ina
                w = torch.where(uns, u - l, torch.ones_like(u))
                chord = torch.where(uns, u / w, torch.zeros_like(u))
                icpt = torch.where(uns, -u * l / w, torch.zeros_like(u))
                ngt = a < 0
                one = (pos | act).to(a.dtype).expand_as(a)
                D = torch.where(uns & ~ngt, al.expand_as(a), one)
                D = torch.where(uns & ngt, chord.expand_as(a), D)
                c = c + (a * torch.where(uns & ngt, icpt.expand_as(a), torch.zeros_like(a))).sum(1)
                v = a * D + S * be
                coef[n["src"]] = coef[n["src"]] + v if n["src"] in coef else v
            elif n["kind"] == "add":
                for s_ in (n["src"], n["src2"]):
                    coef[s_] = coef[s_] + a if s_ in coef else a
        a0 = coef[0]
        return torch.minimum(a0 * self.lo, a0 * self.hi).sum(1) + c

    def load(self, pb, sid, rf):
        """Subproblem state (bounds, splits, parameters) copied from the library to torch tensors."""
        torch = self.torch
        R = len(self.relus)
        st = []
        for m in range(R):
            l, u, S = pb.get_bounds(int(sid), m)
            st.append([torch.tensor(l, device=self.dev), torch.tensor(u, device=self.dev),
                       torch.tensor(S.astype(np.float32), device=self.dev)])
        sets = [0] + [s for m in range(max(rf, 1), R) for s in (2 * m - 1, 2 * m)]
        par = {}
        for si in sets:
            a_, b_, _ = pb.get_params(int(sid), si)
            nm = R if si == 0 else (si + 1) // 2
            par[si] = [[torch.tensor(a_[self.offs[k]:self.offs[k + 1]], device=self.dev),
                        torch.tensor(b_[self.offs[k]:self.offs[k + 1]], device=self.dev)] for k in range(nm)]
        return st, par, list(range(max(rf, 1), R))

    def run(self, state, parent_lb, steps, lr):
        torch = self.torch
        st, par0, layers = state
        st = [[x.clone() for x in s] for s in st]
        par = {si: [[x.detach().clone().requires_grad_() for x in pr] for pr in par0[si]] for si in par0}
        rows = {m: torch.nonzero((st[m][0] < 0) & (st[m][1] > 0)).flatten() for m in layers}
        opts = {si: torch.optim.Adam([t for pr in par[si] for t in pr], lr=lr, maximize=True) for si in par}
        best = torch.tensor(parent_lb, device=self.dev)
        last = len(self.nodes) - 1
        for t in range(steps + 1):
            objs = []
            for m in layers:
                js = rows[m]
                if len(js) == 0:
                    continue
                src = self.nodes[self.relus[m]]["src"]
                d = int(np.prod(self.shapes[src]))
                for sgn, si in ((1.0, 2 * m - 1), (-1.0, 2 * m)):
                    E = torch.zeros(len(js), d, device=self.dev)
                    E[torch.arange(len(js), device=self.dev), js] = sgn
                    lbm = self._bound(src, E, torch.zeros(len(js), device=self.dev), st, par[si])
                    objs.append((si, lbm.sum()))
                    with torch.no_grad():
                        k = 0 if sgn > 0 else 1
                        cur = st[m][k].clone()
                        cur[js] = torch.maximum(cur[js], lbm) if sgn > 0 else torch.minimum(cur[js], -lbm)
                        st[m][k] = cur
            lbf = self._bound(last, self.C, self.c0, st, par[0])
            objs.append((0, lbf.sum()))
            best = torch.maximum(best, lbf.detach())
            if t == steps:
                break
            for si, obj in objs:
                opts[si].zero_grad()
                obj.backward()
                opts[si].step()
                with torch.no_grad():
                    for al, be in par[si]:
                        al.clamp_(0.0, 1.0)
                        be.clamp_(min=0.0)
        return best


def torch_loop(wl, pb, ids, rfs, parent_lb, kw, budget_s):
    import torch
    tl = TorchLoop(wl)
    states = [tl.load(pb, sid, rf) for sid, rf in list(zip(ids, rfs))[:64]]   # untimed: state resident in HBM
    tl.run(states[-1], parent_lb, 1, kw["lr"])                      # untimed warm-up (library kernels load)
    torch.cuda.synchronize()
    lat, lbs = [], []
    t0 = time.perf_counter()
    for s in states:
        ts = time.perf_counter()
        b = tl.run(s, parent_lb, kw["steps"], kw["lr"])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        lbs.append(b.cpu().numpy())
        if time.perf_counter() - t0 > budget_s:
            break
    return len(lbs) / (time.perf_counter() - t0), lat, np.array(lbs)


def loop_summary(name, rate, lat, lbs, ref):
    d = np.abs(lbs - ref[: len(lbs)])
    return {"kind": name, "value": round(rate, 3), "unit": "subproblems/s", "sample": len(lbs),
            "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
            "lb_mean": float(lbs.min(1).mean()), "batched_lb_mean": float(ref[: len(lbs)].min(1).mean()),
            "max_abs_lb_diff_vs_batched": float(d.max()),
            "max_rel_lb_diff_vs_batched": float((d / np.maximum(1.0, np.abs(ref[: len(lbs)]))).max())}


# --------------------------------------------------------------------------- serving stream
SERVE_SEED = 5005


def make_stream(W, nodes, n, rate, seed=SERVE_SEED):
    """Poisson arrivals; each query: a random net of the list, x0 ~ U[0,1], eps ~ U[0.005, 0.03],
    one spec row against a random class."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate))
        ni = int(rng.integers(0, len(nodes)))
        eps = float(rng.uniform(0.005, 0.03))
        x0, lo, hi = W.make_input(nodes[ni][0]["shape"], eps, int(rng.integers(0, 2**31)))
        Cm, c0, _ = W.make_spec(nodes[ni], x0, n_spec=1, seed=int(rng.integers(0, 2**31)))
        out.append((t, ni, lo, hi, Cm, c0))
    return out


def loop_bab(pb, lo, hi, Cm, c0, kw, timeout_s, queue_cap, t_start):
    """BaB of one query with one subproblem per bound_optimize call (lowest lb first)."""
    import heapq
    rid, lb, ub = pb.bound_init(lo, hi, Cm, c0)
    if (ub < 0).any():
        pb.release([rid])
        return "falsified", 1
    if (lb > 0).all():
        pb.release([rid])
        return "verified", 1
    heap, order, n_sub, verdict = [(float(lb.min()), 0, rid)], 1, 0, "verified"
    while heap:
        if time.perf_counter() - t_start > timeout_s:
            verdict = "timeout"
            break
        _, _, sid = heapq.heappop(heap)
        lb, ub, bl, bn = pb.bound_optimize([sid], want_branch=True, **kw)
        n_sub += 1
        if (ub[0] < 0).any():
            pb.release([sid])
            verdict = "falsified"
            break
        if (lb[0] > 0).all():
            pb.release([sid])
            continue
        if bl[0] < 0 or len(heap) + 2 > queue_cap:
            pb.release([sid])
            verdict = "unknown"
            break
        kids = pb.branch_split([sid], [int(bl[0])], [int(bn[0])])
        pb.release([sid])
        for k in kids:
            heapq.heappush(heap, (float(lb[0].min()), order, int(k)))
            order += 1
    if heap:
        pb.release([h[2] for h in heap])
    return verdict, n_sub


def serving(args):
    import collections
    import torch
    import paper_2205_00263_amd as P
    import workloads as W
    torch.cuda.set_device(0)
    cfgs = [int(c) for c in args.serve_nets.split(",")]
    nodes = [W.make_net(c) for c in cfgs]
    nets = [P.Net(n) for n in nodes]
    stream = make_stream(W, nodes, args.serve_queries, args.serve_rate)
    kw = dict(steps=args.adam_steps, lr=0.1)
    srv = P.Server(nets, max_batch=args.serve_batch, steps=args.adam_steps, lr=0.1)
    # untimed warm-up: one query per net (problem pools are created on first use)
    for ni in range(len(nets)):
        q = next(s for s in stream if s[1] == ni)
        srv.wait(srv.query_submit(ni, *q[2:], timeout_s=5.0), timeout=600)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for (ta, ni, lo, hi, Cm, c0) in stream:
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.query_submit(ni, lo, hi, Cm, c0, timeout_s=args.serve_timeout))
    print(f"[serving] {len(tickets)} queries submitted at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    res, step = [], max(1, len(tickets) // 10)
    for k, tk in enumerate(tickets):
        res.append(srv.wait(tk, timeout=args.serve_timeout + 3600))
        if (k + 1) % step == 0:
            print(f"[serving] {k + 1} results at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.array([r["latency"] for r in res])
    n_sub = int(sum(r["subproblems"] for r in res))
    mix = collections.Counter(r["verdict"] for r in res)
    per_net = {f"cfg{c}": {"queries": int(sum(1 for s in stream if s[1] == i)),
                           "p50_s": round(float(np.percentile([r["latency"] for r, s in zip(res, stream)
                                                               if s[1] == i] or [0], 50)), 4),
                           "subproblems": int(sum(r["subproblems"] for r, s in zip(res, stream) if s[1] == i))}
               for i, c in enumerate(cfgs)}
    out = {"metric": "BaB subproblems bounded/sec + p50/p99 query latency (serving stream)",
           "value": round(n_sub / wall, 2), "unit": "subproblems/s", "n_gpus": 1, "higher_is_better": True,
           "dtype": "f32", "data": "synthetic",
           "p50_s": round(float(np.percentile(lat, 50)), 4), "p99_s": round(float(np.percentile(lat, 99)), 4),
           "wall_s": round(wall, 2), "queries": len(res), "subproblems": n_sub, "verdicts": dict(mix),
           "per_net": per_net,
           "config": {"workload": "serving_stream", "nets": [f"cfg{c}" for c in cfgs], "n_spec": 1,
                      "eps": "U[0.005,0.03]", "arrivals": f"Poisson {args.serve_rate}/s",
                      "timeout_s": args.serve_timeout, "max_batch": args.serve_batch, "adam_steps": args.adam_steps,
                      "mem_budget_GiB": 64, "queue_cap": 4096}}
    if args.serve_loop_budget > 0:
        # the plain per-subproblem loop: queries in arrival order, one at a time, batch 1
        pbs = [P.Problem(n, n_spec=1, capacity=4096 + 64) for n in nets]
        for ni in range(len(nets)):   # untimed warm-up
            q = next(s for s in stream if s[1] == ni)
            loop_bab(pbs[ni], *q[2:], kw, 2.0, 4096, time.perf_counter())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat_l, verd_l, nsub_l, done = [], [], 0, 0
        for (ta, ni, lo, hi, Cm, c0) in stream:
            now = time.perf_counter() - t0
            if now > args.serve_loop_budget:
                break
            if ta > now:
                time.sleep(ta - now)
            v, ns = loop_bab(pbs[ni], lo, hi, Cm, c0, kw, args.serve_timeout, 4096, t0 + ta)
            lat_l.append(time.perf_counter() - t0 - ta)
            verd_l.append(v)
            nsub_l += ns
            done += 1
        wall_l = time.perf_counter() - t0
        srv_lat = lat[:done]
        out["per_subproblem_loop"] = {
            "kind": "library, one subproblem per bound_optimize, queries FIFO", "queries_done": done,
            "budget_s": args.serve_loop_budget, "value": round(nsub_l / wall_l, 2), "unit": "subproblems/s",
            "p50_s": round(float(np.percentile(lat_l, 50)), 4), "p99_s": round(float(np.percentile(lat_l, 99)), 4),
            "server_p50_s_same_queries": round(float(np.percentile(srv_lat, 50)), 4),
            "server_p99_s_same_queries": round(float(np.percentile(srv_lat, 99)), 4),
            "verdicts": dict(collections.Counter(verd_l)),
            "verdicts_agree_with_server": int(sum(a == r["verdict"] for a, r in zip(verd_l, res)))}
    print(json.dumps(out), flush=True)


# --------------------------------------------------------------------------- full BaB (ResNet6)
def bab_run(args):
    """Complete verification of queries on the ResNet6-shaped net: the first inputs (seeded
    x0 ~ U[0,1]) whose DeepPoly root is neither verified nor falsified, each run to a verdict
    through the server (batches <= max_batch, queue cap 4096, 20 Adam steps per batch)."""
    import torch
    import paper_2205_00263_amd as P
    import workloads as W
    torch.cuda.set_device(0)
    nodes = W.make_net(4)
    net = P.Net(nodes)
    pb = P.Problem(net, n_spec=9, capacity=64)
    open_q, scanned = [], 0
    for sd in range(7000, 7400):
        x0, lo, hi = W.make_input(nodes[0]["shape"], args.bab_eps, sd)
        Cm, c0, _ = W.make_spec(nodes, x0)
        rid, lb, ub = pb.bound_init(lo, hi, Cm, c0)
        pb.release([rid])
        scanned += 1
        if not (ub < 0).any() and not (lb > 0).all():
            open_q.append((sd, lo, hi, Cm, c0, float(lb.min())))
        if len(open_q) >= args.bab_queries:
            break
    srv = P.Server([net], max_batch=args.serve_batch, queue_cap=4096, steps=args.adam_steps, lr=0.1)
    res, tot_sub, t_all = [], 0, time.perf_counter()
    for sd, lo, hi, Cm, c0, lb0 in open_q:
        t = time.perf_counter()
        r = srv.wait(srv.query_submit(0, lo, hi, Cm, c0, timeout_s=args.serve_timeout), timeout=3600)
        el = time.perf_counter() - t
        tot_sub += r["subproblems"]
        res.append({"seed": sd, "verdict": r["verdict"], "subproblems": int(r["subproblems"]),
                    "seconds": round(el, 3), "deeppoly_lb": round(lb0, 4), "root_opt_lb": round(float(r["lb"]), 4)})
        print(f"[bab] seed {sd}: {r['verdict']} {r['subproblems']} subproblems {el:.2f} s", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - t_all
    srv.close()
    print(json.dumps({"metric": "BaB subproblems bounded/sec (complete verification, ResNet6)",
                      "value": round(tot_sub / wall, 2), "unit": "subproblems/s", "n_gpus": 1,
                      "higher_is_better": True, "dtype": "f32", "data": "synthetic",
                      "config": {"workload": "resnet6_bab", "eps": args.bab_eps, "n_spec": 9,
                                 "max_batch": args.serve_batch, "queue_cap": 4096, "adam_steps": args.adam_steps,
                                 "timeout_s": args.serve_timeout, "inputs_scanned": scanned,
                                 "selection": "first seeds whose DeepPoly root is undecided"},
                      "queries": res}), flush=True)


def roofline_of(kstats, traffic=None):
    """Roofline object of one timed kernel class: its bound follows from its algorithmic intensity
    against the MI355X ridge point (FP32 MFMA 157.3 TFLOP/s over HBM 8 TB/s = 19.7 flop/byte)."""
    if not kstats or kstats["count"] == 0:
        return None
    avg_s = kstats["ms"] / kstats["count"] / 1e3
    flops = kstats["flops"] / kstats["count"]
    byts = kstats["bytes"] / kstats["count"]
    ridge = 157.3e12 / 8.0e12
    if byts > 0 and (flops == 0 or flops / byts < ridge):
        achieved = byts / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                "frac": round(achieved / 8000.0, 4)}
    else:
        achieved = flops / avg_s / 1e12
        roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": 157.3, "unit": "TFLOP/s",
                "frac": round(achieved / 157.3, 4)}
    roof.update({"traffic": traffic, "kernel": kstats["name"], "launches": kstats["count"],
                 "avg_us": round(avg_s * 1e6, 2), "algorithmic_gflop_per_launch": round(flops / 1e9, 4),
                 "algorithmic_mb_per_launch": round(byts / 1e6, 3),
                 "flop_per_byte": round(flops / byts, 2) if byts > 0 else None})
    return roof


def convsmall_batch(args):
    """The ConvSmall batch (--config 2): one step = one bound_optimize of 512 subproblems."""
    import torch
    import paper_2205_00263_amd as P
    import workloads as W

    args.batch = args.batch or 512
    args.roofline_kernel = args.roofline_kernel or "bottom"

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    P.use_torch_plumbing(True)
    wl = W.make_workload(2)
    net = P.Net(wl.nodes)
    n_steps = args.warmup + args.steps
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=args.batch * (n_steps + 5) + 64)
    rid, root_lb, root_ub = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    unstable = []
    for m in range(net.n_relu):
        l, u, _ = pb.get_bounds(rid, m)
        unstable.append(np.nonzero((l < 0) & (u > 0))[0])
    splits = W.make_split_sets(unstable, args.batch, 1, 8, seed=SPLIT_SEED_CS)
    batches = [make_batch(P, pb, rid, splits) for _ in range(n_steps)]
    kw = dict(steps=args.adam_steps, lr=0.1)

    timer = P.KernelTimer(net, kind=args.roofline_kernel)
    for b in batches[: args.warmup]:
        pb.bound_optimize(b, **kw)
    torch.cuda.synchronize()
    timer.start()
    lat = []
    t0 = time.perf_counter()
    lbs = []
    for b in batches[args.warmup:]:
        ts = time.perf_counter()
        lb, ub = pb.bound_optimize(b, **kw)
        lat.append(time.perf_counter() - ts)
        lbs.append(lb)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kstats = timer.stop()
    n_bounded = args.batch * args.steps
    value = n_bounded / el
    roof = roofline_of(kstats, measured_traffic("convsmall", args.roofline_kernel))
    out = {
        "metric": "BaB subproblems bounded/sec (alpha,beta-optimised, 20 Adam steps) + p50/p99 batch latency",
        "value": round(value, 2), "unit": "subproblems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "config": {"workload": "convsmall_bab_batch", "net": "ConvSmall 1x28x28 c16k4s2 c32k4s2 fc100 fc10",
                   "eps": 0.03, "n_spec": int(wl.C.shape[0]), "batch": args.batch, "split_depth": "1-8",
                   "adam_steps": args.adam_steps, "lr": 0.1},
        "bound_summary": {"root_lb_min": float(root_lb.min()),
                          "batch_lb_mean": float(np.mean([x.min(1).mean() for x in lbs]))},
        "roofline": roof,
    }
    if not args.no_loop_baseline:
        ref = lbs[0]
        ids = make_batch(P, pb, rid, splits)
        r = engine_loop(pb, ids, kw, args.loop_budget)
        loops = [loop_summary("library, one subproblem per call", *r, ref)]
        pb.release(ids)
        ids = make_batch(P, pb, rid, splits)
        rfs = [min(m for m, _, _ in sp) + 1 for sp in splits]
        r = torch_loop(wl, pb, ids, rfs, root_lb, kw, args.loop_budget)
        loops.append(loop_summary("PyTorch ops + autograd + torch.optim.Adam, one subproblem at a time", *r, ref))
        pb.release(ids)
        out["per_subproblem_loops"] = loops
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, splits, args.cpu_budget)
    print(json.dumps(out), flush=True)



def host_cores():
    """(cores this process may run on, CPU model) of the host."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return int(n), model


def cpu_baseline_convbig(wl, mean_rows, threads, rows_per_layer=128):
    """The FP64 oracle on a bounded sample of the ConvBig workload: one Adam iteration's work (the
    back-substitution of Eq. 2 / Eq. 5 / Eq. 6 and the analytic gradient) of a few rows of every
    recomputed layer and of the spec rows, timed per row and scaled by the batch's mean rows per
    subproblem and layer, with BLAS limited to `threads` threads.  The oracle's own bounds come from an
    interval pass of the same net and box (the work per row does not depend on the bound values)."""
    from threadpoolctl import threadpool_limits
    from oracle import backsub as ob
    from oracle import net as onet
    from oracle import optimize as oo
    net = onet.Net(wl.nodes)
    lo, hi = np.asarray(wl.lo, np.float64), np.asarray(wl.hi, np.float64)
    states = {}
    for i in net.relus:
        src = net.nodes[i]["src"]
        L, U = onet.interval_forward(net, lo, hi, {k: (st.l, st.u) for k, st in states.items()}, src)
        states[i] = ob.ReluState(L[src], U[src])
    params = {i: {"alpha": ob.heuristic_alpha(st), "beta": np.zeros(st.l.shape)} for i, st in states.items()}
    t_row, t_total = {}, 0.0
    with threadpool_limits(limits=threads):
        for m, i in enumerate(net.relus):
            if m == 0 or mean_rows.get(m, 0.0) == 0.0:
                continue
            js = np.nonzero((states[i].l < 0) & (states[i].u > 0))[0][:rows_per_layer]
            t0 = time.perf_counter()
            out = ob.backsub(net, ob.neuron_start(net, i, js, 1), np.zeros(len(js)), states, params, None, lo, hi)
            oo.bound_grads(net, out)
            dt = time.perf_counter() - t0
            t_row[m] = dt / len(js)
            t_total += dt
        t0 = time.perf_counter()
        out = ob.backsub(net, ob.spec_start(net, wl.C), wl.c0, states, params, None, lo, hi)
        oo.bound_grads(net, out)
        t_spec = time.perf_counter() - t0
        t_total += t_spec
    per_iter = sum(mean_rows[m] * t for m, t in t_row.items()) + t_spec
    return {"value": 1.0 / (20.0 * per_iter), "unit": "subproblems/s", "cores": int(threads), "kind": "oracle",
            "sample": f"FP64 numpy back-substitution + analytic gradient of {rows_per_layer} rows of each recomputed "
                      f"layer and the {len(wl.C)} spec rows ({t_total:.1f} s), scaled by the batch's mean rows per "
                      f"subproblem and layer {dict((m, round(v, 1)) for m, v in mean_rows.items())} and 20 Adam "
                      f"steps: {per_iter:.1f} s of CPU per subproblem step",
            "seconds_per_row": {str(m): round(t, 4) for m, t in t_row.items()}}


def query_stream(args, n_queries):
    """A short Poisson stream of queries on the FC / ConvSmall / ConvBig nets through the server: p50/p99
    query latency, subproblems/s and the verdict mix."""
    import collections
    import paper_2205_00263_amd as P
    import workloads as W
    cfgs = [int(c) for c in args.serve_nets.split(",")]
    nodes = [W.make_net(c) for c in cfgs]
    nets = [P.Net(n) for n in nodes]
    stream = make_stream(W, nodes, n_queries, args.serve_rate)
    srv = P.Server(nets, max_batch=args.serve_batch, steps=args.adam_steps, lr=0.1)
    for ni in range(len(nets)):   # untimed warm-up: problem pools are created on first use
        q = next(x for x in stream if x[1] == ni)
        srv.wait(srv.query_submit(ni, *q[2:], timeout_s=5.0), timeout=600)
    t0 = time.perf_counter()
    tickets = []
    for (ta, ni, lo, hi, Cm, c0) in stream:
        dt = ta - (time.perf_counter() - t0)
        if dt > 0:
            time.sleep(dt)
        tickets.append(srv.query_submit(ni, lo, hi, Cm, c0, timeout_s=args.serve_timeout))
    res = [srv.wait(tk, timeout=args.serve_timeout + 600) for tk in tickets]
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.array([r["latency"] for r in res])
    n_sub = int(sum(r["subproblems"] for r in res))
    return {"queries": len(res), "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4), "subproblems_per_s": round(n_sub / wall, 1),
            "wall_s": round(wall, 2), "verdicts": dict(collections.Counter(r["verdict"] for r in res)),
            "nets": [f"cfg{c}" for c in cfgs], "arrivals": f"Poisson {args.serve_rate}/s", "n_spec": 1,
            "eps": "U[0.005,0.03]", "timeout_s": args.serve_timeout}


def convbig_batch(args):
    """The headline: ConvBig with generated multi-neuron constraints, 1024 subproblems, alpha, beta and
    gamma; one timed step = one Adam iteration of the whole batch."""
    import torch
    import paper_2205_00263_amd as P
    import workloads as W

    B = args.batch or 1024
    # the dominant kernel: the forward convolution of the adjoint at ConvBig's second convolution
    # (every launch of that class runs the 128 x 32 gather GEMM)
    kind = args.roofline_kernel or "conv_forward"
    node = args.roofline_node if args.roofline_node is not None else 3
    T = args.adam_steps

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(1 << 28, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    P.use_torch_plumbing(True)
    wl = W.make_workload(3)
    net = P.Net(wl.nodes)
    pb = P.Problem(net, n_spec=wl.C.shape[0], capacity=3 * B + 64, max_mnc=MNC_CAP)
    t = time.perf_counter()
    rid, root_lb, root_ub = pb.bound_init(wl.lo, wl.hi, wl.C, wl.c0)
    t_init = time.perf_counter() - t
    t = time.perf_counter()
    n_mnc = pb.mnc_generate(rid, cap=MNC_CAP)
    t_mnc = time.perf_counter() - t
    unstable = []
    for m in range(net.n_relu):
        l, u, _ = pb.get_bounds(rid, m)
        unstable.append(np.nonzero((l < 0) & (u > 0))[0])
    splits = W.make_split_sets(unstable, B, 1, 8, seed=SPLIT_SEED_CB)
    ids = make_batch(P, pb, rid, splits)
    # rows each subproblem recomputes per layer (2 per unstable neuron of the layers after its
    # earliest split), on a sample of the batch: the CPU baseline's scale
    mean_rows = {}
    sample = list(range(0, B, max(1, B // 64)))
    for m in range(1, net.n_relu):
        tot = 0
        for b in sample:
            if min(sp[0] for sp in splits[b]) + 1 <= m:
                l, u, _ = pb.get_bounds(int(ids[b]), m)
                tot += 2 * int(np.sum((l < 0) & (u > 0)))
        mean_rows[m] = tot / len(sample)
    log(f"root lb {root_lb.min():.3f}, constraints per layer {n_mnc.tolist()} ({t_mnc:.2f} s), batch of {B} ready")
    sess = pb.optimize_begin(ids, steps=T, lr=0.1)
    for w in range(args.warmup):
        sess.step()
        torch.cuda.synchronize()
        log(f"warm-up step {w + 1}/{args.warmup}")
    timer = P.KernelTimer(net, kind=kind, node=node)
    timer.start()
    lat = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        sess.step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        log(f"step {k + 1}/{args.steps}: {lat[-1] * 1e3:.1f} ms")
    el = time.perf_counter() - t0
    kstats = timer.stop()
    t = time.perf_counter()
    lb, ub = sess.end()
    torch.cuda.synchronize()
    t_end = time.perf_counter() - t
    step_s = el / args.steps
    value = B / (T * step_s + t_end)
    out = {
        "metric": "BaB subproblems bounded/sec (alpha,beta,gamma-optimised) + p50/p99 query latency",
        "value": round(value, 3), "unit": "subproblems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "convbig_mnc_batch",
                   "net": "ConvBig 3x32x32 c32k3s1p1 c32k4s2p1 c64k3s1p1 c64k4s2p1 fc512 fc512 fc10",
                   "eps": round(2 / 255, 6), "n_spec": int(wl.C.shape[0]), "batch": B, "split_depth": "1-8",
                   "adam_steps": T, "lr": 0.1, "mnc_cap": MNC_CAP, "mnc_per_layer": n_mnc.tolist(),
                   "step": "one Adam iteration (evaluation with intermediate recompute, adjoint, update) of the "
                           "whole batch",
                   "value": "batch / (adam_steps x step time + final evaluation)"},
        "timing": {"final_evaluation_ms": round(t_end * 1e3, 2), "bound_init_ms": round(t_init * 1e3, 2),
                   "mnc_generate_ms": round(t_mnc * 1e3, 2),
                   "step_p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                   "step_p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3)},
        "bound_summary": {"root_lb_min": float(root_lb.min()), "root_ub_min": float(root_ub.min()),
                          "batch_lb_mean": float(lb.min(1).mean())},
        "roofline": roofline_of(kstats, measured_traffic("convbig", kind, node)),
    }
    if args.stream_queries > 0:
        log(f"query stream: {args.stream_queries} queries")
        qs = query_stream(args, args.stream_queries)
        out["p50_s"], out["p99_s"] = qs["p50_s"], qs["p99_s"]
        out["query_stream"] = qs
    if not args.no_cpu_baseline:
        log("cpu baseline")
        n, model = host_cores()
        cb = cpu_baseline_convbig(wl, mean_rows, n)
        cb1 = cpu_baseline_convbig(wl, mean_rows, 1)
        cb["cpu_model"] = model
        cb["single_thread"] = {"value": cb1["value"], "cores": 1}
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=3, choices=[2, 3],
                    help="3: ConvBig with multi-neuron constraints (default); 2: ConvSmall")
    ap.add_argument("--batch", type=int, default=None, help="subproblems per batch (default 1024 / 512)")
    ap.add_argument("--adam-steps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-loop-baseline", action="store_true",
                    help="skip the per-subproblem loops (library at batch 1, PyTorch autograd)")
    ap.add_argument("--loop-budget", type=float, default=10.0, help="seconds per per-subproblem loop")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device copy first (a kernel of known traffic for counter calibration)")
    ap.add_argument("--roofline-node", type=int, default=None,
                    help="network node whose launches the roofline times (default: ConvBig's second convolution)")
    ap.add_argument("--roofline-kernel", default=None,
                    help="kernel class timed for the roofline object (dominant one for this workload)")
    ap.add_argument("--serving", action="store_true", help="serving stream instead of the batch benchmark")
    ap.add_argument("--bab", action="store_true", help="complete BaB of ResNet6 queries instead of the batch benchmark")
    ap.add_argument("--bab-eps", type=float, default=1 / 255)
    ap.add_argument("--bab-queries", type=int, default=4)
    ap.add_argument("--serve-queries", type=int, default=1000)
    ap.add_argument("--serve-rate", type=float, default=10.0, help="Poisson arrival rate (queries/s)")
    ap.add_argument("--serve-timeout", type=float, default=60.0)
    ap.add_argument("--serve-batch", type=int, default=1024)
    ap.add_argument("--serve-nets", default="1,2,3", help="configurations whose nets the stream draws from")
    ap.add_argument("--serve-loop-budget", type=float, default=60.0,
                    help="seconds for the per-subproblem FIFO loop on the same stream (0: skip)")
    ap.add_argument("--stream-queries", type=int, default=200,
                    help="Poisson queries served after the ConvBig batch for the latency keys (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(subproblems shard across GPUs without collectives; see the design notes)", file=sys.stderr)
        sys.exit(2)

    if args.serving:
        serving(args)
        return
    if args.bab:
        bab_run(args)
        return
    if args.config == 2:
        args.roofline_node = -1 if args.roofline_node is None else args.roofline_node
        convsmall_batch(args)
    else:
        args.roofline_node = 3 if args.roofline_node is None else args.roofline_node
        convbig_batch(args)


if __name__ == "__main__":
    main()
