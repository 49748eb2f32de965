"""Root pass, parameter sets, analytic gradient and Adam (oracle; test infrastructure only).

Section 3.1 of the paper:
* every intermediate bound l/u is computed with the same back-substitution
  procedure, with one parameter set shared by all neurons of a layer and
  separate sets for the lower and the upper bounds;
* any alpha in [0,1], beta >= 0, gamma >= 0 gives a sound bound, so the
  parameters are tightened by projected gradient ascent;
* for every subproblem a DeepPoly bound (heuristic alpha, beta = gamma = 0)
  comes first (Section 4, experimental setup).

The gradient of a bound with respect to (alpha, beta, gamma) is written out
analytically: D and b-underline are piecewise constant in a', so
d lb / d a^(0) = x* and, going back up, every layer's gradient is the
forward image of x* through the row's linearised network
(g at an affine output = W g_in + b; at a ReLU output = D g_hat + b-underline).
Then  d/d alpha_j = a'_j g_hat_j  (unstable j, a'_j >= 0),
      d/d beta_j  = S_jj g_hat_j,
      d/d gamma   = P g + Phat g_hat - p.
Intermediate bounds l/u are treated as constants of a set's objective.
"""
from __future__ import annotations

import copy

import numpy as np

from .net import AFFINE_KINDS, affine_apply, bias_vector, forward, interval_forward
from .backsub import (ReluState, backsub, heuristic_alpha, neuron_start,
                      spec_start)

ADAM_DEFAULTS = dict(lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8)


# --------------------------------------------------------------------------- gradient
def bound_grads(net, out, mncs=None, per_row=False):
    """Analytic d lb / d params for the rows of one back-substitution result `out`.

    Returns dict relu-node -> dict(alpha=, beta=, gamma=) summed over rows
    (per_row=False, one shared set) or per row ([R, ...]).
    """
    mncs = mncs or {}
    recs = out["records"]
    if not recs:
        return {}
    top = max(recs)
    g = {0: out["xstar"]}
    grads = {}
    for i in range(1, top + 1):
        n = net.nodes[i]
        k = n["kind"]
        if k in AFFINE_KINDS:
            if n["src"] in g:
                g[i] = affine_apply(net, i, g[n["src"]]) + bias_vector(net, i)
        elif k == "add":
            if n["src"] in g and n["src2"] in g:
                g[i] = g[n["src"]] + g[n["src2"]]
        elif k == "relu":
            if i not in recs:
                continue
            rec = recs[i]
            ghat = g[n["src"]]
            g[i] = rec["D"] * ghat + rec["bl"]
            ap = rec["ap"]
            da = np.where(rec["unstable"][None, :] & (ap >= 0), ap * ghat, 0.0)
            db = rec["S"][None, :] * ghat
            if i in mncs and mncs[i].e > 0:
                m = mncs[i]
                dg = g[i] @ m.P.T + ghat @ m.Phat.T - m.p[None, :]
            else:
                dg = np.zeros((ghat.shape[0], 0))
            if per_row:
                grads[i] = {"alpha": da, "beta": db, "gamma": dg}
            else:
                grads[i] = {"alpha": da.sum(0), "beta": db.sum(0), "gamma": dg.sum(0)}
    return grads


# --------------------------------------------------------------------------- Adam
class Adam:
    """Adam ascent on a dict of parameter arrays, PyTorch's bias-corrected update."""

    def __init__(self, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m, self.v, self.t = {}, {}, 0

    def step(self, params, grads):
        self.t += 1
        for key, g in grads.items():
            if key not in self.m:
                self.m[key] = np.zeros_like(g)
                self.v[key] = np.zeros_like(g)
            self.m[key] = self.b1 * self.m[key] + (1 - self.b1) * g
            self.v[key] = self.b2 * self.v[key] + (1 - self.b2) * g * g
            mh = self.m[key] / (1 - self.b1 ** self.t)
            vh = self.v[key] / (1 - self.b2 ** self.t)
            params[key] = params[key] + self.lr * mh / (np.sqrt(vh) + self.eps)


def project(pset):
    """alpha in [0,1]; beta, gamma >= 0."""
    for i, p in pset.items():
        p["alpha"] = np.clip(p["alpha"], 0.0, 1.0)
        p["beta"] = np.maximum(p["beta"], 0.0)
        if "gamma" in p:
            p["gamma"] = np.maximum(p["gamma"], 0.0)


# --------------------------------------------------------------------------- query / subproblem
class Query:
    """One verification problem: net, box, spec rows and optional MNC sets."""

    def __init__(self, net, lo, hi, C, c0, mncs=None, margin=0.0):
        self.net = net
        self.margin = float(margin)   # rounding margin of the reported spec-row bounds (0: exact Eq. 6)
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)
        self.C = np.asarray(C, dtype=np.float64)
        self.c0 = np.asarray(c0, dtype=np.float64)
        self.mncs = mncs or {}

    @property
    def n_spec(self):
        return self.C.shape[0]


class Subproblem:
    """BaB subproblem: bounds l/u and split diagonal per ReLU node, parameter sets, best bounds.

    Parameter sets are keyed "final" (the spec rows) or (m, +1) / (m, -1) for the
    lower / upper bounds of ReLU layer m (m indexes net.relus); each maps
    relu-node -> dict(alpha, beta, gamma) for the ReLU nodes below its objective.
    """

    def __init__(self, states, sets, lb, ub, recompute_from):
        self.states = states
        self.sets = sets
        self.lb = lb
        self.ub = ub
        self.recompute_from = recompute_from  # ReLU layer index, len(relus) = nothing pending
        self.splits = []

    def clone(self):
        return copy.deepcopy(self)


def set_keys(net):
    keys = ["final"]
    for m in range(1, len(net.relus)):
        keys += [(m, 1), (m, -1)]
    return keys


def set_scope(net, key):
    """ReLU nodes a set's parameters cover (those below its objective)."""
    if key == "final":
        return list(net.relus)
    m = key[0]
    return net.relus[:m]


def init_sets(net, states, mncs):
    sets = {}
    for key in set_keys(net):
        ps = {}
        for i in set_scope(net, key):
            e = mncs[i].e if i in mncs else 0
            ps[i] = {"alpha": heuristic_alpha(states[i]),
                     "beta": np.zeros(states[i].l.shape),
                     "gamma": np.zeros(e)}
        sets[key] = ps
    return sets


def attach_mncs(q: Query, sub: Subproblem, mncs):
    """Give the query its MNC sets (generated from the root bounds) and size gamma = 0 in every set."""
    q.mncs = mncs
    for ps in sub.sets.values():
        for i, p in ps.items():
            p["gamma"] = np.zeros(mncs[i].e if i in mncs else 0)


def spec_ub(q: Query, xstar):
    """ub_r = C_r f(x*_r) + c0_r: the spec evaluated at the concretisation minimiser."""
    fx = forward(q.net, xstar)
    return np.einsum("rk,rk->r", q.C, fx) + q.c0


# --------------------------------------------------------------------------- root pass
def root_pass(q: Query):
    """DeepPoly bound of the root (heuristic alpha, beta = gamma = 0).

    ReLU layer 0: exact interval of the first affine layer.  Layer m >= 1: an
    interval pass marks neurons that are already stable; rows +e_j / -e_j of
    the others are back-substituted, and the result is intersected with the
    interval bound.
    """
    net = q.net
    states = {}
    for m, i in enumerate(net.relus):
        src = net.nodes[i]["src"]
        L, U = interval_forward(net, q.lo, q.hi, {k: (s.l, s.u) for k, s in states.items()}, src)
        l, u = L[src].copy(), U[src].copy()
        if m > 0:
            js = np.nonzero((l < 0) & (u > 0))[0]
            if len(js):
                params = {k: {"alpha": heuristic_alpha(s), "beta": np.zeros(s.l.shape)}
                          for k, s in states.items()}
                lo_out = backsub(net, neuron_start(net, i, js, +1), np.zeros(len(js)),
                                 states, params, None, q.lo, q.hi)
                up_out = backsub(net, neuron_start(net, i, js, -1), np.zeros(len(js)),
                                 states, params, None, q.lo, q.hi)
                l[js] = np.maximum(l[js], lo_out["lb"])
                u[js] = np.minimum(u[js], -up_out["lb"])
        states[i] = ReluState(l, u)
    params = {k: {"alpha": heuristic_alpha(s), "beta": np.zeros(s.l.shape)}
              for k, s in states.items()}
    out = backsub(net, spec_start(net, q.C), q.c0, states, params, None, q.lo, q.hi, q.margin)
    ub = spec_ub(q, out["xstar"])
    sub = Subproblem(states, init_sets(net, states, q.mncs), out["lb"].copy(), ub,
                     recompute_from=len(net.relus))
    sub.best_x = out["xstar"]
    sub.final_records = out["records"]
    return sub, out


# --------------------------------------------------------------------------- optimisation
def recompute_layers(net, sub):
    start = max(1, sub.recompute_from)
    return list(range(start, len(net.relus)))


def bound_optimize(q: Query, sub: Subproblem, steps=20, lr=0.1, beta1=0.9, beta2=0.999,
                   eps=1e-8, trace=None, teacher=None):
    """Optimise (alpha, beta, gamma) of one subproblem with `steps` Adam updates.

    Evaluations t = 0..steps: recompute the intermediate bounds of the ReLU
    layers after the earliest pending split (rows fixed to the neurons unstable
    at call start; new l/u are intersected with the old), then bound the spec
    rows; keep the best lb per row and its x*; between evaluations take one
    Adam ascent step per set on the sum of the set's row bounds, then project.
    ub = spec at the x* of each row's best evaluation.  Reported lb =
    max(best, previous lb of the subproblem).

    trace: optional list receiving per-evaluation dicts (lb, grads, params).
    teacher: optional list of parameter-set dicts to use at evaluation t
             instead of the optimiser's own iterate (fixed-parameter parity).
    Returns the updated subproblem (modified in place).
    """
    net = q.net
    layers = recompute_layers(net, sub)
    rows = {}
    for m in layers:
        st = sub.states[net.relus[m]]
        rows[m] = np.nonzero((st.l < 0) & (st.u > 0))[0]
    keys = ["final"] + [(m, s) for m in layers for s in (1, -1)]
    opts = {k: Adam(lr, beta1, beta2, eps) for k in keys}
    best = np.full(q.n_spec, -np.inf)
    best_x = np.zeros((q.n_spec, net.sizes[0]))
    for t in range(steps + 1):
        if teacher is not None:
            for k in keys:
                sub.sets[k] = copy.deepcopy(teacher[t][k])
        outs = {}
        for m in layers:
            i = net.relus[m]
            js = rows[m]
            if len(js) == 0:
                continue
            for s in (1, -1):
                outs[(m, s)] = backsub(net, neuron_start(net, i, js, s), np.zeros(len(js)),
                                       sub.states, sub.sets[(m, s)], q.mncs, q.lo, q.hi)
            st = sub.states[i]
            st.l[js] = np.maximum(st.l[js], outs[(m, 1)]["lb"])
            st.u[js] = np.minimum(st.u[js], -outs[(m, -1)]["lb"])
        outs["final"] = backsub(net, spec_start(net, q.C), q.c0, sub.states, sub.sets["final"],
                                q.mncs, q.lo, q.hi, q.margin)
        lb = outs["final"]["lb"]
        better = lb > best
        best = np.where(better, lb, best)
        best_x[better] = outs["final"]["xstar"][better]
        rec = {"t": t, "lb": lb.copy(), "params": copy.deepcopy({k: sub.sets[k] for k in keys}),
               "l": {i: sub.states[i].l.copy() for i in net.relus},
               "u": {i: sub.states[i].u.copy() for i in net.relus}}
        if t == steps:
            if trace is not None:
                trace.append(rec)
            break
        grads_all = {}
        for k, out in outs.items():
            grads = bound_grads(net, out, q.mncs)
            grads_all[k] = grads
            flat_p, flat_g = {}, {}
            for i, gi in grads.items():
                for name in ("alpha", "beta", "gamma"):
                    if name in gi and name in sub.sets[k][i]:
                        flat_p[(i, name)] = sub.sets[k][i][name]
                        flat_g[(i, name)] = gi[name]
            opts[k].step(flat_p, flat_g)
            for (i, name), v in flat_p.items():
                sub.sets[k][i][name] = v
            project(sub.sets[k])
        rec["grads"] = grads_all
        if trace is not None:
            trace.append(rec)
    sub.lb = np.maximum(best, sub.lb)
    sub.ub = spec_ub(q, best_x)
    sub.best_x = best_x
    sub.final_records = outs["final"]["records"]
    sub.recompute_from = len(net.relus)
    return sub
