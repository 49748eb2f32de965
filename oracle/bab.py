"""Branching and the BaB loop (oracle; test infrastructure only).

Section 2.2: bound every subproblem; lb > 0 verifies it, ub < 0 is a
counterexample; otherwise split an unstable ReLU into its two phases.
Section 3.2 ("Enforcing Splits"): a split sets the corresponding entry of the
split matrix S (Eq. 4) in both children; intermediate bounds of layers up to
and including the split layer are kept, later layers are recomputed.

Readings (where the paper is silent):
* a child starts from its parent's parameters, with beta of the new split
  neuron set to 0, and its reported lb is max(child, parent);
* the split neuron's bound is tightened to the phase (l = 0 for the positive
  child, u = 0 for the negative child);
* branching score (the ResNet workload's rule): score_j =
  sum over the spec rows r of |a'_{r,j}| * (-u_j l_j / (u_j - l_j)) over
  unstable, unsplit neurons, taken from the last evaluation of the spec rows;
  ties go to the lowest (layer, index);
* the queue pops the subproblems with the lowest key (min over spec rows of
  lb) first, ties by creation order.
"""
from __future__ import annotations

import numpy as np

from .backsub import relu_cases
from .optimize import bound_optimize, root_pass

VERIFIED, FALSIFIED, UNKNOWN = "verified", "falsified", "unknown"


def branch_split(net, sub, m, j):
    """Two children of `sub` split on neuron j of ReLU layer m: (positive child, negative child)."""
    i = net.relus[m]
    kids = []
    for S_val in (-1, 1):                     # -1: zhat >= 0 (positive), +1: zhat <= 0
        ch = sub.clone()
        st = ch.states[i]
        st.S[j] = S_val
        if S_val == -1:
            st.l[j] = max(st.l[j], 0.0)
        else:
            st.u[j] = min(st.u[j], 0.0)
        for key, ps in ch.sets.items():
            if i in ps:
                ps[i]["beta"][j] = 0.0
        ch.recompute_from = min(sub.recompute_from, m + 1)
        ch.splits = list(sub.splits) + [(m, int(j), 1 if S_val == -1 else -1)]
        kids.append(ch)
    return kids[0], kids[1]


def branching_score(net, sub, final_records):
    """Per-layer score arrays (c.f. module docstring); -inf where not eligible."""
    scores = []
    for m, i in enumerate(net.relus):
        st = sub.states[i]
        _, _, _, _, unstable = relu_cases(st)
        with np.errstate(divide="ignore", invalid="ignore"):
            height = np.where(unstable, -st.u * st.l / (st.u - st.l), 0.0)
        rec = final_records.get(i)
        if rec is None:
            scores.append(np.full(st.l.shape, -np.inf))
            continue
        s = np.sum(np.abs(rec["ap"]), axis=0) * height
        scores.append(np.where(unstable, s, -np.inf))
    return scores


def pick_branch(scores):
    """argmax over (layer, index) with ties to the lowest layer then index; None if nothing eligible."""
    best, arg = -np.inf, None
    for m, s in enumerate(scores):
        if s.size == 0:
            continue
        j = int(np.argmax(s))
        if s[j] > best:
            best, arg = s[j], (m, j)
    return arg


def bab(q, steps=20, lr=0.1, batch=8, max_subproblems=4096, root_steps=None):
    """Full BaB loop on one query.  Returns (verdict, stats dict)."""
    net = q.net
    root, _ = root_pass(q)
    n_bounded = 1
    if np.any(root.ub < 0):
        return FALSIFIED, {"bounded": n_bounded}
    bound_optimize(q, root, steps=steps if root_steps is None else root_steps, lr=lr)
    if np.any(root.ub < 0):
        return FALSIFIED, {"bounded": n_bounded}
    if np.all(root.lb > 0):
        return VERIFIED, {"bounded": n_bounded}
    queue = [(float(np.min(root.lb)), 0, root)]
    created = 1
    while queue:
        queue.sort(key=lambda e: (e[0], e[1]))
        take, queue = queue[:batch], queue[batch:]
        for _, _, sub in take:
            arg = pick_branch(branching_score(net, sub, sub.final_records))
            if arg is None:
                return UNKNOWN, {"bounded": n_bounded, "reason": "no unstable neuron left"}
            for ch in branch_split(net, sub, *arg):
                bound_optimize(q, ch, steps=steps, lr=lr)
                n_bounded += 1
                if np.any(ch.ub < 0):
                    return FALSIFIED, {"bounded": n_bounded}
                if np.all(ch.lb > 0):
                    continue
                queue.append((float(np.min(ch.lb)), created, ch))
                created += 1
        if len(queue) > max_subproblems:
            return UNKNOWN, {"bounded": n_bounded, "reason": "queue cap"}
    return VERIFIED, {"bounded": n_bounded}
