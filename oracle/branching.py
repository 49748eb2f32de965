"""Branching scores of Section 3.4 (oracle; test infrastructure only).

Active constraint score (multi-neuron constraint guided branching): the
Lagrange parameter gamma of a multi-neuron constraint P z + Phat zhat <= p
(Eq. 3) measures how strongly the bound depends on that constraint, and
gamma^T P, gamma^T Phat are those sensitivities with respect to the ReLU
outputs and inputs.  The score of neuron j of ReLU layer i sums both in
absolute value:

    s_ij = |(gamma_i^T P_i)_j| + |(gamma_i^T Phat_i)_j|,

with gamma of the spec rows' parameter set.  Only unstable (l < 0 < u),
unsplit neurons are candidates.  Cost adjusted branching divides each score
by the direct cost of a split in its layer (Appendix B, `oracle.cost`) and
picks the highest score per cost.
"""
from __future__ import annotations

import numpy as np


def candidates(state):
    """Unstable, unsplit neurons of one ReLU layer."""
    return (state.l < 0) & (state.u > 0) & (state.S == 0)


def acs_scores(net, sub, mncs, key="final"):
    """relu node -> scores [d] (-inf where the neuron is no candidate)."""
    out = {}
    for i in net.relus:
        d = net.sizes[i]
        val = np.zeros(d)
        m = mncs.get(i) if mncs else None
        if m is not None and m.e > 0:
            g = np.asarray(sub.sets[key][i]["gamma"], dtype=np.float64)
            val = np.abs(g @ m.P) + np.abs(g @ m.Phat)
        s = np.full(d, -np.inf)
        c = candidates(sub.states[i])
        s[c] = val[c]
        out[i] = s
    return out


def cab_scores(scores, costs):
    """Scores divided by the split cost of their layer (costs: relu node -> cost > 0)."""
    return {i: s / costs[i] for i, s in scores.items()}


def select(net, scores):
    """(ReLU layer index, neuron) of the highest score, ties to the lowest layer and
    neuron; (-1, -1) without a candidate."""
    best = (-1, -1, -np.inf)
    for t, i in enumerate(net.relus):
        s = scores[i]
        if not np.any(np.isfinite(s)):
            continue
        j = int(np.argmax(s))
        if s[j] > best[2]:
            best = (t, j, s[j])
    return best[0], best[1]
