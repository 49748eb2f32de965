"""Back-substitution through the network (oracle; test infrastructure only).

Follows Section 3.1 of the paper:

* affine layer (Eq. 2):  a^(i-1) = ahat^(i) W^(i),  c^(i-1) = ahat^(i) b^(i) + c^(i)
* ReLU layer (Eq. 5), in the paper's order
    1. multi-neuron constraints:  a' = a + gamma^T P,  c gains -gamma^T p, and
       gamma^T Phat becomes a coefficient on zhat;
    2. single-neuron DeepPoly relaxation (the D / b-underline case table);
    3. split constraints:  ahat = a' D + beta^T S + gamma^T Phat.
* concretisation (Eq. 6) over the input box:  min_x a^(0) x + c^(0)
* the minimiser x* used for the upper bound (Section 3.1, "Upper Bounding").

Readings where the paper is loose (each listed in the design notes):
* the sign test that selects D and b-underline uses a' = a + gamma^T P, the
  coefficient D actually multiplies in Eq. 5;
* a split takes precedence over the stable cases, and a stable case over the
  unstable one;
* the input region is the box [lo, hi] (the L-infinity ball clipped to the
  valid input range); without clipping this equals Hoelder's form of Eq. 6
  with q = 1;
* on a residual join the coefficient is passed unchanged to both operands and
  the contributions meeting at a common producer are summed (linearity).

Optional rounding margin (`margin`, default 0 = the exact bound of Eq. 6): an
FP32 implementation may lower the bounds it reports by
margin * (sum_j |a_j| max(|lo_j|, |hi_j|) + |c|) to cover its own rounding
where the bound is exact; with the margin set, this oracle computes that
bound in FP64.  The optimiser applies it to the spec rows only (the reported
lower bounds); intermediate bounds are the exact values of Eq. 6.

Parameter arrays may be shared by all rows of a set (shape [d]) or per row
(shape [R, d]); numpy broadcasting covers both.
"""
from __future__ import annotations

import numpy as np

from .net import AFFINE_KINDS, affine_adjoint, bias_vector


class ReluState:
    """Per-ReLU-node data of one subproblem: input bounds l/u, split matrix diagonal S."""

    def __init__(self, l, u, S=None):
        self.l = np.asarray(l, dtype=np.float64)
        self.u = np.asarray(u, dtype=np.float64)
        self.S = np.zeros(self.l.shape, dtype=np.int64) if S is None else np.asarray(S, dtype=np.int64)


class Mnc:
    """Multi-neuron constraints P z + Phat zhat <= p of one ReLU layer (Eq. 3), dense [e, d]."""

    def __init__(self, P, Phat, p):
        self.P = np.asarray(P, dtype=np.float64)
        self.Phat = np.asarray(Phat, dtype=np.float64)
        self.p = np.asarray(p, dtype=np.float64)

    @property
    def e(self):
        return self.p.shape[0]


def relu_cases(st: ReluState):
    """Boolean masks of the D case table (split first, then stable, then unstable)."""
    pos_split = st.S == -1          # S_jj = -1 : zhat_j >= 0 (Eq. 4)
    neg_split = st.S == 1           # S_jj = +1 : zhat_j <= 0
    split = pos_split | neg_split
    active = ~split & (st.l >= 0)
    inactive = ~split & ~active & (st.u <= 0)
    unstable = ~split & ~active & ~inactive
    return pos_split, neg_split, active, inactive, unstable


def relu_backsub(a, st: ReluState, alpha, beta, mnc: Mnc | None = None, gamma=None):
    """One ReLU step of Eq. 5 for rows a [R, d] (coefficients on z = relu(zhat)).

    Returns (ahat [R, d] coefficients on zhat, dc [R], record) where record holds
    what the analytic gradient needs.
    """
    a = np.asarray(a, dtype=np.float64)
    R, d = a.shape
    if mnc is not None and mnc.e > 0:
        gamma = np.asarray(gamma, dtype=np.float64)
        gP = gamma @ mnc.P if gamma.ndim == 1 else np.einsum("re,ed->rd", gamma, mnc.P)
        gPh = gamma @ mnc.Phat if gamma.ndim == 1 else np.einsum("re,ed->rd", gamma, mnc.Phat)
        gp = gamma @ mnc.p if gamma.ndim == 1 else gamma @ mnc.p
    else:
        gP, gPh, gp = 0.0, 0.0, 0.0
    ap = a + gP                                  # step 1: a' = a + gamma^T P
    pos_split, neg_split, active, inactive, unstable = relu_cases(st)
    l, u = st.l, st.u
    with np.errstate(divide="ignore", invalid="ignore"):
        chord = np.where(unstable, u / (u - l), 0.0)
        icpt = np.where(unstable, -u * l / (u - l), 0.0)
    alpha = np.broadcast_to(np.asarray(alpha, dtype=np.float64), (R, d))
    D = np.zeros((R, d))
    D[:, pos_split | active] = 1.0
    neg = ap < 0
    unst = np.broadcast_to(unstable, (R, d))
    D = np.where(unst & ~neg, alpha, D)
    D = np.where(unst & neg, np.broadcast_to(chord, (R, d)), D)
    bl = np.where(unst & neg, np.broadcast_to(icpt, (R, d)), 0.0)
    beta = np.asarray(beta, dtype=np.float64)
    ahat = ap * D + st.S * beta + gPh             # steps 2 and 3
    dc = np.sum(ap * bl, axis=1) - gp
    rec = {"ap": ap, "D": D, "bl": bl, "unstable": unstable, "S": st.S}
    return ahat, dc, rec


def concretize(a0, c, lo, hi, margin=0.0):
    """Eq. 6 over the box: lb = sum_j min(a_j lo_j, a_j hi_j) + c; x*_j = hi_j if a_j < 0 else lo_j.

    With margin > 0, lb is lowered by margin * (sum_j |a_j| max(|lo_j|, |hi_j|) + |c|)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    lb = np.sum(np.minimum(a0 * lo, a0 * hi), axis=1) + c
    if margin:
        lb = lb - margin * (np.abs(a0) @ np.maximum(np.abs(lo), np.abs(hi)) + np.abs(c))
    xstar = np.where(a0 < 0, hi, lo)
    return lb, xstar


def backsub(net, start, c0, states, params, mncs=None, lo=None, hi=None, margin=0.0):
    """Back-substitute rows from `start` down to the input and concretise.

    start  : dict node -> [R, size(node)] coefficients on that node's output
             (for a spec row: the output node; for an intermediate bound of a
             ReLU's input: the node feeding that ReLU)
    c0     : [R] constant terms
    states : dict relu-node -> ReluState
    params : dict relu-node -> dict(alpha=, beta=, gamma=)
    mncs   : dict relu-node -> Mnc (optional)
    margin : rounding margin of the concretisation (see concretize)
    Returns dict(lb, xstar, a0, c, records) with records[relu-node] as in relu_backsub.
    """
    mncs = mncs or {}
    coef = {k: np.array(v, dtype=np.float64) for k, v in start.items()}
    c = np.array(c0, dtype=np.float64)
    records = {}
    for i in range(len(net.nodes) - 1, 0, -1):
        if i not in coef:
            continue
        a = coef.pop(i)
        n = net.nodes[i]
        kind = n["kind"]
        if kind in AFFINE_KINDS:
            c = c + a @ bias_vector(net, i)            # Eq. 2 constant
            _accumulate(coef, n["src"], affine_adjoint(net, i, a))
        elif kind == "relu":
            p = params[i]
            ahat, dc, rec = relu_backsub(a, states[i], p["alpha"], p["beta"],
                                         mncs.get(i), p.get("gamma"))
            c = c + dc
            records[i] = rec
            _accumulate(coef, n["src"], ahat)
        elif kind == "add":
            _accumulate(coef, n["src"], a)
            _accumulate(coef, n["src2"], a)
        else:
            raise ValueError(kind)
    a0 = coef.pop(0)
    out = {"a0": a0, "c": c, "records": records}
    if lo is not None:
        out["lb"], out["xstar"] = concretize(a0, c, lo, hi, margin)
    return out


def _accumulate(coef, node, val):
    if node in coef:
        coef[node] = coef[node] + val
    else:
        coef[node] = val


# --------------------------------------------------------------------------- objectives
def spec_start(net, C):
    """Start rows of the spec objective: the property encoded as an extra affine layer on the output."""
    return {len(net.nodes) - 1: np.asarray(C, dtype=np.float64)}


def neuron_start(net, relu_node, js, sign):
    """Start rows +e_j (lower bound, sign=+1) or -e_j (upper bound, sign=-1) on the input of a ReLU."""
    src = net.nodes[relu_node]["src"]
    d = net.sizes[src]
    E = np.zeros((len(js), d))
    E[np.arange(len(js)), np.asarray(js, dtype=np.int64)] = float(sign)
    return {src: E}


def default_params(net, states, alpha_of=None, mncs=None):
    """beta = 0, gamma = 0 and the given alpha (default: heuristic) for every ReLU node."""
    mncs = mncs or {}
    out = {}
    for i in net.relus:
        st = states.get(i)
        if st is None:
            continue
        alpha = heuristic_alpha(st) if alpha_of is None else alpha_of[i]
        e = mncs[i].e if i in mncs else 0
        out[i] = {"alpha": alpha, "beta": np.zeros(st.l.shape), "gamma": np.zeros(e)}
    return out


def heuristic_alpha(st: ReluState):
    """Lower-slope heuristic (DeepPoly's area rule): alpha_j = 1 if u_j > -l_j else 0."""
    return np.where(st.u > -st.l, 1.0, 0.0)
