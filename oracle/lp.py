"""LP of the relaxation that back-substitution dualises (oracle; test infrastructure only).

Section 2.5 and the weak-duality step of Section 3.1: the back-substitution
bound with any feasible (alpha, beta, gamma) is a lower bound of the LP that
keeps, with the same intermediate bounds l/u,

* the affine layers as equalities,
* per unstable ReLU the triangle  z >= 0,  z >= zhat,  z <= u (zhat - l)/(u - l),
* stable / split ReLUs as z = zhat (active or positive split) or z = 0,
  and the split rows  -zhat <= 0 (positive) / zhat <= 0 (negative)  of Eq. 4,
* the multi-neuron rows  P z + Phat zhat <= p  of Eq. 3,
* the input box.

By LP strong duality the best per-row (alpha, beta, gamma) reaches the LP
value; `lp_bound` also maps the LP duals to such parameters
(alpha_j = lambda(z >= zhat) / (lambda(z >= 0) + lambda(z >= zhat)),
beta = split-row duals, gamma = MNC-row duals).  scipy's HiGHS solves it.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize
import scipy.sparse as sp

from .backsub import relu_cases
from .net import AFFINE_KINDS, affine_apply, bias_vector


def _affine_matrix(net, i):
    """Dense matrix of the linear part of affine node i (built column by column)."""
    n = net.nodes[i]
    if n["kind"] == "fc":
        return n["W"]
    d_in = net.sizes[n["src"]]
    return affine_apply(net, i, np.eye(d_in)).T


def lp_bound(net, states, mncs, lo, hi, start, c0=0.0, upto=None):
    """min over the LP of  sum_node start[node] . v_node + c0.

    start: dict node -> coefficient vector [size] (one objective row).
    Returns dict(value, x, params) where params[relu-node] = dict(alpha, beta, gamma)
    is the dual-derived parameter set (per-row parameters for this row).
    """
    mncs = mncs or {}
    top = max(start) if upto is None else upto
    offs = np.cumsum([0] + net.sizes[: top + 1])
    nvar = int(offs[-1])
    eq_rows, eq_b = [], []
    ub_rows, ub_b, ub_tag = [], [], []

    def row(entries):
        r = sp.lil_matrix((1, nvar))
        for idx, val in entries:
            r[0, idx] += val
        return r

    for i in range(1, top + 1):
        n = net.nodes[i]
        k = n["kind"]
        o, d = int(offs[i]), net.sizes[i]
        if k in AFFINE_KINDS:
            A = _affine_matrix(net, i)
            os_ = int(offs[n["src"]])
            blk = sp.lil_matrix((d, nvar))
            blk[:, o:o + d] = sp.identity(d)
            blk[:, os_:os_ + A.shape[1]] = -A
            eq_rows.append(blk.tocsr())
            eq_b.append(bias_vector(net, i))
        elif k == "add":
            o1, o2 = int(offs[n["src"]]), int(offs[n["src2"]])
            blk = sp.lil_matrix((d, nvar))
            blk[:, o:o + d] = sp.identity(d)
            blk[:, o1:o1 + d] = -sp.identity(d)
            blk[:, o2:o2 + d] = -sp.identity(d)
            eq_rows.append(blk.tocsr())
            eq_b.append(np.zeros(d))
        elif k == "relu":
            st = states[i]
            os_ = int(offs[n["src"]])
            pos, neg, act, ina, uns = relu_cases(st)
            for j in range(d):
                z, zh = o + j, os_ + j
                if pos[j] or act[j]:
                    eq_rows.append(row([(z, 1.0), (zh, -1.0)]).tocsr()); eq_b.append([0.0])
                    if pos[j]:
                        ub_rows.append(row([(zh, -1.0)])); ub_b.append(0.0); ub_tag.append(("split", i, j))
                elif neg[j] or ina[j]:
                    eq_rows.append(row([(z, 1.0)]).tocsr()); eq_b.append([0.0])
                    if neg[j]:
                        ub_rows.append(row([(zh, 1.0)])); ub_b.append(0.0); ub_tag.append(("split", i, j))
                else:
                    l, u = st.l[j], st.u[j]
                    kk = u / (u - l)
                    ub_rows.append(row([(z, -1.0)])); ub_b.append(0.0); ub_tag.append(("lo0", i, j))
                    ub_rows.append(row([(zh, 1.0), (z, -1.0)])); ub_b.append(0.0); ub_tag.append(("lo1", i, j))
                    ub_rows.append(row([(z, 1.0), (zh, -kk)])); ub_b.append(-kk * l); ub_tag.append(("up", i, j))
            if i in mncs and mncs[i].e > 0:
                m = mncs[i]
                for e in range(m.e):
                    ents = [(o + j, m.P[e, j]) for j in np.nonzero(m.P[e])[0]]
                    ents += [(os_ + j, m.Phat[e, j]) for j in np.nonzero(m.Phat[e])[0]]
                    ub_rows.append(row(ents)); ub_b.append(m.p[e]); ub_tag.append(("mnc", i, e))
    cvec = np.zeros(nvar)
    for node, coef in start.items():
        cvec[int(offs[node]):int(offs[node]) + net.sizes[node]] += np.asarray(coef, dtype=np.float64).ravel()
    bounds = [(None, None)] * nvar
    for j in range(net.sizes[0]):
        bounds[j] = (float(lo[j]), float(hi[j]))
    A_eq = sp.vstack(eq_rows).tocsr() if eq_rows else None
    b_eq = np.concatenate([np.atleast_1d(b) for b in eq_b]) if eq_b else None
    A_ub = sp.vstack([r.tocsr() for r in ub_rows]).tocsr() if ub_rows else None
    b_ub = np.asarray(ub_b) if ub_rows else None
    res = scipy.optimize.linprog(cvec, A_ub=A_ub, b_ub=b_ub, A_eq=A_eq, b_eq=b_eq,
                                 bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(f"LP failed: {res.message}")
    value = float(res.fun) + float(c0)
    lam = -np.asarray(res.ineqlin.marginals) if ub_rows else np.zeros(0)
    params = {}
    for i in net.relus:
        if i > top:
            continue
        d = net.sizes[i]
        e = mncs[i].e if i in mncs else 0
        params[i] = {"alpha": np.zeros(d), "beta": np.zeros(d), "gamma": np.zeros(e)}
    lo0 = {}
    lo1 = {}
    for (tag, i, j), lv in zip(ub_tag, lam):
        lv = max(float(lv), 0.0)
        if tag == "split":
            params[i]["beta"][j] = lv
        elif tag == "mnc":
            params[i]["gamma"][j] = lv
        elif tag == "lo0":
            lo0[(i, j)] = lv
        elif tag == "lo1":
            lo1[(i, j)] = lv
    for key, l1 in lo1.items():
        tot = lo0[key] + l1
        params[key[0]]["alpha"][key[1]] = l1 / tot if tot > 0 else 0.0
    return {"value": value, "x": res.x[: net.sizes[0]], "params": params}
