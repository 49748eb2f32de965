"""Exact minimum by activation-pattern enumeration (oracle; test infrastructure only).

Completeness argument of Section 3.3: once every ReLU is fixed to a phase the
network is affine, so the exact minimum of the objective over a subdomain is
the minimum, over all activation patterns consistent with the subdomain's
splits, of an LP over the input box with the pattern's sign constraints.
Exponential; for nets with at most ~12 free ReLUs.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize

from .net import AFFINE_KINDS, affine_apply, bias_vector


def _affine_of_pattern(net, pattern):
    """Every node value as an affine map A x + c of the input, given ReLU phases."""
    d0 = net.sizes[0]
    maps = [(np.eye(d0), np.zeros(d0))]
    for i in range(1, len(net.nodes)):
        n = net.nodes[i]
        k = n["kind"]
        if k in AFFINE_KINDS:
            A, c = maps[n["src"]]
            maps.append((affine_apply(net, i, A.T).T, affine_apply(net, i, c[None, :])[0] + bias_vector(net, i)))
        elif k == "relu":
            A, c = maps[n["src"]]
            on = pattern[i].astype(np.float64)
            maps.append((A * on[:, None], c * on))
        elif k == "add":
            A1, c1 = maps[n["src"]]
            A2, c2 = maps[n["src2"]]
            maps.append((A1 + A2, c1 + c2))
    return maps


def exact_min(net, lo, hi, start, c0=0.0, S=None, max_free=14):
    """Exact min over {x in box, split constraints} of sum_node start[node] . v_node + c0.

    S: optional dict relu-node -> split diagonal (-1 positive, +1 negative, 0 free).
    Returns (value, minimiser x) or (inf, None) if the subdomain is empty.
    """
    S = S or {}
    free = []
    fixed = {}
    for i in net.relus:
        s = np.asarray(S.get(i, np.zeros(net.sizes[i], dtype=np.int64)))
        fixed[i] = s
        free += [(i, j) for j in range(net.sizes[i]) if s[j] == 0]
    if len(free) > max_free:
        raise ValueError(f"{len(free)} free ReLUs: too many to enumerate")
    best, best_x = np.inf, None
    bounds = list(zip(np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)))
    for bits in itertools.product((0, 1), repeat=len(free)):
        pattern = {i: (fixed[i] == -1).astype(np.int64) for i in net.relus}
        for (i, j), b in zip(free, bits):
            pattern[i][j] = b
        maps = _affine_of_pattern(net, pattern)
        rows, rhs = [], []
        for i in net.relus:
            A, c = maps[net.nodes[i]["src"]]
            for j in range(net.sizes[i]):
                if pattern[i][j]:      # zhat >= 0  ->  -A x <= c
                    rows.append(-A[j]); rhs.append(c[j])
                else:                  # zhat <= 0  ->  A x <= -c
                    rows.append(A[j]); rhs.append(-c[j])
        obj = np.zeros(net.sizes[0])
        const = float(c0)
        for node, coef in start.items():
            A, c = maps[node]
            coef = np.asarray(coef, dtype=np.float64).ravel()
            obj += coef @ A
            const += float(coef @ c)
        res = scipy.optimize.linprog(obj, A_ub=np.array(rows) if rows else None,
                                     b_ub=np.array(rhs) if rhs else None,
                                     bounds=bounds, method="highs")
        if res.status == 0 and res.fun + const < best:
            best, best_x = res.fun + const, res.x
    return best, best_x
