"""Multi-neuron constraint generation from the exact 3-neuron ReLU hull (oracle; test infrastructure only).

The paper takes its multi-neuron constraints (Eq. 3) from PRIMA and does not
describe their construction.  This generator produces constraints of the same
form, P z + Phat zhat <= p over groups of three neurons of one ReLU layer,
from the exact convex hull of the ReLU graph over an input polytope:

* the polytope Q is given by octahedral bounds s . zhat >= lb_s for the 26
  directions s in {-1,0,1}^3 \\ {0}, each computed by back-substitution with
  the root's (heuristic) parameters;  over a plain box the hull would be the
  product of the single-neuron triangles, so Q must carry these joint bounds;
* relu is linear on each orthant piece of Q, so the hull of the graph is the
  hull of the points (v, relu(v)) over the vertices v of Q intersected with
  each orthant;
* facets come from Qhull in 6-D; each facet's offset is reset to the maximum
  of the facet over the generating points, which makes it valid however
  Qhull rounds;
* facets that involve a single neuron only are dropped (the triangle already
  implies them), and at most `cap` constraints per layer are kept.

Groups: unstable neurons sorted by the triangle height -l u / (u - l),
largest first (ties by index), split into consecutive disjoint triples.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.spatial import ConvexHull, QhullError

from .backsub import Mnc, backsub, heuristic_alpha

DIRS = np.array([s for s in itertools.product((-1, 0, 1), repeat=3) if any(s)], dtype=np.float64)


def octahedral_bounds(net, states, relu_node, group, lo, hi):
    """lb_s of s . zhat over the group for the 26 directions (root parameters)."""
    src = net.nodes[relu_node]["src"]
    d = net.sizes[src]
    E = np.zeros((len(DIRS), d))
    E[:, group] = DIRS
    params = {k: {"alpha": heuristic_alpha(s), "beta": np.zeros(s.l.shape)}
              for k, s in states.items() if k < relu_node}
    out = backsub(net, {src: E}, np.zeros(len(DIRS)), states, params, None, lo, hi)
    return out["lb"]


def polytope_vertices(A, b, tol=1e-9):
    """Vertices of {x in R^3 : A x <= b} by enumerating triples of planes."""
    verts = []
    for i, j, k in itertools.combinations(range(len(A)), 3):
        M = A[[i, j, k]]
        if abs(np.linalg.det(M)) < 1e-12:
            continue
        v = np.linalg.solve(M, b[[i, j, k]])
        if np.all(A @ v <= b + tol * (1 + np.abs(b))):
            verts.append(v)
    if not verts:
        return np.zeros((0, 3))
    V = np.unique(np.round(np.array(verts), 12), axis=0)
    return V


def hull_points(lb):
    """Points (zhat, relu(zhat)) over the vertices of every orthant piece of Q."""
    A0 = -DIRS
    b0 = -np.asarray(lb)
    pts = []
    for o in itertools.product((-1.0, 1.0), repeat=3):
        A = np.vstack([A0, -np.diag(o)])
        b = np.concatenate([b0, np.zeros(3)])
        V = polytope_vertices(A, b)
        for v in V:
            pts.append(np.concatenate([v, np.maximum(v, 0.0)]))
    if not pts:
        return np.zeros((0, 6))
    return np.unique(np.round(np.array(pts), 12), axis=0)


def hull_facets(pts):
    """Facets (Phat [3], P [3], p) of conv(pts) with offsets forced to be valid."""
    if len(pts) < 7:
        return []
    try:
        hull = ConvexHull(pts)
    except QhullError:
        try:
            hull = ConvexHull(pts, qhull_options="QJ")
        except QhullError:
            return []
    seen = set()
    out = []
    for eq in hull.equations:
        nrm = eq[:6]
        scale = np.max(np.abs(nrm))
        if scale == 0:
            continue
        nrm = nrm / scale
        key = tuple(np.round(nrm, 7))
        if key in seen:
            continue
        seen.add(key)
        Phat, P = nrm[:3], nrm[3:]
        p = float(np.max(pts @ nrm))         # sound offset: max over generating points
        support = [t for t in range(3) if abs(Phat[t]) > 1e-12 or abs(P[t]) > 1e-12]
        if len(support) <= 1:
            continue
        out.append((Phat, P, p))
    return out


def make_groups(st, max_groups=None):
    uns = np.nonzero((st.l < 0) & (st.u > 0))[0]
    height = -st.l[uns] * st.u[uns] / (st.u[uns] - st.l[uns])
    order = sorted(range(len(uns)), key=lambda t: (-height[t], uns[t]))
    idx = [int(uns[t]) for t in order]
    groups = [idx[g:g + 3] for g in range(0, len(idx) - 2, 3)]
    if max_groups is not None:
        groups = groups[:max_groups]
    return groups


def generate(net, states, lo, hi, cap=500, layers=None, max_groups=None):
    """MNC sets for every ReLU layer (dict relu-node -> Mnc), from the root bounds `states`."""
    mncs = {}
    for m, i in enumerate(net.relus):
        if layers is not None and m not in layers:
            continue
        d = net.sizes[i]
        rows = []
        for grp in make_groups(states[i], max_groups):
            if len(rows) >= cap:
                break
            lb = octahedral_bounds(net, states, i, grp, lo, hi)
            for Phat, P, p in hull_facets(hull_points(lb)):
                if len(rows) >= cap:
                    break
                rows.append((grp, Phat, P, p))
        e = len(rows)
        Pm = np.zeros((e, d)); Ph = np.zeros((e, d)); pv = np.zeros(e)
        for r, (grp, Phat, P, p) in enumerate(rows):
            Pm[r, grp] = P
            Ph[r, grp] = Phat
            pv[r] = p
        mncs[i] = Mnc(Pm, Ph, pv)
    return mncs
