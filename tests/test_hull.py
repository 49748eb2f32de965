"""The library's constraint generator (host code, no GPU): the exact 3-neuron ReLU hull over an
octahedral polytope, computed by double description in mnb_relu_hull, against the oracle's hull
(scipy's Qhull over the same points, oracle/mnc.py) and against what the hull must satisfy."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import mnc as omnc
from oracle import net as onet
from oracle import optimize as oo

LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2205_00263_amd",
                   "libmnbab.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _groups(cfg, per_layer=3):
    # the small residual net is nearly stable at its own radius: a wider box gives it unstable groups
    wl = W.make_workload(cfg, scale="small", eps=0.05 if cfg == 4 else None)
    net = onet.Net(wl.nodes)
    root, _ = oo.root_pass(oo.Query(net, wl.lo, wl.hi, wl.C, wl.c0))
    for i in net.relus:
        for g in omnc.make_groups(root.states[i])[:per_layer]:
            yield omnc.octahedral_bounds(net, root.states, i, g, wl.lo, wl.hi)


def _close(x, Y, tol=1e-6):
    return len(Y) > 0 and np.min(np.abs(Y - x).max(1)) <= tol * (1.0 + np.abs(x).max())


def _is_facet(x, pts):
    """The hyperplane of constraint x = (Phat, P, p) holds on every point and touches points that span
    five dimensions (a facet of the 6-dimensional hull)."""
    n, b = x[:6], x[6]
    v = pts @ n
    scale = 1.0 + np.abs(b)
    tight = pts[np.abs(v - b) <= 1e-7 * scale]
    return np.all(v <= b + 1e-9 * scale) and len(tight) >= 6 and \
        np.linalg.matrix_rank(np.hstack([tight, np.ones((len(tight), 1))]), tol=1e-7) == 6


def _multi(x):
    """The constraint involves at least two neurons (coefficients below 1e-4 count as zero: the joggled
    hull's single-neuron facets carry residues of up to ~1e-5)."""
    return int(np.sum((np.abs(x[:3]) > 1e-4) | (np.abs(x[3:6]) > 1e-4))) >= 2


@pytest.mark.parametrize("cfg", [1, 2, 3, 4])
def test_hull_matches_oracle_qhull(cfg):
    """Every library constraint is a facet of the hull (valid, offset attained, touching five
    dimensions' worth of the generating points), and every oracle facet is one of them.  Where Qhull
    handles the points as they are, the two sets are equal (compared within 1e-6: Qhull triangulates
    and may list a facet twice with normals that differ in the 7th digit).  Where Qhull needs its
    joggled mode, the oracle also lists near-facets of the perturbed points (each made valid by its
    forced offset) and single-neuron facets whose normals carry joggling residues, which the exact
    hull does not contain; only its true multi-neuron facets are required."""
    from scipy.spatial import ConvexHull, QhullError
    from paper_2205_00263_amd import relu_hull
    n_groups = n_plain = 0
    for lb in _groups(cfg):
        pts = omnc.hull_points(lb)
        ref = omnc.hull_facets(pts)
        R = np.array([np.concatenate([a, b, [c]]) for a, b, c in ref]) if ref else np.zeros((0, 7))
        Ph, Pz, p = relu_hull(lb)
        G = np.concatenate([Ph, Pz, p[:, None]], 1)
        assert all(_is_facet(x, pts) for x in G), "a library constraint is not a facet of the hull"
        try:
            ConvexHull(pts)
            plain = True
        except QhullError:
            plain = False
        # joggled normals deviate by up to ~1e-5 from the facets they stand for
        assert all(_close(x, G, 1e-6 if plain else 1e-4) for x in R if _is_facet(x, pts) and _multi(x)), \
            "an oracle facet is missing"
        if plain:
            assert all(_close(x, G) for x in R), "an oracle constraint is missing"
            assert all(_close(x, R) for x in G), "a facet the oracle does not have"
            n_plain += 1
        n_groups += 1
    assert n_groups > 0 and n_plain > 0


def test_hull_constraints_are_valid_and_tight():
    """Every constraint holds on (v, relu(v)) for v sampled in Q (rejection sampling in its bounding box)
    and is attained at a vertex point (offset = max over the generating points)."""
    from paper_2205_00263_amd import relu_hull
    dirs = omnc.DIRS
    rng = np.random.default_rng(3)
    checked = 0
    for lb in _groups(3, per_layer=2):
        Ph, Pz, p = relu_hull(lb)
        if len(p) == 0:
            continue
        e = {tuple(s): k for k, s in enumerate(dirs.astype(int))}
        lo = np.array([lb[e[(1, 0, 0)]], lb[e[(0, 1, 0)]], lb[e[(0, 0, 1)]]])
        hi = -np.array([lb[e[(-1, 0, 0)]], lb[e[(0, -1, 0)]], lb[e[(0, 0, -1)]]])
        V = rng.uniform(lo, hi, size=(20000, 3))
        V = V[np.all(V @ dirs.T >= lb - 1e-12, axis=1)]
        X = np.maximum(V, 0.0)
        lhs = V @ Ph.T + X @ Pz.T
        assert np.all(lhs <= p + 1e-9 * (1 + np.abs(p))), "a constraint cuts off a point of the ReLU graph"
        pts = omnc.hull_points(lb)
        att = pts[:, :3] @ Ph.T + pts[:, 3:] @ Pz.T
        np.testing.assert_allclose(att.max(0), p, rtol=0, atol=1e-9 * (1 + np.abs(p).max()))
        checked += 1
    assert checked > 0


def test_hull_over_a_box_adds_nothing():
    """Over a box the hull of the ReLU graph is the product of the single-neuron triangles: every facet
    involves one neuron, so no constraint is produced."""
    from paper_2205_00263_amd import relu_hull
    l, u = np.array([-1.0, -0.5, -2.0]), np.array([2.0, 1.5, 0.7])
    lb = np.array([np.sum(np.where(s > 0, s * l, s * u)) for s in omnc.DIRS])
    Ph, Pz, p = relu_hull(lb)
    assert len(p) == 0


def test_hull_rejects_non_finite_bounds():
    from paper_2205_00263_amd import relu_hull
    from paper_2205_00263_amd._lib import MnbError
    lb = np.zeros(26)
    lb[3] = np.inf
    with pytest.raises(MnbError):
        relu_hull(lb)
