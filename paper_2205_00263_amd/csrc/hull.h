// Host-side convex hull of the 3-neuron ReLU graph (multi-neuron constraints, Eq. 3).
#pragma once

#include <array>
#include <vector>

namespace mnb {

// The 26 directions s in {-1,0,1}^3 \ {0} of the octahedral bounds s . zhat >= lb_s, in
// lexicographic order of (s0, s1, s2) with -1 < 0 < 1.
extern const int kOctDirs[26][3];

// One constraint  Phat . zhat + P . z <= p  over a group of three neurons.
struct GroupConstraint {
    double Phat[3], P[3], p;
};

// Facets a . x <= b of the convex hull of `pts` (points of R^D, D <= 8) by the double description
// method, with the normals scaled to max |a_i| = 1 (entries below 1e-9 set to 0) and b = max over
// the points of a . x (valid whatever the rounding).  Returns false (and no facets) when the
// points do not span R^D.
bool hull_facets(const std::vector<std::vector<double>>& pts, int D, std::vector<std::vector<double>>* normals,
                 std::vector<double>* offsets);

// The points (v, relu(v)) over the vertices v of Q intersected with each orthant (below),
// deduplicated at 1e-12; empty if a bound is not finite.
void relu_hull_points(const double lb[26], std::vector<std::vector<double>>* pts);

// Constraints of the exact convex hull of {(v, relu(v)) : v in Q} for the polytope
// Q = {v in R^3 : s . v >= lb_s for the 26 directions s}: relu is linear on each orthant, so the
// hull is that of the points (v, relu(v)) over the vertices v of Q intersected with each orthant.
// Facets that involve a single neuron are dropped (its triangle relaxation already implies them).
// At most max_out constraints are appended to out, in the lexicographic order of their normals.
void relu_hull_constraints(const double lb[26], int max_out, std::vector<GroupConstraint>* out);

}  // namespace mnb
