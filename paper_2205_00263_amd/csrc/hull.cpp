// Host-side convex hull of the 3-neuron ReLU graph, the constraint generator behind the
// multi-neuron constraints of Eq. 3 (the paper takes them from PRIMA; here they are the exact
// hull over an octahedral input polytope, see hull.h).
//
// Facets come from the double description method (Motzkin's incremental algorithm): the valid
// inequalities a . x <= b of conv(X) form the cone K = {(a, b) : a . x_i - b <= 0 for all i}, whose
// extreme rays are the facets of conv(X) plus the trivial (0, 1).  Starting from the simplicial
// cone of d = D+1 linearly independent constraints, each further constraint h splits the rays into
// R+ (violating), R0 and R-; the new cone keeps R0 and R- and adds one ray on h for every adjacent
// pair (p in R+, n in R-).  Adjacency is the combinatorial test on the sets of tight constraints:
// p and n are adjacent iff no third ray is tight on every constraint both are tight on (and those
// are at least d - 2).  Degenerate inputs (many coplanar points, as here) need no special care.
#include "hull.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <set>
#include <tuple>

namespace mnb {

const int kOctDirs[26][3] = {
    {-1, -1, -1}, {-1, -1, 0}, {-1, -1, 1}, {-1, 0, -1}, {-1, 0, 0}, {-1, 0, 1}, {-1, 1, -1}, {-1, 1, 0},
    {-1, 1, 1},   {0, -1, -1}, {0, -1, 0},  {0, -1, 1},  {0, 0, -1}, {0, 0, 1},  {0, 1, -1},  {0, 1, 0},
    {0, 1, 1},    {1, -1, -1}, {1, -1, 0},  {1, -1, 1},  {1, 0, -1}, {1, 0, 0},  {1, 0, 1},   {1, 1, -1},
    {1, 1, 0},    {1, 1, 1}};

namespace {

using Bits = std::vector<uint64_t>;

inline bool subset_of(const Bits& a, const Bits& b) {   // a is a subset of b
    for (size_t w = 0; w < a.size(); ++w)
        if (a[w] & ~b[w]) return false;
    return true;
}
inline int popcount(const Bits& a) {
    int c = 0;
    for (uint64_t w : a) c += __builtin_popcountll(w);
    return c;
}
inline void set_bit(Bits& a, int i) { a[i >> 6] |= 1ull << (i & 63); }

struct Ray {
    std::vector<double> y;
    Bits z;
};

void normalize(std::vector<double>& y) {
    double m = 0.0;
    for (double v : y) m = std::max(m, std::fabs(v));
    if (m > 0.0)
        for (double& v : y) v /= m;
}

// Inverse of a d x d matrix by Gauss-Jordan elimination with partial pivoting.
bool invert(std::vector<std::vector<double>> M, std::vector<std::vector<double>>* inv) {
    const int d = (int)M.size();
    std::vector<std::vector<double>> I(d, std::vector<double>(d, 0.0));
    for (int i = 0; i < d; ++i) I[i][i] = 1.0;
    for (int c = 0; c < d; ++c) {
        int piv = c;
        for (int r = c + 1; r < d; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (std::fabs(M[piv][c]) < 1e-14) return false;
        std::swap(M[c], M[piv]);
        std::swap(I[c], I[piv]);
        const double f = 1.0 / M[c][c];
        for (int k = 0; k < d; ++k) {
            M[c][k] *= f;
            I[c][k] *= f;
        }
        for (int r = 0; r < d; ++r) {
            if (r == c || M[r][c] == 0.0) continue;
            const double g = M[r][c];
            for (int k = 0; k < d; ++k) {
                M[r][k] -= g * M[c][k];
                I[r][k] -= g * I[c][k];
            }
        }
    }
    *inv = I;
    return true;
}

}  // namespace

bool hull_facets(const std::vector<std::vector<double>>& pts, int D, std::vector<std::vector<double>>* normals,
                 std::vector<double>* offsets) {
    normals->clear();
    offsets->clear();
    const int n = (int)pts.size(), d = D + 1;
    if (D < 1 || D > 8 || n < d) return false;
    // points moved into a unit box (the facet directions do not change)
    std::vector<double> lo(D, INFINITY), hi(D, -INFINITY);
    for (const auto& p : pts)
        for (int k = 0; k < D; ++k) {
            lo[k] = std::min(lo[k], p[k]);
            hi[k] = std::max(hi[k], p[k]);
        }
    double span = 0.0;
    for (int k = 0; k < D; ++k) span = std::max(span, hi[k] - lo[k]);
    if (!(span > 0.0) || !std::isfinite(span)) return false;
    std::vector<std::vector<double>> A(n, std::vector<double>(d));
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < D; ++k) A[i][k] = (pts[i][k] - 0.5 * (lo[k] + hi[k])) / span;
        A[i][D] = -1.0;
    }
    auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) s += a[k] * b[k];
        return s;
    };
    // d linearly independent constraints (Gram-Schmidt on the rows, in order)
    std::vector<int> basis;
    std::vector<std::vector<double>> Q;
    for (int i = 0; i < n && (int)basis.size() < d; ++i) {
        std::vector<double> v = A[i];
        for (int pass = 0; pass < 2; ++pass)
            for (const auto& q : Q) {
                const double c = dot(v, q);
                for (int k = 0; k < d; ++k) v[k] -= c * q[k];
            }
        const double nv = std::sqrt(dot(v, v)), na = std::sqrt(dot(A[i], A[i]));
        if (nv > 1e-9 * na) {
            for (double& x : v) x /= nv;
            Q.push_back(v);
            basis.push_back(i);
        }
    }
    if ((int)basis.size() < d) return false;   // the points lie in a hyperplane
    std::vector<std::vector<double>> B(d), inv;
    for (int j = 0; j < d; ++j) B[j] = A[basis[j]];
    if (!invert(B, &inv)) return false;
    const int words = (n + 63) / 64;
    std::vector<Ray> rays;
    for (int j = 0; j < d; ++j) {
        Ray r;
        r.y.resize(d);
        for (int k = 0; k < d; ++k) r.y[k] = -inv[k][j];   // A_B y = -e_j
        normalize(r.y);
        r.z.assign(words, 0);
        for (int t = 0; t < d; ++t)
            if (t != j) set_bit(r.z, basis[t]);
        rays.push_back(std::move(r));
    }
    std::vector<char> in_basis(n, 0);
    for (int b : basis) in_basis[b] = 1;
    const double tol = 1e-9;
    std::vector<double> val;
    std::vector<int> plus, minus, zero;
    for (int h = 0; h < n; ++h) {
        if (in_basis[h]) continue;
        val.resize(rays.size());
        plus.clear();
        minus.clear();
        zero.clear();
        for (size_t r = 0; r < rays.size(); ++r) {
            val[r] = dot(A[h], rays[r].y);
            if (val[r] > tol)
                plus.push_back((int)r);
            else if (val[r] < -tol)
                minus.push_back((int)r);
            else
                zero.push_back((int)r);
        }
        if (plus.empty()) {
            for (int r : zero) set_bit(rays[r].z, h);
            continue;
        }
        std::vector<Ray> next;
        next.reserve(minus.size() + zero.size() + plus.size() * 2);
        for (int p : plus)
            for (int m : minus) {
                Bits common(words);
                for (int w = 0; w < words; ++w) common[w] = rays[p].z[w] & rays[m].z[w];
                if (popcount(common) < d - 2) continue;
                bool adjacent = true;
                for (size_t r = 0; r < rays.size() && adjacent; ++r)
                    if ((int)r != p && (int)r != m && subset_of(common, rays[r].z)) adjacent = false;
                if (!adjacent) continue;
                Ray nr;
                nr.y.resize(d);
                for (int k = 0; k < d; ++k) nr.y[k] = val[p] * rays[m].y[k] - val[m] * rays[p].y[k];
                normalize(nr.y);
                nr.z = common;
                set_bit(nr.z, h);
                next.push_back(std::move(nr));
            }
        for (int m : minus) next.push_back(std::move(rays[m]));
        for (int r : zero) {
            set_bit(rays[r].z, h);
            next.push_back(std::move(rays[r]));
        }
        rays.swap(next);
    }
    for (const Ray& r : rays) {
        std::vector<double> a(r.y.begin(), r.y.begin() + D);
        double m = 0.0;
        for (double v : a) m = std::max(m, std::fabs(v));
        if (m < 1e-9) continue;   // the trivial inequality 0 <= b
        for (double& v : a) {
            v /= m;
            if (std::fabs(v) < 1e-9) v = 0.0;   // rounding residue of the ray combinations
        }
        double b = -INFINITY;
        for (const auto& p : pts) {
            double s = 0.0;
            for (int k = 0; k < D; ++k) s += a[k] * p[k];
            b = std::max(b, s);
        }
        normals->push_back(a);
        offsets->push_back(b);
    }
    return true;
}

namespace {

double det3(const double M[3][3]) {
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

// Vertices of {v in R^3 : A v <= b} from every triple of planes, deduplicated at 1e-12.
void polytope_vertices(const std::vector<std::array<double, 3>>& A, const std::vector<double>& b,
                       std::vector<std::array<double, 3>>* out) {
    const int m = (int)A.size();
    std::set<std::array<long long, 3>> seen;
    for (int i = 0; i < m; ++i)
        for (int j = i + 1; j < m; ++j)
            for (int k = j + 1; k < m; ++k) {
                const double M[3][3] = {{A[i][0], A[i][1], A[i][2]},
                                        {A[j][0], A[j][1], A[j][2]},
                                        {A[k][0], A[k][1], A[k][2]}};
                const double rhs[3] = {b[i], b[j], b[k]};
                const double det = det3(M);
                if (std::fabs(det) < 1e-12) continue;
                std::array<double, 3> v;
                for (int col = 0; col < 3; ++col) {   // Cramer's rule
                    double Mc[3][3];
                    for (int r = 0; r < 3; ++r)
                        for (int c = 0; c < 3; ++c) Mc[r][c] = c == col ? rhs[r] : M[r][c];
                    v[col] = det3(Mc) / det;
                }
                bool ok = true;
                for (int t = 0; t < m && ok; ++t)
                    ok = A[t][0] * v[0] + A[t][1] * v[1] + A[t][2] * v[2] <= b[t] + 1e-9 * (1.0 + std::fabs(b[t]));
                if (!ok) continue;
                std::array<long long, 3> key;
                for (int t = 0; t < 3; ++t) key[t] = std::llround(v[t] * 1e12);
                if (seen.insert(key).second) out->push_back(v);
            }
}

}  // namespace

void relu_hull_points(const double lb[26], std::vector<std::vector<double>>* out) {
    out->clear();
    for (int s = 0; s < 26; ++s)
        if (!std::isfinite(lb[s])) return;
    // Q: s . v >= lb_s, i.e. -s . v <= -lb_s
    std::vector<std::array<double, 3>> A0(26);
    std::vector<double> b0(26);
    for (int s = 0; s < 26; ++s) {
        for (int t = 0; t < 3; ++t) A0[s][t] = -(double)kOctDirs[s][t];
        b0[s] = -lb[s];
    }
    std::set<std::array<long long, 6>> seen;
    for (int o = 0; o < 8; ++o) {
        const double sg[3] = {(o & 4) ? 1.0 : -1.0, (o & 2) ? 1.0 : -1.0, (o & 1) ? 1.0 : -1.0};
        std::vector<std::array<double, 3>> A = A0;
        std::vector<double> b = b0;
        for (int t = 0; t < 3; ++t) {   // orthant: sg_t v_t >= 0
            std::array<double, 3> row{0.0, 0.0, 0.0};
            row[t] = -sg[t];
            A.push_back(row);
            b.push_back(0.0);
        }
        std::vector<std::array<double, 3>> V;
        polytope_vertices(A, b, &V);
        for (const auto& v : V) {
            std::vector<double> p = {v[0], v[1], v[2], std::max(v[0], 0.0), std::max(v[1], 0.0), std::max(v[2], 0.0)};
            std::array<long long, 6> key;
            for (int t = 0; t < 6; ++t) key[t] = std::llround(p[t] * 1e12);
            if (seen.insert(key).second) out->push_back(p);
        }
    }
}

void relu_hull_constraints(const double lb[26], int max_out, std::vector<GroupConstraint>* out) {
    if (max_out <= 0) return;
    std::vector<std::vector<double>> pts;
    relu_hull_points(lb, &pts);
    if (pts.size() < 7) return;
    std::vector<std::vector<double>> nrm;
    std::vector<double> off;
    if (!hull_facets(pts, 6, &nrm, &off)) return;
    // distinct facets in a canonical order (normals rounded to 1e-7), single-neuron ones dropped
    std::vector<std::tuple<std::array<long long, 6>, int>> keys;
    for (size_t f = 0; f < nrm.size(); ++f) {
        std::array<long long, 6> key;
        for (int t = 0; t < 6; ++t) key[t] = std::llround(nrm[f][t] * 1e7);
        keys.emplace_back(key, (int)f);
    }
    std::sort(keys.begin(), keys.end());
    for (size_t i = 0; i < keys.size() && (int)out->size() < max_out; ++i) {
        if (i > 0 && std::get<0>(keys[i]) == std::get<0>(keys[i - 1])) continue;
        const auto& a = nrm[std::get<1>(keys[i])];
        int support = 0;
        for (int t = 0; t < 3; ++t) support += (std::fabs(a[t]) > 1e-12 || std::fabs(a[3 + t]) > 1e-12) ? 1 : 0;
        if (support <= 1) continue;
        GroupConstraint g;
        for (int t = 0; t < 3; ++t) {
            g.Phat[t] = a[t];
            g.P[t] = a[3 + t];
        }
        g.p = off[std::get<1>(keys[i])];
        out->push_back(g);
    }
}

}  // namespace mnb
