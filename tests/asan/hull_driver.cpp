// Host-side driver of the library's ReLU-hull code for a sanitizer build (tests/test_host_asan.py):
// random octahedral polytopes, the constraints of their ReLU-graph hull, each checked on the
// hull's own points.  Exits non-zero on a violated constraint.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2205_00263_amd/csrc/hull.h"

int main() {
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> U(-1.0, 1.0), W(0.05, 1.0);
    int total = 0;
    for (int g = 0; g < 300; ++g) {
        // a box around a random centre, cut by every octahedral direction at a random depth
        double c[3], h[3];
        for (int t = 0; t < 3; ++t) {
            c[t] = 0.5 * U(rng);
            h[t] = W(rng);
        }
        double lb[26];
        for (int d = 0; d < 26; ++d) {
            double lo = 0.0;   // min of s . v over the box
            for (int t = 0; t < 3; ++t) lo += mnb::kOctDirs[d][t] * c[t] - std::abs(mnb::kOctDirs[d][t]) * h[t];
            const int nz = std::abs(mnb::kOctDirs[d][0]) + std::abs(mnb::kOctDirs[d][1]) + std::abs(mnb::kOctDirs[d][2]);
            lb[d] = nz > 1 ? lo + 0.3 * W(rng) * h[0] : lo;   // tighter than the box for mixed directions
        }
        std::vector<std::vector<double>> pts;
        mnb::relu_hull_points(lb, &pts);
        std::vector<mnb::GroupConstraint> cons;
        mnb::relu_hull_constraints(lb, 200, &cons);
        for (const auto& k : cons)
            for (const auto& x : pts) {
                double v = 0.0;
                for (int t = 0; t < 3; ++t) v += k.Phat[t] * x[t] + k.P[t] * x[3 + t];
                if (v > k.p + 1e-9 * (1.0 + std::abs(k.p))) {
                    std::printf("violated: group %d value %.17g offset %.17g\n", g, v, k.p);
                    return 1;
                }
            }
        total += (int)cons.size();
    }
    std::printf("ok %d constraints\n", total);
    return 0;
}
