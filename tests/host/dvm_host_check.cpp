// Host driver of the moment-matrix builder (paper_1411_6697_amd/csrc/dvm_host.cpp), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py:
// for the velocity sets of the paper's runs (Secs. IV and VI) the block matrices are built,
// reassembled into the dense 24 x 24 M and M^-1, and M M^-1 is checked against the
// identity; a degenerate set (all three group speeds equal) must be refused as singular.
#include <cmath>
#include <cstdio>

#include "lbkm_internal.h"

int main() {
    const double sets[][6] = {
        {2.5, 2.2, 1.2, 6.5, 3.0, 0.0},    // Sod
        {2.7, 2.2, 1.2, 5.0, 3.0, 1.1},    // steady detonation
        {2.7, 2.2, 1.2, 1.5, 0.5, 5.0},    // unsteady detonation, Kelvin-Helmholtz, batch, adjoint
        {4.7, 3.3, 1.0, 6.0, 2.5, 0.9},    // Lax
        {0.4, 1.0, 1.8, 0.3, 1.9, 1.5},    // Sjogren
        {1.0, 2.7, 2.9, 1.0, 2.9, 0.96},   // shock reflection
        {0.8, 1.2, 1.3, 1.0, 2.7, 0.8},    // Couette velocity
        {0.8, 1.2, 1.3, 1.1, 3.1, 0.7},    // Couette temperature, panel (a)
    };
    const int n = lbkm::NV;
    static double M[lbkm::NV * lbkm::NV], Mi[lbkm::NV * lbkm::NV];
    int failures = 0;
    for (const auto& dvm : sets) {
        lbkm::Consts c{};
        double cond = 0.0;
        const int r = lbkm::build_moment_blocks(dvm, &c, &cond);
        if (r != 0) {
            std::printf("set (%g %g %g %g %g %g): build returned %d\n", dvm[0], dvm[1], dvm[2], dvm[3], dvm[4],
                        dvm[5], r);
            ++failures;
            continue;
        }
        lbkm::dense_from_blocks(&c, M, Mi);
        double worst = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                long double s = 0.0L;
                for (int k = 0; k < n; ++k) s += (long double)M[i * n + k] * Mi[k * n + j];
                worst = std::fmax(worst, std::fabs((double)s - (i == j ? 1.0 : 0.0)));
            }
        std::printf("set (%g %g %g %g %g %g): cond %.3g, max |M M^-1 - I| %.3g\n", dvm[0], dvm[1], dvm[2], dvm[3],
                    dvm[4], dvm[5], cond, worst);
        if (!(worst <= 1e-15 * cond) && !(worst <= 1e-12)) ++failures;
    }
    lbkm::Consts c{};
    double cond = 0.0;
    const double same[6] = {1.5, 1.5, 1.5, 1.0, 2.0, 3.0};
    const int r = lbkm::build_moment_blocks(same, &c, &cond);
    std::printf("equal group speeds: build returned %d\n", r);
    if (r != -2) ++failures;
    std::printf(failures ? "FAILED\n" : "ok\n");
    return failures ? 1 : 0;
}
