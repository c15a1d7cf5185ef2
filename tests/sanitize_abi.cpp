// Host sanitizer driver for the C-ABI: workspace queries (including the
// sizes of the largest workloads, so the size arithmetic runs under
// UndefinedBehaviorSanitizer's overflow checks) and the argument checks that
// every entry point makes before it touches a device.  Built with the
// library sources by tests/test_sanitize.py; host code only is instrumented.
// No pointer passed here is dereferenced: the calls must return first.
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include "bdg.h"

static int bad = 0;
#define EXPECT(cond)                                                                  \
    do {                                                                              \
        if (!(cond)) {                                                                \
            fprintf(stderr, "sanitize_abi: line %d: %s failed\n", __LINE__, #cond);   \
            bad = 1;                                                                  \
        }                                                                             \
    } while (0)

int main() {
    void *X = (void *)(uintptr_t)256;  // placeholder device pointer, never used
    size_t nb = 0;
    bdg_opts o;
    memset(&o, 0, sizeof(o));
    for (int64_t n : {1, 2, 3, 100, 2304, 27648, 49152, 65536}) {
        nb = 0;
        EXPECT(bdg_eigh_workspace(n, &o, &nb) == 0 && nb > 0);
        o.precision = BDG_FP32_REFINED;
        EXPECT(bdg_eigh_workspace(n, &o, &nb) == 0 && nb > 0);
        o.precision = BDG_FP64;
        EXPECT(bdg_refine_workspace(n, n / 2 + 1, &nb) == 0 && nb > 0);
        EXPECT(bdg_eigh1_workspace(n, 0, n, &nb) == 0 && nb > 0);
        EXPECT(bdg_eigh1_workspace(n, 1, n, &nb) == 0 && nb > 0);
    }
    EXPECT(bdg_eigh_workspace(0, &o, &nb) != 0);
    EXPECT(bdg_eigh_workspace(-5, &o, &nb) != 0);
    EXPECT(bdg_eigh1_workspace(10, 2, 1, &nb) == -2);
    {
        int64_t m = 0;
        EXPECT(bdg_eigh1(10, 0, (double *)X, 5, 0.0, 1.0, (double *)X, (double *)X, 10, 10, &m, X, 1 << 30,
                         nullptr, nullptr) == -4);
        EXPECT(bdg_eigh1(10, 0, (double *)X, 10, 2.0, 1.0, (double *)X, (double *)X, 10, 10, &m, X, 1 << 30,
                         nullptr, nullptr) == -5);
        EXPECT(bdg_eigh1(10, 0, (double *)X, 10, 0.0, 1.0, (double *)X, (double *)X, 10, 10, &m, X, 16, nullptr,
                         nullptr) == BDG_ERR_WORKSPACE);
    }
    bdg_lattice lat;
    memset(&lat, 0, sizeof(lat));
    const int lats[][4] = {{1, 64, 0, 0}, {2, 32, 32, 0}, {3, 24, 24, 24}, {3, 32, 32, 32}, {2, 64, 64, 0}};
    for (auto &l : lats) {
        lat.ndim = l[0];
        for (int d = 0; d < 3; ++d) lat.dims[d] = d < l[0] ? l[1 + d] : 0;
        EXPECT(bdg_scf_workspace(&lat, &nb) == 0 && nb > 0);
    }
    lat.ndim = 4;
    EXPECT(bdg_scf_workspace(&lat, &nb) != 0);
    lat.ndim = 2;
    lat.dims[0] = 7;
    lat.dims[1] = 8;
    EXPECT(bdg_scf_workspace(&lat, &nb) != 0);  // odd side
    // TDSLDA: workspace, refusal above 4096 sites, bad time step
    lat.ndim = 3;
    lat.dims[0] = lat.dims[1] = lat.dims[2] = 16;
    EXPECT(bdg_td_workspace(&lat, 2796, &nb) == 0 && nb > 0);
    bdg_td_params tp = {0.0, 0.0, 1, 0};
    lat.dims[2] = 18;
    EXPECT(bdg_td_evolve(&lat, (const double *)X, 1.0, &tp, 2, (double *)X, 9216, 0.01, 1, nullptr, nullptr, X,
                         (size_t)1 << 40, nullptr) == BDG_ERR_NOT_IMPLEMENTED);
    lat.dims[2] = 8;
    EXPECT(bdg_td_evolve(&lat, (const double *)X, 1.0, &tp, 2, (double *)X, 4096, -0.01, 1, nullptr, nullptr, X,
                         (size_t)1 << 40, nullptr) == -8);
    // regrid between incompatible lattices
    bdg_lattice a, b;
    memset(&a, 0, sizeof(a));
    memset(&b, 0, sizeof(b));
    a.ndim = b.ndim = 2;
    a.dims[0] = a.dims[1] = 12;
    b.dims[0] = 8;
    b.dims[1] = 14;
    EXPECT(bdg_regrid(&a, (const double *)X, &b, (double *)X, 1.0, nullptr) == -3);
    // INT8-sliced products: workspace and slice-count check
    EXPECT(bdg_gemm_int8_workspace(1, 8192, 8192, 8192, 8, &nb) == 0 && nb > 0);
    const double one[2] = {1.0, 0.0};
    EXPECT(bdg_gemm_int8(1, 2, 'N', 'N', 4, 4, 4, one, (const double *)X, 4, (const double *)X, 4, one,
                         (double *)X, 4, X, 1 << 30, nullptr) == -2);
    // network shapes
    bdg_net_shape sh = {32, 64, 64, 8};
    EXPECT(bdg_net_nparams(&sh) > 0);
    EXPECT(bdg_net_workspace(&sh, &nb) == 0 && nb > 0);
    sh.batch = 2;
    EXPECT(bdg_net_start_fields(&sh, (const float *)X, 2, (const double *)X, (double *)X, (double *)X, nullptr) ==
           -3);
    EXPECT(bdg_version() != nullptr && strlen(bdg_version()) > 0);
    EXPECT(bdg_last_error() != nullptr);
    printf("sanitize_abi: %s\n", bad ? "FAILED" : "ok");
    return bad;
}
