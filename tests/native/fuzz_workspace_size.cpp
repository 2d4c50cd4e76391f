// Host-only fuzz of the library's size queries and host-side planning:
// numag_workspace_size (argument validation and the work planning of every path
// and mode: object tables, rotation groups, splits), the snapshot and 2D
// correlation workspace sizes, object-mode plans (create, size, destroy) and the
// launch-shape table (reads, and writes of random shapes that later requests
// then plan with), on random and invalid requests.  Never touches a GPU (the
// pointers are tags that validation does not dereference).  Built with
// AddressSanitizer on the host code by tests/test_host_fuzz_asan.py.
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <random>
#include <vector>
#include "numag.h"
int main()
{
    std::mt19937_64 rng(12345);
    auto U = [&](int64_t lo, int64_t hi) { return std::uniform_int_distribution<int64_t>(lo, hi)(rng); };
    size_t acc = 0;
    for (int it = 0; it < 20000; ++it) {
        int64_t K = U(1, 70);
        std::vector<int64_t> off(K + 1, 0);
        for (int64_t k = 1; k <= K; ++k) off[k] = off[k - 1] + U(0, it % 7 == 0 ? 200000 : 300);
        if (it % 50 == 0 && K > 1) off[K / 2] = off[K / 2 + 1] + 5;  // invalid: decreasing
        numag_sample s;
        std::memset(&s, 0, sizeof(s));
        s.n_points = off[K];
        s.pos = (const double *)0x1000;
        s.nuc = (it & 1) ? (const double *)0x2000 : nullptr;
        s.mag = (it & 2) ? (const double *)0x3000 : nullptr;
        s.n_objects = K;
        s.obj_offsets = K > 1 ? off.data() : nullptr;
        numag_regular reg;
        if (it % 11 == 0) {
            reg.n[0] = (int)U(1, 70); reg.n[1] = (int)U(1, 70); reg.n[2] = (int)U(1, 70); reg.reserved = 0;
            for (int a = 0; a < 3; ++a) { reg.origin[a] = -1.0; reg.step[a] = 0.5; }
            s.regular = &reg; s.n_objects = 1; s.obj_offsets = nullptr;
            s.n_points = (int64_t)reg.n[0] * reg.n[1] * reg.n[2];
        }
        numag_qgrid g;
        g.kind = (int)U(0, 1); g.n0 = (int)U(it % 13 == 0 ? -2 : 1, 600); g.n1 = (int)U(1, 600); g.reserved = 0;
        if (it % 5 == 0) g.n1 = (int)U(1, 4);  // odd and tiny theta counts
        g.qmax = (it % 17 == 0) ? -1.0 : 0.1 + U(0, 30) * 0.1;
        const int64_t n_rot = U(it % 19 == 0 ? 0 : 1, 1500);
        const int path = (int)U(-1, 6), mode = (int)U(-1, 3);
        acc += numag_workspace_size(&s, n_rot, &g, path, mode);
        // the other host-only queries
        numag_regular rg;
        rg.n[0] = (int)U(it % 23 == 0 ? 0 : 1, 40); rg.n[1] = (int)U(1, 40); rg.n[2] = (int)U(1, 40); rg.reserved = 0;
        for (int a = 0; a < 3; ++a) { rg.origin[a] = -1.0; rg.step[a] = 0.25; }
        acc += numag_snapshots_workspace_size(&rg, U(-1, 300), &g, (int)U(-1, 6));
        numag_qgrid rgr = g;
        rgr.kind = (int)U(0, 1); rgr.n0 = (int)U(it % 29 == 0 ? 0 : 1, 300); rgr.n1 = (int)U(1, 300);
        rgr.qmax = 0.5 + (double)U(0, 50);
        acc += numag_correlation_2d_workspace_size(&g, &rgr);
        numag_tune_shape dsh, csh;
        acc += (size_t)(numag_tune_get((int)U(-1, 3), &g, (int)U(-1, 4), U(-1, 1 << 22), &dsh, &csh) + 8);
        if (it % 3 == 0) {
            const numag_tune_shape t{(int)U(-2, 80), (int)U(-5, 70000)};
            (void)numag_tune_set((int)U(-1, 3), &g, (int)U(-1, 4), U(0, 1 << 22), &t);
        }
        if (it % 4 == 0) {
            const int64_t nr = U(it % 31 == 0 ? 0 : 1, 16);
            std::vector<double> rot(9 * (size_t)(nr > 0 ? nr : 1), 0.0);
            for (int64_t r = 0; r < nr; ++r) rot[9 * r] = rot[9 * r + 4] = rot[9 * r + 8] = 1.0;
            if (it % 37 == 0) rot[0] = 2.0;  // invalid: not orthonormal
            numag_plan *plan = nullptr;
            if (numag_plan_create(&s, nr, rot.data(), &g, path, mode, (int)U(0, 1), &plan) == 0)
                acc += numag_plan_workspace_size(plan);
            numag_plan_destroy(plan);
        }
    }
    std::printf("ok %zu\n", acc);
    return 0;
}
