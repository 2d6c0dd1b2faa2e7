// The library's host-side planner under AddressSanitizer and UndefinedBehaviorSanitizer
// (host-only build, no GPU needed): descriptor validation, the multigrid hierarchy, the
// coarse-kernel LDS layout, launch planning and the workspace layout of single stacks
// and of the whole list as one batch, plus descriptors that must be rejected.  Prints
// the workspace sizes (compared with the regular build by the test).
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/ferrox.h"
extern "C" {
#include "stacks.h"
}

static fx_stack_desc desc_of(const san_stack &s) {
    fx_stack_desc d;
    std::memset(&d, 0, sizeof d);
    d.nx = s.nx; d.ny = s.ny; d.nz = s.nz; d.h = s.h;
    d.plane_mat = s.mat; d.plane_eps_r = s.eps; d.plane_Na = s.Na; d.plane_Nd = s.Nd;
    d.alpha = -2.5e9; d.beta = 6e10; d.gamma = 1.5e11; d.g11 = d.g44 = 1e-10; d.Gamma = 100.0;
    d.pbc = s.pbc; d.lambda = s.lambda; d.ni = s.ni; d.T = s.T; d.v_top = s.v_top;
    d.tol_rel = 1e-10; d.max_cycles = 60; d.prec = FX_PREC_FP64; d.warm_start = 3; d.time_order = 1;
    d.carriers = s.carriers; d.m_e = 1.08; d.m_p = 0.81; d.Eg = 1.12;
    return d;
}

int main(int argc, char **argv) {
    san_stack *v;
    const int n = argc > 1 ? san_read(argv[1], &v) : -1;
    if (n <= 0) { std::fprintf(stderr, "no stacks\n"); return 2; }
    std::vector<fx_stack_desc> ds;
    for (int i = 0; i < n; ++i) ds.push_back(desc_of(v[i]));
    for (int prec = 0; prec < 2; ++prec)
        for (int order = 1; order <= 2; ++order) {
            for (auto &d : ds) { d.prec = prec; d.time_order = order; }
            for (int i = 0; i < n; ++i)
                std::printf("stack %d prec %d order %d: %zu\n", i, prec, order, stack_workspace_bytes(&ds[i]));
            std::printf("batch prec %d order %d: %zu\n", prec, order, batch_workspace_bytes(ds.data(), n));
        }
    // rejected descriptors: each must give 0 bytes and a message
    fx_stack_desc bad = ds[0];
    int rejected = 0;
    auto expect_zero = [&](const fx_stack_desc &d, const char *what) {
        const size_t b = stack_workspace_bytes(&d);
        std::printf("reject %s: %zu (%s)\n", what, b, last_error());
        rejected += b == 0;
    };
    bad.nx = 0; expect_zero(bad, "nx = 0"); bad = ds[0];
    bad.h = -1; expect_zero(bad, "h < 0"); bad = ds[0];
    bad.warm_start = 7; expect_zero(bad, "warm_start 7"); bad = ds[0];
    bad.plane_mat = nullptr; expect_zero(bad, "no plane table"); bad = ds[0];
    std::vector<int> mat(v[0].mat, v[0].mat + v[0].nz);
    mat[v[0].nz / 2] = FX_MAT_METAL; bad.plane_mat = mat.data(); expect_zero(bad, "metal inside"); bad = ds[0];
    std::printf("batch of 0: %zu\n", batch_workspace_bytes(ds.data(), 0));
    san_free(v, n);
    return rejected == 5 ? 0 : 1;
}
