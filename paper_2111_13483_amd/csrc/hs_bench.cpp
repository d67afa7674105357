// hs_bench: one build + setup + solve step through the C-ABI only (no
// Python), for hardware-counter runs. Reads a workload file written by
// `bench.py --write-workload` and optionally first runs one device-to-device
// copy of a known size, which calibrates the HBM byte counters.
//
// Usage: hs_bench WORKLOAD_FILE [COPY_MIB]
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hschur.h"

namespace {

struct Header {
    int64_t n;
    double k, self_h;
    int32_t leaf_max, restart;
    double aca_tol, fill_tol, tol;
};

bool ok(int32_t st, const char* what) {
    if (st == HS_OK || st == HS_NOT_CONVERGED) return true;
    std::fprintf(stderr, "%s: %s (%s)\n", what, hs_status_string(st), hs_last_error());
    return false;
}

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) {
        std::fprintf(stderr, "usage: %s WORKLOAD_FILE [COPY_MIB]\n", argv[0]);
        return 2;
    }
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", argv[1]);
        return 2;
    }
    Header h{};
    if (std::fread(&h, sizeof(h), 1, f) != 1 || h.n < 1) {
        std::fprintf(stderr, "bad workload header\n");
        return 2;
    }
    std::vector<double> pts(3 * h.n), rhs(2 * h.n);
    if (std::fread(pts.data(), sizeof(double), pts.size(), f) != pts.size() ||
        std::fread(rhs.data(), sizeof(double), rhs.size(), f) != rhs.size()) {
        std::fprintf(stderr, "truncated workload file\n");
        return 2;
    }
    std::fclose(f);
    const long copy_mib = argc > 2 ? std::atol(argv[2]) : 0;

    double *d_pts = nullptr, *d_b = nullptr, *d_x = nullptr;
    if (hipMalloc(&d_pts, pts.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_b, rhs.size() * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_x, rhs.size() * sizeof(double)) != hipSuccess) {
        std::fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    hipMemcpy(d_pts, pts.data(), pts.size() * sizeof(double), hipMemcpyHostToDevice);
    hipMemcpy(d_b, rhs.data(), rhs.size() * sizeof(double), hipMemcpyHostToDevice);
    if (copy_mib > 0) {
        const size_t bytes = (size_t)copy_mib << 20;
        void *a = nullptr, *b = nullptr;
        if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
            std::fprintf(stderr, "hipMalloc of the copy buffers failed\n");
            return 1;
        }
        hipMemset(a, 0, bytes);
        hipDeviceSynchronize();
        hipMemcpy(b, a, bytes, hipMemcpyDeviceToDevice);
        hipDeviceSynchronize();
        hipFree(a);
        hipFree(b);
        std::printf("copy %ld MiB done\n", copy_mib);
    }

    hs_context* ctx = nullptr;
    if (!ok(hs_context_create(&ctx, 0, nullptr, nullptr, nullptr, nullptr), "context")) return 1;
    const double t0 = now();
    hs_build_opts bo{h.leaf_max, h.aca_tol, 0, 0};
    hs_hmatrix* H = nullptr;
    if (!ok(hs_h_build(ctx, d_pts, h.n, h.k, h.self_h, &bo, &H), "h_build")) return 1;
    const double t1 = now();
    hs_precond_opts po{HS_ORDER_RCM, h.fill_tol, HS_PREC_FP64, 0, 0};
    hs_precond* P = nullptr;
    if (!ok(hs_precond_setup(ctx, H, &po, &P), "precond_setup")) return 1;
    const double t2 = now();
    hs_solve_opts so{HS_SOLVE_GMRES, h.restart, h.tol, 0, 0, 0, 0.0};
    hs_solve_stats st{};
    if (!ok(hs_solve(ctx, H, P, d_b, d_x, 1, &so, &st), "solve")) return 1;
    const double t3 = now();
    std::printf("n %lld h_build %.4f s setup %.4f s solve %.4f s iters %d relres %.3e\n", (long long)h.n, t1 - t0,
                t2 - t1, t3 - t2, st.iters, st.relres);
    hs_precond_destroy(P);
    hs_hmatrix_destroy(H);
    hs_context_destroy(ctx);
    hipFree(d_pts);
    hipFree(d_b);
    hipFree(d_x);
    return 0;
}
