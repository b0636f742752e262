// Host driver of the exact line-solve core (paper_2006_07583_amd/csrc/
// direct_core.h), built with g++ for the CPU tests.
//   direct_core_check solve   : stdin "method n S H mode inv_h src_s aF" then
//                               A, B, K, R (n + 2 values each); prints U, V
//                               (n + 2 values each) after solving every window
//   direct_core_check margin method c2 tol : prints the window margin
#define DIRECT_HD inline
#define DIRECT_HOST_ONLY
#include "direct_core.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace adi::direct;

int main(int argc, char** argv) {
    if (argc >= 5 && !std::strcmp(argv[1], "margin")) {
        std::printf("%d\n", direct_margin(std::atoi(argv[2]), std::atof(argv[3]), std::atof(argv[4])));
        return 0;
    }
    if (argc < 2 || std::strcmp(argv[1], "solve")) return 2;
    int method, n, S, H, mode, src_s;
    double inv_h, aF;
    if (std::scanf("%d %d %d %d %d %lf %d %lf", &method, &n, &S, &H, &mode, &inv_h, &src_s, &aF) != 8) return 3;
    std::vector<double> a(n + 2), b(n + 2), k(n + 2), r(n + 2), u(n + 2, 0.0), v(n + 2, 0.0);
    for (auto* arr : {&a, &b, &k, &r})
        for (auto& x : *arr)
            if (std::scanf("%lf", &x) != 1) return 4;
    const int rows = direct_rows(method, n, S, H);
    std::vector<double> fs((size_t)rows * 8, 0.0);
    HostLine<double> io{a.data(), b.data(), k.data(), r.data(), u.data(), v.data(), fs.data(), rows};
    // the library's dispatch: windows 1..narrow_last with the interior band
    const int nw = direct_nwin(method, n, S);
    int wa, wb;
    narrow_range(method, n, S, H, wa, wb);
    for (int w = 0; w < nw; ++w) {
        const bool narrow = w >= wa && w <= wb;
        if (method == MFD) {
            if (narrow) solve_window<double, MFD, false>(io, n, S, H, w, inv_h, mode, src_s, aF);
            else solve_window<double, MFD, true>(io, n, S, H, w, inv_h, mode, src_s, aF);
        } else {
            if (narrow) solve_window<double, CFD, false>(io, n, S, H, w, inv_h, mode, src_s, aF);
            else solve_window<double, CFD, true>(io, n, S, H, w, inv_h, mode, src_s, aF);
        }
    }
    std::fprintf(stderr, "windows %d, interior-band windows %d\n", nw, wb >= wa ? wb - wa + 1 : 0);
    for (auto* arr : {&u, &v}) {
        for (double x : *arr) std::printf("%.17g ", x);
        std::printf("\n");
    }
    return 0;
}
