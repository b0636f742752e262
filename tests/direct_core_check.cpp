// Host driver of the exact line-solve core (paper_2006_07583_amd/csrc/
// direct_core.h), built with g++ for the CPU tests.
//   direct_core_check solve   : stdin "method n S Se H mode inv_h src_s aF" then
//                               A, B, K, R (n + 2 values each); prints U, V
//                               (n + 2 values each) after solving every window
//   direct_core_check margin method c2 tol : prints the window margin
//   direct_core_check plan    : checks the window-plan invariants, prints the
//                               number of violations (exit status 0 = none)
//   direct_core_check sink    : checks the gathered pressure stores against
//                               one store per slot, prints the number of
//                               violations (exit status 0 = none)
#define DIRECT_HD inline
#define DIRECT_HOST_ONLY
#include "direct_core.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

using namespace adi::direct;

// A transposed pressure row for GatherSink: slot s at row[s - 1], the row
// 32-byte aligned; counts the stores per slot and flags a piece store that
// does not start a 32-byte piece.
template <typename T>
struct SinkRow {
    T* row;
    int* count;
    int* misplaced;
    bool live = true;
    T* uptr(int s) const {
        const int ch = GatherSink<T>::CH;
        if ((s - 1) % ch != 0 || ((uintptr_t)(row + s - 1)) % 32 != 0) ++*misplaced;
        for (int k = 0; k < ch; ++k) ++count[s - 1 + k];
        return row + s - 1;
    }
    void putU(int s, T x) const {
        row[s - 1] = x;
        ++count[s - 1];
    }
};

// Every window o0..o1 within 1..nmax, the slots put in descending order as
// the backward passes do: each output slot must hold its value and have
// been stored once, nothing else touched.
template <typename T>
int check_sink(bool on) {
    constexpr int nmax = 80;
    alignas(32) T row[nmax + 8];
    int count[nmax + 8], misplaced = 0, bad = 0;
    for (int o0 = 1; o0 <= nmax; ++o0)
        for (int o1 = o0 - 1; o1 <= nmax; ++o1) {
            for (int i = 0; i < nmax + 8; ++i) {
                row[i] = T(-1);
                count[i] = 0;
            }
            SinkRow<T> io{row, count, &misplaced};
            auto sk = GatherSink<T>::make(o0, o1, on);
            for (int s = o1; s >= o0; --s) sk.put(io, s, T(1000 + s));
            for (int s = 1; s <= nmax + 8; ++s) {
                const bool out = s >= o0 && s <= o1;
                bad += count[s - 1] != (out ? 1 : 0);
                bad += row[s - 1] != (out ? T(1000 + s) : T(-1));
            }
        }
    return bad + misplaced;
}

int main(int argc, char** argv) {
    if (argc >= 2 && !std::strcmp(argv[1], "sink")) {
        const int bad = check_sink<float>(true) + check_sink<double>(true) + check_sink<float>(false) +
                        check_sink<double>(false);
        std::printf("%d\n", bad);
        return bad ? 1 : 0;
    }
    if (argc >= 5 && !std::strcmp(argv[1], "margin")) {
        std::printf("%d\n", direct_margin(std::atoi(argv[2]), std::atof(argv[3]), std::atof(argv[4])));
        return 0;
    }
    if (argc >= 2 && !std::strcmp(argv[1], "plan")) {
        // window-plan invariants over many sizes: exact partition of the
        // output slots, interior-band windows inside the interior rows, kept
        // rows within the per-thread stride, and the lowest row the interior
        // backward loop reads (MFD: o0 - 1) among the kept rows
        int bad = 0;
        for (int method = 0; method <= 1; ++method)
            for (int n = 8; n <= 700; n += (n < 64 ? 1 : 37))
                for (int H = 6; H <= 140; H += 7)
                    for (int S : {H, 2 * H, 16, 40, 128, n + 1})
                      for (int Se : {0, H + 4}) {
                        if (S <= 0) continue;
                        const int smin = direct_smin(method), nw = direct_nwin(method, n, S, Se);
                        const int rows = direct_rows(method, n, S, Se, H);
                        int wa, wb, next = smin;
                        narrow_range(method, n, S, Se, H, wa, wb);
                        const int lo = method == MFD ? 4 : 2, hi = method == MFD ? n - 3 : n - 2;
                        for (int w = 0; w < nw; ++w) {
                            const Win W = window(smin, n, S, Se, H, w);
                            const int r1 = method == MFD ? W.w1 : 2 * W.w1 + 1;
                            const int rb = first_kept_row(method, W);
                            bad += W.o0 != next || W.o1 < W.o0 || W.w0 > W.o0 || W.w1 < W.o1;
                            bad += r1 - rb + 1 > rows || rb < (method == MFD ? W.w0 : 2 * W.w0);
                            next = W.o1 + 1;
                            if (w >= wa && w <= wb) {
                                bad += W.w0 < lo || W.w1 > hi || w == 0 || w == nw - 1;
                                if (method == MFD) bad += W.o0 - 1 < rb;
                            }
                        }
                        bad += next != n + 1;
                    }
        std::printf("%d\n", bad);
        return bad ? 1 : 0;
    }
    if (argc < 2 || std::strcmp(argv[1], "solve")) return 2;
    int method, n, S, Se, H, mode, src_s;
    double inv_h, aF;
    if (std::scanf("%d %d %d %d %d %d %lf %d %lf", &method, &n, &S, &Se, &H, &mode, &inv_h, &src_s, &aF) != 9)
        return 3;
    std::vector<double> a(n + 2), b(n + 2), k(n + 2), r(n + 2), u(n + 2, 0.0), v(n + 2, 0.0);
    for (auto* arr : {&a, &b, &k, &r})
        for (auto& x : *arr)
            if (std::scanf("%lf", &x) != 1) return 4;
    const int rows = direct_rows(method, n, S, Se, H);
    std::vector<double> fs((size_t)rows * 8, 0.0);
    HostLine<double> io{a.data(), b.data(), k.data(), r.data(), u.data(), v.data(), fs.data(), rows};
    // the library's dispatch: windows 1..narrow_last with the interior band
    const int nw = direct_nwin(method, n, S, Se);
    int wa, wb;
    narrow_range(method, n, S, Se, H, wa, wb);
    for (int w = 0; w < nw; ++w) {
        const bool narrow = w >= wa && w <= wb;
        if (method == MFD) {
            if (narrow) solve_window<double, MFD, false>(io, n, S, Se, H, w, inv_h, mode, src_s, aF);
            else solve_window<double, MFD, true>(io, n, S, Se, H, w, inv_h, mode, src_s, aF);
        } else {
            if (narrow) solve_window<double, CFD, false>(io, n, S, Se, H, w, inv_h, mode, src_s, aF);
            else solve_window<double, CFD, true>(io, n, S, Se, H, w, inv_h, mode, src_s, aF);
        }
    }
    std::fprintf(stderr, "windows %d, interior-band windows %d\n", nw, wb >= wa ? wb - wa + 1 : 0);
    for (auto* arr : {&u, &v}) {
        for (double x : *arr) std::printf("%.17g ", x);
        std::printf("\n");
    }
    return 0;
}
