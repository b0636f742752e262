// Output stage shared by the line-pass kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "line_pass.h"

namespace adi {

// Item and tile of this workgroup in a grouped launch (-1: idle block).
// Consecutive tiles go to the same XCD: block b runs on XCD b % 8.
template <typename T>
__device__ __forceinline__ int group_item(const GroupArgs<T>& g, int& tile) {
    const int b = (int)blockIdx.x;
    const int per = (g.total + 7) / 8;
    tile = (b % 8) * per + b / 8;
    if (tile >= g.total) return -1;
    int lo = 0, hi = g.nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.starts[mid] <= tile) lo = mid; else hi = mid - 1;
    }
    tile -= g.starts[lo];
    return lo;
}

// Damping rate at a point `lo` cells from the line's first wall (the line
// has n cells), from the layer parameters of LinePassArgs.
template <typename T>
__device__ __forceinline__ T damp_at(const LinePassArgs<T>& a, T lo) {
    if (a.dmpiw == T(0)) return a.dmp0;
    T r = T(0);
    if (a.dmpm & 1) {
        const T x = T(1) - lo * a.dmpiw;
        r += x > T(0) ? a.dmp0 * x * x : T(0);
    }
    if (a.dmpm & 2) {
        const T x = T(1) - (T(a.n) - lo) * a.dmpiw;
        r += x > T(0) ? a.dmp0 * x * x : T(0);
    }
    return r;
}
// Position (cells from the first wall) of pressure slot s: nodes (compact)
// or the faces and cell centres (mimetic).
template <int METHOD, typename T>
__device__ __forceinline__ T pres_pos(int s, int n) {
    if (METHOD == 0) return T(s);
    return s <= 0 ? T(0) : (s >= n + 1 ? T(n) : T(s) - T(0.5));
}

// hi + lo + inc as a new (hi, lo) pair: TwoSum of hi and the increment, its
// rounding error folded into the low word, then renormalised.
template <typename T>
__device__ __forceinline__ void acc_two_sum(T hi, T lo, T inc, T& oh, T& ol) {
    const T s = hi + inc;
    const T bb = s - hi;
    const T e = (hi - (s - bb)) + (inc - bb);
    const T l = lo + e;
    oh = s + l;
    ol = l - (oh - s);
}

// Writes the velocity (native layout) and pressure (natural or transposed
// through an LDS tile) results of the central slots [c0, c1) of a lane.
// COMP: vv and uu are increments of the state read from vin / uin (plus
// their low words); the sums are accumulated as (hi, lo) pairs, and the low
// words are stored when the output has a low-word array.
template <typename T, int R, int LW, int NT, int TILEP, bool COMP>
__device__ __forceinline__ void pass_outputs(const LinePassArgs<T>& a, T* smem, T (&vv)[R], T (&uu)[R],
                                             int s0, int q, bool qok, int lq, int lg, int c0, int c1,
                                             int uhi, int n, int tid, bool add_src) {
    if (add_src) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            if (q == a.src_q && s0 + k == a.src_s) uu[k] += a.aF;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const int s = s0 + k;
        if (qok && s >= c0 && s < c1 && s <= n) {
            const int64_t iv = (int64_t)s * a.vin_ld + q, ov = (int64_t)s * a.vout_ld + q;
            if (COMP) {
                const T hi = a.vin[iv];
                const T lo = a.vin_lo ? a.vin_lo[iv] : T(0);
                T oh, ol;
                acc_two_sum(hi, lo, vv[k], oh, ol);
                a.vout[ov] = oh;
                if (a.vout_lo) a.vout_lo[ov] = ol;
            } else {
                a.vout[ov] = vv[k];
            }
        }
    }
    if (COMP) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int s = s0 + k;
            if (qok && s >= c0 && s < c1 && s >= 1 && s <= uhi) {
                const int64_t iu = (int64_t)(s - 1) * a.uin_ld + q;
                const T hi = a.uin[iu];
                const T lo = a.uin_lo ? a.uin_lo[iu] : T(0);
                acc_two_sum(hi, lo, uu[k], uu[k], vv[k]);   // vv now holds the low words
            }
        }
    }
    const bool wlo = COMP && a.uout_lo != nullptr;
    if (!a.utrans) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int s = s0 + k;
            if (qok && s >= c0 && s < c1 && s >= 1 && s <= uhi) {
                const int64_t o = (int64_t)(s - 1) * a.uout_ld + q;
                a.uout[o] = uu[k];
                if (wlo) a.uout_lo[o] = vv[k];
            }
        }
        return;
    }
    const int lo = max(c0, 1), hi = min(c1 - 1, uhi);
    const int nv = hi - lo + 1;
    for (int part = 0; part < (wlo ? 2 : 1); ++part) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int s = s0 + k;
            if (s >= c0 && s < c1) smem[lq * TILEP + (s - c0)] = part == 0 ? uu[k] : vv[k];
        }
        __syncthreads();
        T* dst = part == 0 ? a.uout : a.uout_lo;
        for (int idx = tid; idx < LW * nv; idx += NT) {
            const int l = idx / nv, j = idx - l * nv;
            const int qq = lg * LW + l;
            if (qq < a.nlines) dst[(int64_t)qq * a.uout_ld + (lo + j - 1)] = smem[l * TILEP + (lo - c0) + j];
        }
    }
}

}  // namespace adi
