// Streaming reference kernel (adi_stream_ceiling): the HBM pattern of a line
// pass without its arithmetic.  A pass reads the pressure hand-off, the
// velocity and a kappa and writes the velocity and the next hand-off, each
// element once; this kernel reads three arrays and writes two of the same
// length in 16-byte vectors, which sets the rate such a pass can reach on
// the device (the roofline's achievable ceiling, below the nominal peak).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/adi.h"
#include "problem.h"

namespace {

template <typename T>
struct Vec;
template <>
struct Vec<float> { using type = float4; };
template <>
struct Vec<double> { using type = double2; };

template <typename V>
__device__ __forceinline__ V comb1(const V& a, const V& b, const V& c);
template <>
__device__ __forceinline__ float4 comb1(const float4& a, const float4& b, const float4& c) {
    return make_float4(fmaf(-c.x, b.x, a.x), fmaf(-c.y, b.y, a.y), fmaf(-c.z, b.z, a.z), fmaf(-c.w, b.w, a.w));
}
template <>
__device__ __forceinline__ double2 comb1(const double2& a, const double2& b, const double2& c) {
    return make_double2(fma(-c.x, b.x, a.x), fma(-c.y, b.y, a.y));
}
template <typename V>
__device__ __forceinline__ V comb2(const V& a, const V& b);
template <>
__device__ __forceinline__ float4 comb2(const float4& a, const float4& b) {
    return make_float4(b.x - a.x, b.y - a.y, b.z - a.z, b.w - a.w);
}
template <>
__device__ __forceinline__ double2 comb2(const double2& a, const double2& b) {
    return make_double2(b.x - a.x, b.y - a.y);
}

// x = a - c b, y = b - a over nv vectors; two vectors per thread and
// iteration keep six loads in flight.
template <typename T>
__global__ void __launch_bounds__(256) stream_kernel(const typename Vec<T>::type* __restrict__ a,
                                                     const typename Vec<T>::type* __restrict__ b,
                                                     const typename Vec<T>::type* __restrict__ c,
                                                     typename Vec<T>::type* __restrict__ x,
                                                     typename Vec<T>::type* __restrict__ y, int64_t nv) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv; i += 2 * stride) {
        const int64_t j = i + stride;
        const bool two = j < nv;
        const auto a0 = a[i], b0 = b[i], c0 = c[i];
        typename Vec<T>::type a1{}, b1{}, c1{};
        if (two) {
            a1 = a[j];
            b1 = b[j];
            c1 = c[j];
        }
        x[i] = comb1(a0, b0, c0);
        y[i] = comb2(a0, b0);
        if (two) {
            x[j] = comb1(a1, b1, c1);
            y[j] = comb2(a1, b1);
        }
    }
}

template <typename T>
int launch(const void* a, const void* b, const void* c, void* x, void* y, int64_t n, hipStream_t st) {
    using V = typename Vec<T>::type;
    const int64_t nv = n * (int64_t)sizeof(T) / 16;
    // blocks: two vectors per thread, at most 64 workgroups per compute unit
    const int64_t want = (nv + 511) / 512;
    const unsigned blocks = (unsigned)(want < 16384 ? (want > 0 ? want : 1) : 16384);
    hipLaunchKernelGGL(stream_kernel<T>, dim3(blocks), dim3(256), 0, st, (const V*)a, (const V*)b, (const V*)c,
                       (V*)x, (V*)y, nv);
    HIP_TRY(hipGetLastError(), "stream kernel");
    return ADI_OK;
}

}  // namespace

extern "C" int adi_stream_ceiling(int dtype, const void* a, const void* b, const void* c, void* x, void* y, int64_t n,
                                  void* hip_stream) {
    if (dtype != ADI_FP32 && dtype != ADI_FP64) return adi::fail(ADI_EINVAL, "dtype must be ADI_FP32 or ADI_FP64");
    if (!a || !b || !c || !x || !y) return adi::fail(ADI_EINVAL, "NULL array");
    if (n < 0) return adi::fail(ADI_EINVAL, "n < 0");
    const int64_t esz = dtype == ADI_FP64 ? 8 : 4;
    if ((n * esz) % 16) return adi::fail(ADI_EINVAL, "n * element size must be a multiple of 16 bytes");
    for (const void* p : {a, b, c, (const void*)x, (const void*)y})
        if ((uintptr_t)p % 16) return adi::fail(ADI_EINVAL, "arrays must be 16-byte aligned");
    hipStream_t st = (hipStream_t)hip_stream;
    return dtype == ADI_FP64 ? launch<double>(a, b, c, x, y, n, st) : launch<float>(a, b, c, x, y, n, st);
}
