// Device helpers shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qsv {

template <typename R>
struct V2T;
template <>
struct V2T<double> { using type = double2; };
template <>
struct V2T<float> { using type = float2; };

template <typename R>
struct M2 { R v[8]; };   // 2x2 row-major (re, im)
template <typename R>
struct M4 { R v[32]; };  // 4x4 row-major (re, im)

// Zero-bit insertion (Sec. 2.1): the bits of j at positions >= p move up by
// one and bit p becomes 0.  This is the paper's (j & m_R) + ((j & m_L) << 1)
// with m_R = 2^p - 1, written for 64-bit indices.
__device__ __forceinline__ uint64_t insert0(uint64_t j, int p) {
    const uint64_t lo = j & ((uint64_t(1) << p) - 1);
    return ((j ^ lo) << 1) | lo;
}
__device__ __forceinline__ uint32_t insert0_32(uint32_t j, int p) {
    const uint32_t lo = j & ((1u << p) - 1);
    return ((j ^ lo) << 1) | lo;
}

// (oa, ob) = U (a, b) for a 2x2 complex U.
template <typename R, typename V>
__device__ __forceinline__ void mv2(const R* u, const V& a, const V& b, V& oa, V& ob) {
    oa.x = u[0] * a.x - u[1] * a.y + u[2] * b.x - u[3] * b.y;
    oa.y = u[0] * a.y + u[1] * a.x + u[2] * b.y + u[3] * b.x;
    ob.x = u[4] * a.x - u[5] * a.y + u[6] * b.x - u[7] * b.y;
    ob.y = u[4] * a.y + u[5] * a.x + u[6] * b.y + u[7] * b.x;
}

// o[r] = sum_c U[r][c] v[c] for a 4x4 complex U (accumulation starts from
// the first product, so every term is one multiply-add).
template <typename R, typename V>
__device__ __forceinline__ void mv4(const R* u, const V* v, V* o) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        R re = u[8 * r] * v[0].x - u[8 * r + 1] * v[0].y;
        R im = u[8 * r] * v[0].y + u[8 * r + 1] * v[0].x;
#pragma unroll
        for (int c = 1; c < 4; ++c) {
            const R ur = u[2 * (4 * r + c)], ui = u[2 * (4 * r + c) + 1];
            re += ur * v[c].x - ui * v[c].y;
            im += ur * v[c].y + ui * v[c].x;
        }
        o[r].x = re;
        o[r].y = im;
    }
}

}  // namespace qsv

namespace qsv {

// Fixed-order tree over a 256-thread block; red holds NT rows of 256 values.
// After the call, out[t] (t < NT) holds row t's sum (written by thread t).
template <int NT>
__device__ __forceinline__ void block_tree256(double (*red)[256], double* out) {
    for (int stride = 128; stride > 0; stride >>= 1) {
        __syncthreads();
        if (int(threadIdx.x) < stride) {
#pragma unroll
            for (int t = 0; t < NT; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + stride];
        }
    }
    __syncthreads();
    if (threadIdx.x < NT) out[threadIdx.x] = red[threadIdx.x][0];
}

}  // namespace qsv
