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

// A dispatch covers at most 2^32 - 1 work-items (grid x block), so kernels
// whose natural grid could exceed that at 32+ qubits loop over blocks
// (grid-stride) with their grid capped here: 2^22 blocks of 256 threads.
constexpr uint64_t kMaxGridBlocks = uint64_t(1) << 22;
inline unsigned capped_grid(uint64_t blocks) {
    return unsigned(blocks < 1 ? 1 : (blocks > kMaxGridBlocks ? kMaxGridBlocks : blocks));
}

// Order in which a grid-stride kernel visits its nblk logical blocks.  The
// chip dispatches workgroups to its 8 XCDs round-robin (workgroup b runs on
// XCD b mod 8).  In XCD order the workgroups of one XCD take one contiguous
// eighth of the blocks, in steps of gridDim/8, so at any moment each XCD
// streams its own region of the state rather than all eight interleaving
// on the same lines and DRAM pages: at 32 qubits this raised a controlled
// gate from 5.1-5.3 to 6.2-6.5 TB/s.  It needs nblk and gridDim.x to be
// multiples of 8; otherwise the blocks are visited in plain order.
struct BlockWalk {
    uint64_t first, end, step;
    __device__ __forceinline__ explicit BlockWalk(uint64_t nblk) {
        const uint64_t G = gridDim.x;
        if ((nblk & 7) == 0 && (G & 7) == 0) {
            const uint64_t e = nblk >> 3, x = blockIdx.x & 7u;
            first = x * e + (blockIdx.x >> 3);
            end = x * e + e;
            step = G >> 3;
        } else {
            first = blockIdx.x;
            end = nblk;
            step = G;
        }
    }
};
inline __device__ __forceinline__ uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

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

// Non-temporal load and store of one amplitude: passes stream the state
// through once, so its lines should not displace other cached data.
template <typename V>
__device__ __forceinline__ V ld_nt(const V* p) {
    using R = decltype(p->x);
    typedef R VX __attribute__((ext_vector_type(2)));
    const VX x = __builtin_nontemporal_load(reinterpret_cast<const VX*>(p));
    V v;
    v.x = x.x;
    v.y = x.y;
    return v;
}
template <typename V>
__device__ __forceinline__ void st_nt(V* p, const V& v) {
    using R = decltype(p->x);
    typedef R VX __attribute__((ext_vector_type(2)));
    VX x;
    x.x = v.x;
    x.y = v.y;
    __builtin_nontemporal_store(x, reinterpret_cast<VX*>(p));
}

// Fused multiply-add in the state's real type.
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Complex multiply-accumulate chains: each term is two fused multiply-adds
// on the real part and two on the imaginary part; the first term starts
// from a product.
template <typename R, typename V>
__device__ __forceinline__ void cmac_first(R ur, R ui, const V& x, R& re, R& im) {
    re = fmaR(-ui, x.y, ur * x.x);
    im = fmaR(ui, x.x, ur * x.y);
}
template <typename R, typename V>
__device__ __forceinline__ void cmac(R ur, R ui, const V& x, R& re, R& im) {
    re = fmaR(ur, x.x, re);
    re = fmaR(-ui, x.y, re);
    im = fmaR(ur, x.y, im);
    im = fmaR(ui, x.x, im);
}

// (oa, ob) = U (a, b) for a 2x2 complex U.
template <typename R, typename V>
__device__ __forceinline__ void mv2(const R* u, const V& a, const V& b, V& oa, V& ob) {
    R r0, i0, r1, i1;
    cmac_first(u[0], u[1], a, r0, i0);
    cmac(u[2], u[3], b, r0, i0);
    cmac_first(u[4], u[5], a, r1, i1);
    cmac(u[6], u[7], b, r1, i1);
    oa.x = r0; oa.y = i0;
    ob.x = r1; ob.y = i1;
}

// o[r] = sum_c U[r][c] v[c] for a 4x4 complex U.
template <typename R, typename V>
__device__ __forceinline__ void mv4(const R* u, const V* v, V* o) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        R re, im;
        cmac_first(u[8 * r], u[8 * r + 1], v[0], re, im);
#pragma unroll
        for (int c = 1; c < 4; ++c) cmac(u[2 * (4 * r + c)], u[2 * (4 * r + c) + 1], v[c], re, im);
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
