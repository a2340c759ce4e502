// Device-side helpers shared by the kernels of libspmvsel (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spmvsel {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Value traits: stored type V -> accumulation / vector type A.
template <class V> struct VT;
template <> struct VT<double> {
    using A = double;
    static __device__ __forceinline__ double cvt(double v) { return v; }
};
template <> struct VT<float> {
    using A = float;
    static __device__ __forceinline__ float cvt(float v) { return v; }
};
template <> struct VT<uint16_t> {  // bfloat16 bit pattern
    using A = float;
    static __device__ __forceinline__ float cvt(uint16_t v) {
        return __uint_as_float(static_cast<uint32_t>(v) << 16);
    }
};

template <class T>
__device__ __forceinline__ T ld_nt(const T *p) {
    return __builtin_nontemporal_load(p);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Give each XCD a contiguous range of logical tiles so that
// neighbouring tiles, which touch neighbouring parts of x, share an L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb) {
    const int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Load 8 consecutive elements starting at an 8-aligned index with 16-byte
// vector loads (non-temporal: streamed once).
template <class T>
__device__ __forceinline__ void load8_nt(const T *p, T out[8]) {
    static_assert(sizeof(T) == 2 || sizeof(T) == 4 || sizeof(T) == 8, "");
    constexpr int nv = sizeof(T) / 2;  // number of 16-byte loads
    const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
    union {
        u32x4 v[nv];
        T t[8];
    } u;
#pragma unroll
    for (int i = 0; i < nv; ++i) u.v[i] = __builtin_nontemporal_load(q + i);
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = u.t[i];
}

// ------------------------------------------------------------ DPP reductions
// Butterfly sum over aligned groups of W lanes (W a power of two <= 64).
// Every lane of the group ends with the same value; the pairing is fixed, so
// the result is deterministic.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float swz16_f(float v) {  // lane ^ 16 within 32
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}
__device__ __forceinline__ double swz16_d(double v) {
    const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float x32_f(float v) {  // lane ^ 32
    return __shfl_xor(v, 32, 64);
}
__device__ __forceinline__ double x32_d(double v) { return __shfl_xor(v, 32, 64); }

constexpr int kQuadSwap1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

template <int W>
__device__ __forceinline__ double group_sum(double v) {
    if (W >= 2) v = v + dpp_d<kQuadSwap1>(v);
    if (W >= 4) v = v + dpp_d<kQuadSwap2>(v);
    if (W >= 8) v = v + dpp_d<kRowHalfMirror>(v);
    if (W >= 16) v = v + dpp_d<kRowMirror>(v);
    if (W >= 32) v = v + swz16_d(v);
    if (W >= 64) v = v + x32_d(v);
    return v;
}
template <int W>
__device__ __forceinline__ float group_sum(float v) {
    if (W >= 2) v = v + dpp_f<kQuadSwap1>(v);
    if (W >= 4) v = v + dpp_f<kQuadSwap2>(v);
    if (W >= 8) v = v + dpp_f<kRowHalfMirror>(v);
    if (W >= 16) v = v + dpp_f<kRowMirror>(v);
    if (W >= 32) v = v + swz16_f(v);
    if (W >= 64) v = v + x32_f(v);
    return v;
}

// Minimum over the 64 lanes of a wavefront (every lane gets it).
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp_i<kQuadSwap1>(v));
    v = min(v, dpp_i<kQuadSwap2>(v));
    v = min(v, dpp_i<kRowHalfMirror>(v));
    v = min(v, dpp_i<kRowMirror>(v));
    v = min(v, __builtin_amdgcn_ds_swizzle(v, 0x401F));
    v = min(v, __shfl_xor(v, 32, 64));
    return v;
}

// ------------------------------------------------------------ accumulation
// Plain sum from +0, or Kahan's compensated sum (Kahan 1965) for FP32 rows
// longer than 256 nonzeros.  Compiled without contraction, so every
// operation rounds separately.
template <class A>
struct Sum {
    A s = A(0), c = A(0);
    __device__ __forceinline__ void add(A v) { s = s + v; }
    __device__ __forceinline__ void add_comp(A v) {
        const A yv = v - c;
        const A t = s + yv;
        c = (t - s) - yv;
        s = t;
    }
    __device__ __forceinline__ void add(A v, bool comp) {
        if (comp) add_comp(v); else add(v);
    }
    __device__ __forceinline__ void reset() { s = A(0); c = A(0); }
};

template <class A> __device__ __forceinline__ constexpr bool is_f32() { return sizeof(A) == 4; }

}  // namespace spmvsel
