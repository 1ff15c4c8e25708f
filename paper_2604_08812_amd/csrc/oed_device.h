// Device-side helpers shared by the liboed kernel units: vector types, the 16x16x4 MFMA
// wrappers, vector loads/stores, triangular index maths and the batched-launch lookup.
#pragma once
#include <math.h>

#include "oed_internal.h"

namespace oed {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <typename T>
struct V4;
template <>
struct V4<float> {
    typedef floatx4 type;
};
template <>
struct V4<double> {
    typedef doublex4 type;
};

__device__ __forceinline__ floatx4 mfma16(float a, float b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4 mfma16(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Lane whose stored operand row the A operand of `lane` must carry.  The FP32 16x16x4 MFMA
// returns output row m of a 16x16 block at lane 16*(m/4) + n, register m%4; the FP64 one at
// lane 16*(m%4) + n, register m/4.  Feeding the FP64 A operand the rows in the order
// pi(r) = 4*(r%4) + r/4 (an involution) makes both land in the same accumulator storage order.
template <typename T>
__device__ __forceinline__ int a_lane(int lane)
{
    return lane;
}
template <>
__device__ __forceinline__ int a_lane<double>(int lane)
{
    return (lane & 48) | ((lane & 3) << 2) | ((lane & 15) >> 2);
}

// BF16 (stored as its 16 bits): round to nearest even from FP32, and back.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float x)
{
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// D += A B on 16 x 16 x 32 BF16 operands (8 per lane, passed as 4 dwords), FP32 accumulation.
__device__ __forceinline__ floatx4 mfma_bf16(u32x4 a, u32x4 b, floatx4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

template <typename T>
__device__ __forceinline__ typename V4<T>::type ld4(const T *p)
{
    return *reinterpret_cast<const typename V4<T>::type *>(p);
}
template <typename T>
__device__ __forceinline__ void st4(T *p, typename V4<T>::type v)
{
    *reinterpret_cast<typename V4<T>::type *>(p) = v;
}

// Streaming (non-temporal) vector access: the downdate reads and writes each block of R once per
// launch, and marking those accesses streaming keeps them from evicting the W panels that the
// tiles of an XCD share in its L2.
template <typename T>
__device__ __forceinline__ typename V4<T>::type ld4_stream(const T *p)
{
    return __builtin_nontemporal_load(reinterpret_cast<const typename V4<T>::type *>(p));
}
template <typename T>
__device__ __forceinline__ void st4_stream(T *p, typename V4<T>::type v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<typename V4<T>::type *>(p));
}

// Row of the packed lower triangle: element (t, u), u <= t, at tri(t) + u.
__device__ __forceinline__ int tri(int t) { return t * (t + 1) / 2; }

// Largest i with i(i+1)/2 <= b.
__device__ __forceinline__ int64_t tri_row(int64_t b)
{
    if (b <= 0) return b < 0 ? -1 : 0;
    int64_t i = (int64_t)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((i + 1) * (i + 2) / 2 <= b) ++i;
    while (i * (i + 1) / 2 > b) --i;
    return i;
}

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// A wave-uniform element of a device array, kept in a scalar register.  Where the array's address
// itself comes from memory (a batched launch's descriptor) the compiler reads it with a vector load;
// without this every address derived from the value would occupy vector registers.
__device__ __forceinline__ int uniform_at(const int *__restrict__ p, int k)
{
    return __builtin_amdgcn_readfirstlane(p[k]);
}

// Instance of a batched launch that owns work item `item`: the last descriptor with
// item0 <= item (descriptors are sorted by item0).  -1 if no instance owns the item.
__device__ __forceinline__ int find_instance(const StepDesc *ds, int n, int64_t item)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ds[mid].item0 <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    // work-group uniform: keeps the descriptor loads scalar
    lo = __builtin_amdgcn_readfirstlane(lo);
    return (item >= ds[lo].item0 && item < ds[lo].item0 + ds[lo].nitems) ? lo : -1;
}

// Downdate tile order: the 128 x 128 tiles (P, Q), Q <= P, of the lower triangle are grouped
// in super-tiles of b x b tiles (b = 2^(stl & 7), 8 for stl & 7 == 0), taken in lower-triangular
// order, so that super-tile row SP (a band of b tile rows) is swept column after column.  Inside
// a super-tile the b^2 slots run down the columns (the b tiles that share a column panel of W
// are consecutive, and the band's b row panels are reused by every super-tile of the band) or,
// with stl & 8, along the rows.  The work-groups an XCD runs at a time then share a few row and
// column panels of W in that XCD's L2 instead of sweeping all of W.
// Returns false for slots outside the triangle or past the last tile row T.
__device__ __forceinline__ bool super_tile(int64_t slot, int64_t T, int stl, int64_t &P, int64_t &Q)
{
    if (slot < 0) return false;
    const int lb = (stl & 7) ? (stl & 7) : 3;
    const int64_t st = slot >> (2 * lb), r = slot & ((1 << (2 * lb)) - 1);
    const int64_t SP = tri_row(st), SQ = st - SP * (SP + 1) / 2;
    const int64_t lo = r & ((1 << lb) - 1), hi = r >> lb;
    P = (SP << lb) + ((stl & 8) ? hi : lo);
    Q = (SQ << lb) + ((stl & 8) ? lo : hi);
    return P < T && Q <= P;
}

// Work-group id -> work item, XCD by XCD: work-group g runs on XCD g % 8, and the items are
// handed out so that each XCD processes one contiguous eighth of them.
__device__ __forceinline__ int64_t xcd_item(int64_t wg, int64_t per_xcd) { return (wg & 7) * per_xcd + (wg >> 3); }

}  // namespace oed
