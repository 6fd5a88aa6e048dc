// Small device helpers shared by the kernel files of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecnt {

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2.  Remap the hardware block id so that each XCD walks a
// contiguous range of logical tiles: neighbouring rows (stencil neighbours,
// rows sharing CSR columns) then meet in the same L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nb)
{
    const int64_t per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

template <typename T>
__device__ __forceinline__ double ld(const T *p, size_t i)
{
    return static_cast<double>(p[i]);
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Segment holding x: off[b] <= x < off[b+1] (off ascending, off[0] = 0).
__device__ __forceinline__ int find_seg(const int64_t *__restrict__ off, int nseg, int64_t x)
{
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Two-phase column sums, second phase: the sum over the row chunks
// [ch0, ch1) of part[(ch * rows + row) * C + c] for column c = lane's column,
// computed by the kFinWaves wavefronts of a block (wavefront w takes chunks
// ch0 + w, ch0 + w + kFinWaves, ...; the partial sums are added in wavefront
// order, so the result is reproducible).  Every thread of the block must call
// it (it synchronizes the block); the sum is returned to all of them.
constexpr int kFinWaves = 8;

__device__ __forceinline__ double block_chunk_sum(const double *__restrict__ part, int rows,
                                                  int C, int row, int c, int64_t ch0, int64_t ch1,
                                                  bool valid)
{
    __shared__ double red[kFinWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // four running sums per wavefront (chunks ch, ch + kFinWaves, ... taken in
    // turn), so four loads are in flight; combined in a fixed order
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (valid) {
        int64_t ch = ch0 + w;
        for (; ch + 3 * kFinWaves < ch1; ch += 4 * kFinWaves) {
            s0 += part[((size_t)ch * rows + row) * C + c];
            s1 += part[((size_t)(ch + kFinWaves) * rows + row) * C + c];
            s2 += part[((size_t)(ch + 2 * kFinWaves) * rows + row) * C + c];
            s3 += part[((size_t)(ch + 3 * kFinWaves) * rows + row) * C + c];
        }
        for (; ch < ch1; ch += kFinWaves) s0 += part[((size_t)ch * rows + row) * C + c];
    }
    const double s = (s0 + s1) + (s2 + s3);
    red[w][lane] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kFinWaves; ++q) t += red[q][lane];
    __syncthreads();
    return t;
}

// VW consecutive columns per lane, moved as one vector load/store.
template <typename T, int VW> struct VecT;
template <> struct VecT<double, 1> { using type = double; };
template <> struct VecT<double, 2> { using type = double2; };
template <> struct VecT<float, 1> { using type = float; };
template <> struct VecT<float, 2> { using type = float2; };
template <> struct VecT<float, 4> { using type = float4; };

template <typename T, int VW>
__device__ __forceinline__ void vload(const T *__restrict__ p, size_t e, double (&o)[VW])
{
    using V = typename VecT<T, VW>::type;
    const V v = *reinterpret_cast<const V *>(p + e);
    if constexpr (VW == 1) {
        o[0] = static_cast<double>(v);
    } else if constexpr (VW == 2) {
        o[0] = static_cast<double>(v.x);
        o[1] = static_cast<double>(v.y);
    } else {
        o[0] = static_cast<double>(v.x);
        o[1] = static_cast<double>(v.y);
        o[2] = static_cast<double>(v.z);
        o[3] = static_cast<double>(v.w);
    }
}

// The same load marked non-temporal: for streams read once per launch (the
// Lanczos basis in the reorthogonalization sweeps), so that they do not evict
// what is reused from the caches.
template <typename T, int VW>
__device__ __forceinline__ void vload_nt(const T *__restrict__ p, size_t e, double (&o)[VW])
{
    if constexpr (sizeof(T) * VW == 8) {
        const double raw = __builtin_nontemporal_load(reinterpret_cast<const double *>(p + e));
        if constexpr (VW == 1) {
            o[0] = raw;
        } else {
            T t[VW];
            __builtin_memcpy(t, &raw, sizeof raw);
#pragma unroll
            for (int v = 0; v < VW; ++v) o[v] = static_cast<double>(t[v]);
        }
    } else if constexpr (sizeof(T) * VW == 4) {
        o[0] = static_cast<double>(__builtin_nontemporal_load(reinterpret_cast<const float *>(p + e)));
    } else {
        vload<T, VW>(p, e, o);
    }
}

// vload_nt without the conversion: the values stay in the storage type (half
// the registers for FP32) until they are used
template <typename T, int VW>
__device__ __forceinline__ void vload_nt_raw(const T *__restrict__ p, size_t e, T (&o)[VW])
{
    if constexpr (sizeof(T) * VW == 8 && VW == 1) {
        o[0] = __builtin_nontemporal_load(reinterpret_cast<const double *>(p + e));
    } else if constexpr (sizeof(T) * VW == 8 && VW == 2) {
        // two floats in one 8-byte load, split by bit casts (no memory copy)
        const unsigned long long bits =
            __builtin_nontemporal_load(reinterpret_cast<const unsigned long long *>(p + e));
        o[0] = __uint_as_float((unsigned)(bits & 0xffffffffull));
        o[1] = __uint_as_float((unsigned)(bits >> 32));
    } else if constexpr (sizeof(T) * VW == 4) {
        o[0] = __builtin_nontemporal_load(reinterpret_cast<const float *>(p + e));
    } else {
        double t[VW];
        vload<T, VW>(p, e, t);
#pragma unroll
        for (int v = 0; v < VW; ++v) o[v] = static_cast<T>(t[v]);
    }
}

template <typename T, int VW>
__device__ __forceinline__ void vstore(T *__restrict__ p, size_t e, const double (&o)[VW])
{
    using V = typename VecT<T, VW>::type;
    V v;
    if constexpr (VW == 1) {
        v = static_cast<T>(o[0]);
    } else if constexpr (VW == 2) {
        v.x = static_cast<T>(o[0]);
        v.y = static_cast<T>(o[1]);
    } else {
        v.x = static_cast<T>(o[0]);
        v.y = static_cast<T>(o[1]);
        v.z = static_cast<T>(o[2]);
        v.w = static_cast<T>(o[3]);
    }
    *reinterpret_cast<V *>(p + e) = v;
}

// vstore with the non-temporal hint: the line is not kept in the caches for
// reuse (outputs that no later access of the same launch reads).
template <typename T, int VW>
__device__ __forceinline__ void vstore_nt(T *__restrict__ p, size_t e, const double (&o)[VW])
{
    if constexpr (VW == 1) {
        __builtin_nontemporal_store(static_cast<T>(o[0]), p + e);
    } else {
        typedef T TV __attribute__((ext_vector_type(VW)));
        TV v;
#pragma unroll
        for (int i = 0; i < VW; ++i) v[i] = static_cast<T>(o[i]);
        __builtin_nontemporal_store(v, reinterpret_cast<TV *>(p + e));
    }
}

// Value after rounding to the storage type T (what a later load returns).
template <typename T>
__device__ __forceinline__ double rounded(double x)
{
    return static_cast<double>(static_cast<T>(x));
}

// sum over the 16 lanes of a row of the wavefront (every lane gets the same
// value: each butterfly stage adds two equal partial sums in either order)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    // every lane has a source under a row rotation: bound_ctrl set, no old value
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row_sum16(double x)
{
    x += dpp_f64<0x128>(x);   // row_ror:8
    x += dpp_f64<0x124>(x);   // row_ror:4
    x += dpp_f64<0x122>(x);   // row_ror:2
    x += dpp_f64<0x121>(x);   // row_ror:1
    return x;
}
// sum over the 4 rows of the wavefront (lanes l, l^16, l^32, l^48), by the
// row swaps of v_permlane16_swap / v_permlane32_swap (both halves of a pair
// get the same operands in the same order, so all four lanes agree)
__device__ __forceinline__ double group_sum4(double x)
{
    int lo = __double2loint(x), hi = __double2hiint(x);
    auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    x = __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
    lo = __double2loint(x);
    hi = __double2hiint(x);
    a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}

// sum over the wavefront in VALU (DPP row rotations, then the row swaps):
// every lane gets the same value, in a fixed order
__device__ __forceinline__ double wave_sum_dpp(double x) { return group_sum4(row_sum16(x)); }

// 1/sqrt(x) for a positive, finite, normal x (no special-case handling): the
// hardware estimate y0 refined by the series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8
// + ... to second order, e = 1 - x y0^2.
__device__ __forceinline__ double rsqrt_pos(double x)
{
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y0, y0, 1.0);
    return fma(y0 * e, fma(e, 0.375, 0.5), y0);
}

}  // namespace ecnt
