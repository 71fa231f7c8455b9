// Device-side building blocks of the shifted COCG solve (gfx950, wave64).
//
// Every function here runs inside ONE workgroup that owns one right-hand
// side from start to finish: vectors are split over the workgroup's threads
// by scalar row (row i belongs to thread i mod NT), reductions go through a
// wave butterfly and then a fixed-order sum over the waves in LDS, so that a
// run is bitwise reproducible.  The only synchronisation is __syncthreads().
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace scocg {

// ---------------------------------------------------------------------------
// complex helpers (double2 / float2 hold (re, im))
// ---------------------------------------------------------------------------
template <class T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float>  { using type = float2; };
template <class T> using v2 = typename vec2<T>::type;

struct zc { double re, im; };   // FP64 complex scalar in registers

__device__ __forceinline__ zc zmk(double r, double i) { return zc{r, i}; }
__device__ __forceinline__ zc zadd(zc a, zc b) { return zc{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ zc zsub(zc a, zc b) { return zc{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ zc zmul(zc a, zc b) {
    return zc{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// Smith's algorithm for a / b (scaled, avoids overflow for large |b|).
__device__ __forceinline__ zc zdiv(zc a, zc b) {
    if (fabs(b.re) >= fabs(b.im)) {
        double t = b.im / b.re, den = b.re + b.im * t;
        return zc{(a.re + a.im * t) / den, (a.im - a.re * t) / den};
    } else {
        double t = b.re / b.im, den = b.re * t + b.im;
        return zc{(a.re * t + a.im) / den, (a.im * t - a.re) / den};
    }
}
__device__ __forceinline__ double zabs(zc a) { return hypot(a.re, a.im); }
__device__ __forceinline__ bool zfinite(zc a) { return isfinite(a.re) && isfinite(a.im); }
__device__ __forceinline__ bool zzero(zc a) { return a.re == 0.0 && a.im == 0.0; }

template <class T> __device__ __forceinline__ zc ld(const v2<T>* p, int64_t i) {
    v2<T> v = p[i];
    return zc{(double)v.x, (double)v.y};
}
// The value a complex number takes once stored in precision T (no memory trip).
template <class T> __device__ __forceinline__ zc rnd(zc a) {
    return zc{(double)(T)a.re, (double)(T)a.im};
}
template <class T> __device__ __forceinline__ void st(v2<T>* p, int64_t i, zc a) {
    v2<T> v;
    v.x = (T)a.re;
    v.y = (T)a.im;
    p[i] = v;
}

// ---------------------------------------------------------------------------
// block storage: FP64, FP32 or bfloat16 (upper half of an IEEE float)
// ---------------------------------------------------------------------------
struct bf16_t { uint16_t bits; };
__device__ __forceinline__ double bval(const double* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float  bval(const float* p, int64_t i) { return p[i]; }
__device__ __forceinline__ float  bval(const bf16_t* p, int64_t i) {
    return __uint_as_float(((uint32_t)p[i].bits) << 16);
}

// ---------------------------------------------------------------------------
// quad broadcast: every lane of a group of four gets lane C's value (DPP
// quad_perm, no LDS traffic).  Used where the four rows of a 4x4 block row
// sit in the four lanes of a quad and each needs all four vector entries.
// ---------------------------------------------------------------------------
template <int C>
__device__ __forceinline__ int quad_bcast_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, C * 0x55, 0xF, 0xF, false);
}
template <int C>
__device__ __forceinline__ double quad_bcast(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)quad_bcast_i32<C>((int)(unsigned)(b & 0xffffffffLL));
    const unsigned hi = (unsigned)quad_bcast_i32<C>((int)(unsigned)((unsigned long long)b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int C>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(quad_bcast_i32<C>(__float_as_int(v)));
}
template <int C, class V>
__device__ __forceinline__ V quad_bcast2(const V& v) {
    V o;
    o.x = quad_bcast<C>(v.x);
    o.y = quad_bcast<C>(v.y);
    return o;
}

// ---------------------------------------------------------------------------
// wavefront reductions by DPP row operations (no LDS traffic); every lane of
// the wavefront must be active
// ---------------------------------------------------------------------------
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffLL), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)((unsigned long long)b >> 32), CTRL, ROWS, 0xF,
                                               false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double readlane64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffLL), lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Sum over the 16 lanes of each row (every lane gets its row's sum).
__device__ __forceinline__ double row16_sum(double v) {
    v += dpp64<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp64<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp64<0x124, 0xF>(v);   // row_ror 4: the neighbouring quad
    v += dpp64<0x128, 0xF>(v);   // row_ror 8: the other two quads
    return v;
}
// Sum over the whole wavefront (returned in every lane, a uniform value).
__device__ __forceinline__ double wave_total(double v) {
    v = row16_sum(v);
    v += dpp64<0x142, 0xA>(v);   // row_bcast 15: rows 1, 3 add the last lane of rows 0, 2
    v += dpp64<0x143, 0xC>(v);   // row_bcast 31: rows 2, 3 add lane 31 (rows 0 + 1)
    return readlane64(v, 63);
}

// ---------------------------------------------------------------------------
// workgroup reductions (deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) { return wave_total(v); }

// Sum N doubles over the workgroup; every thread gets the totals.
// `red` is LDS scratch of at least (NT/64)*N doubles.
template <int NT, int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < N; ++n) v[n] = wave_sum(v[n]);
    if (lane == 0) {
#pragma unroll
        for (int n = 0; n < N; ++n) red[w * N + n] = v[n];
    }
    __syncthreads();
#pragma unroll
    for (int n = 0; n < N; ++n) {
        double s = 0.0;
        for (int q = 0; q < NW; ++q) s += red[q * N + n];
        v[n] = s;
    }
    __syncthreads();
}

}  // namespace scocg
