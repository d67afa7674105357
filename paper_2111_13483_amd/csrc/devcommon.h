// Device helpers shared by the gfx950 kernels: complex arithmetic on
// interleaved doubles, wavefront (64-lane) and workgroup reductions, and the
// device-side error flag.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"

namespace hs {

typedef double2 cd;   // {re, im}
typedef float2 cf;    // complex64 storage of the mixed-precision operator copies

// matrix element loads: complex128 as stored, complex64 widened to complex128
__device__ __forceinline__ cd to_cd(cd v) { return v; }
__device__ __forceinline__ cd to_cd(cf v) {
    cd z;
    z.x = (double)v.x;
    z.y = (double)v.y;
    return z;
}

__device__ __forceinline__ cd cmk(double r, double i) { cd z; z.x = r; z.y = i; return z; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return cmk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd csub(cd a, cd b) { return cmk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd cmul(cd a, cd b) { return cmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cd cconj(cd a) { return cmk(a.x, -a.y); }
__device__ __forceinline__ cd cscale(cd a, double s) { return cmk(a.x * s, a.y * s); }
// a + b * c
__device__ __forceinline__ cd cfma(cd b, cd c, cd a) {
    return cmk(fma(b.x, c.x, fma(-b.y, c.y, a.x)), fma(b.x, c.y, fma(b.y, c.x, a.y)));
}
// a + conj(b) * c
__device__ __forceinline__ cd cfmac(cd b, cd c, cd a) {
    return cmk(fma(b.x, c.x, fma(b.y, c.y, a.x)), fma(b.x, c.y, fma(-b.y, c.x, a.y)));
}
// |a|^2 rounded as re*re + im*im with no contraction (pivot decisions)
__device__ __forceinline__ double cabs2_exact(cd a) {
    double r2 = __dmul_rn(a.x, a.x);
    double i2 = __dmul_rn(a.y, a.y);
    return __dadd_rn(r2, i2);
}
__device__ __forceinline__ double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ cd cdiv(cd a, cd b) {
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return cmk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        double r = b.x / b.y, d = b.y + b.x * r;
        return cmk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}

constexpr int kWave = 64;

// Lane moves of a double by DPP (the whole wave must be active) and a read
// of one lane's value into every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the wave (every lane active), the same value in every lane: DPP
// sums within each row of 16 lanes (quad_perm [1,0,3,2], [2,3,0,1], then
// row_ror 4 and 8), then lane 0's sums of the four rows. DPP moves run in the
// vector ALU; lane shuffles would go through the LDS crossbar.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x124>(v);
    v += dpp_f64<0x128>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}
__device__ __forceinline__ cd wave_sum(cd v) { return cmk(wave_sum(v.x), wave_sum(v.y)); }

// ---- complex64 arithmetic (the mixed path's copies compute in FP32) ----
// Arith<T>: the type a kernel computes in for matrix storage T. complex128
// storage computes in FP64; complex64 copies compute in FP32 with FP32
// accumulation, their FP64 input vectors narrowed on load and the results
// widened on store.
template <class T> struct Arith;
template <> struct Arith<cd> { typedef cd type; };
template <> struct Arith<cf> { typedef cf type; };
template <class T> using arith_t = typename Arith<T>::type;

__device__ __forceinline__ cf cmkf(float r, float i) { cf z; z.x = r; z.y = i; return z; }
template <class A> __device__ __forceinline__ A czero();
template <> __device__ __forceinline__ cd czero<cd>() { return cmk(0.0, 0.0); }
template <> __device__ __forceinline__ cf czero<cf>() { return cmkf(0.0f, 0.0f); }
template <class A> __device__ __forceinline__ A to_arith(cd v);
template <> __device__ __forceinline__ cd to_arith<cd>(cd v) { return v; }
template <> __device__ __forceinline__ cf to_arith<cf>(cd v) { return cmkf((float)v.x, (float)v.y); }
template <class A> __device__ __forceinline__ A to_arith(cf v);
template <> __device__ __forceinline__ cf to_arith<cf>(cf v) { return v; }
template <> __device__ __forceinline__ cd to_arith<cd>(cf v) { return to_cd(v); }
__device__ __forceinline__ cf cadd(cf a, cf b) { return cmkf(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cf cmul(cf a, cf b) { return cmkf(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ cf cfma(cf b, cf c, cf a) {
    return cmkf(fmaf(b.x, c.x, fmaf(-b.y, c.y, a.x)), fmaf(b.x, c.y, fmaf(b.y, c.x, a.y)));
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float readlane_f32(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// the same reduction order as the FP64 wave_sum
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f32<0xB1>(v);
    v += dpp_f32<0x4E>(v);
    v += dpp_f32<0x124>(v);
    v += dpp_f32<0x128>(v);
    return (readlane_f32(v, 0) + readlane_f32(v, 16)) + (readlane_f32(v, 32) + readlane_f32(v, 48));
}
__device__ __forceinline__ cf wave_sum(cf v) { return cmkf(wave_sum(v.x), wave_sum(v.y)); }

// Argmax with ties to the lowest index; key < 0 marks "no candidate".
struct ArgMax { double v; int i; };
__device__ __forceinline__ ArgMax amax_pick(ArgMax a, ArgMax b) {
    if (b.v > a.v || (b.v == a.v && b.i < a.i && b.v >= 0.0)) return b;
    return a;
}
// Over the wave (every lane active): the largest value, ties to the lowest
// index among the lanes holding it (NaN never wins).
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ ArgMax wave_argmax(ArgMax a) {
    double vm = a.v;
    vm = fmax(vm, dpp_f64<0xB1>(vm));
    vm = fmax(vm, dpp_f64<0x4E>(vm));
    vm = fmax(vm, dpp_f64<0x124>(vm));
    vm = fmax(vm, dpp_f64<0x128>(vm));
    vm = fmax(fmax(readlane_f64(vm, 0), readlane_f64(vm, 16)), fmax(readlane_f64(vm, 32), readlane_f64(vm, 48)));
    int im = (a.v == vm) ? a.i : 0x7fffffff;
    im = min(im, dpp_i32<0xB1>(im));
    im = min(im, dpp_i32<0x4E>(im));
    im = min(im, dpp_i32<0x124>(im));
    im = min(im, dpp_i32<0x128>(im));
    im = min(min(__builtin_amdgcn_readlane(im, 0), __builtin_amdgcn_readlane(im, 16)),
             min(__builtin_amdgcn_readlane(im, 32), __builtin_amdgcn_readlane(im, 48)));
    ArgMax r;
    r.v = vm;
    r.i = im;
    return r;
}

// Workgroup reductions through a caller-provided LDS scratch of >= nwaves entries.
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red) {
    constexpr int NW = NT / kWave;
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NW; ++i) s += red[i];
    return s;
}

template <int NT>
__device__ __forceinline__ ArgMax wg_argmax(ArgMax a, double* redv, int* redi) {
    constexpr int NW = NT / kWave;
    a = wave_argmax(a);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) { redv[w] = a.v; redi[w] = a.i; }
    __syncthreads();
    ArgMax r; r.v = redv[0]; r.i = redi[0];
#pragma unroll
    for (int i = 1; i < NW; ++i) { ArgMax b; b.v = redv[i]; b.i = redi[i]; r = amax_pick(r, b); }
    return r;
}

// Device error flags: bitwise OR into a global word (codes in kernels.h).
__device__ __forceinline__ void raise_err(int* flag, int bits) { atomicOr(flag, bits); }

}  // namespace hs
