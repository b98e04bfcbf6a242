// Device helpers shared by the fKK-EC kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace fkk {
namespace dev {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// l = 1/2 ln(x r); ratios that are not finite or not above the floor are
// replaced by the floor.
__device__ __forceinline__ float log_ratio(float x, float r, float floor, bool& bad) {
    float q = x * r;
    bad = !(q > floor && q < INFINITY);
    q = bad ? floor : q;
    return 0.5f * logf(q);
}

__device__ __forceinline__ float4 load4_guarded(const float* row, int col, int N, bool vec) {
    if (vec && col + 3 < N) return *reinterpret_cast<const float4*>(row + col);
    float4 v;
    v.x = (col + 0 < N) ? row[col + 0] : 0.f;
    v.y = (col + 1 < N) ? row[col + 1] : 0.f;
    v.z = (col + 2 < N) ? row[col + 2] : 0.f;
    v.w = (col + 3 < N) ? row[col + 3] : 0.f;
    return v;
}

__device__ __forceinline__ float f4get(const float4& v, int q) {
    return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

// exp(x) = 2^(x log2 e) on the hardware exp2 (relative error a few ulp for
// the exponent range of log-ratio spectra).
__device__ __forceinline__ float exp_fast(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// sin and cos by reduction to r in [-pi/4, pi/4] (three-part Cody-Waite
// split of pi/2; n * 1.5703125 is exact for |n| < 2^16) and Taylor
// polynomials through r^9 (sin) and r^10 (cos), truncation error below
// 2e-9 and 2e-11.
__device__ __forceinline__ void sincos_fast(float x, float* sn, float* cs) {
    const float n = rintf(x * 0.636619772367581343f);
    float r = fmaf(-n, 1.5703125f, x);
    r = fmaf(-n, 4.83826794896619231e-4f, r);
    r = fmaf(-n, 2.56328311e-12f, r);
    const float r2 = r * r;
    float ps = fmaf(r2, 2.75573192e-6f, -1.98412698e-4f);
    ps = fmaf(r2, ps, 8.33333333e-3f);
    ps = fmaf(r2, ps, -1.66666667e-1f);
    const float s = fmaf(r * r2, ps, r);
    float pc = fmaf(r2, -2.75573192e-7f, 2.48015873e-5f);
    pc = fmaf(r2, pc, -1.38888889e-3f);
    pc = fmaf(r2, pc, 4.16666667e-2f);
    pc = fmaf(r2, pc, -0.5f);
    const float c = fmaf(r2, pc, 1.0f);
    const int q = ((int)n) & 3;
    *sn = (q == 0) ? s : (q == 1) ? c : (q == 2) ? -s : -c;
    *cs = (q == 0) ? c : (q == 1) ? -s : (q == 2) ? -c : s;
}

}  // namespace dev
}  // namespace fkk
