// Device helpers shared by the fKK-EC kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

namespace fkk {
namespace dev {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ln q for a normal, finite q > 0: the hardware base-2 logarithm times ln 2
// carried as two floats (0x3f317217 + 0x3377d1cf), with the product's
// rounding error put back.  These are the operations logf performs for such
// an argument, so the results are logf's bit for bit; logf's other steps
// (scaling a subnormal argument, passing infinity through) are left out.
__device__ __forceinline__ float log_normal(float q) {
    const float y = __builtin_amdgcn_logf(q);
    const float hi = __builtin_bit_cast(float, 0x3f317217u), lo = __builtin_bit_cast(float, 0x3377d1cfu);
    const float p = hi * y;
    float e = fmaf(y, hi, -p);
    e = fmaf(y, lo, e);
    return fmaf(hi, y, e);
}

// l = 1/2 ln(x r) with r = 1/I_ref given as rh + rl (two floats): one
// rounding of the product x (rh + rl).  A single-float r would shift every
// l of a column by the same ~3e-8 and that offset adds up coherently over
// all rows of the Gram.  Ratios that are not finite or not above the floor
// are replaced by the floor, which the host keeps at or above 2^-126, so
// the logarithm always sees a normal number.
__device__ __forceinline__ float log_ratio(float x, float rh, float rl, float floor, bool& bad) {
    float q = fmaf(x, rh, x * rl);
    bad = !(q > floor && q < INFINITY);
    q = bad ? floor : q;
    return 0.5f * log_normal(q);
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


// Output plane PLANE of K = exp(re) exp(i im) (Eq. 23): 0 Im, 1 Re, 2 |K|.
template <int PLANE>
__device__ __forceinline__ float epilogue(float re, float im) {
    const float mag = exp_fast(re);
    if (PLANE == 2) return mag;
    float sn, cs;
    sincos_fast(im, &sn, &cs);
    return mag * (PLANE == 0 ? sn : cs);
}

// Same with the hardware sine / cosine (v_sin_f32 / v_cos_f32 take the
// angle in revolutions; the fraction of a revolution keeps the argument in
// [-1/2, 1/2]).  Absolute error of order 1e-6: used where the operands are
// BF16 and contribute far more.
template <int PLANE>
__device__ __forceinline__ float epilogue_hw(float re, float im) {
    const float mag = exp_fast(re);
    if (PLANE == 2) return mag;
    float t = im * 0.159154943091895336f;
    t -= rintf(t);
    return mag * (PLANE == 0 ? __builtin_amdgcn_sinf(t) : __builtin_amdgcn_cosf(t));
}

// Epilogue of a 128-spectrum reconstruction tile over 16 NIB wavenumbers:
// lane l of wave w holds, in acc[ib][jb][v], wavenumber j0 + 16 ib +
// 4 (l/16) + v of spectrum r0 + 32 w + 16 jb + l%16.  All values of a lane
// are evaluated in one straight-line block before any store; only the
// stores are guarded, and a tile that lies inside the matrix takes an
// unguarded path.
template <int PLANE, bool VEC_OUT, bool HW_SIN, int NIB>
__device__ __forceinline__ void store_plane(float* __restrict__ out, int64_t ld_out, int64_t M, int N, int64_t r0,
                                            int wave, int lane, int j0, const floatx4 (&are)[NIB][2],
                                            const floatx4 (&aim)[NIB][2]) {
    float o[NIB][2][4];
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                o[ib][jb][v] = HW_SIN ? epilogue_hw<PLANE>(are[ib][jb][v], aim[ib][jb][v])
                                      : epilogue<PLANE>(are[ib][jb][v], aim[ib][jb][v]);
    const int64_t row0 = r0 + wave * 32 + (lane & 15);
    const int col0 = j0 + 4 * (lane >> 4);
    if (VEC_OUT && j0 + 16 * NIB <= N && r0 + 128 <= M) {  // uniform: whole tile inside
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb)
                *reinterpret_cast<float4*>(out + (row0 + jb * 16) * ld_out + col0 + ib * 16) =
                    make_float4(o[ib][jb][0], o[ib][jb][1], o[ib][jb][2], o[ib][jb][3]);
        return;
    }
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            const int64_t row = row0 + jb * 16;
            const int col = col0 + ib * 16;
            if (row >= M) continue;
            float* dst = out + row * ld_out + col;
            if (VEC_OUT && col + 3 < N) {
                *reinterpret_cast<float4*>(dst) = make_float4(o[ib][jb][0], o[ib][jb][1], o[ib][jb][2], o[ib][jb][3]);
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (col + v < N) dst[v] = o[ib][jb][v];
            }
        }
}

// The plane is chosen once per tile, outside the per-value code.
template <bool VEC_OUT, bool HW_SIN = false, int NIB = 4>
__device__ __forceinline__ void store_out(float* __restrict__ out, int64_t ld_out, int64_t M, int N, int64_t r0,
                                          int wave, int lane, int j0, const floatx4 (&are)[NIB][2],
                                          const floatx4 (&aim)[NIB][2], int plane) {
    if (plane == 0) store_plane<0, VEC_OUT, HW_SIN, NIB>(out, ld_out, M, N, r0, wave, lane, j0, are, aim);
    else if (plane == 1) store_plane<1, VEC_OUT, HW_SIN, NIB>(out, ld_out, M, N, r0, wave, lane, j0, are, aim);
    else store_plane<2, VEC_OUT, HW_SIN, NIB>(out, ld_out, M, N, r0, wave, lane, j0, are, aim);
}


// ---- per-spectrum sums for the basis residual (retraining criterion, Sec. 5)
// With A = l diag(f), a spectrum's relative residual against the basis is
// ||A_m - A_m V V^T||^2 / ||A_m||^2 = 1 - ||A_m V||^2 / ||A_m||^2; the kernels
// below write the two sums of each row m as norms[2m] and norms[2m + 1].

// Sum over the 16 lanes that differ in their four low bits.
__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

// ||A_m||^2 from the staging loop's partial sums: thread t of the block
// staged rows (t >> 4) + 16 p (p < 8), four columns at a time.
__device__ __forceinline__ void store_anorms(const float (&asq)[8], float* __restrict__ norms, int64_t r0,
                                             int64_t M) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const float v = sum16(asq[p]);
        const int64_t row = r0 + (tid >> 4) + 16 * p;
        if ((tid & 15) == 0 && row < M) norms[2 * row] = v;
    }
}

// ||A_m V||^2 from a projection tile held as in project_finish (acc[rb][cb][v]
// = Z[r0 + 32 w + 16 rb + 4 (l/16) + v][16 cb + l%16]), with Z = A W and
// g[c] = 1 / shrink_c (0 for a dropped vector), so Z_c g_c = (A V)_c.
template <int KB>
__device__ __forceinline__ void store_znorms(const floatx4 (&acc)[2][KB], const float* __restrict__ g,
                                             float* __restrict__ norms, int64_t r0, int64_t M) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float gl[KB];
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) gl[cb] = g[16 * cb + (lane & 15)];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            float sq = 0.f;
#pragma unroll
            for (int cb = 0; cb < KB; ++cb) {
                const float z = acc[rb][cb][v] * gl[cb];
                sq = fmaf(z, z, sq);
            }
            sq = sum16(sq);
            const int64_t row = r0 + wave * 32 + rb * 16 + 4 * (lane >> 4) + v;
            if ((lane & 15) == 0 && row < M) norms[2 * row + 1] = sq;
        }
}

__device__ __forceinline__ void better_max(float& v, int& i, float ov, int oi) {
    if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
}
__device__ __forceinline__ void better_min(float& v, int& i, float ov, int oi) {
    if (ov < v || (ov == v && oi < i)) { v = ov; i = oi; }
}

// End of a projection block of 128 spectra: lane l of wave w holds, in
// acc[rb][cb][v], Z[r0 + 32 w + 16 rb + 4 (l/16) + v][16 cb + l%16].  Stores
// the first k_store columns of Z and, when pmaxv != nullptr, the block's
// per-column arg-extrema (first row on ties) for the first k_arg columns.
template <int KB>
__device__ __forceinline__ void project_finish(const floatx4 (&acc)[2][KB], int64_t r0, int64_t M,
                                               float* __restrict__ Z, int64_t ld_z, int k_store, float* pmaxv,
                                               float* pminv, long long* pmaxi, long long* pmini, int k_arg) {
    constexpr int KP = KB * 16;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Z[row][c]: acc[rb][cb][v], row = wave*32 + rb*16 + 4*(lane/16) + v, c = cb*16 + lane%16
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < KB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = r0 + wave * 32 + rb * 16 + 4 * (lane >> 4) + v;
                const int c = cb * 16 + (lane & 15);
                if (row < M && c < k_store) Z[row * ld_z + c] = acc[rb][cb][v];
            }

    if (pmaxv == nullptr) return;
    __shared__ float smx[4][KP], smn[4][KP];
    __shared__ int smxi[4][KP], smni[4][KP];
#pragma unroll
    for (int cb = 0; cb < KB; ++cb) {
        float mx = -INFINITY, mn = INFINITY;
        int ix = INT_MAX, in = INT_MAX;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = wave * 32 + rb * 16 + 4 * (lane >> 4) + v;
                if (r0 + rl < M) {
                    better_max(mx, ix, acc[rb][cb][v], rl);
                    better_min(mn, in, acc[rb][cb][v], rl);
                }
            }
#pragma unroll
        for (int off = 16; off <= 32; off <<= 1) {
            const float omx = __shfl_xor(mx, off), omn = __shfl_xor(mn, off);
            const int oix = __shfl_xor(ix, off), oin = __shfl_xor(in, off);
            better_max(mx, ix, omx, oix);
            better_min(mn, in, omn, oin);
        }
        if (lane < 16) {
            smx[wave][cb * 16 + lane] = mx;
            smxi[wave][cb * 16 + lane] = ix;
            smn[wave][cb * 16 + lane] = mn;
            smni[wave][cb * 16 + lane] = in;
        }
    }
    __syncthreads();
    if (tid < KP && tid < k_arg) {
        float mx = smx[0][tid], mn = smn[0][tid];
        int ix = smxi[0][tid], in = smni[0][tid];
        for (int w = 1; w < 4; ++w) {
            better_max(mx, ix, smx[w][tid], smxi[w][tid]);
            better_min(mn, in, smn[w][tid], smni[w][tid]);
        }
        const size_t o = (size_t)blockIdx.x * KP + tid;
        pmaxv[o] = mx;
        pminv[o] = mn;
        pmaxi[o] = (ix == INT_MAX) ? -1 : (long long)(r0 + ix);
        pmini[o] = (in == INT_MAX) ? -1 : (long long)(r0 + in);
    }
}

}  // namespace dev
}  // namespace fkk
