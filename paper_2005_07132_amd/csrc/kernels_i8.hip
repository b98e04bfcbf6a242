// Gram of the log ratio (Eq. 6) to FP64 accuracy on the int8 matrix cores:
// error-free splitting of the operands (Ozaki, Ogita, Oishi & Rump 2012;
// for integer matrix units, Ootomo, Ozaki & Yokota 2024).
//
//   stats:  column sums of I (FP64), clamp count and max |l| per column
//           (FP32 log ratio), one pass over I.
//   exps:   e_j with max_j |l_j| < 2^e_j (with a margin for the FP64 l).
//   slices: l = 1/2 ln(I / I_ref) in FP64 (log_cells), x = l 2^-e_j in
//           (-1, 1), X = rint(x 2^27) cut into balanced base-128 digits:
//               x = 2^-6 (a1 + 2^-7 a2 + 2^-14 a3 + 2^-21 a4) + d,
//           a2..a4 in [-64, 63], |a1| <= 64, |d| <= 2^-28.
//   gram:   for each 128 x 128 tile and row chunk,
//           the int8 products S_i^T S_j summed exactly in int32, grouped by
//           level t = i + j, t = 2..6 (13 products), and
//           G_chunk = 2^(e_a + e_b - 12) sum_t 2^(-7 (t - 2)) C_t, exact in
//           FP64 (54 significant bits at most, see the flush), into the
//           chunk partials that the FP32 path reduces.  Level 6 holds the
//           (3, 3) product, which is never negative on the diagonal: dropping
//           it would bias G_aa by ~2^-40 E[a3^2] per row.  The dropped levels
//           7 and 8 are products of different digits (zero mean) and (4, 4)
//           (~2^-54 per row).
//
// Slices are stored row-group major, slice-major within a row group:
// S[g][s][j] is a 16-byte unit holding rows 16 g .. 16 g + 15 of column j,
// slice s.  v_mfma_i32_32x32x32_i8: lane l holds A[l%32][16 (l/32) + q]
// and B[16 (l/32) + q][l%32] (q = byte 0..15) and receives
// D[8 (v/4) + 4 (l/32) + v%4][l%32] in element v (measured with a one-wave
// probe), so a lane's operand is one 16-byte unit of one row group.
#include "kernels.h"
#include "device_common.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace fkk {
namespace dev {

namespace {

typedef int8_t i8x16 __attribute__((ext_vector_type(16)));
typedef int int32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

constexpr int ST_ROWS = 256;  // rows per stats block
constexpr int GT = kGramTile;
constexpr int I8_THREADS = 512;  // 8 waves: 2 (a) x 4 (b), 64 x 32 of the tile each
constexpr int KROWS = 64;        // rows per K step (4 row groups)

// ---------------------------------------------------------------------------
// stats: column sums of I, clamp count, per-block max |l| (FP32 log ratio)
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256) void stats_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                    const float* __restrict__ rinv, float floor, int npad,
                                                    double* __restrict__ colsum_part, float* __restrict__ colmax_part,
                                                    unsigned long long* __restrict__ clamps) {
    const int64_t r0 = (int64_t)blockIdx.x * ST_ROWS;
    const int64_t r1 = (r0 + ST_ROWS < M) ? r0 + ST_ROWS : M;
    unsigned int cnt = 0;
    for (int g0 = 0; g0 < npad; g0 += 1024) {
        const int c = g0 + 4 * (int)threadIdx.x;
        if (c >= npad) continue;
        float r[4], rl[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            r[q] = (c + q < N) ? rinv[c + q] : 0.f;
            rl[q] = (c + q < N) ? rinv[N + c + q] : 0.f;
        }
        double cs[4] = {0.0, 0.0, 0.0, 0.0};
        float mx[4] = {0.f, 0.f, 0.f, 0.f};
        for (int64_t row0 = r0; row0 < r1; row0 += 4) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                x[u] = (row0 + u < r1) ? load4_guarded(I + (row0 + u) * ld, c, N, VEC) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (row0 + u >= r1) break;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (c + q >= N) continue;
                    bool bad;
                    const float xv = f4get(x[u], q);
                    const float l = log_ratio(xv, r[q], rl[q], floor, bad);
                    cnt += bad ? 1u : 0u;
                    cs[q] += (double)xv;
                    mx[q] = fmaxf(mx[q], fabsf(l));
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            colsum_part[(size_t)blockIdx.x * npad + c + q] = cs[q];
            colmax_part[(size_t)blockIdx.x * npad + c + q] = mx[q];
        }
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(clamps, (unsigned long long)cnt);
}

// Column maxima over the per-block partials in two steps: colmax_group_kernel
// takes the max over part groups (grid.y of them) for 64 columns per block,
// colexp_kernel the max over the groups and the exponent e_j with
// |l_j| < 2^e_j over all rows, from the FP32 maximum with room for the FP64
// log ratio (within 2^-21 relative + 2^-24 absolute of the FP32 one).
constexpr int kMaxGroups = 32;
__global__ __launch_bounds__(256) void colmax_group_kernel(const float* __restrict__ colmax_part, int64_t nparts,
                                                           int npad, float* __restrict__ gmax) {
    __shared__ float red[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), sub = threadIdx.x >> 6;
    const int64_t stride = (int64_t)gridDim.y * 4;
    float m = 0.f;
    if (c < npad)
        for (int64_t b = (int64_t)blockIdx.y * 4 + sub; b < nparts; b += stride)
            m = fmaxf(m, colmax_part[(size_t)b * npad + c]);
    red[sub][threadIdx.x & 63] = m;
    __syncthreads();
    if (sub == 0 && c < npad) {
        m = fmaxf(fmaxf(red[0][threadIdx.x], red[1][threadIdx.x]), fmaxf(red[2][threadIdx.x], red[3][threadIdx.x]));
        gmax[(size_t)blockIdx.y * npad + c] = m;
    }
}

__global__ void colexp_kernel(const float* __restrict__ gmax, int groups, int npad, int N, int margin,
                              int* __restrict__ colexp) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= npad) return;
    float m = 0.f;
    if (j < N)
        for (int g = 0; g < groups; ++g) m = fmaxf(m, gmax[(size_t)g * npad + j]);
    const double bound = (double)m * (1.0 + 0x1p-16) + 0x1p-20;
    int e;
    frexp(bound, &e);  // bound = f 2^e, 1/2 <= f < 1, so bound < 2^e
    colexp[j] = e + margin;
}

// Column maxima of |l| over every stride-th row only (FP32 log ratio as in
// stats_kernel): SAMPLE_ROWS sampled rows per block.  The exponents taken
// from them get one bit of headroom; a row outside it is caught by the
// slicing pass's overflow flag.
constexpr int SAMPLE_ROWS = 64;
constexpr int SAMPLE_BATCH = 8;  // sampled rows whose loads are in flight together
template <bool VEC>
__global__ __launch_bounds__(256) void sample_max_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                         const float* __restrict__ rinv, float floor, int npad,
                                                         int stride, float* __restrict__ colmax_part) {
    const int64_t nsamp = (M + stride - 1) / stride;
    const int64_t t0 = (int64_t)blockIdx.x * SAMPLE_ROWS;
    const int64_t t1 = (t0 + SAMPLE_ROWS < nsamp) ? t0 + SAMPLE_ROWS : nsamp;
    for (int g0 = 0; g0 < npad; g0 += 1024) {
        const int c = g0 + 4 * (int)threadIdx.x;
        if (c >= npad) continue;
        float r[4], rl[4], mx[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            r[q] = (c + q < N) ? rinv[c + q] : 0.f;
            rl[q] = (c + q < N) ? rinv[N + c + q] : 0.f;
        }
        // batches of SAMPLE_BATCH rows: all loads first (rows past the
        // block's last sample read that sample again, which changes no
        // maximum), then the log ratios
        for (int64_t tb = t0; tb < t1; tb += SAMPLE_BATCH) {
            float4 x[SAMPLE_BATCH];
#pragma unroll
            for (int u = 0; u < SAMPLE_BATCH; ++u) {
                const int64_t t = (tb + u < t1) ? tb + u : t1 - 1;
                x[u] = load4_guarded(I + t * stride * ld, c, N, VEC);
            }
#pragma unroll
            for (int u = 0; u < SAMPLE_BATCH; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (c + q >= N) continue;
                    bool bad;
                    const float l = log_ratio(f4get(x[u], q), r[q], rl[q], floor, bad);
                    mx[q] = fmaxf(mx[q], fabsf(l));
                }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) colmax_part[(size_t)blockIdx.x * npad + c + q] = mx[q];
    }
}

// ---------------------------------------------------------------------------
// slices: one thread per (row group, column)
// ---------------------------------------------------------------------------
// ln q in FP64 for q > 0 (finite): q = mant 2^k, mant in [1/2, 1); mant =
// c (1 + u) with c the centre of mant's 1/128-wide cell (tab: 1/c, ln c), so
// |u| <= 1/128 and ln(1 + u) = u - u^2/2 + ... + u^5/5 leaves below 4e-14.
__device__ __forceinline__ double log_cells(double q, const double* tab) {
    int k;
    const double mant = frexp(q, &k);
    const int i = (int)fma(mant, 128.0, -64.0);  // 0..63
    const double u = fma(mant, tab[2 * i], -1.0);
    double p = fma(u, 0.2, -0.25);
    p = fma(u, p, 1.0 / 3.0);
    p = fma(u, p, -0.5);
    p = fma(u, p, 1.0);
    return fma((double)k, 0.69314718055994530942, fma(u, p, tab[2 * i + 1]));
}

// Slices, FP64 column sums and the clamp count in one pass over I.  A block
// takes ST_ROWS rows (16 row groups) of 256 columns, one column per thread,
// rows in order, so the column-sum partials have stats_kernel's layout and
// summation order; the next row group's loads are in flight while one is
// computed.  Digits: with Y = X + 64 (1 + 2^7 + 2^14 + 2^21) > 0, the
// balanced digits are a_s = y_s - 64 for the base-128 digits y_s of Y (a1
// from y1 = Y >> 21 <= 128), so each is one bit-field extract; four rows'
// bytes are packed per dword and moved to two's complement together:
// (y + 64) ^ 0x80 for y1, ((y | 0x80) - 0x40) ^ 0x80 for y < 128 (no carry or
// borrow between bytes in either).  flags[0] counts clamped ratios;
// flags[1] is set when some |X| would reach 2^27 (exponent too small).
__global__ __launch_bounds__(256) void slice_kernel(const float* __restrict__ I, int64_t M, int64_t Mpad, int N,
                                                    int64_t ld, const double* __restrict__ rinv64, double floor,
                                                    const int* __restrict__ colexp, int npad, u32x4v* __restrict__ S,
                                                    double* __restrict__ colsum_part,
                                                    unsigned long long* __restrict__ flags) {
    __shared__ double tab[128];
    if (threadIdx.x < 64) {
        const double c = 0.5 + (threadIdx.x + 0.5) / 128.0;
        tab[2 * threadIdx.x] = 1.0 / c;
        tab[2 * threadIdx.x + 1] = log(c);
    }
    __syncthreads();
    const int j = blockIdx.y * 256 + threadIdx.x;
    if (j >= npad) return;
    const bool live = j < N;
    const double r = live ? rinv64[j] : 0.0;
    // X = rint(x 2^27) with x = l 2^-e and l = ln(q) / 2
    const double scale = live ? ldexp(0.5, 27 - colexp[j]) : 0.0;
    const int64_t r0 = (int64_t)blockIdx.x * ST_ROWS;
    const int64_t g0 = r0 / 16;
    const int64_t g1 = ((r0 + ST_ROWS < Mpad) ? r0 + ST_ROWS : Mpad) / 16;
    constexpr int B = 64 * (1 + (1 << 7) + (1 << 14) + (1 << 21));
    double cs = 0.0;
    unsigned int bad = 0;
    bool ovf = false;
    // loads from an in-range column (columns past N are computed and dropped)
    const float* colp = I + (live ? j : N - 1);
    // 16 rows of the column from row mb; rows past M read row M - 1 (and are
    // masked below).  The pointer steps one row at a time in registers of
    // its own (the empty asm keeps the compiler from holding 16 row offsets
    // in scalar registers).
    auto load = [&](int64_t mb, float (&x)[16]) {
        const float* p = colp + (mb < M ? mb : M - 1) * ld;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            x[q] = *p;
            if (mb + q + 1 < M) p += ld;
            asm volatile("" : "+v"(p));
        }
    };
    auto slice_group = [&](int64_t g, const float (&xs)[16]) {
        unsigned int w1[4] = {0u, 0u, 0u, 0u}, w2[4] = {0u, 0u, 0u, 0u};
        unsigned int w3[4] = {0u, 0u, 0u, 0u}, w4[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            // every element is computed; rows past M and columns past N count
            // for nothing and slice to zero
            const bool valid = live && (16 * g + q < M);
            const double x = valid ? (double)xs[q] : 0.0;
            cs += x;
            double ratio = x * r;
            const bool b = !(ratio > floor) || !(ratio < INFINITY);
            bad += (b && valid) ? 1u : 0u;
            ratio = b ? floor : ratio;
            const double v = log_cells(ratio, tab) * scale;
            ovf = ovf || (valid && !(fabs(v) < 0x1p27 - 0.5));
            const int X = valid ? (int)rint(v) : 0;
            const unsigned int Y = (unsigned int)(X + B);
            const int sh = 8 * (q & 3), u = q >> 2;
            w1[u] |= (Y >> 21) << sh;
            w2[u] |= __builtin_amdgcn_ubfe(Y, 14, 7) << sh;
            w3[u] |= __builtin_amdgcn_ubfe(Y, 7, 7) << sh;
            w4[u] |= (Y & 127u) << sh;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            w1[u] = (w1[u] + 0x40404040u) ^ 0x80808080u;
            w2[u] = ((w2[u] | 0x80808080u) - 0x40404040u) ^ 0x80808080u;
            w3[u] = ((w3[u] | 0x80808080u) - 0x40404040u) ^ 0x80808080u;
            w4[u] = ((w4[u] | 0x80808080u) - 0x40404040u) ^ 0x80808080u;
        }
        u32x4v* out = S + g * 4 * (int64_t)npad + j;
        out[0] = u32x4v{w1[0], w1[1], w1[2], w1[3]};
        out[npad] = u32x4v{w2[0], w2[1], w2[2], w2[3]};
        out[2 * npad] = u32x4v{w3[0], w3[1], w3[2], w3[3]};
        out[3 * npad] = u32x4v{w4[0], w4[1], w4[2], w4[3]};
    };
    float xs[16], xn[16];
    if (g0 < g1) load(16 * g0, xs);
    for (int64_t g = g0; g < g1; ++g) {
        if (g + 1 < g1) load(16 * (g + 1), xn);
        slice_group(g, xs);
#pragma unroll
        for (int q = 0; q < 16; ++q) xs[q] = xn[q];
    }
    colsum_part[(size_t)blockIdx.x * npad + j] = live ? cs : 0.0;
    for (int off = 32; off >= 1; off >>= 1) bad += __shfl_xor(bad, off);
    if ((threadIdx.x & 63) == 0 && bad) atomicAdd(&flags[0], (unsigned long long)bad);
    if (ovf) atomicOr(reinterpret_cast<unsigned int*>(&flags[1]), 1u);
}

// ---------------------------------------------------------------------------
// gram: 128 x 128 tiles, 64-row K steps staged in LDS as sX[slice][row
// group][column] (16-byte units), double-buffered
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32x16 mfma_i8(const u32x4v& a, const u32x4v& b, int32x16 c) {
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i8x16, a), __builtin_bit_cast(i8x16, b), c, 0,
                                                 0, 0);
}

// s_waitcnt immediate (gfx9 encoding) that waits until at most n vector
// memory operations of the wave are outstanding, ignoring the other counters.
template <int n>
__device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((n & 15) | (7 << 4) | (15 << 8) | ((n >> 4) << 14));
}

// Workgroup barrier without a memory fence: __syncthreads() also waits for
// every outstanding vector memory operation, which would drain the direct
// loads in flight for later half steps.  Ordering is explicit instead: the
// loads a half step reads are waited for (wait_vm) before the barrier, its
// LDS reads are consumed by the matrix cores before the barrier, and the
// clobber keeps the compiler from moving memory accesses across it.
__device__ __forceinline__ void barrier_only() { asm volatile("s_barrier" ::: "memory"); }

constexpr int HROWS = 32;  // rows per half step (2 row groups)
constexpr int RING = 4;    // half steps held in LDS

__global__ __launch_bounds__(I8_THREADS) void gram_i8_kernel(const u32x4v* __restrict__ S, int npad, int64_t M,
                                                             int T, int64_t rpc, const int* __restrict__ tiles,
                                                             const int* __restrict__ colexp,
                                                             double* __restrict__ partial) {
    // ring of half steps: [slot][operand][slice 4][row group 2][column 128]
    // (16-byte units, 32 KB per slot)
    __shared__ u32x4v sm[RING][2][4 * 2 * GT];

    // blockIdx -> (chunk, tile): consecutive blocks go to different XCDs, so
    // the 8 XCDs each take every 8th chunk.  Past 32 tiles (the CUs of an
    // XCD) an XCD first runs tiles 0..31 of each of its chunks, one chunk per
    // round of 32 blocks that stream the chunk's rows together, and then the
    // remaining tiles of all its chunks.
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int rr = b >> 3;
    const int nc8 = (int)(gridDim.x / (8 * T));  // chunks per XCD
    int tile, jc;
    if (T > 32 && rr < nc8 * 32) {
        jc = rr / 32;
        tile = rr % 32;
    } else if (T > 32) {
        const int u = rr - nc8 * 32;
        jc = u / (T - 32);
        tile = 32 + u % (T - 32);
    } else {
        jc = rr / T;
        tile = rr % T;
    }
    const int chunk = jc * 8 + xcd;
    const int bi = tiles[2 * tile], bj = tiles[2 * tile + 1];
    const bool diag = (bi == bj);
    const int64_t m0 = (int64_t)chunk * rpc;
    const int64_t m1 = (m0 + rpc < M) ? m0 + rpc : M;
    // half steps (zero rows past M in the slices, which cover whole 64-row steps)
    const int64_t nh = (m1 > m0) ? 2 * ((m1 - m0 + KROWS - 1) / KROWS) : 0;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 2, wc = wave & 3;  // a columns 64 wr.., b columns 32 wc..
    // a wave of a diagonal tile below the diagonal computes nothing needed
    const bool idle = diag && (64 * wr >= 32 * wc + 32);

    // Strips go from HBM to LDS by direct loads (global_load_lds, 16 bytes
    // per lane, lane i to the instruction's LDS base + 16 i): instruction p
    // (< 2) of wave w moves units u = 64 (2 w + p) + lane of a half-step
    // strip, i.e. row group u / 512, slice (u / 128) % 4, columns
    // (u % 128) .. + 63, contiguous in both layouts.
    auto fetch = [&](int64_t h, int blk, int op) {
        const int64_t g0 = (m0 + h * HROWS) / 16;
        const int slot = (int)(h & (RING - 1));
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int u0 = 64 * (2 * wave + p);
            const int rg = u0 >> 9, s = (u0 >> 7) & 3, col0 = u0 & 127;
            const u32x4v* src = S + ((size_t)(g0 + rg) * 4 + s) * npad + blk * GT + col0 + lane;
            __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(src),
                                             (__attribute__((address_space(3))) void*)(
                                                 &sm[slot][op][(s * 2 + rg) * GT + col0]),
                                             16, 0, 0);
        }
    };
    auto fetch_step = [&](int64_t h) {
        fetch(h, bi, 0);
        if (!diag) fetch(h, bj, 1);
    };

    // acc[level t - 2][ti]: (32 x 32) blocks at a columns 64 wr + 32 ti
    int32x16 acc[5][2];
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[t][i][v] = 0;

    for (int64_t h = 0; h < 3 && h < nh; ++h) fetch_step(h);
    if (diag) {  // two loads per half step
        if (nh > 2) wait_vm<4>(); else if (nh > 1) wait_vm<2>(); else wait_vm<0>();
    } else {
        if (nh > 2) wait_vm<8>(); else if (nh > 1) wait_vm<4>(); else wait_vm<0>();
    }
    barrier_only();
    for (int64_t h = 0; h < nh; ++h) {
        const int slot = (int)(h & (RING - 1));
        const u32x4v* A = sm[slot][0];
        const u32x4v* B = diag ? sm[slot][0] : sm[slot][1];
        // half step h + 3 goes to the slot of h - 1, which every wave
        // finished reading before the last barrier
        if (h + 3 < nh) fetch_step(h + 3);
        if (!idle) {
            const int rg = lane >> 5;
            u32x4v bv[4], av[2][4];
#pragma unroll
            for (int s = 0; s < 4; ++s) bv[s] = B[(s * 2 + rg) * GT + wc * 32 + (lane & 31)];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int s = 0; s < 4; ++s) av[i][s] = A[(s * 2 + rg) * GT + wr * 64 + i * 32 + (lane & 31)];
            // level t = s_a + s_b (slices counted from 1), t <= 6: the r-th
            // product of every level of both blocks in turn, so that the
            // products added to one accumulator issue 6 to 10 apart; the
            // scheduling barriers keep the operand reads ahead of the
            // products and the rounds in this order
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int t = 0; t < 5; ++t) {
                        // with slices counted from 0, level t + 2 pairs
                        // (a, t - a): a = 0..t for t <= 3, a = 1..3 for t = 4
                        const int nprod = (t <= 3) ? t + 1 : 3;
                        if (r < nprod) {
                            const int sa = (t <= 3) ? r : r + 1;
                            acc[t][i] = mfma_i8(av[i][sa], bv[t - sa], acc[t][i]);
                        }
                    }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        // half step h + 1 must have landed: the loads issued after it (of
        // h + 2 and h + 3, where they exist) may still be in flight
        if (diag) {
            if (h + 3 < nh) wait_vm<4>(); else if (h + 2 < nh) wait_vm<2>(); else wait_vm<0>();
        } else {
            if (h + 3 < nh) wait_vm<8>(); else if (h + 2 < nh) wait_vm<4>(); else wait_vm<0>();
        }
        barrier_only();
    }
    if (idle) return;

    // Flush: |C_t| <= (t - 1) 2^12 rpc <= 2^30, so sum_t 2^(-7 (t-2)) C_t
    // spans bits 2^30 .. 2^-28: the two halves below are exact in FP64 and
    // their sum rounds once.
    double* P = partial + ((size_t)chunk * T + tile) * (size_t)(GT * GT);
    const int c = wc * 32 + (lane & 31);
    const int ec = colexp[bj * GT + c] - 12;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int r = wr * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
            const double hi = (double)acc[0][i][v] + 0x1p-7 * (double)acc[1][i][v];
            const double lo = 0x1p-14 * (double)acc[2][i][v] + 0x1p-21 * (double)acc[3][i][v] +
                              0x1p-28 * (double)acc[4][i][v];
            P[r * GT + c] = ldexp(hi + lo, colexp[bi * GT + r] + ec);
        }
}

}  // namespace

int64_t stats_blocks(int64_t M) { return (M + ST_ROWS - 1) / ST_ROWS; }

size_t stats_colmax_floats(int64_t M, int npad) { return (size_t)(stats_blocks(M) + kMaxGroups) * npad; }

size_t split_bytes(int64_t M, int npad) { return (size_t)((M + KROWS - 1) / KROWS) * KROWS * (size_t)npad * 4; }

GramPlan split_gram_plan(int64_t M, int N) {
    // int32 levels stay exact while a chunk has at most 2^31 / (4 * 64 * 64)
    // = 131,072 rows: chunks of at most 65,536
    GramPlan p = gram_plan(M, N, 64, KROWS);
    if (p.rows_per_chunk > 65536) p = gram_plan(M, N, (int)((M + 65535) / 65536), KROWS);
    return p;
}

namespace {

// Column maxima partials (nb rows of npad) -> group maxima -> exponents.
hipError_t colexp_from_parts(float* colmax_part, int64_t nb, int npad, int N, int margin, int* colexp, hipStream_t s) {
    // group maxima go to the rows past the last partial, so no block
    // overwrites partials that another block still reads
    float* gmax = colmax_part + (size_t)nb * npad;
    const int groups = (int)std::min<int64_t>(kMaxGroups, (nb + 3) / 4);
    hipLaunchKernelGGL(colmax_group_kernel, dim3((unsigned)((npad + 63) / 64), (unsigned)groups), dim3(256), 0, s,
                       colmax_part, nb, npad, gmax);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colexp_kernel, dim3((unsigned)((npad + 255) / 256)), dim3(256), 0, s, gmax, groups, npad, N,
                       margin, colexp);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_split_stats(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor, int npad,
                              double* colsum_part, float* colmax_part, unsigned long long* clamps, int* colexp,
                              hipStream_t s) {
    if (npad % 4 != 0 || npad < N) return hipErrorInvalidValue;
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    const int64_t nb = stats_blocks(M);
    if (vec)
        hipLaunchKernelGGL(stats_kernel<true>, dim3((unsigned)nb), dim3(256), 0, s, I, M, N, ld, rinv, floor, npad,
                           colsum_part, colmax_part, clamps);
    else
        hipLaunchKernelGGL(stats_kernel<false>, dim3((unsigned)nb), dim3(256), 0, s, I, M, N, ld, rinv, floor, npad,
                           colsum_part, colmax_part, clamps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return colexp_from_parts(colmax_part, nb, npad, N, 0, colexp, s);
}

int64_t sample_blocks(int64_t M, int stride) { return ((M + stride - 1) / stride + SAMPLE_ROWS - 1) / SAMPLE_ROWS; }

hipError_t launch_split_sample(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor, int npad,
                               int stride, float* colmax_part, int* colexp, hipStream_t s) {
    if (npad % 4 != 0 || npad < N || stride < 1 || M < 1) return hipErrorInvalidValue;
    const int64_t nb = sample_blocks(M, stride);
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    if (vec)
        hipLaunchKernelGGL(sample_max_kernel<true>, dim3((unsigned)nb), dim3(256), 0, s, I, M, N, ld, rinv, floor,
                           npad, stride, colmax_part);
    else
        hipLaunchKernelGGL(sample_max_kernel<false>, dim3((unsigned)nb), dim3(256), 0, s, I, M, N, ld, rinv, floor,
                           npad, stride, colmax_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return colexp_from_parts(colmax_part, nb, npad, N, 1, colexp, s);
}

hipError_t launch_split_slices(const float* I, int64_t M, int N, int64_t ld, const double* rinv64, double floor,
                               const int* colexp, int npad, void* S, double* colsum_part,
                               unsigned long long* flags, hipStream_t s) {
    if (npad % 128 != 0 || npad < N || M < 1) return hipErrorInvalidValue;
    const int64_t Mpad = (M + KROWS - 1) / KROWS * KROWS;
    dim3 grid((unsigned)stats_blocks(M), (unsigned)((npad + 255) / 256));
    hipLaunchKernelGGL(slice_kernel, grid, dim3(256), 0, s, I, M, Mpad, N, ld, rinv64, floor, colexp, npad,
                       static_cast<u32x4v*>(S), colsum_part, flags);
    return hipGetLastError();
}

hipError_t launch_gram_split(const void* S, int npad, int64_t M, const GramPlan& plan, const int* d_tiles,
                             const int* colexp, double* partial, hipStream_t s) {
    if (plan.tiles < 1 || plan.chunks < 1 || M < 1 || plan.rows_per_chunk % KROWS != 0 ||
        plan.rows_per_chunk > 65536 || plan.nb * GT > npad)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)(plan.tiles * plan.chunks)), block(I8_THREADS);
    hipLaunchKernelGGL(gram_i8_kernel, grid, block, 0, s, static_cast<const u32x4v*>(S), npad, M, plan.tiles,
                       plan.rows_per_chunk, d_tiles, colexp, partial);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace fkk
