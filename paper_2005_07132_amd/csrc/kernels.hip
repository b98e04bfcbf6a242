// gfx950 kernels of the fKK-EC hot path: log ratio + Gram (Eq. 2, 6),
// projection with per-column arg-extrema (Eq. 13-15, 25), and the
// reconstruction GEMM fused with the exp / sin epilogue (Eq. 23).
//
// Matrix products use v_mfma_f32_16x16x4_f32 (FP32 in, FP32 accumulate).
// For a 16x16x4 block, lane l holds A[l%16][l/16] and B[l/16][l%16] and
// receives D[4*(l/16)+v][l%16] in accumulator element v.  Which physical
// row or column plays "k" inside a block is free as long as A and B agree,
// which lets every lane read four consecutive k values with one 128-bit
// LDS load.
#include "kernels.h"
#include "device_common.h"

#include <algorithm>
#include <climits>
#include <cmath>

namespace fkk {
namespace dev {

// ===========================================================================
// Gram of the log ratio.
// ===========================================================================
constexpr int GT = kGramTile;  // output tile
constexpr int GKC = 32;        // rows per LDS stage
constexpr int GLD = GT + 16;   // LDS row stride: rows 0/1 of a wave read hit disjoint banks

GramPlan gram_plan(int64_t M, int N, int target_chunks, int row_quantum) {
    GramPlan p;
    p.nb = (N + GT - 1) / GT;
    p.tiles = p.nb * (p.nb + 1) / 2;
    int64_t want = target_chunks > 0 ? target_chunks : 64;
    int64_t rpc = (M + want - 1) / want;
    rpc = ((rpc + row_quantum - 1) / row_quantum) * row_quantum;
    if (rpc < row_quantum) rpc = row_quantum;
    int64_t chunks = (M + rpc - 1) / rpc;
    if (chunks < 1) chunks = 1;
    chunks = ((chunks + 7) / 8) * 8;
    p.chunks = (int)chunks;
    p.rows_per_chunk = rpc;
    return p;
}

void gram_tile_list(int nb, int* pairs) {
    int t = 0;
    for (int bi = 0; bi < nb; ++bi)
        for (int bj = bi; bj < nb; ++bj) {
            pairs[2 * t] = bi;
            pairs[2 * t + 1] = bj;
            ++t;
        }
}

// ---------------------------------------------------------------------------
// Log-ratio pass: l = 1/2 ln(I r) written once as FP32 (row stride ldl, zero
// beyond column N), with FP64 column sums of I and the clamp count.
// ---------------------------------------------------------------------------
constexpr int LR_ROWS = 256;  // rows per block

template <bool VEC>
__global__ __launch_bounds__(256) void logratio_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                       const float* __restrict__ rinv, float floor,
                                                       float* __restrict__ L, int64_t ldl, int npad,
                                                       double* __restrict__ colsum_part,
                                                       unsigned long long* __restrict__ clamps) {
    const int64_t r0 = (int64_t)blockIdx.x * LR_ROWS;
    const int64_t r1 = (r0 + LR_ROWS < M) ? r0 + LR_ROWS : M;
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
        for (int64_t row0 = r0; row0 < r1; row0 += 4) {
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                x[u] = (row0 + u < r1) ? load4_guarded(I + (row0 + u) * ld, c, N, VEC) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (row0 + u >= r1) break;
                float l[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bool bad;
                    const float xv = f4get(x[u], q);
                    l[q] = log_ratio(xv, r[q], rl[q], floor, bad);
                    if (c + q < N) {
                        cnt += bad ? 1u : 0u;
                        cs[q] += (double)xv;
                    } else {
                        l[q] = 0.f;
                    }
                }
                *reinterpret_cast<float4*>(L + (row0 + u) * ldl + c) = make_float4(l[0], l[1], l[2], l[3]);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) colsum_part[(size_t)blockIdx.x * npad + c + q] = cs[q];
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(clamps, (unsigned long long)cnt);
}

// ---------------------------------------------------------------------------
// Gram of the log ratio from l (no bounds checks on columns: l is zero past
// N up to the padded width).  FP32: each 32-row LDS stage is accumulated by
// the matrix cores in FP32 and then added into FP64 registers, so the error
// does not grow with the rows of a chunk.
// ---------------------------------------------------------------------------
constexpr int kGramThreads = 512;  // 8 waves, each 32 x 64 of the 128 x 128 tile

typedef double doublex4 __attribute__((ext_vector_type(4)));

// F64: the FP32 l is promoted to FP64 (products exact) and accumulated by
// v_mfma_f64_16x16x4f64 (operands laid out as for the FP32 instruction; the
// result rows are interleaved differently, see the store).  Needed
// where the Gram must resolve eigenvalue gaps below the rounding of the
// FP32 matrix cores, which do not round each sum correctly.
// Tile (bi, bj) of the list is the product of columns 128 bi.. of L and
// columns 128 bj.. of R (R = L for the Gram itself).
template <bool F64>
__global__ __launch_bounds__(kGramThreads) void gram_kernel(const float* __restrict__ L, int64_t ldl,
                                                            const float* __restrict__ R, int64_t ldr, int64_t M,
                                                            int T, int64_t rpc, const int* __restrict__ tiles,
                                                            double* __restrict__ partial) {
    __shared__ __attribute__((aligned(16))) float sA[2][GKC][GLD];
    __shared__ __attribute__((aligned(16))) float sB[2][GKC][GLD];

    // blockIdx -> (chunk, tile): consecutive blocks go to different XCDs, so
    // the 8 XCDs each take every 8th chunk and run all tiles of a chunk.
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int rr = b >> 3;
    const int tile = rr % T;
    const int chunk = (rr / T) * 8 + xcd;
    const int bi = tiles[2 * tile], bj = tiles[2 * tile + 1];
    const bool diag = (bi == bj) && (L == R);
    const int64_t m0 = (int64_t)chunk * rpc;
    const int64_t m1 = (m0 + rpc < M) ? m0 + rpc : M;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;  // rows 32 wr.., columns 64 wc..
    const int lr = tid >> 5;                  // 0..15
    const int lc = (tid & 31) * 4;
    const float* La = L + bi * GT + lc;
    const float* Lb = R + bj * GT + lc;

    doublex4 acc64[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc64[i][j] = doublex4{0.0, 0.0, 0.0, 0.0};

    float4 xa[2], xb[2];
    float keep[2];
    // Rows past the chunk are loaded from the chunk's last row (always valid)
    // and zeroed when written to LDS, so the loads are unconditional and the
    // loaded registers are first used after the MFMA block.
    auto load = [&](int64_t base) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const int64_t row = base + lr + 16 * p;
            const int64_t rc = row < m1 ? row : m1 - 1;
            keep[p] = row < m1 ? 1.f : 0.f;
            xa[p] = *reinterpret_cast<const float4*>(La + rc * ldl);
            xb[p] = *reinterpret_cast<const float4*>(Lb + rc * ldr);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float k = keep[p];
            *reinterpret_cast<float4*>(&sA[buf][lr + 16 * p][lc]) =
                make_float4(xa[p].x * k, xa[p].y * k, xa[p].z * k, xa[p].w * k);
            if (!diag)
                *reinterpret_cast<float4*>(&sB[buf][lr + 16 * p][lc]) =
                    make_float4(xb[p].x * k, xb[p].y * k, xb[p].z * k, xb[p].w * k);
        }
    };

    const int64_t nst = (m1 > m0) ? (m1 - m0 + GKC - 1) / GKC : 0;
    if (nst > 0) {
        load(m0);
        store(0);
    }
    __syncthreads();
    for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nst) load(m0 + (s + 1) * GKC);
        const float(*A)[GLD] = sA[buf];
        const float(*B)[GLD] = diag ? sA[buf] : sB[buf];
        if constexpr (F64) {
#pragma unroll
            for (int ks = 0; ks < GKC / 4; ++ks) {
                const int row = ks * 4 + (lane >> 4);
                double av[2], bv[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) av[i] = (double)A[row][wr * 32 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = (double)B[row][wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc64[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc64[i][j], 0, 0, 0);
            }
            if (s + 1 < nst) store(buf ^ 1);
        } else {
            floatx4 acc[2][4];
#pragma unroll
            for (int ks = 0; ks < GKC / 4; ++ks) {
                const int row = ks * 4 + (lane >> 4);
                float av[2], bv[4];
#pragma unroll
                for (int i = 0; i < 2; ++i) av[i] = A[row][wr * 32 + i * 16 + (lane & 15)];
#pragma unroll
                for (int j = 0; j < 4; ++j) bv[j] = B[row][wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        acc[i][j] = mfma4(av[i], bv[j], ks == 0 ? floatx4{0.f, 0.f, 0.f, 0.f} : acc[i][j]);
            }
            if (s + 1 < nst) store(buf ^ 1);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
        }
        __syncthreads();
    }

    double* P = partial + ((size_t)chunk * T + tile) * (size_t)(GT * GT);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // element v of lane l: row 4 (l/16) + v (FP32 instruction),
                // row l/16 + 4 v (FP64 instruction); column l % 16 in both
                const int r = wr * 32 + i * 16 + (F64 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v);
                const int c = wc * 64 + j * 16 + (lane & 15);
                P[r * GT + c] = acc64[i][j][v];
            }
}

__global__ void gram_reduce_kernel(const double* __restrict__ partial, int T, int C,
                                   const int* __restrict__ tiles, int N, double* __restrict__ G) {
    const int tile = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= GT * GT) return;
    const int bi = tiles[2 * tile], bj = tiles[2 * tile + 1];
    double s = 0.0;
    for (int ch = 0; ch < C; ++ch) s += partial[((size_t)ch * T + tile) * (size_t)(GT * GT) + e];
    const int r = e / GT, c = e % GT;
    const int gi = bi * GT + r, gj = bj * GT + c;
    if (gi >= N || gj >= N) return;
    if (bi != bj || r <= c) {
        G[(size_t)gi * N + gj] = s;
        G[(size_t)gj * N + gi] = s;
    }
}

// Column sums over the partials in a fixed order: stage 1 sums groups of
// partials (grid.y groups), stage 2 sums the groups.
__global__ void colsum_stage1_kernel(const double* __restrict__ part, int64_t C, int stride, int N,
                                     double* __restrict__ mid) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int64_t g = blockIdx.y, G = gridDim.y;
    const int64_t c0 = C * g / G, c1 = C * (g + 1) / G;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t c = c0;
    for (; c + 3 < c1; c += 4) {
        s0 += part[(size_t)c * stride + j];
        s1 += part[(size_t)(c + 1) * stride + j];
        s2 += part[(size_t)(c + 2) * stride + j];
        s3 += part[(size_t)(c + 3) * stride + j];
    }
    for (; c < c1; ++c) s0 += part[(size_t)c * stride + j];
    mid[(size_t)g * N + j] = (s0 + s1) + (s2 + s3);
}

__global__ void colsum_stage2_kernel(const double* __restrict__ mid, int G, int N, double* __restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    double s = 0.0;
    for (int g = 0; g < G; ++g) s += mid[(size_t)g * N + j];
    out[j] = s;
}

int64_t logratio_blocks(int64_t M) { return (M + LR_ROWS - 1) / LR_ROWS; }

hipError_t launch_logratio(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor, float* L,
                           int64_t ldl, int npad, double* colsum_part, unsigned long long* clamps, hipStream_t s) {
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    dim3 grid((unsigned)logratio_blocks(M)), block(256);
    if (vec)
        hipLaunchKernelGGL(logratio_kernel<true>, grid, block, 0, s, I, M, N, ld, rinv, floor, L, ldl, npad,
                           colsum_part, clamps);
    else
        hipLaunchKernelGGL(logratio_kernel<false>, grid, block, 0, s, I, M, N, ld, rinv, floor, L, ldl, npad,
                           colsum_part, clamps);
    return hipGetLastError();
}

hipError_t launch_gram(const float* L, int64_t ldl, int64_t M, const GramPlan& plan, const int* d_tiles,
                       double* partial, hipStream_t s, bool fp64) {
    return launch_gram_pair(L, ldl, L, ldl, M, plan, d_tiles, partial, s, fp64);
}

hipError_t launch_gram_pair(const float* L, int64_t ldl, const float* R, int64_t ldr, int64_t M,
                            const GramPlan& plan, const int* d_tiles, double* partial, hipStream_t s, bool fp64) {
    if (plan.tiles < 1 || plan.chunks < 1 || M < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)(plan.tiles * plan.chunks)), block(kGramThreads);
    if (fp64)
        hipLaunchKernelGGL(gram_kernel<true>, grid, block, 0, s, L, ldl, R, ldr, M, plan.tiles, plan.rows_per_chunk,
                           d_tiles, partial);
    else
        hipLaunchKernelGGL(gram_kernel<false>, grid, block, 0, s, L, ldl, R, ldr, M, plan.tiles,
                           plan.rows_per_chunk, d_tiles, partial);
    return hipGetLastError();
}

// Sum of the chunk partials of each listed tile, in chunk order, into the
// rows x cols block of out (tile (bi, bj) at rows 128 bi.., columns 128 bj..).
__global__ void gram_reduce_rect_kernel(const double* __restrict__ partial, int T, int C,
                                        const int* __restrict__ tiles, int rows, int cols, double* __restrict__ out,
                                        int64_t ld_out) {
    const int tile = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= GT * GT) return;
    const int r = tiles[2 * tile] * GT + e / GT, c = tiles[2 * tile + 1] * GT + e % GT;
    if (r >= rows || c >= cols) return;
    double acc = 0.0;
    for (int ch = 0; ch < C; ++ch) acc += partial[((size_t)ch * T + tile) * (size_t)(GT * GT) + e];
    out[(int64_t)r * ld_out + c] = acc;
}

hipError_t launch_gram_reduce_rect(const double* partial, const GramPlan& plan, const int* d_tiles, int rows,
                                   int cols, double* out, int64_t ld_out, hipStream_t s) {
    if (plan.tiles < 1 || ld_out < cols) return hipErrorInvalidValue;
    dim3 grid(GT * GT / 256, plan.tiles);
    hipLaunchKernelGGL(gram_reduce_rect_kernel, grid, dim3(256), 0, s, partial, plan.tiles, plan.chunks, d_tiles,
                       rows, cols, out, ld_out);
    return hipGetLastError();
}

hipError_t launch_gram_reduce(const double* partial, const GramPlan& plan, const int* d_tiles, int N, double* G,
                              hipStream_t s) {
    dim3 grid(GT * GT / 256, plan.tiles);
    hipLaunchKernelGGL(gram_reduce_kernel, grid, dim3(256), 0, s, partial, plan.tiles, plan.chunks, d_tiles, N, G);
    return hipGetLastError();
}

constexpr int kColsumGroups = 64;
size_t colsum_scratch_doubles(int N) { return (size_t)kColsumGroups * N; }

hipError_t launch_colsum_reduce(const double* part, int64_t nparts, int stride, int N, double* mid, double* out,
                                hipStream_t s) {
    const int G = (int)std::min<int64_t>(kColsumGroups, nparts);
    hipLaunchKernelGGL(colsum_stage1_kernel, dim3((N + 255) / 256, G), dim3(256), 0, s, part, nparts, stride, N, mid);
    hipLaunchKernelGGL(colsum_stage2_kernel, dim3((N + 255) / 256), dim3(256), 0, s, mid, G, N, out);
    return hipGetLastError();
}

// ===========================================================================
// Projection Z = l W with per-column arg-extrema.
// ===========================================================================
constexpr int PR = kProjRows;  // rows per block (4 waves x 32)
constexpr int PNC = 64;        // wavenumbers per LDS stage
constexpr int PLD = PNC + 4;

// Stage one 128 x 64 tile of l = 1/2 ln(I r) into LDS (zeros outside).
// NORMS: also adds (l f)^2 of the staged values to asq[p] (row lrow + 16 p).
template <bool VEC, bool NORMS = false>
__device__ __forceinline__ void stage_logratio(float (*sL)[PLD], const float* __restrict__ I, int64_t r0,
                                               int64_t M, int N, int64_t ld, int j0,
                                               const float* __restrict__ rinv, float floor,
                                               const float* __restrict__ f = nullptr, float* asq = nullptr) {
    const int tid = threadIdx.x;
    const int lrow = tid >> 4;
    const int lcol = (tid & 15) * 4;
    const int col = j0 + lcol;
    float r[4], rl[4], fq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        r[q] = (col + q < N) ? rinv[col + q] : 0.f;
        rl[q] = (col + q < N) ? rinv[N + col + q] : 0.f;
        if (NORMS) fq[q] = (col + q < N) ? f[col + q] : 0.f;
    }
    float4 x[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int64_t row = r0 + lrow + 16 * p;
        x[p] = (row < M) ? load4_guarded(I + row * ld, col, N, VEC) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int64_t row = r0 + lrow + 16 * p;
        float l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bool bad;
            l[q] = (row < M && col + q < N) ? log_ratio(f4get(x[p], q), r[q], rl[q], floor, bad) : 0.f;
            if (NORMS) {
                const float a = l[q] * fq[q];
                asq[p] = fmaf(a, a, asq[p]);
            }
        }
        *reinterpret_cast<float4*>(&sL[lrow + 16 * p][lcol]) = make_float4(l[0], l[1], l[2], l[3]);
    }
}

// Stage one 128 x 64 tile of a precomputed l (row stride ldl, zero past N).
__device__ __forceinline__ void stage_loaded(float (*sL)[PLD], const float* __restrict__ L, int64_t r0, int64_t M,
                                             int64_t ldl, int j0) {
    const int tid = threadIdx.x;
    const int lrow = tid >> 4;
    const int lcol = (tid & 15) * 4;
    float4 x[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const int64_t row = r0 + lrow + 16 * p;
        const int64_t rc = row < M ? row : M - 1;
        x[p] = *reinterpret_cast<const float4*>(L + rc * ldl + j0 + lcol);
    }
#pragma unroll
    for (int p = 0; p < 8; ++p) {
        const float k = (r0 + lrow + 16 * p < M) ? 1.f : 0.f;
        *reinterpret_cast<float4*>(&sL[lrow + 16 * p][lcol]) = make_float4(x[p].x * k, x[p].y * k, x[p].z * k, x[p].w * k);
    }
}

template <int KB>
__device__ __forceinline__ void stage_weights(float (*sW)[PLD], const float* __restrict__ Wt, int ldw, int j0) {
    const int tid = threadIdx.x;
    const int lcol = (tid & 15) * 4;
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        const int c = (tid >> 4) + 16 * p;
        *reinterpret_cast<float4*>(&sW[c][lcol]) =
            *reinterpret_cast<const float4*>(Wt + (size_t)c * ldw + j0 + lcol);
    }
}

// acc[rb][cb] += l(rows of this wave) * W over one 64-wide stage
template <int KB>
__device__ __forceinline__ void project_stage(floatx4 (&acc)[2][KB], const float (*sL)[PLD],
                                              const float (*sW)[PLD], int wave, int lane) {
#pragma unroll
    for (int gq = 0; gq < PNC / 16; ++gq) {
        float4 a[2], w[KB];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
            a[rb] = *reinterpret_cast<const float4*>(&sL[wave * 32 + rb * 16 + (lane & 15)][gq * 16 + 4 * (lane >> 4)]);
#pragma unroll
        for (int cb = 0; cb < KB; ++cb)
            w[cb] = *reinterpret_cast<const float4*>(&sW[cb * 16 + (lane & 15)][gq * 16 + 4 * (lane >> 4)]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                for (int cb = 0; cb < KB; ++cb) acc[rb][cb] = mfma4(f4get(a[rb], q), f4get(w[cb], q), acc[rb][cb]);
    }
}

template <int KB, bool VEC, bool LOGGED>
__global__ __launch_bounds__(256) void project_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                      const float* __restrict__ rinv, float floor,
                                                      const float* __restrict__ Wt, int ldw, int k_store,
                                                      float* __restrict__ Z, int64_t ld_z, float* pmaxv,
                                                      float* pminv, long long* pmaxi, long long* pmini,
                                                      int k_arg) {
    constexpr int KP = KB * 16;
    __shared__ __attribute__((aligned(16))) float sL[PR][PLD];
    __shared__ __attribute__((aligned(16))) float sW[KP][PLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PR;

    floatx4 acc[2][KB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < KB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    for (int j0 = 0; j0 < N; j0 += PNC) {
        if (LOGGED) stage_loaded(sL, I, r0, M, ld, j0);
        else stage_logratio<VEC>(sL, I, r0, M, N, ld, j0, rinv, floor);
        stage_weights<KB>(sW, Wt, ldw, j0);
        __syncthreads();
        project_stage<KB>(acc, sL, sW, wave, lane);
        __syncthreads();
    }

    project_finish<KB>(acc, r0, M, Z, ld_z, k_store, pmaxv, pminv, pmaxi, pmini, k_arg);
}

__global__ void argext_reduce_kernel(ArgPart part, int64_t nblocks, int kp, long long* qmax, long long* qmin) {
    const int c = blockIdx.x;
    float mx = -INFINITY, mn = INFINITY;
    long long ix = LLONG_MAX, in = LLONG_MAX;
    for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const size_t o = (size_t)b * kp + c;
        const long long bi = part.maxi[o], ni = part.mini[o];
        if (bi >= 0 && (part.maxv[o] > mx || (part.maxv[o] == mx && bi < ix))) { mx = part.maxv[o]; ix = bi; }
        if (ni >= 0 && (part.minv[o] < mn || (part.minv[o] == mn && ni < in))) { mn = part.minv[o]; in = ni; }
    }
    __shared__ float smx[256], smn[256];
    __shared__ long long sx[256], sn[256];
    smx[threadIdx.x] = mx; smn[threadIdx.x] = mn; sx[threadIdx.x] = ix; sn[threadIdx.x] = in;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const int o = threadIdx.x + st;
            if (smx[o] > smx[threadIdx.x] || (smx[o] == smx[threadIdx.x] && sx[o] < sx[threadIdx.x])) {
                smx[threadIdx.x] = smx[o]; sx[threadIdx.x] = sx[o];
            }
            if (smn[o] < smn[threadIdx.x] || (smn[o] == smn[threadIdx.x] && sn[o] < sn[threadIdx.x])) {
                smn[threadIdx.x] = smn[o]; sn[threadIdx.x] = sn[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        qmax[c] = (sx[0] == LLONG_MAX) ? -1 : sx[0];
        qmin[c] = (sn[0] == LLONG_MAX) ? -1 : sn[0];
    }
}

// Optional sub-sample between the column extrema (Sec. 2.3, after Eq. 15).
// For column c and level j = 1..s the target is min_c + (max_c - min_c) j /
// (s + 1), from the stored Z at the arg-extrema rows; each block stages
// kBetweenFloats / kp rows of Z in LDS (rows padded by one float, so a
// wave reading one column of 64 rows hits 64 banks) and reports, per
// (column, level) pair, its row nearest to the target (smallest |Z - target|,
// lowest row on ties).  A column without extrema (qmax or qmin < 0) reports
// no row.
constexpr int kBetweenFloats = 8192;

__global__ __launch_bounds__(256) void between_partial_kernel(const float* __restrict__ Z, int64_t M, int64_t ld_z,
                                                              int kp, int k, int s, const long long* __restrict__ qmax,
                                                              const long long* __restrict__ qmin,
                                                              float* __restrict__ pval, long long* __restrict__ pidx) {
    __shared__ float zs[kBetweenFloats + kBetweenFloats / 16];
    const int rows = kBetweenFloats / kp;  // kp in {16, 32, 64, 128}
    const int ldl = kp + 1;
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    for (int e = threadIdx.x; e < rows * kp; e += blockDim.x) {
        const int rr = e / kp, c = e - rr * kp;
        zs[rr * ldl + c] = (r0 + rr < M) ? Z[(r0 + rr) * ld_z + c] : 0.f;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int npairs = k * s;
    for (int pr = wave; pr < npairs; pr += (int)(blockDim.x >> 6)) {
        const int c = pr / s, j = pr - c * s + 1;
        const long long ix = qmax[c], in = qmin[c];
        float best = INFINITY;
        long long brow = LLONG_MAX;
        if (ix >= 0 && in >= 0) {
            const float hi = Z[ix * ld_z + c], lo = Z[in * ld_z + c];
            const float level = lo + (hi - lo) * ((float)j / (float)(s + 1));
            for (int rr = lane; rr < rows; rr += 64) {
                if (r0 + rr >= M) break;
                const float d = fabsf(zs[rr * ldl + c] - level);
                if (d < best) {
                    best = d;
                    brow = r0 + rr;
                }
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const float ob = __shfl_xor(best, off);
            const long long orow = __shfl_xor(brow, off);
            if (ob < best || (ob == best && orow < brow)) {
                best = ob;
                brow = orow;
            }
        }
        if (lane == 0) {
            pval[(size_t)blockIdx.x * npairs + pr] = best;
            pidx[(size_t)blockIdx.x * npairs + pr] = brow;
        }
    }
}

// One block per (column, level) pair: the nearest row over the partials of
// every row block (lowest row on ties), -1 when there is none.
__global__ void between_reduce_kernel(const float* __restrict__ pval, const long long* __restrict__ pidx,
                                      int64_t nblocks, int npairs, long long* __restrict__ q) {
    const int pr = blockIdx.x;
    float best = INFINITY;
    long long brow = LLONG_MAX;
    for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
        const float v = pval[(size_t)b * npairs + pr];
        const long long r = pidx[(size_t)b * npairs + pr];
        if (r != LLONG_MAX && (v < best || (v == best && r < brow))) {
            best = v;
            brow = r;
        }
    }
    __shared__ float sv[256];
    __shared__ long long sr[256];
    sv[threadIdx.x] = best;
    sr[threadIdx.x] = brow;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const int o = threadIdx.x + st;
            if (sv[o] < sv[threadIdx.x] || (sv[o] == sv[threadIdx.x] && sr[o] < sr[threadIdx.x])) {
                sv[threadIdx.x] = sv[o];
                sr[threadIdx.x] = sr[o];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) q[pr] = (sr[0] == LLONG_MAX) ? -1 : sr[0];
}

template <int KB>
static hipError_t project_dispatch(int mode, dim3 grid, hipStream_t s, const float* I, int64_t M, int N, int64_t ld,
                                   const float* rinv, float floor, const float* Wt, int ldw, int k_store, float* Z,
                                   int64_t ld_z, ArgPart part, int k_arg) {
#define FKK_PJ(a, b)                                                                                               \
    hipLaunchKernelGGL((project_kernel<KB, a, b>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, Wt, ldw, k_store, \
                       Z, ld_z, part.maxv, part.minv, part.maxi, part.mini, k_arg)
    if (mode == 2) FKK_PJ(true, true);
    else if (mode == 1) FKK_PJ(true, false);
    else FKK_PJ(false, false);
#undef FKK_PJ
    return hipGetLastError();
}

// logged: I already holds l (row stride ld, 16-byte aligned, zero past N up
// to a multiple of 64 columns).
hipError_t launch_project(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                          const float* Wt, int ldw, int kp, int k_store, float* Z, int64_t ld_z, ArgPart part,
                          int k_arg, hipStream_t s, bool logged) {
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    const int mode = logged ? 2 : (vec ? 1 : 0);
    dim3 grid((unsigned)proj_blocks(M));
    switch (kp) {
        case 16: return project_dispatch<1>(mode, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, k_store, Z, ld_z, part, k_arg);
        case 32: return project_dispatch<2>(mode, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, k_store, Z, ld_z, part, k_arg);
        case 64: return project_dispatch<4>(mode, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, k_store, Z, ld_z, part, k_arg);
        case 128: return project_dispatch<8>(mode, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, k_store, Z, ld_z, part, k_arg);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_argext_reduce(ArgPart part, int64_t nblocks, int kp, int k, long long* qmax, long long* qmin,
                                hipStream_t s) {
    hipLaunchKernelGGL(argext_reduce_kernel, dim3(k), dim3(256), 0, s, part, nblocks, kp, qmax, qmin);
    return hipGetLastError();
}

int64_t between_blocks(int64_t M, int kp) { return (M + kBetweenFloats / kp - 1) / (kBetweenFloats / kp); }

hipError_t launch_between(const float* Z, int64_t M, int64_t ld_z, int kp, int k, int s, const long long* qmax,
                          const long long* qmin, float* pval, long long* pidx, long long* q, hipStream_t st) {
    if (M < 1 || k < 1 || s < 1 || (kp != 16 && kp != 32 && kp != 64 && kp != 128) || k > kp || ld_z < kp)
        return hipErrorInvalidValue;
    const int64_t nb = between_blocks(M, kp);
    hipLaunchKernelGGL(between_partial_kernel, dim3((unsigned)nb), dim3(256), 0, st, Z, M, ld_z, kp, k, s, qmax, qmin,
                       pval, pidx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(between_reduce_kernel, dim3(k * s), dim3(256), 0, st, pval, pidx, nb, k * s, q);
    return hipGetLastError();
}

// Basis residual (retraining criterion, Sec. 5) without an output: the
// projection of a 128-spectrum block onto the basis, the two sums of every
// spectrum (store_anorms / store_znorms, FP32), and their FP64 sums over the
// block in a fixed order into part[2 b], part[2 b + 1].
template <int KB, bool VEC>
__global__ __launch_bounds__(256) void residual_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                       const float* __restrict__ rinv, float floor,
                                                       const float* __restrict__ Wt, int ldw,
                                                       const float* __restrict__ f, const float* __restrict__ g,
                                                       double* __restrict__ part) {
    constexpr int KP = KB * 16;
    __shared__ __attribute__((aligned(16))) float sL[PR][PLD];
    __shared__ __attribute__((aligned(16))) float sW[KP][PLD];
    __shared__ float sN[2 * PR];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PR;
    const int64_t rows = M - r0 < PR ? M - r0 : PR;
    floatx4 acc[2][KB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < KB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    float asq[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < N; j0 += PNC) {
        stage_logratio<VEC, true>(sL, I, r0, M, N, ld, j0, rinv, floor, f, asq);
        stage_weights<KB>(sW, Wt, ldw, j0);
        __syncthreads();
        project_stage<KB>(acc, sL, sW, wave, lane);
        __syncthreads();
    }
    sN[tid] = 0.f;
    __syncthreads();
    store_anorms(asq, sN, 0, rows);  // rows of this block, in LDS
    store_znorms<KB>(acc, g, sN, 0, rows);
    __syncthreads();
    if (wave == 0) {
        double a = (double)sN[2 * lane] + (double)sN[2 * (lane + 64)];
        double z = (double)sN[2 * lane + 1] + (double)sN[2 * (lane + 64) + 1];
        for (int off = 32; off >= 1; off >>= 1) {
            a += __shfl_xor(a, off);
            z += __shfl_xor(z, off);
        }
        if (lane == 0) {
            part[2 * blockIdx.x] = a;
            part[2 * blockIdx.x + 1] = z;
        }
    }
}

// Sum of nparts (a, z) pairs in a fixed order: out[0], out[1].
__global__ __launch_bounds__(256) void residual_total_kernel(const double* __restrict__ part, int64_t nparts,
                                                             double* __restrict__ out) {
    __shared__ double red[2][4];
    double a = 0.0, z = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += 256) {
        a += part[2 * i];
        z += part[2 * i + 1];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off);
        z += __shfl_xor(z, off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        out[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Per segment s (rows offs[s] .. offs[s+1]-1 of a norms array), the FP64
// sums of both norms: out[2 s], out[2 s + 1].  One block per segment.
__global__ __launch_bounds__(256) void segment_sums_kernel(const float* __restrict__ norms,
                                                           const long long* __restrict__ offs,
                                                           double* __restrict__ out) {
    __shared__ double red[2][4];
    const long long b = offs[blockIdx.x], e = offs[blockIdx.x + 1];
    double a = 0.0, z = 0.0;
    for (long long r = b + threadIdx.x; r < e; r += 256) {
        a += norms[2 * r];
        z += norms[2 * r + 1];
    }
    for (int off = 32; off >= 1; off >>= 1) {
        a += __shfl_xor(a, off);
        z += __shfl_xor(z, off);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = a;
        red[1][wave] = z;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        out[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

hipError_t launch_residual_partials(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                                    const float* Wt, int ldw, int kp, const float* f, const float* g, double* part,
                                    hipStream_t s) {
    if (M < 1) return hipSuccess;
    if (!f || !g || !part) return hipErrorInvalidValue;
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    dim3 grid((unsigned)proj_blocks(M));
#define FKK_RS(KB)                                                                                                  \
    do {                                                                                                            \
        if (vec)                                                                                                    \
            hipLaunchKernelGGL((residual_kernel<KB, true>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, Wt,   \
                               ldw, f, g, part);                                                                    \
        else                                                                                                        \
            hipLaunchKernelGGL((residual_kernel<KB, false>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, Wt,  \
                               ldw, f, g, part);                                                                    \
    } while (0)
    switch (kp) {
        case 16: FKK_RS(1); break;
        case 32: FKK_RS(2); break;
        case 64: FKK_RS(4); break;
        case 128: FKK_RS(8); break;
        default: return hipErrorInvalidValue;
    }
#undef FKK_RS
    return hipGetLastError();
}

hipError_t launch_residual_total(const double* part, int64_t nparts, double* out, hipStream_t s) {
    hipLaunchKernelGGL(residual_total_kernel, dim3(1), dim3(256), 0, s, part, nparts, out);
    return hipGetLastError();
}

hipError_t launch_segment_sums(const float* norms, const long long* offs, int nseg, double* out, hipStream_t s) {
    if (nseg < 1) return hipSuccess;
    hipLaunchKernelGGL(segment_sums_kernel, dim3((unsigned)nseg), dim3(256), 0, s, norms, offs, out);
    return hipGetLastError();
}

__global__ void gather_rows_kernel(const float* __restrict__ Z, int64_t ld_z, int k, const long long* __restrict__ q,
                                   int n_q, float* __restrict__ X) {
    const int r = blockIdx.x;
    if (r >= n_q) return;
    const long long row = q[r];
    for (int c = threadIdx.x; c < k; c += blockDim.x) X[(size_t)r * k + c] = Z[row * ld_z + c];
}

hipError_t launch_gather_rows(const float* Z, int64_t ld_z, int k, const long long* q, int n_q, float* X,
                              hipStream_t s) {
    if (n_q <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(n_q), dim3(64), 0, s, Z, ld_z, k, q, n_q, X);
    return hipGetLastError();
}

// ===========================================================================
// Reconstruction: out = plane of exp(Z B_re) exp(i Z B_im).
// The product is formed transposed (A = B^T, B = Z^T) so that every lane
// ends with four consecutive wavenumbers of one spectrum: one 128-bit store.
// Within each group of 16 basis vectors, lane group g = lane/16 holds the
// values of vectors 4q + g (q = 0..3) contiguously (B^T is stored with the
// 4 x 4 transposed order, see kgroup_pos), so matrix-core step q covers the
// consecutive vectors 4q..4q+3 and the steps past k are skipped.
// ===========================================================================
constexpr int RR = 128;  // rows per block (4 waves x 32)
constexpr int RCN = 64;  // wavenumbers per chunk

// Matrix-core steps q < Q of basis group kg (vectors 16 kg + 4q .. +3).
template <int KB, int Q>
__device__ __forceinline__ void recon_group(const float4 (&zf)[2][KB], const float* sRe, const float* sIm, int bld,
                                            int lane, int kg, floatx4 (&are)[4][2], floatx4 (&aim)[4][2]) {
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) {
        const int off = (ib * 16 + (lane & 15)) * bld + kg * 16 + 4 * (lane >> 4);
        const float4 bre = *reinterpret_cast<const float4*>(sRe + off);
        const float4 bim = *reinterpret_cast<const float4*>(sIm + off);
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                are[ib][jb] = mfma4(f4get(bre, q), f4get(zf[jb][kg], q), are[ib][jb]);
                aim[ib][jb] = mfma4(f4get(bim, q), f4get(zf[jb][kg], q), aim[ib][jb]);
            }
    }
}

// QL: steps of the last group that hold vectors below k (1..4).
template <int KB, int QL>
__device__ __forceinline__ void recon_chunk(const float4 (&zf)[2][KB], const float* sRe, const float* sIm, int bld,
                                            int lane, floatx4 (&are)[4][2], floatx4 (&aim)[4][2]) {
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            are[ib][jb] = floatx4{0.f, 0.f, 0.f, 0.f};
            aim[ib][jb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
    for (int kg = 0; kg + 1 < KB; ++kg) recon_group<KB, 4>(zf, sRe, sIm, bld, lane, kg, are, aim);
    recon_group<KB, QL>(zf, sRe, sIm, bld, lane, KB - 1, are, aim);
}

template <int KB, int QL, bool VEC_OUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void recon_kernel(const float* __restrict__ Z, int64_t M, int64_t ld_z, int k,
                                                    const float* __restrict__ BreT, const float* __restrict__ BimT,
                                                    int N, float* __restrict__ out, int64_t ld_out, int plane) {
    constexpr int KP = KB * 16;
    constexpr int BLD = KP + 4;
    __shared__ __attribute__((aligned(16))) float sRe[RCN * BLD];
    __shared__ __attribute__((aligned(16))) float sIm[RCN * BLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * RR;

    float4 zf[2][KB];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kg = 0; kg < KB; ++kg) {
            const int64_t row = r0 + wave * 32 + jb * 16 + (lane & 15);
            const int c = kg * 16 + (lane >> 4);  // vectors c + 4q
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = (row < M && c + 4 * q < k) ? Z[row * ld_z + c + 4 * q] : 0.f;
            zf[jb][kg] = make_float4(v[0], v[1], v[2], v[3]);
        }

    floatx4 are[4][2], aim[4][2];
    constexpr int PER_ROW = KP / 4;
    floatx4 nre[KB], nim[KB];  // native vectors stay in registers
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        const int idx = threadIdx.x + 256 * p;
        const size_t src = (size_t)(idx / PER_ROW) * KP + (idx % PER_ROW) * 4;
        nre[p] = *reinterpret_cast<const floatx4*>(BreT + src);
        nim[p] = *reinterpret_cast<const floatx4*>(BimT + src);
    }
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        const int idx = threadIdx.x + 256 * p;
        const int dst = (idx / PER_ROW) * BLD + (idx % PER_ROW) * 4;
        *reinterpret_cast<floatx4*>(sRe + dst) = nre[p];
        *reinterpret_cast<floatx4*>(sIm + dst) = nim[p];
    }
    __syncthreads();
    for (int j0 = 0; j0 < N; j0 += RCN) {
        // the last chunk reloads itself (harmless) so loads stay unconditional
        const int jn = (j0 + RCN < N) ? j0 + RCN : j0;
#pragma unroll
        for (int p = 0; p < KB; ++p) {
            const int idx = threadIdx.x + 256 * p;
            const size_t src = (size_t)(jn + idx / PER_ROW) * KP + (idx % PER_ROW) * 4;
            nre[p] = *reinterpret_cast<const floatx4*>(BreT + src);
            nim[p] = *reinterpret_cast<const floatx4*>(BimT + src);
        }
        recon_chunk<KB, QL>(zf, sRe, sIm, BLD, lane, are, aim);
        __syncthreads();
#pragma unroll
        for (int p = 0; p < KB; ++p) {
            const int idx = threadIdx.x + 256 * p;
            const int dst = (idx / PER_ROW) * BLD + (idx % PER_ROW) * 4;
            *reinterpret_cast<floatx4*>(sRe + dst) = nre[p];
            *reinterpret_cast<floatx4*>(sIm + dst) = nim[p];
        }
        store_out<VEC_OUT>(out, ld_out, M, N, r0, wave, lane, j0, are, aim, plane);
        __syncthreads();
    }
}

template <int KB>
static hipError_t recon_dispatch(bool vec, dim3 grid, hipStream_t s, const float* Z, int64_t M, int64_t ld_z, int k,
                                 const float* BreT, const float* BimT, int N, float* out, int64_t ld_out, int plane) {
    // steps of the last basis group below k; the unaligned-output variant
    // runs all four (the padded vectors are zero)
    const int ql = ((k - 1 - 16 * (KB - 1)) >> 2) + 1;
#define FKK_RC(Q, V) \
    hipLaunchKernelGGL((recon_kernel<KB, Q, V>), grid, dim3(256), 0, s, Z, M, ld_z, k, BreT, BimT, N, out, ld_out, plane)
    if (!vec) FKK_RC(4, false);
    else if (ql == 1) FKK_RC(1, true);
    else if (ql == 2) FKK_RC(2, true);
    else if (ql == 3) FKK_RC(3, true);
    else FKK_RC(4, true);
#undef FKK_RC
    return hipGetLastError();
}

hipError_t launch_reconstruct(const float* Z, int64_t M, int64_t ld_z, int k, const float* BreT, const float* BimT,
                              int kp, int N, float* out, int64_t ld_out, int plane, hipStream_t s) {
    const bool vec = ((reinterpret_cast<uintptr_t>(out) & 15) == 0) && (ld_out % 4 == 0);
    dim3 grid((unsigned)((M + RR - 1) / RR));
    switch (kp) {
        case 16: return recon_dispatch<1>(vec, grid, s, Z, M, ld_z, k, BreT, BimT, N, out, ld_out, plane);
        case 32: return recon_dispatch<2>(vec, grid, s, Z, M, ld_z, k, BreT, BimT, N, out, ld_out, plane);
        case 64: return recon_dispatch<4>(vec, grid, s, Z, M, ld_z, k, BreT, BimT, N, out, ld_out, plane);
        case 128: return recon_dispatch<8>(vec, grid, s, Z, M, ld_z, k, BreT, BimT, N, out, ld_out, plane);
        default: return hipErrorInvalidValue;
    }
}

// ===========================================================================
// Fused stored-basis transform: each block projects its 128 spectra onto W
// (Z tile kept in LDS) and reconstructs them; I is read once, out written
// once.
// ===========================================================================
// NORMS: also the residual sums of every spectrum (store_anorms /
// store_znorms) into norms, from the same loads and the same projection.
template <int KB, int QL, bool VEC_IN, bool VEC_OUT, bool NORMS>
__global__ __launch_bounds__(256) void transform_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                        const float* __restrict__ rinv, float floor,
                                                        const float* __restrict__ Wt, int ldw,
                                                        const float* __restrict__ BreT,
                                                        const float* __restrict__ BimT, int k,
                                                        float* __restrict__ out, int64_t ld_out, int plane,
                                                        const float* __restrict__ f, const float* __restrict__ g,
                                                        float* __restrict__ norms) {
    constexpr int KP = KB * 16;
    constexpr int BLD = KP + 4;
    constexpr int P1 = PR * PLD + KP * PLD;             // projection phase
    constexpr int P2 = PR * BLD + 2 * RCN * BLD;         // reconstruction phase
    constexpr int SMEM = P1 > P2 ? P1 : P2;
    __shared__ __attribute__((aligned(16))) float smem[SMEM];
    float(*sL)[PLD] = reinterpret_cast<float(*)[PLD]>(smem);
    float(*sW)[PLD] = reinterpret_cast<float(*)[PLD]>(smem + PR * PLD);
    float* sZ = smem;
    float* sRe = smem + PR * BLD;
    float* sIm = sRe + RCN * BLD;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PR;

    floatx4 acc[2][KB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < KB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    float asq[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < N; j0 += PNC) {
        stage_logratio<VEC_IN, NORMS>(sL, I, r0, M, N, ld, j0, rinv, floor, f, asq);
        stage_weights<KB>(sW, Wt, ldw, j0);
        __syncthreads();
        project_stage<KB>(acc, sL, sW, wave, lane);
        __syncthreads();
    }
    if (NORMS) {
        store_anorms(asq, norms, r0, M);
        store_znorms<KB>(acc, g, norms, r0, M);
    }
    // Z tile to LDS: sZ[row][c]
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < KB; ++cb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = wave * 32 + rb * 16 + 4 * (lane >> 4) + v;
                const int kk = lane & 15;  // vector 16 cb + kk at position 4 (kk % 4) + kk / 4
                sZ[row * BLD + cb * 16 + 4 * (kk & 3) + (kk >> 2)] = acc[rb][cb][v];
            }
    __syncthreads();
    float4 zf[2][KB];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kg = 0; kg < KB; ++kg)
            zf[jb][kg] = *reinterpret_cast<const float4*>(sZ + (wave * 32 + jb * 16 + (lane & 15)) * BLD + kg * 16 +
                                                          4 * (lane >> 4));
    // sRe / sIm live beyond sZ, so no barrier is needed before staging them.
    floatx4 are[4][2], aim[4][2];
    constexpr int PER_ROW = KP / 4;
    floatx4 nre[KB], nim[KB];  // native vectors stay in registers
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        const int idx = threadIdx.x + 256 * p;
        const size_t src = (size_t)(idx / PER_ROW) * KP + (idx % PER_ROW) * 4;
        nre[p] = *reinterpret_cast<const floatx4*>(BreT + src);
        nim[p] = *reinterpret_cast<const floatx4*>(BimT + src);
    }
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        const int idx = threadIdx.x + 256 * p;
        const int dst = (idx / PER_ROW) * BLD + (idx % PER_ROW) * 4;
        *reinterpret_cast<floatx4*>(sRe + dst) = nre[p];
        *reinterpret_cast<floatx4*>(sIm + dst) = nim[p];
    }
    __syncthreads();
    for (int j0 = 0; j0 < N; j0 += RCN) {
        // the last chunk reloads itself (harmless) so loads stay unconditional
        const int jn = (j0 + RCN < N) ? j0 + RCN : j0;
#pragma unroll
        for (int p = 0; p < KB; ++p) {
            const int idx = threadIdx.x + 256 * p;
            const size_t src = (size_t)(jn + idx / PER_ROW) * KP + (idx % PER_ROW) * 4;
            nre[p] = *reinterpret_cast<const floatx4*>(BreT + src);
            nim[p] = *reinterpret_cast<const floatx4*>(BimT + src);
        }
        recon_chunk<KB, QL>(zf, sRe, sIm, BLD, lane, are, aim);
        __syncthreads();
#pragma unroll
        for (int p = 0; p < KB; ++p) {
            const int idx = threadIdx.x + 256 * p;
            const int dst = (idx / PER_ROW) * BLD + (idx % PER_ROW) * 4;
            *reinterpret_cast<floatx4*>(sRe + dst) = nre[p];
            *reinterpret_cast<floatx4*>(sIm + dst) = nim[p];
        }
        store_out<VEC_OUT>(out, ld_out, M, N, r0, wave, lane, j0, are, aim, plane);
        __syncthreads();
    }
}

template <int KB, bool NORMS>
static hipError_t transform_dispatch(bool vin, bool vout, dim3 grid, hipStream_t s, const float* I, int64_t M, int N,
                                     int64_t ld, const float* rinv, float floor, const float* Wt, int ldw,
                                     const float* BreT, const float* BimT, int k, float* out, int64_t ld_out,
                                     int plane, const float* f, const float* g, float* norms) {
    const int ql = ((k - 1 - 16 * (KB - 1)) >> 2) + 1;  // as in recon_dispatch
#define FKK_TR(Q, a, b)                                                                                              \
    hipLaunchKernelGGL((transform_kernel<KB, Q, a, b, NORMS>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, Wt, \
                       ldw, BreT, BimT, k, out, ld_out, plane, f, g, norms)
    if (vin && vout) {
        if (ql == 1) FKK_TR(1, true, true);
        else if (ql == 2) FKK_TR(2, true, true);
        else if (ql == 3) FKK_TR(3, true, true);
        else FKK_TR(4, true, true);
    } else if (vin) FKK_TR(4, true, false);
    else if (vout) FKK_TR(4, false, true);
    else FKK_TR(4, false, false);
#undef FKK_TR
    return hipGetLastError();
}

template <int KB>
static hipError_t transform_dispatch_n(bool vin, bool vout, dim3 grid, hipStream_t s, const float* I, int64_t M,
                                       int N, int64_t ld, const float* rinv, float floor, const float* Wt, int ldw,
                                       const float* BreT, const float* BimT, int k, float* out, int64_t ld_out,
                                       int plane, const float* f, const float* g, float* norms) {
    if (norms)
        return transform_dispatch<KB, true>(vin, vout, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, BreT, BimT, k,
                                            out, ld_out, plane, f, g, norms);
    return transform_dispatch<KB, false>(vin, vout, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, BreT, BimT, k, out,
                                         ld_out, plane, f, g, norms);
}

hipError_t launch_transform(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                            const float* Wt, int ldw, int kp, int k, const float* BreT, const float* BimT, float* out,
                            int64_t ld_out, int plane, hipStream_t s, const ResidualArgs& res) {
    const bool vin = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    const bool vout = ((reinterpret_cast<uintptr_t>(out) & 15) == 0) && (ld_out % 4 == 0);
    if (res.norms && (!res.f || !res.g)) return hipErrorInvalidValue;
    dim3 grid((unsigned)proj_blocks(M));
#define FKK_TD(KB)                                                                                                 \
    return transform_dispatch_n<KB>(vin, vout, grid, s, I, M, N, ld, rinv, floor, Wt, ldw, BreT, BimT, k, out,    \
                                    ld_out, plane, res.f, res.g, res.norms)
    switch (kp) {
        case 16: FKK_TD(1);
        case 32: FKK_TD(2);
        case 64: FKK_TD(4);
        case 128: FKK_TD(8);
        default: return hipErrorInvalidValue;
    }
#undef FKK_TD
}

}  // namespace dev
}  // namespace fkk
