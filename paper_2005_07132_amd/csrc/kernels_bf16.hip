// BF16 variants of the fKK-EC contractions: the Gram of Eq. 6, the
// projections of Eq. 13 and Eq. 25 and the reconstruction of Eq. 23, on
// v_mfma_f32_16x16x32_bf16.  Operands are rounded to BF16 (nearest even)
// when they are staged; accumulation, the log ratio and the exp / sin
// epilogue stay FP32.
//
// For a 16x16x32 block lane l supplies A[l%16][k] and B[k][l%16] for eight
// k values, taken here as k = 8 (l/16) + e, e = 0..7 (any assignment is
// valid as long as A and B use the same one), and receives D[4 (l/16) + v]
// [l%16] in accumulator element v.  Every operand fragment is then eight
// consecutive k of one row: one 128-bit LDS load when rows are stored
// k-contiguous.  Element e of a fragment sits in bits 16 (e%2) of dword e/2.
#include "kernels.h"
#include "device_common.h"

#include <algorithm>

namespace fkk {
namespace dev {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma16(const u32x4& a, const u32x4& b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                   0, 0);
}

// Two floats rounded to BF16, lo in bits 0-15.
__device__ __forceinline__ unsigned pack2(float lo, float hi) {
    const bf16x2 v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(unsigned, v);
}

constexpr int GT = kGramTile;
constexpr int G16 = 8;        // 8-row groups per Gram LDS stage (64 rows)
constexpr int LR_ROWS = 256;  // rows per log-ratio block (a multiple of 8)
constexpr int PR = kProjRows; // spectra per projection / transform block
constexpr int PNC = 64;       // wavenumbers per projection stage
constexpr int SLD = PNC + 8;  // BF16 row stride of staged tiles (144 bytes)
constexpr int RCN = 64;       // wavenumbers per reconstruction chunk

// ---------------------------------------------------------------------------
// Log-ratio pass for the BF16 Gram: l = 1/2 ln(I r) rounded to BF16 in
// row-group-packed order: for each group of 8 rows g and column n, the 8
// values l[8g..8g+7][n] are one 16-byte unit Lp[g * npad + n] (rows past M
// and columns past N are zero).  Column sums and the clamp count as in the
// FP32 pass (same block layout of the partial sums).
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ __launch_bounds__(256) void logratio16_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                         const float* __restrict__ rinv, float floor,
                                                         u32x4* __restrict__ Lp, int npad,
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
        for (int64_t row0 = r0; row0 < r1; row0 += 8) {
            float4 x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                x[u] = (row0 + u < r1) ? load4_guarded(I + (row0 + u) * ld, c, N, VEC) : make_float4(0.f, 0.f, 0.f, 0.f);
            float l[8][4];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    bool bad;
                    const float xv = f4get(x[u], q);
                    float lv = log_ratio(xv, r[q], rl[q], floor, bad);
                    if (row0 + u < r1 && c + q < N) {
                        cnt += bad ? 1u : 0u;
                        cs[q] += (double)xv;
                    } else {
                        lv = 0.f;
                    }
                    l[u][q] = lv;
                }
            u32x4* dst = Lp + (size_t)(row0 >> 3) * npad + c;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                dst[q] = u32x4{pack2(l[0][q], l[1][q]), pack2(l[2][q], l[3][q]), pack2(l[4][q], l[5][q]),
                               pack2(l[6][q], l[7][q])};
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) colsum_part[(size_t)blockIdx.x * npad + c + q] = cs[q];
    }
    for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(clamps, (unsigned long long)cnt);
}

// ---------------------------------------------------------------------------
// Gram partials from the packed BF16 log ratio: same tiles, chunks and
// XCD-aware block order as the FP32 kernel; a stage holds 8 row groups of
// the two 128-column strips, stored unit for unit as they are in memory.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gram16_kernel(const u32x4* __restrict__ Lp, int npad, int64_t ngroups, int T,
                                                     int64_t gpc, const int* __restrict__ tiles,
                                                     double* __restrict__ partial) {
    __shared__ u32x4 sA[2][G16][GT];
    __shared__ u32x4 sB[2][G16][GT];

    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int rr = b >> 3;
    const int tile = rr % T;
    const int chunk = (rr / T) * 8 + xcd;
    const int bi = tiles[2 * tile], bj = tiles[2 * tile + 1];
    const bool diag = (bi == bj);
    const int64_t g0 = (int64_t)chunk * gpc;
    const int64_t g1 = (g0 + gpc < ngroups) ? g0 + gpc : ngroups;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lg = tid >> 7, lc = tid & 127;
    const u32x4* La = Lp + bi * GT + lc;
    const u32x4* Lb = Lp + bj * GT + lc;

    floatx4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

    u32x4 xa[4], xb[4];
    unsigned keep[4];
    // Groups past the chunk are loaded from its last group and masked to
    // zero at the LDS store, so the loads are unconditional.
    auto load = [&](int64_t base) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int64_t g = base + lg + 2 * p;
            const int64_t gc = g < g1 ? g : g1 - 1;
            keep[p] = g < g1 ? 0xffffffffu : 0u;
            xa[p] = La[gc * npad];
            if (!diag) xb[p] = Lb[gc * npad];
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            sA[buf][lg + 2 * p][lc] = xa[p] & keep[p];
            if (!diag) sB[buf][lg + 2 * p][lc] = xb[p] & keep[p];
        }
    };

    const int64_t nst = (g1 > g0) ? (g1 - g0 + G16 - 1) / G16 : 0;
    if (nst > 0) {
        load(g0);
        store(0);
    }
    __syncthreads();
    for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        if (s + 1 < nst) load(g0 + (s + 1) * G16);
        const u32x4(*A)[GT] = sA[buf];
        const u32x4(*B)[GT] = diag ? sA[buf] : sB[buf];
#pragma unroll
        for (int ks = 0; ks < G16 / 4; ++ks) {
            const int grp = ks * 4 + (lane >> 4);
            u32x4 av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = A[grp][wr * 64 + i * 16 + (lane & 15)];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = B[grp][wc * 64 + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = mfma16(av[i], bv[j], acc[i][j]);
        }
        if (s + 1 < nst) store(buf ^ 1);
        __syncthreads();
    }

    double* P = partial + ((size_t)chunk * T + tile) * (size_t)(GT * GT);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = wr * 64 + i * 16 + 4 * (lane >> 4) + v;
                const int c = wc * 64 + j * 16 + (lane & 15);
                P[r * GT + c] = (double)acc[i][j][v];
            }
}

// ---------------------------------------------------------------------------
// Projection Z = l W (BF16 operands).
// ---------------------------------------------------------------------------

// One 128 x 64 tile of l = 1/2 ln(I r) into LDS as BF16 (zeros outside).
// NORMS: also adds (l f)^2 of the FP32 log ratio (before the BF16 rounding)
// to asq[p] (row lrow + 16 p).
template <bool VEC, bool NORMS = false>
__device__ __forceinline__ void stage_logratio16(unsigned short (*sL)[SLD], const float* __restrict__ I, int64_t r0,
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
        *reinterpret_cast<uint2*>(&sL[lrow + 16 * p][lcol]) = make_uint2(pack2(l[0], l[1]), pack2(l[2], l[3]));
    }
}

// Rows 0..KQ-1, columns j0..j0+63 of W^T (BF16, row stride ldw, zero past
// k and N) into LDS.
template <int KQ>
__device__ __forceinline__ void stage_weights16(unsigned short (*sW)[SLD], const unsigned short* __restrict__ Wt,
                                                int ldw, int j0) {
#pragma unroll
    for (int p = 0; p < KQ / 32; ++p) {
        const int u = threadIdx.x + 256 * p;
        const int c = u >> 3, c8 = (u & 7) * 8;
        *reinterpret_cast<u32x4*>(&sW[c][c8]) = *reinterpret_cast<const u32x4*>(Wt + (size_t)c * ldw + j0 + c8);
    }
}

// acc[rb][cb] (rows in the accumulator elements) += l W over one stage.
template <int NCB>
__device__ __forceinline__ void project16_stage(floatx4 (&acc)[2][NCB], const unsigned short (*sL)[SLD],
                                                const unsigned short (*sW)[SLD], int wave, int lane) {
#pragma unroll
    for (int ks = 0; ks < PNC / 32; ++ks) {
        const int kc = ks * 32 + 8 * (lane >> 4);
        u32x4 a[2], w[NCB];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) a[rb] = *reinterpret_cast<const u32x4*>(&sL[wave * 32 + rb * 16 + (lane & 15)][kc]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) w[cb] = *reinterpret_cast<const u32x4*>(&sW[cb * 16 + (lane & 15)][kc]);
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = mfma16(a[rb], w[cb], acc[rb][cb]);
    }
}

// Same product transposed: accT[cb][rb] holds 4 consecutive columns of one
// spectrum per lane (column 16 cb + 4 (l/16) + v of spectrum 32 w + 16 rb + l%16).
template <int NCB>
__device__ __forceinline__ void project16_stage_t(floatx4 (&accT)[NCB][2], const unsigned short (*sL)[SLD],
                                                  const unsigned short (*sW)[SLD], int wave, int lane) {
#pragma unroll
    for (int ks = 0; ks < PNC / 32; ++ks) {
        const int kc = ks * 32 + 8 * (lane >> 4);
        u32x4 a[2], w[NCB];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) a[rb] = *reinterpret_cast<const u32x4*>(&sL[wave * 32 + rb * 16 + (lane & 15)][kc]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) w[cb] = *reinterpret_cast<const u32x4*>(&sW[cb * 16 + (lane & 15)][kc]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) accT[cb][rb] = mfma16(w[cb], a[rb], accT[cb][rb]);
    }
}

template <int NCB, bool VEC>
__global__ __launch_bounds__(256) void project16_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                        const float* __restrict__ rinv, float floor,
                                                        const unsigned short* __restrict__ Wt, int ldw, int k_store,
                                                        float* __restrict__ Z, int64_t ld_z, float* pmaxv,
                                                        float* pminv, long long* pmaxi, long long* pmini,
                                                        int k_arg) {
    constexpr int KQ = NCB * 16;
    __shared__ __attribute__((aligned(16))) unsigned short sL[PR][SLD];
    __shared__ __attribute__((aligned(16))) unsigned short sW[KQ][SLD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PR;
    floatx4 acc[2][NCB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < N; j0 += PNC) {
        stage_logratio16<VEC>(sL, I, r0, M, N, ld, j0, rinv, floor);
        stage_weights16<KQ>(sW, Wt, ldw, j0);
        __syncthreads();
        project16_stage<NCB>(acc, sL, sW, wave, lane);
        __syncthreads();
    }
    project_finish<NCB>(acc, r0, M, Z, ld_z, k_store, pmaxv, pminv, pmaxi, pmini, k_arg);
}

// ---------------------------------------------------------------------------
// Reconstruction (transposed as in the FP32 kernel: A = B^T from LDS, B = Z^T
// in registers).  B^T is (rows = wavenumbers) x KQ BF16, 16-byte units
// staged with one unit of padding per row.
// ---------------------------------------------------------------------------
template <int KB2, int NIB = 4>
__device__ __forceinline__ void recon16_chunk(const u32x4 (&zb)[2][KB2], const u32x4* sRe, const u32x4* sIm,
                                              int lane, floatx4 (&are)[NIB][2], floatx4 (&aim)[NIB][2],
                                              int ib0 = 0) {
    constexpr int BLDU = KB2 * 4 + 1;
#pragma unroll
    for (int ib = 0; ib < NIB; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
            are[ib][jb] = floatx4{0.f, 0.f, 0.f, 0.f};
            aim[ib][jb] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
    for (int kg = 0; kg < KB2; ++kg)
#pragma unroll
        for (int ib = 0; ib < NIB; ++ib) {
            const int off = ((ib0 + ib) * 16 + (lane & 15)) * BLDU + kg * 4 + (lane >> 4);
            const u32x4 bre = sRe[off];
            const u32x4 bim = sIm[off];
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                are[ib][jb] = mfma16(bre, zb[jb][kg], are[ib][jb]);
                aim[ib][jb] = mfma16(bim, zb[jb][kg], aim[ib][jb]);
            }
        }
}

// Streams the basis chunks through LDS (next chunk prefetched into registers
// while the current one is multiplied) and writes the output tile.
template <int KB2, bool VEC_OUT>
__device__ __forceinline__ void recon16_loop(const u32x4 (&zb)[2][KB2], const u32x4* __restrict__ BreT,
                                             const u32x4* __restrict__ BimT, u32x4* sRe, u32x4* sIm, int N,
                                             float* __restrict__ out, int64_t ld_out, int64_t M, int64_t r0,
                                             int plane) {
    constexpr int UPR = KB2 * 4;   // 16-byte units per basis row
    constexpr int BLDU = UPR + 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    floatx4 are[4][2], aim[4][2];
    u32x4 nre[KB2], nim[KB2];
#pragma unroll
    for (int p = 0; p < KB2; ++p) {
        const int idx = tid + 256 * p;
        nre[p] = BreT[idx];
        nim[p] = BimT[idx];
    }
#pragma unroll
    for (int p = 0; p < KB2; ++p) {
        const int idx = tid + 256 * p;
        const int dst = (idx / UPR) * BLDU + idx % UPR;
        sRe[dst] = nre[p];
        sIm[dst] = nim[p];
    }
    __syncthreads();
    for (int j0 = 0; j0 < N; j0 += RCN) {
        const int jn = (j0 + RCN < N) ? j0 + RCN : j0;
#pragma unroll
        for (int p = 0; p < KB2; ++p) {
            const size_t src = (size_t)jn * UPR + tid + 256 * p;
            nre[p] = BreT[src];
            nim[p] = BimT[src];
        }
        recon16_chunk<KB2>(zb, sRe, sIm, lane, are, aim);
        __syncthreads();
#pragma unroll
        for (int p = 0; p < KB2; ++p) {
            const int idx = tid + 256 * p;
            const int dst = (idx / UPR) * BLDU + idx % UPR;
            sRe[dst] = nre[p];
            sIm[dst] = nim[p];
        }
        store_out<VEC_OUT, true>(out, ld_out, M, N, r0, wave, lane, j0, are, aim, plane);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Reconstruction with the basis resident in LDS.  A block of W waves holds a
// slice of CW wavenumbers of B_re^T and B_im^T (zero rows past N) for the
// whole launch and walks TPB consecutive tiles of 32 W spectra, 32 per wave.
// The main loop has no barrier and no basis load: its only vector loads are
// the tiles' Z.  With W = 8 the next tile's Z is issued before the current
// tile's stores, so the wait for it (one counter covers loads and stores)
// reaches only stores of two tiles back.  The three-piece form at kq <= 64
// runs W = 12 without that prefetch: the registers then allow three waves
// per SIMD, which hide the Z loads and overlap one wave's stores with
// another's products (1.64 -> 1.52 ms at 703,026 x 1,000, k = 50).
// ---------------------------------------------------------------------------
constexpr int RS_LDS_UNITS = 144 * 1024 / 16;  // LDS for the two basis slices

// Largest slice width (multiple of RCN) whose two planes of P pieces fit the
// LDS budget.
constexpr int rs_cw_max(int kb2, int pieces = 1) { return (RS_LDS_UNITS / (2 * pieces * (kb2 * 4 + 1))) / RCN * RCN; }

// z = z1 + z2 + z3 + r with BF16 pieces z1 = bf16(z), z2 = bf16(z - z1),
// z3 = bf16(z - z1 - z2) (each difference exact in FP32), |r| <= 2^-24 |z|
// roughly; pk[p] packs piece p of two values, lo first.
__device__ __forceinline__ void split3(float a, float b, unsigned (&pk)[3]) {
    const float a1 = (float)(__bf16)a, b1 = (float)(__bf16)b;
    const float ar = a - a1, br = b - b1;
    const float a2 = (float)(__bf16)ar, b2 = (float)(__bf16)br;
    pk[0] = pack2(a1, b1);
    pk[1] = pack2(a2, b2);
    pk[2] = pack2(ar - a2, br - b2);
}

// Raw FP32 Z of one wave's 32 spectra: zr[jb][kg][q] = Z[row][kg 32 + 8 (l/16) + q],
// row = r0 + 16 jb + l%16 (zero past M or k; loads from clamped addresses;
// VEC: rows 16-byte aligned, eight-value groups inside k read as two float4).
template <int KB2, bool VEC>
__device__ __forceinline__ void rs_load_z(float (&zr)[2][KB2][8], const float* __restrict__ Z, int64_t ld_z,
                                          int64_t M, int k, int64_t r0, int lane) {
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        const int64_t row = r0 + jb * 16 + (lane & 15);
        const float* zrow = Z + (row < M ? row : M - 1) * ld_z;
        const float live = row < M ? 1.f : 0.f;
#pragma unroll
        for (int kg = 0; kg < KB2; ++kg) {
            const int c = kg * 32 + 8 * (lane >> 4);
            if (VEC && c + 8 <= k) {
                const float4 a = *reinterpret_cast<const float4*>(zrow + c);
                const float4 b = *reinterpret_cast<const float4*>(zrow + c + 4);
                zr[jb][kg][0] = a.x * live; zr[jb][kg][1] = a.y * live;
                zr[jb][kg][2] = a.z * live; zr[jb][kg][3] = a.w * live;
                zr[jb][kg][4] = b.x * live; zr[jb][kg][5] = b.y * live;
                zr[jb][kg][6] = b.z * live; zr[jb][kg][7] = b.w * live;
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    zr[jb][kg][q] = zrow[c + q < k ? c + q : k - 1] * ((c + q < k) ? live : 0.f);
            }
        }
    }
}

// P = 3: Eq. 23's products to FP32 accuracy on the BF16 matrix cores: B and
// Z each as three BF16 pieces (B's given as consecutive npad x kq planes,
// Z's cut in registers), the six piece products of combined order <= 2,
// smallest first, accumulated in FP32.
template <int KB2, bool VEC_OUT, bool VEC_Z, int P = 1, int W = 8>
__global__ __launch_bounds__(64 * W) void recon16s_kernel(const float* __restrict__ Z, int64_t M, int64_t ld_z,
                                                              int k, const u32x4* __restrict__ BreT,
                                                              const u32x4* __restrict__ BimT, int N, int npad, int cw,
                                                              int nslice, int tpb, float* __restrict__ out,
                                                              int64_t ld_out, int plane) {
    constexpr int UPR = KB2 * 4;   // 16-byte units per basis row
    constexpr int BLDU = UPR + 1;  // padded LDS row
    __shared__ u32x4 sB[RS_LDS_UNITS];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // blockIdx -> (slice, tile group): the nslice blocks of one tile group are
    // 8 apart, so they run on the same XCD and share its L2 for Z
    const int b = blockIdx.x;
    const int xcd = b & 7, rr = b >> 3;
    const int slice = rr % nslice;
    const int64_t group = (int64_t)(rr / nslice) * 8 + xcd;
    constexpr int THREADS = 64 * W, ROWS = 32 * W;
    const int64_t ntiles = (M + ROWS - 1) / ROWS;
    const int64_t t0 = group * tpb;
    if (t0 >= ntiles) return;
    const int64_t t1 = (t0 + tpb < ntiles) ? t0 + tpb : ntiles;
    const int c0 = slice * cw;
    const int c1 = (c0 + cw < N) ? c0 + cw : N;

    // basis slice to LDS: rows c0 .. c0 + cw - 1 (zero past npad); piece pc
    // of plane Re at sB + 2 pc cw BLDU, of plane Im cw BLDU further
    u32x4* sRe = sB;
    u32x4* sIm = sB + cw * BLDU;
#pragma unroll
    for (int pc = 0; pc < P; ++pc) {
        const u32x4* gre = BreT + (size_t)pc * npad * UPR;
        const u32x4* gim = BimT + (size_t)pc * npad * UPR;
        u32x4* lre = sRe + 2 * pc * cw * BLDU;
        u32x4* lim = sIm + 2 * pc * cw * BLDU;
        // (eight units per plane in flight per thread before the LDS writes)
        for (int base = 0; base < cw * UPR; base += 8 * THREADS) {
            u32x4 vre[8], vim[8];
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int idx = base + p * THREADS + tid;
                const int j = c0 + idx / UPR;
                const bool live = idx < cw * UPR && j < npad;
                const size_t src = live ? (size_t)j * UPR + idx % UPR : 0;
                vre[p] = gre[src];
                vim[p] = gim[src];
                if (!live) vre[p] = vim[p] = u32x4{0u, 0u, 0u, 0u};
            }
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int idx = base + p * THREADS + tid;
                if (idx < cw * UPR) {
                    lre[(idx / UPR) * BLDU + idx % UPR] = vre[p];
                    lim[(idx / UPR) * BLDU + idx % UPR] = vim[p];
                }
            }
        }
    }
    __syncthreads();

    // rows of this wave within a tile: group h = wave / 4 of 128 rows, and
    // 32 (wave % 4) .. + 31 within the group (the layout store_out takes)
    // (the next tile's Z is loaded ahead where registers allow: KB2 <= 2
    // with 8 waves)
    constexpr bool PF = KB2 <= 2 && W == 8;
    const int h = wave >> 2, wq = wave & 3;
    float zr[2][KB2][8];
    if (PF) rs_load_z<KB2, VEC_Z>(zr, Z, ld_z, M, k, t0 * ROWS + 128 * h + 32 * wq, lane);
    for (int64_t t = t0; t < t1; ++t) {
        const int64_t r0 = t * ROWS + 128 * h;
        if (!PF) rs_load_z<KB2, VEC_Z>(zr, Z, ld_z, M, k, r0 + 32 * wq, lane);
        u32x4 zb[P][2][KB2];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int kg = 0; kg < KB2; ++kg) {
                if (P == 1) {
                    zb[0][jb][kg] = u32x4{pack2(zr[jb][kg][0], zr[jb][kg][1]), pack2(zr[jb][kg][2], zr[jb][kg][3]),
                                          pack2(zr[jb][kg][4], zr[jb][kg][5]), pack2(zr[jb][kg][6], zr[jb][kg][7])};
                } else {
                    unsigned w[4][3];
#pragma unroll
                    for (int e = 0; e < 4; ++e) split3(zr[jb][kg][2 * e], zr[jb][kg][2 * e + 1], w[e]);
#pragma unroll
                    for (int pc = 0; pc < P; ++pc) zb[pc][jb][kg] = u32x4{w[0][pc], w[1][pc], w[2][pc], w[3][pc]};
                }
            }
        if (PF && t + 1 < t1) rs_load_z<KB2, VEC_Z>(zr, Z, ld_z, M, k, r0 + ROWS + 32 * wq, lane);
        __builtin_amdgcn_sched_barrier(0);
        // each 64-wavenumber chunk in two halves, so that the stores of the
        // first half go out while the second half is multiplied
        for (int j0 = c0; j0 < c1; j0 += RCN)
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                floatx4 are[2][2], aim[2][2];
                if (P == 1) {
                    recon16_chunk<KB2, 2>(zb[0], sRe + (j0 - c0) * BLDU, sIm + (j0 - c0) * BLDU, lane, are, aim,
                                          2 * hh);
                } else {
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int jb = 0; jb < 2; ++jb) are[i][jb] = aim[i][jb] = floatx4{0.f, 0.f, 0.f, 0.f};
                    // piece pairs (z, b) by combined order 2, 1, 0
                    constexpr int PZ[6] = {2, 1, 0, 1, 0, 0}, PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
                    for (int kg = 0; kg < KB2; ++kg)
#pragma unroll
                        for (int i = 0; i < 2; ++i) {
                            const int off = (j0 - c0 + (2 * hh + i) * 16 + (lane & 15)) * BLDU + kg * 4 + (lane >> 4);
#pragma unroll
                            for (int t = 0; t < 6; ++t) {
                                const u32x4 bre = sRe[2 * PB[t] * cw * BLDU + off];
                                const u32x4 bim = sIm[2 * PB[t] * cw * BLDU + off];
#pragma unroll
                                for (int jb = 0; jb < 2; ++jb) {
                                    are[i][jb] = mfma16(bre, zb[PZ[t]][jb][kg], are[i][jb]);
                                    aim[i][jb] = mfma16(bim, zb[PZ[t]][jb][kg], aim[i][jb]);
                                }
                            }
                        }
                }
                store_out<VEC_OUT, P == 1, 2>(out, ld_out, M, N, r0, wq, lane, j0 + 32 * hh, are, aim, plane);
            }
    }
}

// ---------------------------------------------------------------------------
// Projection Z = l W to FP32 accuracy on the BF16 matrix cores: the FP32 log
// ratio staged in LDS and cut into three BF16 pieces as each wave reads its
// operand (split3), W given as three BF16 piece planes (KQ x ldw each,
// consecutive), and the six piece products of combined order <= 2 summed in
// FP32, smallest first within a 32-wavenumber step.  Stages of SW = 32
// wavenumbers at kq <= 64 (38 KB of LDS and 96 registers: four blocks per
// CU, 0.99 ms at 703,026 x 1,000 against 1.19 ms with 64-wavenumber stages
// and two blocks per CU), 64 at kq = 128.
// ---------------------------------------------------------------------------
// One stage of SW wavenumbers (SW = 32 or 64) of the FP32 log ratio of the
// block's PR rows into LDS (row stride SW + 4): thread t takes four columns
// (t % (SW / 4)) * 4 of rows t / (SW / 4) + (1024 / SW) p.
template <bool VEC, int SW>
__device__ __forceinline__ void stage_logratio_f32(float (*sL)[SW + 4], const float* __restrict__ I, int64_t r0,
                                                   int64_t M, int N, int64_t ld, int j0,
                                                   const float* __restrict__ rinv, float floor) {
    constexpr int TPR = SW / 4;           // threads per row
    constexpr int RPP = 256 / TPR;        // rows per pass
    const int tid = threadIdx.x;
    const int lrow = tid / TPR;
    const int lcol = (tid % TPR) * 4;
    const int col = j0 + lcol;
    float r[4], rl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        r[q] = (col + q < N) ? rinv[col + q] : 0.f;
        rl[q] = (col + q < N) ? rinv[N + col + q] : 0.f;
    }
    float4 x[PR / RPP];
#pragma unroll
    for (int p = 0; p < PR / RPP; ++p) {
        const int64_t row = r0 + lrow + RPP * p;
        x[p] = (row < M) ? load4_guarded(I + row * ld, col, N, VEC) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int p = 0; p < PR / RPP; ++p) {
        const int64_t row = r0 + lrow + RPP * p;
        float l[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bool bad;
            l[q] = (row < M && col + q < N) ? log_ratio(f4get(x[p], q), r[q], rl[q], floor, bad) : 0.f;
        }
        *reinterpret_cast<float4*>(&sL[lrow + RPP * p][lcol]) = make_float4(l[0], l[1], l[2], l[3]);
    }
}

// KQ rows of SW BF16 weights (16-byte units) into LDS (row stride SW + 8).
template <int KQ, int SW>
__device__ __forceinline__ void stage_weights16w(unsigned short (*sW)[SW + 8], const unsigned short* __restrict__ Wt,
                                                 int ldw, int j0) {
    constexpr int UPR = SW / 8, UNITS = KQ * UPR;
#pragma unroll
    for (int p = 0; p < (UNITS + 255) / 256; ++p) {
        const int u = threadIdx.x + 256 * p;
        if (UNITS % 256 == 0 || u < UNITS) {
            const int c = u / UPR, c8 = (u % UPR) * 8;
            *reinterpret_cast<u32x4*>(&sW[c][c8]) = *reinterpret_cast<const u32x4*>(Wt + (size_t)c * ldw + j0 + c8);
        }
    }
}

template <int NCB, bool VEC, int SW = (NCB <= 4 ? 32 : PNC)>
__global__ __launch_bounds__(256) void project16x3_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                          const float* __restrict__ rinv, float floor,
                                                          const unsigned short* __restrict__ Wt, int ldw,
                                                          int k_store, float* __restrict__ Z, int64_t ld_z,
                                                          float* pmaxv, float* pminv, long long* pmaxi,
                                                          long long* pmini, int k_arg) {
    constexpr int KQ = NCB * 16;
    __shared__ __attribute__((aligned(16))) float sL[PR][SW + 4];
    __shared__ __attribute__((aligned(16))) unsigned short sW[3][KQ][SW + 8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PR;
    floatx4 acc[2][NCB];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < N; j0 += SW) {
        stage_logratio_f32<VEC, SW>(sL, I, r0, M, N, ld, j0, rinv, floor);
#pragma unroll
        for (int pc = 0; pc < 3; ++pc) stage_weights16w<KQ, SW>(sW[pc], Wt + (size_t)pc * KQ * ldw, ldw, j0);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < SW / 32; ++ks) {
            const int kc = ks * 32 + 8 * (lane >> 4);
            u32x4 a[2][3], w[NCB][3];
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) {
                const float* src = &sL[wave * 32 + rb * 16 + (lane & 15)][kc];
                const float4 x0 = *reinterpret_cast<const float4*>(src);
                const float4 x1 = *reinterpret_cast<const float4*>(src + 4);
                unsigned pk[4][3];
                split3(x0.x, x0.y, pk[0]);
                split3(x0.z, x0.w, pk[1]);
                split3(x1.x, x1.y, pk[2]);
                split3(x1.z, x1.w, pk[3]);
#pragma unroll
                for (int pc = 0; pc < 3; ++pc) a[rb][pc] = u32x4{pk[0][pc], pk[1][pc], pk[2][pc], pk[3][pc]};
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int pc = 0; pc < 3; ++pc) w[cb][pc] = *reinterpret_cast<const u32x4*>(&sW[pc][cb * 16 + (lane & 15)][kc]);
            // piece pairs (l, w) by combined order 2, 1, 0
            constexpr int PA[6] = {2, 1, 0, 1, 0, 0}, PW[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
            for (int t = 0; t < 6; ++t)
#pragma unroll
                for (int rb = 0; rb < 2; ++rb)
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = mfma16(a[rb][PA[t]], w[cb][PW[t]], acc[rb][cb]);
        }
        __syncthreads();
    }
    project_finish<NCB>(acc, r0, M, Z, ld_z, k_store, pmaxv, pminv, pmaxi, pmini, k_arg);
}

// ---------------------------------------------------------------------------
// Fused stored-basis transform in BF16: projection (transposed, so that the
// Z tile goes to LDS as 4-value BF16 stores), then reconstruction.
// ---------------------------------------------------------------------------
// ||A_m V||^2 from the transposed projection tile (accT[cb][rb][v] = Z of
// spectrum 32 w + 16 rb + l%16, column 16 cb + 4 (l/16) + v), with g as in
// store_znorms.  Lanes of one spectrum differ in bits 4 and 5.
template <int NCB>
__device__ __forceinline__ void store_znorms_t(const floatx4 (&accT)[NCB][2], const float* __restrict__ g,
                                               float* __restrict__ norms, int64_t r0, int64_t M) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float sq[2] = {0.f, 0.f};
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const float4 gv = *reinterpret_cast<const float4*>(g + 16 * cb + 4 * (lane >> 4));
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float z = accT[cb][rb][v] * f4get(gv, v);
                sq[rb] = fmaf(z, z, sq[rb]);
            }
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
        float t = sq[rb];
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        const int64_t row = r0 + wave * 32 + 16 * rb + (lane & 15);
        if ((lane >> 4) == 0 && row < M) norms[2 * row + 1] = t;
    }
}

template <int KB2, bool VEC_IN, bool VEC_OUT, bool NORMS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void transform16_kernel(const float* __restrict__ I, int64_t M, int N, int64_t ld,
                                                          const float* __restrict__ rinv, float floor,
                                                          const unsigned short* __restrict__ Wt, int ldw,
                                                          const u32x4* __restrict__ BreT,
                                                          const u32x4* __restrict__ BimT, float* __restrict__ out,
                                                          int64_t ld_out, int plane, const float* __restrict__ f,
                                                          const float* __restrict__ g, float* __restrict__ norms) {
    constexpr int KQ = KB2 * 32, NCB = KB2 * 2;
    constexpr int BLDU = KB2 * 4 + 1;
    constexpr int P1 = (PR * SLD + KQ * SLD) * 2;      // projection phase (bytes)
    constexpr int P2 = (PR * BLDU + 2 * RCN * BLDU) * 16;  // reconstruction phase
    constexpr int SMEM = (P1 > P2 ? P1 : P2) / 16;
    __shared__ u32x4 smem[SMEM];
    unsigned short(*sL)[SLD] = reinterpret_cast<unsigned short(*)[SLD]>(smem);
    unsigned short(*sW)[SLD] = reinterpret_cast<unsigned short(*)[SLD]>(reinterpret_cast<unsigned short*>(smem) + PR * SLD);
    u32x4* sZ = smem;
    u32x4* sRe = smem + PR * BLDU;
    u32x4* sIm = sRe + RCN * BLDU;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PR;

    floatx4 accT[NCB][2];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) accT[cb][rb] = floatx4{0.f, 0.f, 0.f, 0.f};
    float asq[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j0 = 0; j0 < N; j0 += PNC) {
        stage_logratio16<VEC_IN, NORMS>(sL, I, r0, M, N, ld, j0, rinv, floor, f, asq);
        stage_weights16<KQ>(sW, Wt, ldw, j0);
        __syncthreads();
        project16_stage_t<NCB>(accT, sL, sW, wave, lane);
        __syncthreads();
    }
    if (NORMS) {
        store_anorms(asq, norms, r0, M);
        store_znorms_t<NCB>(accT, g, norms, r0, M);
    }
    // Z tile (BF16) to LDS: spectrum row, units of 8 columns.
    unsigned short* sZh = reinterpret_cast<unsigned short*>(sZ);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            const int row = wave * 32 + rb * 16 + (lane & 15);
            const int c = cb * 16 + 4 * (lane >> 4);
            *reinterpret_cast<uint2*>(sZh + row * BLDU * 8 + c) =
                make_uint2(pack2(accT[cb][rb][0], accT[cb][rb][1]), pack2(accT[cb][rb][2], accT[cb][rb][3]));
        }
    __syncthreads();
    u32x4 zb[2][KB2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kg = 0; kg < KB2; ++kg) zb[jb][kg] = sZ[(wave * 32 + jb * 16 + (lane & 15)) * BLDU + kg * 4 + (lane >> 4)];
    // sRe / sIm lie past sZ: no barrier needed before staging them.
    recon16_loop<KB2, VEC_OUT>(zb, BreT, BimT, sRe, sIm, N, out, ld_out, M, r0, plane);
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t logratio16_bytes(int64_t M, int npad) { return (size_t)((M + 7) / 8) * (size_t)npad * 16; }

hipError_t launch_logratio16(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                             uint16_t* Lp, int npad, double* colsum_part, unsigned long long* clamps,
                             hipStream_t s) {
    if (npad % 4 != 0) return hipErrorInvalidValue;
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    dim3 grid((unsigned)((M + LR_ROWS - 1) / LR_ROWS)), block(256);
    u32x4* dst = reinterpret_cast<u32x4*>(Lp);
    if (vec)
        hipLaunchKernelGGL(logratio16_kernel<true>, grid, block, 0, s, I, M, N, ld, rinv, floor, dst, npad,
                           colsum_part, clamps);
    else
        hipLaunchKernelGGL(logratio16_kernel<false>, grid, block, 0, s, I, M, N, ld, rinv, floor, dst, npad,
                           colsum_part, clamps);
    return hipGetLastError();
}

hipError_t launch_gram16(const uint16_t* Lp, int npad, int64_t M, const GramPlan& plan, const int* d_tiles,
                         double* partial, hipStream_t s) {
    if (plan.rows_per_chunk % (8 * G16) != 0 || plan.nb * GT > npad) return hipErrorInvalidValue;
    dim3 grid((unsigned)(plan.tiles * plan.chunks)), block(256);
    hipLaunchKernelGGL(gram16_kernel, grid, block, 0, s, reinterpret_cast<const u32x4*>(Lp), npad, (M + 7) / 8,
                       plan.tiles, plan.rows_per_chunk / 8, d_tiles, partial);
    return hipGetLastError();
}

hipError_t launch_project16(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                            const uint16_t* Wt, int ldw, int kq, int k_store, float* Z, int64_t ld_z, ArgPart part,
                            int k_arg, hipStream_t s, int pieces) {
    if (ldw % 8 != 0 || (pieces != 1 && pieces != 3)) return hipErrorInvalidValue;
    const bool vec = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    dim3 grid((unsigned)proj_blocks(M));
    const unsigned short* w = reinterpret_cast<const unsigned short*>(Wt);
#define FKK_PJ16_K(KERNEL, NCB)                                                                                   \
    do {                                                                                                          \
        if (vec)                                                                                                  \
            hipLaunchKernelGGL((KERNEL<NCB, true>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, w, ldw,      \
                               k_store, Z, ld_z, part.maxv, part.minv, part.maxi, part.mini, k_arg);              \
        else                                                                                                      \
            hipLaunchKernelGGL((KERNEL<NCB, false>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, w, ldw,     \
                               k_store, Z, ld_z, part.maxv, part.minv, part.maxi, part.mini, k_arg);              \
    } while (0)
#define FKK_PJ16(NCB)                                            \
    do {                                                         \
        if (pieces == 3) FKK_PJ16_K(project16x3_kernel, NCB);    \
        else FKK_PJ16_K(project16_kernel, NCB);                  \
    } while (0)
    switch (kq) {
        case 32: FKK_PJ16(2); break;
        case 64: FKK_PJ16(4); break;
        case 128: FKK_PJ16(8); break;
        default: return hipErrorInvalidValue;
    }
#undef FKK_PJ16
#undef FKK_PJ16_K
    return hipGetLastError();
}

hipError_t launch_reconstruct16(const float* Z, int64_t M, int64_t ld_z, int k, const uint16_t* BreT,
                                const uint16_t* BimT, int kq, int N, int npad, float* out, int64_t ld_out, int plane,
                                hipStream_t s, int pieces) {
    if (M <= 0) return hipSuccess;
    if (k < 1 || k > ld_z) return hipErrorInvalidValue;
    if (kq != 32 && kq != 64 && kq != 128) return hipErrorInvalidValue;
    if (pieces != 1 && pieces != 3) return hipErrorInvalidValue;
    if (npad < N) return hipErrorInvalidValue;
    const int kb2 = kq / 32;
    const bool vec = ((reinterpret_cast<uintptr_t>(out) & 15) == 0) && (ld_out % 4 == 0);
    const bool vz = ((reinterpret_cast<uintptr_t>(Z) & 15) == 0) && (ld_z % 4 == 0);
    const u32x4* bre = reinterpret_cast<const u32x4*>(BreT);
    const u32x4* bim = reinterpret_cast<const u32x4*>(BimT);
    // wavenumber slices of equal width (multiple of RCN) that fit LDS
    const int cwm = rs_cw_max(kb2, pieces);
    const int nslice = (N + cwm - 1) / cwm;
    const int cw = ((N + nslice - 1) / nslice + RCN - 1) / RCN * RCN;
    // tiles per block: about 2048 blocks over the whole launch
    // three pieces with kq <= 64: blocks of 12 waves (three per SIMD),
    // otherwise 8
    const int waves = (pieces == 3 && kb2 <= 2) ? 12 : 8;
    const int64_t ntiles = (M + 32 * waves - 1) / (32 * waves);
    int64_t tpb = (ntiles * nslice + 2047) / 2048;
    if (tpb < 1) tpb = 1;
    const int64_t groups = (ntiles + tpb - 1) / tpb;
    // block b -> group 8 (b / 8 / nslice) + b % 8: groups padded to a multiple of 8
    const int64_t nblocks = (groups + 7) / 8 * 8 * nslice;
    if (nblocks > INT_MAX) return hipErrorInvalidValue;
    dim3 grid((unsigned)nblocks), block(64 * waves);
#define FKK_RC16(KB2, VO, VZ, P)                                                                                   \
    hipLaunchKernelGGL((recon16s_kernel<KB2, VO, VZ, P, (P == 3 && KB2 <= 2 ? 12 : 8)>), grid, block, 0, s, Z, M, ld_z, k, bre, bim, N, npad, cw, \
                       nslice, (int)tpb, out, ld_out, plane)
#define FKK_RC16_K(KB2, P)                                          \
    do {                                                            \
        if (vec && vz) FKK_RC16(KB2, true, true, P);                \
        else if (vec) FKK_RC16(KB2, true, false, P);                \
        else if (vz) FKK_RC16(KB2, false, true, P);                 \
        else FKK_RC16(KB2, false, false, P);                        \
    } while (0)
    if (pieces == 1) {
        switch (kb2) {
            case 1: FKK_RC16_K(1, 1); break;
            case 2: FKK_RC16_K(2, 1); break;
            default: FKK_RC16_K(4, 1); break;
        }
    } else {
        switch (kb2) {
            case 1: FKK_RC16_K(1, 3); break;
            case 2: FKK_RC16_K(2, 3); break;
            default: FKK_RC16_K(4, 3); break;
        }
    }
#undef FKK_RC16_K
#undef FKK_RC16
    return hipGetLastError();
}

hipError_t launch_transform16(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                              const uint16_t* Wt, int ldw, int kq, const uint16_t* BreT, const uint16_t* BimT,
                              float* out, int64_t ld_out, int plane, hipStream_t s, const ResidualArgs& res) {
    if (ldw % 8 != 0) return hipErrorInvalidValue;
    if (res.norms && (!res.f || !res.g)) return hipErrorInvalidValue;
    const bool vin = ((reinterpret_cast<uintptr_t>(I) & 15) == 0) && (ld % 4 == 0);
    const bool vout = ((reinterpret_cast<uintptr_t>(out) & 15) == 0) && (ld_out % 4 == 0);
    dim3 grid((unsigned)proj_blocks(M));
    const unsigned short* w = reinterpret_cast<const unsigned short*>(Wt);
    const u32x4* bre = reinterpret_cast<const u32x4*>(BreT);
    const u32x4* bim = reinterpret_cast<const u32x4*>(BimT);
#define FKK_TR16(KB2, A, B, NR)                                                                                    \
    hipLaunchKernelGGL((transform16_kernel<KB2, A, B, NR>), grid, dim3(256), 0, s, I, M, N, ld, rinv, floor, w,   \
                       ldw, bre, bim, out, ld_out, plane, res.f, res.g, res.norms)
#define FKK_TR16_K(KB2)                                                        \
    do {                                                                       \
        if (res.norms) {                                                       \
            if (vin && vout) FKK_TR16(KB2, true, true, true);                  \
            else FKK_TR16(KB2, false, false, true);                            \
        } else if (vin && vout) FKK_TR16(KB2, true, true, false);              \
        else if (vin) FKK_TR16(KB2, true, false, false);                       \
        else if (vout) FKK_TR16(KB2, false, true, false);                      \
        else FKK_TR16(KB2, false, false, false);                               \
    } while (0)
    switch (kq) {
        case 32: FKK_TR16_K(1); break;
        case 64: FKK_TR16_K(2); break;
        case 128: FKK_TR16_K(4); break;
        default: return hipErrorInvalidValue;
    }
#undef FKK_TR16_K
#undef FKK_TR16
    return hipGetLastError();
}

}  // namespace dev
}  // namespace fkk
