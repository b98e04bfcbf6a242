// Launch interface of the gfx950 kernels of the fKK-EC hot path.
//
// rinv arguments hold 1/I_ref as two floats per wavenumber: the nearest
// float in rinv[0..N) and the remainder in rinv[N..2N).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fkk {
namespace dev {

// Gram of the log ratio: tiles of 128 x 128 over the upper triangle, split
// over chunks of rows (a multiple of 8 chunks so that all tiles of a chunk
// run on one XCD).
constexpr int kGramTile = 128;

struct GramPlan {
    int nb = 0;        // column blocks of 128
    int tiles = 0;     // upper-triangle tiles nb(nb+1)/2
    int chunks = 0;    // row chunks (multiple of 8)
    int64_t rows_per_chunk = 0;
    size_t partial_doubles() const { return (size_t)chunks * tiles * kGramTile * kGramTile; }
};
// rows_per_chunk is a multiple of row_quantum (32 for the FP32 kernel, 64
// for the BF16 kernel).
GramPlan gram_plan(int64_t M, int N, int target_chunks, int row_quantum = 32);

// d_tiles: int2[tiles] (bi <= bj) written by the caller from gram_tile_list.
void gram_tile_list(int nb, int* host_pairs /* 2 * tiles */);

// Log-ratio pass: L (M x ldl FP32, zero past column N up to npad) = l,
// per-block FP64 column sums (logratio_blocks(M) x npad) and clamp count.
int64_t logratio_blocks(int64_t M);
hipError_t launch_logratio(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor, float* L,
                           int64_t ldl, int npad, double* colsum_part, unsigned long long* clamps, hipStream_t s);
// FP64 Gram partials of L per chunk of rows (npad must cover plan.nb * 128
// columns), and their sum in chunk order into G (N x N FP64, both triangles).
// fp64: products and sums in FP64 (v_mfma_f64_16x16x4f64).
hipError_t launch_gram(const float* L, int64_t ldl, int64_t M, const GramPlan& plan, const int* d_tiles,
                       double* partial, hipStream_t s, bool fp64 = false);
hipError_t launch_gram_reduce(const double* partial, const GramPlan& plan, const int* d_tiles, int N, double* G,
                              hipStream_t s);
// The same kernels for the product of two tall matrices, L^T R: tile
// (bi, bj) of d_tiles pairs columns 128 bi.. of L with columns 128 bj.. of R
// (both padded with readable columns up to the tile edges); plan.tiles is
// the number of listed tiles.  The rect reduction writes the rows x cols
// block of out (row 128 bi + r, column 128 bj + c) without symmetrising.
hipError_t launch_gram_pair(const float* L, int64_t ldl, const float* R, int64_t ldr, int64_t M,
                            const GramPlan& plan, const int* d_tiles, double* partial, hipStream_t s, bool fp64);
hipError_t launch_gram_reduce_rect(const double* partial, const GramPlan& plan, const int* d_tiles, int rows,
                                   int cols, double* out, int64_t ld_out, hipStream_t s);
size_t colsum_scratch_doubles(int N);
hipError_t launch_colsum_reduce(const double* part, int64_t nparts, int stride, int N, double* mid, double* out,
                                hipStream_t s);

// Projection Z = l W (W given transposed: Wt is kp x ldw, zero beyond k / N),
// with per-block column arg-extrema partials when part != nullptr.
struct ArgPart {
    float* maxv;
    float* minv;
    long long* maxi;
    long long* mini;
};
constexpr int kProjRows = 128;
inline int64_t proj_blocks(int64_t M) { return (M + kProjRows - 1) / kProjRows; }
hipError_t launch_project(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                          const float* Wt, int ldw, int kp, int k_store, float* Z, int64_t ld_z,
                          ArgPart part, int k_arg, hipStream_t s, bool logged = false);
// Basis residual (retraining criterion, Sec. 5).  With A = l diag(f), the
// sums ||A_m||^2 and ||A_m V||^2 of each spectrum (the projection on Wt with
// g[c] = 1 / shrink_c, kp entries, zero past k, so that Z_c g_c = (A V)_c).
// f: N floats.  launch_residual_partials: their FP64 sums per block of
// kProjRows spectra into part[2 b], part[2 b + 1] (proj_blocks(M) pairs);
// launch_residual_total: the sum of nparts pairs in a fixed order into
// out[0..1]; launch_segment_sums: the FP64 sums over the rows offs[s] ..
// offs[s+1]-1 of a per-spectrum norms array (2 floats per row) into
// out[2 s..2 s+1].
hipError_t launch_residual_partials(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                                    const float* Wt, int ldw, int kp, const float* f, const float* g, double* part,
                                    hipStream_t s);
hipError_t launch_residual_total(const double* part, int64_t nparts, double* out, hipStream_t s);
hipError_t launch_segment_sums(const float* norms, const long long* offs, int nseg, double* out, hipStream_t s);
// Optional per-spectrum residual sums of the fused transforms: norms[2 m],
// norms[2 m + 1] = ||A_m||^2, ||A_m V||^2 (FP32) when norms != nullptr.
struct ResidualArgs {
    const float* f = nullptr;  // N
    const float* g = nullptr;  // 128, 1 / shrink, zero past k
    float* norms = nullptr;    // M x 2
};
hipError_t launch_argext_reduce(ArgPart part, int64_t nblocks, int kp, int k, long long* qmax,
                                long long* qmin, hipStream_t s);
// Sub-sample between the extrema (Sec. 2.3): for each of the k columns of Z
// (M rows, stride ld_z, kp in {16, 32, 64, 128} columns stored) and each of
// s levels evenly spaced strictly between Z[qmin[c], c] and Z[qmax[c], c]
// (device), the row nearest to the level (first on ties) into q[c s + j - 1]
// (device, -1 when the column has no extrema).  pval / pidx: scratch of
// between_blocks(M, kp) * k * s entries each.
int64_t between_blocks(int64_t M, int kp);
hipError_t launch_between(const float* Z, int64_t M, int64_t ld_z, int kp, int k, int s, const long long* qmax,
                          const long long* qmin, float* pval, long long* pidx, long long* q, hipStream_t st);

// Reconstruction: out = plane of exp(Z B_re) exp(i Z B_im); BreT / BimT are
// (rows = wavenumbers) x kp with the vectors in kgroup_pos order.
hipError_t launch_reconstruct(const float* Z, int64_t M, int64_t ld_z, int k, const float* BreT,
                              const float* BimT, int kp, int N, float* out, int64_t ld_out, int plane,
                              hipStream_t s);

// Fused stored-basis transform: projection onto Wt then reconstruction.
// B^T (FP32) holds the basis vectors of each group of 16 in the order
// 0,4,8,12,1,5,9,13,2,... (kgroup_pos); Z and W keep the natural order.
inline int kgroup_pos(int c) { return (c & ~15) + 4 * (c & 3) + ((c & 15) >> 2); }
hipError_t launch_transform(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                            const float* Wt, int ldw, int kp, int k, const float* BreT, const float* BimT,
                            float* out, int64_t ld_out, int plane, hipStream_t s,
                            const ResidualArgs& res = ResidualArgs{});

// ---- BF16 operands, FP32 accumulation -------------------------------------
// BF16 arrays are passed as uint16_t (bit patterns).  kq = padded k of the
// BF16 basis copies: 32, 64 or 128.

// Log ratio rounded to BF16 in row-group-packed order (8 rows of one column
// per 16-byte unit, logratio16_bytes(M, npad) bytes), with the column-sum
// partials and clamp count of launch_logratio.
size_t logratio16_bytes(int64_t M, int npad);
hipError_t launch_logratio16(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                             uint16_t* Lp, int npad, double* colsum_part, unsigned long long* clamps,
                             hipStream_t s);
// Gram partials from the packed log ratio (plan from gram_plan(.., 64)).
hipError_t launch_gram16(const uint16_t* Lp, int npad, int64_t M, const GramPlan& plan, const int* d_tiles,
                         double* partial, hipStream_t s);
// Projection from I (log ratio on load), Wt: kq x ldw BF16.  pieces 3: Wt
// holds three BF16 piece planes of W^T (kq x ldw each, consecutive), the log
// ratio is cut into three pieces as well, and Z has FP32 accuracy.
hipError_t launch_project16(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                            const uint16_t* Wt, int ldw, int kq, int k_store, float* Z, int64_t ld_z,
                            ArgPart part, int k_arg, hipStream_t s, int pieces = 1);
// Reconstruction from FP32 Z; BreT / BimT: npad x kq BF16 (npad >= N rows,
// zero past N; the basis keeps N rounded up to 64), read at rows below
// npad only.  pieces = 3: FP32 accuracy on the BF16 matrix cores, BreT /
// BimT then three consecutive npad x kq planes (the BF16 pieces of B) each.
hipError_t launch_reconstruct16(const float* Z, int64_t M, int64_t ld_z, int k, const uint16_t* BreT,
                                const uint16_t* BimT, int kq, int N, int npad, float* out, int64_t ld_out,
                                int plane, hipStream_t s, int pieces = 1);
hipError_t launch_transform16(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor,
                              const uint16_t* Wt, int ldw, int kq, const uint16_t* BreT, const uint16_t* BimT,
                              float* out, int64_t ld_out, int plane, hipStream_t s,
                              const ResidualArgs& res = ResidualArgs{});

// ---- Gram to FP64 accuracy on the int8 matrix cores (error-free splitting)
// stats: FP64 column sums of I (stats_blocks(M) x npad partials, reduced by
// launch_colsum_reduce), the clamp count, per-block max |l| (colmax_part,
// stats_colmax_floats(M, npad) floats) and the column exponents colexp (npad ints).
int64_t stats_blocks(int64_t M);
size_t stats_colmax_floats(int64_t M, int npad);  // colmax_part: partials and group maxima
hipError_t launch_split_stats(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor, int npad,
                              double* colsum_part, float* colmax_part, unsigned long long* clamps, int* colexp,
                              hipStream_t s);
// exponents from the maxima of every stride-th row with one bit of headroom
// (colmax_part as for the stats, at least stats_colmax_floats(M, npad)).
hipError_t launch_split_sample(const float* I, int64_t M, int N, int64_t ld, const float* rinv, float floor, int npad,
                               int stride, float* colmax_part, int* colexp, hipStream_t s);
// slices of the FP64 log ratio (rinv64: 1/I_ref, N doubles) into S,
// split_bytes(M, npad) bytes (rows padded to a multiple of 64 with zeros),
// with the FP64 column-sum partials (stats layout) and flags[0] += clamped
// ratios, flags[1] set when a row does not fit its column's exponent.
size_t split_bytes(int64_t M, int npad);
hipError_t launch_split_slices(const float* I, int64_t M, int N, int64_t ld, const double* rinv64, double floor,
                               const int* colexp, int npad, void* S, double* colsum_part,
                               unsigned long long* flags, hipStream_t s);
// chunk partials of the Gram from the slices (plan from split_gram_plan),
// reduced by launch_gram_reduce.
GramPlan split_gram_plan(int64_t M, int N);
hipError_t launch_gram_split(const void* S, int npad, int64_t M, const GramPlan& plan, const int* d_tiles,
                             const int* colexp, double* partial, hipStream_t s);

// Gather rows q of a row-major FP32 matrix Z (k columns, row stride ld_z)
// into X (n_q x k).
hipError_t launch_gather_rows(const float* Z, int64_t ld_z, int k, const long long* q, int n_q, float* X,
                              hipStream_t s);

}  // namespace dev
}  // namespace fkk
