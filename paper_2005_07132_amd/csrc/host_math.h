// FP64 host-side numerics of fKK-EC that act on the k basis vectors or on
// the N x N Gram matrix (never on the M spectra): FFT-based Hilbert
// transform, ALS / Whittaker detrending, Savitzky-Golay trendline, ridge
// regression through a one-sided Jacobi SVD, and a top-k symmetric
// eigensolver.  Plain C++ (no HIP), so it can be built and checked on any
// host.
#pragma once

#include <cstdint>
#include <functional>
#include <vector>

namespace fkk {

// Runs body(r0, r1) over a split of the rows [0, rows) on the library's
// host thread pool (one call on the caller's thread when there is one).
void parallel_rows(int rows, const std::function<void(int, int)>& body);

// Discrete Hilbert transform of each of `rows` rows of x (rows x n,
// row-major) into y: centred padding to `len` points (edge replication or
// zeros), multiplication of DFT bin nu by -i sgn(nu) (0 at DC and Nyquist),
// inverse DFT, real part, crop.  len must be a power of two >= n.
void hilbert_rows(const double* x, double* y, int rows, int n, int len, int pad_mode);

// Baseline by asymmetric least squares: n_iter solves of
// (diag(w) + lam D^T D) z = w * y, weights p above the baseline, 1 - p
// elsewhere, starting from w = 1.  detrend == 1 (Whittaker) is one solve
// with w = 1.
void detrend_row(const double* y, double* z, int n, int mode, double lam, double p, int n_iter);
void detrend_rows(const double* y, double* z, int rows, int n, int mode, double lam, double p, int n_iter);

// Trendline of each row: Savitzky-Golay (window, order) with least-squares
// polynomial fits on the first / last window near the ends, or the mean.
void trendline_rows(const double* x, double* y, int rows, int n, int mode, int window, int order);

// Ridge regression B = (X^T X + lam I)^-1 X^T Y (X: m x k, Y: m x n,
// B: k x n) with lam = rel * sigma_max(X)^2; rel = 0 gives the minimum-norm
// least-squares solution.  Returns lam.  X = 0 gives B = 0.
double ridge_rel_solve(const double* X, const double* Y, double* B, int m, int k, int n, double rel);

// Top-k eigenpairs of the symmetric n x n matrix a (row-major): values in
// descending order, vectors as the columns of vecs (n x k row-major), each
// with its largest-magnitude entry positive.  Uses `threads` host threads.
// Returns 0 on success.
int eigh_topk(const double* a, int n, int k, double* vals, double* vecs, int threads);

// The same from an existing Householder tridiagonalisation: diagonal d (n),
// off-diagonal e (n-1), reflectors beta (n-2) and vstore (column i packed at
// sum_{j<i} (n-j-1), length n-i-1), with A = Q T Q^T, Q = H_0 ... H_{n-3},
// H_i = I - beta_i v_i v_i^T acting on indices i+1..n-1.
int eig_tridiag_topk(const double* d, const double* e, const double* beta, const double* vstore, int n, int k,
                     double* vals, double* vecs);
// Its two halves: the top-k eigenpairs of T (values descending, vector j of
// T at Y + j n), which need only d and e; then x = Q y for each vector, the
// sign rule, and the transpose into vecs (n x k).  Y has room for k rounded
// up to a multiple of 4 vectors, the ones past k zero.  With rel_cut > 0
// only the pairs whose sqrt(max(value, 0)) exceeds rel_cut times that of
// the largest (at least one) get vectors; *k_out (when given) receives
// their count, and values past it are left as bisected.
int tridiag_eigvecs(const double* d, const double* e, int n, int k, double* vals, double* Y, double rel_cut = 0.0,
                    int* k_out = nullptr);
void tridiag_back_transform(const double* beta, const double* vstore, int n, int k, double* Y, double* vecs);

// Small dense FP64 kernels of the randomized range finder (X: n x l
// row-major, l small): G = X^T X (both triangles; per-thread partial sums
// added in thread order); in place upper-triangular R with G = R^T R (false
// if G is not positive definite); X <- X R^-1; an orthonormal basis of the
// columns of X in place by Cholesky QR applied twice (false on breakdown).
void gram_cols(const double* X, int n, int l, double* G);
bool cholesky_upper(double* G, int l);
void solve_right_upper(double* X, int n, int l, const double* R);
bool orthonormalize_cols(double* X, int n, int l);

// Default readings of parameters the paper leaves open.
int default_fft_len(int n);
double default_als_lambda(int n);
int default_sg_window(int n);

}  // namespace fkk
