// Device Householder tridiagonalisation of a symmetric FP64 matrix.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fkk {
namespace dev {

// Packed reflector storage for an n x n reduction (column i: n - i - 1 values).
size_t tridiag_vstore_doubles(int n);

// Sets the kernels' dynamic LDS size for order n (call before
// launch_tridiag, outside any stream capture).
hipError_t tridiag_prepare(int n);

// A (n x n row-major FP64, symmetric, overwritten) -> tridiagonal (d: n,
// e: n-1), reflectors (vstore, beta: n-2).  p0, p1: n doubles of scratch.
// Kernel launches only (n - 1 of them), so the sequence can be recorded
// into a graph.
hipError_t launch_tridiag(double* A, int n, double* p0, double* p1, double* vstore, double* beta, double* d, double* e,
                          hipStream_t s);

// Whole reduction in one cooperative launch of G blocks (each keeps its rows
// in LDS).  tridiag_resident_grid returns G for order n on `device`, or 0
// when the device cannot run it (no cooperative launch, rows do not fit).
// A is read only.  xch: tridiag_resident_xch_doubles(n) doubles of scratch
// and *err, all zero before the launch; *err != 0 afterwards means a wait
// for exchanged data gave up after spin_limit polls (0: at the first wait)
// and the outputs are invalid.
int tridiag_resident_grid(int n, int device);
size_t tridiag_resident_xch_doubles(int n);
hipError_t launch_tridiag_resident(const double* A, int n, int G, double* xch, int* err, double* vstore,
                                   double* beta, double* d, double* e, int spin_limit, hipStream_t s);

// x = Q y for k eigenvectors y of T (vector j at Y + j n) with the
// reflectors of either reduction above (beta on the device, n - 2 values;
// vstore packed), then the sign rule (largest-magnitude entry positive,
// first on ties) into vecs (n x k row-major).  n <= back_transform_max_n().
// vpad: back_transform_vpad_doubles(n) doubles of scratch (the reflectors
// as zero-padded rows in whole blocks of 16, then the blocks' T factors of
// the compact WY form).
int back_transform_max_n();
size_t back_transform_vpad_doubles(int n);
hipError_t launch_back_transform(const double* beta, const double* vstore, int n, int k, const double* Y,
                                 double* vecs, double* vpad, hipStream_t s);

// G(r, c) *= f(r) f(c).
hipError_t launch_scale_sym(double* G, const double* f, int n, hipStream_t s);

}  // namespace dev
}  // namespace fkk
