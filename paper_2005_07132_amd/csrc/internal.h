// Library-internal definitions shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <vector>

#include "fkkec.h"

// A basis set: FP64 host copies (the stored model of ML:fKK-EC) and the
// device arrays the transform kernels read.
struct fkk_basis {
    int device = -1;
    int N = 0, k = 0, kp = 0, npad = 0;
    int kq = 0;                 // k padded for the BF16 copies: 32, 64 or 128
    int prec = FKK_PREC_FP32;   // precision of transforms with this basis
    std::vector<double> i_ref, f, s, v, b_re, b_im, phi_pec_t, v_sec_t, h_v;
    std::vector<int64_t> q;
    double ml_lambda = 0.0, ratio_floor = 1e-6, ridge_lambda = 0.0;
    mutable std::atomic<int> holders{0}; // servers holding the basis (fkk_basis_free: FKK_EBUSY)
    void* d_arena = nullptr;     // one allocation holding the arrays below
    float* d_rinv = nullptr;     // 2N: 1/I_ref as hi, lo floats
    float* d_wt = nullptr;       // kp x npad: f(j) V(j,c) shrink(c)
    float* d_bre_t = nullptr;    // npad x kp, vectors in group order
    float* d_bim_t = nullptr;    // npad x kp
    uint16_t* d_wt16 = nullptr;  // kq x npad, BF16 of d_wt
    uint16_t* d_bre16 = nullptr; // npad x kq, BF16, natural order
    uint16_t* d_bim16 = nullptr; // npad x kq
    float* d_f = nullptr;        // npad: f of the training data (residual sums)
    float* d_g = nullptr;        // 128: 1 / shrink of each vector, zero past k
    ~fkk_basis() {
        if (d_arena) hipFree(d_arena);
    }
};

