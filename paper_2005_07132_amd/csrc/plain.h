// Conventional per-spectrum KK -> PEC -> SEC on the device (Eq. 2-5, SEC in
// the log form of Eq. 19), the comparator of the factorised method.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace fkk {
namespace plain {

struct Config {
    int N = 0;
    int len = 0;        // FFT length (power of two >= N)
    int pad_mode = 0;   // 0 edge, 1 zero
    int detrend = 0;    // 0 ALS, 1 Whittaker
    double lam = 0.0;
    double p = 1e-3;
    int iters = 10;
    int sec_mode = 0;   // 0 Savitzky-Golay, 1 mean
    int sec_re = 0;     // SEC form: 0 log magnitude minus its trendline (Eq. 19), 1 divide by the trendline of Re (Eq. 4-5)
    int window = 0;
    int order = 2;
    double floor = 1e-6;
    int plane = 0;      // 0 Im, 1 Re, 2 |K|
};

struct Workspace {
    double* ell = nullptr;     // batch x N   log ratio
    double* phi = nullptr;     // batch x N   KK phase, later H{phi_err}
    double* err = nullptr;     // batch x N   phase error phi_err
    double* scratch = nullptr; // 4 x N x batch, interleaved ALS state
    double* twiddle = nullptr; // len / 2 complex (table of the current length)
    std::vector<std::pair<int, double*>> tw_tables;  // one table per FFT length used
    double* sg = nullptr;      // trendline coefficient tables
    int64_t batch = 0;
    size_t cap_row = 0;        // doubles per batch-sized array (batch x N)
    int n = 0, len = 0, tw_len = 0;
    size_t sg_doubles = 0;
    size_t bytes() const;
    void release();
};

// Runs the whole conventional workflow for M spectra of d_I (row stride ld;
// FP64 when in_f64, else FP32), writing the selected plane of K_CARS to d_out
// (row stride ld_out; FP64 when out_f64, else FP32).  All arithmetic is FP64.
hipError_t run(Workspace& ws, const Config& cfg, const void* d_I, bool in_f64, int64_t M, int64_t ld,
               const double* h_iref, void* d_out, bool out_f64, int64_t ld_out, hipStream_t s, std::string* why);

}  // namespace plain
}  // namespace fkk
