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

// Device scratch of one call, carved from one region: batch x N doubles
// each for the log ratio, the KK phase and the phase error, 4 x batch x N
// for the ALS state, the twiddle table of the FFT length and the trendline
// tables.  Spectra run in batches of `batch` rows.
struct Layout {
    double* ell = nullptr;      // batch x N   log ratio
    double* phi = nullptr;      // batch x N   KK phase, later H{phi_err}
    double* err = nullptr;      // batch x N   phase error phi_err
    double* scratch = nullptr;  // 4 x N x batch, interleaved ALS state
    double* twiddle = nullptr;  // len / 2 complex
    double* sg = nullptr;       // I_ref (N), then the trendline tables (16)
    int64_t batch = 0;
};

// Rows per batch for M spectra when the workspace does not limit it.
int64_t full_batch(int64_t M);
// Bytes of a region for batches of `batch` rows (256-byte aligned parts).
size_t layout_bytes(int N, int len, int64_t batch);
// The largest batch (a multiple of 256 rows, at most full_batch(M)) whose
// layout fits in `bytes`; 0 if not even 256 rows fit.
int64_t batch_for_bytes(int N, int len, int64_t M, size_t bytes);
// Carves the layout for `batch` rows out of `base`.
Layout carve(void* base, int N, int len, int64_t batch);

// Runs the whole conventional workflow for M spectra of d_I (row stride ld;
// FP64 when in_f64, else FP32), writing the selected plane of K_CARS to d_out
// (row stride ld_out; FP64 when out_f64, else FP32).  All arithmetic is FP64.
hipError_t run(const Layout& ws, const Config& cfg, const void* d_I, bool in_f64, int64_t M, int64_t ld,
               const double* h_iref, void* d_out, bool out_f64, int64_t ld_out, hipStream_t s, std::string* why);

}  // namespace plain
}  // namespace fkk
