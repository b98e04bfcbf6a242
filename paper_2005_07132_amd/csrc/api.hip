// C ABI of the fKK-EC library (include/fkkec.h): argument checking, device
// workspace, and the orchestration of the fit
//   device: log ratio + Gram  ->  host FP64: eigensolve, fKK / fPEC / fSEC
//   device: projection + arg-extrema  ->  device: reconstruction + epilogue
// and of the stored-basis transform.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cfloat>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fkkec.h"
#include "internal.h"
#include "host_math.h"
#include "eig.h"
#include "kernels.h"
#include "plain.h"

namespace {

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(count, 1) * sizeof(T));
        if (e == hipSuccess) n = std::max<size_t>(count, 1);
        return e;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
    }
};

template <class T>
struct PinnedBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        if (p) hipHostFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p), std::max<size_t>(count, 1) * sizeof(T),
                                     hipHostMallocDefault);
        if (e == hipSuccess) n = std::max<size_t>(count, 1);
        return e;
    }
    void release() {
        if (p) hipHostFree(p);
        p = nullptr;
        n = 0;
    }
};

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

int round_up(int x, int m) { return (x + m - 1) / m * m; }

// 1/I_ref as two floats per wavenumber: hi in out[0..N), lo in out[N..2N).
void split_reciprocal(const double* iref, int N, float* out) {
    for (int j = 0; j < N; ++j) {
        const double r = 1.0 / iref[j];
        out[j] = (float)r;
        out[N + j] = (float)(r - (double)out[j]);
    }
}

// Precisions of projection / reconstruction: FP32, BF16 and SPLIT (FP32
// accuracy on the BF16 matrix cores in the reconstruction; FP32 elsewhere).
bool valid_prec(int p) { return p == FKK_PREC_FP32 || p == FKK_PREC_BF16 || p == FKK_PREC_SPLIT; }
bool valid_gram_prec(int p) { return valid_prec(p) || p == FKK_PREC_FP64; }

// Nearest-even BF16 bit pattern of a finite float.
uint16_t to_bf16(float x) {
    uint32_t u;
    std::memcpy(&u, &x, sizeof u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float from_bf16(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float x;
    std::memcpy(&x, &u, sizeof x);
    return x;
}

int kp_for(int k) {
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    return 128;
}

int host_threads() {
    unsigned hw = std::thread::hardware_concurrency();
    if (hw == 0) hw = 1;
    return (int)std::min(16u, hw);
}

// Consecutive 256-byte aligned parts of one device region.  With a null
// base it only counts bytes: the same code sizes a workspace and lays it out.
struct Carve {
    unsigned char* base;
    size_t off = 0;
    explicit Carve(void* b) : base(static_cast<unsigned char*>(b)) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

}  // namespace

// Fixed device array of fkk_basis_residual_noalloc: the per-block partial
// sums (two doubles per block of 128 spectra) and their total.  Every device
// the library runs on holds its own copy until the process ends.  Host code
// never uses this name as an address: the address on each device comes from
// hipGetSymbolAddress (scratch_address).
constexpr size_t kScratchDoubles = 2 * (size_t)FKK_NOALLOC_MAX_BLOCKS + 2;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Address of `scratch` on `device` (current), looked up once per device.
hipError_t scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[device] = p;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

}  // namespace

struct fkk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // The context's own device workspace, used by calls that get none from
    // the caller (grown on demand, kept until the context is destroyed).
    DevBuf<unsigned char> ws;
    PinnedBuf<double> hG;
    PinnedBuf<double> hstage;  // basis uploads
    hipEvent_t ev[12] = {};  // 0-9 stage timing, 10-11 eigensolve copies
    // The n - 1 launches of the tridiagonalisation, recorded once per order
    // and buffer set on a private stream and replayed on `stream`.
    bool graphs = true;
    // The whole reduction as one cooperative launch when the device and the
    // order allow it (FKK_NO_RESIDENT_TRIDIAG=1 forces the per-column
    // launches); a wait that gives up falls back to the per-column launches.
    bool resident_tri = true;
    int tri_spin_limit = 1 << 22;  // polls of a wait before giving up (FKK_TRIDIAG_SPIN_LIMIT)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t tri_exec = nullptr;
    int tri_n = 0;
    const double* tri_key[2] = {nullptr, nullptr};
    void* scratch = nullptr;  // this device's copy of the library's fixed array

    hipError_t events() {
        for (auto& e : ev)
            if (!e) {
                hipError_t r = hipEventCreate(&e);
                if (r != hipSuccess) return r;
            }
        return hipSuccess;
    }
    float elapsed(int a, int b) const {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[a], ev[b]) != hipSuccess) return -1.f;
        return ms;
    }

    fkk_status fail(fkk_status s, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return s;
    }
    size_t bytes() const { return ws.n; }
};

#define FKK_HIP(ctx, call)                                                                          \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return (ctx)->fail(FKK_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
    } while (0)

namespace {

// Smallest ratio floor: the FP32 kernels take the logarithm of clamped
// ratios as normal numbers (2^-126 and up).
constexpr double kMinRatioFloor = 0x1p-126;

// auto_k: k = 0 (the rank rule of Sec. 4.1) is allowed.
// plain: the conventional method, the only one with the real-part SEC form.
fkk_status check_params(fkk_ctx* ctx, const fkk_params* p, int N, bool auto_k = false, bool plain = false) {
    if (!p) return ctx->fail(FKK_EINVAL, "params is NULL");
    if (p->sec_form != FKK_SEC_FORM_LOG && !(plain && p->sec_form == FKK_SEC_FORM_RE))
        return ctx->fail(FKK_EINVAL, "sec_form=%d (the real-part form is for fkk_plain only)", p->sec_form);
    if (!(auto_k && p->k == 0) && (p->k < 1 || p->k > N))
        return ctx->fail(FKK_EINVAL, "k=%d outside 1..N=%d", p->k, N);
    if (p->k > 128) return ctx->fail(FKK_ERANK, "k=%d above the supported 128", p->k);
    if (p->f_mode != FKK_F_ONE && p->f_mode != FKK_F_NOISE) return ctx->fail(FKK_EINVAL, "bad f_mode");
    if (p->pad_mode != FKK_PAD_EDGE && p->pad_mode != FKK_PAD_ZERO) return ctx->fail(FKK_EINVAL, "bad pad_mode");
    const int len = p->fft_len ? p->fft_len : fkk::default_fft_len(N);
    if (len < N || (len & (len - 1)) != 0)
        return ctx->fail(FKK_EINVAL, "fft_len=%d must be a power of two >= N", p->fft_len);
    if (p->detrend != FKK_DETREND_ALS && p->detrend != FKK_DETREND_WHITTAKER)
        return ctx->fail(FKK_EINVAL, "bad detrend");
    if (!(p->als_lambda >= 0.0) || !(p->als_p > 0.0 && p->als_p < 1.0) || p->als_iters < 1)
        return ctx->fail(FKK_EINVAL, "bad ALS parameters");
    if (!(p->ridge_rel >= 0.0) || !(p->ml_lambda >= 0.0)) return ctx->fail(FKK_EINVAL, "negative ridge weight");
    if (p->sec_mode != FKK_SEC_SAVGOL && p->sec_mode != FKK_SEC_MEAN) return ctx->fail(FKK_EINVAL, "bad sec_mode");
    if (p->sec_mode == FKK_SEC_SAVGOL) {
        const int w = p->sg_window ? p->sg_window : fkk::default_sg_window(N);
        if (w % 2 == 0 || w > N || w <= p->sg_order || p->sg_order < 0)
            return ctx->fail(FKK_EINVAL, "Savitzky-Golay window %d / order %d invalid for N=%d", w, p->sg_order, N);
    }
    if (!(p->ratio_floor >= kMinRatioFloor))
        return ctx->fail(FKK_EINVAL, "ratio_floor must be at least 2^-126 (the smallest normal FP32 number)");
    if (p->output < FKK_OUT_IM || p->output > FKK_OUT_ABS) return ctx->fail(FKK_EINVAL, "bad output plane");
    if (!valid_gram_prec(p->gram_prec) || !valid_prec(p->recon_prec))
        return ctx->fail(FKK_EINVAL, "bad matrix-core precision (gram_prec=%d, recon_prec=%d)", p->gram_prec,
                         p->recon_prec);
    if (p->f_mode == FKK_F_NOISE && !(p->alpha >= 0.0 && p->sigma_g >= 0.0 && (p->alpha > 0.0 || p->sigma_g > 0.0)))
        return ctx->fail(FKK_EINVAL, "f_mode=noise needs alpha >= 0, sigma_g >= 0, not both 0");
    if (p->q_between < 0 || p->q_between > 16) return ctx->fail(FKK_EINVAL, "q_between=%d outside 0..16", p->q_between);
    if (p->svd_mode != FKK_SVD_GRAM && p->svd_mode != FKK_SVD_RANDOMIZED) return ctx->fail(FKK_EINVAL, "bad svd_mode");
    if (p->svd_mode == FKK_SVD_RANDOMIZED) {
        if (p->k == 0) return ctx->fail(FKK_EINVAL, "the randomized SVD needs k >= 1");
        if (p->rrf_oversample < 0 || p->rrf_power_iters < 0 || p->rrf_power_iters > 16)
            return ctx->fail(FKK_EINVAL, "rrf_oversample >= 0 and 0 <= rrf_power_iters <= 16");
        if (p->k + p->rrf_oversample > std::min(N, 128))
            return ctx->fail(FKK_ERANK, "k + rrf_oversample = %d above min(N, 128)", p->k + p->rrf_oversample);
    }
    return FKK_OK;
}

fkk_status check_matrix(fkk_ctx* ctx, const void* d, int64_t M, int N, int64_t ld, const char* what) {
    if (!d) return ctx->fail(FKK_EINVAL, "%s is NULL", what);
    if (M < 1) return ctx->fail(FKK_EINVAL, "%s: M=%lld < 1", what, (long long)M);
    if (N < 4) return ctx->fail(FKK_EINVAL, "%s: N=%d < 4", what, N);
    if (ld < N) return ctx->fail(FKK_EINVAL, "%s: ld=%lld < N=%d", what, (long long)ld, N);
    return FKK_OK;
}

fkk_status check_iref(fkk_ctx* ctx, const double* h_iref, int N) {
    if (!h_iref) return ctx->fail(FKK_EINVAL, "I_ref is NULL");
    for (int j = 0; j < N; ++j)
        if (!(h_iref[j] > 0.0) || !std::isfinite(h_iref[j]))
            return ctx->fail(FKK_EINVAL, "I_ref[%d] must be positive and finite", j);
    return FKK_OK;
}

// Device copies of a basis: 1/I_ref (two floats per wavenumber), the
// projection weights W^T (kp x npad), B_re^T and B_im^T (npad x kp, vectors
// in the kernels' group order) and BF16 copies of the three (natural order,
// k padded to kq).  All live in one device allocation, assembled in the
// context's pinned staging buffer and sent with one copy.
fkk_status upload_basis(fkk_ctx* ctx, fkk_basis* b, double shrink_lambda) {
    const int N = b->N, k = b->k, kp = b->kp, np = b->npad, kq = b->kq;
    auto al = [](size_t bytes) { return (bytes + 255) & ~size_t(255); };
    const size_t o_rinv = 0;
    const size_t o_wt = o_rinv + al(2 * (size_t)N * 4);
    const size_t o_bre = o_wt + al((size_t)kp * np * 4);
    const size_t o_bim = o_bre + al((size_t)np * kp * 4);
    const size_t o_wt16 = o_bim + al((size_t)np * kp * 4);
    const size_t o_bre16 = o_wt16 + al((size_t)kq * np * 2);
    const size_t o_bim16 = o_bre16 + al(3 * (size_t)np * kq * 2);
    const size_t o_f = o_bim16 + al(3 * (size_t)np * kq * 2);
    const size_t o_g = o_f + al((size_t)np * 4);
    const size_t total = o_g + al(128 * 4);
    FKK_HIP(ctx, ctx->hstage.ensure((total + 7) / 8));  // doubles
    unsigned char* h = reinterpret_cast<unsigned char*>(ctx->hstage.p);
    std::memset(h, 0, total);
    float* rinv = reinterpret_cast<float*>(h + o_rinv);
    float* wt = reinterpret_cast<float*>(h + o_wt);
    float* bre = reinterpret_cast<float*>(h + o_bre);
    float* bim = reinterpret_cast<float*>(h + o_bim);
    uint16_t* wt16 = reinterpret_cast<uint16_t*>(h + o_wt16);
    uint16_t* bre16 = reinterpret_cast<uint16_t*>(h + o_bre16);
    uint16_t* bim16 = reinterpret_cast<uint16_t*>(h + o_bim16);
    split_reciprocal(b->i_ref.data(), N, rinv);
    float* fd = reinterpret_cast<float*>(h + o_f);
    float* gd = reinterpret_cast<float*>(h + o_g);
    for (int j = 0; j < N; ++j) fd[j] = (float)b->f[j];
    double smax = 0.0;
    for (int c = 0; c < k; ++c) smax = std::max(smax, b->s[c]);
    // (rows of each array split over the host pool: every element is
    // written by one thread, so the contents do not depend on the split)
    fkk::parallel_rows(k, [&](int c0, int c1) {
        for (int c = c0; c < c1; ++c) {
            double shrink;
            if (shrink_lambda > 0.0) shrink = b->s[c] * b->s[c] / (b->s[c] * b->s[c] + shrink_lambda);
            else shrink = (b->s[c] > 1e-15 * smax) ? 1.0 : 0.0;  // pseudo-inverse of S V^T
            gd[c] = shrink > 0.0 ? (float)(1.0 / shrink) : 0.f;
            for (int j = 0; j < N; ++j) {
                const float w = (float)(b->f[j] * b->v[(size_t)j * k + c] * shrink);
                wt[(size_t)c * np + j] = w;
                wt16[(size_t)c * np + j] = to_bf16(w);
            }
        }
    });
    fkk::parallel_rows(N, [&](int j0, int j1) {
        for (int j = j0; j < j1; ++j)
            for (int c = 0; c < k; ++c) {
                const float re = (float)b->b_re[(size_t)c * N + j], im = (float)b->b_im[(size_t)c * N + j];
                bre[(size_t)j * kp + fkk::dev::kgroup_pos(c)] = re;
                bim[(size_t)j * kp + fkk::dev::kgroup_pos(c)] = im;
                // three BF16 pieces of the FP32 value (planes np kq apart): the
                // first is the BF16 copy, the rest carry the remainders
                float rr = re, ri = im;
                for (int pc = 0; pc < 3; ++pc) {
                    const uint16_t hr = to_bf16(rr), hi = to_bf16(ri);
                    bre16[(size_t)pc * np * kq + (size_t)j * kq + c] = hr;
                    bim16[(size_t)pc * np * kq + (size_t)j * kq + c] = hi;
                    rr -= from_bf16(hr);
                    ri -= from_bf16(hi);
                }
            }
    });
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    if (!b->d_arena) FKK_HIP(ctx, hipMalloc(&b->d_arena, total));
    unsigned char* d = reinterpret_cast<unsigned char*>(b->d_arena);
    FKK_HIP(ctx, hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, ctx->stream));
    FKK_HIP(ctx, hipStreamSynchronize(ctx->stream));  // the staging buffer is reused
    b->d_rinv = reinterpret_cast<float*>(d + o_rinv);
    b->d_wt = reinterpret_cast<float*>(d + o_wt);
    b->d_bre_t = reinterpret_cast<float*>(d + o_bre);
    b->d_bim_t = reinterpret_cast<float*>(d + o_bim);
    b->d_wt16 = reinterpret_cast<uint16_t*>(d + o_wt16);
    b->d_bre16 = reinterpret_cast<uint16_t*>(d + o_bre16);
    b->d_bim16 = reinterpret_cast<uint16_t*>(d + o_bim16);
    b->d_f = reinterpret_cast<float*>(d + o_f);
    b->d_g = reinterpret_cast<float*>(d + o_g);
    b->device = ctx->device;
    return FKK_OK;
}

// fKK on the basis vectors (Eq. 7, 11): H_V = H{V^T / f}, FP64.  Needs only
// V and f, so the fit runs it while the projection is on the device.
void basis_fkk(fkk_basis* b, const fkk_params* p) {
    const int N = b->N, k = b->k;
    const int len = p->fft_len ? p->fft_len : fkk::default_fft_len(N);
    std::vector<double> vt_f((size_t)k * N);
    for (int c = 0; c < k; ++c)
        for (int j = 0; j < N; ++j) vt_f[(size_t)c * N + j] = b->v[(size_t)j * k + c] / b->f[j];
    b->h_v.assign((size_t)k * N, 0.0);
    fkk::hilbert_rows(vt_f.data(), b->h_v.data(), k, N, len, p->pad_mode);
}

// fPEC and fSEC on the basis vectors (Eq. 16-18, 21-23), FP64, after basis_fkk.
void basis_math(fkk_basis* b, const double* X, int n_q, const fkk_params* p) {
    const int N = b->N, k = b->k;
    const int len = p->fft_len ? p->fft_len : fkk::default_fft_len(N);
    const double lam = p->als_lambda > 0.0 ? p->als_lambda : fkk::default_als_lambda(N);
    const int window = p->sg_window ? p->sg_window : fkk::default_sg_window(N);
    std::vector<double> vt_f((size_t)k * N);
    for (int c = 0; c < k; ++c)
        for (int j = 0; j < N; ++j) vt_f[(size_t)c * N + j] = b->v[(size_t)j * k + c] / b->f[j];
    // Phi_raw = X H{V^T/f}; Phi_err = D{Phi_raw} row by row
    std::vector<double> raw((size_t)n_q * N, 0.0), err((size_t)n_q * N);
    fkk::parallel_rows(n_q, [&](int r0, int r1) {
        for (int r = r0; r < r1; ++r)
            for (int c = 0; c < k; ++c) {
                const double x = X[(size_t)r * k + c];
                const double* hv = &b->h_v[(size_t)c * N];
                double* dst = &raw[(size_t)r * N];
                for (int j = 0; j < N; ++j) dst[j] += x * hv[j];
            }
    });
    fkk::detrend_rows(raw.data(), err.data(), n_q, N, p->detrend, lam, p->als_p, p->als_iters);
    b->phi_pec_t.assign((size_t)k * N, 0.0);
    b->ridge_lambda = fkk::ridge_rel_solve(X, err.data(), b->phi_pec_t.data(), n_q, k, N, p->ridge_rel);
    std::vector<double> h_phi((size_t)k * N), t((size_t)k * N);
    fkk::hilbert_rows(b->phi_pec_t.data(), h_phi.data(), k, N, len, p->pad_mode);
    for (size_t i = 0; i < t.size(); ++i) t[i] = vt_f[i] + h_phi[i];
    b->v_sec_t.assign((size_t)k * N, 0.0);
    fkk::trendline_rows(t.data(), b->v_sec_t.data(), k, N, p->sec_mode, window, p->sg_order);
    b->b_re.resize((size_t)k * N);
    b->b_im.resize((size_t)k * N);
    for (size_t i = 0; i < t.size(); ++i) {
        b->b_re[i] = t[i] - b->v_sec_t[i];
        b->b_im[i] = b->h_v[i] - b->phi_pec_t[i];
    }
}

fkk_basis* new_basis(int N, int k, const double* iref, const double* f, const double* s, const double* v,
                     double ml_lambda, double floor) {
    fkk_basis* b = new fkk_basis;
    b->N = N;
    b->k = k;
    b->kp = kp_for(k);
    b->kq = std::max(b->kp, 32);
    b->npad = round_up(N, 64);
    b->i_ref.assign(iref, iref + N);
    b->f.assign(f, f + N);
    b->s.assign(s, s + k);
    b->v.assign(v, v + (size_t)N * k);
    b->ml_lambda = ml_lambda;
    b->ratio_floor = floor;
    return b;
}

int npad_for(int N) { return round_up(N, fkk::dev::kGramTile); }

// Rows between the sampled rows of the split Gram's column exponents.
constexpr int kSplitSampleStride = 16;

// ---- device workspace layouts ------------------------------------------------

// Log ratio, Gram and column sums (Eq. 2, 6, 9).  with_gram false: the
// log-ratio pass and column sums only; rrf: the range finder's products
// (l^T Y, N x 128, and Y^T Y, 128 x 128) in place of the Gram.
struct GramWs {
    float* L = nullptr;                  // M x npad FP32 l, or the packed BF16 l
    double* partial = nullptr;           // FP64 chunk partials of the tiles
    double* G = nullptr;                 // N x N FP64 (rrf: npad x 128 + 128 x 128)
    double* colsum_part = nullptr;       // per-block column sums
    double* colsum = nullptr;            // N sums + reduction scratch
    unsigned long long* clamps = nullptr;  // [0] clamp count, [1] split-slice overflow flag
    int* tiles = nullptr;                // tile pairs
    float* rinv = nullptr;               // 1/I_ref as two floats per wavenumber
    // FKK_PREC_SPLIT only (L then holds the int8 slices)
    float* colmax = nullptr;             // per-block max |l|
    int* colexp = nullptr;               // column exponents (npad)
    double* rinv64 = nullptr;            // 1/I_ref (N)
};

void gram_layout(Carve& c, int64_t M, int N, int prec, bool with_gram, bool rrf, GramWs* w) {
    const int npad = npad_for(N), nb = npad / fkk::dev::kGramTile;
    const bool bf16 = (prec == FKK_PREC_BF16), split = (prec == FKK_PREC_SPLIT);
    const fkk::dev::GramPlan plan =
        split ? fkk::dev::split_gram_plan(M, N) : fkk::dev::gram_plan(M, N, 64, bf16 ? 64 : 32);
    const fkk::dev::GramPlan pr = fkk::dev::gram_plan(M, N, 64, 32);
    w->L = c.take<float>(bf16    ? (fkk::dev::logratio16_bytes(M, npad) + 3) / 4
                         : split ? fkk::dev::split_bytes(M, npad) / 4
                                 : (size_t)M * npad);
    size_t part = 0, g = 0, tiles = 0;
    if (with_gram) {
        part = plan.partial_doubles();
        g = (size_t)N * N;
        tiles = 2 * (size_t)plan.tiles;
    } else if (rrf) {
        part = (size_t)pr.chunks * nb * fkk::dev::kGramTile * fkk::dev::kGramTile;
        g = (size_t)npad * fkk::dev::kGramTile + (size_t)fkk::dev::kGramTile * fkk::dev::kGramTile;
        tiles = 2 * (size_t)(nb + 1);
    }
    w->partial = c.take<double>(part);
    w->G = c.take<double>(g);
    w->colsum_part = c.take<double>((size_t)fkk::dev::logratio_blocks(M) * npad);
    w->colsum = c.take<double>(N + fkk::dev::colsum_scratch_doubles(N));
    w->clamps = c.take<unsigned long long>(2);
    w->tiles = c.take<int>(tiles);
    w->rinv = c.take<float>(2 * (size_t)N);
    if (split) {
        w->colmax = c.take<float>(fkk::dev::stats_colmax_floats(M, npad));
        w->colexp = c.take<int>(npad);
        w->rinv64 = c.take<double>(N);
    }
}

// Everything fkk_fit uses on the device, in one region.
struct FitWs {
    GramWs g;
    double* tri = nullptr;    // p0 | p1 | beta | d | e | reflectors | flags (2) | exchange
    double* fdev = nullptr;   // f (N)
    double* eigv = nullptr;   // Y, x = Q y and the expanded reflectors
    float* Z = nullptr;       // M x kp (range finder: M x 128)
    float* X = nullptr;       // projection weights kp x npad (range finder: 128 x npad)
    float* pmaxv = nullptr;
    float* pminv = nullptr;
    long long* pmaxi = nullptr;
    long long* pmini = nullptr;
    long long* qext = nullptr;
    long long* qdev = nullptr;
    float* bval = nullptr;
    long long* bidx = nullptr;
    long long* qbet = nullptr;
    float* rows = nullptr;    // the sub-sampled input rows, n_q x N
};

// Parameters are assumed valid (check_params).  The layout depends only on
// the sizes and the parameters, never on the device.
size_t fit_layout(void* base, int64_t M, int N, const fkk_params* p, FitWs* w) {
    Carve c(base);
    const bool rrf = (p->svd_mode == FKK_SVD_RANDOMIZED);
    const int gprec = rrf ? FKK_PREC_FP32 : p->gram_prec;
    gram_layout(c, M, N, gprec, !rrf, rrf, &w->g);
    const int npad = npad_for(N);
    const int kcap = p->k > 0 ? p->k : std::min(N, 128);
    const int kp = kp_for(kcap), kq = std::max(kp, 32);
    constexpr int LY = fkk::dev::kGramTile;
    if (!rrf) {
        const size_t nv = fkk::dev::tridiag_vstore_doubles(N), nx = fkk::dev::tridiag_resident_xch_doubles(N);
        w->tri = c.take<double>(5 * (size_t)N + nv + 2 + nx);
        w->eigv = c.take<double>(N <= fkk::dev::back_transform_max_n()
                                     ? 2 * (size_t)N * kcap + fkk::dev::back_transform_vpad_doubles(N)
                                     : 0);
    }
    w->fdev = c.take<double>(N);
    w->Z = c.take<float>((size_t)M * (rrf ? std::max(kp, LY) : kp));
    // the projection weights: kp x npad FP32, kq x npad BF16, or three BF16
    // piece planes (recon_prec FKK_PREC_SPLIT)
    w->X = c.take<float>((size_t)std::max(rrf ? std::max(kp, LY) : kp, (3 * kq + 1) / 2) * npad);
    const int ka = (p->recon_prec == FKK_PREC_BF16 || p->recon_prec == FKK_PREC_SPLIT) ? kq : kp;
    const size_t nblk = (size_t)fkk::dev::proj_blocks(M);
    w->pmaxv = c.take<float>(nblk * ka);
    w->pminv = c.take<float>(nblk * ka);
    w->pmaxi = c.take<long long>(nblk * ka);
    w->pmini = c.take<long long>(nblk * ka);
    w->qext = c.take<long long>(2 * (size_t)ka);
    const bool ovr = p->n_q_override > 0;
    const size_t nq = ovr ? (size_t)p->n_q_override : (size_t)kcap * (2 + p->q_between);
    const size_t nbet = ovr ? 0 : (size_t)kcap * p->q_between;
    const size_t np = nbet ? (size_t)fkk::dev::between_blocks(M, kp) * nbet : 0;
    w->qdev = c.take<long long>(nq);
    w->bval = c.take<float>(np);
    w->bidx = c.take<long long>(np);
    w->qbet = c.take<long long>(nbet);
    w->rows = c.take<float>(nq * N);
    return c.bytes();
}

size_t plain_layout_bytes(int64_t M, int N, const fkk_params* p) {
    const int len = p->fft_len ? p->fft_len : fkk::default_fft_len(N);
    return fkk::plain::layout_bytes(N, len, fkk::plain::full_batch(M));
}

// The region a call works in: the caller's (d_ws, at least `need` bytes,
// 256-byte aligned), or the context's own, grown to `need`.
fkk_status acquire_ws(fkk_ctx* ctx, void* d_ws, size_t ws_bytes, size_t need, void** out) {
    if (d_ws) {
        if (reinterpret_cast<uintptr_t>(d_ws) & 255)
            return ctx->fail(FKK_EINVAL, "workspace must be 256-byte aligned");
        if (ws_bytes < need)
            return ctx->fail(FKK_EINVAL, "workspace of %zu bytes, %zu needed", ws_bytes, need);
        *out = d_ws;
        return FKK_OK;
    }
    if (ws_bytes != 0) return ctx->fail(FKK_EINVAL, "ws_bytes without a workspace");
    FKK_HIP(ctx, ctx->ws.ensure(need));
    *out = ctx->ws.p;
    return FKK_OK;
}

// Log-ratio pass into w.L, Gram G_L = l^T l into w.G (device, FP64, N x N),
// column sums into w.colsum and the clamp count into w.clamps.
// with_gram false: the log-ratio pass and column sums only (FP32 l).
// Split Gram: exact_exp false takes the column exponents from a sample of
// the rows (one bit of headroom); gram_with_sums redoes the pass with exact
// ones when a row did not fit.
fkk_status gram_device(fkk_ctx* ctx, const GramWs& w, const float* d_I, int64_t M, int N, int64_t ld,
                       const double* h_iref, double floor, int prec, bool timed, bool with_gram = true,
                       bool exact_exp = false) {
    const int npad = npad_for(N);
    const bool bf16 = (prec == FKK_PREC_BF16), split = (prec == FKK_PREC_SPLIT) && with_gram;
    const fkk::dev::GramPlan plan =
        split ? fkk::dev::split_gram_plan(M, N) : fkk::dev::gram_plan(M, N, 64, bf16 ? 64 : 32);
    std::vector<int> pairs(2 * plan.tiles);
    fkk::dev::gram_tile_list(plan.nb, pairs.data());
    std::vector<float> rinv(2 * (size_t)N);
    split_reciprocal(h_iref, N, rinv.data());
    const int64_t nlr = fkk::dev::logratio_blocks(M);
    hipStream_t s = ctx->stream;
    if (with_gram)
        FKK_HIP(ctx, hipMemcpyAsync(w.tiles, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, s));
    FKK_HIP(ctx, hipMemcpyAsync(w.rinv, rinv.data(), rinv.size() * sizeof(float), hipMemcpyHostToDevice, s));
    FKK_HIP(ctx, hipMemsetAsync(w.clamps, 0, 2 * sizeof(unsigned long long), s));
    if (split) {
        // column statistics, exponents and the int8 slices of the FP64 log
        // ratio; then the Gram on the int8 matrix cores
        std::vector<double> r64(N);
        for (int j = 0; j < N; ++j) r64[j] = 1.0 / h_iref[j];
        FKK_HIP(ctx, hipMemcpyAsync(w.rinv64, r64.data(), N * sizeof(double), hipMemcpyHostToDevice, s));
        const int64_t nst = fkk::dev::stats_blocks(M);
        if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[8], s));
        if (exact_exp) {
            // the statistics pass's sums and clamp count are recomputed by
            // the slicing pass
            FKK_HIP(ctx, fkk::dev::launch_split_stats(d_I, M, N, ld, w.rinv, (float)floor, npad, w.colsum_part,
                                                      w.colmax, w.clamps, w.colexp, s));
            FKK_HIP(ctx, hipMemsetAsync(w.clamps, 0, 2 * sizeof(unsigned long long), s));
        } else {
            FKK_HIP(ctx, fkk::dev::launch_split_sample(d_I, M, N, ld, w.rinv, (float)floor, npad, kSplitSampleStride,
                                                       w.colmax, w.colexp, s));
        }
        FKK_HIP(ctx, fkk::dev::launch_split_slices(d_I, M, N, ld, w.rinv64, floor, w.colexp, npad, w.L,
                                                   w.colsum_part, w.clamps, s));
        if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[9], s));
        if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[0], s));
        FKK_HIP(ctx, fkk::dev::launch_gram_split(w.L, npad, M, plan, w.tiles, w.colexp, w.partial, s));
        if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[1], s));
        FKK_HIP(ctx, fkk::dev::launch_gram_reduce(w.partial, plan, w.tiles, N, w.G, s));
        FKK_HIP(ctx, fkk::dev::launch_colsum_reduce(w.colsum_part, nst, npad, N, w.colsum + N, w.colsum, s));
        return FKK_OK;
    }
    if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[8], s));
    uint16_t* lp16 = reinterpret_cast<uint16_t*>(w.L);
    if (bf16)
        FKK_HIP(ctx, fkk::dev::launch_logratio16(d_I, M, N, ld, w.rinv, (float)floor, lp16, npad, w.colsum_part,
                                                 w.clamps, s));
    else
        FKK_HIP(ctx, fkk::dev::launch_logratio(d_I, M, N, ld, w.rinv, (float)floor, w.L, npad, npad, w.colsum_part,
                                               w.clamps, s));
    if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[9], s));
    if (!with_gram) {
        FKK_HIP(ctx, fkk::dev::launch_colsum_reduce(w.colsum_part, nlr, npad, N, w.colsum + N, w.colsum, s));
        return FKK_OK;
    }
    if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[0], s));
    if (bf16)
        FKK_HIP(ctx, fkk::dev::launch_gram16(lp16, npad, M, plan, w.tiles, w.partial, s));
    else
        FKK_HIP(ctx, fkk::dev::launch_gram(w.L, npad, M, plan, w.tiles, w.partial, s, prec == FKK_PREC_FP64));
    if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[1], s));
    FKK_HIP(ctx, fkk::dev::launch_gram_reduce(w.partial, plan, w.tiles, N, w.G, s));
    FKK_HIP(ctx, fkk::dev::launch_colsum_reduce(w.colsum_part, nlr, npad, N, w.colsum + N, w.colsum, s));
    return FKK_OK;
}

// Column sums and clamp count back to the host (synchronises the stream);
// *overflow: the split slicing pass found a row past its column exponent.
fkk_status fetch_sums(fkk_ctx* ctx, const GramWs& w, int N, double* h_colsum, int64_t* h_clamps,
                      bool* overflow = nullptr) {
    FKK_HIP(ctx, ctx->hG.ensure((size_t)N + 2));
    hipStream_t s = ctx->stream;
    double* hg = ctx->hG.p;
    FKK_HIP(ctx, hipMemcpyAsync(hg, w.colsum, N * sizeof(double), hipMemcpyDeviceToHost, s));
    FKK_HIP(ctx, hipMemcpyAsync(hg + N, w.clamps, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    FKK_HIP(ctx, hipStreamSynchronize(s));
    std::memcpy(h_colsum, hg, N * sizeof(double));
    unsigned long long c[2];
    std::memcpy(c, hg + N, sizeof c);
    *h_clamps = (int64_t)c[0];
    if (overflow) *overflow = c[1] != 0;
    return FKK_OK;
}

// gram_device and fetch_sums; for the split Gram, once more with exact column
// exponents when the sampled ones were too small for some row.
fkk_status gram_with_sums(fkk_ctx* ctx, const GramWs& w, const float* d_I, int64_t M, int N, int64_t ld,
                          const double* h_iref, double floor, int prec, bool timed, bool with_gram, double* h_colsum,
                          int64_t* h_clamps, bool* redone = nullptr) {
    fkk_status st = gram_device(ctx, w, d_I, M, N, ld, h_iref, floor, prec, timed, with_gram, false);
    bool ovf = false;
    if (st == FKK_OK) st = fetch_sums(ctx, w, N, h_colsum, h_clamps, &ovf);
    if (redone) *redone = false;
    if (st != FKK_OK || !ovf || prec != FKK_PREC_SPLIT || !with_gram) return st;
    if (redone) *redone = true;
    st = gram_device(ctx, w, d_I, M, N, ld, h_iref, floor, prec, timed, with_gram, true);
    if (st == FKK_OK) st = fetch_sums(ctx, w, N, h_colsum, h_clamps, &ovf);
    if (st == FKK_OK && ovf) return ctx->fail(FKK_EINTERNAL, "split Gram: a row exceeds its exact column exponent");
    return st;
}

// Host end of the eigensolve once the reduction is queued on s: the small
// arrays (beta | d | e, and the exchange error flag when flag != nullptr)
// come back to the host, which finds the eigenpairs of T; the vectors go
// back to the device (eigv: 2 N k + expanded reflectors) for x = Q y
// against the reflectors left there (on the host instead, from a copy of
// the reflectors, past the kernel's order limit).  *failed reports a set
// flag (outputs then unused).  With rel_cut > 0 only the pairs above the
// cut (relative to the largest singular value) get vectors: *k_used of
// them, vecs then N x *k_used.
fkk_status eig_finish(fkk_ctx* ctx, double* eigv, int N, int k, size_t nv, const double* beta, const double* flag,
                      double* vals, double* vecs, bool* failed, double rel_cut, int* k_used) {
    hipStream_t s = ctx->stream;
    const bool dev_bt = N <= fkk::dev::back_transform_max_n();
    const size_t k4n = (size_t)(k + 3) / 4 * 4 * N;
    // pinned: beta | d | e | flag | Y (k rounded up to 4 vectors) | x (N k), or the reflectors
    FKK_HIP(ctx, ctx->hG.ensure(3 * (size_t)N + 1 + k4n + (dev_bt ? (size_t)N * k : nv)));
    double* h = ctx->hG.p;
    double* hflag = h + 3 * N;
    double* hY = hflag + 1;
    double* hx = hY + k4n;
    *failed = false;
    FKK_HIP(ctx, hipMemcpyAsync(h, beta, 3 * (size_t)N * sizeof(double), hipMemcpyDeviceToHost, s));
    if (flag) FKK_HIP(ctx, hipMemcpyAsync(hflag, flag, sizeof(double), hipMemcpyDeviceToHost, s));
    FKK_HIP(ctx, hipEventRecord(ctx->ev[10], s));
    if (!dev_bt) {
        FKK_HIP(ctx, hipMemcpyAsync(hx, beta + 3 * N, nv * sizeof(double), hipMemcpyDeviceToHost, s));
        FKK_HIP(ctx, hipEventRecord(ctx->ev[11], s));
    }
    FKK_HIP(ctx, hipEventSynchronize(ctx->ev[10]));
    if (flag) {
        int berr = 0;
        std::memcpy(&berr, hflag, sizeof berr);
        if (berr != 0) {
            *failed = true;
            if (!dev_bt) FKK_HIP(ctx, hipEventSynchronize(ctx->ev[11]));
            return FKK_OK;
        }
    }
    std::fill(hY, hY + k4n, 0.0);
    const int rc = fkk::tridiag_eigvecs(h + N, h + 2 * N, N, k, vals, hY, rel_cut, k_used);
    if (!dev_bt) FKK_HIP(ctx, hipEventSynchronize(ctx->ev[11]));
    if (rc != 0) return ctx->fail(FKK_EINTERNAL, "tridiagonal eigensolver failed");
    const int ku = *k_used;
    if (!dev_bt) {
        fkk::tridiag_back_transform(h, hx, N, ku, hY, vecs);
        return FKK_OK;
    }
    double* dY = eigv;
    double* dx = dY + (size_t)N * ku;
    double* vpad = dx + (size_t)N * ku;
    FKK_HIP(ctx, hipMemcpyAsync(dY, hY, (size_t)N * ku * sizeof(double), hipMemcpyHostToDevice, s));
    FKK_HIP(ctx, fkk::dev::launch_back_transform(beta, beta + 3 * N, N, ku, dY, dx, vpad, s));
    FKK_HIP(ctx, hipMemcpyAsync(hx, dx, (size_t)N * ku * sizeof(double), hipMemcpyDeviceToHost, s));
    FKK_HIP(ctx, hipEventRecord(ctx->ev[11], s));
    FKK_HIP(ctx, hipEventSynchronize(ctx->ev[11]));
    std::memcpy(vecs, hx, (size_t)N * ku * sizeof(double));
    return FKK_OK;
}

// Top-k eigenpairs of diag(f) G diag(f) with G = w.g.G: scaling, the
// Householder reduction and the back-transformation on the device, the
// tridiagonal eigenproblem on the host.  Overwrites G.
fkk_status eig_device(fkk_ctx* ctx, const FitWs& w, int N, int k, const double* f, double* vals, double* vecs,
                      bool timed, double rel_cut, int* k_used, int* path) {
    const size_t nv = fkk::dev::tridiag_vstore_doubles(N);
    const size_t nx = fkk::dev::tridiag_resident_xch_doubles(N);
    hipStream_t s = ctx->stream;
    double* G = w.g.G;
    double* t = w.tri;
    double *p0 = t, *p1 = t + N, *beta = t + 2 * N, *d = t + 3 * N, *e = t + 4 * N, *vs = t + 5 * N;
    double* flags = vs + nv;  // [0]: exchange error (int), [1]: unused
    double* xch = flags + 2;
    FKK_HIP(ctx, hipMemcpyAsync(w.fdev, f, N * sizeof(double), hipMemcpyHostToDevice, s));
    FKK_HIP(ctx, fkk::dev::launch_scale_sym(G, w.fdev, N, s));
    const int rg = ctx->resident_tri ? fkk::dev::tridiag_resident_grid(N, ctx->device) : 0;
    if (rg > 0) {
        // G is read only, so a failed exchange leaves it for the per-column path
        if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[6], s));
        FKK_HIP(ctx, hipMemsetAsync(flags, 0, (2 + nx) * sizeof(double), s));
        if (fkk::dev::launch_tridiag_resident(G, N, rg, xch, reinterpret_cast<int*>(flags), vs, beta, d, e,
                                              ctx->tri_spin_limit, s) == hipSuccess) {
            if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[7], s));
            bool failed = false;
            const fkk_status st =
                eig_finish(ctx, w.eigv, N, k, nv, beta, flags, vals, vecs, &failed, rel_cut, k_used);
            if (st != FKK_OK || !failed) {
                if (path) *path = FKK_TRIDIAG_RESIDENT;
                return st;
            }
        } else {
            (void)hipGetLastError();  // launch refused (e.g. the grid cannot be co-resident)
        }
        ctx->resident_tri = false;
    }
    FKK_HIP(ctx, fkk::dev::tridiag_prepare(N));
    if (ctx->graphs && !(ctx->tri_exec && ctx->tri_n == N && ctx->tri_key[0] == G && ctx->tri_key[1] == t)) {
        if (ctx->tri_exec) {
            hipGraphExecDestroy(ctx->tri_exec);
            ctx->tri_exec = nullptr;
        }
        if (!ctx->cap_stream) FKK_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
        FKK_HIP(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
        const hipError_t le = fkk::dev::launch_tridiag(G, N, p0, p1, vs, beta, d, e, ctx->cap_stream);
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &g);
        hipError_t ie = hipSuccess;
        if (le == hipSuccess && ce == hipSuccess) ie = hipGraphInstantiate(&ctx->tri_exec, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (le != hipSuccess || ce != hipSuccess || ie != hipSuccess) {
            ctx->tri_exec = nullptr;
            return ctx->fail(FKK_EDEVICE, "recording the tridiagonalisation failed: %s",
                             hipGetErrorString(le != hipSuccess ? le : ce != hipSuccess ? ce : ie));
        }
        ctx->tri_n = N;
        ctx->tri_key[0] = G;
        ctx->tri_key[1] = t;
    }
    if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[6], s));
    if (ctx->graphs)
        FKK_HIP(ctx, hipGraphLaunch(ctx->tri_exec, s));
    else
        FKK_HIP(ctx, fkk::dev::launch_tridiag(G, N, p0, p1, vs, beta, d, e, s));
    if (timed) FKK_HIP(ctx, hipEventRecord(ctx->ev[7], s));
    bool failed = false;
    if (path) *path = FKK_TRIDIAG_PER_COLUMN;
    return eig_finish(ctx, w.eigv, N, k, nv, beta, nullptr, vals, vecs, &failed, rel_cut, k_used);
}

// Standard normal numbers for the range finder's test matrix: SplitMix64
// (Steele, Lea & Flood 2014) from `seed`, pairs of uniforms in (0, 1]
// turned into pairs of normals by the Box-Muller transform.
void rrf_gaussian(uint64_t seed, size_t n, double* out) {
    uint64_t x = seed;
    auto next = [&x]() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (size_t i = 0; i < n; i += 2) {
        const double u1 = ((next() >> 11) + 1) * (1.0 / 9007199254740992.0);
        const double u2 = ((next() >> 11) + 1) * (1.0 / 9007199254740992.0);
        const double r = std::sqrt(-2.0 * std::log(u1)), t = 6.283185307179586 * u2;
        out[i] = r * std::cos(t);
        if (i + 1 < n) out[i + 1] = r * std::sin(t);
    }
}

// Top-k singular triplets of A = l diag(f) by the randomized range finder
// with subspace iteration (Halko, Martinsson & Tropp 2011, Algorithms 4.4
// and 5.1) on the FP32 log ratio in w.g.L: Y = A W on the matrix cores
// (projection kernel), Y^T Y with FP64 products and sums, A^T Y as FP64
// partials of FP32 matrix-core stages; the n x l and l x l algebra in FP64
// on the host.  Q = Y R^-1 with R from Cholesky of Y^T Y stays implicit:
// A^T Q = diag(f) (l^T Y) R^-1.  Outputs s (k) and V (N x k, sign rule).
fkk_status rrf_device(fkk_ctx* ctx, const FitWs& w, int64_t M, int N, const double* f, const fkk_params* p, int k,
                      double* sv, double* V) {
    const int l = k + p->rrf_oversample;
    const int npad = npad_for(N), nb = npad / fkk::dev::kGramTile;
    constexpr int LY = fkk::dev::kGramTile;  // Y is M x 128 (columns past l zero)
    hipStream_t s = ctx->stream;
    std::vector<double> W((size_t)N * l);
    if (p->rrf_omega)
        std::memcpy(W.data(), p->rrf_omega, W.size() * sizeof(double));
    else
        rrf_gaussian(p->rrf_seed, W.size(), W.data());
    fkk::dev::GramPlan pc = fkk::dev::gram_plan(M, N, 64, 32), py = pc;
    pc.tiles = nb;  // (bi, 0): l^T Y
    py.tiles = 1;   // (0, 0): Y^T Y
    std::vector<int> pairs(2 * (size_t)(nb + 1), 0);
    for (int bi = 0; bi < nb; ++bi) pairs[2 * bi] = bi;
    FKK_HIP(ctx, ctx->hG.ensure((size_t)npad * LY + (size_t)LY * LY));
    FKK_HIP(ctx, hipMemcpyAsync(w.g.tiles, pairs.data(), pairs.size() * sizeof(int), hipMemcpyHostToDevice, s));
    double* d_c = w.g.G;                         // l^T Y: N x 128
    double* d_gy = w.g.G + (size_t)npad * LY;    // Y^T Y: 128 x 128
    double* h_c = ctx->hG.p;
    double* h_gy = ctx->hG.p + (size_t)npad * LY;
    std::vector<float> wt((size_t)LY * npad);
    std::vector<double> AtQ((size_t)N * l), G((size_t)l * l);
    const fkk::dev::ArgPart none{nullptr, nullptr, nullptr, nullptr};
    for (int it = 0; it <= p->rrf_power_iters; ++it) {
        std::fill(wt.begin(), wt.end(), 0.f);
        for (int c = 0; c < l; ++c)
            for (int j = 0; j < N; ++j) wt[(size_t)c * npad + j] = (float)(f[j] * W[(size_t)j * l + c]);
        FKK_HIP(ctx, hipMemcpyAsync(w.X, wt.data(), wt.size() * sizeof(float), hipMemcpyHostToDevice, s));
        FKK_HIP(ctx, fkk::dev::launch_project(w.g.L, M, N, npad, w.g.rinv, (float)p->ratio_floor, w.X,
                                              npad, LY, LY, w.Z, LY, none, 0, s, true));
        FKK_HIP(ctx, fkk::dev::launch_gram_pair(w.Z, LY, w.Z, LY, M, py, w.g.tiles + 2 * nb,
                                                w.g.partial, s, true));
        FKK_HIP(ctx, fkk::dev::launch_gram_reduce_rect(w.g.partial, py, w.g.tiles + 2 * nb, LY, LY, d_gy, LY,
                                                       s));
        FKK_HIP(ctx, fkk::dev::launch_gram_pair(w.g.L, npad, w.Z, LY, M, pc, w.g.tiles, w.g.partial, s,
                                                false));
        FKK_HIP(ctx, fkk::dev::launch_gram_reduce_rect(w.g.partial, pc, w.g.tiles, N, LY, d_c, LY, s));
        FKK_HIP(ctx, hipMemcpyAsync(h_c, d_c, (size_t)N * LY * sizeof(double), hipMemcpyDeviceToHost, s));
        FKK_HIP(ctx, hipMemcpyAsync(h_gy, d_gy, (size_t)LY * LY * sizeof(double), hipMemcpyDeviceToHost, s));
        FKK_HIP(ctx, hipStreamSynchronize(s));
        for (int a = 0; a < l; ++a)
            for (int b = 0; b < l; ++b) G[(size_t)a * l + b] = h_gy[(size_t)a * LY + b];
        if (!fkk::cholesky_upper(G.data(), l))
            return ctx->fail(FKK_ERANK, "range finder: Y^T Y not positive definite (rank of A below l = %d)", l);
        for (int j = 0; j < N; ++j)
            for (int c = 0; c < l; ++c) AtQ[(size_t)j * l + c] = f[j] * h_c[(size_t)j * LY + c];
        fkk::solve_right_upper(AtQ.data(), N, l, G.data());  // A^T Q = A^T Y R^-1
        if (it < p->rrf_power_iters) {
            W = AtQ;
            if (!fkk::orthonormalize_cols(W.data(), N, l))
                return ctx->fail(FKK_ERANK, "range finder: A^T Q rank deficient (rank of A below l = %d)", l);
        }
    }
    // B = Q^T A = (A^T Q)^T: B B^T = (A^T Q)^T (A^T Q); V = B^T U_B / s
    fkk::gram_cols(AtQ.data(), N, l, G.data());
    std::vector<double> lam(k), ub((size_t)l * k);
    if (fkk::eigh_topk(G.data(), l, k, lam.data(), ub.data(), 1) != 0)
        return ctx->fail(FKK_EINTERNAL, "range finder: small eigensolve failed");
    for (int c = 0; c < k; ++c) sv[c] = std::sqrt(std::max(lam[c], 0.0));
    for (int j = 0; j < N; ++j)
        for (int c = 0; c < k; ++c) {
            double acc = 0.0;
            for (int a = 0; a < l; ++a) acc += AtQ[(size_t)j * l + a] * ub[(size_t)a * k + c];
            V[(size_t)j * k + c] = sv[c] > 0.0 ? acc / sv[c] : 0.0;
        }
    for (int c = 0; c < k; ++c) {  // largest-magnitude entry positive (first on ties)
        int imax = 0;
        for (int j = 1; j < N; ++j)
            if (std::fabs(V[(size_t)j * k + c]) > std::fabs(V[(size_t)imax * k + c])) imax = j;
        if (V[(size_t)imax * k + c] < 0.0)
            for (int j = 0; j < N; ++j) V[(size_t)j * k + c] = -V[(size_t)j * k + c];
    }
    return FKK_OK;
}

}  // namespace

extern "C" {

int fkk_version(void) { return FKK_API_VERSION; }

const char* fkk_status_string(fkk_status s) {
    switch (s) {
        case FKK_OK: return "ok";
        case FKK_EINVAL: return "invalid argument";
        case FKK_ENOMEM: return "out of memory";
        case FKK_EDEVICE: return "device error";
        case FKK_EDOMAIN: return "invalid intensities";
        case FKK_EMISMATCH: return "basis / data mismatch";
        case FKK_ERANK: return "rank not available";
        case FKK_EINTERNAL: return "internal numerical failure";
    }
    return "unknown status";
}

void fkk_params_default(fkk_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->k = 50;
    p->f_mode = FKK_F_ONE;
    p->alpha = 0.0;
    p->sigma_g = 1.0;
    p->pad_mode = FKK_PAD_EDGE;
    p->fft_len = 0;
    p->detrend = FKK_DETREND_ALS;
    p->als_lambda = 0.0;
    p->als_p = 1e-3;
    p->als_iters = 10;
    p->ridge_rel = 1e-6;
    p->sec_mode = FKK_SEC_SAVGOL;
    p->sg_window = 0;
    p->sg_order = 2;
    p->ml_lambda = 0.0;
    p->ratio_floor = 1e-6;
    p->strict = 0;
    p->gram_prec = FKK_PREC_FP32;
    p->recon_prec = FKK_PREC_FP32;
    p->output = FKK_OUT_IM;
    p->q_override = nullptr;
    p->n_q_override = 0;
    p->sec_form = FKK_SEC_FORM_LOG;
    p->svd_mode = FKK_SVD_GRAM;
    p->rrf_oversample = 10;
    p->rrf_power_iters = 1;
    p->rrf_seed = 20200514;
    p->rrf_omega = nullptr;
    p->q_between = 0;
}

fkk_status fkk_ctx_create(int device, void* hip_stream, fkk_ctx** out) {
    if (!out) return FKK_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return FKK_EDEVICE;
    if (device < 0 || device >= count) return FKK_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return FKK_EDEVICE;
    void* scr = nullptr;
    if (scratch_address(device, &scr) != hipSuccess) return FKK_EDEVICE;
    fkk_ctx* c = new fkk_ctx;
    c->device = device;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->scratch = scr;
    const char* ng = std::getenv("FKK_NO_GRAPHS");
    c->graphs = !(ng && ng[0] == '1');
    const char* nr = std::getenv("FKK_NO_RESIDENT_TRIDIAG");
    c->resident_tri = !(nr && nr[0] == '1');
    if (const char* sl = std::getenv("FKK_TRIDIAG_SPIN_LIMIT")) {
        const long v = std::strtol(sl, nullptr, 10);
        if (v >= 0 && v <= (1L << 30)) c->tri_spin_limit = (int)v;
    }
    *out = c;
    return FKK_OK;
}

void fkk_ctx_destroy(fkk_ctx* ctx) {
    if (!ctx) return;
    hipSetDevice(ctx->device);
    hipStreamSynchronize(ctx->stream);
    if (ctx->tri_exec) hipGraphExecDestroy(ctx->tri_exec);
    if (ctx->cap_stream) hipStreamDestroy(ctx->cap_stream);
    ctx->ws.release();
    ctx->hG.release();
    ctx->hstage.release();
    for (auto& e : ctx->ev)
        if (e) hipEventDestroy(e);
    delete ctx;
}

const char* fkk_ctx_last_error(const fkk_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

size_t fkk_ctx_workspace_bytes(const fkk_ctx* ctx) { return ctx ? ctx->bytes() : 0; }

fkk_status fkk_gram(fkk_ctx* ctx, const float* d_I, int64_t M, int32_t N, int64_t ld, const double* h_iref,
                    double ratio_floor, int32_t prec, double* h_gram, double* h_colsum, int64_t* h_clamps) {
    if (!ctx) return FKK_EINVAL;
    fkk_status st;
    if ((st = check_matrix(ctx, d_I, M, N, ld, "I")) != FKK_OK) return st;
    if ((st = check_iref(ctx, h_iref, N)) != FKK_OK) return st;
    if (!(ratio_floor >= kMinRatioFloor))
        return ctx->fail(FKK_EINVAL, "ratio_floor must be at least 2^-126 (the smallest normal FP32 number)");
    if (!valid_gram_prec(prec)) return ctx->fail(FKK_EINVAL, "bad precision %d", prec);
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    GramWs w;
    Carve sizing(nullptr);
    gram_layout(sizing, M, N, prec, true, false, &w);
    void* base = nullptr;
    if ((st = acquire_ws(ctx, nullptr, 0, sizing.bytes(), &base)) != FKK_OK) return st;
    Carve c(base);
    gram_layout(c, M, N, prec, true, false, &w);
    std::vector<double> cs(N);
    int64_t cl = 0;
    if ((st = gram_with_sums(ctx, w, d_I, M, N, ld, h_iref, ratio_floor, prec, false, true, cs.data(), &cl)) !=
        FKK_OK)
        return st;
    if (h_gram) {
        FKK_HIP(ctx, hipMemcpyAsync(h_gram, w.G, (size_t)N * N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        FKK_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (h_colsum) std::memcpy(h_colsum, cs.data(), N * sizeof(double));
    if (h_clamps) *h_clamps = cl;
    return FKK_OK;
}

fkk_status fkk_eigh_topk(const double* h_a, int32_t N, int32_t k, double* h_evals, double* h_evecs) {
    if (!h_a || !h_evals || !h_evecs || N < 1 || k < 1 || k > N) return FKK_EINVAL;
    return fkk::eigh_topk(h_a, N, k, h_evals, h_evecs, host_threads()) == 0 ? FKK_OK : FKK_EINTERNAL;
}

fkk_status fkk_basis_from_factors(fkk_ctx* ctx, int32_t N, int32_t k, const double* h_iref, const double* h_f,
                                  const double* h_s, const double* h_v, const double* h_x, int32_t n_q,
                                  const fkk_params* p, fkk_basis** out_basis) {
    fkk_ctx sink;  // error sink when ctx is NULL (host-only basis)
    fkk_ctx* c = ctx ? ctx : &sink;
    if (!out_basis || !h_iref || !h_f || !h_s || !h_v || !h_x || n_q < 1 || N < 4)
        return c->fail(FKK_EINVAL, "NULL argument or bad size");
    *out_basis = nullptr;
    fkk_status st;
    if ((st = check_params(c, p, N)) != FKK_OK) return st;
    if (p->k != k) return c->fail(FKK_EINVAL, "params.k != k");
    fkk_basis* b = new_basis(N, k, h_iref, h_f, h_s, h_v, p->ml_lambda, p->ratio_floor);
    b->prec = p->recon_prec;
    basis_fkk(b, p);
    basis_math(b, h_x, n_q, p);
    if (ctx) {
        if ((st = upload_basis(ctx, b, p->ml_lambda)) != FKK_OK) {
            delete b;
            return st;
        }
    }
    *out_basis = b;
    return FKK_OK;
}

fkk_status fkk_fit(fkk_ctx* ctx, const float* d_I, int64_t M, int32_t N, int64_t ld, const double* h_iref,
                   const fkk_params* p, fkk_basis** out_basis, float* d_out, int64_t ld_out, void* d_ws,
                   size_t ws_bytes, fkk_fit_report* rep) {
    if (!ctx) return FKK_EINVAL;
    const auto t_all = std::chrono::steady_clock::now();
    fkk_status st;
    if ((st = check_matrix(ctx, d_I, M, N, ld, "I")) != FKK_OK) return st;
    if ((st = check_iref(ctx, h_iref, N)) != FKK_OK) return st;
    if ((st = check_params(ctx, p, N, true)) != FKK_OK) return st;
    if (d_out && ld_out < N) return ctx->fail(FKK_EINVAL, "ld_out=%lld < N", (long long)ld_out);
    if (p->n_q_override > 0) {
        if (!p->q_override) return ctx->fail(FKK_EINVAL, "q_override is NULL");
        for (int i = 0; i < p->n_q_override; ++i)
            if (p->q_override[i] < 0 || p->q_override[i] >= M)
                return ctx->fail(FKK_EINVAL, "q_override[%d] out of range", i);
    }
    if (out_basis) *out_basis = nullptr;
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // k = 0: the top min(N, 128) pairs are computed and the rank rule keeps
    // those above the cut-off (Sec. 4.1)
    const int kcap = p->k > 0 ? p->k : std::min(N, 128);
    fkk_fit_report r{};
    FitWs w;
    void* base = nullptr;
    if ((st = acquire_ws(ctx, d_ws, ws_bytes, fit_layout(nullptr, M, N, p, &w), &base)) != FKK_OK) return st;
    fit_layout(base, M, N, p, &w);

    // 1. log ratio, Gram and column sums on the device (Eq. 2, 6, 9)
    auto t0 = std::chrono::steady_clock::now();
    std::vector<double> colsum(N);
    int64_t clamps = 0;
    FKK_HIP(ctx, ctx->events());
    const bool rrf = (p->svd_mode == FKK_SVD_RANDOMIZED);
    // the range finder works from the FP32 log ratio, whatever gram_prec says
    const int gprec = rrf ? FKK_PREC_FP32 : p->gram_prec;
    if ((st = gram_with_sums(ctx, w.g, d_I, M, N, ld, h_iref, p->ratio_floor, gprec, true, !rrf, colsum.data(),
                             &clamps)) != FKK_OK)
        return st;
    r.dev_ms_gram = rrf ? 0.0 : ctx->elapsed(0, 1);
    r.dev_ms_logratio = ctx->elapsed(8, 9);
    r.clamps = clamps;
    r.ms_gram = ms_since(t0);
    if (p->strict && clamps > 0) return ctx->fail(FKK_EDOMAIN, "%lld intensity ratios clamped", (long long)clamps);

    // 2. f and the FP64 eigensolve of G_A = diag(f) G_L diag(f)
    t0 = std::chrono::steady_clock::now();
    std::vector<double> f(N, 1.0);
    if (p->f_mode == FKK_F_NOISE)
        for (int j = 0; j < N; ++j) {
            const double mean = colsum[j] / (double)M;
            f[j] = 2.0 * mean / std::sqrt(p->alpha * mean + p->sigma_g * p->sigma_g);
        }
    std::vector<double> lam(kcap), V((size_t)N * kcap), sv(kcap);
    // the rank rule keeps singular values above s_max max(M, N) eps, eps of
    // the FP32 input
    const double rank_rel = p->k == 0 ? (double)std::max<int64_t>(M, N) * (double)FLT_EPSILON : 0.0;
    int k = kcap;
    if (rrf) {
        if ((st = rrf_device(ctx, w, M, N, f.data(), p, kcap, sv.data(), V.data())) != FKK_OK) return st;
        for (int c = 0; c < kcap; ++c) lam[c] = sv[c] * sv[c];
    } else {
        // with the rank rule, the eigenvalues come first and only the kept
        // pairs get eigenvectors; V is then N x k
        if ((st = eig_device(ctx, w, N, kcap, f.data(), lam.data(), V.data(), true, rank_rel, &k, &r.tridiag_path)) !=
            FKK_OK)
            return st;
        for (int c = 0; c < k; ++c) sv[c] = std::sqrt(std::max(lam[c], 0.0));
        if (k < kcap) {
            V.resize((size_t)N * k);
            lam.resize(k);
            sv.resize(k);
        }
        r.dev_ms_tridiag = ctx->elapsed(6, 7);
    }
    if (p->k == 0 && rrf) {
        const double cut = sv[0] * rank_rel;
        int cnt = 0;
        for (int c = 0; c < kcap; ++c) cnt += sv[c] > cut ? 1 : 0;
        k = std::max(cnt, 1);
        if (k < kcap) {
            std::vector<double> Vk((size_t)N * k);
            for (int j = 0; j < N; ++j)
                for (int c = 0; c < k; ++c) Vk[(size_t)j * k + c] = V[(size_t)j * kcap + c];
            V.swap(Vk);
            lam.resize(k);
            sv.resize(k);
        }
    }
    const int kp = kp_for(k);
    r.ms_eig = ms_since(t0);

    // 3. projection Z = A V_k and per-column arg-extrema (Eq. 13-15)
    t0 = std::chrono::steady_clock::now();
    fkk_basis* b = new_basis(N, k, h_iref, f.data(), sv.data(), V.data(), p->ml_lambda, p->ratio_floor);
    b->prec = p->recon_prec;
    const bool pbf16 = (p->recon_prec == FKK_PREC_BF16), psplit = (p->recon_prec == FKK_PREC_SPLIT);
    const int kq = b->kq;
    const int ka = (pbf16 || psplit) ? kq : kp;  // column blocks of the arg-extrema partials
    // FP32 weights (kp x npad), and for the BF16 modes their BF16 copy
    // (kq x npad) or three BF16 pieces in consecutive planes (the first is
    // the BF16 copy); rows of W^T split over the host pool
    std::vector<float> wt((size_t)kp * b->npad, 0.f);
    std::vector<uint16_t> wt16;
    const int np16 = psplit ? 3 : (pbf16 ? 1 : 0);
    if (np16) wt16.assign((size_t)np16 * kq * b->npad, 0);
    fkk::parallel_rows(k, [&](int c0, int c1) {
        for (int c = c0; c < c1; ++c)
            for (int j = 0; j < N; ++j) {
                const size_t i = (size_t)c * b->npad + j;
                float rest = wt[i] = (float)(f[j] * V[(size_t)j * k + c]);
                for (int pc = 0; pc < np16; ++pc) {
                    const uint16_t h = to_bf16(rest);
                    wt16[(size_t)pc * kq * b->npad + i] = h;
                    rest -= from_bf16(h);
                }
            }
    });
    auto cleanup = [&](fkk_status e) { delete b; return e; };
    const int64_t nblk = fkk::dev::proj_blocks(M);
    // w.X holds the weights: kp x npad FP32, kq x npad BF16, or three such BF16 planes
    float* d_wt = w.X;  // the fit's projection weights (no ML shrink)
    uint16_t* d_wt16 = reinterpret_cast<uint16_t*>(w.X);
    const hipError_t wcopy =
        (pbf16 || psplit)
            ? hipMemcpyAsync(d_wt16, wt16.data(), wt16.size() * sizeof(uint16_t), hipMemcpyHostToDevice, s)
            : hipMemcpyAsync(d_wt, wt.data(), wt.size() * sizeof(float), hipMemcpyHostToDevice, s);
    if (wcopy != hipSuccess) return cleanup(ctx->fail(FKK_EDEVICE, "copy of projection weights failed"));
    fkk::dev::ArgPart part{w.pmaxv, w.pminv, w.pmaxi, w.pmini};
    hipError_t perr = hipEventRecord(ctx->ev[2], s);
    if (perr == hipSuccess) {
        if (pbf16 || psplit)  // log ratio recomputed from I
            perr = fkk::dev::launch_project16(d_I, M, N, ld, w.g.rinv, (float)p->ratio_floor, d_wt16, b->npad, kq,
                                              kp, w.Z, kp, part, k, s, psplit ? 3 : 1);
        else if (gprec == FKK_PREC_BF16 || gprec == FKK_PREC_SPLIT)  // w.g.L holds no FP32 l: start from I
            perr = fkk::dev::launch_project(d_I, M, N, ld, w.g.rinv, (float)p->ratio_floor, d_wt, b->npad, kp, kp,
                                            w.Z, kp, part, k, s, false);
        else  // the FP32 l of the Gram pass
            perr = fkk::dev::launch_project(w.g.L, M, N, npad_for(N), w.g.rinv, (float)p->ratio_floor, d_wt,
                                            b->npad, kp, kp, w.Z, kp, part, k, s, true);
    }
    if (perr != hipSuccess || hipEventRecord(ctx->ev[3], s) != hipSuccess ||
        fkk::dev::launch_argext_reduce(part, nblk, ka, k, w.qext, w.qext + ka, s) != hipSuccess)
        return cleanup(ctx->fail(FKK_EDEVICE, "projection launch failed"));
    // the optional rows between the extrema (Sec. 2.3), from the stored Z
    const int nbet = (p->n_q_override > 0) ? 0 : k * p->q_between;
    if (nbet > 0) {
        if (fkk::dev::launch_between(w.Z, M, kp, kp, k, p->q_between, w.qext, w.qext + ka, w.bval, w.bidx, w.qbet,
                                     s) != hipSuccess)
            return cleanup(ctx->fail(FKK_EDEVICE, "sub-sample launch failed"));
    }
    basis_fkk(b, p);  // host FP64 while the projection runs
    std::vector<long long> qe(2 * (size_t)ka), qb(nbet);
    if (hipMemcpyAsync(qe.data(), w.qext, qe.size() * sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
        (nbet > 0 && hipMemcpyAsync(qb.data(), w.qbet, qb.size() * sizeof(long long), hipMemcpyDeviceToHost,
                                    s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(ctx->fail(FKK_EDEVICE, "projection failed"));
    r.dev_ms_project = ctx->elapsed(2, 3);
    std::vector<long long> q;
    if (p->n_q_override > 0) {
        q.assign(p->q_override, p->q_override + p->n_q_override);
    } else {
        for (int c = 0; c < k; ++c) {
            if (qe[c] >= 0) q.push_back(qe[c]);
            if (qe[ka + c] >= 0) q.push_back(qe[ka + c]);
        }
        for (long long r : qb)
            if (r >= 0) q.push_back(r);
        std::sort(q.begin(), q.end());
        q.erase(std::unique(q.begin(), q.end()), q.end());
    }
    const int n_q = (int)q.size();
    // U_ss S = A[q] V_k (Eq. 13-15) in FP64 from the FP32 input rows q: the
    // device Z only selects q.  fPEC's ridge solve amplifies errors of X
    // along its weak directions, so X is not taken from the FP32 projection.
    std::vector<float> rows((size_t)n_q * N);
    // (n_q is at most the layout's 2 k + k q_between, or n_q_override)
    if (hipMemcpyAsync(w.qdev, q.data(), n_q * sizeof(long long), hipMemcpyHostToDevice, s) != hipSuccess ||
        fkk::dev::launch_gather_rows(d_I, ld, N, w.qdev, n_q, w.rows, s) != hipSuccess ||
        hipMemcpyAsync(rows.data(), w.rows, rows.size() * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(ctx->fail(FKK_EDEVICE, "gather of sub-sampled rows failed"));
    r.ms_project = ms_since(t0);

    // 4. fKK, fPEC, fSEC on the basis vectors (host FP64)
    t0 = std::chrono::steady_clock::now();
    std::vector<double> X((size_t)n_q * k, 0.0);
    fkk::parallel_rows(n_q, [&](int q0, int q1) {
        std::vector<double> a(N);
        for (int rq = q0; rq < q1; ++rq) {
            for (int j = 0; j < N; ++j) {
                double ratio = (double)rows[(size_t)rq * N + j] / h_iref[j];
                if (!(ratio > p->ratio_floor) || !std::isfinite(ratio)) ratio = p->ratio_floor;
                a[j] = 0.5 * std::log(ratio) * f[j];
            }
            double* xr = &X[(size_t)rq * k];
            for (int j = 0; j < N; ++j) {
                const double aj = a[j];
                const double* vr = &V[(size_t)j * k];
                for (int c = 0; c < k; ++c) xr[c] += aj * vr[c];
            }
        }
    });
    b->q.assign(q.begin(), q.end());
    basis_math(b, X.data(), n_q, p);
    if ((st = upload_basis(ctx, b, p->ml_lambda)) != FKK_OK) return cleanup(st);
    r.n_q = n_q;
    r.ridge_lambda = b->ridge_lambda;
    r.ms_basis = ms_since(t0);

    // 5. reconstruction of Eq. 23 for the training rows
    t0 = std::chrono::steady_clock::now();
    if (d_out) {
        if (hipEventRecord(ctx->ev[4], s) != hipSuccess ||
            (pbf16 || p->recon_prec == FKK_PREC_SPLIT
                 ? fkk::dev::launch_reconstruct16(w.Z, M, kp, k, b->d_bre16, b->d_bim16, kq, N, b->npad, d_out, ld_out,
                                                  p->output, s, pbf16 ? 1 : 3)
                 : fkk::dev::launch_reconstruct(w.Z, M, kp, k, b->d_bre_t, b->d_bim_t, kp, N, d_out, ld_out,
                                                p->output, s)) != hipSuccess ||
            hipEventRecord(ctx->ev[5], s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            return cleanup(ctx->fail(FKK_EDEVICE, "reconstruction failed"));
        r.dev_ms_recon = ctx->elapsed(4, 5);
    }
    r.ms_recon = ms_since(t0);
    r.ms_total = ms_since(t_all);
    if (rep) *rep = r;
    if (out_basis) *out_basis = b;
    else delete b;
    return FKK_OK;
}

fkk_status fkk_transform(fkk_ctx* ctx, const fkk_basis* b, const float* d_I, int64_t M, int64_t ld, float* d_out,
                         int64_t ld_out, int32_t plane, float* d_norms, void* d_ws, size_t ws_bytes) {
    if (!ctx) return FKK_EINVAL;
    if (!b) return ctx->fail(FKK_EINVAL, "basis is NULL");
    fkk_status st;
    if ((st = check_matrix(ctx, d_I, M, b->N, ld, "I")) != FKK_OK) return st;
    if (!d_out || ld_out < b->N) return ctx->fail(FKK_EINVAL, "bad output");
    if (plane < FKK_OUT_IM || plane > FKK_OUT_ABS) return ctx->fail(FKK_EINVAL, "bad output plane %d", plane);
    if (!d_ws && ws_bytes != 0) return ctx->fail(FKK_EINVAL, "ws_bytes without a workspace");
    (void)ws_bytes;  // the fused kernel keeps its Z tile in LDS: no workspace
    if (b->device != ctx->device || !b->d_wt) return ctx->fail(FKK_EMISMATCH, "basis lives on another device");
    if (d_norms && (reinterpret_cast<uintptr_t>(d_norms) & 7) != 0)
        return ctx->fail(FKK_EINVAL, "norms must be 8-byte aligned");
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    fkk::dev::ResidualArgs res;
    if (d_norms) res = {b->d_f, b->d_g, d_norms};
    if (b->prec == FKK_PREC_BF16)
        FKK_HIP(ctx, fkk::dev::launch_transform16(d_I, M, b->N, ld, b->d_rinv, (float)b->ratio_floor, b->d_wt16,
                                                  b->npad, b->kq, b->d_bre16, b->d_bim16, d_out, ld_out, plane,
                                                  ctx->stream, res));
    else
        FKK_HIP(ctx, fkk::dev::launch_transform(d_I, M, b->N, ld, b->d_rinv, (float)b->ratio_floor, b->d_wt, b->npad,
                                                b->kp, b->k, b->d_bre_t, b->d_bim_t, d_out, ld_out, plane,
                                                ctx->stream, res));
    return FKK_OK;
}

fkk_status fkk_project(fkk_ctx* ctx, const fkk_basis* b, const float* d_I, int64_t M, int64_t ld, float* d_z,
                       int64_t ld_z, int64_t* h_qmax, int64_t* h_qmin) {
    if (!ctx) return FKK_EINVAL;
    if (!b) return ctx->fail(FKK_EINVAL, "basis is NULL");
    fkk_status st;
    if ((st = check_matrix(ctx, d_I, M, b->N, ld, "I")) != FKK_OK) return st;
    if (!d_z || ld_z < b->k) return ctx->fail(FKK_EINVAL, "bad Z output");
    if (b->device != ctx->device || !b->d_wt) return ctx->fail(FKK_EMISMATCH, "basis lives on another device");
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t nblk = fkk::dev::proj_blocks(M);
    const bool bf16 = (b->prec == FKK_PREC_BF16);
    const int ka = bf16 ? b->kq : b->kp;
    fkk::dev::ArgPart part{nullptr, nullptr, nullptr, nullptr};
    long long* qext = nullptr;
    const bool want = h_qmax || h_qmin;
    if (want) {
        auto layout = [&](void* base) {
            Carve c(base);
            part.maxv = c.take<float>((size_t)nblk * ka);
            part.minv = c.take<float>((size_t)nblk * ka);
            part.maxi = c.take<long long>((size_t)nblk * ka);
            part.mini = c.take<long long>((size_t)nblk * ka);
            qext = c.take<long long>(2 * (size_t)ka);
            return c.bytes();
        };
        void* base = nullptr;
        if ((st = acquire_ws(ctx, nullptr, 0, layout(nullptr), &base)) != FKK_OK) return st;
        layout(base);
    }
    if (bf16)
        FKK_HIP(ctx, fkk::dev::launch_project16(d_I, M, b->N, ld, b->d_rinv, (float)b->ratio_floor, b->d_wt16, b->npad,
                                                b->kq, b->k, d_z, ld_z, part, b->k, s));
    else
        FKK_HIP(ctx, fkk::dev::launch_project(d_I, M, b->N, ld, b->d_rinv, (float)b->ratio_floor, b->d_wt, b->npad,
                                              b->kp, b->k, d_z, ld_z, part, b->k, s));
    if (!want) return FKK_OK;
    FKK_HIP(ctx, fkk::dev::launch_argext_reduce(part, nblk, ka, b->k, qext, qext + ka, s));
    std::vector<long long> qe(2 * (size_t)ka);
    FKK_HIP(ctx, hipMemcpyAsync(qe.data(), qext, qe.size() * sizeof(long long), hipMemcpyDeviceToHost, s));
    FKK_HIP(ctx, hipStreamSynchronize(s));
    for (int c = 0; c < b->k; ++c) {
        if (h_qmax) h_qmax[c] = qe[c];
        if (h_qmin) h_qmin[c] = qe[ka + c];
    }
    return FKK_OK;
}

namespace {

// Residual of Sec. 5 from the two FP64 sums.
double residual_from_sums(double sa, double sz) { return sa > 0.0 ? std::sqrt(std::max(0.0, 1.0 - sz / sa)) : 0.0; }

fkk_status check_residual_args(fkk_ctx* ctx, const fkk_basis* b, const float* d_I, int64_t M, int64_t ld,
                               const double* h_residual) {
    if (!b || !h_residual) return ctx->fail(FKK_EINVAL, "NULL argument");
    fkk_status st;
    if ((st = check_matrix(ctx, d_I, M, b->N, ld, "I")) != FKK_OK) return st;
    if (b->device != ctx->device || !b->d_wt) return ctx->fail(FKK_EMISMATCH, "basis lives on another device");
    return FKK_OK;
}

// Partials per block of spectra into part, their total into part + 2 nblk,
// the total to the host.  The kernels are those of every residual call.
fkk_status residual_device(fkk_ctx* ctx, const fkk_basis* b, const float* d_I, int64_t M, int64_t ld, double* part,
                           double* h_residual) {
    const int64_t nblk = fkk::dev::proj_blocks(M);
    hipStream_t s = ctx->stream;
    FKK_HIP(ctx, fkk::dev::launch_residual_partials(d_I, M, b->N, ld, b->d_rinv, (float)b->ratio_floor, b->d_wt,
                                                    b->npad, b->kp, b->d_f, b->d_g, part, s));
    FKK_HIP(ctx, fkk::dev::launch_residual_total(part, nblk, part + 2 * nblk, s));
    double h[2] = {0.0, 0.0};
    FKK_HIP(ctx, hipMemcpyAsync(h, part + 2 * nblk, sizeof h, hipMemcpyDeviceToHost, s));
    FKK_HIP(ctx, hipStreamSynchronize(s));
    *h_residual = residual_from_sums(h[0], h[1]);
    return FKK_OK;
}

}  // namespace

fkk_status fkk_basis_residual(fkk_ctx* ctx, const fkk_basis* b, const float* d_I, int64_t M, int64_t ld,
                              double* h_residual) {
    if (!ctx) return FKK_EINVAL;
    fkk_status st;
    if ((st = check_residual_args(ctx, b, d_I, M, ld, h_residual)) != FKK_OK) return st;
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    void* base = nullptr;
    const size_t need = (2 * (size_t)fkk::dev::proj_blocks(M) + 2) * sizeof(double);
    if ((st = acquire_ws(ctx, nullptr, 0, need, &base)) != FKK_OK) return st;
    return residual_device(ctx, b, d_I, M, ld, static_cast<double*>(base), h_residual);
}

fkk_status fkk_basis_residual_noalloc(fkk_ctx* ctx, const fkk_basis* b, const float* d_I, int64_t M, int64_t ld,
                                      double* h_residual) {
    if (!ctx) return FKK_EINVAL;
    fkk_status st;
    if ((st = check_residual_args(ctx, b, d_I, M, ld, h_residual)) != FKK_OK) return st;
    if (M > FKK_NOALLOC_MAX_SPECTRA)
        return ctx->fail(FKK_EINVAL, "M=%lld above the %lld spectra of the fixed scratch array", (long long)M,
                         (long long)FKK_NOALLOC_MAX_SPECTRA);
    if (!ctx->scratch) return ctx->fail(FKK_EDEVICE, "no scratch address for device %d", ctx->device);
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    // the kernels write every partial and the total: nothing to clear
    return residual_device(ctx, b, d_I, M, ld, static_cast<double*>(ctx->scratch), h_residual);
}

fkk_status fkk_reconstruct(fkk_ctx* ctx, const fkk_basis* b, const float* d_z, int64_t M, int64_t ld_z,
                           float* d_out, int64_t ld_out, int32_t plane) {
    if (!ctx) return FKK_EINVAL;
    if (!b) return ctx->fail(FKK_EINVAL, "basis is NULL");
    if (!d_z || M < 1 || ld_z < b->k) return ctx->fail(FKK_EINVAL, "bad Z");
    if (!d_out || ld_out < b->N) return ctx->fail(FKK_EINVAL, "bad output");
    if (plane < FKK_OUT_IM || plane > FKK_OUT_ABS) return ctx->fail(FKK_EINVAL, "bad plane");
    if (b->device != ctx->device || !b->d_bre_t) return ctx->fail(FKK_EMISMATCH, "basis lives on another device");
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    if (b->prec == FKK_PREC_BF16 || b->prec == FKK_PREC_SPLIT)
        FKK_HIP(ctx, fkk::dev::launch_reconstruct16(d_z, M, ld_z, b->k, b->d_bre16, b->d_bim16, b->kq, b->N, b->npad, d_out,
                                                    ld_out, plane, ctx->stream,
                                                    b->prec == FKK_PREC_SPLIT ? 3 : 1));
    else
        FKK_HIP(ctx, fkk::dev::launch_reconstruct(d_z, M, ld_z, b->k, b->d_bre_t, b->d_bim_t, b->kp, b->N, d_out,
                                                  ld_out, plane, ctx->stream));
    return FKK_OK;
}

fkk_status fkk_basis_import(fkk_ctx* ctx, const fkk_basis_desc* d, fkk_basis** out) {
    if (!ctx) return FKK_EINVAL;
    if (!d || !out || !d->i_ref || !d->f || !d->s || !d->v || !d->b_re || !d->b_im)
        return ctx->fail(FKK_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->N < 4 || d->k < 1 || d->k > d->N || d->k > 128) return ctx->fail(FKK_EINVAL, "bad N / k");
    if (!(d->ml_lambda >= 0.0) || !(d->ratio_floor >= kMinRatioFloor)) return ctx->fail(FKK_EINVAL, "bad scalars");
    fkk_status st;
    if ((st = check_iref(ctx, d->i_ref, d->N)) != FKK_OK) return st;
    fkk_basis* b = new_basis(d->N, d->k, d->i_ref, d->f, d->s, d->v, d->ml_lambda, d->ratio_floor);
    b->b_re.assign(d->b_re, d->b_re + (size_t)d->k * d->N);
    b->b_im.assign(d->b_im, d->b_im + (size_t)d->k * d->N);
    if ((st = upload_basis(ctx, b, d->ml_lambda)) != FKK_OK) {
        delete b;
        return st;
    }
    *out = b;
    return FKK_OK;
}

fkk_status fkk_basis_set_precision(fkk_basis* b, int32_t prec) {
    if (!b || !valid_prec(prec)) return FKK_EINVAL;
    b->prec = prec;
    return FKK_OK;
}

fkk_status fkk_basis_get_precision(const fkk_basis* b, int32_t* prec) {
    if (!b || !prec) return FKK_EINVAL;
    *prec = b->prec;
    return FKK_OK;
}

fkk_status fkk_basis_info(const fkk_basis* b, int32_t* N, int32_t* k, int32_t* n_q) {
    if (!b) return FKK_EINVAL;
    if (N) *N = b->N;
    if (k) *k = b->k;
    if (n_q) *n_q = (int32_t)b->q.size();
    return FKK_OK;
}

fkk_status fkk_basis_export(const fkk_basis* b, double* i_ref, double* f, double* s, double* v, double* b_re,
                            double* b_im, double* phi_pec_t, double* v_sec_t, double* h_v, int64_t* q,
                            double* scalars3) {
    if (!b) return FKK_EINVAL;
    auto put = [](double* dst, const std::vector<double>& src) {
        if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(double));
    };
    put(i_ref, b->i_ref);
    put(f, b->f);
    put(s, b->s);
    put(v, b->v);
    put(b_re, b->b_re);
    put(b_im, b->b_im);
    put(phi_pec_t, b->phi_pec_t);
    put(v_sec_t, b->v_sec_t);
    put(h_v, b->h_v);
    if (q && !b->q.empty()) std::memcpy(q, b->q.data(), b->q.size() * sizeof(int64_t));
    if (scalars3) {
        scalars3[0] = b->ml_lambda;
        scalars3[1] = b->ratio_floor;
        scalars3[2] = b->ridge_lambda;
    }
    return FKK_OK;
}

fkk_status fkk_basis_free(fkk_basis* b) {
    if (!b) return FKK_OK;
    if (b->holders.load() > 0) return FKK_EBUSY;  // a server still transforms with it
    delete b;
    return FKK_OK;
}

namespace {

fkk_status plain_any(fkk_ctx* ctx, const void* d_I, bool f64, int64_t M, int32_t N, int64_t ld, const double* h_iref,
                     const fkk_params* p, void* d_out, int64_t ld_out, void* d_ws, size_t ws_bytes) {
    if (!ctx) return FKK_EINVAL;
    fkk_status st;
    if ((st = check_matrix(ctx, d_I, M, N, ld, "I")) != FKK_OK) return st;
    if (f64 && (reinterpret_cast<uintptr_t>(d_I) & 7) != 0) return ctx->fail(FKK_EINVAL, "I must be 8-byte aligned");
    if ((st = check_iref(ctx, h_iref, N)) != FKK_OK) return st;
    if ((st = check_params(ctx, p, N, false, true)) != FKK_OK) return st;
    if (!d_out || ld_out < N) return ctx->fail(FKK_EINVAL, "bad output");
    FKK_HIP(ctx, hipSetDevice(ctx->device));
    fkk::plain::Config cfg;
    cfg.N = N;
    cfg.len = p->fft_len ? p->fft_len : fkk::default_fft_len(N);
    cfg.pad_mode = p->pad_mode;
    cfg.detrend = p->detrend;
    cfg.lam = p->als_lambda > 0.0 ? p->als_lambda : fkk::default_als_lambda(N);
    cfg.p = p->als_p;
    cfg.iters = p->als_iters;
    cfg.sec_mode = p->sec_mode;
    cfg.sec_re = p->sec_form == FKK_SEC_FORM_RE ? 1 : 0;
    cfg.window = p->sg_window ? p->sg_window : fkk::default_sg_window(N);
    cfg.order = p->sg_order;
    cfg.floor = p->ratio_floor;
    cfg.plane = p->output;
    // a caller's workspace may be smaller than the full batch: the spectra
    // then run in smaller batches (at least 256 rows)
    int64_t batch = fkk::plain::full_batch(M);
    void* base = nullptr;
    if (d_ws) {
        if (reinterpret_cast<uintptr_t>(d_ws) & 255) return ctx->fail(FKK_EINVAL, "workspace must be 256-byte aligned");
        batch = fkk::plain::batch_for_bytes(N, cfg.len, M, ws_bytes);
        if (batch < 1)
            return ctx->fail(FKK_EINVAL, "workspace of %zu bytes below the %zu a batch of 256 spectra needs", ws_bytes,
                             fkk::plain::layout_bytes(N, cfg.len, 256));
        base = d_ws;
    } else if ((st = acquire_ws(ctx, nullptr, ws_bytes, fkk::plain::layout_bytes(N, cfg.len, batch), &base)) !=
               FKK_OK) {
        return st;
    }
    const fkk::plain::Layout lay = fkk::plain::carve(base, N, cfg.len, batch);
    std::string why;
    const hipError_t e = fkk::plain::run(lay, cfg, d_I, f64, M, ld, h_iref, d_out, f64, ld_out, ctx->stream, &why);
    if (e != hipSuccess)
        return ctx->fail(FKK_EDEVICE, "plain path: %s (%s)", hipGetErrorString(e), why.c_str());
    return FKK_OK;
}

}  // namespace

fkk_status fkk_plain(fkk_ctx* ctx, const float* d_I, int64_t M, int32_t N, int64_t ld, const double* h_iref,
                     const fkk_params* p, float* d_out, int64_t ld_out, void* d_ws, size_t ws_bytes) {
    return plain_any(ctx, d_I, false, M, N, ld, h_iref, p, d_out, ld_out, d_ws, ws_bytes);
}

fkk_status fkk_plain_f64(fkk_ctx* ctx, const double* d_I, int64_t M, int32_t N, int64_t ld, const double* h_iref,
                         const fkk_params* p, double* d_out, int64_t ld_out, void* d_ws, size_t ws_bytes) {
    return plain_any(ctx, d_I, true, M, N, ld, h_iref, p, d_out, ld_out, d_ws, ws_bytes);
}

fkk_status fkk_workspace_size(const fkk_ctx* ctx, int32_t op, int64_t M, int32_t N, const fkk_params* p,
                              size_t* bytes) {
    (void)ctx;
    if (!bytes) return FKK_EINVAL;
    *bytes = 0;
    if (M < 1 || N < 4) return FKK_EINVAL;
    fkk_ctx sink;  // check_params reports through a context
    switch (op) {
        case FKK_OP_FIT: {
            if (!p || check_params(&sink, p, N, true) != FKK_OK) return FKK_EINVAL;
            FitWs w;
            *bytes = fit_layout(nullptr, M, N, p, &w);
            return FKK_OK;
        }
        case FKK_OP_PLAIN:
            if (!p || check_params(&sink, p, N, false, true) != FKK_OK) return FKK_EINVAL;
            *bytes = plain_layout_bytes(M, N, p);
            return FKK_OK;
        case FKK_OP_TRANSFORM:
            return FKK_OK;  // the fused kernel needs no workspace
        default:
            return FKK_EINVAL;
    }
}

}  // extern "C"
