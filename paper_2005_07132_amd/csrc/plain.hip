// Conventional per-spectrum workflow on the device, FP64 state:
//   kk_kernel     l = 1/2 ln(I / I_ref), phi = H{l}       (Eq. 2)
//   als_kernel    phi_err = D{phi}                         (PEC, Sec. 2.1)
//   sec_kernel    rho = l + H{phi_err}, rho -= M{rho},
//                 out = plane of exp(rho + i (phi - phi_err))  (Eq. 5, 19)
// The Hilbert transform packs two real spectra into one complex FFT held in
// LDS (H is real and complex-linear, so H{a + i b} = H{a} + i H{b}).  ALS
// runs one spectrum per lane with its recurrence state interleaved across
// spectra, so every global access of a wave is one contiguous segment.
#include "plain.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace fkk {
namespace plain {

namespace {
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

int64_t full_batch(int64_t M) { return std::min<int64_t>(((M + 255) / 256) * 256, 131072); }

size_t layout_bytes(int N, int len, int64_t batch) {
    const size_t row = al256((size_t)batch * N * sizeof(double));
    return 3 * row + al256(4 * (size_t)batch * N * sizeof(double)) + al256((size_t)len * sizeof(double)) +
           al256(((size_t)N + 16) * sizeof(double));
}

int64_t batch_for_bytes(int N, int len, int64_t M, size_t bytes) {
    int64_t b = full_batch(M);
    while (b >= 256 && layout_bytes(N, len, b) > bytes) b -= 256;
    return b >= 256 ? b : 0;
}

Layout carve(void* base, int N, int len, int64_t batch) {
    Layout w;
    char* p = static_cast<char*>(base);
    const size_t row = al256((size_t)batch * N * sizeof(double));
    w.ell = reinterpret_cast<double*>(p);
    w.phi = reinterpret_cast<double*>(p + row);
    w.err = reinterpret_cast<double*>(p + 2 * row);
    w.scratch = reinterpret_cast<double*>(p + 3 * row);
    const size_t o_tw = 3 * row + al256(4 * (size_t)batch * N * sizeof(double));
    w.twiddle = reinterpret_cast<double*>(p + o_tw);
    w.sg = reinterpret_cast<double*>(p + o_tw + al256((size_t)len * sizeof(double)));
    w.batch = batch;
    return w;
}

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int bitrev(int i, int bits) { return (int)(__brev((unsigned)i) >> (32 - bits)); }

// In-place FFT stages on LDS data z (L complex), twiddles tw[j] = e^{-2 pi i j / L}.
// dit: input bit-reversed, output natural.  dif: input natural, output bit-reversed.
__device__ void fft_dit(double2* z, const double2* __restrict__ tw, int L) {
    for (int half = 1; half < L; half <<= 1) {
        const int stride = L / (2 * half);
        for (int t = threadIdx.x; t < L / 2; t += blockDim.x) {
            const int j = t & (half - 1);
            const int a = (t - j) * 2 + j;
            const int b = a + half;
            const double2 w = tw[j * stride];
            const double2 x = z[a], y = z[b];
            const double yr = y.x * w.x - y.y * w.y, yi = y.x * w.y + y.y * w.x;
            z[a] = make_double2(x.x + yr, x.y + yi);
            z[b] = make_double2(x.x - yr, x.y - yi);
        }
        __syncthreads();
    }
}

__device__ void fft_dif(double2* z, const double2* __restrict__ tw, int L) {
    for (int half = L / 2; half >= 1; half >>= 1) {
        const int stride = L / (2 * half);
        for (int t = threadIdx.x; t < L / 2; t += blockDim.x) {
            const int j = t & (half - 1);
            const int a = (t - j) * 2 + j;
            const int b = a + half;
            const double2 w = tw[j * stride];
            const double2 x = z[a], y = z[b];
            const double dr = x.x - y.x, di = x.y - y.y;
            z[a] = make_double2(x.x + y.x, x.y + y.y);
            z[b] = make_double2(dr * w.x - di * w.y, dr * w.y + di * w.x);
        }
        __syncthreads();
    }
}

// Hilbert transform of the two rows held (bit-reversed, padded) in z:
// forward DIT, multiply by -i sgn(nu), conjugate, forward DIF.  The result
// R (bit-reversed) gives H{a}[t] = Re R / L and H{b}[t] = -Im R / L.
__device__ void hilbert_pair(double2* z, const double2* __restrict__ tw, int L) {
    fft_dit(z, tw, L);
    for (int b = threadIdx.x; b < L; b += blockDim.x) {
        double2 v = z[b];
        double2 m;
        if (b == 0 || b == L / 2) m = make_double2(0.0, 0.0);
        else if (b < L / 2) m = make_double2(v.y, -v.x);  // * (-i)
        else m = make_double2(-v.y, v.x);                 // * (+i)
        z[b] = make_double2(m.x, -m.y);                   // conjugate
    }
    __syncthreads();
    fft_dif(z, tw, L);
}

__device__ __forceinline__ double log_ratio64(double x, double iref, double floor) {
    double q = x / iref;
    if (!(q > floor && q < INFINITY)) q = floor;
    return 0.5 * log(q);
}

template <typename TIn>
__global__ __launch_bounds__(kThreads) void kk_kernel(const TIn* __restrict__ I, int64_t m0, int64_t nb, int N,
                                                      int64_t ld, const double* __restrict__ iref, double floor,
                                                      int L, int bits, int pad_mode, const double2* __restrict__ tw,
                                                      double* __restrict__ ell, double* __restrict__ phi) {
    extern __shared__ double2 z[];
    const int64_t ra = m0 + 2 * (int64_t)blockIdx.x, rb = ra + 1;
    const bool hb = 2 * (int64_t)blockIdx.x + 1 < nb;
    const int pl = (L - N) / 2;
    const TIn* xa = I + ra * ld;
    const TIn* xb = I + rb * ld;
    const int64_t la = 2 * (int64_t)blockIdx.x, lb = la + 1;  // batch-local rows
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        const int src = i - pl;
        double va = 0.0, vb = 0.0;
        if (src >= 0 && src < N) {
            va = log_ratio64(xa[src], iref[src], floor);
            vb = hb ? log_ratio64(xb[src], iref[src], floor) : 0.0;
            ell[la * N + src] = va;
            if (hb) ell[lb * N + src] = vb;
        } else if (pad_mode == 0) {
            const int e = src < 0 ? 0 : N - 1;
            va = log_ratio64(xa[e], iref[e], floor);
            vb = hb ? log_ratio64(xb[e], iref[e], floor) : 0.0;
        }
        z[bitrev(i, bits)] = make_double2(va, vb);
    }
    __syncthreads();
    hilbert_pair(z, tw, L);
    const double inv = 1.0 / L;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double2 r = z[bitrev(pl + i, bits)];
        phi[la * N + i] = r.x * inv;
        if (hb) phi[lb * N + i] = -r.y * inv;
    }
}

// ALS: one lane per spectrum.  y and the result z are row-major (batch x N);
// the LDL^T state (D, l1, u) and the previous iterate are interleaved
// (index j * nb + m).  The recurrence is the one of the host detrender.
constexpr int JC = 16;  // wavenumbers per LDS tile

__global__ __launch_bounds__(kThreads) void als_kernel(const double* __restrict__ y, double* __restrict__ zout,
                                                       int64_t nb, int N, double lam, double p, int iters,
                                                       double* __restrict__ st) {
    __shared__ double tile[kThreads][JC + 1];
    const int lane = threadIdx.x;
    const int64_t mb0 = (int64_t)blockIdx.x * kThreads;
    const int64_t m = mb0 + lane;
    const bool active = m < nb;
    double* sD = st;
    double* sL1 = st + (size_t)N * nb;
    double* sU = st + 2 * (size_t)N * nb;
    double* sZ = st + 3 * (size_t)N * nb;
    auto IX = [&](int j) { return (size_t)j * nb + m; };
    const int tr = threadIdx.x / JC, tc = threadIdx.x % JC;  // cooperative tile mapping

    for (int it = 0; it < iters; ++it) {
        // ---- forward: factorisation and L u = w y ----
        double dm1 = 0.0, dm2 = 0.0;    // D[j-1], D[j-2]
        double l1m1 = 0.0;              // l1[j] computed at j-1 (= l1 of the current j)
        double l2c = 0.0, l2n = 0.0;    // l2[j], l2[j+1]
        double um1 = 0.0, um2 = 0.0;    // u[j-1], u[j-2]
        for (int j0 = 0; j0 < N; j0 += JC) {
            __syncthreads();
            for (int r = tr; r < kThreads; r += kThreads / JC) {
                const int64_t row = mb0 + r;
                const int col = j0 + tc;
                tile[r][tc] = (row < nb && col < N) ? y[row * N + col] : 0.0;
            }
            __syncthreads();
            if (!active) continue;
            const int jend = min(JC, N - j0);
            for (int jj = 0; jj < jend; ++jj) {
                const int j = j0 + jj;
                const double yj = tile[lane][jj];
                double w = 1.0;
                if (it > 0) w = (yj > sZ[IX(j)]) ? p : 1.0 - p;
                double c0 = 6.0;
                if (j == 0 || j == N - 1) c0 = 1.0;
                else if (j == 1 || j == N - 2) c0 = 5.0;
                double d = w + lam * c0;
                const double l1j = l1m1;
                if (j >= 1) d -= l1j * l1j * dm1;
                if (j >= 2) d -= l2c * l2c * dm2;
                // l1[j+1] and l2[j+2]
                double l1n = 0.0;
                if (j + 1 < N) {
                    const double c1 = (j == 0 || j == N - 2) ? -2.0 : -4.0;
                    double v = lam * c1;
                    if (j >= 1) v -= l2n * l1j * dm1;
                    l1n = v / d;
                }
                const double l2nn = (j + 2 < N) ? lam / d : 0.0;
                double u = w * yj;
                if (j >= 1) u -= l1j * um1;
                if (j >= 2) u -= l2c * um2;
                sD[IX(j)] = d;
                sL1[IX(j)] = l1j;
                sU[IX(j)] = u;
                um2 = um1;
                um1 = u;
                dm2 = dm1;
                dm1 = d;
                l1m1 = l1n;
                l2c = l2n;
                l2n = l2nn;
            }
        }
        // ---- backward: D v = u, L^T z = v ----
        const bool last = (it == iters - 1);
        double z1 = 0.0, z2 = 0.0;        // z[j+1], z[j+2]
        double l1p1 = 0.0;                // l1[j+1]
        const int nch = (N + JC - 1) / JC;
        for (int cidx = nch - 1; cidx >= 0; --cidx) {
            const int j0 = cidx * JC;
            const int jend = min(JC, N - j0);
            if (active) {
                for (int jj = jend - 1; jj >= 0; --jj) {
                    const int j = j0 + jj;
                    const double d = sD[IX(j)];
                    double v = sU[IX(j)] / d;
                    if (j + 1 < N) v -= l1p1 * z1;          // l1[j+1] z[j+1]
                    if (j + 2 < N) v -= (lam / d) * z2;     // l2[j+2] = lam / D[j]
                    z2 = z1;
                    z1 = v;
                    l1p1 = sL1[IX(j)];
                    sZ[IX(j)] = v;
                    if (last) tile[lane][jj] = v;
                }
            }
            if (last) {
                __syncthreads();
                for (int r = tr; r < kThreads; r += kThreads / JC) {
                    const int64_t row = mb0 + r;
                    const int col = j0 + tc;
                    if (row < nb && tc < jend) zout[row * N + col] = tile[r][tc];
                }
                __syncthreads();
            }
        }
    }
}

// SEC: H{phi_err}, rho = l + H{phi_err}, rho -= trend(rho), epilogue.
// The Savitzky-Golay trendline is evaluated from running moment sums:
// for the window of half width h around i, m_p = sum_x (x/h)^p y(i+x),
// value = sum_p g_p m_p with g = row 0 of (V^T V)^-1; near the ends the
// first / last full window is fitted and evaluated at t = (i - centre)/h.
template <typename TOut>
__global__ __launch_bounds__(kThreads) void sec_kernel(int64_t m0, int64_t nb, int N, int L, int bits, int pad_mode,
                                                       const double2* __restrict__ tw, const double* __restrict__ ell,
                                                       const double* __restrict__ phi,
                                                       const double* __restrict__ err, int sec_mode, int sec_re,
                                                       int half, int order, const double* __restrict__ ginv,
                                                       int plane, TOut* __restrict__ out, int64_t ld_out) {
    extern __shared__ double2 z[];
    __shared__ double part[4][kThreads + 1];
    const int64_t la = 2 * (int64_t)blockIdx.x, lb = la + 1;
    const bool hb = lb < nb;
    const int pl = (L - N) / 2;
    for (int i = threadIdx.x; i < L; i += blockDim.x) {
        int src = i - pl;
        double va = 0.0, vb = 0.0;
        if (src >= 0 && src < N) {
            va = err[la * N + src];
            vb = hb ? err[lb * N + src] : 0.0;
        } else if (pad_mode == 0) {
            src = src < 0 ? 0 : N - 1;
            va = err[la * N + src];
            vb = hb ? err[lb * N + src] : 0.0;
        }
        z[bitrev(i, bits)] = make_double2(va, vb);
    }
    __syncthreads();
    hilbert_pair(z, tw, L);
    // LDS after the transform: [4 prefix arrays of N + 1][rho_a | rho_b]
    const double inv = 1.0 / L;
    double* rho = reinterpret_cast<double*>(z) + 4 * (N + 1);
    double hv[2][16];
    int cnt = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x, ++cnt) {
        const double2 r = z[bitrev(pl + i, bits)];
        hv[0][cnt] = r.x * inv;
        hv[1][cnt] = -r.y * inv;
    }
    __syncthreads();
    cnt = 0;
    for (int i = threadIdx.x; i < N; i += blockDim.x, ++cnt) {
        rho[i] = ell[la * N + i] + hv[0][cnt];
        rho[N + i] = hb ? ell[lb * N + i] + hv[1][cnt] : 0.0;
    }
    __syncthreads();
    double* pre = reinterpret_cast<double*>(z);  // 4 prefix arrays of N + 1
    for (int s = 0; s < (hb ? 2 : 1); ++s) {
        double* y = rho + (size_t)s * N;
        const int64_t lrow = la + s;
        TOut* orow = out + (m0 + lrow) * ld_out;
        // the corrected spectrum K' = exp(rho) exp(i (phi - phi_err)); the
        // real-part form of SEC (Eq. 4-5) divides it by the trendline of
        // Re K', so the trendline then acts on Re K' instead of rho
        auto corrected = [&](int i, int cnt_i, double trend) -> TOut {
            const double ph = phi[lrow * N + i] - err[lrow * N + i];
            if (sec_re) {
                const double mag = exp(ell[lrow * N + i] + hv[s][cnt_i]);
                return (TOut)(plane == 0 ? mag * sin(ph) / trend
                                         : (plane == 1 ? mag * cos(ph) / trend : mag / fabs(trend)));
            }
            const double mag = exp(y[i] - trend);
            return (TOut)(plane == 0 ? mag * sin(ph) : (plane == 1 ? mag * cos(ph) : mag));
        };
        if (sec_re) {
            for (int i = threadIdx.x; i < N; i += blockDim.x)
                y[i] = exp(y[i]) * cos(phi[lrow * N + i] - err[lrow * N + i]);
            __syncthreads();
        }
        if (sec_mode == 1) {
            double acc = 0.0;
            for (int i = threadIdx.x; i < N; i += blockDim.x) acc += y[i];
            part[0][threadIdx.x] = acc;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int q = 0; q < (int)blockDim.x; ++q) t += part[0][q];
                part[1][0] = t / N;
            }
            __syncthreads();
            const double mean = part[1][0];
            int ci = 0;
            for (int i = threadIdx.x; i < N; i += blockDim.x, ++ci) orow[i] = corrected(i, ci, mean);
            __syncthreads();
            continue;
        }
        // prefix sums Q_q[i] = sum_{j<i} ((j - c)/h)^q y_j, q <= order
        const double c = 0.5 * (N - 1);
        const double invh = 1.0 / half;
        const int seg = (N + blockDim.x - 1) / blockDim.x;
        const int a0 = threadIdx.x * seg, a1 = min(N, a0 + seg);
        double ls[4] = {0, 0, 0, 0};
        for (int j = a0; j < a1; ++j) {
            const double x = (j - c) * invh;
            double pw = y[j];
            for (int q = 0; q <= order; ++q) { ls[q] += pw; pw *= x; }
        }
        for (int q = 0; q <= order; ++q) part[q][threadIdx.x] = ls[q];
        __syncthreads();
        if (threadIdx.x < 4) {
            const int q = threadIdx.x;
            if (q <= order) {
                double run = 0.0;
                for (int t = 0; t < (int)blockDim.x; ++t) {
                    const double v = part[q][t];
                    part[q][t] = run;
                    run += v;
                }
            }
        }
        __syncthreads();
        {
            double run[4];
            for (int q = 0; q <= order; ++q) run[q] = part[q][threadIdx.x];
            for (int j = a0; j < a1; ++j) {
                const double x = (j - c) * invh;
                double pw = y[j];
                for (int q = 0; q <= order; ++q) {
                    pre[q * (N + 1) + j] = run[q];
                    run[q] += pw;
                    pw *= x;
                }
            }
            if (a1 == N && a0 < a1)
                for (int q = 0; q <= order; ++q) pre[q * (N + 1) + N] = run[q];
        }
        __syncthreads();
        const int m = order + 1;
        int ci = 0;
        for (int i = threadIdx.x; i < N; i += blockDim.x, ++ci) {
            // window [s0, s0 + 2h] and the point's offset from its centre
            int s0 = i - half;
            if (s0 < 0) s0 = 0;
            if (s0 > N - (2 * half + 1)) s0 = N - (2 * half + 1);
            const double ctr = s0 + half;
            // W_q = sum over window of ((j - c)/h)^q y_j ; convert to moments about ctr
            double W[4], mom[4];
            for (int q = 0; q < m; ++q) W[q] = pre[q * (N + 1) + s0 + 2 * half + 1] - pre[q * (N + 1) + s0];
            const double dd = (ctr - c) * invh;  // (j - ctr)/h = (j - c)/h - dd
            for (int pp = 0; pp < m; ++pp) {
                double acc = 0.0, binom = 1.0;
                for (int q = 0; q <= pp; ++q) {
                    // C(pp, q) (-dd)^(pp-q) W_q
                    double pw = 1.0;
                    for (int e = 0; e < pp - q; ++e) pw *= -dd;
                    acc += binom * pw * W[q];
                    binom = binom * (pp - q) / (q + 1);
                }
                mom[pp] = acc;
            }
            const double t = (i - ctr) * invh;
            // value = tvec^T Ginv mom
            double val = 0.0, tp = 1.0;
            for (int r = 0; r < m; ++r) {
                double g = 0.0;
                for (int q = 0; q < m; ++q) g += ginv[r * m + q] * mom[q];
                val += tp * g;
                tp *= t;
            }
            orow[i] = corrected(i, ci, val);
        }
        __syncthreads();
    }
}

}  // namespace

hipError_t run(const Layout& ws, const Config& cfg, const void* d_I, bool in_f64, int64_t M, int64_t ld,
               const double* h_iref, void* d_out, bool out_f64, int64_t ld_out, hipStream_t s, std::string* why) {
    const int N = cfg.N, L = cfg.len;
    int bits = 0;
    while ((1 << bits) < L) ++bits;
    if ((1 << bits) != L || L < N) {
        if (why) *why = "fft length must be a power of two >= N";
        return hipErrorInvalidValue;
    }
    if ((size_t)L * 16 > 160 * 1024) {
        if (why) *why = "fft length above the LDS capacity (8192)";
        return hipErrorInvalidValue;
    }
    if (cfg.sec_mode == 0 && (cfg.order > 3 || cfg.order < 0)) {
        if (why) *why = "Savitzky-Golay order above 3 not supported on the device path";
        return hipErrorInvalidValue;
    }
    if (N > 16 * kThreads) {
        if (why) *why = "N above 4096";
        return hipErrorInvalidValue;
    }
    const int64_t batch = ws.batch;
    if (batch < 1 || !ws.ell) {
        if (why) *why = "no workspace";
        return hipErrorInvalidValue;
    }
    hipError_t e;
    // twiddle table of the length (copied with the call: the workspace is
    // the caller's and holds nothing between calls)
    std::vector<double> tw(L);
    for (int j = 0; j < L / 2; ++j) {
        const double a = -2.0 * M_PI * (double)j / (double)L;
        tw[2 * j] = std::cos(a);
        tw[2 * j + 1] = std::sin(a);
    }
    if ((e = hipMemcpyAsync(ws.twiddle, tw.data(), L * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    // (V^T V)^-1 of the scaled Vandermonde of the window and I_ref
    const int half = cfg.window / 2, m = cfg.order + 1;
    std::vector<double> host((size_t)N + 16, 0.0);
    for (int j = 0; j < N; ++j) host[j] = h_iref[j];
    if (cfg.sec_mode == 0) {
        std::vector<double> g((size_t)m * m, 0.0), inv((size_t)m * m, 0.0);
        for (int x = -half; x <= half; ++x) {
            const double t = (double)x / half;
            std::vector<double> pw(2 * m - 1);
            double v = 1.0;
            for (int q = 0; q < 2 * m - 1; ++q) { pw[q] = v; v *= t; }
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) g[r * m + c] += pw[r + c];
        }
        // Gauss-Jordan inverse (m <= 4)
        for (int r = 0; r < m; ++r) inv[r * m + r] = 1.0;
        for (int c = 0; c < m; ++c) {
            int piv = c;
            for (int r = c + 1; r < m; ++r)
                if (std::fabs(g[r * m + c]) > std::fabs(g[piv * m + c])) piv = r;
            for (int q = 0; q < m; ++q) {
                std::swap(g[c * m + q], g[piv * m + q]);
                std::swap(inv[c * m + q], inv[piv * m + q]);
            }
            const double d = g[c * m + c];
            for (int q = 0; q < m; ++q) { g[c * m + q] /= d; inv[c * m + q] /= d; }
            for (int r = 0; r < m; ++r) {
                if (r == c) continue;
                const double f = g[r * m + c];
                for (int q = 0; q < m; ++q) { g[r * m + q] -= f * g[c * m + q]; inv[r * m + q] -= f * inv[c * m + q]; }
            }
        }
        for (int q = 0; q < m * m; ++q) host[N + q] = inv[q];
    }
    if ((e = hipMemcpyAsync(ws.sg, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, s)) != hipSuccess)
        return e;
    const double* d_iref = ws.sg;
    const double* d_ginv = ws.sg + N;
    const size_t lds = std::max((size_t)L * sizeof(double2), (size_t)(6 * N + 4) * sizeof(double));
    if (lds > 160 * 1024) {
        if (why) *why = "spectrum too long for the LDS-resident transform";
        return hipErrorInvalidValue;
    }
    if (in_f64)
        hipFuncSetAttribute(reinterpret_cast<const void*>(kk_kernel<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else
        hipFuncSetAttribute(reinterpret_cast<const void*>(kk_kernel<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (out_f64)
        hipFuncSetAttribute(reinterpret_cast<const void*>(sec_kernel<double>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    else
        hipFuncSetAttribute(reinterpret_cast<const void*>(sec_kernel<float>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    const int iters = (cfg.detrend == 1) ? 1 : cfg.iters;
    const double p = (cfg.detrend == 1) ? 0.5 : cfg.p;
    for (int64_t m0 = 0; m0 < M; m0 += batch) {
        const int64_t nb = std::min(batch, M - m0);
        const unsigned pairs = (unsigned)((nb + 1) / 2);
        if (in_f64)
            hipLaunchKernelGGL(kk_kernel<double>, dim3(pairs), dim3(kThreads), lds, s,
                               static_cast<const double*>(d_I), m0, nb, N, ld, d_iref, cfg.floor, L, bits,
                               cfg.pad_mode, reinterpret_cast<const double2*>(ws.twiddle), ws.ell, ws.phi);
        else
            hipLaunchKernelGGL(kk_kernel<float>, dim3(pairs), dim3(kThreads), lds, s, static_cast<const float*>(d_I),
                               m0, nb, N, ld, d_iref, cfg.floor, L, bits, cfg.pad_mode,
                               reinterpret_cast<const double2*>(ws.twiddle), ws.ell, ws.phi);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(als_kernel, dim3((unsigned)((nb + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, ws.phi,
                           ws.err, nb, N, cfg.lam, p, iters, ws.scratch);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (out_f64)
            hipLaunchKernelGGL(sec_kernel<double>, dim3(pairs), dim3(kThreads), lds, s, m0, nb, N, L, bits,
                               cfg.pad_mode, reinterpret_cast<const double2*>(ws.twiddle), ws.ell, ws.phi, ws.err,
                               cfg.sec_mode, cfg.sec_re, half, cfg.order, d_ginv, cfg.plane, static_cast<double*>(d_out),
                               ld_out);
        else
            hipLaunchKernelGGL(sec_kernel<float>, dim3(pairs), dim3(kThreads), lds, s, m0, nb, N, L, bits,
                               cfg.pad_mode, reinterpret_cast<const double2*>(ws.twiddle), ws.ell, ws.phi, ws.err,
                               cfg.sec_mode, cfg.sec_re, half, cfg.order, d_ginv, cfg.plane, static_cast<float*>(d_out),
                               ld_out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace plain
}  // namespace fkk
