// FP64 host numerics of fKK-EC on the basis vectors and the Gram matrix.
// See host_math.h for the contracts.
#include "host_math.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <limits>
#include <memory>
#include <chrono>
#include <mutex>
#include <thread>

namespace fkk {

using cplx = std::complex<double>;

// ---------------------------------------------------------------------------
// Host thread pool shared by all host stages.
// ---------------------------------------------------------------------------
namespace {

// Fork-join pool whose workers spin between back-to-back parallel regions
// (the tridiagonalisation issues two regions per column) and sleep once no
// region has come for about 2 ms, so that they do not hold the host's cores
// through the device stages of a fit (15 spinning workers left the calling
// thread and the runtime's threads waiting for a core).
class Pool {
  public:
    explicit Pool(int n) : n_(std::max(1, n)) {
        for (int t = 1; t < n_; ++t) th_.emplace_back([this, t] { worker(t); });
    }
    ~Pool() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
            gen_.fetch_add(1);
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    int size() const { return n_; }
    // run fn(tid, nthreads) on every thread, return when all are done.
    // Callers on different host threads (one context each) take turns: the
    // job slot, the generation and the completion count are the pool's own.
    void run(const std::function<void(int, int)>& fn) {
        std::lock_guard<std::mutex> turn(run_mu_);
        job_ = &fn;
        done_.store(0);
        {
            std::lock_guard<std::mutex> g(mu_);
            gen_.fetch_add(1);
        }
        cv_.notify_all();
        fn(0, n_);
        while (done_.load(std::memory_order_acquire) != n_ - 1) std::this_thread::yield();
    }

  private:
    void worker(int tid) {
        int64_t seen = 0;
        for (;;) {
            const auto t0 = std::chrono::steady_clock::now();
            int spins = 0;
            while (gen_.load(std::memory_order_acquire) == seen) {
                if ((++spins & 63) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000)) {
                    std::unique_lock<std::mutex> lk(mu_);
                    cv_.wait(lk, [&] { return gen_.load() != seen; });
                    break;
                }
                std::this_thread::yield();
            }
            seen = gen_.load(std::memory_order_acquire);
            if (stop_) return;
            (*job_)(tid, n_);
            done_.fetch_add(1, std::memory_order_release);
        }
    }
    int n_;
    std::vector<std::thread> th_;
    std::atomic<int64_t> gen_{0};
    std::atomic<int> done_{0};
    const std::function<void(int, int)>* job_ = nullptr;
    std::mutex mu_;
    std::mutex run_mu_;  // one job at a time
    std::condition_variable cv_;
    bool stop_ = false;
};

void split(int lo, int hi, int tid, int nt, int* a, int* b) {
    const int len = hi - lo;
    *a = lo + (int)((int64_t)len * tid / nt);
    *b = lo + (int)((int64_t)len * (tid + 1) / nt);
}

// Created on first use and never destroyed: its workers sleep in the pool
// until the process ends, so no static destructor joins threads while the
// process (and the runtimes loaded into it) is being torn down.
Pool& host_pool() {
    static Pool* pool = new Pool([] {
        unsigned hw = std::thread::hardware_concurrency();
        return (int)std::min(16u, hw == 0 ? 1u : hw);
    }());
    return *pool;
}

}  // namespace

// Rows [0, rows) split over the pool.
void parallel_rows(int rows, const std::function<void(int, int)>& body) {
    Pool& pool = host_pool();
    if (rows <= 1 || pool.size() == 1) {
        body(0, rows);
        return;
    }
    pool.run([&](int tid, int nthr) {
        int r0, r1;
        split(0, rows, tid, nthr, &r0, &r1);
        if (r0 < r1) body(r0, r1);
    });
}


int default_fft_len(int n) {
    int len = 1;
    while (len < 3 * n) len *= 2;
    return len;
}

double default_als_lambda(int n) {
    const double r = n / 1000.0;
    return 1.0e5 * r * r * r * r;
}

int default_sg_window(int n) {
    int w = n / 2;
    if (w % 2 == 0) w -= 1;
    return std::max(w, 3);
}

// ---------------------------------------------------------------------------
// Radix-2 complex FFT (decimation in time, iterative), length a power of two.
// ---------------------------------------------------------------------------
namespace {

struct FftPlan {
    int n = 0;
    std::vector<int> rev;
    std::vector<cplx> tw;  // exp(-2 pi i j / n), j < n/2
    std::vector<double> stw;  // per stage (half = 1, 2, 4, ...): the half twiddles it uses, re/im interleaved
    explicit FftPlan(int len) : n(len), rev(len), tw(len / 2) {
        int bits = 0;
        while ((1 << bits) < n) ++bits;
        for (int i = 0; i < n; ++i) {
            int r = 0;
            for (int b = 0; b < bits; ++b)
                if (i & (1 << b)) r |= 1 << (bits - 1 - b);
            rev[i] = r;
        }
        for (int j = 0; j < n / 2; ++j) {
            const double ang = -2.0 * M_PI * (double)j / (double)n;
            tw[j] = cplx(std::cos(ang), std::sin(ang));
        }
        stw.resize(2 * (size_t)std::max(n - 1, 1));
        for (int half = 1; half < n; half *= 2)
            for (int j = 0; j < half; ++j) {
                stw[2 * (size_t)(half - 1 + j)] = tw[(size_t)j * (n / (2 * half))].real();
                stw[2 * (size_t)(half - 1 + j) + 1] = tw[(size_t)j * (n / (2 * half))].imag();
            }
    }
    void run(cplx* a, bool inverse) const {
        double* z = reinterpret_cast<double*>(a);
        for (int i = 0; i < n; ++i)
            if (i < rev[i]) std::swap(a[i], a[rev[i]]);
        const double sgn = inverse ? -1.0 : 1.0;
        for (int half = 1; half < n; half *= 2) {
            const double* w = &stw[2 * (size_t)(half - 1)];
            for (int s = 0; s < n; s += 2 * half) {
                for (int j = 0; j < half; ++j) {
                    const double wr = w[2 * j], wi = sgn * w[2 * j + 1];
                    double* x = z + 2 * (s + j);
                    double* y = z + 2 * (s + j + half);
                    const double tr = wr * y[0] - wi * y[1], ti = wr * y[1] + wi * y[0];
                    y[0] = x[0] - tr;
                    y[1] = x[1] - ti;
                    x[0] += tr;
                    x[1] += ti;
                }
            }
        }
        if (inverse) {
            const double inv = 1.0 / n;
            for (int i = 0; i < 2 * n; ++i) z[i] *= inv;
        }
    }
};

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Plans depend only on the length: built once per length and shared.
std::shared_ptr<const FftPlan> fft_plan(int len) {
    static std::mutex mu;
    static std::vector<std::shared_ptr<const FftPlan>> plans;
    std::lock_guard<std::mutex> g(mu);
    for (const auto& p : plans)
        if (p->n == len) return p;
    plans.push_back(std::make_shared<const FftPlan>(len));
    return plans.back();
}

}  // namespace

void hilbert_rows(const double* x, double* y, int rows, int n, int len, int pad_mode) {
    if (!is_pow2(len) || len < n) return;
    const std::shared_ptr<const FftPlan> plan_p = fft_plan(len);
    const FftPlan& plan = *plan_p;
    const int pl = (len - n) / 2;
    // Two real rows per complex transform: H is real and complex-linear, so
    // H{a + i b} = H{a} + i H{b}.
    const int pairs = (rows + 1) / 2;
    parallel_rows(pairs, [&](int p0, int p1) {
        std::vector<cplx> buf(len);
        auto pad_value = [&](const double* row, int i) -> double {
            const int src = i - pl;
            if (src >= 0 && src < n) return row[src];
            if (pad_mode == 1) return 0.0;
            return src < 0 ? row[0] : row[n - 1];
        };
        for (int pr = p0; pr < p1; ++pr) {
            const int r = 2 * pr;
            const double* ra = x + (size_t)r * n;
            const double* rb = (r + 1 < rows) ? x + (size_t)(r + 1) * n : nullptr;
            for (int i = 0; i < len; ++i) buf[i] = cplx(pad_value(ra, i), rb ? pad_value(rb, i) : 0.0);
            plan.run(buf.data(), false);
            buf[0] = 0.0;
            buf[len / 2] = 0.0;
            for (int b = 1; b < len / 2; ++b) buf[b] = cplx(buf[b].imag(), -buf[b].real());        // * (-i)
            for (int b = len / 2 + 1; b < len; ++b) buf[b] = cplx(-buf[b].imag(), buf[b].real());  // * (+i)
            plan.run(buf.data(), true);
            for (int i = 0; i < n; ++i) {
                y[(size_t)r * n + i] = buf[pl + i].real();
                if (rb) y[(size_t)(r + 1) * n + i] = buf[pl + i].imag();
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Detrending: (diag(w) + lam D^T D) z = w y, D the second-difference matrix.
// The matrix is symmetric positive definite and pentadiagonal; it is solved
// by an LDL^T factorisation with unit lower factor of bandwidth two.
// ---------------------------------------------------------------------------
namespace {

void penta_solve(const double* w, const double* y, double* z, int n, double lam,
                 std::vector<double>& dd, std::vector<double>& l1, std::vector<double>& l2) {
    dd.assign(n, 0.0);
    l1.assign(n + 1, 0.0);
    l2.assign(n + 2, 0.0);
    auto a0 = [&](int i) {  // diagonal of lam D^T D plus w
        double c = 6.0;
        if (i == 0 || i == n - 1) c = 1.0;
        else if (i == 1 || i == n - 2) c = 5.0;
        return w[i] + lam * c;
    };
    auto a1 = [&](int i) {  // A[i+1][i]
        double c = -4.0;
        if (i == 0 || i == n - 2) c = -2.0;
        return lam * c;
    };
    const double a2 = lam;  // A[i+2][i]
    for (int i = 0; i < n; ++i) {
        double d = a0(i);
        if (i >= 1) d -= l1[i] * l1[i] * dd[i - 1];
        if (i >= 2) d -= l2[i] * l2[i] * dd[i - 2];
        dd[i] = d;
        if (i + 1 < n) {
            double v = a1(i);
            if (i >= 1) v -= l2[i + 1] * l1[i] * dd[i - 1];
            l1[i + 1] = v / d;
        }
        if (i + 2 < n) l2[i + 2] = a2 / d;
    }
    // L u = w y ; D v = u ; L^T z = v
    for (int i = 0; i < n; ++i) {
        double u = w[i] * y[i];
        if (i >= 1) u -= l1[i] * z[i - 1];
        if (i >= 2) u -= l2[i] * z[i - 2];
        z[i] = u;
    }
    for (int i = 0; i < n; ++i) z[i] /= dd[i];
    for (int i = n - 1; i >= 0; --i) {
        double v = z[i];
        if (i + 1 < n) v -= l1[i + 1] * z[i + 1];
        if (i + 2 < n) v -= l2[i + 2] * z[i + 2];
        z[i] = v;
    }
}

}  // namespace

void detrend_row(const double* y, double* z, int n, int mode, double lam, double p, int n_iter) {
    std::vector<double> w(n, 1.0), dd, l1, l2;
    if (n < 4) {  // D^T D needs at least 4 points to be pentadiagonal
        for (int i = 0; i < n; ++i) z[i] = y[i];
        return;
    }
    const int iters = (mode == 1) ? 1 : n_iter;
    for (int it = 0; it < iters; ++it) {
        penta_solve(w.data(), y, z, n, lam, dd, l1, l2);
        for (int i = 0; i < n; ++i) w[i] = (y[i] > z[i]) ? p : 1.0 - p;
    }
}

namespace {

// detrend_row on four rows at once: the same operations per row, with the
// four factorisation and substitution chains interleaved (their divisions
// and dependent updates overlap).  Rows are independent, so the results
// equal four calls of detrend_row.
void detrend_row4(const double* const* y, double* const* z, int n, int mode, double lam, double p, int n_iter) {
    constexpr int R = 4;
    std::vector<double> w((size_t)R * n, 1.0), dd((size_t)R * n), l1((size_t)R * (n + 1)), l2((size_t)R * (n + 2));
    const int iters = (mode == 1) ? 1 : n_iter;
    const double a2 = lam;
    for (int it = 0; it < iters; ++it) {
        std::fill(l1.begin(), l1.end(), 0.0);
        std::fill(l2.begin(), l2.end(), 0.0);
        for (int i = 0; i < n; ++i) {
            double c0 = 6.0;
            if (i == 0 || i == n - 1) c0 = 1.0;
            else if (i == 1 || i == n - 2) c0 = 5.0;
            double c1 = -4.0;
            if (i == 0 || i == n - 2) c1 = -2.0;
            for (int r = 0; r < R; ++r) {
                double* D = &dd[(size_t)r * n];
                double* L1 = &l1[(size_t)r * (n + 1)];
                double* L2 = &l2[(size_t)r * (n + 2)];
                double d = w[(size_t)r * n + i] + lam * c0;
                if (i >= 1) d -= L1[i] * L1[i] * D[i - 1];
                if (i >= 2) d -= L2[i] * L2[i] * D[i - 2];
                D[i] = d;
                if (i + 1 < n) {
                    double v = lam * c1;
                    if (i >= 1) v -= L2[i + 1] * L1[i] * D[i - 1];
                    L1[i + 1] = v / d;
                }
                if (i + 2 < n) L2[i + 2] = a2 / d;
            }
        }
        for (int i = 0; i < n; ++i)
            for (int r = 0; r < R; ++r) {
                const double* L1 = &l1[(size_t)r * (n + 1)];
                const double* L2 = &l2[(size_t)r * (n + 2)];
                double* zr = z[r];
                double u = w[(size_t)r * n + i] * y[r][i];
                if (i >= 1) u -= L1[i] * zr[i - 1];
                if (i >= 2) u -= L2[i] * zr[i - 2];
                zr[i] = u;
            }
        for (int r = 0; r < R; ++r)
            for (int i = 0; i < n; ++i) z[r][i] /= dd[(size_t)r * n + i];
        for (int i = n - 1; i >= 0; --i)
            for (int r = 0; r < R; ++r) {
                const double* L1 = &l1[(size_t)r * (n + 1)];
                const double* L2 = &l2[(size_t)r * (n + 2)];
                double* zr = z[r];
                double v = zr[i];
                if (i + 1 < n) v -= L1[i + 1] * zr[i + 1];
                if (i + 2 < n) v -= L2[i + 2] * zr[i + 2];
                zr[i] = v;
            }
        for (int r = 0; r < R; ++r)
            for (int i = 0; i < n; ++i) w[(size_t)r * n + i] = (y[r][i] > z[r][i]) ? p : 1.0 - p;
    }
}

}  // namespace

void detrend_rows(const double* y, double* z, int rows, int n, int mode, double lam, double p, int n_iter) {
    // rows 4g..4g+3 go through detrend_row4, the rows - rows % 4 .. rows-1
    // tail through detrend_row: fixed by the row count, not by the threads
    const int groups = (n >= 4) ? rows / 4 : 0;
    parallel_rows(groups + (rows - 4 * groups), [&](int t0, int t1) {
        for (int t = t0; t < t1; ++t) {
            if (t < groups) {
                const int r = 4 * t;
                const double* ys[4] = {y + (size_t)r * n, y + (size_t)(r + 1) * n, y + (size_t)(r + 2) * n,
                                       y + (size_t)(r + 3) * n};
                double* zs[4] = {z + (size_t)r * n, z + (size_t)(r + 1) * n, z + (size_t)(r + 2) * n,
                                 z + (size_t)(r + 3) * n};
                detrend_row4(ys, zs, n, mode, lam, p, n_iter);
            } else {
                const int r = 4 * groups + (t - groups);
                detrend_row(y + (size_t)r * n, z + (size_t)r * n, n, mode, lam, p, n_iter);
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Savitzky-Golay trendline.  The weights of output point i are those of the
// least-squares polynomial of degree `order` through the window evaluated at
// i: c = V (V^T V)^-1 e_0 with V the Vandermonde matrix of the window
// positions relative to i (scaled by the half window for conditioning).
// ---------------------------------------------------------------------------
namespace {

// Solve the small SPD system g x = b in place (Gaussian elimination with
// partial pivoting; g is (order+1)^2).
void small_solve(std::vector<double>& g, std::vector<double>& b, int m) {
    for (int c = 0; c < m; ++c) {
        int piv = c;
        for (int r = c + 1; r < m; ++r)
            if (std::fabs(g[r * m + c]) > std::fabs(g[piv * m + c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < m; ++j) std::swap(g[c * m + j], g[piv * m + j]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < m; ++r) {
            const double f = g[r * m + c] / g[c * m + c];
            for (int j = c; j < m; ++j) g[r * m + j] -= f * g[c * m + j];
            b[r] -= f * b[c];
        }
    }
    for (int c = m - 1; c >= 0; --c) {
        double v = b[c];
        for (int j = c + 1; j < m; ++j) v -= g[c * m + j] * b[j];
        b[c] = v / g[c * m + c];
    }
}

void sg_weights(int start, int window, int at, int order, double scale, double* out) {
    const int m = order + 1;
    std::vector<double> g(m * m, 0.0), b(m, 0.0), pw(2 * m - 1);
    for (int j = 0; j < window; ++j) {
        const double x = (start + j - at) / scale;
        double pi = 1.0;
        for (int e = 0; e < 2 * m - 1; ++e) { pw[e] = pi; pi *= x; }
        for (int r = 0; r < m; ++r)
            for (int c = 0; c < m; ++c) g[r * m + c] += pw[r + c];
    }
    b[0] = 1.0;
    small_solve(g, b, m);  // b = (V^T V)^-1 e0
    for (int j = 0; j < window; ++j) {
        const double x = (start + j - at) / scale;
        double pi = 1.0, v = 0.0;
        for (int e = 0; e < m; ++e) { v += b[e] * pi; pi *= x; }
        out[j] = v;
    }
}

}  // namespace

void trendline_rows(const double* x, double* y, int rows, int n, int mode, int window, int order) {
    if (mode == 1) {
        for (int r = 0; r < rows; ++r) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += x[(size_t)r * n + i];
            s /= n;
            for (int i = 0; i < n; ++i) y[(size_t)r * n + i] = s;
        }
        return;
    }
    const int half = window / 2;
    // Weight tables depend only on (n, window, order): build once, reuse.
    struct Tables {
        int n = -1, window = -1, order = -1;
        // wmid: interior weights; emat: (order+1) x window operator from a
        // window's values to the coefficients of its least-squares polynomial
        // in (position - window centre) / scale; epow: for each edge output
        // (left 0..half-1, then right n-half..n-1) the powers of its offset
        std::vector<double> wmid, emat, epow;
    };
    static std::mutex cache_mu;
    static std::shared_ptr<const Tables> cache;
    std::shared_ptr<const Tables> tp;
    {
        std::lock_guard<std::mutex> g(cache_mu);
        if (cache && cache->n == n && cache->window == window && cache->order == order) tp = cache;
    }
    if (!tp) {
        Tables t;
        const double scale = std::max(1, half);
        t.wmid.resize(window);
        sg_weights(0, window, half, order, scale, t.wmid.data());
        // edges ("interp"): the polynomial fitted to the first (last) window,
        // evaluated at the edge positions; its coefficients are computed once
        // per row and side instead of one window-long sum per edge point
        const int m = order + 1;
        std::vector<double> vp((size_t)window * m), gm((size_t)m * m, 0.0);
        for (int j = 0; j < window; ++j) {
            const double u = (j - half) / scale;
            double pw = 1.0;
            for (int e = 0; e < m; ++e) {
                vp[(size_t)j * m + e] = pw;
                pw *= u;
            }
        }
        for (int j = 0; j < window; ++j)
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) gm[r * m + c] += vp[(size_t)j * m + r] * vp[(size_t)j * m + c];
        t.emat.assign((size_t)m * window, 0.0);
        for (int k = 0; k < m; ++k) {
            std::vector<double> g2(gm), bk(m, 0.0);
            bk[k] = 1.0;
            small_solve(g2, bk, m);  // row k of (V^T V)^-1 (symmetric)
            for (int j = 0; j < window; ++j) {
                double v = 0.0;
                for (int l = 0; l < m; ++l) v += bk[l] * vp[(size_t)j * m + l];
                t.emat[(size_t)k * window + j] = v;
            }
        }
        t.epow.resize((size_t)2 * half * m);
        for (int i = 0; i < half; ++i) {
            const double ul = (i - half) / scale, ur = (i + 1) / scale;  // left: position i; right: n - half + i
            double pl = 1.0, pr = 1.0;
            for (int e = 0; e < m; ++e) {
                t.epow[(size_t)i * m + e] = pl;
                t.epow[(size_t)(half + i) * m + e] = pr;
                pl *= ul;
                pr *= ur;
            }
        }
        t.n = n;
        t.window = window;
        t.order = order;
        tp = std::make_shared<const Tables>(std::move(t));
        std::lock_guard<std::mutex> g(cache_mu);
        cache = tp;
    }
    const std::vector<double>& wmid = tp->wmid;
    const std::vector<double>& emat = tp->emat;
    const std::vector<double>& epow = tp->epow;
    const int m = order + 1;
    parallel_rows(rows, [&](int ra, int rb) {
        std::vector<double> coef(m);
        for (int r = ra; r < rb; ++r) {
            const double* xr = x + (size_t)r * n;
            double* yr = y + (size_t)r * n;
            int i = half;
            // four outputs at once (one 4-wide vector FMA per weight), each
            // summed in the order of the one-output loop below
            for (; i + 4 <= n - half; i += 4) {
                const double* src = xr + i - half;
                double s0[4] = {0, 0, 0, 0}, s1[4] = {0, 0, 0, 0}, s2[4] = {0, 0, 0, 0}, s3[4] = {0, 0, 0, 0};
                int j = 0;
                for (; j + 3 < window; j += 4) {
                    const double w0 = wmid[j], w1 = wmid[j + 1], w2 = wmid[j + 2], w3 = wmid[j + 3];
                    for (int o = 0; o < 4; ++o) {
                        s0[o] += w0 * src[j + o];
                        s1[o] += w1 * src[j + 1 + o];
                        s2[o] += w2 * src[j + 2 + o];
                        s3[o] += w3 * src[j + 3 + o];
                    }
                }
                for (; j < window; ++j)
                    for (int o = 0; o < 4; ++o) s0[o] += wmid[j] * src[j + o];
                for (int o = 0; o < 4; ++o) yr[i + o] = (s0[o] + s1[o]) + (s2[o] + s3[o]);
            }
            for (; i < n - half; ++i) {
                const double* src = xr + i - half;
                double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                int j = 0;
                for (; j + 3 < window; j += 4) {
                    s0 += wmid[j] * src[j];
                    s1 += wmid[j + 1] * src[j + 1];
                    s2 += wmid[j + 2] * src[j + 2];
                    s3 += wmid[j + 3] * src[j + 3];
                }
                for (; j < window; ++j) s0 += wmid[j] * src[j];
                yr[i] = (s0 + s1) + (s2 + s3);
            }
            for (int side = 0; side < 2; ++side) {
                const double* src = xr + (side ? n - window : 0);
                double* c = coef.data();
                for (int k = 0; k < m; ++k) {
                    const double* mk = &emat[(size_t)k * window];
                    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
                    int j = 0;
                    for (; j + 3 < window; j += 4) {
                        s0 += mk[j] * src[j];
                        s1 += mk[j + 1] * src[j + 1];
                        s2 += mk[j + 2] * src[j + 2];
                        s3 += mk[j + 3] * src[j + 3];
                    }
                    for (; j < window; ++j) s0 += mk[j] * src[j];
                    c[k] = (s0 + s1) + (s2 + s3);
                }
                double* dst = yr + (side ? n - half : 0);
                const double* pw = &epow[(size_t)side * half * m];
                for (int i = 0; i < half; ++i) {
                    double v = 0.0;
                    for (int k = m - 1; k >= 0; --k) v += c[k] * pw[(size_t)i * m + k];
                    dst[i] = v;
                }
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Ridge regression through the thin SVD of X (one-sided Jacobi):
//   B = W diag(sigma / (sigma^2 + lam)) U^T Y,  lam = rel * sigma_max^2,
// with singular values below eps * max(m, k) * sigma_max dropped when
// lam = 0 (the minimum-norm least-squares solution).
// ---------------------------------------------------------------------------
// lam > 0: the normal equations (X^T X + lam I) B = X^T Y by Cholesky
// (condition number at most lam_max / lam); false if the factorisation
// breaks down (non-finite input), so the caller can take the SVD route.
static bool ridge_normal_equations(const double* X, const double* Y, double* B, int m, int k, int n, double rel,
                                   double* lam_out) {
    std::vector<double> G((size_t)k * k, 0.0);
    for (int i = 0; i < m; ++i) {
        const double* xr = X + (size_t)i * k;
        for (int a = 0; a < k; ++a)
            for (int b = a; b < k; ++b) G[(size_t)a * k + b] += xr[a] * xr[b];
    }
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < a; ++b) G[(size_t)a * k + b] = G[(size_t)b * k + a];
    double lmax = 0.0;
    std::vector<double> vec(k);
    if (eigh_topk(G.data(), k, 1, &lmax, vec.data(), 1) != 0 || !std::isfinite(lmax)) return false;
    std::fill(B, B + (size_t)k * n, 0.0);
    *lam_out = 0.0;
    if (!(lmax > 0.0)) return true;  // X = 0
    const double lam = rel * lmax;
    for (int a = 0; a < k; ++a) G[(size_t)a * k + a] += lam;
    // G = L L^T, L in the lower triangle
    for (int j = 0; j < k; ++j) {
        double dj = G[(size_t)j * k + j];
        for (int c = 0; c < j; ++c) dj -= G[(size_t)j * k + c] * G[(size_t)j * k + c];
        if (!(dj > 0.0) || !std::isfinite(dj)) return false;
        const double ljj = std::sqrt(dj);
        G[(size_t)j * k + j] = ljj;
        for (int r = j + 1; r < k; ++r) {
            double v = G[(size_t)r * k + j];
            for (int c = 0; c < j; ++c) v -= G[(size_t)r * k + c] * G[(size_t)j * k + c];
            G[(size_t)r * k + j] = v / ljj;
        }
    }
    // X^T Y and the two triangular solves, split over columns of Y
    parallel_rows(n, [&](int c0, int c1) {
        const int w = c1 - c0;
        std::vector<double> R((size_t)k * w, 0.0);
        for (int i = 0; i < m; ++i) {
            const double* xr = X + (size_t)i * k;
            const double* yr = Y + (size_t)i * n + c0;
            for (int a = 0; a < k; ++a) {
                const double xa = xr[a];
                double* ra = &R[(size_t)a * w];
                for (int c = 0; c < w; ++c) ra[c] += xa * yr[c];
            }
        }
        for (int a = 0; a < k; ++a) {  // L z = R
            double* ra = &R[(size_t)a * w];
            for (int b = 0; b < a; ++b) {
                const double l = G[(size_t)a * k + b];
                const double* rb = &R[(size_t)b * w];
                for (int c = 0; c < w; ++c) ra[c] -= l * rb[c];
            }
            const double inv = 1.0 / G[(size_t)a * k + a];
            for (int c = 0; c < w; ++c) ra[c] *= inv;
        }
        for (int a = k - 1; a >= 0; --a) {  // L^T b = z
            double* ra = &R[(size_t)a * w];
            for (int b = a + 1; b < k; ++b) {
                const double l = G[(size_t)b * k + a];
                const double* rb = &R[(size_t)b * w];
                for (int c = 0; c < w; ++c) ra[c] -= l * rb[c];
            }
            const double inv = 1.0 / G[(size_t)a * k + a];
            for (int c = 0; c < w; ++c) ra[c] *= inv;
            std::copy(ra, ra + w, B + (size_t)a * n + c0);
        }
    });
    *lam_out = lam;
    return true;
}

double ridge_rel_solve(const double* X, const double* Y, double* B, int m, int k, int n, double rel) {
    if (rel > 0.0) {
        double lam = 0.0;
        if (ridge_normal_equations(X, Y, B, m, k, n, rel, &lam)) return lam;
    }
    // lam = 0 (minimum-norm least squares): one-sided Jacobi SVD of X
    // columns of X as contiguous vectors
    std::vector<double> cols((size_t)k * m), W((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        for (int i = 0; i < m; ++i) cols[(size_t)j * m + i] = X[(size_t)i * k + j];
        W[(size_t)j * k + j] = 1.0;  // W stored column-major: column j at j*k
    }
    const double eps = std::numeric_limits<double>::epsilon();
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < k - 1; ++p) {
            for (int q = p + 1; q < k; ++q) {
                double* cp = &cols[(size_t)p * m];
                double* cq = &cols[(size_t)q * m];
                double alpha = 0, beta = 0, gamma = 0;
                for (int i = 0; i < m; ++i) {
                    alpha += cp[i] * cp[i];
                    beta += cq[i] * cq[i];
                    gamma += cp[i] * cq[i];
                }
                if (std::fabs(gamma) <= eps * std::sqrt(alpha * beta) || gamma == 0.0) continue;
                rotated = true;
                const double zeta = (beta - alpha) / (2.0 * gamma);
                const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < m; ++i) {
                    const double a = cp[i], b = cq[i];
                    cp[i] = c * a - s * b;
                    cq[i] = s * a + c * b;
                }
                double* wp = &W[(size_t)p * k];
                double* wq = &W[(size_t)q * k];
                for (int i = 0; i < k; ++i) {
                    const double a = wp[i], b = wq[i];
                    wp[i] = c * a - s * b;
                    wq[i] = s * a + c * b;
                }
            }
        }
        if (!rotated) break;
    }
    std::vector<double> sig(k);
    double smax = 0.0;
    for (int j = 0; j < k; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += cols[(size_t)j * m + i] * cols[(size_t)j * m + i];
        sig[j] = std::sqrt(s);
        smax = std::max(smax, sig[j]);
    }
    std::fill(B, B + (size_t)k * n, 0.0);
    if (smax == 0.0) return 0.0;
    const double lam = rel * smax * smax;
    const double cutoff = eps * std::max(m, k) * smax;
    std::vector<double> uty(n);
    for (int j = 0; j < k; ++j) {
        if (sig[j] == 0.0 || (lam == 0.0 && sig[j] <= cutoff)) continue;  // no contribution
        const double g = (lam == 0.0) ? 1.0 / sig[j] : sig[j] / (sig[j] * sig[j] + lam);
        // u_j^T Y with u_j = col_j / sigma_j
        std::fill(uty.begin(), uty.end(), 0.0);
        for (int i = 0; i < m; ++i) {
            const double u = cols[(size_t)j * m + i] / sig[j];
            const double* yr = Y + (size_t)i * n;
            for (int c = 0; c < n; ++c) uty[c] += u * yr[c];
        }
        const double* wj = &W[(size_t)j * k];
        for (int r = 0; r < k; ++r) {
            const double f = wj[r] * g;
            double* br = B + (size_t)r * n;
            for (int c = 0; c < n; ++c) br[c] += f * uty[c];
        }
    }
    return lam;
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver for the top k eigenpairs.
// ---------------------------------------------------------------------------
namespace {

// Number of eigenvalues of the tridiagonal (d, e) that are smaller than x.
int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
    int count = 0;
    double q = d[0] - x;
    if (std::fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++count;
    for (int i = 1; i < n; ++i) {
        q = d[i] - x - e2[i - 1] / q;
        if (std::fabs(q) < pivmin) q = -pivmin;
        if (q < 0) ++count;
    }
    return count;
}

// Four Sturm counts at once (independent recurrences interleaved, so the
// division chains overlap); each lane computes exactly what sturm_count does.
void sturm_count4(const double* d, const double* e2, int n, const double* x, double pivmin, int* count) {
    double q[4];
    int c[4];
    for (int l = 0; l < 4; ++l) {
        q[l] = d[0] - x[l];
        if (std::fabs(q[l]) < pivmin) q[l] = -pivmin;
        c[l] = q[l] < 0 ? 1 : 0;
    }
    for (int i = 1; i < n; ++i) {
        const double di = d[i], ei = e2[i - 1];
        for (int l = 0; l < 4; ++l) {
            double t = di - x[l] - ei / q[l];
            if (std::fabs(t) < pivmin) t = -pivmin;
            c[l] += t < 0 ? 1 : 0;
            q[l] = t;
        }
    }
    for (int l = 0; l < 4; ++l) count[l] = c[l];
}

// Eight Sturm counts at once: two interleaved groups of four, each lane the
// recurrence of sturm_count.
void sturm_count8(const double* d, const double* e2, int n, const double* x, double pivmin, int* count) {
    double q[8];
    int c[8];
    for (int l = 0; l < 8; ++l) {
        q[l] = d[0] - x[l];
        if (std::fabs(q[l]) < pivmin) q[l] = -pivmin;
        c[l] = q[l] < 0 ? 1 : 0;
    }
    for (int i = 1; i < n; ++i) {
        const double di = d[i], ei = e2[i - 1];
        for (int l = 0; l < 8; ++l) {
            double t = di - x[l] - ei / q[l];
            if (std::fabs(t) < pivmin) t = -pivmin;
            c[l] += t < 0 ? 1 : 0;
            q[l] = t;
        }
    }
    for (int l = 0; l < 8; ++l) count[l] = c[l];
}

// Solve (T - lam I) x = b for tridiagonal T by Gaussian elimination with
// partial pivoting (row interchanges between neighbours).  b is overwritten.
void tri_shift_solve(const double* d, const double* e, int n, double lam, double pivmin, double* b,
                     std::vector<double>& dl, std::vector<double>& dd, std::vector<double>& du,
                     std::vector<double>& du2, std::vector<char>& swap) {
    dl.assign(e, e + n - 1);
    dd.resize(n);
    for (int i = 0; i < n; ++i) dd[i] = d[i] - lam;
    du.assign(e, e + n - 1);
    du2.assign(std::max(n - 2, 0), 0.0);
    swap.assign(n, 0);
    for (int i = 0; i + 1 < n; ++i) {
        if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
            if (std::fabs(dd[i]) < pivmin) dd[i] = (dd[i] < 0 ? -pivmin : pivmin);
            const double f = dl[i] / dd[i];
            dl[i] = f;
            dd[i + 1] -= f * du[i];
        } else {
            const double f = dd[i] / dl[i];
            dd[i] = dl[i];
            dl[i] = f;
            const double t = du[i];
            du[i] = dd[i + 1];
            dd[i + 1] = t - f * dd[i + 1];
            if (i + 2 < n) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du[i + 1];
            }
            swap[i] = 1;
        }
    }
    if (std::fabs(dd[n - 1]) < pivmin) dd[n - 1] = (dd[n - 1] < 0 ? -pivmin : pivmin);
    for (int i = 0; i + 1 < n; ++i) {
        if (swap[i]) std::swap(b[i], b[i + 1]);
        b[i + 1] -= dl[i] * b[i];
    }
    b[n - 1] /= dd[n - 1];
    if (n >= 2) b[n - 2] = (b[n - 2] - du[n - 2] * b[n - 1]) / dd[n - 2];
    for (int i = n - 3; i >= 0; --i) b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / dd[i];
}

}  // namespace

int eigh_topk(const double* a_in, int n, int k, double* vals, double* vecs, int threads) {
    if (n <= 0 || k <= 0 || k > n) return -1;
    std::vector<double> A(a_in, a_in + (size_t)n * n);
    std::vector<double> d(n), e(std::max(n - 1, 1), 0.0);
    std::vector<double> vstore;          // Householder vectors, packed
    std::vector<size_t> voff(std::max(n - 2, 0));
    std::vector<double> beta(std::max(n - 2, 0), 0.0);
    Pool& pool = host_pool();
    (void)threads;
    std::vector<double> p(n), pn(n), w(n), v(n), vn(n);

    // ---- Householder reduction to tridiagonal form: A <- H A H ----
    // H_i = I - beta_i v_i v_i^T zeroes row/column i below the subdiagonal.
    // With p_i = beta_i B_i v_i (B_i the trailing block) and
    // w_i = p_i - (beta_i/2)(p_i . v_i) v_i, the block becomes
    // B_i - v_i w_i^T - w_i v_i^T.  The rank-2 update of column i is fused
    // with the product B_{i+1} v_{i+1} of the next column: row i+1 is updated
    // first (it defines v_{i+1}), then every further row is updated and
    // immediately dotted with v_{i+1}, so the block is streamed once per column.
    size_t total = 0;
    for (int i = 0; i + 2 < n; ++i) { voff[i] = total; total += n - i - 1; }
    vstore.resize(std::max<size_t>(total, 1));
    // reflector from row i (columns i+1..n-1); returns false if none is needed
    auto reflector = [&](int i, double* vv, double* bb) {
        const int lo = i + 1, m = n - lo;
        const double* x = &A[(size_t)i * n + lo];
        double sig2 = 0.0;
        for (int j = 1; j < m; ++j) sig2 += x[j] * x[j];
        const double x0 = x[0];
        d[i] = A[(size_t)i * n + i];
        if (sig2 == 0.0) {
            e[i] = x0;
            *bb = 0.0;
            for (int j = 0; j < m; ++j) vv[j] = 0.0;
        } else {
            const double norm = std::sqrt(x0 * x0 + sig2);
            const double alpha = (x0 >= 0) ? -norm : norm;
            for (int j = 0; j < m; ++j) vv[j] = x[j];
            vv[0] = x0 - alpha;
            *bb = 2.0 / (vv[0] * vv[0] + sig2);
            e[i] = alpha;
        }
        beta[i] = *bb;
        std::copy(vv, vv + m, vstore.begin() + voff[i]);
    };
    auto dot = [](const double* a, const double* b, int m) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int c = 0;
        for (; c + 3 < m; c += 4) {
            s0 += a[c] * b[c];
            s1 += a[c + 1] * b[c + 1];
            s2 += a[c + 2] * b[c + 2];
            s3 += a[c + 3] * b[c + 3];
        }
        for (; c < m; ++c) s0 += a[c] * b[c];
        return (s0 + s1) + (s2 + s3);
    };
    if (n >= 3) {
        double b0;
        reflector(0, v.data(), &b0);
        const int lo = 1, m = n - 1;
        pool.run([&](int tid, int nthr) {
            int r0, r1;
            split(lo, n, tid, nthr, &r0, &r1);
            for (int r = r0; r < r1; ++r) p[r - lo] = b0 * dot(&A[(size_t)r * n + lo], v.data(), m);
        });
    }
    for (int i = 0; i + 2 < n; ++i) {
        const int lo = i + 1, m = n - lo;
        const double b = beta[i];
        double ptv = dot(p.data(), v.data(), m);
        const double kk = 0.5 * b * ptv;
        for (int j = 0; j < m; ++j) w[j] = p[j] - kk * v[j];
        // row lo first: it defines the next reflector
        {
            double* row = &A[(size_t)lo * n + lo];
            const double vr = v[0], wr = w[0];
            for (int c = 0; c < m; ++c) row[c] -= vr * w[c] + wr * v[c];
        }
        const bool next = (i + 3 < n);
        double bn = 0.0;
        if (next) reflector(lo, vn.data(), &bn);
        const int lo2 = lo + 1, m2 = n - lo2;
        pool.run([&](int tid, int nthr) {
            int r0, r1;
            split(lo2, n, tid, nthr, &r0, &r1);
            for (int r = r0; r < r1; ++r) {
                double* row = &A[(size_t)r * n + lo];
                const double vr = v[r - lo], wr = w[r - lo];
                for (int c = 0; c < m; ++c) row[c] -= vr * w[c] + wr * v[c];
                if (next) pn[r - lo2] = bn * dot(row + 1, vn.data(), m2);
            }
        });
        if (next) {
            std::swap(v, vn);
            std::swap(p, pn);
        }
    }
    if (n >= 2) {
        d[n - 2] = A[(size_t)(n - 2) * n + (n - 2)];
        e[n - 2] = A[(size_t)(n - 1) * n + (n - 2)];
    }
    d[n - 1] = A[(size_t)(n - 1) * n + (n - 1)];

    return eig_tridiag_topk(d.data(), e.data(), beta.data(), vstore.data(), n, k, vals, vecs);
}

// ---------------------------------------------------------------------------
// Small dense kernels of the randomized range finder (n x l, l <= 128).
// ---------------------------------------------------------------------------
void gram_cols(const double* X, int n, int l, double* G) {
    Pool& pool = host_pool();
    const int nt = pool.size();
    std::vector<double> part((size_t)nt * l * l, 0.0);
    pool.run([&](int tid, int nthr) {
        int r0, r1;
        split(0, n, tid, nthr, &r0, &r1);
        double* g = &part[(size_t)tid * l * l];
        for (int r = r0; r < r1; ++r) {
            const double* x = X + (size_t)r * l;
            for (int a = 0; a < l; ++a) {
                const double xa = x[a];
                double* ga = g + (size_t)a * l;
                for (int b = a; b < l; ++b) ga[b] += xa * x[b];
            }
        }
    });
    std::fill(G, G + (size_t)l * l, 0.0);
    for (int t = 0; t < nt; ++t)  // fixed order: the same sums every call
        for (size_t i = 0; i < (size_t)l * l; ++i) G[i] += part[(size_t)t * l * l + i];
    for (int a = 0; a < l; ++a)
        for (int b = 0; b < a; ++b) G[(size_t)a * l + b] = G[(size_t)b * l + a];
}

bool cholesky_upper(double* G, int l) {
    for (int j = 0; j < l; ++j) {
        double dj = G[(size_t)j * l + j];
        for (int c = 0; c < j; ++c) dj -= G[(size_t)c * l + j] * G[(size_t)c * l + j];
        if (!(dj > 0.0) || !std::isfinite(dj)) return false;
        const double rjj = std::sqrt(dj);
        G[(size_t)j * l + j] = rjj;
        for (int col = j + 1; col < l; ++col) {
            double v = G[(size_t)j * l + col];
            for (int c = 0; c < j; ++c) v -= G[(size_t)c * l + j] * G[(size_t)c * l + col];
            G[(size_t)j * l + col] = v / rjj;
        }
        for (int r = j + 1; r < l; ++r) G[(size_t)r * l + j] = 0.0;
    }
    return true;
}

void solve_right_upper(double* X, int n, int l, const double* R) {
    parallel_rows(n, [&](int r0, int r1) {
        for (int r = r0; r < r1; ++r) {
            double* x = X + (size_t)r * l;
            for (int j = 0; j < l; ++j) {  // y R = x, column by column
                double v = x[j];
                for (int i = 0; i < j; ++i) v -= x[i] * R[(size_t)i * l + j];
                x[j] = v / R[(size_t)j * l + j];
            }
        }
    });
}

bool orthonormalize_cols(double* X, int n, int l) {
    std::vector<double> G((size_t)l * l);
    for (int pass = 0; pass < 2; ++pass) {  // Cholesky QR, twice
        gram_cols(X, n, l, G.data());
        if (!cholesky_upper(G.data(), l)) return false;
        solve_right_upper(X, n, l, G.data());
    }
    return true;
}

int tridiag_eigvecs(const double* d_in, const double* e_in, int n, int k, double* vals, double* Y, double rel_cut,
                    int* k_out) {
    if (n <= 0 || k <= 0 || k > n) return -1;
    if (k_out) *k_out = k;
    Pool& pool = host_pool();
    std::vector<double> d(d_in, d_in + n), e(std::max(n - 1, 1), 0.0);
    for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    // ---- eigenvalues by bisection (Sturm counts) ----
    double tnorm = 0.0, lo = std::numeric_limits<double>::max(), hi = -lo;
    std::vector<double> e2(std::max(n - 1, 1), 0.0);
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, d[i] - r);
        hi = std::max(hi, d[i] + r);
        tnorm = std::max(tnorm, std::fabs(d[i]) + r);
        if (i + 1 < n) e2[i] = e[i] * e[i];
    }
    const double eps = std::numeric_limits<double>::epsilon();
    const double pivmin = std::max(std::numeric_limits<double>::min(), tnorm * eps * eps);
    if (tnorm == 0.0) {  // zero matrix: eigenvalues 0, unit vectors
        for (int j = 0; j < k; ++j) vals[j] = 0.0;
        for (int j = 0; j < k; ++j)
            for (int r = 0; r < n; ++r) Y[(size_t)j * n + r] = (r == j) ? 1.0 : 0.0;
        return 0;
    }
    lo -= 2 * eps * tnorm;
    hi += 2 * eps * tnorm;
    // eigenvalues jfrom..jto-1 (descending order) by trisection over the
    // pool: each pass counts at the two points that cut an eigenvalue's
    // bracket in thirds (four eigenvalues, eight counts in flight), so a
    // pass shrinks the bracket 3x where bisection's shrinks it 2x, at the
    // cost of one division chain more, which overlaps the first
    auto bisect_range = [&](int jfrom, int jto) {
        pool.run([&](int tid, int nthr) {
            int j0, j1;
            split(jfrom, jto, tid, nthr, &j0, &j1);
            for (int jb = j0; jb < j1; jb += 4) {
                double a[4], b[4], pts[8];
                bool live[4];
                int cnt[8];
                for (int l = 0; l < 4; ++l) {
                    a[l] = lo;
                    b[l] = hi;
                    live[l] = (jb + l < j1);
                }
                for (int it = 0; it < 200; ++it) {
                    bool any = false;
                    for (int l = 0; l < 4; ++l) {
                        const double w = (b[l] - a[l]) / 3.0;
                        pts[2 * l] = a[l] + w;
                        pts[2 * l + 1] = b[l] - w;
                        if (live[l] && (b[l] - a[l] <= 2 * eps * std::max(std::fabs(a[l]), std::fabs(b[l])) + pivmin ||
                                        !(a[l] < pts[2 * l] && pts[2 * l] < pts[2 * l + 1] && pts[2 * l + 1] < b[l])))
                            live[l] = false;
                        any = any || live[l];
                    }
                    if (!any) break;
                    sturm_count8(d.data(), e2.data(), n, pts, pivmin, cnt);
                    for (int l = 0; l < 4; ++l) {
                        if (!live[l]) continue;
                        const int idx = n - 1 - (jb + l);  // ascending index of the j-th largest
                        if (cnt[2 * l] > idx) {
                            b[l] = pts[2 * l];
                        } else if (cnt[2 * l + 1] > idx) {
                            a[l] = pts[2 * l];
                            b[l] = pts[2 * l + 1];
                        } else {
                            a[l] = pts[2 * l + 1];
                        }
                    }
                }
                for (int l = 0; l < 4 && jb + l < j1; ++l) vals[jb + l] = 0.5 * (a[l] + b[l]);
            }
        });
    };

    if (rel_cut > 0.0) {
        // the largest eigenvalue first; the number above the cut then comes
        // from one Sturm count at cut^2, and only those are bisected
        bisect_range(0, 1);
        const double cut = std::sqrt(std::max(vals[0], 0.0)) * rel_cut;
        const double x2 = cut * cut;
        const double xs[4] = {x2, x2, x2, x2};
        int below[4];
        sturm_count4(d.data(), e2.data(), n, xs, pivmin, below);
        k = std::min(std::max(n - below[0], 1), k);
        if (k_out) *k_out = k;
        if (k > 1) bisect_range(1, k);
    } else {
        bisect_range(0, k);
    }

    // ---- eigenvectors of T by inverse iteration ----
    // Each vector is iterated with its own shift (independently, in
    // parallel).  Eigenvalues closer than ortol (numerically equal) form a
    // group that is iterated together with re-orthogonalisation; a final
    // modified Gram-Schmidt pass removes the remaining O(eps |T| / gap)
    // overlaps between computed vectors.
    const double ortol = 1e-10 * tnorm;
    std::vector<int> group_start;
    for (int j = 0; j < k; ++j)
        if (j == 0 || std::fabs(vals[j - 1] - vals[j]) > ortol) group_start.push_back(j);
    const int ngroups = (int)group_start.size();
    group_start.push_back(k);
    auto dotn = [n](const double* a, const double* b) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int i = 0;
        for (; i + 3 < n; i += 4) {
            s0 += a[i] * b[i];
            s1 += a[i + 1] * b[i + 1];
            s2 += a[i + 2] * b[i + 2];
            s3 += a[i + 3] * b[i + 3];
        }
        for (; i < n; ++i) s0 += a[i] * b[i];
        return (s0 + s1) + (s2 + s3);
    };
    std::atomic<int> failed{0};
    pool.run([&](int tid, int nthr) {
        std::vector<double> dl, dd, du, du2;
        std::vector<char> sw;
        for (int g = tid; g < ngroups; g += nthr) {
            const int c0 = group_start[g], c1 = group_start[g + 1];
            for (int j = c0; j < c1; ++j) {
                double* b = &Y[(size_t)j * n];
                uint64_t state = 0x9E3779B97F4A7C15ull + (uint64_t)j;  // deterministic start
                for (int i = 0; i < n; ++i) {
                    state = state * 6364136223846793005ull + 1442695040888963407ull;
                    b[i] = 0.5 + (double)(state >> 11) * (1.0 / 9007199254740992.0);
                }
                const int iters = (j > c0) ? 5 : 3;
                for (int it = 0; it < iters; ++it) {
                    tri_shift_solve(d.data(), e.data(), n, vals[j], pivmin + eps * tnorm, b, dl, dd, du, du2, sw);
                    for (int c = c0; c < j; ++c) {
                        const double* yc = &Y[(size_t)c * n];
                        const double s = dotn(yc, b);
                        for (int i = 0; i < n; ++i) b[i] -= s * yc[i];
                    }
                    const double nrm = std::sqrt(dotn(b, b));
                    if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                        failed.store(1);
                        return;
                    }
                    const double inv = 1.0 / nrm;
                    for (int i = 0; i < n; ++i) b[i] *= inv;
                }
            }
        }
    });
    if (failed.load()) return -2;
    // Final modified Gram-Schmidt pass, pipelined over the pool: vector j
    // takes the finished vectors 0..j-1 in order as soon as each one is
    // final, so every vector sees exactly the operations of the sequential
    // pass.  A vector that fails marks the pass failed and every waiter
    // leaves.
    std::unique_ptr<std::atomic<int>[]> fin(new std::atomic<int>[k]);
    for (int j = 0; j < k; ++j) fin[j].store(j == 0 ? 1 : 0, std::memory_order_relaxed);
    pool.run([&](int tid, int nthr) {
        for (int j = 1 + tid; j < k; j += nthr) {
            double* b = &Y[(size_t)j * n];
            for (int c = 0; c < j; ++c) {
                while (!fin[c].load(std::memory_order_acquire)) {
                    if (failed.load(std::memory_order_relaxed)) return;
                    std::this_thread::yield();
                }
                const double* yc = &Y[(size_t)c * n];
                const double s = dotn(yc, b);
                for (int i = 0; i < n; ++i) b[i] -= s * yc[i];
            }
            const double nrm = std::sqrt(dotn(b, b));
            if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                failed.store(1);
                return;
            }
            for (int i = 0; i < n; ++i) b[i] /= nrm;
            fin[j].store(1, std::memory_order_release);
        }
    });
    return failed.load() ? -2 : 0;
}

void tridiag_back_transform(const double* beta, const double* vstore, int n, int k, double* Y, double* vecs) {
    Pool& pool = host_pool();
    std::vector<size_t> voff(std::max(n - 2, 0));
    size_t total = 0;
    for (int i = 0; i + 2 < n; ++i) {
        voff[i] = total;
        total += n - i - 1;
    }
    // ---- back-transformation x = H_0 H_1 ... H_{n-3} y ----
    // Y holds k4 = k rounded up to 4 vectors (the extra ones zero).  Each
    // thread takes whole groups of four vectors and applies every reflector
    // to them while the reflector is in cache; the dot products keep four
    // partial sums per vector (c mod 4) so they run on 4-wide vector FMAs.
    const int groups = (k + 3) / 4;
    pool.run([&](int tid, int nthr) {
        int g0, g1;
        split(0, groups, tid, nthr, &g0, &g1);
        for (int gi = g0; gi < g1; ++gi) {
            double* y0 = Y + (size_t)(4 * gi) * n;
            double* y1 = y0 + n;
            double* y2 = y1 + n;
            double* y3 = y2 + n;
            for (int i = n - 3; i >= 0; --i) {
                if (beta[i] == 0.0) continue;
                const int lo2 = i + 1, m = n - lo2;
                const double* vs = &vstore[voff[i]];
                double* a0 = y0 + lo2;
                double* a1 = y1 + lo2;
                double* a2 = y2 + lo2;
                double* a3 = y3 + lo2;
                double p0[4] = {0, 0, 0, 0}, p1[4] = {0, 0, 0, 0}, p2[4] = {0, 0, 0, 0}, p3[4] = {0, 0, 0, 0};
                int c = 0;
                for (; c + 4 <= m; c += 4)
                    for (int l = 0; l < 4; ++l) {
                        const double vc = vs[c + l];
                        p0[l] += vc * a0[c + l];
                        p1[l] += vc * a1[c + l];
                        p2[l] += vc * a2[c + l];
                        p3[l] += vc * a3[c + l];
                    }
                for (; c < m; ++c) {
                    const double vc = vs[c];
                    p0[0] += vc * a0[c];
                    p1[0] += vc * a1[c];
                    p2[0] += vc * a2[c];
                    p3[0] += vc * a3[c];
                }
                const double s0 = ((p0[0] + p0[1]) + (p0[2] + p0[3])) * beta[i];
                const double s1 = ((p1[0] + p1[1]) + (p1[2] + p1[3])) * beta[i];
                const double s2 = ((p2[0] + p2[1]) + (p2[2] + p2[3])) * beta[i];
                const double s3 = ((p3[0] + p3[1]) + (p3[2] + p3[3])) * beta[i];
                for (int cc = 0; cc < m; ++cc) {
                    const double vc = vs[cc];
                    a0[cc] -= s0 * vc;
                    a1[cc] -= s1 * vc;
                    a2[cc] -= s2 * vc;
                    a3[cc] -= s3 * vc;
                }
            }
            for (int j = 4 * gi; j < 4 * gi + 4 && j < k; ++j) {
                const double* y = Y + (size_t)j * n;
                // sign: largest-magnitude entry positive (first on ties)
                int imax = 0;
                for (int r = 1; r < n; ++r)
                    if (std::fabs(y[r]) > std::fabs(y[imax])) imax = r;
                const double sg = (y[imax] < 0) ? -1.0 : 1.0;
                for (int r = 0; r < n; ++r) vecs[(size_t)r * k + j] = sg * y[r];
            }
        }
    });
}

int eig_tridiag_topk(const double* d, const double* e, const double* beta, const double* vstore, int n, int k,
                     double* vals, double* vecs) {
    if (n <= 0 || k <= 0 || k > n) return -1;
    std::vector<double> Y((size_t)(k + 3) / 4 * 4 * n, 0.0);
    const int rc = tridiag_eigvecs(d, e, n, k, vals, Y.data());
    if (rc != 0) return rc;
    tridiag_back_transform(beta, vstore, n, k, Y.data(), vecs);
    return 0;
}

}  // namespace fkk
