// Householder reduction of the symmetric N x N FP64 matrix G_A to
// tridiagonal form on the device (the O(N^3) part of the eigensolve of
// Eq. 6).  One launch per column i:
//   every block rebuilds, in LDS, w_i = p_i - (beta_i/2)(p_i . v_i) v_i, the
//   updated pivot row i+1 and from it the next reflector v_{i+1}; then the
//   waves of all blocks apply B <- B - v_i w_i^T - w_i v_i^T to the rows
//   below and dot each updated row with v_{i+1} (p_{i+1} = beta_{i+1} B v_{i+1}).
// Rebuilding the O(N) pivot data in every block removes any grid-wide
// synchronisation inside a step; the kernel boundary orders the steps.
// Reflectors are stored packed (column i at i(N-1) - i(i-1)/2, length N-i-1)
// with the same convention as the host reduction, so the host finishes with
// bisection, inverse iteration and back-transformation.
#include "eig.h"

namespace fkk {
namespace dev {

namespace {

constexpr int kThreads = 256;
constexpr int kPrefetch = 16;  // row doubles per lane held in registers (trailing width <= 1024)
static_assert(64 * kPrefetch <= 4 * kThreads, "pivot loads of a prefetching step assume m <= 4 * kThreads");

__device__ __forceinline__ int64_t voff(int64_t i, int64_t n) { return i * (n - 1) - i * (i - 1) / 2; }

// x from the lane `CTRL` names within the same row of 16 lanes (DPP), both
// halves of the double moved alike.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_value(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}

// Sum over the 64 lanes of a wave (all active), returned in every lane:
// rotations by 8, 4, 2 and 1 within each row of 16 lanes leave each lane
// with its row's sum, and the four row sums are read from lanes 0, 16, 32
// and 48 and added in that fixed order.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x128>(v);  // row_ror:8
    v += dpp_move<0x124>(v);  // row_ror:4
    v += dpp_move<0x122>(v);  // row_ror:2
    v += dpp_move<0x121>(v);  // row_ror:1
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// Block-wide sum; every thread gets the result.  red: one double of LDS per wave.
__device__ double block_sum(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

// Block-wide sum with one barrier: red (one double of LDS per wave) must not be read
// by any thread between the barrier here and the next use of the same red
// (callers alternate two buffers, with barriers in between).
__device__ double block_sum_pp(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

// Reflector of x (length m, in LDS): v = x - alpha e1, beta = 2 / v.v,
// alpha = -sign(x0) |x|; zero reflector when x[1:] = 0.
__device__ void make_reflector(const double* x, int m, double* v, double* beta, double* alpha, double* red) {
    double part = 0.0;
    for (int j = 1 + threadIdx.x; j < m; j += blockDim.x) part += x[j] * x[j];
    const double sig2 = block_sum(part, red);
    const double x0 = x[0];
    if (sig2 == 0.0) {
        for (int j = threadIdx.x; j < m; j += blockDim.x) v[j] = 0.0;
        *beta = 0.0;
        *alpha = x0;
    } else {
        const double norm = sqrt(x0 * x0 + sig2);
        const double a = (x0 >= 0.0) ? -norm : norm;
        for (int j = threadIdx.x; j < m; j += blockDim.x) v[j] = (j == 0) ? x0 - a : x[j];
        *beta = 2.0 / ((x0 - a) * (x0 - a) + sig2);
        *alpha = a;
    }
    __syncthreads();
}

// Step 0: reflector of row 0 and p_0 = beta_0 B_0 v_0.
__global__ __launch_bounds__(kThreads) void tridiag_init(const double* __restrict__ A, int n,
                                                         double* __restrict__ p_out, double* __restrict__ vstore,
                                                         double* __restrict__ beta, double* __restrict__ d,
                                                         double* __restrict__ e) {
    extern __shared__ double sm[];
    __shared__ double red[4];
    const int m = n - 1;
    double* x = sm;
    double* v = sm + n;
    for (int j = threadIdx.x; j < m; j += blockDim.x) x[j] = A[1 + j];
    __syncthreads();
    double b, a;
    make_reflector(x, m, v, &b, &a, red);
    if (blockIdx.x == 0) {
        for (int j = threadIdx.x; j < m; j += blockDim.x) vstore[j] = v[j];
        if (threadIdx.x == 0) {
            beta[0] = b;
            d[0] = A[0];
            e[0] = a;
        }
    }
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tw = gridDim.x * (blockDim.x >> 6);
    for (int r = 1 + gw; r < n; r += tw) {
        const double* row = A + (size_t)r * n + 1;
        double s = 0.0;
        for (int c = lane; c < m; c += 64) s += row[c] * v[c];
        s = wave_sum(s);
        if (lane == 0) p_out[r - 1] = b * s;
    }
}

// Step i (0 <= i <= n-3): rank-2 update of column i fused with p_{i+1}.
// The pivot data are built with one round of global reads and two block
// reductions: ptv = p_i . v_i, then |x_{1:}|^2 of the updated pivot row.
// Each wave's first two rows do not depend on the pivot data: with PF > 0
// (trailing width m <= 64 PF) they are loaded into registers before it, so
// their round trip overlaps the reductions; further rows stream as before.
template <int PF>
__global__ __launch_bounds__(kThreads) void tridiag_step(double* __restrict__ A, int n, int i,
                                                         const double* __restrict__ p_in,
                                                         double* __restrict__ p_out, double* __restrict__ vstore,
                                                         double* __restrict__ beta, double* __restrict__ d,
                                                         double* __restrict__ e) {
    extern __shared__ double sm[];
    __shared__ double red[4];
    const int lo = i + 1, m = n - lo;
    double* v = sm;          // v_i        (m)
    double* w = sm + n;      // w_i        (m)
    double* x = sm + 2 * n;  // updated row lo, columns lo..n-1 (m)
    double* vn = sm + 3 * n; // v_{i+1}    (m-1)
    const double* vs = vstore + voff(i, n);
    const double* rlo = A + (size_t)lo * n + lo;
    const double bi = beta[i];
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tw = gridDim.x * (blockDim.x >> 6);
    const int r0 = lo + 1 + gw, r1 = r0 + tw;
    constexpr int PFN = PF > 0 ? PF : 1;
    double ra[PFN], rb[PFN];
    if (PF > 0) {
#pragma unroll
        for (int t = 0; t < PFN; ++t) {
            const int c = lane + 64 * t;
            ra[t] = (r0 < n && c < m) ? A[(size_t)r0 * n + lo + c] : 0.0;
            rb[t] = (r1 < n && c < m) ? A[(size_t)r1 * n + lo + c] : 0.0;
        }
    }
    // one round of independent global reads (issued together with the rows)
    const double v0 = vs[0], p0 = p_in[0];  // w[0] in LDS is rewritten below
    double part = 0.0;
    if (PF > 0) {  // m <= 4 * kThreads: all loads in flight at once
        double tv[4], tp[4], tx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = threadIdx.x + kThreads * u;
            tv[u] = j < m ? vs[j] : 0.0;
            tp[u] = j < m ? p_in[j] : 0.0;
            tx[u] = j < m ? rlo[j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = threadIdx.x + kThreads * u;
            if (j < m) {
                v[j] = tv[u];
                w[j] = tp[u];
                x[j] = tx[u];
                part += tp[u] * tv[u];
            }
        }
    } else {
        for (int j = threadIdx.x; j < m; j += blockDim.x) {
            const double vj = vs[j], pj = p_in[j];
            v[j] = vj;
            w[j] = pj;
            x[j] = rlo[j];
            part += pj * vj;
        }
    }
    const double kk = 0.5 * bi * block_sum(part, red);  // barriers make v, w, x visible
    const double w0 = p0 - kk * v0;
    const bool next = (i + 3 < n);
    double part2 = 0.0;
    for (int j = threadIdx.x; j < m; j += blockDim.x) {
        const double wj = w[j] - kk * v[j];
        const double xj = x[j] - (v0 * wj + w0 * v[j]);
        w[j] = wj;
        x[j] = xj;
        if (j >= 2) part2 += xj * xj;
    }
    double bn = 0.0;
    if (next) {
        const double sig2 = block_sum(part2, red);  // x, w complete after this
        const double x0 = x[1];
        double a;
        if (sig2 == 0.0) {
            a = x0;
            for (int j = threadIdx.x; j < m - 1; j += blockDim.x) vn[j] = 0.0;
        } else {
            const double norm = sqrt(x0 * x0 + sig2);
            a = (x0 >= 0.0) ? -norm : norm;
            bn = 2.0 / ((x0 - a) * (x0 - a) + sig2);
            for (int j = threadIdx.x; j < m - 1; j += blockDim.x) vn[j] = (j == 0) ? x0 - a : x[1 + j];
        }
        if (blockIdx.x == 0) {
            double* vso = vstore + voff(lo, n);
            for (int j = threadIdx.x; j < m - 1; j += blockDim.x) vso[j] = vn[j];
            if (threadIdx.x == 0) {
                beta[lo] = bn;
                d[lo] = x[0];
                e[lo] = a;
            }
        }
    }
    __syncthreads();
    if (!next && blockIdx.x == 0 && threadIdx.x == 0) {
        d[lo] = x[0];
        e[lo] = x[1];
    }
    // rows held in registers
    int rstart = r0;
    if (PF > 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int r = h == 0 ? r0 : r1;
            if (r >= n) break;
            double* row = A + (size_t)r * n + lo;
            const double vr = v[r - lo], wr = w[r - lo];
            double sacc = 0.0;
#pragma unroll
            for (int t = 0; t < PFN; ++t) {
                const int c = lane + 64 * t;
                if (c < m) {
                    const double u = (h == 0 ? ra[t] : rb[t]) - (vr * w[c] + wr * v[c]);
                    row[c] = u;
                    if (next && c >= 1) sacc += u * vn[c - 1];
                    if (!next && r == n - 1 && c == m - 1) d[n - 1] = u;
                }
            }
            if (next) {
                sacc = wave_sum(sacc);
                if (lane == 0) p_out[r - lo - 1] = bn * sacc;
            }
        }
        rstart = r1 + tw;
    }
    for (int r = rstart; r < n; r += tw) {
        double* row = A + (size_t)r * n + lo;
        const double vr = v[r - lo], wr = w[r - lo];
        double sacc = 0.0;
        int c = lane;
        for (; c + 192 < m; c += 256) {  // four independent loads in flight
            const double a0 = row[c], a1 = row[c + 64], a2 = row[c + 128], a3 = row[c + 192];
            const double u0 = a0 - (vr * w[c] + wr * v[c]);
            const double u1 = a1 - (vr * w[c + 64] + wr * v[c + 64]);
            const double u2 = a2 - (vr * w[c + 128] + wr * v[c + 128]);
            const double u3 = a3 - (vr * w[c + 192] + wr * v[c + 192]);
            row[c] = u0;
            row[c + 64] = u1;
            row[c + 128] = u2;
            row[c + 192] = u3;
            if (next) {
                if (c >= 1) sacc += u0 * vn[c - 1];
                sacc += u1 * vn[c + 63] + u2 * vn[c + 127] + u3 * vn[c + 191];
            }
        }
        for (; c < m; c += 64) {
            const double a = row[c] - (vr * w[c] + wr * v[c]);
            row[c] = a;
            if (next && c >= 1) sacc += a * vn[c - 1];
            if (!next && r == n - 1 && c == m - 1) d[n - 1] = a;
        }
        if (next) {
            sacc = wave_sum(sacc);
            if (lane == 0) p_out[r - lo - 1] = bn * sacc;
        }
    }
}

// ---------------------------------------------------------------------------
// Whole reduction in one cooperative launch.  Block b keeps rows b, b+G,
// b+2G, ... of the matrix in LDS for the whole reduction, so the rank-2
// updates never leave the CU.  Per column the blocks exchange only p (one
// entry per row) and the next pivot row.  Each exchanged double travels as
// one 64-bit word: the value rounded to 51 significant bits, its two lowest
// bits replaced by the column number mod 4, which the reader clears again
// (a relative change below 2^-51 that keeps zeros exact and is the same for
// every block, since all read the same word); a reader polls
// its words until all of them carry the expected number, so no separate
// grid barrier is needed.  Two buffers alternate between columns, so the
// word a reader may still find in a slot is that of two columns earlier
// (another number mod 4) or the cleared word (0, and columns 0 and 1
// carry 1 and 2).  A block writes the words of column i+1 only
// after it has read all words of column i, and every block still reading
// column i-1 (the previous content of that buffer) writes at least one word
// of column i after it has read column i-1: a block leaves the column loop
// as soon as it owns no row below the pivot, so every block in the loop
// owns such a row and writes its p entry.  The block owning row n-1, which
// stays in the loop to the end, writes d, e, beta and the reflectors.
// The arithmetic of a column is that of tridiag_step, with the block sums
// split over 512 threads (one owned row per wave) instead of 256.
// ---------------------------------------------------------------------------
constexpr int kMaxOwnedRows = 16;
constexpr int kResThreads = 512;  // threads of a tridiag_resident block (8 waves)
constexpr int kRowsPerBlock = kResThreads / 64;  // preferred rows per block: one per wave
constexpr int kXchPerThread = 8;  // exchange entries per thread and column: n - 1 <= 8 * kResThreads
constexpr size_t kResidentLdsMax = 160 * 1024 - 512;  // dynamic part; the static part is < 200 bytes

typedef unsigned long long u64;

// Agent-coherent (relaxed atomic) accesses: they miss in the per-XCD caches.
// The magnitude is rounded to a multiple of 4 units in the last place (half
// up: the bit pattern of a finite double grows with its magnitude), then
// the two low bits take the tag.
__device__ __forceinline__ void xch_put(u64* slot, double v, unsigned tag) {
    const u64 bits = ((u64)__double_as_longlong(v) + 2ull) & ~3ull;
    __hip_atomic_store(slot, bits | (u64)(tag & 3u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 xch_word(const u64* p) {
    return __hip_atomic_load(const_cast<u64*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool xch_tagged(u64 w, unsigned tag) { return (unsigned)(w & 3ull) == (tag & 3u); }
// the tag bits cleared: a zero travels as an exact zero
__device__ __forceinline__ double xch_value(u64 w) { return __longlong_as_double((long long)(w & ~3ull)); }

// Entries 0..m-1 of p and of the pivot row of column `tag` into w and x
// (LDS), with part += p . v over this thread's entries; NU = ceil(m /
// kResThreads) entries per thread, so a poll loads only live entries.  Gives
// up after spin_limit polls (spin_limit 0: at once), or when *err is set.
template <int NU>
struct XchPoll {
    u64 a[NU], c[NU];
    __device__ __forceinline__ void issue(const u64* pw, const u64* xw, int m) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {  // clamped: every load in bounds, none waits for another
            const int j = min((int)threadIdx.x + kResThreads * u, m - 1);
            a[u] = xch_word(pw + j);
            c[u] = xch_word(xw + j);
        }
    }
    __device__ __forceinline__ bool complete(int m, unsigned tag) const {
        bool all = true;
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = threadIdx.x + kResThreads * u;
            if (j < m) all = all && xch_tagged(a[u], tag) && xch_tagged(c[u], tag);
        }
        return all;
    }
    __device__ __forceinline__ void use(int m, double* w, double* x, const double* v, double& part) const {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int j = threadIdx.x + kResThreads * u;
            if (j < m) {
                const double pj = xch_value(a[u]);
                w[j] = pj;
                x[j] = xch_value(c[u]);
                part += pj * v[j];
            }
        }
    }
};

// Entries 0..m-1 of p and of the pivot row of column `tag` into w and x
// (LDS), with part += p . v over this thread's entries; NU = ceil(m /
// kResThreads) entries per thread, so a poll loads only live entries.  (Two
// polls in flight at a time measured slower: the extra traffic to the
// coherence point costs more than the earlier detection gains.)  Gives up
// after spin_limit polls (spin_limit 0: at once), or when *err is set.
template <int NU>
__device__ bool xch_fetch_n(const u64* pw, const u64* xw, int m, unsigned tag, int spin_limit, const int* err,
                            double* w, double* x, const double* v, double& part) {
    XchPoll<NU> p0;
    for (int spins = 0;; ++spins) {
        if (spins >= spin_limit) return false;
        if ((spins & 63) == 63 &&
            __hip_atomic_load(const_cast<int*>(err), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        p0.issue(pw, xw, m);
        if (p0.complete(m, tag)) break;
        __builtin_amdgcn_s_sleep(1);
    }
    p0.use(m, w, x, v, part);
    return true;
}

__device__ bool xch_fetch(const u64* pw, const u64* xw, int m, unsigned tag, int spin_limit, const int* err,
                          double* w, double* x, const double* v, double& part) {
    switch ((m + kResThreads - 1) / kResThreads) {  // uniform over the block
        case 1: return xch_fetch_n<1>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        case 2: return xch_fetch_n<2>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        case 3: return xch_fetch_n<3>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        case 4: return xch_fetch_n<4>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        case 5: return xch_fetch_n<5>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        case 6: return xch_fetch_n<6>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        case 7: return xch_fetch_n<7>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
        default: return xch_fetch_n<kXchPerThread>(pw, xw, m, tag, spin_limit, err, w, x, v, part);
    }
}

__global__ __launch_bounds__(kResThreads) void tridiag_resident(const double* __restrict__ A, int n, int R, u64* xch,
                                                             double* __restrict__ vstore, double* __restrict__ beta,
                                                             double* __restrict__ d, double* __restrict__ e,
                                                             int* err, int spin_limit) {
    extern __shared__ double sm[];
    __shared__ double red[16];  // [0..7]: p . v, [8..15]: |x_{1:}|^2 (alternating, see block_sum_pp)
    __shared__ double sp0;
    __shared__ int sbad;
    const int G = gridDim.x, b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int writer = (n - 1) % G;                       // owns row n-1: in the loop to the end
    const int last_row = b + ((n - 1 - b) / G) * G;       // largest row this block owns
    double* rows = sm;                   // local row t = matrix row b + t G, all n columns
    double* va = sm + (size_t)R * n;     // v_i
    double* vb = va + n;                 // v_{i+1}
    double* w = vb + n;                  // p_i, then w_i
    double* x = w + n;                   // pivot row
    if (tid == 0) sbad = 0;
    for (int t = 0; t < R; ++t) {
        const int r = b + t * G;
        if (r >= n) break;
        for (int c = tid; c < n; c += kResThreads) rows[(size_t)t * n + c] = A[(size_t)r * n + c];
    }
    // column 0: reflector of row 0 and p_0 = beta_0 B_0 v_0, from A itself
    const int m0 = n - 1;
    for (int j = tid; j < m0; j += kResThreads) x[j] = A[1 + j];
    __syncthreads();
    double bcur, a0;
    make_reflector(x, m0, va, &bcur, &a0, red);
    if (b == writer) {
        for (int j = tid; j < m0; j += kResThreads) vstore[j] = va[j];
        if (tid == 0) {
            beta[0] = bcur;
            d[0] = A[0];
            e[0] = a0;
        }
    }
    for (int t = wave; t < R; t += kResThreads / 64) {
        const int r = b + t * G;
        if (r < 1 || r >= n) continue;
        const double* row = rows + (size_t)t * n + 1;
        double sacc = 0.0;
        for (int c = lane; c < m0; c += 64) {
            sacc += row[c] * va[c];
            if (r == 1) xch_put(xch + 2 * (size_t)n + c, row[c], 1u);  // pivot row of column 0
        }
        sacc = wave_sum(sacc);
        if (lane == 0) xch_put(xch + (r - 1), bcur * sacc, 1u);
    }

    for (int i = 0; i + 2 < n; ++i) {
        const int lo = i + 1, m = n - lo;
        // no row below the pivot left: nothing to update or send from here
        // on (uniform over the block; the writer block never leaves early)
        if (last_row <= lo) return;
        const unsigned tag = (unsigned)i + 1u;  // words of column i
        const double v0 = va[0];
        double part = 0.0;
        __syncthreads();  // LDS of the previous column no longer read
        // words of column i: p at xch + n (i & 1), pivot row at xch + 2n + n (i & 1)
        const size_t half = (i & 1) ? (size_t)n : 0;
        if (!xch_fetch(xch + half, xch + 2 * (size_t)n + half, m, tag, spin_limit, err, w, x, va, part)) sbad = 1;
        // p_0 is copied before the barrier: thread 0 overwrites w[0] with w_0
        // below while other waves may still be about to read it
        if (tid == 0) sp0 = w[0];  // w[0] is this thread's own entry
        // the sum's barrier also publishes sbad, sp0 and the fetched w, x
        const double ptv = block_sum_pp(part, red);
        if (sbad) {
            if (tid == 0) __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;
        }
        const double p0 = sp0;
        const double kk = 0.5 * bcur * ptv;
        const double w0 = p0 - kk * v0;
        const bool next = (i + 3 < n);
        double part2 = 0.0;
        for (int j = tid; j < m; j += kResThreads) {
            const double wj = w[j] - kk * va[j];
            const double xj = x[j] - (v0 * wj + w0 * va[j]);
            w[j] = wj;
            x[j] = xj;
            if (j >= 2) part2 += xj * xj;
        }
        double bn = 0.0;
        if (next) {
            const double sig2 = block_sum_pp(part2, red + 8);  // x, w complete after this
            const double x0 = x[1];
            double a;
            if (sig2 == 0.0) {
                a = x0;
                for (int j = tid; j < m - 1; j += kResThreads) vb[j] = 0.0;
            } else {
                const double norm = sqrt(x0 * x0 + sig2);
                a = (x0 >= 0.0) ? -norm : norm;
                bn = 2.0 / ((x0 - a) * (x0 - a) + sig2);
                for (int j = tid; j < m - 1; j += kResThreads) vb[j] = (j == 0) ? x0 - a : x[1 + j];
            }
            if (b == writer) {
                double* vso = vstore + voff(lo, n);
                for (int j = tid; j < m - 1; j += kResThreads) vso[j] = vb[j];
                if (tid == 0) {
                    beta[lo] = bn;
                    d[lo] = x[0];
                    e[lo] = a;
                }
            }
        } else {
            __syncthreads();
            if (b == writer && tid == 0) {
                d[lo] = x[0];
                e[lo] = x[1];
            }
        }
        __syncthreads();  // vb, w, x complete
        const unsigned ntag = tag + 1u;
        u64* pout = xch + (half ? 0 : (size_t)n);
        u64* xout = xch + 2 * (size_t)n + (half ? 0 : (size_t)n);
        for (int t = wave; t < R; t += kResThreads / 64) {
            const int r = b + t * G;
            if (r <= lo || r >= n) continue;
            double* row = rows + (size_t)t * n + lo;
            const double vr = va[r - lo], wr = w[r - lo];
            const bool pivot = next && r == lo + 1;  // pivot row of the next column
            double sacc = 0.0;
            int c = lane;
            // four columns per lane in flight (m > 192 implies next); sacc
            // takes the columns in the same order as the loop below
            for (; c + 192 < m; c += 256) {
                double u[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cc = c + 64 * q;
                    u[q] = row[cc] - (vr * w[cc] + wr * va[cc]);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int cc = c + 64 * q;
                    row[cc] = u[q];
                    if (cc >= 1) {
                        sacc += u[q] * vb[cc - 1];
                        if (pivot) xch_put(xout + (cc - 1), u[q], ntag);
                    }
                }
            }
            for (; c < m; c += 64) {
                const double u = row[c] - (vr * w[c] + wr * va[c]);
                row[c] = u;
                if (next && c >= 1) {
                    sacc += u * vb[c - 1];
                    if (pivot) xch_put(xout + (c - 1), u, ntag);
                }
                if (!next && r == n - 1 && c == m - 1) d[n - 1] = u;
            }
            if (next) {
                sacc = wave_sum(sacc);
                if (lane == 0) xch_put(pout + (r - lo - 1), bn * sacc, ntag);
            }
        }
        if (!next) break;
        double* tv = va;
        va = vb;
        vb = tv;
        bcur = bn;
    }
}

__global__ void scale_sym_kernel(double* __restrict__ G, const double* __restrict__ f, int n) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * n) return;
    const int r = (int)(idx / n), c = (int)(idx % n);
    G[idx] *= f[r] * f[c];
}

}  // namespace

size_t tridiag_vstore_doubles(int n) { return n >= 3 ? (size_t)(n - 2) * (n - 1) - (size_t)(n - 2) * (n - 3) / 2 : 1; }

hipError_t launch_scale_sym(double* G, const double* f, int n, hipStream_t s) {
    const int64_t total = (int64_t)n * n;
    hipLaunchKernelGGL(scale_sym_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, G, f, n);
    return hipGetLastError();
}


size_t tridiag_resident_lds(int n, int G) {
    const int R = (n + G - 1) / G;
    return ((size_t)R * n + 4 * (size_t)n) * sizeof(double);
}

int tridiag_resident_grid(int n, int device) {
    if (n < 3 || n - 1 > kXchPerThread * kResThreads) return 0;
    int coop = 0, cus = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) return 0;
    // one row per wave where LDS and the CUs allow: fewer blocks exchange
    // less; more blocks where a block's rows would not fit its LDS
    int G = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    const long long rmax = ((long long)(kResidentLdsMax / sizeof(double)) - 4LL * n) / n;
    if (rmax < 1) return 0;
    const int g_lds = (int)((n + rmax - 1) / rmax);
    if (G < g_lds) G = g_lds;
    if (G > cus) G = cus;
    if (G > n) G = n;
    if ((n + G - 1) / G > kMaxOwnedRows) return 0;
    if (tridiag_resident_lds(n, G) > kResidentLdsMax) return 0;
    return G;
}

size_t tridiag_resident_xch_doubles(int n) { return 4 * (size_t)n; }

hipError_t launch_tridiag_resident(const double* A, int n, int G, double* xch, int* err, double* vstore,
                                   double* beta, double* d, double* e, int spin_limit, hipStream_t s) {
    if (n < 3 || n - 1 > kXchPerThread * kResThreads || G < 1 || G > n || spin_limit < 0) return hipErrorInvalidValue;
    const int R = (n + G - 1) / G;
    if (R > kMaxOwnedRows) return hipErrorInvalidValue;
    const size_t lds = tridiag_resident_lds(n, G);
    if (lds > kResidentLdsMax) return hipErrorInvalidValue;
    hipError_t er = hipFuncSetAttribute(reinterpret_cast<const void*>(tridiag_resident),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (er != hipSuccess) return er;
    u64* words = reinterpret_cast<u64*>(xch);
    int nn = n, rr = R;
    void* args[] = {(void*)&A,    (void*)&nn,   (void*)&rr, (void*)&words, (void*)&vstore,
                    (void*)&beta, (void*)&d,    (void*)&e,  (void*)&err,   (void*)&spin_limit};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(tridiag_resident), dim3(G), dim3(kResThreads), args,
                                      (unsigned)lds, s);
}

hipError_t tridiag_prepare(int n) {
    if (n < 3) return hipErrorInvalidValue;
    const size_t lds = (size_t)4 * n * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(tridiag_init),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(tridiag_step<kPrefetch>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(tridiag_step<0>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_tridiag(double* A, int n, double* p0, double* p1, double* vstore, double* beta, double* d, double* e,
                          hipStream_t s) {
    if (n < 3) return hipErrorInvalidValue;
    const size_t lds = (size_t)4 * n * sizeof(double);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    auto blocks_for = [](int rows) {
        int b = (rows + 7) / 8;  // at least two rows per wave
        if (b < 1) b = 1;
        if (b > 256) b = 256;
        return b;
    };
    hipLaunchKernelGGL(tridiag_init, dim3(blocks_for(n - 1)), dim3(kThreads), lds, s, A, n, p0, vstore, beta, d, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    double* pin = p0;
    double* pout = p1;
    for (int i = 0; i + 2 < n; ++i) {
        const int rows = n - (i + 2);
        if (n - (i + 1) <= 64 * kPrefetch)
            hipLaunchKernelGGL(tridiag_step<kPrefetch>, dim3(blocks_for(rows)), dim3(kThreads), lds, s, A, n, i, pin,
                               pout, vstore, beta, d, e);
        else
            hipLaunchKernelGGL(tridiag_step<0>, dim3(blocks_for(rows)), dim3(kThreads), lds, s, A, n, i, pin, pout,
                               vstore, beta, d, e);
        if ((err = hipGetLastError()) != hipSuccess) return err;
        double* t = pin;
        pin = pout;
        pout = t;
    }
    return hipSuccess;
}

namespace {

// Reflector i (packed, rows i+1 .. n-1) into row i of vpad (npad doubles,
// zero at rows <= i and >= n), so the back-transformation loads whole rows
// at one stride without clamping or masking.
// Row i of vpad: reflector i expanded to npad entries (zero outside i+1 ..
// n-1); rows past the last reflector (up to a whole number of blocks) zero.
__global__ void expand_reflectors_kernel(const double* __restrict__ vstore, int n, int npad,
                                         double* __restrict__ vpad) {
    const int i = blockIdx.x;
    double* dst = vpad + (size_t)i * npad;
    if (i >= n - 2) {
        for (int r = threadIdx.x; r < npad; r += blockDim.x) dst[r] = 0.0;
        return;
    }
    const double* vs = vstore + voff(i, n) - (i + 1);
    for (int r = threadIdx.x; r < npad; r += blockDim.x) dst[r] = (r > i && r < n) ? vs[r] : 0.0;
}

// ---------------------------------------------------------------------------
// Blocked back-transformation.  The reflectors are taken kBtB at a time in
// the compact WY form (Schreiber & Van Loan 1989): for reflectors i0 ..
// i0 + B - 1, H_i0 ... H_{i0+B-1} = I - V T V^T with V the reflector rows as
// columns and T upper triangular, built column by column,
//   T(j, j) = beta_j,  T(0:j, j) = -beta_j T(0:j, 0:j) V(:, 0:j)^T v_j.
// x = Q y then takes one block at a time, last to first:
//   x <- x - V (T (V^T x)),
// so a vector meets n / B dependent steps, each with B dot products reduced
// together, instead of n - 2 single ones.
// ---------------------------------------------------------------------------
constexpr int kBtB = 16;         // reflectors per block
constexpr int kBtThreads = 256;  // threads per vector; rows tid + 256 m
constexpr int kBtPairs = kBtB * (kBtB + 1) / 2;

// (a, c), a <= c, of the upper triangle of a kBtB x kBtB matrix in row-major order
struct BtPairTable {
    int a[kBtPairs], c[kBtPairs];
    constexpr BtPairTable() : a(), c() {
        int p = 0;
        for (int i = 0; i < kBtB; ++i)
            for (int j = i; j < kBtB; ++j) {
                a[p] = i;
                c[p] = j;
                ++p;
            }
    }
};
constexpr BtPairTable kBtPairTable{};

// Rows tid + 256 m (m < MR) of reflectors i0 .. i0 + kBtB - 1 (vpad holds
// whole blocks: the rows past the last reflector are zero).
template <int MR>
__device__ __forceinline__ void bt_load_block(double (&v)[kBtB][MR], const double* __restrict__ vpad, int i0) {
    constexpr int NP = kBtThreads * MR;
#pragma unroll
    for (int a = 0; a < kBtB; ++a) {
        const double* row = vpad + (size_t)(i0 + a) * NP + threadIdx.x;
#pragma unroll
        for (int m = 0; m < MR; ++m) v[a][m] = row[kBtThreads * m];
    }
}

// T of reflector block blockIdx.x (reflectors past nr are zero: beta 0).
// G = V^T V from the threads' rows: per round, 16 of the 136 entries a <= c
// as per-thread partials through LDS, each summed by 16 threads; then
// thread a < B builds row a of T.
template <int MR>
__global__ __launch_bounds__(kBtThreads) void tfactor_kernel(const double* __restrict__ beta,
                                                             const double* __restrict__ vpad, int nr,
                                                             double* __restrict__ tmat) {
    __shared__ double sP[kBtB][kBtThreads + 1];
    __shared__ double sGf[kBtPairs];
    __shared__ double sG[kBtB][kBtB + 1];
    __shared__ double sT[kBtB][kBtB + 1];
    const int i0 = blockIdx.x * kBtB, tid = threadIdx.x;
    double v[kBtB][MR];
    bt_load_block<MR>(v, vpad, i0);
    // rounds of kBtB pairs; the pair indices are constants after unrolling,
    // so v stays in registers
#pragma unroll
    for (int p0 = 0; p0 < kBtPairs; p0 += kBtB) {
#pragma unroll
        for (int q = 0; q < kBtB; ++q) {
            double t = 0.0;
            if (p0 + q < kBtPairs) {
                const int a = kBtPairTable.a[p0 + q < kBtPairs ? p0 + q : 0];
                const int c = kBtPairTable.c[p0 + q < kBtPairs ? p0 + q : 0];
#pragma unroll
                for (int m = 0; m < MR; ++m) t += v[a][m] * v[c][m];
            }
            sP[q][tid] = t;
        }
        __syncthreads();
        {
            const int q = tid >> 4, s = tid & 15;
            double t = 0.0;
#pragma unroll
            for (int u = 0; u < kBtThreads / 16; ++u) t += sP[q][16 * u + s];
            t += __shfl_xor(t, 1);
            t += __shfl_xor(t, 2);
            t += __shfl_xor(t, 4);
            t += __shfl_xor(t, 8);
            if (s == 0 && p0 + q < kBtPairs) sGf[p0 + q] = t;
        }
        __syncthreads();
    }
    {  // G(a, c) for a <= c from the pair order (row-major upper triangle)
        const int a = tid / kBtB, c = tid % kBtB;
        if (a <= c) sG[a][c] = sGf[a * kBtB - a * (a - 1) / 2 + (c - a)];
    }
    if (tid < kBtB)
        for (int q = 0; q < kBtB; ++q) sT[tid][q] = 0.0;
    __syncthreads();
    // column j of T: thread a < j takes T(a, j) = -beta_j sum_{a <= l < j} T(a, l) G(l, j)
    for (int j = 0; j < kBtB; ++j) {
        const double bj = (i0 + j < nr) ? beta[i0 + j] : 0.0;
        if (tid < j) {
            double t = 0.0;
            for (int l = tid; l < j; ++l) t += sT[tid][l] * sG[l][j];
            sT[tid][j] = -bj * t;
        } else if (tid == j) {
            sT[j][j] = bj;
        }
        __syncthreads();
    }
    if (tid < kBtB * kBtB) tmat[(size_t)blockIdx.x * kBtB * kBtB + tid] = sT[tid / kBtB][tid % kBtB];
}

// One block per vector j: x (rows tid + 256 m, m < MR, NP = 256 MR) in
// registers; per reflector block, last to first, w = V^T x (sums of the
// threads' partials through LDS), u = T w, x -= V u; then the sign rule
// (the largest-magnitude entry positive, the first on ties) and the
// transposed store into vecs (n x k, row-major).
template <int MR>
__global__ __launch_bounds__(kBtThreads) void back_transform_blocked_kernel(const double* __restrict__ tmat,
                                                                            const double* __restrict__ vpad,
                                                                            int n, int nr, int nblk, int k,
                                                                            const double* __restrict__ Y,
                                                                            double* __restrict__ vecs) {
    __shared__ double sP[kBtB][kBtThreads + 1];
    __shared__ double sW[kBtB], sU[kBtB];
    __shared__ double sBest[kBtThreads / 64], sVal[kBtThreads / 64];
    __shared__ int sRow[kBtThreads / 64];
    const int j = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double x[MR];
    const double* yj = Y + (size_t)j * n;
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tid + kBtThreads * m;
        x[m] = (r < n) ? yj[r] : 0.0;
    }
    // the next block's T row (threads < kBtB) and reflector rows (MR <= 4)
    // are loaded while this one is applied: no step waits for a load it
    // issued itself (one counter covers all loads in flight)
    constexpr bool PF = MR <= 4;
    double v[kBtB][MR], vn[kBtB][MR], trow[kBtB], tn[kBtB];
    auto load_t = [&](int blk, double (&dst)[kBtB]) {
        const double* src = tmat + ((size_t)blk * kBtB + (tid < kBtB ? tid : 0)) * kBtB;
#pragma unroll
        for (int c = 0; c < kBtB; ++c) dst[c] = src[c];
    };
    if (nblk > 0) {
        load_t(nblk - 1, tn);
        if constexpr (PF) bt_load_block<MR>(vn, vpad, (nblk - 1) * kBtB);
    }
    for (int blk = nblk - 1; blk >= 0; --blk) {
        const int i0 = blk * kBtB;
#pragma unroll
        for (int c = 0; c < kBtB; ++c) trow[c] = tn[c];
        if constexpr (PF) {
#pragma unroll
            for (int a = 0; a < kBtB; ++a)
#pragma unroll
                for (int m = 0; m < MR; ++m) v[a][m] = vn[a][m];
        }
        if (blk > 0) load_t(blk - 1, tn);
        if constexpr (PF) {
            if (blk > 0) bt_load_block<MR>(vn, vpad, i0 - kBtB);
        } else {
            bt_load_block<MR>(v, vpad, i0);
        }
#pragma unroll
        for (int a = 0; a < kBtB; ++a) {
            double p = 0.0;
#pragma unroll
            for (int m = 0; m < MR; ++m) p += v[a][m] * x[m];
            sP[a][tid] = p;
        }
        __syncthreads();
        {  // w_a: 16 threads per a, 16 partials each, then a 16-lane sum
            const int a = tid >> 4, s = tid & 15;
            double t = 0.0;
#pragma unroll
            for (int q = 0; q < kBtThreads / 16; ++q) t += sP[a][16 * q + s];
            t += __shfl_xor(t, 1);
            t += __shfl_xor(t, 2);
            t += __shfl_xor(t, 4);
            t += __shfl_xor(t, 8);
            if (s == 0) sW[a] = t;
        }
        __syncthreads();
        if (tid < kBtB) {  // T upper triangular: its zeros below the diagonal add nothing
            double u = 0.0;
#pragma unroll
            for (int c = 0; c < kBtB; ++c) u += trow[c] * sW[c];
            sU[tid] = u;
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < kBtB; ++a) {
            const double ua = sU[a];
#pragma unroll
            for (int m = 0; m < MR; ++m) x[m] -= v[a][m] * ua;
        }
        // no barrier here: sP was last read before the second barrier, and
        // sW and sU are next written after the next block's first one
    }
    // sign rule: (|x|, row, x) of the largest magnitude, the lowest row on ties
    double best = -1.0, bval = 0.0;
    int brow = n;
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tid + kBtThreads * m;
        if (r < n && fabs(x[m]) > best) {
            best = fabs(x[m]);
            bval = x[m];
            brow = r;
        }
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off);
        const double ov = __shfl_xor(bval, off);
        const int orow = __shfl_xor(brow, off);
        if (ob > best || (ob == best && orow < brow)) {
            best = ob;
            bval = ov;
            brow = orow;
        }
    }
    if (lane == 0) {
        sBest[wave] = best;
        sVal[wave] = bval;
        sRow[wave] = brow;
    }
    __syncthreads();
    for (int w = 0; w < kBtThreads / 64; ++w) {
        const double ob = sBest[w];
        const int orow = sRow[w];
        if (ob > best || (ob == best && orow < brow)) {
            best = ob;
            bval = sVal[w];
            brow = orow;
        }
    }
    const double sg = bval < 0.0 ? -1.0 : 1.0;
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tid + kBtThreads * m;
        if (r < n) vecs[(size_t)r * k + j] = sg * x[m];
    }
}

}  // namespace

int back_transform_max_n() { return 64 * 32; }

// padded reflector rows (whole blocks of kBtB), then the T factors
size_t back_transform_vpad_doubles(int n) {
    const int T = n <= 256 ? 4 : n <= 512 ? 8 : n <= 1024 ? 16 : 32;
    const size_t nblk = n >= 3 ? (size_t)(n - 2 + kBtB - 1) / kBtB : 0;
    return n >= 3 ? nblk * kBtB * 64 * T + nblk * kBtB * kBtB : 1;
}

hipError_t launch_back_transform(const double* beta, const double* vstore, int n, int k, const double* Y,
                                 double* vecs, double* vpad, hipStream_t s) {
    if (n < 1 || k < 1 || n > back_transform_max_n()) return hipErrorInvalidValue;
    const int T = n <= 256 ? 4 : n <= 512 ? 8 : n <= 1024 ? 16 : 32;
    // blocked form: padded rows of whole blocks, their T factors, then one
    // block per vector
    const int nr = n >= 3 ? n - 2 : 0, nblk = (nr + kBtB - 1) / kBtB, NP = 64 * T;
    if (nblk > 0) {
        hipLaunchKernelGGL(expand_reflectors_kernel, dim3(nblk * kBtB), dim3(kThreads), 0, s, vstore, n, NP, vpad);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    double* tmat = vpad + (size_t)nblk * kBtB * NP;
    if (nblk > 0) {
        if (T == 4)
            hipLaunchKernelGGL(tfactor_kernel<1>, dim3(nblk), dim3(kBtThreads), 0, s, beta, vpad, nr, tmat);
        else if (T == 8)
            hipLaunchKernelGGL(tfactor_kernel<2>, dim3(nblk), dim3(kBtThreads), 0, s, beta, vpad, nr, tmat);
        else if (T == 16)
            hipLaunchKernelGGL(tfactor_kernel<4>, dim3(nblk), dim3(kBtThreads), 0, s, beta, vpad, nr, tmat);
        else
            hipLaunchKernelGGL(tfactor_kernel<8>, dim3(nblk), dim3(kBtThreads), 0, s, beta, vpad, nr, tmat);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const dim3 grid(k), block(kBtThreads);
    if (T == 4)
        hipLaunchKernelGGL(back_transform_blocked_kernel<1>, grid, block, 0, s, tmat, vpad, n, nr, nblk, k, Y, vecs);
    else if (T == 8)
        hipLaunchKernelGGL(back_transform_blocked_kernel<2>, grid, block, 0, s, tmat, vpad, n, nr, nblk, k, Y, vecs);
    else if (T == 16)
        hipLaunchKernelGGL(back_transform_blocked_kernel<4>, grid, block, 0, s, tmat, vpad, n, nr, nblk, k, Y, vecs);
    else
        hipLaunchKernelGGL(back_transform_blocked_kernel<8>, grid, block, 0, s, tmat, vpad, n, nr, nblk, k, Y, vecs);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace fkk
