// Serving runtime: stored-basis transforms of tiles submitted from host
// memory, with HBM-budget admission and continuous batching (include/fkkec.h).
//
// One scheduler thread per server.  Each pass it retires finished batches
// (freeing their device bytes), then admits queued tiles of one basis in
// arrival order while the budget and the in-flight slots allow, and issues
// for that batch: host-to-device copies (copy stream) -> one transform launch
// over the concatenated rows (compute stream) -> device-to-host copies
// (second copy stream), chained by events.  Batches are not waited for
// before the next is formed, so tiles arriving meanwhile are admitted as
// memory frees and their work overlaps the batches in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "fkkec.h"
#include "internal.h"
#include "kernels.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over one device arena, 256-byte granules, coalescing.
class Arena {
  public:
    void init(size_t bytes) {
        size_ = bytes;
        free_.clear();
        free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }

  private:
    size_t size_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t ticket = 0;
    double residual = 0.0;  // of the tile against its basis (Sec. 5), set when it completes
    int basis = 0;
    const float* in = nullptr;
    int64_t rows = 0, ld = 0;
    float* out = nullptr;
    int64_t ld_out = 0;
    Clock::time_point t_submit;
    size_t bytes = 0;
};

struct Batch {
    std::vector<Request> reqs;
    size_t off = 0, bytes = 0;
    int slot = -1;  // pinned host slot: tile offsets out, residual sums back
    hipEvent_t copied = nullptr, computed = nullptr, done = nullptr;
};

// Device bytes of a tile: input and output (rows x n each), the two residual
// sums of every spectrum, and room for alignment and the batch's per-tile
// offsets and sums.
size_t tile_bytes(int64_t rows, int n) { return (2 * (size_t)rows * n + 2 * (size_t)rows) * sizeof(float) + 512; }

struct Finished {
    double latency_ms = 0.0, residual = 0.0;
};

}  // namespace

struct fkk_server {
    int device = 0;
    fkk_server_config cfg{};
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    char* arena_base = nullptr;
    Arena arena;
    std::vector<const fkk_basis*> bases;
    std::vector<int> base_prec;  // precision captured when the basis was added

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> queue;
    std::vector<Batch> inflight;
    int inflight_tiles = 0;
    std::unordered_map<int64_t, Finished> finished;  // ticket -> latency (ms), residual
    std::vector<double> latencies;
    int64_t next_ticket = 1, submitted = 0, completed = 0, rejected = 0, spectra = 0, launches = 0, batch_tiles = 0;
    int64_t flagged = 0;
    double max_residual = 0.0;
    // pinned host slots, one per batch in flight: max_inflight + 1 tile
    // offsets (int64), then 2 max_inflight residual sums (FP64)
    unsigned char* side = nullptr;
    size_t slot_bytes = 0;
    std::vector<int> free_slots;
    Clock::time_point first_submit, last_done;
    bool any_submit = false, stop = false;
    hipError_t error = hipSuccess;
    std::thread worker;

    void run();
    bool issue(std::vector<Request>& reqs);
};

bool fkk_server::issue(std::vector<Request>& reqs) {
    const int bid = reqs[0].basis;  // reqs is moved from below
    const fkk_basis* b = bases[bid];
    const int prec = base_prec[bid];
    const int n = b->N;
    int64_t rows = 0;
    size_t bytes = 0;
    for (auto& r : reqs) {
        rows += r.rows;
        bytes += r.bytes;
    }
    Batch bt;
    if (free_slots.empty() || !arena.alloc(bytes, &bt.off)) return false;  // reqs untouched: caller requeues
    bt.slot = free_slots.back();
    free_slots.pop_back();
    bt.reqs = std::move(reqs);
    bt.bytes = bytes;
    const int nt = (int)bt.reqs.size();
    // device layout: inputs of all tiles (rows x n, contiguous), outputs, the
    // residual sums of every spectrum (rows x 2), then (256-byte aligned)
    // the tile offsets and the per-tile sums
    float* din = reinterpret_cast<float*>(arena_base + bt.off);
    float* dout = din + (size_t)rows * n;
    float* dnorm = dout + (size_t)rows * n;
    const size_t o_offs = ((size_t)(reinterpret_cast<char*>(dnorm + 2 * rows) - arena_base) + 255) & ~size_t(255);
    long long* doffs = reinterpret_cast<long long*>(arena_base + o_offs);
    double* dsums = reinterpret_cast<double*>(doffs + nt + 1);
    long long* hoffs = reinterpret_cast<long long*>(side + (size_t)bt.slot * slot_bytes);
    double* hsums = reinterpret_cast<double*>(hoffs + cfg.max_inflight + 1);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) {
        if (r != hipSuccess && e == hipSuccess) e = r;
    };
    chk(hipEventCreateWithFlags(&bt.copied, hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&bt.computed, hipEventDisableTiming));
    chk(hipEventCreateWithFlags(&bt.done, hipEventDisableTiming));
    int64_t r0 = 0;
    for (int t = 0; t < nt; ++t) {
        const Request& r = bt.reqs[t];
        hoffs[t] = r0;
        chk(hipMemcpy2DAsync(din + (size_t)r0 * n, n * sizeof(float), r.in, r.ld * sizeof(float), n * sizeof(float),
                             r.rows, hipMemcpyHostToDevice, s_in));
        r0 += r.rows;
    }
    hoffs[nt] = r0;
    chk(hipMemcpyAsync(doffs, hoffs, (nt + 1) * sizeof(long long), hipMemcpyHostToDevice, s_in));
    chk(hipEventRecord(bt.copied, s_in));
    chk(hipStreamWaitEvent(s_comp, bt.copied, 0));
    // the transform also writes each spectrum's residual sums (Sec. 5)
    const fkk::dev::ResidualArgs res{b->d_f, b->d_g, dnorm};
    if (prec == FKK_PREC_BF16)
        chk(fkk::dev::launch_transform16(din, rows, n, n, b->d_rinv, (float)b->ratio_floor, b->d_wt16, b->npad, b->kq,
                                         b->d_bre16, b->d_bim16, dout, n, FKK_OUT_IM, s_comp, res));
    else
        chk(fkk::dev::launch_transform(din, rows, n, n, b->d_rinv, (float)b->ratio_floor, b->d_wt, b->npad, b->kp,
                                       b->k, b->d_bre_t, b->d_bim_t, dout, n, FKK_OUT_IM, s_comp, res));
    chk(fkk::dev::launch_segment_sums(dnorm, doffs, nt, dsums, s_comp));
    chk(hipEventRecord(bt.computed, s_comp));
    chk(hipStreamWaitEvent(s_out, bt.computed, 0));
    r0 = 0;
    for (auto& r : bt.reqs) {
        chk(hipMemcpy2DAsync(r.out, r.ld_out * sizeof(float), dout + (size_t)r0 * n, n * sizeof(float),
                             n * sizeof(float), r.rows, hipMemcpyDeviceToHost, s_out));
        r0 += r.rows;
    }
    chk(hipMemcpyAsync(hsums, dsums, 2 * (size_t)nt * sizeof(double), hipMemcpyDeviceToHost, s_out));
    chk(hipEventRecord(bt.done, s_out));
    if (e != hipSuccess) error = e;
    ++launches;
    batch_tiles += (int64_t)bt.reqs.size();
    inflight_tiles += (int)bt.reqs.size();
    inflight.push_back(std::move(bt));
    return true;
}

void fkk_server::run() {
    hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // 1. retire finished batches
        for (size_t i = 0; i < inflight.size();) {
            const hipError_t q = hipEventQuery(inflight[i].done);
            if (q == hipErrorNotReady) {
                ++i;
                continue;
            }
            if (q != hipSuccess) error = q;
            const auto now = Clock::now();
            Batch& bt = inflight[i];
            const double* hsums = reinterpret_cast<const double*>(side + (size_t)bt.slot * slot_bytes +
                                                                  (cfg.max_inflight + 1) * sizeof(long long));
            for (size_t t = 0; t < bt.reqs.size(); ++t) {
                const Request& r = bt.reqs[t];
                const double lat = ms_between(r.t_submit, now);
                const double sa = hsums[2 * t], sz = hsums[2 * t + 1];
                const double res = sa > 0.0 ? std::sqrt(std::max(0.0, 1.0 - sz / sa)) : 0.0;
                latencies.push_back(lat);
                finished[r.ticket] = Finished{lat, res};
                if (cfg.residual_threshold > 0.0 && res > cfg.residual_threshold) ++flagged;
                max_residual = std::max(max_residual, res);
                spectra += r.rows;
                ++completed;
            }
            free_slots.push_back(bt.slot);
            last_done = now;
            inflight_tiles -= (int)bt.reqs.size();
            arena.release(bt.off, bt.bytes);
            hipEventDestroy(bt.copied);
            hipEventDestroy(bt.computed);
            hipEventDestroy(bt.done);
            inflight.erase(inflight.begin() + (long)i);
            cv_done.notify_all();
        }
        // 2. admit one batch: queued tiles of the front tile's basis, in order
        bool issued = false;
        if (!queue.empty() && inflight_tiles < cfg.max_inflight) {
            const int basis = queue.front().basis;
            std::vector<Request> take;
            size_t bytes = 0;
            int64_t rows = 0;
            size_t probe_off;
            for (auto it = queue.begin(); it != queue.end();) {
                if (it->basis != basis) {
                    ++it;
                    continue;
                }
                if (!take.empty() && (rows + it->rows > cfg.max_batch_rows ||
                                      inflight_tiles + (int)take.size() >= cfg.max_inflight))
                    break;
                // the whole batch must fit in one free range of the arena
                if (!arena.alloc(bytes + it->bytes, &probe_off)) break;
                arena.release(probe_off, bytes + it->bytes);
                bytes += it->bytes;
                rows += it->rows;
                take.push_back(*it);
                it = queue.erase(it);
            }
            if (!take.empty()) {
                issued = issue(take);
                if (!issued)  // cannot happen after the probe; requeue in order
                    for (auto rit = take.rbegin(); rit != take.rend(); ++rit) queue.push_front(*rit);
            }
        }
        if (stop && queue.empty() && inflight.empty()) break;
        if (issued) continue;
        // 3. nothing issued: sleep until a submission, or poll in-flight work
        if (inflight.empty()) {
            if (stop && queue.empty()) break;
            cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        } else {
            cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

extern "C" {

fkk_status fkk_server_create(int device, const fkk_server_config* cfg, fkk_server** out) {
    if (!cfg || !out || cfg->hbm_budget_bytes < (1 << 20) || cfg->max_inflight < 1 || cfg->max_inflight > 4096 ||
        cfg->max_batch_rows < 1 || !(cfg->residual_threshold >= 0.0))
        return FKK_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return FKK_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return FKK_EDEVICE;
    fkk_server* s = new fkk_server;
    s->device = device;
    s->cfg = *cfg;
    if (hipStreamCreateWithFlags(&s->s_in, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->s_out, hipStreamNonBlocking) != hipSuccess) {
        fkk_server_destroy(s);
        return FKK_EDEVICE;
    }
    if (hipMalloc(reinterpret_cast<void**>(&s->arena_base), (size_t)cfg->hbm_budget_bytes) != hipSuccess) {
        fkk_server_destroy(s);
        return FKK_ENOMEM;
    }
    s->arena.init((size_t)cfg->hbm_budget_bytes);
    s->slot_bytes = (((size_t)cfg->max_inflight + 1) * sizeof(long long) + 2 * (size_t)cfg->max_inflight *
                     sizeof(double) + 255) & ~size_t(255);
    if (hipHostMalloc(reinterpret_cast<void**>(&s->side), s->slot_bytes * cfg->max_inflight, hipHostMallocDefault) !=
        hipSuccess) {
        fkk_server_destroy(s);
        return FKK_ENOMEM;
    }
    for (int i = cfg->max_inflight - 1; i >= 0; --i) s->free_slots.push_back(i);
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return FKK_OK;
}

fkk_status fkk_server_add_basis(fkk_server* srv, const fkk_basis* basis, int32_t* basis_id) {
    if (!srv || !basis || !basis_id) return FKK_EINVAL;
    if (basis->device != srv->device || !basis->d_wt) return FKK_EMISMATCH;
    std::lock_guard<std::mutex> g(srv->mu);
    srv->bases.push_back(basis);
    srv->base_prec.push_back(basis->prec);
    basis->holders.fetch_add(1);  // released by fkk_server_destroy
    *basis_id = (int32_t)srv->bases.size() - 1;
    return FKK_OK;
}

fkk_status fkk_server_submit(fkk_server* srv, int32_t basis_id, const float* h_in, int64_t rows, int64_t ld,
                             float* h_out, int64_t ld_out, int64_t* ticket) {
    if (!srv || !h_in || !h_out || !ticket || rows < 1) return FKK_EINVAL;
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->error != hipSuccess) return FKK_EDEVICE;
    if (basis_id < 0 || basis_id >= (int32_t)srv->bases.size()) return FKK_EINVAL;
    const int n = srv->bases[basis_id]->N;
    if (ld < n || ld_out < n) return FKK_EINVAL;
    Request r;
    r.ticket = srv->next_ticket++;
    r.basis = basis_id;
    r.in = h_in;
    r.rows = rows;
    r.ld = ld;
    r.out = h_out;
    r.ld_out = ld_out;
    r.t_submit = Clock::now();
    r.bytes = tile_bytes(rows, n);
    if (r.bytes > srv->arena.size() || rows > srv->cfg.max_batch_rows) {
        ++srv->rejected;
        return FKK_ENOMEM;
    }
    if (!srv->any_submit) {
        srv->first_submit = r.t_submit;
        srv->any_submit = true;
    }
    ++srv->submitted;
    srv->queue.push_back(r);
    *ticket = r.ticket;
    srv->cv_work.notify_one();
    return FKK_OK;
}

fkk_status fkk_server_wait(fkk_server* srv, int64_t ticket, double timeout_ms, double* latency_ms,
                           double* residual) {
    if (!srv) return FKK_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&] { return srv->finished.count(ticket) > 0 || srv->error != hipSuccess; };
    if (timeout_ms < 0) srv->cv_done.wait(lk, ready);
    else if (!srv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready))
        return FKK_EBUSY;
    if (srv->error != hipSuccess) return FKK_EDEVICE;
    const Finished fin = srv->finished[ticket];
    if (latency_ms) *latency_ms = fin.latency_ms;
    if (residual) *residual = fin.residual;
    srv->finished.erase(ticket);
    return FKK_OK;
}

fkk_status fkk_server_drain(fkk_server* srv) {
    if (!srv) return FKK_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] {
        return (srv->queue.empty() && srv->inflight.empty()) || srv->error != hipSuccess;
    });
    return srv->error == hipSuccess ? FKK_OK : FKK_EDEVICE;
}

fkk_status fkk_server_stats_get(fkk_server* srv, fkk_server_stats* st) {
    if (!srv || !st) return FKK_EINVAL;
    std::lock_guard<std::mutex> g(srv->mu);
    std::memset(st, 0, sizeof *st);
    st->submitted = srv->submitted;
    st->completed = srv->completed;
    st->rejected = srv->rejected;
    st->spectra = srv->spectra;
    st->launches = srv->launches;
    st->mean_batch_tiles = srv->launches ? (double)srv->batch_tiles / srv->launches : 0.0;
    st->flagged = srv->flagged;
    st->max_residual = srv->max_residual;
    if (!srv->latencies.empty()) {
        std::vector<double> l = srv->latencies;
        std::sort(l.begin(), l.end());
        auto pct = [&](double p) {
            const size_t i = (size_t)std::min<double>(l.size() - 1, std::max(0.0, p * (l.size() - 1) + 0.5));
            return l[i];
        };
        st->p50_ms = pct(0.50);
        st->p99_ms = pct(0.99);
        st->max_ms = l.back();
        double sum = 0.0;
        for (double v : l) sum += v;
        st->mean_ms = sum / l.size();
        st->busy_s = ms_between(srv->first_submit, srv->last_done) * 1e-3;
    }
    return srv->error == hipSuccess ? FKK_OK : FKK_EDEVICE;
}

fkk_status fkk_server_reset_stats(fkk_server* srv) {
    if (!srv) return FKK_EINVAL;
    std::lock_guard<std::mutex> g(srv->mu);
    srv->latencies.clear();
    srv->finished.clear();
    srv->submitted = srv->completed = srv->rejected = srv->spectra = srv->launches = srv->batch_tiles = 0;
    srv->flagged = 0;
    srv->max_residual = 0.0;
    srv->any_submit = false;
    return FKK_OK;
}

void fkk_server_destroy(fkk_server* srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    hipSetDevice(srv->device);
    if (srv->s_in) hipStreamSynchronize(srv->s_in);
    if (srv->s_comp) hipStreamSynchronize(srv->s_comp);
    if (srv->s_out) hipStreamSynchronize(srv->s_out);
    if (srv->arena_base) hipFree(srv->arena_base);
    if (srv->side) hipHostFree(srv->side);
    if (srv->s_in) hipStreamDestroy(srv->s_in);
    if (srv->s_comp) hipStreamDestroy(srv->s_comp);
    if (srv->s_out) hipStreamDestroy(srv->s_out);
    for (const fkk_basis* b : srv->bases) b->holders.fetch_sub(1);
    delete srv;
}

}  // extern "C"
