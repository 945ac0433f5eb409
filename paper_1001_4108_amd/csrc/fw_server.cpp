// Serving loop: continuous batching of APSP requests on one GPU.
//
// Requests arrive at any time (fw_server_submit).  A dispatcher thread admits
// them in arrival order while their device footprint fits the memory budget,
// copies each admitted payload into a resident slot, and groups work onto a
// small set of worker streams:
//   * every admitted request with n <= small_n that is waiting when a stream
//     frees up (up to max_batch of them and the worker's work-table
//     capacity) goes into ONE batch, run as fw_apsp_batched runs it: stage-
//     batched launches shared by all of its graphs (so a 500-vertex request
//     spreads over the whole GPU), the smallest graphs in one persistent
//     launch -- whatever has arrived is batched together;
//   * a larger request runs the single-graph stage loop (fw_apsp) on its own
//     stream.
// Groups on different streams overlap on the device.  One completion thread
// per stream waits for its groups in order, timestamps them, returns the
// memory of finished requests to the budget and wakes the dispatcher, so new
// requests are admitted as soon as slots and memory free up.
//
// A request's result depends only on its own matrix: both paths share the
// plan table and the per-cell code (see fw_tiles.h), so it is the same alone
// and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fwapsp.h"
#include "fw_internal.h"

namespace fw {
namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

int status_of(hipError_t e) {
    if (e == hipSuccess) return FW_OK;
    if (e == hipErrorOutOfMemory) return FW_ERR_NOMEM;
    return FW_ERR_HIP;
}

constexpr size_t kAlign = 256;

// First-fit allocator over one device arena, with coalescing of free runs.
class Arena {
  public:
    void init(char *base, size_t cap) {
        base_ = base;
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char *at(size_t off) const { return base_ + off; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }
    size_t cap() const { return cap_; }

  private:
    char *base_ = nullptr;
    size_t cap_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    int64_t n = 0;
    const void *src = nullptr;
    int64_t ld_src = 0;
    void *dst_host = nullptr;
    int64_t ld_dst = 0;
    int keep = 0;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    size_t off = 0, bytes = 0;
    int64_t ld_slot = 0;
    int status = FW_OK;
    int group_size = 0;
    bool allocated = false;
    bool done = false;
};

struct Group {
    std::vector<Request *> reqs;
    hipEvent_t done = nullptr;
    int stream = 0;
    bool batched = false;
};

// Work-table capacity of each worker's batched groups (stage-batched
// entries, 8 bytes each): a 512-vertex graph at tile 64 adds about 520.
constexpr size_t kWorkBytes = size_t(8) << 20;

struct Worker {
    hipStream_t st = nullptr;
    void *host_table = nullptr;  // pinned BatchHeader + items for batched groups
    void *dev_table = nullptr;
    void *host_work = nullptr;   // pinned stage-batched work table
    void *dev_work = nullptr;
    bool busy = false;
    std::deque<Group *> queue;   // groups waiting for the completion thread
    std::thread completer;
};

}  // namespace
}  // namespace fw

using namespace fw;

struct fw_server_s {
    fw_server_config cfg{};
    int device = 0;
    void *arena_mem = nullptr;
    Arena arena;
    std::vector<Worker> workers;
    std::mutex mu;
    std::condition_variable cv_dispatch;  // new request, freed memory or stream
    std::condition_variable cv_done;      // completions available / drain
    std::deque<Request *> waiting;        // submitted, not admitted (arrival order)
    std::deque<Request *> admitted;       // admitted, not yet launched
    std::unordered_map<int64_t, Request *> live;  // every request not yet released
    std::deque<fw_completion> completions;
    int64_t next_id = 1;
    bool stop = false;
    fw_server_stats stats{};
    std::thread dispatcher;
    size_t table_bytes = 0;
    int grid = 0;
};

namespace {

void complete_locked(fw_server_s *s, Request *r) {
    r->done = true;
    fw_completion c{};
    c.id = r->id;
    c.n = r->n;
    c.status = r->status;
    c.t_submit_ns = r->t_submit;
    c.t_admit_ns = r->t_admit;
    c.t_done_ns = r->t_done;
    c.group_size = r->group_size;
    s->completions.push_back(c);
    s->stats.completed++;
    if (r->status != FW_OK) s->stats.failed++;
    if (!r->keep || r->status != FW_OK) {
        if (r->allocated) s->arena.release(r->off, r->bytes);
        s->live.erase(r->id);
        delete r;
    }
}

// Enqueue one group on its worker stream; returns a status for all of it.
int enqueue_group(fw_server_s *s, Group *g) {
    Worker &w = s->workers[g->stream];
    hipStream_t st = w.st;
    const int dt = s->cfg.dtype;
    const size_t es = 4;
    hipError_t e = hipSuccess;
    for (Request *r : g->reqs) {
        if (r->n == 0) continue;
        e = hipMemcpy2DAsync(s->arena.at(r->off), (size_t)r->ld_slot * es, r->src,
                             (size_t)r->ld_src * es, (size_t)r->n * es, (size_t)r->n,
                             hipMemcpyDefault, st);
        if (e != hipSuccess) return status_of(e);
    }
    if (g->batched) {
        std::vector<void *> ptrs;
        std::vector<int64_t> ns, lds;
        for (Request *r : g->reqs)
            if (r->n > 1) {
                ptrs.push_back(s->arena.at(r->off));
                ns.push_back(r->n);
                lds.push_back(r->ld_slot);
            }
        const BatchBuffers buf{w.host_table, w.dev_table, s->table_bytes,
                               w.host_work,  w.dev_work,  kWorkBytes};
        const int st2 = enqueue_batch_buffered(ptrs.data(), ns.data(), lds.data(),
                                               (int64_t)ptrs.size(), dt, buf, st);
        if (st2 != FW_OK) return st2;
    } else {
        for (Request *r : g->reqs) {
            int st2 = solve_single(s->arena.at(r->off), dt, r->n, r->ld_slot, nullptr, 0, st);
            if (st2 != FW_OK) return st2;
        }
    }
    for (Request *r : g->reqs) {
        if (!r->dst_host || r->n == 0) continue;
        e = hipMemcpy2DAsync(r->dst_host, (size_t)r->ld_dst * es, s->arena.at(r->off),
                             (size_t)r->ld_slot * es, (size_t)r->n * es, (size_t)r->n,
                             hipMemcpyDefault, st);
        if (e != hipSuccess) return status_of(e);
    }
    e = hipEventRecord(g->done, st);
    return status_of(e);
}

void dispatcher_main(fw_server_s *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        if (s->stop) {
            // shutting down: requests not yet admitted are cancelled
            while (!s->waiting.empty()) {
                Request *r = s->waiting.front();
                s->waiting.pop_front();
                r->status = FW_ERR_BUSY;
                r->t_done = now_ns();
                complete_locked(s, r);
            }
            s->cv_done.notify_all();
        }
        // admission: arrival order, while the footprint fits the budget
        while (!s->waiting.empty()) {
            Request *r = s->waiting.front();
            size_t off = 0;
            if (r->bytes && !s->arena.alloc(r->bytes, &off)) {
                s->stats.deferrals++;
                break;
            }
            r->off = off;
            r->allocated = r->bytes != 0;
            r->t_admit = now_ns();
            s->waiting.pop_front();
            s->admitted.push_back(r);
            s->stats.admitted++;
        }
        int idle = -1;
        for (size_t i = 0; i < s->workers.size(); ++i)
            if (!s->workers[i].busy) {
                idle = (int)i;
                break;
            }
        if (s->stop && s->waiting.empty() && s->admitted.empty()) break;
        if (idle < 0 || s->admitted.empty()) {
            s->cv_dispatch.wait(lk);
            continue;
        }
        // group: the oldest admitted request decides the kind
        Group *g = new Group();
        g->stream = idle;
        Request *head = s->admitted.front();
        if (head->n <= s->cfg.small_n) {
            g->batched = true;
            int64_t entries = 0;
            const int64_t cap = (int64_t)(kWorkBytes / 8);
            for (auto it = s->admitted.begin();
                 it != s->admitted.end() && (int)g->reqs.size() < s->cfg.max_batch;) {
                if ((*it)->n <= s->cfg.small_n) {
                    const int64_t e = batch_work_entries(s->cfg.dtype, (*it)->n, false);
                    if (!g->reqs.empty() && entries + e > cap) break;
                    entries += e;
                    g->reqs.push_back(*it);
                    it = s->admitted.erase(it);
                } else {
                    ++it;
                }
            }
            s->stats.batched_groups++;
        } else {
            g->reqs.push_back(head);
            s->admitted.pop_front();
            s->stats.single_groups++;
        }
        for (Request *r : g->reqs) r->group_size = (int)g->reqs.size();
        s->stats.max_group = std::max<int64_t>(s->stats.max_group, (int64_t)g->reqs.size());
        Worker &w = s->workers[idle];
        w.busy = true;
        lk.unlock();
        int st = FW_OK;
        if (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess) {
            g->done = nullptr;
            st = FW_ERR_HIP;
        } else {
            st = enqueue_group(s, g);
        }
        lk.lock();
        if (st != FW_OK) {
            if (g->done) (void)hipStreamSynchronize(w.st);
            for (Request *r : g->reqs) {
                r->status = st;
                r->t_done = now_ns();
                complete_locked(s, r);
            }
            if (g->done) (void)hipEventDestroy(g->done);
            delete g;
            w.busy = false;
            s->cv_done.notify_all();
            continue;
        }
        w.queue.push_back(g);
        s->cv_dispatch.notify_all();  // wakes this stream's completion thread
    }
    s->cv_dispatch.notify_all();
}

void completer_main(fw_server_s *s, int idx) {
    (void)hipSetDevice(s->device);
    Worker &w = s->workers[idx];
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        while (w.queue.empty() && !(s->stop && s->waiting.empty() && s->admitted.empty() &&
                                    !w.busy))
            s->cv_dispatch.wait(lk);
        if (w.queue.empty()) break;
        Group *g = w.queue.front();
        lk.unlock();
        const hipError_t e = hipEventSynchronize(g->done);
        const int64_t t = now_ns();
        lk.lock();
        w.queue.pop_front();
        for (Request *r : g->reqs) {
            r->t_done = t;
            r->status = status_of(e);
            complete_locked(s, r);
        }
        (void)hipEventDestroy(g->done);
        delete g;
        w.busy = false;
        s->cv_dispatch.notify_all();
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int fw_server_create(const fw_server_config *cfg, fw_server *out) {
    if (!cfg || !out) return FW_ERR_INVALID;
    *out = nullptr;
    if ((cfg->dtype != FW_F32 && cfg->dtype != FW_I32) || cfg->budget_bytes <= 0 ||
        cfg->streams < 1 || cfg->streams > 16 || cfg->max_batch < 1 || cfg->small_n < 0 ||
        cfg->queue_cap < 1)
        return FW_ERR_INVALID;
    auto *s = new fw_server_s();
    s->cfg = *cfg;
    s->cfg.small_n = std::min<int64_t>(cfg->small_n, fw_batched_max_n(cfg->dtype, 0));
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return FW_ERR_HIP;
    }
    int status = FW_OK;
    if (hipMalloc(&s->arena_mem, (size_t)cfg->budget_bytes) != hipSuccess) status = FW_ERR_NOMEM;
    s->arena.init(static_cast<char *>(s->arena_mem), status == FW_OK ? (size_t)cfg->budget_bytes : 0);
    s->grid = batched_resident_grid(cfg->dtype, false);
    if (s->grid <= 0 && status == FW_OK) status = FW_ERR_HIP;
    s->table_bytes = sizeof(BatchHeader) + sizeof(BatchItem) * (size_t)cfg->max_batch;
    s->workers.resize((size_t)cfg->streams);
    for (auto &w : s->workers) {
        if (status != FW_OK) break;
        if (hipStreamCreateWithFlags(&w.st, hipStreamNonBlocking) != hipSuccess ||
            hipHostMalloc(&w.host_table, s->table_bytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&w.dev_table, s->table_bytes) != hipSuccess ||
            hipHostMalloc(&w.host_work, kWorkBytes, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&w.dev_work, kWorkBytes) != hipSuccess)
            status = FW_ERR_NOMEM;
    }
    if (status != FW_OK) {
        for (auto &w : s->workers) {
            if (w.st) (void)hipStreamDestroy(w.st);
            if (w.host_table) (void)hipHostFree(w.host_table);
            if (w.dev_table) (void)hipFree(w.dev_table);
            if (w.host_work) (void)hipHostFree(w.host_work);
            if (w.dev_work) (void)hipFree(w.dev_work);
        }
        if (s->arena_mem) (void)hipFree(s->arena_mem);
        delete s;
        return status;
    }
    s->stats.budget_bytes = cfg->budget_bytes;
    s->dispatcher = std::thread(dispatcher_main, s);
    for (size_t i = 0; i < s->workers.size(); ++i)
        s->workers[i].completer = std::thread(completer_main, s, (int)i);
    *out = s;
    return FW_OK;
}

int fw_server_submit(fw_server s, const void *src, int64_t n, int64_t ld_src, void *dst_host,
                     int64_t ld_dst, int keep, int64_t *id_out) {
    if (!s || n < 0 || n > 0x7fffffffLL || ld_src < n || (n > 0 && !src)) return FW_ERR_INVALID;
    if (dst_host && ld_dst < n) return FW_ERR_INVALID;
    const int64_t ld_slot = (n + 3) / 4 * 4;
    const double fp = (double)n * (double)ld_slot * 4.0;
    if (fp > (double)s->cfg.budget_bytes) return FW_ERR_UNSUPPORTED;
    auto *r = new Request();
    r->n = n;
    r->src = src;
    r->ld_src = ld_src;
    r->dst_host = dst_host;
    r->ld_dst = ld_dst;
    r->keep = keep ? 1 : 0;
    r->ld_slot = ld_slot;
    r->bytes = (size_t)fp;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return FW_ERR_INVALID;
        }
        if ((int64_t)s->waiting.size() >= s->cfg.queue_cap) {
            s->stats.rejected++;
            delete r;
            return FW_ERR_BUSY;
        }
        r->id = s->next_id++;
        r->t_submit = now_ns();
        s->waiting.push_back(r);
        s->live[r->id] = r;
        s->stats.submitted++;
        if (id_out) *id_out = r->id;
    }
    s->cv_dispatch.notify_all();
    return FW_OK;
}

int fw_server_poll(fw_server s, fw_completion *out, int cap, int64_t timeout_us) {
    if (!s || (cap > 0 && !out) || cap < 0) return -FW_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completions.empty() && timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                            [&] { return !s->completions.empty(); });
    int k = 0;
    while (k < cap && !s->completions.empty()) {
        out[k++] = s->completions.front();
        s->completions.pop_front();
    }
    return k;
}

int fw_server_fetch(fw_server s, int64_t id, void *dst, int64_t ld_dst, void *stream) {
    if (!s) return FW_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->live.find(id);
    if (it == s->live.end()) return FW_ERR_NOT_FOUND;
    Request *r = it->second;
    if (!r->done || !r->keep) return FW_ERR_INVALID;
    if (r->n == 0) return FW_OK;
    if (!dst || ld_dst < r->n) return FW_ERR_INVALID;
    return status_of(hipMemcpy2DAsync(dst, (size_t)ld_dst * 4, s->arena.at(r->off),
                                      (size_t)r->ld_slot * 4, (size_t)r->n * 4, (size_t)r->n,
                                      hipMemcpyDefault, (hipStream_t)stream));
}

int fw_server_release(fw_server s, int64_t id) {
    if (!s) return FW_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->live.find(id);
        if (it == s->live.end()) return FW_ERR_NOT_FOUND;
        Request *r = it->second;
        if (!r->done) return FW_ERR_INVALID;
        if (r->allocated) s->arena.release(r->off, r->bytes);
        s->live.erase(it);
        delete r;
    }
    s->cv_dispatch.notify_all();
    return FW_OK;
}

int fw_server_drain(fw_server s, int64_t timeout_us) {
    if (!s) return FW_ERR_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto idle = [&] { return s->stats.completed == s->stats.submitted; };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, idle);
        return FW_OK;
    }
    return s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), idle) ? FW_OK
                                                                               : FW_ERR_BUSY;
}

int fw_server_get_stats(fw_server s, fw_server_stats *out) {
    if (!s || !out) return FW_ERR_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->waiting = (int64_t)s->waiting.size();
    out->bytes_in_use = (int64_t)s->arena.used();
    out->peak_bytes = (int64_t)s->arena.peak();
    return FW_OK;
}

int fw_server_destroy(fw_server s) {
    if (!s) return FW_ERR_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_dispatch.notify_all();
    if (s->dispatcher.joinable()) s->dispatcher.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->cv_dispatch.notify_all();
    }
    for (auto &w : s->workers)
        if (w.completer.joinable()) w.completer.join();
    for (auto &w : s->workers) {
        (void)hipStreamSynchronize(w.st);
        (void)hipStreamDestroy(w.st);
        (void)hipHostFree(w.host_table);
        (void)hipFree(w.dev_table);
        (void)hipHostFree(w.host_work);
        (void)hipFree(w.dev_work);
    }
    for (auto &kv : s->live) delete kv.second;
    (void)hipFree(s->arena_mem);
    delete s;
    return FW_OK;
}

}  // extern "C"
