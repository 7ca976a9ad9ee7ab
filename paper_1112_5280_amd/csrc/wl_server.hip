// wl_server.hip -- the solve server behind wl_server_* (include/wilson.h).
//
// Requests (one lattice problem each) wait in a queue. A fixed set of slots,
// each a host thread with its own non-blocking stream, takes the waiting
// request with the earliest deadline -- submission time plus site_slack
// seconds per lattice site, so with site_slack = 0 the oldest -- as soon as
// the slot is idle and that request's solver workspace fits in the free part
// of the server's device arena; the solve then runs on the slot's stream,
// overlapping on the device with every other admitted solve.
// When it finishes, its workspace returns to the arena and the next request
// is admitted. The arena is one device allocation made at creation and
// carved by a first-fit allocator with coalescing, so admission by memory is
// exact and nothing is allocated per request.
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "wl_host.h"

namespace wl {
namespace {

constexpr size_t kArenaAlign = 256;
// Only lattices up to this volume are merged: a larger solve keeps the device
// busy by itself, and batching it only makes its batch mates finish together.
constexpr long kMergeMaxSites = 1L << 17;

// First-fit allocator over [0, size) with free-block coalescing.
class Arena {
  public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
        size_ = size;
    }
    size_t size() const { return size_; }
    bool can_alloc(size_t n) const {
        for (const auto &f : free_)
            if (f.second >= n) return true;
        return false;
    }
    bool alloc(size_t n, size_t *off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const size_t rest = it->second - n;
            const size_t at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        auto it = free_.emplace(off, n).first;
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

  private:
    std::map<size_t, size_t> free_;   // offset -> length
    size_t size_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    wl_problem p{};
    Geom g{};
    size_t ws_bytes = 0;
    wl_request_times t{};
    wl_solve_stats st{};
    int status = WL_NOCONV;
    bool done = false;
    bool claimed = false;   // a wl_server_wait holds it
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace wl

using namespace wl;

struct wl_server {
    wl_server_config cfg{};
    Phases ph{};
    int dev = 0;
    void *arena_mem = nullptr;
    Arena arena;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> slots;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    std::mutex m;
    std::condition_variable cv_admit, cv_done;
    std::deque<Request *> queue;                       // waiting, in submission order
    std::unordered_map<uint64_t, Request *> live;      // every uncollected request
    std::deque<Request *> finished;                    // finished, not collected
    uint64_t next_ticket = 1;
    bool stopping = false;

    // admission deadline: a lattice of V sites may be passed over by requests
    // submitted up to site_slack * V seconds after it (earliest deadline first
    // keeps small solves from queueing behind large ones, and a large one
    // waits at most that long for the smaller ones that overtake it)
    double deadline(const Request *r) const {
        return r->t.submitted + cfg.site_slack * double(2L * r->g.Vh);
    }
    // queue position of the next request to admit: the earliest deadline, the
    // earliest submission among equal deadlines
    size_t head() const {
        size_t b = 0;
        for (size_t j = 1; j < queue.size(); ++j)
            if (deadline(queue[j]) < deadline(queue[b])) b = j;
        return b;
    }
    bool head_fits() const {
        return !queue.empty() && arena.can_alloc(queue[head()]->ws_bytes);
    }

    // bytes of a merged batch of m requests of geometry g (one request: the
    // solo solver's workspace), rounded to the arena's alignment
    size_t batch_bytes(const Geom &g, int m) const {
        const size_t n = m == 1 ? workspace_bytes(g, cfg.flags) : problem_group_bytes(g, cfg.flags, m);
        return (n + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
    }

    // the head request and, with merging, the waiting requests of its lattice
    // size that fit beside it (in submission order, which for one size is
    // deadline order, so all of them come after the head); removes them from
    // the queue and carves their workspace (lock held, head_fits() true)
    std::vector<Request *> take_batch(size_t *off, size_t *bytes) {
        const size_t h = head();
        std::vector<Request *> grp{queue[h]};
        size_t need = queue[h]->ws_bytes;
        if (cfg.merge > 1 && 2L * grp[0]->g.Vh <= kMergeMaxSites) {
            const Geom &g = grp[0]->g;
            for (size_t j = h + 1; j < queue.size() && int(grp.size()) < cfg.merge; ++j) {
                Request *q = queue[j];
                if (std::memcmp(q->p.dims, grp[0]->p.dims, sizeof(q->p.dims)) != 0) continue;
                const size_t more = batch_bytes(g, int(grp.size()) + 1);
                if (!arena.can_alloc(more)) break;
                grp.push_back(q);
                need = more;
            }
        }
        if (!arena.alloc(need, off)) return {};
        for (Request *r : grp)
            for (auto it = queue.begin(); it != queue.end(); ++it)
                if (*it == r) {
                    queue.erase(it);
                    break;
                }
        *bytes = need;
        return grp;
    }

    void slot_loop(int k) {
        const hipError_t e = hipSetDevice(dev);
        std::unique_lock<std::mutex> lk(m);
        for (;;) {
            cv_admit.wait(lk, [&] { return head_fits() || (stopping && queue.empty()); });
            if (queue.empty()) break;   // stopping and drained
            size_t off = 0, bytes = 0;
            std::vector<Request *> grp = take_batch(&off, &bytes);
            if (grp.empty()) continue;
            const double now = seconds_since(t0);
            for (Request *r : grp) r->t.admitted = now;
            if (head_fits()) cv_admit.notify_one();   // the next one may start too
            lk.unlock();

            std::string why;
            const int n = int(grp.size());
            std::vector<wl_solve_stats> st(n);
            std::vector<int> status(n, WL_EHIP);
            if (e != hipSuccess) {
                for (int i = 0; i < n; ++i) st[i].status = WL_EHIP;
            } else if (n == 1) {
                Request *r = grp[0];
                SolveIn in{};
                in.gauge = r->p.gauge;
                in.b = r->p.b;
                in.x = r->p.x;
                in.g = r->g;
                in.kappa = r->p.kappa;
                in.ph = ph;
                in.tol = cfg.tol;
                in.maxiter = cfg.maxiter;
                in.flags = cfg.flags;
                in.work = static_cast<char *>(arena_mem) + off;
                in.s = streams[k];
                in.own_stream = true;
                status[0] = run_solver(false, in, &st[0], &why);
            } else {
                std::vector<const wl_problem *> ps(n);
                for (int i = 0; i < n; ++i) ps[i] = &grp[i]->p;
                run_problem_group(ps.data(), n, grp[0]->g, ph, cfg.tol, cfg.maxiter, cfg.flags,
                                  static_cast<char *>(arena_mem) + off, streams[k], st.data(),
                                  &why);
                for (int i = 0; i < n; ++i) status[i] = st[i].status;
            }

            lk.lock();
            arena.release(off, bytes);
            const double fin = seconds_since(t0);
            for (int i = 0; i < n; ++i) {
                Request *r = grp[i];
                r->st = st[i];
                r->status = status[i];
                r->t.finished = fin;
                r->done = true;
                finished.push_back(r);
            }
            cv_done.notify_all();
            cv_admit.notify_all();
        }
    }

    static void collect(Request *r, wl_solve_stats *st, wl_request_times *t) {
        if (st) *st = r->st;
        if (t) *t = r->t;
    }

    // remove a finished request from the bookkeeping (lock held)
    void forget(Request *r) {
        for (auto it = finished.begin(); it != finished.end(); ++it)
            if (*it == r) {
                finished.erase(it);
                break;
            }
        live.erase(r->ticket);
        delete r;
    }
};

namespace wl {

int server_create(const wl_server_config &cfg, const Phases &ph, wl_server **out,
                  std::string *why) {
    auto *s = new wl_server;
    s->cfg = cfg;
    s->ph = ph;
    hipError_t e = hipGetDevice(&s->dev);
    if (e == hipSuccess) e = hipMalloc(&s->arena_mem, cfg.hbm_budget);
    for (int k = 0; e == hipSuccess && k < cfg.slots; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
    }
    if (e != hipSuccess) {
        *why = std::string("server setup: ") + hipGetErrorString(e);
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
        if (s->arena_mem) (void)hipFree(s->arena_mem);
        delete s;
        return WL_EHIP;
    }
    s->arena.reset(cfg.hbm_budget / kArenaAlign * kArenaAlign);
    for (int k = 0; k < cfg.slots; ++k) s->slots.emplace_back(&wl_server::slot_loop, s, k);
    *out = s;
    return WL_OK;
}

int server_submit(wl_server *s, const wl_problem &p, const Geom &g, uint64_t *ticket,
                  std::string *why) {
    const size_t need = (workspace_bytes(g, s->cfg.flags) + kArenaAlign - 1) / kArenaAlign *
                        kArenaAlign;
    if (need > s->arena.size()) {
        *why = "request workspace (" + std::to_string(need) + " bytes) exceeds the server's "
               "HBM budget (" + std::to_string(s->arena.size()) + " bytes)";
        return WL_EWORKSPACE;
    }
    auto *r = new Request;
    r->p = p;
    r->g = g;
    r->ws_bytes = need;
    std::lock_guard<std::mutex> lk(s->m);
    if (s->stopping) {
        delete r;
        *why = "server is shutting down";
        return WL_EINVAL;
    }
    r->ticket = s->next_ticket++;
    r->t.submitted = seconds_since(s->t0);
    s->live[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_admit.notify_one();
    return WL_OK;
}

int server_wait(wl_server *s, uint64_t ticket, wl_solve_stats *st, wl_request_times *t,
                std::string *why) {
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->live.find(ticket);
    if (it == s->live.end() || it->second->claimed) {
        *why = "unknown or already collected ticket " + std::to_string(ticket);
        return WL_EINVAL;
    }
    Request *r = it->second;
    r->claimed = true;
    s->cv_done.wait(lk, [&] { return r->done; });
    wl_server::collect(r, st, t);
    const int status = r->status;
    s->forget(r);
    return status;
}

int server_next(wl_server *s, uint64_t *ticket, wl_solve_stats *st, wl_request_times *t,
                std::string *why) {
    std::unique_lock<std::mutex> lk(s->m);
    auto pick = [&]() -> Request * {
        for (Request *r : s->finished)
            if (!r->claimed) return r;
        return nullptr;
    };
    auto unclaimed = [&] {
        for (const auto &kv : s->live)
            if (!kv.second->claimed) return true;
        return false;
    };
    if (!unclaimed()) {
        *why = "no request is pending";
        return WL_EINVAL;
    }
    Request *r = nullptr;
    s->cv_done.wait(lk, [&] { return (r = pick()) != nullptr || !unclaimed(); });
    if (!r) {
        *why = "no request is pending";
        return WL_EINVAL;
    }
    *ticket = r->ticket;
    wl_server::collect(r, st, t);
    const int status = r->status;
    s->forget(r);
    return status;
}

int server_pending(wl_server *s) {
    std::lock_guard<std::mutex> lk(s->m);
    return int(s->live.size());
}

int server_destroy(wl_server *s) {
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stopping = true;
    }
    s->cv_admit.notify_all();
    for (auto &th : s->slots) th.join();
    int ret = WL_OK;
    for (hipStream_t st : s->streams)
        if (hipStreamDestroy(st) != hipSuccess) ret = WL_EHIP;
    if (hipFree(s->arena_mem) != hipSuccess) ret = WL_EHIP;
    for (auto &kv : s->live) delete kv.second;
    delete s;
    return ret;
}

}  // namespace wl
