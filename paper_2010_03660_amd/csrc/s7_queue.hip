// Request queue with continuous batching: the serving form.  The paper points
// to real-time and in-the-loop simulation (section VIII-A), where solves arrive
// continuously.
//
// * The caller hands over a device arena, which is the HBM budget.  Its head
//   holds the batch engine's tables; the rest is carved first-fit, on the host,
//   into the workspaces of admitted requests.
// * submit() copies the request descriptor into a FIFO and returns a ticket.
//   A request whose workspace could never fit in the arena is refused with
//   S7_ENOMEM.
// * The serving thread admits requests from the FIFO head while their
//   workspace fits.
//   - Small requests join the batch engine.  Each engine step is one
//     persistent launch in which every resident request runs its solve
//     (iterations, refinement steps, epilogue) for a time slice of about 2 ms,
//     or a fixed number of iterations if the options set one.  Requests that
//     arrive during a step join at the next one; the others keep their Krylov
//     state on the device.
//   - Large requests (split_cells and up) gain nothing from batching and run
//     best on the single-system path.  A second thread solves them one at a
//     time on its own stream, concurrently with the engine's launches.
//   A finished request frees its workspace for the next admission.
// * 2D 9-point requests (s7_queue_submit_2d9) share the arena, the FIFO, the
//   large-request thread and the batch engine: one persistent launch runs the
//   resident requests of both operators, each system with its own phase
//   functions.
// * poll() never blocks; wait() blocks until the request is done.  A finished
//   request's result is handed out once, then its ticket is released.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "s7_host.hpp"

using namespace s7;

namespace {

constexpr double kSliceMs = 2.0;      // target length of one persistent launch
constexpr int kQueueCapacity = 2048;  // resident engine requests at most
constexpr long long kSplitCells = 1ll << 21;

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// First-fit allocator of 256-byte aligned ranges inside [0, size).
class Arena {
  public:
    explicit Arena(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
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

  private:
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Req {
    uint64_t ticket;
    EngineJob job;
    bool big = false;
    size_t off = 0, bytes = 0;
    double t_submit = 0, t_admit = 0;
    bool done = false;
};

}  // namespace

struct s7_queue {
    char* arena;
    size_t arena_bytes;
    size_t table_bytes;
    int device;
    s7_options opt;
    int epoch_iters;
    long long split_cells;
    Arena heap;
    hipStream_t stream = nullptr, big_stream = nullptr;
    std::unique_ptr<BatchEngine> engine;  // resident requests of both operators

    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_big;
    std::deque<Req*> pending;    // submitted, not admitted
    std::deque<Req*> big_ready;  // admitted large requests
    std::map<uint64_t, std::unique_ptr<Req>> reqs;
    uint64_t next_ticket = 1;
    uint64_t gen = 0;  // bumped by every submission and every release
    bool stop = false, stop_big = false;
    int error = S7_OK;
    std::string error_msg;
    std::thread worker, big_worker;

    s7_queue(char* a, size_t ab, size_t tb, int dev, const s7_options& o)
        : arena(a), arena_bytes(ab), table_bytes(tb), device(dev), opt(o), heap(ab - tb) {
        epoch_iters = o.graph_iters > 0 ? o.graph_iters : 0;  // 0: time slices
        split_cells = o.split_cells < 0 ? (1ll << 62) : (o.split_cells > 0 ? o.split_cells : kSplitCells);
    }

    // Marks every unfinished request failed with rc and stops both threads (lock held).
    void fail_all(int rc, std::vector<Req*>& resident) {
        error = rc;
        for (Req* r : resident) r->job.info.status = rc, r->done = true;
        for (Req* r : pending) r->job.info.status = rc, r->done = true;
        for (Req* r : big_ready) r->job.info.status = rc, r->done = true;
        pending.clear();
        big_ready.clear();
        resident.clear();
        stop = stop_big = true;
        cv_done.notify_all();
        cv_big.notify_all();
    }

    void finish(Req* r) {  // lock held
        r->job.info.t_wait_ms = r->t_admit - r->t_submit;
        r->done = true;
        heap.release(r->off, r->bytes);
        ++gen;
    }

    // The serving thread: admission and the batch engine.
    void run() {
        (void)hipSetDevice(device);
        std::vector<Req*> resident;
        uint64_t seen = ~0ull;
        for (;;) {
            {
                std::unique_lock<std::mutex> lk(mu);
                // sleep while there is nothing to run and nothing new could be admitted
                cv_work.wait(lk, [&] {
                    return !resident.empty() || (!pending.empty() && gen != seen) ||
                           (stop && pending.empty());
                });
                if (stop && pending.empty() && resident.empty()) break;
                while (!pending.empty() && (int)resident.size() < kQueueCapacity) {
                    Req* r = pending.front();
                    size_t off;
                    if (!heap.alloc(r->bytes, &off)) break;
                    pending.pop_front();
                    r->off = off;
                    r->job.ws = arena + table_bytes + off;
                    r->t_admit = now_ms();
                    if (r->big) {
                        big_ready.push_back(r);
                        cv_big.notify_one();
                    } else {
                        resident.push_back(r);
                        engine->add(&r->job);
                    }
                }
                seen = gen;
            }
            if (resident.empty()) continue;
            const int rc = engine->step(epoch_iters, kSliceMs);
            std::lock_guard<std::mutex> lk(mu);
            if (rc != S7_OK) {
                error_msg = s7_last_error();
                fail_all(rc, resident);
                return;
            }
            std::vector<Req*> keep;
            bool any = false;
            for (Req* r : resident) {
                if (r->job.finished) {
                    finish(r);
                    any = true;
                } else {
                    keep.push_back(r);
                }
            }
            resident.swap(keep);
            if (any) cv_done.notify_all();
        }
        std::lock_guard<std::mutex> lk(mu);
        stop_big = true;  // everything admitted: the large-request thread drains and leaves
        cv_big.notify_all();
    }

    // The second thread: large requests, one at a time, on the single-system path.
    void run_big() {
        (void)hipSetDevice(device);
        for (;;) {
            Req* r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_big.wait(lk, [&] { return !big_ready.empty() || stop_big; });
                if (big_ready.empty()) return;
                r = big_ready.front();
                big_ready.pop_front();
            }
            const EngineJob& j = r->job;
            s7_info info;
            int rc;
            if (j.op) {
                const float* c9[9];
                for (int a = 0; a < 7; ++a) c9[a] = j.coef[a];
                c9[7] = j.coef9[0];
                c9[8] = j.coef9[1];
                rc = s7_bicgstab_solve_2d9(j.d.nx, j.d.ny, c9, j.b, j.x, j.rtol, j.max_iter, j.prec, j.ws,
                                           j.ws_bytes, &opt, &info, big_stream);
            } else {
                rc = s7_bicgstab_solve(j.d, j.coef, j.b, j.x, j.rtol, j.max_iter, j.prec, j.ws, j.ws_bytes,
                                       &opt, &info, big_stream);
            }
            std::lock_guard<std::mutex> lk(mu);
            if (rc < 0) {
                if (error == S7_OK) {
                    error = rc;
                    error_msg = s7_last_error();
                }
                info.status = rc;
            }
            info.t_ms = now_ms() - r->t_submit;
            r->job.info = info;
            finish(r);
            cv_done.notify_all();
            cv_work.notify_one();  // memory came free
        }
    }
};

extern "C" {

// Two engine tables: the 7-point engine's, then the 9-point engine's.
static size_t one_table_bytes() { return align256(engine_table_bytes(kQueueCapacity)); }

size_t s7_queue_table_bytes(void) { return one_table_bytes(); }

int s7_queue_create(s7_queue** q, void* arena, size_t arena_bytes, const s7_options* opt) {
    clear_error();
    if (!q || !arena || ((uintptr_t)arena & 255u) != 0) {
        set_error("s7_queue_create: invalid argument");
        return S7_EINVAL;
    }
    s7_options o;
    options_or_default(opt, o);
    const size_t tb = s7_queue_table_bytes();
    if (arena_bytes <= tb + 256) {
        set_error("s7_queue_create: arena smaller than the engine tables (%zu bytes)", tb);
        return S7_EINVAL;
    }
    int dev = 0;
    S7_HIP(hipGetDevice(&dev));
    s7_queue* Q = new (std::nothrow) s7_queue((char*)arena, arena_bytes, tb, dev, o);
    if (!Q) return S7_EINVAL;
    hipError_t e = hipStreamCreateWithFlags(&Q->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&Q->big_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (Q->stream) (void)hipStreamDestroy(Q->stream);
        delete Q;
        set_error("s7_queue_create: %s", hipGetErrorString(e));
        return S7_EHIP;
    }
    Q->engine.reset(new BatchEngine((char*)arena, kQueueCapacity, o, Q->stream));
    Q->worker = std::thread([Q] { Q->run(); });
    Q->big_worker = std::thread([Q] { Q->run_big(); });
    *q = Q;
    return S7_OK;
}

}  // extern "C"

// Queues a request whose job descriptor is filled in; bytes is its workspace.
static int enqueue(s7_queue* q, const EngineJob& job, int op, size_t bytes, uint64_t* ticket, const char* who) {
    if (align256(bytes) > q->arena_bytes - q->table_bytes) {
        set_error("%s: request needs %zu bytes, the arena has %zu", who, bytes, q->arena_bytes - q->table_bytes);
        return S7_ENOMEM;
    }
    std::unique_ptr<Req> r(new Req());
    r->job = job;
    r->job.ws_bytes = bytes;
    r->job.op = op;  // 0: 3D 7-point, 1: 2D 9-point
    r->bytes = bytes;
    r->big = (long long)job.d.nx * job.d.ny * job.d.nz >= q->split_cells;
    r->t_submit = now_ms();
    r->job.t_start_ms = r->t_submit;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        if (q->stop) {
            set_error("%s: queue stopped (%s)", who, q->error_msg.c_str());
            return q->error ? q->error : S7_EINVAL;
        }
        r->ticket = q->next_ticket++;
        *ticket = r->ticket;
        q->pending.push_back(r.get());
        q->reqs[r->ticket] = std::move(r);
        ++q->gen;
    }
    q->cv_work.notify_one();
    return S7_OK;
}

extern "C" {

int s7_queue_submit(s7_queue* q, const s7_request* req, uint64_t* ticket) {
    clear_error();
    if (!q || !req || !ticket || !dims_ok(req->d) || !req->b || !req->x || !(req->rtol > 0.0) ||
        req->max_iter < 0 || req->prec < S7_FP32 || req->prec > S7_FP16_IR) {
        set_error("s7_queue_submit: invalid argument");
        return S7_EINVAL;
    }
    for (int a = 0; a < 7; ++a)
        if (!req->coef[a]) {
            set_error("s7_queue_submit: invalid argument");
            return S7_EINVAL;
        }
    EngineJob j;
    std::memset(&j, 0, sizeof(j));
    j.d = req->d;
    for (int a = 0; a < 7; ++a) j.coef[a] = req->coef[a];
    j.b = req->b;
    j.x = req->x;
    j.rtol = req->rtol;
    j.max_iter = req->max_iter;
    j.prec = req->prec;
    return enqueue(q, j, 0, make_layout(req->d, req->prec, q->opt).bytes, ticket, "s7_queue_submit");
}

int s7_queue_submit_2d9(s7_queue* q, const s7_request_2d9* req, uint64_t* ticket) {
    clear_error();
    bool ok = q && req && ticket && req->nx >= 1 && req->ny >= 1 &&
              (long long)req->nx * req->ny <= kMaxCells && req->b && req->x && req->rtol > 0.0 &&
              req->max_iter >= 0 && req->prec >= S7_FP32 && req->prec <= S7_FP16_IR;
    for (int a = 0; a < 9 && ok; ++a) ok = req->coef[a] != nullptr;
    if (!ok) {
        set_error("s7_queue_submit_2d9: invalid argument");
        return S7_EINVAL;
    }
    EngineJob j;
    std::memset(&j, 0, sizeof(j));
    j.d = s7_dims{req->nx, req->ny, 1};
    for (int a = 0; a < 7; ++a) j.coef[a] = req->coef[a];
    j.coef9[0] = req->coef[7];
    j.coef9[1] = req->coef[8];
    j.b = req->b;
    j.x = req->x;
    j.rtol = req->rtol;
    j.max_iter = req->max_iter;
    j.prec = req->prec;
    const size_t bytes = make_layout(j.d, req->prec, q->opt, q->opt.jacobi ? 8 : 9).bytes;
    return enqueue(q, j, 1, bytes, ticket, "s7_queue_submit_2d9");
}

int s7_queue_poll(s7_queue* q, uint64_t ticket, s7_info* info) {
    clear_error();
    if (!q) return S7_EINVAL;
    std::lock_guard<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return S7_ENOTFOUND;
    if (!it->second->done) return S7_EAGAIN;
    if (info) *info = it->second->job.info;
    const int st = it->second->job.info.status;
    q->reqs.erase(it);
    return st;
}

int s7_queue_wait(s7_queue* q, uint64_t ticket, s7_info* info) {
    clear_error();
    if (!q) return S7_EINVAL;
    std::unique_lock<std::mutex> lk(q->mu);
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return S7_ENOTFOUND;
    Req* r = it->second.get();
    q->cv_done.wait(lk, [&] { return r->done; });
    if (info) *info = r->job.info;
    const int st = r->job.info.status;
    q->reqs.erase(ticket);
    return st;
}

int s7_queue_destroy(s7_queue* q) {
    clear_error();
    if (!q) return S7_EINVAL;
    {
        std::lock_guard<std::mutex> lk(q->mu);
        q->stop = true;
    }
    q->cv_work.notify_all();
    if (q->worker.joinable()) q->worker.join();  // drains, then releases the large-request thread
    if (q->big_worker.joinable()) q->big_worker.join();
    const int err = q->error;
    if (q->stream) (void)hipStreamDestroy(q->stream);
    if (q->big_stream) (void)hipStreamDestroy(q->big_stream);
    delete q;
    return err == S7_OK ? S7_OK : err;
}

}  // extern "C"
