// Many molecules on one device: the batched solver and the serving loop.
//
// Both run the same round structure as a single solve (m Arnoldi steps,
// update, FP64 residual, next-cycle start) over every active molecule at
// once: each launch covers all of them, the product drains one tile queue
// holding the tiles of every molecule.  A molecule's decomposition depends
// only on its own size, so its arithmetic is the same alone or in a batch.
//
// Serving (continuous batching): requests wait in a FIFO queue; the head is
// admitted when a slot is free and its footprint fits in the device arena
// (first fit).  Admitted requests are initialised (source terms, norms,
// first cycle start) and join the active set at the next round boundary;
// finished ones leave it, their energies are evaluated and their memory
// returns to the arena.  Krylov state stays on the device for the whole
// solve.  The paper budgets 11N + 6Nc doubles per solve (Section 2.4) for a
// host-driven GMRES; a device-resident GMRES(m) also holds the basis
// (m+1)*2N and the split partial sums, which gabi_solve_footprint counts.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include "gabi_internal.h"

namespace gabi {
namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// ------------------------------------------------------------- staged input
struct Staged {
    int64_t n = 0, nc = 0;
    std::vector<double4> pos, nrm;
    std::vector<float4> geo32;
    std::vector<double> chg;  // 4 nc
    double eps1 = 1, eps2 = 80, kappa = 0;
    double *u_out = nullptr;
    int64_t tag = 0;
    int64_t ticket = 0;
    int64_t bytes = 0;
    double t_submit = 0;
};

int stage_problem(const gabi_problem &p, int m, Staged &out, std::string &err) {
    int rc = validate_surface(p.n, p.cx, p.cy, p.cz, p.nx, p.ny, p.nz, p.area, err);
    if (rc) return rc;
    if ((rc = validate_charges(p.nc, p.px, p.py, p.pz, p.q, err))) return rc;
    if ((rc = check_charges_vs_centroids(p.n, p.cx, p.cy, p.cz, p.nc, p.px, p.py, p.pz, err)))
        return rc;
    if (!params_valid(p.eps1, p.eps2, p.kappa)) {
        err = "need eps1 > 0, eps2 > 0, kappa >= 0, all finite";
        return GABI_EINVAL;
    }
    out.n = p.n;
    out.nc = p.nc;
    stage_surface(p.n, p.cx, p.cy, p.cz, p.nx, p.ny, p.nz, p.area, out.pos, out.nrm, out.geo32);
    out.chg.resize((size_t)(4 * p.nc));
    for (int64_t k = 0; k < p.nc; ++k) {
        out.chg[4 * k] = p.px[k];
        out.chg[4 * k + 1] = p.py[k];
        out.chg[4 * k + 2] = p.pz[k];
        out.chg[4 * k + 3] = p.q[k];
    }
    out.eps1 = p.eps1;
    out.eps2 = p.eps2;
    out.kappa = p.kappa;
    out.u_out = p.u_out;
    out.tag = p.tag;
    out.bytes = slot_bytes(p.n, p.nc, m);
    return GABI_OK;
}

// ------------------------------------------------------------------ arena
// First-fit allocator over [0, cap) with coalescing of free ranges.
class Arena {
   public:
    explicit Arena(int64_t cap) : cap_(cap) {
        if (cap > 0) free_[0] = cap;
    }
    bool alloc(int64_t size, int64_t &off) {
        size = (size + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= size) {
                off = it->first;
                const int64_t rest = it->second - size;
                free_.erase(it);
                if (rest > 0) free_[off + size] = rest;
                used_ += size;
                return true;
            }
        }
        return false;
    }
    bool fits(int64_t size) const {
        size = (size + 255) & ~int64_t(255);
        for (auto &f : free_)
            if (f.second >= size) return true;
        return false;
    }
    void release(int64_t off, int64_t size) {
        size = (size + 255) & ~int64_t(255);
        used_ -= size;
        auto it = free_.emplace(off, size).first;
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
    int64_t used() const { return used_; }
    int64_t cap() const { return cap_; }

   private:
    int64_t cap_, used_ = 0;
    std::map<int64_t, int64_t> free_;
};

// --------------------------------------------------------------- executors
struct Executor {
    virtual ~Executor() {}
    virtual int start(int64_t arena_bytes, std::string &err) = 0;
    virtual int admit(Slot &s, const Staged &p, int64_t off, const gabi_solve_opts &o,
                      std::string &err) = 0;
    virtual int init(std::vector<Slot *> &fresh, std::string &err) = 0;
    virtual int round(std::vector<Slot *> &active, std::string &err) = 0;
    virtual int finish(std::vector<Slot *> &done, std::string &err) = 0;
    virtual void stop() {}
};

class HipExecutor : public Executor {
   public:
    HipExecutor(int device, bool use_graph) : device_(device), use_graph_(use_graph) {}
    ~HipExecutor() override { stop(); }

    int start(int64_t arena_bytes, std::string &err) override {
        if (hipSetDevice(device_) != hipSuccess) {
            err = "cannot use device " + std::to_string(device_);
            return GABI_EDEVICE;
        }
        if (hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess ||
            hipStreamCreateWithFlags(&capture_, hipStreamNonBlocking) != hipSuccess) {
            err = "stream creation failed";
            return GABI_EDEVICE;
        }
        if (hipMalloc(&base_, std::max<int64_t>(arena_bytes, 256)) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            err = "arena allocation of " + std::to_string(arena_bytes) + " bytes failed";
            return GABI_ENOMEM;
        }
        return GABI_OK;
    }

    void stop() override {
        if (stream_) (void)hipStreamSynchronize(stream_);
        batch_free(active_);
        batch_free(tmp_);
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
        if (stream_) (void)hipStreamDestroy(stream_);
        if (capture_) (void)hipStreamDestroy(capture_);
        stream_ = capture_ = nullptr;
    }

    int admit(Slot &s, const Staged &p, int64_t off, const gabi_solve_opts &o,
              std::string &err) override {
        s.mem = static_cast<char *>(base_) + off;
        s.uid = next_slot_uid();
        s.mol = Mol{};
        slot_carve(s, p.n, p.nc, o.restart);
        slot_set_params(s, p.eps1, p.eps2, p.kappa);
        slot_set_mode(s, o.mode == GABI_SOLVE_MIXED_IR ? kModeMixed : kModeFP64);
        set_solve_targets(s, o.tol, o.inner_tol, o.maxit);
        s.mol.m = o.restart;
        if (upload_geometry(s, p.pos.data(), p.nrm.data(), p.geo32.data(), stream_) ||
            upload_charges(s, p.chg.data(), stream_)) {
            err = "upload failed";
            return GABI_EDEVICE;
        }
        return GABI_OK;
    }

    int init(std::vector<Slot *> &fresh, std::string &err) override {
        if (fresh.empty()) return GABI_OK;
        int rc = use(tmp_, fresh, err);
        if (rc) return rc;
        enqueue_init(tmp_, stream_, false, nullptr);
        return read(tmp_, err);
    }

    int round(std::vector<Slot *> &active, std::string &err) override {
        if (active.empty()) return GABI_OK;
        std::vector<int64_t> uids;
        for (const Slot *s : active) uids.push_back(s->uid);
        if (uids != active_uids_) {
            int rc = use(active_, active, err);
            if (rc) return rc;
            active_uids_ = uids;
            rounds_since_build_ = 0;
        }
        // capture once the set has been stable for a round
        const bool graph = use_graph_ && rounds_since_build_ >= 1;
        int rc = run_round(active_, stream_, capture_, nullptr, graph, err);
        if (rc) return rc;
        ++rounds_since_build_;
        return read(active_, err);
    }

    int finish(std::vector<Slot *> &done, std::string &err) override {
        if (done.empty()) return GABI_OK;
        int rc = use(tmp_, done, err);
        if (rc) return rc;
        enqueue_finalize(tmp_, stream_);
        for (Slot *s : done)
            if (s->u_out)
                (void)hipMemcpyAsync(s->u_out, s->mol.sol, sizeof(double) * 2 * s->mol.n,
                                     hipMemcpyDeviceToHost, stream_);
        return read(tmp_, err);
    }

   private:
    int use(Batch &b, std::vector<Slot *> &slots, std::string &err) {
        b.slots = slots;
        b.mode = slots.empty() ? 0 : slots[0]->mol.mode;
        return batch_build(b, stream_, err);
    }
    int read(Batch &b, std::string &err) {
        enqueue_gather(b, stream_);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(stream_);
        if (e != hipSuccess) {
            err = std::string("device error: ") + hipGetErrorString(e);
            return GABI_EDEVICE;
        }
        for (size_t k = 0; k < b.slots.size(); ++k) b.slots[k]->host_st = b.h_status[k];
        return GABI_OK;
    }

    int device_;
    bool use_graph_;
    hipStream_t stream_ = nullptr, capture_ = nullptr;
    void *base_ = nullptr;
    Batch active_, tmp_;
    std::vector<int64_t> active_uids_;  // slots active_ was built for
    int rounds_since_build_ = 0;
};

// Host-only executor: the scheduler's admission and accounting without a
// device.  A request converges after ceil(N / 4096) rounds; each round
// takes round_seconds.
class MockExecutor : public Executor {
   public:
    explicit MockExecutor(double round_seconds) : dt_(round_seconds) {}
    int start(int64_t, std::string &) override { return GABI_OK; }
    int admit(Slot &s, const Staged &p, int64_t, const gabi_solve_opts &o,
              std::string &) override {
        s.uid = next_slot_uid();
        s.mol = Mol{};
        s.mol.n = (int32_t)p.n;
        s.mol.nc = (int32_t)p.nc;
        s.mol.m = o.restart;
        s.mol.mode = o.mode == GABI_SOLVE_MIXED_IR ? kModeMixed : kModeFP64;
        s.mol.maxit = o.maxit;
        s.mol.tol0 = o.tol;
        return GABI_OK;
    }
    int init(std::vector<Slot *> &fresh, std::string &) override {
        for (Slot *s : fresh) {
            s->host_st = KrylovStatus{};
            s->host_st.beta0 = 1.0;
            s->host_st.rnorm = 1.0;
            s->host_st.maxit = s->mol.maxit;
            s->host_st.tol0 = s->mol.tol0;
        }
        return GABI_OK;
    }
    int round(std::vector<Slot *> &active, std::string &) override {
        if (dt_ > 0) std::this_thread::sleep_for(std::chrono::duration<double>(dt_));
        for (Slot *s : active) {
            KrylovStatus &st = s->host_st;
            const int need = (s->mol.n + 4095) / 4096;
            st.iters += std::min(s->mol.m, std::max(1, st.maxit - st.iters));
            const int done_rounds = s->rounds + 1;
            st.rnorm = std::pow(0.1, done_rounds);
            st.converged = done_rounds >= need ? 1 : 0;
            if (st.converged) st.rnorm = 0.0;
        }
        return GABI_OK;
    }
    int finish(std::vector<Slot *> &done, std::string &) override {
        for (Slot *s : done) s->host_st.energy = -(double)s->mol.n;
        return GABI_OK;
    }

   private:
    double dt_;
};

// ---------------------------------------------------------------- results
bool slot_finished(const Slot &s, const gabi_solve_opts &o) {
    const KrylovStatus &st = s.host_st;
    if (st.converged) return true;
    if (st.iters >= st.maxit) return true;
    if (s.mol.mode == kModeMixed && s.rounds >= o.max_outer) return true;
    return false;
}

gabi_result make_result(const Slot &s) {
    const KrylovStatus &st = s.host_st;
    gabi_result r{};
    r.tag = s.tag;
    r.ticket = s.ticket;
    r.status = st.converged ? GABI_OK : GABI_NOT_CONVERGED;
    r.energy = st.energy;
    r.info.iterations = st.iters;
    r.info.restarts = s.rounds;
    if (s.mol.mode == kModeMixed) {
        r.info.matvecs_fp32 = st.iters;
        r.info.matvecs_fp64 = s.rounds;
        r.info.outer = s.rounds;
    } else {
        r.info.matvecs_fp64 = st.iters + s.rounds;
    }
    r.info.rel_residual = st.beta0 > 0 ? st.rnorm / st.beta0 : 0.0;
    r.info.converged = st.converged;
    r.info.seconds = s.t_done - s.t_admit;
    r.t_submit = s.t_submit;
    r.t_admit = s.t_admit;
    r.t_done = s.t_done;
    r.device_bytes = s.bytes;
    return r;
}

}  // namespace
}  // namespace gabi

using namespace gabi;

// ------------------------------------------------------------------ server
struct gabi_server {
    std::unique_ptr<Executor> ex;
    gabi_solve_opts opts{};
    int32_t max_slots = 1;
    double t0 = 0;
    std::unique_ptr<Arena> arena;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Staged>> queue;
    std::deque<gabi_result> results;
    std::vector<std::unique_ptr<Slot>> active;
    bool stop = false;
    std::string err;
    gabi_server_stats stats{};
    int64_t seq = 0;
    std::thread worker;

    // round cap (gabi_server_set_round_cap): slack < 0 runs every active
    // request each round
    std::atomic<double> cap_slack{-1.0};
    std::atomic<int64_t> cap_floor_n{0};

    double clock() const { return now_s() - t0; }
    void run();
    std::vector<Slot *> capped_round(const std::vector<Slot *> &iterate) const;
};

// The requests of a round under the cap: in admission order (the active
// list's order), the oldest always, then each one whose work keeps the
// round's total within max((1 + slack) x the oldest's work, floor^2), where
// a request's work is N^2 (its products' pairs).  The others wait for a
// later round; no request's arithmetic depends on which rounds it joins.
std::vector<Slot *> gabi_server::capped_round(const std::vector<Slot *> &iterate) const {
    if (iterate.empty()) return iterate;
    auto work = [](const Slot *s) { return (double)s->mol.n * (double)s->mol.n; };
    const double floor_n = (double)cap_floor_n.load();
    const double cap = std::max((1.0 + cap_slack.load()) * work(iterate[0]), floor_n * floor_n);
    std::vector<Slot *> out;
    double sum = 0.0;
    for (Slot *s : iterate) {
        const double w = work(s);
        if (out.empty() || sum + w <= cap) {
            out.push_back(s);
            sum += w;
        }
    }
    return out;
}

void gabi_server::run() {
    std::string e;
    for (;;) {
        std::vector<std::pair<std::unique_ptr<Staged>, int64_t>> fresh;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) return;
                while (!queue.empty() && (int32_t)active.size() + (int32_t)fresh.size() < max_slots) {
                    int64_t off = 0;
                    if (!arena->alloc(queue.front()->bytes, off)) break;
                    fresh.emplace_back(std::move(queue.front()), off);
                    queue.pop_front();
                }
                if (!fresh.empty() || !active.empty()) break;
                cv_work.wait(lk);
            }
        }
        // admit and initialise the new requests (outside the lock)
        std::vector<Slot *> init_list;
        std::vector<std::unique_ptr<Slot>> admitted;
        for (auto &f : fresh) {
            auto s = std::make_unique<Slot>();
            s->tag = f.first->tag;
            s->ticket = f.first->ticket;
            s->u_out = f.first->u_out;
            s->t_submit = f.first->t_submit;
            s->t_admit = clock();
            s->bytes = f.first->bytes;
            s->arena_off = f.second;
            s->from_arena = true;
            int rc = ex->admit(*s, *f.first, f.second, opts, e);
            if (rc) {
                std::lock_guard<std::mutex> lk(mu);
                err = e;
                gabi_result r{};
                r.tag = s->tag;
                r.ticket = s->ticket;
                r.status = rc;
                r.t_submit = s->t_submit;
                r.t_admit = s->t_admit;
                r.t_done = clock();
                results.push_back(r);
                arena->release(s->arena_off, s->bytes);
                stats.failed++;
                stats.completed++;
                cv_done.notify_all();
                continue;
            }
            init_list.push_back(s.get());
            admitted.push_back(std::move(s));
        }
        int rc = ex->init(init_list, e);
        std::vector<Slot *> run_list;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (auto &s : admitted) active.push_back(std::move(s));
            stats.admitted += (int64_t)init_list.size();
            stats.peak_bytes = std::max(stats.peak_bytes, arena->used());
            stats.max_active = std::max<int64_t>(stats.max_active, (int64_t)active.size());
            for (auto &s : active) run_list.push_back(s.get());
        }
        // one round for the active requests that still iterate: all of them,
        // or under a round cap those that fit, oldest first
        std::vector<Slot *> iterate;
        for (Slot *s : run_list)
            if (!slot_finished(*s, opts)) iterate.push_back(s);
        if (cap_slack >= 0.0) iterate = capped_round(iterate);
        if (rc == GABI_OK && !iterate.empty()) {
            rc = ex->round(iterate, e);
            for (Slot *s : iterate) s->rounds++;
            std::lock_guard<std::mutex> lk(mu);
            stats.rounds++;
        }
        if (rc) {  // device failure: fail every active request and stop
            std::lock_guard<std::mutex> lk(mu);
            err = e;
            for (auto &s : active) {
                gabi_result r = make_result(*s);
                r.status = rc;
                r.t_done = clock();
                results.push_back(r);
                stats.failed++;
                stats.completed++;
            }
            active.clear();
            stop = true;
            cv_done.notify_all();
            return;
        }
        std::vector<Slot *> done;
        for (Slot *s : run_list)
            if (slot_finished(*s, opts)) done.push_back(s);
        if (!done.empty()) {
            rc = ex->finish(done, e);
            std::lock_guard<std::mutex> lk(mu);
            const double t = clock();
            for (Slot *s : done) {
                s->t_done = t;
                gabi_result r = make_result(*s);
                if (rc) r.status = rc;
                results.push_back(r);
                arena->release(s->arena_off, s->bytes);
                stats.completed++;
                if (r.status < 0) stats.failed++;
            }
            active.erase(std::remove_if(active.begin(), active.end(),
                                        [&](const std::unique_ptr<Slot> &p) {
                                            return std::find(done.begin(), done.end(), p.get()) !=
                                                   done.end();
                                        }),
                         active.end());
            cv_done.notify_all();
        }
    }
}

extern "C" {

int64_t gabi_solve_footprint(int64_t n, int64_t nc, int32_t restart) {
    if (n < 1 || nc < 0 || restart < 1 || restart > kMaxRestart) return -1;
    return slot_bytes(n, nc, restart);
}

int gabi_batch_solve(int device, int64_t nprob, const gabi_problem *probs,
                     const gabi_solve_opts *opts, gabi_result *results) {
    if (nprob < 0 || (nprob > 0 && (!probs || !results))) return GABI_EINVAL;
    gabi_solve_opts o;
    std::string err;
    if (opts_check(opts, &o, err)) return GABI_EINVAL;
    if (o.mode == GABI_SOLVE_TREE_IR) return GABI_EINVAL;  // single contexts only
    std::vector<Staged> staged((size_t)nprob);
    int64_t total = 0;
    std::vector<int64_t> offs((size_t)nprob);
    for (int64_t k = 0; k < nprob; ++k) {
        results[k] = gabi_result{};
        results[k].tag = probs[k].tag;
        results[k].ticket = k;
        int rc = stage_problem(probs[k], o.restart, staged[k], err);
        if (rc) {
            results[k].status = rc;
            staged[k].n = 0;
            continue;
        }
        offs[k] = total;
        total += (staged[k].bytes + 255) & ~int64_t(255);
    }
    HipExecutor ex(device, o.use_graph != 0);
    int rc = ex.start(total, err);
    if (rc) return rc;
    const double t0 = now_s();
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<Slot *> active;
    std::vector<int64_t> index;
    for (int64_t k = 0; k < nprob; ++k) {
        if (staged[k].n == 0) continue;
        auto s = std::make_unique<Slot>();
        s->tag = staged[k].tag;
        s->ticket = k;
        s->u_out = staged[k].u_out;
        s->bytes = staged[k].bytes;
        s->t_submit = s->t_admit = 0.0;
        if ((rc = ex.admit(*s, staged[k], offs[k], o, err))) return rc;
        active.push_back(s.get());
        index.push_back(k);
        slots.push_back(std::move(s));
    }
    if ((rc = ex.init(active, err))) return rc;
    std::map<Slot *, int64_t> where;
    for (size_t i = 0; i < active.size(); ++i) where[active[i]] = index[i];
    auto retire = [&](std::vector<Slot *> &done) -> int {
        if (done.empty()) return GABI_OK;
        int e = ex.finish(done, err);
        if (e) return e;
        const double t = now_s() - t0;
        for (Slot *s : done) {
            s->t_done = t;
            results[where[s]] = make_result(*s);
        }
        return GABI_OK;
    };
    for (;;) {
        std::vector<Slot *> done, keep;
        for (Slot *s : active) (slot_finished(*s, o) ? done : keep).push_back(s);
        if ((rc = retire(done))) return rc;
        active.swap(keep);
        if (active.empty()) break;
        if ((rc = ex.round(active, err))) return rc;
        for (Slot *s : active) s->rounds++;
    }
    ex.stop();
    return GABI_OK;
}

int gabi_server_create(gabi_server **out, int device, int64_t budget_bytes,
                       int32_t max_slots, const gabi_solve_opts *opts,
                       double mock_round_seconds) {
    if (!out || budget_bytes <= 0 || max_slots < 1) return GABI_EINVAL;
    *out = nullptr;
    auto srv = std::make_unique<gabi_server>();
    std::string err;
    if (opts_check(opts, &srv->opts, err) || srv->opts.mode == GABI_SOLVE_TREE_IR)
        return GABI_EINVAL;  // the treecode refinement is for single contexts
    srv->max_slots = max_slots;
    srv->arena = std::make_unique<Arena>(budget_bytes);
    srv->stats.budget_bytes = budget_bytes;
    if (device >= 0)
        srv->ex = std::make_unique<HipExecutor>(device, srv->opts.use_graph != 0);
    else
        srv->ex = std::make_unique<MockExecutor>(mock_round_seconds);
    int rc = srv->ex->start(budget_bytes, err);
    if (rc) return rc;
    srv->t0 = now_s();
    gabi_server *s = srv.release();
    s->worker = std::thread([s, device]() {
        if (device >= 0) (void)hipSetDevice(device);
        s->run();
    });
    *out = s;
    return GABI_OK;
}

int gabi_server_submit(gabi_server *srv, const gabi_problem *p, int64_t *ticket) {
    if (!srv || !p) return GABI_EINVAL;
    auto st = std::make_unique<Staged>();
    std::string err;
    int rc = stage_problem(*p, srv->opts.restart, *st, err);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (rc) {
        srv->err = err;
        return rc;
    }
    if (st->bytes > srv->arena->cap()) {
        srv->err = "request needs " + std::to_string(st->bytes) +
                   " device bytes, more than the whole budget";
        return GABI_ENOMEM;
    }
    if (srv->stop) {
        srv->err = "server stopped";
        return GABI_EBUSY;
    }
    st->t_submit = srv->clock();
    st->ticket = srv->seq;
    if (ticket) *ticket = srv->seq;
    srv->seq++;
    srv->queue.push_back(std::move(st));
    srv->stats.submitted++;
    srv->cv_work.notify_all();
    return GABI_OK;
}

int gabi_server_poll(gabi_server *srv, gabi_result *out, int32_t max, int32_t *count) {
    if (!srv || (max > 0 && !out)) return GABI_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    int32_t c = 0;
    while (c < max && !srv->results.empty()) {
        out[c++] = srv->results.front();
        srv->results.pop_front();
    }
    if (count) *count = c;
    return GABI_OK;
}

int gabi_server_drain(gabi_server *srv, double timeout_s) {
    if (!srv) return GABI_EINVAL;
    std::unique_lock<std::mutex> lk(srv->mu);
    const bool ok = srv->cv_done.wait_for(
        lk, std::chrono::duration<double>(std::max(0.0, timeout_s)),
        [&] { return srv->stats.completed >= srv->stats.submitted || srv->stop; });
    return ok && srv->stats.completed >= srv->stats.submitted ? GABI_OK : GABI_EBUSY;
}

int gabi_server_set_round_cap(gabi_server *srv, double slack, int64_t floor_elements) {
    if (!srv || !std::isfinite(slack) || floor_elements < 0) return GABI_EINVAL;
    srv->cap_slack.store(slack);
    srv->cap_floor_n.store(floor_elements);
    return GABI_OK;
}

int gabi_server_stats_get(gabi_server *srv, gabi_server_stats *out) {
    if (!srv || !out) return GABI_EINVAL;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->stats;
    out->queued = (int64_t)srv->queue.size();
    out->active = (int64_t)srv->active.size();
    out->bytes_in_use = srv->arena->used();
    out->peak_bytes = std::max(srv->stats.peak_bytes, out->bytes_in_use);
    return GABI_OK;
}

double gabi_server_clock(gabi_server *srv) { return srv ? srv->clock() : 0.0; }

const char *gabi_server_last_error(gabi_server *srv) {
    return srv ? srv->err.c_str() : "null server";
}

void gabi_server_destroy(gabi_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        srv->cv_work.notify_all();
    }
    if (srv->worker.joinable()) srv->worker.join();
    srv->ex->stop();
    delete srv;
}

}  // extern "C"
