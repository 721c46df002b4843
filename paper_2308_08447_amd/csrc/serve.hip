// serve.hip -- continuous batching of independent LLG simulations on one GPU.
//
// Two threads with a HIP stream each:
//   worker       loops: (1) admits queued requests while their device memory
//                fits the budget (the transformed tensor of a mesh is counted
//                once for all resident requests of that mesh and shared through
//                the process-wide cache), scanning the queue in arrival order:
//                a request that fits may pass one that does not, until the one
//                at the head has been passed MAX_BYPASS times, after which the
//                freed memory is held for it; (2) moves requests whose set-up
//                is done into the active set; (3) advances every active request
//                by q RK4 steps, q = the fewest steps any active request still
//                needs (at most QUANTUM; prepared requests join in groups, see
//                MERGE_COUNT), with shared launches: one launch per
//                FFT stage and transform length, one LLG launch per 16 meshes;
//                with SERVE_GRAPHS the launches of one step are captured into a
//                HIP graph once per distinct active set and replayed; (4)
//                retires finished requests (copy m to host, free their memory).
//   preparation  creates the plans of admitted requests (a new mesh's FP64
//                tensor set-up included) and uploads m0 on its own stream, so
//                that this work overlaps the worker's steps instead of stalling
//                them.
// Each request's arithmetic does not depend on which other requests share its
// launches, so a result is bit-identical to running the request alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "plan.h"

namespace {

using Clock = std::chrono::steady_clock;
constexpr int QUANTUM = 16;
constexpr int MAX_BYPASS = 16;  // admissions that may pass the request at the head
constexpr int MERGE_COUNT = 16;  // ready requests that join the active set at once
constexpr auto MERGE_WAIT = std::chrono::milliseconds(20);

struct Request {
    uint64_t id = 0;
    demag_mesh mesh{};
    llg_params prm{};
    double dt = 0.0;
    int nsteps = 0;
    std::vector<float> host;  // m0 on submission, the result on completion
    int steps_done = 0;
    enum { QUEUED, PREPARING, READY, ACTIVE, DONE } state = QUEUED;
    size_t need = 0;          // budget reserved at admission
    int bypassed = 0;         // admissions that passed this request while it waited
    int status = DEMAG_OK;
    std::string error;
    Clock::time_point t_submit, t_done, t_ready;
    demag_plan* plan = nullptr;
    float* m = nullptr;
    size_t bytes = 0;         // workspace + RK4 + m
    dm::Geometry g{};
};

using ShapeKey = std::tuple<int, int, int, double, double, double>;
ShapeKey shape_key(const demag_mesh& m) { return ShapeKey{m.nx, m.ny, m.nz, m.dx, m.dy, m.dz}; }

}  // namespace

struct demag_server {
    size_t budget = 0;
    int max_active = 1;
    uint32_t flags = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t prep_stream = nullptr;  // plan set-up and m0 uploads (default priority)
    std::thread worker, prep;
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_prep;
    std::deque<Request*> queue;
    std::deque<Request*> preparing;      // admitted, set-up pending
    std::vector<Request*> ready;         // set up, not yet in the active set
    std::vector<Request*> active;
    int admitted = 0;                    // preparing + ready + active
    int in_prep = 0;                     // requests the preparation thread is setting up
    std::unordered_map<uint64_t, Request*> reqs;
    std::map<ShapeKey, int> active_shapes;  // active requests per mesh (tensor held once)
    uint64_t next_id = 1;
    bool stop = false;
    size_t used = 0;
    serve_stats st{};
    // graph of one RK4 step of the current active set
    hipGraphExec_t exec = nullptr;
    std::vector<uint64_t> graph_ids;
};

namespace {

size_t spectrum_bytes(const dm::Geometry& g) { return g.k_elems() * sizeof(float); }

void release(demag_server* s, Request* r) {
    if (r->plan) dm::free_plan(r->plan);
    if (r->m) (void)hipFree(r->m);
    r->plan = nullptr;
    r->m = nullptr;
}

// Called with the lock held; returns the bytes to add if r were admitted now.
size_t admission_bytes(demag_server* s, const Request* r) {
    size_t b = r->bytes;
    if (s->active_shapes[shape_key(r->mesh)] == 0) b += spectrum_bytes(r->g);
    return b;
}

// bytes returned to the budget when r retires (lock held): its own memory plus
// the tensor if no other active request holds the mesh
size_t admission_bytes_release(demag_server* s, Request* r) {
    size_t b = r->bytes;
    int& n = s->active_shapes[shape_key(r->mesh)];
    if (--n == 0) b += spectrum_bytes(r->g);
    return b;
}

void finish(demag_server* s, Request* r, int status, const std::string& err) {
    r->status = status;
    r->error = err;
    r->state = Request::DONE;
    r->t_done = Clock::now();
    if (status == DEMAG_OK) {
        s->st.completed++;
        s->st.cell_steps += (double)r->g.cells() * r->nsteps;
    } else {
        s->st.failed++;
    }
}

// Admits queued requests (worker thread): reserves their budget and hands them
// to the preparation thread.  Requests are taken in arrival order; one that
// does not fit yet may be passed by later ones that do, until it has been
// passed MAX_BYPASS times.
void admit(demag_server* s) {
    std::lock_guard<std::mutex> lk(s->mu);
    bool handed = false;
    for (auto it = s->queue.begin(); it != s->queue.end() && s->admitted < s->max_active;) {
        Request* r = *it;
        const size_t need = admission_bytes(s, r);
        if (need > s->budget) {  // can never fit
            it = s->queue.erase(it);
            finish(s, r, DEMAG_ENOMEM, "request needs more device memory than the budget");
            s->cv_done.notify_all();
            continue;
        }
        if (s->used + need > s->budget) {
            if (r->bypassed >= MAX_BYPASS) break;  // hold the memory that frees up for it
            ++it;
            continue;
        }
        for (auto jt = s->queue.begin(); jt != it; ++jt) (*jt)->bypassed++;
        it = s->queue.erase(it);
        r->need = need;
        s->used += need;
        s->active_shapes[shape_key(r->mesh)]++;
        if (s->used > s->st.peak_bytes) s->st.peak_bytes = s->used;
        r->state = Request::PREPARING;
        s->preparing.push_back(r);
        s->admitted++;
        handed = true;
    }
    if (handed) s->cv_prep.notify_one();
}

// Preparation thread: plan (tensor set-up on first use of a mesh), RK4
// buffers, m0 upload, on its own stream.  It takes every request admitted so
// far as one group and hands the group over when all of it is ready, so a
// burst of arrivals joins the active set together.
void prep_main(demag_server* s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        std::deque<Request*> group;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_prep.wait(lk, [&] { return s->stop || !s->preparing.empty(); });
            if (s->stop) return;
            group.swap(s->preparing);
            s->in_prep = (int)group.size();
        }
        std::vector<std::tuple<Request*, int, std::string>> failed;
        std::vector<Request*> ok;
        for (Request* r : group) {
            int rc = dm::create_plan(&r->mesh, DEMAG_FP32, s->prep_stream, &r->plan);
            if (!rc) rc = dm::ensure_rk(r->plan);
            if (!rc) rc = dm::dev_alloc((void**)&r->m, r->host.size() * sizeof(float), "request m");
            if (!rc && hipMemcpyAsync(r->m, r->host.data(), r->host.size() * sizeof(float),
                                      hipMemcpyHostToDevice, s->prep_stream) != hipSuccess)
                rc = dm::fail(DEMAG_EHIP, "copy of m0 to the device failed");
            if (rc) {
                failed.emplace_back(r, rc, std::string(demag_last_error()));
                release(s, r);
            } else {
                ok.push_back(r);
            }
        }
        if (!ok.empty() && hipStreamSynchronize(s->prep_stream) != hipSuccess) {
            for (Request* r : ok) {
                failed.emplace_back(r, DEMAG_EHIP, "stream synchronisation failed");
                release(s, r);
            }
            ok.clear();
        }
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& f : failed) {
            Request* r = std::get<0>(f);
            s->used -= admission_bytes_release(s, r);
            s->admitted--;
            finish(s, r, std::get<1>(f), std::get<2>(f));
        }
        const auto now = Clock::now();
        for (Request* r : ok) {
            r->state = Request::READY;
            r->t_ready = now;
            s->ready.push_back(r);
        }
        s->in_prep = 0;
        if (!failed.empty()) s->cv_done.notify_all();
        s->cv_work.notify_one();
    }
}

int capture_step(demag_server* s, const std::vector<dm::LLGStep>& steps) {
    if (s->exec) {
        (void)hipGraphExecDestroy(s->exec);
        s->exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    DM_HIP(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    int rc = dm::rk4_step_batch(steps.data(), (int)steps.size(), s->stream);
    hipError_t e = hipStreamEndCapture(s->stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return dm::fail(DEMAG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&s->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        s->exec = nullptr;
        return dm::fail(DEMAG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    s->st.graph_captures++;
    return DEMAG_OK;
}

// Advances every active request by q steps and retires the finished ones.
void iterate(demag_server* s) {
    std::vector<Request*> act;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        act = s->active;
    }
    int q = QUANTUM;
    std::vector<dm::LLGStep> steps;
    std::vector<uint64_t> ids;
    for (Request* r : act) {
        q = std::min(q, r->nsteps - r->steps_done);
        steps.push_back(dm::LLGStep{r->plan, r->m, r->prm, r->dt});
        ids.push_back(r->id);
    }
    int rc = DEMAG_OK;
    if (q > 0) {
        if (s->flags & SERVE_GRAPHS) {
            if (!s->exec || ids != s->graph_ids) {
                rc = capture_step(s, steps);
                s->graph_ids = rc ? std::vector<uint64_t>() : ids;
            }
            for (int i = 0; i < q && !rc; ++i)
                if (hipGraphLaunch(s->exec, s->stream) != hipSuccess)
                    rc = dm::fail(DEMAG_EHIP, "graph launch failed");
        } else {
            for (int i = 0; i < q && !rc; ++i)
                rc = dm::rk4_step_batch(steps.data(), (int)steps.size(), s->stream);
        }
        if (!rc && hipStreamSynchronize(s->stream) != hipSuccess)
            rc = dm::fail(DEMAG_EHIP, "stream synchronisation failed");
    }
    std::string err = rc ? demag_last_error() : std::string();
    std::vector<Request*> done;
    for (Request* r : act) {
        if (rc) {
            done.push_back(r);
            continue;
        }
        r->steps_done += q;
        if (r->steps_done >= r->nsteps) done.push_back(r);
    }
    for (Request* r : done) {
        int frc = rc;
        if (!frc && hipMemcpy(r->host.data(), r->m, r->host.size() * sizeof(float),
                              hipMemcpyDeviceToHost) != hipSuccess)
            frc = dm::fail(DEMAG_EHIP, "copy of the result to the host failed");
        std::string ferr = frc ? (rc ? err : std::string(demag_last_error())) : std::string();
        release(s, r);
        std::lock_guard<std::mutex> lk(s->mu);
        s->used -= admission_bytes_release(s, r);
        s->admitted--;
        finish(s, r, frc, ferr);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.iterations++;
    if (!done.empty()) {
        std::vector<Request*> keep;
        for (Request* r : s->active)
            if (r->state == Request::ACTIVE) keep.push_back(r);
        s->active.swap(keep);
        s->cv_done.notify_all();
    }
}

void worker_main(demag_server* s) {
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            // sleep while nothing can advance: no active request, nothing ready,
            // and the queue empty or blocked until memory frees up
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] {
                return s->stop || !s->active.empty() || !s->ready.empty() ||
                       (!s->queue.empty() && s->admitted < s->max_active && s->preparing.empty() &&
                        s->in_prep == 0);
            });
            if (s->stop) return;
        }
        admit(s);
        bool any;
        {
            // Ready requests join the active set together, so that a burst of
            // arrivals changes the captured step once, not once per request:
            // when nothing is active, when nothing else is being prepared, when
            // MERGE_COUNT are waiting or the oldest has waited MERGE_WAIT.
            std::lock_guard<std::mutex> lk(s->mu);
            const bool merge = !s->ready.empty() &&
                               (s->active.empty() || (s->preparing.empty() && s->in_prep == 0) ||
                                (int)s->ready.size() >= MERGE_COUNT ||
                                Clock::now() - s->ready.front()->t_ready >= MERGE_WAIT);
            if (merge) {
                for (Request* r : s->ready) {
                    r->state = Request::ACTIVE;
                    s->active.push_back(r);
                }
                s->ready.clear();
            }
            any = !s->active.empty();
        }
        if (any) iterate(s);
    }
}

}  // namespace

extern "C" {

int serve_open(size_t hbm_budget_bytes, int32_t max_active, uint32_t flags, demag_server** out) {
    if (!out) return dm::fail(DEMAG_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return dm::fail(DEMAG_EINVAL, "budget must be > 0");
    if (max_active < 1 || max_active > 1024) return dm::fail(DEMAG_EINVAL, "max_active must be in 1..1024");
    if (flags & ~(uint32_t)SERVE_GRAPHS) return dm::fail(DEMAG_EINVAL, "unknown flags");
    demag_server* s = new (std::nothrow) demag_server();
    if (!s) return dm::fail(DEMAG_ENOMEM, "host allocation failed");
    s->budget = hbm_budget_bytes;
    s->max_active = max_active;
    s->flags = flags;
    (void)hipGetDevice(&s->device);
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return dm::fail(DEMAG_EHIP, "hipStreamCreate failed");
    }
    if (hipStreamCreateWithFlags(&s->prep_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipStreamDestroy(s->stream);
        delete s;
        return dm::fail(DEMAG_EHIP, "hipStreamCreate failed");
    }
    s->worker = std::thread(worker_main, s);
    s->prep = std::thread(prep_main, s);
    *out = s;
    return DEMAG_OK;
}

int serve_submit(demag_server* s, const demag_mesh* mesh, const llg_params* params, double dt,
                 int32_t nsteps, const float* m0_host, uint64_t* request_id) {
    if (!s || !mesh || !params || !m0_host || !request_id)
        return dm::fail(DEMAG_EINVAL, "NULL argument");
    dm::Geometry g;
    int rc = dm::check_mesh(mesh, &g);
    if (rc) return rc;
    if ((rc = dm::check_llg_params(params, dt, nsteps))) return rc;
    Request* r = new (std::nothrow) Request();
    if (!r) return dm::fail(DEMAG_ENOMEM, "host allocation failed");
    r->mesh = *mesh;
    r->prm = *params;
    r->dt = dt;
    r->nsteps = nsteps;
    r->g = g;
    r->host.assign(m0_host, m0_host + 3 * g.cells());
    r->bytes = dm::workspace_bytes(g, DEMAG_FP32) + dm::rk_bytes(g) + 3 * g.cells() * sizeof(float);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->st.submitted++;
        if (nsteps == 0) {
            finish(s, r, DEMAG_OK, "");
            s->cv_done.notify_all();
        } else {
            s->queue.push_back(r);
        }
        *request_id = r->id;
    }
    s->cv_work.notify_one();
    return DEMAG_OK;
}

int serve_wait(demag_server* s, uint64_t id, float* m_out_host, double* latency_s) {
    if (!s || !m_out_host) return dm::fail(DEMAG_EINVAL, "NULL argument");
    Request* r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end()) return dm::fail(DEMAG_EINVAL, "unknown request id");
        r = it->second;
        // the wait releases the lock: a concurrent serve_submit may insert into
        // (and rehash) the map, so the iterator is not used after it
        s->cv_done.wait(lk, [&] { return r->state == Request::DONE || s->stop; });
        if (r->state != Request::DONE) return dm::fail(DEMAG_EBUSY, "server closed before the request finished");
        s->reqs.erase(id);
    }
    std::copy(r->host.begin(), r->host.end(), m_out_host);
    if (latency_s) latency_s[0] = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    int status = r->status;
    std::string err = r->error;
    delete r;
    if (status) return dm::fail(status, err);
    return DEMAG_OK;
}

int serve_get_stats(demag_server* s, serve_stats* out) {
    if (!s || !out) return dm::fail(DEMAG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->active = (int32_t)s->active.size();
    out->queued = (int32_t)s->queue.size();
    out->bytes_in_use = s->used;
    return DEMAG_OK;
}

int serve_close(demag_server* s) {
    if (!s) return dm::fail(DEMAG_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    s->cv_prep.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->prep.joinable()) s->prep.join();
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamSynchronize(s->prep_stream);
    for (auto& kv : s->reqs) {
        release(s, kv.second);
        delete kv.second;
    }
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    (void)hipStreamDestroy(s->stream);
    (void)hipStreamDestroy(s->prep_stream);
    delete s;
    return DEMAG_OK;
}

}  // extern "C"
