// Serving loop of the shsph C ABI: a host thread per context that admits
// STEP / EVAL jobs in arrival order under an HBM budget and runs every pass
// as one batched pass over all running jobs (continuous batching: jobs join
// and leave at pass boundaries).  The one-at-a-time policy runs the same
// queue with a single job on the device, the plain baseline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/shsph.h"

// Internal entry points of api.cpp.
int shsph_internal_pass(shsph_ctx* c, const int64_t* handles, const double* dt, int32_t count);
int shsph_internal_inst_state(shsph_ctx* c, int64_t h, int64_t* n, int* has_force, double* dt_cfl,
                              int busy_delta);
void*& shsph_internal_server(shsph_ctx* c);
int shsph_internal_dtype(shsph_ctx* c);

namespace {

// HBM charged per particle by the admission rule.  State: the 14 pooled
// fields of the dtype plus the 32-bit id.  Work: what one pass allocates per
// particle -- keys and values of the sort (x2), the three key-order float4
// arrays, h copies, mask / scan / leaf arrays, Karras tables at 8 particles
// per leaf, the parent and box rows (2 n rows in a captured pass: leaves
// start at row n - instances), thermo / acc / Omega, and the ELL neighbour
// cache (32 words of 8 B per particle at the default capacity, 25 % headroom).
double state_per_particle(int dtype) { return 14.0 * (dtype == SHSPH_F32 ? 4 : 8) + 4.0; }
double work_per_particle(int dtype) { return dtype == SHSPH_F32 ? 544.0 : 880.0; }

struct Job {
    shsph_job spec;
    shsph_particles init;
    bool has_init = false;
    int64_t n = 0;
    double need_state = 0, need_work = 0;
    shsph_job_status st;
};

struct Server {
    shsph_ctx* ctx = nullptr;
    shsph_serve_config cfg;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> queue;          // pending, arrival order
    std::vector<uint64_t> running;
    std::unordered_map<uint64_t, Job> jobs;
    uint64_t next_ticket = 1;
    int admitting = 0;                   // jobs off the queue, instance being created
    double running_work = 0;             // work bytes charged to running jobs
    size_t pass_cap = 0;                 // jobs per pass (halved when a pass runs out of memory)
    size_t rot = 0;                      // first running job of the next capped pass
    bool stop = false;
    shsph_serve_counters stats;
    std::thread th;
};

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

double pool_state_bytes(Server* S)
{
    int64_t used = 0;
    shsph_pool_usage(S->ctx, &used, nullptr, nullptr);
    const int dt = shsph_internal_dtype(S->ctx);
    return (double)used * state_per_particle(dt < 0 ? SHSPH_F32 : dt);
}

bool handle_running(Server* S, int64_t h)
{
    for (uint64_t t : S->running)
        if (S->jobs[t].st.handle == h) return true;
    return false;
}

void finish(Server* S, Job& j, int state, int err, double t)
{
    j.st.state = state;
    j.st.error = err;
    j.st.t_done = t;
    if (state == SHSPH_JOB_DONE) ++S->stats.jobs_done; else ++S->stats.jobs_failed;
}

// Admit from the head of the queue while the rules allow (no overtaking).
void admit(Server* S, std::unique_lock<std::mutex>& lk)
{
    while (!S->queue.empty()) {
        const uint64_t t = S->queue.front();
        Job& j = S->jobs[t];
        const int cap = S->cfg.policy == SHSPH_SERVE_ONE_AT_A_TIME ? 1 : S->cfg.max_batch;
        if ((int)S->running.size() >= cap) return;
        if (S->cfg.max_batch_particles > 0 && !S->running.empty()) {
            int64_t np = 0;
            for (uint64_t r : S->running) np += S->jobs[r].n;
            if (np + j.n > S->cfg.max_batch_particles) return;
        }
        if (!j.has_init && handle_running(S, j.spec.handle)) return;
        const double need = (j.has_init ? j.need_state : 0.0) + j.need_work;
        const double used = pool_state_bytes(S) + S->running_work;
        if (used + need > S->cfg.budget_bytes) return;
        S->queue.pop_front();
        int64_t h = j.spec.handle;
        if (j.has_init) {
            ++S->admitting;
            lk.unlock();
            const int rc = shsph_instance_create(S->ctx, &j.init, &h);
            lk.lock();
            --S->admitting;
            if (rc != SHSPH_OK) { finish(S, j, SHSPH_JOB_FAILED, rc, now_s()); S->cv_done.notify_all(); continue; }
        }
        if (shsph_internal_inst_state(S->ctx, h, nullptr, nullptr, nullptr, +1) != SHSPH_OK) {
            finish(S, j, SHSPH_JOB_FAILED, SHSPH_EINVAL, now_s());
            S->cv_done.notify_all();
            continue;
        }
        j.st.handle = h;
        j.st.state = SHSPH_JOB_RUNNING;
        j.st.t_start = now_s();
        S->running.push_back(t);
        S->running_work += j.need_work;
        S->stats.peak_bytes = std::max(S->stats.peak_bytes, used + need);
    }
}

void loop(Server* S)
{
    std::unique_lock<std::mutex> lk(S->m);
    for (;;) {
        admit(S, lk);
        if (S->running.empty()) {
            if (S->stop && S->queue.empty()) break;
            // wait for a submission, or re-check the budget (instances
            // destroyed by the client free pool memory without a signal)
            S->cv_work.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        // one pass over the running jobs (all of them unless a pass ran out
        // of memory; then a rotating share): 0 = first derivatives of a CFL
        // job, 1 = evaluation, 2 = a step
        const size_t nr = S->running.size();
        const size_t m = std::min(nr, S->pass_cap ? S->pass_cap : nr);
        std::vector<int64_t> hs(m);
        std::vector<double> dts(m);
        std::vector<int> kind(m);
        std::vector<uint64_t> tk(m);
        for (size_t i = 0; i < m; ++i) tk[i] = S->running[(S->rot + i) % nr];
        S->rot = (S->rot + m) % nr;
        double np = 0;
        for (size_t i = 0; i < m; ++i) {
            Job& j = S->jobs[tk[i]];
            int64_t n = 0;
            int hf = 0;
            double dcfl = 0;
            shsph_internal_inst_state(S->ctx, j.st.handle, &n, &hf, &dcfl, 0);
            hs[i] = j.st.handle;
            np += (double)n;
            if (j.spec.kind == SHSPH_JOB_EVAL) { kind[i] = 1; dts[i] = 0.0; }
            else if (j.spec.dt > 0) { kind[i] = 2; dts[i] = j.spec.dt; }
            else if (!hf) { kind[i] = 0; dts[i] = 0.0; }
            else { kind[i] = 2; dts[i] = (std::isfinite(dcfl) && dcfl > 0) ? dcfl : -1.0; }
        }
        lk.unlock();
        // a CFL job without a usable dt is evaluated again (dt = 0) instead
        for (size_t i = 0; i < m; ++i)
            if (dts[i] < 0) { dts[i] = 0.0; kind[i] = 0; }
        const double t0 = now_s();
        const int rc = shsph_internal_pass(S->ctx, hs.data(), dts.data(), (int32_t)m);
        const double t1 = now_s();
        lk.lock();
        ++S->stats.passes;
        S->stats.particle_passes += np;
        S->stats.busy_s += t1 - t0;
        S->stats.peak_jobs = std::max<int64_t>(S->stats.peak_jobs, (int64_t)m);
        if (rc == SHSPH_ENOMEM && m > 1) {     // retry with half the jobs per pass
            S->pass_cap = m / 2;
            continue;
        }
        std::vector<uint64_t> done_now;
        for (size_t i = 0; i < m; ++i) {
            Job& j = S->jobs[tk[i]];
            ++j.st.passes;
            int end = 0, err = SHSPH_OK;
            if (rc != SHSPH_OK && rc != SHSPH_ENOCONV) { end = SHSPH_JOB_FAILED; err = rc; }
            else {
                shsph_info inf;
                if (shsph_instance_info(S->ctx, j.st.handle, &inf) == SHSPH_OK && inf.n_noconv > 0) {
                    end = SHSPH_JOB_FAILED;
                    err = SHSPH_ENOCONV;
                } else if (kind[i] == 1) {
                    end = SHSPH_JOB_DONE;
                } else if (kind[i] == 2 && ++j.st.steps_done >= j.spec.nsteps) {
                    end = SHSPH_JOB_DONE;
                }
            }
            if (!end) continue;
            done_now.push_back(tk[i]);
            finish(S, j, end, err, t1);
            shsph_internal_inst_state(S->ctx, j.st.handle, nullptr, nullptr, nullptr, -1);
            S->running_work -= j.need_work;
            if (j.spec.release) {
                shsph_instance_destroy(S->ctx, j.st.handle);
                j.st.handle = 0;
            }
        }
        std::vector<uint64_t> keep;
        for (uint64_t t : S->running)
            if (std::find(done_now.begin(), done_now.end(), t) == done_now.end()) keep.push_back(t);
        S->running.swap(keep);
        if (S->running.empty()) {
            S->running_work = 0;                       // no drift from rounding
            S->rot = 0;
        } else {
            S->rot %= S->running.size();
        }
        S->cv_done.notify_all();
    }
    S->cv_done.notify_all();
}

Server* server_of(shsph_ctx* c) { return c ? (Server*)shsph_internal_server(c) : nullptr; }

}  // namespace

extern "C" {

double shsph_clock(void) { return now_s(); }

int shsph_footprint(shsph_ctx* c, int64_t n, int32_t dtype, double* state_bytes, double* work_bytes)
{
    if (!c || n < 0 || (dtype != SHSPH_F32 && dtype != SHSPH_F64)) return SHSPH_EINVAL;
    if (state_bytes) *state_bytes = (double)n * state_per_particle(dtype);
    if (work_bytes) *work_bytes = (double)n * work_per_particle(dtype);
    return SHSPH_OK;
}

int shsph_serve_start(shsph_ctx* c, const shsph_serve_config* cfg)
{
    if (!c || !cfg) return SHSPH_EINVAL;
    if (server_of(c)) return SHSPH_ESTATE;
    if (!(cfg->budget_bytes > 0) || cfg->max_batch < 1 || cfg->max_batch > 2048 ||
        cfg->max_batch_particles < 0 ||
        (cfg->policy != SHSPH_SERVE_CONTINUOUS && cfg->policy != SHSPH_SERVE_ONE_AT_A_TIME))
        return SHSPH_EINVAL;
    Server* S = new Server();
    S->ctx = c;
    S->cfg = *cfg;
    memset(&S->stats, 0, sizeof(S->stats));
    shsph_internal_server(c) = S;
    S->th = std::thread(loop, S);
    return SHSPH_OK;
}

int shsph_submit(shsph_ctx* c, const shsph_job* job, uint64_t* ticket)
{
    Server* S = server_of(c);
    if (!S) return SHSPH_ESTATE;
    if (!job || !ticket) return SHSPH_EINVAL;
    if (job->kind != SHSPH_JOB_STEP && job->kind != SHSPH_JOB_EVAL) return SHSPH_EINVAL;
    if (job->kind == SHSPH_JOB_STEP && job->nsteps < 1) return SHSPH_EINVAL;
    if (!std::isfinite(job->dt)) return SHSPH_EINVAL;
    Job j;
    j.spec = *job;
    int dtype;
    if (job->init) {
        j.init = *job->init;
        j.has_init = true;
        j.n = j.init.n;
        dtype = j.init.dtype;
        if (j.n < 1 || (dtype != SHSPH_F32 && dtype != SHSPH_F64)) return SHSPH_EINVAL;
    } else {
        if (shsph_internal_inst_state(c, job->handle, &j.n, nullptr, nullptr, 0) != SHSPH_OK)
            return SHSPH_EINVAL;
        dtype = shsph_internal_dtype(c);
    }
    j.spec.init = nullptr;
    j.need_state = (double)j.n * state_per_particle(dtype);
    j.need_work = (double)j.n * work_per_particle(dtype);
    if ((j.has_init ? j.need_state : 0.0) + j.need_work > S->cfg.budget_bytes) return SHSPH_ENOMEM;
    memset(&j.st, 0, sizeof(j.st));
    j.st.state = SHSPH_JOB_PENDING;
    j.st.handle = j.has_init ? 0 : job->handle;
    std::lock_guard<std::mutex> lk(S->m);
    if (S->stop) return SHSPH_ESTATE;
    j.st.t_submit = now_s();
    const uint64_t t = S->next_ticket++;
    S->jobs[t] = j;
    S->queue.push_back(t);
    *ticket = t;
    S->cv_work.notify_one();
    return SHSPH_OK;
}

int shsph_poll(shsph_ctx* c, uint64_t ticket, shsph_job_status* st)
{
    Server* S = server_of(c);
    if (!S) return SHSPH_ESTATE;
    if (!st) return SHSPH_EINVAL;
    std::lock_guard<std::mutex> lk(S->m);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) return SHSPH_EINVAL;
    *st = it->second.st;
    return SHSPH_OK;
}

int shsph_serve_drain(shsph_ctx* c, double timeout_s)
{
    Server* S = server_of(c);
    if (!S) return SHSPH_ESTATE;
    std::unique_lock<std::mutex> lk(S->m);
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                           std::chrono::duration<double>(std::max(timeout_s, 0.0)));
    const bool ok = S->cv_done.wait_until(lk, until, [S] {
        return S->queue.empty() && S->running.empty() && S->admitting == 0;
    });
    return ok ? SHSPH_OK : SHSPH_ESTATE;
}

int shsph_serve_stats(shsph_ctx* c, shsph_serve_counters* out)
{
    Server* S = server_of(c);
    if (!S) return SHSPH_ESTATE;
    if (!out) return SHSPH_EINVAL;
    std::lock_guard<std::mutex> lk(S->m);
    *out = S->stats;
    return SHSPH_OK;
}

int shsph_serve_stop(shsph_ctx* c)
{
    Server* S = server_of(c);
    if (!S) return SHSPH_ESTATE;
    {
        std::lock_guard<std::mutex> lk(S->m);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();
    shsph_internal_server(c) = nullptr;
    delete S;
    return SHSPH_OK;
}

}  // extern "C"
