// Host side of the shsph C ABI: context, device buffers, and the sequences
// of kernel launches behind shsph_build_tree / _density / _force / _step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/shsph.h"
#include "kernels.hpp"

using namespace shsph;

namespace {

struct Buf {
    void* p = nullptr;
    size_t cap = 0;
};

enum State { ST_NONE = 0, ST_TREE = 1, ST_DENSITY = 2, ST_FORCE = 3 };

// Stages timed by the optional HIP-event profiler (one entry per launch group).
enum Stage {
    S_MORTON, S_SORT, S_GATHER, S_LEAVES, S_KARRAS, S_BOXES, S_STAGE1, S_STAGE2, S_DENSITY,
    S_FORCE, S_CORRECT, S_DENSITY_FORCE, S_NUM
};
const char* const STAGE_NAMES[S_NUM] = {
    "predict_morton", "radix_sort", "gather", "mask_reduce_compact", "karras", "boxes",
    "group_leaf_cache", "particle_cache", "density", "force", "correct", "density_force"
};

// A pooled instance: its fields live at [off, off + n) of the pool arrays.
struct Inst {
    i64 off = 0, n = 0;
    double mass = 0, lo[3] = { 0, 0, 0 }, hi[3] = { 0, 0, 0 };
    int periodic = 0;
    bool has_force = false;     // a derivative pass has run (CFL dt known)
    InstStat stat;              // reductions of the last pass
    double lambda_cfl = 1.0;    // CFL multiplier (App. G)
    int reruns = 0;             // corrector re-runs of the last pass
    int busy = 0;               // held by a running serving job
};

// Field pools of the context's instances (structure of arrays, one dtype).
// The free list maps offset -> length; neighbouring free ranges are merged.
enum PoolField { PF_X, PF_Y, PF_Z, PF_VX, PF_VY, PF_VZ, PF_U, PF_H, PF_AX, PF_AY, PF_AZ, PF_DU,
                 PF_RHO, PF_OMEGA, PF_PID, PF_NUM };
struct Pool {
    int dtype = -1;
    i64 cap = 0, used = 0;
    void* fld[PF_NUM] = {};
    std::map<i64, i64> free_;
};

struct Prof {
    bool on = false;
    std::vector<int> stage;
    std::vector<hipEvent_t> ev;     // 2 per record
    size_t used = 0;
    double ms[S_NUM] = {};
    long long launches[S_NUM] = {};
};

}  // namespace

struct shsph_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    shsph_params prm;
    std::string err;

    // shape of the current build
    int dtype = 0;
    i64 n = 0;
    int ninst = 0;
    i64 n_leaf = 0, n_internal = 0, n_groups = 0;
    i64 lbase = 0;                              // node of leaf 0: n - ninst (fixed per pass shape)
    bool capturing = false;                     // launches are being captured: no host reads
    // captured batched passes
    u64 alloc_gen = 0;                          // counts (re)allocations of device buffers
    u64 param_gen = 0;                          // counts parameter changes
    std::vector<i64> gkey;                      // the pass shape gexec was captured for
    std::vector<i64> last_key;                  // the shape of the last launch-by-launch pass
    std::vector<i64> nocap_key;                 // a shape whose capture failed (not retried)
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;           // records captures (launches go on `stream`)
    i64 graph_passes = 0, graph_aborts = 0;
    int graph_backoff = 0, graph_wait = 0;      // passes run launch by launch after an abort
    u32 graph_abort_why = 0;                    // abort word of the last switched-off replay
    i64 cap_leaf = 256;                         // per-group union leaves (stage 1)
    // stage-2 cache: capacity per group (words of 4 entries per lane), planned
    // each build from the need of the previous one (valid for gneed_groups)
    i64 gneed_groups = -1;
    u64 cache_words = 0;                        // words laid out by the last build
    int state = ST_NONE;
    int restarts = 0;
    int vals_sel = 0;       // which value buffer holds eps after the sort
    double lambda_cfl = 1.0;  // CFL multiplier of the plain step (App. G)
    int key_bits_built = 63;  // Morton width of the current tree
    int reruns_last = 0;      // corrector re-runs of the last plain step
    int xi_sel = 0;         // which mask buffer holds the final keep mask

    // device buffers (grown on demand, never shrunk)
    Buf keys[2], vals[2], hist, scan_tmp, bbox;          // hist: radix sort state
    Buf posh, velu, vhalf, hn, hcache, pid_s, thermo, omega, acc, vsig, status;
    Buf alpha_s;                                // viscosity alpha in key order (switch)
    Buf xi[2], xscan, id, mu_leaf, lvstate;     // lvstate: fused leaf pass (ticket + look-back)
    Buf lchild, rchild, endrange, lflag, rflag, child, parent, arrive, blo, bhi;
    Buf rec, nrec, rscan;                       // bottom-up box records
    Buf glo, ghi, uleaf, uslot, ucnt, ustot;    // stage 1, per group
    Buf nlist, ncnt, flags;                     // stage 2, per particle (ELL)
    Buf gcap, gbase, gneed, gredo;
    Buf gstate;                                 // captured passes: gate words, gates, re-runs              // stage 2, per group capacity / layout
    Buf bpart;                                  // corrector partial sums
    Buf work[3];                                // work counters (profiling)
    i64 parts_pending = 0;                      // corrector blocks not yet folded
    Buf inst_d, poff_d, goff_d, leaf_off_d, ioff_d, root_d, stat_d, dt_inst_d, dt_host_d;
    Buf pbox, plen, xoff, xlist;                // export only

    Buf redo_d, rhmax_d;                        // per-instance density redo flags, root h_max

    // pinned host staging for counters
    void* pinned = nullptr;                     // PINNED_BYTES read-back + UPLOAD_BYTES upload
    hipEvent_t up_done = nullptr;               // last upload from the pinned area

    std::vector<InstDev> inst_h;
    std::vector<i64> poff_h, goff_h;
    Prof prof;

    // pooled instances (batched passes and serving)
    Pool pool;
    std::map<int64_t, Inst> insts;
    int64_t next_handle = 1;
    std::recursive_mutex mu;                    // one API call at a time on this context
    void* server = nullptr;                     // serving loop (serve.cpp), if started

    // shsph_step_noalloc runs on a second context (`sc`) whose device buffers
    // are all carved, by a bump pointer reset at every call, from the
    // device's static scratch array (`arena`); it shares the pinned staging
    // area and upload event of its parent and keeps its per-instance
    // reductions (the CFL dt of its last step) on the host between calls.
    shsph_ctx* sc = nullptr;
    char* arena = nullptr;
    size_t arena_used = 0;
    InstStat stat_keep{};
    bool stat_kept = false;
};

namespace {

const size_t PINNED_BYTES = 1 << 20;      // read-back staging
// device flag words: 0..3 tree traversal / cache capacity (reset per cache
// build), FLAG_SORT = radix sort look-back overrun, FLAG_LEAVES (+1) = fused
// leaf pass unresolved tile (look-back overrun)
constexpr int FLAG_WORDS = 8, FLAG_SORT = 4, FLAG_LEAVES = 5;
// stage-2 capacity of a group without history: 32 words of 4 entries per lane
constexpr u32 CACHE_WORDS0 = 32;
const size_t UPLOAD_BYTES = 1 << 20;      // upload staging (instance tables), after it
const int MAX_BATCH = 2048;           // instances per batched pass (stats fit the staging)

int fail(shsph_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}



#define HIPTRY(ctx, expr)                                                                \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(ctx, e_ == hipErrorOutOfMemory ? SHSPH_ENOMEM : SHSPH_EHIP,       \
                        std::string(#expr ": ") + hipGetErrorString(e_));                \
    } while (0)

#define TRY(expr)                                                                        \
    do {                                                                                 \
        int r_ = (expr);                                                                 \
        if (r_ != SHSPH_OK) return r_;                                                   \
    } while (0)

// Working memory of shsph_step_noalloc: one static array per device, its
// address taken once per device at context creation.
constexpr size_t SCRATCH_BYTES = (size_t)128 << 20;
constexpr int64_t SCRATCH_MAX_N = (int64_t)1 << 17;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
std::mutex scratch_mu;
std::map<int, char*> scratch_addr;          // device -> its copy of `scratch`

// Address of `scratch` on `device` (the current device), or nullptr.
char* scratch_on(int device)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    auto it = scratch_addr.find(device);
    if (it != scratch_addr.end()) return it->second;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    scratch_addr[device] = (char*)ptr;
    return (char*)ptr;
}

// Make `b` hold at least `bytes`; grows by 25 % beyond the request.  On a
// context with an arena the bytes come from the arena (exactly, 256-byte
// aligned) and nothing is allocated; an arena that cannot hold them is a
// capacity error.
int ensure(shsph_ctx* c, Buf& b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    if (b.cap >= bytes) return SHSPH_OK;
    if (c->capturing) return fail(c, SHSPH_EHIP, "a buffer would grow while a pass is captured");
    ++c->alloc_gen;
    if (c->arena) {
        const size_t off = (c->arena_used + 255) & ~(size_t)255;
        const size_t want = (bytes + 255) & ~(size_t)255;
        if (off + want > SCRATCH_BYTES)
            return fail(c, SHSPH_ECAPACITY, "the static scratch array (" +
                        std::to_string(SCRATCH_BYTES >> 20) + " MiB) cannot hold this step's working memory");
        b.p = c->arena + off;
        b.cap = want;
        c->arena_used = off + want;
        return SHSPH_OK;
    }
    if (b.p) {
        HIPTRY(c, hipStreamSynchronize(c->stream));
        HIPTRY(c, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();                 // do not leave the failure to later launches
        return fail(c, SHSPH_ENOMEM, "device memory exhausted (" + std::to_string(want >> 20) + " MiB)");
    }
    b.cap = want;
    return SHSPH_OK;
}

// Grow `b` to at least `bytes` keeping its first `keep` bytes.
int ensure_keep(shsph_ctx* c, Buf& b, size_t bytes, size_t keep)
{
    if (b.cap >= bytes) return SHSPH_OK;
    Buf nb;
    TRY(ensure(c, nb, bytes));
    if (b.p && keep) {
        HIPTRY(c, hipMemcpyAsync(nb.p, b.p, std::min(keep, b.cap), hipMemcpyDeviceToDevice, c->stream));
    }
    if (b.p && !c->arena) {
        HIPTRY(c, hipStreamSynchronize(c->stream));
        HIPTRY(c, hipFree(b.p));
    }
    b = nb;
    return SHSPH_OK;
}

template <class T> T* P(Buf& b) { return (T*)b.p; }

// --- optional stage timing with HIP events on the context's stream -----------
void prof_begin(shsph_ctx* c, int stage)
{
    Prof& p = c->prof;
    if (!p.on) return;
    if (p.used == p.stage.size()) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return;
        p.stage.push_back(stage);
        p.ev.push_back(e0);
        p.ev.push_back(e1);
    }
    p.stage[p.used] = stage;
    hipEventRecord(p.ev[2 * p.used], c->stream);
}

void prof_end(shsph_ctx* c)
{
    Prof& p = c->prof;
    if (!p.on || p.used >= p.stage.size()) return;
    hipEventRecord(p.ev[2 * p.used + 1], c->stream);
    ++p.used;
}

void prof_collect(shsph_ctx* c)
{
    Prof& p = c->prof;
    if (!p.on || p.used == 0) return;
    hipEventSynchronize(p.ev[2 * p.used - 1]);
    for (size_t i = 0; i < p.used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.ev[2 * i], p.ev[2 * i + 1]) == hipSuccess) {
            p.ms[p.stage[i]] += ms;
            p.launches[p.stage[i]] += 1;
        }
    }
    p.used = 0;
}

int check_launch(shsph_ctx* c, const char* where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, SHSPH_EHIP, std::string(where) + ": " + hipGetErrorString(e));
    return SHSPH_OK;
}

// Copy `bytes` from device to the pinned staging area and wait.
int read_back(shsph_ctx* c, const void* dev, size_t bytes, size_t off = 0)
{
    HIPTRY(c, hipMemcpyAsync((char*)c->pinned + off, dev, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return SHSPH_OK;
}

bool finite_box(const shsph_particles* p)
{
    for (int d = 0; d < 3; ++d)
        if (!(std::isfinite(p->lo[d]) && std::isfinite(p->hi[d]) && p->hi[d] > p->lo[d])) return false;
    return true;
}

int validate(shsph_ctx* c, const shsph_particles* p, bool need_v, bool need_a)
{
    if (!p) return fail(c, SHSPH_EINVAL, "particles is NULL");
    if (p->n < 1 || p->n > (int64_t)0x7fffffff) return fail(c, SHSPH_EINVAL, "n must be in [1, 2^31)");
    if (p->dtype != SHSPH_F32 && p->dtype != SHSPH_F64) return fail(c, SHSPH_EINVAL, "bad dtype");
    if (!p->x || !p->y || !p->z || !p->h) return fail(c, SHSPH_EINVAL, "x, y, z, h are required");
    if (p->periodic && !finite_box(p)) return fail(c, SHSPH_EINVAL, "periodic box needs hi > lo");
    if (!(p->mass > 0) || !std::isfinite(p->mass)) return fail(c, SHSPH_EINVAL, "mass must be > 0");
    if (need_v && (!p->vx || !p->vy || !p->vz || !p->u))
        return fail(c, SHSPH_EINVAL, "vx, vy, vz, u are required");
    if (need_a && (!p->ax || !p->ay || !p->az || !p->dudt))
        return fail(c, SHSPH_EINVAL, "ax, ay, az, dudt are required");
    return SHSPH_OK;
}

SphParams sph_params(const shsph_params& q)
{
    SphParams s;
    s.hfact = q.hfact; s.gamma = q.gamma; s.alpha = q.alpha_av; s.beta = q.beta_av;
    s.beta_u = q.beta_u; s.chi = q.chi; s.lambda = q.lambda; s.eps_h = q.eps_h;
    s.c_cour = q.c_cour; s.c_force = q.c_force; s.max_iter = q.max_iter;
    s.kernel = q.kernel;
    s.r_kern = kernel_support(q.kernel);
    s.alpha_min = q.alpha_min; s.alpha_max = q.alpha_max; s.sigma_decay = q.sigma_decay;
    s.force_split = q.force_split;
    return s;
}

template <class T> FieldPtrs<T> fields(const shsph_particles* p)
{
    FieldPtrs<T> f;
    f.x = (const T*)p->x; f.y = (const T*)p->y; f.z = (const T*)p->z;
    f.vx = (const T*)p->vx; f.vy = (const T*)p->vy; f.vz = (const T*)p->vz;
    f.u = (const T*)p->u; f.h = (const T*)p->h;
    f.ax = (const T*)p->ax; f.ay = (const T*)p->ay; f.az = (const T*)p->az;
    f.du = (const T*)p->dudt;
    f.pid = p->pid;
    return f;
}

template <class T> SortedPtrs<T> sorted(shsph_ctx* c, bool with_step)
{
    SortedPtrs<T> s;
    s.posh = P<vec4<T>>(c->posh);
    s.velu = P<vec4<T>>(c->velu);
    s.vhalf = with_step ? P<vec4<T>>(c->vhalf) : nullptr;
    s.hn = P<T>(c->hn);
    s.hcache = P<T>(c->hcache);
    s.pid = P<u32>(c->pid_s);
    return s;
}

// Size the per-instance device tables for c->ninst and upload the instance
// table and the particle / group offsets.
int upload_instances(shsph_ctx* c)
{
    const int k = c->ninst;
    TRY(ensure(c, c->inst_d, k * sizeof(InstDev)));
    TRY(ensure(c, c->poff_d, (k + 1) * sizeof(i64)));
    TRY(ensure(c, c->goff_d, (k + 1) * sizeof(i64)));
    TRY(ensure(c, c->stat_d, k * sizeof(InstStat)));
    TRY(ensure(c, c->dt_inst_d, k * sizeof(double)));
    TRY(ensure(c, c->dt_host_d, k * sizeof(double)));
    TRY(ensure(c, c->leaf_off_d, (k + 1) * sizeof(i64)));
    TRY(ensure(c, c->ioff_d, (k + 1) * sizeof(i64)));
    TRY(ensure(c, c->root_d, k * sizeof(u32)));
    TRY(ensure(c, c->bbox, 6 * k * sizeof(u64)));
    TRY(ensure(c, c->redo_d, k));
    TRY(ensure(c, c->rhmax_d, k * sizeof(double)));
    // stage through the pinned upload area (the previous upload must have left it)
    if (c->up_done) HIPTRY(c, hipEventSynchronize(c->up_done));
    char* up = (char*)c->pinned + PINNED_BYTES;
    const size_t b0 = k * sizeof(InstDev), b1 = (k + 1) * sizeof(i64);
    memcpy(up, c->inst_h.data(), b0);
    memcpy(up + b0, c->poff_h.data(), b1);
    memcpy(up + b0 + b1, c->goff_h.data(), b1);
    HIPTRY(c, hipMemcpyAsync(c->inst_d.p, up, b0, hipMemcpyHostToDevice, c->stream));
    HIPTRY(c, hipMemcpyAsync(c->poff_d.p, up + b0, b1, hipMemcpyHostToDevice, c->stream));
    HIPTRY(c, hipMemcpyAsync(c->goff_d.p, up + b0 + b1, b1, hipMemcpyHostToDevice, c->stream));
    if (!c->up_done) HIPTRY(c, hipEventCreateWithFlags(&c->up_done, hipEventDisableTiming));
    HIPTRY(c, hipEventRecord(c->up_done, c->stream));
    return SHSPH_OK;
}

// Upload `bytes` from host memory to device through the pinned upload area,
// after the instance tables (same wait rule), `at` bytes further on (uploads
// enqueued without a wait between them use different `at`).
int upload_extra(shsph_ctx* c, void* dst, const void* src, size_t bytes, size_t at = 0)
{
    const int k = c->ninst;
    const size_t off = k * sizeof(InstDev) + 2 * (k + 1) * sizeof(i64) + at;
    if (off + bytes > UPLOAD_BYTES) return fail(c, SHSPH_EINVAL, "upload area too small");
    char* up = (char*)c->pinned + PINNED_BYTES + off;
    memcpy(up, src, bytes);
    HIPTRY(c, hipMemcpyAsync(dst, up, bytes, hipMemcpyHostToDevice, c->stream));
    HIPTRY(c, hipEventRecord(c->up_done, c->stream));
    return SHSPH_OK;
}

// Instance table for a single instance.
int set_single_instance(shsph_ctx* c, const shsph_particles* p)
{
    c->ninst = 1;
    c->inst_h.assign(1, InstDev());
    InstDev& in = c->inst_h[0];
    in.p_off = 0;
    in.p_cnt = p->n;
    in.shift = 0;
    for (int d = 0; d < 3; ++d) { in.lo[d] = p->lo[d]; in.hi[d] = p->hi[d]; }
    in.mass = p->mass;
    in.periodic = p->periodic ? 1 : 0;
    in.pad = 0;
    c->poff_h = { 0, p->n };
    c->n_groups = (p->n + GROUP - 1) / GROUP;
    c->goff_h = { 0, c->n_groups };
    return upload_instances(c);
}

GroupMap group_map(shsph_ctx* c)
{
    GroupMap g;
    g.goff = P<i64>(c->goff_d);
    g.p_off = P<i64>(c->poff_d);
    g.ninst = c->ninst;
    return g;
}

// Work counters: kernel kind 0 = particle cache, 1 = density, 2 = force;
// 64 slots x 2 u64 each, accumulated on the device while profiling is on.
u64* work_ptr(shsph_ctx* c, int kind)
{
    if (!c->prof.on || !c->work[kind].p) return nullptr;
    return P<u64>(c->work[kind]);
}

CacheView cache_view(shsph_ctx* c)
{
    CacheView v;
    v.work = nullptr;
    v.skip = nullptr;
    v.uleaf = P<u32>(c->uleaf); v.uslot = P<u32>(c->uslot);
    v.ucnt = P<u32>(c->ucnt); v.ustot = P<u32>(c->ustot);
    v.cap = c->cap_leaf;
    v.nlist = P<u64>(c->nlist); v.ncnt = P<u32>(c->ncnt);
    v.gbase = P<u64>(c->gbase);
    v.glo = c->glo.p; v.ghi = c->ghi.p; v.blo = c->blo.p;
    v.root = P<u32>(c->root_d);
    v.rk = kernel_support(c->prm.kernel) * c->prm.chi;
    return v;
}

// ---------------------------------------------------------------------------
// Tree build: keys -> sort -> gather -> mask/reduce/compact -> Karras ->
// boxes -> caches.  `dt_dev` non-NULL: positions are the leapfrog-predicted
// ones (stepping); the gather then also forms v*, u*, v^{n+1/2}, u^{n+1/2}.
// ---------------------------------------------------------------------------
template <class T>
int build_caches(shsph_ctx* c, const u8* redo = nullptr, const u32* skip = nullptr);
template <class T> int build_tree_tables(shsph_ctx* c, i64 nl);

template <class T> int build(shsph_ctx* c, const FieldPtrs<T>& f, i64 n, const double* dt_dev, bool step)
{
    hipStream_t st = c->stream;
    const int nred = c->prm.n_red < 0 ? 3 : c->prm.n_red;

    TRY(ensure(c, c->keys[0], n * sizeof(u64)));
    TRY(ensure(c, c->keys[1], n * sizeof(u64)));
    TRY(ensure(c, c->vals[0], n * sizeof(u32)));
    TRY(ensure(c, c->vals[1], n * sizeof(u32)));
    TRY(ensure(c, c->hist, radix_state_words(n, c->ninst) * sizeof(u32)));
    TRY(ensure(c, c->scan_tmp, scan_tmp_bytes(n + 1)));
    if (!c->flags.p) {
        TRY(ensure(c, c->flags, FLAG_WORDS * sizeof(u32)));
        launch_fill_u32(P<u32>(c->flags), FLAG_WORDS, 0u, st);
    }
    TRY(ensure(c, c->posh, n * sizeof(vec4<T>)));
    TRY(ensure(c, c->velu, n * sizeof(vec4<T>)));
    if (step) TRY(ensure(c, c->vhalf, n * sizeof(vec4<T>)));
    TRY(ensure(c, c->hn, n * sizeof(T)));
    TRY(ensure(c, c->hcache, n * sizeof(T)));
    TRY(ensure(c, c->pid_s, n * sizeof(u32)));
    TRY(ensure(c, c->xi[0], n));
    TRY(ensure(c, c->xi[1], n));
    TRY(ensure(c, c->xscan, (n + 1) * sizeof(u32)));
    TRY(ensure(c, c->id, (n + 1) * sizeof(u32)));
    TRY(ensure(c, c->mu_leaf, n * sizeof(u64)));

    InstDev* inst = P<InstDev>(c->inst_d);
    const i64* poff = P<i64>(c->poff_d);
    const int ninst = c->ninst;

    // leapfrog prediction (+ isolated box) -> Morton keys
    bool any_isolated = false;
    for (const InstDev& in : c->inst_h) any_isolated |= !in.periodic;
    if (any_isolated) launch_bbox<T>(f, n, inst, poff, ninst, dt_dev, P<u64>(c->bbox), st);
    prof_begin(c, S_MORTON);
    const int kbits = c->prm.key_bits == 30 ? 30 : 63;    // 30-bit or 63-bit Morton codes
    launch_predict_morton<T>(f, n, inst, poff, ninst, dt_dev, P<u64>(c->keys[0]), P<u32>(c->vals[0]),
                             kbits / 3, st);
    prof_end(c);
    TRY(check_launch(c, "morton"));
    // stable radix sort of (key, index), then gather into key order
    prof_begin(c, S_SORT);
    // (the nearly-sorted path reads a count on the host: not while capturing)
    const int sel = radix_sort_pairs(P<u64>(c->keys[0]), P<u32>(c->vals[0]), P<u64>(c->keys[1]),
                                     P<u32>(c->vals[1]), n, kbits, poff, ninst, P<u32>(c->hist),
                                     P<u32>(c->flags) + FLAG_SORT,
                                     c->capturing ? nullptr : (u32*)c->pinned, st);
    prof_end(c);
    if (sel == -2) return fail(c, SHSPH_EHIP, "radix sort: reading the out-of-place count failed");
    if (sel < 0) return fail(c, SHSPH_ECAPACITY, "more than 2^30 - 2 particles in one pass");
    c->vals_sel = sel;
    c->key_bits_built = kbits;
    const u64* mu = P<u64>(c->keys[sel]);
    const u32* eps = P<u32>(c->vals[sel]);
    TRY(check_launch(c, "sort"));
    SortedPtrs<T> s = sorted<T>(c, step);
    prof_begin(c, S_GATHER);
    launch_gather<T>(f, n, inst, poff, ninst, dt_dev, eps, s, st);
    prof_end(c);
    TRY(check_launch(c, "gather"));
    // keep mask, reduction passes, scan and compaction: one kernel that runs
    // the passes tile by tile in LDS; the separate passes (double-buffered
    // mask) only when some tile could not be resolved within its window
    prof_begin(c, S_LEAVES);
    TRY(ensure(c, c->lvstate, leaves_fused_state_words(n) * sizeof(u32)));
    launch_fill_u32(P<u32>(c->flags) + FLAG_LEAVES, 2, 0u, st);
    launch_leaves_fused(mu, n, poff, ninst, nred, P<u32>(c->lvstate), P<u8>(c->xi[0]),
                        P<u32>(c->xscan), P<u32>(c->id), P<u64>(c->mu_leaf),
                        P<u32>(c->flags) + FLAG_LEAVES, st);
    c->xi_sel = 0;
    prof_end(c);
    TRY(check_launch(c, "leaves"));
    // captured: the flags go to the pass's gate, the leaf count stays on the device
    if (c->capturing) return build_tree_tables<T>(c, n);
    HIPTRY(c, hipMemcpyAsync(c->pinned, P<u32>(c->xscan) + n, sizeof(u32), hipMemcpyDeviceToHost, st));
    HIPTRY(c, hipMemcpyAsync((char*)c->pinned + 8, P<u32>(c->flags) + FLAG_LEAVES, 2 * sizeof(u32),
                             hipMemcpyDeviceToHost, st));
    HIPTRY(c, hipStreamSynchronize(st));
    u32 lvf[2];
    memcpy(lvf, (char*)c->pinned + 8, sizeof(lvf));
    if (lvf[1]) return fail(c, SHSPH_EHIP, "leaf pass: a look-back wait ran past its bound");
    if (lvf[0]) {
        prof_begin(c, S_LEAVES);
        launch_mask_init(mu, n, poff, ninst, P<u8>(c->xi[0]), st);
        int xs = 0;
        for (int r = 0; r < nred; ++r) {
            launch_reduce_pass(mu, n, poff, ninst, P<u8>(c->xi[xs]), P<u8>(c->xi[xs ^ 1]), st);
            xs ^= 1;
        }
        c->xi_sel = xs;
        scan_u8_u32(P<u8>(c->xi[xs]), P<u32>(c->xscan), n, c->scan_tmp.p, st);
        launch_compact(mu, P<u8>(c->xi[xs]), P<u32>(c->xscan), n, P<u32>(c->id), P<u64>(c->mu_leaf), st);
        prof_end(c);
        TRY(check_launch(c, "compact"));
        TRY(read_back(c, P<u32>(c->xscan) + n, sizeof(u32)));
    }
    const i64 nl = *(u32*)c->pinned;
    c->n_leaf = nl;
    c->n_internal = nl - ninst;
    return build_tree_tables<T>(c, nl);
}

// Karras tables, parents, then the boxes and caches.  Leaf j is node
// lbase + j with lbase = n - ninst; nl bounds the launches (the leaf count,
// or n while capturing, when the kernels find the count on the device).
template <class T> int build_tree_tables(shsph_ctx* c, i64 nl)
{
    hipStream_t st = c->stream;
    const i64 n = c->n;
    const int ninst = c->ninst;
    const i64* poff = P<i64>(c->poff_d);
    const i64 lbase = n - ninst;
    c->lbase = lbase;
    const i64 ni = nl - ninst, nn = lbase + nl;
    TRY(ensure(c, c->lchild, std::max<i64>(ni, 1) * sizeof(u32)));
    TRY(ensure(c, c->rchild, std::max<i64>(ni, 1) * sizeof(u32)));
    TRY(ensure(c, c->endrange, std::max<i64>(ni, 1) * sizeof(u32)));
    TRY(ensure(c, c->lflag, std::max<i64>(ni, 1)));
    TRY(ensure(c, c->rflag, std::max<i64>(ni, 1)));
    TRY(ensure(c, c->child, 2 * std::max<i64>(ni, 1) * sizeof(u32)));
    TRY(ensure(c, c->parent, nn * sizeof(u32)));
    TRY(ensure(c, c->arrive, std::max<i64>(ni, 1) * sizeof(u32)));
    TRY(ensure(c, c->blo, nn * sizeof(vec4<T>)));
    TRY(ensure(c, c->bhi, nn * sizeof(vec4<T>)));
    prof_begin(c, S_KARRAS);
    launch_inst_leaves(poff, ninst, P<u32>(c->xscan), n, P<i64>(c->leaf_off_d), P<i64>(c->ioff_d),
                       P<u32>(c->root_d), P<u32>(c->parent), lbase, st);
    TreePtrs t;
    t.lchild = P<u32>(c->lchild); t.rchild = P<u32>(c->rchild); t.endrange = P<u32>(c->endrange);
    t.lflag = P<u8>(c->lflag); t.rflag = P<u8>(c->rflag);
    t.child = P<u32>(c->child); t.parent = P<u32>(c->parent);
    launch_karras(P<u64>(c->mu_leaf), P<i64>(c->leaf_off_d), P<i64>(c->ioff_d), ninst, lbase, ni,
                  t, st);
    prof_end(c);
    TRY(check_launch(c, "karras"));
    c->restarts = 0;
    return build_caches<T>(c);
}

// Boxes, stage-1 and stage-2 caches on the current tree, with h_cache = posh.w.
// Capacities (leaves per group, entries per particle) grow and the stage is
// redone when a build reports more than fits.
// `redo` (device, per instance, optional): only instances flagged 1 get new
// caches; the others keep the ones of the previous build (valid: their h
// stayed within chi h_cache).  A capacity regrow changes the layout, so the
// retry rebuilds every group.
// While capturing, `skip` (a device word) switches the box launches off.
// With `redo` the layout is kept: the instances concerned write into their
// groups' ranges (a group that outgrows its range gets a new one appended).
template <class T> int build_caches(shsph_ctx* c, const u8* redo, const u32* skip)
{
    hipStream_t st = c->stream;
    // launch bounds: the leaf and internal counts, or their largest values
    // while capturing (the kernels read the counts on the device)
    const i64 n = c->n, lb = c->lbase, G = c->n_groups;
    const i64 nl = c->capturing ? n : c->n_leaf, ni = c->capturing ? lb : c->n_internal;
    const InstDev* inst = P<InstDev>(c->inst_d);
    const int ninst = c->ninst;
    const vec4<T>* posh = P<vec4<T>>(c->posh);
    const GroupMap gm = group_map(c);
    const double rk = kernel_support(c->prm.kernel) * c->prm.chi;
    // bottom-up boxes and h_max
    const size_t nrc = boxes_rec_count(nl);
    const i64 nbb = (i64)(nrc / 128) + 1;
    TRY(ensure(c, c->rec, nrc * sizeof(u32)));
    TRY(ensure(c, c->nrec, (nbb + 1) * sizeof(u32)));
    TRY(ensure(c, c->rscan, (nbb + 1) * sizeof(u32)));
    TRY(ensure(c, c->glo, G * sizeof(vec4<T>)));
    TRY(ensure(c, c->ghi, G * sizeof(vec4<T>)));
    TRY(ensure(c, c->ucnt, G * sizeof(u32)));
    TRY(ensure(c, c->ustot, G * sizeof(u32)));
    TRY(ensure(c, c->ncnt, n * sizeof(u32)));
    prof_begin(c, S_BOXES);
    launch_fill_u32(P<u32>(c->arrive), std::max<i64>(ni, 1), 0u, st);
    launch_fill_u32(P<u32>(c->flags), 4, 0u, st);
    launch_boxes_up<T>(posh, P<u32>(c->id), nl, lb, P<u32>(c->child), P<u32>(c->parent),
                       P<u32>(c->endrange), P<i64>(c->ioff_d), P<i64>(c->leaf_off_d), ninst,
                       P<u32>(c->arrive), P<u32>(c->rec), P<u32>(c->nrec), P<u32>(c->rscan),
                       c->scan_tmp.p, P<vec4<T>>(c->blo), P<vec4<T>>(c->bhi), P<u32>(c->flags), st,
                       skip);
    launch_group_boxes<T>(posh, gm, G, P<vec4<T>>(c->glo), P<vec4<T>>(c->ghi), st, skip);
    prof_end(c);
    TRY(check_launch(c, "boxes"));
    TRY(ensure(c, c->gcap, G * sizeof(u32)));
    TRY(ensure(c, c->gbase, (G + 1) * sizeof(u64)));
    TRY(ensure(c, c->gneed, G * sizeof(u32)));
    TRY(ensure(c, c->gredo, G));
    const size_t WORD_BYTES = (size_t)GROUP * sizeof(u64);    // one word of every lane of a group
    bool run_stage1 = true;
    bool plan = redo == nullptr;     // a rebuild of some instances keeps the others' layout
    const u8* gredo = nullptr;       // regrow retry: only the groups that overflowed
    for (int attempt = 0;; ++attempt) {
        // stage 1: neighbour leaves of each group
        TRY(ensure(c, c->uleaf, (size_t)G * c->cap_leaf * sizeof(u32)));
        TRY(ensure(c, c->uslot, (size_t)G * c->cap_leaf * sizeof(u32)));
        if (run_stage1) {
        prof_begin(c, S_STAGE1);
        launch_group_leaves<T>(P<vec4<T>>(c->blo), P<vec4<T>>(c->bhi), P<u32>(c->child),
                               P<u32>(c->id), P<u32>(c->xscan), lb, P<vec4<T>>(c->glo), P<vec4<T>>(c->ghi), G, gm,
                               P<u32>(c->root_d), inst, rk, c->cap_leaf,
                               (u32)c->prm.spread_slots, c->prm.stage1_serial != 0,
                               P<u32>(c->uleaf),
                               P<u32>(c->uslot), P<u32>(c->ucnt), P<u32>(c->ustot),
                               P<u32>(c->flags), attempt ? nullptr : redo, st);
        prof_end(c);
        TRY(check_launch(c, "stage1"));
        }
        // stage-2 capacities: each group's need in the previous build (same
        // groups) or a default, never above its union; laid out by a scan
        if (plan) {
            const bool hist = c->gneed_groups == G;
            launch_cache_plan(P<u32>(c->ustot), hist ? P<u32>(c->gneed) : nullptr, G, CACHE_WORDS0,
                              P<u32>(c->gcap), P<u64>(c->gbase), c->scan_tmp.p, st, skip);
            if (!c->nlist.p)    // first build: room for the default capacity
                TRY(ensure(c, c->nlist, (size_t)G * CACHE_WORDS0 * WORD_BYTES));
            plan = false;
        }
        // stage 2: particle neighbours as union slots (a layout larger than
        // the buffer is flagged, nothing written)
        prof_begin(c, S_STAGE2);
        launch_group_cache<T>(posh, P<vec4<T>>(c->blo), P<vec4<T>>(c->bhi), P<u32>(c->id),
                              P<u32>(c->xscan), lb, gm, G,
                              inst, rk, rk, c->cap_leaf, P<u32>(c->uleaf), P<u32>(c->uslot),
                              P<u32>(c->ucnt), P<u32>(c->ustot), P<u64>(c->gbase), P<u32>(c->gcap),
                              (u64)(c->nlist.cap / WORD_BYTES), P<u32>(c->gneed), gredo,
                              P<u64>(c->nlist), P<u32>(c->ncnt), P<u32>(c->flags), P<vec4<T>>(c->glo),
                              P<vec4<T>>(c->ghi), P<u32>(c->root_d), work_ptr(c, 0),
                              c->prm.stage2_mode, attempt ? nullptr : redo, st);
        prof_end(c);
        TRY(check_launch(c, "stage2"));
        launch_root_hmax<T>(P<vec4<T>>(c->blo), P<u32>(c->root_d), ninst, P<double>(c->rhmax_d), st);
        if (c->capturing) {
            // groups that outgrew their capacity get a larger range at the end
            // of the layout and run stage 2 again, as below (device-side; a
            // layout past the buffer is flagged); the other flags and the
            // radii go to the pass's gate
            launch_cache_regrow(P<u32>(c->gneed), G, P<u32>(c->gcap), P<u64>(c->gbase),
                                P<u8>(c->gredo), st);
            launch_flag_and(P<u32>(c->flags), ~4u, st);
            launch_group_cache<T>(posh, P<vec4<T>>(c->blo), P<vec4<T>>(c->bhi), P<u32>(c->id),
                                  P<u32>(c->xscan), lb, gm, G, inst, rk, rk, c->cap_leaf,
                                  P<u32>(c->uleaf), P<u32>(c->uslot), P<u32>(c->ucnt),
                                  P<u32>(c->ustot), P<u64>(c->gbase), P<u32>(c->gcap),
                                  (u64)(c->nlist.cap / WORD_BYTES), P<u32>(c->gneed),
                                  P<u8>(c->gredo), P<u64>(c->nlist), P<u32>(c->ncnt),
                                  P<u32>(c->flags), P<vec4<T>>(c->glo), P<vec4<T>>(c->ghi),
                                  P<u32>(c->root_d), nullptr, c->prm.stage2_mode, nullptr, st);
            c->gneed_groups = G;
            return check_launch(c, "stage2 (regrow)");
        }
        HIPTRY(c, hipMemcpyAsync(c->pinned, c->flags.p, FLAG_WORDS * sizeof(u32),
                                 hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipMemcpyAsync((char*)c->pinned + FLAG_WORDS * sizeof(u32), c->rhmax_d.p,
                                 ninst * sizeof(double), hipMemcpyDeviceToHost, st));
        const size_t tot_at = FLAG_WORDS * sizeof(u32) + ninst * sizeof(double);
        HIPTRY(c, hipMemcpyAsync((char*)c->pinned + tot_at, P<u64>(c->gbase) + G, sizeof(u64),
                                 hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipStreamSynchronize(st));
        u32 fl[FLAG_WORDS];
        memcpy(fl, c->pinned, sizeof(fl));
        u64 words = 0;
        memcpy(&words, (char*)c->pinned + tot_at, sizeof(u64));
        if (fl[FLAG_SORT]) {
            launch_fill_u32(P<u32>(c->flags) + FLAG_SORT, 1, 0u, st);
            return fail(c, SHSPH_EHIP, "radix sort: a look-back wait ran past its bound");
        }
        if (fl[0] & 1u) return fail(c, SHSPH_ECAPACITY, "tree traversal stack overflow");
        if (fl[0] & 16u) return fail(c, SHSPH_ECAPACITY, "bottom-up box records overflow");
        // periodic minimum image needs the cache radius below half the box
        const double* rh = (const double*)((char*)c->pinned + FLAG_WORDS * sizeof(u32));
        for (int k = 0; k < ninst; ++k) {
            const InstDev& in = c->inst_h[k];
            if (!in.periodic) continue;
            for (int d = 0; d < 3; ++d)
                if (rk * rh[k] >= 0.5 * (in.hi[d] - in.lo[d]))
                    return fail(c, SHSPH_EINVAL, "periodic box smaller than twice the cache radius" +
                                (ninst > 1 ? " (batch instance " + std::to_string(k) + ")" : std::string()));
        }
        if (!(fl[0] & 38u)) {
            c->gneed_groups = G;
            c->cache_words = words;
            break;
        }
        if (attempt >= 6) return fail(c, SHSPH_ECAPACITY, "neighbour cache capacity");
        launch_fill_u32(P<u32>(c->flags), 4, 0u, st);
        gredo = nullptr;
        if (fl[0] & 2u) {
            // stage 1 overflowed: half again the largest request, then stage 1
            // and a fresh plan for every group
            c->cap_leaf = std::max<i64>(c->cap_leaf, (i64)fl[1] + fl[1] / 2 + 16);
            run_stage1 = true;
            plan = redo == nullptr;
            continue;
        }
        run_stage1 = false;
        if (fl[0] & 32u) {
            // the planned layout did not fit the buffer: grow it (nothing was
            // written) and run stage 2 again
            TRY(ensure(c, c->nlist, (size_t)(words + words / 4 + G) * WORD_BYTES));
            continue;
        }
        // some groups outgrew their capacity: they get a larger range at the
        // end of the layout and only they run stage 2 again (the others keep
        // what they wrote)
        launch_cache_regrow(P<u32>(c->gneed), G, P<u32>(c->gcap), P<u64>(c->gbase), P<u8>(c->gredo), st);
        TRY(read_back(c, P<u64>(c->gbase) + G, sizeof(u64)));
        memcpy(&words, c->pinned, sizeof(u64));
        TRY(ensure_keep(c, c->nlist, (size_t)(words + words / 8) * WORD_BYTES, c->nlist.cap));
        gredo = P<u8>(c->gredo);
    }
    return SHSPH_OK;
}

// Density / h iteration with cache rebuilds while some h leaves chi h_cache.
// `force` (optional): the first pass runs density and force in one
// persistent launch (k_density_force); *force_done tells whether that force
// stands (no particle left chi h_cache), else the caller runs the force.
template <class T> struct FusedForce {
    vec4<T>* acc;
    bool* done;
};

template <class T> int run_density(shsph_ctx* c, bool with_thermo, const FusedForce<T>* force = nullptr)
{
    hipStream_t st = c->stream;
    const i64 n = c->n;
    TRY(ensure(c, c->omega, n * sizeof(T)));
    TRY(ensure(c, c->thermo, n * sizeof(vec4<T>)));
    TRY(ensure(c, c->status, n));
    const SphParams sp = sph_params(c->prm);
    SortedPtrs<T> s = sorted<T>(c, false);
    if (!with_thermo) s.velu = nullptr;
    if (force) *force->done = false;
    // Instances whose h all settled keep their result; only those with a
    // particle past chi h_cache iterate again on the rebuilt caches, so an
    // instance gets the same h whatever else shares the pass.
    const int ninst = c->ninst;
    std::vector<u8> redo(ninst, 1);
    for (int attempt = 0;; ++attempt) {
        const u8* rd = attempt ? P<u8>(c->redo_d) : nullptr;
        CacheView cvd = cache_view(c);
        cvd.work = work_ptr(c, 1);
        bool fused = false;
        if (attempt == 0 && force && with_thermo) {
            launch_stat_reset(P<InstStat>(c->stat_d), ninst, 3, nullptr, st);
            CacheView cvf = cache_view(c);
            cvf.work = work_ptr(c, 2);
            prof_begin(c, S_DENSITY_FORCE);
            fused = launch_density_force<T>(s, P<vec4<T>>(c->thermo), P<u32>(c->id), group_map(c),
                                            c->n_groups, ninst, P<InstDev>(c->inst_d), sp, cvd, cvf,
                                            P<T>(c->omega), P<u8>(c->status), P<InstStat>(c->stat_d),
                                            force->acc, nullptr, st) == 0;
            prof_end(c);
            if (!fused) (void)hipGetLastError();
        }
        if (!fused) {
            launch_stat_reset(P<InstStat>(c->stat_d), ninst, 1, rd, st);
            prof_begin(c, S_DENSITY);
            launch_density<T>(s, P<u32>(c->id), group_map(c), c->n_groups, P<InstDev>(c->inst_d), sp,
                              cvd, P<T>(c->omega),
                              with_thermo ? P<vec4<T>>(c->thermo) : nullptr, P<u8>(c->status),
                              P<InstStat>(c->stat_d), rd, st);
            prof_end(c);
        }
        TRY(check_launch(c, "density"));
        TRY(read_back(c, c->stat_d.p, ninst * sizeof(InstStat)));
        const InstStat* hs = (const InstStat*)c->pinned;
        u32 ex = 0, nc = 0;
        for (int k = 0; k < ninst; ++k) {
            redo[k] = hs[k].n_exceed ? 1 : 0;
            ex += hs[k].n_exceed;
            nc += hs[k].n_noconv;
        }
        if (ex == 0) {
            if (fused) *force->done = true;
            if (nc) return fail(c, SHSPH_ENOCONV, "h iteration did not converge for " + std::to_string(nc) + " particles");
            return SHSPH_OK;
        }
        if (attempt >= c->prm.max_restarts)
            return fail(c, SHSPH_ENOCONV, "h kept exceeding the cache tolerance after rebuilds");
        // rebuild the caches with the current h as the cache h
        ++c->restarts;
        TRY(upload_extra(c, c->redo_d.p, redo.data(), ninst));
        launch_copy_h<T>(s.posh, s.hcache, n, st);
        TRY(build_caches<T>(c, ninst > 1 ? P<u8>(c->redo_d) : nullptr));
    }
}

template <class T> int do_build(shsph_ctx* c, const shsph_particles* p)
{
    TRY(set_single_instance(c, p));
    c->n = p->n;
    c->dtype = p->dtype;
    c->state = ST_NONE;
    launch_stat_reset(P<InstStat>(c->stat_d), 1, 3, nullptr, c->stream);
    TRY(build<T>(c, fields<T>(p), p->n, nullptr, false));
    prof_collect(c);
    c->state = ST_TREE;
    return SHSPH_OK;
}

template <class T> int do_density(shsph_ctx* c, shsph_particles* p)
{
    hipStream_t st = c->stream;
    const i64 n = c->n;
    const u32* eps = P<u32>(c->vals[c->vals_sel]);
    const bool with_u = p->u && p->vx && p->vy && p->vz;
    if (with_u)
        launch_gather_velu<T>(eps, n, (const T*)p->vx, (const T*)p->vy, (const T*)p->vz,
                              (const T*)p->u, P<vec4<T>>(c->velu), st);
    // the velocity part is only used by force; zeros are fine when absent
    int rc = run_density<T>(c, with_u);
    if (rc != SHSPH_OK && rc != SHSPH_ENOCONV) return rc;
    launch_scatter<T>(eps, n, P<vec4<T>>(c->posh), 3, nullptr, (T*)p->h, st);
    launch_scatter<T>(eps, n, nullptr, 0, P<T>(c->omega), (T*)p->omega, st);
    launch_scatter_rho<T>(eps, n, P<vec4<T>>(c->posh), P<i64>(c->poff_d), c->ninst,
                          P<InstDev>(c->inst_d), c->prm.hfact, (T*)p->rho, st);
    TRY(check_launch(c, "density scatter"));
    HIPTRY(c, hipStreamSynchronize(st));
    prof_collect(c);
    c->state = ST_DENSITY;
    return rc;
}

template <class T> int do_force(shsph_ctx* c, shsph_particles* p)
{
    hipStream_t st = c->stream;
    const i64 n = c->n;
    const u32* eps = P<u32>(c->vals[c->vals_sel]);
    TRY(ensure(c, c->acc, n * sizeof(vec4<T>)));
    TRY(ensure(c, c->vsig, n * sizeof(T)));
    launch_gather_velu<T>(eps, n, (const T*)p->vx, (const T*)p->vy, (const T*)p->vz, (const T*)p->u,
                          P<vec4<T>>(c->velu), st);
    const T* al = nullptr;
    if (p->alpha) {           // per-particle viscosity alpha, gathered into key order
        TRY(ensure(c, c->alpha_s, n * sizeof(T)));
        launch_gather1<T>(eps, n, (const T*)p->alpha, P<T>(c->alpha_s), st);
        al = P<T>(c->alpha_s);
    }
    launch_thermo<T>(P<vec4<T>>(c->posh), P<vec4<T>>(c->velu), P<T>(c->omega), n, P<i64>(c->poff_d),
                     c->ninst, P<InstDev>(c->inst_d), c->prm.hfact, c->prm.gamma, c->prm.alpha_av,
                     al, P<vec4<T>>(c->thermo), st);
    launch_stat_reset(P<InstStat>(c->stat_d), c->ninst, 2, nullptr, st);
    c->parts_pending = 0;
    const SphParams sp = sph_params(c->prm);
    prof_begin(c, S_FORCE);
    launch_force<T>(sorted<T>(c, false), P<vec4<T>>(c->thermo), P<u32>(c->id), group_map(c),
                    c->n_groups, P<InstDev>(c->inst_d), sp, cache_view(c), P<vec4<T>>(c->acc),
                    P<T>(c->vsig), P<InstStat>(c->stat_d), st);
    prof_end(c);
    TRY(check_launch(c, "force"));
    const vec4<T>* acc = P<vec4<T>>(c->acc);
    launch_scatter<T>(eps, n, acc, 0, nullptr, (T*)p->ax, st);
    launch_scatter<T>(eps, n, acc, 1, nullptr, (T*)p->ay, st);
    launch_scatter<T>(eps, n, acc, 2, nullptr, (T*)p->az, st);
    launch_scatter<T>(eps, n, acc, 3, nullptr, (T*)p->dudt, st);
    TRY(check_launch(c, "force scatter"));
    HIPTRY(c, hipStreamSynchronize(st));
    prof_collect(c);
    c->state = ST_FORCE;
    return SHSPH_OK;
}

// Corrector re-runs (App. G.1): an instance whose max |dv| exceeds eps_v
// times its rms velocity gets v* <- v^{n+1}, u* <- u^{n+1} and the force and
// corrector again, at most max_reruns times.  The derivative kernels run
// over the whole pass; instances that passed keep v*, so they recompute
// exactly what they had.  Leaves the folded reductions in stat_d and the
// re-run count of each instance in `reruns`.
template <class T>
int corrector_reruns(shsph_ctx* c, const OutPtrs<T>& o, const double* dt_dev, std::vector<int>& reruns,
                     const T* alpha_s = nullptr)
{
    hipStream_t st = c->stream;
    const int ninst = c->ninst;
    const i64 n = c->n, nb = (n + GROUP - 1) / GROUP;
    reruns.assign(ninst, 0);
    if (!(c->prm.eps_v > 0)) return SHSPH_OK;
    std::vector<u8> redo(ninst, 0);
    for (;;) {
        if (c->parts_pending > 0) {
            launch_fold_parts(P<BlockPart>(c->bpart), c->parts_pending, ninst,
                              P<InstStat>(c->stat_d), st);
            c->parts_pending = 0;
        }
        TRY(read_back(c, c->stat_d.p, ninst * sizeof(InstStat)));
        const InstStat* hs = (const InstStat*)c->pinned;
        bool any = false;
        for (int k = 0; k < ninst; ++k) {
            float dv;
            memcpy(&dv, &hs[k].dvmax_bits, 4);
            double v2 = 0;
            for (int i = 0; i < STAT_SLOTS; ++i) v2 += hs[k].v2_part[i];
            const double cnt = (double)std::max<i64>(c->poff_h[k + 1] - c->poff_h[k], 1);
            const bool fail_k = (double)dv > c->prm.eps_v * std::sqrt(v2 / cnt);
            redo[k] = (fail_k && reruns[k] < c->prm.max_reruns) ? 1 : 0;
            if (redo[k]) { ++reruns[k]; any = true; }
        }
        if (!any) return SHSPH_OK;
        TRY(upload_extra(c, c->redo_d.p, redo.data(), ninst));
        launch_velu_from_out<T>(o, n, P<i64>(c->poff_d), ninst, P<InstDev>(c->inst_d),
                                P<u8>(c->redo_d), P<vec4<T>>(c->velu), st);
        launch_thermo<T>(P<vec4<T>>(c->posh), P<vec4<T>>(c->velu), P<T>(c->omega), n,
                         P<i64>(c->poff_d), ninst, P<InstDev>(c->inst_d), c->prm.hfact,
                         c->prm.gamma, c->prm.alpha_av, alpha_s, P<vec4<T>>(c->thermo), st);
        launch_stat_reset(P<InstStat>(c->stat_d), ninst, 2, nullptr, st);
        const SphParams sp = sph_params(c->prm);
        prof_begin(c, S_FORCE);
        launch_force<T>(sorted<T>(c, true), P<vec4<T>>(c->thermo), P<u32>(c->id), group_map(c),
                        c->n_groups, P<InstDev>(c->inst_d), sp, cache_view(c), P<vec4<T>>(c->acc),
                        nullptr, P<InstStat>(c->stat_d), st);
        prof_end(c);
        TRY(check_launch(c, "force (corrector re-run)"));
        prof_begin(c, S_CORRECT);
        launch_correct<T>(sorted<T>(c, true), P<vec4<T>>(c->acc), P<T>(c->omega), n,
                          P<i64>(c->poff_d), ninst, P<InstDev>(c->inst_d), dt_dev, c->prm.hfact,
                          o, P<InstStat>(c->stat_d), P<BlockPart>(c->bpart), st);
        c->parts_pending = nb;
        prof_end(c);
        TRY(check_launch(c, "correct (re-run)"));
    }
}

// CFL multiplier (App. G): halved after a step that re-ran its corrector,
// else relaxed towards 1 as (1 + s lambda) / (1 + s).
double next_multiplier(const shsph_params& q, double lam, int reruns)
{
    if (!(q.eps_v > 0)) return 1.0;
    return reruns ? 0.5 * lam : (1.0 + q.lambda_stiff * lam) / (1.0 + q.lambda_stiff);
}

template <class T> int do_step(shsph_ctx* c, shsph_particles* p, double dt, double* dt_used)
{
    hipStream_t st = c->stream;
    // dt for this step: caller's value, else the CFL dt of the last force pass
    if (!(dt > 0) && c->state != ST_FORCE)
        return fail(c, SHSPH_ESTATE, "dt <= 0 needs a preceding force evaluation (CFL dt)");
    const bool keep_stat = (c->arena ? c->stat_kept : c->stat_d.p != nullptr) && c->ninst == 1;
    TRY(set_single_instance(c, p));
    if (!keep_stat && !(dt > 0)) return fail(c, SHSPH_ESTATE, "no CFL dt available");
    if (c->arena && keep_stat)   // the reductions of this context's last step
        TRY(upload_extra(c, c->stat_d.p, &c->stat_keep, sizeof(InstStat), 256));
    // a CFL step takes the CFL multiplier (encoded as -lambda)
    const double dt_req = dt > 0 ? dt : -c->lambda_cfl;
    TRY(upload_extra(c, c->dt_host_d.p, &dt_req, sizeof(double)));
    launch_dt_select(P<double>(c->dt_inst_d), P<InstStat>(c->stat_d), P<double>(c->dt_host_d), 1, st);
    c->n = p->n;
    c->dtype = p->dtype;
    c->state = ST_NONE;
    const double* dt_dev = P<double>(c->dt_inst_d);
    TRY(build<T>(c, fields<T>(p), p->n, dt_dev, true));
    c->state = ST_TREE;
    const i64 n = c->n;
    TRY(ensure(c, c->acc, n * sizeof(vec4<T>)));
    const bool sw = c->prm.alpha_switch && p->alpha;
    if (sw) {   // alpha^n and a^n into key order for the shock detector
        const u32* eps = P<u32>(c->vals[c->vals_sel]);
        TRY(ensure(c, c->alpha_s, n * sizeof(T)));
        launch_gather1<T>(eps, n, (const T*)p->alpha, P<T>(c->alpha_s), st);
        launch_gather_velu<T>(eps, n, (const T*)p->ax, (const T*)p->ay, (const T*)p->az,
                              (const T*)p->dudt, P<vec4<T>>(c->acc), st);
    }
    // with the alpha switch the force needs alpha^{n+1} first: no fusion
    bool fdone = false;
    const FusedForce<T> ff{P<vec4<T>>(c->acc), &fdone};
    int rc = run_density<T>(c, true, (c->prm.fused_density_force && !sw) ? &ff : nullptr);
    if (rc != SHSPH_OK) return rc;
    if (sw) {   // alpha^{n+1} from v*, grad v*, grad a^n; alpha c staged for the force
        launch_alpha<T>(sorted<T>(c, true), P<vec4<T>>(c->acc), P<T>(c->omega), P<u32>(c->id),
                        group_map(c), c->n_groups, P<InstDev>(c->inst_d), sph_params(c->prm),
                        cache_view(c), dt_dev, P<T>(c->alpha_s), P<vec4<T>>(c->thermo), st);
        TRY(check_launch(c, "alpha switch"));
    }
    c->parts_pending = 0;
    const SphParams sp = sph_params(c->prm);
    if (!fdone) {
        launch_stat_reset(P<InstStat>(c->stat_d), c->ninst, 2, nullptr, st);
        prof_begin(c, S_FORCE);
        CacheView cvf = cache_view(c);
        cvf.work = work_ptr(c, 2);
        launch_force<T>(sorted<T>(c, true), P<vec4<T>>(c->thermo), P<u32>(c->id), group_map(c),
                        c->n_groups, P<InstDev>(c->inst_d), sp, cvf, P<vec4<T>>(c->acc),
                        nullptr, P<InstStat>(c->stat_d), st);
        prof_end(c);
        TRY(check_launch(c, "force"));
    }
    OutPtrs<T> o;
    o.x = (T*)p->x; o.y = (T*)p->y; o.z = (T*)p->z;
    o.vx = (T*)p->vx; o.vy = (T*)p->vy; o.vz = (T*)p->vz;
    o.u = (T*)p->u; o.h = (T*)p->h;
    o.ax = (T*)p->ax; o.ay = (T*)p->ay; o.az = (T*)p->az; o.du = (T*)p->dudt;
    o.rho = (T*)p->rho; o.omega = (T*)p->omega; o.pid = p->pid;
    TRY(ensure(c, c->bpart, ((n + GROUP - 1) / GROUP) * sizeof(BlockPart)));
    prof_begin(c, S_CORRECT);
    launch_correct<T>(sorted<T>(c, true), P<vec4<T>>(c->acc), P<T>(c->omega), n, P<i64>(c->poff_d),
                      c->ninst, P<InstDev>(c->inst_d), dt_dev, c->prm.hfact, o,
                      P<InstStat>(c->stat_d), P<BlockPart>(c->bpart), st);
    c->parts_pending = (n + GROUP - 1) / GROUP;
    prof_end(c);
    TRY(check_launch(c, "correct"));
    std::vector<int> rr;
    TRY(corrector_reruns<T>(c, o, dt_dev, rr, sw ? P<T>(c->alpha_s) : nullptr));
    c->reruns_last = rr.empty() ? 0 : rr[0];
    if (sw)   // alpha^{n+1} back to the caller, in the new key order like every field
        HIPTRY(c, hipMemcpyAsync(p->alpha, c->alpha_s.p, n * sizeof(T), hipMemcpyDeviceToDevice, st));
    c->lambda_cfl = next_multiplier(c->prm, c->lambda_cfl, c->reruns_last);
    if (dt_used) {
        TRY(read_back(c, dt_dev, sizeof(double)));
        *dt_used = *(double*)c->pinned;
    }
    prof_collect(c);
    c->state = ST_FORCE;
    return SHSPH_OK;
}

// Sum of a device u32 array (through the exclusive scan; waits).
int sum_u32(shsph_ctx* c, const u32* p, i64 count, u64* out)
{
    *out = 0;
    if (count <= 0) return SHSPH_OK;
    TRY(ensure(c, c->xoff, (count + 1) * sizeof(u64)));
    TRY(ensure(c, c->scan_tmp, scan_tmp_bytes(count + 1)));
    scan_u32_u64(p, P<u64>(c->xoff), count, c->scan_tmp.p, c->stream);
    TRY(read_back(c, P<u64>(c->xoff) + count, 8));
    *out = *(u64*)c->pinned;
    return SHSPH_OK;
}

// ---------------------------------------------------------------------------
// Instance pool: one array per field for all pooled instances; an instance
// is a contiguous range [off, off + n).  Ranges are handed out first-fit and
// merged on release; the arrays grow (copy + free) when no range fits.
// ---------------------------------------------------------------------------
size_t pool_elem(int f, int dtype) { return f == PF_PID ? 4 : (dtype == SHSPH_F32 ? 4 : 8); }

void pool_release(shsph_ctx* c)
{
    Pool& q = c->pool;
    for (int f = 0; f < PF_NUM; ++f)
        if (q.fld[f]) { (void)hipFree(q.fld[f]); q.fld[f] = nullptr; }
    q.cap = 0;
    q.used = 0;
    q.free_.clear();
}

void pool_put(Pool& q, i64 off, i64 len)
{
    auto it = q.free_.emplace(off, len).first;
    if (it != q.free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) { pv->second += it->second; q.free_.erase(it); it = pv; }
    }
    auto nx = std::next(it);
    if (nx != q.free_.end() && it->first + it->second == nx->first) { it->second += nx->second; q.free_.erase(nx); }
}

int pool_grow(shsph_ctx* c, i64 need)
{
    Pool& q = c->pool;
    const i64 ncap = std::max<i64>(q.cap + std::max<i64>(need, q.cap / 2), (i64)1 << 16);
    HIPTRY(c, hipStreamSynchronize(c->stream));
    void* nf[PF_NUM] = {};
    for (int f = 0; f < PF_NUM; ++f) {
        if (hipMalloc(&nf[f], ncap * pool_elem(f, q.dtype)) != hipSuccess) {
            for (int g = 0; g < PF_NUM; ++g) if (nf[g]) hipFree(nf[g]);
            (void)hipGetLastError();
            return fail(c, SHSPH_ENOMEM, "instance pool: device memory exhausted");
        }
    }
    for (int f = 0; f < PF_NUM; ++f) {
        if (q.cap)
            HIPTRY(c, hipMemcpyAsync(nf[f], q.fld[f], q.cap * pool_elem(f, q.dtype),
                                     hipMemcpyDeviceToDevice, c->stream));
    }
    HIPTRY(c, hipStreamSynchronize(c->stream));
    for (int f = 0; f < PF_NUM; ++f) {
        if (q.fld[f]) hipFree(q.fld[f]);
        q.fld[f] = nf[f];
    }
    pool_put(q, q.cap, ncap - q.cap);
    q.cap = ncap;
    ++c->alloc_gen;
    return SHSPH_OK;
}

int pool_alloc(shsph_ctx* c, i64 n, i64* off)
{
    Pool& q = c->pool;
    for (int pass = 0; pass < 2; ++pass) {
        for (auto it = q.free_.begin(); it != q.free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const i64 rest = it->second - n, roff = it->first + n;
            q.free_.erase(it);
            if (rest) q.free_.emplace(roff, rest);
            q.used += n;
            return SHSPH_OK;
        }
        if (pass == 0) TRY(pool_grow(c, n));
    }
    return fail(c, SHSPH_ENOMEM, "instance pool: no range fits");
}

template <class T> FieldPtrs<T> pool_fields(shsph_ctx* c)
{
    void* const* f = c->pool.fld;
    FieldPtrs<T> r;
    r.x = (const T*)f[PF_X]; r.y = (const T*)f[PF_Y]; r.z = (const T*)f[PF_Z];
    r.vx = (const T*)f[PF_VX]; r.vy = (const T*)f[PF_VY]; r.vz = (const T*)f[PF_VZ];
    r.u = (const T*)f[PF_U]; r.h = (const T*)f[PF_H];
    r.ax = (const T*)f[PF_AX]; r.ay = (const T*)f[PF_AY]; r.az = (const T*)f[PF_AZ];
    r.du = (const T*)f[PF_DU];
    r.pid = (const u32*)f[PF_PID];
    return r;
}

template <class T> OutPtrs<T> pool_out(shsph_ctx* c)
{
    void* const* f = c->pool.fld;
    OutPtrs<T> o;
    o.x = (T*)f[PF_X]; o.y = (T*)f[PF_Y]; o.z = (T*)f[PF_Z];
    o.vx = (T*)f[PF_VX]; o.vy = (T*)f[PF_VY]; o.vz = (T*)f[PF_VZ];
    o.u = (T*)f[PF_U]; o.h = (T*)f[PF_H];
    o.ax = (T*)f[PF_AX]; o.ay = (T*)f[PF_AY]; o.az = (T*)f[PF_AZ]; o.du = (T*)f[PF_DU];
    o.rho = (T*)f[PF_RHO]; o.omega = (T*)f[PF_OMEGA]; o.pid = (u32*)f[PF_PID];
    return o;
}

// One pass of the whole step over pooled instances b with per-instance dt
// (dt = 0: derivatives at the current state, the state itself unchanged).
// Every stage is one launch over all of them.  Instances whose h iteration
// does not settle are reported through their stats (SHSPH_ENOCONV); the
// others are complete.
// ---------------------------------------------------------------------------
// Captured batched passes.  A pass whose shape repeats the previous pass's
// (same particle and group counts, instance boundary types, parameters,
// buffers and stream) is recorded once as a hipGraph and then replayed: the
// launch sequence is the launch-by-launch pass's, with every decision the
// host takes between launches moved to the device (no read-back until the
// end).  Leaf and internal counts stay on the device (leaf j at node lbase +
// j, launches sized for n leaves, the kernels bounded by the count); the
// nearly-sorted path of the sort is not used; capacity, sort, leaf-pass and
// box conditions and an h past chi h_cache set an abort word that switches
// every later launch off, after which the host runs the pass again launch by
// launch (the caller's arrays are written only by the corrector, which the
// abort switches off); the corrector re-runs are max_reruns rounds, each
// switched on by the previous round's check on the device.  Results are the
// launch-by-launch pass's, bit for bit.
// ---------------------------------------------------------------------------
// gate words: [0] abort, [1 + r] corrector re-run round r off (r < GS_ROUNDS),
// [GS_RB0 + b] cache-rebuild round b off (b < GS_RBMAX)
constexpr int GS_WORDS = 64, GS_ROUNDS = 40, GS_RB0 = 48, GS_RBMAX = 2;

bool graph_usable(shsph_ctx* c)
{
    return c->prm.graph_batch && !c->prof.on && !c->arena && c->prm.max_reruns <= GS_ROUNDS;
}

std::vector<i64> pass_key(shsph_ctx* c)
{
    std::vector<i64> k = {c->n, c->n_groups, c->ninst, c->dtype, (i64)c->alloc_gen,
                          (i64)c->param_gen, c->cap_leaf, c->gneed_groups == c->n_groups ? 1 : 0,
                          (i64)(intptr_t)c->stream};
    for (const InstDev& in : c->inst_h) k.push_back(in.periodic);
    return k;
}

void graph_drop(shsph_ctx* c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->gkey.clear();
    c->graph_backoff = c->graph_wait = 0;
}

// Buffers a captured pass uses at their largest (node tables for n leaves)
// or with headroom (the neighbour cache), allocated before the capture.
template <class T> int presize_capture(shsph_ctx* c)
{
    const i64 n = c->n, ninst = c->ninst, lb = n - ninst, G = c->n_groups;
    const i64 ni = std::max<i64>(lb, 1), nn = lb + n;
    TRY(ensure(c, c->lchild, ni * sizeof(u32)));
    TRY(ensure(c, c->rchild, ni * sizeof(u32)));
    TRY(ensure(c, c->endrange, ni * sizeof(u32)));
    TRY(ensure(c, c->lflag, ni));
    TRY(ensure(c, c->rflag, ni));
    TRY(ensure(c, c->child, 2 * ni * sizeof(u32)));
    TRY(ensure(c, c->arrive, ni * sizeof(u32)));
    TRY(ensure(c, c->parent, nn * sizeof(u32)));
    TRY(ensure(c, c->blo, nn * sizeof(vec4<T>)));
    TRY(ensure(c, c->bhi, nn * sizeof(vec4<T>)));
    const size_t nrc = boxes_rec_count(n);
    const i64 nbb = (i64)(nrc / 128) + 1;
    TRY(ensure(c, c->rec, nrc * sizeof(u32)));
    TRY(ensure(c, c->nrec, (nbb + 1) * sizeof(u32)));
    TRY(ensure(c, c->rscan, (nbb + 1) * sizeof(u32)));
    const size_t WORD_BYTES = (size_t)GROUP * sizeof(u64);
    TRY(ensure(c, c->nlist, (size_t)(c->cache_words + c->cache_words / 4 + 2 * G) * WORD_BYTES));
    TRY(ensure(c, c->acc, n * sizeof(vec4<T>)));
    TRY(ensure(c, c->bpart, ((n + GROUP - 1) / GROUP) * sizeof(BlockPart)));
    TRY(ensure(c, c->gstate, GS_WORDS * sizeof(u32) + ninst * (sizeof(u32) + 3)));
    return SHSPH_OK;
}

// The launches of one captured pass (see above).
template <class T> int graph_body(shsph_ctx* c)
{
    hipStream_t st = c->stream;
    const int ninst = c->ninst;
    const i64 n = c->n;
    const double* dt_dev = P<double>(c->dt_inst_d);
    u32* gs = P<u32>(c->gstate);
    u32* reruns = gs + GS_WORDS;
    u8* gate = (u8*)(reruns + ninst);
    u8* redo = gate + ninst;
    u8* rx = redo + ninst;                      // instances of a cache-rebuild round
    InstStat* stat = P<InstStat>(c->stat_d);
    const InstDev* inst = P<InstDev>(c->inst_d);
    const i64* poff = P<i64>(c->poff_d);
    launch_stat_reset(stat, ninst, 3, nullptr, st);
    TRY(build<T>(c, pool_fields<T>(c), n, dt_dev, true));
    const double rk = kernel_support(c->prm.kernel) * c->prm.chi;
    launch_gate_build(P<u32>(c->flags), 0x37u, FLAG_SORT, FLAG_LEAVES, P<double>(c->rhmax_d), inst,
                      ninst, rk, gs, gate, reruns, st);
    // density: the first attempt of the launch-by-launch pass
    const SphParams sp = sph_params(c->prm);
    SphParams sp1 = sp;       // the first force: the fused launch's (one thread per particle)
    if (c->prm.fused_density_force) sp1.force_split = 1;
    SortedPtrs<T> s = sorted<T>(c, false);
    launch_stat_reset(stat, ninst, 1, nullptr, st);
    launch_density<T>(s, P<u32>(c->id), group_map(c), c->n_groups, inst, sp, cache_view(c),
                      P<T>(c->omega), P<vec4<T>>(c->thermo), P<u8>(c->status), stat, gate, st);
    TRY(check_launch(c, "density"));
    // cache-rebuild rounds (the launch-by-launch pass's restarts), each
    // switched on by a particle past chi h_cache; past the last, the pass
    // switches itself off
    const int RB = std::min(c->prm.max_restarts, GS_RBMAX);
    for (int b = 0; b < RB; ++b) {
        u32* skw = gs + GS_RB0 + b;
        launch_gate_exceed(stat, ninst, gs, skw, rx, st);
        launch_copy_h<T>(s.posh, s.hcache, n, st, skw);
        // the layout is kept (no new plan inside the pass): a plan's scan
        // would recompute every group's offset, also in a round that is
        // switched off, and so move groups that an earlier regrow placed at
        // the end of the layout away from what stage 2 wrote
        TRY(build_caches<T>(c, rx, skw));
        launch_gate_round(P<u32>(c->flags), 0x37u, P<double>(c->rhmax_d), inst, ninst, rk, skw, gs,
                          rx, st);
        launch_stat_reset(stat, ninst, 1, rx, st);
        launch_density<T>(s, P<u32>(c->id), group_map(c), c->n_groups, inst, sp, cache_view(c),
                          P<T>(c->omega), P<vec4<T>>(c->thermo), P<u8>(c->status), stat, rx, st);
        TRY(check_launch(c, "density (rebuild round)"));
    }
    launch_gate_density(stat, ninst, gs, gate, st);
    // force and corrector
    const SortedPtrs<T> s1 = sorted<T>(c, true);
    const OutPtrs<T> o = pool_out<T>(c);
    const i64 nb = (n + GROUP - 1) / GROUP;
    auto force_correct = [&](const u32* skip, const SphParams& spf) {
        launch_stat_reset(stat, ninst, 2, nullptr, st, skip);
        CacheView cvf = cache_view(c);
        cvf.skip = skip;
        launch_force<T>(s1, P<vec4<T>>(c->thermo), P<u32>(c->id), group_map(c), c->n_groups, inst,
                        spf, cvf, P<vec4<T>>(c->acc), nullptr, stat, st);
        launch_correct<T>(s1, P<vec4<T>>(c->acc), P<T>(c->omega), n, poff, ninst, inst, dt_dev,
                          c->prm.hfact, o, stat, P<BlockPart>(c->bpart), st, skip);
    };
    force_correct(gs, sp1);
    TRY(check_launch(c, "force"));
    const int R = c->prm.eps_v > 0 ? c->prm.max_reruns : 0;
    for (int r = 0; r < R; ++r) {
        launch_fold_parts(P<BlockPart>(c->bpart), nb, ninst, stat, st, gs + r);
        launch_rerun_decide(stat, poff, ninst, c->prm.eps_v, c->prm.max_reruns, r, gs, redo, reruns,
                            st);
        launch_velu_from_out<T>(o, n, poff, ninst, inst, redo, P<vec4<T>>(c->velu), st);
        launch_thermo<T>(P<vec4<T>>(c->posh), P<vec4<T>>(c->velu), P<T>(c->omega), n, poff, ninst,
                         inst, c->prm.hfact, c->prm.gamma, c->prm.alpha_av, nullptr,
                         P<vec4<T>>(c->thermo), st, gs + 1 + r);
        force_correct(gs + 1 + r, sp);
        TRY(check_launch(c, "corrector re-run"));
    }
    launch_fold_parts(P<BlockPart>(c->bpart), nb, ninst, stat, st, gs + R);
    return check_launch(c, "fold");
}

// Runs the pass from a captured graph when its shape allows (capturing it
// first when the previous pass had this shape).  *done = false: the caller
// runs the pass launch by launch (no graph, or the graph's pass aborted).
// On success the instance stats are in the pinned staging, the re-run
// counts in rr, and *rc is SHSPH_OK or SHSPH_ENOCONV.
template <class T> int graph_pass(shsph_ctx* c, std::vector<int>& rr, int* rc, bool* done)
{
    *done = false;
    if (!graph_usable(c)) return SHSPH_OK;
    hipStream_t st = c->stream;
    const int ninst = c->ninst;
    std::vector<i64> key = pass_key(c);
    // after a replay that switched itself off, the next passes of the shape
    // (1, 2, 4 .. 16 of them, doubling while replays keep aborting) run
    // launch by launch: a batch that rebuilds its caches in most passes
    // would otherwise pay for both
    if (c->gexec && key == c->gkey && c->graph_wait > 0) {
        --c->graph_wait;
        return SHSPH_OK;
    }
    if (!(c->gexec && key == c->gkey)) {
        if (key != c->last_key || key == c->nocap_key) return SHSPH_OK;
        graph_drop(c);
        TRY(presize_capture<T>(c));
        key = pass_key(c);
        // recorded on a stream of our own (the caller's may be the null
        // stream, which cannot be captured); nothing runs while recording
        if (!c->cap_stream) HIPTRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        int brc = SHSPH_EHIP;
        hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            c->stream = c->cap_stream;
            c->capturing = true;
            brc = graph_body<T>(c);
            c->capturing = false;
            c->stream = st;
            e = hipStreamEndCapture(c->cap_stream, &g);
        }
        hipGraphExec_t x = nullptr;
        const bool ok = brc == SHSPH_OK && e == hipSuccess && g &&
                        hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (!ok) {          // this shape runs launch by launch from now on
            (void)hipGetLastError();
            c->nocap_key = key;
            c->err.clear();
            return SHSPH_OK;
        }
        c->gexec = x;
        c->gkey = key;
    }
    HIPTRY(c, hipGraphLaunch(c->gexec, st));
    // one read-back: stats, re-run counts, abort word, leaf count, cache words
    const size_t o_rr = (size_t)ninst * sizeof(InstStat), o_gs = o_rr + ninst * sizeof(u32);
    char* pin = (char*)c->pinned;
    u32* gs = P<u32>(c->gstate);
    HIPTRY(c, hipMemcpyAsync(pin, c->stat_d.p, o_rr, hipMemcpyDeviceToHost, st));
    HIPTRY(c, hipMemcpyAsync(pin + o_rr, gs + GS_WORDS, ninst * sizeof(u32), hipMemcpyDeviceToHost, st));
    const size_t o_x = o_gs + GS_WORDS * sizeof(u32);
    HIPTRY(c, hipMemcpyAsync(pin + o_gs, gs, GS_WORDS * sizeof(u32), hipMemcpyDeviceToHost, st));
    HIPTRY(c, hipMemcpyAsync(pin + o_x, P<u32>(c->xscan) + c->n, sizeof(u32),
                             hipMemcpyDeviceToHost, st));
    HIPTRY(c, hipMemcpyAsync(pin + o_x + 8, P<u64>(c->gbase) + c->n_groups, sizeof(u64),
                             hipMemcpyDeviceToHost, st));
    HIPTRY(c, hipStreamSynchronize(st));
    u32 gw[GS_WORDS], nl = 0;
    u64 words = 0;
    memcpy(gw, pin + o_gs, sizeof(gw));
    memcpy(&nl, pin + o_x, 4);
    memcpy(&words, pin + o_x + 8, 8);
    const u32 abort_w = gw[0];
    if (abort_w) {
        ++c->graph_aborts;
        c->graph_abort_why = abort_w;
        c->graph_backoff = std::min(2 * c->graph_backoff + 1, 16);
        c->graph_wait = c->graph_backoff;
        return SHSPH_OK;
    }
    ++c->graph_passes;
    c->graph_backoff = 0;
    c->n_leaf = nl;
    c->n_internal = (i64)nl - ninst;
    c->cache_words = words;
    c->restarts = 0;
    for (int b = 0; b < std::min(c->prm.max_restarts, GS_RBMAX); ++b) c->restarts += gw[GS_RB0 + b] == 0u;
    c->parts_pending = 0;
    rr.assign(ninst, 0);
    u32 nc = 0;
    const InstStat* hs = (const InstStat*)pin;
    for (int k = 0; k < ninst; ++k) {
        u32 r;
        memcpy(&r, pin + o_rr + k * sizeof(u32), 4);
        rr[k] = (int)r;
        nc += hs[k].n_noconv;
    }
    *rc = nc ? fail(c, SHSPH_ENOCONV, "h iteration did not converge for " + std::to_string(nc) + " particles")
             : SHSPH_OK;
    *done = true;
    return SHSPH_OK;
}

// The pass launch by launch; leaves the stats in the pinned staging.
template <class T> int eager_pass(shsph_ctx* c, std::vector<int>& rr, int* rc_out)
{
    hipStream_t st = c->stream;
    const int ninst = c->ninst;
    launch_stat_reset(P<InstStat>(c->stat_d), ninst, 3, nullptr, st);
    const double* dt_dev = P<double>(c->dt_inst_d);
    TRY(build<T>(c, pool_fields<T>(c), c->n, dt_dev, true));
    const i64 n = c->n;
    TRY(ensure(c, c->acc, n * sizeof(vec4<T>)));
    bool fdone = false;
    const FusedForce<T> ff{P<vec4<T>>(c->acc), &fdone};
    const int rc = run_density<T>(c, true, c->prm.fused_density_force ? &ff : nullptr);
    if (rc != SHSPH_OK && rc != SHSPH_ENOCONV) return rc;
    const SphParams sp = sph_params(c->prm);
    if (!fdone) {
        launch_stat_reset(P<InstStat>(c->stat_d), ninst, 2, nullptr, st);
        prof_begin(c, S_FORCE);
        CacheView cvf = cache_view(c);
        cvf.work = work_ptr(c, 2);
        launch_force<T>(sorted<T>(c, true), P<vec4<T>>(c->thermo), P<u32>(c->id), group_map(c),
                        c->n_groups, P<InstDev>(c->inst_d), sp, cvf, P<vec4<T>>(c->acc), nullptr,
                        P<InstStat>(c->stat_d), st);
        prof_end(c);
        TRY(check_launch(c, "force"));
    }
    const i64 nb = (n + GROUP - 1) / GROUP;
    TRY(ensure(c, c->bpart, nb * sizeof(BlockPart)));
    prof_begin(c, S_CORRECT);
    launch_correct<T>(sorted<T>(c, true), P<vec4<T>>(c->acc), P<T>(c->omega), n, P<i64>(c->poff_d),
                      ninst, P<InstDev>(c->inst_d), dt_dev, c->prm.hfact, pool_out<T>(c),
                      P<InstStat>(c->stat_d), P<BlockPart>(c->bpart), st);
    prof_end(c);
    c->parts_pending = nb;
    TRY(check_launch(c, "correct"));
    TRY(corrector_reruns<T>(c, pool_out<T>(c), dt_dev, rr));
    if (c->parts_pending > 0) {
        launch_fold_parts(P<BlockPart>(c->bpart), c->parts_pending, ninst, P<InstStat>(c->stat_d), st);
        c->parts_pending = 0;
    }
    TRY(read_back(c, c->stat_d.p, ninst * sizeof(InstStat)));
    *rc_out = rc;
    return SHSPH_OK;
}

template <class T> int batch_pass(shsph_ctx* c, const std::vector<Inst*>& b, const std::vector<double>& dt)
{
    const int ninst = (int)b.size();
    c->state = ST_NONE;
    c->ninst = ninst;
    c->inst_h.assign(ninst, InstDev());
    c->poff_h.assign(ninst + 1, 0);
    c->goff_h.assign(ninst + 1, 0);
    i64 off = 0, g = 0;
    for (int k = 0; k < ninst; ++k) {
        InstDev& in = c->inst_h[k];
        in.p_off = off;
        in.p_cnt = b[k]->n;
        in.shift = b[k]->off - off;
        for (int d = 0; d < 3; ++d) { in.lo[d] = b[k]->lo[d]; in.hi[d] = b[k]->hi[d]; }
        in.mass = b[k]->mass;
        in.periodic = b[k]->periodic;
        in.pad = 0;
        c->poff_h[k] = off;
        c->goff_h[k] = g;
        off += b[k]->n;
        g += (b[k]->n + GROUP - 1) / GROUP;
    }
    c->poff_h[ninst] = off;
    c->goff_h[ninst] = g;
    c->n = off;
    c->n_groups = g;
    c->dtype = c->pool.dtype;
    TRY(upload_instances(c));
    TRY(upload_extra(c, c->dt_inst_d.p, dt.data(), ninst * sizeof(double)));
    std::vector<int> rr;
    int rc = SHSPH_OK;
    bool done = false;
    TRY(graph_pass<T>(c, rr, &rc, &done));
    if (!done) {
        TRY(eager_pass<T>(c, rr, &rc));
        c->last_key = pass_key(c);
    }
    prof_collect(c);
    const InstStat* hs = (const InstStat*)c->pinned;
    for (int k = 0; k < ninst; ++k) {
        b[k]->stat = hs[k];
        // particles still past chi h_cache when the rebuilds ran out did not
        // converge either
        b[k]->stat.n_noconv += hs[k].n_exceed;
        b[k]->has_force = true;
        // an evaluation pass (dt 0) is not a step: the multiplier stays
        if (dt[k] > 0) {
            b[k]->reruns = rr[k];
            b[k]->lambda_cfl = next_multiplier(c->prm, b[k]->lambda_cfl, rr[k]);
        }
    }
    return rc;
}

Inst* find_inst(shsph_ctx* c, int64_t h)
{
    auto it = c->insts.find(h);
    return it == c->insts.end() ? nullptr : &it->second;
}

double inst_dt_cfl(const Inst& in)
{
    float f;
    memcpy(&f, &in.stat.dt_bits, 4);
    return (double)f;
}

// dt of an instance's next CFL step: the CFL dt times its multiplier.
double inst_dt_step(const Inst& in) { return in.lambda_cfl * inst_dt_cfl(in); }

// Resolve handles and the dt of each instance for a stepping pass; CFL
// instances without a derivative pass get one first (dt = 0).
int gather_batch(shsph_ctx* c, const int64_t* handles, int32_t count, std::vector<Inst*>& b,
                 bool server = false)
{
    if (!handles || count < 1 || count > MAX_BATCH)
        return fail(c, SHSPH_EINVAL, "batch needs 1.." + std::to_string(MAX_BATCH) + " handles");
    b.clear();
    for (int k = 0; k < count; ++k) {
        Inst* in = find_inst(c, handles[k]);
        if (!in) return fail(c, SHSPH_EINVAL, "unknown instance handle " + std::to_string(handles[k]));
        if (in->busy && !server) return fail(c, SHSPH_ESTATE, "instance is held by a serving job");
        for (Inst* o : b)
            if (o == in) return fail(c, SHSPH_EINVAL, "a handle appears twice in the batch");
        b.push_back(in);
    }
    return SHSPH_OK;
}

int run_pass(shsph_ctx* c, const std::vector<Inst*>& b, const std::vector<double>& dt)
{
    return c->pool.dtype == SHSPH_F32 ? batch_pass<float>(c, b, dt) : batch_pass<double>(c, b, dt);
}

}  // namespace

// Internal entry points of the serving loop (serve.cpp): a pass over pooled
// instances, their sizes, and the context lock.
int shsph_internal_pass(shsph_ctx* c, const int64_t* handles, const double* dt, int32_t count)
{
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    std::vector<Inst*> b;
    TRY(gather_batch(c, handles, count, b, true));
    HIPTRY(c, hipSetDevice(c->device));
    return run_pass(c, b, std::vector<double>(dt, dt + count));
}

int shsph_internal_inst_state(shsph_ctx* c, int64_t h, int64_t* n, int* has_force, double* dt_cfl, int busy_delta)
{
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    Inst* in = find_inst(c, h);
    if (!in) return SHSPH_EINVAL;
    if (n) *n = in->n;
    if (has_force) *has_force = in->has_force ? 1 : 0;
    if (dt_cfl) *dt_cfl = inst_dt_step(*in);
    in->busy += busy_delta;
    return SHSPH_OK;
}

void*& shsph_internal_server(shsph_ctx* c) { return c->server; }
int shsph_internal_dtype(shsph_ctx* c) { return c->pool.dtype; }

// =========================================================== C interface ===
extern "C" {

void shsph_params_default(shsph_params* p)
{
    if (!p) return;
    p->hfact = 1.2;
    p->gamma = 5.0 / 3.0;
    p->alpha_av = 1.0;
    p->beta_av = 2.0;
    p->beta_u = 1.0;
    p->chi = 1.1;
    p->lambda = 1.2;
    p->eps_h = 1e-6;
    p->c_cour = 0.3;
    p->c_force = 0.25;
    p->max_iter = 50;
    p->n_red = 3;
    p->max_restarts = 8;
    p->spread_slots = 8192;
    p->stage1_serial = 0;
    p->stage2_mode = 1;
    p->kernel = SHSPH_KERNEL_M4;
    p->key_bits = 63;
    p->eps_v = 0.0;
    p->max_reruns = 3;
    p->alpha_switch = 0;
    p->lambda_stiff = 1.0;
    p->alpha_min = 0.0;
    p->alpha_max = 1.0;
    p->sigma_decay = 0.1;
    p->force_split = 2;
    p->fused_density_force = 0;
    p->graph_batch = 1;
}

// Every device buffer of a context.
static std::vector<Buf*> all_bufs(shsph_ctx* c)
{
    return { &c->keys[0], &c->keys[1], &c->vals[0], &c->vals[1], &c->hist,
             &c->scan_tmp, &c->bbox, &c->posh, &c->velu, &c->vhalf, &c->hn, &c->hcache,
             &c->pid_s, &c->thermo, &c->omega, &c->acc, &c->vsig, &c->status, &c->xi[0],
             &c->xi[1], &c->xscan, &c->id, &c->mu_leaf, &c->lchild, &c->rchild, &c->endrange,
             &c->lflag, &c->rflag, &c->child, &c->parent, &c->arrive, &c->blo, &c->bhi,
             &c->rec, &c->nrec, &c->rscan, &c->glo, &c->ghi, &c->uleaf, &c->uslot,
             &c->ucnt, &c->ustot, &c->nlist, &c->ncnt, &c->flags, &c->inst_d, &c->poff_d,
             &c->goff_d, &c->leaf_off_d, &c->ioff_d, &c->root_d, &c->stat_d,
             &c->dt_inst_d, &c->dt_host_d, &c->pbox, &c->plen, &c->xoff, &c->xlist,
             &c->bpart, &c->work[0], &c->work[1], &c->work[2], &c->redo_d, &c->rhmax_d,
             &c->alpha_s, &c->lvstate, &c->gcap, &c->gbase, &c->gneed, &c->gredo };
}

// Parameter ranges accepted by shsph_create and shsph_set_params.
static bool params_valid(const shsph_params& q)
{
    return (q.hfact > 0) && (q.chi >= 1) && (q.lambda > 1) && (q.eps_h > 0) &&
           !(q.max_iter < 1 || q.n_red > 20 || q.max_restarts < 0 ||
             q.spread_slots < 1 || q.stage2_mode < 0 || q.stage2_mode > 2 ||
             q.kernel < 0 || q.kernel >= KERNEL_COUNT ||
             (q.key_bits != 63 && q.key_bits != 30) || !(q.eps_v >= 0) ||
             q.max_reruns < 0 || !(q.lambda_stiff >= 0) || !(q.sigma_decay > 0) ||
             !(q.alpha_min >= 0) || !(q.alpha_max >= q.alpha_min) ||
             (q.force_split != 1 && q.force_split != 2) ||
             (q.fused_density_force != 0 && q.fused_density_force != 1) ||
             (q.graph_batch != 0 && q.graph_batch != 1));
}

int shsph_create(int device, const shsph_params* p, shsph_ctx** out)
{
    if (!out) return SHSPH_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SHSPH_EINVAL;
    shsph_ctx* c = new shsph_ctx();
    c->device = device;
    if (p) c->prm = *p; else shsph_params_default(&c->prm);
    if (!params_valid(c->prm)) {
        delete c;
        return SHSPH_EINVAL;
    }

    if (hipSetDevice(device) != hipSuccess || hipHostMalloc(&c->pinned, PINNED_BYTES + UPLOAD_BYTES) != hipSuccess) {
        delete c;
        return SHSPH_EHIP;
    }
    if (hipEventCreateWithFlags(&c->up_done, hipEventDisableTiming) != hipSuccess) {
        if (c->up_done) hipEventDestroy(c->up_done);
        hipHostFree(c->pinned);
        delete c;
        return SHSPH_EHIP;
    }
    c->stream = nullptr;
    // the allocation-free step's context: buffers in this device's scratch
    // array, staging shared with this context
    c->sc = new shsph_ctx();
    c->sc->device = device;
    c->sc->pinned = c->pinned;
    c->sc->up_done = c->up_done;
    c->sc->arena = scratch_on(device);
    *out = c;
    return SHSPH_OK;
}

int shsph_destroy(shsph_ctx* c)
{
    if (!c) return SHSPH_EINVAL;
    if (c->server) shsph_serve_stop(c);
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    pool_release(c);
    graph_drop(c);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    if (c->up_done) hipEventDestroy(c->up_done);
    for (Buf* b : all_bufs(c))
        if (b->p) hipFree(b->p);
    delete c->sc;                 // its buffers live in the scratch array, its staging is ours
    if (c->pinned) hipHostFree(c->pinned);
    for (hipEvent_t e : c->prof.ev) hipEventDestroy(e);
    delete c;
    return SHSPH_OK;
}

int shsph_set_params(shsph_ctx* c, const shsph_params* p)
{
    if (!c || !p) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    if (c->server) return fail(c, SHSPH_ESTATE, "parameters cannot change while serving");
    if (!params_valid(*p)) return fail(c, SHSPH_EINVAL, "parameter out of range");
    c->prm = *p;
    ++c->param_gen;
    return SHSPH_OK;
}

int shsph_get_params(shsph_ctx* c, shsph_params* out)
{
    if (!c || !out) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    *out = c->prm;
    return SHSPH_OK;
}

int shsph_set_stream(shsph_ctx* c, void* stream)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->stream = (hipStream_t)stream;
    return SHSPH_OK;
}

const char* shsph_last_error(const shsph_ctx* c) { return c ? c->err.c_str() : "null context"; }

int shsph_build_tree(shsph_ctx* c, const shsph_particles* p)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    TRY(validate(c, p, false, false));
    HIPTRY(c, hipSetDevice(c->device));
    return p->dtype == SHSPH_F32 ? do_build<float>(c, p) : do_build<double>(c, p);
}

int shsph_density(shsph_ctx* c, shsph_particles* p)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    TRY(validate(c, p, false, false));
    if (c->state < ST_TREE || p->n != c->n || p->dtype != c->dtype)
        return fail(c, SHSPH_ESTATE, "shsph_density needs shsph_build_tree on the same particles");
    HIPTRY(c, hipSetDevice(c->device));
    return p->dtype == SHSPH_F32 ? do_density<float>(c, p) : do_density<double>(c, p);
}

int shsph_force(shsph_ctx* c, shsph_particles* p)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    TRY(validate(c, p, true, true));
    if (c->state < ST_DENSITY || p->n != c->n || p->dtype != c->dtype)
        return fail(c, SHSPH_ESTATE, "shsph_force needs shsph_density on the same particles");
    HIPTRY(c, hipSetDevice(c->device));
    return p->dtype == SHSPH_F32 ? do_force<float>(c, p) : do_force<double>(c, p);
}

int shsph_step(shsph_ctx* c, shsph_particles* p, double dt, double* dt_used)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    TRY(validate(c, p, true, true));
    if (!std::isfinite(dt)) return fail(c, SHSPH_EINVAL, "dt must be finite");
    HIPTRY(c, hipSetDevice(c->device));
    return p->dtype == SHSPH_F32 ? do_step<float>(c, p, dt, dt_used)
                                 : do_step<double>(c, p, dt, dt_used);
}

int shsph_step_noalloc(shsph_ctx* c, shsph_particles* p, double dt, double* dt_used)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    shsph_ctx* s = c->sc;
    if (!s || !s->arena) return fail(c, SHSPH_EHIP, "the static scratch array is not available on this device");
    TRY(validate(c, p, true, true));
    if (!std::isfinite(dt)) return fail(c, SHSPH_EINVAL, "dt must be finite");
    if (p->n > SCRATCH_MAX_N)
        return fail(c, SHSPH_ECAPACITY, "shsph_step_noalloc takes at most " +
                    std::to_string(SCRATCH_MAX_N) + " particles (n = " + std::to_string(p->n) + ")");
    HIPTRY(c, hipSetDevice(c->device));
    s->prm = c->prm;
    s->stream = c->stream;
    s->err.clear();
    // every buffer is laid out afresh in the array for this call; device
    // contents of earlier calls (the cache capacity history) are not kept
    for (Buf* b : all_bufs(s)) { b->p = nullptr; b->cap = 0; }
    s->arena_used = 0;
    s->gneed_groups = -1;
    int rc = p->dtype == SHSPH_F32 ? do_step<float>(s, p, dt, dt_used)
                                   : do_step<double>(s, p, dt, dt_used);
    if (rc == SHSPH_OK) {
        // keep this step's reductions (its CFL dt) for the next call, and
        // leave no work of this call running on the array
        if (s->parts_pending > 0) {
            launch_fold_parts(P<BlockPart>(s->bpart), s->parts_pending, s->ninst,
                              P<InstStat>(s->stat_d), s->stream);
            s->parts_pending = 0;
        }
        rc = read_back(s, s->stat_d.p, sizeof(InstStat));
        if (rc == SHSPH_OK) memcpy(&s->stat_keep, s->pinned, sizeof(InstStat));
    }
    s->stat_kept = rc == SHSPH_OK;
    if (rc != SHSPH_OK) {
        s->state = ST_NONE;
        (void)hipStreamSynchronize(s->stream);
        c->err = s->err;
    }
    return rc;
}

int shsph_set_profiling(shsph_ctx* c, int on)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->prof.on = on != 0;
    c->prof.used = 0;
    HIPTRY(c, hipSetDevice(c->device));
    for (int k = 0; k < 3; ++k) {
        TRY(ensure(c, c->work[k], 128 * sizeof(u64)));
        launch_fill_u32(P<u32>(c->work[k]), 256, 0u, c->stream);
    }
    for (int i = 0; i < S_NUM; ++i) { c->prof.ms[i] = 0; c->prof.launches[i] = 0; }
    return SHSPH_OK;
}

int shsph_get_work(shsph_ctx* c, double* out6)
{
    if (!c || !out6) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (int k = 0; k < 6; ++k) out6[k] = 0.0;
    HIPTRY(c, hipSetDevice(c->device));
    for (int k = 0; k < 3; ++k) {
        if (!c->work[k].p) continue;
        u64 w[128];
        HIPTRY(c, hipMemcpyAsync(w, c->work[k].p, sizeof(w), hipMemcpyDeviceToHost, c->stream));
        HIPTRY(c, hipStreamSynchronize(c->stream));
        for (int s = 0; s < 64; ++s) { out6[2 * k] += (double)w[2 * s]; out6[2 * k + 1] += (double)w[2 * s + 1]; }
    }
    return SHSPH_OK;
}

int shsph_get_stage_times(shsph_ctx* c, double* ms, int64_t* launches, int32_t n)
{
    if (!c || n < 0) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (int i = 0; i < n && i < S_NUM; ++i) {
        if (ms) ms[i] = c->prof.ms[i];
        if (launches) launches[i] = c->prof.launches[i];
    }
    return SHSPH_OK;
}

const char* shsph_stage_name(int32_t i) { return (i >= 0 && i < S_NUM) ? STAGE_NAMES[i] : ""; }

int shsph_get_info(shsph_ctx* c, shsph_info* o)
{
    if (!c || !o) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    memset(o, 0, sizeof(*o));
    o->n = c->n;
    o->n_leaf = c->n_leaf;
    o->n_groups = c->n_groups;
    o->n_red = c->prm.n_red;
    o->restarts = c->restarts;
    o->reruns = c->reruns_last;
    o->cache_capacity = c->n > 0 ? (int32_t)(4 * c->cache_words * GROUP / c->n) : 0;
    o->cfl_multiplier = c->lambda_cfl;
    o->graph_passes = c->graph_passes;
    o->graph_aborts = c->graph_aborts;
    o->graph_abort_why = (int32_t)c->graph_abort_why;
    HIPTRY(c, hipSetDevice(c->device));
    if (c->state >= ST_TREE) {
        u64 t1 = 0, t2 = 0;
        TRY(sum_u32(c, P<u32>(c->ucnt), c->n_groups, &t1));
        TRY(sum_u32(c, P<u32>(c->ncnt), c->n, &t2));
        o->n_leaf_neigh = (int64_t)t1;
        o->n_neigh = (int64_t)t2;
    }
    if (c->stat_d.p && c->ninst >= 1) {
        if (c->parts_pending > 0) {
            launch_fold_parts(P<BlockPart>(c->bpart), c->parts_pending, c->ninst,
                              P<InstStat>(c->stat_d), c->stream);
            c->parts_pending = 0;
        }
        InstStat s;
        HIPTRY(c, hipMemcpyAsync(c->pinned, c->stat_d.p, sizeof(InstStat), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPTRY(c, hipStreamSynchronize(c->stream));
        memcpy(&s, c->pinned, sizeof(s));
        float dt, dv;
        memcpy(&dt, &s.dt_bits, 4);
        memcpy(&dv, &s.dvmax_bits, 4);
        o->dt_cfl = dt;
        o->dv_max = dv;
        for (int i = 0; i < STAT_SLOTS; ++i) { o->dv2_sum += s.dv2_part[i]; o->v2_sum += s.v2_part[i]; }
        o->max_iter_seen = (int32_t)s.max_iter_seen;
        o->n_noconv = (int32_t)s.n_noconv;
    }
    return SHSPH_OK;
}

int shsph_export_tree(shsph_ctx* c, const shsph_tree_export* o)
{
    if (!c || !o) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (c->state < ST_TREE) return fail(c, SHSPH_ESTATE, "no tree built");
    HIPTRY(c, hipSetDevice(c->device));
    hipStream_t st = c->stream;
    // rows in compact numbering: internal nodes, then leaf j at ni + j (on
    // the device leaf j is node lbase + j)
    const i64 n = c->n, nl = c->n_leaf, ni = c->n_internal, nn = ni + nl, G = c->n_groups;
    const i64 lb = c->lbase;
    const size_t T = c->dtype == SHSPH_F32 ? 4 : 8;
    auto cp = [&](void* dst, const void* src, size_t bytes) -> int {
        if (dst && bytes) HIPTRY(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st));
        return SHSPH_OK;
    };
    // keys in caller order are not kept after the sort: scatter back through eps
    if (o->keys) {
        std::vector<u64> mu(n);
        std::vector<u32> eps(n);
        HIPTRY(c, hipMemcpyAsync(mu.data(), c->keys[c->vals_sel].p, n * 8, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipMemcpyAsync(eps.data(), c->vals[c->vals_sel].p, n * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipStreamSynchronize(st));
        for (i64 i = 0; i < n; ++i) o->keys[eps[i]] = mu[i];
    }
    TRY(cp(o->eps, c->vals[c->vals_sel].p, n * 4));
    TRY(cp(o->mu, c->keys[c->vals_sel].p, n * 8));
    TRY(cp(o->xi, c->xi[c->xi_sel].p, n));
    TRY(cp(o->id, c->id.p, (nl + 1) * 4));
    TRY(cp(o->mu_leaf, c->mu_leaf.p, nl * 8));
    if (ni > 0) {
        TRY(cp(o->lchild, c->lchild.p, ni * 4));
        TRY(cp(o->rchild, c->rchild.p, ni * 4));
        TRY(cp(o->endrange, c->endrange.p, ni * 4));
        TRY(cp(o->lflag, c->lflag.p, ni));
        TRY(cp(o->rflag, c->rflag.p, ni));
    }
    if (o->parent) {
        TRY(cp(o->parent, c->parent.p, ni * 4));
        TRY(cp(o->parent + ni, P<u32>(c->parent) + lb, nl * 4));
    }
    if (o->bmin || o->bmax || o->hmax) {
        const size_t row = 4 * T;
        std::vector<char> lo(nn * row), hi(nn * row);
        HIPTRY(c, hipMemcpyAsync(lo.data(), c->blo.p, ni * row, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipMemcpyAsync(hi.data(), c->bhi.p, ni * row, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipMemcpyAsync(lo.data() + ni * row, (char*)c->blo.p + lb * row, nl * row,
                                 hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipMemcpyAsync(hi.data() + ni * row, (char*)c->bhi.p + lb * row, nl * row,
                                 hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipStreamSynchronize(st));
        for (i64 v = 0; v < nn; ++v) {
            for (int d = 0; d < 3; ++d) {
                if (o->bmin) memcpy((char*)o->bmin + (3 * v + d) * T, &lo[(4 * v + d) * T], T);
                if (o->bmax) memcpy((char*)o->bmax + (3 * v + d) * T, &hi[(4 * v + d) * T], T);
            }
            if (o->hmax) memcpy((char*)o->hmax + v * T, &lo[(4 * v + 3) * T], T);
        }
    }
    if (o->pbox || o->plen) {
        TRY(ensure(c, c->pbox, 6 * nn * sizeof(u32)));
        TRY(ensure(c, c->plen, nn * sizeof(i32)));
        launch_prefix_boxes(P<u64>(c->mu_leaf), P<i64>(c->leaf_off_d), P<i64>(c->ioff_d), c->ninst,
                            ni, nl, lb, P<u32>(c->endrange), P<u32>(c->parent), P<u32>(c->pbox),
                            P<i32>(c->plen), c->key_bits_built == 30 ? 33 : 0, st);
        TRY(check_launch(c, "prefix boxes"));
        TRY(cp(o->pbox, c->pbox.p, 6 * nn * 4));
        TRY(cp(o->plen, c->plen.p, nn * 4));
    }
    if (o->group_off || o->group_leaves) {
        std::vector<u32> cnt(G), ul((size_t)G * c->cap_leaf);
        HIPTRY(c, hipMemcpyAsync(cnt.data(), c->ucnt.p, G * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipMemcpyAsync(ul.data(), c->uleaf.p, ul.size() * 4, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipStreamSynchronize(st));
        u64 off = 0;
        for (i64 g = 0; g < G; ++g) {
            if (o->group_off) o->group_off[g] = off;
            if (o->group_leaves)
                memcpy(o->group_leaves + off, &ul[(size_t)g * c->cap_leaf], cnt[g] * 4);
            off += cnt[g];
        }
        if (o->group_off) o->group_off[G] = off;
    }
    if (o->neigh_off || o->neigh_list) {
        u64 total = 0;
        TRY(ensure(c, c->xoff, (n + 1) * sizeof(u64)));
        TRY(ensure(c, c->scan_tmp, scan_tmp_bytes(n + 1)));
        scan_u32_u64(P<u32>(c->ncnt), P<u64>(c->xoff), n, c->scan_tmp.p, st);
        TRY(read_back(c, P<u64>(c->xoff) + n, 8));
        total = *(u64*)c->pinned;
        TRY(ensure(c, c->xlist, std::max<u64>(total, 1) * sizeof(u32)));
        launch_cache_to_global(P<u32>(c->id), group_map(c), G, c->cap_leaf, P<u32>(c->uleaf),
                               P<u32>(c->uslot), P<u32>(c->ucnt), P<u32>(c->ustot),
                               P<u64>(c->gbase), P<u64>(c->nlist),
                               P<u32>(c->ncnt), P<u64>(c->xoff), P<u32>(c->xlist), st);
        TRY(check_launch(c, "cache export"));
        TRY(cp(o->neigh_off, c->xoff.p, (n + 1) * 8));
        TRY(cp(o->neigh_list, c->xlist.p, total * 4));
    }
    if (o->h_sorted) {
        std::vector<char> ph(n * 4 * T);
        HIPTRY(c, hipMemcpyAsync(ph.data(), c->posh.p, n * 4 * T, hipMemcpyDeviceToHost, st));
        HIPTRY(c, hipStreamSynchronize(st));
        for (i64 i = 0; i < n; ++i) memcpy((char*)o->h_sorted + i * T, &ph[(4 * i + 3) * T], T);
    }
    TRY(cp(o->h_cache, c->hcache.p, n * T));
    HIPTRY(c, hipStreamSynchronize(st));
    return SHSPH_OK;
}


// ----------------------------------------------- pooled instances, batches ---
int shsph_instance_create(shsph_ctx* c, const shsph_particles* p, int64_t* handle)
{
    if (!c || !handle) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    TRY(validate(c, p, true, false));
    HIPTRY(c, hipSetDevice(c->device));
    Pool& q = c->pool;
    if (q.used == 0 && q.dtype != p->dtype) {
        HIPTRY(c, hipStreamSynchronize(c->stream));
        pool_release(c);
        q.dtype = p->dtype;
    }
    if (q.dtype != p->dtype)
        return fail(c, SHSPH_EINVAL, "all pooled instances of a context share one dtype");
    const i64 n = p->n;
    i64 off = 0;
    TRY(pool_alloc(c, n, &off));
    const size_t es = pool_elem(PF_X, q.dtype);
    const void* src[PF_NUM] = { p->x, p->y, p->z, p->vx, p->vy, p->vz, p->u, p->h,
                                p->ax, p->ay, p->az, p->dudt, p->rho, p->omega, p->pid };
    int rc = SHSPH_OK;
    for (int f = 0; f < PF_NUM && rc == SHSPH_OK; ++f) {
        char* dst = (char*)q.fld[f] + off * pool_elem(f, q.dtype);
        hipError_t e;
        if (src[f]) e = hipMemcpyAsync(dst, src[f], n * pool_elem(f, q.dtype), hipMemcpyDefault, c->stream);
        else if (f == PF_PID) { launch_iota_u32((u32*)dst, n, c->stream); e = hipGetLastError(); }
        else e = hipMemsetAsync(dst, 0, n * es, c->stream);
        if (e != hipSuccess) rc = fail(c, SHSPH_EHIP, std::string("instance copy: ") + hipGetErrorString(e));
    }
    if (rc == SHSPH_OK && hipStreamSynchronize(c->stream) != hipSuccess)
        rc = fail(c, SHSPH_EHIP, "instance copy failed");
    if (rc != SHSPH_OK) {
        pool_put(q, off, n);
        q.used -= n;
        return rc;
    }
    Inst in;
    in.off = off;
    in.n = n;
    in.mass = p->mass;
    for (int d = 0; d < 3; ++d) { in.lo[d] = p->lo[d]; in.hi[d] = p->hi[d]; }
    in.periodic = p->periodic ? 1 : 0;
    memset(&in.stat, 0, sizeof(in.stat));
    in.stat.dt_bits = 0x7f800000u;
    *handle = c->next_handle++;
    c->insts[*handle] = in;
    return SHSPH_OK;
}

int shsph_instance_destroy(shsph_ctx* c, int64_t handle)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    Inst* in = find_inst(c, handle);
    if (!in) return fail(c, SHSPH_EINVAL, "unknown instance handle");
    if (in->busy) return fail(c, SHSPH_ESTATE, "instance is held by a serving job");
    pool_put(c->pool, in->off, in->n);
    c->pool.used -= in->n;
    c->insts.erase(handle);
    return SHSPH_OK;
}

int shsph_instance_read(shsph_ctx* c, int64_t handle, const shsph_particles* out)
{
    if (!c || !out) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    Inst* in = find_inst(c, handle);
    if (!in) return fail(c, SHSPH_EINVAL, "unknown instance handle");
    if (out->n != in->n || out->dtype != c->pool.dtype)
        return fail(c, SHSPH_EINVAL, "output size or dtype differs from the instance");
    HIPTRY(c, hipSetDevice(c->device));
    Pool& q = c->pool;
    void* dst[PF_NUM] = { out->x, out->y, out->z, out->vx, out->vy, out->vz, out->u, out->h,
                          out->ax, out->ay, out->az, out->dudt, out->rho, out->omega, out->pid };
    for (int f = 0; f < PF_NUM; ++f) {
        if (!dst[f]) continue;
        const size_t es = pool_elem(f, q.dtype);
        HIPTRY(c, hipMemcpyAsync(dst[f], (char*)q.fld[f] + in->off * es, in->n * es,
                                 hipMemcpyDefault, c->stream));
    }
    HIPTRY(c, hipStreamSynchronize(c->stream));
    return SHSPH_OK;
}

int shsph_instance_info(shsph_ctx* c, int64_t handle, shsph_info* o)
{
    if (!c || !o) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    Inst* in = find_inst(c, handle);
    if (!in) return fail(c, SHSPH_EINVAL, "unknown instance handle");
    memset(o, 0, sizeof(*o));
    o->n = in->n;
    o->n_red = c->prm.n_red;
    const InstStat& s = in->stat;
    float dv;
    memcpy(&dv, &s.dvmax_bits, 4);
    o->dt_cfl = inst_dt_cfl(*in);
    o->dv_max = dv;
    for (int i = 0; i < STAT_SLOTS; ++i) { o->dv2_sum += s.dv2_part[i]; o->v2_sum += s.v2_part[i]; }
    o->max_iter_seen = (int32_t)s.max_iter_seen;
    o->n_noconv = (int32_t)s.n_noconv;
    o->reruns = in->reruns;
    o->cfl_multiplier = in->lambda_cfl;
    return SHSPH_OK;
}

int shsph_step_batch(shsph_ctx* c, const int64_t* handles, int32_t count, const double* dt,
                     double* dt_used)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    std::vector<Inst*> b;
    TRY(gather_batch(c, handles, count, b));
    HIPTRY(c, hipSetDevice(c->device));
    std::vector<Inst*> pre;
    for (int k = 0; k < count; ++k) {
        const double d = dt ? dt[k] : 0.0;
        if (!std::isfinite(d)) return fail(c, SHSPH_EINVAL, "dt must be finite");
        if (!(d > 0) && !b[k]->has_force) pre.push_back(b[k]);
    }
    int rc = SHSPH_OK;
    if (!pre.empty()) {
        rc = run_pass(c, pre, std::vector<double>(pre.size(), 0.0));
        if (rc != SHSPH_OK) return rc;
    }
    std::vector<double> d(count);
    for (int k = 0; k < count; ++k) {
        d[k] = (dt && dt[k] > 0) ? dt[k] : inst_dt_step(*b[k]);
        if (!(d[k] > 0) || !std::isfinite(d[k]))
            return fail(c, SHSPH_ESTATE, "no finite CFL dt for instance " + std::to_string(handles[k]));
    }
    rc = run_pass(c, b, d);
    if (dt_used && (rc == SHSPH_OK || rc == SHSPH_ENOCONV))
        for (int k = 0; k < count; ++k) dt_used[k] = d[k];
    return rc;
}

int shsph_eval_batch(shsph_ctx* c, const int64_t* handles, int32_t count)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    std::vector<Inst*> b;
    TRY(gather_batch(c, handles, count, b));
    HIPTRY(c, hipSetDevice(c->device));
    return run_pass(c, b, std::vector<double>(count, 0.0));
}

int shsph_pool_usage(shsph_ctx* c, int64_t* particles_used, int64_t* particles_cap, int64_t* n_instances)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (particles_used) *particles_used = c->pool.used;
    if (particles_cap) *particles_cap = c->pool.cap;
    if (n_instances) *n_instances = (int64_t)c->insts.size();
    return SHSPH_OK;
}


// Autotuner for batched passes: leaf size (n_red) x stage-2 walk, timed on
// evaluation passes of the given instances; the fastest is kept.
int shsph_autotune(shsph_ctx* c, const int64_t* handles, int32_t count, int32_t* n_red_out,
                   int32_t* mode_out, int32_t* split_out, double* ms_out)
{
    if (!c) return SHSPH_EINVAL;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    c->err.clear();
    std::vector<Inst*> b;
    TRY(gather_batch(c, handles, count, b));
    HIPTRY(c, hipSetDevice(c->device));
    const std::vector<double> zero(count, 0.0);
    const shsph_params keep = c->prm;
    double best = 1e300;
    int best_nr = keep.n_red, best_md = keep.stage2_mode, best_fs = keep.force_split;
    for (int nr = 2; nr <= 4; ++nr) {
        for (int md = 0; md <= 2; ++md) {
            for (int fs = 0; fs <= 2; ++fs) {     // 0: the fused density + force launch
                c->prm.n_red = nr;
                c->prm.stage2_mode = md;
                c->prm.force_split = fs ? fs : 1;
                c->prm.fused_density_force = fs ? 0 : 1;
                ++c->param_gen;
                double t = 0;
                // the first pass sizes buffers, the second records a captured
                // pass (when those are on), the third is timed
                for (int rep = 0; rep < 3; ++rep) {
                    const auto t0 = std::chrono::steady_clock::now();
                    const int rc = run_pass(c, b, zero);
                    if (rc != SHSPH_OK && rc != SHSPH_ENOCONV) {
                        c->prm = keep;
                        ++c->param_gen;
                        return rc;
                    }
                    t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                }
                if (t < best) { best = t; best_nr = nr; best_md = md; best_fs = fs; }
            }
        }
    }
    c->prm = keep;
    c->prm.n_red = best_nr;
    c->prm.stage2_mode = best_md;
    c->prm.force_split = best_fs ? best_fs : 1;
    c->prm.fused_density_force = best_fs ? 0 : 1;
    ++c->param_gen;
    if (n_red_out) *n_red_out = best_nr;
    if (mode_out) *mode_out = best_md;
    if (split_out) *split_out = best_fs;
    if (ms_out) *ms_out = best;
    return SHSPH_OK;
}

}  // extern "C"
