// host_jobs.hpp -- host side of batches and of the server: job layout in one
// arena, the job table, the persistent launch of k_jobs, and (server) a host
// thread that admits queued jobs by device memory, publishes them to the
// running kernel and collects finished jobs.  Included once, by ptmi.hip.
#pragma once
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

namespace {

constexpr int kJobEvents = 64;

double now_s()
{
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

pt_status validate_job(const pt_job_desc &j)
{
    pt_status st = validate(j.L, j.q, j.sigma, j.T, j.R);
    if (st != PT_OK) return st;
    if (j.sweeps < 0 || j.sweeps > INT32_MAX) return fail(PT_EINVAL, "sweeps must be in [0, 2^31)");
    if (j.exchange_every < 1) return fail(PT_EINVAL, "exchange_every must be >= 1");
    if (j.init != PT_INIT_RANDOM && j.init != PT_INIT_ORDERED) return fail(PT_EINVAL, "bad init");
    return PT_OK;
}

// Device bytes of a server: the job arena, the ticket counter, and one pair of
// ready / finished words per job slot.
size_t server_bytes(size_t arena_bytes, int32_t max_jobs)
{
    return Layout::up(arena_bytes) + Layout::up(sizeof(JobControl)) +
           Layout::up(sizeof(unsigned long long) * kJcWords * static_cast<size_t>(max_jobs));
}

size_t job_bytes(const pt_job_desc &j, int prec)
{
    return Layout::up(layout_of(j.L, j.q, j.R, prec, 0, kJobEvents).total);
}

// Carve of one job inside a workgroup LDS budget, and which kernel variant
// runs it: the table in LDS if it fits; else, for q <= 7 (at most six stored
// rows), in HBM (two, four or six register rows per flush: 1.7x faster than
// direct sums on the 16384-site, q = 5 instance), and for larger q direct sums
// with no table (an HBM flush of eight rows, or row by row, per flip ran the
// 256-job batch at half the speed of direct sums); int32 tables always keep
// their table.
pt_status job_plan(const pt_job_desc &j, int prec, int budget, int threads, LdsPlan *plan, int32_t *variant)
{
    const size_t b = static_cast<size_t>(budget);
    const bool in_lds = make_plan(j.L, j.q, j.R, prec, true, kPlLds, b, threads, plan);
    const int spill = (j.q <= 7 || prec == PT_PREC_I32) ? kPlHbm : kPlDirect;
    if (!in_lds && !make_plan(j.L, j.q, j.R, prec, true, spill, b, threads, plan))
        return fail(PT_EINVAL, "job with L = %d, R = %d does not fit an LDS budget of %d B", j.L, j.R, budget);
    *variant = job_variant(plan->place, j.q, plan->j64_in_lds != 0);
    return PT_OK;
}

const void *jobs_fn_prec(int prec)
{
    if (prec == PT_PREC_F32) return jobs_kernel_f32();
    if (prec == PT_PREC_I32) return jobs_kernel_i32();
    return jobs_kernel_f64();
}

// Resident workgroups of k_jobs for (threads, budget) on this device.
pt_status jobs_capacity(int prec, int threads, int budget, int *cap)
{
    int dev = 0, cus = 0, per_cu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const void *fn = jobs_fn_prec(prec);
    HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, budget));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, budget));
    *cap = per_cu * cus;
    return PT_OK;
}

void job_slot(JobSlot &S, const pt_job_desc &j, int prec, unsigned char *base, const double *Tdev,
              const LdsPlan &plan, int32_t variant, int32_t wbase, unsigned long long *jc)
{
    const Layout lay = layout_of(j.L, j.q, j.R, prec, 0, kJobEvents);
    std::memset(&S, 0, sizeof S);
    fill_inst(S.inst, base, lay, j.L, j.q, j.R, j.seed, 0, 0, kJobEvents);
    S.plan = plan;
    S.T = Tdev;
    S.jc = jc;
    S.sigma = j.sigma;
    S.sweeps = j.sweeps;
    S.xevery = j.exchange_every;
    S.init = j.init;
    S.wbase = wbase;
    S.variant = variant;
}

// Walker workgroup shape: threads (default 256: four waves, one per SIMD),
// and LDS bytes per workgroup (default: all the device allows beside k_jobs'
// own static LDS, so that as many jobs as possible keep their field table in
// LDS; one walker per CU either way once a budget exceeds half the LDS).
pt_status shape_defaults(const pt_options &o, int prec, int *threads, int *budget)
{
    *threads = o.threads ? o.threads : 256;
    int dev = 0, lds_max = 0;
    hipFuncAttributes fa;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    HIPCHK(hipFuncGetAttributes(&fa, jobs_fn_prec(prec)));
    const int cap = (lds_max - static_cast<int>(fa.sharedSizeBytes)) & ~255;
    *budget = o.lds_budget > 0 ? std::min(cap, o.lds_budget) : cap;
    if (*threads % kWave || *threads < kWave || *threads > kMaxJobThreads)
        return fail(PT_EINVAL, "threads must be a multiple of 64 in [64, %d]", kMaxJobThreads);
    if (*budget < 4096) return fail(PT_EINVAL, "lds_budget must be at least 4096 B");
    return PT_OK;
}

pt_status fetch_spins(const Inst &P, hipStream_t st, uint8_t *spins, int32_t *perm)
{
    const size_t n = static_cast<size_t>(P.R) * P.L;
    if (spins) {
        HIPCHK(hipMemcpyAsync(spins, P.spins, n, hipMemcpyDeviceToHost, st));
    }
    if (perm) HIPCHK(hipMemcpyAsync(perm, P.perm, sizeof(int32_t) * P.R, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (spins)
        for (size_t e = 0; e < n; ++e) spins[e] = static_cast<uint8_t>(spins[e] + 1);
    return PT_OK;
}

}  // namespace

// ===========================================================================
// Batches
// ===========================================================================
struct pt_batch {
    int32_t njobs = 0, prec = 0, threads = 256, budget = 0, grid = 0;
    hipStream_t stream = nullptr;
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false, ran = false;
    std::vector<JobSlot> slots;       // by job index
    std::vector<JobSlot> exec_slots;  // in launch order (the device's job table)
    std::vector<pt_job_desc> jobs;
    JobSlot *d_slots = nullptr;
    JobControl *d_ctl = nullptr;
    unsigned long long *d_jc = nullptr;  // [njobs][kJcWords] ready / finished words, clocks
    double *d_T = nullptr;
    std::vector<double> Tall;
    size_t slots_off = 0, ctl_off = 0, jc_off = 0, T_off = 0, total = 0;
    std::vector<size_t> job_off;
};

namespace {

pt_status batch_layout(const pt_job_desc *jobs, int32_t n, const pt_options &o, pt_batch *b)
{
    if (!jobs || n < 1) return fail(PT_EINVAL, "no jobs");
    if (!valid_prec(o.precision)) return fail(PT_EINVAL, "bad precision");
    size_t off = 0, nT = 0;
    b->job_off.resize(n);
    for (int j = 0; j < n; ++j) {
        const pt_status st = validate_job(jobs[j]);
        if (st != PT_OK) return fail(st, "job %d: %s", j, pt_last_error());
        b->job_off[j] = off;
        off += job_bytes(jobs[j], o.precision);
        nT += static_cast<size_t>(jobs[j].R);
    }
    b->slots_off = off;
    off += Layout::up(sizeof(JobSlot) * n);
    b->ctl_off = off;
    off += Layout::up(sizeof(JobControl));
    b->jc_off = off;
    off += Layout::up(sizeof(unsigned long long) * kJcWords * static_cast<size_t>(n));
    b->T_off = off;
    off += Layout::up(sizeof(double) * nT);
    b->total = off;
    return PT_OK;
}

}  // namespace

extern "C" {

pt_status pt_batch_workspace_size(const pt_job_desc *jobs, int32_t njobs, const pt_options *opt, size_t *bytes)
{
    if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
    pt_options d;
    pt_default_options(&d);
    pt_batch tmp;
    const pt_status st = batch_layout(jobs, njobs, opt ? *opt : d, &tmp);
    if (st != PT_OK) return st;
    *bytes = tmp.total;
    return PT_OK;
}

pt_status pt_batch_create(pt_batch **out, const pt_job_desc *jobs, int32_t njobs, const pt_options *opt)
{
    if (!out) return fail(PT_EINVAL, "out is NULL");
    *out = nullptr;
    pt_options d;
    pt_default_options(&d);
    const pt_options &o = opt ? *opt : d;
    pt_batch *b = new (std::nothrow) pt_batch();
    if (!b) return fail(PT_ENOMEM, "host allocation failed");
    auto bail = [&](pt_status st) {
        if (b->own_ws && b->ws) (void)hipFree(b->ws);
        delete b;
        return st;
    };
    pt_status st = batch_layout(jobs, njobs, o, b);
    if (st != PT_OK) return bail(st);
    b->njobs = njobs;
    b->prec = o.precision;
    b->stream = static_cast<hipStream_t>(o.stream);
    if ((st = shape_defaults(o, b->prec, &b->threads, &b->budget)) != PT_OK) return bail(st);
    if (o.lds_budget <= 0) {
        // default budget: raised, in 4 KiB steps up to what the device allows,
        // until the largest job fits with its table in HBM
        int cap = 0, dev = 0;
        hipFuncAttributes fa;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
            hipFuncGetAttributes(&fa, jobs_fn_prec(b->prec)) != hipSuccess)
            return bail(fail(PT_EDEVICE, "device query failed"));
        cap = (cap - static_cast<int>(fa.sharedSizeBytes)) & ~255;
        for (int j = 0; j < njobs; ++j) {
            LdsPlan pl;
            while (b->budget < cap &&
                   !make_plan(jobs[j].L, jobs[j].q, jobs[j].R, b->prec, true, kPlHbm, b->budget, b->threads, &pl))
                b->budget = std::min(cap, b->budget + 4096);
        }
    }
    if (o.workspace) {
        if (o.workspace_bytes < b->total) return bail(fail(PT_ENOMEM, "workspace of %zu B < %zu B", o.workspace_bytes, b->total));
        b->ws = static_cast<unsigned char *>(o.workspace);
        b->ws_bytes = o.workspace_bytes;
    } else {
        if (hipMalloc(&b->ws, b->total) != hipSuccess) return bail(fail(PT_ENOMEM, "hipMalloc(%zu) failed", b->total));
        b->own_ws = true;
        b->ws_bytes = b->total;
    }
    b->d_slots = reinterpret_cast<JobSlot *>(b->ws + b->slots_off);
    b->d_ctl = reinterpret_cast<JobControl *>(b->ws + b->ctl_off);
    b->d_jc = reinterpret_cast<unsigned long long *>(b->ws + b->jc_off);
    b->d_T = reinterpret_cast<double *>(b->ws + b->T_off);
    b->slots.resize(njobs);
    b->jobs.assign(jobs, jobs + njobs);
    // Launch order: the costliest jobs first (tickets go out job by job, so a
    // large job taken last would run alone at the end of the launch).  Cost
    // estimate: attempts, times L / 256 more for direct sums (each attempt an
    // O(L) sum).  Each job's trajectory does not depend on the order.
    std::vector<LdsPlan> plans(njobs);
    std::vector<int32_t> variants(njobs);
    std::vector<double> cost(njobs);
    for (int j = 0; j < njobs; ++j) {
        if ((st = job_plan(jobs[j], b->prec, b->budget, b->threads, &plans[j], &variants[j])) != PT_OK) return bail(st);
        const double att = static_cast<double>(jobs[j].L) * jobs[j].R * static_cast<double>(jobs[j].sweeps);
        cost[j] = plans[j].place == kPlDirect ? att * (1.0 + jobs[j].L / 256.0) : att;
    }
    std::vector<int32_t> order(njobs);
    for (int j = 0; j < njobs; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost[x] > cost[y]; });
    int32_t wbase = 0, maxR = 0;
    size_t toff = 0;
    std::vector<size_t> T_at(njobs);
    for (int j = 0; j < njobs; ++j) {
        T_at[j] = toff;
        b->Tall.insert(b->Tall.end(), jobs[j].T, jobs[j].T + jobs[j].R);
        toff += jobs[j].R;
        b->jobs[j].T = nullptr;
        maxR = std::max(maxR, jobs[j].R);
    }
    b->exec_slots.resize(njobs);
    for (int k = 0; k < njobs; ++k) {
        const int j = order[k];
        job_slot(b->slots[j], jobs[j], b->prec, b->ws + b->job_off[j], b->d_T + T_at[j], plans[j], variants[j], wbase,
                 b->d_jc + kJcWords * static_cast<size_t>(j));
        b->exec_slots[k] = b->slots[j];
        wbase += jobs[j].R;
    }
    int cap = 0;
    if ((st = jobs_capacity(b->prec, b->threads, b->budget, &cap)) != PT_OK) return bail(st);
    if (cap < maxR)
        return bail(fail(PT_EINVAL, "only %d workgroups fit at once but a job has %d replicas", cap, maxR));
    b->grid = std::min(cap, wbase);
    *out = b;
    return PT_OK;
}

pt_status pt_batch_run(pt_batch *b)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    if (b->ran) return fail(PT_ESTATE, "batch already ran");
    pt_status st = zero_async(b->ws, b->slots_off, b->stream);
    if (st == PT_OK) st = zero_async(b->d_ctl, b->T_off - b->ctl_off, b->stream);  // ticket and ready/finished words
    if (st != PT_OK) return st;
    HIPCHK(hipMemcpyAsync(b->d_slots, b->exec_slots.data(), sizeof(JobSlot) * b->njobs, hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipMemcpyAsync(b->d_T, b->Tall.data(), sizeof(double) * b->Tall.size(), hipMemcpyHostToDevice, b->stream));
    const JobSlot *slots = b->d_slots;
    int32_t nstatic = b->njobs;
    const int32_t *pub = nullptr, *stop = nullptr;
    JobControl *ctl = b->d_ctl;
    int32_t *done = nullptr;
    void *args[] = {&slots, &nstatic, &pub, &stop, &ctl, &done};
    HIPCHK(hipLaunchKernel(jobs_fn_prec(b->prec), dim3(b->grid), dim3(b->threads), args, b->budget, b->stream));
    b->ran = true;
    return PT_OK;
}

pt_status pt_batch_observables(pt_batch *b, int32_t job, pt_obs *out)
{
    if (!b || !out) return fail(PT_EINVAL, "null argument");
    if (job < 0 || job >= b->njobs) return fail(PT_EINVAL, "job index out of range");
    HIPCHK(hipStreamSynchronize(b->stream));
    HostObs h;
    const pt_status st = h.fetch(b->slots[job].inst, b->stream);
    if (st != PT_OK) return st;
    if (h.ctr[kCtrError]) return fail(PT_EDEVICE, "job %d reported error bits 0x%llx", job, h.ctr[kCtrError]);
    const int64_t sw = b->ran ? b->jobs[job].sweeps : 0;
    h.fill(out, sw, sw / b->jobs[job].exchange_every, sw);
    return PT_OK;
}

pt_status pt_batch_get_spins(pt_batch *b, int32_t job, uint8_t *spins, int32_t *perm)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    if (job < 0 || job >= b->njobs) return fail(PT_EINVAL, "job index out of range");
    HIPCHK(hipStreamSynchronize(b->stream));
    return fetch_spins(b->slots[job].inst, b->stream, spins, perm);
}

pt_status pt_batch_shape(pt_batch *b, int32_t *wgs, int32_t *threads, int32_t *lds)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    if (wgs) *wgs = b->grid;
    if (threads) *threads = b->threads;
    if (lds) *lds = b->budget;
    return PT_OK;
}

pt_status pt_batch_job_stats(pt_batch *b, int32_t job, int32_t *placement, double *start_s, double *end_s)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    if (job < 0 || job >= b->njobs) return fail(PT_EINVAL, "job index out of range");
    if (placement) *placement = b->slots[job].plan.place;
    if (!start_s && !end_s) return PT_OK;
    if (!b->ran) return fail(PT_ESTATE, "batch has not run");
    HIPCHK(hipStreamSynchronize(b->stream));
    unsigned long long w[kJcWords];
    HIPCHK(hipMemcpy(w, b->d_jc + kJcWords * static_cast<size_t>(job), sizeof w, hipMemcpyDeviceToHost));
    int dev = 0, khz = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    if (khz <= 0) return fail(PT_EDEVICE, "no device wall-clock rate");
    const double per_s = 1e3 * khz;
    if (start_s) *start_s = static_cast<double>(w[2]) / per_s;
    if (end_s) *end_s = static_cast<double>(w[3]) / per_s;
    return PT_OK;
}

pt_status pt_batch_free(pt_batch *b)
{
    if (!b) return fail(PT_EINVAL, "null batch");
    (void)hipStreamSynchronize(b->stream);
    if (b->own_ws && b->ws) (void)hipFree(b->ws);
    delete b;
    return PT_OK;
}

}  // extern "C"

// ===========================================================================
// Server
// ===========================================================================
struct ServerJob {
    pt_job_desc desc{};
    std::vector<double> T;
    int64_t id = 0;
    int32_t slot = -1;          // index in the job table once admitted
    size_t off = 0, bytes = 0;  // arena block
    double t_submit = 0, t_admit = 0, t_done = 0;
    int state = 0;              // 0 queued, 1 running, 2 done, 3 failed, 4 cancelled
    HostObs obs;
    std::vector<uint8_t> spins;
};

struct pt_server {
    int32_t prec = 0, threads = 256, budget = 0, grid = 0, max_jobs = 0;
    size_t arena_bytes = 0;
    unsigned char *mem = nullptr;   // device: arena | control | ready/finished words
    bool own_mem = false;
    size_t ctl_off = 0, jc_off = 0;
    JobControl *d_ctl = nullptr;
    unsigned long long *d_jc = nullptr;  // [max_jobs][kJcWords]
    int32_t *h_ctl = nullptr;       // pinned: [0] published, [1] stop
    int32_t *h_done = nullptr;      // pinned: [max_jobs]
    JobSlot *h_slots = nullptr;     // pinned: [max_jobs] job table read by the running kernel
    double *h_T = nullptr;          // pinned: [max_jobs][64] temperatures
    hipStream_t kstream = nullptr, cstream = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int64_t> queue;
    std::map<int64_t, ServerJob> jobs;
    std::vector<int64_t> running;
    std::map<size_t, size_t> free_blocks;  // offset -> bytes
    int64_t next_id = 0;
    int32_t published = 0;
    int32_t wbase = 0;
    int32_t inflight = 0, inflight_max = 0;  // walkers admitted and not yet finished
    bool quit = false, failed = false;
    std::string fail_msg;
    std::thread th;
    double t0 = 0;
};

namespace {

constexpr int kServerMaxR = 64;

bool arena_alloc(pt_server *s, size_t bytes, size_t *off)
{
    for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
        if (it->second >= bytes) {
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            s->free_blocks.erase(it);
            if (rest) s->free_blocks[at] = rest;
            return true;
        }
    }
    return false;
}

void arena_free(pt_server *s, size_t off, size_t bytes)
{
    auto it = s->free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != s->free_blocks.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        s->free_blocks.erase(nx);
    }
    if (it != s->free_blocks.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            s->free_blocks.erase(it);
        }
    }
}

// Admit the queue's head jobs that fit, in order; publish them.  A job is
// admitted when its state fits in the arena and the walkers admitted and not
// yet finished stay within inflight_max (or none are): the device always has
// published tickets to take, and the rest of the backlog waits on the host,
// where it can still be cancelled.
bool server_admit(pt_server *s)
{
    bool any = false;
    while (!s->queue.empty() && s->published < s->max_jobs) {
        ServerJob &J = s->jobs[s->queue.front()];
        if (s->inflight > 0 && s->inflight + J.desc.R > s->inflight_max) break;
        size_t off = 0;
        if (!arena_alloc(s, J.bytes, &off)) break;  // head-of-line: wait for memory
        s->queue.pop_front();
        J.off = off;
        J.slot = s->published;
        LdsPlan plan;
        int32_t variant = 0;
        job_plan(J.desc, s->prec, s->budget, s->threads, &plan, &variant);
        // the slot and ladder go straight into pinned host memory, before the
        // published count that makes them visible to the kernel
        double *Th = s->h_T + static_cast<size_t>(J.slot) * kServerMaxR;
        std::memcpy(Th, J.T.data(), sizeof(double) * J.desc.R);
        job_slot(s->h_slots[J.slot], J.desc, s->prec, s->mem + off, Th, plan, variant, s->wbase,
                 s->d_jc + kJcWords * static_cast<size_t>(J.slot));
        s->wbase += J.desc.R;
        s->inflight += J.desc.R;
        s->published += 1;
        J.state = 1;
        J.t_admit = now_s() - s->t0;
        s->running.push_back(J.id);
        __atomic_store_n(&s->h_ctl[0], s->published, __ATOMIC_RELEASE);
        any = true;
    }
    return any;
}

// Collect jobs whose last walker has finished.
bool server_collect(pt_server *s, std::unique_lock<std::mutex> &lk)
{
    bool any = false;
    for (size_t k = 0; k < s->running.size();) {
        ServerJob &J = s->jobs[s->running[k]];
        if (__atomic_load_n(&s->h_done[J.slot], __ATOMIC_ACQUIRE) == 0) {
            ++k;
            continue;
        }
        JobSlot S;
        const Layout lay = layout_of(J.desc.L, J.desc.q, J.desc.R, s->prec, 0, kJobEvents);
        fill_inst(S.inst, s->mem + J.off, lay, J.desc.L, J.desc.q, J.desc.R, J.desc.seed, 0, 0, kJobEvents);
        lk.unlock();
        J.spins.resize(static_cast<size_t>(J.desc.R) * J.desc.L);
        const bool ok = J.obs.fetch(S.inst, s->cstream) == PT_OK &&
                        hipMemcpyAsync(J.spins.data(), S.inst.spins, J.spins.size(), hipMemcpyDeviceToHost,
                                       s->cstream) == hipSuccess &&
                        hipStreamSynchronize(s->cstream) == hipSuccess;
        lk.lock();
        J.t_done = now_s() - s->t0;
        J.state = ok && J.obs.ctr[kCtrError] == 0 ? 2 : 3;
        arena_free(s, J.off, J.bytes);
        s->inflight -= J.desc.R;
        s->running.erase(s->running.begin() + static_cast<long>(k));
        any = true;
    }
    return any;
}

void server_loop(pt_server *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    while (!s->failed) {
        const bool a = server_admit(s);
        const bool c = server_collect(s, lk);
        if (a || c) s->cv.notify_all();
        if (s->quit && s->queue.empty() && s->running.empty()) break;
        s->cv.wait_for(lk, std::chrono::microseconds(200));
    }
    s->cv.notify_all();
}

}  // namespace

extern "C" {

pt_status pt_server_start(pt_server **out, size_t arena_bytes, int32_t max_jobs, const pt_options *opt)
{
    if (!out) return fail(PT_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_jobs < 1 || arena_bytes < 4096) return fail(PT_EINVAL, "bad arena size or job count");
    pt_options d;
    pt_default_options(&d);
    const pt_options &o = opt ? *opt : d;
    if (!valid_prec(o.precision)) return fail(PT_EINVAL, "bad precision");
    pt_server *s = new (std::nothrow) pt_server();
    if (!s) return fail(PT_ENOMEM, "host allocation failed");
    auto bail = [&](pt_status st) {
        if (s->kstream) (void)hipStreamDestroy(s->kstream);
        if (s->cstream) (void)hipStreamDestroy(s->cstream);
        if (s->own_mem && s->mem) (void)hipFree(s->mem);
        if (s->h_ctl) (void)hipHostFree(s->h_ctl);
        if (s->h_done) (void)hipHostFree(s->h_done);
        if (s->h_slots) (void)hipHostFree(s->h_slots);
        if (s->h_T) (void)hipHostFree(s->h_T);
        delete s;
        return st;
    };
    s->prec = o.precision;
    s->max_jobs = max_jobs;
    pt_status st0 = shape_defaults(o, s->prec, &s->threads, &s->budget);
    if (st0 != PT_OK) return bail(st0);
    s->arena_bytes = Layout::up(arena_bytes);
    s->ctl_off = s->arena_bytes;
    s->jc_off = s->ctl_off + Layout::up(sizeof(JobControl));
    const size_t total = server_bytes(arena_bytes, max_jobs);
    if (o.workspace) {
        if (o.workspace_bytes < total) return bail(fail(PT_ENOMEM, "workspace of %zu B < %zu B", o.workspace_bytes, total));
        s->mem = static_cast<unsigned char *>(o.workspace);
    } else {
        if (hipMalloc(&s->mem, total) != hipSuccess) return bail(fail(PT_ENOMEM, "hipMalloc(%zu) failed", total));
        s->own_mem = true;
    }
    s->d_ctl = reinterpret_cast<JobControl *>(s->mem + s->ctl_off);
    s->d_jc = reinterpret_cast<unsigned long long *>(s->mem + s->jc_off);
    // The running kernel polls these words and reads the job table while the
    // host writes them, so they must be coherent during the launch: default
    // pinned memory (coherent only at dispatch boundaries unless the
    // HIP_HOST_COHERENT environment variable says otherwise) may serve the
    // device stale lines.
    constexpr unsigned kCoh = hipHostMallocCoherent;
    if (hipHostMalloc(&s->h_ctl, 256, kCoh) != hipSuccess ||
        hipHostMalloc(&s->h_done, sizeof(int32_t) * max_jobs, kCoh) != hipSuccess ||
        hipHostMalloc(&s->h_slots, sizeof(JobSlot) * max_jobs, kCoh) != hipSuccess ||
        hipHostMalloc(&s->h_T, sizeof(double) * kServerMaxR * max_jobs, kCoh) != hipSuccess)
        return bail(fail(PT_ENOMEM, "pinned host allocation failed"));
    std::memset(s->h_ctl, 0, 256);
    std::memset(s->h_done, 0, sizeof(int32_t) * max_jobs);
    std::memset(static_cast<void *>(s->h_slots), 0, sizeof(JobSlot) * max_jobs);
    if (hipStreamCreateWithFlags(&s->kstream, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&s->cstream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(PT_EDEVICE, "stream creation failed"));
    int cap = 0;
    pt_status st = jobs_capacity(s->prec, s->threads, s->budget, &cap);
    if (st != PT_OK) return bail(st);
    if (cap < kServerMaxR) return bail(fail(PT_EINVAL, "only %d workgroups fit at once (need %d)", cap, kServerMaxR));
    s->grid = cap;
    s->inflight_max = 2 * cap;
    s->free_blocks[0] = s->arena_bytes;
    // ticket and every slot's ready/finished words start at zero with the launch
    if (zero_async(s->d_ctl, total - s->ctl_off, s->kstream) != PT_OK) return bail(PT_EDEVICE);
    const JobSlot *slots = s->h_slots;
    int32_t nstatic = -1;
    const int32_t *pub = s->h_ctl, *stop = s->h_ctl + 1;
    JobControl *ctl = s->d_ctl;
    int32_t *done = s->h_done;
    void *args[] = {&slots, &nstatic, &pub, &stop, &ctl, &done};
    if (hipLaunchKernel(jobs_fn_prec(s->prec), dim3(s->grid), dim3(s->threads), args, s->budget, s->kstream) !=
        hipSuccess)
        return bail(fail(PT_EDEVICE, "server launch failed"));
    s->t0 = now_s();
    s->th = std::thread(server_loop, s);
    *out = s;
    return PT_OK;
}

pt_status pt_server_workspace_size(size_t arena_bytes, int32_t max_jobs, size_t *bytes)
{
    if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
    if (max_jobs < 1) return fail(PT_EINVAL, "max_jobs must be >= 1");
    *bytes = server_bytes(arena_bytes, max_jobs);
    return PT_OK;
}

pt_status pt_server_submit(pt_server *s, const pt_job_desc *job, int64_t *id_out)
{
    if (!s || !job) return fail(PT_EINVAL, "null argument");
    pt_status st = validate_job(*job);
    if (st != PT_OK) return st;
    if (job->R > kServerMaxR) return fail(PT_EINVAL, "server jobs have at most %d replicas", kServerMaxR);
    LdsPlan plan;
    int32_t variant = 0;
    if ((st = job_plan(*job, s->prec, s->budget, s->threads, &plan, &variant)) != PT_OK) return st;
    const size_t bytes = job_bytes(*job, s->prec);
    if (bytes > s->arena_bytes) return fail(PT_ENOMEM, "job needs %zu B, arena has %zu B", bytes, s->arena_bytes);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->failed) return fail(PT_EDEVICE, "server failed: %s", s->fail_msg.c_str());
    if (s->quit) return fail(PT_ESTATE, "server is stopping");
    if (s->next_id >= s->max_jobs) return fail(PT_ENOMEM, "server job table full (%d jobs)", s->max_jobs);
    ServerJob J;
    J.desc = *job;
    J.T.assign(job->T, job->T + job->R);
    J.desc.T = nullptr;
    J.id = s->next_id++;
    J.bytes = bytes;
    J.t_submit = now_s() - s->t0;
    s->jobs[J.id] = std::move(J);
    s->queue.push_back(s->next_id - 1);
    if (id_out) *id_out = s->next_id - 1;
    s->cv.notify_all();
    return PT_OK;
}

static pt_status server_result(pt_server *s, const ServerJob &J, pt_obs *out)
{
    if (J.state == 3) return fail(PT_EDEVICE, "job %lld failed on the device", static_cast<long long>(J.id));
    if (J.state == 4) return fail(PT_ESTATE, "job %lld was cancelled", static_cast<long long>(J.id));
    if (out) J.obs.fill(out, J.desc.sweeps, J.desc.sweeps / J.desc.exchange_every, J.desc.sweeps);
    (void)s;
    return PT_OK;
}

pt_status pt_server_poll(pt_server *s, int64_t id, int32_t *done, pt_obs *out)
{
    if (!s) return fail(PT_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(PT_EINVAL, "unknown job id");
    const bool fin = it->second.state >= 2;
    if (done) *done = fin ? 1 : 0;  // cancelled jobs count as ended (and report PT_ESTATE)
    if (fin) return server_result(s, it->second, out);
    return PT_OK;
}

pt_status pt_server_wait(pt_server *s, int64_t id, double timeout_s, pt_obs *out)
{
    if (!s) return fail(PT_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(PT_EINVAL, "unknown job id");
    const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (it->second.state < 2) {
        if (s->failed) return fail(PT_EDEVICE, "server failed: %s", s->fail_msg.c_str());
        if (s->cv.wait_until(lk, until) == std::cv_status::timeout && it->second.state < 2)
            return fail(PT_ESTATE, "job %lld not finished after %.1f s", static_cast<long long>(id), timeout_s);
    }
    return server_result(s, it->second, out);
}

pt_status pt_server_cancel(pt_server *s, int64_t id)
{
    if (!s) return fail(PT_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(PT_EINVAL, "unknown job id");
    ServerJob &J = it->second;
    if (J.state == 4) return PT_OK;
    if (J.state != 0) return fail(PT_ESTATE, "job %lld was already admitted", static_cast<long long>(id));
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
        if (*q == id) {
            s->queue.erase(q);
            break;
        }
    J.state = 4;
    J.t_done = now_s() - s->t0;
    s->cv.notify_all();
    return PT_OK;
}

pt_status pt_server_times(pt_server *s, int64_t id, double *sub, double *adm, double *fin)
{
    if (!s) return fail(PT_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(PT_EINVAL, "unknown job id");
    if (sub) *sub = it->second.t_submit;
    if (adm) *adm = it->second.t_admit;
    if (fin) *fin = it->second.t_done;
    return PT_OK;
}

pt_status pt_server_get_spins(pt_server *s, int64_t id, uint8_t *spins, int32_t *perm)
{
    if (!s) return fail(PT_EINVAL, "null server");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return fail(PT_EINVAL, "unknown job id");
    const ServerJob &J = it->second;
    if (J.state != 2) return fail(PT_ESTATE, "job not finished");
    if (spins)
        for (size_t e = 0; e < J.spins.size(); ++e) spins[e] = static_cast<uint8_t>(J.spins[e] + 1);
    if (perm) std::memcpy(perm, J.obs.perm.data(), sizeof(int32_t) * J.desc.R);
    return PT_OK;
}

pt_status pt_server_stop(pt_server *s)
{
    if (!s) return fail(PT_EINVAL, "null server");
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->quit = true;
        s->cv.notify_all();
    }
    if (s->th.joinable()) s->th.join();
    __atomic_store_n(&s->h_ctl[1], 1, __ATOMIC_RELEASE);
    const hipError_t e = hipStreamSynchronize(s->kstream);
    const bool failed = s->failed;
    (void)hipStreamDestroy(s->kstream);
    (void)hipStreamDestroy(s->cstream);
    if (s->own_mem && s->mem) (void)hipFree(s->mem);
    (void)hipHostFree(s->h_ctl);
    (void)hipHostFree(s->h_done);
    (void)hipHostFree(s->h_slots);
    (void)hipHostFree(s->h_T);
    delete s;
    if (e != hipSuccess) return fail(PT_EDEVICE, "server kernel: %s", hipGetErrorString(e));
    if (failed) return fail(PT_EDEVICE, "server failed");
    return PT_OK;
}

}  // extern "C"
