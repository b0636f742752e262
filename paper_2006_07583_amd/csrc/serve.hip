// Served form of the library (include/adi.h, adi_server_*): requests with
// host arrays arrive at any time; a scheduler thread advances every active
// problem by one step per tick with grouped launches (one grid per kernel
// variant and half-step, as in batch.hip) while an upload thread admits and
// uploads requests and a download thread returns finished ones, each on a
// stream of its own.
//
// Device memory comes from an arena of hbm_budget_bytes allocated once at
// creation: admission is first come, first served, as soon as the request's
// arrays and workspace fit; nothing is allocated or freed on the device
// while serving.  Results are written back into the request's host arrays,
// or held in the arena until adi_fetch (ADI_REQUEST_HOLD).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/adi.h"
#include "admission.h"
#include "line_pass.h"
#include "problem.h"

namespace {

using adi::fail;
using adi::hip_fail;

using adi::Arena;

enum { ST_QUEUED = 0, ST_RUNNING = 1, ST_DONE = 2 };

struct Req {
    uint64_t ticket = 0;
    adi_request r{};
    int64_t ld[6] = {};
    size_t arr_off[6] = {};   // arena offsets of U, V, W, K, Rv, Rw (relative to off)
    size_t ws_off = 0;
    size_t bytes = 0, off = 0;
    adi_problem* pb = nullptr;
    int64_t s = 0;
    int state = ST_QUEUED;
    int status = ADI_OK;
    bool held = false;       // result kept in the arena until adi_fetch
    bool fetching = false;
    double t_submit = 0, t_start = 0, t_done = 0;
    hipEvent_t ev = nullptr;
};

// rows x cols of the six arrays of a problem
void array_shapes(const adi_params& p, int64_t rows[6], int64_t cols[6]) {
    const bool cfd = p.method == ADI_CFD;
    const int64_t ru = cfd ? p.ny + 1 : p.ny + 2, cu = cfd ? p.nx + 1 : p.nx + 2;
    const int64_t rv = cfd ? p.ny + 1 : p.ny + 2, cv = p.nx + 1;
    const int64_t rw = p.ny + 1, cw = cfd ? p.nx + 1 : p.nx + 2;
    const int64_t r[6] = {ru, rv, rw, ru, rv, rw}, c[6] = {cu, cv, cw, cu, cv, cw};
    for (int i = 0; i < 6; ++i) {
        rows[i] = r[i];
        cols[i] = c[i];
    }
}

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Descriptor staging of one tick: host (pinned) and device copies.
struct Slot {
    char* host = nullptr;
    char* dev = nullptr;
    hipEvent_t ev = nullptr;
    bool used = false;
};

}  // namespace

struct adi_server {
    adi_server_params prm{};
    int dev = 0;
    // compute stream; two upload and two download threads, each with a
    // stream of its own: the runtime maps streams onto a few hardware
    // queues, and an upload or download stream that shares the compute
    // stream's queue waits behind its ticks (one such upload took 8.8 ms
    // instead of 2 ms); with two of each, work goes on while one waits
    static constexpr int kUp = 2, kDown = 2;
    hipStream_t cs = nullptr, us[kUp] = {}, ds[kDown] = {};
    char* mem = nullptr;
    Arena arena;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req*> pending;
    std::vector<Req*> ready, active;
    std::deque<Req*> finishing;
    std::unordered_map<uint64_t, Req*> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    bool sched_done = false;
    int fatal = ADI_OK;
    int64_t admitted = 0;   // admitted and not yet done (bounded by max_active)
    std::thread sched, up[kUp], down[kDown];
    // tick staging
    static constexpr int NSLOT = 4;
    Slot slot[NSLOT];
    size_t slot_bytes = 0;
    int cur_slot = 0;
    int* dzero = nullptr;
    // statistics
    int64_t ticks = 0, done = 0, peak_active = 0, launches = 0;
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Append the grouped items of one dtype and half to the staging buffer and
// launch them.
template <typename T>
int stage_and_launch(adi_server* S, std::vector<adi::PassDesc<T>>& v, char* host, char* dev, size_t& used) {
    if (v.empty()) return ADI_OK;
    std::stable_sort(v.begin(), v.end(),
                     [](const adi::PassDesc<T>& x, const adi::PassDesc<T>& y) { return x.key() < y.key(); });
    size_t i = 0;
    while (i < v.size()) {
        size_t j = i;
        while (j < v.size() && v[j].key() == v[i].key()) ++j;
        const size_t cnt = j - i;
        const size_t ib = align256(cnt * sizeof(adi::LinePassArgs<T>)), sb = align256((cnt + 1) * sizeof(int));
        if (used + ib + sb > S->slot_bytes) return fail(ADI_EINVAL, "tick descriptors exceed the staging buffer");
        auto* items = (adi::LinePassArgs<T>*)(host + used);
        int* starts = (int*)(host + used + ib);
        int tot = 0;
        for (size_t k = 0; k < cnt; ++k) {
            items[k] = v[i + k].a;
            starts[k] = tot;
            tot += v[i + k].tiles();
        }
        starts[cnt] = tot;
        adi::GroupArgs<T> ga;
        ga.items = (const adi::LinePassArgs<T>*)(dev + used);
        ga.starts = (const int*)(dev + used + ib);
        ga.tick = S->dzero;
        ga.nitems = (int)cnt;
        ga.total = tot;
        used += ib + sb;
        // the copy of everything staged so far precedes the launch
        HIP_TRY(hipMemcpyAsync(dev + used - ib - sb, host + used - ib - sb, ib + sb, hipMemcpyHostToDevice, S->cs),
                "descriptor upload");
        HIP_TRY(adi::launch_grouped<T>(v[i], ga, S->cs), "grouped line pass");
        ++S->launches;
        i = j;
    }
    return ADI_OK;
}

int tick(adi_server* S) {
    Slot& sl = S->slot[S->cur_slot];
    S->cur_slot = (S->cur_slot + 1) % adi_server::NSLOT;
    if (sl.used) HIP_TRY(hipEventSynchronize(sl.ev), "hipEventSynchronize");
    size_t used = 0;
    for (int h = 0; h < 2; ++h) {
        std::vector<adi::PassDesc<float>> vf;
        std::vector<adi::PassDesc<double>> vd;
        for (Req* r : S->active) {
            if (r->pb->p.dtype == ADI_FP64)
                vd.push_back(adi::run_pass<double>(r->pb, r->s, h, h == 1 && r->s == r->r.nsteps - 1, nullptr));
            else
                vf.push_back(adi::run_pass<float>(r->pb, r->s, h, h == 1 && r->s == r->r.nsteps - 1, nullptr));
        }
        int rc = stage_and_launch<float>(S, vf, sl.host, sl.dev, used);
        if (rc == ADI_OK) rc = stage_and_launch<double>(S, vd, sl.host, sl.dev, used);
        if (rc != ADI_OK) return rc;
    }
    HIP_TRY(hipEventRecord(sl.ev, S->cs), "hipEventRecord");
    sl.used = true;
    ++S->ticks;
    return ADI_OK;
}

void fail_all(adi_server* S, int code) {
    // caller holds the lock
    S->fatal = code;
    for (auto& kv : S->all)
        if (kv.second->state != ST_DONE) {
            kv.second->state = ST_DONE;
            kv.second->status = code;
        }
    S->cv.notify_all();
}

void scheduler(adi_server* S) {
    (void)hipSetDevice(S->dev);
    for (;;) {
        std::vector<Req*> joining;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // leave only when stopping and nothing is pending, uploading,
            // running or downloading
            const auto drained = [&] { return S->stop && S->pending.empty() && S->admitted == 0; };
            S->cv.wait(lk, [&] { return S->fatal || !S->ready.empty() || !S->active.empty() || drained(); });
            if (S->fatal || (S->ready.empty() && S->active.empty())) {
                S->sched_done = true;
                S->cv.notify_all();
                return;
            }
            joining.swap(S->ready);
        }
        int rc = ADI_OK;
        std::vector<Req*> started;
        for (Req* r : joining) {
            rc = r->pb->p.dtype == ADI_FP64 ? adi::run_begin<double>(r->pb, S->cs) : adi::run_begin<float>(r->pb, S->cs);
            if (rc != ADI_OK) break;
            r->s = 0;
            started.push_back(r);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Req* r : started) {
                r->state = ST_RUNNING;
                r->t_start = now_s(S->t0);
                S->active.push_back(r);
            }
        }
        if (rc == ADI_OK && !S->active.empty()) rc = tick(S);
        std::vector<Req*> fin, keep;
        if (rc == ADI_OK) {
            for (Req* r : S->active) {
                if (++r->s == r->r.nsteps) {
                    rc = r->pb->p.dtype == ADI_FP64 ? adi::run_end<double>(r->pb, S->cs, r->r.nsteps)
                                                    : adi::run_end<float>(r->pb, S->cs, r->r.nsteps);
                    if (rc != ADI_OK) break;
                    hipError_t e = hipEventRecord(r->ev, S->cs);
                    if (e != hipSuccess) {
                        rc = hip_fail(e, "hipEventRecord");
                        break;
                    }
                    fin.push_back(r);
                } else {
                    keep.push_back(r);
                }
            }
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (rc != ADI_OK) {
            fail_all(S, rc);
            S->sched_done = true;
            return;
        }
        S->peak_active = std::max<int64_t>(S->peak_active, (int64_t)S->active.size());
        S->active.swap(keep);
        for (Req* r : fin) S->finishing.push_back(r);
        if (!fin.empty()) S->cv.notify_all();
    }
}

// Upload one admitted request and bind its problem (upload stream).
int start_request(adi_server* S, Req* r, hipStream_t us) {
    const adi_params& p = r->r.params;
    const size_t esz = p.dtype == ADI_FP64 ? 8 : 4;
    int64_t rows[6], cols[6];
    array_shapes(p, rows, cols);
    const void* src[6] = {r->r.U, r->r.V, r->r.W, r->r.K, r->r.Rv, r->r.Rw};
    void* dptr[6] = {};
    for (int i = 0; i < 6; ++i) {
        if (!src[i]) continue;
        dptr[i] = S->mem + r->off + r->arr_off[i];
        HIP_TRY(hipMemcpy2DAsync(dptr[i], cols[i] * esz, src[i], r->ld[i] * esz, cols[i] * esz, rows[i],
                                 hipMemcpyHostToDevice, us), "request upload");
    }
    // no wait here: the problem's bind work is queued on the same stream,
    // after the copies, and waits for the stream once (its material check).
    // Each wait on this stream can sit behind compute work when the runtime
    // maps it onto the compute stream's hardware queue.
    int rc = adi_create(&p, us, &r->pb);
    if (rc != ADI_OK) return rc;
    const int64_t ld0[6] = {0, 0, 0, 0, 0, 0};
    rc = adi_bind(r->pb, dptr[0], dptr[1], dptr[2], dptr[3], dptr[4], dptr[5], ld0, S->mem + r->off + r->ws_off,
                  r->bytes - r->ws_off);
    if (rc != ADI_OK) return rc;
    return adi_set_step(r->pb, 0);
}

// Copy the results of a finished request back into its host arrays (held
// requests only wait for their last step).
int finish_request(adi_server* S, Req* r, hipStream_t ds) {
    HIP_TRY(hipEventSynchronize(r->ev), "hipEventSynchronize");
    if (r->r.flags & ADI_REQUEST_HOLD) return ADI_OK;
    const adi_params& p = r->r.params;
    const size_t esz = p.dtype == ADI_FP64 ? 8 : 4;
    int64_t rows[6], cols[6];
    array_shapes(p, rows, cols);
    void* dst[3] = {r->r.U, r->r.V, r->r.W};
    for (int i = 0; i < 3; ++i)
        HIP_TRY(hipMemcpy2DAsync(dst[i], r->ld[i] * esz, S->mem + r->off + r->arr_off[i], cols[i] * esz,
                                 cols[i] * esz, rows[i], hipMemcpyDeviceToHost, ds), "result download");
    HIP_TRY(hipStreamSynchronize(ds), "hipStreamSynchronize");
    return ADI_OK;
}

// Admission and uploads, oldest request first.
void uploader(adi_server* S, int k) {
    (void)hipSetDevice(S->dev);
    for (;;) {
        Req* adm = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // reserves arena memory for the oldest pending request when it fits
            auto admissible = [&] { return adi::admissible(S->pending, S->admitted, S->prm.max_active, S->arena); };
            S->cv.wait(lk, [&] { return S->fatal || admissible() || (S->stop && S->pending.empty()); });
            if (S->fatal || !admissible()) return;
            adm = S->pending.front();
            S->pending.pop_front();
            ++S->admitted;
        }
        const int rc = start_request(S, adm, S->us[k]);
        std::lock_guard<std::mutex> lk(S->mu);
        if (rc != ADI_OK) {
            // this request fails alone; its memory goes back
            if (adm->pb) adi_destroy(adm->pb);
            adm->pb = nullptr;
            S->arena.release(adm->off, adm->bytes);
            adm->state = ST_DONE;
            adm->status = rc;
            adm->t_done = now_s(S->t0);
            --S->admitted;
            S->cv.notify_all();
            continue;
        }
        S->ready.push_back(adm);
        S->cv.notify_all();
    }
}

// Downloads of finished requests, in completion order.
void downloader(adi_server* S, int k) {
    (void)hipSetDevice(S->dev);
    for (;;) {
        Req* fin = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->fatal || !S->finishing.empty() || S->sched_done; });
            if (S->fatal) return;
            if (S->finishing.empty()) return;   // scheduler done and nothing left
            fin = S->finishing.front();
            S->finishing.pop_front();
        }
        const int rc = finish_request(S, fin, S->ds[k]);
        std::lock_guard<std::mutex> lk(S->mu);
        if (rc != ADI_OK) {
            fail_all(S, rc);
            return;
        }
        adi_destroy(fin->pb);
        fin->pb = nullptr;
        if (fin->r.flags & ADI_REQUEST_HOLD)
            fin->held = true;
        else
            S->arena.release(fin->off, fin->bytes);
        fin->state = ST_DONE;
        fin->t_done = now_s(S->t0);
        ++S->done;
        --S->admitted;
        S->cv.notify_all();
    }
}

void release_server(adi_server* S) {
    (void)hipSetDevice(S->dev);
    if (S->cs) (void)hipStreamSynchronize(S->cs);
    for (auto st : S->us)
        if (st) (void)hipStreamSynchronize(st);
    for (auto st : S->ds)
        if (st) (void)hipStreamSynchronize(st);
    for (auto& kv : S->all) {
        Req* r = kv.second;
        if (r->pb) adi_destroy(r->pb);
        if (r->ev) (void)hipEventDestroy(r->ev);
        delete r;
    }
    for (auto& sl : S->slot) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.host) (void)hipHostFree(sl.host);
        if (sl.dev) (void)hipFree(sl.dev);
    }
    if (S->dzero) (void)hipFree(S->dzero);
    if (S->mem) (void)hipFree(S->mem);
    if (S->cs) (void)hipStreamDestroy(S->cs);
    for (auto st : S->us)
        if (st) (void)hipStreamDestroy(st);
    for (auto st : S->ds)
        if (st) (void)hipStreamDestroy(st);
    delete S;
}

}  // namespace

extern "C" {

int adi_server_params_init(adi_server_params* p) {
    if (!p) return fail(ADI_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(adi_server_params);
    p->hbm_budget_bytes = (uint64_t)16 << 30;
    p->max_active = 256;
    return ADI_OK;
}

int adi_server_create(const adi_server_params* p, adi_server** out) {
    if (!out) return fail(ADI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || p->struct_size != sizeof(adi_server_params)) return fail(ADI_EINVAL, "bad adi_server_params");
    if (p->hbm_budget_bytes < ((uint64_t)1 << 20)) return fail(ADI_EINVAL, "hbm_budget_bytes below 1 MiB");
    if (p->max_active < 1 || p->max_active > 4096) return fail(ADI_EINVAL, "max_active must be in [1, 4096]");
    adi_server* S = new (std::nothrow) adi_server();
    if (!S) return fail(ADI_ENOMEM, "host allocation failed");
    S->prm = *p;
    S->t0 = std::chrono::steady_clock::now();
    hipError_t e = hipGetDevice(&S->dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&S->cs, hipStreamNonBlocking);
    for (int k = 0; k < adi_server::kUp && e == hipSuccess; ++k)
        e = hipStreamCreateWithFlags(&S->us[k], hipStreamNonBlocking);
    for (int k = 0; k < adi_server::kDown && e == hipSuccess; ++k)
        e = hipStreamCreateWithFlags(&S->ds[k], hipStreamNonBlocking);
    if (e != hipSuccess) {
        release_server(S);
        return hip_fail(e, "server streams");
    }
    void* m = nullptr;
    e = hipMalloc(&m, p->hbm_budget_bytes);
    if (e != hipSuccess) {
        release_server(S);
        return fail(ADI_ENOMEM, "arena of %llu bytes: %s", (unsigned long long)p->hbm_budget_bytes,
                    hipGetErrorString(e));
    }
    S->mem = (char*)m;
    S->arena.reset(p->hbm_budget_bytes);
    // per tick: both halves of every active problem, grouped (prefix sums included)
    S->slot_bytes = align256((size_t)2 * p->max_active * (sizeof(adi::LinePassArgs<double>) + 2 * sizeof(int) + 512) + 65536);
    for (auto& sl : S->slot) {
        e = hipHostMalloc((void**)&sl.host, S->slot_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&sl.dev, S->slot_bytes);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_server(S);
            return hip_fail(e, "tick staging");
        }
    }
    e = hipMalloc((void**)&S->dzero, 256);
    if (e == hipSuccess) e = hipMemsetAsync(S->dzero, 0, 256, S->cs);
    if (e == hipSuccess) e = hipStreamSynchronize(S->cs);
    if (e != hipSuccess) {
        release_server(S);
        return hip_fail(e, "server set-up");
    }
    S->sched = std::thread(scheduler, S);
    for (int k = 0; k < adi_server::kUp; ++k) S->up[k] = std::thread(uploader, S, k);
    for (int k = 0; k < adi_server::kDown; ++k) S->down[k] = std::thread(downloader, S, k);
    *out = S;
    return ADI_OK;
}

int adi_submit(adi_server* S, const adi_request* rq, uint64_t* ticket) {
    if (!S || !rq || !ticket) return fail(ADI_EINVAL, "NULL argument");
    if (rq->struct_size != sizeof(adi_request)) return fail(ADI_EINVAL, "bad adi_request struct_size");
    if (!rq->U || !rq->V || !rq->W) return fail(ADI_EINVAL, "U, V and W are required");
    if (rq->nsteps < 1) return fail(ADI_EINVAL, "nsteps must be >= 1");
    if (rq->params.sweeps == 0) return fail(ADI_EINVAL, "direct solves (sweeps 0) are not served");
    if (rq->flags & ~ADI_REQUEST_HOLD) return fail(ADI_EINVAL, "unknown request flags 0x%x", rq->flags);
    size_t ws = 0;
    int rc = adi_workspace_size(&rq->params, rq->K != nullptr, rq->Rv != nullptr, rq->Rw != nullptr, &ws);
    if (rc != ADI_OK) return rc;
    Req* r = new (std::nothrow) Req();
    if (!r) return fail(ADI_ENOMEM, "host allocation failed");
    r->r = *rq;
    int64_t rows[6], cols[6];
    array_shapes(rq->params, rows, cols);
    const size_t esz = rq->params.dtype == ADI_FP64 ? 8 : 4;
    const void* src[6] = {rq->U, rq->V, rq->W, rq->K, rq->Rv, rq->Rw};
    size_t cur = 0;
    for (int i = 0; i < 6; ++i) {
        r->ld[i] = rq->ld[i] ? rq->ld[i] : cols[i];
        if (r->ld[i] < cols[i]) {
            delete r;
            return fail(ADI_EINVAL, "ld[%d] below the row length", i);
        }
        r->arr_off[i] = cur;
        if (src[i]) cur += align256((size_t)rows[i] * cols[i] * esz);
    }
    r->ws_off = cur;
    r->bytes = cur + ws;
    if (r->bytes > S->prm.hbm_budget_bytes) {
        delete r;
        return fail(ADI_EINVAL, "request needs %zu bytes, more than the whole budget", (size_t)(cur + ws));
    }
    hipError_t e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete r;
        return hip_fail(e, "hipEventCreate");
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fatal) {
        (void)hipEventDestroy(r->ev);
        delete r;
        return fail(S->fatal, "server stopped after an error");
    }
    r->ticket = S->next_ticket++;
    r->off = (size_t)-1;
    r->t_submit = now_s(S->t0);
    S->all[r->ticket] = r;
    S->pending.push_back(r);
    *ticket = r->ticket;
    S->cv.notify_all();
    return ADI_OK;
}

int adi_poll(adi_server* S, uint64_t ticket, int* state) {
    if (!S || !state) return fail(ADI_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(ADI_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    *state = it->second->state;
    return it->second->state == ST_DONE ? it->second->status : ADI_OK;
}

int adi_wait(adi_server* S, uint64_t ticket) {
    if (!S) return fail(ADI_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(ADI_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Req* r = it->second;
    S->cv.wait(lk, [&] { return r->state == ST_DONE; });
    return r->status == ADI_OK ? ADI_OK : fail(r->status, "request failed");
}

int adi_fetch(adi_server* S, uint64_t ticket, void* U, void* V, void* W) {
    if (!S) return fail(ADI_EINVAL, "server is NULL");
    Req* r = nullptr;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return fail(ADI_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
        r = it->second;
        S->cv.wait(lk, [&] { return r->state == ST_DONE; });
        if (r->status != ADI_OK) return fail(r->status, "request failed");
        if (r->r.flags & ADI_REQUEST_HOLD) {
            if (!r->held || r->fetching) return fail(ADI_EINVAL, "result of ticket %llu already fetched",
                                                     (unsigned long long)ticket);
            r->fetching = true;   // this thread copies; the arena block stays reserved
        }
    }
    const adi_params& p = r->r.params;
    const size_t esz = p.dtype == ADI_FP64 ? 8 : 4;
    int64_t rows[6], cols[6];
    array_shapes(p, rows, cols);
    void* dst[3] = {U, V, W};
    const void* hsrc[3] = {r->r.U, r->r.V, r->r.W};
    int rc = ADI_OK;
    for (int i = 0; i < 3 && rc == ADI_OK; ++i) {
        if (!dst[i]) continue;
        if (r->held) {
            const hipError_t e = hipMemcpy2D(dst[i], r->ld[i] * esz, S->mem + r->off + r->arr_off[i], cols[i] * esz,
                                             cols[i] * esz, rows[i], hipMemcpyDeviceToHost);
            if (e != hipSuccess) rc = hip_fail(e, "result download");
        } else if (dst[i] != hsrc[i]) {
            for (int64_t j = 0; j < rows[i]; ++j)
                std::memcpy((char*)dst[i] + j * r->ld[i] * esz, (const char*)hsrc[i] + j * r->ld[i] * esz,
                            cols[i] * esz);
        }
    }
    if (r->held) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->arena.release(r->off, r->bytes);
        r->held = false;
        S->cv.notify_all();
    }
    return rc;
}

int adi_request_times(adi_server* S, uint64_t ticket, double* t_submit, double* t_start, double* t_done) {
    if (!S) return fail(ADI_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(ADI_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (t_submit) *t_submit = it->second->t_submit;
    if (t_start) *t_start = it->second->t_start;
    if (t_done) *t_done = it->second->t_done;
    return ADI_OK;
}

int adi_server_get_stats(adi_server* S, adi_server_stats* st) {
    if (!S || !st) return fail(ADI_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->queued = (int64_t)S->pending.size();
    st->active = (int64_t)(S->active.size() + S->ready.size());
    st->done = S->done;
    st->peak_active = S->peak_active;
    st->ticks = S->ticks;
    st->launches = S->launches;
    st->arena_used = S->arena.used();
    return ADI_OK;
}

int adi_server_destroy(adi_server* S) {
    if (!S) return ADI_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    // the uploader leaves once nothing is pending, the scheduler once nothing
    // is pending, uploading, running or downloading, the downloader after the
    // last download
    if (S->sched.joinable()) S->sched.join();
    for (auto& t : S->up)
        if (t.joinable()) t.join();
    for (auto& t : S->down)
        if (t.joinable()) t.join();
    release_server(S);
    return ADI_OK;
}

}  // extern "C"
