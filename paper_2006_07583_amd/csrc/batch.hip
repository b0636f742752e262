// Batched runs: many independent problems advanced in lockstep, with one
// grouped launch per kernel variant and half-step (include/adi.h,
// adi_batch_*).
//
// Every step of every problem is two line passes (run_pass half 0 and 1).
// Within a batch the passes of one half-step are independent, so they are
// collected across problems, sorted by kernel variant (tile shape, method,
// mode) and issued as one grid per variant; each workgroup finds its pass
// by a binary search over the prefix sums of the block counts.  The pass
// descriptors depend on the step only through the ping-pong parity and the
// source term, so the descriptor sets (even steps, odd steps, last step) are
// uploaded once per run and the source term is read from a per-run table
// indexed by a device-side step counter.  With ADI_BATCH_GRAPH the launches
// of two consecutive steps are captured once into a hipGraph and replayed.
// As after adi_run, every problem's state stays in its workspace
// (adi_get_state writes it out).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/adi.h"
#include "line_pass.h"
#include "problem.h"

namespace {

__global__ void tick_kernel(int* tick, int set, int value) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *tick = set ? value : *tick + 1;
}

// One grouped launch: passes [first, first + count) of a sorted set.
struct Group {
    int key;
    int first, count, total;
    size_t starts_off;   // offset (ints) of its prefix sums in the starts array
};

template <typename T>
struct TypedPart {
    std::vector<adi::PassDesc<T>> set[3][2];   // [even, odd, last][half]
    std::vector<Group> groups[3][2];
    std::vector<adi::PassDesc<T>> proto[3][2];  // kernel variant of each group
    std::vector<adi::LinePassArgs<T>> items;   // all sets, grouped, for upload
    std::vector<T> aF;                         // [problem][step]
    size_t items_off[3][2] = {};               // first item of each set
    adi::LinePassArgs<T>* ditems = nullptr;
    T* daF = nullptr;
};

}  // namespace

struct adi_batch {
    int dev = 0;
    hipStream_t st = nullptr;
    int flags = 0;
    std::vector<adi_problem*> probs;
    std::vector<hipEvent_t> ev;   // per problem: orders its own stream with the batch stream
    hipEvent_t done = nullptr;
    TypedPart<float> f32;
    TypedPart<double> f64;
    std::vector<int> starts;
    char* dmem = nullptr;
    size_t dmem_bytes = 0;
    int* dtick = nullptr;
    int* dstarts = nullptr;
    // extra streams of the concurrent grouped launches and the fork / join
    // events of a half-step
    static constexpr int kAux = 3;
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr, join[kAux] = {};
    hipGraph_t graph = nullptr;   // graph of the last run (kept until the next run)
    hipGraphExec_t exec = nullptr;
    int64_t launches = 0;         // grouped launches in the last run, graph replays included
};

namespace {

using adi::fail;
using adi::hip_fail;

template <typename T>
bool is_type(const adi_problem* pb) {
    return (pb->p.dtype == ADI_FP64) == std::is_same<T, double>::value;
}

// Descriptor sets of one dtype.  run_pass is called in the order a
// sequential run would call it, so the ping-pong state of every problem
// ends where adi_run would leave it.
template <typename T>
void build_sets(adi_batch* b, TypedPart<T>& part, int64_t nsteps, std::vector<size_t>& aF_index) {
    for (auto& s : part.set)
        for (auto& h : s) h.clear();
    part.aF.clear();
    std::vector<int> np_idx;
    for (size_t i = 0; i < b->probs.size(); ++i)
        if (is_type<T>(b->probs[i])) np_idx.push_back((int)i);
    const size_t np = np_idx.size();
    part.aF.assign(np * (size_t)nsteps, T(0));
    for (size_t k = 0; k < np; ++k) {
        adi_problem* pb = b->probs[np_idx[k]];
        for (int64_t s = 0; s < nsteps; ++s) part.aF[k * nsteps + s] = (T)adi::source_term(*pb, pb->step + s + 1);
        aF_index[np_idx[k]] = k * nsteps;
    }
    // aF table pointers are filled in after the device buffer is placed
    for (size_t k = 0; k < np; ++k) {
        adi_problem* pb = b->probs[np_idx[k]];
        const int v0 = pb->vcur, w0 = pb->wcur;
        const T* tab = (const T*)(uintptr_t)(aF_index[np_idx[k]] + 1);   // placeholder: index + 1
        if (nsteps >= 2)
            for (int h = 0; h < 2; ++h) part.set[0][h].push_back(adi::run_pass<T>(pb, 0, h, false, tab));
        if (nsteps >= 3)
            for (int h = 0; h < 2; ++h) part.set[1][h].push_back(adi::run_pass<T>(pb, 1, h, false, tab));
        pb->vcur = v0;
        pb->wcur = w0;
        if ((nsteps - 1) % 2)
            for (int h = 0; h < 2; ++h) (void)adi::run_pass<T>(pb, 0, h, false, tab);
        for (int h = 0; h < 2; ++h) part.set[2][h].push_back(adi::run_pass<T>(pb, nsteps - 1, h, false, tab));
    }
}

// Sort each set by kernel variant, cut it into groups, append the items and
// the prefix sums.
template <typename T>
void build_groups(TypedPart<T>& part, std::vector<int>& starts) {
    part.items.clear();
    for (int k = 0; k < 3; ++k)
        for (int h = 0; h < 2; ++h) {
            auto& v = part.set[k][h];
            std::stable_sort(v.begin(), v.end(),
                             [](const adi::PassDesc<T>& x, const adi::PassDesc<T>& y) { return x.key() < y.key(); });
            part.groups[k][h].clear();
            part.proto[k][h].clear();
            part.items_off[k][h] = part.items.size();
            size_t i = 0;
            while (i < v.size()) {
                size_t j = i;
                Group g{};
                g.key = v[i].key();
                part.proto[k][h].push_back(v[i]);
                g.first = (int)part.items.size();
                g.starts_off = starts.size();
                int tot = 0;
                while (j < v.size() && v[j].key() == g.key) {
                    starts.push_back(tot);
                    tot += v[j].tiles();
                    part.items.push_back(v[j].a);
                    ++j;
                }
                starts.push_back(tot);
                g.count = (int)(j - i);
                g.total = tot;
                part.groups[k][h].push_back(g);
                i = j;
            }
        }
}

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

void drop_graph(adi_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

template <typename T>
hipError_t launch_group(adi_batch* b, TypedPart<T>& part, int k, int h, size_t gi, hipStream_t st) {
    const Group& g = part.groups[k][h][gi];
    adi::GroupArgs<T> ga;
    ga.items = part.ditems + g.first;
    ga.starts = b->dstarts + g.starts_off;
    ga.tick = b->dtick;
    ga.nitems = g.count;
    ga.total = g.total;
    ++b->launches;
    return adi::launch_grouped<T>(part.proto[k][h][gi], ga, st);
}

// Work of a group, in element-slots: tiles x the slots one tile covers
// (lines per workgroup x window), for balancing the streams.
template <typename T>
double group_work(const TypedPart<T>& part, int k, int h, size_t gi) {
    const auto& d = part.proto[k][h][gi];
    const int dt = sizeof(T) == 8 ? 1 : 0;
    const double per = d.ver == 1 ? (double)adi::line_lanes(dt, d.cfg) * adi::line_ws(d.cfg)
                                  : (double)adi::line3_lanes(dt) * adi::LINE_WS;
    return (double)part.groups[k][h][gi].total * per * sizeof(T);
}

int launch_step(adi_batch* b, int k) {
    const bool one = (b->flags & ADI_BATCH_ONE_STREAM) != 0;
    for (int h = 0; h < 2; ++h) {
        // the groups of this half-step, largest first, each to the stream
        // with the least work so far (the batch stream is stream 0)
        struct Item { double w; int dt; size_t gi; };
        std::vector<Item> items;
        for (size_t gi = 0; gi < b->f32.groups[k][h].size(); ++gi)
            items.push_back({group_work(b->f32, k, h, gi), 0, gi});
        for (size_t gi = 0; gi < b->f64.groups[k][h].size(); ++gi)
            items.push_back({group_work(b->f64, k, h, gi), 1, gi});
        std::stable_sort(items.begin(), items.end(), [](const Item& x, const Item& y) { return x.w > y.w; });
        const int ns = one ? 1 : std::min<int>(1 + adi_batch::kAux, (int)items.size());
        double load[1 + adi_batch::kAux] = {};
        if (ns > 1) {
            HIP_TRY(hipEventRecord(b->fork, b->st), "fork");
            for (int j = 1; j < ns; ++j) HIP_TRY(hipStreamWaitEvent(b->aux[j - 1], b->fork, 0), "fork");
        }
        for (const Item& it : items) {
            int j = 0;
            for (int q = 1; q < ns; ++q)
                if (load[q] < load[j]) j = q;
            load[j] += it.w;
            hipStream_t st = j == 0 ? b->st : b->aux[j - 1];
            if (it.dt == 0)
                HIP_TRY(launch_group<float>(b, b->f32, k, h, it.gi, st), "grouped line pass");
            else
                HIP_TRY(launch_group<double>(b, b->f64, k, h, it.gi, st), "grouped line pass");
        }
        for (int j = 1; j < ns; ++j) {
            HIP_TRY(hipEventRecord(b->join[j - 1], b->aux[j - 1]), "join");
            HIP_TRY(hipStreamWaitEvent(b->st, b->join[j - 1], 0), "join");
        }
    }
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, b->st, b->dtick, 0, 0);
    HIP_TRY(hipGetLastError(), "step counter");
    return ADI_OK;
}

int run_batch(adi_batch* b, int64_t nsteps) {
    const size_t np = b->probs.size();
    // order the batch stream after the problems' own streams
    for (size_t i = 0; i < np; ++i) {
        adi_problem* pb = b->probs[i];
        if (pb->st != b->st) {
            HIP_TRY(hipEventRecord(b->ev[i], pb->st), "hipEventRecord");
            HIP_TRY(hipStreamWaitEvent(b->st, b->ev[i], 0), "hipStreamWaitEvent");
        }
    }
    // the previous run's uploads and graph must be done with before they change
    HIP_TRY(hipStreamSynchronize(b->st), "hipStreamSynchronize");
    drop_graph(b);

    // set-up copies and explicit pass of every problem whose state is still
    // in its bound arrays
    for (size_t i = 0; i < np; ++i) {
        adi_problem* pb = b->probs[i];
        if (pb->ready) continue;
        const int rc = pb->p.dtype == ADI_FP64 ? adi::run_begin<double>(pb, b->st) : adi::run_begin<float>(pb, b->st);
        if (rc != ADI_OK) return rc;
    }

    std::vector<size_t> aF_index(np, 0);
    build_sets<float>(b, b->f32, nsteps, aF_index);
    build_sets<double>(b, b->f64, nsteps, aF_index);
    b->starts.clear();
    build_groups<float>(b->f32, b->starts);
    build_groups<double>(b->f64, b->starts);

    // device buffer: items f32 | items f64 | aF f32 | aF f64 | starts | tick
    const size_t o_i32 = 0;
    const size_t o_i64 = o_i32 + align256(b->f32.items.size() * sizeof(adi::LinePassArgs<float>));
    const size_t o_a32 = o_i64 + align256(b->f64.items.size() * sizeof(adi::LinePassArgs<double>));
    const size_t o_a64 = o_a32 + align256(b->f32.aF.size() * sizeof(float));
    const size_t o_st = o_a64 + align256(b->f64.aF.size() * sizeof(double));
    const size_t o_tk = o_st + align256(b->starts.size() * sizeof(int));
    const size_t need = o_tk + 256;
    if (need > b->dmem_bytes) {
        if (b->dmem) (void)hipFree(b->dmem);
        b->dmem = nullptr;
        b->dmem_bytes = 0;
        void* m = nullptr;
        hipError_t e = hipMalloc(&m, need);
        if (e != hipSuccess) return fail(ADI_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
        b->dmem = (char*)m;
        b->dmem_bytes = need;
    }
    b->f32.ditems = (adi::LinePassArgs<float>*)(b->dmem + o_i32);
    b->f64.ditems = (adi::LinePassArgs<double>*)(b->dmem + o_i64);
    b->f32.daF = (float*)(b->dmem + o_a32);
    b->f64.daF = (double*)(b->dmem + o_a64);
    b->dstarts = (int*)(b->dmem + o_st);
    b->dtick = (int*)(b->dmem + o_tk);
    // replace the placeholder table indices by device addresses
    for (auto& a : b->f32.items)
        if (a.aFtab) a.aFtab = b->f32.daF + ((uintptr_t)a.aFtab - 1);
    for (auto& a : b->f64.items)
        if (a.aFtab) a.aFtab = b->f64.daF + ((uintptr_t)a.aFtab - 1);
    auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, b->st) : hipSuccess;
    };
    HIP_TRY(up(b->f32.ditems, b->f32.items.data(), b->f32.items.size() * sizeof(adi::LinePassArgs<float>)), "upload");
    HIP_TRY(up(b->f64.ditems, b->f64.items.data(), b->f64.items.size() * sizeof(adi::LinePassArgs<double>)), "upload");
    HIP_TRY(up(b->f32.daF, b->f32.aF.data(), b->f32.aF.size() * sizeof(float)), "upload");
    HIP_TRY(up(b->f64.daF, b->f64.aF.data(), b->f64.aF.size() * sizeof(double)), "upload");
    HIP_TRY(up(b->dstarts, b->starts.data(), b->starts.size() * sizeof(int)), "upload");
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, b->st, b->dtick, 1, 0);
    HIP_TRY(hipGetLastError(), "step counter");

    b->launches = 0;
    int64_t s = 0;
    const int64_t pairs = (nsteps - 1) / 2;
    if ((b->flags & ADI_BATCH_GRAPH) && pairs >= 1) {
        // steps 0 .. 2*pairs-1 from a graph of two steps
        HIP_TRY(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        int rc = launch_step(b, 0);
        if (rc == ADI_OK) rc = launch_step(b, 1);
        hipError_t e = hipStreamEndCapture(b->st, &b->graph);
        if (rc != ADI_OK) return rc;
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        for (int64_t r = 0; r < pairs; ++r) HIP_TRY(hipGraphLaunch(b->exec, b->st), "hipGraphLaunch");
        b->launches *= pairs;
        s = 2 * pairs;
    }
    for (; s < nsteps; ++s) {
        const int k = s == nsteps - 1 ? 2 : (int)(s % 2);
        const int rc = launch_step(b, k);
        if (rc != ADI_OK) return rc;
    }

    for (size_t i = 0; i < np; ++i) adi::run_advance(b->probs[i], nsteps);
    // later work on a problem's own stream waits for the batch
    HIP_TRY(hipEventRecord(b->done, b->st), "hipEventRecord");
    for (size_t i = 0; i < np; ++i)
        if (b->probs[i]->st != b->st) HIP_TRY(hipStreamWaitEvent(b->probs[i]->st, b->done, 0), "hipStreamWaitEvent");
    return ADI_OK;
}

void release(adi_batch* b) {
    if (!b) return;
    (void)hipSetDevice(b->dev);
    (void)hipStreamSynchronize(b->st);
    drop_graph(b);
    for (auto e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->fork) (void)hipEventDestroy(b->fork);
    for (int j = 0; j < adi_batch::kAux; ++j) {
        if (b->join[j]) (void)hipEventDestroy(b->join[j]);
        if (b->aux[j]) {
            (void)hipStreamSynchronize(b->aux[j]);
            (void)hipStreamDestroy(b->aux[j]);
        }
    }
    if (b->dmem) (void)hipFree(b->dmem);
    delete b;
}

}  // namespace

extern "C" {

int adi_batch_create(adi_problem* const* problems, int count, void* hip_stream, int flags, adi_batch** out) {
    if (!out) return fail(ADI_EINVAL, "out is NULL");
    *out = nullptr;
    if (!problems || count <= 0) return fail(ADI_EINVAL, "need at least one problem");
    if (flags & ~(ADI_BATCH_GRAPH | ADI_BATCH_ONE_STREAM)) return fail(ADI_EINVAL, "unknown flags 0x%x", flags);
    if ((flags & ADI_BATCH_GRAPH) && !hip_stream)
        return fail(ADI_EINVAL, "ADI_BATCH_GRAPH needs a stream other than the null stream");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    for (int i = 0; i < count; ++i) {
        const adi_problem* pb = problems[i];
        if (!pb) return fail(ADI_EINVAL, "problem %d is NULL", i);
        if (!pb->bound) return fail(ADI_ENOTREADY, "problem %d has no bound arrays", i);
        if (pb->dev != dev) return fail(ADI_EINVAL, "problem %d lives on device %d, not the current %d", i, pb->dev, dev);
        if (pb->eps > 0.0)
            return fail(ADI_EINVAL, "problem %d uses tolerance-tested stages, which batches do not run", i);
        if (pb->p.sweeps == 0)
            return fail(ADI_EINVAL, "problem %d uses direct solves (sweeps 0), which batches do not run", i);
        if (pb->fsig.kind || pb->bsig.kind)
            return fail(ADI_EINVAL, "problem %d has a forcing field or wall data, which batches do not run", i);
        for (int j = 0; j < i; ++j)
            if (problems[j] == pb) return fail(ADI_EINVAL, "problem %d appears twice", i);
    }
    adi_batch* b = new (std::nothrow) adi_batch();
    if (!b) return fail(ADI_ENOMEM, "host allocation failed");
    b->dev = dev;
    b->st = (hipStream_t)hip_stream;
    b->flags = flags;
    b->probs.assign(problems, problems + count);
    b->ev.assign(count, nullptr);
    for (int i = 0; i < count; ++i) {
        hipError_t e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
        if (e != hipSuccess) {
            release(b);
            return hip_fail(e, "hipEventCreate");
        }
    }
    hipError_t e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int j = 0; j < adi_batch::kAux && e == hipSuccess && !(flags & ADI_BATCH_ONE_STREAM); ++j) {
        e = hipEventCreateWithFlags(&b->join[j], hipEventDisableTiming);
        // default priority, like every stream of the library
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->aux[j], hipStreamNonBlocking);
    }
    if (e != hipSuccess) {
        release(b);
        return hip_fail(e, "hipEventCreate");
    }
    *out = b;
    return ADI_OK;
}

int adi_batch_run(adi_batch* b, int64_t nsteps) {
    if (!b) return fail(ADI_EINVAL, "batch is NULL");
    if (nsteps < 0) return fail(ADI_EINVAL, "nsteps < 0");
    if (nsteps == 0) return ADI_OK;
    for (size_t i = 0; i < b->probs.size(); ++i)
        if (!b->probs[i]->bound) return fail(ADI_ENOTREADY, "problem %zu has no bound arrays", i);
    HIP_TRY(hipSetDevice(b->dev), "hipSetDevice");
    return run_batch(b, nsteps);
}

int adi_batch_sync(adi_batch* b) {
    if (!b) return fail(ADI_EINVAL, "batch is NULL");
    HIP_TRY(hipSetDevice(b->dev), "hipSetDevice");
    HIP_TRY(hipStreamSynchronize(b->st), "hipStreamSynchronize");
    return ADI_OK;
}

int adi_batch_launches(const adi_batch* b, int64_t* n) {
    if (!b || !n) return fail(ADI_EINVAL, "NULL argument");
    *n = b->launches;
    return ADI_OK;
}

int adi_batch_destroy(adi_batch* b) {
    release(b);
    return ADI_OK;
}

}  // extern "C"
