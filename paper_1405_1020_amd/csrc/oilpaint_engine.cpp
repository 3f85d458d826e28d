// Batched and served forms of the filter: one persistent launch over a
// flattened tile queue (oilpaint_batch), the same launch captured once in a
// hipGraph and replayed (oilpaint_plan_*), and a continuous-batching request
// queue that packs waiting work into successive persistent launches
// (oilpaint_queue_*).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "oilpaint_internal.h"

namespace oilpaint_impl {

int make_job(const oilpaint_desc& d, const oilpaint_variant* v, int device, Job& j, bool& empty);
int apply_variant(Job& j, const oilpaint_variant& v, int device);
int check_device_ptr(const void* p);
oilpaint_variant choose_variant(int width, int height, int reff, int levels, bool paper, int device);

namespace {

// Smallest radius whose batch tiles use four wavefronts per strip.  A batch
// runs several classes at once, which already gives the GPU many wavefronts,
// so below this the split's barriers and tile hand-off cost more than its
// latency hiding gains (64-image batch of radii 2-8: 74.5 GP/s with one
// wavefront per strip from radius 8 on, 67.5 with four).
constexpr int kBatchSplitMinRadius = 10;
// Smallest radius whose jobs tuned to the column layout's several-wavefront
// form run in its four-wavefront batch classes.
constexpr int kBatchColumnMinRadius = 7;

// Layout of a job inside a persistent launch: the streamed layouts as the
// job's own choice (four wavefronts sharing a strip where that is its plain
// shape and the radius is at least kBatchSplitMinRadius, else one); the
// column layout's radius <= 15 form with several wavefronts as four from
// kBatchColumnMinRadius, else the streamed layout (one wavefront of the
// column form in the paper form); every other layout with one computing
// wavefront per workgroup (a tile-staged shape of several wavefronts becomes
// the streamed layout when it applies); shrunk (wavefronts, then rows, then
// lanes) until its on-chip footprint fits.  The rows are set afterwards for
// the whole launch (shape_rows).
int batch_shape(Job& j, int device) {
    oilpaint_variant v = choose_variant(j.width, j.height, j.radius, j.levels, j.paper != 0, device);
    if (v.hist == OILPAINT_HIST_REGS) {  // no persistent form: the streamed layout's classes
        v.hist = OILPAINT_HIST_STREAM;
        v.waves = 1;
        v.lanes = 64;
        v.rows = 0;
        v.per_cu = 8;
    }
    if (is_stream(v.hist) && v.waves > 1 && j.radius < kBatchSplitMinRadius) {
        v.waves = 1;
        v.per_cu = 8;
    }
    if (v.hist == OILPAINT_HIST_COLUMN && v.waves > 1 && j.radius > kPackedMaxRadius) {
        // the radius 16..31 form has no persistent kernel: the generic column classes
        v.waves = 1;
        v.rows = 0;
        v.per_cu = 8;
    }
    if (v.hist == OILPAINT_HIST_COLUMN && v.waves > 1) {
        // the column layout's four-wavefront classes from
        // kBatchColumnMinRadius; below it the streamed layout's classes,
        // whose one-wavefront batch forms beat the column layout's (its
        // one-wavefront form for the paper form)
        if (j.radius >= kBatchColumnMinRadius && j.radius <= kPackedMaxRadius && j.levels <= kColumn15MaxLevels) {
            v.waves = 4;
            v.rows = 0;
        } else if (!j.paper) {
            v.hist = OILPAINT_HIST_STREAM;
            v.lanes = 64;
            v.rows = 0;
            v.waves = j.radius >= kBatchSplitMinRadius ? kSplitWaves : 1;
            v.per_cu = v.waves > 1 ? 5 : 8;
        } else {
            v.waves = 1;
            v.per_cu = 8;
        }
    }
    if (!is_stream(v.hist) && v.hist != OILPAINT_HIST_COLUMN && v.waves > 1) {
        if (j.radius <= kPackedMaxRadius && j.levels <= 64 && !j.paper) {
            v.hist = OILPAINT_HIST_STREAM;
            v.lanes = 64;
            v.rows = 0;
            v.per_cu = 8;
        }
        v.waves = 1;
    }
    for (;;) {
        const int st = apply_variant(j, v, device);
        if (st == OILPAINT_OK) return st;
        if (v.waves > 1)
            v.waves = 1;
        else if (v.rows > 8)
            v.rows >>= 1;
        else if (v.lanes > 16)
            v.lanes >>= 1;
        else
            return st;
    }
}

// Shortest run worth a tile: about 5(2r+1) rows, so that the (2r+1)^2 first
// window costs at most ~10 % of the run's sliding updates (or the whole
// band when it is shorter).
int min_run_rows(const Job& j) {
    return std::max(1, std::min(j.row_end - j.row_begin, std::max(8, 5 * (2 * j.radius + 1))));
}

// Rows per tile for every job of one launch, from the launch's total work:
// about kTilesPerSlot tiles per resident workgroup over the whole launch
// (the batch, not a single image, supplies the parallelism; long runs pay
// the first window and the per-tile prologue rarely), at least
// min_run_rows and at most the band or 1024 rows.  A job whose layout does
// not fit the new rows keeps its own.
constexpr int kTilesPerSlot = 32;
constexpr int kSlotsPerCu = 8;  // typical resident workgroups (one-wavefront classes)

void shape_rows(std::vector<Job>& jobs, int device) {
    const DeviceInfo d = device_info(device);
    const double slots = (double)(d.ok ? d.cus : 256) * kSlotsPerCu;
    double strip_rows = 0;
    for (const Job& j : jobs)
        strip_rows += (double)((j.width + j.lanes - 1) / j.lanes) * (j.row_end - j.row_begin);
    const int target = (int)std::min(1024.0, std::ceil(strip_rows / (kTilesPerSlot * slots)));
    for (Job& j : jobs) {
        const int band = j.row_end - j.row_begin;
        const int rows = std::max(min_run_rows(j), std::min(target, std::min(band, 1024)));
        oilpaint_variant v;
        v.waves = j.waves;
        v.hist = j.hist;
        v.lanes = j.lanes;
        v.per_cu = 1;
        const int runs = runs_per_tile(j.hist, j.waves);
        v.rows = std::max(1, (rows + runs - 1) / runs);
        Job t = j;
        if (apply_variant(t, v, device) == OILPAINT_OK) {
            j = t;
        } else {  // own rows, tiles over this band
            const long per_tile = (long)runs * j.rows;
            j.tiles_y = (int)((band + per_tile - 1) / per_tile);
        }
    }
}

// Relative cost of one tile: window updates plus the mode search per output
// pixel, plus the first window of every lane.
double tile_cost(const Job& j) {
    const double span = 2.0 * j.radius + 1.0;
    const int runs = runs_per_tile(j.hist, j.waves);
    const double px = (double)j.lanes * j.rows * runs;
    return px * (2.0 * span + j.levels * 0.5 + 4.0) + (double)j.lanes * runs * span * span;
}

// One kernel class of a batch (batch_class): its jobs in queue order and
// its flattened tile queue.
struct ClassLayout {
    int cls = kGenericClass;
    std::vector<Job> jobs;        // queue order
    std::vector<int32_t> first;   // njobs + 1
    size_t lds = 0;
    int ntiles = 0;
    double cost = 0;              // total tile cost
    size_t first_off = 0, jobs_off = 0;  // offsets in the argument block
};

// Argument block: [counters, one per class, kCounterWords apart][first_tile
// arrays][job arrays].
constexpr int kCounterWords = 32;  // 128 bytes: one counter per cache line
constexpr int kMaxBranches = 4;    // classes run on at most this many streams

struct Layout {
    std::vector<ClassLayout> classes;  // costliest first
    size_t bytes = 0;
    int ntiles = 0;
};

// Group jobs by kernel class, order each class's jobs by tile cost
// (costliest first, so that long tiles start early and cheap ones fill the
// tail) and lay out the argument block.
void build_layout(const std::vector<Job>& jobs, Layout& out) {
    std::map<int, ClassLayout> by;
    for (const Job& j : jobs) {
        ClassLayout& c = by[batch_class(j)];
        c.cls = batch_class(j);
        c.jobs.push_back(j);
    }
    out = Layout();
    for (auto& kv : by) out.classes.push_back(std::move(kv.second));
    for (ClassLayout& c : out.classes) {
        std::stable_sort(c.jobs.begin(), c.jobs.end(),
                         [&](const Job& a, const Job& b) { return tile_cost(a) > tile_cost(b); });
        c.first.assign(c.jobs.size() + 1, 0);
        long total = 0;
        for (size_t i = 0; i < c.jobs.size(); ++i) {
            const long t = (long)c.jobs[i].tiles_x * c.jobs[i].tiles_y;
            c.first[i] = (int32_t)total;
            total += t;
            c.lds = std::max(c.lds, lds_bytes(c.jobs[i]));
            c.cost += tile_cost(c.jobs[i]) * (double)t;
        }
        c.first[c.jobs.size()] = (int32_t)total;
        c.ntiles = (int)total;
        out.ntiles += c.ntiles;
    }
    std::stable_sort(out.classes.begin(), out.classes.end(),
                     [](const ClassLayout& a, const ClassLayout& b) { return a.cost > b.cost; });
    size_t off = ((size_t)kCounterWords * 4 * out.classes.size() + 255) & ~(size_t)255;
    for (ClassLayout& c : out.classes) {
        c.first_off = off;
        off += (sizeof(int32_t) * c.first.size() + 15) & ~(size_t)15;
    }
    off = (off + 255) & ~(size_t)255;
    for (ClassLayout& c : out.classes) {
        c.jobs_off = off;
        off += sizeof(Job) * c.jobs.size();
    }
    out.bytes = off;
}

void pack_args(const Layout& L, uint8_t* host) {
    std::memset(host, 0, L.bytes);
    for (const ClassLayout& c : L.classes) {
        std::memcpy(host + c.first_off, c.first.data(), sizeof(int32_t) * c.first.size());
        std::memcpy(host + c.jobs_off, c.jobs.data(), sizeof(Job) * c.jobs.size());
    }
}

BatchArgs class_args(const Layout& L, size_t k, uint8_t* dev) {
    const ClassLayout& c = L.classes[k];
    BatchArgs a;
    a.counter = reinterpret_cast<uint32_t*>(dev) + k * kCounterWords;
    a.first_tile = reinterpret_cast<const int32_t*>(dev + c.first_off);
    a.jobs = reinterpret_cast<const Job*>(dev + c.jobs_off);
    a.njobs = (int32_t)c.jobs.size();
    a.ntiles = c.ntiles;
    return a;
}

// Side streams and events that spread a batch's classes over concurrent
// streams.  Inside a stream capture the branches become parallel graph
// branches.
struct Branches {
    hipStream_t side[kMaxBranches] = {};
    hipEvent_t join[kMaxBranches] = {};
    hipEvent_t fork = nullptr;
    int made = 0;

    Branches() = default;
    Branches(const Branches&) = delete;
    Branches& operator=(const Branches&) = delete;
    ~Branches() {
        for (int b = 0; b < made; ++b) {
            (void)hipStreamSynchronize(side[b]);
            (void)hipStreamDestroy(side[b]);
            (void)hipEventDestroy(join[b]);
        }
        if (fork) (void)hipEventDestroy(fork);
    }
    // Make sure side streams 0 .. n-1 exist.
    bool ensure(int n) {
        if (!fork && hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return false;
        while (made < n) {
            if (hipStreamCreateWithFlags(&side[made], hipStreamNonBlocking) != hipSuccess) return false;
            if (hipEventCreateWithFlags(&join[made], hipEventDisableTiming) != hipSuccess) {
                (void)hipStreamDestroy(side[made]);
                return false;
            }
            ++made;
        }
        return true;
    }
};

// Enqueue the counter reset and every class's persistent kernel, the
// classes spread over branches by total cost (each to the least loaded).
//   join:      branch 0 is `stream` itself and the side branches join back
//              into it, so the whole batch is ordered before later work on
//              `stream` (batches and plans).
//   detached:  every class runs on a side stream that waits for the reset
//              on `stream`, and nothing joins back, so the next launch's
//              classes start while this one's last tiles finish (the
//              request queue).  The streams carrying work are returned in
//              ends[0 .. *nends-1]; the caller records completion there.
// Returns the number of workgroups launched in `workgroups`.
int enqueue_classes(const Layout& L, uint8_t* dev, int device, Branches& br, hipStream_t stream, bool join,
                    int* workgroups, hipStream_t* ends, int* nends) {
    const int nc = (int)L.classes.size();
    if (workgroups) *workgroups = 0;
    if (nends) *nends = 0;
    if (L.ntiles == 0) return OILPAINT_OK;
    if (launch_reset_counters(reinterpret_cast<uint32_t*>(dev), nc, kCounterWords, stream) != hipSuccess)
        return OILPAINT_ERR_HIP;
    const int nb = std::min(nc, kMaxBranches);
    const int nside = join ? nb - 1 : nb;
    hipStream_t bs[kMaxBranches];
    if (!br.ensure(nside)) {
        (void)note_hip("branch streams", hipGetLastError());
        return OILPAINT_ERR_HIP;
    }
    for (int b = 0; b < nb; ++b) bs[b] = join ? (b == 0 ? stream : br.side[b - 1]) : br.side[b];
    if (nside > 0) {
        if (note_hip("hipEventRecord", hipEventRecord(br.fork, stream)) != hipSuccess) return OILPAINT_ERR_HIP;
        for (int b = 0; b < nside; ++b)
            if (note_hip("hipStreamWaitEvent", hipStreamWaitEvent(br.side[b], br.fork, 0)) != hipSuccess)
                return OILPAINT_ERR_HIP;
    }
    double load[kMaxBranches] = {};
    int total = 0;
    for (int k = 0; k < nc; ++k) {
        const ClassLayout& c = L.classes[k];
        if (c.ntiles == 0) continue;
        const int b = (int)(std::min_element(load, load + nb) - load);
        load[b] += c.cost;
        const int waves = batch_waves(c.cls);
        const int grid = std::min(batch_grid(device, c.cls, waves, c.lds), c.ntiles);
        if (launch_batch(class_args(L, (size_t)k, dev), c.cls, waves, c.lds, grid, bs[b]) != hipSuccess)
            return OILPAINT_ERR_HIP;
        total += grid;
    }
    if (join) {
        for (int b = 0; b < nside; ++b) {
            if (note_hip("hipEventRecord", hipEventRecord(br.join[b], br.side[b])) != hipSuccess ||
                note_hip("hipStreamWaitEvent", hipStreamWaitEvent(stream, br.join[b], 0)) != hipSuccess)
                return OILPAINT_ERR_HIP;
        }
        if (ends) ends[0] = stream;
        if (nends) *nends = 1;
    } else {
        for (int b = 0; b < nb; ++b)
            if (ends) ends[b] = bs[b];
        if (nends) *nends = nb;
    }
    if (workgroups) *workgroups = total;
    return OILPAINT_OK;
}

// A small ring of (pinned host, device) argument buffers.  A slot is reused
// only after the events recorded behind its last launch (one per stream that
// carried it) have completed.
struct ArgSlot {
    uint8_t* dev = nullptr;
    uint8_t* host = nullptr;
    size_t cap = 0;
    hipEvent_t done[kMaxBranches] = {};
    int pending = 0;  // events recorded
};

class ArgRing {
  public:
    explicit ArgRing(int n) : slots_(n) {}
    ~ArgRing() {
        for (auto& s : slots_) {
            for (int i = 0; i < s.pending; ++i) (void)hipEventSynchronize(s.done[i]);
            if (s.dev) (void)hipFree(s.dev);
            if (s.host) (void)hipHostFree(s.host);
            for (hipEvent_t e : s.done)
                if (e) (void)hipEventDestroy(e);
        }
    }
    // Returns a slot with at least `bytes` of capacity, or nullptr.
    ArgSlot* acquire(size_t bytes) {
        ArgSlot* s = &slots_[next_];
        next_ = (next_ + 1) % slots_.size();
        for (int i = 0; i < s->pending; ++i)
            if (hipEventSynchronize(s->done[i]) != hipSuccess) return nullptr;
        s->pending = 0;
        if (s->cap < bytes) {
            if (s->dev) (void)hipFree(s->dev);
            if (s->host) (void)hipHostFree(s->host);
            s->dev = nullptr;
            s->host = nullptr;
            s->cap = 0;
            const size_t cap = std::max(bytes, (size_t)65536);
            if (hipMalloc(&s->dev, cap) != hipSuccess) return nullptr;
            if (hipHostMalloc(reinterpret_cast<void**>(&s->host), cap, hipHostMallocDefault) != hipSuccess) {
                (void)hipFree(s->dev);
                s->dev = nullptr;
                return nullptr;
            }
            s->cap = cap;
        }
        return s;
    }
    // The slot is in use by the work enqueued so far on streams[0 .. n-1].
    void release(ArgSlot* s, const hipStream_t* streams, int n) {
        for (int i = 0; i < n && i < kMaxBranches; ++i) {
            if (!s->done[i] && hipEventCreateWithFlags(&s->done[i], hipEventDisableTiming) != hipSuccess) break;
            if (hipEventRecord(s->done[i], streams[i]) != hipSuccess) break;
            s->pending = i + 1;
        }
    }

  private:
    std::vector<ArgSlot> slots_;
    size_t next_ = 0;
};

// Upload `L` through `ring` and enqueue its classes (see enqueue_classes).
int enqueue_layout(const Layout& L, int device, ArgRing& ring, Branches& br, hipStream_t stream, bool join,
                   hipStream_t* ends, int* nends) {
    if (nends) *nends = 0;
    if (L.ntiles == 0) return OILPAINT_OK;
    ArgSlot* s = ring.acquire(L.bytes);
    if (!s) return OILPAINT_ERR_NOMEM;
    pack_args(L, s->host);
    if (note_hip("hipMemcpyAsync", hipMemcpyAsync(s->dev, s->host, L.bytes, hipMemcpyHostToDevice, stream)) !=
        hipSuccess)
        return OILPAINT_ERR_HIP;
    hipStream_t es[kMaxBranches];
    int ne = 0;
    const int st = enqueue_classes(L, s->dev, device, br, stream, join, nullptr, es, &ne);
    if (st != OILPAINT_OK) return st;
    // every stream in es[] is ordered after the upload and the reset
    ring.release(s, es, ne);
    for (int i = 0; i < ne; ++i)
        if (ends) ends[i] = es[i];
    if (nends) *nends = ne;
    return OILPAINT_OK;
}

ArgRing& device_ring(int device) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<ArgRing>> rings;
    std::lock_guard<std::mutex> lock(mu);
    auto& p = rings[device];
    if (!p) p.reset(new ArgRing(8));
    return *p;
}

Branches& device_branches(int device) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<Branches>> m;
    std::lock_guard<std::mutex> lock(mu);
    auto& p = m[device];
    if (!p) p.reset(new Branches);
    return *p;
}

std::mutex& ring_mutex(int device) {
    static std::mutex mu;
    static std::map<int, std::unique_ptr<std::mutex>> m;
    std::lock_guard<std::mutex> lock(mu);
    auto& p = m[device];
    if (!p) p.reset(new std::mutex);
    return *p;
}

// Validate all descriptors into jobs (empty images dropped).
int collect_jobs(const oilpaint_desc* descs, int n, int device, std::vector<Job>& jobs, int* bad_index) {
    if (n < 0) return OILPAINT_ERR_ARG;
    if (n > 0 && !descs) return OILPAINT_ERR_NULL;
    jobs.clear();
    jobs.reserve(n);
    for (int i = 0; i < n; ++i) {
        Job j;
        bool empty = false;
        int st = make_job(descs[i], nullptr, device, j, empty);
        if (st == OILPAINT_OK && !empty) st = batch_shape(j, device);
        if (st == OILPAINT_OK && !empty) st = check_device_ptr(j.src);
        if (st == OILPAINT_OK && !empty) st = check_device_ptr(j.dst);
        if (st != OILPAINT_OK) {
            if (bad_index) *bad_index = i;
            return st;
        }
        if (!empty) jobs.push_back(j);
    }
    if (bad_index) *bad_index = -1;
    shape_rows(jobs, device);
    return OILPAINT_OK;
}

}  // namespace
}  // namespace oilpaint_impl

using namespace oilpaint_impl;

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
struct oilpaint_plan {
    int device = 0;
    Layout layout;
    uint8_t* dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int grid = 0;  // workgroups over all classes
    oilpaint_plan() = default;
    oilpaint_plan(const oilpaint_plan&) = delete;
    oilpaint_plan& operator=(const oilpaint_plan&) = delete;
    // also on a failed create, which returns before handing the plan out
    ~oilpaint_plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (dev) (void)hipFree(dev);
    }
};

// ---------------------------------------------------------------------------
// Queue
// ---------------------------------------------------------------------------
constexpr int kQueueDepth = 4;  // launches in flight on a queue's stream

struct QueueReq {
    Job job;              // whole request (row_begin .. row_end), batch shape
    oilpaint_desc desc;   // as pushed: a lone request runs as a plain launch
    int next_row;         // first output row not yet launched
    int launches_left = 0;
    bool all_launched = false;
    bool done = false;
    int status = OILPAINT_OK;  // an error code once a launch of its rows failed
};

struct Inflight {
    std::vector<hipEvent_t> evs;    // one per stream that carries the launch
    std::vector<uint64_t> tickets;  // requests with a band in this launch
};

struct oilpaint_queue {
    int device = 0;
    hipStream_t stream = nullptr;
    int capacity = 0;
    int64_t step_pixels = 0;
    uint64_t next_ticket = 1;
    std::unordered_map<uint64_t, QueueReq> reqs;
    std::deque<uint64_t> waiting;  // arrival order, some rows not launched
    std::deque<Inflight> inflight;
    std::vector<hipEvent_t> free_events;
    std::unique_ptr<ArgRing> ring;
    std::unique_ptr<Branches> branches;
    std::deque<uint64_t> finished;  // completed, in completion order (may hold
                                    // tickets already reported by poll)
    size_t held = 0;  // requests not yet complete
    unsigned next_side = 0;  // side stream of the next single-band launch
    bool last_direct = false;  // the last launch was one large request alone
    int fail_next = 0;  // test hook: launches still to be treated as failed
};

namespace {

// Retire every launch that has completed (launches on different streams may
// complete out of order); with `block`, first wait for the oldest.  A
// request is complete when all launches holding one of its bands are.
int retire(oilpaint_queue* q, bool block) {
    if (block && !q->inflight.empty())
        for (hipEvent_t e : q->inflight.front().evs)
            if (note_hip("hipEventSynchronize", hipEventSynchronize(e)) != hipSuccess) return OILPAINT_ERR_HIP;
    for (auto it = q->inflight.begin(); it != q->inflight.end();) {
        bool done = true;
        for (hipEvent_t e : it->evs) {
            const hipError_t st = hipEventQuery(e);
            if (st == hipSuccess) continue;
            if (st != hipErrorNotReady) {
                (void)note_hip("hipEventQuery", st);
                return OILPAINT_ERR_HIP;
            }
            done = false;
            break;
        }
        if (!done) {
            ++it;
            continue;
        }
        for (uint64_t t : it->tickets) {
            auto r_it = q->reqs.find(t);
            if (r_it == q->reqs.end()) continue;
            QueueReq& r = r_it->second;
            if (--r.launches_left == 0 && r.all_launched && !r.done) {
                r.done = true;
                --q->held;
                q->finished.push_back(t);
            }
        }
        for (hipEvent_t e : it->evs) q->free_events.push_back(e);
        it = q->inflight.erase(it);
    }
    return OILPAINT_OK;
}

// Waiting work goes out in launches.  Small requests are packed together:
// each gets an equal share of the launch's pixels (at least one tile row of
// its own shape), so a small request that arrives behind others finishes in
// the next launch instead of waiting for them to drain.  Such a launch covers
// step_pixels, or a quarter of the waiting small pixels when the backlog is
// larger (at most 64 x step_pixels), so that a backlog keeps enough work in
// flight.  A launch of a single band uses the plain kernel with the
// request's own launch shape.  A request with at least kDirectPixels left
// fills the GPU alone: it goes out whole as one plain launch with its own
// tuned shape instead of in bands, on a side stream of its own, so that
// batches of small requests run beside it.
constexpr int64_t kDirectPixels = 4 << 20;

int64_t pixels_left(const QueueReq& r) { return (int64_t)(r.job.row_end - r.next_row) * r.job.width; }

// Rows [rb, re) of request t as one plain launch on the next side stream.
int launch_direct(oilpaint_queue* q, uint64_t t, int rb, int re, hipStream_t* end) {
    oilpaint_desc d = q->reqs[t].desc;
    d.row_begin = rb;
    d.row_end = re;
    Job pj;
    bool empty = false;
    const hipStream_t side = q->branches->side[q->next_side++ % kMaxBranches];
    *end = side;
    const int st = make_job(d, nullptr, q->device, pj, empty);
    if (st != OILPAINT_OK) return st;
    if (!empty && launch_plain(pj, pj.waves, lds_bytes(pj), side) != hipSuccess) return OILPAINT_ERR_HIP;
    return OILPAINT_OK;
}

// A launch that could not be enqueued, or whose completion cannot be
// tracked, fails the requests that had rows in it: none of their rows is
// launched again, and each is complete, with `st` as its status, as soon as
// the launches holding its earlier bands have retired (their kernels may
// still write its dst until then).
void fail_launch(oilpaint_queue* q, const std::vector<uint64_t>& tickets, int st) {
    for (uint64_t t : tickets) {
        QueueReq& r = q->reqs[t];
        r.status = st;
        r.all_launched = true;
        if (--r.launches_left == 0 && !r.done) {
            r.done = true;
            --q->held;
            q->finished.push_back(t);
        }
    }
    std::deque<uint64_t> still;
    for (uint64_t t : q->waiting)
        if (q->reqs[t].status == OILPAINT_OK) still.push_back(t);
    q->waiting.swap(still);
}

// One launch of waiting work (returns 1, 0 if there was none, or an error):
//   * a lone request with nothing in flight: the whole request, plain;
//   * a large request (kDirectPixels): the whole request, plain -- at most
//     every other launch while small requests wait, so that neither kind
//     starves the other;
//   * otherwise every waiting small request gets an equal share of the
//     launch's pixels (at least one run of min_run_rows), one batch launch.
// A launch that fails fails its requests (fail_launch) and still counts as a
// step: the queue goes on with the other requests.
int launch_step(oilpaint_queue* q) {
    if (q->waiting.empty()) return 0;
    // The work goes to side streams only, so that nothing on the queue's own
    // stream (uploads, counter resets) waits for a running launch.
    if (!q->branches->ensure(kMaxBranches)) {
        (void)note_hip("branch streams", hipGetLastError());
        return OILPAINT_ERR_HIP;
    }
    bool any_small = false;
    auto big = q->waiting.end();
    for (auto it = q->waiting.begin(); it != q->waiting.end(); ++it) {
        const int64_t left = pixels_left(q->reqs[*it]);
        if (left >= kDirectPixels) {
            if (big == q->waiting.end()) big = it;
        } else {
            any_small = true;
        }
    }
    const bool lone = q->waiting.size() == 1 && q->inflight.empty();
    hipStream_t ends[kMaxBranches];
    int nends = 0;
    std::vector<uint64_t> tickets;
    int st = OILPAINT_OK;
    if (lone || (big != q->waiting.end() && (!q->last_direct || !any_small))) {
        const uint64_t t = lone ? q->waiting.front() : *big;
        QueueReq& r = q->reqs[t];
        if (q->fail_next > 0) {
            --q->fail_next;
            st = OILPAINT_ERR_HIP;
        } else {
            st = launch_direct(q, t, r.next_row, r.job.row_end, &ends[0]);
        }
        nends = 1;
        r.next_row = r.job.row_end;
        r.launches_left += 1;
        r.all_launched = true;
        q->waiting.erase(lone ? q->waiting.begin() : big);
        tickets.push_back(t);
        q->last_direct = !lone;
    } else {
        q->last_direct = false;
        int64_t small_px = 0;
        int nsmall = 0;
        for (uint64_t t : q->waiting) {
            const int64_t left = pixels_left(q->reqs[t]);
            if (left < kDirectPixels) small_px += left, ++nsmall;
        }
        int64_t budget = std::max(q->step_pixels, std::min(64 * q->step_pixels, small_px / 4));
        const int64_t share = std::max<int64_t>(1, budget / (int64_t)std::max(nsmall, 1));
        std::vector<Job> jobs;
        std::deque<uint64_t> still;
        for (uint64_t t : q->waiting) {
            QueueReq& r = q->reqs[t];
            if (budget <= 0 || pixels_left(r) >= kDirectPixels) {
                still.push_back(t);
                continue;
            }
            const Job& w = r.job;
            const int64_t row_px = (int64_t)w.width;
            const int rb = r.next_row;
            Job band = w;
            band.row_begin = rb;
            band.row_end = w.row_end;
            const int64_t unit = min_run_rows(band);  // shortest band worth a tile
            const int64_t want_rows =
                std::max<int64_t>(unit, std::min<int64_t>(share, budget) / std::max<int64_t>(row_px, 1));
            const int re = (int)std::min<int64_t>(w.row_end, rb + want_rows);
            band.row_end = re;
            jobs.push_back(band);
            tickets.push_back(t);
            r.next_row = re;
            r.launches_left += 1;
            budget -= (int64_t)(re - rb) * row_px;
            if (re >= w.row_end)
                r.all_launched = true;
            else
                still.push_back(t);
        }
        q->waiting.swap(still);
        if (jobs.empty()) return 0;
        if (q->fail_next > 0) {
            --q->fail_next;
            st = OILPAINT_ERR_HIP;
        } else if (jobs.size() == 1) {
            st = launch_direct(q, tickets[0], jobs[0].row_begin, jobs[0].row_end, &ends[0]);
            nends = 1;
        } else {
            shape_rows(jobs, q->device);
            Layout L;
            build_layout(jobs, L);
            st = enqueue_layout(L, q->device, *q->ring, *q->branches, q->stream, false, ends, &nends);
        }
    }
    if (st != OILPAINT_OK) {
        fail_launch(q, tickets, st);
        return 1;
    }
    Inflight f;
    for (int i = 0; i < nends; ++i) {
        hipEvent_t ev = nullptr;
        if (!q->free_events.empty()) {
            ev = q->free_events.back();
            q->free_events.pop_back();
        } else if (note_hip("hipEventCreate", hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
            ev = nullptr;
        }
        if (ev && note_hip("hipEventRecord", hipEventRecord(ev, ends[i])) != hipSuccess) {
            q->free_events.push_back(ev);
            ev = nullptr;
        }
        if (!ev) {
            // the launch is enqueued but cannot be tracked: wait for it, then
            // fail its requests
            for (int k = 0; k < nends; ++k) (void)hipStreamSynchronize(ends[k]);
            for (hipEvent_t e : f.evs) q->free_events.push_back(e);
            fail_launch(q, tickets, OILPAINT_ERR_HIP);
            return 1;
        }
        f.evs.push_back(ev);
    }
    f.tickets = tickets;
    q->inflight.push_back(f);
    return 1;
}

int queue_progress(oilpaint_queue* q) {
    const int rs = retire(q, false);
    if (rs != OILPAINT_OK) return rs;
    int launched = 0;
    while (q->inflight.size() < (size_t)kQueueDepth && !q->waiting.empty()) {
        const int st = launch_step(q);
        if (st < 0) return st;
        if (st == 0) break;
        launched += st;
    }
    return launched;
}

}  // namespace

extern "C" {

int oilpaint_batch(const oilpaint_desc* descs, int n, void* stream, int* bad_index) {
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return OILPAINT_ERR_HIP;
    std::vector<Job> jobs;
    int st = collect_jobs(descs, n, device, jobs, bad_index);
    if (st != OILPAINT_OK || jobs.empty()) return st;
    Layout L;
    build_layout(jobs, L);
    std::lock_guard<std::mutex> lock(ring_mutex(device));
    return enqueue_layout(L, device, device_ring(device), device_branches(device), (hipStream_t)stream, true,
                          nullptr, nullptr);
}

// ---------------------------------------------------------------------------
// Batches without allocation: the argument block (class counters, tile
// prefix sums, job descriptors) lives in a file-scope device array instead
// of the library's argument ring.  Each GPU holds its own copy of the array
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
}  // extern "C"

namespace oilpaint_impl {
namespace {

static __device__ __align__(256) uint8_t scratch[OILPAINT_NOALLOC_SCRATCH_BYTES];

// Per-device set-up, made once per device with that device current: the
// array's address on that device, and a host staging block of the same size
// (pageable, so that an upload from it completes before hipMemcpyAsync
// returns and the block may be refilled at once).
struct NoAllocDevice {
    uint8_t* dev = nullptr;
    std::vector<uint8_t> host;
};

NoAllocDevice* noalloc_device(int device) {
    static std::mutex mu;
    static std::map<int, NoAllocDevice> m;
    std::lock_guard<std::mutex> lock(mu);
    auto it = m.find(device);
    if (it != m.end()) return &it->second;
    void* p = nullptr;
    if (note_hip("hipGetSymbolAddress", hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess || !p)
        return nullptr;
    NoAllocDevice& d = m[device];
    d.dev = static_cast<uint8_t*>(p);
    d.host.assign(OILPAINT_NOALLOC_SCRATCH_BYTES, 0);
    if (!device_branches(device).ensure(kMaxBranches - 1)) {
        (void)note_hip("branch streams", hipGetLastError());
        m.erase(device);
        return nullptr;
    }
    return &d;
}

}  // namespace
}  // namespace oilpaint_impl

extern "C" {

int oilpaint_batch_noalloc(const oilpaint_desc* descs, int n, void* stream, int* bad_index) {
    int device = 0;
    if (note_hip("hipGetDevice", hipGetDevice(&device)) != hipSuccess) return OILPAINT_ERR_HIP;
    std::vector<Job> jobs;
    int st = collect_jobs(descs, n, device, jobs, bad_index);
    if (st != OILPAINT_OK || jobs.empty()) return st;
    Layout L;
    build_layout(jobs, L);
    if (L.bytes > (size_t)OILPAINT_NOALLOC_SCRATCH_BYTES) {
        char text[160];
        std::snprintf(text, sizeof(text),
                      "oilpaint_batch_noalloc: argument block of %zu bytes exceeds the %d-byte static scratch",
                      L.bytes, OILPAINT_NOALLOC_SCRATCH_BYTES);
        note_error(text);
        return OILPAINT_ERR_ARG;
    }
    std::lock_guard<std::mutex> lock(ring_mutex(device));
    NoAllocDevice* d = noalloc_device(device);
    if (!d) return OILPAINT_ERR_HIP;
    pack_args(L, d->host.data());
    const hipStream_t s = (hipStream_t)stream;
    if (note_hip("hipMemcpyAsync", hipMemcpyAsync(d->dev, d->host.data(), L.bytes, hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return OILPAINT_ERR_HIP;
    // the counters are cleared by enqueue_classes' reset kernel
    return enqueue_classes(L, d->dev, device, device_branches(device), s, true, nullptr, nullptr, nullptr);
}

int oilpaint_plan_create(const oilpaint_desc* descs, int n, void* stream, oilpaint_plan** out, int* bad_index) {
    if (!out) return OILPAINT_ERR_NULL;
    *out = nullptr;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return OILPAINT_ERR_HIP;
    std::vector<Job> jobs;
    int st = collect_jobs(descs, n, device, jobs, bad_index);
    if (st != OILPAINT_OK) return st;
    std::unique_ptr<oilpaint_plan> p(new oilpaint_plan);
    p->device = device;
    build_layout(jobs, p->layout);
    const size_t bytes = std::max<size_t>(p->layout.bytes, 256);
    if (hipMalloc(&p->dev, bytes) != hipSuccess) return OILPAINT_ERR_NOMEM;
    std::vector<uint8_t> host(bytes);
    pack_args(p->layout, host.data());
    if (hipMemcpy(p->dev, host.data(), p->layout.bytes, hipMemcpyHostToDevice) != hipSuccess) return OILPAINT_ERR_HIP;
    if (p->layout.ntiles > 0) {
        hipStream_t cap;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return OILPAINT_ERR_HIP;
        hipGraph_t g = nullptr;
        bool ok = false, ended = false;
        {
            Branches br;
            ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
            // counters are cleared by a kernel, not a memset node
            ok = ok && enqueue_classes(p->layout, p->dev, device, br, cap, true, &p->grid, nullptr, nullptr) ==
                           OILPAINT_OK;
            ended = hipStreamEndCapture(cap, &g) == hipSuccess;
        }
        (void)hipStreamDestroy(cap);
        if (!ok || !ended || !g) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return OILPAINT_ERR_HIP;
        }
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) return OILPAINT_ERR_HIP;
    }
    (void)stream;
    *out = p.release();
    return OILPAINT_OK;
}

int oilpaint_plan_launch(oilpaint_plan* plan, void* stream) {
    if (!plan) return OILPAINT_ERR_NULL;
    if (!plan->exec) return OILPAINT_OK;  // nothing to compute
    return hipGraphLaunch(plan->exec, (hipStream_t)stream) == hipSuccess ? OILPAINT_OK : OILPAINT_ERR_HIP;
}

int oilpaint_plan_info(const oilpaint_plan* plan, int* tiles, int* workgroups) {
    if (!plan) return OILPAINT_ERR_NULL;
    if (tiles) *tiles = plan->layout.ntiles;
    if (workgroups) *workgroups = plan->grid;
    return OILPAINT_OK;
}

int oilpaint_plan_destroy(oilpaint_plan* plan) {
    delete plan;  // its graph and device block with it
    return OILPAINT_OK;
}

int oilpaint_queue_create(int capacity, int64_t step_pixels, oilpaint_queue** out) {
    if (!out) return OILPAINT_ERR_NULL;
    *out = nullptr;
    if (capacity < 1 || step_pixels < 0) return OILPAINT_ERR_ARG;
    std::unique_ptr<oilpaint_queue> q(new oilpaint_queue);
    if (hipGetDevice(&q->device) != hipSuccess) return OILPAINT_ERR_HIP;
    if (hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking) != hipSuccess) return OILPAINT_ERR_HIP;
    q->capacity = capacity;
    q->step_pixels = step_pixels > 0 ? step_pixels : (int64_t)8 << 20;
    q->ring.reset(new ArgRing(kQueueDepth + 2));
    q->branches.reset(new Branches);
    *out = q.release();
    return OILPAINT_OK;
}

int oilpaint_queue_push(oilpaint_queue* q, const oilpaint_desc* desc, uint64_t* ticket) {
    if (!q || !desc || !ticket) return OILPAINT_ERR_NULL;
    const int rs = retire(q, false);
    if (rs != OILPAINT_OK) return rs;
    if ((int)q->held >= q->capacity) return OILPAINT_ERR_FULL;
    Job j;
    bool empty = false;
    int st = make_job(*desc, nullptr, q->device, j, empty);
    if (st == OILPAINT_OK && !empty) st = batch_shape(j, q->device);
    if (st == OILPAINT_OK && !empty) st = check_device_ptr(j.src);
    if (st == OILPAINT_OK && !empty) st = check_device_ptr(j.dst);
    if (st != OILPAINT_OK) return st;
    const uint64_t t = q->next_ticket++;
    QueueReq r;
    r.job = j;
    r.desc = *desc;
    r.next_row = j.row_begin;
    r.all_launched = empty;
    r.done = empty;
    q->reqs[t] = r;
    if (!empty) {
        q->waiting.push_back(t);
        ++q->held;
    } else {
        q->finished.push_back(t);
    }
    *ticket = t;
    // The request is accepted: an error of the progress step below recurs
    // on the next step, poll or completed call, which reports it.
    (void)queue_progress(q);
    return OILPAINT_OK;
}

int oilpaint_queue_step(oilpaint_queue* q) {
    if (!q) return OILPAINT_ERR_NULL;
    return queue_progress(q);
}

int oilpaint_queue_poll(oilpaint_queue* q, uint64_t ticket) {
    if (!q) return OILPAINT_ERR_NULL;
    auto it = q->reqs.find(ticket);
    if (it == q->reqs.end()) return OILPAINT_ERR_ARG;
    if (!it->second.done) {
        const int st = queue_progress(q);
        if (st < 0) return st;
        if (!it->second.done) return 0;
    }
    // reported complete (or failed): the ticket is forgotten
    const int status = it->second.status;
    q->reqs.erase(it);
    if (q->finished.size() > 2 * (size_t)q->capacity + 1024) {
        std::deque<uint64_t> keep;
        for (uint64_t t : q->finished)
            if (q->reqs.count(t)) keep.push_back(t);
        q->finished.swap(keep);
    }
    return status != OILPAINT_OK ? status : 1;
}

int oilpaint_queue_completed(oilpaint_queue* q, uint64_t* tickets, int* status, int max) {
    if (!q || (!tickets && max > 0)) return OILPAINT_ERR_NULL;
    if (max < 0) return OILPAINT_ERR_ARG;
    const int st = queue_progress(q);
    if (st < 0) return st;
    int n = 0;
    while (n < max && !q->finished.empty()) {
        const uint64_t t = q->finished.front();
        q->finished.pop_front();
        auto it = q->reqs.find(t);
        if (it == q->reqs.end()) continue;  // already reported by poll
        if (status) status[n] = it->second.status;
        tickets[n++] = t;
        q->reqs.erase(it);
    }
    return n;
}

int oilpaint_queue_drain(oilpaint_queue* q) {
    if (!q) return OILPAINT_ERR_NULL;
    for (;;) {
        const int st = queue_progress(q);
        if (st < 0) return st;
        if (q->inflight.empty() && q->waiting.empty()) return OILPAINT_OK;
        const int rs = retire(q, true);
        if (rs != OILPAINT_OK) return rs;
    }
}

void* oilpaint_queue_stream(oilpaint_queue* q) { return q ? (void*)q->stream : nullptr; }

int oilpaint_queue_fail_next(oilpaint_queue* q, int n) {
    if (!q) return OILPAINT_ERR_NULL;
    if (n < 0) return OILPAINT_ERR_ARG;
    q->fail_next = n;
    return OILPAINT_OK;
}

int oilpaint_queue_destroy(oilpaint_queue* q) {
    if (!q) return OILPAINT_OK;
    (void)hipStreamSynchronize(q->stream);
    q->branches.reset();  // synchronizes the side streams
    for (auto& f : q->inflight)
        for (hipEvent_t e : f.evs) (void)hipEventDestroy(e);
    for (auto e : q->free_events) (void)hipEventDestroy(e);
    q->ring.reset();
    (void)hipStreamDestroy(q->stream);
    delete q;
    return OILPAINT_OK;
}

}  // extern "C"
