// Serving loop: continuous batching of correlation requests (include/dic.h,
// "Serving").
//
// References are library contexts made resident once.  Each request gets its
// own frame scratch (deformed coefficients, parent keys, frontier lists, wave
// sizes, seed buffers) from a per-reference reuse pool, so steady-state
// admission allocates nothing.  A launch step runs one wave kernel per group of
// active requests with the same shape, threads per subset and reduction
// precision; every request in it is at its own wave (step - k_base).  The host
// reads the size of each request's next wave once per dic_server_step call and
// retires the requests whose propagation has ended.
#include "dic_context.h"

#include <deque>
#include <map>
#include <tuple>
#include <unordered_map>

using namespace dicmi;

namespace {

constexpr int kMaxSeeds = 64;
constexpr int kMaxActive = 64;

// Device scratch of one request, sized for one reference context.
struct ReqBuf {
    dic_ctx *ref = nullptr;
    void *dcoef_base = nullptr;
    uint64_t *pkey = nullptr;
    int32_t *list0 = nullptr, *list1 = nullptr, *counts = nullptr;
    double *seed_p = nullptr;
    int32_t *seed_nodes = nullptr;
    int32_t *centre = nullptr;
    double *zbuf = nullptr;
    unsigned long long *stat = nullptr;
    FrameState *d_frame = nullptr;
    // pinned host staging of the seed nodes, search centres and frame record,
    // read by asynchronous copies while the request is active
    char *h_stage = nullptr;
    size_t bytes = 0;
};

constexpr size_t kStageBytes = sizeof(FrameState) + sizeof(int32_t) * 3 * kMaxSeeds;

struct Request {
    int64_t ticket = 0;
    dic_ctx *ref = nullptr;
    int32_t ref_id = -1;
    dic_image def{};
    std::vector<dic_seed> seeds;
    dic_result out{};
    int state = 0;  // 0 waiting, 1 active, 2 done
    dic_status result = DIC_OK;
    ReqBuf *buf = nullptr;
    FrameState F{};
    int slot = -1;  // index into the gather array while active
    dic_stats stats{};
};

size_t request_bytes(const dic_ctx *c)
{
    const size_t esz = c->prm.coef_fp16 ? sizeof(__half) : sizeof(float);
    const size_t side = 2 * static_cast<size_t>(c->prm.seed_radius) + 1;
    return c->coef_elems() * esz + static_cast<size_t>(c->nodes) * (8 + 4 + 4) +
           (static_cast<size_t>(c->nodes) + 2) * 4 + kMaxSeeds * (16 + 4 + 8 + 8 * side * side) + 32 +
           sizeof(FrameState);
}

// Device bytes dic_set_reference allocates for an image of W x H pixels.
size_t reference_bytes(int W, int H, int pixel, const dic_params &p)
{
    const int64_t nx = (W - p.subset_size) / p.step + 1, ny = (H - p.subset_size) / p.step + 1;
    const size_t nodes = static_cast<size_t>(nx) * ny;
    const size_t cpitch = round_up(W + 2 * kPad, 64), ppitch = round_up(W, 64);
    return cpitch * (H + 2 * kPad) * sizeof(float) + ppitch * H * sizeof(float) * 4 +
           sizeof(double) * cache_slots(p.shape) * nodes + nodes + static_cast<size_t>(W) * pixel_size(pixel) * H +
           sizeof(int32_t) * (nodes + 130) + sizeof(RefView);
}

} // namespace

struct dic_server {
    int device = 0;
    hipStream_t stream = nullptr;
    dic_server_params prm{};
    std::string err;
    std::vector<dic_ctx *> refs;        // nullptr once removed
    std::vector<double> ref_size;       // bytes counted for each reference
    std::deque<Request *> waiting;
    std::vector<Request *> active;
    std::unordered_map<int64_t, Request *> all;
    std::map<dic_ctx *, std::vector<ReqBuf *>> pool;
    int64_t next_ticket = 1, submitted = 0, admitted = 0, completed = 0;
    int step = 0;
    double ref_bytes = 0, active_bytes = 0, pool_bytes = 0;
    FrameState *d_frames = nullptr;   // device copies of the active frames (gather)
    int32_t *d_next = nullptr;
    int32_t *h_next = nullptr;        // pinned
    FrameState *h_frames = nullptr;   // pinned
    hipStream_t stream2 = nullptr;    // second launch chain (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

#define SFAIL(code, ...)                                                                                              \
    do {                                                                                                              \
        char buf_[512];                                                                                               \
        snprintf(buf_, sizeof(buf_), __VA_ARGS__);                                                                    \
        s->err = buf_;                                                                                                \
        return code;                                                                                                  \
    } while (0)

#define SHIP(expr)                                                                                                    \
    do {                                                                                                              \
        hipError_t e_ = (expr);                                                                                       \
        if (e_ != hipSuccess) {                                                                                       \
            if (e_ == hipErrorOutOfMemory) SFAIL(DIC_E_NOMEM, "%s: %s", #expr, hipGetErrorString(e_));              \
            SFAIL(DIC_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_));                                             \
        }                                                                                                             \
    } while (0)

namespace {

void free_buf(ReqBuf *b)
{
    dfree(b->dcoef_base);
    dfree(b->pkey);
    dfree(b->list0);
    dfree(b->list1);
    dfree(b->counts);
    dfree(b->seed_p);
    dfree(b->seed_nodes);
    dfree(b->centre);
    dfree(b->zbuf);
    dfree(b->stat);
    dfree(b->d_frame);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    delete b;
}

dic_status alloc_buf(dic_server *s, dic_ctx *c, ReqBuf **out)
{
    ReqBuf *b = new ReqBuf();
    b->ref = c;
    b->bytes = request_bytes(c);
    const size_t esz = c->prm.coef_fp16 ? sizeof(__half) : sizeof(float);
    const int side = 2 * c->prm.seed_radius + 1;
    hipError_t e = hipSuccess;
    e = e ? e : hipMalloc(&b->dcoef_base, c->coef_elems() * esz);
    e = e ? e : hipMalloc(&b->pkey, sizeof(uint64_t) * c->nodes);
    e = e ? e : hipMalloc(&b->list0, sizeof(int32_t) * c->nodes);
    e = e ? e : hipMalloc(&b->list1, sizeof(int32_t) * c->nodes);
    e = e ? e : hipMalloc(&b->counts, sizeof(int32_t) * (c->nodes + 2));
    e = e ? e : hipMalloc(&b->seed_p, sizeof(double) * 2 * kMaxSeeds);
    e = e ? e : hipMalloc(&b->seed_nodes, sizeof(int32_t) * kMaxSeeds);
    e = e ? e : hipMalloc(&b->centre, sizeof(int32_t) * 2 * kMaxSeeds);
    e = e ? e : hipMalloc(&b->zbuf, sizeof(double) * kMaxSeeds * side * side);
    e = e ? e : hipMalloc(&b->stat, sizeof(unsigned long long) * 4);
    e = e ? e : hipMalloc(&b->d_frame, sizeof(FrameState));
    e = e ? e : hipHostMalloc(reinterpret_cast<void **>(&b->h_stage), kStageBytes);
    if (e != hipSuccess) {
        free_buf(b);
        SFAIL(e == hipErrorOutOfMemory ? DIC_E_NOMEM : DIC_E_DEVICE, "request scratch: %s", hipGetErrorString(e));
    }
    *out = b;
    return DIC_OK;
}

// Give up pooled (idle) scratch until `need` more bytes fit the budget.
void trim_pool(dic_server *s, double need)
{
    for (auto &kv : s->pool) {
        auto &v = kv.second;
        while (!v.empty() && s->ref_bytes + s->active_bytes + s->pool_bytes + need > s->prm.hbm_budget_bytes) {
            s->pool_bytes -= v.back()->bytes;
            free_buf(v.back());
            v.pop_back();
        }
    }
}

// Seed nodes of a request on its reference's active nodes, de-duplicated, with
// the integer search centre of each.
void request_seeds(const Request *r, std::vector<int32_t> &nodes, std::vector<int32_t> &centre)
{
    for (const dic_seed &sd : r->seeds) {
        const int64_t node = snap_seed(r->ref, sd.x, sd.y);
        if (node < 0) continue;
        bool dup = false;
        for (int32_t q : nodes) dup = dup || q == node;
        if (dup) continue;
        nodes.push_back(static_cast<int32_t>(node));
        centre.push_back(static_cast<int32_t>(std::lround(sd.u0)));
        centre.push_back(static_cast<int32_t>(std::lround(sd.v0)));
    }
}

// Start a request: scratch from the pool (or a new allocation), deformed
// prefilter, frame initialisation, seed search.  Everything is queued on the
// server stream; nothing waits.
dic_status admit(dic_server *s, Request *r, const std::vector<int32_t> &nodes, const std::vector<int32_t> &centre)
{
    dic_ctx *c = r->ref;
    hipStream_t st = s->stream;
    ReqBuf *b = nullptr;
    auto &pl = s->pool[c];
    if (!pl.empty()) {
        b = pl.back();
        pl.pop_back();
        s->pool_bytes -= b->bytes;
    } else {
        trim_pool(s, static_cast<double>(request_bytes(c)));
        dic_status rc = alloc_buf(s, c, &b);
        if (rc != DIC_OK) return rc;
    }
    r->buf = b;
    s->active_bytes += b->bytes;

    FrameState &F = r->F;
    const size_t esz = c->prm.coef_fp16 ? sizeof(__half) : sizeof(float);
    F.dcoef = static_cast<char *>(b->dcoef_base) + (kPad * c->cpitch + kPad) * esz;
    F.dpitch = c->cpitch;
    F.draw = r->def.data;
    F.draw_pitch = r->def.pitch_bytes;
    F.dpixel = r->def.pixel;
    F.p = r->out.p;
    F.zncc = r->out.zncc;
    F.iters = r->out.iters;
    F.status = r->out.status;
    F.wave = r->out.wave;
    F.pkey = b->pkey;
    F.list0 = b->list0;
    F.list1 = b->list1;
    F.counts = b->counts;
    F.seed_p = b->seed_p;
    F.seed_nodes = b->seed_nodes;
    F.nseeds = static_cast<int32_t>(nodes.size());
    F.stat = b->stat;
    F.ref = c->d_view;
    F.k_base = s->step;
    F.kmax = static_cast<int>(c->nodes + 1);
    const int ns = static_cast<int>(nodes.size());
    std::memcpy(b->h_stage, &F, sizeof(FrameState));
    int32_t *hs = reinterpret_cast<int32_t *>(b->h_stage + sizeof(FrameState));
    std::memcpy(hs, nodes.data(), sizeof(int32_t) * ns);
    std::memcpy(hs + kMaxSeeds, centre.data(), sizeof(int32_t) * 2 * ns);

    RefView R = c->view();
    launch_prefilter(r->def.data, r->def.pitch_bytes, r->def.pixel, c->W, c->H, c->tmp, c->tpitch,
                     const_cast<void *>(F.dcoef), c->cpitch, c->prm.coef_fp16 != 0, st);
    launch_init_frame(R, F, c->np, st);
    SHIP(hipMemsetAsync(b->stat, 0, sizeof(unsigned long long) * 4, st));
    SHIP(hipMemcpyAsync(b->d_frame, b->h_stage, sizeof(FrameState), hipMemcpyHostToDevice, st));
    SHIP(hipMemcpyAsync(b->seed_nodes, hs, sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    SHIP(hipMemcpyAsync(b->centre, hs + kMaxSeeds, sizeof(int32_t) * 2 * ns, hipMemcpyHostToDevice, st));
    launch_seed_search(R, b->d_frame, 1, ns, c->prm.seed_radius, b->centre, b->zbuf, st);
    launch_seed_pick(R, b->d_frame, 1, ns, c->prm.seed_radius, b->centre, b->zbuf, st);
    SHIP(hipGetLastError());
    return DIC_OK;
}

void release(dic_server *s, Request *r)
{
    if (r->buf) {
        s->active_bytes -= r->buf->bytes;
        s->pool[r->ref].push_back(r->buf);
        s->pool_bytes += r->buf->bytes;
        r->buf = nullptr;
    }
}

} // namespace

extern "C" {

dic_status dic_server_create(dic_server **out, int device, void *hip_stream, const dic_server_params *prm)
{
    if (!out || !prm) return DIC_E_INVAL;
    *out = nullptr;
    if (prm->max_active < 1 || prm->max_active > kMaxActive || !(prm->hbm_budget_bytes > 0)) return DIC_E_INVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return DIC_E_DEVICE;
    if (device < 0 || device >= ndev) return DIC_E_INVAL;
    if (hipSetDevice(device) != hipSuccess) return DIC_E_DEVICE;
    dic_server *s = new dic_server();
    s->device = device;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->prm = *prm;
    if (hipMalloc(&s->d_frames, sizeof(FrameState) * kMaxActive) != hipSuccess ||
        hipMalloc(&s->d_next, sizeof(int32_t) * kMaxActive) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&s->h_next), sizeof(int32_t) * kMaxActive) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&s->h_frames), sizeof(FrameState) * kMaxActive) != hipSuccess) {
        dfree(s->d_frames);
        dfree(s->d_next);
        if (s->h_next) (void)hipHostFree(s->h_next);
        delete s;
        return DIC_E_NOMEM;
    }
    *out = s;
    return DIC_OK;
}

const char *dic_server_last_error(const dic_server *s) { return s ? s->err.c_str() : "null server"; }

dic_status dic_server_add_reference(dic_server *s, const dic_image *ref, const uint8_t *roi_mask_dev,
                                    const dic_params *prm, int32_t *ref_id)
{
    if (!s || !ref_id) return DIC_E_INVAL;
    s->err.clear();
    if (!ref || !prm) SFAIL(DIC_E_INVAL, "reference image or params is NULL");
    if (prm->shape == DIC_SHAPE_RIGID || prm->cost != DIC_COST_ZNSSD || prm->lm_lambda != 0.0)
        SFAIL(DIC_E_UNSUPPORTED, "the serving loop runs ZNSSD with the affine or quadratic shape and lm_lambda 0");
    if (ref->width >= prm->subset_size && ref->height >= prm->subset_size && prm->step >= 1 &&
        (prm->shape == DIC_SHAPE_AFFINE || prm->shape == DIC_SHAPE_QUADRATIC)) {
        // budget check before anything is allocated; idle pooled scratch goes first
        const double bytes = static_cast<double>(reference_bytes(ref->width, ref->height, ref->pixel, *prm));
        if (s->ref_bytes + s->active_bytes + s->pool_bytes + bytes > s->prm.hbm_budget_bytes) trim_pool(s, bytes);
        if (s->ref_bytes + s->active_bytes + s->pool_bytes + bytes > s->prm.hbm_budget_bytes)
            SFAIL(DIC_E_NOMEM, "reference of %.0f MB exceeds the HBM budget (%.0f MB in use)", bytes / 1e6,
                  (s->ref_bytes + s->active_bytes) / 1e6);
    }
    SHIP(hipSetDevice(s->device));
    dic_ctx *c = nullptr;
    dic_status rc = dic_create(&c, s->device, s->stream);
    if (rc != DIC_OK) SFAIL(rc, "context creation failed");
    rc = dic_set_reference(c, ref, roi_mask_dev, prm);
    if (rc != DIC_OK) {
        s->err = c->err;
        dic_destroy(c);
        return rc;
    }
    const double bytes = static_cast<double>(reference_bytes(c->W, c->H, c->ref_pixel, c->prm));
    s->ref_bytes += bytes;
    s->refs.push_back(c);
    s->ref_size.push_back(bytes);
    *ref_id = static_cast<int32_t>(s->refs.size() - 1);
    return DIC_OK;
}

dic_status dic_server_remove_reference(dic_server *s, int32_t ref_id)
{
    if (!s) return DIC_E_INVAL;
    s->err.clear();
    if (ref_id < 0 || ref_id >= static_cast<int32_t>(s->refs.size()) || !s->refs[ref_id])
        SFAIL(DIC_E_INVAL, "unknown reference %d", ref_id);
    dic_ctx *c = s->refs[ref_id];
    for (const Request *r : s->waiting)
        if (r->ref == c) SFAIL(DIC_E_STATE, "reference %d has waiting requests", ref_id);
    for (const Request *r : s->active)
        if (r->ref == c) SFAIL(DIC_E_STATE, "reference %d has active requests", ref_id);
    SHIP(hipSetDevice(s->device));
    auto it = s->pool.find(c);
    if (it != s->pool.end()) {
        for (ReqBuf *b : it->second) {
            s->pool_bytes -= b->bytes;
            free_buf(b);
        }
        s->pool.erase(it);
    }
    // finished requests keep their ticket but no longer point at the context
    for (auto &kv : s->all)
        if (kv.second->ref == c) kv.second->ref = nullptr;
    dic_destroy(c);
    s->refs[ref_id] = nullptr;
    s->ref_bytes -= s->ref_size[ref_id];
    return DIC_OK;
}

dic_status dic_server_submit(dic_server *s, int32_t ref_id, const dic_image *def, const dic_seed *seeds,
                             int32_t nseeds, dic_result *out, int64_t *ticket)
{
    if (!s || !ticket) return DIC_E_INVAL;
    s->err.clear();
    if (ref_id < 0 || ref_id >= static_cast<int32_t>(s->refs.size()) || !s->refs[ref_id])
        SFAIL(DIC_E_INVAL, "unknown reference %d", ref_id);
    dic_ctx *c = s->refs[ref_id];
    if (!def || !def->data) SFAIL(DIC_E_INVAL, "deformed image is NULL");
    if (def->width != c->W || def->height != c->H) SFAIL(DIC_E_INVAL, "deformed image size differs from the reference");
    if (def->pixel < DIC_PIX_U8 || def->pixel > DIC_PIX_F32 ||
        def->pitch_bytes < static_cast<int64_t>(def->width * pixel_size(def->pixel)))
        SFAIL(DIC_E_INVAL, "deformed image layout");
    if (!seeds || nseeds < 1 || nseeds > kMaxSeeds) SFAIL(DIC_E_INVAL, "nseeds %d (1..%d)", nseeds, kMaxSeeds);
    if (!out || !out->p || !out->zncc || !out->iters || !out->status || !out->wave)
        SFAIL(DIC_E_INVAL, "result has a NULL array");
    for (int q = 0; q < nseeds; ++q)
        if (!std::isfinite(seeds[q].x) || !std::isfinite(seeds[q].y) || !std::isfinite(seeds[q].u0) ||
            !std::isfinite(seeds[q].v0))
            SFAIL(DIC_E_INVAL, "seed %d is not finite", q);
    Request *r = new Request();
    r->ticket = s->next_ticket++;
    r->ref = c;
    r->ref_id = ref_id;
    r->def = *def;
    r->seeds.assign(seeds, seeds + nseeds);
    r->out = *out;
    s->waiting.push_back(r);
    s->all[r->ticket] = r;
    ++s->submitted;
    *ticket = r->ticket;
    return DIC_OK;
}

dic_status dic_server_step(dic_server *s, int32_t steps)
{
    if (!s) return DIC_E_INVAL;
    s->err.clear();
    if (steps < 1 || steps > 256) SFAIL(DIC_E_INVAL, "steps %d (1..256)", steps);
    SHIP(hipSetDevice(s->device));
    hipStream_t st = s->stream;

    // ---- admission, FIFO: a request that cannot fit even beside its own reference
    // alone fails; one that does not fit now waits (for active requests to finish,
    // or for the caller to remove references)
    while (!s->waiting.empty() && static_cast<int>(s->active.size()) < s->prm.max_active) {
        Request *r = s->waiting.front();
        const double need = static_cast<double>(request_bytes(r->ref));
        const bool pooled = !s->pool[r->ref].empty();
        if (!pooled && s->ref_size[r->ref_id] + need > s->prm.hbm_budget_bytes) {
            s->waiting.pop_front();
            r->state = 2;
            r->result = DIC_E_NOMEM;
            ++s->completed;
            continue;
        }
        if (!pooled && s->ref_bytes + s->active_bytes + need > s->prm.hbm_budget_bytes) {
            trim_pool(s, need);
            if (s->ref_bytes + s->active_bytes + need > s->prm.hbm_budget_bytes) break;
        }
        s->waiting.pop_front();
        std::vector<int32_t> nodes, centre;
        request_seeds(r, nodes, centre);
        if (nodes.empty()) {   // no seed on an active node: done without propagation
            r->state = 2;
            r->result = DIC_E_NOSEED;
            ++s->completed;
            continue;
        }
        dic_status rc = admit(s, r, nodes, centre);
        if (rc != DIC_OK) {
            release(s, r);
            r->state = 2;
            r->result = rc;
            ++s->completed;
            if (rc == DIC_E_DEVICE) return rc;
            continue;
        }
        ++s->admitted;
        r->state = 1;
        s->active.push_back(r);
    }

    // ---- launch steps: one launch per (shape, threads per subset, precision) group
    // and launch chain.  The requests are independent, so with two or more active
    // ones every group is split into two chains on two streams (alternate requests):
    // a request's waves stay in order on its chain's stream, and one chain's launch
    // fills the GPU while the other's last workgroups finish.
    std::map<std::tuple<int, int, int>, std::vector<Request *>> groups[2];
    const int nchain = s->active.size() >= 2 ? 2 : 1;
    if (nchain == 2 && !s->stream2) {
        SHIP(hipStreamCreateWithFlags(&s->stream2, hipStreamNonBlocking));
        SHIP(hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming));
        SHIP(hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming));
    }
    const hipStream_t chain_stream[2] = {st, nchain == 2 ? s->stream2 : st};
    std::map<std::tuple<int, int, int>, int> seen;
    for (Request *r : s->active) {
        const dic_ctx *c = r->ref;
        const auto key = std::make_tuple(c->np, c->tps, c->prm.reduce_fp64);
        const int nth = seen[key]++;
        groups[nchain == 2 ? nth % 2 : 0][key].push_back(r);
    }
    if (nchain == 2) {
        // the second chain starts after this call's admissions on the serving stream
        SHIP(hipEventRecord(s->ev_fork, st));
        SHIP(hipStreamWaitEvent(s->stream2, s->ev_fork, 0));
    }
    for (int q = 0; q < steps; ++q) {
        for (int ch = 0; ch < nchain; ++ch)
        for (auto &g : groups[ch]) {
            const auto &reqs = g.second;
            for (size_t i0 = 0; i0 < reqs.size(); i0 += kMaxFrames) {
                FrameTable table;
                std::memset(&table, 0, sizeof(table));
                int nmax = 0, tsmax = 0, ldsmax = 0;
                const size_t i1 = std::min(reqs.size(), i0 + kMaxFrames);
                for (size_t i = i0; i < i1; ++i) {
                    table.f[i - i0] = reqs[i]->F;
                    const int n = reqs[i]->ref->prm.subset_size, ts = reqs[i]->ref->window_side();
                    nmax = std::max(nmax, n);
                    tsmax = std::max(tsmax, ts);
                    ldsmax = std::max(ldsmax, ts * lds_pitch(n, ts));
                }
                table.n = static_cast<int>(i1 - i0);
                const int np = std::get<0>(g.first), tps = std::get<1>(g.first);
                // the one-chain grid even with two chains: the serving launches carry few
                // subsets per request, and 8 workgroups per compute unit measured slower
                // there (20 requests/s: p50 291 ms against 256 ms)
                const int grid = wave_grid_hint(np, tps, s->device, 1);
                if (!launch_wave(table, s->step, np, nmax, tps, std::get<2>(g.first) != 0, tsmax, ldsmax, grid,
                                 chain_stream[ch])) {
                    if (nchain == 2) {
                        SHIP(hipEventRecord(s->ev_join, s->stream2));
                        SHIP(hipStreamWaitEvent(st, s->ev_join, 0));
                    }
                    SFAIL(DIC_E_UNSUPPORTED, "no kernel for shape %d, %d threads, subset %d", np, tps, nmax);
                }
            }
        }
        ++s->step;
    }
    if (nchain == 2) {
        // the serving stream continues after both chains
        SHIP(hipEventRecord(s->ev_join, s->stream2));
        SHIP(hipStreamWaitEvent(st, s->ev_join, 0));
    }
    SHIP(hipGetLastError());

    // ---- which requests have an empty next wave: retire them
    const int na = static_cast<int>(s->active.size());
    if (na > 0) {
        for (int i = 0; i < na; ++i) s->h_frames[i] = s->active[i]->F;
        SHIP(hipMemcpyAsync(s->d_frames, s->h_frames, sizeof(FrameState) * na, hipMemcpyHostToDevice, st));
        launch_gather_next(s->d_frames, na, s->step, s->d_next, st);
        SHIP(hipMemcpyAsync(s->h_next, s->d_next, sizeof(int32_t) * na, hipMemcpyDeviceToHost, st));
        SHIP(hipStreamSynchronize(st));
        std::vector<Request *> keep;
        std::vector<Request *> done;
        for (int i = 0; i < na; ++i) (s->h_next[i] == 0 ? done : keep).push_back(s->active[i]);
        for (Request *r : done) {
            RefView R = r->ref->view();
            launch_frame_stats(R, r->F, st);
            launch_finalize(R, r->F, r->ref->np, r->ref->prm.nan_unconverged != 0, st);
        }
        if (!done.empty()) {
            std::vector<unsigned long long> stat(4 * done.size());
            for (size_t i = 0; i < done.size(); ++i)
                SHIP(hipMemcpyAsync(stat.data() + 4 * i, done[i]->buf->stat, sizeof(unsigned long long) * 4,
                                    hipMemcpyDeviceToHost, st));
            SHIP(hipStreamSynchronize(st));
            for (size_t i = 0; i < done.size(); ++i) {
                Request *r = done[i];
                dic_stats &S = r->stats;
                S.nodes = r->ref->nodes;
                S.active = r->ref->active;
                S.computed = static_cast<int64_t>(stat[4 * i]);
                S.converged = static_cast<int64_t>(stat[4 * i + 1]);
                S.iterations = static_cast<int64_t>(stat[4 * i + 2]);
                S.frames = 1;
                S.threads_per_subset = r->ref->tps;
                S.waves = static_cast<int32_t>(stat[4 * i + 3]);
                S.launch_chains = 1;
                release(s, r);
                r->state = 2;
                ++s->completed;
            }
        }
        s->active = keep;
    }
    return DIC_OK;
}

dic_status dic_server_poll(dic_server *s, int64_t ticket, int32_t *done, int32_t *status, dic_stats *st)
{
    if (!s || !done) return DIC_E_INVAL;
    auto it = s->all.find(ticket);
    if (it == s->all.end()) SFAIL(DIC_E_INVAL, "unknown ticket %lld", static_cast<long long>(ticket));
    Request *r = it->second;
    *done = r->state == 2;
    if (status) *status = r->state == 2 ? r->result : DIC_OK;
    if (st) *st = r->stats;
    return DIC_OK;
}

dic_status dic_server_forget(dic_server *s, int64_t ticket)
{
    if (!s) return DIC_E_INVAL;
    s->err.clear();
    auto it = s->all.find(ticket);
    if (it == s->all.end()) SFAIL(DIC_E_INVAL, "unknown ticket %lld", static_cast<long long>(ticket));
    if (it->second->state != 2) SFAIL(DIC_E_STATE, "ticket %lld is not done", static_cast<long long>(ticket));
    delete it->second;
    s->all.erase(it);
    return DIC_OK;
}

dic_status dic_server_get_stats(const dic_server *s, dic_server_stats *out)
{
    if (!s || !out) return DIC_E_INVAL;
    out->submitted = s->submitted;
    out->admitted = s->admitted;
    out->completed = s->completed;
    out->active = static_cast<int32_t>(s->active.size());
    out->waiting = static_cast<int32_t>(s->waiting.size());
    out->steps = s->step;
    out->used_bytes = s->ref_bytes + s->active_bytes;
    out->pool_bytes = s->pool_bytes;
    return DIC_OK;
}

dic_status dic_server_destroy(dic_server *s)
{
    if (!s) return DIC_E_INVAL;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    else (void)hipDeviceSynchronize();
    for (auto &kv : s->all) {
        if (kv.second->buf) free_buf(kv.second->buf);
        delete kv.second;
    }
    for (auto &kv : s->pool)
        for (ReqBuf *b : kv.second) free_buf(b);
    for (dic_ctx *c : s->refs)
        if (c) dic_destroy(c);
    dfree(s->d_frames);
    dfree(s->d_next);
    if (s->h_next) (void)hipHostFree(s->h_next);
    if (s->h_frames) (void)hipHostFree(s->h_frames);
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    if (s->stream2) {
        (void)hipStreamSynchronize(s->stream2);
        (void)hipStreamDestroy(s->stream2);
    }
    delete s;
    return DIC_OK;
}

} // extern "C"
