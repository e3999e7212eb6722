// server.cpp -- the frame server behind nis_server_start ... nis_server_stop.
//
// A scheduler thread admits queued frame requests in arrival order onto a fixed
// set of slots.  A slot is one HIP stream with its own light state (path
// density fields and site tables), query workspace and frame buffers, so frames
// in different slots share nothing writable and each frame's result is the one
// it would get alone.  Admission needs an idle slot and room in the device
// memory budget for the slot's growth and the frame's image; when the budget
// is short the server first frees cached images and the buffers of idle
// slots.  A slot keeps its light fields between frames and skips the sweep
// when the next frame has the same medium, pyramid and light.  Completion is
// observed by polling an event per slot.
//
// With batch_gather, the small grey frames (at most 2^18 pixels) admitted in
// one scheduling pass share their gather: each runs its light fields, camera
// rays and collisions on its own slot's stream, then one launch of the
// gather on the first frame's stream covers every frame's collisions
// (k_features_multi, each frame's medium and light from a table), after
// which each frame's backbone and image run on its own stream again.  Two
// sets of batch buffers let one batch gather while the previous one's
// backbones still read theirs.  Larger frames run alone as before.  A
// frame's image is bit for bit the one it gets alone.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>

#include "runtime.h"

using namespace nis;

namespace {

using Clock = std::chrono::steady_clock;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    hipEvent_t pre = nullptr;        // batch mode: the frame's collisions and light fields are ready
    hipEvent_t read = nullptr;       // batch mode: the frame's backbone has read the batch buffers
    int* pinned_count = nullptr;     // host copy of the frame's collision count
    Workspace ws;
    FrameWork fw;
    LightState ls;
    int32_t medium = 0;              // medium ls was laid out for
    uint64_t req = 0;                // request on the device, 0 when idle
    size_t bytes() const { return ws.bytes() + fw.bytes() + ls.bytes(); }
    void release_buffers()
    {
        ws.release();
        fw.release();
        ls.release();
        ls.valid = false;
        medium = 0;
    }
};

struct Request {
    nis_frame_req req;
    Params P;
    CamArgs C;
    double l[3];
    int32_t status = NIS_QUEUED;
    std::string err;
    double t_submit = 0, t_start = 0, t_done = 0;
    int64_t n_points = 0;
    DevBuf image;
    int slot = -1;
};

}  // namespace

struct Server {
    nis_server_cfg cfg;
    std::vector<Slot> slots;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Request> reqs;
    std::vector<DevBuf> spare_images;
    // batch mode, two sets: descriptors, single-scatter terms, gather table;
    // an event recorded once every backbone of the set's last batch read it
    DevBuf bdesc[2], bf0[2], btab[2];
    hipEvent_t gathered = nullptr, bdone[2] = {nullptr, nullptr};
    bool bdone_rec[2] = {false, false};
    int bset = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread thread;
    std::condition_variable wake;     // submit, release, stop
    std::condition_variable finished; // a frame completed or failed
    Clock::time_point t0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    size_t held() const
    {
        size_t b = 0;
        for (const Slot& s : slots) b += s.bytes();
        for (const auto& kv : reqs) b += kv.second.image.bytes;
        for (const DevBuf& d : spare_images) b += d.bytes;
        for (int i = 0; i < 2; i++) b += bdesc[i].bytes + bf0[i].bytes + btab[i].bytes;
        return b;
    }
};

namespace {

size_t image_bytes(const Request& r)
{
    return (size_t)r.C.width * r.C.height * r.P.channels * sizeof(float);
}

// Device memory a slot must hold to run the request (workspace, frame buffers
// and light fields).
void slot_need(int prec, const Medium* M, const Request& r, size_t* ws, size_t* fw, size_t* ls)
{
    const int64_t npix = (int64_t)r.C.width * r.C.height;
    *ws = workspace_bytes(prec, npix);
    *fw = frame_work_bytes(npix) + (r.P.channels == 3 ? (size_t)npix * 3 * sizeof(float) : 0);
    LightState tmp;
    light_layout(M, r.l, &tmp);
    *ls = (size_t)tmp.rt_floats * sizeof(float) + (size_t)(tmp.pair_count + tmp.dpair_count) * sizeof(float2) +
          sizeof(SiteTables);
}

size_t grow(size_t need, size_t have) { return need > have ? need - have : 0; }

size_t slot_growth(const Server* S, const Slot& s, const Medium* M, const Request& r)
{
    size_t ws, fw, ls;
    slot_need(S->cfg.precision, M, r, &ws, &fw, &ls);
    return grow(ws, s.ws.bytes()) + grow(fw, s.fw.bytes()) + grow(ls, s.ls.bytes());
}

bool same_light(const Slot& s, int32_t medium, const Medium* M, const double l[3])
{
    return s.ls.valid && s.medium == medium && !s.ls.stale && s.ls.swept_version == M->version &&
           s.ls.l[0] == l[0] && s.ls.l[1] == l[1] && s.ls.l[2] == l[2];
}

void fail_request(Server* S, Request& r, int32_t code, const std::string& msg)
{
    r.status = code;
    r.err = msg;
    r.t_done = S->now();
    if (r.image.p) {
        S->spare_images.push_back(r.image);
        r.image = DevBuf();
    }
    S->finished.notify_all();
}

// Observes finished frames.
void retire(nis_ctx* ctx, Server* S)
{
    (void)ctx;
    for (size_t k = 0; k < S->slots.size(); k++) {
        Slot& s = S->slots[k];
        if (!s.req) continue;
        hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) continue;
        Request& r = S->reqs[s.req];
        if (e == hipSuccess) {
            r.status = NIS_OK;
            r.t_done = S->now();
            r.n_points = *s.pinned_count;
            S->finished.notify_all();
        } else {
            fail_request(S, r, NIS_E_DEVICE, std::string("frame failed: ") + hipGetErrorString(e));
        }
        s.req = 0;
    }
}

// Light state and image of request `id` on slot k.
Medium* begin(nis_ctx* ctx, Server* S, int k, uint64_t id)
{
    Slot& s = S->slots[k];
    Request& r = S->reqs[id];
    Medium* M = get_medium(ctx, r.req.medium);
    if (!same_light(s, r.req.medium, M, r.l)) {
        set_light_state(M, r.l, &s.ls);
        s.medium = r.req.medium;
    }
    const size_t ib = image_bytes(r);
    // the smallest spare image that fits, else a new one
    int best = -1;
    for (size_t i = 0; i < S->spare_images.size(); i++)
        if (S->spare_images[i].bytes >= ib && (best < 0 || S->spare_images[i].bytes < S->spare_images[best].bytes))
            best = (int)i;
    if (best >= 0) {
        r.image = S->spare_images[best];
        S->spare_images.erase(S->spare_images.begin() + best);
    } else {
        r.image.reserve(ib, "frame image");
    }
    return M;
}

// The frame of request `id` on slot k is queued up to its image on stream st:
// its count comes back and its completion is recorded there.
void finish(Server* S, int k, uint64_t id, hipStream_t st)
{
    Slot& s = S->slots[k];
    Request& r = S->reqs[id];
    hip_check(hipMemcpyAsync(s.pinned_count, s.fw.count.p, sizeof(int), hipMemcpyDeviceToHost, st),
              "count download");
    hip_check(hipEventRecord(s.done, st), "hipEventRecord");
    r.status = NIS_RUNNING;
    r.slot = k;
    r.t_start = S->now();
    s.req = id;
}

// Queues the whole frame of request `id` on slot k.
void launch(nis_ctx* ctx, Server* S, int k, uint64_t id)
{
    Slot& s = S->slots[k];
    Request& r = S->reqs[id];
    Medium* M = begin(ctx, S, k, id);
    render_frame(s.ws, s.fw, ctx->net, S->cfg.precision, M, &s.ls, r.P, r.C, r.req.seed, r.image.as<float>(),
                 s.stream);
    finish(S, k, id, s.stream);
}

// Queues the frames of `batch` (slot, request) with one gather launch.
constexpr int64_t kBatchPix = 1 << 18;   // the largest frame that shares its gather

void launch_batch(nis_ctx* ctx, Server* S, const std::vector<std::pair<int, uint64_t>>& batch)
{
    const int prec = S->cfg.precision;
    const Net* net = ctx->net;
    const int n = (int)batch.size();
    std::vector<FeatArgs> tab(n);
    FeatMulti fm;
    std::memset(&fm, 0, sizeof(fm));
    fm.n = n;
    int64_t rows = 0, blocks = 0;
    for (int i = 0; i < n; i++) {
        const int k = batch[i].first;
        Slot& s = S->slots[k];
        Request& r = S->reqs[batch[i].second];
        Medium* M = begin(ctx, S, k, batch[i].second);
        CamArgs Cb = r.C;
        Cb.band = kRenderBand;   // as render_frame: collisions in bands of rows
        frame_points(s.fw, M, r.P, Cb, r.req.seed, nullptr, nullptr, nullptr, nullptr, s.stream);
        tab[i] = prepare_feat_args(net, prec, M, &s.ls, r.P, s.stream);
        const FrameBuffers fb = s.fw.view();
        tab[i].pts = fb.cpts;
        tab[i].dirs = fb.cdirs;
        tab[i].npts = (int64_t)r.C.width * r.C.height;
        tab[i].count = fb.count;
        fm.first[i] = (int)blocks;
        blocks += features_blocks(tab[i].npts);
        rows += tab[i].npts;
        hip_check(hipEventRecord(s.pre, s.stream), "hipEventRecord");
    }
    fm.first[n] = (int)blocks;
    const int b = S->bset;
    S->bset ^= 1;
    const hipStream_t bs = S->slots[batch[0].first].stream;
    for (int i = 1; i < n; i++) hip_check(hipStreamWaitEvent(bs, S->slots[batch[i].first].pre, 0), "wait");
    // this buffer set's previous batch: its backbones have read it
    if (S->bdone_rec[b]) hip_check(hipStreamWaitEvent(bs, S->bdone[b], 0), "wait");
    const size_t rb = desc_row_bytes(prec);
    S->bdesc[b].reserve((size_t)rows * rb, "batch descriptors");
    S->bf0[b].reserve((size_t)rows * sizeof(float), "batch single-scatter terms");
    S->btab[b].reserve(sizeof(FeatArgs) * n, "batch table");
    int64_t base = 0;
    for (int i = 0; i < n; i++) {
        tab[i].desc = static_cast<char*>(S->bdesc[b].p) + (size_t)base * rb;
        tab[i].f0 = S->bf0[b].as<float>() + base;
        base += tab[i].npts;
    }
    // the table from pageable memory: the copy has read it when the call returns
    hip_check(hipMemcpyAsync(S->btab[b].p, tab.data(), sizeof(FeatArgs) * n, hipMemcpyHostToDevice, bs),
              "batch table");
    fm.table = S->btab[b].as<FeatArgs>();
    bool big = false;
    for (int i = 0; i < n; i++) big |= big_fields(tab[i].mv);
    hip_check(launch_features_multi(prec, fm, big, bs), "features");
    hip_check(hipEventRecord(S->gathered, bs), "hipEventRecord");
    // each frame's backbone and image on its own stream
    for (int i = 0; i < n; i++) {
        const int k = batch[i].first;
        Slot& s = S->slots[k];
        Request& r = S->reqs[batch[i].second];
        const FrameBuffers fb = s.fw.view();
        if (i > 0) hip_check(hipStreamWaitEvent(s.stream, S->gathered, 0), "wait");
        MlpArgs ma = mlp_args(net, prec);
        ma.x = tab[i].desc;
        ma.npts = tab[i].npts;
        ma.count = fb.count;
        ma.f0 = tab[i].f0;
        ma.radiance = r.P.radiance;
        ma.out = s.fw.L.as<float>();
        ma.albedo_gamma = (float)std::pow((double)r.P.albedo, (double)net->gamma);
        hip_check(launch_mlp(prec, ma, s.stream), "backbone");
        hip_check(hipEventRecord(s.read, s.stream), "hipEventRecord");
        hip_check(launch_image(fb, tab[i].npts, s.fw.L.as<float>(), r.P.albedo, r.image.as<float>(), s.stream),
                  "image");
        finish(S, k, batch[i].second, s.stream);
    }
    for (int i = 1; i < n; i++) hip_check(hipStreamWaitEvent(bs, S->slots[batch[i].first].read, 0), "wait");
    hip_check(hipEventRecord(S->bdone[b], bs), "hipEventRecord");
    S->bdone_rec[b] = true;
}

// Admits queued requests in order while a slot is idle and memory allows.
void admit(nis_ctx* ctx, Server* S)
{
    std::vector<std::pair<int, uint64_t>> batch;   // batch mode: the pass's grey frames
    int64_t batch_pix = 0;
    auto flush = [&] {
        if (batch.empty()) return;
        try {
            launch_batch(ctx, S, batch);
        } catch (const Error& e) {
            for (auto& b : batch) {
                (void)hipStreamSynchronize(S->slots[b.first].stream);   // nothing may still write the image
                S->slots[b.first].req = 0;
                fail_request(S, S->reqs[b.second], e.code, e.msg);
            }
        } catch (...) {
            for (auto& b : batch) {
                (void)hipStreamSynchronize(S->slots[b.first].stream);
                S->slots[b.first].req = 0;
                fail_request(S, S->reqs[b.second], NIS_E_INTERNAL, "internal error");
            }
        }
        batch.clear();
        batch_pix = 0;
    };
    while (!S->queue.empty()) {
        const uint64_t id = S->queue.front();
        Request& r = S->reqs[id];
        auto mit = ctx->media.find(r.req.medium);
        if (mit == ctx->media.end()) {
            S->queue.pop_front();
            fail_request(S, r, NIS_E_STATE, "medium was unloaded");
            continue;
        }
        const Medium* M = mit->second;
        // an idle slot, preferring one that already holds this light
        int k = -1;
        for (size_t i = 0; i < S->slots.size(); i++) {
            if (S->slots[i].req) continue;
            if (k < 0) k = (int)i;
            if (same_light(S->slots[i], r.req.medium, M, r.l)) {
                k = (int)i;
                break;
            }
        }
        if (k < 0) break;
        size_t ib = image_bytes(r), img_growth = ib;
        for (const DevBuf& d : S->spare_images)
            if (d.bytes >= ib) img_growth = 0;
        size_t need = slot_growth(S, S->slots[k], M, r) + img_growth;
        if (S->held() + need > S->cfg.hbm_budget_bytes) {
            for (DevBuf& d : S->spare_images) d.release();
            S->spare_images.clear();
            img_growth = ib;
            need = slot_growth(S, S->slots[k], M, r) + img_growth;
        }
        if (S->held() + need > S->cfg.hbm_budget_bytes) {
            for (size_t i = 0; i < S->slots.size(); i++)
                if ((int)i != k && !S->slots[i].req) S->slots[i].release_buffers();
        }
        if (S->held() + need > S->cfg.hbm_budget_bytes) {
            // the frame fits the budget alone (checked at submit); shrink the
            // chosen slot too if it holds oversized buffers, else wait
            S->slots[k].release_buffers();
            need = slot_growth(S, S->slots[k], M, r) + img_growth;
            if (S->held() + need > S->cfg.hbm_budget_bytes) break;
        }
        S->queue.pop_front();
        const int64_t npix = (int64_t)r.C.width * r.C.height;
        if (S->cfg.batch_gather && r.P.channels == 1 && npix <= kBatchPix) {
            if (batch_pix + npix > kChunk || (int)batch.size() == kMaxBatch) flush();
            batch.emplace_back(k, id);
            batch_pix += npix;
            S->slots[k].req = id;   // taken; begin() and finish() fill in the rest
            continue;
        }
        try {
            launch(ctx, S, k, id);
        } catch (const Error& e) {
            (void)hipStreamSynchronize(S->slots[k].stream);   // nothing may still write the image
            fail_request(S, r, e.code, e.msg);
        } catch (...) {
            (void)hipStreamSynchronize(S->slots[k].stream);
            fail_request(S, r, NIS_E_INTERNAL, "internal error");
        }
    }
    flush();
}

void scheduler(nis_ctx* ctx, Server* S)
{
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(ctx->mu);
    while (!S->stop) {
        retire(ctx, S);
        admit(ctx, S);
        bool busy = false;
        for (const Slot& s : S->slots) busy |= s.req != 0;
        if (busy)
            S->wake.wait_for(lk, std::chrono::microseconds(20));
        else
            S->wake.wait(lk);
    }
}

Server* running(nis_ctx* ctx)
{
    if (!ctx->server) fail(NIS_E_STATE, "no frame server is running");
    return ctx->server;
}

void fill_result(const Request& r, nis_frame_result* out)
{
    out->status = r.status;
    out->width = r.C.width;
    out->height = r.C.height;
    out->channels = r.P.channels;
    out->n_points = r.n_points;
    out->d_image = r.status == NIS_OK ? r.image.as<float>() : nullptr;
    out->t_submit = r.t_submit;
    out->t_start = r.t_start;
    out->t_done = r.t_done;
}

void check(nis_ctx* ctx)
{
    if (!ctx) fail(NIS_E_INVALID, "context is NULL");
    g_prof = nullptr;
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
}

// Validates a request and derives its camera, unit light and parameters.
Request make_request(nis_ctx* ctx, const nis_frame_req* req)
{
    if (!req) fail(NIS_E_INVALID, "req is NULL");
    Medium* M = get_medium(ctx, req->medium);
    Request r;
    r.req = *req;
    r.C = camera_args(&req->camera);
    for (int d = 0; d < 3; d++)
        if (!std::isfinite(req->light_dir[d])) fail(NIS_E_INVALID, "light must be finite");
    if (!std::isfinite(req->radiance)) fail(NIS_E_INVALID, "radiance must be finite");
    if (!(std::isfinite(req->g) && req->g > -1.f && req->g < 1.f)) fail(NIS_E_INVALID, "g must be in (-1,1)");
    double l[3] = {req->light_dir[0], req->light_dir[1], req->light_dir[2]};
    const double nrm = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    if (!(nrm > 0.0)) fail(NIS_E_INVALID, "light direction is zero");
    for (int d = 0; d < 3; d++) r.l[d] = l[d] / nrm;
    r.P = Params{M->sigma_t, M->albedo, single_lobe(req->g), req->radiance, M->volume_phase};
    if (!grey_albedo(M)) {
        // a coloured medium renders an RGB frame (one backbone pass per channel)
        r.P.channels = 3;
        for (int c = 0; c < 3; c++) r.P.rgb[c] = M->albedo_rgb[c];
        r.P.albedo = r.P.rgb[0];
    }
    return r;
}

// Device memory one frame holds: slot buffers plus its image.
size_t frame_need(int prec, const Medium* M, const Request& r)
{
    size_t ws, fw, ls;
    slot_need(prec, M, r, &ws, &fw, &ls);
    return ws + fw + ls + image_bytes(r);
}

void free_server(Server* S)
{
    for (Slot& s : S->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        s.release_buffers();
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.pre) (void)hipEventDestroy(s.pre);
        if (s.read) (void)hipEventDestroy(s.read);
        if (s.pinned_count) (void)hipHostFree(s.pinned_count);
        if (s.stream) (void)hipStreamDestroy(s.stream);
    }
    for (auto& kv : S->reqs) kv.second.image.release();
    for (DevBuf& d : S->spare_images) d.release();
    for (int i = 0; i < 2; i++) {
        S->bdesc[i].release();
        S->bf0[i].release();
        S->btab[i].release();
        if (S->bdone[i]) (void)hipEventDestroy(S->bdone[i]);
    }
    if (S->gathered) (void)hipEventDestroy(S->gathered);
    delete S;
}

}  // namespace

namespace nis {

void server_shutdown(nis_ctx* ctx)
{
    Server* S;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        S = ctx->server;
        if (!S) return;
        S->stop = true;
        S->wake.notify_all();
    }
    if (S->thread.joinable()) S->thread.join();
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->server = nullptr;
    for (auto& kv : S->reqs)
        if (kv.second.status == NIS_QUEUED || kv.second.status == NIS_RUNNING) kv.second.status = NIS_E_STATE;
    S->finished.notify_all();
    free_server(S);
}

}  // namespace nis

extern "C" {

int32_t nis_server_start(nis_ctx* ctx, const nis_server_cfg* cfg)
{
    return guard([&] {
        check(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (ctx->server) fail(NIS_E_STATE, "a frame server is already running");
        if (!ctx->net) fail(NIS_E_STATE, "no weights set");
        if (!cfg) fail(NIS_E_INVALID, "cfg is NULL");
        if (cfg->precision != NIS_FP32 && cfg->precision != NIS_BF16 && cfg->precision != NIS_FP8)
            fail(NIS_E_INVALID, "unknown precision");
        if (cfg->precision == NIS_FP8 && !ctx->net->has_fp8)
            fail(NIS_E_UNSUPPORTED, "FP8 needs the activation scales: pass them in the weight blob or call "
                                    "nis_calibrate_fp8");
        if (cfg->max_inflight < 1 || cfg->max_inflight > 16) fail(NIS_E_INVALID, "max_inflight must be in [1,16]");
        if (cfg->hbm_budget_bytes == 0) fail(NIS_E_INVALID, "budget is zero");
        if (cfg->batch_gather != 0 && cfg->batch_gather != 1) fail(NIS_E_INVALID, "batch_gather must be 0 or 1");
        if (cfg->reserved != 0) fail(NIS_E_INVALID, "reserved must be 0");
        Server* S = new Server();
        S->cfg = *cfg;
        S->t0 = Clock::now();
        S->slots.resize(cfg->max_inflight);
        try {
            for (Slot& s : S->slots) {
                hip_check(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking), "hipStreamCreate");
                hip_check(hipEventCreateWithFlags(&s.done, hipEventDisableTiming), "hipEventCreate");
                hip_check(hipEventCreateWithFlags(&s.pre, hipEventDisableTiming), "hipEventCreate");
                hip_check(hipEventCreateWithFlags(&s.read, hipEventDisableTiming), "hipEventCreate");
                hip_check(hipHostMalloc((void**)&s.pinned_count, sizeof(int), hipHostMallocDefault), "hipHostMalloc");
                *s.pinned_count = 0;
            }
            for (int i = 0; i < 2; i++)
                hip_check(hipEventCreateWithFlags(&S->bdone[i], hipEventDisableTiming), "hipEventCreate");
            hip_check(hipEventCreateWithFlags(&S->gathered, hipEventDisableTiming), "hipEventCreate");
            S->thread = std::thread(scheduler, ctx, S);
        } catch (...) {
            free_server(S);
            throw;
        }
        ctx->server = S;
    });
}

int32_t nis_frame_memory(nis_ctx* ctx, const nis_frame_req* req, int32_t precision, uint64_t* bytes)
{
    return guard([&] {
        check(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!bytes) fail(NIS_E_INVALID, "bytes is NULL");
        if (precision != NIS_FP32 && precision != NIS_BF16 && precision != NIS_FP8)
            fail(NIS_E_INVALID, "unknown precision");
        Request r = make_request(ctx, req);
        *bytes = frame_need(precision, get_medium(ctx, req->medium), r);
    });
}

int32_t nis_submit_frame(nis_ctx* ctx, const nis_frame_req* req, uint64_t* id)
{
    return guard([&] {
        check(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Server* S = running(ctx);
        if (!id) fail(NIS_E_INVALID, "id is NULL");
        Request r = make_request(ctx, req);
        if (frame_need(S->cfg.precision, get_medium(ctx, req->medium), r) > S->cfg.hbm_budget_bytes)
            fail(NIS_E_NOMEM, "the frame needs more device memory than the server's whole budget");
        r.t_submit = S->now();
        const uint64_t k = S->next_id++;
        S->reqs.emplace(k, std::move(r));
        S->queue.push_back(k);
        *id = k;
        S->wake.notify_all();
    });
}

int32_t nis_poll(nis_ctx* ctx, uint64_t id, nis_frame_result* out)
{
    return guard([&] {
        check(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Server* S = running(ctx);
        if (!out) fail(NIS_E_INVALID, "out is NULL");
        auto it = S->reqs.find(id);
        if (it == S->reqs.end()) fail(NIS_E_INVALID, "unknown frame id");
        fill_result(it->second, out);
    });
}

int32_t nis_wait(nis_ctx* ctx, uint64_t id, nis_frame_result* out)
{
    return guard([&] {
        check(ctx);
        std::unique_lock<std::mutex> lk(ctx->mu);
        Server* S = running(ctx);
        if (!out) fail(NIS_E_INVALID, "out is NULL");
        for (;;) {
            auto it = S->reqs.find(id);
            if (it == S->reqs.end()) fail(NIS_E_INVALID, "unknown frame id");
            if (it->second.status != NIS_QUEUED && it->second.status != NIS_RUNNING) {
                fill_result(it->second, out);
                return;
            }
            S->finished.wait(lk);
            if (ctx->server != S) fail(NIS_E_STATE, "the frame server stopped");
        }
    });
}

int32_t nis_release(nis_ctx* ctx, uint64_t id)
{
    return guard([&] {
        check(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Server* S = running(ctx);
        auto it = S->reqs.find(id);
        if (it == S->reqs.end()) fail(NIS_E_INVALID, "unknown frame id");
        if (it->second.status == NIS_QUEUED || it->second.status == NIS_RUNNING)
            fail(NIS_E_STATE, "the frame is still queued or running");
        if (it->second.image.p) S->spare_images.push_back(it->second.image);
        S->reqs.erase(it);
        S->wake.notify_all();
    });
}

int32_t nis_server_stop(nis_ctx* ctx)
{
    return guard([&] {
        check(ctx);
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            running(ctx);
        }
        server_shutdown(ctx);
    });
}

}  // extern "C"
