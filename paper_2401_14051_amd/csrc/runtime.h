// runtime.h -- host-side state behind the C ABI: device buffers, media, light
// states, packed networks, per-stream workspaces and the frame pipeline.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/nis.h"
#include "launch_args.h"

namespace nis {

// ---- errors: every ABI call runs inside guard(), which maps these to codes --

struct Error {
    int32_t code;
    std::string msg;
};

extern thread_local std::string g_err;

[[noreturn]] void fail(int32_t code, const std::string& msg);
void hip_check(hipError_t e, const char* what);

template <class F> int32_t guard(F&& f)
{
    try {
        f();
        g_err.clear();
        return NIS_OK;
    } catch (const Error& e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_err = "host allocation failed";
        return NIS_E_NOMEM;
    } catch (...) {
        g_err = "internal error";
        return NIS_E_INTERNAL;
    }
}

// ---- device memory -----------------------------------------------------------

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    void reserve(size_t nbytes, const char* what);   // grows (contents not kept)
    void release();
    template <class T> T* as() const { return reinterpret_cast<T*>(p); }
};

// ---- media and lights --------------------------------------------------------

// Everything that depends on the light direction: the light frame (dominant
// axis, shears, lattice offsets), each level's sheared-ray ranges, the path
// density fields (stored only as pairs along V), the light-axis density pairs
// and the per-site direction/phase tables; for a light dominated by x also a
// copy of the pyramid with y fastest, so that the sweep's lanes (along the
// lateral axis b = y) read neighbouring floats.
struct LightState {
    bool valid = false;
    double l[3] = {0, 0, 0};                // unit vector towards the light
    int a = 0, b = 1, c = 2, sigma = 1;
    double sb = 0, sc = 0, la = 1;
    double qoff[3][9] = {};
    Level lev[kMaxLevels] = {};             // medium's n and rho_off plus this light's ray ranges
    int64_t rt_floats = 0;                  // transposed pyramid (x-dominant lights only)
    int64_t pair_count = 0;                 // light-axis density pairs of all levels
    int64_t dpair_count = 0;                // path-density pairs of all levels
    DevBuf RT, P, DP, tab, vtab, tpl;
    std::vector<TplTables> tpl_host;        // host copy of the template tables (kept while a copy may run)
    bool tpl_valid = false;
    Phase tpl_phase = {};                   // phase the template tables were computed for
    bool stale = true;                      // D, P and DP must be recomputed
    uint64_t swept_version = 0;             // pyramid version they were computed from
    bool tab_valid = false;
    Phase tab_phase = {};                   // phase the site tables were computed for
    bool tab_volume = false;                // ... and whether as volume phases (then vtab too)
    size_t bytes() const { return RT.bytes + P.bytes + DP.bytes + tab.bytes + vtab.bytes + tpl.bytes; }
    void release()
    {
        RT.release();
        P.release();
        DP.release();
        tab.release();
        vtab.release();
        tpl.release();
        tab_valid = false;
        tpl_valid = false;
        stale = true;
    }
};

struct Medium {
    int n = 0, levels = 0;
    float sigma_t = 0, albedo = 0;
    float albedo_rgb[3] = {0, 0, 0};        // per colour channel; all three equal albedo for a grey medium
    Phase phase = {1, {1.f}, {0.f}};
    bool volume_phase = false;              // phase features from volume phases (eq. 9)
    float rmax = 0;                         // largest density of level 0
    Level lev[kMaxLevels] = {};             // n and rho_off of every level
    DevBuf rho;
    int64_t rho_floats = 0;
    uint64_t version = 1;                   // bumped whenever the pyramid is rebuilt
    LightState light;                       // the light of the synchronous API
    float radiance = 1.f;
};

// Medium parameters a computation runs with.
struct Params {
    float sigma_t, albedo;
    Phase phase;
    float radiance;
    bool volume = false;   // volume phases (eq. 9) in the phase features
    int channels = 1;      // 3: one radiance per colour channel, albedo rgb[c]
    float rgb[3] = {0, 0, 0};
    int templates = 0;     // NIS_TEMPLATES_LATTICE or NIS_TEMPLATES_PAPER
    int modules = 0;       // 1: the paper's backbone modules between the templates and the MLP
};

inline bool grey_albedo(const Medium* M)
{
    return M->albedo_rgb[0] == M->albedo_rgb[1] && M->albedo_rgb[1] == M->albedo_rgb[2];
}

inline Phase single_lobe(float g) { return Phase{1, {1.f}, {g}}; }
inline bool same_phase(const Phase& a, const Phase& b)
{
    if (a.n != b.n) return false;
    for (int i = 0; i < a.n; i++)
        if (a.w[i] != b.w[i] || a.g[i] != b.g[i]) return false;
    return true;
}

// Fills the light frame and level ranges of `ls` for direction l (unit);
// reserves nothing.  Fails with NIS_E_UNSUPPORTED if a level's field would
// exceed 2^31 entries.
void light_layout(const Medium* M, const double l[3], LightState* ls);
// light_layout plus the allocation of D; marks D and the tables stale.
void set_light_state(const Medium* M, const double l[3], LightState* ls);

// ---- networks ------------------------------------------------------------------

struct PackedNet {
    DevBuf w1t[2], w2t[2], cb[2];
    DevBuf W[kMaxLinear], bias[kMaxLinear], wexp[kMaxLinear], wout;
};

struct Net {
    int width = 0, n_linear = 0, wpad = 0;
    float lam = 0.6f, gamma = 4.f;
    bool has_fp8 = false;              // activation scales known (blob or calibration); FP8 packed
    bool has_modules = false;          // the blob holds the paper's backbone modules
    std::vector<float> modules;        // their weights, blob order
    DevBuf mod;                        // ... on the device, in the module kernel's packed layout (FP32)
    std::vector<float> groups[2];      // 3844 floats each, blob order
    std::vector<std::vector<float>> A, beta;
    // dequantisation scales of the FP8 activations (x = code * scale): conv1
    // input, conv2 input (unused: the CNN runs in BF16), then the input of
    // each backbone layer
    std::vector<float> fp8_scales;
    PackedNet packed[3];               // fp32, bf16, fp8
};

// ---- profiling -------------------------------------------------------------------

struct Profiler {
    bool on = false;
    struct Rec {
        const char* name;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    void clear();
    ~Profiler();
};

extern thread_local Profiler* g_prof;   // profiler of the context this thread is calling into

// ---- workspaces ------------------------------------------------------------------

constexpr int64_t kChunk = 1 << 21;   // points per feature/backbone pass
constexpr int kRenderBand = 8;         // rows per band of a rendered frame's collision order

// Descriptor and single-scatter scratch of one stream (and, for the paper's
// backbone modules, the FP32 template feature rows they read).
struct Workspace {
    DevBuf desc, f0, feat;
    size_t bytes() const { return desc.bytes + f0.bytes + feat.bytes; }
    void release()
    {
        desc.release();
        f0.release();
        feat.release();
    }
};
constexpr int64_t kModuleChunk = 1 << 16;   // points per pass with the backbone modules

// Per-pixel buffers of one frame on one stream.
struct FrameWork {
    DevBuf flag, offset, pts, dirs, cpts, cdirs, cpix, count, scan, L;
    DevBuf L3;   // RGB radiance of the collisions, reserved by the first RGB frame
    int64_t npix = 0;
    void reserve(int64_t npix);
    FrameBuffers view() const;
    size_t bytes() const;
    void release();
};

size_t workspace_bytes(int prec, int64_t npts);   // what run_query reserves for npts points
size_t frame_work_bytes(int64_t npix);            // what FrameWork::reserve(npix) allocates

struct QueryOut {
    float* radiance = nullptr;
    float* y = nullptr;
    float* tbar = nullptr;
    float* rho = nullptr;
    float* phi = nullptr;
    float* stats = nullptr;
    float* tp = nullptr;
    float* f0 = nullptr;
    void* desc = nullptr;     // raw descriptor copy (precision's row layout), [n][desc_row_bytes]
    float* absmax = nullptr;  // FP32 backbone only: device [n_linear], running max |input| of each layer
    bool run_mlp = true;
};

// Device addresses of the scratch one pass of the query uses: the descriptor
// rows [chunk][desc_row_bytes] and the single-scatter terms [chunk].
struct WsView {
    void* desc = nullptr;
    float* f0 = nullptr;
    float* feat = nullptr;   // backbone modules only: FP32 template feature rows [chunk][kDescPad]
    int64_t chunk = 0;       // points per pass
};

// Sweep if stale, refresh the site tables, then features and backbone over
// n points (or min(n, *d_count) when d_count is given), in chunks.
void run_query(Workspace& ws, const Net* net, int prec, const Medium* M, LightState* ls, const Params& P,
               const float* d_pts, const float* d_dirs, int64_t n, const int* d_count, const QueryOut& o,
               hipStream_t s);
// The same on caller-provided scratch; allocates nothing (fails with
// NIS_E_STATE where the light's tables would have to be allocated first).
void run_query_in(const WsView& w, const Net* net, int prec, const Medium* M, LightState* ls, const Params& P,
                  const float* d_pts, const float* d_dirs, int64_t n, const int* d_count, const QueryOut& o,
                  hipStream_t s, bool may_alloc);

// The gather's arguments for a query of medium M under light state ls (its
// points, count, outputs not set), after bringing the light's fields and
// site tables up to date on stream s; the backbone's weight arguments.
FeatArgs prepare_feat_args(const Net* net, int prec, const Medium* M, LightState* ls, const Params& P,
                           hipStream_t s);
MlpArgs mlp_args(const Net* net, int prec);

// Validates a camera and converts it to kernel arguments.
CamArgs camera_args(const nis_camera* cam);

// Camera rays, delta tracking and compaction into fw (or into the caller's
// arrays when d_pts is given), all on stream s.
void frame_points(FrameWork& fw, const Medium* M, const Params& P, const CamArgs& C, uint64_t seed,
                  float* d_pts, float* d_dirs, int* d_pix, int* d_count, hipStream_t s);

// A whole frame: frame_points, query of the collisions, image = albedo * L.
void render_frame(Workspace& ws, FrameWork& fw, const Net* net, int prec, const Medium* M, LightState* ls,
                  const Params& P, const CamArgs& C, uint64_t seed, float* d_image, hipStream_t s);

const char* precision_name(int prec);

}  // namespace nis

struct Server;

struct nis_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::map<int32_t, nis::Medium*> media;
    int32_t next_id = 1;
    nis::Net* net = nullptr;
    int precision = nis::kPrecFP32;
    int templates = 0;                 // NIS_TEMPLATES_LATTICE (default) or NIS_TEMPLATES_PAPER
    int backbone = 0;                  // NIS_BACKBONE_MLP (default) or NIS_BACKBONE_PAPER
    nis::Workspace ws;
    nis::FrameWork fw;
    nis::DevBuf io;
    nis::DevBuf batch_y, batch_tab;    // nis_query_batch: network outputs, gather argument table
    nis::Profiler prof;
    std::mutex mu;             // taken by every ABI call and by the server's scheduler
    Server* server = nullptr;
    hipEvent_t order = nullptr;        // recorded after each call's work
    hipStream_t order_stream = nullptr;
    bool ordered = false;              // order has been recorded
};

namespace nis {
// The work of one context is ordered across streams: a call's work on stream
// s starts after the work of the context's earlier calls, on whatever stream.
// StreamUse makes s wait for the previous call's event (when the streams
// differ) and records the event on s when the call ends.
struct StreamUse {
    nis_ctx* ctx;
    hipStream_t s;
    StreamUse(nis_ctx* c, hipStream_t stream);
    ~StreamUse();
};

Medium* get_medium(nis_ctx* ctx, int32_t id);
Params medium_params(const Medium* M);
void server_shutdown(nis_ctx* ctx);   // stops and frees the server, if any (ctx->mu held)
}  // namespace nis
