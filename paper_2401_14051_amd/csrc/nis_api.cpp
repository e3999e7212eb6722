// nis_api.cpp -- host runtime behind the C ABI declared in include/nis.h.
//
// Owns the device memory of every medium (density pyramid, path-density
// fields, per-light site tables), the packed network weights for each
// precision, and the per-stream workspaces, and queues the kernels on HIP
// streams.  Double-precision set-up values (light frame, lattice offsets,
// per-layer coefficients, camera frames) are computed here term by term; this
// file is built with -ffp-contract=off so that each product and sum is rounded
// once.
#include <cmath>
#include <cstdio>

#include "runtime.h"

// Scratch of the allocation-free query (nis_query_device_noalloc): room for
// the descriptor rows and single-scatter terms of NIS_NOALLOC_MAX_POINTS
// points at the widest precision (FP32 descriptor),
// each part starting on a 256-byte boundary.  Every GPU the library runs on
// holds its own copy until the process ends.  Host code never passes this
// name to a kernel or a copy: it reaches the memory only through the device
// address that scratch_setup() looks up per device.
constexpr size_t kScratchBytes =
    ((size_t)NIS_NOALLOC_MAX_POINTS * nis::kDescPad * 4 + 255) / 256 * 256 + ((size_t)NIS_NOALLOC_MAX_POINTS * 4 + 255) / 256 * 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace nis {

thread_local std::string g_err;
thread_local Profiler* g_prof = nullptr;

void fail(int32_t code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what)
{
    if (e == hipSuccess) return;
    if (e == hipErrorOutOfMemory) fail(NIS_E_NOMEM, std::string(what) + ": out of device memory");
    fail(NIS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void DevBuf::reserve(size_t nbytes, const char* what)
{
    if (nbytes <= bytes) return;
    release();
    hip_check(hipMalloc(&p, nbytes), what);
    bytes = nbytes;
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

hipEvent_t Profiler::get()
{
    if (pool.empty()) {
        hipEvent_t e;
        hip_check(hipEventCreate(&e), "hipEventCreate");
        return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
}

void Profiler::clear()
{
    for (auto& r : recs) {
        pool.push_back(r.a);
        pool.push_back(r.b);
    }
    recs.clear();
}

Profiler::~Profiler()
{
    clear();
    for (auto e : pool) (void)hipEventDestroy(e);
}

namespace {

uint16_t bf16_bits(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                              // round to nearest even
    return (uint16_t)(u >> 16);
}

constexpr int kGroupFloats = 216 + 8 + 3456 + 16 + 64 + 4 + 64 + 16;

void check_ctx(nis_ctx* ctx)
{
    if (!ctx) fail(NIS_E_INVALID, "context is NULL");
    g_prof = &ctx->prof;
    hip_check(hipSetDevice(ctx->device), "hipSetDevice");
}

void no_server(nis_ctx* ctx, const char* what)
{
    if (ctx->server) fail(NIS_E_STATE, std::string(what) + " is not allowed while the frame server runs");
}

bool finite3(const float* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

void validate_params(float sigma_t, float albedo, float g)
{
    if (!(std::isfinite(sigma_t) && sigma_t >= 0.f)) fail(NIS_E_INVALID, "sigma_t must be finite and >= 0");
    if (!(std::isfinite(albedo) && albedo >= 0.f && albedo <= 1.f)) fail(NIS_E_INVALID, "albedo must be in [0,1]");
    if (!(std::isfinite(g) && g > -1.f && g < 1.f)) fail(NIS_E_INVALID, "g must be in (-1,1)");
}

void ray_range(double s, int nm, int* lo, int* hi)
{
    double a = (nm - 1) * s;
    *lo = (int)std::floor(a < 0.0 ? a : 0.0) - 1;
    *hi = (int)std::ceil((double)(nm - 1) + (a > 0.0 ? a : 0.0)) + 1;
}

MediumView make_view(const Medium* M, const LightState* ls, const Params& P, const Net* net)
{
    MediumView v;
    std::memset(&v, 0, sizeof(v));
    v.rho = M->rho.as<float>();
    if (ls->a == 0) {
        // x-dominant light: the transposed copy, [x][z][y] per level
        v.rho_s = ls->RT.as<float>();
        v.se[0] = 2, v.se[1] = 0, v.se[2] = 1;
    } else {
        v.rho_s = v.rho;
        v.se[0] = 0, v.se[1] = 1, v.se[2] = 2;
    }
    v.pairs = ls->P.as<float2>();
    v.dpairs = ls->DP.as<float2>();
    for (int m = 0; m < M->levels; m++) v.lev[m] = ls->lev[m];
    v.levels = M->levels;
    v.n0 = M->n;
    v.a = ls->a;
    v.b = ls->b;
    v.c = ls->c;
    v.sigma = ls->sigma;
    v.sb = ls->sb;
    v.sc = ls->sc;
    for (int d = 0; d < 3; d++) v.l[d] = ls->l[d];
    v.la = ls->la;
    std::memcpy(v.qoff, ls->qoff, sizeof(v.qoff));
    v.sigma_t = P.sigma_t;
    v.albedo = P.albedo;
    v.radiance = P.radiance;
    v.volume = P.volume ? 1 : 0;
    v.lam = net ? net->lam : 0.6f;
    v.gamma = net ? net->gamma : 4.f;
    v.nl = P.phase.n;
    double mc = 0.0;
    for (int i = 0; i < P.phase.n; i++) {
        const double g = P.phase.g[i], w = P.phase.w[i];
        mc += w * g;
        v.hg_a[i] = 1.0 + g * g;
        v.hg_b[i] = 2.0 * g;
        v.hg_k[i] = w * ((1.0 - g * g) / (4.0 * M_PI));
        const double ga = std::fabs(g);
        v.ph_a[i] = (float)ga;
        v.ph_s[i] = g < 0.0 ? -1.f : 1.f;
        v.ph_c[i] = (float)((1.0 - ga) * (1.0 - ga));
        v.ph_k[i] = (float)v.hg_k[i];
    }
    v.g = (float)mc;
    return v;
}

template <class F> void timed(const char* name, hipStream_t s, F&& launch)
{
    if (!g_prof || !g_prof->on) {
        hip_check(launch(), name);
        return;
    }
    hipEvent_t a = g_prof->get(), b = g_prof->get();
    hip_check(hipEventRecord(a, s), "hipEventRecord");
    hip_check(launch(), name);
    hip_check(hipEventRecord(b, s), "hipEventRecord");
    g_prof->recs.push_back({name, a, b});
}

// 64-point Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on
// the Legendre polynomial P_64 from the Chebyshev-like initial guesses
// cos(pi (i + 3/4) / (n + 1/2)); the weights are 2 / ((1 - x^2) P'_64(x)^2).
static const GaussLegendre64& gauss_legendre64()
{
    static const GaussLegendre64 gl = [] {
        GaussLegendre64 r;
        const int n = 64;
        for (int i = 0; i < n; i++) {
            double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dpn = 1.0;
            for (int it = 0; it < 100; it++) {
                double pm = 1.0, pn = x;
                for (int k = 2; k <= n; k++) {
                    const double pk = ((2 * k - 1) * x * pn - (k - 1) * pm) / k;
                    pm = pn;
                    pn = pk;
                }
                dpn = n * (x * pn - pm) / (x * x - 1.0);
                const double step = pn / dpn;
                x -= step;
                if (std::fabs(step) < 1e-16) break;
            }
            r.x[i] = x;
            r.w[i] = 2.0 / ((1.0 - x * x) * dpn * dpn);
        }
        return r;
    }();
    return gl;
}

void refresh_tables(const Medium* M, LightState* ls, const Phase& ph, bool volume, hipStream_t s,
                    bool may_alloc = true)
{
    if (ls->tab_valid && same_phase(ls->tab_phase, ph) && ls->tab_volume == volume) return;
    if (!may_alloc && (ls->tab.bytes < sizeof(SiteTables) ||
                       (volume && ls->vtab.bytes < (size_t)kSites * kVBins * sizeof(float))))
        fail(NIS_E_STATE, "the light's site tables are not allocated: set the light (after enabling volume phases)");
    ls->tab.reserve(sizeof(SiteTables), "site tables");
    Params P = medium_params(M);
    P.phase = ph;
    P.volume = volume;
    MediumView mv = make_view(M, ls, P, nullptr);
    timed("site_tables", s, [&] { return launch_site_tables(mv, ls->tab.as<SiteTables>(), s); });
    if (volume) {
        ls->vtab.reserve((size_t)kSites * kVBins * sizeof(float), "volume phase tables");
        timed("volume_tables", s, [&] {
            return launch_volume_tables(mv, gauss_legendre64(), ls->tab.as<SiteTables>(), ls->vtab.as<float>(), s);
        });
    }
    ls->tab_valid = true;
    ls->tab_phase = ph;
    ls->tab_volume = volume;
}

// ---- the paper's templates (Sec. III.B.2, eq. 2-4) -------------------------
//
// Unit templates (the paper leaves the construction open; these readings are
// shared with the checks of this library):
//  * diffuse layer 0: the centre and 5 points on the unit sphere; layer i >= 1:
//    n_i points in the shell 1/2 <= |u| <= 1.  Directions are spherical
//    Fibonacci points (z stratified, golden-angle azimuth), and in the shell
//    each point takes an equal-volume radial stratum from the additive
//    sequence frac(1/2 + k c), c = 0.5698402909980532 (decorrelated from the
//    golden angle);
//  * highlight layer h (cone with apex at the point, axis l, unit length and
//    unit base radius): axial t dividing the layer's frustum volume at
//    (k + 1/2)/n, radius sqrt(frac(1/2 + k c)) t, golden-angle azimuth, in the
//    orthonormal frame of l of Duff et al. (2017);
//  * eq. (3): D(S) is the mean nearest-neighbour distance of a unit set;
//    eq. (4): r_i = 2^(i-1) xi_i / (2^8 D(S_i)), xi_i = 1 - 0.08 min(i, 5).
// All in double precision, built with contraction off (each product and sum
// rounded once), so that the sampled positions' in-cube decisions are those
// of the definition.
namespace {

struct TplGeometry {
    double unit[kTplSites][3];   // diffuse: world axes; highlight: (t, x1, x2) in the frame of l
    double D[kLayers];
    double radius[kDiffuse];
};

void tpl_unit_point(int layer, int k, double u[3])
{
    const double golden = 2.39996322972865332, step = 0.5698402909980532;
    const int n = tpl_count(layer);
    if (layer < kDiffuse) {
        int kk = k, nn = n;
        double rad;
        if (layer == 0) {
            if (k == 0) {
                u[0] = u[1] = u[2] = 0.0;
                return;
            }
            kk = k - 1;
            nn = n - 1;
            rad = 1.0;
        } else {
            const double a = 0.5 + kk * step;
            const double wv = a - std::floor(a);
            rad = std::cbrt(0.125 + wv * 0.875);
        }
        const double z = 1.0 - (2.0 * kk + 1.0) / nn;
        const double rxy = std::sqrt(1.0 - z * z);
        const double az = kk * golden;
        u[0] = rad * (rxy * std::cos(az));
        u[1] = rad * (rxy * std::sin(az));
        u[2] = rad * z;
    } else {
        const int h = layer - kDiffuse;
        const double lo = h / 4.0, hi = (h + 1) / 4.0;
        const double t = std::cbrt(lo * lo * lo + ((k + 0.5) / n) * (hi * hi * hi - lo * lo * lo));
        const double a = 0.5 + k * step;
        const double wv = a - std::floor(a);
        const double rad = std::sqrt(wv) * t;
        const double az = k * golden;
        u[0] = t;
        u[1] = rad * std::cos(az);
        u[2] = rad * std::sin(az);
    }
}

const TplGeometry& tpl_geometry()
{
    static const TplGeometry G = [] {
        TplGeometry g;
        for (int k = 0; k < kLayers; k++)
            for (int j = 0; j < tpl_count(k); j++) tpl_unit_point(k, j, g.unit[tpl_first(k) + j]);
        for (int k = 0; k < kLayers; k++) {
            const int n = tpl_count(k), f = tpl_first(k);
            double sum = 0.0;
            for (int j = 0; j < n; j++) {
                double best = INFINITY;
                for (int i = 0; i < n; i++) {
                    if (i == j) continue;
                    const double dx = g.unit[f + j][0] - g.unit[f + i][0];
                    const double dy = g.unit[f + j][1] - g.unit[f + i][1];
                    const double dz = g.unit[f + j][2] - g.unit[f + i][2];
                    const double d = std::sqrt(dx * dx + dy * dy + dz * dz);
                    if (d < best) best = d;
                }
                sum += best;
            }
            g.D[k] = sum / n;
        }
        for (int i = 0; i < kDiffuse; i++) {
            const double xi = 1.0 - 0.08 * (i < 5 ? i : 5);
            g.radius[i] = std::ldexp(1.0, i - 1) * xi / (256.0 * g.D[i]);
        }
        return g;
    }();
    return G;
}

// level whose voxel matches a point spacing on an n^3 grid (below L)
int tpl_level_host(double spacing, int n, int L)
{
    const double x = spacing * n;
    int m = 0;
    while (m < L - 1 && x >= 1.4142135623730951 * std::ldexp(1.0, m)) m++;
    return m;
}

// the medium's phase (its lobes summed with their weights) in double precision
double phase_value(const Phase& ph, double mu)
{
    double v = 0.0;
    for (int i = 0; i < ph.n; i++) {
        const double g = ph.g[i];
        const double den = 1.0 + g * g - 2.0 * g * mu;
        v += ph.w[i] * ((1.0 - g * g) / (4.0 * M_PI)) / (den * std::sqrt(den));
    }
    return v;
}

}  // namespace

// Template tables of a light and phase: the highlight points in world axes
// (o = t l + x1 e1 + x2 e2) and every point's unit direction and f(d . l).
void refresh_tpl_tables(LightState* ls, const Phase& ph, hipStream_t s, bool may_alloc)
{
    if (ls->tpl_valid && same_phase(ls->tpl_phase, ph)) return;
    if (!may_alloc && ls->tpl.bytes < sizeof(TplTables))
        fail(NIS_E_STATE, "the light's template tables are not allocated: set the light first");
    ls->tpl.reserve(sizeof(TplTables), "template tables");
    const TplGeometry& G = tpl_geometry();
    const double* l = ls->l;
    // orthonormal frame of l (Duff et al. 2017)
    const double sg = l[2] >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (sg + l[2]);
    const double b = l[0] * l[1] * a;
    const double e1[3] = {1.0 + sg * l[0] * l[0] * a, sg * b, -sg * l[0]};
    const double e2[3] = {b, sg + l[1] * l[1] * a, -l[1]};
    if (ls->tpl_host.size() != 1) ls->tpl_host.resize(1);
    TplTables& T = ls->tpl_host[0];
    for (int k = 0; k < kLayers; k++)
        for (int j = 0; j < tpl_count(k); j++) {
            const int t = tpl_first(k) + j;
            const double* u = G.unit[t];
            double o[3];
            for (int d = 0; d < 3; d++) o[d] = k < kDiffuse ? u[d] : u[0] * l[d] + u[1] * e1[d] + u[2] * e2[d];
            for (int d = 0; d < 3; d++) T.off[t][d] = o[d];
            const double on = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
            if (on > 0.0) {
                const double dd[3] = {o[0] / on, o[1] / on, o[2] / on};
                const double mu = dd[0] * l[0] + dd[1] * l[1] + dd[2] * l[2];
                T.site[t] = make_float4((float)dd[0], (float)dd[1], (float)dd[2], (float)phase_value(ph, mu));
            } else {
                T.site[t] = make_float4((float)l[0], (float)l[1], (float)l[2], 1.f);   // the centre: f(w.l)
            }
        }
    hip_check(hipMemcpyAsync(ls->tpl.p, &T, sizeof(TplTables), hipMemcpyHostToDevice, s), "template tables");
    ls->tpl_valid = true;
    ls->tpl_phase = ph;
}

void ensure_sweep(const Medium* M, LightState* ls, hipStream_t s)
{
    if (!ls->valid) fail(NIS_E_STATE, "no light set for this medium");
    if (!ls->stale && ls->swept_version == M->version) return;
    MediumView mv = make_view(M, ls, medium_params(M), nullptr);
    if (ls->a == 0) timed("transpose", s, [&] { return launch_transpose(mv, s); });
    timed("sweep", s, [&] { return launch_sweep(mv, s); });
    timed("pairs", s, [&] { return launch_pairs(mv, s); });
    ls->stale = false;
    ls->swept_version = M->version;
}

// ---- weights --------------------------------------------------------------

struct BlobHeader {
    char magic[4];
    uint32_t version, din, width, n_linear, groups;
    float lam, gamma;
    uint32_t has_fp8_scales;
    uint32_t has_modules;
    uint32_t reserved[6];
};
static_assert(sizeof(BlobHeader) == 64, "blob header is 64 bytes");

void upload(DevBuf& buf, const void* host, size_t bytes, const char* what)
{
    buf.reserve(bytes, what);
    hip_check(hipMemcpy(buf.p, host, bytes, hipMemcpyHostToDevice), what);
}

template <class T> void upload_vec(DevBuf& buf, const std::vector<T>& v, const char* what)
{
    upload(buf, v.data(), v.size() * sizeof(T), what);
}

// OCP E4M3FN code of f with round-to-nearest-even, saturating at +-448
// (1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits; 0x7f is NaN).
uint8_t fp8_e4m3(float f)
{
    const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
    const float a = std::fabs(f);
    if (std::isnan(f)) return 0x7f;
    if (a >= 464.f) return sign | 0x7e;
    int e;
    std::frexp(a, &e);                 // a in [2^(e-1), 2^e)
    int E = e - 1 + 7;                 // biased exponent of a normal encoding
    if (a == 0.f) return sign;
    if (E >= 1) {
        float r = std::nearbyint(std::ldexp(a, 3 - (e - 1)));   // 8 <= r <= 16
        if (r == 16.f) {
            r = 8.f;
            E += 1;
        }
        if (E > 15 || (E == 15 && r > 14.f)) return sign | 0x7e;
        return sign | (uint8_t)(E << 3) | (uint8_t)((int)r - 8);
    }
    const float r = std::nearbyint(std::ldexp(a, 9));            // subnormal: r * 2^-9
    if (r >= 8.f) return sign | 0x08;
    return sign | (uint8_t)r;
}

// The FP8 backbone (k_mlp_f8): every layer's scales folded into its weights
// and bias, weights as E4M3 codes with one power-of-two (E8M0) scale per
// output channel, in the kernel's A-fragment order.  Layer l reads codes of
// x_l / s_l and writes codes of ReLU(z_l) / s_{l+1}, so its weights are
// W_l s_l / s_{l+1} and its bias beta_l / s_{l+1}; the output weights carry
// s_{n-1}.  Needs the activation scales (net->has_fp8).
void pack_fp8_backbone(Net* net, PackedNet& P)
{
    const int W = net->width, Wp = net->wpad, NO = (Wp + 31) / 32, Wb = NO * 32;
    const float* sc = net->fp8_scales.data() + 2;   // input scale of each backbone layer
    for (int li = 0; li + 1 < net->n_linear; li++) {
        const int din = li == 0 ? kDesc : W;
        const int KC = li == 0 ? kDescF8 / 64 : hidden_k(kPrecFP8, Wp) / 64;
        const double f = (double)sc[li] / (double)sc[li + 1];
        std::vector<int> ex(Wb, 0);
        std::vector<uint32_t> eb(Wb, 127u);
        std::vector<float> bb(Wb, 0.f);
        for (int o = 0; o < W; o++) {
            double amax = 0.0;
            for (int i = 0; i < din; i++) amax = std::fmax(amax, std::fabs(net->A[li][(size_t)o * din + i] * f));
            int e = amax > 0.0 ? (int)std::ceil(std::log2(amax / 448.0)) : 0;
            e = e < -127 ? -127 : e > 127 ? 127 : e;
            ex[o] = e;
            eb[o] = (uint32_t)(e + 127);
            bb[o] = (float)((double)net->beta[li][o] / (double)sc[li + 1]);
        }
        // step kc, tile ct, half h, lane l = r + 32 g, byte e16: weight row
        // ct*32 + r, K slot e = 16 h + e16 of lane group g, whose input column
        // is (first layer) the descriptor byte (kc/2)*128 + 64 g + 32 (kc%2) + e,
        // (hidden layers) the previous layer's channel held in that slot
        std::vector<uint8_t> frag((size_t)KC * NO * 2048, 0);
        size_t pos = 0;
        for (int kc = 0; kc < KC; kc++)
            for (int ct = 0; ct < NO; ct++)
                for (int h = 0; h < 2; h++)
                    for (int l = 0; l < 64; l++)
                        for (int e16 = 0; e16 < 16; e16++) {
                            const int g = l / 32, row = ct * 32 + l % 32, e = 16 * h + e16;
                            int col;
                            if (li == 0) {
                                col = (kc / 2) * 128 + 64 * g + 32 * (kc % 2) + e;
                            } else {
                                const int t = 2 * kc + e / 16, rr = e % 16;
                                col = t < NO ? t * 32 + 8 * (rr / 4) + 4 * g + rr % 4 : din;
                            }
                            uint8_t code = 0;
                            if (row < W && col < din)
                                code = fp8_e4m3((float)std::ldexp(net->A[li][(size_t)row * din + col] * f, -ex[row]));
                            frag[pos++] = code;
                        }
        upload_vec(P.W[li], frag, "backbone weights");
        upload_vec(P.bias[li], bb, "backbone biases");
        upload_vec(P.wexp[li], eb, "backbone weight scales");
    }
    std::vector<float> wo(Wb, 0.f);
    const float slast = sc[net->n_linear - 1];
    for (int i = 0; i < W; i++) wo[i] = (float)((double)net->A[net->n_linear - 1][i] * (double)slast);
    upload_vec(P.wout, wo, "output weights");
}

// Pack one precision: conv weights [out][k] zero padded (float32 for FP32,
// bfloat16 otherwise: the FP8 path runs the CNN in BF16); backbone matrices
// zero padded to the kernel's tile sizes and stored in fragment order, in
// float32 or bfloat16 (FP8: pack_fp8_backbone, once the activation scales
// are known); biases and the last layer stay float32.
void pack_net(Net* net, int prec)
{
    PackedNet& P = net->packed[prec];
    auto put = [&](DevBuf& buf, const std::vector<float>& v, const char* what) {
        if (prec == kPrecFP32) {
            upload_vec(buf, v, what);
        } else {
            std::vector<uint16_t> h(v.size());
            for (size_t i = 0; i < v.size(); i++) h[i] = bf16_bits(v[i]);
            upload_vec(buf, h, what);
        }
    };
    for (int gi = 0; gi < 2; gi++) {
        const float* G = net->groups[gi].data();
        const float *w1 = G, *b1 = w1 + 216, *w2 = b1 + 8, *b2 = w2 + 3456;
        const float *s1 = b2 + 16, *c1 = s1 + 64, *s2 = c1 + 4, *c2 = s2 + 64;
        std::vector<float> t1(16 * kConv1K, 0.f), t2(16 * kConv2K, 0.f);
        // One MFMA tile convolves two points: rows 0-7 are the first point's
        // channels, rows 8-15 the second's, each with zero weights on the other
        // point's K slots.  A tap-row (dz * 3 + dy) takes 4 slots, dx and a zero.
        // FP32 (K step 4): the first point's tap-row tr at K 4 tr, the second's
        // at 36 + 4 tr.  BF16 (K step 32): tap-rows 0-7 of the first point fill
        // step 0 and those of the second step 1; tap-row 8 takes slots 0-3 of
        // step 2 (first point) and slots 4-7 (second).  Both points then sum
        // their products with the same grouping, the other point's steps
        // adding exact zeros, so that a point's result does not depend on its
        // place in the batch (the tests compare frames rendered in two point
        // orders bit for bit).
        auto k1 = [&](int second, int tr) {
            if (prec == kPrecFP32) return 36 * second + 4 * tr;
            return tr < 8 ? 32 * second + 4 * tr : 64 + 4 * second;
        };
        for (int o = 0; o < 8; o++)
            for (int tr = 0; tr < 9; tr++)
                for (int dx = 0; dx < 3; dx++) {
                    t1[o * kConv1K + k1(0, tr) + dx] = w1[o * 27 + tr * 3 + dx];
                    t1[(o + 8) * kConv1K + k1(1, tr) + dx] = w1[o * 27 + tr * 3 + dx];
                }
        // conv2 K order is tap-major (k = tap * 8 + input channel), matching the
        // channels-fastest layout of the conv1 output the kernel reads
        for (int o = 0; o < 16; o++)
            for (int ci = 0; ci < 8; ci++)
                for (int tap = 0; tap < 27; tap++) t2[o * kConv2K + tap * 8 + ci] = w2[(o * 8 + ci) * 27 + tap];
        put(P.w1t[gi], t1, "conv1 weights");
        put(P.w2t[gi], t2, "conv2 weights");
        std::vector<float> cb;
        cb.insert(cb.end(), b1, b1 + 8);
        cb.insert(cb.end(), b2, b2 + 16);
        cb.insert(cb.end(), s1, s1 + 64);
        cb.insert(cb.end(), c1, c1 + 4);
        cb.insert(cb.end(), s2, s2 + 64);
        cb.insert(cb.end(), c2, c2 + 16);
        upload_vec(P.cb[gi], cb, "attention weights");
    }
    if (prec == kPrecFP8) {
        if (net->has_fp8) pack_fp8_backbone(net, P);
        return;
    }
    const int W = net->width, Wp = net->wpad;
    const int Wb = (Wp + 31) / 32 * 32;   // biases and output weights padded to whole 32-channel tiles
    for (int li = 0; li + 1 < net->n_linear; li++) {
        const int din = li == 0 ? kDesc : W, kpad = li == 0 ? input_k(prec) : mlp_hidden_k(prec, Wp);
        std::vector<float> t((size_t)Wp * kpad, 0.f), bb(Wb, 0.f);
        for (int o = 0; o < W; o++) {
            for (int i = 0; i < din; i++) t[(size_t)o * kpad + i] = net->A[li][(size_t)o * din + i];
            bb[o] = net->beta[li][o];
        }
        const int KS = mlp_k_step(prec), KPL = mlp_k_per_lane(prec), KC = kpad / KS;
        std::vector<float> f(t.size());
        size_t pos = 0;
        if (prec == kPrecBF16) {
            // A-fragment order of the BF16 kernel (32x32x16 tiles, weights as
            // the A operand): K step kc holds, for output tile ct (32 channels)
            // and lane l = r + 32 g, the elements W[ct*32 + r][col(kc, g, e)],
            // e < 8.  First layer: col = (kc/4)*64 + g*32 + (kc%4)*8 + e, so a
            // lane's descriptor elements of four consecutive K steps are one
            // contiguous run.  Hidden layers: col is the previous layer's
            // channel that the lane holds in register (kc%2)*8 + e of its
            // output tile kc/2, i.e. (kc/2)*32 + (2 (kc%2) + e/4)*8 + g*4 + e%4.
            const int NO = (Wp + 31) / 32, KCb = li == 0 ? kDescPad / 16 : Wp / 16;
            f.assign((size_t)KCb * NO * 512, 0.f);
            for (int kc = 0; kc < KCb; kc++)
                for (int ct = 0; ct < NO; ct++)
                    for (int l = 0; l < 64; l++)
                        for (int e = 0; e < 8; e++) {
                            const int g = l / 32, row = ct * 32 + l % 32;
                            const int col = li == 0 ? (kc / 4) * 64 + g * 32 + (kc % 4) * 8 + e
                                                    : (kc / 2) * 32 + (2 * (kc % 2) + e / 4) * 8 + g * 4 + e % 4;
                            f[pos++] = row < Wp && col < kpad ? t[(size_t)row * kpad + col] : 0.f;
                        }
        } else {
            // B-fragment order: block (ct, kc) holds, for lane l = r + 16 g, the
            // elements W[ct*16 + r][kc*KS + g*KPL + e], e < KPL, contiguously
            for (int ct = 0; ct < Wp / 16; ct++)
                for (int kc = 0; kc < KC; kc++)
                    for (int l = 0; l < 64; l++)
                        for (int e = 0; e < KPL; e++)
                            f[pos++] = t[(size_t)(ct * 16 + l % 16) * kpad + kc * KS + (l / 16) * KPL + e];
        }
        put(P.W[li], f, "backbone weights");
        upload_vec(P.bias[li], bb, "backbone biases");
    }
    std::vector<float> wo(Wb, 0.f);
    for (int i = 0; i < W; i++) wo[i] = net->A[net->n_linear - 1][i];
    upload_vec(P.wout, wo, "output weights");
}

void free_net(Net* net)
{
    if (!net) return;
    for (auto& P : net->packed) {
        for (int g = 0; g < 2; g++) {
            P.w1t[g].release();
            P.w2t[g].release();
            P.cb[g].release();
        }
        for (auto& b : P.W) b.release();
        for (auto& b : P.bias) b.release();
        for (auto& b : P.wexp) b.release();
        P.wout.release();
    }
    net->mod.release();
    delete net;
}

void free_medium(Medium* M)
{
    M->rho.release();
    M->light.release();
    delete M;
}

// bytes of one FrameWork buffer set for npix pixels, scan storage excluded
size_t frame_fixed_bytes(int64_t npix) { return (size_t)npix * (4 + 4 + 12 + 12 + 12 + 12 + 4 + 4) + 256; }

}  // namespace

StreamUse::StreamUse(nis_ctx* c, hipStream_t stream) : ctx(c), s(stream)
{
    if (ctx->ordered && ctx->order_stream != s)
        hip_check(hipStreamWaitEvent(s, ctx->order, 0), "hipStreamWaitEvent");
}

StreamUse::~StreamUse()
{
    if (hipEventRecord(ctx->order, s) == hipSuccess) {
        ctx->order_stream = s;
        ctx->ordered = true;
    }
}

// ---- media and lights --------------------------------------------------------

Medium* get_medium(nis_ctx* ctx, int32_t id)
{
    auto it = ctx->media.find(id);
    if (it == ctx->media.end()) fail(NIS_E_STATE, "unknown medium handle");
    return it->second;
}

Params medium_params(const Medium* M) { return Params{M->sigma_t, M->albedo, M->phase, M->radiance, M->volume_phase}; }

// Parameters of a one-channel result: the albedo must be grey.
Params grey_params(const Medium* M)
{
    if (!grey_albedo(M)) fail(NIS_E_STATE, "the medium has a coloured albedo: use the RGB calls");
    return medium_params(M);
}

// Parameters of an RGB result; channel 0's albedo goes into the features.
Params rgb_params(const Medium* M)
{
    Params P = medium_params(M);
    P.channels = 3;
    for (int c = 0; c < 3; c++) P.rgb[c] = M->albedo_rgb[c];
    P.albedo = P.rgb[0];
    return P;
}

// The parameters of a query through the context: its template and backbone
// choices added.
Params with_templates(const nis_ctx* ctx, Params P)
{
    P.templates = ctx->templates;
    P.modules = ctx->backbone == NIS_BACKBONE_PAPER ? 1 : 0;
    return P;
}

// The levels of an n^3 medium's pyramid (edge n >> m, densities at rho_off);
// returns their count.
int pyramid_levels(Medium* M, int n)
{
    int L = 1;
    while ((1 << (L - 1)) < n) L++;
    M->n = n;
    M->levels = L;
    int64_t off = 0;
    for (int m = 0; m < L; m++) {
        M->lev[m].n = n >> m;
        M->lev[m].rho_off = off;
        const int64_t nm = n >> m;
        off += nm * nm * nm;
    }
    M->rho_floats = off;
    return L;
}

// A light direction normalised, or NIS_E_INVALID.
void unit_light(const float dir[3], double l[3])
{
    if (!dir || !finite3(dir)) fail(NIS_E_INVALID, "light must be finite");
    for (int d = 0; d < 3; d++) l[d] = dir[d];
    const double nrm = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    if (!(nrm > 0.0)) fail(NIS_E_INVALID, "light direction is zero");
    for (int d = 0; d < 3; d++) l[d] /= nrm;
}

void light_layout(const Medium* M, const double l[3], LightState* ls)
{
    for (int d = 0; d < 3; d++) ls->l[d] = l[d];
    int a = 0;
    for (int i = 1; i < 3; i++)
        if (std::fabs(l[i]) > std::fabs(l[a])) a = i;
    ls->a = a;
    ls->b = a == 0 ? 1 : 0;
    ls->c = a == 2 ? 1 : 2;
    ls->sigma = l[a] > 0.0 ? 1 : -1;
    ls->la = std::fabs(l[a]);
    ls->sb = l[ls->b] / ls->la;
    ls->sc = l[ls->c] / ls->la;
    for (int d = 0; d < 3; d++)
        for (int qi = 0; qi < 9; qi++) ls->qoff[d][qi] = (qi - 4) * l[d] / ls->la;
    int64_t poff = 0, qoff = 0;
    for (int m = 0; m < M->levels; m++) {
        Level& lv = ls->lev[m];
        lv = M->lev[m];
        int uhi, vhi;
        ray_range(ls->sb, lv.n, &lv.ulo, &uhi);
        ray_range(ls->sc, lv.n, &lv.vlo, &vhi);
        lv.ulo -= kRayPad;
        uhi += kRayPad;
        lv.nu = uhi - lv.ulo + 1;
        lv.nv = vhi - lv.vlo + 1;
        lv.p_off = poff;
        lv.q_off = qoff;
        lv.ds = (float)((1.0 / lv.n) / ls->la);
        // the kernels address a level's density and light-axis pairs, and one
        // slice of its path-density pairs, with 32-bit byte offsets (a whole
        // level of path-density pairs may pass 4 GiB: the gather then reads it
        // through 64-bit addresses)
        const int64_t pn = (int64_t)(lv.n + 1) * lv.n * (lv.n + 2 * kPairPad);
        const int64_t qn = (int64_t)lv.nu * (lv.nv + 1) * lv.n;
        if ((int64_t)lv.nu * (lv.nv + 1) * 8 >= ((int64_t)1 << 32) || pn * 8 >= ((int64_t)1 << 32) ||
            (int64_t)lv.n * lv.n * lv.n * 4 >= ((int64_t)1 << 32))
            fail(NIS_E_UNSUPPORTED, "a level's fields exceed the 32-bit offsets for this light (media up to 512^3 are served)");
        poff += pn;
        qoff += qn;
    }
    ls->pair_count = poff;
    ls->rt_floats = a == 0 ? M->rho_floats : 0;
    ls->dpair_count = qoff;
}

void set_light_state(const Medium* M, const double l[3], LightState* ls)
{
    light_layout(M, l, ls);
    if (ls->rt_floats > 0)
        ls->RT.reserve((size_t)ls->rt_floats * sizeof(float), "transposed pyramid");
    else
        ls->RT.release();
    ls->P.reserve((size_t)ls->pair_count * sizeof(float2), "light-axis density pairs");
    ls->DP.reserve((size_t)ls->dpair_count * sizeof(float2), "path-density pairs");
    // the site and template tables too, so that a query under this light allocates nothing
    ls->tab.reserve(sizeof(SiteTables), "site tables");
    ls->tpl.reserve(sizeof(TplTables), "template tables");
    if (M->volume_phase) ls->vtab.reserve((size_t)kSites * kVBins * sizeof(float), "volume phase tables");
    ls->valid = true;
    ls->stale = true;
    ls->tab_valid = false;
    ls->tpl_valid = false;
}

const char* precision_name(int prec) { return prec == kPrecFP32 ? "fp32" : prec == kPrecBF16 ? "bf16" : "fp8"; }

// ---- allocation-free scratch ------------------------------------------------

namespace {

struct ScratchSlot {
    bool done = false;
    hipError_t err = hipSuccess;
    void* ptr = nullptr;   // device address of this device's copy of `scratch`
};
std::mutex g_scratch_mu;
std::map<int, ScratchSlot> g_scratch;

// Looks up the device address of `scratch` on `device`, which must be the
// current device; once per device, the result (or the HIP error) kept.
void scratch_setup(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    ScratchSlot& sl = g_scratch[device];
    if (sl.done) return;
    void* ptr = nullptr;
    sl.err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    sl.ptr = sl.err == hipSuccess ? ptr : nullptr;
    sl.done = true;
}

// The scratch of `device` cut into the parts of one pass of n points.
WsView scratch_view(int device, int prec, int64_t n)
{
    ScratchSlot sl;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        auto it = g_scratch.find(device);
        if (it != g_scratch.end()) sl = it->second;
    }
    if (!sl.done) fail(NIS_E_INTERNAL, "scratch not set up for this device");
    if (!sl.ptr) fail(NIS_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(sl.err));
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t d = up((size_t)n * desc_row_bytes(prec)), f = up((size_t)n * 4);
    if (d + f > kScratchBytes) fail(NIS_E_INTERNAL, "scratch too small");
    char* base = static_cast<char*>(sl.ptr);
    WsView w;
    w.desc = base;
    w.f0 = reinterpret_cast<float*>(base + d);
    w.chunk = n;
    return w;
}

}  // namespace

// ---- query ----------------------------------------------------------------

size_t workspace_bytes(int prec, int64_t npts)
{
    const int64_t chunk = npts < kChunk ? npts : kChunk;
    return (size_t)chunk * desc_row_bytes(prec) + (size_t)chunk * 4;
}

namespace {
size_t module_feat_bytes(int64_t chunk) { return (size_t)chunk * kDescPad * sizeof(float); }
}  // namespace

void run_query(Workspace& ws, const Net* net, int prec, const Medium* M, LightState* ls, const Params& Pm,
               const float* d_pts, const float* d_dirs, int64_t n, const int* d_count, const QueryOut& o,
               hipStream_t s)
{
    if (!net) fail(NIS_E_STATE, "no weights set");
    const int64_t cap = Pm.modules ? kModuleChunk : kChunk;
    const int64_t chunk = n < cap ? n : cap;
    ws.desc.reserve((size_t)chunk * desc_row_bytes(prec), "descriptor workspace");
    ws.f0.reserve((size_t)chunk * sizeof(float), "single-scatter workspace");
    WsView w;
    w.desc = ws.desc.p;
    w.f0 = ws.f0.as<float>();
    w.chunk = chunk;
    if (Pm.modules) {
        ws.feat.reserve(module_feat_bytes(chunk), "template feature workspace");
        w.feat = ws.feat.as<float>();
    }
    run_query_in(w, net, prec, M, ls, Pm, d_pts, d_dirs, n, d_count, o, s, true);
}

// The gather's arguments that do not depend on the points: medium view,
// light tables, layer coefficients, CNN weights, descriptor scale.
FeatArgs feat_args(const Net* net, int prec, const Medium* M, const LightState* ls, const Params& Pm,
                   const MediumView& mv)
{
    const PackedNet& P = net->packed[prec];
    FeatArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.mv = mv;
    fa.tab = ls->tab.as<SiteTables>();
    fa.vtab = Pm.volume ? ls->vtab.as<float>() : nullptr;
    for (int k = 0; k < kLayers; k++) {
        int m = k < M->levels - 1 ? k : M->levels - 1;
        fa.coef[k] = (float)(std::pow((double)net->lam, m + 1) * (double)Pm.sigma_t);
    }
    for (int gi = 0; gi < 2; gi++) {
        fa.w1t[gi] = P.w1t[gi].p;
        fa.w2t[gi] = P.w2t[gi].p;
        fa.cb[gi] = P.cb[gi].as<float>();
    }
    fa.desc_inv_scale = prec == kPrecFP8 ? 1.f / net->fp8_scales[2] : 1.f;
    return fa;
}

// The backbone's arguments that do not depend on the points: its weights.
MlpArgs mlp_args(const Net* net, int prec)
{
    const PackedNet& P = net->packed[prec];
    MlpArgs ma;
    std::memset(&ma, 0, sizeof(ma));
    for (int li = 0; li + 1 < net->n_linear; li++) {
        ma.W[li] = P.W[li].p;
        ma.bias[li] = P.bias[li].as<float>();
        ma.wexp[li] = P.wexp[li].as<uint32_t>();
    }
    ma.wout = P.wout.as<float>();
    ma.bout = net->beta[net->n_linear - 1][0];
    ma.n_linear = net->n_linear;
    ma.wpad = net->wpad;
    ma.out_stride = 1;
    return ma;
}

FeatArgs prepare_feat_args(const Net* net, int prec, const Medium* M, LightState* ls, const Params& P,
                           hipStream_t s)
{
    ensure_sweep(M, ls, s);
    refresh_tables(M, ls, P.phase, P.volume, s, true);
    return feat_args(net, prec, M, ls, P, make_view(M, ls, P, net));
}

void run_query_in(const WsView& ws, const Net* net, int prec, const Medium* M, LightState* ls, const Params& Pm,
                  const float* d_pts, const float* d_dirs, int64_t n, const int* d_count, const QueryOut& o,
                  hipStream_t s, bool may_alloc)
{
    if (!net) fail(NIS_E_STATE, "no weights set");
    if (Pm.channels != 1 && (Pm.channels != 3 || o.y || o.desc)) fail(NIS_E_INVALID, "bad channel count");
    if (ws.chunk <= 0 || !ws.desc || !ws.f0) fail(NIS_E_INTERNAL, "no scratch");
    if (prec == kPrecFP8 && !net->has_fp8)
        fail(NIS_E_UNSUPPORTED, "FP8 needs the activation scales: pass them in the weight blob or call nis_calibrate_fp8");
    if (Pm.templates && Pm.volume)
        fail(NIS_E_UNSUPPORTED, "volume phases are not available with the paper's templates");
    if (Pm.modules) {
        if (!Pm.templates) fail(NIS_E_STATE, "the paper's backbone reads the paper's templates (nis_set_templates)");
        if (!net->has_modules) fail(NIS_E_STATE, "the weights hold no backbone modules");
        if (!ws.feat) fail(NIS_E_UNSUPPORTED, "the paper's backbone needs a template feature workspace");
        if (ws.chunk > kModuleChunk) fail(NIS_E_INTERNAL, "module pass too large");
    }
    ensure_sweep(M, ls, s);
    if (Pm.templates) refresh_tpl_tables(ls, Pm.phase, s, may_alloc);
    else refresh_tables(M, ls, Pm.phase, Pm.volume, s, may_alloc);
    const int64_t chunk = ws.chunk;
    MediumView mv = make_view(M, ls, Pm, net);
    for (int64_t p0 = 0; p0 < n; p0 += chunk) {
        const int64_t cn = (n - p0) < chunk ? (n - p0) : chunk;
        FeatArgs fa = feat_args(net, prec, M, ls, Pm, mv);
        fa.pts = d_pts + 3 * p0;
        fa.dirs = d_dirs + 3 * p0;
        fa.npts = cn;
        fa.count = d_count;
        fa.count_off = p0;
        fa.desc = ws.desc;
        fa.f0 = o.f0 ? o.f0 + p0 : ws.f0;
        auto off = [&](float* base, int64_t per) { return base ? base + p0 * per : nullptr; };
        fa.dbg_tbar = off(o.tbar, kLayers * kSites);
        fa.dbg_rho = off(o.rho, kLayers * kSites);
        fa.dbg_phi = off(o.phi, kSites);
        fa.dbg_stats = off(o.stats, kLayers * kStats);
        fa.dbg_tp = off(o.tp, 1);
        if (Pm.templates) {
            TplArgs ta;
            std::memset(&ta, 0, sizeof(ta));
            const TplGeometry& G = tpl_geometry();
            ta.mv = mv;
            ta.tab = ls->tpl.as<TplTables>();
            ta.pts = fa.pts;
            ta.dirs = fa.dirs;
            ta.npts = cn;
            for (int m = 0; m < M->levels; m++)
                ta.coef[m] = (float)(std::pow((double)net->lam, m + 1) * (double)Pm.sigma_t);
            for (int k = 0; k < kDiffuse; k++) {
                ta.radius[k] = G.radius[k];
                ta.mdiff[k] = tpl_level_host(G.radius[k] * G.D[k], M->n, M->levels);
            }
            for (int h = 0; h < kLayers - kDiffuse; h++) ta.dh[h] = G.D[kDiffuse + h];
            // with the backbone modules the features go to the FP32 rows they read
            ta.desc = Pm.modules ? (void*)ws.feat : fa.desc;
            ta.desc_inv_scale = Pm.modules ? 1.f : fa.desc_inv_scale;
            ta.feat_only = Pm.modules ? 1 : 0;
            ta.f0 = fa.f0;
            ta.dbg_tbar = o.tbar ? o.tbar + p0 * kTplSites : nullptr;
            ta.dbg_rho = o.rho ? o.rho + p0 * kTplSites : nullptr;
            ta.dbg_phi = o.phi ? o.phi + p0 * kTplSites : nullptr;
            ta.dbg_stats = fa.dbg_stats;
            ta.count = d_count;
            ta.count_off = p0;
            const int tprec = Pm.modules ? kPrecFP32 : prec;
            timed("features", s, [&] { return launch_template_features(tprec, ta, s); });
            if (Pm.modules)
                timed("modules", s, [&] {
                    return launch_modules(prec, ws.feat, net->mod.as<float>(), cn, d_count, p0, ws.desc,
                                          fa.desc_inv_scale, Pm.albedo, s);
                });
        } else {
            timed("features", s, [&] { return launch_features(prec, fa, s); });
        }
        if (o.desc) {
            size_t eb = desc_row_bytes(prec);
            hip_check(hipMemcpyAsync((char*)o.desc + p0 * eb, ws.desc, cn * eb, hipMemcpyDeviceToDevice, s),
                      "descriptor copy");
        }
        if (!o.run_mlp) continue;
        MlpArgs ma = mlp_args(net, prec);
        ma.x = ws.desc;
        ma.npts = cn;
        ma.count = d_count;
        ma.count_off = p0;
        ma.absmax = o.absmax;
        ma.f0 = fa.f0;
        ma.radiance = Pm.radiance;
        ma.out_stride = Pm.channels;
        // colour channels share the features; each rewrites the albedo entry
        // (the features stored channel 0's) and runs the backbone
        for (int c = 0; c < Pm.channels; c++) {
            const float eta = Pm.channels == 3 ? Pm.rgb[c] : Pm.albedo;
            if (c > 0) {
                const float stored = prec == kPrecFP8 ? eta * fa.desc_inv_scale : eta;
                timed("albedo_entry", s,
                      [&] { return launch_albedo_entry(prec, ws.desc, cn, d_count, p0, stored, s); });
            }
            ma.out = o.radiance ? o.radiance + p0 * Pm.channels + c : nullptr;
            ma.y_out = o.y && c == 0 ? o.y + p0 : nullptr;
            ma.albedo_gamma = (float)std::pow((double)eta, (double)net->gamma);
            timed("backbone", s, [&] { return launch_mlp(prec, ma, s); });
        }
    }
}

// ---- frames -----------------------------------------------------------------

size_t frame_work_bytes(int64_t npix)
{
    size_t scan = 0;
    hip_check(frame_scan_bytes(npix, &scan), "scan storage size");
    return frame_fixed_bytes(npix) + scan;
}

void FrameWork::reserve(int64_t n)
{
    if (n <= npix) return;
    const size_t N = (size_t)n;
    flag.reserve(N * 4, "frame flags");
    offset.reserve(N * 4, "frame offsets");
    pts.reserve(N * 12, "frame points");
    dirs.reserve(N * 12, "frame directions");
    cpts.reserve(N * 12, "frame points");
    cdirs.reserve(N * 12, "frame directions");
    cpix.reserve(N * 4, "frame pixels");
    L.reserve(N * 4, "frame radiance");
    count.reserve(256, "frame count");
    size_t sb = 0;
    hip_check(frame_scan_bytes(n, &sb), "scan storage size");
    scan.reserve(sb ? sb : 1, "scan storage");
    npix = n;
}

FrameBuffers FrameWork::view() const
{
    FrameBuffers fb;
    fb.flag = flag.as<int>();
    fb.offset = offset.as<int>();
    fb.pts = pts.as<float>();
    fb.dirs = dirs.as<float>();
    fb.cpts = cpts.as<float>();
    fb.cdirs = cdirs.as<float>();
    fb.cpix = cpix.as<int>();
    fb.count = count.as<int>();
    fb.scan_tmp = scan.p;
    fb.scan_bytes = scan.bytes;
    return fb;
}

size_t FrameWork::bytes() const
{
    return flag.bytes + offset.bytes + pts.bytes + dirs.bytes + cpts.bytes + cdirs.bytes + cpix.bytes + L.bytes +
           count.bytes + scan.bytes + L3.bytes;
}

void FrameWork::release()
{
    for (DevBuf* b : {&flag, &offset, &pts, &dirs, &cpts, &cdirs, &cpix, &count, &scan, &L, &L3}) b->release();
    npix = 0;
}

CamArgs camera_args(const nis_camera* cam)
{
    if (!cam) fail(NIS_E_INVALID, "camera is NULL");
    if (cam->width < 1 || cam->height < 1 || (int64_t)cam->width * cam->height > ((int64_t)1 << 28))
        fail(NIS_E_INVALID, "image size must be positive with at most 2^28 pixels");
    CamArgs C;
    std::memset(&C, 0, sizeof(C));
    C.width = cam->width;
    C.height = cam->height;
    if (cam->vfov_deg == 0.0) {
        if (!std::isfinite(cam->ortho_z)) fail(NIS_E_INVALID, "ortho_z must be finite");
        C.ortho = 1;
        C.oz = cam->ortho_z;
        return C;
    }
    if (!(cam->vfov_deg > 0.0 && cam->vfov_deg < 180.0)) fail(NIS_E_INVALID, "vfov_deg must be 0 or in (0,180)");
    double f[3], up[3];
    for (int d = 0; d < 3; d++) {
        if (!std::isfinite(cam->eye[d]) || !std::isfinite(cam->target[d]) || !std::isfinite(cam->up[d]))
            fail(NIS_E_INVALID, "camera vectors must be finite");
        C.eye[d] = cam->eye[d];
        f[d] = cam->target[d] - cam->eye[d];
        up[d] = cam->up[d];
    }
    const double fn = std::sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    if (!(fn > 0.0)) fail(NIS_E_INVALID, "eye and target coincide");
    for (int d = 0; d < 3; d++) C.f[d] = f[d] / fn;
    double r[3] = {C.f[1] * up[2] - C.f[2] * up[1], C.f[2] * up[0] - C.f[0] * up[2], C.f[0] * up[1] - C.f[1] * up[0]};
    const double rn = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    if (!(rn > 0.0)) fail(NIS_E_INVALID, "up is parallel to the view direction");
    for (int d = 0; d < 3; d++) C.r[d] = r[d] / rn;
    C.u[0] = C.r[1] * C.f[2] - C.r[2] * C.f[1];
    C.u[1] = C.r[2] * C.f[0] - C.r[0] * C.f[2];
    C.u[2] = C.r[0] * C.f[1] - C.r[1] * C.f[0];
    C.aspect = (double)cam->width / (double)cam->height;
    C.tan_half = std::tan(cam->vfov_deg * (M_PI / 180.0) * 0.5);
    return C;
}

void frame_points(FrameWork& fw, const Medium* M, const Params& P, const CamArgs& C, uint64_t seed, float* d_pts,
                  float* d_dirs, int* d_pix, int* d_count, hipStream_t s)
{
    const int64_t npix = (int64_t)C.width * C.height;
    fw.reserve(npix);
    FrameBuffers fb = fw.view();
    if (d_pts) {
        fb.cpts = d_pts;
        fb.cdirs = d_dirs;
        fb.cpix = d_pix;
        fb.count = d_count;
    }
    const double sigma_t = P.sigma_t, majorant = sigma_t * (double)M->rmax;
    timed("raygen", s,
          [&] { return launch_raygen(C, M->rho.as<float>(), M->n, sigma_t, majorant, seed, fb, s); });
}

void render_frame(Workspace& ws, FrameWork& fw, const Net* net, int prec, const Medium* M, LightState* ls,
                  const Params& P, const CamArgs& C, uint64_t seed, float* d_image, hipStream_t s)
{
    if (!net) fail(NIS_E_STATE, "no weights set");
    if (!ls->valid) fail(NIS_E_STATE, "no light set for this medium");
    const int64_t npix = (int64_t)C.width * C.height;
    // collisions in bands of rows: the result of a point does not depend on
    // its place in the batch, and compact patches share more of their bricks
    CamArgs Cb = C;
    Cb.band = kRenderBand;
    frame_points(fw, M, P, Cb, seed, nullptr, nullptr, nullptr, nullptr, s);
    FrameBuffers fb = fw.view();
    QueryOut o;
    o.radiance = fw.L.as<float>();
    if (P.channels == 3) {
        fw.L3.reserve((size_t)fw.npix * 3 * sizeof(float), "frame radiance");
        o.radiance = fw.L3.as<float>();
    }
    run_query(ws, net, prec, M, ls, P, fb.cpts, fb.cdirs, npix, fb.count, o, s);
    if (P.channels == 3)
        timed("image", s, [&] { return launch_image_rgb(fb, npix, fw.L3.as<float>(), P.rgb, d_image, s); });
    else
        timed("image", s, [&] { return launch_image(fb, npix, fw.L.as<float>(), P.albedo, d_image, s); });
}

// Synchronous query of host arrays: channels = 1 (grey) or 3 (RGB, [n][3] out).
void query_host(nis_ctx* ctx, int32_t medium, const float* points, const float* dirs, int64_t n, float* out,
                int channels)
{
    check_ctx(ctx);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!points || !dirs || !out || n <= 0) fail(NIS_E_INVALID, "bad query arguments");
    for (int64_t i = 0; i < n; i++) {
        if (!finite3(points + 3 * i) || !finite3(dirs + 3 * i)) fail(NIS_E_INVALID, "non-finite query input");
        const float* d = dirs + 3 * i;
        if (d[0] == 0.f && d[1] == 0.f && d[2] == 0.f) fail(NIS_E_INVALID, "zero view direction");
    }
    Medium* M = get_medium(ctx, medium);
    const Params P = with_templates(ctx, channels == 3 ? rgb_params(M) : grey_params(M));
    if (!ctx->net) fail(NIS_E_STATE, "no weights set");
    if (!M->light.valid) fail(NIS_E_STATE, "no light set for this medium");
    const size_t bytes = (size_t)n * (6 + channels) * sizeof(float);
    StreamUse su(ctx, ctx->stream);
    ctx->io.reserve(bytes, "query staging");
    float* d_pts = ctx->io.as<float>();
    float* d_dirs = d_pts + 3 * n;
    float* d_out = d_dirs + 3 * n;
    hip_check(hipMemcpyAsync(d_pts, points, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, ctx->stream),
              "upload");
    hip_check(hipMemcpyAsync(d_dirs, dirs, (size_t)n * 3 * sizeof(float), hipMemcpyHostToDevice, ctx->stream),
              "upload");
    QueryOut o;
    o.radiance = d_out;
    run_query(ctx->ws, ctx->net, ctx->precision, M, &M->light, P, d_pts, d_dirs, n, nullptr, o, ctx->stream);
    hip_check(hipMemcpyAsync(out, d_out, (size_t)n * channels * sizeof(float), hipMemcpyDeviceToHost, ctx->stream),
              "download");
    hip_check(hipStreamSynchronize(ctx->stream), "query");
}

}  // namespace nis

using namespace nis;

// ---- C ABI ------------------------------------------------------------------

extern "C" {

const char* nis_last_error(void) { return g_err.c_str(); }

int32_t nis_create(int32_t hip_device, nis_ctx** out)
{
    return guard([&] {
        if (!out) fail(NIS_E_INVALID, "out is NULL");
        *out = nullptr;
        int count = 0;
        hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
        if (hip_device < 0 || hip_device >= count) fail(NIS_E_INVALID, "no such HIP device");
        hip_check(hipSetDevice(hip_device), "hipSetDevice");
        scratch_setup(hip_device);
        nis_ctx* ctx = new nis_ctx();
        ctx->device = hip_device;
        hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->order, hipEventDisableTiming);
        if (e != hipSuccess) {
            if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
            delete ctx;
            hip_check(e, "hipStreamCreate");
        }
        *out = ctx;
    });
}

int32_t nis_destroy(nis_ctx* ctx)
{
    if (!ctx) return NIS_OK;
    return guard([&] {
        (void)hipSetDevice(ctx->device);
        server_shutdown(ctx);
        (void)hipDeviceSynchronize();
        for (auto& kv : ctx->media) free_medium(kv.second);
        free_net(ctx->net);
        ctx->ws.release();
        ctx->fw.release();
        ctx->io.release();
        ctx->batch_y.release();
        ctx->batch_tab.release();
        (void)hipEventDestroy(ctx->order);
        (void)hipStreamDestroy(ctx->stream);
        delete ctx;
    });
}

int32_t nis_load_medium(nis_ctx* ctx, const float* density, int32_t n, float sigma_t, float albedo, float g,
                        int32_t* medium_out)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!density || !medium_out) fail(NIS_E_INVALID, "density or medium_out is NULL");
        if (n < 1 || n > 1024 || (n & (n - 1)) != 0) fail(NIS_E_INVALID, "n must be a power of two in [1,1024]");
        validate_params(sigma_t, albedo, g);
        const int64_t n3 = (int64_t)n * n * n;
        float rmax = 0.f;
        for (int64_t i = 0; i < n3; i++) {
            if (!(std::isfinite(density[i]) && density[i] >= 0.f)) fail(NIS_E_INVALID, "density must be finite and >= 0");
            rmax = density[i] > rmax ? density[i] : rmax;
        }
        Medium* M = new Medium();
        try {
            M->n = n;
            M->sigma_t = sigma_t;
            M->albedo = albedo;
            for (int c = 0; c < 3; c++) M->albedo_rgb[c] = albedo;
            M->phase = single_lobe(g);
            M->rmax = rmax;
            const int L = pyramid_levels(M, n);
            const int64_t off = M->rho_floats;
            M->rho.reserve((size_t)off * sizeof(float), "density pyramid");
            hip_check(hipMemcpyAsync(M->rho.p, density, (size_t)n3 * sizeof(float), hipMemcpyHostToDevice,
                                     ctx->stream), "density upload");
            hip_check(launch_pyramid(M->rho.as<float>(), M->lev, L, ctx->stream), "pyramid launch");
            hip_check(hipStreamSynchronize(ctx->stream), "pyramid");
        } catch (...) {
            free_medium(M);
            throw;
        }
        int32_t id = ctx->next_id++;
        ctx->media[id] = M;
        *medium_out = id;
    });
}

int32_t nis_rebuild_pyramid(nis_ctx* ctx, int32_t medium, void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        no_server(ctx, "rebuilding a pyramid");
        Medium* M = get_medium(ctx, medium);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        hipStream_t s = su.s;
        timed("pyramid", s, [&] { return launch_pyramid(M->rho.as<float>(), M->lev, M->levels, s); });
        M->version++;
    });
}

int32_t nis_set_medium_params(nis_ctx* ctx, int32_t medium, float sigma_t, float albedo, float g)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        validate_params(sigma_t, albedo, g);
        M->sigma_t = sigma_t;
        M->albedo = albedo;
        for (int c = 0; c < 3; c++) M->albedo_rgb[c] = albedo;
        M->phase = single_lobe(g);
    });
}

int32_t nis_set_albedo_rgb(nis_ctx* ctx, int32_t medium, const float* albedo_rgb)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (!albedo_rgb) fail(NIS_E_INVALID, "albedo_rgb is NULL");
        for (int c = 0; c < 3; c++)
            if (!(std::isfinite(albedo_rgb[c]) && albedo_rgb[c] >= 0.f && albedo_rgb[c] <= 1.f))
                fail(NIS_E_INVALID, "albedo must be in [0,1]");
        for (int c = 0; c < 3; c++) M->albedo_rgb[c] = albedo_rgb[c];
        if (grey_albedo(M)) M->albedo = albedo_rgb[0];
    });
}

int32_t nis_set_volume_phase(nis_ctx* ctx, int32_t medium, int32_t enable)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (enable != 0 && enable != 1) fail(NIS_E_INVALID, "enable must be 0 or 1");
        if (enable == 1 && M->light.valid)
            M->light.vtab.reserve((size_t)kSites * kVBins * sizeof(float), "volume phase tables");
        M->volume_phase = enable == 1;
    });
}

int32_t nis_set_phase_lobes(nis_ctx* ctx, int32_t medium, int32_t n, const float* weights, const float* g)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (!weights || !g) fail(NIS_E_INVALID, "weights or g is NULL");
        if (n < 1 || n > kMaxLobes) fail(NIS_E_INVALID, "the phase takes 1 to 4 lobes");
        Phase ph = {};
        ph.n = n;
        double sum = 0.0;
        for (int i = 0; i < n; i++) {
            if (!(std::isfinite(weights[i]) && weights[i] >= 0.f)) fail(NIS_E_INVALID, "lobe weights must be >= 0");
            if (!(std::isfinite(g[i]) && g[i] > -1.f && g[i] < 1.f)) fail(NIS_E_INVALID, "lobe g must be in (-1,1)");
            ph.w[i] = weights[i];
            ph.g[i] = g[i];
            sum += weights[i];
        }
        if (std::fabs(sum - 1.0) > 1e-5) fail(NIS_E_INVALID, "lobe weights must sum to 1");
        M->phase = ph;
    });
}

int32_t nis_unload_medium(nis_ctx* ctx, int32_t medium)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        no_server(ctx, "unloading a medium");
        Medium* M = get_medium(ctx, medium);
        hip_check(hipDeviceSynchronize(), "unload");   // work on any stream may still read it
        ctx->media.erase(medium);
        free_medium(M);
    });
}

int32_t nis_set_light(nis_ctx* ctx, int32_t medium, const float dir[3], float radiance, int32_t flags)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (!std::isfinite(radiance)) fail(NIS_E_INVALID, "light must be finite");
        double l[3];
        unit_light(dir, l);
        set_light_state(M, l, &M->light);
        M->radiance = radiance;
        if (flags & NIS_EAGER) {
            StreamUse su(ctx, ctx->stream);
            ensure_sweep(M, &M->light, su.s);
        }
    });
}

int32_t nis_light_footprint(int32_t n, const float dir[3], int64_t* bytes_out, int64_t* level_bytes)
{
    return guard([&] {
        if (!bytes_out) fail(NIS_E_INVALID, "bytes_out is NULL");
        if (n < 1 || n > 1024 || (n & (n - 1)) != 0) fail(NIS_E_INVALID, "n must be a power of two in [1,1024]");
        double l[3];
        unit_light(dir, l);
        // the layout alone: no device memory is touched
        Medium M;
        pyramid_levels(&M, n);
        LightState ls;
        light_layout(&M, l, &ls);
        *bytes_out = ls.dpair_count * (int64_t)sizeof(float2) + ls.pair_count * (int64_t)sizeof(float2) +
                     ls.rt_floats * (int64_t)sizeof(float);
        if (level_bytes)
            for (int m = 0; m < M.levels; m++) {
                const Level& lv = ls.lev[m];
                level_bytes[m] = (int64_t)lv.nu * (lv.nv + 1) * lv.n * (int64_t)sizeof(float2);
            }
    });
}

int32_t nis_set_weights(nis_ctx* ctx, const void* blob, size_t nbytes)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        no_server(ctx, "replacing the weights");
        if (!blob || nbytes < sizeof(BlobHeader)) fail(NIS_E_INVALID, "weight blob too short");
        BlobHeader h;
        std::memcpy(&h, blob, sizeof(h));
        if (std::memcmp(h.magic, "NISW", 4) != 0 || h.version != 1) fail(NIS_E_INVALID, "bad blob magic/version");
        if (h.din != (uint32_t)kDesc || h.groups != 2) fail(NIS_E_INVALID, "blob din/groups mismatch");
        if (h.n_linear < 2 || h.n_linear > 16) fail(NIS_E_INVALID, "n_linear must be in [2,16]");
        if (h.width < 1 || mlp_padded_width((int)h.width) < 0) fail(NIS_E_INVALID, "unsupported width");
        if (!(std::isfinite(h.lam) && h.lam > 0.f && h.lam <= 1.f)) fail(NIS_E_INVALID, "lambda must be in (0,1]");
        if (!(std::isfinite(h.gamma) && h.gamma >= 0.f)) fail(NIS_E_INVALID, "gamma must be >= 0");
        size_t need = 2 * (size_t)kGroupFloats;
        std::vector<int> din(h.n_linear), dout(h.n_linear);
        for (uint32_t i = 0; i < h.n_linear; i++) {
            din[i] = i == 0 ? kDesc : (int)h.width;
            dout[i] = i + 1 == h.n_linear ? 1 : (int)h.width;
            need += (size_t)din[i] * dout[i] + dout[i];
        }
        if (h.has_fp8_scales) need += 2 + h.n_linear;
        if (h.has_modules > 1) fail(NIS_E_INVALID, "has_modules must be 0 or 1");
        if (h.has_modules) need += (size_t)module_floats_total();
        if (nbytes != sizeof(BlobHeader) + need * sizeof(float)) fail(NIS_E_INVALID, "blob size mismatch");
        const float* f = reinterpret_cast<const float*>((const char*)blob + sizeof(BlobHeader));
        std::vector<float> all(f, f + need);
        for (float v : all)
            if (!std::isfinite(v)) fail(NIS_E_INVALID, "blob holds a non-finite value");
        Net* net = new Net();
        try {
            net->width = (int)h.width;
            net->n_linear = (int)h.n_linear;
            net->wpad = mlp_padded_width(net->width);
            net->lam = h.lam;
            net->gamma = h.gamma;
            net->has_fp8 = h.has_fp8_scales != 0;
            net->has_modules = h.has_modules != 0;
            size_t pos = 0;
            for (int gi = 0; gi < 2; gi++) {
                net->groups[gi].assign(all.begin() + pos, all.begin() + pos + kGroupFloats);
                pos += kGroupFloats;
            }
            for (int i = 0; i < net->n_linear; i++) {
                size_t na = (size_t)din[i] * dout[i];
                net->A.emplace_back(all.begin() + pos, all.begin() + pos + na);
                pos += na;
                net->beta.emplace_back(all.begin() + pos, all.begin() + pos + dout[i]);
                pos += dout[i];
            }
            if (net->has_fp8) {
                net->fp8_scales.assign(all.begin() + pos, all.begin() + pos + 2 + net->n_linear);
                pos += 2 + net->n_linear;
                for (float v : net->fp8_scales)
                    if (!(v > 0.f)) fail(NIS_E_INVALID, "FP8 activation scales must be > 0");
            }
            if (net->has_modules) {
                net->modules.assign(all.begin() + pos, all.end());
                std::vector<float> packed((size_t)module_packed_floats());
                pack_modules(net->modules.data(), packed.data());
                upload_vec(net->mod, packed, "backbone modules");
            }
            pack_net(net, kPrecFP32);
            pack_net(net, kPrecBF16);
            pack_net(net, kPrecFP8);
        } catch (...) {
            free_net(net);
            throw;
        }
        hip_check(hipDeviceSynchronize(), "weights");   // queries on any stream may read the old ones
        free_net(ctx->net);
        ctx->net = net;
    });
}

int32_t nis_set_precision(nis_ctx* ctx, int32_t precision)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (precision != NIS_FP32 && precision != NIS_BF16 && precision != NIS_FP8)
            fail(NIS_E_INVALID, "unknown precision");
        if (precision == NIS_FP8 && ctx->net && !ctx->net->has_fp8)
            fail(NIS_E_UNSUPPORTED, "FP8 needs the activation scales: pass them in the weight blob or call "
                                    "nis_calibrate_fp8");
        ctx->precision = precision;
    });
}

int32_t nis_query_device(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs, int64_t n,
                         float* d_out, void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || !d_out || n <= 0) fail(NIS_E_INVALID, "bad query arguments");
        Medium* M = get_medium(ctx, medium);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        hipStream_t s = su.s;
        QueryOut o;
        o.radiance = d_out;
        run_query(ctx->ws, ctx->net, ctx->precision, M, &M->light, with_templates(ctx, grey_params(M)), d_points, d_dirs, n, nullptr,
                  o, s);
    });
}

int32_t nis_set_templates(nis_ctx* ctx, int32_t kind)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (kind != NIS_TEMPLATES_LATTICE && kind != NIS_TEMPLATES_PAPER) fail(NIS_E_INVALID, "unknown template kind");
        ctx->templates = kind;
    });
}

int32_t nis_set_backbone(nis_ctx* ctx, int32_t kind)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (kind != NIS_BACKBONE_MLP && kind != NIS_BACKBONE_PAPER) fail(NIS_E_INVALID, "unknown backbone kind");
        if (kind == NIS_BACKBONE_PAPER && ctx->net && !ctx->net->has_modules)
            fail(NIS_E_STATE, "the weights hold no backbone modules");
        ctx->backbone = kind;
    });
}

int32_t nis_debug_template_features(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs,
                                    int64_t n, float* d_tbar, float* d_rho, float* d_phi, float* d_stats,
                                    float* d_f0)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || n <= 0 || !d_tbar || !d_rho || !d_phi || !d_stats)
            fail(NIS_E_INVALID, "bad arguments");
        Medium* M = get_medium(ctx, medium);
        hip_check(hipDeviceSynchronize(), "sync");
        QueryOut o;
        o.tbar = d_tbar;
        o.rho = d_rho;
        o.phi = d_phi;
        o.stats = d_stats;
        o.f0 = d_f0;
        o.run_mlp = false;
        Params P = grey_params(M);
        P.templates = NIS_TEMPLATES_PAPER;
        run_query(ctx->ws, ctx->net, ctx->precision, M, &M->light, P, d_points, d_dirs, n, nullptr, o, ctx->stream);
        hip_check(hipStreamSynchronize(ctx->stream), "template features");
    });
}

int32_t nis_calibrate_fp8(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs, int64_t n,
                          void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        no_server(ctx, "calibrating the FP8 scales");
        if (!d_points || !d_dirs || n <= 0) fail(NIS_E_INVALID, "bad calibration arguments");
        Medium* M = get_medium(ctx, medium);
        if (!ctx->net) fail(NIS_E_STATE, "no weights set");
        Net* net = ctx->net;
        const Params P = with_templates(ctx, grey_params(M));
        DevBuf amax;
        amax.reserve((size_t)net->n_linear * sizeof(float), "calibration maxima");
        std::vector<float> h(net->n_linear, 0.f);
        try {
            StreamUse su(ctx, (hipStream_t)hip_stream);
            hip_check(hipMemsetAsync(amax.p, 0, amax.bytes, su.s), "calibration maxima");
            QueryOut o;
            o.absmax = amax.as<float>();
            run_query(ctx->ws, net, kPrecFP32, M, &M->light, P, d_points, d_dirs, n, nullptr, o, su.s);
            hip_check(hipMemcpyAsync(h.data(), amax.p, h.size() * sizeof(float), hipMemcpyDeviceToHost, su.s),
                      "calibration maxima");
            hip_check(hipStreamSynchronize(su.s), "calibration");
        } catch (...) {
            amax.release();
            throw;
        }
        amax.release();
        // x = code * s with s = 2 max|x| / 448: a factor of two of headroom
        // above the calibration points' range (codes saturate at 448)
        std::vector<float> sc(2 + net->n_linear, 1.f);
        for (int i = 0; i < net->n_linear; i++) {
            if (!std::isfinite(h[i])) fail(NIS_E_INTERNAL, "non-finite calibration maximum");
            sc[2 + i] = h[i] > 0.f ? 2.f * h[i] / 448.f : 1.f;
        }
        hip_check(hipDeviceSynchronize(), "calibration");   // FP8 queries on any stream may read the old weights
        net->fp8_scales = sc;
        net->has_fp8 = true;
        pack_net(net, kPrecFP8);
    });
}

int32_t nis_query_device_noalloc(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs,
                                 int64_t n, float* d_out, void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || !d_out || n <= 0) fail(NIS_E_INVALID, "bad query arguments");
        if (n > NIS_NOALLOC_MAX_POINTS)
            fail(NIS_E_INVALID, "the allocation-free query takes at most " + std::to_string(NIS_NOALLOC_MAX_POINTS) +
                                    " points per call");
        Medium* M = get_medium(ctx, medium);
        const Params P = with_templates(ctx, grey_params(M));
        if (!M->light.valid) fail(NIS_E_STATE, "no light set for this medium");
        const WsView w = scratch_view(ctx->device, ctx->precision, n);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        QueryOut o;
        o.radiance = d_out;
        run_query_in(w, ctx->net, ctx->precision, M, &M->light, P, d_points, d_dirs, n, nullptr, o, su.s, false);
    });
}

int32_t nis_query_batch(nis_ctx* ctx, const nis_query_item* items, int32_t count, void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!items || count <= 0 || count > kMaxBatch) fail(NIS_E_INVALID, "a batch holds 1 to 64 queries");
        const Net* net = ctx->net;
        if (!net) fail(NIS_E_STATE, "no weights set");
        const int prec = ctx->precision;
        if (prec == kPrecFP8 && !net->has_fp8)
            fail(NIS_E_UNSUPPORTED, "FP8 needs the activation scales: pass them in the weight blob or call nis_calibrate_fp8");
        if (ctx->templates != NIS_TEMPLATES_LATTICE)
            fail(NIS_E_UNSUPPORTED, "batched queries sample the lattice templates");
        int64_t total = 0;
        std::vector<Medium*> media(count);
        for (int32_t i = 0; i < count; i++) {
            const nis_query_item& it = items[i];
            if (it.n < 0 || it.reserved != 0 || (it.n > 0 && (!it.d_points || !it.d_view_dirs || !it.d_radiance_out)))
                fail(NIS_E_INVALID, "bad batch item");
            media[i] = get_medium(ctx, it.medium);
            if (!grey_albedo(media[i])) fail(NIS_E_STATE, "a coloured medium needs the RGB query");
            total += it.n;
        }
        if (total > kChunk) fail(NIS_E_INVALID, "a batch holds at most 2^21 points");
        if (total == 0) return;
        StreamUse su(ctx, (hipStream_t)hip_stream);
        const hipStream_t s = su.s;
        Workspace& ws = ctx->ws;
        const size_t rb = desc_row_bytes(prec);
        ws.desc.reserve((size_t)total * rb, "descriptor workspace");
        ws.f0.reserve((size_t)total * sizeof(float), "single-scatter workspace");
        ctx->batch_y.reserve((size_t)total * sizeof(float), "batch network outputs");
        // each query's light fields and tables, then its gather arguments
        std::vector<FeatArgs> tab(count);
        FeatMulti fm;
        std::memset(&fm, 0, sizeof(fm));
        fm.n = count;
        int64_t base = 0, blocks = 0;
        for (int32_t i = 0; i < count; i++) {
            Medium* M = media[i];
            tab[i] = prepare_feat_args(net, prec, M, &M->light, grey_params(M), s);
            tab[i].pts = items[i].d_points;
            tab[i].dirs = items[i].d_view_dirs;
            tab[i].npts = items[i].n;
            tab[i].desc = static_cast<char*>(ws.desc.p) + (size_t)base * rb;
            tab[i].f0 = ws.f0.as<float>() + base;
            fm.first[i] = (int)blocks;
            blocks += items[i].n > 0 ? features_blocks(items[i].n) : 0;
            base += items[i].n;
        }
        if (blocks > 0x7fffffff) fail(NIS_E_INVALID, "batch too large");
        fm.first[count] = (int)blocks;
        // the table from pageable memory: the copy has read it when the call returns
        ctx->batch_tab.reserve(sizeof(FeatArgs) * count, "batch table");
        hip_check(hipMemcpyAsync(ctx->batch_tab.p, tab.data(), sizeof(FeatArgs) * count, hipMemcpyHostToDevice, s),
                  "batch table");
        fm.table = ctx->batch_tab.as<FeatArgs>();
        bool big = false;
        for (int32_t i = 0; i < count; i++) big |= big_fields(tab[i].mv);
        timed("features", s, [&] { return launch_features_multi(prec, fm, big, s); });
        // one backbone pass over every query's rows, then each query's decode
        MlpArgs ma = mlp_args(net, prec);
        ma.x = ws.desc.p;
        ma.npts = total;
        ma.f0 = ws.f0.as<float>();
        ma.y_out = ctx->batch_y.as<float>();
        timed("backbone", s, [&] { return launch_mlp(prec, ma, s); });
        base = 0;
        for (int32_t i = 0; i < count; i++) {
            const Medium* M = media[i];
            const float ag = (float)std::pow((double)M->albedo, (double)net->gamma);
            timed("decode", s, [&] {
                return launch_decode(ctx->batch_y.as<float>() + base, ws.f0.as<float>() + base, items[i].n,
                                     M->radiance, ag, items[i].d_radiance_out, s);
            });
            base += items[i].n;
        }
    });
}

int32_t nis_query(nis_ctx* ctx, int32_t medium, const float* points, const float* dirs, int64_t n,
                  float* radiance_out)
{
    return guard([&] { query_host(ctx, medium, points, dirs, n, radiance_out, 1); });
}

int32_t nis_query_rgb(nis_ctx* ctx, int32_t medium, const float* points, const float* dirs, int64_t n,
                      float* radiance_out)
{
    return guard([&] { query_host(ctx, medium, points, dirs, n, radiance_out, 3); });
}

int32_t nis_query_rgb_device(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs, int64_t n,
                             float* d_out, void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || !d_out || n <= 0) fail(NIS_E_INVALID, "bad query arguments");
        Medium* M = get_medium(ctx, medium);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        QueryOut o;
        o.radiance = d_out;
        run_query(ctx->ws, ctx->net, ctx->precision, M, &M->light, with_templates(ctx, rgb_params(M)), d_points, d_dirs, n, nullptr, o,
                  su.s);
    });
}

int32_t nis_frame_points(nis_ctx* ctx, int32_t medium, const nis_camera* camera, uint64_t seed, float* d_points,
                         float* d_dirs, int32_t* d_pixel, int32_t* d_count, void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || !d_pixel || !d_count) fail(NIS_E_INVALID, "output arrays must not be NULL");
        Medium* M = get_medium(ctx, medium);
        CamArgs C = camera_args(camera);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        hipStream_t s = su.s;
        frame_points(ctx->fw, M, medium_params(M), C, seed, d_points, d_dirs, d_pixel, d_count, s);
    });
}

int32_t nis_render(nis_ctx* ctx, int32_t medium, const nis_camera* camera, uint64_t seed, float* d_image,
                   void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_image) fail(NIS_E_INVALID, "image is NULL");
        Medium* M = get_medium(ctx, medium);
        CamArgs C = camera_args(camera);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        hipStream_t s = su.s;
        render_frame(ctx->ws, ctx->fw, ctx->net, ctx->precision, M, &M->light, with_templates(ctx, grey_params(M)), C, seed, d_image,
                     s);
    });
}

int32_t nis_render_rgb(nis_ctx* ctx, int32_t medium, const nis_camera* camera, uint64_t seed, float* d_image,
                       void* hip_stream)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_image) fail(NIS_E_INVALID, "image is NULL");
        Medium* M = get_medium(ctx, medium);
        CamArgs C = camera_args(camera);
        StreamUse su(ctx, (hipStream_t)hip_stream);
        render_frame(ctx->ws, ctx->fw, ctx->net, ctx->precision, M, &M->light, with_templates(ctx, rgb_params(M)), C, seed, d_image,
                     su.s);
    });
}

int32_t nis_profile(nis_ctx* ctx, int32_t enable)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        hip_check(hipDeviceSynchronize(), "sync");
        ctx->prof.clear();
        ctx->prof.on = enable != 0;
    });
}

int32_t nis_profile_report(nis_ctx* ctx, char* buf, size_t capacity)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!buf || capacity == 0) fail(NIS_E_INVALID, "buffer is NULL");
        std::map<std::string, std::pair<int64_t, double>> agg;
        for (auto& r : ctx->prof.recs) {
            hip_check(hipEventSynchronize(r.b), "hipEventSynchronize");
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
            auto& e = agg[r.name];
            e.first += 1;
            e.second += ms;
        }
        std::string out;
        char line[160];
        for (auto& kv : agg) {
            std::snprintf(line, sizeof(line), "%s %lld %.6f\n", kv.first.c_str(), (long long)kv.second.first,
                          kv.second.second);
            out += line;
        }
        if (out.size() + 1 > capacity) fail(NIS_E_INVALID, "buffer too small");
        std::memcpy(buf, out.c_str(), out.size() + 1);
    });
}

int32_t nis_medium_info(nis_ctx* ctx, int32_t medium, int32_t* levels, int64_t* pyramid_floats)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (levels) *levels = M->levels;
        if (pyramid_floats) *pyramid_floats = M->rho_floats;
    });
}

int32_t nis_debug_pyramid(nis_ctx* ctx, int32_t medium, float* out, int64_t capacity)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (!out || capacity < M->rho_floats) fail(NIS_E_INVALID, "output too small");
        hip_check(hipDeviceSynchronize(), "sync");
        hip_check(hipMemcpy(out, M->rho.p, (size_t)M->rho_floats * sizeof(float), hipMemcpyDeviceToHost), "download");
    });
}

int32_t nis_debug_path_density(nis_ctx* ctx, int32_t medium, int32_t level, float* out, int64_t capacity,
                               int32_t dims[5])
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (!dims) fail(NIS_E_INVALID, "dims is NULL");
        if (level < 0 || level >= M->levels) fail(NIS_E_INVALID, "no such level");
        hip_check(hipDeviceSynchronize(), "sync");   // the debug calls see all earlier work
        ensure_sweep(M, &M->light, ctx->stream);
        const Level& lv = M->light.lev[level];
        // the rays of the definition, without the layout's padding
        const int nu = lv.nu - 2 * kRayPad;
        dims[0] = lv.ulo + kRayPad;
        dims[1] = lv.ulo + kRayPad + nu - 1;
        dims[2] = lv.vlo;
        dims[3] = lv.vlo + lv.nv - 1;
        dims[4] = lv.n;
        if (!out) return;
        const int64_t count = (int64_t)nu * lv.nv * lv.n;
        if (capacity < count) fail(NIS_E_INVALID, "output too small");
        // D is stored only inside its pairs along V: D(V) is the second
        // member of pair V' = V
        std::vector<float2> q((size_t)lv.nu * (lv.nv + 1) * lv.n);
        hip_check(hipStreamSynchronize(ctx->stream), "sync");
        hip_check(hipMemcpy(q.data(), M->light.DP.as<float2>() + lv.q_off, q.size() * sizeof(float2),
                            hipMemcpyDeviceToHost),
                  "download");
        for (int64_t j = 0; j < lv.n; j++)
            for (int64_t v = 0; v < lv.nv; v++)
                for (int64_t u = 0; u < nu; u++)
                    out[(j * lv.nv + v) * nu + u] = q[(size_t)((j * (lv.nv + 1) + v) * lv.nu + kRayPad + u)].y;
    });
}

int32_t nis_debug_path_pairs(nis_ctx* ctx, int32_t medium, int32_t level, float* out, int64_t capacity)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        Medium* M = get_medium(ctx, medium);
        if (!out) fail(NIS_E_INVALID, "out is NULL");
        if (level < 0 || level >= M->levels) fail(NIS_E_INVALID, "no such level");
        hip_check(hipDeviceSynchronize(), "sync");
        ensure_sweep(M, &M->light, ctx->stream);
        const Level& lv = M->light.lev[level];
        const int nu = lv.nu - 2 * kRayPad;
        const int64_t count = 2 * (int64_t)nu * (lv.nv + 1) * lv.n;
        if (capacity < count) fail(NIS_E_INVALID, "output too small");
        std::vector<float2> q((size_t)lv.nu * (lv.nv + 1) * lv.n);
        hip_check(hipStreamSynchronize(ctx->stream), "sync");
        hip_check(hipMemcpy(q.data(), M->light.DP.as<float2>() + lv.q_off, q.size() * sizeof(float2),
                            hipMemcpyDeviceToHost),
                  "download");
        // the rays of the definition, without the layout's padding
        for (int64_t r = 0; r < (int64_t)(lv.nv + 1) * lv.n; r++)
            std::memcpy(out + 2 * r * nu, q.data() + r * lv.nu + kRayPad, (size_t)nu * sizeof(float2));
    });
}

int32_t nis_debug_features(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs, int64_t n,
                           float* d_tbar, float* d_rho, float* d_phi, float* d_stats, float* d_tp, float* d_f0)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || n <= 0) fail(NIS_E_INVALID, "bad arguments");
        Medium* M = get_medium(ctx, medium);
        hip_check(hipDeviceSynchronize(), "sync");
        QueryOut o;
        o.tbar = d_tbar;
        o.rho = d_rho;
        o.phi = d_phi;
        o.stats = d_stats;
        o.tp = d_tp;
        o.f0 = d_f0;
        o.run_mlp = false;
        run_query(ctx->ws, ctx->net, ctx->precision, M, &M->light, grey_params(M), d_points, d_dirs, n, nullptr, o,
                  ctx->stream);
        hip_check(hipStreamSynchronize(ctx->stream), "features");
    });
}

int32_t nis_debug_network(nis_ctx* ctx, int32_t medium, const float* d_points, const float* d_dirs, int64_t n,
                          float* d_desc, float* d_y)
{
    return guard([&] {
        check_ctx(ctx);
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (!d_points || !d_dirs || n <= 0) fail(NIS_E_INVALID, "bad arguments");
        Medium* M = get_medium(ctx, medium);
        hip_check(hipDeviceSynchronize(), "sync");
        const int prec = ctx->precision;
        DevBuf raw;
        QueryOut o;
        o.y = d_y;
        if (d_desc) {
            raw.reserve((size_t)n * desc_row_bytes(prec), "descriptor copy");
            o.desc = raw.p;
        }
        try {
            run_query(ctx->ws, ctx->net, prec, M, &M->light, with_templates(ctx, grey_params(M)), d_points, d_dirs, n, nullptr, o,
                      ctx->stream);
            const float dscale = prec == kPrecFP8 ? ctx->net->fp8_scales[2] : 1.f;
            if (d_desc) hip_check(launch_desc_to_f32(prec, raw.p, d_desc, n, dscale, ctx->stream), "descriptor convert");
            hip_check(hipStreamSynchronize(ctx->stream), "network");
        } catch (...) {
            (void)hipStreamSynchronize(ctx->stream);
            raw.release();
            throw;
        }
        raw.release();
    });
}

}  // extern "C"
