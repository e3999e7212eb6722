// launch_args.h -- argument blocks and launchers of the library's kernels.
#pragma once

#include "nis_internal.h"

namespace nis {

constexpr int kMaxLinear = 16;

struct FeatArgs {
    MediumView mv;
    const SiteTables* tab;
    const float* vtab;           // volume phase only: [kSites][kVBins] w-side cone means over the angle
    const float* pts;
    const float* dirs;
    int64_t npts;
    float coef[kLayers];         // lambda^(m+1) * sigma_t per layer
    const void* w1t[2];          // conv1 weights [16 out][32 k], k = tap, zero padded
    const void* w2t[2];          // conv2 weights [16 out][224 k], k = c*27 + tap
    const float* cb[2];          // b1[8] b2[16] s1[64] c1[4] s2[64] c2[16]
    void* desc;                  // [npts][kDescPad] (FP8 output: [npts][kDescF8] E4M3 codes)
    float desc_inv_scale;        // FP8 output only: 1 / the backbone's first input scale
    float* f0;                   // [npts] HG(w.l) T(p)
    float* dbg_tbar;             // optional [npts][12][225]
    float* dbg_rho;              // optional [npts][12][225]
    float* dbg_phi;              // optional [npts][225]
    float* dbg_stats;            // optional [npts][12][8]
    float* dbg_tp;               // optional [npts]
    const int* count;            // optional device point count: the kernel serves
    int64_t count_off;           // min(npts, *count - count_off) points
};

// Several gathers in one launch (nis_query_batch): query r's arguments are
// table[r] (device memory) and its workgroups first[r] .. first[r + 1] - 1,
// features_blocks(npts) of them.
constexpr int kMaxBatch = 64;
struct FeatMulti {
    const FeatArgs* table;
    int n;
    int first[kMaxBatch + 1];
};

// The gather at the paper's templates (k_template_features).
struct TplArgs {
    MediumView mv;
    const TplTables* tab;
    const float* pts;
    const float* dirs;
    int64_t npts;
    float coef[kMaxLevels];      // lambda^(m+1) * sigma_t per level m
    double radius[kDiffuse];     // diffuse layer radii (eq. 4), unit-cube lengths
    int mdiff[kDiffuse];         // diffuse layer levels
    double dh[kLayers - kDiffuse];   // highlight layers' eq. (3) measure of the unit cone sets
    void* desc;                  // [npts][kDescPad] (FP8 output: [npts][kDescF8] E4M3 codes)
    float desc_inv_scale;        // FP8 output only: 1 / the backbone's first input scale
    int feat_only;               // FP32 rows in the backbone modules' layout (mf_block, mf_stats) instead
    float* f0;                   // [npts] f(w.l) T(p)
    float* dbg_tbar;             // optional [npts][kTplSites]
    float* dbg_rho;              // optional [npts][kTplSites]
    float* dbg_phi;              // optional [npts][kTplSites]
    float* dbg_stats;            // optional [npts][12][8]
    const int* count;            // optional device point count, as in FeatArgs
    int64_t count_off;
};

struct MlpArgs {
    const void* x;                   // [npts][kDescPad] descriptor ([npts][kDescF8] codes for FP8)
    int64_t npts;
    const void* W[kMaxLinear];       // layer i, in the kernel's fragment order
    const float* bias[kMaxLinear];   // [wpad], zero padded (FP8: divided by the layer's output scale)
    const uint32_t* wexp[kMaxLinear];// FP8 only: E8M0 weight scale of each output channel, [tiles * 32]
    float* absmax;                   // FP32 only, optional: [n_linear] running max |input| of each layer
    const float* wout;               // [wpad] last-layer weights (float32; FP8: times its input scale)
    float bout;
    int n_linear, wpad;
    const float* f0;                 // [npts]
    float* out;                      // radiance of row r at out[r * out_stride] (may be NULL)
    int64_t out_stride;              // 1, or 3 for one channel of an RGB result
    float* y_out;                    // [npts] network output (may be NULL)
    float albedo_gamma;              // albedo^gamma
    float radiance;
    const int* count;                // optional device point count, as in FeatArgs
    int64_t count_off;
};

constexpr int kMaxTrackingSteps = 100000;   // free flights per camera ray before it is dropped

// Camera of a frame: orthographic rays along -z through the pixel centres of
// the unit square at height oz, or pinhole rays from eye along the
// orthonormal frame (f forward, r right, u up); double precision.
struct CamArgs {
    int ortho;
    int width, height;
    int band;   // order of the ray slots: 0 pixel order; B > 1 bands of B rows, each walked column by column
    double oz, aspect, tan_half;
    double eye[3], f[3], r[3], u[3];
};

// Device buffers of one frame (npix = width * height entries each, except count).
struct FrameBuffers {
    int* flag;          // 1 where the ray collides inside the medium
    int* offset;        // exclusive prefix sum of flag
    float* pts;         // [npix][3] collision points (0 on a miss)
    float* dirs;        // [npix][3] ray directions
    float* cpts;        // [npix][3] compacted points, pixel order
    float* cdirs;       // [npix][3] compacted directions
    int* cpix;          // [npix] pixel of each compacted point
    int* count;         // [1] number of collisions
    void* scan_tmp;
    size_t scan_bytes;
};

hipError_t launch_pyramid(const float* rho, const Level* lev, int levels, hipStream_t s);
hipError_t launch_transpose(const MediumView& mv, hipStream_t s);
hipError_t launch_sweep(const MediumView& mv, hipStream_t s);
hipError_t launch_pairs(const MediumView& mv, hipStream_t s);
hipError_t launch_site_tables(const MediumView& mv, SiteTables* tab, hipStream_t s);
// 64-point Gauss-Legendre rule on [-1, 1] for the volume-phase tables
struct GaussLegendre64 {
    double x[64], w[64];
};
hipError_t launch_volume_tables(const MediumView& mv, const GaussLegendre64& gl, SiteTables* tab, float* vtab,
                                hipStream_t s);
hipError_t launch_features(int prec, const FeatArgs& a, hipStream_t s);
int64_t features_blocks(int64_t npts);   // workgroups launch_features uses for npts points
// big: some query's medium holds a level of path-density pairs of 4 GiB or more
hipError_t launch_features_multi(int prec, const FeatMulti& m, bool big, hipStream_t s);
bool big_fields(const MediumView& mv);
// L[i] = radiance (f0[i] + albedo_gamma expm1(y[i])) for n points (the backbone's decode)
hipError_t launch_decode(const float* y, const float* f0, int64_t n, float radiance, float albedo_gamma, float* out,
                         hipStream_t s);
hipError_t launch_template_features(int prec, const TplArgs& a, hipStream_t s);
// The paper's backbone modules: FP32 template feature rows [npts][kDescPad]
// -> descriptor rows in the precision's layout.
hipError_t launch_modules(int prec, const float* feat, const float* wm, int64_t npts, const int* count,
                          int64_t count_off, void* desc, float desc_inv_scale, float albedo, hipStream_t s);
int module_floats_total();   // floats of the module block of the weight blob
int module_packed_floats();  // floats of that block in the kernel's packed layout
void pack_modules(const float* raw, float* out);   // blob order -> packed layout
hipError_t launch_desc_to_f32(int prec, const void* src, float* dst, int64_t n, float scale, hipStream_t s);
hipError_t launch_mlp(int prec, const MlpArgs& a, hipStream_t s);
// eta: the albedo entry as stored (FP8: already divided by the descriptor's scale)
hipError_t launch_albedo_entry(int prec, void* desc, int64_t n, const int* count, int64_t count_off, float eta,
                               hipStream_t s);
int mlp_padded_width(int width);
hipError_t frame_scan_bytes(int64_t npix, size_t* bytes);
hipError_t launch_raygen(const CamArgs& C, const float* rho0, int n, double sigma_t, double majorant,
                         uint64_t seed, const FrameBuffers& fb, hipStream_t s);
hipError_t launch_image(const FrameBuffers& fb, int64_t npix, const float* L, float scale, float* image,
                        hipStream_t s);
// RGB image [npix][3] from RGB radiance [count][3], channel c scaled by scale[c].
hipError_t launch_image_rgb(const FrameBuffers& fb, int64_t npix, const float* L, const float scale[3],
                            float* image, hipStream_t s);
int mlp_hidden_k(int prec, int wpad);
int mlp_k_step(int prec);       // K per MFMA instruction
int mlp_k_per_lane(int prec);   // K elements a lane holds in one B fragment

// K of the backbone's hidden layers: the padded width rounded up to the MFMA
// K step (4 for FP32, 32 for BF16); the extra weight columns are zero.
__host__ __device__ constexpr int hidden_k(int prec, int wpad)
{
    return prec == kPrecFP32 ? wpad : prec == kPrecBF16 ? (wpad + 31) / 32 * 32 : (wpad + 63) / 64 * 64;
}

// K of the backbone's first layer: the descriptor padded to the MFMA K step.
__host__ __device__ constexpr int input_k(int prec)
{
    return prec == kPrecFP8 ? kDescF8 : kDescPad;
}

// Bytes of one stored descriptor row.
__host__ __device__ constexpr int desc_row_bytes(int prec)
{
    return prec == kPrecFP32 ? kDescPad * 4 : prec == kPrecBF16 ? kDescPad * 2 : kDescF8;
}

}  // namespace nis
