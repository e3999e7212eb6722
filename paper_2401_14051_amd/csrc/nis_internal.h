// nis_internal.h -- device-side data layout shared by the library's kernels
// and its host runtime.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nis {

constexpr int kLayers = 12;       // template layers: 0-7 diffuse, 8-11 highlight
constexpr int kDiffuse = 8;
constexpr int kSites = 225;       // 9 (along the light) x 5 x 5
constexpr int kStats = 8;         // squeeze vector, eq. (24)
constexpr int kFeat = 80;         // 16 channels x 5 positions after the CNN
constexpr int kPerLayer = kFeat + kStats;
constexpr int kDesc = kLayers * kPerLayer + 1;   // 1057
constexpr int kDescPad = 1088;    // row stride of the descriptor in elements, FP32 and BF16 (multiple of 64)
constexpr int kDescF8 = 1152;     // row stride of the FP8 descriptor in bytes (E4M3 codes; 18 K steps of 64)
constexpr int kMaxLevels = 11;    // 1024^3 .. 1^3
constexpr int kMaxWidth = 256;    // backbone width limit
constexpr int kConv1K = 96;       // two points x 9 tap-rows x 4 (3 taps + a zero), padded to the MFMA step
constexpr int kConv2K = 224;      // 8 channels x 27 taps padded
constexpr int kPrecFP32 = 0, kPrecBF16 = 1, kPrecFP8 = 2;

// Padding of the gather's layouts, so that the bricks of every point inside
// the unit cube lie within the stored rows and load as whole runs: the
// path-density fields hold kRayPad extra rays (all zero: they miss the cube)
// on each side along U, and the light-axis density pairs kPairPad extra
// entries (index-clamped copies) on each side along b, where the outermost
// slab of an in-cube point's lattice reaches 4 voxels out and its brick 2 more.
constexpr int kRayPad = 2;
constexpr int kPairPad = 8;

// Phase function of a medium: n HG lobes with weights w summing to one and
// asymmetries g (Sec. III.A, eq. 6); one lobe of weight 1 is plain HG (eq. 5).
constexpr int kMaxLobes = 4;
// Volume phase (eq. 9): bins of the per-site tables over the angle between w and d
constexpr int kVBins = 2048;
constexpr int kCentreSite = 112;   // q = j = i = 0
struct Phase {
    int n;
    float w[kMaxLobes], g[kMaxLobes];
};

// Geometry of one pyramid level and its light-sheared path-density field.
struct Level {
    int n;              // edge n_m
    int ulo, vlo;       // first ray indices along the lateral axes b, c (ulo includes kRayPad)
    int nu, nv;         // ray counts (nu includes 2 kRayPad)
    int64_t rho_off;    // offset of the level in the density pyramid
    int64_t p_off;      // offset (in pairs) of the level's light-axis density pairs
    int64_t q_off;      // offset (in pairs) of the level's path-density pairs
    float ds;           // slice step along the ray, h_m / |l_a|
};

// Everything a kernel needs to know about a medium under a light.
struct MediumView {
    const float* rho;   // density pyramid, each level [z][y][x]
    const float* rho_s; // the pyramid in the layout the sweep and the light-axis pairs read
    int se[3];          // its stride along axis d (0 = x, 1 = y, 2 = z) is n_m^se[d]
    float2* pairs;      // per level [A' = 0..n][c][b + kPairPad < n + 2 kPairPad]: (rho(a = A'-1), rho(a = A') - rho(a = A'-1)), index-clamped
    float2* dpairs;     // per level [J][V' = 0..nv][U]: (D(V'-1), D(V')), index-clamped
    Level lev[kMaxLevels];
    int levels;
    int n0;             // finest edge
    int a, b, c;        // dominant axis and lateral axes (0 = x, 1 = y, 2 = z)
    int sigma;          // sign of l_a
    int st[3];          // unused by kernels that take strides per level
    double sb, sc;      // lateral shears l_b/|l_a|, l_c/|l_a|
    double l[3];        // unit light direction (towards the light)
    double la;          // |l_a|
    double qoff[3][9];  // (q * l_d) / |l_a| for q = -4..4, the lattice's along-light offsets
    float sigma_t, albedo, g, radiance;   // g: the phase's mean cosine, sum of w_i g_i
    float lam;          // graded-field coefficient base (eq. 1)
    float gamma;        // decode exponent (eq. 21)
    int volume;                // phase features from volume phases (eq. 9) rather than point phases
    int nl;                    // phase lobes; per lobe i:
    double hg_a[kMaxLobes], hg_b[kMaxLobes], hg_k[kMaxLobes];   // 1+g^2, 2g, w (1-g^2)/(4 pi)
    float ph_a[kMaxLobes], ph_s[kMaxLobes], ph_c[kMaxLobes], ph_k[kMaxLobes];   // |g|, sign g, (1-|g|)^2, float(hg_k)
};

// The paper's own templates (Sec. III.B.2): 8 diffuse sphere layers and 4
// highlight cone layers, kTplSites points in all.
constexpr int kTplSites = 266;
constexpr int kTplFeat = 3 * kTplSites + kLayers * kStats;   // descriptor entries before the zero gap (894)
__host__ __device__ constexpr int tpl_count(int k)
{
    return k == 0 ? 6 : k == 1 ? 8 : k == 2 ? 12 : k == 3 ? 16 : k == 4 ? 24 : k == 5 ? 32 : k < 8 ? 48
         : k == 8 ? 32 : k < 11 ? 16 : 8;
}
__host__ __device__ constexpr int tpl_first(int k)
{
    int f = 0;
    for (int i = 0; i < k; i++) f += tpl_count(i);
    return f;
}

// The decode of eq. (21) and the radiance of eq. (19): L = I (f(w.l) T + F),
// F = eta^gamma expm1(y); one definition for every kernel that decodes.
__device__ __forceinline__ float decode_radiance(float radiance, float f0, float albedo_gamma, float y)
{
    return radiance * __builtin_fmaf(albedo_gamma, expm1f(y), f0);
}

// The feature rows the paper's backbone modules read, written by the
// template gather: per feature type (graded transmittance, density, phase)
// the layers' values, each layer's block padded to a multiple of 4 floats
// (16-byte loads), then the 12 squeeze vectors.  A module of one type reads
// one contiguous third of the row.
__host__ __device__ constexpr int mf_pad4(int n) { return (n + 3) / 4 * 4; }
__host__ __device__ constexpr int mf_type_len()
{
    int s = 0;
    for (int k = 0; k < kLayers; k++) s += mf_pad4(tpl_count(k));
    return s;
}
__host__ __device__ constexpr int mf_block(int tau, int k)
{
    int s = tau * mf_type_len();
    for (int i = 0; i < k; i++) s += mf_pad4(tpl_count(i));
    return s;
}
__host__ __device__ constexpr int mf_stats(int k) { return 3 * mf_type_len() + kStats * k; }
constexpr int kModFeat = 3 * mf_type_len() + kLayers * kStats;   // 900 floats

// Per-light template tables: each point's offset (diffuse layers: the unit
// template point, scaled per layer by its radius; highlight layers: the unit
// cone point in world axes, scaled per query point by its light extent) and
// its (direction from the centre, f(direction . l)) for the phase feature.
struct TplTables {
    double off[kTplSites][3];
    float4 site[kTplSites];
};

// Per-light constant tables for the gather (one copy per medium).
struct SiteTables {
    // (d_t, f(d_t . l)) per site: the unit lattice offset direction and the
    // incident-side value of the medium's phase f; the centre site holds (l, 1)
    float4 site[kSites];
};

}  // namespace nis
