// k_features.hip -- template gather, 3D-CNN and squeeze-excitation for a tile
// of shading points, writing each point's 1057-entry descriptor.
//
// For every point p (view direction w) and template layer k = 0..11:
//  * gather (Sec. III.B.2-4, eq. 1, eq. 8): the 225 sites of the light-aligned
//    5x5x9 lattice at spacing 2^k voxels sample the density of level
//    m = min(k, L-1) (zero outside the unit cube) and its graded transmittance
//    exp(-lambda^(m+1) sigma_t D_m); per-layer means and maxima form the
//    squeeze vector of eq. (24) together with the phase statistics, g and
//    alpha = acos(w.l);
//  * 3D-CNN (Fig. 3): the 9x5x5 transmittance lattice goes through conv 3^3
//    1->8 + ReLU and conv 3^3 8->16 + ReLU (valid padding), computed as two
//    implicit-im2col GEMMs on MFMA with the lattice staged in LDS;
//  * squeeze-excitation (eq. 24-26): channel means -> FC 16->4 -> ReLU ->
//    FC 4->16 -> sigmoid gate on the 16x5 feature map.
// Layers 0-7 use the diffuse weight group and layers 8-11 the highlight group.
//
// Site geometry.  In level-m index units the 225 sites of layer k sit at
// integer offsets c*(i, j, -q), c = 2^(k-m), from the point's light-sheared
// coordinates, so the path-density lookups of a layer share one trilinear
// weight set and the density lookups share one set per slab q.  Whether a site
// lies inside the closed unit cube is decided on its double-precision position
// p + 2^k h_0 (q l/|l_a| + i e_b + j e_c), evaluated term by term without
// contraction, because that decision is discontinuous in the position.
//
// Work split.  A workgroup is one wave and holds kTP = 4 points; the 16 lanes
// of a point share its work, so no stage waits for another wave.  Per layer
// the path densities around the point (index-clamped) are first staged in LDS
// as a small brick from the per-light path-density pairs, as 48-byte runs
// with one lane per brick row; a lane then evaluates up to three rows of 5
// transmittance sites (one slab q, one lateral j, i = -2..2) from the brick
// with the shared weights.  The densities need no staging: lane q < 9 of a
// point loads its slab's 6 rows of light-axis density pairs (48-byte runs)
// into registers and evaluates the slab's 25 sites.  Each lane keeps its own
// running sums and maxima, reduced over the point's 16 lanes by shuffles.

// Lattice layout for conv1.  Each 5-site row of the transmittance lattice is
// stored as three 4-wide windows starting at i = 0, 1, 2 (the last padded with
// a zero), so the 3 taps of a kernel row -- plus a fourth tap with zero weight
// -- are one aligned 4-element read for every output position.  conv1's K
// index is tap-row * 4 + dx over 9 tap-rows (K = 36, padded to the MFMA step).
#include "launch_args.h"
#include "mfma.h"

namespace nis {

constexpr int kTP = 4;                    // points per workgroup (one wave)
constexpr int kXcds = 8;                  // accelerator complex dies of the MI355X
constexpr int kCbFloats = 8 + 16 + 64 + 4 + 64 + 16;   // b1 b2 s1 c1 s2 c2 (in memory)
constexpr int kCbLds = 8 + 16 + 4 + 16;                 // b1 b2 c1 c2 (in LDS)
constexpr int kRows = 45;                 // site rows per point and layer
constexpr int kLatRow = 12;               // three 4-wide windows of a 5-site row
constexpr int kLatStride = kRows * kLatRow + 4;
constexpr int kY1Pos = 64;                // 63 conv1 positions + 1
constexpr int kBufferFlags = 0x00020000;  // buffer resource word 3 for gfx9-family raw loads
constexpr int kBrickJ = 10, kBrickV = 6, kBrickU = 6;   // path-density brick of one point-layer

struct PointLayer {           // per point and layer (path-density lookups)
    int iu, iv, ij, pad;      // sheared base indices
    float w00, w10, w01, w11; // bilinear weights over (J, V): (J0,V0) (J0+1,V0) (J0,V0+1) (J0+1,V0+1)
    float wu, wv, wj, pad1;
};

struct SlabParams {           // per point, layer and slab q (density lookups)
    int16_t ia, cbase, bbase;     // a base of the slab, first c and b of its brick (clamped to
                                  // [-1, n], [-6, n], [-6, n]: the reads they give do not change)
    uint16_t mask;                // in-cube bits (0-4 i, 5-9 j, 10 slab)
    float wa, wc, wb;             // the weights along a, c, b
};

// Shared memory of one wave.  The lattice is dead once conv1 has read it, so
// the attention stage reuses its space.  The brick area holds the
// path-density bricks, then conv1's output, which in turn stages the
// descriptor rows once conv2 has read it.
template <class E> struct FeatShared {
    union {
        E lat[kTP][kLatStride];
        struct {
            float H[kTP][16][5];
        } se;
    } __attribute__((aligned(16))) u0;
    union {
        float brick[kTP][kBrickJ * kBrickV * kBrickU];
        E y1[kTP][kY1Pos][8];                  // conv1 output, channels fastest
    } __attribute__((aligned(16))) u1;
    float pstat[kTP][kStats];
    float pfix[kTP][3];
    double px[kTP][3];
    PointLayer pl[kTP];
    SlabParams sp[kTP][9];
    float cb[kCbLds];                          // the group's conv and attention biases
    uint16_t smask[kTP][kLayers][9];           // in-cube bits of every slab of every layer
    uint16_t posoff[kY1Pos];                   // conv1: lattice offset of output position p (the 64th = the 63rd)
    uint16_t goff[24];                         // conv1 (BF16): lattice offset of 4-slot K group g
    double qo[3][9];                           // the light's lattice offsets, per axis and slab
};

__device__ __forceinline__ double site_coord(double x, double scale, double qo, int i)
{
#pragma clang fp contract(off)
    return x + scale * (qo + (double)i);
}

__device__ __forceinline__ double site_coord_a(double x, double scale, double qo)
{
#pragma clang fp contract(off)
    return x + scale * qo;
}

// the medium's phase (its HG lobes summed with their weights, eq. 6) in FP64
__device__ __forceinline__ double hg64(const MediumView& mv, double mu)
{
    double v = 0.0;
    for (int i = 0; i < mv.nl; i++) {
        const double den = mv.hg_a[i] - mv.hg_b[i] * mu;
        v += mv.hg_k[i] / (den * sqrt(den));
    }
    return v;
}

__device__ __forceinline__ float lerpf(float a, float b, float w) { return __builtin_fmaf(w, b - a, a); }
// the same value from a and its step d = b - a (rounded as lerpf rounds it)
__device__ __forceinline__ float lerp_step(float a, float d, float w) { return __builtin_fmaf(w, d, a); }


__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

// The value unchanged, but opaque to the optimiser: per-lane index arithmetic
// derived from it inside the layer loop is recomputed each layer instead of
// being hoisted out of the loop and kept live (and spilled) across it.
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// light-sheared continuous coordinates of x at level m
__device__ __forceinline__ void sheared(const MediumView& mv, int nm, const double x[3], double& Uf,
                                        double& Vf, double& Jf)
{
    double g[3];
    for (int d = 0; d < 3; d++) g[d] = x[d] * nm - 0.5;
    Jf = mv.sigma > 0 ? (nm - 1) - g[mv.a] : g[mv.a];
    Uf = g[mv.b] + Jf * mv.sb;
    Vf = g[mv.c] + Jf * mv.sc;
}

// Index-clamped trilinear lookup in a path-density field, read from its
// pairs along V: pair V' = V + 1 (clamped into 0..n_V) holds D at the clamped
// rows V and V + 1, the two rows the lookup interpolates between.
__device__ __forceinline__ float sample_D(const float2* __restrict__ Q, const Level& lv, int U, int V,
                                          int J, float wu, float wv, float wj)
{
    const int u0 = clampi(U - lv.ulo, 0, lv.nu - 1), u1 = clampi(U + 1 - lv.ulo, 0, lv.nu - 1);
    const int vp = clampi(V + 1 - lv.vlo, 0, lv.nv);
    const int j0 = clampi(J, 0, lv.n - 1), j1 = clampi(J + 1, 0, lv.n - 1);
    const int64_t qplane = (int64_t)lv.nu * (lv.nv + 1);
    const float2* q0 = Q + j0 * qplane + (int64_t)vp * lv.nu;
    const float2* q1 = Q + j1 * qplane + (int64_t)vp * lv.nu;
    const float2 p00 = q0[u0], p10 = q0[u1], p01 = q1[u0], p11 = q1[u1];
    float a00 = lerpf(p00.x, p10.x, wu);
    float a01 = lerpf(p00.y, p10.y, wu);
    float a10 = lerpf(p01.x, p11.x, wu);
    float a11 = lerpf(p01.y, p11.y, wu);
    return lerpf(lerpf(a00, a01, wv), lerpf(a10, a11, wv), wj);
}

// As sample_D, with the pairs at U and U + 1 of each slice read as one
// 16-byte load (from U clamped to n_U - 2, the two members picked to match
// the index clamping).
__device__ __forceinline__ float sample_D2(const float2* __restrict__ Q, const Level& lv, int U, int V, int J,
                                           float wu, float wv, float wj)
{
    const int u0 = clampi(U - lv.ulo, 0, lv.nu - 1), u1 = clampi(U + 1 - lv.ulo, 0, lv.nu - 1);
    const int ub = min(u0, lv.nu - 2);
    const int vp = clampi(V + 1 - lv.vlo, 0, lv.nv);
    const int j0 = clampi(J, 0, lv.n - 1), j1 = clampi(J + 1, 0, lv.n - 1);
    const int64_t qplane = (int64_t)lv.nu * (lv.nv + 1);
    const float4 a = *reinterpret_cast<const float4*>(Q + j0 * qplane + (int64_t)vp * lv.nu + ub);
    const float4 b = *reinterpret_cast<const float4*>(Q + j1 * qplane + (int64_t)vp * lv.nu + ub);
    const float2 p00 = u0 == ub ? make_float2(a.x, a.y) : make_float2(a.z, a.w);
    const float2 p10 = u1 == ub ? make_float2(a.x, a.y) : make_float2(a.z, a.w);
    const float2 p01 = u0 == ub ? make_float2(b.x, b.y) : make_float2(b.z, b.w);
    const float2 p11 = u1 == ub ? make_float2(b.x, b.y) : make_float2(b.z, b.w);
    float a00 = lerpf(p00.x, p10.x, wu);
    float a01 = lerpf(p00.y, p10.y, wu);
    float a10 = lerpf(p01.x, p11.x, wu);
    float a11 = lerpf(p01.y, p11.y, wu);
    return lerpf(lerpf(a00, a01, wv), lerpf(a10, a11, wv), wj);
}

// One row of 5 sites from 4 rows of 6 samples: bilinear across the rows with
// the shared weights, then linear along the row.
__device__ __forceinline__ void row5(const float* r00, const float* r10, const float* r01, const float* r11,
                                     float w00, float w10, float w01, float w11, float wr, float out[5])
{
    float b[6];
#pragma unroll
    for (int u = 0; u < 6; u++) b[u] = w00 * r00[u] + w10 * r10[u] + w01 * r01[u] + w11 * r11[u];
#pragma unroll
    for (int i = 0; i < 5; i++) out[i] = lerpf(b[i], b[i + 1], wr);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    bf16x2 v = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, v);
}

// bfloat16 pair {lo, hi} rounded to nearest even, packed low half first: one
// v_cvt_pk_bf16_f32, written as a vector conversion so that the compiler sees
// it (and keeps the wait states an MFMA result needs before it is read)
__device__ __forceinline__ uint32_t cvt_pk_bf16(float lo, float hi)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2v));
}

// The three 4-wide windows of a lattice row of 5 values.
template <class E> __device__ __forceinline__ void store_windows(E* row, const float t[5]);

template <> __device__ __forceinline__ void store_windows<float>(float* row, const float t[5])
{
    *reinterpret_cast<float4*>(row + 0) = make_float4(t[0], t[1], t[2], t[3]);
    *reinterpret_cast<float4*>(row + 4) = make_float4(t[1], t[2], t[3], t[4]);
    *reinterpret_cast<float4*>(row + 8) = make_float4(t[2], t[3], t[4], 0.f);
}

template <> __device__ __forceinline__ void store_windows<__bf16>(__bf16* row, const float t[5])
{
    const uint32_t p01 = pack_bf16(t[0], t[1]), p12 = pack_bf16(t[1], t[2]), p23 = pack_bf16(t[2], t[3]);
    const uint32_t p34 = pack_bf16(t[3], t[4]), p40 = pack_bf16(t[4], 0.f);
    *reinterpret_cast<uint2*>(row + 0) = make_uint2(p01, p23);
    *reinterpret_cast<uint2*>(row + 4) = make_uint2(p12, p34);
    *reinterpret_cast<uint2*>(row + 8) = make_uint2(p23, p40);
}

// element offset in a point's lattice of tap-row tr = dz * 3 + dy
__device__ __forceinline__ int taprow_off(int tr) { return ((tr / 3) * 5 + tr % 3) * kLatRow; }

// E4M3 code of x (saturated at +-448), rounded to nearest even
__device__ __forceinline__ uint8_t fp8_code(float x)
{
    x = __builtin_amdgcn_fmed3f(x, -448.f, 448.f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
}

// F8: the descriptor is stored as E4M3 codes of the entries divided by the
// backbone's first input scale (the CNN itself runs in BF16).
//
// The body takes the workgroup's index within its query's grid, so that one
// launch can serve several queries (k_features_multi).
template <int PREC, bool DBG, bool F8, bool BIG>
__device__ __forceinline__ void features_body(const FeatArgs& A, int64_t block)
{
    typedef Mfma<PREC> M;
    typedef typename M::elem E;
    __shared__ FeatShared<E> sh;
    E(*lat)[kLatStride] = sh.u0.lat;
    E(*y1)[kY1Pos][8] = sh.u1.y1;
    float(*brick)[kBrickJ * kBrickV * kBrickU] = sh.u1.brick;
    SlabParams(*sp)[9] = sh.sp;
    float* cbl = sh.cb;
    uint16_t(*smask)[kLayers][9] = sh.smask;
    float(*H)[16][5] = sh.u0.se.H;
    float(*pstat)[kStats] = sh.pstat;
    float(*pfix)[3] = sh.pfix;
    double(*px)[3] = sh.px;
    PointLayer* pl = sh.pl;

    const MediumView& mv = A.mv;
    const int lane = threadIdx.x;
    const int lr = lane % 16, lg = lane / 16;   // point lg of the tile, lane lr of the point
    // Workgroups are dealt to the 8 XCDs in turn (workgroup i runs on XCD i mod
    // 8), each with its own L2; give every XCD one contiguous run of tiles so
    // that neighbouring points share an L2.  The grid is a multiple of 8.
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    const int64_t per_xcd = ((npts + kTP - 1) / kTP + kXcds - 1) / kXcds;   // of the live tiles
    const int64_t slot = block / kXcds;
    if (slot >= per_xcd) return;
    const int64_t tile0 = ((block % kXcds) * per_xcd + slot) * kTP;
    // (the point count may live in device memory: frames whose hit count the
    // device computed; workgroups past it leave at once)
    if (tile0 >= npts) return;

    // tables read by every lane: the lattice offsets (a dynamic index into
    // the kernel arguments would be a vector load from them at every use) and
    // conv1's position offsets
    if (lane < 27) sh.qo[lane / 9][lane % 9] = mv.qoff[lane / 9][lane % 9];
    {
        const int pc = lane < 63 ? lane : 62;
        sh.posoff[lane] = (uint16_t)(((pc / 9) * 5 + (pc / 3) % 3) * kLatRow + (pc % 3) * 4);
        // BF16 conv1 reads the 4-slot groups g of its K steps: g < 8 is
        // tap-row g of the pair's first point, 8 <= g < 16 tap-row g - 8 of
        // the second, g = 16 tap-row 8 of the first and g = 17 of the second;
        // groups g >= 18 meet zero weights and read any entry (offset 0)
        const int g = lane;
        if (g < 24)
            sh.goff[g] = (uint16_t)(g < 16 ? (g >= 8 ? kLatStride : 0) + taprow_off(g % 8)
                                    : g == 16 ? taprow_off(8) : g == 17 ? kLatStride + taprow_off(8) : 0);
    }
    __syncthreads();

    // ---- per point: position, phase features, transmittance to the light ----
    {
        const int pt = lg, sub = lr;
        const int64_t p = tile0 + pt;
        const bool live = p < npts;
        const int64_t pc = live ? p : npts - 1;
        double x[3], w[3];
        for (int d = 0; d < 3; d++) {
            x[d] = A.pts[3 * pc + d];
            w[d] = A.dirs[3 * pc + d];
        }
        const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int d = 0; d < 3; d++) w[d] /= wn;
        const double wl = w[0] * mv.l[0] + w[1] * mv.l[1] + w[2] * mv.l[2];
        // Phase features in FP32 through a denominator without cancellation:
        // for unit vectors 1 + g^2 - 2g w.d = (1-|g|)^2 + |g| |w - sign(g) d|^2,
        // every term non-negative, so a few roundings in relative terms;
        // den^(-3/2) as rsq^3, summed over the phase's lobes (eq. 6).  The
        // centre site's table entry is (l, 1).
        const float wf[3] = {(float)w[0], (float)w[1], (float)w[2]};
        // one lobe's term of the phase at w . d for a site table entry e
        auto lobe = [&](int i, const float4& e) __attribute__((always_inline)) {
            const float gs = mv.ph_s[i];
            const float dx = wf[0] - gs * e.x, dy = wf[1] - gs * e.y, dz = wf[2] - gs * e.z;
            const float den = mv.ph_c[i] + mv.ph_a[i] * (dx * dx + dy * dy + dz * dz);
            const float r = __builtin_amdgcn_rsqf(den);
            return mv.ph_k[i] * e.w * (r * r * r);
        };
        const bool one_lobe = mv.nl == 1;
        float phs = 0.f, phm = -INFINITY;
        auto accum_phase = [&](int t, float P) __attribute__((always_inline)) {
            // log(1 + P) with the hardware logarithm: P >= 0, so 1 + P rounds
            // to within 6e-8 and the absolute error stays near 1e-7
            const float ph = __logf(1.f + P);
            phs += ph;
            phm = fmaxf(phm, ph);
            if (DBG && live) A.dbg_phi[p * kSites + t] = ph;
        };
        if (mv.volume == 0) {
            for (int t = sub; t < kSites; t += 16) {
                const float4 e = A.tab->site[t];
                float P = lobe(0, e);
                if (!one_lobe) {
#pragma unroll
                    for (int i = 1; i < kMaxLobes; i++)
                        if (i < mv.nl) P += lobe(i, e);
                }
                accum_phase(t, P);
            }
        } else {
            for (int t = sub; t < kSites; t += 16) {
                const float4 e = A.tab->site[t];
                float P;
                if (t != kCentreSite) {
                    // volume phase (eq. 9): the site's table of cone means, linear
                    // in the angle between w and d (2 asin(|w - d|/2), or pi minus
                    // 2 asin(|w + d|/2) past a right angle: both exact near their
                    // end), times the incident-side cone mean
                    const float mu0 = wf[0] * e.x + wf[1] * e.y + wf[2] * e.z;
                    const float sg = mu0 >= 0.f ? 1.f : -1.f;
                    const float ex = wf[0] - sg * e.x, ey = wf[1] - sg * e.y, ez = wf[2] - sg * e.z;
                    const float h = 2.f * asinf(fminf(1.f, 0.5f * sqrtf(ex * ex + ey * ey + ez * ez)));
                    const float ang = mu0 >= 0.f ? h : (float)M_PI - h;
                    const float xf = ang * (float)((kVBins - 1) / M_PI);
                    const int i0 = min((int)xf, kVBins - 2);
                    const float fr = xf - (float)i0;
                    const float* row = A.vtab + t * kVBins;
                    const float v0 = row[i0], v1 = row[i0 + 1];
                    P = e.w * (v0 + fr * (v1 - v0));
                } else {
                    P = lobe(0, e);
                    for (int i = 1; i < mv.nl; i++) P += lobe(i, e);
                }
                accum_phase(t, P);
            }
        }
        for (int o = 1; o < 16; o <<= 1) {
            phs += __shfl_xor(phs, o);
            phm = fmaxf(phm, __shfl_xor(phm, o));
        }
        // in-cube bits of the sites of every slab of every layer (bits 0-4: i
        // along b, 5-9: j along c, 10: the slab along a), decided on the
        // double-precision site positions
        for (int e = sub; e < kLayers * 9; e += 16) {
            const int kk = e / 9, qi = e % 9;
            const double scale = ldexp(1.0 / mv.n0, kk);
            int mask = 0;
            const double sa = site_coord_a(x[mv.a], scale, sh.qo[mv.a][qi]);
            if (sa >= 0.0 && sa <= 1.0) mask |= 1 << 10;
            for (int i = -2; i <= 2; i++) {
                const double sb = site_coord(x[mv.b], scale, sh.qo[mv.b][qi], i);
                const double sc = site_coord(x[mv.c], scale, sh.qo[mv.c][qi], i);
                if (sb >= 0.0 && sb <= 1.0) mask |= 1 << (i + 2);
                if (sc >= 0.0 && sc <= 1.0) mask |= 1 << (i + 7);
            }
            smask[pt][kk][qi] = (uint16_t)mask;
        }
        if (sub == 0) {
            pfix[pt][0] = phs * (1.f / kSites);
            pfix[pt][1] = phm;
            pfix[pt][2] = (float)acos(fmin(1.0, fmax(-1.0, wl)));
            for (int d = 0; d < 3; d++) px[pt][d] = x[d];
        }
        if (sub == 1 && live) {
            const Level& l0 = mv.lev[0];
            double Uf, Vf, Jf;
            sheared(mv, l0.n, x, Uf, Vf, Jf);
            double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
            float D0 = sample_D(mv.dpairs + l0.q_off, l0, (int)fu, (int)fv, (int)fj, (float)(Uf - fu),
                                (float)(Vf - fv), (float)(Jf - fj));
            float T = expf(-mv.sigma_t * D0);
            A.f0[p] = (float)(hg64(mv, wl) * (double)T);
            if (DBG) A.dbg_tp[p] = T;
        }
    }

    E* desc = reinterpret_cast<E*>(A.desc);
    uint8_t* desc8 = reinterpret_cast<uint8_t*>(A.desc);


    // conv1 A fragments of the current weight group (reloaded when it changes)
    constexpr int KC1 = PREC == kPrecFP32 ? 18 : 3;
    typename M::frag aw[KC1];
    for (int k = 0; k < kLayers; k++) {
        const int m = k < mv.levels - 1 ? k : mv.levels - 1;
        const Level lv = mv.lev[m];
        const int nm = lv.n;
        const int c = 1 << (k - m);
        const float coef = A.coef[k];
        const int grp = k < kDiffuse ? 0 : 1;
        const int rsize = nm * nm * nm;
        const __amdgpu_buffer_rsrc_t rR =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(mv.rho + lv.rho_off), 0, rsize * 4, kBufferFlags);
        // the path-density pairs of the level: below 2^32 bytes but for the
        // finest level of a 512^3 medium under a light near a diagonal (BIG
        // launches, where such a level is read through 64-bit addresses);
        // sizes and offsets are unsigned
        const uint32_t qrow = (uint32_t)lv.nu * (lv.nv + 1);
        const bool qbig = BIG && (uint64_t)qrow * nm * 8 >= ((uint64_t)1 << 32);
        const float* qbase = reinterpret_cast<const float*>(mv.dpairs + lv.q_off);
        const __amdgpu_buffer_rsrc_t rQ =
            __builtin_amdgcn_make_buffer_rsrc(mv.dpairs + lv.q_off, 0, (int)(qrow * nm * 8), kBufferFlags);
        auto ldQ = [&](uint32_t o) {
            return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rQ, (int)(o * 4), 0, 0));
        };
        auto ldR = [&](int o) { return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rR, o * 4, 0, 0)); };
        __syncthreads();   // the previous layer's readers of the shared tables are done
        const int ln = opaque(lane), lrl = ln & 15;
        if (k == 0 || k == kDiffuse) {
            const E* w1 = reinterpret_cast<const E*>(A.w1t[grp]);
#pragma unroll
            for (int kc = 0; kc < KC1; kc++) aw[kc] = M::load(w1 + lr * kConv1K + kc * M::KS + lg * M::KPL);
            if (ln < kCbLds) cbl[ln] = A.cb[grp][ln < 24 ? ln : ln < 28 ? 88 + (ln - 24) : 156 + (ln - 28)];
        }

        // ---- set-up: sheared path-density bases (one lane per point) and the
        // density bases, in-cube bits and weights of each slab (one lane per slab)
        if (ln < kTP * 10) {
            // one path for both: three FP64 coordinates of the point, each an
            // offset of g = x n_m - 1/2, then their floors and fractions
            const bool slab = ln < kTP * 9;
            const int spt = slab ? ln / 9 : ln - kTP * 9, qi = slab ? ln % 9 : 0;
            const double x[3] = {px[spt][0], px[spt][1], px[spt][2]};
            const double ga = x[mv.a] * nm - 0.5, gb = x[mv.b] * nm - 0.5, gc = x[mv.c] * nm - 0.5;
            // slab q: (a, b, c) = (g_a, g_b + c o_b(q), g_c + c o_c(q)); point:
            // the sheared (J, U, V) with J = g_a (or n_m - 1 - g_a against the
            // axis) and U = g_b + J s_b, V = g_c + J s_c
            const double t0 = !slab && mv.sigma > 0 ? (nm - 1) - ga : ga;
            const double t1 = gb + (slab ? c * sh.qo[mv.b][qi] : t0 * mv.sb);
            const double t2 = gc + (slab ? c * sh.qo[mv.c][qi] : t0 * mv.sc);
            const double f0 = floor(t0), f1 = floor(t1), f2 = floor(t2);
            const int i0 = (int)f0, i1 = (int)f1, i2 = (int)f2;
            const float w0 = (float)(t0 - f0), w1 = (float)(t1 - f1), w2 = (float)(t2 - f2);
            if (slab) {
                SlabParams sp1;
                sp1.ia = (int16_t)clampi(i0 + (qi - 4) * mv.sigma, -1, nm);
                sp1.cbase = (int16_t)clampi(i2 - 2, -6, nm);
                sp1.bbase = (int16_t)clampi(i1 - 2, -6, nm);
                sp1.mask = smask[spt][k][qi];
                sp1.wa = w0;
                sp1.wc = w2;
                sp1.wb = w1;
                sp[spt][qi] = sp1;
            } else {
                PointLayer q;
                q.iu = i1;
                q.iv = i2;
                q.ij = i0;
                q.pad = 0;
                q.wu = w1;
                q.wv = w2;
                q.wj = w0;
                q.w00 = (1.f - w0) * (1.f - w2);
                q.w10 = w0 * (1.f - w2);
                q.w01 = (1.f - w0) * w2;
                q.w11 = w0 * w2;
                q.pad1 = 0.f;
                pl[spt] = q;
            }
        }
        __syncthreads();
        const int pt = ln >> 4;
        const PointLayer P = pl[pt];

        // ---- path-density bricks: for each point the rows J = ij-4..ij+5,
        // V = iv-2..iv+3 of 6 samples U = iu-2..iu+3 (index-clamped), shared by
        // the point's 45 site rows.  One lane per row (16 + 8 byte loads); the
        // loads of all its rows are issued before the first store.  The
        // single-voxel level (c > 1) is one 3 x 3 slice, copied whole.
        if (c == 1) {
            // two V rows at a time from the path-density pairs: a pair row is 6
            // pairs, 48 contiguous bytes
            constexpr int kDPairs = kTP * kBrickJ * (kBrickV / 2), kDIt = (kDPairs + 63) / 64;
            float dv[kDIt][12];
#pragma unroll
            for (int it = 0; it < kDIt; it++) {
                const int rr = ln + 64 * it;
                if (rr < kDPairs) {
                    const int bp = rr / (kBrickJ * 3), loc = rr % (kBrickJ * 3);
                    const PointLayer Q = pl[bp];
                    // J and V are clamped per row; only a row that crosses a U
                    // edge of the padded field (none does for a point inside
                    // the cube) is read sample by sample
                    const int J = clampi(Q.ij - 4 + loc / 3, 0, nm - 1);
                    const int Vp = clampi(Q.iv - 1 + 2 * (loc % 3) - lv.vlo, 0, lv.nv);
                    const int U0 = Q.iu - 2 - lv.ulo;
                    if (qbig) {
                        const float* q = qbase + ((int64_t)J * qrow + (int64_t)Vp * lv.nu) * 2;
#pragma unroll
                        for (int u = 0; u < 6; u++) {
                            const int64_t o = (int64_t)clampi(U0 + u, 0, lv.nu - 1) * 2;
                            dv[it][2 * u] = q[o];
                            dv[it][2 * u + 1] = q[o + 1];
                        }
                    } else if (U0 >= 0 && U0 + 5 < lv.nu) {
                        const uint32_t o = ((uint32_t)J * qrow + (uint32_t)Vp * lv.nu + U0) * 2;
#pragma unroll
                        for (int e = 0; e < 12; e++) dv[it][e] = ldQ(o + e);
                    } else {
                        const uint32_t ro = (uint32_t)J * qrow + (uint32_t)Vp * lv.nu;
#pragma unroll
                        for (int u = 0; u < 6; u++) {
                            const uint32_t o = (ro + clampi(U0 + u, 0, lv.nu - 1)) * 2;
                            dv[it][2 * u] = ldQ(o);
                            dv[it][2 * u + 1] = ldQ(o + 1);
                        }
                    }
                }
            }
#pragma unroll
            for (int it = 0; it < kDIt; it++) {
                const int rr = ln + 64 * it;
                if (rr < kDPairs) {
                    // the pair row holds brick rows bv = 2 (loc % 3) and bv + 1,
                    // which are adjacent in the brick
                    const int bp = rr / (kBrickJ * 3), loc = rr % (kBrickJ * 3);
                    float2* dst = reinterpret_cast<float2*>(&brick[bp][(loc / 3 * kBrickV + 2 * (loc % 3)) * kBrickU]);
#pragma unroll
                    for (int e = 0; e < 3; e++) {
                        dst[e] = make_float2(dv[it][4 * e], dv[it][4 * e + 2]);
                        dst[3 + e] = make_float2(dv[it][4 * e + 1], dv[it][4 * e + 3]);
                    }
                }
            }
        } else {
            // the 1^3 level's field is 1 slice of 3 x 3 rays; D(U, V) is the
            // second member of pair V' = V
            const int u = ln & 7, v = ln >> 3;
            if (u < lv.nu && v < lv.nv) brick[0][v * lv.nu + u] = ldQ(((uint32_t)v * lv.nu + u) * 2 + 1);
        }
        __syncthreads();

        // ---- transmittance lattice: up to three rows of 5 sites per lane --------
        // (one loop per case, so that the single-voxel level's set-up is not
        // paid on the other levels; exp(-coef D) as exp2 of one product)
        float ts = 0.f, tmx = -INFINITY;
        const float nl2c = -coef * 1.44269504088896341f;
        auto emit = [&](int r, const float* Dv) __attribute__((always_inline)) {
            float T[5];
#pragma unroll
            for (int i = 0; i < 5; i++) T[i] = __builtin_amdgcn_exp2f(nl2c * Dv[i]);
            store_windows<E>(lat[pt] + r * kLatRow, T);
            const int64_t p = tile0 + pt;
#pragma unroll
            for (int i = 0; i < 5; i++) {
                ts += T[i];
                tmx = fmaxf(tmx, T[i]);
                if (DBG && p < npts) A.dbg_tbar[(p * kLayers + k) * kSites + r * 5 + i] = T[i];
            }
        };
        if (c == 1) {
            for (int r = lrl; r < kRows; r += 16) {
                const int qi = r / 5, jj = r % 5, q = qi - 4;
                // rows (J0, V0), (J0, V0+1), (J0+1, V0), (J0+1, V0+1) of the brick,
                // J0 = ij - q -> bj = 4 - q, V0 = iv + j -> bv = j + 2
                const float* b0 = &brick[pt][((4 - q) * kBrickV + jj) * kBrickU];
                float d00[6], d01[6], d10[6], d11[6];
#pragma unroll
                for (int h = 0; h < 3; h++) {
                    const float2 e00 = reinterpret_cast<const float2*>(b0)[h];
                    const float2 e01 = reinterpret_cast<const float2*>(b0 + kBrickU)[h];
                    const float2 e10 = reinterpret_cast<const float2*>(b0 + kBrickV * kBrickU)[h];
                    const float2 e11 = reinterpret_cast<const float2*>(b0 + kBrickV * kBrickU + kBrickU)[h];
                    d00[2 * h] = e00.x, d00[2 * h + 1] = e00.y;
                    d01[2 * h] = e01.x, d01[2 * h + 1] = e01.y;
                    d10[2 * h] = e10.x, d10[2 * h + 1] = e10.y;
                    d11[2 * h] = e11.x, d11[2 * h + 1] = e11.y;
                }
                float Dv[5];
                row5(d00, d10, d01, d11, P.w00, P.w10, P.w01, P.w11, P.wu, Dv);
                emit(r, Dv);
            }
        } else {
            // c > 1 only on the single-voxel level (one slice, so no
            // interpolation along J): sites are c apart; the U samples of a
            // site are the same in every row
            const float* sl = &brick[0][0];   // the whole slice, staged above
            int u0[5], u1[5];
#pragma unroll
            for (int i = 0; i < 5; i++) {
                u0[i] = clampi(P.iu + c * (i - 2) - lv.ulo, 0, lv.nu - 1);
                u1[i] = clampi(P.iu + c * (i - 2) + 1 - lv.ulo, 0, lv.nu - 1);
            }
            for (int r = lrl; r < kRows; r += 16) {
                const int j = r % 5 - 2;
                const float* s0 = sl + clampi(P.iv + c * j - lv.vlo, 0, lv.nv - 1) * lv.nu;
                const float* s1 = sl + clampi(P.iv + c * j + 1 - lv.vlo, 0, lv.nv - 1) * lv.nu;
                float Dv[5];
#pragma unroll
                for (int i = 0; i < 5; i++) {
                    const float e0 = lerpf(s0[u0[i]], s0[u1[i]], P.wu);
                    const float e1 = lerpf(s1[u0[i]], s1[u1[i]], P.wu);
                    Dv[i] = lerpf(e0, e1, P.wv);
                }
                emit(r, Dv);
            }
        }
        // ---- densities and their statistics: lane q < 9 of each point's 16
        // takes slab q.  It loads the slab's brick rows c = cbase..+5 of 6
        // samples b = bbase..+5 straight into registers, an a-plane and its
        // step to the next side by side from the light-axis pairs (a row is 6
        // pairs, 48 contiguous bytes), interpolates along a with the slab's
        // shared weight, then
        // evaluates the slab's 5 site rows (c, then b) and accumulates their
        // statistics.  The single-voxel level reads its voxel once.
        float rs = 0.f, rmx = -INFINITY;
        // row jj of slab r / 5 = qi (r = 5 qi + jj): a site is inside the
        // cube when its slab, its lateral j (bit 5 + jj) and its i (bit i) are
        auto accum = [&](int r, int jj, int mask, const float* Rv) __attribute__((always_inline)) {
            const bool row_in = (mask >> 10) & (mask >> (jj + 5)) & 1;
            const int64_t p = tile0 + pt;
#pragma unroll
            for (int i = 0; i < 5; i++) {
                const float rv = row_in && ((mask >> i) & 1) ? Rv[i] : 0.f;
                rs += rv;
                rmx = fmaxf(rmx, rv);
                if (DBG && p < npts) A.dbg_rho[(p * kLayers + k) * kSites + r * 5 + i] = rv;
            }
        };
        if (nm == 1) {
            const float r0 = ldR(0);
            const float Rv[5] = {r0, r0, r0, r0, r0};
            for (int r = lrl; r < kRows; r += 16) accum(r, r % 5, sp[pt][r / 5].mask, Rv);
        } else if (lrl < 9) {
            const int qi = lrl;
            const SlabParams S = sp[pt][qi];
            const int nb = nm + 2 * kPairPad;   // stored row length of the pairs
            const __amdgpu_buffer_rsrc_t rP = __builtin_amdgcn_make_buffer_rsrc(
                mv.pairs + lv.p_off, 0, (nm + 1) * nm * nb * 8, kBufferFlags);
            auto ldP = [&](int o) { return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rP, o * 4, 0, 0)); };
            // a is clamped once, c per row; a row within the padded b range
            // (every row of an in-cube point) is one run, others are read
            // sample by sample
            const int Ap = clampi(S.ia + 1, 0, nm), B0 = S.bbase;
            const bool run = B0 >= -kPairPad && B0 + 5 < nm + kPairPad;
            float pr[kBrickV][12];
#pragma unroll
            for (int cc = 0; cc < kBrickV; cc++) {
                const int C = clampi(S.cbase + cc, 0, nm - 1);
                const int ro = (Ap * nm + C) * nb + kPairPad;
                if (run) {
#pragma unroll
                    for (int e = 0; e < 12; e++) pr[cc][e] = ldP((ro + B0) * 2 + e);
                } else {
#pragma unroll
                    for (int u = 0; u < 6; u++) {
                        const int o = (ro + clampi(B0 + u, 0, nm - 1)) * 2;
                        pr[cc][2 * u] = ldP(o);
                        pr[cc][2 * u + 1] = ldP(o + 1);
                    }
                }
            }
            float R[kBrickV][6];
#pragma unroll
            for (int cc = 0; cc < kBrickV; cc++)
#pragma unroll
                for (int u = 0; u < 6; u++) R[cc][u] = lerp_step(pr[cc][2 * u], pr[cc][2 * u + 1], S.wa);
            auto rows = [&](bool masked) __attribute__((always_inline)) {
#pragma unroll
                for (int jj = 0; jj < 5; jj++) {
                    float bb[6], Rv[5];
#pragma unroll
                    for (int u = 0; u < 6; u++) bb[u] = lerpf(R[jj][u], R[jj + 1][u], S.wc);
#pragma unroll
                    for (int i = 0; i < 5; i++) Rv[i] = lerpf(bb[i], bb[i + 1], S.wb);
                    if (masked) {
                        accum(qi * 5 + jj, jj, S.mask, Rv);
                    } else {
                        const int64_t p = tile0 + pt;
#pragma unroll
                        for (int i = 0; i < 5; i++) {
                            rs += Rv[i];
                            rmx = fmaxf(rmx, Rv[i]);
                            if (DBG && p < npts) A.dbg_rho[(p * kLayers + k) * kSites + (qi * 5 + jj) * 5 + i] = Rv[i];
                        }
                    }
                }
            };
            // when every site of every slab lane is inside the cube (interior
            // points on the finer layers), the wave skips the in-cube selects
            if (__ballot((S.mask & 0x7ff) != 0x7ff) == 0) rows(false);
            else rows(true);
        }

        // ---- per-point statistics (eq. 24) over the point's 16 lanes ------------
        for (int o = 1; o < 16; o <<= 1) {
            rs += __shfl_xor(rs, o);
            ts += __shfl_xor(ts, o);
            rmx = fmaxf(rmx, __shfl_xor(rmx, o));
            tmx = fmaxf(tmx, __shfl_xor(tmx, o));
        }
        if (lr == 0) {
            pstat[pt][0] = rs * (1.f / kSites);
            pstat[pt][2] = ts * (1.f / kSites);
            pstat[pt][3] = rmx;
            pstat[pt][5] = tmx;
        } else if (lr == 1) {
            pstat[pt][1] = pfix[pt][0];
            pstat[pt][4] = pfix[pt][1];
            pstat[pt][6] = mv.g;
            pstat[pt][7] = pfix[pt][2];
        }
        __syncthreads();

        // conv2's weight fragments (BF16: all 7 stay in registers for both of
        // its tiles) are requested now, so that their latency overlaps conv1
        constexpr int KC2 = kConv2K / M::KS;
        typename M::frag bw[M::KPL == 8 ? KC2 : 1];
        const E* w2 = reinterpret_cast<const E*>(A.w2t[grp]);
        if constexpr (M::KPL == 8) {
#pragma unroll
            for (int kc = 0; kc < KC2; kc++) bw[kc] = M::load(w2 + lr * kConv2K + kc * M::KS + lg * M::KPL);
        }

        // ---- conv1, two points per MFMA tile: out^T [16 x 16 positions] =
        // W1 (tp0's rows 0-7 and tp0 + 1's rows 8-15, each zero on the other's
        // K slots) . [im2col of tp0 and tp0 + 1 on their K slots], the bias as
        // the C operand of the first K step
        {
            f32x4 bias;
#pragma unroll
            for (int e = 0; e < 4; e++) bias[e] = cbl[(lg & 1) * 4 + e];
            // BF16: lane group lg reads the 4-slot groups g = kc*8 + 2lg + h of K
            // step kc: g < 8 is tap-row g of tp0, 8 <= g < 16 tap-row g - 8 of
            // tp0 + 1, g = 16 tap-row 8 of tp0 and g = 17 tap-row 8 of tp0 + 1,
            // so that both points group their products alike.  Groups g >= 18
            // meet zero weights: they read any lattice entry (all finite), which
            // keeps every read unconditional.
            int goff[KC1 < 3 ? KC1 : 3][2];
#pragma unroll
            for (int kc = 0; kc < (KC1 < 3 ? KC1 : 3); kc++)
#pragma unroll
                for (int h = 0; h < 2; h++) goff[kc][h] = sh.goff[kc * 8 + 2 * (ln >> 4) + h];
#pragma unroll 1
            for (int tp0 = 0; tp0 < kTP; tp0 += 2)
#pragma unroll
            for (int t4 = 0; t4 < 4; t4++) {
                const int pos = t4 * 16 + lrl;
                const E* base = lat[tp0] + sh.posoff[pos];
                f32x4 acc = bias;
                if constexpr (PREC == kPrecFP32) {
                    // K step kc is the 4-slot group kc: tap-row kc % 9 of point tp0 + kc / 9
#pragma unroll
                    for (int kc = 0; kc < KC1; kc++)
                        acc = M::mma(aw[kc], base[(kc >= 9 ? kLatStride : 0) + taprow_off(kc % 9) + lg], acc);
                    float v[4];
#pragma unroll
                    for (int e = 0; e < 4; e++) v[e] = fmaxf(acc[e], 0.f);
                    if (pos < 63)
                        *reinterpret_cast<float4*>(&y1[tp0 + (lg >> 1)][pos][(lg & 1) * 4]) =
                            make_float4(v[0], v[1], v[2], v[3]);
                } else {
                    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
                    for (int kc = 0; kc < KC1; kc++) {
                        const uint2 r0 = *reinterpret_cast<const uint2*>(base + goff[kc][0]);
                        const uint2 r1 = *reinterpret_cast<const uint2*>(base + goff[kc][1]);
                        const u32x4 bv = {r0.x, r0.y, r1.x, r1.y};
                        acc = M::mma(aw[kc], __builtin_bit_cast(bf16x8, bv), acc);
                    }
                    // ReLU after rounding, as a signed 16-bit max on the bfloat16
                    // patterns (rounding keeps the sign); position 63 is padding
                    typedef short i16x4 __attribute__((ext_vector_type(4)));
                    const uint2 pk = make_uint2(cvt_pk_bf16(acc[0], acc[1]), cvt_pk_bf16(acc[2], acc[3]));
                    const i16x4 rl = __builtin_elementwise_max(__builtin_bit_cast(i16x4, pk), i16x4{});
                    *reinterpret_cast<uint2*>(&y1[tp0 + (lg >> 1)][pos][(lg & 1) * 4]) = __builtin_bit_cast(uint2, rl);
                }
            }
        }
        __syncthreads();

        // the attention weights this lane needs (a row of 4 of s1, one of s2),
        // from memory: requested now so that conv2 covers their latency, and
        // kept out of LDS, which limits the waves per compute unit
        const float4 s1v = *reinterpret_cast<const float4*>(A.cb[grp] + 24 + (lr & 3) * 16 + (lr & ~3));
        const float4 s2v = *reinterpret_cast<const float4*>(A.cb[grp] + 92 + lr * 4);

        // ---- conv2: [rows = (point, z)] x [K = 27 taps x 8 channels] x [16 channels]
        {
            const float* b2 = cbl + 8;
#pragma unroll
            for (int tile = 0; tile < 2; tile++) {
                const int row = tile * 16 + lrl;
                const int rc = row < kTP * 5 ? row : kTP * 5 - 1;
                const int tp = rc / 5, z = rc % 5;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 8
                for (int kc = 0; kc < KC2; kc++) {
                    const int k0 = kc * M::KS + lg * M::KPL;     // K index = tap * 8 + channel
                    const int tap = k0 >> 3 < 27 ? k0 >> 3 : 0;
                    if constexpr (M::KPL == 8) {
                        acc = M::mma(M::load(&y1[tp][z * 9 + tap][0]), bw[kc], acc);
                    } else {
                        acc = M::mma(y1[tp][z * 9 + tap][k0 & 7], M::load(w2 + lr * kConv2K + k0), acc);
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const int row2 = tile * 16 + lg * 4 + e;
                    if (row2 < kTP * 5) H[row2 / 5][lr][row2 % 5] = fmaxf(acc[e] + b2[lr], 0.f);
                }
            }
        }
        __syncthreads();

        // ---- squeeze-excitation gate and the layer's descriptor entries ---------
        {
            const float *c1 = cbl + 24, *c2 = cbl + 28;
            const int o = lr, pbase = lane & ~15;
            float hv[5];
#pragma unroll
            for (int z = 0; z < 5; z++) hv[z] = H[pt][o][z];
            const float zo = (hv[0] + hv[1] + hv[2] + hv[3] + hv[4]) * 0.2f;   // squeeze of channel o
            // hidden unit h = o % 4 over the inputs 4 (o/4) .. +3, summed over the
            // point's four lanes with the same h: every lane then holds unit o % 4
            const int h = o & 3, i0 = o & ~3;
            const float s1r[4] = {s1v.x, s1v.y, s1v.z, s1v.w}, s2r[4] = {s2v.x, s2v.y, s2v.z, s2v.w};
            float part = 0.f;
#pragma unroll
            for (int d = 0; d < 4; d++) part += s1r[d] * __shfl(zo, pbase | (i0 + d));
            part += __shfl_xor(part, 4);
            part += __shfl_xor(part, 8);
            const float hid_h = fmaxf(part + c1[h], 0.f);
            float s = c2[o];
#pragma unroll
            for (int hh = 0; hh < 4; hh++) s += s2r[hh] * __shfl(hid_h, pbase | hh);
            // sigmoid with the hardware exponential and reciprocal (each about 1 ulp)
            const float gate = __builtin_amdgcn_rcpf(1.f + __expf(-s));
            // stage the 88 entries of the layer in the (now free) conv1 output
            if constexpr (F8) {
                uint8_t* stage = reinterpret_cast<uint8_t*>(&y1[pt][0][0]);
                const float inv = A.desc_inv_scale;
#pragma unroll
                for (int z = 0; z < 5; z++) stage[o * 5 + z] = fp8_code(gate * hv[z] * inv);
                if (o < kStats) stage[kFeat + o] = fp8_code(pstat[pt][o] * inv);
            } else {
                E* stage = &y1[pt][0][0];
#pragma unroll
                for (int z = 0; z < 5; z++) stage[o * 5 + z] = M::cvt(gate * hv[z]);
                if (o < kStats) stage[kFeat + o] = M::cvt(pstat[pt][o]);
            }
            if (DBG && o < kStats && tile0 + pt < npts)
                A.dbg_stats[((tile0 + pt) * kLayers + k) * kStats + o] = pstat[pt][o];
            __syncthreads();
            if constexpr (F8) {
                // 8-byte stores of the staged codes (88 per point)
                constexpr int kChunks = kPerLayer / 8;
                for (int e = lane; e < kTP * kChunks; e += 64) {
                    const int tq = e / kChunks, ch = e % kChunks;
                    const int64_t pp = tile0 + tq;
                    if (pp < npts)
                        *reinterpret_cast<uint2*>(desc8 + pp * kDescF8 + k * kPerLayer + ch * 8) =
                            *reinterpret_cast<const uint2*>(reinterpret_cast<const uint8_t*>(&y1[tq][0][0]) + ch * 8);
                }
            } else {
                // 16-byte stores of the staged rows (88 entries per point)
                constexpr int kVec = 16 / sizeof(E), kChunks = kPerLayer / kVec;
                for (int e = lane; e < kTP * kChunks; e += 64) {
                    const int tq = e / kChunks, ch = e % kChunks;
                    const int64_t pp = tile0 + tq;
                    if (pp < npts)
                        *reinterpret_cast<uint4*>(desc + pp * kDescPad + k * kPerLayer + ch * kVec) =
                            *reinterpret_cast<const uint4*>(&y1[tq][0][0] + ch * kVec);
                }
            }
        }
    }
    // albedo entry and zero padding
    if constexpr (F8) {
        constexpr int kTail = kDescF8 - kDesc + 1;
        for (int e = lane; e < kTP * kTail; e += 64) {
            const int tq = e / kTail, f = kDesc - 1 + e % kTail;
            const int64_t pp = tile0 + tq;
            if (pp < npts) desc8[pp * kDescF8 + f] = f == kDesc - 1 ? fp8_code(mv.albedo * A.desc_inv_scale) : 0;
        }
    } else {
        for (int e = lane; e < kTP * (kDescPad - kDesc + 1); e += 64) {
            const int tq = e / (kDescPad - kDesc + 1), f = kDesc - 1 + e % (kDescPad - kDesc + 1);
            const int64_t pp = tile0 + tq;
            if (pp < npts) desc[pp * kDescPad + f] = M::cvt(f == kDesc - 1 ? mv.albedo : 0.f);
        }
    }
}

template <int PREC, bool DBG, bool F8, bool BIG>
__global__ void __launch_bounds__(64, 3)
k_features(FeatArgs A)
{
    features_body<PREC, DBG, F8, BIG>(A, blockIdx.x);
}

// Several queries in one launch: query r's workgroups are first[r] ..
// first[r + 1] - 1 (each count a multiple of 8, so that a workgroup's XCD is
// the one its own grid would give it); its arguments are read from the table.
template <int PREC, bool F8, bool BIG>
__global__ void __launch_bounds__(64, 3)
k_features_multi(FeatMulti M)
{
    int r = 0;
    for (int i = 1; i < M.n; i++) r = (int)blockIdx.x >= M.first[i] ? i : r;
    features_body<PREC, false, F8, BIG>(M.table[r], (int64_t)blockIdx.x - M.first[r]);
}

// whether a level of mv holds path-density pairs of 4 GiB or more
bool big_fields(const MediumView& mv)
{
    for (int m = 0; m < mv.levels; m++) {
        const Level& lv = mv.lev[m];
        if ((uint64_t)lv.nu * (lv.nv + 1) * lv.n * 8 >= ((uint64_t)1 << 32)) return true;
    }
    return false;
}

// ---- the gather at the paper's own templates (Sec. III.B.2, eq. 2-4) -----
//
// Diffuse layer k < 8: point s = p + r_k u (u its unit template point, r_k its
// radius by eq. 4), level m_k matched to the layer's point spacing.
// Highlight layer h: point s = p + d_l o, o the unit cone point along l and
// d_l the distance from p towards the light to where that ray leaves the
// unit cube; the level is matched to the spacing D(C_h) d_l.  At each point:
// the density (zero outside the closed cube), the graded transmittance
// exp(-lambda^(m+1) sigma_t D_m) and the phase feature log1p(f(w.d) f(d.l))
// (f(w.l) where the point is p itself); per layer the squeeze vector of
// eq. (24).  The descriptor holds, per layer, its transmittances, densities
// and phase features in template order and its squeeze vector, then zeros up
// to the albedo entry (index 1056, as in the lattice descriptor).
//
// Work split: a workgroup of 4 waves, one point per wave, a lane per template
// point (266 points, five rounds of 64 lanes); values are staged in LDS for
// the per-layer statistics (a lane per layer) and the descriptor row.
constexpr int kTplWaves = 4;

__device__ __forceinline__ int tpl_layer_of(int t)
{
    int k = 0;
#pragma unroll
    for (int i = 1; i < kLayers; i++) k += t >= tpl_first(i) ? 1 : 0;
    return k;
}

// the level whose voxel matches a point spacing (unit-cube length) on an n^3
// grid: the number of m >= 0 with spacing * n >= sqrt(2) 2^m, below L
__device__ __forceinline__ int tpl_level(double spacing, int n, int L)
{
#pragma clang fp contract(off)
    const double x = spacing * n;
    int m = 0;
    while (m < L - 1 && x >= 1.4142135623730951 * ldexp(1.0, m)) m++;
    return m;
}

// distance from x towards the light to where that ray leaves the unit cube
// (0 when it misses the cube or the cube lies behind x)
__device__ __forceinline__ double tpl_light_extent(const double l[3], const double x[3])
{
#pragma clang fp contract(off)
    double t0 = -INFINITY, t1 = INFINITY;
    for (int d = 0; d < 3; d++) {
        if (l[d] == 0.0) {
            if (x[d] < 0.0 || x[d] > 1.0) return 0.0;
            continue;
        }
        const double a = (0.0 - x[d]) / l[d], b = (1.0 - x[d]) / l[d];
        const double lo = a < b ? a : b, hi = a < b ? b : a;
        if (lo > t0) t0 = lo;
        if (hi < t1) t1 = hi;
    }
    if (t1 < t0 || t1 <= 0.0) return 0.0;
    return t1;
}

__device__ __forceinline__ double tpl_coord(double x, double scale, double o)
{
#pragma clang fp contract(off)
    return x + scale * o;
}

// density of level lv at s: zero outside the closed unit cube, else
// index-clamped trilinear, from the light-axis density pairs: rows c and
// c + 1, each one 16-byte load of the pairs at b and b + 1 (each pair holds
// the density at a and its step to a + 1).  An in-cube site has
// -1 <= b <= n - 1, inside the stored row's padding of index-clamped copies.
__device__ __forceinline__ float tpl_rho(const MediumView& mv, const Level& lv, const double s[3])
{
    if (s[0] < 0.0 || s[0] > 1.0 || s[1] < 0.0 || s[1] > 1.0 || s[2] < 0.0 || s[2] > 1.0) return 0.f;
    const int nm = lv.n, nb = nm + 2 * kPairPad;
    const double ga = s[mv.a] * nm - 0.5, gb = s[mv.b] * nm - 0.5, gc = s[mv.c] * nm - 0.5;
    const double fa = floor(ga), fb = floor(gb), fc = floor(gc);
    const float wa = (float)(ga - fa), wb = (float)(gb - fb), wc = (float)(gc - fc);
    const int ia = (int)fa, ib = clampi((int)fb, -1, nm - 1), ic = (int)fc;
    const float2* P = mv.pairs + lv.p_off + (int64_t)clampi(ia + 1, 0, nm) * nm * nb + kPairPad + ib;
    const float4 q0 = *reinterpret_cast<const float4*>(P + (int64_t)clampi(ic, 0, nm - 1) * nb);
    const float4 q1 = *reinterpret_cast<const float4*>(P + (int64_t)clampi(ic + 1, 0, nm - 1) * nb);
    const float2 p00 = make_float2(q0.x, q0.y), p01 = make_float2(q0.z, q0.w);
    const float2 p10 = make_float2(q1.x, q1.y), p11 = make_float2(q1.z, q1.w);
    const float r00 = lerp_step(p00.x, p00.y, wa), r01 = lerp_step(p01.x, p01.y, wa);
    const float r10 = lerp_step(p10.x, p10.y, wa), r11 = lerp_step(p11.x, p11.y, wa);
    return lerpf(lerpf(r00, r01, wb), lerpf(r10, r11, wb), wc);
}

// Where each descriptor entry below kTplFeat comes from in a wave's staged
// values [tbar (266), rho (266), phi (266), squeeze vectors (12 x 8)].
struct TplDescMap {
    uint16_t src[kTplFeat];
};
constexpr TplDescMap make_tpl_desc_map()
{
    TplDescMap m{};
    int e = 0;
    for (int k = 0; k < kLayers; k++) {
        const int n = tpl_count(k), f = tpl_first(k);
        for (int ty = 0; ty < 3; ty++)
            for (int j = 0; j < n; j++) m.src[e++] = (uint16_t)(ty * kTplSites + f + j);
        for (int i = 0; i < kStats; i++) m.src[e++] = (uint16_t)(3 * kTplSites + k * kStats + i);
    }
    return m;
}
__constant__ TplDescMap kTplMap = make_tpl_desc_map();

// The same for the backbone modules' feature rows (0xffff: padding, zero).
struct TplModMap {
    uint16_t src[kModFeat];
};
constexpr TplModMap make_tpl_mod_map()
{
    TplModMap m{};
    for (int f = 0; f < kModFeat; f++) m.src[f] = 0xffff;
    for (int k = 0; k < kLayers; k++) {
        const int n = tpl_count(k), f = tpl_first(k);
        for (int ty = 0; ty < 3; ty++)
            for (int j = 0; j < n; j++) m.src[mf_block(ty, k) + j] = (uint16_t)(ty * kTplSites + f + j);
        for (int i = 0; i < kStats; i++) m.src[mf_stats(k) + i] = (uint16_t)(3 * kTplSites + k * kStats + i);
    }
    return m;
}
__constant__ TplModMap kTplModMap = make_tpl_mod_map();
constexpr int kTplStage = 3 * kTplSites + kLayers * kStats;

template <int PREC, bool DBG, bool F8>
__global__ void __launch_bounds__(64 * kTplWaves) __attribute__((amdgpu_waves_per_eu(8)))
k_template_features(TplArgs A)
{
    typedef Mfma<PREC> M;
    typedef typename M::elem E;
    // per wave: tbar, rho, phi of each template point, then the squeeze vectors
    __shared__ float stage[kTplWaves][kTplStage];
    float* vals = stage[threadIdx.x / 64];
    float* stv = vals + 3 * kTplSites;
    // per-level and per-layer parameters a site picks by a run-time index
    // (dynamic indices into the kernel arguments would go through private
    // memory): levels and their coefficients, diffuse radii and levels, and
    // each wave's highlight levels
    __shared__ Level slev[kMaxLevels];
    __shared__ float scoef[kMaxLevels];
    __shared__ double srad[kDiffuse];
    __shared__ int smd[kDiffuse];
    __shared__ int smh[kTplWaves][kLayers - kDiffuse];
    __shared__ uint8_t slayer[kTplSites];      // the layer of each template site
    const MediumView& mv = A.mv;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < kMaxLevels; i++) {
            slev[i] = mv.lev[i];
            scoef[i] = A.coef[i];
        }
#pragma unroll
        for (int i = 0; i < kDiffuse; i++) {
            srad[i] = A.radius[i];
            smd[i] = A.mdiff[i];
        }
    }
    for (int t = threadIdx.x; t < kTplSites; t += 64 * kTplWaves) slayer[t] = (uint8_t)tpl_layer_of(t);
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    const int64_t p = (int64_t)blockIdx.x * kTplWaves + wave;
    if ((int64_t)blockIdx.x * kTplWaves >= npts) return;
    const bool live = p < npts;
    const int64_t pc = live ? p : npts - 1;

    double x[3], w[3];
    for (int d = 0; d < 3; d++) {
        x[d] = A.pts[3 * pc + d];
        w[d] = A.dirs[3 * pc + d];
    }
    const double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (int d = 0; d < 3; d++) w[d] /= wn;
    const double wl = w[0] * mv.l[0] + w[1] * mv.l[1] + w[2] * mv.l[2];
    const float wf[3] = {(float)w[0], (float)w[1], (float)w[2]};
    const double dlen = tpl_light_extent(mv.l, x);
    if (lane == 0) {
#pragma unroll
        for (int h = 0; h < kLayers - kDiffuse; h++) smh[wave][h] = tpl_level(A.dh[h] * dlen, mv.n0, mv.levels);
    }
    __syncthreads();
    // one lobe's term of the phase at w . d for a site table entry (as in k_features)
    auto lobe = [&](int i, const float4& e) __attribute__((always_inline)) {
        const float gs = mv.ph_s[i];
        const float dx = wf[0] - gs * e.x, dy = wf[1] - gs * e.y, dz = wf[2] - gs * e.z;
        const float den = mv.ph_c[i] + mv.ph_a[i] * (dx * dx + dy * dy + dz * dz);
        const float r = __builtin_amdgcn_rsqf(den);
        return mv.ph_k[i] * e.w * (r * r * r);
    };
    const float4 centre = make_float4((float)mv.l[0], (float)mv.l[1], (float)mv.l[2], 1.f);

    for (int t = lane; t < kTplSites; t += 64) {
        const int k = slayer[t];
        const bool diffuse = k < kDiffuse;
        const double scale = diffuse ? srad[k] : dlen;
        const int m = diffuse ? smd[k] : smh[wave][k - kDiffuse];
        double s[3];
        for (int d = 0; d < 3; d++) s[d] = tpl_coord(x[d], scale, A.tab->off[t][d]);
        const Level lv = slev[m];
        const int nm = lv.n;
        const float r = tpl_rho(mv, lv, s);
        // path density at s (sheared lookup, index-clamped trilinear)
        double g[3];
        for (int d = 0; d < 3; d++) g[d] = s[d] * nm - 0.5;
        const double Jf = mv.sigma > 0 ? (nm - 1) - g[mv.a] : g[mv.a];
        const double Uf = g[mv.b] + Jf * mv.sb, Vf = g[mv.c] + Jf * mv.sc;
        const double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
        const float Dv = sample_D2(mv.dpairs + lv.q_off, lv, (int)fu, (int)fv, (int)fj, (float)(Uf - fu),
                                   (float)(Vf - fv), (float)(Jf - fj));
        const float T = __builtin_amdgcn_exp2f(-scoef[m] * 1.44269504088896341f * Dv);
        const bool at_p = s[0] == x[0] && s[1] == x[1] && s[2] == x[2];
        const float4 e = at_p ? centre : A.tab->site[t];
        float P = lobe(0, e);
        for (int i = 1; i < mv.nl; i++) P += lobe(i, e);
        const float ph = __logf(1.f + P);
        vals[t] = T;
        vals[kTplSites + t] = r;
        vals[2 * kTplSites + t] = ph;
        if (DBG && live) {
            A.dbg_tbar[p * kTplSites + t] = T;
            A.dbg_rho[p * kTplSites + t] = r;
            A.dbg_phi[p * kTplSites + t] = ph;
        }
    }
    __syncthreads();
    // squeeze vector of eq. (24) per layer: four lanes per layer, each over
    // every fourth point, then summed over the four
    {
        const int k = min(lane >> 2, kLayers - 1), sub = lane & 3, f = tpl_first(k), n = tpl_count(k);
        float ts = 0.f, rs = 0.f, ps = 0.f, tm = -INFINITY, rm = -INFINITY, pm = -INFINITY;
        for (int j = sub; j < n; j += 4) {
            const float T = vals[f + j], r = vals[kTplSites + f + j], ph = vals[2 * kTplSites + f + j];
            ts += T, rs += r, ps += ph;
            tm = fmaxf(tm, T), rm = fmaxf(rm, r), pm = fmaxf(pm, ph);
        }
#pragma unroll
        for (int o = 1; o < 4; o <<= 1) {
            ts += __shfl_xor(ts, o);
            rs += __shfl_xor(rs, o);
            ps += __shfl_xor(ps, o);
            tm = fmaxf(tm, __shfl_xor(tm, o));
            rm = fmaxf(rm, __shfl_xor(rm, o));
            pm = fmaxf(pm, __shfl_xor(pm, o));
        }
        if (lane < 4 * kLayers && sub == 0) {
            const float inv = 1.f / (float)n;
            const float v[kStats] = {rs * inv, ps * inv, ts * inv, rm, pm, tm, mv.g,
                                     (float)acos(fmin(1.0, fmax(-1.0, wl)))};
            for (int i = 0; i < kStats; i++) {
                stv[k * kStats + i] = v[i];
                if (DBG && live) A.dbg_stats[(p * kLayers + k) * kStats + i] = v[i];
            }
        }
    }
    if (lane == 4 * kLayers && live) {
        // single-scatter term f(w.l) T(p) (eq. 19, eq. 15)
        const Level& l0 = mv.lev[0];
        double g[3];
        for (int d = 0; d < 3; d++) g[d] = x[d] * l0.n - 0.5;
        const double Jf = mv.sigma > 0 ? (l0.n - 1) - g[mv.a] : g[mv.a];
        const double Uf = g[mv.b] + Jf * mv.sb, Vf = g[mv.c] + Jf * mv.sc;
        const double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
        const float D0 = sample_D(mv.dpairs + l0.q_off, l0, (int)fu, (int)fv, (int)fj, (float)(Uf - fu),
                                  (float)(Vf - fv), (float)(Jf - fj));
        A.f0[p] = (float)(hg64(mv, wl) * (double)expf(-mv.sigma_t * D0));
    }
    __syncthreads();
    if (!live) return;
    // the descriptor row: per layer tbar, rho, phi (template order), squeeze vector
    if (A.feat_only) {
        // the backbone modules' feature row (FP32)
        for (int e = lane; e < kModFeat; e += 64) {
            const int src = kTplModMap.src[e];
            reinterpret_cast<float*>(A.desc)[p * kDescPad + e] = src == 0xffff ? 0.f : vals[src];
        }
        return;
    }
    const int rowlen = F8 ? kDescF8 : kDescPad;
    for (int e = lane; e < rowlen; e += 64) {
        const float v = e < kTplFeat ? vals[kTplMap.src[e]] : e == kDesc - 1 ? mv.albedo : 0.f;
        if constexpr (F8) {
            reinterpret_cast<uint8_t*>(A.desc)[p * kDescF8 + e] = e < kTplFeat || e == kDesc - 1 ? fp8_code(v * A.desc_inv_scale) : 0;
        } else {
            reinterpret_cast<E*>(A.desc)[p * kDescPad + e] = M::cvt(v);
        }
    }
}

hipError_t launch_template_features(int prec, const TplArgs& a, hipStream_t s)
{
    if (a.npts <= 0) return hipSuccess;
    const int64_t blocks = (a.npts + kTplWaves - 1) / kTplWaves;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const bool dbg = a.dbg_tbar || a.dbg_rho || a.dbg_phi || a.dbg_stats;
    if (dbg && !(a.dbg_tbar && a.dbg_rho && a.dbg_phi && a.dbg_stats)) return hipErrorInvalidValue;
    const dim3 g((int)blocks), b(64 * kTplWaves);
    if (prec == kPrecFP8) {
        if (dbg) hipLaunchKernelGGL((k_template_features<kPrecBF16, true, true>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_template_features<kPrecBF16, false, true>), g, b, 0, s, a);
    } else if (prec == kPrecBF16) {
        if (dbg) hipLaunchKernelGGL((k_template_features<kPrecBF16, true, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_template_features<kPrecBF16, false, false>), g, b, 0, s, a);
    } else {
        if (dbg) hipLaunchKernelGGL((k_template_features<kPrecFP32, true, false>), g, b, 0, s, a);
        else hipLaunchKernelGGL((k_template_features<kPrecFP32, false, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

// Rewrites the albedo entry of n descriptor rows: the channels of a coloured
// albedo share every other entry.  eta is the entry's value as stored (for
// the FP8 descriptor, already divided by its scale).
// Rows beyond a device count (count[0] - count_off, when count is given) are
// left alone, as the backbone does not read them.
template <int PREC>
__global__ void k_albedo_entry(void* desc, int64_t n, const int* count, int64_t count_off, float eta)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nv = count ? (int64_t)*count - count_off : n;
    if (!(i < n && i < nv)) return;
    if constexpr (PREC == kPrecFP8) {
        reinterpret_cast<uint8_t*>(desc)[i * kDescF8 + kDesc - 1] = fp8_code(eta);
    } else {
        typedef typename Mfma<PREC>::elem E;
        reinterpret_cast<E*>(desc)[i * kDescPad + kDesc - 1] = Mfma<PREC>::cvt(eta);
    }
}

hipError_t launch_albedo_entry(int prec, void* desc, int64_t n, const int* count, int64_t count_off, float eta,
                               hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    if (prec == kPrecFP8)
        hipLaunchKernelGGL(k_albedo_entry<kPrecFP8>, dim3((int)blocks), dim3(256), 0, s, desc, n, count, count_off,
                           eta);
    else if (prec == kPrecBF16)
        hipLaunchKernelGGL(k_albedo_entry<kPrecBF16>, dim3((int)blocks), dim3(256), 0, s, desc, n, count, count_off,
                           eta);
    else
        hipLaunchKernelGGL(k_albedo_entry<kPrecFP32>, dim3((int)blocks), dim3(256), 0, s, desc, n, count, count_off,
                           eta);
    return hipGetLastError();
}

// Widen a descriptor of the given precision to float32 [n][1057] (FP8: the
// codes times the descriptor's scale).
template <int PREC>
__global__ void k_desc_to_f32(const void* src, float* dst, int64_t n, float scale)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kDesc) return;
    int64_t row = i / kDesc, col = i % kDesc;
    if constexpr (PREC == kPrecFP8) {
        const int c = reinterpret_cast<const uint8_t*>(src)[row * kDescF8 + col];
        dst[i] = __builtin_amdgcn_cvt_f32_fp8(c, 0) * scale;
    } else {
        typedef typename Mfma<PREC>::elem E;
        dst[i] = (float)reinterpret_cast<const E*>(src)[row * kDescPad + col];
    }
}

hipError_t launch_desc_to_f32(int prec, const void* src, float* dst, int64_t n, float scale, hipStream_t s)
{
    int blocks = (int)((n * kDesc + 255) / 256);
    if (prec == kPrecFP8)
        hipLaunchKernelGGL(k_desc_to_f32<kPrecFP8>, dim3(blocks), dim3(256), 0, s, src, dst, n, scale);
    else if (prec == kPrecBF16)
        hipLaunchKernelGGL(k_desc_to_f32<kPrecBF16>, dim3(blocks), dim3(256), 0, s, src, dst, n, scale);
    else
        hipLaunchKernelGGL(k_desc_to_f32<kPrecFP32>, dim3(blocks), dim3(256), 0, s, src, dst, n, scale);
    return hipGetLastError();
}

int64_t features_blocks(int64_t npts) { return ((npts + kTP - 1) / kTP + kXcds - 1) / kXcds * kXcds; }

hipError_t launch_features_multi(int prec, const FeatMulti& m, bool big, hipStream_t s)
{
    if (m.n <= 0 || m.n > kMaxBatch) return hipErrorInvalidValue;
    const int blocks = m.first[m.n];
    if (blocks <= 0) return hipSuccess;
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), 0, s, m); };
    if (prec == kPrecFP8) big ? go(k_features_multi<kPrecBF16, true, true>) : go(k_features_multi<kPrecBF16, true, false>);
    else if (prec == kPrecBF16) big ? go(k_features_multi<kPrecBF16, false, true>) : go(k_features_multi<kPrecBF16, false, false>);
    else big ? go(k_features_multi<kPrecFP32, false, true>) : go(k_features_multi<kPrecFP32, false, false>);
    return hipGetLastError();
}

hipError_t launch_features(int prec, const FeatArgs& a, hipStream_t s)
{
    if (a.npts <= 0) return hipSuccess;
    const int64_t blocks = ((a.npts + kTP - 1) / kTP + kXcds - 1) / kXcds * kXcds;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const bool dbg = a.dbg_tbar || a.dbg_rho || a.dbg_phi || a.dbg_stats || a.dbg_tp;
    if (dbg && !(a.dbg_tbar && a.dbg_rho && a.dbg_phi && a.dbg_stats && a.dbg_tp))
        return hipErrorInvalidValue;   // the debug variant writes every stage output
    // the FP8 path runs the CNN in BF16 and stores the descriptor as E4M3 codes
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, dim3((int)blocks), dim3(64), 0, s, a); };
    const bool big = big_fields(a.mv);
    if (prec == kPrecFP8) {
        if (dbg) big ? go(k_features<kPrecBF16, true, true, true>) : go(k_features<kPrecBF16, true, true, false>);
        else big ? go(k_features<kPrecBF16, false, true, true>) : go(k_features<kPrecBF16, false, true, false>);
    } else if (prec == kPrecBF16) {
        if (dbg) big ? go(k_features<kPrecBF16, true, false, true>) : go(k_features<kPrecBF16, true, false, false>);
        else big ? go(k_features<kPrecBF16, false, false, true>) : go(k_features<kPrecBF16, false, false, false>);
    } else {
        if (dbg) big ? go(k_features<kPrecFP32, true, false, true>) : go(k_features<kPrecFP32, true, false, false>);
        else big ? go(k_features<kPrecFP32, false, false, true>) : go(k_features<kPrecFP32, false, false, false>);
    }
    return hipGetLastError();
}

}  // namespace nis
