// k_volume.hip -- density pyramid and light-direction path-density sweep.
//
// Pyramid (Sec. III.B.1): each coarser level is the 2x2x2 box mean of the
// level below, down to 1^3.
//
// Sweep (eq. 1 with the extinction of eq. 15): for every level m and every
// light-sheared ray (U,V) the kernel walks the n_m slices J from the
// light-facing face and computes the path density
//     D_m(U,V,J) = ds_m * ( sum_{J'<J} r(J') + r(J)/2 ),
// where r(J) is the bilinear density on slice J at lateral index coordinates
// (U - J sb, V - J sc), or 0 outside [-1/2, n_m - 1/2].  The graded
// transmittance exp(-lambda^(m+1) sigma_t D) is applied at lookup time, so
// the field does not depend on sigma_t.  Running sums are compensated
// (Neumaier) float32 within a segment of slices and double across segments.
// D is stored only in the layout the gather reads, the pairs
// (D(V'-1), D(V')) along V, V' = 0..n_V with both rows clamped into the ray
// range: the pairs hold every value of D.  Lanes run along U: for a light dominated by y or z the lateral
// axis b is x, so neighbouring lanes read neighbouring voxels and write
// neighbouring entries.
#include "launch_args.h"

namespace nis {

// One thread per two neighbouring coarse voxels along x (nc >= 2; the 1^3
// level takes one thread): four 16-byte rows of the fine level in, one
// 8-byte pair out.  Edges are powers of two, so the index splits by shifts.
__global__ void __launch_bounds__(256)
k_mip(const float* __restrict__ fine, float* __restrict__ coarse, int nc, int lg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nf = 2 * nc;
    if (nc == 1) {
        if (i > 0) return;
        const float* f = fine;
        coarse[0] = (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) * 0.125f;
        return;
    }
    if (i >= (nc * nc * nc) >> 1) return;
    const int x = (i & ((nc >> 1) - 1)) * 2, y = (i >> (lg - 1)) & (nc - 1), z = i >> (2 * lg - 1);
    const float* f = fine + ((2 * z) * nf + 2 * y) * nf + 2 * x;
    const float4 a = *reinterpret_cast<const float4*>(f);
    const float4 b = *reinterpret_cast<const float4*>(f + nf);
    const float4 c = *reinterpret_cast<const float4*>(f + nf * nf);
    const float4 d = *reinterpret_cast<const float4*>(f + nf * nf + nf);
    const float s0 = ((a.x + a.y) + (b.x + b.y)) + ((c.x + c.y) + (d.x + d.y));
    const float s1 = ((a.z + a.w) + (b.z + b.w)) + ((c.z + c.w) + (d.z + d.w));
    *reinterpret_cast<float2*>(coarse + (z * nc + y) * nc + x) = make_float2(s0 * 0.125f, s1 * 0.125f);
}

// Copy of a level with y fastest, [x][z][y], for lights dominated by x: their
// lateral axes are y and z, and the sweep's and the light-axis pairs' lanes
// run along b = y.  32 x 32 tiles of one z-plane through LDS, so that both
// the reads (along x) and the writes (along y) are whole rows.
__global__ void __launch_bounds__(256)
k_transpose_x(const float* __restrict__ in, float* __restrict__ out, int n)
{
    __shared__ float t[32][33];
    const int x0 = blockIdx.x * 32, y0 = blockIdx.y * 32, z = blockIdx.z;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int x = x0 + tx, y = y0 + j;
        if (x < n && y < n) t[j][tx] = in[((int64_t)z * n + y) * n + x];
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int x = x0 + j, y = y0 + tx;
        if (x < n && y < n) out[((int64_t)x * n + z) * n + y] = t[tx][j];
    }
}

// Work split of the sweep.  A workgroup owns a tile of 64 rays along U (one
// per lane) by kSwRays rays along V, and its kSwWaves waves cut the slices
// into consecutive segments of up to kSwSeg slices each (a chunk of kSwWaves
// segments; finer levels take several chunks in turn).  Every wave keeps its
// segment's samples in registers, sums them, and after one barrier starts its
// running sums from the earlier segments' totals.  Each lane also samples the
// ray just below its tile (V0 - 1), so that it can write the path-density
// pairs (D(V'-1), D(V')) of its own rays whole; and since ray V+1 at slice J
// samples the density rows one above those of ray V, the rays of a lane share
// their row loads.  The pairs leave as non-temporal stores: they are read
// back only by the gather, and cached dirty lines of them would otherwise be
// written back during the passes that follow.
constexpr int kSwRays = 4;
constexpr int kSwSeg = 4;
constexpr int kSwWaves = 8;

struct SweepArgs {
    int blk_off[kMaxLevels + 1];   // prefix sums of workgroups per level
};

__device__ __forceinline__ void neumaier(float& sum, float& comp, float r)
{
    const float t = sum + r;
    comp += fabsf(sum) >= fabsf(r) ? (sum - t) + r : (r - t) + sum;
    sum = t;
}

constexpr int kBufFlags = 0x00020000;   // buffer resource word 3 for gfx9-family raw accesses
constexpr int kStream = 2;               // cache policy of a buffer access: non-temporal
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(64 * kSwWaves)
k_sweep(MediumView mv, SweepArgs sa)
{
    constexpr int R = kSwRays, K = kSwRays + 1;   // rays written, rays sampled
    __shared__ double tot[kSwWaves][K][64];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int bid = blockIdx.x;
    int m = 0;
    while (m + 1 < mv.levels && bid >= sa.blk_off[m + 1]) m++;
    const Level lv = mv.lev[m];
    const int local = bid - sa.blk_off[m];
    const int tiles_u = (lv.nu + 63) >> 6;
    const int iu = (local % tiles_u) * 64 + lane;
    const int V0 = (local / tiles_u) * R;          // first ray written (local index)
    const int n = lv.n, nu = lv.nu, nv = lv.nv;
    const int seg = n >= kSwWaves * kSwSeg ? kSwSeg : (n >= kSwWaves ? n / kSwWaves : 1);
    const int chunk = kSwWaves * seg;
    auto stride = [&](int axis) { return mv.se[axis] == 0 ? 1 : mv.se[axis] == 1 ? n : n * n; };
    const int sta = stride(mv.a) * 4, stb = stride(mv.b) * 4, stc = stride(mv.c) * 4;   // bytes
    const double hi = n - 0.5;
    const double dU = (double)(lv.ulo + iu), dV = (double)(lv.vlo + V0 - 1);   // sampled ray k is V = dV + k
    const bool lane_out = iu < nu;
    // byte sizes and offsets within a level's density and within one slice
    // of its path-density pairs stay below 2^32 (the light's layout refuses
    // larger ones); a level's pairs may pass 4 GiB (512^3 under a light near
    // a diagonal), so each slice's stores use a resource based at the slice
    const uint32_t qplane = (uint32_t)nu * (nv + 1) * 8;
    const __amdgpu_buffer_rsrc_t rR = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(mv.rho_s + lv.rho_off), 0, (int)((uint32_t)n * n * n * 4), kBufFlags);
    auto slice_rsrc = [&](int J) {
        return __builtin_amdgcn_make_buffer_rsrc(mv.dpairs + lv.q_off + (int64_t)J * nu * (nv + 1), 0, (int)qplane,
                                                 kBufFlags);
    };
    auto ld = [&](int off) { return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rR, off, 0, 0)); };
    // When the lateral axis b is x, the two samples u0, u0+1 of a density row
    // are adjacent floats: one 8-byte load from clamp(u0, 0, n-2) then holds
    // both clamped samples, and u0 alone picks which member each one is.
    const bool wide = stb == 4 && n >= 2;

    // The K samples of slice J.  (U - J s) is a product then a difference,
    // each rounded once (no contraction): the in-range test must be decided
    // exactly as the definition states it.
    auto sample = [&](int J, float (&r)[K]) {
#pragma clang fp contract(off)
        const int sl = (mv.sigma > 0 ? n - 1 - J : J) * sta;
        const double pb = (double)J * mv.sb, pc = (double)J * mv.sc;
        const double u = dU - pb;
        const bool uin = u >= -0.5 && u <= hi;
        const double fu = floor(u);
        const float wu = (float)(u - fu);
        const int u0 = (int)fu;
        const int cu0 = min(max(u0, 0), n - 1), cu1 = min(max(u0 + 1, 0), n - 1);
        const int ou0 = sl + cu0 * stb, ou1 = sl + cu1 * stb;
        const int cb = min(max(u0, 0), n - 2), ob = sl + cb * 4;
        const bool hiA = cu0 != cb, hiB = cu1 != cb;
        double v[K];
        int f[K];
        bool in[K], any = false;
#pragma unroll
        for (int k = 0; k < K; k++) {
            v[k] = (dV + k) - pc;
            f[k] = (int)floor(v[k]);
            in[k] = uin && v[k] >= -0.5 && v[k] <= hi;
            any |= in[k];
        }
        float a[K + 1], b[K + 1];
#pragma unroll
        for (int q = 0; q <= K; q++) a[q] = b[q] = 0.f;
        if (any && wide) {
#pragma unroll
            for (int q = 0; q <= K; q++) {
                const int oy = min(max(f[0] + q, 0), n - 1) * stc;
                const u32x2 p = __builtin_amdgcn_raw_buffer_load_b64(rR, ob + oy, 0, 0);
                a[q] = __uint_as_float(hiA ? p.y : p.x);
                b[q] = __uint_as_float(hiB ? p.y : p.x);
            }
        } else if (any) {
#pragma unroll
            for (int q = 0; q <= K; q++) {
                const int oy = min(max(f[0] + q, 0), n - 1) * stc;
                a[q] = ld(ou0 + oy);
                b[q] = ld(ou1 + oy);
            }
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            float r00 = a[k], r10 = b[k], r01 = a[k + 1], r11 = b[k + 1];
            if (in[k] && f[k] != f[0] + k) {
                // the rows of ray k are not those of ray 0 shifted by k (a
                // rounding of U - J s at another magnitude): load its own
                const int oy0 = min(max(f[k], 0), n - 1) * stc, oy1 = min(max(f[k] + 1, 0), n - 1) * stc;
                r00 = ld(ou0 + oy0);
                r10 = ld(ou1 + oy0);
                r01 = ld(ou0 + oy1);
                r11 = ld(ou1 + oy1);
            }
            const float wv = (float)(v[k] - (double)f[k]);
            const float r0 = r00 + wu * (r10 - r00);
            const float r1 = r01 + wu * (r11 - r01);
            r[k] = in[k] ? r0 + wv * (r1 - r0) : 0.f;
        }
    };

    double carry[K];
#pragma unroll
    for (int k = 0; k < K; k++) carry[k] = 0.0;
    for (int J0 = 0; J0 < n; J0 += chunk) {
        const int Js = J0 + w * seg;
        const int cnt = min(seg, n - Js);   // slices of this wave's segment (may be <= 0)
        float rs[kSwSeg][K];
        float sm[K], cp[K];
#pragma unroll
        for (int k = 0; k < K; k++) sm[k] = cp[k] = 0.f;
#pragma unroll
        for (int j = 0; j < kSwSeg; j++) {
            if (j < cnt) {
                sample(Js + j, rs[j]);
#pragma unroll
                for (int k = 0; k < K; k++) neumaier(sm[k], cp[k], rs[j][k]);
            }
        }
#pragma unroll
        for (int k = 0; k < K; k++) tot[w][k][lane] = (double)sm[k] + (double)cp[k];
        __syncthreads();
        // this segment starts from the earlier chunks and the earlier segments
        double P[K];
#pragma unroll
        for (int k = 0; k < K; k++) P[k] = carry[k];
#pragma unroll 1
        for (int q = 0; q < w; q++) {
#pragma unroll
            for (int k = 0; k < K; k++) P[k] += tot[q][k][lane];
        }
        if (J0 + chunk < n) {
#pragma unroll
            for (int k = 0; k < K; k++) carry[k] = P[k];
#pragma unroll 1
            for (int q = w; q < kSwWaves; q++) {
#pragma unroll
                for (int k = 0; k < K; k++) carry[k] += tot[q][k][lane];
            }
        }
#pragma unroll
        for (int k = 0; k < K; k++) {
            sm[k] = (float)P[k];
            cp[k] = (float)(P[k] - (double)sm[k]);
        }
        const uint32_t o0 = ((uint32_t)V0 * nu + iu) * 8;   // pair of the first written ray at J = 0
#pragma unroll
        for (int j = 0; j < kSwSeg; j++) {
            if (j < cnt) {
                const int J = Js + j;
                float d[K];
#pragma unroll
                for (int k = 0; k < K; k++) {
                    d[k] = lv.ds * ((sm[k] + cp[k]) + 0.5f * rs[j][k]);
                    neumaier(sm[k], cp[k], rs[j][k]);
                }
                if (lane_out) {
                    const __amdgpu_buffer_rsrc_t rQ = slice_rsrc(J);   // J is the same on every lane
#pragma unroll
                    for (int k = 1; k < K; k++) {
                        const int iv = V0 + k - 1;
                        if (iv < nv) {
                            const float dm = iv == 0 ? d[k] : d[k - 1];
                            const uint32_t oq = o0 + (uint32_t)(k - 1) * nu * 8;
                            __builtin_amdgcn_raw_buffer_store_b64(u32x2{__float_as_uint(dm), __float_as_uint(d[k])},
                                                                  rQ, (int)oq, 0, kStream);
                            if (iv == nv - 1)
                                __builtin_amdgcn_raw_buffer_store_b64(
                                    u32x2{__float_as_uint(d[k]), __float_as_uint(d[k])}, rQ,
                                    (int)(oq + (uint32_t)nu * 8), 0, kStream);
                        }
                    }
                }
            }
        }
        if (J0 + chunk < n) __syncthreads();   // tot is rewritten by the next chunk
    }
}

// Per-light lattice tables: unit offset directions d_t = o_t / |o_t| and the
// incident-side phase f(d_t . l) of the phase feature (eq. 8) for the
// medium's phase f (its HG lobes, eq. 6).  The centre site (o = 0) has no
// direction; its phase feature is f(w . l), so it stores (l, 1).
__global__ void k_site_tables(MediumView mv, SiteTables* tab)
{
    const int t = threadIdx.x;
    if (t >= kSites) return;
    const int qi = t / 25, j = (t / 5) % 5 - 2, i = t % 5 - 2;
    double o[3];
    for (int d = 0; d < 3; d++) o[d] = mv.qoff[d][qi];
    o[mv.b] += i;
    o[mv.c] += j;
    const double on = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    if (on == 0.0) {
        tab->site[t] = make_float4((float)mv.l[0], (float)mv.l[1], (float)mv.l[2], 1.f);
        return;
    }
    const double dl = (o[0] * mv.l[0] + o[1] * mv.l[1] + o[2] * mv.l[2]) / on;
    double ph = 0.0;   // the medium's phase at d_t . l: its lobes summed with their weights (eq. 6)
    for (int k = 0; k < mv.nl; k++) {
        const double den = mv.hg_a[k] - mv.hg_b[k] * dl;
        ph += mv.hg_k[k] / (den * sqrt(den));
    }
    tab->site[t] = make_float4((float)(o[0] / on), (float)(o[1] / on), (float)(o[2] / on), (float)ph);
}

// ---- volume phase (eq. 9) ----------------------------------------------------
// A site seen from the point is read as a ball of half the lattice spacing,
// so it subtends a cone of half-angle beta = asin(1 / (2 |o|)) around the
// site direction d; the volume phase is the medium's phase averaged over the
// cone.  For a direction v with v . d = mu0, a cone direction at polar angle
// theta and azimuth psi has v . phi = mu0 cos theta + sqrt(1 - mu0^2) sin theta
// cos psi, so an HG lobe's denominator is A - B cos psi; its azimuthal
// integral, of (A - B cos psi)^(-3/2), is 4 E(m) / ((A - B) sqrt(A + B)) with
// m = 2B / (A + B) (B >= 0), and cos theta over [cos beta, 1] is integrated
// with 64-point Gauss-Legendre.

// complete elliptic integral of the second kind by the arithmetic-geometric mean
__device__ double ellip_e(double m)
{
    double a = 1.0, b = sqrt(1.0 - m), c = sqrt(m), s = 0.5 * m, p = 0.5;
    for (int it = 0; it < 40 && c > 1e-17; it++) {
        const double an = 0.5 * (a + b);
        c = 0.5 * (a - b);
        b = sqrt(a * b);
        a = an;
        p *= 2.0;
        s += p * c * c;
    }
    return (M_PI / (2.0 * a)) * (1.0 - s);
}

// the medium's phase averaged over a cone of half-angle beta around d, mu0 = v . d
__device__ double cone_phase(const MediumView& mv, const GaussLegendre64& gl, double mu0, double beta)
{
    const double cb = cos(beta), s0 = sqrt(fmax(0.0, 1.0 - mu0 * mu0));
    const double half = 0.5 * (1.0 - cb), mid = 0.5 * (1.0 + cb);
    double total = 0.0;
    for (int k = 0; k < mv.nl; k++) {
        const double g2 = 0.5 * mv.hg_b[k];   // g
        double acc = 0.0;
        for (int i = 0; i < 64; i++) {
            const double t = mid + half * gl.x[i];
            const double A = mv.hg_a[k] - mv.hg_b[k] * mu0 * t;
            const double B = fabs(2.0 * g2 * s0 * sqrt(fmax(0.0, 1.0 - t * t)));
            acc += gl.w[i] * half * (4.0 * ellip_e(2.0 * B / (A + B)) / ((A - B) * sqrt(A + B)));
        }
        total += mv.hg_k[k] * acc;   // hg_k carries the lobe's weight and (1 - g^2) / (4 pi)
    }
    return total / (2.0 * M_PI * (1.0 - cb));
}

// Volume-phase tables of the current light and phase: block t (a site other
// than the centre) replaces its site-table entry's incident-side phase by the
// cone mean at d_t . l, and fills row t of vtab with the cone means at angles
// pi b / (kVBins - 1), b < kVBins, between w and d_t (uniform in the angle,
// so that forward and backward lobes are resolved alike).
__global__ void __launch_bounds__(256) k_volume_tables(MediumView mv, GaussLegendre64 gl, SiteTables* tab, float* vtab)
{
    const int t = blockIdx.x;
    if (t == kCentreSite) return;
    const int qi = t / 25, j = (t / 5) % 5 - 2, i = t % 5 - 2;
    double o[3];
    for (int d = 0; d < 3; d++) o[d] = mv.qoff[d][qi];
    o[mv.b] += i;
    o[mv.c] += j;
    const double on = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    const double beta = asin(0.5 / on);
    for (int b = threadIdx.x; b < kVBins; b += blockDim.x) {
        vtab[(int64_t)t * kVBins + b] = (float)cone_phase(mv, gl, cos(M_PI * b / (kVBins - 1)), beta);
    }
    if (threadIdx.x == 0) {
        const double dl = (o[0] * mv.l[0] + o[1] * mv.l[1] + o[2] * mv.l[2]) / on;
        tab->site[t].w = (float)cone_phase(mv, gl, dl, beta);
    }
}

hipError_t launch_volume_tables(const MediumView& mv, const GaussLegendre64& gl, SiteTables* tab, float* vtab,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_volume_tables, dim3(kSites), dim3(256), 0, s, mv, gl, tab, vtab);
    return hipGetLastError();
}

// Light-axis density pairs (a layout of the pyramid for the gather): for each
// level, entry (A', c, b), A' = 0..n, b = -kPairPad..n-1+kPairPad, holds the
// density at a = A'-1 and its step to a = A' along the light's dominant axis,
// (rho(A'-1), rho(A') - rho(A'-1)), each index (b too) clamped into [0, n-1],
// stored with b fastest; so the two a-planes of a density row sit side by
// side, a row of 6 pairs is 48 contiguous bytes whatever the light, and the
// gather's interpolation along a is one fused multiply-add (the same
// rounding as rho0 + w (rho1 - rho0) evaluated there).
// One thread per four neighbouring entries along b (n >= 4; smaller levels
// one entry per thread): 16-byte loads of the two a-planes when b is x, two
// 16-byte stores.
template <int E>
__global__ void __launch_bounds__(256)
k_pairs(const float* __restrict__ rho, float2* __restrict__ out, int n, int lg, int sa, int sb, int sc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ((n + 1) << (2 * lg)) / E) return;
    const int lq = lg - (E == 4 ? 2 : 0);
    const int bb = (t & ((n / E) - 1)) * E, cc = (t >> lq) & (n - 1), ap = t >> (lq + lg);
    const int a0 = ap - 1 < 0 ? 0 : ap - 1, a1 = ap > n - 1 ? n - 1 : ap;
    const float* r0 = rho + a0 * sa + cc * sc + bb * sb;
    const float* r1 = rho + a1 * sa + cc * sc + bb * sb;
    float v0[E], v1[E];
    if (E == 4 && sb == 1) {
        const float4 p = *reinterpret_cast<const float4*>(r0), q = *reinterpret_cast<const float4*>(r1);
        v0[0] = p.x, v0[1] = p.y, v0[2] = p.z, v0[3] = p.w;
        v1[0] = q.x, v1[1] = q.y, v1[2] = q.z, v1[3] = q.w;
    } else {
#pragma unroll
        for (int e = 0; e < E; e++) v0[e] = r0[e * sb], v1[e] = r1[e * sb];
    }
#pragma unroll
    for (int e = 0; e < E; e++) v1[e] -= v0[e];   // the step along a
    // non-temporal stores: the pairs are read back only by the gather, long
    // after this pass, so they should not displace cached lines on the way
    const int nb = n + 2 * kPairPad;
    float2* row = out + ((ap << lg) + cc) * nb;
    float2* o = row + kPairPad + bb;
    // the padding entries of the row repeat its end samples
    if (bb == 0)
        for (int e = 0; e < kPairPad; e++) row[e] = make_float2(v0[0], v1[0]);
    if (bb + E == n)
        for (int e = 0; e < kPairPad; e++) row[kPairPad + n + e] = make_float2(v0[E - 1], v1[E - 1]);
    if (E == 4) {
        typedef float f32x4 __attribute__((ext_vector_type(4)));
        __builtin_nontemporal_store(f32x4{v0[0], v1[0], v0[1], v1[1]}, reinterpret_cast<f32x4*>(o));
        __builtin_nontemporal_store(f32x4{v0[2], v1[2], v0[3], v1[3]}, reinterpret_cast<f32x4*>(o) + 1);
    } else {
        o[0] = make_float2(v0[0], v1[0]);
    }
}

hipError_t launch_pairs(const MediumView& mv, hipStream_t s)
{
    for (int m = 0; m < mv.levels; m++) {
        const Level& lv = mv.lev[m];
        const int lg = __builtin_ctz(lv.n);
        const int total = (lv.n + 1) << (2 * lg);
        auto stride = [&](int axis) { return 1 << (lg * mv.se[axis]); };
        const int sa = stride(mv.a), sb = stride(mv.b), sc = stride(mv.c);
        if (lv.n >= 4)
            hipLaunchKernelGGL(k_pairs<4>, dim3((total / 4 + 255) / 256), dim3(256), 0, s, mv.rho_s + lv.rho_off,
                               mv.pairs + lv.p_off, lv.n, lg, sa, sb, sc);
        else
            hipLaunchKernelGGL(k_pairs<1>, dim3((total + 255) / 256), dim3(256), 0, s, mv.rho_s + lv.rho_off,
                               mv.pairs + lv.p_off, lv.n, lg, sa, sb, sc);
    }
    return hipGetLastError();
}

hipError_t launch_site_tables(const MediumView& mv, SiteTables* tab, hipStream_t s)
{
    hipLaunchKernelGGL(k_site_tables, dim3(1), dim3(256), 0, s, mv, tab);
    return hipGetLastError();
}

hipError_t launch_pyramid(const float* rho, const Level* lev, int levels, hipStream_t s)
{
    for (int m = 0; m + 1 < levels; m++) {
        const int nc = lev[m + 1].n, lg = __builtin_ctz(nc);
        const int threads = nc == 1 ? 1 : (nc * nc * nc) / 2;
        hipLaunchKernelGGL(k_mip, dim3((threads + 255) / 256), dim3(256), 0, s, rho + lev[m].rho_off,
                           const_cast<float*>(rho) + lev[m + 1].rho_off, nc, lg);
    }
    return hipGetLastError();
}

hipError_t launch_transpose(const MediumView& mv, hipStream_t s)
{
    for (int m = 0; m < mv.levels; m++) {
        const Level& lv = mv.lev[m];
        const int t = (lv.n + 31) / 32;
        hipLaunchKernelGGL(k_transpose_x, dim3(t, t, lv.n), dim3(256), 0, s, mv.rho + lv.rho_off,
                           const_cast<float*>(mv.rho_s) + lv.rho_off, lv.n);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const MediumView& mv, hipStream_t s)
{
    SweepArgs sa;
    sa.blk_off[0] = 0;
    for (int m = 0; m < kMaxLevels; m++) {
        const Level& lv = mv.lev[m];
        const int blocks = m < mv.levels ? ((lv.nu + 63) / 64) * ((lv.nv + kSwRays - 1) / kSwRays) : 0;
        sa.blk_off[m + 1] = sa.blk_off[m] + blocks;
    }
    hipLaunchKernelGGL(k_sweep, dim3(sa.blk_off[mv.levels]), dim3(64 * kSwWaves), 0, s, mv, sa);
    return hipGetLastError();
}

}  // namespace nis
