// k_volume.hip -- density pyramid and light-direction path-density sweep.
//
// Pyramid (Sec. III.B.1): each coarser level is the 2x2x2 box mean of the
// level below, down to 1^3.
//
// Sweep (eq. 1 with the extinction of eq. 15): for every level m and every
// light-sheared ray (U,V) the kernel walks the n_m slices J from the
// light-facing face and writes the path density
//     D_m(U,V,J) = ds_m * ( sum_{J'<J} r(J') + r(J)/2 ),
// where r(J) is the bilinear density on slice J at lateral index coordinates
// (U - J sb, V - J sc), or 0 outside [-1/2, n_m - 1/2].  The graded
// transmittance exp(-lambda^(m+1) sigma_t D) is applied at lookup time, so
// the field does not depend on sigma_t.  The running sum is compensated
// (Neumaier) float32.  One lane per ray, lanes along U: for a light dominated
// by y or z the lateral axis b is x, so neighbouring lanes read neighbouring
// voxels and write neighbouring D entries.
#include "launch_args.h"

namespace nis {

__global__ void __launch_bounds__(256)
k_mip(const float* __restrict__ fine, float* __restrict__ coarse, int nc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nc * nc * nc;
    if (i >= total) return;
    int x = (int)(i % nc);
    int y = (int)((i / nc) % nc);
    int z = (int)(i / ((int64_t)nc * nc));
    int64_t nf = 2 * (int64_t)nc;
    const float* f = fine + ((2 * z) * nf + 2 * y) * nf + 2 * x;
    float2 a = *reinterpret_cast<const float2*>(f);
    float2 b = *reinterpret_cast<const float2*>(f + nf);
    float2 c = *reinterpret_cast<const float2*>(f + nf * nf);
    float2 d = *reinterpret_cast<const float2*>(f + nf * nf + nf);
    float s = ((a.x + a.y) + (b.x + b.y)) + ((c.x + c.y) + (d.x + d.y));
    coarse[i] = s * 0.125f;
}

// (U - J s) evaluated as a product then a difference, each rounded once: the
// in-range test below must be decided exactly as the definition states it.
__device__ __forceinline__ double lateral(int U, int J, double s)
{
#pragma clang fp contract(off)
    return (double)U - (double)J * s;
}

struct SweepArgs {
    int64_t ray_off[kMaxLevels + 1];   // prefix sums of rays per level
};

__global__ void __launch_bounds__(256)
k_sweep(MediumView mv, SweepArgs sa)
{
    int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= sa.ray_off[mv.levels]) return;
    int m = 0;
    while (m + 1 < mv.levels && gid >= sa.ray_off[m + 1]) m++;
    const Level lv = mv.lev[m];
    int64_t local = gid - sa.ray_off[m];
    int iu = (int)(local % lv.nu), iv = (int)(local / lv.nu);
    int U = lv.ulo + iu, V = lv.vlo + iv;
    const int n = lv.n;
    const float* rho = mv.rho + lv.rho_off;
    float* D = mv.D + lv.d_off + (int64_t)iv * lv.nu + iu;
    const int64_t plane = (int64_t)lv.nu * lv.nv;
    int64_t st[3] = {1, n, (int64_t)n * n};
    const int64_t sta = st[mv.a], stb = st[mv.b], stc = st[mv.c];
    const double hi = n - 0.5;
    float sum = 0.f, comp = 0.f;
#pragma unroll 4
    for (int J = 0; J < n; J++) {
        int ia = mv.sigma > 0 ? n - 1 - J : J;
        double u = lateral(U, J, mv.sb);
        double v = lateral(V, J, mv.sc);
        float r = 0.f;
        if (u >= -0.5 && u <= hi && v >= -0.5 && v <= hi) {
            double fu = floor(u), fv = floor(v);
            int u0 = (int)fu, v0 = (int)fv;
            float wu = (float)(u - fu), wv = (float)(v - fv);
            int u1 = min(u0 + 1, n - 1), v1 = min(v0 + 1, n - 1);
            u0 = max(u0, 0);
            v0 = max(v0, 0);
            const float* s = rho + ia * sta;
            float r00 = s[u0 * stb + v0 * stc], r10 = s[u1 * stb + v0 * stc];
            float r01 = s[u0 * stb + v1 * stc], r11 = s[u1 * stb + v1 * stc];
            float r0 = r00 + wu * (r10 - r00);
            float r1 = r01 + wu * (r11 - r01);
            r = r0 + wv * (r1 - r0);
        }
        D[J * plane] = lv.ds * ((sum + comp) + 0.5f * r);
        float t = sum + r;
        comp += fabsf(sum) >= fabsf(r) ? (sum - t) + r : (r - t) + sum;
        sum = t;
    }
}

// Per-light lattice tables: unit offset directions d_t = o_t / |o_t| and the
// incident-side phase HG(d_t . l) of the phase feature (eq. 8) for the
// current g.  The centre site (o = 0) has no direction; its phase feature is
// HG(w . l), so it stores (l, 1).
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
    const double den = mv.hg_a - mv.hg_b * dl;
    tab->site[t] = make_float4((float)(o[0] / on), (float)(o[1] / on), (float)(o[2] / on),
                               (float)(mv.hg_k / (den * sqrt(den))));
}

// Light-axis density pairs (a layout of the pyramid for the gather): for each
// level, entry (A', c, b), A' = 0..n, holds the densities at a = A'-1 and
// a = A' along the light's dominant axis, each index clamped into [0, n-1],
// stored with b fastest; so the two a-planes of a density row sit side by
// side and a row of 6 pairs is 48 contiguous bytes whatever the light.
__global__ void __launch_bounds__(256)
k_pairs(const float* __restrict__ rho, float2* __restrict__ out, int n, int a, int b, int c)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)(n + 1) * n * n) return;
    const int bb = (int)(i % n), cc = (int)((i / n) % n), ap = (int)(i / ((int64_t)n * n));
    const int a0 = ap - 1 < 0 ? 0 : ap - 1, a1 = ap > n - 1 ? n - 1 : ap;
    int p0[3], p1[3];
    p0[a] = a0, p1[a] = a1;
    p0[b] = p1[b] = bb;
    p0[c] = p1[c] = cc;
    out[i] = make_float2(rho[((int64_t)p0[2] * n + p0[1]) * n + p0[0]], rho[((int64_t)p1[2] * n + p1[1]) * n + p1[0]]);
}

hipError_t launch_pairs(const MediumView& mv, hipStream_t s)
{
    for (int m = 0; m < mv.levels; m++) {
        const Level& lv = mv.lev[m];
        const int64_t total = (int64_t)(lv.n + 1) * lv.n * lv.n;
        const int blocks = (int)((total + 255) / 256);
        hipLaunchKernelGGL(k_pairs, dim3(blocks), dim3(256), 0, s, mv.rho + lv.rho_off, mv.pairs + lv.p_off, lv.n,
                           mv.a, mv.b, mv.c);
    }
    return hipGetLastError();
}

// Path-density pairs along V (a layout of D for the gather): entry (J, V', U),
// V' = 0..nv, holds D at V = V'-1 and V = V', each index clamped into
// [0, nv-1], so two neighbouring V rows of a brick are one contiguous run.
__global__ void __launch_bounds__(256)
k_dpairs(const float* __restrict__ D, float2* __restrict__ out, int n, int nv, int nu)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n * (nv + 1) * nu) return;
    const int u = (int)(i % nu), vp = (int)((i / nu) % (nv + 1)), j = (int)(i / ((int64_t)nu * (nv + 1)));
    const int v0 = vp - 1 < 0 ? 0 : vp - 1, v1 = vp > nv - 1 ? nv - 1 : vp;
    const float* row = D + (int64_t)j * nv * nu + u;
    out[i] = make_float2(row[(int64_t)v0 * nu], row[(int64_t)v1 * nu]);
}

hipError_t launch_dpairs(const MediumView& mv, hipStream_t s)
{
    for (int m = 0; m < mv.levels; m++) {
        const Level& lv = mv.lev[m];
        const int64_t total = (int64_t)lv.n * (lv.nv + 1) * lv.nu;
        const int blocks = (int)((total + 255) / 256);
        hipLaunchKernelGGL(k_dpairs, dim3(blocks), dim3(256), 0, s, mv.D + lv.d_off, mv.dpairs + lv.q_off, lv.n, lv.nv,
                           lv.nu);
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
        int nc = lev[m + 1].n;
        int64_t total = (int64_t)nc * nc * nc;
        int blocks = (int)((total + 255) / 256);
        hipLaunchKernelGGL(k_mip, dim3(blocks), dim3(256), 0, s, rho + lev[m].rho_off,
                           const_cast<float*>(rho) + lev[m + 1].rho_off, nc);
    }
    return hipGetLastError();
}

hipError_t launch_sweep(const MediumView& mv, hipStream_t s)
{
    SweepArgs sa;
    sa.ray_off[0] = 0;
    for (int m = 0; m < kMaxLevels; m++)
        sa.ray_off[m + 1] = sa.ray_off[m] + (m < mv.levels ? (int64_t)mv.lev[m].nu * mv.lev[m].nv : 0);
    int64_t total = sa.ray_off[mv.levels];
    int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_sweep, dim3(blocks), dim3(256), 0, s, mv, sa);
    return hipGetLastError();
}

}  // namespace nis
