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
#include "launch_args.h"
#include "mfma.h"

namespace nis {

constexpr int kTP = 32;          // points per workgroup
constexpr int kTPT = 8;          // gather threads per point
constexpr int kLatStride = 232;  // 225 sites + padding
constexpr int kY1Stride = 72;    // 63 conv1 positions + zero padding

struct Slab {
    int ib0, ic0;                // density base indices along b, c for this slab
    float wb, wc;                // their weights
    int mask;                    // bits 0-4: i in range, 5-9: j in range, 10: slab in range
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

__device__ __forceinline__ double hg64(const MediumView& mv, double mu)
{
    double den = mv.hg_a - mv.hg_b * mu;
    return mv.hg_k / (den * sqrt(den));
}

__device__ __forceinline__ float lerpf(float a, float b, float w) { return a + w * (b - a); }

// index-clamped trilinear lookup in a path-density field D[J][V][U]
__device__ __forceinline__ float sample_D(const float* __restrict__ D, const Level& lv, int U, int V,
                                          int J, float wu, float wv, float wj)
{
    int u0 = min(max(U - lv.ulo, 0), lv.nu - 1), u1 = min(max(U + 1 - lv.ulo, 0), lv.nu - 1);
    int v0 = min(max(V - lv.vlo, 0), lv.nv - 1), v1 = min(max(V + 1 - lv.vlo, 0), lv.nv - 1);
    int j0 = min(max(J, 0), lv.n - 1), j1 = min(max(J + 1, 0), lv.n - 1);
    const int64_t plane = (int64_t)lv.nu * lv.nv;
    const float* d0 = D + j0 * plane;
    const float* d1 = D + j1 * plane;
    float a00 = lerpf(d0[v0 * lv.nu + u0], d0[v0 * lv.nu + u1], wu);
    float a01 = lerpf(d0[v1 * lv.nu + u0], d0[v1 * lv.nu + u1], wu);
    float a10 = lerpf(d1[v0 * lv.nu + u0], d1[v0 * lv.nu + u1], wu);
    float a11 = lerpf(d1[v1 * lv.nu + u0], d1[v1 * lv.nu + u1], wu);
    return lerpf(lerpf(a00, a01, wv), lerpf(a10, a11, wv), wj);
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

__device__ __forceinline__ int tap_offset(int k)   // conv1 tap (dz,dy,dx) in the 9x5x5 lattice
{
    return (k / 9) * 25 + ((k / 3) % 3) * 5 + (k % 3);
}

template <int PREC>
__global__ void __launch_bounds__(256)
k_features(FeatArgs A)
{
    typedef Mfma<PREC> M;
    typedef typename M::elem E;
    __shared__ E lat[kTP][kLatStride];
    __shared__ E y1[kTP][8][kY1Stride];
    __shared__ float H[kTP][16][5];
    __shared__ float gate[kTP][16];
    __shared__ Slab slab[kTP][9];
    __shared__ float pstat[kTP][kStats];
    __shared__ float pfix[kTP][3];

    const MediumView& mv = A.mv;
    const int tid = threadIdx.x;
    const int lp = tid / kTPT, r = tid % kTPT;
    const int64_t p = (int64_t)blockIdx.x * kTP + lp;
    const bool live = p < A.npts;
    const int64_t pc = live ? p : A.npts - 1;

    // zero the conv1 output padding once (read with zero weights by conv2)
    for (int e = tid; e < kTP * 8 * kY1Stride; e += 256) {
        int pt = e / (8 * kY1Stride), rem = e % (8 * kY1Stride);
        y1[pt][rem / kY1Stride][rem % kY1Stride] = M::zero();
    }

    double x[3], w[3];
    for (int d = 0; d < 3; d++) {
        x[d] = A.pts[3 * pc + d];
        w[d] = A.dirs[3 * pc + d];
    }
    {
        double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int d = 0; d < 3; d++) w[d] /= wn;
    }
    const double wl = w[0] * mv.l[0] + w[1] * mv.l[1] + w[2] * mv.l[2];

    // ---- phase features (independent of the layer) -------------------------
    {
        const float wf0 = (float)w[0], wf1 = (float)w[1], wf2 = (float)w[2];
        const float ha = (float)mv.hg_a, hb = (float)mv.hg_b, hk = (float)mv.hg_k;
        float phs = 0.f, phm = -INFINITY;
        for (int t = r; t < kSites; t += kTPT) {
            float P;
            if (t == kSites / 2) {
                P = (float)hg64(mv, wl);
            } else {
                float mu = wf0 * A.tab->dir[t][0] + wf1 * A.tab->dir[t][1] + wf2 * A.tab->dir[t][2];
                float den = fmaf(-hb, mu, ha);
                P = hk / (den * sqrtf(den)) * A.tab->hg_dl[t];
            }
            float ph = log1pf(P);
            phs += ph;
            phm = fmaxf(phm, ph);
            if (A.dbg_phi && live) A.dbg_phi[p * kSites + t] = ph;
        }
        for (int o = 1; o < kTPT; o <<= 1) {
            phs += __shfl_xor(phs, o);
            phm = fmaxf(phm, __shfl_xor(phm, o));
        }
        if (r == 0) {
            pfix[lp][0] = phs / kSites;
            pfix[lp][1] = phm;
            pfix[lp][2] = (float)acos(fmin(1.0, fmax(-1.0, wl)));
        }
    }
    // ---- transmittance to the light and the single-scatter term -------------
    if (r == 0 && live) {
        const Level& l0 = mv.lev[0];
        double Uf, Vf, Jf;
        sheared(mv, l0.n, x, Uf, Vf, Jf);
        double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
        float D0 = sample_D(mv.D + l0.d_off, l0, (int)fu, (int)fv, (int)fj, (float)(Uf - fu),
                            (float)(Vf - fv), (float)(Jf - fj));
        float T = expf(-mv.sigma_t * D0);
        A.f0[p] = (float)(hg64(mv, wl) * (double)T);
        if (A.dbg_tp) A.dbg_tp[p] = T;
    }

    const int wave = tid / 64, lane = tid % 64;
    const int lr = lane % 16, lg = lane / 16;
    E* desc = reinterpret_cast<E*>(A.desc);

    for (int k = 0; k < kLayers; k++) {
        const int m = k < mv.levels - 1 ? k : mv.levels - 1;
        const Level lv = mv.lev[m];
        const int nm = lv.n;
        const int c = 1 << (k - m);
        const double scale = ldexp(1.0 / mv.n0, k);
        const int grp = k < kDiffuse ? 0 : 1;

        // per-slab density bases and exact in-cube masks
        for (int qi = r; qi < 9; qi += kTPT) {
            Slab s;
            int mask = 0;
            double sa = site_coord_a(x[mv.a], scale, mv.qoff[mv.a][qi]);
            if (sa >= 0.0 && sa <= 1.0) mask |= 1 << 10;
            for (int i = -2; i <= 2; i++) {
                double sb = site_coord(x[mv.b], scale, mv.qoff[mv.b][qi], i);
                double sc = site_coord(x[mv.c], scale, mv.qoff[mv.c][qi], i);
                if (sb >= 0.0 && sb <= 1.0) mask |= 1 << (i + 2);
                if (sc >= 0.0 && sc <= 1.0) mask |= 1 << (i + 7);
            }
            double gb = x[mv.b] * nm - 0.5 + c * mv.qoff[mv.b][qi];
            double gc = x[mv.c] * nm - 0.5 + c * mv.qoff[mv.c][qi];
            double fb = floor(gb), fc = floor(gc);
            s.ib0 = (int)fb;
            s.ic0 = (int)fc;
            s.wb = (float)(gb - fb);
            s.wc = (float)(gc - fc);
            s.mask = mask;
            slab[lp][qi] = s;
        }
        double Uf, Vf, Jf;
        sheared(mv, nm, x, Uf, Vf, Jf);
        const double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
        const int iu = (int)fu, iv = (int)fv, ij = (int)fj;
        const float wu = (float)(Uf - fu), wv = (float)(Vf - fv), wj = (float)(Jf - fj);
        const double ga = x[mv.a] * nm - 0.5;
        const double fa = floor(ga);
        const int ia0 = (int)fa;
        const float wa = (float)(ga - fa);
        const float coef = A.coef[k];
        const float* rho = mv.rho + lv.rho_off;
        const float* D = mv.D + lv.d_off;
        const int64_t st[3] = {1, nm, (int64_t)nm * nm};
        __syncthreads();

        float rs = 0.f, rmx = -INFINITY, ts = 0.f, tmx = -INFINITY;
        for (int t = r; t < kSites; t += kTPT) {
            const int qi = t / 25, j = (t / 5) % 5 - 2, i = t % 5 - 2;
            const int q = qi - 4;
            const Slab s = slab[lp][qi];
            float rv = 0.f;
            if ((s.mask >> 10) & (s.mask >> (i + 2)) & (s.mask >> (j + 7)) & 1) {
                int ja = ia0 + c * q * mv.sigma, jb = s.ib0 + c * i, jc = s.ic0 + c * j;
                int a0 = min(max(ja, 0), nm - 1), a1 = min(max(ja + 1, 0), nm - 1);
                int b0 = min(max(jb, 0), nm - 1), b1 = min(max(jb + 1, 0), nm - 1);
                int c0 = min(max(jc, 0), nm - 1), c1 = min(max(jc + 1, 0), nm - 1);
                int64_t A0 = a0 * st[mv.a], A1 = a1 * st[mv.a];
                int64_t B0 = b0 * st[mv.b], B1 = b1 * st[mv.b];
                int64_t C0 = c0 * st[mv.c], C1 = c1 * st[mv.c];
                float v00 = lerpf(rho[A0 + B0 + C0], rho[A1 + B0 + C0], wa);
                float v10 = lerpf(rho[A0 + B1 + C0], rho[A1 + B1 + C0], wa);
                float v01 = lerpf(rho[A0 + B0 + C1], rho[A1 + B0 + C1], wa);
                float v11 = lerpf(rho[A0 + B1 + C1], rho[A1 + B1 + C1], wa);
                rv = lerpf(lerpf(v00, v10, s.wb), lerpf(v01, v11, s.wb), s.wc);
            }
            float Dv = sample_D(D, lv, iu + c * i, iv + c * j, ij - c * q, wu, wv, wj);
            float T = expf(-coef * Dv);
            lat[lp][t] = M::cvt(T);
            rs += rv;
            rmx = fmaxf(rmx, rv);
            ts += T;
            tmx = fmaxf(tmx, T);
            if (live && A.dbg_tbar) A.dbg_tbar[(p * kLayers + k) * kSites + t] = T;
            if (live && A.dbg_rho) A.dbg_rho[(p * kLayers + k) * kSites + t] = rv;
        }
        for (int o = 1; o < kTPT; o <<= 1) {
            rs += __shfl_xor(rs, o);
            ts += __shfl_xor(ts, o);
            rmx = fmaxf(rmx, __shfl_xor(rmx, o));
            tmx = fmaxf(tmx, __shfl_xor(tmx, o));
        }
        if (r == 0) {
            float* v = pstat[lp];
            v[0] = rs / kSites;
            v[1] = pfix[lp][0];
            v[2] = ts / kSites;
            v[3] = rmx;
            v[4] = pfix[lp][1];
            v[5] = tmx;
            v[6] = mv.g;
            v[7] = pfix[lp][2];
            if (live && A.dbg_stats)
                for (int e = 0; e < kStats; e++) A.dbg_stats[(p * kLayers + k) * kStats + e] = v[e];
        }
        __syncthreads();

        // ---- conv1: [rows = (point, position)] x [K = 27 taps] x [8 channels]
        {
            const E* w1 = reinterpret_cast<const E*>(A.w1t[grp]);
            const float* b1 = A.cb[grp];
            typename M::frag bw[kConv1K / M::KS];
#pragma unroll
            for (int kc = 0; kc < kConv1K / M::KS; kc++)
                bw[kc] = M::load(w1 + lr * kConv1K + kc * M::KS + lg * M::KPL);
            for (int tile = wave; tile < kTP * 4; tile += 4) {
                const int pt = tile >> 2, pos = (tile & 3) * 16 + lr;
                const int base = pos < 63 ? (pos / 9) * 25 + ((pos / 3) % 3) * 5 + pos % 3 : 0;
                const E* L = lat[pt] + base;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < kConv1K / M::KS; kc++) {
                    auto get = [&](int kk) -> E { return kk < 27 ? L[tap_offset(kk)] : M::zero(); };
                    acc = M::mma(M::gather(get, kc * M::KS + lg * M::KPL), bw[kc], acc);
                }
                if (lr < 8) {
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        int pos2 = (tile & 3) * 16 + lg * 4 + e;
                        if (pos2 < 63) y1[pt][lr][pos2] = M::cvt(fmaxf(acc[e] + b1[lr], 0.f));
                    }
                }
            }
        }
        __syncthreads();

        // ---- conv2: [rows = (point, z)] x [K = 8 x 27] x [16 channels]
        {
            const E* w2 = reinterpret_cast<const E*>(A.w2t[grp]);
            const float* b2 = A.cb[grp] + 8;
            for (int tile = wave; tile < kTP * 5 / 16; tile += 4) {
                const int row = tile * 16 + lr;
                const int pt = row / 5, z = row % 5;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
                for (int kc = 0; kc < kConv2K / M::KS; kc++) {
                    auto get = [&](int kk) -> E {
                        return kk < 216 ? y1[pt][kk / 27][z * 9 + kk % 27] : M::zero();
                    };
                    typename M::frag b = M::load(w2 + lr * kConv2K + kc * M::KS + lg * M::KPL);
                    acc = M::mma(M::gather(get, kc * M::KS + lg * M::KPL), b, acc);
                }
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int row2 = tile * 16 + lg * 4 + e;
                    H[row2 / 5][lr][row2 % 5] = fmaxf(acc[e] + b2[lr], 0.f);
                }
            }
        }
        __syncthreads();

        // ---- squeeze-excitation gate per point
        if (tid < kTP) {
            const float* cb = A.cb[grp];
            const float *s1 = cb + 24, *c1 = cb + 88, *s2 = cb + 92, *c2 = cb + 156;
            float zc[16], hid[4];
            for (int o = 0; o < 16; o++) {
                float s = 0.f;
                for (int z = 0; z < 5; z++) s += H[tid][o][z];
                zc[o] = s / 5.f;
            }
            for (int h = 0; h < 4; h++) {
                float s = c1[h];
                for (int o = 0; o < 16; o++) s += s1[h * 16 + o] * zc[o];
                hid[h] = fmaxf(s, 0.f);
            }
            for (int o = 0; o < 16; o++) {
                float s = c2[o];
                for (int h = 0; h < 4; h++) s += s2[o * 4 + h] * hid[h];
                gate[tid][o] = 1.f / (1.f + expf(-s));
            }
        }
        __syncthreads();

        // ---- descriptor entries of layer k
        for (int e = tid; e < kTP * kPerLayer; e += 256) {
            const int pt = e / kPerLayer, f = e % kPerLayer;
            const int64_t pp = (int64_t)blockIdx.x * kTP + pt;
            if (pp >= A.npts) continue;
            float v = f < kFeat ? gate[pt][f / 5] * H[pt][f / 5][f % 5] : pstat[pt][f - kFeat];
            desc[pp * kDescPad + k * kPerLayer + f] = M::cvt(v);
        }
        __syncthreads();
    }
    // albedo entry and zero padding
    for (int e = tid; e < kTP * (kDescPad - kDesc + 1); e += 256) {
        const int pt = e / (kDescPad - kDesc + 1), f = kDesc - 1 + e % (kDescPad - kDesc + 1);
        const int64_t pp = (int64_t)blockIdx.x * kTP + pt;
        if (pp < A.npts) desc[pp * kDescPad + f] = M::cvt(f == kDesc - 1 ? mv.albedo : 0.f);
    }
}

// Widen a descriptor of the given precision to float32 [n][1057].
template <int PREC>
__global__ void k_desc_to_f32(const void* src, float* dst, int64_t n)
{
    typedef typename Mfma<PREC>::elem E;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * kDesc) return;
    int64_t row = i / kDesc, col = i % kDesc;
    dst[i] = (float)reinterpret_cast<const E*>(src)[row * kDescPad + col];
}

hipError_t launch_desc_to_f32(int prec, const void* src, float* dst, int64_t n, hipStream_t s)
{
    int blocks = (int)((n * kDesc + 255) / 256);
    if (prec == kPrecBF16)
        hipLaunchKernelGGL(k_desc_to_f32<kPrecBF16>, dim3(blocks), dim3(256), 0, s, src, dst, n);
    else
        hipLaunchKernelGGL(k_desc_to_f32<kPrecFP32>, dim3(blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_features(int prec, const FeatArgs& a, hipStream_t s)
{
    if (a.npts <= 0) return hipSuccess;
    int blocks = (int)((a.npts + kTP - 1) / kTP);
    if (prec == kPrecBF16)
        hipLaunchKernelGGL(k_features<kPrecBF16>, dim3(blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_features<kPrecFP32>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace nis
