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
// Work split.  A workgroup holds kTP points.  Per layer, every thread of the
// workgroup evaluates rows of 5 sites (one slab q, one lateral j, i = -2..2):
// a row needs 4 rows of 6 path densities and 4 rows of 6 densities, which it
// reads contiguously and interpolates separably (along the slice or the light
// axis first, then the lateral axes).  Rows whose indices all lie inside the
// field take a path without clamping; the others clamp every index.  Levels
// with at most 8^3 voxels are copied whole into LDS first and read from there.
#include "launch_args.h"
#include "mfma.h"

namespace nis {

constexpr int kTP = 16;                   // points per workgroup
constexpr int kRows = 45;                 // site rows per point and layer
constexpr int kLatStride = 232;           // 225 sites + padding
constexpr int kY1Pos = 64;                // 63 conv1 positions + 1
constexpr int kSmallLevel = 4096;         // floats of a level staged whole in LDS
constexpr int kBufferFlags = 0x00020000;  // buffer resource word 3 for gfx9-family raw loads

struct PointLayer {           // per point and layer
    int iu, iv, ij, ia0;      // sheared base indices (path density) and light-axis base (density)
    float wu, wv, wj, wa;     // their interpolation weights
};

struct SlabParams {           // per point, layer and slab q
    int ib0, ic0, mask, pad;  // density lateral bases; in-cube bits (0-4 i, 5-9 j, 10 slab)
    float wb, wc, pad1, pad2;
};

// Shared memory of one workgroup.  The whole-level copy is only live during
// the gather and the conv1 output only afterwards; the per-row statistics only
// until conv2 writes its output.
template <class E> struct FeatShared {
    E lat[kTP][kLatStride];
    union {
        float small_lvl[kSmallLevel];
        E y1[kTP][kY1Pos][8];                // conv1 output, channels fastest
    } __attribute__((aligned(16))) u1;
    union {
        float part[kTP * kRows][4];
        struct {
            float H[kTP][16][5];
            float zc[kTP][16];
            float hid[kTP][4];
            float gate[kTP][16];
        } se;
    } u2;
    float pstat[kTP][kStats];
    float pfix[kTP][3];
    double px[kTP][3];
    PointLayer pl[kTP];
    SlabParams sp[kTP][9];
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

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return min(max(v, lo), hi); }

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

// index-clamped trilinear lookup in a path-density field D[J][V][U]
__device__ __forceinline__ float sample_D(const float* __restrict__ D, const Level& lv, int U, int V,
                                          int J, float wu, float wv, float wj)
{
    int u0 = clampi(U - lv.ulo, 0, lv.nu - 1), u1 = clampi(U + 1 - lv.ulo, 0, lv.nu - 1);
    int v0 = clampi(V - lv.vlo, 0, lv.nv - 1), v1 = clampi(V + 1 - lv.vlo, 0, lv.nv - 1);
    int j0 = clampi(J, 0, lv.n - 1), j1 = clampi(J + 1, 0, lv.n - 1);
    const int64_t plane = (int64_t)lv.nu * lv.nv;
    const float* d0 = D + j0 * plane;
    const float* d1 = D + j1 * plane;
    float a00 = lerpf(d0[v0 * lv.nu + u0], d0[v0 * lv.nu + u1], wu);
    float a01 = lerpf(d0[v1 * lv.nu + u0], d0[v1 * lv.nu + u1], wu);
    float a10 = lerpf(d1[v0 * lv.nu + u0], d1[v0 * lv.nu + u1], wu);
    float a11 = lerpf(d1[v1 * lv.nu + u0], d1[v1 * lv.nu + u1], wu);
    return lerpf(lerpf(a00, a01, wv), lerpf(a10, a11, wv), wj);
}

// Separable interpolation of one row of 5 sites from 4 rows of 6 samples:
// first between rows (r00,r10) and (r01,r11) with weight w1, then between the
// two results with w2, then along the row with w3.
__device__ __forceinline__ void row5(const float* r00, const float* r10, const float* r01, const float* r11,
                                     float w1, float w2, float w3, float out[5])
{
    float b[6];
#pragma unroll
    for (int u = 0; u < 6; u++) b[u] = lerpf(lerpf(r00[u], r10[u], w1), lerpf(r01[u], r11[u], w1), w2);
#pragma unroll
    for (int i = 0; i < 5; i++) out[i] = lerpf(b[i], b[i + 1], w3);
}

template <class T>
__device__ __forceinline__ void load6(const T* p, float v[6])
{
#pragma unroll
    for (int u = 0; u < 6; u++) v[u] = p[u];
}

template <int PREC, bool DBG>
__global__ void __launch_bounds__(256)
k_features(FeatArgs A)
{
    typedef Mfma<PREC> M;
    typedef typename M::elem E;
    __shared__ FeatShared<E> sh;
    E(*lat)[kLatStride] = sh.lat;
    E(*y1)[kY1Pos][8] = sh.u1.y1;
    float* small_lvl = sh.u1.small_lvl;
    float(*part)[4] = sh.u2.part;
    float(*H)[16][5] = sh.u2.se.H;
    float(*zc)[16] = sh.u2.se.zc;
    float(*hid)[4] = sh.u2.se.hid;
    float(*gate)[16] = sh.u2.se.gate;
    float(*pstat)[kStats] = sh.pstat;
    float(*pfix)[3] = sh.pfix;
    double(*px)[3] = sh.px;
    PointLayer* pl = sh.pl;
    SlabParams(*sp)[9] = sh.sp;

    const MediumView& mv = A.mv;
    const int tid = threadIdx.x;
    const int wave = tid / 64, lane = tid % 64;
    const int lr = lane % 16, lg = lane / 16;
    const int64_t tile0 = (int64_t)blockIdx.x * kTP;
    // the point count may live in device memory (frames whose hit count the
    // device computed); blocks past it leave before any barrier
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    if (tile0 >= npts) return;

    // ---- per point: position, phase features, transmittance to the light ----
    {
        const int pt = tid / 16, sub = tid % 16;
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
        float phs = 0.f, phm = -INFINITY;
        for (int t = sub; t < kSites; t += 16) {
            double P;
            if (t == kSites / 2) {
                P = hg64(mv, wl);
            } else {
                const double* dt = A.tab->dir[t];
                P = hg64(mv, w[0] * dt[0] + w[1] * dt[1] + w[2] * dt[2]) * (double)A.tab->hg_dl[t];
            }
            float ph = log1pf((float)P);
            phs += ph;
            phm = fmaxf(phm, ph);
            if (DBG && live) A.dbg_phi[p * kSites + t] = ph;
        }
        for (int o = 1; o < 16; o <<= 1) {
            phs += __shfl_xor(phs, o);
            phm = fmaxf(phm, __shfl_xor(phm, o));
        }
        if (sub == 0) {
            pfix[pt][0] = phs / kSites;
            pfix[pt][1] = phm;
            pfix[pt][2] = (float)acos(fmin(1.0, fmax(-1.0, wl)));
            for (int d = 0; d < 3; d++) px[pt][d] = x[d];
        }
        if (sub == 1 && live) {
            const Level& l0 = mv.lev[0];
            double Uf, Vf, Jf;
            sheared(mv, l0.n, x, Uf, Vf, Jf);
            double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
            float D0 = sample_D(mv.D + l0.d_off, l0, (int)fu, (int)fv, (int)fj, (float)(Uf - fu),
                                (float)(Vf - fv), (float)(Jf - fj));
            float T = expf(-mv.sigma_t * D0);
            A.f0[p] = (float)(hg64(mv, wl) * (double)T);
            if (DBG) A.dbg_tp[p] = T;
        }
    }

    // conv1 B-fragment lattice offsets of this lane's taps (fixed for all tiles)
    int tapoff[M::KPL * (kConv1K / M::KS)];
#pragma unroll
    for (int kc = 0; kc < kConv1K / M::KS; kc++)
#pragma unroll
        for (int e = 0; e < M::KPL; e++) {
            const int kk = kc * M::KS + lg * M::KPL + e;
            tapoff[kc * M::KPL + e] = kk < 27 ? (kk / 9) * 25 + ((kk / 3) % 3) * 5 + (kk % 3) : -1;
        }
    E* desc = reinterpret_cast<E*>(A.desc);

    float row_absmax = 0.f;   // thread (point, o): max |stored entry| of its point so far
    for (int k = 0; k < kLayers; k++) {
        const int m = k < mv.levels - 1 ? k : mv.levels - 1;
        const Level lv = mv.lev[m];
        const int nm = lv.n;
        const int c = 1 << (k - m);
        const double scale = ldexp(1.0 / mv.n0, k);
        const float coef = A.coef[k];
        const int grp = k < kDiffuse ? 0 : 1;
        const int st[3] = {1, nm, nm * nm};
        const int sta = st[mv.a], stb = st[mv.b], stc = st[mv.c];
        const int plane = lv.nu * lv.nv;
        const int dsize = plane * nm, rsize = nm * nm * nm;
        const bool small = dsize + rsize <= kSmallLevel;
        __syncthreads();   // previous layer's users of the shared tables are done

        // ---- per point-layer and per slab set-up --------------------------------
        if (tid < kTP * 9) {
            const int pt = tid / 9, qi = tid % 9;
            const double x[3] = {px[pt][0], px[pt][1], px[pt][2]};
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
            SlabParams s;
            s.ib0 = (int)fb;
            s.ic0 = (int)fc;
            s.mask = mask;
            s.pad = 0;
            s.wb = (float)(gb - fb);
            s.wc = (float)(gc - fc);
            s.pad1 = s.pad2 = 0.f;
            sp[pt][qi] = s;
        } else if (tid < kTP * 10) {
            const int pt = tid - kTP * 9;
            const double x[3] = {px[pt][0], px[pt][1], px[pt][2]};
            double Uf, Vf, Jf;
            sheared(mv, nm, x, Uf, Vf, Jf);
            const double fu = floor(Uf), fv = floor(Vf), fj = floor(Jf);
            const double ga = x[mv.a] * nm - 0.5;
            const double fa = floor(ga);
            PointLayer q;
            q.iu = (int)fu;
            q.iv = (int)fv;
            q.ij = (int)fj;
            q.ia0 = (int)fa;
            q.wu = (float)(Uf - fu);
            q.wv = (float)(Vf - fv);
            q.wj = (float)(Jf - fj);
            q.wa = (float)(ga - fa);
            pl[pt] = q;
        }
        if (small) {
            const float* srcD = mv.D + lv.d_off;
            const float* srcR = mv.rho + lv.rho_off;
            for (int e = tid; e < dsize; e += 256) small_lvl[e] = srcD[e];
            for (int e = tid; e < rsize; e += 256) small_lvl[dsize + e] = srcR[e];
        }
        __syncthreads();

        // ---- gather: rows of 5 sites ---------------------------------------------
        // One instantiation per source: LDS for whole small levels, raw buffer
        // loads (32-bit offsets, immediate offsets along a row) for the others.
        auto gather = [&](auto ldD, auto ldR) __attribute__((always_inline)) {
        for (int R = tid; R < kTP * kRows; R += 256) {
            const int pt = R / kRows, r = R % kRows;
            const int qi = r / 5, jj = r % 5;
            const int q = qi - 4, j = jj - 2;
            const PointLayer P = pl[pt];
            const SlabParams S = sp[pt][qi];
            float Dv[5], Rv[5];
            // path density rows: J = ij - c q (+1), V = iv + c j (+1), U = iu + c i (+1)
            if (c == 1) {
                const int J0 = P.ij - q, V0 = P.iv + j - lv.vlo, U0 = P.iu - 2 - lv.ulo;
                const bool inside = J0 >= 0 && J0 + 1 < nm && V0 >= 0 && V0 + 1 < lv.nv && U0 >= 0 && U0 + 5 < lv.nu;
                float a0[6], a1[6], b0[6], b1[6];
                if (inside) {
                    const int o = (J0 * lv.nv + V0) * lv.nu + U0;
#pragma unroll
                    for (int u = 0; u < 6; u++) {
                        a0[u] = ldD(o + u);
                        b0[u] = ldD(o + lv.nu + u);
                        a1[u] = ldD(o + plane + u);
                        b1[u] = ldD(o + plane + lv.nu + u);
                    }
                } else {
                    const int j0 = clampi(J0, 0, nm - 1) * plane, j1 = clampi(J0 + 1, 0, nm - 1) * plane;
                    const int v0 = clampi(V0, 0, lv.nv - 1) * lv.nu, v1 = clampi(V0 + 1, 0, lv.nv - 1) * lv.nu;
#pragma unroll
                    for (int u = 0; u < 6; u++) {
                        const int uc = clampi(U0 + u, 0, lv.nu - 1);
                        a0[u] = ldD(j0 + v0 + uc);
                        b0[u] = ldD(j0 + v1 + uc);
                        a1[u] = ldD(j1 + v0 + uc);
                        b1[u] = ldD(j1 + v1 + uc);
                    }
                }
                row5(a0, a1, b0, b1, P.wj, P.wv, P.wu, Dv);
            } else {
                // c > 1 only on the single-voxel level (one slice): sites are c apart
                const int v0 = clampi(P.iv + c * j - lv.vlo, 0, lv.nv - 1) * lv.nu;
                const int v1 = clampi(P.iv + c * j + 1 - lv.vlo, 0, lv.nv - 1) * lv.nu;
#pragma unroll
                for (int i = 0; i < 5; i++) {
                    const int u0 = clampi(P.iu + c * (i - 2) - lv.ulo, 0, lv.nu - 1);
                    const int u1 = clampi(P.iu + c * (i - 2) + 1 - lv.ulo, 0, lv.nu - 1);
                    const float d0 = lerpf(ldD(v0 + u0), ldD(v0 + u1), P.wu);
                    const float d1 = lerpf(ldD(v1 + u0), ldD(v1 + u1), P.wu);
                    const float dd = lerpf(d0, d1, P.wv);
                    Dv[i] = lerpf(dd, dd, P.wj);
                }
            }
            // density rows: a = ia0 + c q sigma (+1), c-axis ic0(q) + c j (+1), b-axis ib0(q) + c i (+1)
            if (nm == 1) {
                const float r0 = ldR(0);
#pragma unroll
                for (int i = 0; i < 5; i++) Rv[i] = r0;
            } else {
                const int A0 = P.ia0 + q * mv.sigma, C0 = S.ic0 + j, B0 = S.ib0 - 2;
                const bool inside = A0 >= 0 && A0 + 1 < nm && C0 >= 0 && C0 + 1 < nm && B0 >= 0 && B0 + 5 < nm &&
                                    stb == 1;
                float a0[6], a1[6], b0[6], b1[6];
                if (inside) {
                    const int o = A0 * sta + C0 * stc + B0;
#pragma unroll
                    for (int u = 0; u < 6; u++) {
                        a0[u] = ldR(o + u);
                        a1[u] = ldR(o + sta + u);
                        b0[u] = ldR(o + stc + u);
                        b1[u] = ldR(o + sta + stc + u);
                    }
                } else {
                    const int x0 = clampi(A0, 0, nm - 1) * sta, x1 = clampi(A0 + 1, 0, nm - 1) * sta;
                    const int z0 = clampi(C0, 0, nm - 1) * stc, z1 = clampi(C0 + 1, 0, nm - 1) * stc;
#pragma unroll
                    for (int u = 0; u < 6; u++) {
                        const int bc = clampi(B0 + u, 0, nm - 1) * stb;
                        a0[u] = ldR(x0 + z0 + bc);
                        a1[u] = ldR(x1 + z0 + bc);
                        b0[u] = ldR(x0 + z1 + bc);
                        b1[u] = ldR(x1 + z1 + bc);
                    }
                }
                row5(a0, a1, b0, b1, P.wa, S.wc, S.wb, Rv);
            }
            float rs = 0.f, rmx = -INFINITY, ts = 0.f, tmx = -INFINITY;
            const int64_t p = tile0 + pt;
#pragma unroll
            for (int i = 0; i < 5; i++) {
                const float T = __expf(-coef * Dv[i]);
                const float rv = ((S.mask >> 10) & (S.mask >> i) & (S.mask >> (jj + 5)) & 1) ? Rv[i] : 0.f;
                lat[pt][r * 5 + i] = M::cvt(T);
                rs += rv;
                rmx = fmaxf(rmx, rv);
                ts += T;
                tmx = fmaxf(tmx, T);
                if (DBG && p < npts) {
                    A.dbg_tbar[(p * kLayers + k) * kSites + r * 5 + i] = T;
                    A.dbg_rho[(p * kLayers + k) * kSites + r * 5 + i] = rv;
                }
            }
            part[R][0] = rs;
            part[R][1] = rmx;
            part[R][2] = ts;
            part[R][3] = tmx;
        }
        };
        if (small) {
            const float* sD = small_lvl;
            const float* sR = small_lvl + dsize;
            gather([&](int o) { return sD[o]; }, [&](int o) { return sR[o]; });
        } else {
            const __amdgpu_buffer_rsrc_t rD =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(mv.D + lv.d_off), 0, dsize * 4, kBufferFlags);
            const __amdgpu_buffer_rsrc_t rR =
                __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(mv.rho + lv.rho_off), 0, rsize * 4, kBufferFlags);
            gather([&](int o) { return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rD, o * 4, 0, 0)); },
                   [&](int o) { return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rR, o * 4, 0, 0)); });
        }
        __syncthreads();

        // ---- per-point statistics (eq. 24) ----------------------------------------
        if (tid < kTP * 4) {
            const int pt = tid / 4, s = tid % 4;
            float v = s & 1 ? -INFINITY : 0.f;
            for (int r = 0; r < kRows; r++) v = s & 1 ? fmaxf(v, part[pt * kRows + r][s]) : v + part[pt * kRows + r][s];
            const int slot = s == 0 ? 0 : s == 1 ? 3 : s == 2 ? 2 : 5;
            pstat[pt][slot] = s & 1 ? v : v / kSites;
        } else if (tid < kTP * 5) {
            const int pt = tid - kTP * 4;
            pstat[pt][1] = pfix[pt][0];
            pstat[pt][4] = pfix[pt][1];
            pstat[pt][6] = mv.g;
            pstat[pt][7] = pfix[pt][2];
        }

        // ---- conv1: out^T [8 ch x 16 positions] = W1 [8 x 27] . im2col [27 x 16]
        {
            const E* w1 = reinterpret_cast<const E*>(A.w1t[grp]);
            const float* b1 = A.cb[grp];
            typename M::frag aw[kConv1K / M::KS];
#pragma unroll
            for (int kc = 0; kc < kConv1K / M::KS; kc++)
                aw[kc] = M::load(w1 + lr * kConv1K + kc * M::KS + lg * M::KPL);
            for (int tile = wave; tile < kTP * 4; tile += 4) {
                const int pt = tile >> 2, pos = (tile & 3) * 16 + lr;
                const int base = pos < 63 ? (pos / 9) * 25 + ((pos / 3) % 3) * 5 + pos % 3 : 0;
                const E* L = lat[pt] + base;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < kConv1K / M::KS; kc++) {
                    auto get = [&](int kk) -> E {
                        const int o = tapoff[kk - lg * M::KPL - kc * M::KS + kc * M::KPL];
                        return o >= 0 ? L[o] : M::zero();
                    };
                    acc = M::mma(aw[kc], M::gather(get, kc * M::KS + lg * M::KPL), acc);
                }
                if (lg < 2 && pos < 63) {
#pragma unroll
                    for (int e = 0; e < 4; e++) y1[pt][pos][lg * 4 + e] = M::cvt(fmaxf(acc[e] + b1[lg * 4 + e], 0.f));
                }
            }
        }
        __syncthreads();

        // ---- conv2: [rows = (point, z)] x [K = 27 taps x 8 channels] x [16 channels]
        {
            const E* w2 = reinterpret_cast<const E*>(A.w2t[grp]);
            const float* b2 = A.cb[grp] + 8;
            for (int tile = wave; tile < kTP * 5 / 16; tile += 4) {
                const int row = tile * 16 + lr;
                const int pt = row / 5, z = row % 5;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kc = 0; kc < kConv2K / M::KS; kc++) {
                    const int k0 = kc * M::KS + lg * M::KPL;     // K index = tap * 8 + channel
                    typename M::frag a;
                    if constexpr (M::KPL == 8) {
                        const int tap = k0 >> 3 < 27 ? k0 >> 3 : 0;
                        const int pos = z * 9 + tap;
                        a = M::load(&y1[pt][pos][0]);
                    } else {
                        const int tap = k0 >> 3 < 27 ? k0 >> 3 : 0;
                        a = y1[pt][z * 9 + tap][k0 & 7];
                    }
                    typename M::frag b = M::load(w2 + lr * kConv2K + k0);
                    acc = M::mma(a, b, acc);
                }
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    int row2 = tile * 16 + lg * 4 + e;
                    H[row2 / 5][lr][row2 % 5] = fmaxf(acc[e] + b2[lr], 0.f);
                }
            }
        }
        __syncthreads();

        // ---- squeeze-excitation gate
        {
            const float* cb = A.cb[grp];
            const float *s1 = cb + 24, *c1 = cb + 88, *s2 = cb + 92, *c2 = cb + 156;
            const int pt = tid / 16, o = tid % 16;
            zc[pt][o] = (H[pt][o][0] + H[pt][o][1] + H[pt][o][2] + H[pt][o][3] + H[pt][o][4]) / 5.f;
            __syncthreads();
            if (o < 4) {
                float s = c1[o];
                for (int i = 0; i < 16; i++) s += s1[o * 16 + i] * zc[pt][i];
                hid[pt][o] = fmaxf(s, 0.f);
            }
            __syncthreads();
            float s = c2[o];
            for (int h = 0; h < 4; h++) s += s2[o * 4 + h] * hid[pt][h];
            gate[pt][o] = 1.f / (1.f + expf(-s));
            // descriptor entries of layer k: 5 features of channel o, and stat o
            const int64_t pp = tile0 + pt;
            float lmax = 0.f;
            E q[6];
#pragma unroll
            for (int z = 0; z < 5; z++) {
                q[z] = M::cvt(gate[pt][o] * H[pt][o][z]);
                lmax = fmaxf(lmax, fabsf((float)q[z]));
            }
            q[5] = M::cvt(o < kStats ? pstat[pt][o] : 0.f);
            lmax = fmaxf(lmax, fabsf((float)q[5]));
            if (pp < npts) {
                E* d = desc + pp * kDescPad + k * kPerLayer;
#pragma unroll
                for (int z = 0; z < 5; z++) d[o * 5 + z] = q[z];
                if (o < kStats) d[kFeat + o] = q[5];
                if (DBG && o < kStats) A.dbg_stats[(pp * kLayers + k) * kStats + o] = pstat[pt][o];
            }
            // running maximum |entry| of the point's stored descriptor (the 16
            // threads of a point are 16 consecutive lanes of one wave)
            for (int s = 1; s < 16; s <<= 1) lmax = fmaxf(lmax, __shfl_xor(lmax, s));
            row_absmax = fmaxf(row_absmax, lmax);
        }
    }
    // albedo entry and zero padding
    for (int e = tid; e < kTP * (kDescPad - kDesc + 1); e += 256) {
        const int pt = e / (kDescPad - kDesc + 1), f = kDesc - 1 + e % (kDescPad - kDesc + 1);
        const int64_t pp = tile0 + pt;
        if (pp < npts) desc[pp * kDescPad + f] = M::cvt(f == kDesc - 1 ? mv.albedo : 0.f);
    }
    if (A.rowmax && tid % 16 == 0 && tile0 + tid / 16 < npts)
        A.rowmax[tile0 + tid / 16] = fmaxf(row_absmax, fabsf((float)M::cvt(mv.albedo)));
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
    if (prec == kPrecBF16 || prec == kPrecFP8)
        hipLaunchKernelGGL(k_desc_to_f32<kPrecBF16>, dim3(blocks), dim3(256), 0, s, src, dst, n);
    else
        hipLaunchKernelGGL(k_desc_to_f32<kPrecFP32>, dim3(blocks), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_features(int prec, const FeatArgs& a, hipStream_t s)
{
    if (a.npts <= 0) return hipSuccess;
    const int blocks = (int)((a.npts + kTP - 1) / kTP);
    const bool dbg = a.dbg_tbar || a.dbg_rho || a.dbg_phi || a.dbg_stats || a.dbg_tp;
    if (dbg && !(a.dbg_tbar && a.dbg_rho && a.dbg_phi && a.dbg_stats && a.dbg_tp))
        return hipErrorInvalidValue;   // the debug variant writes every stage output
    // the FP8 path runs the CNN and stores the descriptor in BF16
    if (prec == kPrecBF16 || prec == kPrecFP8) {
        if (dbg) hipLaunchKernelGGL((k_features<kPrecBF16, true>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_features<kPrecBF16, false>), dim3(blocks), dim3(256), 0, s, a);
    } else {
        if (dbg) hipLaunchKernelGGL((k_features<kPrecFP32, true>), dim3(blocks), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_features<kPrecFP32, false>), dim3(blocks), dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace nis
