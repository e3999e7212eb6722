// k_modules.hip -- the paper's backbone modules (Sec. III.C.2, Fig. 6) over
// the features sampled at the paper's templates.
//
// Six identical modules, one per feature type (graded transmittance,
// density, phase) and template group (diffuse layers 0-7, highlight layers
// 8-11), carry the features of their current layer h through the group's
// layers.  A step from layer k to k+1:
//   u  = [h; g; alpha]                       fusion with the configuration parameters
//   z  = ReLU(S1 v_k + e1)                   squeeze (v_k: eq. 24) and excitation (eq. 25)
//   a  = sigmoid(S2 z + e2) * u              attention gate (eq. 26)
//   y  = x_{k+1} + F1 a + f1                 FC-1 to the next layer's size, fused with its features
//   h  = ReLU(F2 y + f2) + x_{k+1}           FC-2, fused with them again
// Per type, the two groups' final states merge through a full connection,
// m = ReLU(M [h_diffuse; h_highlight] + mb), and the descriptor the backbone
// MLP reads is [m_T; m_rho; m_phi; g; alpha], zeros, albedo at index 1056.
//
// Work split: a wave takes 32 points and runs every contraction as a chain
// of 32x32x2 FP32 MFMAs with the points as the N dimension (lane l holds
// point l % 32).  A vector of R rows per point lives in the accumulator
// layout: tile t (32 rows), register r, lane half hh = l / 32 hold row
// 32 t + 8 (r / 4) + 4 hh + r % 4.  One register of that layout is exactly a
// B operand (its two K entries are the rows of the two lane halves), so a
// layer's output feeds the next contraction without any data movement: the
// host packs each weight matrix's columns in that order.  The attention's
// excitation is one more MFMA pair per input tile whose B operand is
// (z_0 | z_1) and (1 | 0) and whose A holds S2 and e2, which yields the gate
// logits in the same layout.  Only the registers holding a row below R take
// part in the K loop; the rest are zero.
//
// A workgroup of 8 waves (256 points, two waves per SIMD) copies one feature
// type's packed weights (108 KiB) into LDS at a time and reads every A
// fragment from there, one 4-byte word per lane.  Each step issues its reads
// of the next layer's features and squeeze vector before its MFMAs, and the
// feature rows are laid out by type (mf_block), so that a module reads one
// contiguous third of its points' rows with 16-byte loads.  The kernel fits
// 256 registers, so the second wave of a SIMD covers the first one's
// dependency stalls (gate, FC-1, FC-2 each wait for the previous result);
// two groups of 32 points per wave (sharing each A fragment) measured the
// same at one wave per SIMD, and three waves per SIMD spill.
#include "launch_args.h"
#include "mfma.h"

namespace nis {

typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int V> using ICm = std::integral_constant<int, V>;

template <int I, int N, class F> __device__ __forceinline__ void static_loop(F&& f)
{
    if constexpr (I < N) {
        f(ICm<I>{});
        static_loop<I + 1, N>(f);
    }
}

constexpr int kMerge = 64;                 // width of a type's merge
constexpr int kCat = 48 + 8;               // last diffuse layer + last highlight layer
constexpr int kNT = 1;                     // groups of 32 points per wave (the MFMAs' N tiles)
constexpr int kModPts = 32 * kNT;          // points per wave
constexpr int kModWaves = 8;

// ---- layout of a per-point vector over the accumulator registers -----------

__host__ __device__ constexpr int mtiles(int rows) { return (rows + 31) / 32; }
__host__ __device__ constexpr int mrow(int t, int r, int hh) { return 32 * t + 8 * (r / 4) + 4 * hh + r % 4; }
// registers of tile t holding some row below `rows` (a prefix: rows grow with r)
__host__ __device__ constexpr int muse(int t, int rows)
{
    int c = 0;
    for (int r = 0; r < 16; r++) c += mrow(t, r, 0) < rows ? 1 : 0;
    return c;
}
// K steps of a contraction over a vector of `rows` rows
__host__ __device__ constexpr int mksteps(int rows)
{
    int c = 0;
    for (int t = 0; t < mtiles(rows); t++) c += muse(t, rows);
    return c;
}

// ---- packed weights ----------------------------------------------------------
// Per step: S1 (16) and e1 (2), padded to 32 floats; per input tile the two
// gate fragments (S2 columns, e2); f1 as [out tile][hh][16]; F1's fragments
// [out tile][K step][64 lanes]; f2; F2's fragments.  Per type after its two
// modules: mb as [tile][hh][16], then M's fragments [tile][K step][64].
constexpr int kHdr = 32;

__host__ __device__ constexpr int pk_step_floats(int k)
{
    const int a = tpl_count(k) + 2, b = tpl_count(k + 1), tb = mtiles(b);
    return kHdr + mtiles(a) * 128 + tb * 32 + tb * mksteps(a) * 64 + tb * 32 + tb * mksteps(b) * 64;
}
constexpr int kMergeK = mksteps(48) + mksteps(8);
__host__ __device__ constexpr int pk_merge_floats() { return 2 * 32 + 2 * kMergeK * 64; }
__host__ __device__ constexpr int pk_type_floats()
{
    int s = pk_merge_floats();
    for (int k = 0; k < kLayers - 1; k++)
        if (k != kDiffuse - 1) s += pk_step_floats(k);
    return s;
}

// floats of one step's weights in the weight blob (from layer k)
constexpr int raw_step_floats(int k)
{
    const int n = tpl_count(k), a = n + 2, b = tpl_count(k + 1);
    return 16 + 2 + 2 * a + a + b * a + b + b * b + b;
}
constexpr int raw_total()
{
    int s = 0;
    for (int k = 0; k < kLayers - 1; k++)
        if (k != kDiffuse - 1) s += raw_step_floats(k);
    return 3 * s + 3 * (kMerge * kCat + kMerge);
}

__device__ __forceinline__ f32x16 mma(float a, float b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigmoidf_(float x) { return __builtin_amdgcn_rcpf(1.f + __expf(-x)); }

// One step from layer K for the wave's kNT groups of 32 points: h (tiles of
// n_K rows) -> h (tiles of n_{K+1} rows).  row[tn]: the lane's point's
// feature row in group tn; wp: the step's packed weights.  Every A fragment
// read from LDS feeds one MFMA per group.
template <int K>
__device__ __forceinline__ void mod_step(const float* __restrict__& wp, const float* const (&row)[kNT], int tau,
                                         const float (&g)[kNT], const float (&alpha)[kNT], int lane,
                                         f32x16 (&h)[2][kNT], float4 (&vsq)[kNT][2])
{
    constexpr int n = tpl_count(K), a = n + 2, b = tpl_count(K + 1);
    constexpr int TA = mtiles(a), TB = mtiles(b);
    const int hh = lane >> 5;
    // the step's reads from memory first, so that their latency passes under
    // the MFMAs: the next layer's features of this type and its squeeze
    // vector (the next step's)
    float4 xq[TB][4][kNT], vn[kNT][2];
#pragma unroll
    for (int tn = 0; tn < kNT; tn++) {
        const float* xr = row[tn] + mf_block(0, K + 1) + tau * mf_type_len();
#pragma unroll
        for (int mt = 0; mt < TB; mt++)
#pragma unroll
            for (int q = 0; q < 4; q++)   // rows 32 mt + 8 q + 4 hh .. + 3 (in the row: always readable)
                xq[mt][q][tn] = *reinterpret_cast<const float4*>(xr + 32 * mt + 8 * q + 4 * hh);
        vn[tn][0] = *reinterpret_cast<const float4*>(row[tn] + mf_stats(K + 1));
        vn[tn][1] = *reinterpret_cast<const float4*>(row[tn] + mf_stats(K + 1) + 4);
    }
    // u = [h; g; alpha] (rows n and n + 1, zero so far, take g and alpha),
    // gated by the excitation of the layer's squeeze vector (eq. 25, 26):
    // logits S2 z + e2 in the same layout, then a = sigmoid * u
    f32x16 u[TA][kNT];
#pragma unroll
    for (int tn = 0; tn < kNT; tn++) {
        const float v[8] = {vsq[tn][0].x, vsq[tn][0].y, vsq[tn][0].z, vsq[tn][0].w,
                            vsq[tn][1].x, vsq[tn][1].y, vsq[tn][1].z, vsq[tn][1].w};
        float z0 = wp[16], z1 = wp[17];
#pragma unroll
        for (int i = 0; i < 8; i++) {
            z0 += wp[i] * v[i];
            z1 += wp[8 + i] * v[i];
        }
        z0 = fmaxf(z0, 0.f);
        z1 = fmaxf(z1, 0.f);
#pragma unroll
        for (int t = 0; t < TA; t++) u[t][tn] = t < mtiles(n) ? h[t < 2 ? t : 0][tn] : f32x16{};
        constexpr int tg = n / 32, rg = 4 * ((n % 32) / 8) + n % 4, hg = (n % 8) / 4;
        constexpr int ta = (n + 1) / 32, ra = 4 * (((n + 1) % 32) / 8) + (n + 1) % 4, ha = ((n + 1) % 8) / 4;
        if (hh == hg) u[tg][tn][rg] = g[tn];
        if (hh == ha) u[ta][tn][ra] = alpha[tn];
        const float bz0 = hh ? z1 : z0, bz1 = hh ? 0.f : 1.f;
#pragma unroll
        for (int t = 0; t < TA; t++) {
            f32x16 gl = mma(wp[kHdr + t * 128 + lane], bz0, f32x16{});
            gl = mma(wp[kHdr + t * 128 + 64 + lane], bz1, gl);
#pragma unroll
            for (int r = 0; r < muse(t, a); r++) u[t][tn][r] *= sigmoidf_(gl[r]);
        }
    }
    wp += kHdr + TA * 128;
    // FC-1, fused with the next layer's features: y = x + (F1 a + f1)
    f32x16 x[TB][kNT], y[TB][kNT];
#pragma unroll
    for (int mt = 0; mt < TB; mt++) {
        const float* b1 = wp + mt * 32 + hh * 16;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float bv = b1[r];
#pragma unroll
            for (int tn = 0; tn < kNT; tn++) y[mt][tn][r] = bv;
        }
    }
    wp += TB * 32;
#pragma unroll
    for (int mt = 0; mt < TB; mt++) {
        int s = 0;
#pragma unroll
        for (int t = 0; t < TA; t++)
#pragma unroll
            for (int r = 0; r < muse(t, a); r++, s++) {
                const float w = wp[(mt * mksteps(a) + s) * 64 + lane];
#pragma unroll
                for (int tn = 0; tn < kNT; tn++) y[mt][tn] = mma(w, u[t][tn][r], y[mt][tn]);
            }
    }
    wp += TB * mksteps(a) * 64;
#pragma unroll
    for (int mt = 0; mt < TB; mt++)
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
            for (int tn = 0; tn < kNT; tn++) {
                const int r0 = 32 * mt + 8 * q + 4 * hh;
                const float e[4] = {xq[mt][q][tn].x, xq[mt][q][tn].y, xq[mt][q][tn].z, xq[mt][q][tn].w};
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    x[mt][tn][4 * q + i] = r0 + i < b ? e[i] : 0.f;
                    y[mt][tn][4 * q + i] = x[mt][tn][4 * q + i] + y[mt][tn][4 * q + i];
                }
            }
#pragma unroll
    for (int tn = 0; tn < kNT; tn++) {
        vsq[tn][0] = vn[tn][0];
        vsq[tn][1] = vn[tn][1];
    }
    // FC-2, fused again: h = ReLU(F2 y + f2) + x
    f32x16 acc[TB][kNT];
#pragma unroll
    for (int mt = 0; mt < TB; mt++) {
        const float* b2 = wp + mt * 32 + hh * 16;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float bv = b2[r];
#pragma unroll
            for (int tn = 0; tn < kNT; tn++) acc[mt][tn][r] = bv;
        }
    }
    wp += TB * 32;
#pragma unroll
    for (int mt = 0; mt < TB; mt++) {
        int s = 0;
#pragma unroll
        for (int t = 0; t < TB; t++)
#pragma unroll
            for (int r = 0; r < muse(t, b); r++, s++) {
                const float w = wp[(mt * mksteps(b) + s) * 64 + lane];
#pragma unroll
                for (int tn = 0; tn < kNT; tn++) acc[mt][tn] = mma(w, y[t][tn][r], acc[mt][tn]);
            }
    }
    wp += TB * mksteps(b) * 64;
#pragma unroll
    for (int mt = 0; mt < 2; mt++)
#pragma unroll
        for (int tn = 0; tn < kNT; tn++) {
            if (mt < TB) {
#pragma unroll
                for (int r = 0; r < 16; r++)
                    h[mt][tn][r] = fmaxf(acc[mt < TB ? mt : 0][tn][r], 0.f) + x[mt < TB ? mt : 0][tn][r];
            } else {
                h[mt][tn] = f32x16{};
            }
        }
}

// A module of group G over its layers: h enters as the group's first layer's
// features of type tau and leaves as its final state.
template <int G>
__device__ __forceinline__ void run_module(const float* __restrict__& wp, const float* const (&row)[kNT], int tau,
                                           const float (&g)[kNT], const float (&alpha)[kNT], int lane,
                                           f32x16 (&h)[2][kNT])
{
    constexpr int k0 = G ? kDiffuse : 0, k1 = G ? kLayers - 1 : kDiffuse - 1;
    constexpr int n0 = tpl_count(k0);
    const int hh = lane >> 5;
#pragma unroll
    for (int tn = 0; tn < kNT; tn++) {
        const float* x0 = row[tn] + mf_block(0, k0) + tau * mf_type_len();
        h[0][tn] = f32x16{};
        h[1][tn] = f32x16{};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int r0 = 8 * q + 4 * hh;
            const float4 x4 = *reinterpret_cast<const float4*>(x0 + r0);
            const float e[4] = {x4.x, x4.y, x4.z, x4.w};
#pragma unroll
            for (int i = 0; i < 4; i++) h[0][tn][4 * q + i] = r0 + i < n0 ? e[i] : 0.f;
        }
    }
    float4 vsq[kNT][2];   // the current layer's squeeze vector
#pragma unroll
    for (int tn = 0; tn < kNT; tn++) {
        vsq[tn][0] = *reinterpret_cast<const float4*>(row[tn] + mf_stats(k0));
        vsq[tn][1] = *reinterpret_cast<const float4*>(row[tn] + mf_stats(k0) + 4);
    }
    static_loop<k0, k1>([&](auto kc) __attribute__((always_inline)) {
        mod_step<decltype(kc)::value>(wp, row, tau, g, alpha, lane, h, vsq);
    });
}

template <int PREC, bool F8>
__global__ void __launch_bounds__(64 * kModWaves)
k_modules(const float* __restrict__ feat, const float* __restrict__ wm, int64_t npts, const int* count,
          int64_t count_off, void* desc, float desc_inv_scale, float albedo)
{
    typedef typename Mfma<PREC>::elem E;
    __shared__ __attribute__((aligned(16))) float wl[pk_type_floats()];
    const int64_t nv = count ? min(max((int64_t)*count - count_off, (int64_t)0), npts) : npts;
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, hh = lane >> 5;
    // the whole workgroup leaves together (it shares barriers); a wave past
    // the last point computes on that point and writes nothing
    if ((int64_t)blockIdx.x * kModWaves * kModPts >= nv) return;
    const int64_t p0 = ((int64_t)blockIdx.x * kModWaves + wave) * kModPts;
    int64_t p[kNT];
    bool live[kNT];
    const float* row[kNT];
    float g[kNT], alpha[kNT];
#pragma unroll
    for (int tn = 0; tn < kNT; tn++) {
        p[tn] = p0 + 32 * tn + (lane & 31);
        live[tn] = p[tn] < nv;
        row[tn] = feat + (live[tn] ? p[tn] : nv - 1) * kDescPad;
        g[tn] = row[tn][mf_stats(0) + 6];
        alpha[tn] = row[tn][mf_stats(0) + 7];
    }
    const int rowlen = F8 ? kDescF8 : kDescPad;
    // four consecutive entries e .. e + 3 of descriptor row pp
    auto put4 = [&](int64_t pp, int e, const float (&v)[4]) __attribute__((always_inline)) {
        if constexpr (F8) {
            const float s = desc_inv_scale;
            auto q = [&](float x) { return __builtin_amdgcn_fmed3f(x * s, -448.f, 448.f); };
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(q(v[0]), q(v[1]), 0, false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(q(v[2]), q(v[3]), w, true);
            *reinterpret_cast<int*>(reinterpret_cast<uint8_t*>(desc) + pp * kDescF8 + e) = w;
        } else if constexpr (PREC == kPrecBF16) {
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
            const uint32_t a = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{v[0], v[1]}, bf16x2v));
            const uint32_t c = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{v[2], v[3]}, bf16x2v));
            *reinterpret_cast<uint2*>(reinterpret_cast<E*>(desc) + pp * kDescPad + e) = make_uint2(a, c);
        } else {
            *reinterpret_cast<float4*>(reinterpret_cast<float*>(desc) + pp * kDescPad + e) =
                make_float4(v[0], v[1], v[2], v[3]);
        }
    };
#pragma unroll 1
    for (int tau = 0; tau < 3; tau++) {
        // this type's weights into LDS
        __syncthreads();
        {
            const float4* src = reinterpret_cast<const float4*>(wm + (size_t)tau * pk_type_floats());
            float4* dst = reinterpret_cast<float4*>(wl);
            constexpr int n4 = pk_type_floats() / 4;
#pragma unroll 9
            for (int e = threadIdx.x; e < n4; e += 64 * kModWaves) dst[e] = src[e];
        }
        __syncthreads();
        const float* wp = wl;
        f32x16 hd[2][kNT], hl[2][kNT];
        run_module<0>(wp, row, tau, g, alpha, lane, hd);
        run_module<1>(wp, row, tau, g, alpha, lane, hl);
        // the type's merge of its two groups
        f32x16 acc[2][kNT];
#pragma unroll
        for (int mt = 0; mt < 2; mt++) {
            const float* bm = wp + mt * 32 + hh * 16;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const float bv = bm[r];
#pragma unroll
                for (int tn = 0; tn < kNT; tn++) acc[mt][tn][r] = bv;
            }
        }
        wp += 64;
#pragma unroll
        for (int mt = 0; mt < 2; mt++) {
            int s = 0;
#pragma unroll
            for (int t = 0; t < 2; t++)
#pragma unroll
                for (int r = 0; r < muse(t, 48); r++, s++) {
                    const float w = wp[(mt * kMergeK + s) * 64 + lane];
#pragma unroll
                    for (int tn = 0; tn < kNT; tn++) acc[mt][tn] = mma(w, hd[t][tn][r], acc[mt][tn]);
                }
#pragma unroll
            for (int r = 0; r < muse(0, 8); r++, s++) {
                const float w = wp[(mt * kMergeK + s) * 64 + lane];
#pragma unroll
                for (int tn = 0; tn < kNT; tn++) acc[mt][tn] = mma(w, hl[0][tn][r], acc[mt][tn]);
            }
        }
#pragma unroll
        for (int tn = 0; tn < kNT; tn++)
            if (live[tn]) {
#pragma unroll
                for (int mt = 0; mt < 2; mt++)
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const float v[4] = {fmaxf(acc[mt][tn][4 * q], 0.f), fmaxf(acc[mt][tn][4 * q + 1], 0.f),
                                            fmaxf(acc[mt][tn][4 * q + 2], 0.f), fmaxf(acc[mt][tn][4 * q + 3], 0.f)};
                        put4(p[tn], tau * kMerge + mrow(mt, 4 * q, hh), v);
                    }
            }
    }
    // then g, alpha, zeros up to the albedo entry at 1056, and zero padding:
    // the wave writes the tails of its points one row after another, four
    // entries per lane
    const int64_t pend = max(min(p0 + kModPts, nv), p0);
    for (int64_t pp = p0; pp < pend; pp++) {
        const int src = (int)((pp - p0) & 31), grp = (int)((pp - p0) >> 5);
        float gp = __shfl(g[0], src), ap = __shfl(alpha[0], src);
#pragma unroll
        for (int tn = 1; tn < kNT; tn++) {
            const float gt = __shfl(g[tn], src), at = __shfl(alpha[tn], src);
            gp = grp == tn ? gt : gp;
            ap = grp == tn ? at : ap;
        }
        for (int e = 3 * kMerge + 4 * lane; e < rowlen; e += 256) {
            float v[4];
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const int ei = e + i;
                v[i] = ei == 3 * kMerge ? gp : ei == 3 * kMerge + 1 ? ap : ei == kDesc - 1 ? albedo : 0.f;
            }
            put4(pp, e, v);
        }
    }
}

static_assert(raw_total() == 56706, "module block size (documented at nis_set_weights)");

int module_floats_total() { return raw_total(); }
int module_packed_floats() { return 3 * pk_type_floats(); }

// The blob's module block (its own order) -> the kernel's packed layout.
void pack_modules(const float* raw, float* out)
{
    int step_off[3][kLayers] = {}, merge_off[3] = {};
    int o = 0;
    for (int tau = 0; tau < 3; tau++)
        for (int k = 0; k < kLayers - 1; k++)
            if (k != kDiffuse - 1) {
                step_off[tau][k] = o;
                o += raw_step_floats(k);
            }
    for (int tau = 0; tau < 3; tau++) merge_off[tau] = o + tau * (kMerge * kCat + kMerge);
    float* w = out;
    for (int tau = 0; tau < 3; tau++) {
        for (int k = 0; k < kLayers - 1; k++) {
            if (k == kDiffuse - 1) continue;
            const int n = tpl_count(k), a = n + 2, b = tpl_count(k + 1), ta = mtiles(a), tb = mtiles(b);
            const float* S1 = raw + step_off[tau][k];
            const float* e1 = S1 + 16;
            const float* S2 = e1 + 2;
            const float* e2 = S2 + 2 * a;
            const float* F1 = e2 + a;
            const float* f1 = F1 + b * a;
            const float* F2 = f1 + b;
            const float* f2 = F2 + b * b;
            for (int i = 0; i < kHdr; i++) w[i] = i < 16 ? S1[i] : i < 18 ? e1[i - 16] : 0.f;
            w += kHdr;
            for (int t = 0; t < ta; t++) {
                for (int l = 0; l < 64; l++) {
                    const int rr = 32 * t + l % 32, hh = l / 32;
                    w[l] = rr < a ? S2[rr * 2 + hh] : 0.f;
                    w[64 + l] = rr < a && hh == 0 ? e2[rr] : 0.f;
                }
                w += 128;
            }
            auto bias = [&](const float* f) {
                for (int mt = 0; mt < tb; mt++)
                    for (int hh = 0; hh < 2; hh++)
                        for (int r = 0; r < 16; r++) {
                            const int rr = mrow(mt, r, hh);
                            w[(mt * 2 + hh) * 16 + r] = rr < b ? f[rr] : 0.f;
                        }
                w += tb * 32;
            };
            // fragments of W (b rows, `cols` columns) over a K vector of `cols` rows
            auto frags = [&](const float* W, int cols) {
                for (int mt = 0; mt < tb; mt++) {
                    int s = 0;
                    for (int t = 0; t < mtiles(cols); t++)
                        for (int r = 0; r < muse(t, cols); r++, s++)
                            for (int l = 0; l < 64; l++) {
                                const int orow = 32 * mt + l % 32, c = mrow(t, r, l / 32);
                                w[(mt * mksteps(cols) + s) * 64 + l] = orow < b && c < cols ? W[orow * cols + c] : 0.f;
                            }
                }
                w += tb * mksteps(cols) * 64;
            };
            bias(f1);
            frags(F1, a);
            bias(f2);
            frags(F2, b);
        }
        const float* M = raw + merge_off[tau];
        const float* mb = M + kMerge * kCat;
        for (int mt = 0; mt < 2; mt++)
            for (int hh = 0; hh < 2; hh++)
                for (int r = 0; r < 16; r++) w[(mt * 2 + hh) * 16 + r] = mb[mrow(mt, r, hh)];
        w += 64;
        for (int mt = 0; mt < 2; mt++) {
            int s = 0;
            for (int t = 0; t < 2; t++)
                for (int r = 0; r < muse(t, 48); r++, s++)
                    for (int l = 0; l < 64; l++) {
                        const int c = mrow(t, r, l / 32);
                        w[(mt * kMergeK + s) * 64 + l] = c < 48 ? M[(32 * mt + l % 32) * kCat + c] : 0.f;
                    }
            for (int r = 0; r < muse(0, 8); r++, s++)
                for (int l = 0; l < 64; l++) {
                    const int c = mrow(0, r, l / 32);
                    w[(mt * kMergeK + s) * 64 + l] = c < 8 ? M[(32 * mt + l % 32) * kCat + 48 + c] : 0.f;
                }
        }
        w += 2 * kMergeK * 64;
    }
}

hipError_t launch_modules(int prec, const float* feat, const float* wm, int64_t npts, const int* count,
                          int64_t count_off, void* desc, float desc_inv_scale, float albedo, hipStream_t s)
{
    if (npts <= 0) return hipSuccess;
    const int64_t per = (int64_t)kModWaves * kModPts;
    const int64_t blocks = (npts + per - 1) / per;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((int)blocks), b(64 * kModWaves);
    if (prec == kPrecFP8)
        hipLaunchKernelGGL((k_modules<kPrecBF16, true>), g, b, 0, s, feat, wm, npts, count, count_off, desc,
                           desc_inv_scale, albedo);
    else if (prec == kPrecBF16)
        hipLaunchKernelGGL((k_modules<kPrecBF16, false>), g, b, 0, s, feat, wm, npts, count, count_off, desc,
                           desc_inv_scale, albedo);
    else
        hipLaunchKernelGGL((k_modules<kPrecFP32, false>), g, b, 0, s, feat, wm, npts, count, count_off, desc,
                           desc_inv_scale, albedo);
    return hipGetLastError();
}

}  // namespace nis
