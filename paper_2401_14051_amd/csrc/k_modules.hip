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
// Work split: one lane per point; every weight is the same for all lanes of
// a wave (scalar loads), so the contractions are per-lane FMA chains with a
// scalar operand.  The layers' sizes are compile-time constants, so the
// per-point state stays in registers.
#include "launch_args.h"
#include "mfma.h"

namespace nis {

template <int V> using ICm = std::integral_constant<int, V>;

template <int I, int N, class F> __device__ __forceinline__ void static_loop(F&& f)
{
    if constexpr (I < N) {
        f(ICm<I>{});
        static_loop<I + 1, N>(f);
    }
}

__device__ __forceinline__ float sigmoidf_(float x) { return 1.f / (1.f + __expf(-x)); }

// offset (in floats) of a layer's block in a feature row: per layer its
// tbar, rho, phi (n each) and squeeze vector (8)
constexpr int feat_base(int k)
{
    int b = 0;
    for (int i = 0; i < k; i++) b += 3 * tpl_count(i) + kStats;
    return b;
}

// floats of one step's weights from layer k
constexpr int step_floats(int k)
{
    return 16 + 2 + 2 * (tpl_count(k) + 2) + (tpl_count(k) + 2) + tpl_count(k + 1) * (tpl_count(k) + 2) +
           tpl_count(k + 1) + tpl_count(k + 1) * tpl_count(k + 1) + tpl_count(k + 1);
}

// floats of a module's steps (group 0: layers 0..7, group 1: 8..11)
constexpr int module_floats(int grp)
{
    int s = 0;
    for (int k = grp ? kDiffuse : 0; k < (grp ? kLayers - 1 : kDiffuse - 1); k++) s += step_floats(k);
    return s;
}

constexpr int kMerge = 64;
constexpr int kCat = 48 + 8;   // last diffuse layer + last highlight layer
constexpr int kModuleFloats = 3 * (module_floats(0) + module_floats(1)) + 3 * (kMerge * kCat + kMerge);

// One module: h (the group's first layer's features of type tau on entry,
// its final state on exit); w points at its first step's weights.
template <int G>
__device__ __forceinline__ void run_module(const float* __restrict__ w, int tau, const float* __restrict__ row,
                                           float g, float alpha, float (&h)[48])
{
    constexpr int k0 = G ? kDiffuse : 0, k1 = G ? kLayers - 1 : kDiffuse - 1;
    static_loop<k0, k1>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;
        constexpr int n = tpl_count(k), a = n + 2, b = tpl_count(k + 1);
        const float* S1 = w;
        const float* e1 = S1 + 16;
        const float* S2 = e1 + 2;
        const float* e2 = S2 + 2 * a;
        const float* F1 = e2 + a;
        const float* f1 = F1 + b * a;
        const float* F2 = f1 + b;
        const float* f2 = F2 + b * b;
        w = f2 + b;
        const float* v = row + feat_base(k) + 3 * n;
        const float* xn = row + feat_base(k + 1) + tau * b;
        float z[2];
#pragma unroll
        for (int r = 0; r < 2; r++) {
            float acc = e1[r];
#pragma unroll
            for (int i = 0; i < 8; i++) acc += S1[r * 8 + i] * v[i];
            z[r] = fmaxf(acc, 0.f);
        }
        float av[a];
#pragma unroll
        for (int i = 0; i < a; i++) {
            const float ui = i < n ? h[i < n ? i : 0] : i == n ? g : alpha;
            av[i] = sigmoidf_(e2[i] + S2[2 * i] * z[0] + S2[2 * i + 1] * z[1]) * ui;
        }
        float x[b], y[b];
#pragma unroll
        for (int o = 0; o < b; o++) {
            x[o] = xn[o];
            float acc = f1[o];
#pragma unroll
            for (int i = 0; i < a; i++) acc += F1[o * a + i] * av[i];
            y[o] = x[o] + acc;
        }
#pragma unroll
        for (int o = 0; o < b; o++) {
            float acc = f2[o];
#pragma unroll
            for (int i = 0; i < b; i++) acc += F2[o * b + i] * y[i];
            h[o] = fmaxf(acc, 0.f) + x[o];
        }
    });
}

template <int PREC, bool F8>
__global__ void __launch_bounds__(256)
k_modules(const float* __restrict__ feat, const float* __restrict__ wm, int64_t npts, const int* count,
          int64_t count_off, void* desc, float desc_inv_scale, float albedo)
{
    typedef typename Mfma<PREC>::elem E;
    const int64_t nv = count ? min(max((int64_t)*count - count_off, (int64_t)0), npts) : npts;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nv) return;
    const float* row = feat + p * kDescPad;
    const float g = row[3 * tpl_count(0) + 6], alpha = row[3 * tpl_count(0) + 7];
    // a descriptor entry in the backbone's precision
    auto put = [&](int e, float x) __attribute__((always_inline)) {
        if constexpr (F8) {
            x = __builtin_amdgcn_fmed3f(x * desc_inv_scale, -448.f, 448.f);
            reinterpret_cast<uint8_t*>(desc)[p * kDescF8 + e] =
                (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xff);
        } else {
            reinterpret_cast<E*>(desc)[p * kDescPad + e] = Mfma<PREC>::cvt(x);
        }
    };
    const float* w = wm;
    const float* wmerge = wm + 3 * (module_floats(0) + module_floats(1));
#pragma unroll 1
    for (int tau = 0; tau < 3; tau++) {
        float cat[kCat];
        {
            float h[48];
#pragma unroll
            for (int j = 0; j < tpl_count(0); j++) h[j] = row[feat_base(0) + tau * tpl_count(0) + j];
            run_module<0>(w, tau, row, g, alpha, h);
            w += module_floats(0);
#pragma unroll
            for (int j = 0; j < 48; j++) cat[j] = h[j];
        }
        {
            float h[48];
#pragma unroll
            for (int j = 0; j < tpl_count(kDiffuse); j++) h[j] = row[feat_base(kDiffuse) + tau * tpl_count(kDiffuse) + j];
            run_module<1>(w, tau, row, g, alpha, h);
            w += module_floats(1);
#pragma unroll
            for (int j = 0; j < 8; j++) cat[48 + j] = h[j];
        }
        // the type's merge of its two groups, written as it is formed
        const float* M = wmerge + tau * (kMerge * kCat + kMerge);
        const float* mb = M + kMerge * kCat;
#pragma unroll 4
        for (int o = 0; o < kMerge; o++) {
            float acc = mb[o];
#pragma unroll
            for (int i = 0; i < kCat; i++) acc += M[o * kCat + i] * cat[i];
            put(tau * kMerge + o, fmaxf(acc, 0.f));
        }
    }
    // then g, alpha, zeros, the albedo entry at 1056 and zero padding
    put(3 * kMerge, g);
    put(3 * kMerge + 1, alpha);
    const int rowlen = F8 ? kDescF8 : kDescPad;
    for (int e = 3 * kMerge + 2; e < rowlen; e++) put(e, e == kDesc - 1 ? albedo : 0.f);
}

int module_floats_total() { return kModuleFloats; }

hipError_t launch_modules(int prec, const float* feat, const float* wm, int64_t npts, const int* count,
                          int64_t count_off, void* desc, float desc_inv_scale, float albedo, hipStream_t s)
{
    if (npts <= 0) return hipSuccess;
    const int64_t blocks = (npts + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 g((int)blocks), b(256);
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
