// k_mlp.hip -- backbone network and output decode for a tile of points.
//
// Backbone (Sec. III.C.2, Fig. 6, in MLP form): h_1 = ReLU(A_1 x + beta_1),
// h_i = ReLU(A_i h_{i-1} + beta_i) for the hidden layers, y = a_out . h + b.
// Decode (eq. 21 inverted, eq. 19): F = albedo^gamma * expm1(y) and the
// radiance L = I * (HG(w.l) T(p) + F).
//
// Each wave owns ROWS points (64 in BF16, 32 in FP32) and keeps their
// activations in its own LDS slice; every hidden layer is a [ROWS x K] x
// [K x W] MFMA GEMM whose output overwrites the slice in place.  Weights are
// stored pre-arranged in MFMA B-fragment order: for output tile ct and K step
// kc, the 64 lanes' fragments are one contiguous block, so a wave loads each
// fragment with fully used cache lines and every fragment feeds ROWS/16 MFMAs.
// The last layer is a float32 dot product per row, fused with the decode.
#include "launch_args.h"
#include "mfma.h"

namespace nis {

constexpr int kMlpWaves = 4;

template <int PREC> struct MlpShape {
    static constexpr int ROWS = PREC == kPrecFP32 ? 32 : 64;   // rows per wave
};

template <int PREC, int NT>
__global__ void __launch_bounds__(256)
k_mlp(MlpArgs A)
{
    typedef Mfma<PREC> M;
    typedef typename M::elem E;
    constexpr int ROWS = MlpShape<PREC>::ROWS;
    constexpr int RT = ROWS / 16;                           // row tiles per wave
    constexpr int W = NT * 16;
    constexpr int KH = hidden_k(PREC, W);                   // K of the hidden layers (zero padded)
    constexpr int HS = KH + (PREC == kPrecFP32 ? 4 : 8);   // row stride, keeps 16 B alignment
    constexpr int FRAG = 64 * M::KPL;                       // elements of one B-fragment block
    __shared__ __attribute__((aligned(16))) E hbuf[kMlpWaves][ROWS][HS];

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int lr = lane % 16, lg = lane / 16;
    const int64_t row0 = ((int64_t)blockIdx.x * kMlpWaves + wave) * ROWS;
    E(*h)[HS] = hbuf[wave];
    const E* x = reinterpret_cast<const E*>(A.x);

    // activation columns W..KH-1 only ever meet zero weights; keep them finite
    if constexpr (KH > W) {
        for (int e = lane; e < ROWS * (KH - W); e += 64) h[e / (KH - W)][W + e % (KH - W)] = M::zero();
    }
    f32x4 acc[RT][NT];
    for (int li = 0; li + 1 < A.n_linear; li++) {
        const E* Wf = reinterpret_cast<const E*>(A.W[li]) + lane * M::KPL;
        const int K = li == 0 ? kDescPad : KH;
        const int KC = K / M::KS;
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < NT; ct++) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (li == 0) {
            const E* xr[RT];
#pragma unroll
            for (int rt = 0; rt < RT; rt++) {
                int64_t r = row0 + rt * 16 + lr;
                r = r < A.npts ? r : A.npts - 1;
                xr[rt] = x + r * kDescPad + lg * M::KPL;
            }
            for (int kc = 0; kc < KC; kc++) {
                typename M::frag a[RT];
#pragma unroll
                for (int rt = 0; rt < RT; rt++) a[rt] = M::load(xr[rt] + kc * M::KS);
#pragma unroll
                for (int ct = 0; ct < NT; ct++) {
                    typename M::frag b = M::load(Wf + (ct * KC + kc) * FRAG);
#pragma unroll
                    for (int rt = 0; rt < RT; rt++) acc[rt][ct] = M::mma(a[rt], b, acc[rt][ct]);
                }
            }
        } else {
            for (int kc = 0; kc < KC; kc++) {
                typename M::frag a[RT];
#pragma unroll
                for (int rt = 0; rt < RT; rt++) a[rt] = M::load(&h[rt * 16 + lr][kc * M::KS + lg * M::KPL]);
#pragma unroll
                for (int ct = 0; ct < NT; ct++) {
                    typename M::frag b = M::load(Wf + (ct * KC + kc) * FRAG);
#pragma unroll
                    for (int rt = 0; rt < RT; rt++) acc[rt][ct] = M::mma(a[rt], b, acc[rt][ct]);
                }
            }
        }
        __syncthreads();   // every lane's reads of h precede the in-place overwrite
        const float* bias = A.bias[li];
#pragma unroll
        for (int ct = 0; ct < NT; ct++) {
            const float bb = bias[ct * 16 + lr];
#pragma unroll
            for (int rt = 0; rt < RT; rt++)
#pragma unroll
                for (int e = 0; e < 4; e++)
                    h[rt * 16 + lg * 4 + e][ct * 16 + lr] = M::cvt(fmaxf(acc[rt][ct][e] + bb, 0.f));
        }
        __syncthreads();
    }
    // last layer + decode, one row per lane
    for (int rr = lane; rr < ROWS; rr += 64) {
        const int64_t row = row0 + rr;
        float y = A.bout;
        for (int k = 0; k < W; k++) y += (float)h[rr][k] * A.wout[k];
        if (row < A.npts) {
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row] = A.radiance * (A.f0[row] + A.albedo_gamma * expm1f(y));
        }
    }
}

template <int PREC>
static hipError_t launch_mlp_prec(const MlpArgs& a, hipStream_t s)
{
    constexpr int per = kMlpWaves * MlpShape<PREC>::ROWS;
    int blocks = (int)((a.npts + per - 1) / per);
    dim3 g(blocks), b(256);
    switch (a.wpad / 16) {
    case 1: hipLaunchKernelGGL((k_mlp<PREC, 1>), g, b, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_mlp<PREC, 2>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_mlp<PREC, 4>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((k_mlp<PREC, 8>), g, b, 0, s, a); break;
    case 13: hipLaunchKernelGGL((k_mlp<PREC, 13>), g, b, 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_mlp<PREC, 16>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// K of the hidden layers for a padded width: a multiple of the MFMA K step.
int mlp_hidden_k(int prec, int wpad) { return hidden_k(prec, wpad); }

// MFMA K step and elements per lane of a B fragment for a precision.
int mlp_k_step(int prec) { return prec == kPrecFP32 ? Mfma<kPrecFP32>::KS : Mfma<kPrecBF16>::KS; }
int mlp_k_per_lane(int prec) { return prec == kPrecFP32 ? Mfma<kPrecFP32>::KPL : Mfma<kPrecBF16>::KPL; }

// Padded width the kernel is instantiated for: the smallest of
// 16, 32, 64, 128, 208, 256 that holds `width`.
int mlp_padded_width(int width)
{
    static const int sizes[] = {16, 32, 64, 128, 208, 256};
    for (int s : sizes)
        if (width <= s) return s;
    return -1;
}

hipError_t launch_mlp(int prec, const MlpArgs& a, hipStream_t s)
{
    if (a.npts <= 0) return hipSuccess;
    if (prec == kPrecBF16) return launch_mlp_prec<kPrecBF16>(a, s);
    return launch_mlp_prec<kPrecFP32>(a, s);
}

}  // namespace nis
