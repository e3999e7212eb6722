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
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    if ((int64_t)blockIdx.x * kMlpWaves * ROWS >= npts) return;
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
                r = r < npts ? r : npts - 1;
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
        if (row < npts) {
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row] = A.radiance * (A.f0[row] + A.albedo_gamma * expm1f(y));
        }
    }
}

// FP8 backbone.  Every GEMM is E4M3 x E4M3 -> FP32 on MFMA with two scales:
// one per output column of the weights (absmax / 448, fixed at set_weights)
// and one per row of the activations (absmax / 448 of that point's layer
// input, computed here), so a point's result never depends on the others in
// its batch.  The descriptor arrives in BF16 with its row maxima and is
// quantised while it is loaded; hidden activations are stored in LDS as E4M3.
template <int NT>
__global__ void __launch_bounds__(256)
k_mlp_fp8(MlpArgs A)
{
    typedef Mfma<kPrecFP8> M;
    constexpr int ROWS = 64, RT = 4;
    constexpr int W = NT * 16;
    constexpr int KH = hidden_k(kPrecFP8, W);
    constexpr int K0 = input_k(kPrecFP8);
    constexpr int HS = KH + 16;                  // bytes per activation row
    constexpr int FRAG = 64 * M::KPL;
    // scaling to 447.5 keeps every rounded code finite (the conversion does not saturate)
    constexpr float kTarget = 447.5f;
    __shared__ __attribute__((aligned(16))) uint8_t hbuf[kMlpWaves][ROWS][HS];
    __shared__ float rsc[kMlpWaves][ROWS];      // dequantisation scale of each row's activations

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int lr = lane % 16, lg = lane / 16;
    const int64_t row0 = ((int64_t)blockIdx.x * kMlpWaves + wave) * ROWS;
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    if ((int64_t)blockIdx.x * kMlpWaves * ROWS >= npts) return;
    uint8_t(*h)[HS] = hbuf[wave];
    float* rs = rsc[wave];
    const __bf16* x = reinterpret_cast<const __bf16*>(A.x);

    if constexpr (KH > W) {
        for (int e = lane; e < ROWS * (KH - W); e += 64) h[e / (KH - W)][W + e % (KH - W)] = 0;
    }
    // row scales of the descriptor
    float qs[RT];
    const __bf16* xr[RT];
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
        int64_t r = row0 + rt * 16 + lr;
        r = r < npts ? r : npts - 1;
        xr[rt] = x + r * kDescPad + lg * M::KPL;
        const float m = A.rowmax[r];
        qs[rt] = m > 0.f ? kTarget / m : 1.f;
        if (lg == 0) rs[rt * 16 + lr] = m > 0.f ? m / kTarget : 1.f;
    }
    __syncthreads();

    f32x4 acc[RT][NT];
    for (int li = 0; li + 1 < A.n_linear; li++) {
        const uint8_t* Wf = reinterpret_cast<const uint8_t*>(A.W[li]) + lane * M::KPL;
        const int K = li == 0 ? K0 : KH;
        const int KC = K / M::KS;
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < NT; ct++) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < KC; kc++) {
            typename M::frag a[RT];
            if (li == 0) {
                const bool valid = kc * M::KS + lg * M::KPL < kDescPad;
#pragma unroll
                for (int rt = 0; rt < RT; rt++) {
                    if (valid) {
                        const bf16x8* src = reinterpret_cast<const bf16x8*>(xr[rt] + kc * M::KS);
#pragma unroll
                        for (int v = 0; v < 4; v++) {
                            const bf16x8 u = src[v];
                            a[rt][2 * v] = pack_fp8x4_inrange((float)u[0] * qs[rt], (float)u[1] * qs[rt],
                                                              (float)u[2] * qs[rt], (float)u[3] * qs[rt]);
                            a[rt][2 * v + 1] = pack_fp8x4_inrange((float)u[4] * qs[rt], (float)u[5] * qs[rt],
                                                                  (float)u[6] * qs[rt], (float)u[7] * qs[rt]);
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < 8; v++) a[rt][v] = 0;
                    }
                }
            } else {
#pragma unroll
                for (int rt = 0; rt < RT; rt++) a[rt] = M::load(&h[rt * 16 + lr][kc * M::KS + lg * M::KPL]);
            }
#pragma unroll
            for (int ct = 0; ct < NT; ct++) {
                typename M::frag b = M::load(Wf + (ct * KC + kc) * FRAG);
#pragma unroll
                for (int rt = 0; rt < RT; rt++) acc[rt][ct] = M::mma(a[rt], b, acc[rt][ct]);
            }
        }
        __syncthreads();   // every lane's reads of h and rs precede their overwrite
        const float* bias = A.bias[li];
        const float* wsc = A.wscale[li];
#pragma unroll
        for (int rt = 0; rt < RT; rt++) {
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = rt * 16 + lg * 4 + e;
                const float din = rs[row];
                float m = 0.f;
#pragma unroll
                for (int ct = 0; ct < NT; ct++) {
                    const int col = ct * 16 + lr;
                    const float v = fmaxf(acc[rt][ct][e] * din * wsc[col] + bias[col], 0.f);
                    acc[rt][ct][e] = v;
                    m = fmaxf(m, v);
                }
                for (int o = 1; o < 16; o <<= 1) m = fmaxf(m, __shfl_xor(m, o));
                const float q = m > 0.f ? kTarget / m : 1.f;
#pragma unroll
                for (int ct = 0; ct < NT; ct++) {
                    const int w = __builtin_amdgcn_cvt_pk_fp8_f32(acc[rt][ct][e] * q, 0.f, 0, false);
                    h[row][ct * 16 + lr] = (uint8_t)(w & 0xff);
                }
                // the row's 16 lanes read rs[row] above, in this wave, before this write
                if (lr == 0) rs[row] = m > 0.f ? m / kTarget : 1.f;
            }
        }
        __syncthreads();
    }
    // last layer + decode, one row per lane
    for (int rr = lane; rr < ROWS; rr += 64) {
        const int64_t row = row0 + rr;
        float y = 0.f;
        for (int k = 0; k < W; k++) y += __builtin_amdgcn_cvt_f32_fp8((int)h[rr][k], 0) * A.wout[k];
        y = A.bout + y * rs[rr];
        if (row < npts) {
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row] = A.radiance * (A.f0[row] + A.albedo_gamma * expm1f(y));
        }
    }
}

// BF16 backbone with the weights as the MFMA A operand and the activations as
// B.  A layer's output tile D[channel][point] leaves each lane holding 4
// consecutive channels of one point, which after bias and ReLU are exactly the
// lane's B fragment of the next layer once that layer's K index is permuted
// to match: K slot s = kc*32 + g*8 + e (lane group g) is channel
// (2 kc + e/4) * 16 + g * 4 + e % 4 (the weights are packed in that order).
// So activations stay in registers from layer to layer.  A workgroup of 4
// waves covers 256 points (4 tiles of 16 per wave); for every K step the
// group stages the step's NT weight fragments (NT KiB) in LDS once, double
// buffered, and all four waves read them there.  P point tiles of 16 per
// wave (fewer for wide layers, whose accumulators and inputs must fit in the
// register file).
template <int NT, int P>
__global__ void __launch_bounds__(256)
k_mlp_bf16(MlpArgs A)
{
    typedef Mfma<kPrecBF16> M;
    constexpr int KCH = hidden_k(kPrecBF16, NT * 16) / 32;
    constexpr int KC0 = kDescPad / 32;
    constexpr int BLK = NT * 64 * 8;           // bf16 elements of one K step's fragments
    constexpr int CH = BLK / 8;                // their 16-byte chunks
    constexpr int SJ = (CH + 255) / 256;
    __shared__ __attribute__((aligned(16))) __bf16 abuf[2][BLK];

    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, lr = lane % 16, lg = lane / 16;
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    const int64_t wg0 = (int64_t)blockIdx.x * (4 * 16 * P);
    if (wg0 >= npts) return;
    const int64_t row0 = wg0 + wave * 16 * P;
    const __bf16* x = reinterpret_cast<const __bf16*>(A.x);

    // staging of one K step: chunk tid + 256 j, clamped to the last chunk (a
    // clamped thread stores a copy of that chunk's own value)
    struct Stage {
        uint4 v[SJ];
    };
    auto stage_load = [&](const __bf16* src) __attribute__((always_inline)) {
        Stage t;
#pragma unroll
        for (int j = 0; j < SJ; j++) t.v[j] = reinterpret_cast<const uint4*>(src)[min(tid + 256 * j, CH - 1)];
        return t;
    };
    auto stage_store = [&](int b, Stage t) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < SJ; j++) reinterpret_cast<uint4*>(abuf[b])[min(tid + 256 * j, CH - 1)] = t.v[j];
    };

    f32x4 acc[NT][P];
    bf16x8 hin[KCH][P];
    for (int li = 0; li + 1 < A.n_linear; li++) {
        const __bf16* Wl = reinterpret_cast<const __bf16*>(A.W[li]);
        const int KC = li == 0 ? KC0 : KCH;
#pragma unroll
        for (int ct = 0; ct < NT; ct++)
#pragma unroll
            for (int p = 0; p < P; p++) acc[ct][p] = f32x4{0.f, 0.f, 0.f, 0.f};
        stage_store(0, stage_load(Wl));
        __syncthreads();
        // K step kc from buffer kc & 1 while the next step's fragments are
        // fetched (past the last step: the last again, into the idle buffer)
        auto step = [&](int kc, const bf16x8* bx) __attribute__((always_inline)) {
            const int b = kc & 1;
            const Stage nxt = stage_load(Wl + (int64_t)min(kc + 1, KC - 1) * BLK);
#pragma unroll
            for (int ct = 0; ct < NT; ct++) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&abuf[b][(ct * 64 + lane) * 8]);
#pragma unroll
                for (int p = 0; p < P; p++) acc[ct][p] = M::mma(a, bx[p], acc[ct][p]);
            }
            stage_store(b ^ 1, nxt);
            __syncthreads();
        };
        if (li == 0) {
            const __bf16* xr[P];
#pragma unroll
            for (int p = 0; p < P; p++) {
                int64_t r = row0 + p * 16 + lr;
                r = r < npts ? r : npts - 1;
                xr[p] = x + r * kDescPad + lg * 8;
            }
            // descriptor fragments one K step ahead
            bf16x8 bx[P], bn[P];
#pragma unroll
            for (int p = 0; p < P; p++) bx[p] = *reinterpret_cast<const bf16x8*>(xr[p]);
            for (int kc = 0; kc < KC0; kc++) {
#pragma unroll
                for (int p = 0; p < P; p++)
                    bn[p] = *reinterpret_cast<const bf16x8*>(xr[p] + min(kc + 1, KC0 - 1) * 32);
                step(kc, bx);
#pragma unroll
                for (int p = 0; p < P; p++) bx[p] = bn[p];
            }
        } else {
#pragma unroll
            for (int kc = 0; kc < KCH; kc++) step(kc, hin[kc]);
        }
        // bias + ReLU into the next layer's B fragments (channels >= 16 NT are zero)
        const float* bias = A.bias[li];
#pragma unroll
        for (int kc = 0; kc < KCH; kc++)
#pragma unroll
            for (int p = 0; p < P; p++) {
                bf16x8 f;
#pragma unroll
                for (int e = 0; e < 8; e++) {
                    const int ct = 2 * kc + e / 4;
                    float v = 0.f;
                    if (ct < NT) v = fmaxf(acc[ct][p][e % 4] + bias[ct * 16 + lg * 4 + e % 4], 0.f);
                    f[e] = (__bf16)v;
                }
                hin[kc][p] = f;
            }
    }
    // last layer (a dot product over the channels, spread over the lane groups) + decode
#pragma unroll
    for (int p = 0; p < P; p++) {
        float s = 0.f;
#pragma unroll
        for (int kc = 0; kc < KCH; kc++)
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int ct = 2 * kc + e / 4;
                if (ct < NT) s += (float)hin[kc][p][e] * A.wout[ct * 16 + lg * 4 + e % 4];
            }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        const int64_t row = row0 + p * 16 + lr;
        if (lg == 0 && row < npts) {
            const float y = A.bout + s;
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row] = A.radiance * (A.f0[row] + A.albedo_gamma * expm1f(y));
        }
    }
}

template <int NT, int P>
static void launch_bf16_nt(const MlpArgs& a, hipStream_t s)
{
    const int per = 4 * 16 * P;
    hipLaunchKernelGGL((k_mlp_bf16<NT, P>), dim3((int)((a.npts + per - 1) / per)), dim3(256), 0, s, a);
}

static hipError_t launch_mlp_bf16(const MlpArgs& a, hipStream_t s)
{
    switch (a.wpad / 16) {
    case 1: launch_bf16_nt<1, 4>(a, s); break;
    case 2: launch_bf16_nt<2, 4>(a, s); break;
    case 4: launch_bf16_nt<4, 4>(a, s); break;
    case 8: launch_bf16_nt<8, 4>(a, s); break;
    case 13: launch_bf16_nt<13, 3>(a, s); break;
    case 16: launch_bf16_nt<16, 2>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NT>
static void launch_fp8_nt(const MlpArgs& a, dim3 g, dim3 b, hipStream_t s)
{
    hipLaunchKernelGGL((k_mlp_fp8<NT>), g, b, 0, s, a);
}

static hipError_t launch_mlp_fp8(const MlpArgs& a, hipStream_t s)
{
    constexpr int per = kMlpWaves * 64;
    int blocks = (int)((a.npts + per - 1) / per);
    dim3 g(blocks), b(256);
    switch (a.wpad / 16) {
    case 1: launch_fp8_nt<1>(a, g, b, s); break;
    case 2: launch_fp8_nt<2>(a, g, b, s); break;
    case 4: launch_fp8_nt<4>(a, g, b, s); break;
    case 8: launch_fp8_nt<8>(a, g, b, s); break;
    case 13: launch_fp8_nt<13>(a, g, b, s); break;
    case 16: launch_fp8_nt<16>(a, g, b, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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
int mlp_k_step(int prec)
{
    return prec == kPrecFP32 ? Mfma<kPrecFP32>::KS : prec == kPrecBF16 ? Mfma<kPrecBF16>::KS : Mfma<kPrecFP8>::KS;
}
int mlp_k_per_lane(int prec)
{
    return prec == kPrecFP32 ? Mfma<kPrecFP32>::KPL : prec == kPrecBF16 ? Mfma<kPrecBF16>::KPL : Mfma<kPrecFP8>::KPL;
}

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
    if (prec == kPrecFP8) return launch_mlp_fp8(a, s);
    if (prec == kPrecBF16) return launch_mlp_bf16(a, s);
    return launch_mlp_prec<kPrecFP32>(a, s);
}

}  // namespace nis
