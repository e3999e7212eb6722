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
    // calibration (FP32 only): the largest |input| of every layer, per lane,
    // then per wave, into A.absmax with an atomic maximum on the float bits
    const bool track = PREC == kPrecFP32 && A.absmax != nullptr;
    auto publish = [&](float v, int li) __attribute__((always_inline)) {
        for (int o = 1; o < 64; o <<= 1) v = fmaxf(v, __shfl_xor(v, o));
        if (lane == 0) atomicMax(reinterpret_cast<unsigned int*>(A.absmax) + li, __float_as_uint(v));
    };
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
            float imx = 0.f;
            // the fragments of K step kc + 1 are requested before the MFMAs of
            // step kc, so that their latency overlaps them
            typename M::frag a[RT], b[NT], an[RT], bn[NT];
            auto fetch = [&](int kc, typename M::frag* af, typename M::frag* bf) __attribute__((always_inline)) {
#pragma unroll
                for (int rt = 0; rt < RT; rt++) af[rt] = M::load(xr[rt] + kc * M::KS);
#pragma unroll
                for (int ct = 0; ct < NT; ct++) bf[ct] = M::load(Wf + (ct * KC + kc) * FRAG);
            };
            fetch(0, an, bn);
            for (int kc = 0; kc < KC; kc++) {
#pragma unroll
                for (int rt = 0; rt < RT; rt++) a[rt] = an[rt];
#pragma unroll
                for (int ct = 0; ct < NT; ct++) b[ct] = bn[ct];
                if (kc + 1 < KC) fetch(kc + 1, an, bn);
                if constexpr (PREC == kPrecFP32) {
                    if (track) {
#pragma unroll
                        for (int rt = 0; rt < RT; rt++) imx = fmaxf(imx, fabsf(a[rt]));
                    }
                }
#pragma unroll
                for (int ct = 0; ct < NT; ct++)
#pragma unroll
                    for (int rt = 0; rt < RT; rt++) acc[rt][ct] = M::mma(a[rt], b[ct], acc[rt][ct]);
            }
            if (track) publish(imx, 0);
        } else {
            typename M::frag a[RT], b[NT], an[RT], bn[NT];
            auto fetch = [&](int kc, typename M::frag* af, typename M::frag* bf) __attribute__((always_inline)) {
#pragma unroll
                for (int rt = 0; rt < RT; rt++) af[rt] = M::load(&h[rt * 16 + lr][kc * M::KS + lg * M::KPL]);
#pragma unroll
                for (int ct = 0; ct < NT; ct++) bf[ct] = M::load(Wf + (ct * KC + kc) * FRAG);
            };
            fetch(0, an, bn);
            for (int kc = 0; kc < KC; kc++) {
#pragma unroll
                for (int rt = 0; rt < RT; rt++) a[rt] = an[rt];
#pragma unroll
                for (int ct = 0; ct < NT; ct++) b[ct] = bn[ct];
                if (kc + 1 < KC) fetch(kc + 1, an, bn);
#pragma unroll
                for (int ct = 0; ct < NT; ct++)
#pragma unroll
                    for (int rt = 0; rt < RT; rt++) acc[rt][ct] = M::mma(a[rt], b[ct], acc[rt][ct]);
            }
        }
        __syncthreads();   // every lane's reads of h precede the in-place overwrite
        const float* bias = A.bias[li];
        float omx = 0.f;
#pragma unroll
        for (int ct = 0; ct < NT; ct++) {
            const float bb = bias[ct * 16 + lr];
#pragma unroll
            for (int rt = 0; rt < RT; rt++)
#pragma unroll
                for (int e = 0; e < 4; e++) {
                    const float v = fmaxf(acc[rt][ct][e] + bb, 0.f);
                    omx = fmaxf(omx, v);
                    h[rt * 16 + lg * 4 + e][ct * 16 + lr] = M::cvt(v);
                }
        }
        if (track) publish(omx, li + 1);
        __syncthreads();
    }
    // last layer + decode, one row per lane
    for (int rr = lane; rr < ROWS; rr += 64) {
        const int64_t row = row0 + rr;
        float y = A.bout;
        for (int k = 0; k < W; k++) y += (float)h[rr][k] * A.wout[k];
        if (row < npts) {
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row * A.out_stride] = decode_radiance(A.radiance, A.f0[row], A.albedo_gamma, y);
        }
    }
}

// BF16 backbone on 32x32x16 MFMA tiles, the weights as the A operand and the
// activations as B.  A layer's output tile D[channel][point] leaves lane
// l = p + 32 g holding, for point p, the 16 channels 8 (r/4) + 4 g + r%4 of
// the tile (r < 16).  Split into two halves of 8 registers these are exactly
// the lane's B fragments of two K steps of the next layer once that layer's K
// index is permuted to match (the weights are packed in that order), so the
// activations stay in registers from layer to layer.  For the first layer the
// descriptor columns are permuted instead, so that a lane's elements of four
// consecutive K steps are one 64-byte run of its descriptor row.
//
// A workgroup of 4 waves covers 4 * 32 * PT points.  The weights stream
// through LDS in stages of kStage K steps (NO KiB per step), copied from
// global memory straight into LDS and double buffered, so one barrier covers
// kStage steps.  The first layer's descriptor fragments take the same route
// into per-wave LDS regions, two stages ahead (three buffers), which keeps
// the HBM latency of the descriptor stream off the MFMA pipeline.
constexpr int kStage = 4;

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

// bfloat16 pair {lo, hi} rounded to nearest even, packed low half first: one
// v_cvt_pk_bf16_f32, written as a vector conversion so that the compiler sees
// it (and keeps the wait states an MFMA result needs before it is read)
__device__ __forceinline__ uint32_t cvt_pk_bf16(float lo, float hi)
{
    typedef float f32x2 __attribute__((ext_vector_type(2)));
    typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2v));
}

__device__ __forceinline__ f32x16 mfma32(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// buffer resource over bytes bytes at base (reads past the end return zero)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, int64_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// 16 bytes per lane from buffer r at voff + soff into LDS at lds + 16 * lane
// (lds is wave-uniform)
__device__ __forceinline__ void copy_lds16(__amdgpu_buffer_rsrc_t r, void* lds, int voff, int soff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, voff, soff, 0, 0);
}

// as copy_lds16 with the non-temporal cache policy, for data read exactly
// once (the descriptor stream), so that it does not displace the weights
__device__ __forceinline__ void copy_lds16_stream(__amdgpu_buffer_rsrc_t r, void* lds, int voff, int soff)
{
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void*)lds, 16, voff, soff, 0, 2);
}

// an empty use of x that the compiler must keep: x stays allocated up to here
__device__ __forceinline__ void keep_alive(const f32x16& x) { asm volatile("" ::"v"(x)); }

// waits until at most N of this wave's loads are outstanding
template <int N> __device__ __forceinline__ void wait_vm()
{
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

template <int V> using IC = std::integral_constant<int, V>;

// f(IC<I>), f(IC<I+1>), ..., f(IC<N-1>)
template <int I, int N, class F> __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (I < N) {
        f(IC<I>{});
        static_for<I + 1, N>(f);
    }
}

// Every LDS buffer is a variable of its own and each access names its buffer
// at compile time: the compiler can then tell that the copies in flight into
// one buffer do not alias the reads of another, and does not wait for them.
template <int NO, int KH, int PT, int NW>
__global__ void __launch_bounds__(64 * NW)
k_mlp_bf16(MlpArgs A)
{
    constexpr int KC0 = kDescPad / 16;          // K steps of the first layer
    constexpr int NQ0 = KC0 / kStage;           // its stages
    static_assert(KC0 % kStage == 0, "first-layer stages must tile the descriptor");
    constexpr int FRB = NO * 1024;              // bytes of one K step's weight fragments
    constexpr int STB = kStage * FRB;           // bytes of one weight stage
    constexpr int DTB = kStage * 1024;          // one wave's descriptor fragments of one point tile and stage
    constexpr int ND = PT * kStage;             // descriptor copies per wave and stage
    static_assert(PT <= 2, "descriptor buffers exist for two point tiles");
    // The weight buffers are the largest variables, which places them first,
    // where every read's offset fits the instruction's immediate field.
    __shared__ __attribute__((aligned(16))) uint8_t wb0[STB];
    __shared__ __attribute__((aligned(16))) uint8_t wb1[STB];
    __shared__ __attribute__((aligned(16))) uint8_t db00[NW][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db01[PT > 1 ? NW : 1][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db10[NW][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db11[PT > 1 ? NW : 1][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db20[NW][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db21[PT > 1 ? NW : 1][DTB];

    const int tid = threadIdx.x, lane = tid % 64, lp = lane % 32, lg = lane / 32;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    const int64_t wg0 = (int64_t)blockIdx.x * (NW * 32 * PT);
    if (wg0 >= npts) return;
    const int64_t row0 = wg0 + wave * 32 * PT;

    auto wbuf = [&](auto bc) __attribute__((always_inline)) -> uint8_t* {
        if constexpr (decltype(bc)::value == 0) return wb0;
        else return wb1;
    };
    // descriptor buffer d (of three) of point tile p, this wave's part
    auto dbuf = [&](auto dc, auto pc) __attribute__((always_inline)) -> uint8_t* {
        constexpr int d = decltype(dc)::value, p = decltype(pc)::value;
        if constexpr (p == 0) {
            if constexpr (d == 0) return db00[wave];
            else if constexpr (d == 1) return db10[wave];
            else return db20[wave];
        } else {
            if constexpr (d == 0) return db01[wave];
            else if constexpr (d == 1) return db11[wave];
            else return db21[wave];
        }
    };

    // The copies into LDS are buffer loads: the hardware checks each against
    // its buffer's size, and the compiler counts them as vector-memory loads
    // only, so they do not force waits on the LDS reads issued around them.
    // Copies of weight stages: nch chunks of 1 KiB from byte offset off of a
    // layer's weights, chunk c by wave c % NW; copy u of this wave is chunk
    // wave + NW u (at most NWC per stage).  A chunk index past the stage
    // repeats its last chunk (chunk 0 of an empty stage), so every wave
    // issues the same number of copies.
    constexpr int NWC = (kStage * NO + NW - 1) / NW;
    auto copy_w = [&](__amdgpu_buffer_rsrc_t r, int off, int nch, uint8_t* dst, int u) __attribute__((always_inline)) {
        const int c = min(wave + NW * u, max(nch, 1) - 1);
        copy_lds16(r, dst + c * 1024, lane * 16, off + c * 1024);
    };
    // A first-layer stage of a point tile is the 128-byte slice 128 q.. of
    // each of its 32 descriptor rows (K steps 4q..4q+3 of both lane groups).
    // In LDS row r's slice holds its 16-byte segment s at slot s ^ ((r/2)%8):
    // each copy instruction then fills 8 whole rows (8 cache lines), and the
    // 16 lanes of a B-fragment read phase (16 rows, one segment) fall on
    // distinct banks.  Lane v of copy i of tile p fetches row 8i + v/8, slot
    // v%8; rows past the live count repeat the last live row.  Offsets are
    // taken from the workgroup's first row, so the base is wave-uniform.
    const __amdgpu_buffer_rsrc_t xr = rsrc(reinterpret_cast<const uint8_t*>(A.x) + wg0 * (kDescPad * 2),
                                           min(npts - wg0, (int64_t)(NW * 32 * PT)) * (kDescPad * 2));
    uint32_t doff[PT][4];
#pragma unroll
    for (int p = 0; p < PT; p++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 8 * i + lane / 8, sl = lane % 8, seg = sl ^ ((r >> 1) & 7);
            int64_t row = row0 + p * 32 + r;
            row = row < npts ? row : npts - 1;
            doff[p][i] = (uint32_t)((row - wg0) * (kDescPad * 2) + seg * 16);
        }
    // copy k (of ND) of this wave's descriptor stage q into buffer d: tile k/4,
    // rows 8 (k%4)..
    auto copy_d = [&](int q, auto dc, int k) __attribute__((always_inline)) {
        const int p = k / 4, i = k % 4;
        uint8_t* dst = p == 0 ? dbuf(dc, IC<0>{}) : dbuf(dc, IC<PT - 1>{});
        copy_lds16_stream(xr, dst + i * 1024, doff[p][i], q * 128);
    };
    // byte offset of this lane's B fragment of step j within a tile's slice
    int roff[kStage];
#pragma unroll
    for (int j = 0; j < kStage; j++) roff[j] = lp * 128 + (((lg * 4 + j) ^ ((lp >> 1) & 7)) << 4);

    f32x16 acc[NO][PT];
    // A fragment of output tile ct at K step j of a weight buffer
    auto read_a = [&](const uint8_t* wsrc, int j, int ct) __attribute__((always_inline)) {
        return *reinterpret_cast<const bf16x8*>(wsrc + j * FRB + ct * 1024 + lane * 16);
    };
    // accumulators start at the layer's bias (register r of tile ct holds
    // channel ct*32 + (r/4)*8 + 4 g + r%4; the bias is padded to whole tiles)
    auto init_acc = [&](const float* bias, int np) __attribute__((always_inline)) {
#pragma unroll
        for (int ct = 0; ct < NO; ct++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float4 bv = *reinterpret_cast<const float4*>(bias + ct * 32 + j * 8 + lg * 4);
#pragma unroll
                for (int p = 0; p < PT; p++)
                    if (p < np) {
                        acc[ct][p][j * 4 + 0] = bv.x;
                        acc[ct][p][j * 4 + 1] = bv.y;
                        acc[ct][p][j * 4 + 2] = bv.z;
                        acc[ct][p][j * 4 + 3] = bv.w;
                    }
            }
    };
    init_acc(A.bias[0], PT);

    const int nhid = A.n_linear - 2;   // hidden layers after the first
    const __amdgpu_buffer_rsrc_t W0 = rsrc(A.W[0], KC0 * FRB);
    const __amdgpu_buffer_rsrc_t W1 = nhid > 0 ? rsrc(A.W[1], KH * FRB) : W0;

    // A K step is issued as NO units in a fixed order: the PT MFMAs of
    // output tile ct and one of the stage's copies (copy u = j*NO + ct while
    // any are left), so that copies trickle out between MFMAs instead of
    // stalling the wave in a burst; the first unit also reads all of the next
    // step's fragments, which leaves the rest of the step to cover their
    // latency.

    // ---- first layer.  Stage q multiplies from weight buffer q % 2 and
    // descriptor buffer q % 3 while the weights of stage q + 1 and the
    // descriptors of stage q + 2 are copied (past the last stage the copies
    // repeat the last descriptor stage into an idle buffer, which keeps the
    // count of loads in flight the same at every stage end).
    auto stage0 = [&](auto bc, auto dc, int q) __attribute__((always_inline)) {
        constexpr int B = decltype(bc)::value, D = decltype(dc)::value;
        const IC<(D + 2) % 3> dn{};   // descriptor buffer being filled
        const bool last = q + 1 == NQ0;
        const uint8_t* wcur = wbuf(IC<B>{});
        uint8_t* wnx = wbuf(IC<1 - B>{});
        const __amdgpu_buffer_rsrc_t wsrc = last ? W1 : W0;
        const int woff = last ? 0 : (q + 1) * STB;
        const int wnch = !last ? kStage * NO : nhid > 0 ? min(kStage, KH) * NO : 0;
        const int qd = min(q + 2, NQ0 - 1);
        const uint8_t* dcur[PT];
        static_for<0, PT>([&](auto pc) __attribute__((always_inline)) { dcur[decltype(pc)::value] = dbuf(IC<D>{}, pc); });
        bf16x8 a[2][NO], bx[2][PT];
#pragma unroll
        for (int ct = 0; ct < NO; ct++) a[0][ct] = read_a(wcur, 0, ct);
#pragma unroll
        for (int p = 0; p < PT; p++) bx[0][p] = *reinterpret_cast<const bf16x8*>(dcur[p] + roff[0]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < kStage; j++)
#pragma unroll
            for (int ct = 0; ct < NO; ct++) {
                const int u = j * NO + ct;
#pragma unroll
                for (int p = 0; p < PT; p++) acc[ct][p] = mfma32(a[j % 2][ct], bx[j % 2][p], acc[ct][p]);
                __builtin_amdgcn_sched_barrier(0);
                if (j + 1 < kStage && ct == 0) {
#pragma unroll
                    for (int c2 = 0; c2 < NO; c2++) a[(j + 1) % 2][c2] = read_a(wcur, j + 1, c2);
#pragma unroll
                    for (int p = 0; p < PT; p++)
                        bx[(j + 1) % 2][p] = *reinterpret_cast<const bf16x8*>(dcur[p] + roff[j + 1]);
                }
                if (u < NWC) copy_w(wsrc, woff, wnch, wnx, u);
                else if (u - NWC < ND) copy_d(qd, dn, u - NWC);
                __builtin_amdgcn_sched_barrier(0);
            }
        // copies that found no unit (small widths)
#pragma unroll
        for (int u = kStage * NO; u < NWC + ND; u++) {
            if (u < NWC) copy_w(wsrc, woff, wnch, wnx, u);
            else copy_d(qd, dn, u - NWC);
        }
        // the last stage's copies are waited for after the epilogue
        if (!last) {
            wait_vm<ND>();
            __syncthreads();
        }
    };
#pragma unroll
    for (int u = 0; u < NWC; u++) copy_w(W0, 0, kStage * NO, wbuf(IC<0>{}), u);
#pragma unroll
    for (int k = 0; k < ND; k++) copy_d(0, IC<0>{}, k);
#pragma unroll
    for (int k = 0; k < ND; k++) copy_d(1, IC<1>{}, k);
    wait_vm<ND>();
    __syncthreads();
    for (int q = 0; q < NQ0; q += 6) {
        stage0(IC<0>{}, IC<0>{}, q);
        if (q + 1 < NQ0) stage0(IC<1>{}, IC<1>{}, q + 1);
        if (q + 2 < NQ0) stage0(IC<0>{}, IC<2>{}, q + 2);
        if (q + 3 < NQ0) stage0(IC<1>{}, IC<0>{}, q + 3);
        if (q + 4 < NQ0) stage0(IC<0>{}, IC<1>{}, q + 4);
        if (q + 5 < NQ0) stage0(IC<1>{}, IC<2>{}, q + 5);
    }

    // ---- ReLU of a finished layer into the next layer's B fragments.  The
    // ReLU is applied after rounding, as a signed 16-bit max on the bfloat16
    // bit patterns (rounding keeps the sign, so both orders agree).
    bf16x8 hin[KH][PT];
    auto epilogue = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int kc = 0; kc < KH; kc++)
#pragma unroll
            for (int p = 0; p < PT; p++) {
                const f32x16& c = acc[kc / 2][p];
                const int o = (kc % 2) * 8;
                const uint4 f = {cvt_pk_bf16(c[o + 0], c[o + 1]), cvt_pk_bf16(c[o + 2], c[o + 3]),
                                 cvt_pk_bf16(c[o + 4], c[o + 5]), cvt_pk_bf16(c[o + 6], c[o + 7])};
                const i16x8 v = __builtin_elementwise_max(__builtin_bit_cast(i16x8, f), i16x8{});
                hin[kc][p] = __builtin_bit_cast(bf16x8, v);
            }
        // With an odd number of K steps the second half of the last tile's
        // accumulator is never read.  When the accumulators live in VGPRs (one
        // point tile per wave), keep it allocated until the epilogue's end:
        // otherwise its registers can be handed to the conversions above while
        // the MFMA that writes them is still in flight, and its late write
        // overwrites their results.  (With two tiles the accumulators are in
        // AGPRs, which the conversions never write.)
        if constexpr (KH % 2 == 1 && PT == 1) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int p = 0; p < PT; p++) keep_alive(acc[NO - 1][p]);
        }
    };
    epilogue();
    wait_vm<0>();
    __syncthreads();

    // ---- hidden layers: B fragments from registers; a layer whose stages
    // start at weight buffer B0 copies the next layer's first stage during
    // its own last stage, and waits for it after its epilogue.  The bias is
    // loaded into the accumulators of point tile 0 only: in the layer's first
    // K step the other tiles take it as their C operand before tile 0
    // overwrites it.
    constexpr int NQH = (KH + kStage - 1) / kStage;
    auto hidden = [&](auto b0c, int li) __attribute__((always_inline)) {
        constexpr int B0 = decltype(b0c)::value;
        const __amdgpu_buffer_rsrc_t Wl = rsrc(A.W[li], KH * FRB);
        const __amdgpu_buffer_rsrc_t Wn = li < nhid ? rsrc(A.W[li + 1], KH * FRB) : Wl;
        init_acc(A.bias[li], 1);
        static_for<0, NQH>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value, B = (B0 + q) % 2, k0 = q * kStage;
            constexpr int ns = KH - k0 < kStage ? KH - k0 : kStage;
            // copies of this layer's next stage, or of the next layer's first
            constexpr bool inner = q + 1 < NQH;
            constexpr int nn = !inner ? 0 : KH - k0 - kStage < kStage ? KH - k0 - kStage : kStage;
            const __amdgpu_buffer_rsrc_t wsrc = inner ? Wl : Wn;
            const int woff = inner ? (k0 + kStage) * FRB : 0;
            const int wnch = inner ? nn * NO : li < nhid ? (KH < kStage ? KH : kStage) * NO : 0;
            const uint8_t* wcur = wbuf(IC<B>{});
            uint8_t* wnx = wbuf(IC<1 - B>{});
            bf16x8 a[2][NO];
#pragma unroll
            for (int ct = 0; ct < NO; ct++) a[0][ct] = read_a(wcur, 0, ct);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < ns; j++)
#pragma unroll
                for (int ct = 0; ct < NO; ct++) {
                    const int u = j * NO + ct;
                    if (q == 0 && j == 0) {
#pragma unroll
                        for (int p = PT - 1; p >= 0; p--) acc[ct][p] = mfma32(a[0][ct], hin[k0][p], acc[ct][0]);
                    } else {
#pragma unroll
                        for (int p = 0; p < PT; p++) acc[ct][p] = mfma32(a[j % 2][ct], hin[k0 + j][p], acc[ct][p]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (j + 1 < ns && ct == 0) {
#pragma unroll
                        for (int c2 = 0; c2 < NO; c2++) a[(j + 1) % 2][c2] = read_a(wcur, j + 1, c2);
                    }
                    if (u < NWC) copy_w(wsrc, woff, wnch, wnx, u);
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
            for (int u = ns * NO; u < NWC; u++) copy_w(wsrc, woff, wnch, wnx, u);
            if constexpr (q + 1 < NQH) {
                wait_vm<0>();
                __syncthreads();
            }
        });
        epilogue();
        wait_vm<0>();
        __syncthreads();
    };
    constexpr int HB = NQ0 % 2;   // weight buffer of the first hidden stage
    if constexpr (NQH % 2 == 0) {
        for (int li = 1; li <= nhid; li++) hidden(IC<HB>{}, li);
    } else {
        for (int li = 1; li <= nhid; li += 2) {
            hidden(IC<HB>{}, li);
            if (li + 1 <= nhid) hidden(IC<1 - HB>{}, li + 1);
        }
    }

    // ---- last layer (a dot product over the lane's channels, then across the
    // two lane groups) + decode
#pragma unroll
    for (int p = 0; p < PT; p++) {
        float s = 0.f;
#pragma unroll
        for (int kc = 0; kc < KH; kc++)
#pragma unroll
            for (int hf = 0; hf < 2; hf++) {
                const float4 w = *reinterpret_cast<const float4*>(A.wout + (kc / 2) * 32 + (2 * (kc % 2) + hf) * 8 + lg * 4);
                s += (float)hin[kc][p][hf * 4 + 0] * w.x + (float)hin[kc][p][hf * 4 + 1] * w.y +
                     (float)hin[kc][p][hf * 4 + 2] * w.z + (float)hin[kc][p][hf * 4 + 3] * w.w;
            }
        s += __shfl_xor(s, 32);
        const int64_t row = row0 + p * 32 + lp;
        if (lg == 0 && row < npts) {
            const float y = A.bout + s;
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row * A.out_stride] = decode_radiance(A.radiance, A.f0[row], A.albedo_gamma, y);
        }
    }
}

// FP8 backbone on 32x32x64 E4M3 MFMA tiles with hardware block scales
// (v_mfma_scale_f32_32x32x64_f8f6f4), the weights as the A operand and the
// activations as B, in the layout of the BF16 kernel above.  Every layer
// input x_l is stored as E4M3 codes q = x_l / s_l with one static scale s_l
// per layer (calibrated on representative points, nis_calibrate_fp8).  The
// host folds the scales into the packed network: layer l's weights become
// W_l s_l / s_{l+1}, quantised per output channel with a power-of-two scale
// that the MFMA applies (its E8M0 block scale; the activations' block scale
// is 1), and its bias beta_l / s_{l+1}.  The accumulator then holds
// z_l / s_{l+1}, and the next layer's codes are med3(acc, 0, 448) converted
// to E4M3: ReLU and saturation in one instruction.  Nothing depends on the
// other points of the batch.
//
// A K step is 64 inputs.  The output tile pair (2 kc, 2 kc + 1) leaves lane
// l = p + 32 g holding 32 values of point p, which are exactly its B fragment
// of the next layer's K step kc once that layer's K order is permuted to
// match (slot e < 16: channel 32 (2 kc) + 8 (e/4) + 4 g + e%4 of tile 2 kc;
// e >= 16: the same in tile 2 kc + 1, zero past the last tile).  For the
// first layer, a stage of two K steps is the 128-byte slice of each
// descriptor row, lane group g taking its bytes 64 g .. 64 g + 63 (32 per
// step).  A lane's 32-byte A fragment of one tile and step is stored as two
// 16-byte halves, the 64 lanes' first halves before their second halves, so
// that each 16-byte LDS read is one contiguous 1 KiB row of the wave.
constexpr int kStage8 = 2;   // K steps per weight stage (FP8)

// The value unchanged, but opaque to the optimiser (it cannot be hoisted or
// shared across the places that ask for it).
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

typedef int i32x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x16 mfma32_f8(const i32x8& a, const i32x8& b, f32x16 c, int ea)
{
    // formats: E4M3 for both operands; block scales: ea for A, 2^0 for B
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, ea, 0, 127);
}

// four floats -> four E4M3 codes (little-endian) after med3(x, lo, 448)
__device__ __forceinline__ int fp8x4_clamped(float a, float b, float c, float d, float lo)
{
    a = __builtin_amdgcn_fmed3f(a, lo, 448.f);
    b = __builtin_amdgcn_fmed3f(b, lo, 448.f);
    c = __builtin_amdgcn_fmed3f(c, lo, 448.f);
    d = __builtin_amdgcn_fmed3f(d, lo, 448.f);
    const int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
    return __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
}

template <int NO, int KH, int PT, int NW>
__global__ void __launch_bounds__(64 * NW)
k_mlp_f8(MlpArgs A)
{
    constexpr int KC0 = kDescF8 / 64;           // K steps of the first layer
    constexpr int NQ0 = KC0 / kStage8;          // its stages
    static_assert(KC0 % kStage8 == 0, "first-layer stages must tile the descriptor");
    constexpr int FRB = NO * 2048;              // bytes of one K step's weight fragments
    constexpr int STB = kStage8 * FRB;          // bytes of one weight stage
    constexpr int DTB = 4096;                   // one wave's descriptor slices of one point tile and stage
    constexpr int ND = PT * 4;                  // descriptor copies (1 KiB) per wave and stage
    static_assert(PT <= 2, "descriptor buffers exist for two point tiles");
    __shared__ __attribute__((aligned(16))) uint8_t wb0[STB];
    __shared__ __attribute__((aligned(16))) uint8_t wb1[STB];
    __shared__ __attribute__((aligned(16))) uint8_t db00[NW][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db01[PT > 1 ? NW : 1][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db10[NW][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db11[PT > 1 ? NW : 1][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db20[NW][DTB];
    __shared__ __attribute__((aligned(16))) uint8_t db21[PT > 1 ? NW : 1][DTB];

    const int tid = threadIdx.x, lane = tid % 64, lp = lane % 32, lg = lane / 32;
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const int64_t npts = A.count ? min(max((int64_t)*A.count - A.count_off, (int64_t)0), A.npts) : A.npts;
    const int64_t wg0 = (int64_t)blockIdx.x * (NW * 32 * PT);
    if (wg0 >= npts) return;
    const int64_t row0 = wg0 + wave * 32 * PT;

    auto wbuf = [&](auto bc) __attribute__((always_inline)) -> uint8_t* {
        if constexpr (decltype(bc)::value == 0) return wb0;
        else return wb1;
    };
    auto dbuf = [&](auto dc, auto pc) __attribute__((always_inline)) -> uint8_t* {
        constexpr int d = decltype(dc)::value, p = decltype(pc)::value;
        if constexpr (p == 0) {
            if constexpr (d == 0) return db00[wave];
            else if constexpr (d == 1) return db10[wave];
            else return db20[wave];
        } else {
            if constexpr (d == 0) return db01[wave];
            else if constexpr (d == 1) return db11[wave];
            else return db21[wave];
        }
    };

    // weight stages as in the BF16 kernel: chunks of 1 KiB, chunk c by wave c % NW
    constexpr int NWC = (kStage8 * NO * 2 + NW - 1) / NW;
    auto copy_w = [&](__amdgpu_buffer_rsrc_t r, int off, int nch, uint8_t* dst, int u) __attribute__((always_inline)) {
        const int c = min(wave + NW * u, max(nch, 1) - 1);
        copy_lds16(r, dst + c * 1024, lane * 16, off + c * 1024);
    };
    // descriptor slices: 128 bytes of each of 32 rows per tile and stage, row
    // r's 16-byte segment s at slot s ^ ((r/2) % 8), as in the BF16 kernel
    const __amdgpu_buffer_rsrc_t xr = rsrc(reinterpret_cast<const uint8_t*>(A.x) + wg0 * kDescF8,
                                           min(npts - wg0, (int64_t)(NW * 32 * PT)) * kDescF8);
    uint32_t doff[PT][4];
#pragma unroll
    for (int p = 0; p < PT; p++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 8 * i + lane / 8, sl = lane % 8, seg = sl ^ ((r >> 1) & 7);
            int64_t row = row0 + p * 32 + r;
            row = row < npts ? row : npts - 1;
            doff[p][i] = (uint32_t)((row - wg0) * kDescF8 + seg * 16);
        }
    auto copy_d = [&](int q, auto dc, int k) __attribute__((always_inline)) {
        const int p = k / 4, i = k % 4;
        uint8_t* dst = p == 0 ? dbuf(dc, IC<0>{}) : dbuf(dc, IC<PT - 1>{});
        copy_lds16_stream(xr, dst + i * 1024, doff[p][i], q * 128);
    };
    // byte offsets of the two 16-byte halves of this lane's B fragment of step j
    int roff[kStage8][2];
#pragma unroll
    for (int j = 0; j < kStage8; j++)
#pragma unroll
        for (int h = 0; h < 2; h++) roff[j][h] = lp * 128 + (((lg * 4 + 2 * j + h) ^ ((lp >> 1) & 7)) << 4);

    f32x16 acc[NO][PT];
    // (the per-lane parts of the LDS addresses pass through opaque() once per
    // stage, so that the compiler forms each stage's addresses anew instead of
    // keeping every buffer's precomputed addresses live across the kernel)
    auto read_a = [&](const uint8_t* wsrc, int j, int ct, int lo16) __attribute__((always_inline)) {
        const uint8_t* base = wsrc + j * FRB + ct * 2048 + lo16;
        const int4 lo = *reinterpret_cast<const int4*>(base), hi = *reinterpret_cast<const int4*>(base + 1024);
        return i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    };
    auto read_b = [&](const uint8_t* dsrc, int o0, int o1) __attribute__((always_inline)) {
        const int4 lo = *reinterpret_cast<const int4*>(dsrc + o0);
        const int4 hi = *reinterpret_cast<const int4*>(dsrc + o1);
        return i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    };
    auto init_acc = [&](const float* bias, int np) __attribute__((always_inline)) {
#pragma unroll
        for (int ct = 0; ct < NO; ct++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float4 bv = *reinterpret_cast<const float4*>(bias + ct * 32 + j * 8 + lg * 4);
#pragma unroll
                for (int p = 0; p < PT; p++)
                    if (p < np) {
                        acc[ct][p][j * 4 + 0] = bv.x;
                        acc[ct][p][j * 4 + 1] = bv.y;
                        acc[ct][p][j * 4 + 2] = bv.z;
                        acc[ct][p][j * 4 + 3] = bv.w;
                    }
            }
    };
    // the E8M0 weight scales of this lane's row (channel ct*32 + lp) of a layer
    int ea[NO];
    auto load_scales = [&](int li) __attribute__((always_inline)) {
#pragma unroll
        for (int ct = 0; ct < NO; ct++) ea[ct] = (int)A.wexp[li][ct * 32 + lp];
    };
    init_acc(A.bias[0], PT);
    load_scales(0);

    const int nhid = A.n_linear - 2;
    const __amdgpu_buffer_rsrc_t W0 = rsrc(A.W[0], KC0 * FRB);
    const __amdgpu_buffer_rsrc_t W1 = nhid > 0 ? rsrc(A.W[1], KH * FRB) : W0;

    // ---- first layer: stage q from weight buffer q % 2 and descriptor buffer
    // q % 3 while stage q + 1's weights and stage q + 2's descriptors load
    auto stage0 = [&](auto bc, auto dc, int q) __attribute__((always_inline)) {
        constexpr int B = decltype(bc)::value, D = decltype(dc)::value;
        const IC<(D + 2) % 3> dn{};
        const bool last = q + 1 == NQ0;
        const uint8_t* wcur = wbuf(IC<B>{});
        uint8_t* wnx = wbuf(IC<1 - B>{});
        const __amdgpu_buffer_rsrc_t wsrc = last ? W1 : W0;
        const int woff = last ? 0 : (q + 1) * STB;
        const int wnch = !last ? kStage8 * NO * 2 : nhid > 0 ? min(kStage8, KH) * NO * 2 : 0;
        const int qd = min(q + 2, NQ0 - 1);
        const uint8_t* dcur[PT];
        static_for<0, PT>([&](auto pc) __attribute__((always_inline)) { dcur[decltype(pc)::value] = dbuf(IC<D>{}, pc); });
        // A fragments are read one unit ahead (one tile's worth in flight),
        // B fragments one step ahead
        const int la = opaque(lane * 16);
        int ro[kStage8][2];
#pragma unroll
        for (int j = 0; j < kStage8; j++)
#pragma unroll
            for (int h = 0; h < 2; h++) ro[j][h] = opaque(roff[j][h]);
        i32x8 a[2], bx[2][PT];
        a[0] = read_a(wcur, 0, 0, la);
#pragma unroll
        for (int p = 0; p < PT; p++) bx[0][p] = read_b(dcur[p], ro[0][0], ro[0][1]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < kStage8; j++)
#pragma unroll
            for (int ct = 0; ct < NO; ct++) {
                const int u = j * NO + ct;
                // (each read's address passes through opaque() here, so that
                // the read cannot be hoisted above this unit)
                if (u + 1 < kStage8 * NO) a[(u + 1) % 2] = read_a(wcur, (u + 1) / NO, (u + 1) % NO, opaque(la));
                if (j + 1 < kStage8 && ct == 0) {
#pragma unroll
                    for (int p = 0; p < PT; p++)
                        bx[(j + 1) % 2][p] = read_b(dcur[p], opaque(ro[j + 1][0]), opaque(ro[j + 1][1]));
                }
#pragma unroll
                for (int p = 0; p < PT; p++) acc[ct][p] = mfma32_f8(a[u % 2], bx[j % 2][p], acc[ct][p], ea[ct]);
                __builtin_amdgcn_sched_barrier(0);
                if (u < NWC) copy_w(wsrc, woff, wnch, wnx, u);
                else if (u - NWC < ND) copy_d(qd, dn, u - NWC);
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
        for (int u = kStage8 * NO; u < NWC + ND; u++) {
            if (u < NWC) copy_w(wsrc, woff, wnch, wnx, u);
            else copy_d(qd, dn, u - NWC);
        }
        // (unconditional: a branch here would let the compiler sink this
        // stage's MFMAs past it into one block, with every fragment live)
        wait_vm<ND>();
        __syncthreads();
    };
#pragma unroll
    for (int u = 0; u < NWC; u++) copy_w(W0, 0, kStage8 * NO * 2, wbuf(IC<0>{}), u);
#pragma unroll
    for (int k = 0; k < ND; k++) copy_d(0, IC<0>{}, k);
#pragma unroll
    for (int k = 0; k < ND; k++) copy_d(1, IC<1>{}, k);
    wait_vm<ND>();
    __syncthreads();
    for (int q = 0; q < NQ0; q += 6) {
        stage0(IC<0>{}, IC<0>{}, q);
        if (q + 1 < NQ0) stage0(IC<1>{}, IC<1>{}, q + 1);
        if (q + 2 < NQ0) stage0(IC<0>{}, IC<2>{}, q + 2);
        if (q + 3 < NQ0) stage0(IC<1>{}, IC<0>{}, q + 3);
        if (q + 4 < NQ0) stage0(IC<0>{}, IC<1>{}, q + 4);
        if (q + 5 < NQ0) stage0(IC<1>{}, IC<2>{}, q + 5);
    }

    // ---- a finished layer's accumulators (z / s_next) into the next layer's
    // B fragments: ReLU and saturation by med3, then E4M3
    i32x8 hin[KH][PT];
    auto epilogue = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int kc = 0; kc < KH; kc++)
#pragma unroll
            for (int p = 0; p < PT; p++) {
                i32x8 f;
#pragma unroll
                for (int hf = 0; hf < 2; hf++) {
                    const int t = 2 * kc + hf;
                    if (t < NO) {
                        const f32x16& c = acc[t < NO ? t : 0][p];
#pragma unroll
                        for (int v = 0; v < 4; v++)
                            f[hf * 4 + v] = fp8x4_clamped(c[4 * v], c[4 * v + 1], c[4 * v + 2], c[4 * v + 3], 0.f);
                    } else {
#pragma unroll
                        for (int v = 0; v < 4; v++) f[hf * 4 + v] = 0;
                    }
                }
                hin[kc][p] = f;
            }
    };
    epilogue();
    wait_vm<0>();
    __syncthreads();

    // ---- hidden layers, B fragments from registers (as in the BF16 kernel)
    constexpr int NQH = (KH + kStage8 - 1) / kStage8;
    auto hidden = [&](auto b0c, int li) __attribute__((always_inline)) {
        constexpr int B0 = decltype(b0c)::value;
        const __amdgpu_buffer_rsrc_t Wl = rsrc(A.W[li], KH * FRB);
        const __amdgpu_buffer_rsrc_t Wn = li < nhid ? rsrc(A.W[li + 1], KH * FRB) : Wl;
        init_acc(A.bias[li], 1);
        load_scales(li);
        static_for<0, NQH>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value, B = (B0 + q) % 2, k0 = q * kStage8;
            constexpr int ns = KH - k0 < kStage8 ? KH - k0 : kStage8;
            constexpr bool inner = q + 1 < NQH;
            constexpr int nn = !inner ? 0 : KH - k0 - kStage8 < kStage8 ? KH - k0 - kStage8 : kStage8;
            const __amdgpu_buffer_rsrc_t wsrc = inner ? Wl : Wn;
            const int woff = inner ? (k0 + kStage8) * FRB : 0;
            const int wnch = inner ? nn * NO * 2 : li < nhid ? (KH < kStage8 ? KH : kStage8) * NO * 2 : 0;
            const uint8_t* wcur = wbuf(IC<B>{});
            uint8_t* wnx = wbuf(IC<1 - B>{});
            const int la = opaque(lane * 16);
            i32x8 a[2];
            a[0] = read_a(wcur, 0, 0, la);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < ns; j++)
#pragma unroll
                for (int ct = 0; ct < NO; ct++) {
                    const int u = j * NO + ct;
                    if (u + 1 < ns * NO) a[(u + 1) % 2] = read_a(wcur, (u + 1) / NO, (u + 1) % NO, opaque(la));
                    if (q == 0 && j == 0) {
#pragma unroll
                        for (int p = PT - 1; p >= 0; p--)
                            acc[ct][p] = mfma32_f8(a[u % 2], hin[k0][p], acc[ct][0], ea[ct]);
                    } else {
#pragma unroll
                        for (int p = 0; p < PT; p++)
                            acc[ct][p] = mfma32_f8(a[u % 2], hin[k0 + j][p], acc[ct][p], ea[ct]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (u < NWC) copy_w(wsrc, woff, wnch, wnx, u);
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
            for (int u = ns * NO; u < NWC; u++) copy_w(wsrc, woff, wnch, wnx, u);
            if constexpr (q + 1 < NQH) {
                wait_vm<0>();
                __syncthreads();
            }
        });
        epilogue();
        wait_vm<0>();
        __syncthreads();
    };
    constexpr int HB = NQ0 % 2;
    if constexpr (NQH % 2 == 0) {
        for (int li = 1; li <= nhid; li++) hidden(IC<HB>{}, li);
    } else {
        for (int li = 1; li <= nhid; li += 2) {
            hidden(IC<HB>{}, li);
            if (li + 1 <= nhid) hidden(IC<1 - HB>{}, li + 1);
        }
    }

    // ---- last layer: the codes times the output weights (which carry the
    // last input scale), over the lane's channels and across its two groups
#pragma unroll
    for (int p = 0; p < PT; p++) {
        float s = 0.f;
#pragma unroll
        for (int kc = 0; kc < KH; kc++)
#pragma unroll
            for (int hf = 0; hf < 2; hf++) {
                const int t = 2 * kc + hf;
                if (t < NO) {
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int w4 = hin[kc][p][hf * 4 + v];
                        const float4 w = *reinterpret_cast<const float4*>(A.wout + t * 32 + v * 8 + lg * 4);
                        s += __builtin_amdgcn_cvt_f32_fp8(w4, 0) * w.x + __builtin_amdgcn_cvt_f32_fp8(w4, 1) * w.y +
                             __builtin_amdgcn_cvt_f32_fp8(w4, 2) * w.z + __builtin_amdgcn_cvt_f32_fp8(w4, 3) * w.w;
                    }
                }
            }
        s += __shfl_xor(s, 32);
        const int64_t row = row0 + p * 32 + lp;
        if (lg == 0 && row < npts) {
            const float y = A.bout + s;
            if (A.y_out) A.y_out[row] = y;
            if (A.out) A.out[row * A.out_stride] = decode_radiance(A.radiance, A.f0[row], A.albedo_gamma, y);
        }
    }
}

template <int NO, int KH, int PT, int NW>
static void launch_bf16_nt(const MlpArgs& a, hipStream_t s)
{
    const int per = NW * 32 * PT;
    hipLaunchKernelGGL((k_mlp_bf16<NO, KH, PT, NW>), dim3((int)((a.npts + per - 1) / per)), dim3(64 * NW), 0, s, a);
}

static hipError_t launch_mlp_bf16(const MlpArgs& a, hipStream_t s)
{
    switch (a.wpad) {
    case 16: launch_bf16_nt<1, 1, 2, 4>(a, s); break;
    case 32: launch_bf16_nt<1, 2, 2, 4>(a, s); break;
    case 64: launch_bf16_nt<2, 4, 2, 4>(a, s); break;
    case 128: launch_bf16_nt<4, 8, 2, 4>(a, s); break;
    case 208: launch_bf16_nt<7, 13, 2, 4>(a, s); break;
    case 256: launch_bf16_nt<8, 16, 1, 4>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NO, int KH, int PT, int NW>
static void launch_f8_nt(const MlpArgs& a, hipStream_t s)
{
    const int per = NW * 32 * PT;
    hipLaunchKernelGGL((k_mlp_f8<NO, KH, PT, NW>), dim3((int)((a.npts + per - 1) / per)), dim3(64 * NW), 0, s, a);
}

static hipError_t launch_mlp_fp8(const MlpArgs& a, hipStream_t s)
{
    switch (a.wpad) {
    case 16: launch_f8_nt<1, 1, 2, 4>(a, s); break;
    case 32: launch_f8_nt<1, 1, 2, 4>(a, s); break;
    case 64: launch_f8_nt<2, 1, 2, 4>(a, s); break;
    case 128: launch_f8_nt<4, 2, 2, 4>(a, s); break;
    case 208: launch_f8_nt<7, 4, 2, 4>(a, s); break;
    case 256: launch_f8_nt<8, 4, 1, 4>(a, s); break;
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

// MFMA K step and elements per lane of a B fragment of the FP32 kernel.
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

__global__ void k_decode(const float* __restrict__ y, const float* __restrict__ f0, int64_t n, float radiance,
                         float albedo_gamma, float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = decode_radiance(radiance, f0[i], albedo_gamma, y[i]);
}

hipError_t launch_decode(const float* y, const float* f0, int64_t n, float radiance, float albedo_gamma, float* out,
                         hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_decode, dim3((int)blocks), dim3(256), 0, s, y, f0, n, radiance, albedo_gamma, out);
    return hipGetLastError();
}

hipError_t launch_mlp(int prec, const MlpArgs& a, hipStream_t s)
{
    if (a.npts <= 0) return hipSuccess;
    if (prec == kPrecFP8) return launch_mlp_fp8(a, s);
    if (prec == kPrecBF16) return launch_mlp_bf16(a, s);
    return launch_mlp_prec<kPrecFP32>(a, s);
}

}  // namespace nis
